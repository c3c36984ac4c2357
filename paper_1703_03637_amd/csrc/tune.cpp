// Schedule selection for the product kernels: defaults, the autotuner
// (hphi_hv_tune) and its on-disk cache.
//
// The tuner times candidate schedules of the real product on the caller's
// buffers -- window budget and number of passes of the windowed full-space
// kernel with or without staged copies (or the single-pass kernel), lanes
// per row, resident blocks per CU, LDS or global tables, cache hints on the
// streaming accesses -- and pins the fastest for (Hamiltonian, nvec, dtype).  With
// HPHI_TUNE_CACHE set, choices are appended to that file, keyed by a
// signature of the device, the space and the packed operators, and are
// reused by later processes without timing.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hphi_internal.h"

namespace hphi {
namespace {

int env_int(const char* name, int dflt) {
    const char* e = getenv(name);
    return (e && *e) ? atoi(e) : dflt;
}

Schedule default_schedule(const hphi_basis* B, int nvec) {
    Schedule s;
    s.windowed = 1;
    s.window_kb = 2048;
    s.max_passes = 3;
    s.lpr = nvec >= 16 ? 4 : (nvec >= 8 ? 2 : 1);
    // sectors wider than 32 bits: 6 resident blocks per CU measured fastest
    // (more waves in flight thrash the L2 on the 36-bit kagome sector)
    s.blocks_per_cu = (B->dev.sector != 0 && B->nbits > 32) ? 6 : 0;
    s.nt_streams = nvec >= 8 ? 1 : 0;
    // overrides for experiments
    s.windowed = env_int("HPHI_WINDOWED", s.windowed);
    s.window_kb = env_int("HPHI_L2_WINDOW_KB", s.window_kb);
    s.max_passes = env_int("HPHI_PASSES", s.max_passes);
    const int l = env_int("HPHI_LPR", 0);
    if ((l == 1 || l == 2 || l == 4 || l == 8) && l <= nvec) s.lpr = l;
    s.blocks_per_cu = env_int("HPHI_BLOCKS_PER_CU", s.blocks_per_cu);
    s.stage_tables = std::min(2, std::max(0, env_int("HPHI_STAGE_TABLES", s.stage_tables)));
    s.nt_streams = env_int("HPHI_NT_STREAMS", s.nt_streams) ? 1 : 0;
    s.sector_blocks = env_int("HPHI_SECTOR_BLOCKS", s.sector_blocks);
    if (s.window_kb < 1) s.window_kb = 2048;
    if (s.max_passes < 1) s.max_passes = 1;
    return s;
}

std::string signature(const hphi_ham* H, int nvec, int dtype) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    for (char& c : arch)
        if (c == ' ' || c == '|') c = '_';
    uint64_t h = 1469598103934665603ull;   // FNV-1a over the packed operators
    const unsigned char* p = reinterpret_cast<const unsigned char*>(H->ops.data());
    for (size_t i = 0; i < H->ops.size() * sizeof(DevOp); ++i) h = (h ^ p[i]) * 1099511628211ull;
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|bits%d|sector%d|dim%lld|ops%zu|%016llx|nvec%d|dtype%d", arch.c_str(),
             H->basis->nbits, H->basis->desc.sector, (long long)H->basis->dim, H->ops.size(),
             (unsigned long long)h, nvec, dtype);
    return buf;
}

bool cache_lookup(const std::string& sig, Schedule& out) {
    const char* path = getenv("HPHI_TUNE_CACHE");
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof(line), f)) {
        char key[300];
        Schedule s;
        const int n = sscanf(line, "%299s %d %d %d %d %d %d %d %d", key, &s.windowed, &s.window_kb, &s.max_passes,
                             &s.lpr, &s.blocks_per_cu, &s.stage_tables, &s.nt_streams, &s.sector_blocks);
        if (n == 8) s.sector_blocks = 0;   // entries written before the block-staged sector kernel
        if (n >= 8 && sig == key) {
            out = s;   // the last entry for a key wins
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const std::string& sig, const Schedule& s, double us) {
    const char* path = getenv("HPHI_TUNE_CACHE");
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d %d %d %d %d %d %d %.2f\n", sig.c_str(), s.windowed, s.window_kb, s.max_passes, s.lpr,
            s.blocks_per_cu, s.stage_tables, s.nt_streams, s.sector_blocks, us);
    fclose(f);
}

}  // namespace

Schedule schedule_for(const hphi_ham* ham, int nvec, int dtype) {
    hphi_ham* H = const_cast<hphi_ham*>(ham);
    {
        std::lock_guard<std::mutex> lock(H->plan_mu);
        for (const auto& t : H->tuned)
            if (t.nvec == nvec && t.dtype == dtype) return t.s;
    }
    Schedule s = default_schedule(H->basis, nvec);
    if (getenv("HPHI_TUNE_CACHE")) {
        Schedule c;
        if (cache_lookup(signature(H, nvec, dtype), c)) s = c;
        std::lock_guard<std::mutex> lock(H->plan_mu);
        H->tuned.push_back({nvec, dtype, s});
    }
    return s;
}

}  // namespace hphi

using namespace hphi;

extern "C" int hphi_hv_tune(const hphi_ham* ham, const void* v, void* u, int64_t nvec, int32_t dtype,
                            int32_t* sched_out, void* stream) {
    if (!ham || !v || !u) return set_error(HPHI_EINVAL, "hphi_hv_tune: null argument");
    if (u == v) return set_error(HPHI_EINVAL, "hphi_hv_tune: u must not alias v");
    if (!(nvec == 1 || nvec == 2 || nvec == 4 || nvec == 8 || nvec == 16))
        return set_error(HPHI_EINVAL, "hphi_hv_tune: nvec must be 1, 2, 4, 8 or 16");
    if (dtype < HPHI_F64 || dtype > HPHI_C64) return set_error(HPHI_EINVAL, "hphi_hv_tune: bad dtype");
    if (ham->is_complex && !dtype_complex(dtype))
        return set_error(HPHI_EDTYPE, "hphi_hv_tune: complex Hamiltonian with real storage");
    hipStream_t st = (hipStream_t)stream;
    const hphi_basis* B = ham->basis;
    const bool windowable = B->dev.sector == 0 && B->nbits >= 6 && B->nbits <= 32;
    const bool blockable = B->dev.sector != 0 && B->d_t1 && nvec <= 4;

    std::vector<Schedule> cands;
    std::vector<int> lprs = {1};
    if (nvec >= 8) lprs = {1, 2, 4, 8};
    else if (nvec >= 2) lprs = nvec >= 4 ? std::vector<int>{1, 2, 4} : std::vector<int>{1, 2};
    const bool wide_sector = B->dev.sector != 0 && B->nbits > 32;
    for (int bpc : (wide_sector ? std::vector<int>{0, 4, 6} : std::vector<int>{0, 4})) {
        for (int lpr : lprs) {
            Schedule s;
            s.sector_blocks = 0;
            s.lpr = lpr;
            s.blocks_per_cu = bpc;
            s.windowed = 0;
            s.window_kb = 2048;
            s.max_passes = 1;
            for (int tables : {1, 0}) {
                s.stage_tables = tables;
                cands.push_back(s);
            }
            if (B->dev.sector != 0 && B->nbits > 32 && B->d_t1) {
                s.stage_tables = 2;   // only the pattern table in LDS, not the two-level rank table
                cands.push_back(s);
            }
            s.stage_tables = 1;
            if (!windowable) continue;
            s.windowed = 1;
            cands.push_back(s);   // single natural pass, compact operators
            for (int nt : (nvec >= 8 ? std::vector<int>{1, 0} : std::vector<int>{0}))
                for (int wkb : {1024, 2048, 4096})
                    for (int mp : {2, 3})
                        for (int staged : {1, 2}) {
                            s.windowed = staged;
                            s.window_kb = wkb;
                            s.max_passes = mp;
                            s.nt_streams = nt;
                            cands.push_back(s);
                        }
            s.nt_streams = 0;
        }
    }
    if (blockable)
        for (int bpc : {1, 2, 3}) {
            Schedule s;
            s.windowed = 0;
            s.sector_blocks = 1;
            s.blocks_per_cu = bpc;
            cands.push_back(s);
        }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return set_error(HPHI_EDEVICE, "hphi_hv_tune: event creation failed");
    std::vector<double> times(cands.size(), 1e300);
    // microseconds per product of candidate ci: the best of `rounds` timings of `reps` calls
    auto time_cand = [&](size_t ci, int rounds, int reps) -> double {
        const Schedule& s = cands[ci];
        HvLaunch L{};
        L.ham = ham;
        L.v = v;
        L.u = u;
        L.a = 1.0;
        L.b = 0.0;
        L.nvec = int(nvec);
        L.dtype = dtype;
        L.sched = &s;
        int rc = launch_hv(L, st);   // warm-up (builds the plan)
        if (rc) return 1e300;
        double best = 1e300;
        for (int q = 0; q < rounds; ++q) {
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps && !rc; ++r) rc = launch_hv(L, st);
            (void)hipEventRecord(e1, st);
            if (rc || hipEventSynchronize(e1) != hipSuccess) return 1e300;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            best = std::min(best, 1e3 * double(ms) / reps);
        }
        return best;
    };
    for (size_t ci = 0; ci < cands.size(); ++ci) times[ci] = time_cand(ci, 1, 2);
    double fastest = 1e300;
    for (double t : times) fastest = t < fastest ? t : fastest;
    if (fastest >= 1e300) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return set_error(HPHI_EDEVICE, "hphi_hv_tune: no schedule ran");
    }
    // the candidates within 5% of the fastest are timed again, longer (one
    // short timing is a few percent noisy)
    const double first_fastest = fastest;
    fastest = 1e300;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        if (times[ci] > first_fastest * 1.05) continue;
        times[ci] = time_cand(ci, 3, 3);
        fastest = std::min(fastest, times[ci]);
    }
    for (size_t ci = 0; ci < cands.size(); ++ci)
        if (times[ci] > first_fastest * 1.05) times[ci] = 1e300;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (fastest >= 1e300) return set_error(HPHI_EDEVICE, "hphi_hv_tune: no schedule ran twice");
    // the first candidate within 1% of the fastest wins, so repeated tuning
    // settles on the same schedule
    size_t pick = 0;
    while (times[pick] > fastest * 1.01) ++pick;
    const Schedule best = cands[pick];
    const double best_us = times[pick];
    {
        hphi_ham* H = const_cast<hphi_ham*>(ham);
        std::lock_guard<std::mutex> lock(H->plan_mu);
        bool set = false;
        for (auto& t : H->tuned)
            if (t.nvec == int(nvec) && t.dtype == dtype) {
                t.s = best;
                set = true;
            }
        if (!set) H->tuned.push_back({int(nvec), dtype, best});
    }
    cache_store(signature(ham, int(nvec), dtype), best, best_us);
    if (sched_out) {
        sched_out[0] = best.windowed;
        sched_out[1] = best.window_kb;
        sched_out[2] = best.max_passes;
        sched_out[3] = best.lpr;
        sched_out[4] = best.blocks_per_cu;
        sched_out[5] = best.stage_tables;
        sched_out[6] = best.nt_streams;
        sched_out[7] = best.sector_blocks;
        sched_out[8] = int(best_us);
    }
    return HPHI_OK;
}
