// C entry points: argument checks, the Lanczos driver (Sec. 3.4) and the
// TPQ step (Sec. 3.5) on top of the product kernels.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hphi_internal.h"

namespace hphi {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int check_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return HPHI_OK;
    return set_error(e == hipErrorOutOfMemory ? HPHI_ENOMEM : HPHI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool alloc_fails() {
    static std::mutex mu;
    static std::string armed;
    static long count = 0;
    const char* e = std::getenv("HPHI_FAIL_ALLOC");
    std::lock_guard<std::mutex> g(mu);
    const std::string cur = e ? e : "";
    if (cur != armed) {
        armed = cur;
        count = 0;
    }
    const long n = cur.empty() ? 0 : std::strtol(cur.c_str(), nullptr, 10);
    if (n <= 0) return false;
    return ++count == n;
}

int dev_alloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (alloc_fails()) return set_error(HPHI_ENOMEM, "%s: device allocation of %zu bytes failed (injected)", what, bytes);
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return set_error(e == hipErrorOutOfMemory ? HPHI_ENOMEM : HPHI_EDEVICE, "%s: device allocation of %zu bytes: %s",
                         what, bytes, hipGetErrorString(e));
    }
    return HPHI_OK;
}

// Opt-in progress report of long Lanczos runs (HPHI_PROGRESS=N): every N
// steps the host waits for the stream and prints the step reached.
static int progress_every() {
    const char* e = std::getenv("HPHI_PROGRESS");
    return e ? std::atoi(e) : 0;
}

static void report_progress(hipStream_t st, const char* what, int k, int n) {
    (void)hipStreamSynchronize(st);
    std::fprintf(stderr, "[hphi] %s: step %d of %d done\n", what, k, n);
    std::fflush(stderr);
}

// Capture `body` (which enqueues work on the stream it is given) once into a
// graph and replay it `reps` times on a side stream joined to `st`.
template <typename Body>
int replay_pairs(hipStream_t st, Body body, int reps, const char* what = nullptr, int k0 = 0, int n = 0) {
    hipStream_t cs;
    int rc = check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "graph stream");
    if (rc) return rc;
    hipEvent_t ev;
    (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    (void)hipEventRecord(ev, st);
    (void)hipStreamWaitEvent(cs, ev, 0);
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    rc = check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
    if (!rc) {
        const int r = body(cs);
        const hipError_t e = hipStreamEndCapture(cs, &g);
        rc = r ? r : check_hip(e, "end capture");
    }
    if (!rc) rc = check_hip(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "graph instantiate");
    const int every = what ? progress_every() : 0;
    for (int k = 0; !rc && k < reps; ++k) {
        rc = check_hip(hipGraphLaunch(ge, cs), "graph launch");
        if (every > 0 && (k + 1) % ((every + 1) / 2) == 0) report_progress(cs, what, k0 + 2 * (k + 1), n);
    }
    (void)hipEventRecord(ev, cs);
    (void)hipStreamWaitEvent(st, ev, 0);
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
    (void)hipEventDestroy(ev);
    return rc;
}

static bool valid_dtype(int dt) { return dt == HPHI_F64 || dt == HPHI_C128 || dt == HPHI_F32 || dt == HPHI_C64; }
static bool valid_nvec(int64_t n) { return n == 1 || n == 2 || n == 4 || n == 8 || n == 16; }

}  // namespace hphi

using namespace hphi;

extern "C" const char* hphi_last_error(void) { return g_err; }

extern "C" const char* hphi_version(void) { return "hphi-mi355x 0.1 (gfx950)"; }

extern "C" int hphi_hv(const hphi_ham* ham, const void* v, void* u, int64_t nvec, int32_t dtype,
                       const hphi_hv_opts* opts, void* stream) {
    if (!ham || !v) return set_error(HPHI_EINVAL, "hphi_hv: null ham or v");
    if (u && u == v) return set_error(HPHI_EINVAL, "hphi_hv: u must not alias v");
    if (!valid_nvec(nvec)) return set_error(HPHI_EINVAL, "hphi_hv: nvec must be 1, 2, 4, 8 or 16");
    if (!valid_dtype(dtype)) return set_error(HPHI_EINVAL, "hphi_hv: bad dtype %d", dtype);
    if (ham->is_complex && !dtype_complex(dtype))
        return set_error(HPHI_EDTYPE, "hphi_hv: complex Hamiltonian with real storage");
    hphi_hv_opts o = opts ? *opts : hphi_hv_opts{1.0, 0.0, nullptr, nullptr};
    if (!std::isfinite(o.a) || !std::isfinite(o.b)) return set_error(HPHI_EINVAL, "hphi_hv: non-finite a or b");
    HvLaunch L{};
    L.ham = ham;
    L.v = v;
    L.u = u;
    L.y = nullptr;
    L.cy = nullptr;
    L.sx = o.in_scale;
    L.a = o.a;
    L.b = o.b;
    L.nvec = int(nvec);
    L.dtype = dtype;
    L.stop = nullptr;
    L.reduce_out = o.reduce;
    return launch_hv(L, (hipStream_t)stream);
}

extern "C" int hphi_hv_cma(const hphi_ham* ham, const void* v, void* u, int64_t nvec, int32_t dtype,
                           int32_t cluster_bits, const hphi_hv_opts* opts, void* stream) {
    if (!ham || !v || !u) return set_error(HPHI_EINVAL, "hphi_hv_cma: null ham, v or u");
    if (u == v) return set_error(HPHI_EINVAL, "hphi_hv_cma: u must not alias v");
    if (!valid_nvec(nvec)) return set_error(HPHI_EINVAL, "hphi_hv_cma: nvec must be 1, 2, 4, 8 or 16");
    if (!valid_dtype(dtype)) return set_error(HPHI_EINVAL, "hphi_hv_cma: bad dtype %d", dtype);
    if (ham->is_complex) return set_error(HPHI_EDTYPE, "hphi_hv_cma: complex matrix elements");
    hphi_hv_opts o = opts ? *opts : hphi_hv_opts{1.0, 0.0, nullptr, nullptr};
    if (!std::isfinite(o.a) || !std::isfinite(o.b)) return set_error(HPHI_EINVAL, "hphi_hv_cma: non-finite a or b");
    if ((dtype == HPHI_F64 || dtype == HPHI_C128) && cluster_bits > 6)
        return set_error(HPHI_EINVAL, "hphi_hv_cma: FP64 storage allows cluster_bits <= 6");
    const CmaPlan* P = nullptr;
    const int rc = get_cma_plan(ham, cluster_bits, &P);
    if (rc) return rc;
    HvLaunch L{};
    L.ham = ham;
    L.v = v;
    L.u = u;
    L.sx = o.in_scale;
    L.a = o.a;
    L.b = o.b;
    L.nvec = int(nvec);
    L.dtype = dtype;
    L.reduce_out = o.reduce;
    return launch_hv_cma(L, P, (hipStream_t)stream);
}

extern "C" int hphi_hv_cma_plan(const hphi_ham* ham, int32_t cluster_bits, int32_t* n_clusters, int32_t* sites) {
    if (!ham || !n_clusters) return set_error(HPHI_EINVAL, "hphi_hv_cma_plan: null ham or n_clusters");
    const CmaPlan* P = nullptr;
    const int rc = get_cma_plan(ham, cluster_bits, &P);
    if (rc) return rc;
    *n_clusters = P->n_stage;
    if (sites) {
        // cluster bits in ascending order (the plan lists them so)
        for (int c = 0; c < P->n_stage; ++c)
            for (int j = 0; j < P->M; ++j) sites[c * P->M + j] = P->bits[size_t(c) * 64 + j];
    }
    return HPHI_OK;
}

extern "C" int hphi_hv_elements(const hphi_ham* ham, int64_t row0, int64_t nrows, int32_t cap, int64_t nvec,
                                int32_t dtype, int64_t* cols, double* re, double* im, int32_t* term_id,
                                int32_t* counts, void* stream) {
    if (!ham) return set_error(HPHI_EINVAL, "hphi_hv_elements: null ham");
    const hphi_basis* B = ham->basis;
    if (row0 < 0 || nrows < 0 || row0 + nrows > B->dim)
        return set_error(HPHI_EINVAL, "hphi_hv_elements: rows out of range");
    if (nrows > (int64_t(1) << 22)) return set_error(HPHI_EINVAL, "hphi_hv_elements: at most 2^22 rows per call");
    if (cap < 1 || !cols || !re || !im || !term_id || !counts)
        return set_error(HPHI_EINVAL, "hphi_hv_elements: bad output arrays");
    if (!valid_nvec(nvec) || (B->nbits > 32 && nvec > 4))
        return set_error(HPHI_EINVAL, "hphi_hv_elements: nvec not supported by the product for this space");
    if (dtype != HPHI_C128 && dtype != HPHI_C64)
        return set_error(HPHI_EINVAL, "hphi_hv_elements: the export follows a complex storage type (C128 or C64)");
    if (nrows == 0) return HPHI_OK;
    hipStream_t st = (hipStream_t)stream;
    constexpr int kExportPasses = 8;
    ExportArgs ex;
    ex.row0 = row0;
    ex.nrows = nrows;
    ex.n_slots = int(ham->ops.size());
    ex.n_pass = kExportPasses;
    // tiles of the single-pass kernel that hold the rows
    auto tile_of = [&](int64_t r) -> int64_t {
        if (B->dev.sector == 0) return r / kTile;
        const int64_t k = int64_t(std::upper_bound(B->h_row.begin(), B->h_row.end() - 1, r) - B->h_row.begin()) - 1;
        return B->h_tile[size_t(k)] + (r - B->h_row[size_t(k)]) / kTile;
    };
    ex.t0 = tile_of(row0);
    ex.t1 = tile_of(row0 + nrows - 1) + 1;
    const size_t nrec = size_t(nrows) * size_t(ex.n_slots > 0 ? ex.n_slots : 1);
    const size_t bytes = nrec * 24 + size_t(nrows) * kExportPasses * 8;
    char* mem = nullptr;
    if (int rc = dev_alloc((void**)&mem, bytes, "hphi_hv_elements: records")) return rc;
    ex.col = reinterpret_cast<int64_t*>(mem);
    ex.cr = reinterpret_cast<double*>(mem + nrec * 8);
    ex.ci = reinterpret_cast<double*>(mem + nrec * 16);
    ex.diag = reinterpret_cast<double*>(mem + nrec * 24);
    int rc = launch_fill_zero(mem, int64_t(bytes), st);
    HvLaunch L{};
    L.ham = ham;
    L.a = 1.0;
    L.b = 0.0;
    L.nvec = int(nvec);
    L.dtype = dtype;
    L.ex = &ex;
    if (!rc) rc = launch_hv(L, st);
    if (!rc) rc = launch_elements_compact(ham, ex, cap, cols, re, im, term_id, counts, st);
    const hipError_t e = hipStreamSynchronize(st);
    (void)hipFree(mem);
    return rc ? rc : check_hip(e, "hphi_hv_elements sync");
}

extern "C" int hphi_expect(const hphi_ham* obs, const void* psi, int64_t nvec, int32_t dtype, double* out,
                           void* stream) {
    if (!obs || !psi || !out) return set_error(HPHI_EINVAL, "hphi_expect: null argument");
    if (!valid_nvec(nvec)) return set_error(HPHI_EINVAL, "hphi_expect: nvec must be 1, 2, 4, 8 or 16");
    if (!valid_dtype(dtype)) return set_error(HPHI_EINVAL, "hphi_expect: bad dtype");
    if (obs->is_complex && !dtype_complex(dtype))
        return set_error(HPHI_EDTYPE, "hphi_expect: complex observable with real storage");
    HvLaunch L{};
    L.ham = obs;
    L.v = psi;
    L.u = nullptr;       // reductions only
    L.a = 1.0;
    L.b = 0.0;
    L.nvec = int(nvec);
    L.dtype = dtype;
    L.reduce_out = obs->d_red;
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_hv(L, st);
    if (rc) return rc;
    return launch_expect(obs->d_red, out, int(nvec), st);
}

extern "C" int hphi_tpq_step(const hphi_ham* ham, const void* psi_in, void* psi_out, int64_t nvec, int32_t dtype,
                             double l, int32_t k, const double* in_scale, double* obs, void* stream) {
    if (!ham || !psi_in || !psi_out || !obs) return set_error(HPHI_EINVAL, "hphi_tpq_step: null argument");
    if (psi_in == psi_out) return set_error(HPHI_EINVAL, "hphi_tpq_step: psi_out must not alias psi_in");
    if (!valid_nvec(nvec)) return set_error(HPHI_EINVAL, "hphi_tpq_step: nvec must be 1, 2, 4, 8 or 16");
    if (!valid_dtype(dtype)) return set_error(HPHI_EINVAL, "hphi_tpq_step: bad dtype");
    if (ham->is_complex && !dtype_complex(dtype))
        return set_error(HPHI_EDTYPE, "hphi_tpq_step: complex Hamiltonian with real storage");
    if (k < 1 || !std::isfinite(l)) return set_error(HPHI_EINVAL, "hphi_tpq_step: need k >= 1 and finite l");
    const double ns = double(ham->n_sites);
    HvLaunch L{};
    L.ham = ham;
    L.v = psi_in;
    L.u = psi_out;
    L.sx = in_scale;
    L.a = -1.0 / ns;
    L.b = l;
    L.nvec = int(nvec);
    L.dtype = dtype;
    L.reduce_out = ham->d_red;
    hipStream_t st = (hipStream_t)stream;
    int rc = launch_hv(L, st);
    if (rc) return rc;
    return launch_tpq_obs(ham->d_red, obs, int(nvec), ns, l, k, st);
}

extern "C" int hphi_tpq_run(const hphi_ham* ham, void* psi_a, void* psi_b, int64_t nvec, int32_t dtype, double l,
                            int32_t k0, int32_t n_steps, const double* in_scale, double* obs_log, int32_t use_graph,
                            void* stream) {
    if (!ham || !psi_a || !psi_b || !obs_log) return set_error(HPHI_EINVAL, "hphi_tpq_run: null argument");
    if (psi_a == psi_b) return set_error(HPHI_EINVAL, "hphi_tpq_run: the two state buffers must differ");
    if (!valid_nvec(nvec)) return set_error(HPHI_EINVAL, "hphi_tpq_run: nvec must be 1, 2, 4, 8 or 16");
    if (!valid_dtype(dtype)) return set_error(HPHI_EINVAL, "hphi_tpq_run: bad dtype");
    if (ham->is_complex && !dtype_complex(dtype))
        return set_error(HPHI_EDTYPE, "hphi_tpq_run: complex Hamiltonian with real storage");
    if (k0 < 1 || n_steps < 0 || !std::isfinite(l))
        return set_error(HPHI_EINVAL, "hphi_tpq_run: need k0 >= 1, n_steps >= 0 and finite l");
    if (n_steps == 0) return HPHI_OK;
    hipStream_t st = (hipStream_t)stream;
    TpqRunState* S = nullptr;
    if (int rc = dev_alloc((void**)&S, sizeof(TpqRunState), "hphi_tpq_run: state")) return rc;
    const double ns = double(ham->n_sites);
    // step of parity p reads buffer p (a or b) and writes the other; its input
    // scale is the caller's for the first step, else the previous step's
    auto step = [&](int parity, bool first, hipStream_t s) {
        HvLaunch L{};
        L.ham = ham;
        L.v = parity ? psi_b : psi_a;
        L.u = parity ? psi_a : psi_b;
        L.sx = first ? in_scale : S->scale[parity ^ 1];
        L.a = -1.0 / ns;
        L.b = l;
        L.nvec = int(nvec);
        L.dtype = dtype;
        L.reduce_out = ham->d_red;
        int rc = launch_hv(L, s);
        return rc ? rc : launch_tpq_obs_run(ham->d_red, S, obs_log, int(nvec), ns, l, s);
    };
    int rc = launch_tpq_run_init(S, k0, st);
    if (!rc) rc = step(0, true, st);      // eager: allocates lazily built plans before any capture
    int j = 1;
    if (!rc && use_graph && n_steps - j >= 4) {
        rc = replay_pairs(st, [&](hipStream_t cs) {
            int r = step(1, false, cs);
            return r ? r : step(0, false, cs);
        }, (n_steps - j) / 2);
        if (!rc) j += (n_steps - j) / 2 * 2;
    }
    for (; !rc && j < n_steps; ++j) rc = step(j & 1, false, st);
    const hipError_t e = hipStreamSynchronize(st);
    (void)hipFree(S);
    return rc ? rc : check_hip(e, "hphi_tpq_run sync");
}

extern "C" int hphi_tpq_run_noalloc(const hphi_ham* ham, void* psi_a, void* psi_b, int64_t nvec, int32_t dtype,
                                    double l, int32_t k0, int32_t n_steps, const double* in_scale, double* obs_log,
                                    void* stream) {
    if (!ham || !psi_a || !psi_b || !obs_log) return set_error(HPHI_EINVAL, "hphi_tpq_run_noalloc: null argument");
    if (psi_a == psi_b) return set_error(HPHI_EINVAL, "hphi_tpq_run_noalloc: the two state buffers must differ");
    if (!valid_nvec(nvec) || nvec > kMaxNvec)
        return set_error(HPHI_EINVAL, "hphi_tpq_run_noalloc: nvec must be 1, 2, 4, 8 or 16 (the static state holds "
                                      "the scales of at most %d samples)", kMaxNvec);
    if (!valid_dtype(dtype)) return set_error(HPHI_EINVAL, "hphi_tpq_run_noalloc: bad dtype");
    if (ham->is_complex && !dtype_complex(dtype))
        return set_error(HPHI_EDTYPE, "hphi_tpq_run_noalloc: complex Hamiltonian with real storage");
    if (k0 < 1 || n_steps < 0 || !std::isfinite(l))
        return set_error(HPHI_EINVAL, "hphi_tpq_run_noalloc: need k0 >= 1, n_steps >= 0 and finite l");
    if (n_steps == 0) return HPHI_OK;
    TpqRunState* S = nullptr;
    if (int rc = tpq_static_state(&S)) return rc;
    hipStream_t st = (hipStream_t)stream;
    const double ns = double(ham->n_sites);
    int rc = launch_tpq_run_init(S, k0, st);
    for (int j = 0; !rc && j < n_steps; ++j) {
        const int parity = j & 1;
        HvLaunch L{};
        L.ham = ham;
        L.v = parity ? psi_b : psi_a;
        L.u = parity ? psi_a : psi_b;
        L.sx = j == 0 ? in_scale : S->scale[parity ^ 1];
        L.a = -1.0 / ns;
        L.b = l;
        L.nvec = int(nvec);
        L.dtype = dtype;
        L.reduce_out = ham->d_red;
        L.no_alloc = true;
        rc = launch_hv(L, st);
        if (!rc) rc = launch_tpq_obs_run(ham->d_red, S, obs_log, int(nvec), ns, l, st);
    }
    return rc;
}

// ---------------------------------------------------------------- Lanczos

namespace {

struct LzDev {
    LzScalars* sc = nullptr;
    double* alpha = nullptr;
    double* beta = nullptr;
    double* evec = nullptr;
    double* red = nullptr;
    double* spart = nullptr;   // partials of the streaming kernels
    void* mem = nullptr;
};

constexpr int kStreamGrid = 1024;

int lz_alloc(LzDev& D, int n) {
    const size_t bytes = 256 + 3 * size_t(n) * 8 + 64 * 8 + size_t(kStreamGrid) * 8 + 1024;
    char* p = nullptr;
    if (int rc = dev_alloc((void**)&p, bytes, "hphi_lanczos: scalar workspace")) return rc;
    D.mem = p;
    D.sc = (LzScalars*)p;
    p += 256;
    D.alpha = (double*)p;
    p += size_t(n) * 8;
    D.beta = (double*)p;
    p += size_t(n) * 8;
    D.evec = (double*)p;
    p += size_t(n) * 8;
    D.red = (double*)p;
    p += 64 * 8;
    D.spart = (double*)p;
    return HPHI_OK;
}

int stream_grid_for(int64_t scalars) {
    int64_t g = (scalars + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > kStreamGrid) g = kStreamGrid;
    return int(g);
}

// One Lanczos iteration: pass 1 (product, alpha) and pass 2 (update, beta).
int lz_iteration(const hphi_ham* H, int dtype, void* X, void* Y, bool first, LzDev& D, void* acc, int grid,
                 hipStream_t st) {
    const int* stop = &D.sc->stop;
    HvLaunch L{};
    L.ham = H;
    L.v = X;
    L.u = Y;
    L.y = first ? nullptr : Y;
    L.cy = &D.sc->cy;
    L.sx = &D.sc->s_cur;
    L.a = 1.0;
    L.b = 0.0;
    L.nvec = 1;
    L.dtype = dtype;
    L.stop = stop;
    L.reduce_out = D.red;
    // each reduction launch also takes the scalar step that reads its sums
    L.lz_sc = D.sc;
    L.lz_alpha = D.alpha;
    L.lz_evec = acc ? D.evec : nullptr;
    int rc = launch_hv(L, st);
    if (rc) return rc;
    return launch_lanczos_update_lz(Y, X, H->basis->dim, dtype, D.sc, acc, D.spart, grid, D.red, D.beta, D.alpha,
                                    H->d_flag, st);
}

// Run the recurrence from v0 for n_max steps (pass 1 or the eigenvector pass).
int lz_run(const hphi_ham* H, int dtype, const void* v0, void* A, void* B, LzDev& D, int n_max, double tol,
           void* acc, bool use_graph, hipStream_t st) {
    const int64_t dim = H->basis->dim;
    const int64_t scalars = dim * (dtype_complex(dtype) ? 2 : 1);
    const int grid = stream_grid_for(scalars);
    int rc = launch_copy_norm(v0, A, dim, dtype, D.spart, grid, D.red, H->d_flag, st);
    if (rc) return rc;
    // the eigenvector accumulator starts at zero; it may share v0's buffer,
    // which is not read again after the copy above
    if (acc) rc = launch_fill_zero(acc, dim * int64_t(dtype_complex(dtype) ? 16 : 8), st);
    if (rc) return rc;
    rc = launch_lz_init(D.sc, D.red, tol, n_max, st);
    if (rc) return rc;
    rc = lz_iteration(H, dtype, A, B, true, D, acc, grid, st);
    if (rc) return rc;
    int k = 1;
    const char* what = acc ? "lanczos second pass" : "lanczos";
    if (use_graph && n_max >= 3) {
        // iterations (odd, even) captured once and replayed; the device-side
        // step counter and stop flag make every replay advance the recurrence
        rc = replay_pairs(st, [&](hipStream_t cs) {
            int r = lz_iteration(H, dtype, B, A, false, D, acc, grid, cs);
            return r ? r : lz_iteration(H, dtype, A, B, false, D, acc, grid, cs);
        }, (n_max - 1) / 2, what, 1, n_max);
        if (rc) return rc;
        k += (n_max - 1) / 2 * 2;
    }
    const int every = progress_every();
    for (; k < n_max; ++k) {
        void* X = (k & 1) ? B : A;
        void* Y = (k & 1) ? A : B;
        rc = lz_iteration(H, dtype, X, Y, false, D, acc, grid, st);
        if (rc) return rc;
        if (every > 0 && (k + 1) % every == 0) report_progress(st, what, k + 1, n_max);
    }
    return HPHI_OK;
}

// ---- batched recurrence: several problems advance together, one launch
// per kernel and step (uneven sizes share the persistent grid)

struct LzBatch {
    LzScalars* sc = nullptr;   // [n]
    double* alpha = nullptr;   // [n][n_iter]
    double* beta = nullptr;
    double* evec = nullptr;
    double* red = nullptr;     // [n][kNQ]
    double* spart = nullptr;   // [kStreamGrid]
    void* mem = nullptr;
};

int lzb_alloc(LzBatch& D, int n, int n_iter) {
    const size_t sc_b = (size_t(n) * sizeof(LzScalars) + 255) / 256 * 256;
    const size_t arr = size_t(n) * n_iter * 8;
    const size_t bytes = sc_b + 3 * arr + size_t(n) * kNQ * 8 + size_t(kStreamGrid) * 8 + 1024;
    char* p = nullptr;
    if (int rc = dev_alloc((void**)&p, bytes, "hphi_lanczos: batched workspace")) return rc;
    D.mem = p;
    D.sc = (LzScalars*)p;
    p += sc_b;
    D.alpha = (double*)p;
    p += arr;
    D.beta = (double*)p;
    p += arr;
    D.evec = (double*)p;
    p += arr;
    D.red = (double*)p;
    p += size_t(n) * kNQ * 8;
    D.spart = (double*)p;
    return HPHI_OK;
}

struct BatchPlans {
    MultiPlan hv_first, hv[2];
    UpdPlan upd[2];
    void release() {
        for (void* m : {hv_first.mem, hv[0].mem, hv[1].mem, upd[0].mem, upd[1].mem})
            if (m) (void)hipFree(m);
        hv_first.mem = hv[0].mem = hv[1].mem = upd[0].mem = upd[1].mem = nullptr;
    }
};

// parity 0: X = A, Y = B; parity 1: X = B, Y = A
int lzb_plans(const hphi_ham* const* H, int n, int dtype, void* const* A, void* const* Bv, LzBatch& D,
              void* const* acc, BatchPlans& P) {
    std::vector<HvLaunch> Ls(n);
    std::vector<UpdDesc> U(n);
    std::vector<double*> ured(n);
    for (int first = 1; first >= 0; --first)
        for (int q = 0; q < (first ? 1 : 2); ++q) {
            for (int p = 0; p < n; ++p) {
                void* X = q ? Bv[p] : A[p];
                void* Y = q ? A[p] : Bv[p];
                HvLaunch& L = Ls[p];
                L = HvLaunch{};
                L.ham = H[p];
                L.v = X;
                L.u = Y;
                L.y = first ? nullptr : Y;
                L.cy = &D.sc[p].cy;
                L.sx = &D.sc[p].s_cur;
                L.a = 1.0;
                L.b = 0.0;
                L.nvec = 1;
                L.dtype = dtype;
                L.stop = &D.sc[p].stop;
                L.reduce_out = D.red + size_t(kNQ) * p;
                if (!first) {
                    UpdDesc& u = U[p];
                    u = UpdDesc{};
                    u.y = Y;
                    u.x = X;
                    u.n = H[p]->basis->dim * (dtype_complex(dtype) ? 2 : 1);
                    u.c2 = &D.sc[p].c2;
                    u.acc = acc ? static_cast<double*>(acc[p]) : nullptr;
                    u.ec = &D.sc[p].ecoef;
                    u.stop = &D.sc[p].stop;
                    u.flag = H[p]->d_flag;
                    ured[p] = D.red + size_t(kNQ) * p;
                }
            }
            int rc = hv_multi_prepare(Ls.data(), n, first ? &P.hv_first : &P.hv[q]);
            if (!rc && !first) rc = upd_multi_prepare(U.data(), ured.data(), n, dtype, &P.upd[q]);
            if (rc) return rc;
        }
    return HPHI_OK;
}

int lzb_iteration(const BatchPlans& P, int parity, bool first, LzBatch& D, bool acc, int n_iter, hipStream_t st) {
    // each reduction launch also takes the scalar steps that read its sums
    const LzMulti lz{D.sc, D.alpha, D.beta, acc ? D.evec : nullptr, n_iter};
    int rc = hv_multi_launch(first ? P.hv_first : P.hv[parity], &lz, st);
    if (!rc) rc = upd_multi_launch(P.upd[parity], &lz, st);
    return rc;
}

// Run all recurrences from v0 for up to n_max[p] steps (pass 1, or the
// eigenvector pass when acc != nullptr).
int lzb_run(const hphi_ham* const* H, int n, int dtype, const void* const* v0, void* const* A, void* const* Bv,
            LzBatch& D, const int* n_max, double tol, void* const* acc, bool use_graph, int n_iter, hipStream_t st) {
    int N = 0;
    for (int p = 0; p < n; ++p) {
        const int64_t dim = H[p]->basis->dim;
        const int grid = stream_grid_for(dim * (dtype_complex(dtype) ? 2 : 1));
        double* red = D.red + size_t(kNQ) * p;
        int rc = launch_copy_norm(v0[p], A[p], dim, dtype, D.spart, grid, red, H[p]->d_flag, st);
        // eigenvector accumulator (may share v0's buffer, not read again)
        if (!rc && acc) rc = launch_fill_zero(acc[p], dim * int64_t(dtype_complex(dtype) ? 16 : 8), st);
        if (!rc) rc = launch_lz_init(D.sc + p, red, tol, n_max[p], st);
        if (rc) return rc;
        if (n_max[p] > N) N = n_max[p];
    }
    BatchPlans P;
    int rc = lzb_plans(H, n, dtype, A, Bv, D, acc, P);
    if (!rc) rc = lzb_iteration(P, 0, true, D, acc != nullptr, n_iter, st);
    int k = 1;
    if (!rc && use_graph && N >= 3) {
        hipStream_t cs;
        rc = check_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "graph stream");
        if (!rc) {
            hipEvent_t ev;
            (void)hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            (void)hipEventRecord(ev, st);
            (void)hipStreamWaitEvent(cs, ev, 0);
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            rc = check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
            if (!rc) {
                int r1 = lzb_iteration(P, 1, false, D, acc != nullptr, n_iter, cs);
                int r2 = r1 ? r1 : lzb_iteration(P, 0, false, D, acc != nullptr, n_iter, cs);
                hipError_t e = hipStreamEndCapture(cs, &g);
                rc = r2 ? r2 : check_hip(e, "end capture");
            }
            if (!rc) rc = check_hip(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "graph instantiate");
            for (; !rc && k + 2 <= N; k += 2) rc = check_hip(hipGraphLaunch(ge, cs), "graph launch");
            (void)hipEventRecord(ev, cs);
            (void)hipStreamWaitEvent(st, ev, 0);
            if (ge) (void)hipGraphExecDestroy(ge);
            if (g) (void)hipGraphDestroy(g);
            (void)hipStreamSynchronize(cs);
            (void)hipStreamDestroy(cs);
            (void)hipEventDestroy(ev);
        }
    }
    for (; !rc && k < N; ++k) rc = lzb_iteration(P, k & 1, false, D, acc != nullptr, n_iter, st);
    // plans are read by kernels still in flight: release after the stream drains
    hipError_t e = hipStreamSynchronize(st);
    P.release();
    if (!rc) rc = check_hip(e, "batched lanczos sync");
    return rc;
}

// FP64 check of a Ritz vector x: <x|x>, <x|Hx>, |Hx|^2, then |Hx - E x|^2
int refine_one(const hphi_ham* H, const void* x, int x_dtype, double* red, hphi_lanczos_result& r,
               hipStream_t st) {
    HvLaunch L{};
    L.ham = H;
    L.v = x;
    L.u = nullptr;
    L.a = 1.0;
    L.b = 0.0;
    L.nvec = 1;
    L.dtype = x_dtype;
    L.reduce_out = red;
    int rc = launch_hv(L, st);
    double q[4];
    if (!rc) rc = check_hip(hipMemcpyAsync(q, red, 32, hipMemcpyDeviceToHost, st), "copy red");
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "refine sync");
    if (rc) return rc;
    const double E = q[1] / q[0];
    r.e0_refined = E;
    r.variance = q[2] / q[0] - E * E;
    L.b = -E;
    rc = launch_hv(L, st);
    if (!rc) rc = check_hip(hipMemcpyAsync(q, red, 32, hipMemcpyDeviceToHost, st), "copy red");
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "refine sync");
    if (rc) return rc;
    r.residual = std::sqrt(q[3] / q[0]);
    return HPHI_OK;
}

// Batched Lanczos (all problems in one launch per kernel and step).
int lanczos_batched(const hphi_ham* const* hams, int n, const hphi_lanczos_opts& o, double tol,
                    const void* const* v0, void* const* work, void* const* x_out, hphi_lanczos_result* res,
                    hipStream_t st) {
    const int x_dtype = dtype_complex(o.dtype) ? HPHI_C128 : HPHI_F64;
    LzBatch D;
    int rc = lzb_alloc(D, n, o.n_iter);
    if (rc) return rc;
    std::vector<int> n_max(n);
    std::vector<void*> A(n), Bv(n);
    for (int h = 0; h < n; ++h) {
        const int64_t dim = hams[h]->basis->dim;
        n_max[h] = int(dim < o.n_iter ? dim : o.n_iter);
        A[h] = work[h];
        Bv[h] = (char*)work[h] + size_t(dim) * dtype_size(o.dtype);
    }
    rc = lzb_run(hams, n, o.dtype, v0, A.data(), Bv.data(), D, n_max.data(), tol, nullptr, o.use_graph != 0,
                 o.n_iter, st);
    std::vector<LzScalars> sc(n);
    std::vector<double> alpha(size_t(n) * o.n_iter), beta(size_t(n) * o.n_iter);
    if (!rc) rc = check_hip(hipMemcpyAsync(sc.data(), D.sc, size_t(n) * sizeof(LzScalars), hipMemcpyDeviceToHost, st),
                            "copy scalars");
    if (!rc) rc = check_hip(hipMemcpyAsync(alpha.data(), D.alpha, alpha.size() * 8, hipMemcpyDeviceToHost, st), "copy alpha");
    if (!rc) rc = check_hip(hipMemcpyAsync(beta.data(), D.beta, beta.size() * 8, hipMemcpyDeviceToHost, st), "copy beta");
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "lanczos sync");
    std::vector<double> evecs(size_t(n) * o.n_iter, 0.0);
    std::vector<int> n_done(n, 0);
    for (int h = 0; h < n && !rc; ++h) {
        const int nd = sc[h].n_done;
        n_done[h] = nd;
        res[h].n_done = nd;
        res[h].info = (sc[h].breakdown || nd < o.n_iter) ? HPHI_INFO_BREAKDOWN : HPHI_OK;
        for (int k = 0; k < o.n_iter; ++k) {
            res[h].alpha[k] = k < nd ? alpha[size_t(h) * o.n_iter + k] : 0.0;
            res[h].beta[k] = k < nd ? beta[size_t(h) * o.n_iter + k] : 0.0;
        }
        if (nd < 1) rc = set_error(HPHI_EINVAL, "hphi_lanczos: zero start vector for problem %d", h);
        else res[h].e0_ritz = tridiag_lowest(res[h].alpha, res[h].beta, nd, evecs.data() + size_t(h) * o.n_iter);
        res[h].e0_refined = res[h].variance = res[h].residual = NAN;
    }
    if (!rc && o.refine) {
        // second pass: replay every recurrence and accumulate x = sum_k e~_k v_k
        rc = check_hip(hipMemcpyAsync(D.evec, evecs.data(), evecs.size() * 8, hipMemcpyHostToDevice, st), "copy evec");
        if (!rc) rc = lzb_run(hams, n, o.dtype, v0, A.data(), Bv.data(), D, n_done.data(), tol, x_out,
                              o.use_graph != 0, o.n_iter, st);
        for (int h = 0; h < n && !rc; ++h) rc = refine_one(hams[h], x_out[h], x_dtype, D.red, res[h], st);
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(D.mem);
    return rc;
}

int lanczos_each(const hphi_ham* const* hams, int n_hams, const hphi_lanczos_opts& o, double tol,
                 const void* const* v0, void* const* work, void* const* x_out, hphi_lanczos_result* res,
                 hipStream_t st);

// all problems can share one launch: same coefficient type, space kind and width
bool batchable(const hphi_ham* const* hams, int n) {
    if (n < 2 || n > 64) return false;
    for (int h = 1; h < n; ++h) {
        if (hams[h]->is_complex != hams[0]->is_complex) return false;
        if ((hams[h]->basis->dev.sector != 0) != (hams[0]->basis->dev.sector != 0)) return false;
        if ((hams[h]->basis->nbits > 32) != (hams[0]->basis->nbits > 32)) return false;
    }
    return true;
}

}  // namespace

extern "C" int hphi_lanczos(const hphi_ham* const* hams, int32_t n_hams, const hphi_lanczos_opts* opts,
                            const void* const* v0, void* const* work, void* const* x_out, hphi_lanczos_result* res,
                            void* stream) {
    if (!hams || n_hams < 1 || !opts || !v0 || !work || !res) return set_error(HPHI_EINVAL, "hphi_lanczos: null argument");
    const hphi_lanczos_opts o = *opts;
    if (o.n_iter < 1 || o.n_iter > 100000) return set_error(HPHI_EINVAL, "hphi_lanczos: n_iter out of range");
    if (!valid_dtype(o.dtype)) return set_error(HPHI_EINVAL, "hphi_lanczos: bad dtype");
    if (o.refine && !x_out) return set_error(HPHI_EINVAL, "hphi_lanczos: refine needs x_out");
    for (int h = 0; h < n_hams; ++h) {
        if (!hams[h] || !v0[h] || !work[h] || !res[h].alpha || !res[h].beta)
            return set_error(HPHI_EINVAL, "hphi_lanczos: null entry for problem %d", h);
        if (o.refine && !x_out[h]) return set_error(HPHI_EINVAL, "hphi_lanczos: null x_out for problem %d", h);
        if (hams[h]->is_complex && !dtype_complex(o.dtype))
            return set_error(HPHI_EDTYPE, "hphi_lanczos: complex Hamiltonian with real storage");
    }
    const double tol = o.breakdown_tol > 0 ? o.breakdown_tol : 1e-13;
    hipStream_t st = (hipStream_t)stream;
    for (int h = 0; h < n_hams; ++h)
        if (int rc = launch_fill_zero(hams[h]->d_flag, sizeof(int32_t), st)) return rc;
    const int rc_run = batchable(hams, n_hams) ? lanczos_batched(hams, n_hams, o, tol, v0, work, x_out, res, st)
                                               : lanczos_each(hams, n_hams, o, tol, v0, work, x_out, res, st);
    // a NaN or Inf start vector also ends the recurrence at once (its norm is
    // not positive): the flag word names the cause
    if (rc_run != HPHI_OK && rc_run != HPHI_EINVAL) return rc_run;
    const std::string msg = hphi_last_error();
    for (int h = 0; h < n_hams; ++h) {
        int32_t f = 0;
        int rc = check_hip(hipMemcpyAsync(&f, hams[h]->d_flag, sizeof(f), hipMemcpyDeviceToHost, st), "copy flag");
        if (!rc) rc = check_hip(hipStreamSynchronize(st), "lanczos sync");
        if (rc) return rc;
        if (f) return set_error(HPHI_ENONFINITE, "hphi_lanczos: non-finite norm or sum in problem %d (flags %d)", h, f);
    }
    if (rc_run) set_error(rc_run, "%s", msg.c_str());
    return rc_run;
}

extern "C" int hphi_ham_nonfinite(const hphi_ham* ham, int32_t* flags, int32_t clear, void* stream) {
    if (!ham || !flags) return set_error(HPHI_EINVAL, "hphi_ham_nonfinite: null argument");
    hipStream_t st = (hipStream_t)stream;
    int rc = check_hip(hipMemcpyAsync(flags, ham->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st), "copy flag");
    if (!rc && clear) rc = launch_fill_zero(ham->d_flag, sizeof(int32_t), st);
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "flag sync");
    return rc;
}

namespace {

// one problem after the other (problems that cannot share a launch)
int lanczos_each(const hphi_ham* const* hams, int n_hams, const hphi_lanczos_opts& o, double tol,
                 const void* const* v0, void* const* work, void* const* x_out, hphi_lanczos_result* res,
                 hipStream_t st) {
    const int x_dtype = dtype_complex(o.dtype) ? HPHI_C128 : HPHI_F64;

    for (int h = 0; h < n_hams; ++h) {
        const hphi_ham* H = hams[h];
        const int64_t dim = H->basis->dim;
        const int n_max = int(dim < o.n_iter ? dim : o.n_iter);
        const size_t vbytes = size_t(dim) * dtype_size(o.dtype);
        void* A = work[h];
        void* Bv = (char*)work[h] + vbytes;
        LzDev D;
        int rc = lz_alloc(D, o.n_iter);
        if (rc) return rc;
        auto fail = [&](int code) {
            (void)hipFree(D.mem);
            return code;
        };
        rc = lz_run(H, o.dtype, v0[h], A, Bv, D, n_max, tol, nullptr, o.use_graph != 0, st);
        if (rc) return fail(rc);
        LzScalars sc{};
        rc = check_hip(hipMemcpyAsync(&sc, D.sc, sizeof(sc), hipMemcpyDeviceToHost, st), "copy scalars");
        if (!rc) rc = check_hip(hipMemcpyAsync(res[h].alpha, D.alpha, size_t(o.n_iter) * 8, hipMemcpyDeviceToHost, st), "copy alpha");
        if (!rc) rc = check_hip(hipMemcpyAsync(res[h].beta, D.beta, size_t(o.n_iter) * 8, hipMemcpyDeviceToHost, st), "copy beta");
        if (!rc) rc = check_hip(hipStreamSynchronize(st), "lanczos sync");
        if (rc) return fail(rc);
        const int n = sc.n_done;
        res[h].n_done = n;
        res[h].info = (sc.breakdown || n < o.n_iter) ? HPHI_INFO_BREAKDOWN : HPHI_OK;
        for (int k = n; k < o.n_iter; ++k) {
            res[h].alpha[k] = 0.0;
            res[h].beta[k] = 0.0;
        }
        if (n < 1) return fail(set_error(HPHI_EINVAL, "hphi_lanczos: zero start vector for problem %d", h));
        std::vector<double> evec(n);
        res[h].e0_ritz = tridiag_lowest(res[h].alpha, res[h].beta, n, evec.data());
        res[h].e0_refined = res[h].variance = res[h].residual = NAN;
        if (o.refine) {
            // second pass: replay the recurrence and accumulate x = sum_k e~_k v_k
            rc = check_hip(hipMemcpyAsync(D.evec, evec.data(), size_t(n) * 8, hipMemcpyHostToDevice, st), "copy evec");
            if (!rc) rc = lz_run(H, o.dtype, v0[h], A, Bv, D, n, tol, x_out[h], o.use_graph != 0, st);
            if (rc) return fail(rc);
            rc = refine_one(H, x_out[h], x_dtype, D.red, res[h], st);
            if (rc) return fail(rc);
        }
        (void)hipFree(D.mem);
    }
    return HPHI_OK;
}

}  // namespace

extern "C" int hphi_cg_refine(const hphi_ham* ham, void* x, int32_t dtype, double e_approx,
                              const hphi_cg_opts* opts, void* work, hphi_cg_result* res, void* stream) {
    if (!ham || !x || !work || !res) return set_error(HPHI_EINVAL, "hphi_cg_refine: null argument");
    if (dtype != HPHI_F64 && dtype != HPHI_C128)
        return set_error(HPHI_EINVAL, "hphi_cg_refine: the vector must be FP64 (F64 or C128)");
    if (ham->is_complex && dtype != HPHI_C128)
        return set_error(HPHI_EDTYPE, "hphi_cg_refine: complex Hamiltonian with real storage");
    const hphi_cg_opts o = opts ? *opts : hphi_cg_opts{1e-6, 2, 1000, 1e-12};
    if (!(o.shift > 0) || !std::isfinite(o.shift) || o.n_inverse < 1 || o.cg_max_iter < 1 || !(o.cg_tol > 0) ||
        !std::isfinite(e_approx))
        return set_error(HPHI_EINVAL, "hphi_cg_refine: bad options");
    hipStream_t st = (hipStream_t)stream;
    const int64_t dim = ham->basis->dim;
    const int64_t n = dim * (dtype == HPHI_C128 ? 2 : 1);   // FP64 scalars per vector
    double* X = static_cast<double*>(x);
    double* R = static_cast<double*>(work);
    double* P = R + n;
    double* Q = P + n;
    double* mem = nullptr;
    if (int rc0 = dev_alloc((void**)&mem, (2048 + 64) * sizeof(double), "hphi_cg_refine: workspace")) return rc0;
    double* partials = mem;
    double* red = mem + 2048;                // [0..3] product sums, [8] a norm
    const double Ep = e_approx + o.shift;
    int rc = HPHI_OK;
    res->cg_iters = 0;
    res->info = HPHI_OK;
    auto host = [&](double* dst, const double* src, int cnt) {
        int r = check_hip(hipMemcpyAsync(dst, src, size_t(cnt) * 8, hipMemcpyDeviceToHost, st), "copy scalar");
        return r ? r : check_hip(hipStreamSynchronize(st), "cg sync");
    };
    // A v = (H - E') v in one product call: a = 1, b = -E'
    auto apply = [&](const double* v, double* u, double* pap) {
        HvLaunch L{};
        L.ham = ham;
        L.v = v;
        L.u = u;
        L.a = 1.0;
        L.b = -Ep;
        L.nvec = 1;
        L.dtype = dtype;
        L.reduce_out = red;
        int r = launch_hv(L, st);
        double q[2];
        if (!r) r = host(q, red, 2);
        if (!r) *pap = q[1] - Ep * q[0];     // <v|Hv> - E' <v|v>
        return r;
    };
    for (int it = 0; it < o.n_inverse && !rc; ++it) {
        // CG for A y = b with b = y_k (|b| = 1) from x_0 = y_k: r = b - A b
        double pap = 0.0, rr = 0.0;
        rc = apply(X, Q, &pap);
        if (!rc) rc = launch_lincomb(R, X, Q, n, 1.0, -1.0, partials, red + 8, st);
        if (!rc) rc = host(&rr, red + 8, 1);
        if (!rc) rc = launch_lincomb(P, R, R, n, 1.0, 0.0, partials, nullptr, st);
        int j = 0;
        bool done = std::sqrt(rr) <= o.cg_tol;
        for (; !rc && !done && j < o.cg_max_iter; ++j) {
            rc = apply(P, Q, &pap);
            if (rc) break;
            if (!std::isfinite(pap) || pap == 0.0) break;    // breakdown: keep the current iterate
            const double alpha = rr / pap;
            rc = launch_lincomb(X, X, P, n, 1.0, alpha, partials, nullptr, st);
            double rn = 0.0;
            if (!rc) rc = launch_lincomb(R, R, Q, n, 1.0, -alpha, partials, red + 8, st);
            if (!rc) rc = host(&rn, red + 8, 1);
            if (rc) break;
            if (std::sqrt(rn) <= o.cg_tol) {
                done = true;
                ++j;
                break;
            }
            rc = launch_lincomb(P, R, P, n, 1.0, rn / rr, partials, nullptr, st);
            rr = rn;
        }
        res->cg_iters += j;
        if (!rc && !done && j >= o.cg_max_iter) res->info = HPHI_INFO_MAXITER;
        // normalize y_{k+1}
        double xx = 0.0;
        if (!rc) rc = launch_lincomb(X, X, X, n, 1.0, 0.0, partials, red + 8, st);
        if (!rc) rc = host(&xx, red + 8, 1);
        if (!rc && !(xx > 0.0 && std::isfinite(xx))) rc = set_error(HPHI_EDEVICE, "hphi_cg_refine: vector vanished");
        if (!rc) rc = launch_lincomb(X, X, X, n, 1.0 / std::sqrt(xx), 0.0, partials, nullptr, st);
    }
    if (!rc) {
        hphi_lanczos_result lr{};
        rc = refine_one(ham, X, dtype, red, lr, st);
        res->e_refined = lr.e0_refined;
        res->variance = lr.variance;
        res->residual = lr.residual;
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(mem);
    return rc;
}
