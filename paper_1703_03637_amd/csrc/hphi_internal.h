// Internal data layout shared by the host code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "hphi.h"

namespace hphi {

// Rows per tile: one wavefront of 64 lanes, one row per lane.
constexpr int kTile = 64;
constexpr int kBlock = 256;              // threads per block (4 wavefronts)
constexpr int kWavesPerBlock = kBlock / 64;
constexpr int kMaxGrid = 4096;           // blocks of the persistent H.v grid
constexpr int kMaxNvec = 16;
constexpr int kNQ = 4;                   // reduced quantities per vector
constexpr int kMaxPassOps = 1024;        // operators per windowed pass (LDS pattern table <= 128 KB)

// One packed operator of the on-the-fly product (Sec. 3.3).
//
// The row pattern p = bit(s, bi) | bit(s, bj) << 1 selects the diagonal
// contribution d[p] and the pulled off-diagonal element
//   <s| H_term |s ^ xmask> = (cr[p] + i ci[p]) * (-1)^popcount(s & smask).
// xmask == 0 marks a diagonal-only operator.  smask is nonzero only for
// fermion operators (the Jordan-Wigner parity of the orbitals outside the
// pattern).  cmask != 0 adds a condition: the element and the diagonal part
// apply only to rows with (s & cmask) == cval (operators on more than two
// orbitals, e.g. the two-body Green's function; single-pass kernel only).
struct DevOp {
    uint64_t xmask;
    uint64_t smask;
    uint32_t bi;
    uint32_t bj;
    int32_t term;
    int32_t has_off;      // any nonzero off-diagonal element
    double d[4];
    double cr[4];
    double ci[4];
    uint64_t cmask;
    uint64_t cval;
};

// Launch schedule of the product kernels (chosen by hphi_hv_tune or by
// defaults).  Zero fields mean "default".
struct Schedule {
    // 0: single-pass product kernel; 1: windowed full-space kernel when it
    // applies; 2: windowed, and every pass after the first gathers from a
    // copy of v stored in that pass's processing order (written by the
    // previous pass), so its window is one contiguous block of memory
    int windowed = 1;
    int window_kb = 2048;   // L2 budget per XCD for a window block
    int max_passes = 3;     // passes of the windowed kernel (1 = natural order)
    int lpr = 0;            // lanes per row (nvec >= 8); 0 = default
    int blocks_per_cu = 0;  // resident blocks per CU; 0 = as many as fit
    int stage_tables = 1;   // single-pass kernel: stage pattern and rank tables in LDS when they fit
                            // (spaces wider than 32 bits: 1 = the two-level low-rank table in LDS,
                            // 2 = only the pattern table, the full low table read through the caches)
    int nt_streams = 0;     // windowed kernel: non-temporal hints on partial sums, output and staged copies
    int sector_blocks = 0;  // sector bases: 1 = block-staged kernel (high-half blocks in LDS), 0 = the
                            // per-tile kernel (measured as fast or faster on every workload here)
};

// Compact kernel-side operator of the windowed product (configurations of
// at most 32 bits), FP64 values.  Element for row
// pattern p = bit(s,bi) | bit(s,bj) << 1: (c[p] + i ci[p]) times the sign
// (-1)^popcount(s & sm); diagonal part d[p].  xm == 0 marks a padding or
// diagonal-only entry.  lq is the flip mask in the pass's processing-index
// bits when the partner row lies in the same 64-row tile (lq < 64), else
// ~0u: a wavefront that holds both rows exchanges them between lanes.
template <typename T>
struct alignas(128) KOp {
    uint32_t xm;
    uint32_t sm;
    uint32_t bi;
    uint32_t bj;
    T c[4];
    T ci[4];
    T d[4];
    uint32_t lq;
    int32_t op;   // index of the operator in the Hamiltonian's list (-1 for padding)
};

// Pass plan of the windowed full-space product.  Each pass applies the
// operators whose flip bits all lie in its window of `wbits` configuration
// bits; the window bits are placed in the low bits of the processing
// index, so every partner row of a pass lies inside an L2-sized block of
// rows that is processed at the same time.
struct PassPlan {
    int row_bytes = 0;
    int window_kb = 0;              // L2 budget the window was sized for
    int max_passes = 0;             // operators of further windows are folded back
    int n_pass = 0;
    int wbits = 0;
    std::vector<int32_t> perm;      // [n_pass][64]: processing-index bit -> configuration bit
    std::vector<int32_t> op_begin;  // [n_pass + 1] ranges into the pass-ordered operator list
    DevOp* d_ops = nullptr;         // operators ordered by pass
    int32_t* d_perm = nullptr;      // device copy of perm
    // compact operators, each pass padded to a multiple of 4 entries
    std::vector<int32_t> kop_begin; // [n_pass + 1]
    KOp<double>* d_kop64 = nullptr;
    // staged variant: the same records with the flip mask of every pass
    // after the first expressed in that pass's processing-index bits
    KOp<double>* d_kopq = nullptr;
    std::vector<int32_t> inv;       // [n_pass][64]: configuration bit -> processing-index bit
    int32_t* d_inv = nullptr;
};

// Dense-block plan (clusters of M configuration bits).  Stage c applies the
// dense partial Hamiltonian of cluster c, H_c[r][t] (row r pulls from
// column t, both M-bit local configurations), to every block of 2^M rows
// that share all configuration bits outside the cluster.
struct CmaPlan {
    int M = 0;
    int n_stage = 0;
    // [n_stage][64]: local bit j < M -> configuration bit of the cluster,
    // then the configuration bits outside it, ascending (block index bits)
    std::vector<int32_t> bits;
    std::vector<int32_t> n_ops;     // [n_stage] operators folded into each cluster
    float* d_hf = nullptr;          // [n_stage][2^M][2^M], row-major
    double* d_hd = nullptr;         // same, FP64
    int32_t* d_bits = nullptr;      // device copy of bits
};

// Device view of a basis, passed by value to kernels.
struct BasisDev {
    int32_t sector;       // 0 = full space (index = bit string)
    int32_t nbits;
    int32_t b_lo;         // width of the low half of the split tables
    int32_t pad;
    uint64_t mask_lo;
    int64_t dim;
    int64_t n_tiles;      // tiles of kTile rows
    int64_t n_high;       // valid high halves (sector only)
    const uint32_t* j_lo;     // [2^b_lo]   rank of a low half within its charge class
    const int64_t* j_hi;      // [2^b_hi]   first index of a high half, -1 if none
    const uint64_t* h_val;    // [n_high]   valid high halves, ascending
    const int64_t* h_row;     // [n_high+1] first row of each high half (prefix)
    const int64_t* h_tile;    // [n_high+1] first tile of each high half (prefix)
    const uint32_t* h_lobase; // [n_high]   offset of its low list in `lows`
    const uint32_t* lows;     // low halves grouped by charge class, ascending
};

}  // namespace hphi

struct hphi_basis {
    hphi_basis_desc desc;
    int nbits = 0;
    int b_lo = 0;
    int b_hi = 0;
    int64_t dim = 0;
    int device = 0;
    hphi::BasisDev dev{};
    void* dmem = nullptr;
    // host copies (validation, host-side rank checks, row -> tile for exports)
    std::vector<uint32_t> j_lo;
    std::vector<int64_t> j_hi;
    std::vector<int64_t> h_row, h_tile;
    int64_t max_block_rows = 0;   // rows of the largest high-half block
    // two-level low-rank tables of the block-staged sector product: the low
    // half l = (a, b), b its low lr_b2 bits, has rank T1[a][class(l)] + T2[b]
    // among the low halves of its class (null if they would not fit in LDS)
    int lr_b2 = 0, lr_ncls = 0, lr_pairs = 0, lr_nsl = 0;
    // their compact 16-bit form for the single-pass kernel (null if it does
    // not apply): rank(l) = T1c[a][T2p[b] >> 10] + (T2p[b] & 1023)
    int lr_n2 = 0;                // classes of a b2-bit part
    uint16_t* d_t1c = nullptr;    // [2^(b_lo - lr_b2)][lr_n2]
    uint16_t* d_t2p = nullptr;    // [2^lr_b2]
    uint32_t* d_t1 = nullptr;     // [2^(b_lo - lr_b2)][lr_ncls]
    uint16_t* d_t2 = nullptr;     // [2^lr_b2]
    size_t lr_bytes = 0;          // bytes of T1 and T2 as the kernel stages them
};

struct hphi_ham {
    ~hphi_ham();
    const hphi_basis* basis = nullptr;
    int n_sites = 0;
    bool is_complex = false;
    bool has_cond = false;        // some operator carries a row condition (cmask)
    std::vector<hphi::DevOp> ops;
    hphi::DevOp* d_ops = nullptr;  // ops padded with inert entries to n_ops_pad
    int n_ops_pad = 0;            // multiple of 4
    double* d_ptab = nullptr;     // [n_ops_pad][4 patterns][Re c, Im c, d, 0]
    int grid = 0;                 // persistent grid of the product kernels
    double* d_partials = nullptr; // [kMaxGrid][kNQ * kMaxNvec]
    double* d_red = nullptr;      // [kNQ * kMaxNvec]
    int32_t* d_flag = nullptr;    // sticky non-finite flag word of the reductions (device, one int)
    std::mutex plan_mu;           // guards the lazily built pass plans, staging buffers and tuned schedules
    void* d_stage[2] = {nullptr, nullptr};   // copies of v in a later pass's order (staged schedule)
    size_t stage_bytes[2] = {0, 0};
    std::vector<hphi::PassPlan*> plans;
    std::vector<hphi::CmaPlan*> cma_plans;
    struct Tuned {
        int nvec, dtype;
        hphi::Schedule s;
    };
    std::vector<Tuned> tuned;
};

namespace hphi {

// error state (thread-local message)
int set_error(int code, const char* fmt, ...);
int check_hip(hipError_t e, const char* what);

// Every device allocation of the library goes through dev_alloc, and the
// large host structures of the builders check alloc_fails first.  Test hook:
// if the environment variable HPHI_FAIL_ALLOC holds a number N > 0, the N-th
// allocation counted from the moment the variable took its current value
// fails as if memory were exhausted (status HPHI_ENOMEM).
bool alloc_fails();
int dev_alloc(void** p, size_t bytes, const char* what);

// Element export through the product kernels (hphi_hv_elements): instead of
// gathering and accumulating, the kernel records for every row in
// [row0, row0 + nrows) and every operator slot o < n_slots the target index
// and the signed element it decoded (col[r][o], cr[r][o], ci[r][o]; rows are
// relative to row0), and the diagonal sum of its pass in diag[r][pass].
// Tiles [t0, t1) of the single-pass kernel cover the rows (the windowed
// kernel visits every tile).
struct ExportArgs {
    int64_t row0 = 0, nrows = 0;
    int64_t t0 = 0, t1 = 0;
    int n_slots = 0;
    int n_pass = 1;
    int64_t* col = nullptr;
    double* cr = nullptr;
    double* ci = nullptr;
    double* diag = nullptr;
};

// launch wrappers (kernels.hip)
struct LzScalars;
struct HvLaunch {
    const hphi_ham* ham;
    const void* v;
    void* u;
    const void* y;           // optional extra input (may alias u), coefficient cy[b]
    const double* cy;        // device [nvec]
    const double* sx;        // device [nvec] or nullptr
    double a, b;
    int nvec;
    int dtype;
    const int* stop;         // device flag: skip all work if nonzero (nullptr = never)
    double* reduce_out;      // device [kNQ * nvec] or nullptr (quantity-major)
    const Schedule* sched;   // nullptr: the tuned or default schedule
    const ExportArgs* ex;    // non-null: element export instead of the product
    bool no_alloc;           // allocate nothing: only plans and staging buffers that exist already
    // one Lanczos recurrence (nvec 1, stop == &lz_sc->stop): the launch that
    // reduces the sums also takes the scalar step after the product
    LzScalars* lz_sc;
    double* lz_alpha;
    const double* lz_evec;
};
Schedule schedule_for(const hphi_ham* ham, int nvec, int dtype);
int launch_hv(const HvLaunch& L, hipStream_t st);
// compact the records of an export into the element lists of hphi_hv_elements
int launch_elements_compact(const hphi_ham* ham, const ExportArgs& ex, int cap, int64_t* cols, double* re,
                            double* im, int32_t* term, int32_t* counts, hipStream_t st);
int launch_rank(const hphi_basis* b, const uint64_t* cfg, int64_t* idx, int64_t n, hipStream_t st);
int launch_unrank(const hphi_basis* b, const int64_t* idx, uint64_t* cfg, int64_t n, hipStream_t st);

// Lanczos / TPQ support kernels
int launch_copy_norm(const void* src, void* dst, int64_t n, int dtype, double* partials, int grid,
                     double* red, int32_t* flag, hipStream_t st);
int launch_lanczos_update(void* y, const void* x, int64_t n, int dtype, const double* c2,
                          void* acc, const double* ecoef, double* partials, int grid, double* red,
                          const int* stop, int32_t* flag, hipStream_t st);
// the same update, with the reduction of |y|^2 and the scalar step after the
// update (beta, stop test, next scales) in one launch
int launch_lanczos_update_lz(void* y, const void* x, int64_t n, int dtype, LzScalars* sc, void* acc,
                             double* partials, int grid, double* red, double* beta, const double* alpha,
                             int32_t* flag, hipStream_t st);
int launch_fill_zero(void* p, int64_t bytes, hipStream_t st);
// w = a x + b y (FP64, n scalars; w may alias x or y); |w|^2 into *norm2 if non-null
int launch_lincomb(double* w, const double* x, const double* y, int64_t n, double a, double b, double* partials,
                   double* norm2, hipStream_t st);
int launch_expect(const double* red, double* out, int nvec, hipStream_t st);
int launch_tpq_obs(const double* red, double* obs, int nvec, double n_sites, double l, int k,
                   hipStream_t st);
// device state of a multi-step TPQ run (hphi_tpq_run): the next step's index
// k, the step counter j, and the normalizing scales of the last two states
struct TpqRunState {
    int32_t k;
    int32_t j;
    int32_t pad[2];
    double scale[2][kMaxNvec];
};
int launch_tpq_run_init(TpqRunState* s, int k0, hipStream_t st);
// The device state of the allocation-free TPQ run: a file-scope static
// device array of one TpqRunState, its address on the current device
// (resolved once per device).  Returns an error code or HPHI_OK.
int tpq_static_state(TpqRunState** out);
int launch_tpq_obs_run(const double* red, TpqRunState* s, double* obs_log, int nvec, double n_sites, double l,
                       hipStream_t st);

// per-iteration scalar bookkeeping of the Lanczos recurrence (device, one thread)
struct LzScalars {
    double s_cur;     // scale of the stored v_k (1/beta_k folded into loads)
    double cy;        // coefficient of v_{k-1} in pass 1: -beta_k * s_prev
    double c2;        // coefficient of v_k in pass 2: -alpha_k * s_cur
    double ecoef;     // eigenvector coefficient e~_k * s_cur (second pass)
    double beta_k;    // beta_k of the current step
    double tol;
    int32_t k;        // current step
    int32_t n_max;    // min(n_iter, dim)
    int32_t stop;     // 1 once the recurrence has ended
    int32_t n_done;
    int32_t breakdown;
    int32_t pad;
};
int launch_lz_init(LzScalars* sc, const double* red, double tol, int n_max, hipStream_t st);

// ---- several problems per launch (batched Lanczos over uneven sectors)
struct RedDesc {             // reduce partials[n_parts][nq] into out[nq]
    const double* partials;
    int n_parts;
    int pad;
    double* out;
    const int* stop;
    int32_t* flag;           // non-finite flag word of the problem (or nullptr)
};
struct UpdDesc {             // y += c2 x, |y|^2 partials, acc += ec x
    void* y;
    const void* x;
    int64_t n;               // scalars
    const double* c2;
    double* acc;
    const double* ec;
    double* partials;        // set by the plan
    const int* stop;
    int32_t* flag;           // non-finite flag word of the problem's Hamiltonian
};
// Launch plan of one batched product: per-problem arguments, block ranges
// (multiples of 8) and reductions, uploaded once and replayed by graphs.
struct MultiPlan {
    int n = 0;
    int grid = 0;
    size_t lds = 0;
    bool gtab = false;
    int dtype = 0;
    bool cc = false, sector = false, w64 = false;
    void* mem = nullptr;     // device: args, begin, partials, reductions
    const void* d_args = nullptr;
    const int* d_begin = nullptr;
    const RedDesc* d_red = nullptr;
};
// Problems must agree on dtype, coefficient type, sector/full space and
// configuration width (else HPHI_EINVAL); nvec must be 1.
int hv_multi_prepare(const HvLaunch* Ls, int n, MultiPlan* out);
// the scalars of several recurrences (alpha/beta/evec: `stride` per problem);
// with it, the launches that reduce the sums also take the scalar steps
struct LzMulti {
    LzScalars* sc;
    double* alpha;
    double* beta;
    const double* evec;
    int stride;
};
int hv_multi_launch(const MultiPlan& P, const LzMulti* lz, hipStream_t st);
struct UpdPlan {
    int n = 0;
    int grid = 0;
    bool fp64 = true;
    void* mem = nullptr;
    const UpdDesc* d_desc = nullptr;
    const int* d_begin = nullptr;
    const RedDesc* d_red = nullptr;
};
// red_out[p]: device [1] receiving |y_p|^2
int upd_multi_prepare(const UpdDesc* descs, double* const* red_out, int n, int dtype, UpdPlan* out);
int upd_multi_launch(const UpdPlan& P, const LzMulti* lz, hipStream_t st);

// dense-block plan for clusters of M bits (cma.cpp); an error code if the
// space or the operators do not fit
int get_cma_plan(const hphi_ham* ham, int M, const CmaPlan** out);
// one dense-block product (kernels.hip): stages into u, then the epilogue
int launch_hv_cma(const HvLaunch& L, const CmaPlan* P, hipStream_t st);

// pass plan of the windowed product (plan.cpp); nullptr if not applicable
// may_build = false: only a plan built earlier (no allocation)
const PassPlan* get_plan(const hphi_ham* ham, int row_bytes, int window_kb, int max_passes, bool may_build = true);
// staging buffers of at least `bytes` each (grown on demand, kept with the
// Hamiltonian); returns nonzero if they cannot be had
int get_stage_buffers(const hphi_ham* ham, size_t bytes, int count, void** out);

// host tridiagonal eigensolver (tridiag.cpp)
double tridiag_lowest(const double* alpha, const double* beta, int n, double* evec);

size_t dtype_size(int dtype);
bool dtype_complex(int dtype);

}  // namespace hphi
