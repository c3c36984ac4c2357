/*
 * hphi.h -- C ABI of the MI355X matrix-free H.v / Lanczos / TPQ library.
 *
 * Implements the hot path of Kawamura et al., "Quantum Lattice Model
 * Solver HPhi" (arXiv:1703.03637) on one AMD Instinct MI355X (gfx950):
 *   - the bit-string Hilbert space and its canonical (fixed Sz or fixed
 *     particle number) restriction with two-dimensional (split-table)
 *     reverse lookup                                     (Sec. 3.1)
 *   - the on-the-fly Hamiltonian-vector product: diagonal terms, XOR
 *     exchange / hopping after a bit test, fermion sign from the parity
 *     of a masked bit count                              (Sec. 3.3)
 *   - the Lanczos ground-state iteration with the second pass for the
 *     eigenvector and the energy/variance check (Sec. 3.4, App. A.3)
 *   - the microcanonical TPQ step                         (Sec. 3.5)
 *   - a dense-block variant of the product after the continuous-memory-
 *     access method, on the matrix cores                 (Sec. 4.3)
 *
 * Conventions (bind every entry point):
 *   * Site i of a spin-1/2 system is bit i (bit 0 least significant);
 *     bit value 1 = up.  A fermion system of N sites uses 2N bits,
 *     orbital k = 2*site + sigma (sigma 0 = up, 1 = down), i.e. the
 *     4-ary site digit of Sec. 3.1 split with up in the low bit.
 *   * Fermion signs use the Jordan-Wigner order ascending in k; a hop
 *     c+_a c_b picks up (-1)^(number of occupied orbitals strictly
 *     between a and b).
 *   * A full-space index is the bit string itself; a sector index is
 *     the rank of the bit string among the sector's bit strings in
 *     ascending order (the order of the Sec. 3.3 example).
 *   * Vectors are device memory in one of four storage types (hphi_dtype).
 *     nvec > 1 vectors are interleaved: element b of row r is at
 *     v[r * nvec + b].  Complex vectors store (re, im) pairs.
 *   * Every call returns an int status (HPHI_OK = 0, negative = error).
 *     Arguments are validated on the host before anything is launched;
 *     on error nothing is written and hphi_last_error() (thread-local)
 *     holds a message.  No exception crosses the ABI.
 *   * Unless stated otherwise calls are asynchronous on the HIP stream
 *     passed as `stream` (a hipStream_t; NULL = the legacy default stream).
 *   * Handles (hphi_basis, hphi_ham) are library-owned and immutable
 *     after build.  A hphi_ham holds a small reduction workspace:
 *     calls that share one hphi_ham must not overlap in time on
 *     different streams.
 */
#ifndef HPHI_H
#define HPHI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    HPHI_OK = 0,
    HPHI_EINVAL = -1,       /* bad argument (checked before any launch)            */
    HPHI_ENOMEM = -2,       /* device or host allocation failed                   */
    HPHI_EDEVICE = -3,      /* HIP runtime error (message in hphi_last_error)      */
    HPHI_ESECTOR = -4,      /* a term maps a sector state outside the sector       */
    HPHI_EDTYPE = -5,       /* complex matrix elements with a real storage type    */
    HPHI_ENONFINITE = -6,   /* a reduction of the run was NaN or Inf (hphi_lanczos) */
    HPHI_INFO_BREAKDOWN = 1, /* Lanczos stopped early: beta below tolerance or dim */
    HPHI_INFO_MAXITER = 2    /* a CG solve reached its iteration limit             */
};

enum { HPHI_SPIN_HALF = 0, HPHI_FERMION = 1 };

enum {
    HPHI_SECTOR_NONE = 0,     /* full 2^nbits space (grand canonical)            */
    HPHI_SECTOR_SZ = 1,       /* spins: fixed 2*Sz = (#up - #down)              */
    HPHI_SECTOR_NUP_NDN = 2,  /* fermions: fixed number of up and of down        */
    HPHI_SECTOR_NTOT = 3      /* fermions: fixed total particle number           */
};

typedef enum {
    HPHI_F64 = 0,   /* real double                                               */
    HPHI_C128 = 1,  /* complex double (re, im)                                   */
    HPHI_F32 = 2,   /* real float storage; products, sums, reductions in FP64    */
    HPHI_C64 = 3    /* complex float storage (re, im), as HPHI_F32               */
} hphi_dtype;

/* ------------------------------------------------------------------ basis */

/* Hilbert-space descriptor (Sec. 3.1).
 *   particle   HPHI_SPIN_HALF (nbits = n_sites) or HPHI_FERMION (nbits = 2*n_sites)
 *   sector     HPHI_SECTOR_*; two_sz for SZ (parity of n_sites), n_up/n_dn for
 *              NUP_NDN, n_tot for NTOT
 *   split_bits width of the low half of the split rank tables (0 = nbits/2,
 *              rounded down to even for fermions so a site is never split).
 * Limits: full space nbits <= 40; sector spaces nbits <= 62 with
 * 2^split_bits and 2^(nbits - split_bits) table entries each <= 2^26. */
typedef struct {
    int32_t particle;
    int32_t n_sites;
    int32_t sector;
    int32_t two_sz;
    int32_t n_up;
    int32_t n_dn;
    int32_t n_tot;
    int32_t split_bits;
} hphi_basis_desc;

typedef struct hphi_basis hphi_basis;

/* Build the space and, for a sector, the split rank tables of the
 * two-dimensional search (Sec. 3.1): for a bit string s = (h << b_lo) | l,
 *   index(s) = J_hi[h] + J_lo[l],
 * J_lo[l] = rank of l among low halves with the same charge, J_hi[h] = index
 * of the first sector state with high half h.  Tables are enumerated on the
 * host with the same-popcount successor and copied to the current device.
 * Synchronous.  *out receives a handle to free with hphi_basis_free. */
int hphi_basis_build(const hphi_basis_desc* desc, hphi_basis** out);

/* Dimension of the space (host value). */
int hphi_basis_dim(const hphi_basis* basis, int64_t* dim);

/* Device arrays, n entries each.  rank: idx[k] = index of cfg[k] or -1 if
 * cfg[k] is not in the space.  unrank: cfg[k] = configuration of idx[k];
 * indices outside [0, dim) give cfg = ~0. */
int hphi_basis_rank(const hphi_basis* basis, const uint64_t* cfg, int64_t* idx, int64_t n,
                    void* stream);
int hphi_basis_unrank(const hphi_basis* basis, const int64_t* idx, uint64_t* cfg, int64_t n,
                      void* stream);

void hphi_basis_free(hphi_basis* basis);

/* ------------------------------------------------------------ Hamiltonian */

enum {
    /* spins (Sec. 2.3 "Spin"): site indices i != j < n_sites                    */
    HPHI_TERM_SPIN_BOND = 0,   /* sum_ab c[3a+b] S_i^a S_j^b, a,b in (x,y,z)     */
    HPHI_TERM_SPIN_FIELD = 1,  /* sum_a c[a] S_i^a                                */
    /* fermions (Sec. 2.3 "Fermion Hubbard"): orbital indices < 2*n_sites        */
    HPHI_TERM_HOP = 2,         /* t c+_i c_j + conj(t) c+_j c_i, t = c[0] + i c[1], i != j */
    HPHI_TERM_DENS = 3,        /* c[0] n_i n_j, i != j                             */
    HPHI_TERM_NUM = 4,         /* c[0] n_i                                         */
    HPHI_TERM_HUBBARD_U = 5,   /* c[0] n_{i,up} n_{i,down}, i a site index         */
    /* observables: the two-body Green's function of Sec. 2.2 (output from
     * eigenvectors and TPQ states) as a Hermitian operator,
     *   t c+_i c_j c+_k c_l + conj(t) c+_l c_k c+_j c_i,  t = c[0] + i c[1],
     *   k = (int)c[2], l = (int)c[3]  (orbitals; repeats allowed),
     * so that <O> = 2 Re(t <c+_i c_j c+_k c_l>): t = 1 gives 2 Re G, t = i gives
     * -2 Im G.  Packed for the single-pass product kernel only (use with
     * hphi_expect; the windowed, block-staged and dense-block kernels decline). */
    HPHI_TERM_GREEN2 = 6
};

/* One term of the Hamiltonian.  Unused fields are ignored.  Each term is
 * Hermitian on its own; the Hamiltonian is the sum of the list as given
 * (an undirected bond is listed once). */
typedef struct {
    int32_t kind;
    int32_t i;
    int32_t j;
    int32_t reserved;
    double c[9];
} hphi_term;

typedef struct hphi_ham hphi_ham;

/* Validate and pack terms for the on-the-fly product (Sec. 3.3): each term
 * becomes per-bit-pattern diagonal values and, per flip mask, the pulled
 * matrix elements <s|H|s ^ mask>.  Returns HPHI_ESECTOR if a term has a
 * nonzero element that leaves the basis' sector (e.g. a transverse field or
 * a Kitaev coupling on an Sz sector), HPHI_EINVAL for bad indices.
 * The basis must outlive the ham.  Synchronous. */
int hphi_ham_build(const hphi_basis* basis, const hphi_term* terms, int64_t n_terms,
                   hphi_ham** out);

/* 1 if any matrix element is complex (then only C128/C64 storage is allowed). */
int hphi_ham_is_complex(const hphi_ham* ham, int32_t* is_complex);

/* Non-finite flag word of a Hamiltonian (fault detection for the fused
 * reductions of Sec. 3.4 and 3.5).  Every reduction the library computes for
 * calls on this ham -- the four sums of hphi_hv, hphi_tpq_step and
 * hphi_expect, and the norms of the Lanczos recurrence -- ORs a bit into a
 * sticky device word when its result is NaN or Inf (a non-finite input
 * entry, or overflow):
 *   HPHI_NONFINITE_PRODUCT  a sum of a product call (<x|x>, <x|Hx>, |Hx|^2, |u|^2)
 *   HPHI_NONFINITE_NORM     a norm of a Lanczos vector (start vector or update)
 * Products without reductions (opts->reduce == NULL) set nothing.  Writes the
 * word to *flags (host) and, if clear != 0, resets it to zero.  Synchronizes
 * `stream`.  hphi_lanczos clears the words of its hams when it starts and
 * returns HPHI_ENONFINITE if one is set when it ends. */
enum { HPHI_NONFINITE_PRODUCT = 1, HPHI_NONFINITE_NORM = 2 };
int hphi_ham_nonfinite(const hphi_ham* ham, int32_t* flags, int32_t clear, void* stream);

void hphi_ham_free(hphi_ham* ham);

/* ------------------------------------------------------------------ H . v */

/* Options of hphi_hv.  With x_b = s_b * v_b (s_b = in_scale[b], or 1):
 *     u_b = a * (H x_b) + b * x_b
 * and, if reduce != NULL, FP64 sums written to reduce[q * nvec + b]:
 *     q = 0: <x_b|x_b>   q = 1: Re<x_b|H x_b>   q = 2: <H x_b|H x_b>   q = 3: <u_b|u_b>
 * reduced in a fixed order (bitwise reproducible for a fixed launch shape).
 * u may be NULL (reductions only). */
typedef struct {
    double a;
    double b;
    const double* in_scale; /* device [nvec] or NULL */
    double* reduce;         /* device [4 * nvec] or NULL */
} hphi_hv_opts;

/* Matrix-free product over all rows of the space.  v, u: device, dim*nvec
 * elements of `dtype`, interleaved; u must not alias v.  nvec in
 * {1, 2, 4, 8, 16}; configurations wider than 32 bits allow nvec <= 4
 * (HPHI_EINVAL otherwise).  FP32/C64 are storage formats only: every product,
 * row sum and reduction is FP64 with FP64 coefficients, and results are
 * rounded once when stored (a multi-pass schedule also rounds the partial
 * sums it passes between passes).  opts NULL = {1, 0, NULL, NULL}.
 * Workspace lives with the ham: reduction partials, and for a staged
 * multi-pass schedule one or two device buffers of dim*nvec elements
 * (copies of v in a later pass's row order), allocated on first use and
 * kept until hphi_ham_free.  Calls that share a ham must therefore not run
 * concurrently on different streams.
 * Returns HPHI_EDTYPE for a complex Hamiltonian with a real dtype. */
int hphi_hv(const hphi_ham* ham, const void* v, void* u, int64_t nvec, int32_t dtype,
            const hphi_hv_opts* opts, void* stream);

/* Autotuner of the product's launch schedule.  Times candidate schedules of
 * hphi_hv on the caller's buffers (v: input, u: scratch output of the same
 * size, overwritten) -- for full-space bases of 6..32 bits the windowed
 * multi-pass traversal with 1, 2 or 4 MB L2 windows and up to 3 passes,
 * gathering from v itself or from staged copies of v in each pass's row
 * order, or a single natural-order pass; lanes per row (nvec >= 2); resident blocks
 * per CU, table placement -- and pins the fastest for this (ham, nvec, dtype) (the
 * candidates within 5% of the fastest are timed again, best of 3 x 3 calls): later
 * hphi_hv / hphi_tpq_step / hphi_lanczos calls with that nvec and dtype use
 * it.  Results are bitwise reproducible for a fixed schedule; a different
 * schedule may change the last bits of the reductions.  sched_out (host,
 * may be NULL) receives 9 ints: windowed (0: single pass, 1: windowed,
 * 2: windowed with staged copies), window_kb, max_passes,
 * lanes_per_row, blocks_per_cu, stage_tables (single-pass kernel: 1 =
 * pattern and rank tables staged in LDS when they fit -- on sectors wider
 * than 32 bits the two-level low-rank table --, 2 = only the pattern table
 * in LDS, 0 = read from global memory), nt_streams (windowed kernel, nvec >= 8: 1 = partial
 * sums, output and staged copies move with non-temporal hints so they do
 * not evict the gather window from L2), sector_blocks (sector bases: 1 = the
 * block-staged kernel that keeps each high-half block of rows in LDS, 0 =
 * the per-tile kernel), microseconds per product call (9 ints in all).  If the
 * environment variable HPHI_TUNE_CACHE names a file, the choice is
 * appended there and reused by later processes for the same device,
 * space and operators.  Synchronizes `stream`. */
int hphi_hv_tune(const hphi_ham* ham, const void* v, void* u, int64_t nvec, int32_t dtype,
                 int32_t* sched_out, void* stream);

/* Dense-block variant of the product, after the paper's continuous-memory-
 * access method (Sec. 4.3): any sum of terms acting on M chosen sites is a
 * dense 2^M x 2^M matrix acting on the 2^M rows that share all other bits.
 * The terms are covered by clusters of at most `cluster_bits` = M sites
 * (greedily, deterministic; every term must fit in one cluster); for each
 * cluster the library builds its dense partial Hamiltonian once, and one
 * pass multiplies every 2^M-row block by it with matrix-core (MFMA)
 * instructions, gathering the block's rows through the cluster's bit
 * positions instead of permuting the vector, and accumulating into u.  The
 * last cluster's pass also applies a, b, in_scale and the reductions exactly
 * as hphi_hv does.  The result equals hphi_hv's up to rounding: the dense blocks sum in
 * the storage precision (FP32 for F32/C64 storage, FP64 for F64/C128), and
 * partial sums pass between clusters in u.
 * Applies to spin-1/2 full spaces of 6..32 bits with real matrix elements;
 * cluster_bits in 4..7 and at most the number of sites (6 for F64/C128).
 * v, u: device, dim*nvec elements, interleaved; u must not alias v and must
 * be non-NULL.  nvec in {1, 2, 4, 8, 16}.  opts as for hphi_hv (NULL =
 * {1, 0, NULL, NULL}).  The dense matrices and the cluster plan are cached
 * with the ham (2^(2M) values per cluster) until hphi_ham_free; calls that
 * share a ham must not run concurrently on different streams.
 * Returns HPHI_EINVAL if the space or the terms do not fit these limits,
 * HPHI_EDTYPE for a complex Hamiltonian. */
int hphi_hv_cma(const hphi_ham* ham, const void* v, void* u, int64_t nvec, int32_t dtype,
                int32_t cluster_bits, const hphi_hv_opts* opts, void* stream);

/* The cluster cover hphi_hv_cma uses for `cluster_bits` (building it if
 * needed): *n_clusters receives the number of clusters (one pass each) and,
 * if sites != NULL (host, n_clusters * cluster_bits entries, caller-owned),
 * the sites of cluster c in ascending order at sites[c * cluster_bits ...].
 * Call once with sites = NULL to learn the count.  Same limits and errors as
 * hphi_hv_cma. */
int hphi_hv_cma_plan(const hphi_ham* ham, int32_t cluster_bits, int32_t* n_clusters, int32_t* sites);

/* Element export through the product kernels themselves (parity checks of
 * the Sec. 3.3 decode: bit test, XOR target, parity sign, split-table rank).
 * The product that hphi_hv runs for `nvec` vectors of storage type `dtype`
 * (C128 or C64: the export follows the complex lane layouts) -- the same
 * kernel, schedule and operator records -- runs in an export mode: in place
 * of each gather it records the target index it decoded (for partners that
 * the windowed kernel takes from its LDS row tile or from another lane, the
 * partner's configuration as it arrives through that on-chip path) and the
 * signed element.  For rows row0 .. row0+nrows-1 (at most 2^22 per call)
 * it then writes up to `cap` elements per row:
 *   the diagonal (col = row, term_id = -1, value = sum of diagonal parts) if nonzero,
 *   then one entry per packed off-diagonal operator whose element is nonzero,
 *   in the order of the operators (col = target index, term_id = index into
 *   the term list, value = signed matrix element <row|H|col>).
 * cols/re/im/term_id: device [nrows * cap]; counts: device [nrows], the full
 * element count of each row (may exceed cap; extra elements are dropped).
 * Allocates a record buffer of nrows * (24 * n_operators + 64) bytes for the
 * call and synchronizes `stream`. */
int hphi_hv_elements(const hphi_ham* ham, int64_t row0, int64_t nrows, int32_t cap, int64_t nvec, int32_t dtype,
                     int64_t* cols, double* re, double* im, int32_t* term_id, int32_t* counts, void* stream);

/* ---------------------------------------------------------------- Lanczos */

typedef struct {
    int32_t n_iter;        /* number of Lanczos steps (size of T_n), >= 1        */
    int32_t dtype;         /* storage type of the Lanczos vectors                */
    int32_t refine;        /* 1: second pass for the eigenvector + FP64 check    */
    int32_t use_graph;     /* 1: replay the iteration from a captured HIP graph  */
    double breakdown_tol;  /* relative beta tolerance, <= 0 selects 1e-13        */
} hphi_lanczos_opts;

typedef struct {
    double* alpha;         /* host, caller-owned [n_iter]: alpha_k               */
    double* beta;          /* host, caller-owned [n_iter]: beta[k] = beta_{k+1}  */
    int32_t n_done;        /* steps taken (size of T)                            */
    int32_t info;          /* HPHI_OK or HPHI_INFO_BREAKDOWN                      */
    double e0_ritz;        /* lowest eigenvalue of T_n                           */
    double e0_refined;     /* <x|H|x>/<x|x> of the eigenvector, FP64 (refine)    */
    double variance;       /* <H^2> - <H>^2 of x (refine)                        */
    double residual;       /* |Hx - E x| / |x| (refine)                          */
} hphi_lanczos_result;

/* Lanczos ground state (Sec. 3.4): v_0 = x_0/|x_0|, beta_0 = 0,
 *   alpha_k = (H v_k, v_k), w = H v_k - beta_k v_{k-1} - alpha_k v_k,
 *   beta_{k+1} = |w|, v_{k+1} = w / beta_{k+1},
 * two stored vectors, no reorthogonalization; the lowest Ritz value of T_n
 * comes from a host FP64 tridiagonal eigensolver.  The recurrence stops
 * early (info = HPHI_INFO_BREAKDOWN) when k+1 reaches the dimension or
 * beta_{k+1} <= tol * max(|alpha_k|, beta_k, 1).  With refine, the
 * recurrence is replayed bit-for-bit to accumulate x = sum_k e~_k v_k in
 * FP64 (App. A.3) and E, variance and residual are measured with an FP64
 * product.
 * Several problems (n_hams > 1, up to 64) that share the coefficient type,
 * the space kind (sector or full) and the configuration width run as one
 * batched recurrence: each step is one persistent product launch, one
 * update launch and one scalar launch for all of them (uneven sizes split
 * the grid in proportion to their tiles), each odd/even step pair replayed
 * from one captured graph; other combinations run one problem at a time.
 *   hams[n_hams]  one Hamiltonian per independent problem (e.g. Sz sectors)
 *   v0[h]         device start vector, storage dtype, dim_h entries
 *   work[h]       device scratch of 2 * dim_h storage elements
 *   x_out[h]      device FP64 (C128 for complex dtypes) [dim_h], required if refine.
 *                 It may be the buffer of v0[h] when that buffer holds dim_h
 *                 FP64 (C128) elements: the second pass copies v0 before x is
 *                 accumulated, so v0 is then overwritten by the eigenvector
 *                 (this saves one vector of memory on the largest spaces)
 *   res[h]        results; alpha/beta arrays of n_iter entries each
 * A non-finite norm or sum anywhere in the recurrence (NaN or Inf in v0, or
 * overflow) returns HPHI_ENONFINITE after the run (see hphi_ham_nonfinite).
 * Synchronizes `stream` before returning. */
int hphi_lanczos(const hphi_ham* const* hams, int32_t n_hams, const hphi_lanczos_opts* opts,
                 const void* const* v0, void* const* work, void* const* x_out,
                 hphi_lanczos_result* res, void* stream);

/* Inverse-iteration refinement of an eigenvector (Sec. 3.4, inverse
 * iteration method; App. A.3): starting from y_0 = x (the Lanczos
 * eigenvector), n_inverse times solve (H - E') y_{k+1} = y_k by conjugate
 * gradients, starting each solve from y_k, and normalize; E' = e_approx +
 * shift, the small positive shift that stabilizes CG.  All FP64.
 *   x      device, dim elements of dtype F64 or C128 (the x_out of
 *          hphi_lanczos); in: approximate eigenvector, out: refined, |x| = 1
 *   work   device scratch of 3 * dim elements of dtype (r, p, q: with x the
 *          four vectors of the method)
 *   res    host: E = <x|H|x>, variance, residual |Hx - Ex| of the result, the
 *          CG iterations taken, info = HPHI_OK or HPHI_INFO_MAXITER
 * opts NULL = {1e-6, 2, 1000, 1e-12}.  Synchronizes `stream` (each CG step
 * reads its two FP64 scalars on the host). */
typedef struct {
    double shift;         /* added to e_approx (> 0)                            */
    int32_t n_inverse;    /* inverse-iteration steps (>= 1)                     */
    int32_t cg_max_iter;  /* per solve                                          */
    double cg_tol;        /* stop when |r| <= cg_tol |y_k| (|y_k| = 1)          */
} hphi_cg_opts;

typedef struct {
    double e_refined;
    double variance;
    double residual;
    int32_t cg_iters;
    int32_t info;
} hphi_cg_result;

int hphi_cg_refine(const hphi_ham* ham, void* x, int32_t dtype, double e_approx, const hphi_cg_opts* opts,
                   void* work, hphi_cg_result* res, void* stream);

/* ------------------------------------------------------------ observables */

/* Expectation values of a Hermitian observable O in nvec states (Sec. 3.5:
 * observables of TPQ states and eigenvectors, e.g. the doublon density of
 * Sec. 5.1).  O is given as a term list built into its own hphi_ham on the
 * same basis: the Hubbard-U kind with U = 1 counts doublons, a HOP term
 * t c+_a c_b + conj(t) c+_b c_a measures 2 Re <c+_a c_b> at t = 1 and
 * -2 Im <c+_a c_b> at t = i (together the one-body Green's function), DENS
 * measures n_a n_b, a spin bond S^a_i S^b_j (the density and spin two-body
 * correlations).  psi: device, dim*nvec
 * elements of dtype, interleaved as for hphi_hv.  out: device [2 * nvec]
 * (FP64): out[b] = Re<psi_b|O|psi_b> / <psi_b|psi_b>, out[nvec + b] =
 * <psi_b|psi_b>.  Uses the product kernels in reduce-only mode (no output
 * vector) and the reduction workspace of `obs`.  Asynchronous on stream. */
int hphi_expect(const hphi_ham* obs, const void* psi, int64_t nvec, int32_t dtype, double* out,
                void* stream);

/* -------------------------------------------------------------------- TPQ */

/* One microcanonical TPQ step (Sec. 3.5) for nvec independent samples:
 * with psi = s * psi_in (s = in_scale[b] or 1),
 *     phi = (l - H / N_s) psi,   psi_out = phi (unnormalized)
 * and obs (device, [4 * nvec], layout obs[q * nvec + b]):
 *     q = 0: u_{k-1}   = <psi|H|psi> / (<psi|psi> N_s)   energy per site of the input
 *     q = 1: <H^2>/N_s^2 of the input state
 *     q = 2: beta_{k-1} = (2 (k-1) / N_s) / (l - u_{k-1})
 *     q = 3: 1 / |phi|, the scale that normalizes psi_out (pass &obs[3*nvec]
 *            as in_scale of the next step)
 * k >= 1 is the index of the produced state psi_k.  N_s = n_sites.
 * psi_out must not alias psi_in. */
int hphi_tpq_step(const hphi_ham* ham, const void* psi_in, void* psi_out, int64_t nvec,
                  int32_t dtype, double l, int32_t k, const double* in_scale, double* obs,
                  void* stream);

/* n_steps consecutive mTPQ steps (Sec. 3.5) of nvec samples, the states
 * alternating between two caller-owned device buffers: step j = 0 .. n_steps-1
 * is hphi_tpq_step with k = k0 + j reading psi_a (j even) or psi_b (j odd) and
 * writing the other, with input scale in_scale (device [nvec] or NULL = 1)
 * for j = 0 and the previous step's 1/|phi| after that.  The step index and
 * the scales stay on the device, so with use_graph the steps after the first
 * are replayed in pairs from one captured HIP graph (no host work per step).
 *   obs_log  device FP64 [n_steps][4][nvec]: entry [j][q][b] is obs[q*nvec+b]
 *            of step j as hphi_tpq_step defines it (u, <H^2>/N_s^2, beta of
 *            the step's input state; 1/|phi| of its output)
 * The state psi_{k0+n_steps-1} ends in psi_a if n_steps is even, else in
 * psi_b, unnormalized: its normalizing scale is obs_log[n_steps-1][3][.].
 * k0 >= 1; n_steps = 0 does nothing.  Allocates a small device state for
 * the run and synchronizes `stream` before returning. */
int hphi_tpq_run(const hphi_ham* ham, void* psi_a, void* psi_b, int64_t nvec, int32_t dtype, double l,
                 int32_t k0, int32_t n_steps, const double* in_scale, double* obs_log, int32_t use_graph,
                 void* stream);

/* hphi_tpq_run for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, steps, obs_log layout and final-state placement as
 * hphi_tpq_run, with these differences:
 *   - allocates nothing: the run's device state (step index, step counter
 *     and the scales of the last two states, 272 bytes) lives in a static
 *     device array of the library, one per GPU, held until the process ends;
 *     the product uses only pass plans and staging buffers that earlier calls
 *     on this ham built (else it takes the single-pass kernel, which needs
 *     none), and the ham's own reduction workspace;
 *   - launches every step eagerly on `stream` and returns without
 *     synchronizing, so the whole run may itself be captured into a graph;
 *   - maximum: nvec <= 16 (the static state holds 16 scales); larger values
 *     return HPHI_EINVAL.
 * The static state is shared by every call on a GPU and keeps the last
 * call's contents (each call resets its counters first): calls that overlap
 * in time on one GPU race, even on different hams. */
int hphi_tpq_run_noalloc(const hphi_ham* ham, void* psi_a, void* psi_b, int64_t nvec, int32_t dtype, double l,
                         int32_t k0, int32_t n_steps, const double* in_scale, double* obs_log, void* stream);

/* ------------------------------------------------------------------ misc */

/* Message of the last error on this thread ("" if none). */
const char* hphi_last_error(void);

/* Library version string. */
const char* hphi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HPHI_H */
