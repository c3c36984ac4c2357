// gfx950 kernels of the matrix-free product and its reductions.
//
// Product (Sec. 3.3): each lane owns one row s of the output ("pull").  For
// every packed operator it reads the two bits that select the pattern p,
// adds the diagonal part d[p], and, if the pulled element <s|H|s^mask> is
// nonzero, forms the target t = s ^ mask, applies the fermion sign
// (-1)^popcount(s & smask), ranks t (identity on the full space, split-table
// lookup J_hi[t >> b_lo] + J_lo[t & mask_lo] on a sector, Sec. 3.1) and
// gathers the nvec interleaved values of row t.  One writer per output
// element, no atomics: results are reproducible bit for bit.
//
// Work split: a tile is 64 consecutive rows (one wavefront).  Tiles are
// dealt to wavefronts XCD by XCD: blocks i, i+8, ... run on the same XCD
// (round-robin dispatch), so each XCD sweeps its own contiguous eighth of
// the row space and neighbouring rows share that XCD's L2.
//
// Reductions: per row FP64 products, a per-tile wavefront reduce-scatter
// (each lane ends up owning one vector's sum), a fixed-order block sum and
// a fixed-order second-stage kernel.
#include <hip/hip_runtime.h>

#include "hphi_internal.h"

namespace hphi {
namespace {

template <int B>
struct Log2 {
    static constexpr int value = B == 1 ? 0 : B == 2 ? 1 : B == 4 ? 2 : B == 8 ? 3 : 4;
};

template <typename T>
__device__ __forceinline__ T sel4(int p, T c0, T c1, T c2, T c3) {
    const T lo = (p & 1) ? c1 : c0;
    const T hi = (p & 1) ? c3 : c2;
    return (p & 2) ? hi : lo;
}

__device__ __forceinline__ int wave_uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// largest k in [0, n) with h_tile[k] <= tile (h_tile ascending)
__device__ __forceinline__ int64_t find_high(const int64_t* __restrict__ h_tile, int64_t n, int64_t tile) {
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (h_tile[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// largest k in [0, n) with h_row[k] <= row
__device__ __forceinline__ int64_t find_high_row(const int64_t* __restrict__ h_row, int64_t n, int64_t row) {
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (h_row[mid] <= row) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <bool SECTOR>
__device__ __forceinline__ int64_t rank_of(const BasisDev& b, uint64_t t) {
    if constexpr (!SECTOR) {
        return int64_t(t);
    } else {
        return b.j_hi[t >> b.b_lo] + int64_t(b.j_lo[t & b.mask_lo]);
    }
}

// unrank one row (per-lane binary search; used outside the product kernel)
__device__ __forceinline__ uint64_t unrank_row(const BasisDev& b, int64_t row) {
    if (b.sector == 0) return uint64_t(row);
    const int64_t k = find_high_row(b.h_row, b.n_high, row);
    return (b.h_val[k] << b.b_lo) | uint64_t(b.lows[b.h_lobase[k] + (row - b.h_row[k])]);
}

// ---- row loads/stores of NE scalars (vectorised by size)
template <typename S, int NE>
__device__ __forceinline__ void load_row(const S* __restrict__ base, int64_t idx, S (&out)[NE]) {
    constexpr int BYTES = NE * int(sizeof(S));
    const char* p = reinterpret_cast<const char*>(base) + idx * BYTES;
    if constexpr (BYTES % 16 == 0) {
#pragma unroll
        for (int k = 0; k < BYTES / 16; ++k) {
            const uint4 w = reinterpret_cast<const uint4*>(p)[k];
            __builtin_memcpy(reinterpret_cast<char*>(out) + 16 * k, &w, 16);
        }
    } else if constexpr (BYTES % 8 == 0) {
#pragma unroll
        for (int k = 0; k < BYTES / 8; ++k) {
            const uint2 w = reinterpret_cast<const uint2*>(p)[k];
            __builtin_memcpy(reinterpret_cast<char*>(out) + 8 * k, &w, 8);
        }
    } else {
#pragma unroll
        for (int k = 0; k < NE; ++k) out[k] = reinterpret_cast<const S*>(p)[k];
    }
}

template <typename S, int NE>
__device__ __forceinline__ void store_row(S* __restrict__ base, int64_t idx, const S (&in)[NE]) {
    constexpr int BYTES = NE * int(sizeof(S));
    char* p = reinterpret_cast<char*>(base) + idx * BYTES;
    if constexpr (BYTES % 16 == 0) {
#pragma unroll
        for (int k = 0; k < BYTES / 16; ++k) {
            uint4 w;
            __builtin_memcpy(&w, reinterpret_cast<const char*>(in) + 16 * k, 16);
            reinterpret_cast<uint4*>(p)[k] = w;
        }
    } else if constexpr (BYTES % 8 == 0) {
#pragma unroll
        for (int k = 0; k < BYTES / 8; ++k) {
            uint2 w;
            __builtin_memcpy(&w, reinterpret_cast<const char*>(in) + 8 * k, 8);
            reinterpret_cast<uint2*>(p)[k] = w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NE; ++k) reinterpret_cast<S*>(p)[k] = in[k];
    }
}

// Wavefront reduce-scatter of B values per lane: afterwards every lane L
// holds the wave sum of x[L >> (6 - log2 B)].  Fixed exchange pattern.
template <int B>
__device__ __forceinline__ double wave_reduce_scatter(double (&x)[B], int lane) {
    constexpr int LOGB = Log2<B>::value;
#pragma unroll
    for (int j = 0; j < LOGB; ++j) {
        const int n = B >> j, half = n >> 1, off = 32 >> j;
        const bool upper = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const double send = upper ? x[i] : x[i + half];
            const double keep = upper ? x[i + half] : x[i];
            x[i] = keep + __shfl_xor(send, off, 64);
        }
    }
    double r = x[0];
#pragma unroll
    for (int off = 32 >> LOGB; off >= 1; off >>= 1) r += __shfl_xor(r, off, 64);
    return r;
}

struct HvArgs {
    BasisDev bs;
    const DevOp* ops;
    int n_ops;
    const void* v;
    void* u;
    const void* y;
    const double* cy;
    const double* sx;
    double a, b;
    const int* stop;
    double* partials;
};

// S: storage scalar, CPLX: complex vectors, CCOEF: complex coefficients,
// SECTOR: split-table rank, B: interleaved vectors per row.
template <typename S, bool CPLX, bool CCOEF, bool SECTOR, int B>
__global__ __launch_bounds__(kBlock) void hv_kernel(HvArgs A) {
    constexpr int NC = CPLX ? 2 : 1;
    constexpr int NE = B * NC;
    constexpr int LOGB = Log2<B>::value;
    if (A.stop && *A.stop) return;

    const int lane = threadIdx.x & 63;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const S* __restrict__ v = static_cast<const S*>(A.v);
    S* __restrict__ u = static_cast<S*>(A.u);
    const S* __restrict__ y = static_cast<const S*>(A.y);
    const DevOp* __restrict__ ops = A.ops;
    const BasisDev& bs = A.bs;

    double sx[B], cy[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        sx[b] = A.sx ? A.sx[b] : 1.0;
        cy[b] = (A.y && A.cy) ? A.cy[b] : 0.0;
    }

    // XCD-aware tile range
    const int xcd = blockIdx.x & 7;
    const int waves_x = int(gridDim.x >> 3) * kWavesPerBlock;
    const int wl = int(blockIdx.x >> 3) * kWavesPerBlock + wave;
    const int64_t T = bs.n_tiles;
    const int64_t Tx = (T + 7) >> 3;
    const int64_t t_begin = xcd * Tx;
    const int64_t t_end = (t_begin + Tx < T) ? t_begin + Tx : T;

    double wq[kNQ] = {0.0, 0.0, 0.0, 0.0};

    for (int64_t tile = t_begin + wl; tile < t_end; tile += waves_x) {
        int64_t row;
        uint64_t s;
        bool valid;
        if constexpr (!SECTOR) {
            row = tile * kTile + lane;
            valid = row < bs.dim;
            s = uint64_t(row);
        } else {
            const int64_t k = find_high(bs.h_tile, bs.n_high, tile);
            const int64_t start = (tile - bs.h_tile[k]) * kTile + lane;
            const int64_t cnt = bs.h_row[k + 1] - bs.h_row[k];
            valid = start < cnt;
            row = bs.h_row[k] + start;
            s = valid ? ((bs.h_val[k] << bs.b_lo) | uint64_t(bs.lows[bs.h_lobase[k] + start])) : 0;
        }

        S acc[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) acc[e] = S(0);
        double dsum = 0.0;

        if (valid) {
            for (int o = 0; o < A.n_ops; ++o) {
                const DevOp& op = ops[o];
                const int p = int((s >> op.bi) & 1u) | (int((s >> op.bj) & 1u) << 1);
                dsum += sel4(p, op.d[0], op.d[1], op.d[2], op.d[3]);
                if (op.xmask == 0) continue;
                S cr, ci;
                if constexpr (sizeof(S) == 4) {
                    cr = sel4(p, op.fr[0], op.fr[1], op.fr[2], op.fr[3]);
                    ci = CCOEF ? sel4(p, op.fi[0], op.fi[1], op.fi[2], op.fi[3]) : 0.0f;
                } else {
                    cr = sel4(p, op.cr[0], op.cr[1], op.cr[2], op.cr[3]);
                    ci = CCOEF ? sel4(p, op.ci[0], op.ci[1], op.ci[2], op.ci[3]) : 0.0;
                }
                const bool active = (cr != S(0)) || (CCOEF && ci != S(0));
                if (active) {
                    const uint64_t t = s ^ op.xmask;
                    if (op.smask != 0 && (__popcll(s & op.smask) & 1)) {
                        cr = -cr;
                        ci = -ci;
                    }
                    const int64_t idx = rank_of<SECTOR>(bs, t);
                    alignas(16) S g[NE];
                    load_row<S, NE>(v, idx, g);
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        if constexpr (CPLX) {
                            const S gr = g[2 * b], gi = g[2 * b + 1];
                            if constexpr (CCOEF) {
                                acc[2 * b] += cr * gr - ci * gi;
                                acc[2 * b + 1] += cr * gi + ci * gr;
                            } else {
                                acc[2 * b] += cr * gr;
                                acc[2 * b + 1] += cr * gi;
                            }
                        } else {
                            acc[b] += cr * g[b];
                        }
                    }
                }
            }
        }

        // epilogue: u = a * H x + b * x + cy * y with x = sx * v, in FP64
        double q[kNQ][B];
        if (valid) {
            alignas(16) S vr[NE];
            load_row<S, NE>(v, row, vr);
            alignas(16) S yr[NE];
            if (y) load_row<S, NE>(y, row, yr);
            alignas(16) S ur[NE];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if constexpr (CPLX) {
                    const double xr = sx[b] * double(vr[2 * b]), xi = sx[b] * double(vr[2 * b + 1]);
                    const double hr = sx[b] * (double(acc[2 * b]) + dsum * double(vr[2 * b]));
                    const double hi = sx[b] * (double(acc[2 * b + 1]) + dsum * double(vr[2 * b + 1]));
                    double ore = A.a * hr + A.b * xr, oim = A.a * hi + A.b * xi;
                    if (y) {
                        ore += cy[b] * double(yr[2 * b]);
                        oim += cy[b] * double(yr[2 * b + 1]);
                    }
                    ur[2 * b] = S(ore);
                    ur[2 * b + 1] = S(oim);
                    q[0][b] = xr * xr + xi * xi;
                    q[1][b] = xr * hr + xi * hi;
                    q[2][b] = hr * hr + hi * hi;
                    q[3][b] = ore * ore + oim * oim;
                } else {
                    const double x = sx[b] * double(vr[b]);
                    const double h = sx[b] * (double(acc[b]) + dsum * double(vr[b]));
                    double o = A.a * h + A.b * x;
                    if (y) o += cy[b] * double(yr[b]);
                    ur[b] = S(o);
                    q[0][b] = x * x;
                    q[1][b] = x * h;
                    q[2][b] = h * h;
                    q[3][b] = o * o;
                }
            }
            if (u) store_row<S, NE>(u, row, ur);
        } else {
#pragma unroll
            for (int k = 0; k < kNQ; ++k)
#pragma unroll
                for (int b = 0; b < B; ++b) q[k][b] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < kNQ; ++k) wq[k] += wave_reduce_scatter<B>(q[k], lane);
    }

    __shared__ double sh[kWavesPerBlock][kNQ][64];
#pragma unroll
    for (int k = 0; k < kNQ; ++k) sh[wave][k][lane] = wq[k];
    __syncthreads();
    if (int(threadIdx.x) < kNQ * B) {
        const int k = threadIdx.x / B, b = threadIdx.x % B;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) s += sh[w][k][b << (6 - LOGB)];
        A.partials[size_t(blockIdx.x) * (kNQ * B) + threadIdx.x] = s;
    }
}

// out[q] = sum over g of partials[g * nq + q], fixed order; one block per q.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partials, int n_parts,
                                                              int nq, double* __restrict__ out,
                                                              const int* stop) {
    if (stop && *stop) return;
    const int q = blockIdx.x;
    double s = 0.0;
    for (int g = threadIdx.x; g < n_parts; g += 256) s += partials[size_t(g) * nq + q];
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = sh[0];
}

// ---- element export (same operator evaluation as hv_kernel, FP64 values)
template <bool SECTOR>
__global__ __launch_bounds__(256) void elements_kernel(BasisDev bs, const DevOp* __restrict__ ops, int n_ops,
                                                       int64_t row0, int64_t nrows, int cap,
                                                       int64_t* __restrict__ cols, double* __restrict__ re,
                                                       double* __restrict__ im, int32_t* __restrict__ term,
                                                       int32_t* __restrict__ counts) {
    const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (r >= nrows) return;
    const int64_t row = row0 + r;
    const uint64_t s = unrank_row(bs, row);
    int n = 0;
    double dsum = 0.0;
    for (int o = 0; o < n_ops; ++o) {
        const DevOp& op = ops[o];
        const int p = int((s >> op.bi) & 1u) | (int((s >> op.bj) & 1u) << 1);
        dsum += sel4(p, op.d[0], op.d[1], op.d[2], op.d[3]);
    }
    const size_t base = size_t(r) * cap;
    if (dsum != 0.0) {
        if (n < cap) {
            cols[base + n] = row;
            re[base + n] = dsum;
            im[base + n] = 0.0;
            term[base + n] = -1;
        }
        ++n;
    }
    for (int o = 0; o < n_ops; ++o) {
        const DevOp& op = ops[o];
        if (op.xmask == 0) continue;
        const int p = int((s >> op.bi) & 1u) | (int((s >> op.bj) & 1u) << 1);
        double cr = sel4(p, op.cr[0], op.cr[1], op.cr[2], op.cr[3]);
        double ci = sel4(p, op.ci[0], op.ci[1], op.ci[2], op.ci[3]);
        if (cr == 0.0 && ci == 0.0) continue;
        const uint64_t t = s ^ op.xmask;
        if (op.smask != 0 && (__popcll(s & op.smask) & 1)) {
            cr = -cr;
            ci = -ci;
        }
        if (n < cap) {
            cols[base + n] = rank_of<SECTOR>(bs, t);
            re[base + n] = cr;
            im[base + n] = ci;
            term[base + n] = op.term;
        }
        ++n;
    }
    counts[r] = n;
}

__global__ void rank_kernel(BasisDev bs, int32_t particle, int32_t sector, int32_t ta, int32_t tb,
                            const uint64_t* __restrict__ cfg, int64_t* __restrict__ idx, int64_t n) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= n) return;
    const uint64_t c = cfg[k];
    if (bs.nbits < 64 && (c >> bs.nbits) != 0) {
        idx[k] = -1;
        return;
    }
    bool ok = true;
    if (sector == HPHI_SECTOR_SZ || sector == HPHI_SECTOR_NTOT) {
        ok = __popcll(c) == ta;
    } else if (sector == HPHI_SECTOR_NUP_NDN) {
        ok = __popcll(c & 0x5555555555555555ull) == ta && __popcll(c & 0xAAAAAAAAAAAAAAAAull) == tb;
    }
    (void)particle;
    if (!ok) {
        idx[k] = -1;
        return;
    }
    idx[k] = sector == 0 ? int64_t(c) : rank_of<true>(bs, c);
}

__global__ void unrank_kernel(BasisDev bs, const int64_t* __restrict__ idx, uint64_t* __restrict__ cfg, int64_t n) {
    const int64_t k = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (k >= n) return;
    const int64_t r = idx[k];
    cfg[k] = (r < 0 || r >= bs.dim) ? ~uint64_t(0) : unrank_row(bs, r);
}

// ---- streaming kernels of the Lanczos recurrence (real scalars; a complex
// vector is 2n scalars and all coefficients here are real)
template <typename S>
__global__ __launch_bounds__(256) void copy_norm_kernel(const S* __restrict__ src, S* __restrict__ dst, int64_t n,
                                                        double* __restrict__ partials) {
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const S x = src[i];
        if (dst) dst[i] = x;
        s += double(x) * double(x);
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// y += c2 * x, |y|^2; optionally acc += ecoef * x (FP64 accumulator)
template <typename S>
__global__ __launch_bounds__(256) void lanczos_update_kernel(S* __restrict__ y, const S* __restrict__ x, int64_t n,
                                                             const double* __restrict__ c2p,
                                                             double* __restrict__ acc,
                                                             const double* __restrict__ ecp,
                                                             double* __restrict__ partials, const int* stop) {
    if (stop && *stop) return;
    const double c2 = *c2p;
    const double ec = acc ? *ecp : 0.0;
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const double xv = double(x[i]);
        const S w = S(double(y[i]) + c2 * xv);
        y[i] = w;
        s += double(w) * double(w);
        if (acc) acc[i] += ec * xv;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void fill_zero_kernel(uint32_t* __restrict__ p, int64_t n_words) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n_words; i += int64_t(gridDim.x) * 256) p[i] = 0u;
}

__global__ void tpq_obs_kernel(const double* __restrict__ red, double* __restrict__ obs, int nvec, double ns,
                               double l, int k) {
    const int b = threadIdx.x;
    if (b >= nvec) return;
    const double xx = red[0 * nvec + b], xh = red[1 * nvec + b], hh = red[2 * nvec + b],
                 uu = red[3 * nvec + b];
    const double uk = xh / xx / ns;
    obs[0 * nvec + b] = uk;
    obs[1 * nvec + b] = hh / xx / (ns * ns);
    obs[2 * nvec + b] = (2.0 * double(k - 1) / ns) / (l - uk);
    obs[3 * nvec + b] = 1.0 / sqrt(uu);
}

__global__ void lz_init_kernel(LzScalars* sc, const double* red, double tol, int n_max) {
    const double nn = red[0];
    sc->s_cur = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    sc->cy = 0.0;
    sc->c2 = 0.0;
    sc->ecoef = 0.0;
    sc->beta_k = 0.0;
    sc->tol = tol;
    sc->k = 0;
    sc->n_max = n_max;
    sc->stop = nn > 0.0 ? 0 : 1;
    sc->n_done = 0;
    sc->breakdown = nn > 0.0 ? 0 : 1;
}

__global__ void lz_after_hv_kernel(LzScalars* sc, const double* red, double* alpha, const double* evec) {
    if (sc->stop) return;
    const double a = red[1];          // Re<v_k|H v_k>, v_k = s_cur * X
    alpha[sc->k] = a;
    sc->c2 = -a * sc->s_cur;
    sc->ecoef = evec ? evec[sc->k] * sc->s_cur : 0.0;
}

__global__ void lz_after_update_kernel(LzScalars* sc, const double* red, double* beta, const double* alpha) {
    if (sc->stop) return;
    const int k = sc->k;
    const double b = sqrt(red[0]);
    beta[k] = b;
    sc->n_done = k + 1;
    const double a = fabs(alpha[k]);
    double scale = a > sc->beta_k ? a : sc->beta_k;
    if (scale < 1.0) scale = 1.0;
    if (k + 1 >= sc->n_max || b <= sc->tol * scale) {
        sc->stop = 1;
        if (k + 1 < sc->n_max) sc->breakdown = 1;
        return;
    }
    sc->cy = -b * sc->s_cur;   // -beta_{k+1} times the scale of v_k (next step's v_{k-1})
    sc->s_cur = 1.0 / b;
    sc->beta_k = b;
    sc->k = k + 1;
}

}  // namespace

// ------------------------------------------------------------------ launchers

size_t dtype_size(int dtype) {
    switch (dtype) {
        case HPHI_F64: return 8;
        case HPHI_C128: return 16;
        case HPHI_F32: return 4;
        case HPHI_C64: return 8;
    }
    return 0;
}

bool dtype_complex(int dtype) { return dtype == HPHI_C128 || dtype == HPHI_C64; }

template <typename S, bool CPLX, bool CCOEF, bool SECTOR, int B>
static int launch_hv_t(const HvLaunch& L, hipStream_t st) {
    const hphi_ham* H = L.ham;
    HvArgs A;
    A.bs = H->basis->dev;
    A.ops = H->d_ops;
    A.n_ops = int(H->ops.size());
    A.v = L.v;
    A.u = L.u;
    A.y = L.y;
    A.cy = L.cy;
    A.sx = L.sx;
    A.a = L.a;
    A.b = L.b;
    A.stop = L.stop;
    A.partials = H->d_partials;
    hv_kernel<S, CPLX, CCOEF, SECTOR, B><<<H->grid, kBlock, 0, st>>>(A);
    int rc = check_hip(hipGetLastError(), "hv_kernel launch");
    if (rc) return rc;
    if (L.reduce_out) {
        reduce_partials_kernel<<<kNQ * B, 256, 0, st>>>(H->d_partials, H->grid, kNQ * B, L.reduce_out, L.stop);
        rc = check_hip(hipGetLastError(), "reduce launch");
    }
    return rc;
}

template <typename S, bool CPLX, bool CCOEF, bool SECTOR>
static int launch_hv_b(const HvLaunch& L, hipStream_t st) {
    switch (L.nvec) {
        case 1: return launch_hv_t<S, CPLX, CCOEF, SECTOR, 1>(L, st);
        case 2: return launch_hv_t<S, CPLX, CCOEF, SECTOR, 2>(L, st);
        case 4: return launch_hv_t<S, CPLX, CCOEF, SECTOR, 4>(L, st);
        case 8: return launch_hv_t<S, CPLX, CCOEF, SECTOR, 8>(L, st);
        case 16: return launch_hv_t<S, CPLX, CCOEF, SECTOR, 16>(L, st);
    }
    return set_error(HPHI_EINVAL, "nvec must be 1, 2, 4, 8 or 16 (got %d)", L.nvec);
}

template <typename S, bool CPLX, bool CCOEF>
static int launch_hv_s(const HvLaunch& L, hipStream_t st) {
    if (L.ham->basis->dev.sector != 0) return launch_hv_b<S, CPLX, CCOEF, true>(L, st);
    return launch_hv_b<S, CPLX, CCOEF, false>(L, st);
}

int launch_hv(const HvLaunch& L, hipStream_t st) {
    const bool cc = L.ham->is_complex;
    switch (L.dtype) {
        case HPHI_F64:
            if (cc) return set_error(HPHI_EDTYPE, "complex Hamiltonian with real storage");
            return launch_hv_s<double, false, false>(L, st);
        case HPHI_F32:
            if (cc) return set_error(HPHI_EDTYPE, "complex Hamiltonian with real storage");
            return launch_hv_s<float, false, false>(L, st);
        case HPHI_C128:
            return cc ? launch_hv_s<double, true, true>(L, st) : launch_hv_s<double, true, false>(L, st);
        case HPHI_C64:
            return cc ? launch_hv_s<float, true, true>(L, st) : launch_hv_s<float, true, false>(L, st);
    }
    return set_error(HPHI_EINVAL, "bad dtype %d", L.dtype);
}

int launch_elements(const hphi_ham* H, int64_t row0, int64_t nrows, int cap, int64_t* cols, double* re, double* im,
                    int32_t* term, int32_t* counts, hipStream_t st) {
    const int64_t blocks = (nrows + 255) / 256;
    if (H->basis->dev.sector != 0)
        elements_kernel<true><<<dim3(unsigned(blocks)), 256, 0, st>>>(H->basis->dev, H->d_ops, int(H->ops.size()),
                                                                        row0, nrows, cap, cols, re, im, term, counts);
    else
        elements_kernel<false><<<dim3(unsigned(blocks)), 256, 0, st>>>(H->basis->dev, H->d_ops, int(H->ops.size()),
                                                                         row0, nrows, cap, cols, re, im, term, counts);
    return check_hip(hipGetLastError(), "elements_kernel launch");
}

int launch_rank(const hphi_basis* b, const uint64_t* cfg, int64_t* idx, int64_t n, hipStream_t st) {
    int ta = 0, tb = 0;
    const hphi_basis_desc& d = b->desc;
    if (d.sector == HPHI_SECTOR_SZ) ta = (d.n_sites + d.two_sz) / 2;
    if (d.sector == HPHI_SECTOR_NUP_NDN) {
        ta = d.n_up;
        tb = d.n_dn;
    }
    if (d.sector == HPHI_SECTOR_NTOT) ta = d.n_tot;
    rank_kernel<<<dim3(unsigned((n + 255) / 256)), 256, 0, st>>>(b->dev, d.particle, d.sector, ta, tb, cfg, idx, n);
    return check_hip(hipGetLastError(), "rank_kernel launch");
}

int launch_unrank(const hphi_basis* b, const int64_t* idx, uint64_t* cfg, int64_t n, hipStream_t st) {
    unrank_kernel<<<dim3(unsigned((n + 255) / 256)), 256, 0, st>>>(b->dev, idx, cfg, n);
    return check_hip(hipGetLastError(), "unrank_kernel launch");
}

static int stream_grid(int64_t n) {
    int64_t g = (n + 1023) / 1024;
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    return int(g);
}

int launch_copy_norm(const void* src, void* dst, int64_t n, int dtype, double* partials, int grid, double* red,
                     hipStream_t st) {
    const int64_t ns = n * (dtype_complex(dtype) ? 2 : 1);
    if (grid <= 0) grid = stream_grid(ns);
    if (dtype == HPHI_F64 || dtype == HPHI_C128)
        copy_norm_kernel<double><<<grid, 256, 0, st>>>((const double*)src, (double*)dst, ns, partials);
    else
        copy_norm_kernel<float><<<grid, 256, 0, st>>>((const float*)src, (float*)dst, ns, partials);
    int rc = check_hip(hipGetLastError(), "copy_norm launch");
    if (rc) return rc;
    reduce_partials_kernel<<<1, 256, 0, st>>>(partials, grid, 1, red, nullptr);
    return check_hip(hipGetLastError(), "reduce launch");
}

int launch_lanczos_update(void* y, const void* x, int64_t n, int dtype, const double* c2, void* acc,
                          const double* ecoef, double* partials, int grid, double* red, const int* stop,
                          hipStream_t st) {
    const int64_t ns = n * (dtype_complex(dtype) ? 2 : 1);
    if (grid <= 0) grid = stream_grid(ns);
    if (dtype == HPHI_F64 || dtype == HPHI_C128)
        lanczos_update_kernel<double><<<grid, 256, 0, st>>>((double*)y, (const double*)x, ns, c2, (double*)acc,
                                                            ecoef, partials, stop);
    else
        lanczos_update_kernel<float><<<grid, 256, 0, st>>>((float*)y, (const float*)x, ns, c2, (double*)acc, ecoef,
                                                           partials, stop);
    int rc = check_hip(hipGetLastError(), "lanczos_update launch");
    if (rc) return rc;
    reduce_partials_kernel<<<1, 256, 0, st>>>(partials, grid, 1, red, stop);
    return check_hip(hipGetLastError(), "reduce launch");
}

int launch_fill_zero(void* p, int64_t bytes, hipStream_t st) {
    const int64_t words = bytes / 4;
    fill_zero_kernel<<<stream_grid(words), 256, 0, st>>>((uint32_t*)p, words);
    return check_hip(hipGetLastError(), "fill_zero launch");
}

int launch_tpq_obs(const double* red, double* obs, int nvec, double n_sites, double l, int k, hipStream_t st) {
    tpq_obs_kernel<<<1, 64, 0, st>>>(red, obs, nvec, n_sites, l, k);
    return check_hip(hipGetLastError(), "tpq_obs launch");
}

int launch_lz_init(LzScalars* sc, const double* red, double tol, int n_max, hipStream_t st) {
    lz_init_kernel<<<1, 1, 0, st>>>(sc, red, tol, n_max);
    return check_hip(hipGetLastError(), "lz_init launch");
}

int launch_lz_after_hv(LzScalars* sc, const double* red, double* alpha, const double* evec, hipStream_t st) {
    lz_after_hv_kernel<<<1, 1, 0, st>>>(sc, red, alpha, evec);
    return check_hip(hipGetLastError(), "lz_after_hv launch");
}

int launch_lz_after_update(LzScalars* sc, const double* red, double* beta, const double* alpha, hipStream_t st) {
    lz_after_update_kernel<<<1, 1, 0, st>>>(sc, red, beta, alpha);
    return check_hip(hipGetLastError(), "lz_after_update launch");
}

}  // namespace hphi
