// gfx950 kernels of the matrix-free product and its reductions.
//
// Product (Sec. 3.3): each row s of the output is owned by one lane, or by
// LPR = 2, 4 or 8 lanes that split its vectors when nvec >= 8 ("pull").  For
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

#include <algorithm>
#include <mutex>
#include <cstdlib>
#include <vector>

#include <type_traits>

#include "hphi_internal.h"

namespace hphi {
namespace {

constexpr int ilog2(int b) { return b <= 1 ? 0 : 1 + ilog2(b / 2); }

template <int B>
struct Log2 {
    static_assert(B > 0 && (B & (B - 1)) == 0, "power of two");
    static constexpr int value = ilog2(B);
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

// charge class of a low half: its popcount, or (fermions at fixed up and
// down counts) n_even * (nsl + 1) + n_odd over its nsl sites
__device__ __forceinline__ int low_class(uint32_t l, int cls_pairs, int nsl) {
    if (!cls_pairs) return __popc(l);
    return __popc(l & 0x55555555u) * (nsl + 1) + __popc(l & 0xAAAAAAAAu);
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

// ---- lane share of an interleaved row.  A row of nvec vectors is split
// over LPR lanes in chunks of CB = min(16, lane bytes) bytes, dealt
// round-robin: lane `sub` owns chunks sub, sub + LPR, sub + 2 LPR, ...  One
// 16-byte load instruction of the LPR lanes of a row therefore reads
// LPR * 16 contiguous bytes of it (a whole 128-byte line at LPR = 8), so
// no line is requested by several instructions.
template <typename S, int NE, int LPR>
struct LaneLayout {
    static constexpr int LB = NE * int(sizeof(S));     // bytes per lane per row
    static constexpr int CB = LB >= 16 ? 16 : LB;      // chunk bytes
    static constexpr int NCH = LB / CB;                // chunks per lane
    static constexpr int CPS = CB / int(sizeof(S));    // scalars per chunk
    static constexpr int RB = LB * LPR;                // row bytes
};

template <int CB>
__device__ __forceinline__ void copy_chunk(char* dst, const char* src) {
    if constexpr (CB == 16) {
        const uint4 w = *reinterpret_cast<const uint4*>(src);
        __builtin_memcpy(dst, &w, 16);
    } else if constexpr (CB == 8) {
        const uint2 w = *reinterpret_cast<const uint2*>(src);
        __builtin_memcpy(dst, &w, 8);
    } else {
        static_assert(CB == 4, "chunk of 4, 8 or 16 bytes");
        const uint32_t w = *reinterpret_cast<const uint32_t*>(src);
        __builtin_memcpy(dst, &w, 4);
    }
}

template <int CB>
__device__ __forceinline__ void put_chunk(char* dst, const char* src) {
    if constexpr (CB == 16) {
        uint4 w;
        __builtin_memcpy(&w, src, 16);
        *reinterpret_cast<uint4*>(dst) = w;
    } else if constexpr (CB == 8) {
        uint2 w;
        __builtin_memcpy(&w, src, 8);
        *reinterpret_cast<uint2*>(dst) = w;
    } else {
        uint32_t w;
        __builtin_memcpy(&w, src, 4);
        *reinterpret_cast<uint32_t*>(dst) = w;
    }
}

// streaming variants: non-temporal hint (data not reused, should not evict
// the L2 window of the gathers)
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));

template <int CB>
__device__ __forceinline__ void copy_chunk_nt(char* dst, const char* src) {
    if constexpr (CB == 16) {
        const u32x4_t w = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(src));
        __builtin_memcpy(dst, &w, 16);
    } else if constexpr (CB == 8) {
        const u32x2_t w = __builtin_nontemporal_load(reinterpret_cast<const u32x2_t*>(src));
        __builtin_memcpy(dst, &w, 8);
    } else {
        const uint32_t w = __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(src));
        __builtin_memcpy(dst, &w, 4);
    }
}

template <int CB>
__device__ __forceinline__ void put_chunk_nt(char* dst, const char* src) {
    if constexpr (CB == 16) {
        u32x4_t w;
        __builtin_memcpy(&w, src, 16);
        __builtin_nontemporal_store(w, reinterpret_cast<u32x4_t*>(dst));
    } else if constexpr (CB == 8) {
        u32x2_t w;
        __builtin_memcpy(&w, src, 8);
        __builtin_nontemporal_store(w, reinterpret_cast<u32x2_t*>(dst));
    } else {
        uint32_t w;
        __builtin_memcpy(&w, src, 4);
        __builtin_nontemporal_store(w, reinterpret_cast<uint32_t*>(dst));
    }
}

template <typename S, int NE, int LPR>
__device__ __forceinline__ void load_lane_nt(const S* __restrict__ base, int64_t row, int sub, S (&out)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
    const char* p = reinterpret_cast<const char*>(base) + row * Ly::RB + sub * Ly::CB;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        copy_chunk_nt<Ly::CB>(reinterpret_cast<char*>(out) + j * Ly::CB, p + j * LPR * Ly::CB);
}

template <typename S, int NE, int LPR>
__device__ __forceinline__ void store_lane_nt(S* __restrict__ base, int64_t row, int sub, const S (&in)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
    char* p = reinterpret_cast<char*>(base) + row * Ly::RB + sub * Ly::CB;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        put_chunk_nt<Ly::CB>(p + j * LPR * Ly::CB, reinterpret_cast<const char*>(in) + j * Ly::CB);
}

// Values of another lane of the wavefront (byte address 4 * lane); every
// lane of the wavefront must take part.
template <typename S, int NE>
__device__ __forceinline__ void exchange_lane(const S (&x)[NE], int addr, S (&out)[NE]) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        if constexpr (sizeof(S) == 4) {
            out[e] = __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x[e])));
        } else {
            const long long w = __double_as_longlong(x[e]);
            const int lo = __builtin_amdgcn_ds_bpermute(addr, int(w));
            const int hi = __builtin_amdgcn_ds_bpermute(addr, int(w >> 32));
            out[e] = __longlong_as_double(static_cast<long long>(static_cast<unsigned>(lo)) |
                                          (static_cast<long long>(hi) << 32));
        }
    }
}

// Whether the windowed product keeps a wavefront's 64-row tile of v in LDS
// (8 lanes per row measured slower with it).
__host__ __device__ constexpr bool tile_in_lds(int row_bytes, int lpr) { return 64 * row_bytes <= 8192 && lpr <= 4; }

// A wavefront's 64-row tile of v in LDS, rows in the lane layout of
// memory; odd rows swap the two halves of their chunks, so that lanes
// reading consecutive rows spread over all banks.
template <typename S, int NE, int LPR>
__device__ __forceinline__ int tile_chunk(int r, int c) {
    using Ly = LaneLayout<S, NE, LPR>;
    constexpr int NCR = Ly::RB / Ly::CB;
    return r * Ly::RB + (NCR >= 2 ? (c ^ ((r & 1) * (NCR / 2))) : c) * Ly::CB;
}

template <typename S, int NE, int LPR>
__device__ __forceinline__ void tile_put(char* tb, int r, int sub, const S (&in)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        put_chunk<Ly::CB>(tb + tile_chunk<S, NE, LPR>(r, j * LPR + sub), reinterpret_cast<const char*>(in) + j * Ly::CB);
}

template <typename S, int NE, int LPR>
__device__ __forceinline__ void tile_get(const char* tb, int r, int sub, S (&out)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        copy_chunk<Ly::CB>(reinterpret_cast<char*>(out) + j * Ly::CB, tb + tile_chunk<S, NE, LPR>(r, j * LPR + sub));
}

template <typename S, int NE, int LPR>
__device__ __forceinline__ void load_lane(const S* __restrict__ base, int64_t row, int sub, S (&out)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
    const char* p = reinterpret_cast<const char*>(base) + row * Ly::RB + sub * Ly::CB;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        copy_chunk<Ly::CB>(reinterpret_cast<char*>(out) + j * Ly::CB, p + j * LPR * Ly::CB);
}

template <typename S, int NE, int LPR>
__device__ __forceinline__ void store_lane(S* __restrict__ base, int64_t row, int sub, const S (&in)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
    char* p = reinterpret_cast<char*>(base) + row * Ly::RB + sub * Ly::CB;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        put_chunk<Ly::CB>(p + j * LPR * Ly::CB, reinterpret_cast<const char*>(in) + j * Ly::CB);
}

// A row of zeros in device memory (the widest row: 16 complex128 values).
// In the windowed and block-staged kernels, lanes whose element is zero read
// it instead of a partner row, so the accumulation adds exact zeros.
__device__ __align__(256) uint32_t kZeroRow[64] = {};

// the lane's share of the row at byte address rowp
template <typename S, int NE, int LPR>
__device__ __forceinline__ void load_lane_at(const char* rowp, int sub, S (&out)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
    const char* p = rowp + sub * Ly::CB;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        copy_chunk<Ly::CB>(reinterpret_cast<char*>(out) + j * Ly::CB, p + j * LPR * Ly::CB);
}

// row `idx` of v for an active lane, the zero row otherwise
template <typename S, int NE, int LPR>
__device__ __forceinline__ const char* row_or_zero(const S* v, int64_t idx, bool act) {
    return act ? reinterpret_cast<const char*>(v) + idx * int64_t(LaneLayout<S, NE, LPR>::RB)
               : reinterpret_cast<const char*>(kZeroRow);
}

// Byte offset in a wavefront's LDS tile of the lane's first chunk of row r
// (the layout of tile_chunk: odd rows swap the two halves of the row); its
// chunk j then sits at offset ^ (j * LPR * CB)
template <typename S, int NE, int LPR>
__device__ __forceinline__ uint32_t tile_off(int r, uint32_t sub_cb) {
    using Ly = LaneLayout<S, NE, LPR>;
    constexpr int NCR = Ly::RB / Ly::CB;
    uint32_t off = uint32_t(r) * uint32_t(Ly::RB) | sub_cb;
    if constexpr (NCR >= 2) off ^= (uint32_t(r) & 1u) * uint32_t(Ly::RB / 2);
    return off;
}

template <typename S, int NE, int LPR>
__device__ __forceinline__ void tile_get_off(const char* tb, uint32_t off, S (&out)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        copy_chunk<Ly::CB>(reinterpret_cast<char*>(out) + j * Ly::CB, tb + (off ^ uint32_t(j * LPR * Ly::CB)));
}

// the lane's share of a row, from the lane's own chunk address p
template <typename S, int NE, int LPR>
__device__ __forceinline__ void load_sub_at(const char* p, S (&out)[NE]) {
    using Ly = LaneLayout<S, NE, LPR>;
#pragma unroll
    for (int j = 0; j < Ly::NCH; ++j)
        copy_chunk<Ly::CB>(reinterpret_cast<char*>(out) + j * Ly::CB, p + j * LPR * Ly::CB);
}

// vector index of the lane's b-th vector (b < NE / NC)
template <typename S, int NE, int LPR, int NC>
__device__ __forceinline__ int lane_vec(int sub, int b) {
    using Ly = LaneLayout<S, NE, LPR>;
    const int e = NC * b;
    return ((e / Ly::CPS * LPR + sub) * Ly::CPS + e % Ly::CPS) / NC;
}

// inverse: lane share `sub` and local index `bi` of vector g
template <typename S, int NE, int LPR, int NC>
__host__ __device__ constexpr void vec_lane(int g, int& sub, int& bi) {
    using Ly = LaneLayout<S, NE, LPR>;
    const int eg = NC * g;
    const int c = eg / Ly::CPS;
    sub = c % LPR;
    bi = ((c / LPR) * Ly::CPS + eg % Ly::CPS) / NC;
}

// acc += c * g for one gathered row (c = cr + i ci), FP64.  With SEL, a lane
// whose element is zero (act false) adds exactly zero: it skipped its gather,
// so its g registers hold a stale row that may be non-finite, and 0 * Inf
// would be NaN.  Without SEL the caller has made g a zero row for such lanes
// (or a row that the lane's own output depends on anyway).
template <typename S, bool CPLX, bool CCOEF, int VPL, bool SEL = false>
__device__ __forceinline__ void accumulate(double (&acc)[VPL * (CPLX ? 2 : 1)], const S (&g)[VPL * (CPLX ? 2 : 1)],
                                           bool act, double cr, double ci) {
#pragma unroll
    for (int b = 0; b < VPL; ++b) {
        if constexpr (CPLX) {
            const double gr = SEL && !act ? 0.0 : double(g[2 * b]);
            const double gi = SEL && !act ? 0.0 : double(g[2 * b + 1]);
            if constexpr (CCOEF) {
                acc[2 * b] += cr * gr - ci * gi;
                acc[2 * b + 1] += cr * gi + ci * gr;
            } else {
                acc[2 * b] += cr * gr;
                acc[2 * b + 1] += cr * gi;
            }
        } else {
            acc[b] += cr * (SEL && !act ? 0.0 : double(g[b]));
        }
    }
}

struct HvArgs {
    BasisDev bs;
    const DevOp* ops;    // padded to n_ops (a multiple of 4)
    int n_ops;
    const double* ptab;  // [n_ops][4][Re c, Im c, d, 0] pattern table
    const void* v;
    void* u;
    const void* y;
    const double* cy;
    const double* sx;
    double a, b;
    const int* stop;
    double* partials;
    ExportArgs ex;       // element export (EXPORT instantiations only)
    // two-level low-rank table (TAB 3), compact form: with l = (a, b), b its
    // low b2 bits, rank(l) = T1c[a][class(b)] + (T2p[b] & 1023); class(b) is
    // popcount(b), or for fermions at fixed up and down counts
    // popcount(b & even) * w2 + popcount(b & odd)
    const uint16_t* t1c; // [2^(b_lo - b2)][n2]
    const uint16_t* t2p; // [2^b2]
    int32_t b2, n2, cls_pairs, w2;
};

// the packed operator table seen through the constant address space
typedef const __attribute__((address_space(4))) DevOp ConstOp;

template <bool W64>
struct StateT {
    using type = uint32_t;
};
template <>
struct StateT<true> {
    using type = uint64_t;
};

// bit `pos` of a configuration (pos uniform across the wavefront)
template <bool W64>
__device__ __forceinline__ uint32_t bit_at(typename StateT<W64>::type s, uint32_t pos) {
    if constexpr (W64) {
        return uint32_t(s >> pos) & 1u;
    } else {
        return __builtin_amdgcn_ubfe(s, pos, 1u);
    }
}

template <bool W64>
__device__ __forceinline__ uint32_t parity_masked(typename StateT<W64>::type s, uint64_t m) {
    if constexpr (W64) {
        return uint32_t(__popcll(s & m)) & 1u;
    } else {
        return uint32_t(__popc(s & uint32_t(m))) & 1u;
    }
}

// branch-free choice between two values by a lane mask (all ones / zero):
// a bitwise select, so no register array is ever indexed per lane
__device__ __forceinline__ double pick(uint32_t m, double a, double b) {
    const uint64_t mm = (uint64_t(m) << 32) | m;
    const uint64_t ua = __double_as_longlong(a), ub = __double_as_longlong(b);
    return __longlong_as_double(static_cast<long long>((ua & mm) | (ub & ~mm)));
}

// Reduce one quantity over the rows held by a wavefront.  Each lane holds
// VPL per-row values (its share of the vectors); afterwards lane L holds the
// wave sum for the local vector L >> (6 - log2 VPL) of share L & (LPR-1)
// (vec_lane maps a vector to its share and local index).  Every step is
// FP64.
template <typename R, int VPL, int LPR>
__device__ __forceinline__ double wave_reduce_rows(R (&x)[VPL], int lane) {
    constexpr int LOGV = Log2<VPL>::value;
#pragma unroll
    for (int j = 0; j < LOGV; ++j) {
        const int half = (VPL >> j) >> 1, off = 32 >> j;
        const uint32_t up = (lane & off) ? 0xffffffffu : 0u;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const R lo = x[i], hi = x[i + half];
            const R send = pick(up, lo, hi);
            const R keep = pick(up, hi, lo);
            x[i] = keep + __shfl_xor(send, off, 64);
        }
    }
    double r = double(x[0]);
#pragma unroll
    for (int off = 32 >> LOGV; off >= LPR; off >>= 1) r += __shfl_xor(r, off, 64);
    return r;
}

// The four per-row FP64 products (|x|^2, Re x*h, |h|^2, |u|^2) of this
// lane's vectors, each reduced over the wavefront's rows into wq.
template <int VPL, int LPR, int NC, int NE>
__device__ __forceinline__ void wave_reduce_quantities(const double (&x)[NE], const double (&h)[NE],
                                                       const double (&u)[NE], double (&wq)[kNQ], int lane) {
    double q[VPL];
#pragma unroll
    for (int b = 0; b < VPL; ++b) {
        q[b] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) q[b] += x[NC * b + c] * x[NC * b + c];
    }
    wq[0] += wave_reduce_rows<double, VPL, LPR>(q, lane);
#pragma unroll
    for (int b = 0; b < VPL; ++b) {
        q[b] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) q[b] += x[NC * b + c] * h[NC * b + c];
    }
    wq[1] += wave_reduce_rows<double, VPL, LPR>(q, lane);
#pragma unroll
    for (int b = 0; b < VPL; ++b) {
        q[b] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) q[b] += h[NC * b + c] * h[NC * b + c];
    }
    wq[2] += wave_reduce_rows<double, VPL, LPR>(q, lane);
#pragma unroll
    for (int b = 0; b < VPL; ++b) {
        q[b] = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) q[b] += u[NC * b + c] * u[NC * b + c];
    }
    wq[3] += wave_reduce_rows<double, VPL, LPR>(q, lane);
}

// dynamic LDS of the product kernels (pattern tables, staged rank tables)
extern __shared__ double lds_dyn[];

// Block-wide copy of `bytes` (a multiple of 4) from global memory to LDS:
// 16-byte pieces, four loads in flight per thread before their stores.
__device__ __forceinline__ void stage_to_lds(void* dst, const void* src, size_t bytes) {
    const size_t n16 = bytes / 16;
    const uint4* s4 = static_cast<const uint4*>(src);
    uint4* d4 = static_cast<uint4*>(dst);
    size_t i = threadIdx.x;
    for (; i + 3 * kBlock < n16; i += 4 * kBlock) {
        const uint4 a = s4[i], b = s4[i + kBlock], c = s4[i + 2 * kBlock], d = s4[i + 3 * kBlock];
        d4[i] = a;
        d4[i + kBlock] = b;
        d4[i + 2 * kBlock] = c;
        d4[i + 3 * kBlock] = d;
    }
    for (; i < n16; i += kBlock) d4[i] = s4[i];
    const uint32_t* s1 = static_cast<const uint32_t*>(src);
    uint32_t* d1 = static_cast<uint32_t*>(dst);
    for (size_t k = n16 * 4 + threadIdx.x; k < bytes / 4; k += kBlock) d1[k] = s1[k];
}

// Bytes of LDS the single-pass product stages: the pattern table, and on a
// sector basis the low split rank table.  A table that does not fit under
// kLdsStageBytes is read from global memory instead (TAB).
constexpr size_t kLdsStageBytes = 64 * 1024;

// Body of the single-pass product for the block `blk` of `nblk` (a multiple
// of 8) working on the problem A.
// S: storage scalar, CPLX: complex vectors, CCOEF: complex coefficients,
// SECTOR: split-table rank, B: interleaved vectors per row, LPR: lanes per
// row (each lane owns B/LPR of the vectors, in interleaved chunks),
// W64: configurations above 32 bits, TAB: table placement (0: pattern and
// low rank tables staged in LDS, 1: both read from global memory, 2: pattern
// table in LDS, low rank table from global memory).
// EXPORT: the element export of the same decode (no gathers, no output):
// per row in the export range and operator slot o, the target index and the
// signed element are recorded; the diagonal sum goes to the row's pass-0 slot.
template <typename S, bool CPLX, bool CCOEF, bool SECTOR, int B, int LPR, bool W64, int TAB, bool EXPORT = false>
__device__ __forceinline__ void hv_body(const HvArgs& A, const int blk, const int nblk) {
    using ST = typename StateT<W64>::type;
    constexpr int NC = CPLX ? 2 : 1;
    constexpr int VPL = B / LPR;          // vectors per lane
    constexpr int NE = VPL * NC;          // scalars per lane per row
    constexpr int RPW = 64 / LPR;         // rows per wavefront pass
    constexpr int LOGV = Log2<VPL>::value;
    constexpr int LOGL = Log2<LPR>::value;
    static_assert(VPL * LPR == B, "LPR must divide B");
    if (A.stop && *A.stop) return;

    const int lane = threadIdx.x & 63;
    const int sub = lane & (LPR - 1);      // which share of the vectors
    const int rlane = lane >> LOGL;        // row within the pass
    const int wave = wave_uniform(threadIdx.x >> 6);
    const S* __restrict__ v = static_cast<const S*>(A.v);
    S* __restrict__ u = static_cast<S*>(A.u);
    const S* __restrict__ y = static_cast<const S*>(A.y);
    // operator records through the constant address space: uniform indices
    // become scalar loads
    const ConstOp* ops = (const ConstOp*)(A.ops);
    const BasisDev& bs = A.bs;
    const int n_ops = A.n_ops;

    // pattern table and (sector) low rank table: staged in LDS, or global.
    // The high rank table is read with scalar loads: every row of a tile
    // shares its high half, so the target's high half is uniform.  TAB 3
    // (spaces whose full low table is too large for LDS): the two-level
    // low-rank table in LDS, 16-bit entries.
    const double* tab;
    const uint32_t* jlo = nullptr;
    const uint16_t* lt1 = nullptr;
    const uint16_t* lt2 = nullptr;
    typedef const __attribute__((address_space(4))) int64_t ConstI64;
    const ConstI64* jhi = (const ConstI64*)(bs.j_hi);
    if constexpr (TAB == 1) {
        tab = A.ptab;
        if constexpr (SECTOR) jlo = bs.j_lo;
    } else {
        double* lt = lds_dyn;
        stage_to_lds(lt, A.ptab, size_t(n_ops) * 16 * sizeof(double));
        tab = lt;
        if constexpr (SECTOR) {
            if constexpr (TAB == 0) {
                uint32_t* ll = reinterpret_cast<uint32_t*>(lt + n_ops * 16);
                const int n_lo = 1 << bs.b_lo;
                stage_to_lds(ll, bs.j_lo, size_t(n_lo) * 4);
                jlo = ll;
            } else if constexpr (TAB == 3) {
                uint16_t* s1 = reinterpret_cast<uint16_t*>(lt + n_ops * 16);
                const int n1 = (1 << (bs.b_lo - A.b2)) * A.n2;
                uint16_t* s2 = s1 + (n1 + 7) / 8 * 8;
                stage_to_lds(s1, A.t1c, (size_t(n1) * 2 + 3) / 4 * 4);
                stage_to_lds(s2, A.t2p, (size_t(1) << A.b2) * 2);
                lt1 = s1;
                lt2 = s2;
            } else {
                jlo = bs.j_lo;   // too large for LDS: read through the caches
            }
        }
        __syncthreads();
    }

    // all arithmetic in FP64: FP32 types are a storage format only
    double sx[VPL], cy[VPL];
#pragma unroll
    for (int b = 0; b < VPL; ++b) {
        const int gv = lane_vec<S, NE, LPR, NC>(sub, b);
        sx[b] = A.sx ? A.sx[gv] : 1.0;
        cy[b] = (A.y && A.cy) ? A.cy[gv] : 0.0;
    }
    const double ca = A.a, cb = A.b;

    // XCD-aware tile range: blocks blk, blk + 8, ... share an XCD and sweep
    // its contiguous eighth of the tiles
    const int xcd = blk & 7;
    int64_t tile_first, t_end, tile_step;
    if constexpr (EXPORT) {
        // the tiles that hold the export's rows, dealt over every wavefront
        tile_first = A.ex.t0 + int64_t(blk) * kWavesPerBlock + wave;
        t_end = A.ex.t1;
        tile_step = int64_t(nblk) * kWavesPerBlock;
    } else {
        const int waves_x = (nblk >> 3) * kWavesPerBlock;
        const int wl = (blk >> 3) * kWavesPerBlock + wave;
        const int64_t T = bs.n_tiles;
        const int64_t Tx = (T + 7) >> 3;
        const int64_t t_begin = xcd * Tx;
        t_end = (t_begin + Tx < T) ? t_begin + Tx : T;
        tile_first = t_begin + wl;
        tile_step = waves_x;
    }

    double wq[kNQ] = {0.0, 0.0, 0.0, 0.0};
    // gathered rows: a lane whose element is zero skips its gather and adds
    // zero in its place, so a non-finite entry of v reaches only the rows it
    // couples to
    alignas(16) S g[4][NE];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < NE; ++e) g[k][e] = S(0);

    for (int64_t tile = tile_first; tile < t_end; tile += tile_step) {
        int64_t k_hi = 0, tile_row0 = 0, cnt = kTile, hrow = 0;
        ST hbits = 0;
        uint64_t hval = 0;
        uint32_t lobase = 0;
        if constexpr (SECTOR) {
            k_hi = find_high(bs.h_tile, bs.n_high, tile);
            tile_row0 = (tile - bs.h_tile[k_hi]) * kTile;
            hrow = bs.h_row[k_hi];
            cnt = bs.h_row[k_hi + 1] - hrow;
            hval = bs.h_val[k_hi];
            hbits = ST(hval << bs.b_lo);
            lobase = bs.h_lobase[k_hi];
        }
#pragma unroll 1
        for (int pass = 0; pass < LPR; ++pass) {
            const int r_in_tile = pass * RPW + rlane;
            int64_t row;
            ST s;
            bool valid;
            if constexpr (!SECTOR) {
                row = tile * kTile + r_in_tile;
                valid = row < bs.dim;
                s = ST(row);
            } else {
                const int64_t start = tile_row0 + r_in_tile;
                valid = start < cnt;
                row = bs.h_row[k_hi] + start;
                s = valid ? (hbits | ST(bs.lows[lobase + start])) : ST(0);
            }

            double acc[NE];
#pragma unroll
            for (int e = 0; e < NE; ++e) acc[e] = 0.0;
            double dsum = 0.0;

            // operators in groups of 4: decode all, issue every gather, then
            // accumulate (FP64 coefficients and sums). Wave priority rises with
            // the phase (decode 1, gather issue 2, accumulation 0), so the SIMD's
            // arbiter favours waves about to put loads in flight over waves that
            // wait on theirs, and more gathers overlap.
            for (int o = 0; o < n_ops; o += 4) {
                if constexpr (!EXPORT) __builtin_amdgcn_s_setprio(1);
                double crk[4], cik[4];
                int64_t ik[4];
                bool actk[4];
                // the group's four records first, with one wait: scalar loads and
                // LDS reads share a wait counter, so a record loaded between two
                // pattern-table reads would also wait for the earlier read (with one
                // vector per lane; wider lanes hold too many scalar registers for it)
                constexpr bool kPre = !EXPORT && VPL == 1;
                uint32_t rbi[4], rbj[4];
                uint64_t rxm[4], rsm[4], rcm[4];
                if constexpr (kPre) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        rbi[k] = ops[o + k].bi;
                        rbj[k] = ops[o + k].bj;
                        rxm[k] = ops[o + k].xmask;
                        rsm[k] = ops[o + k].smask;
                        rcm[k] = ops[o + k].cmask;
                    }
                    asm volatile("" : "+s"(rbi[0]), "+s"(rbi[1]), "+s"(rbi[2]), "+s"(rbi[3]), "+s"(rbj[0]), "+s"(rbj[1]),
                                      "+s"(rbj[2]), "+s"(rbj[3]), "+s"(rxm[0]), "+s"(rxm[1]), "+s"(rxm[2]), "+s"(rxm[3]),
                                      "+s"(rsm[0]), "+s"(rsm[1]), "+s"(rsm[2]), "+s"(rsm[3]),
                                      "+s"(rcm[0]), "+s"(rcm[1]), "+s"(rcm[2]), "+s"(rcm[3]));
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const ConstOp& op = ops[o + k];
                    const uint32_t bi = kPre ? rbi[k] : op.bi, bj = kPre ? rbj[k] : op.bj;
                    const uint64_t xmask = kPre ? rxm[k] : op.xmask, smask = kPre ? rsm[k] : op.smask,
                                   cmask = kPre ? rcm[k] : op.cmask;
                    const uint32_t pat = bit_at<W64>(s, bi) | (bit_at<W64>(s, bj) << 1);
                    const double* te = tab + ((o + k) * 4 + int(pat)) * 4;
                    double cr = te[0];
                    double ci = CCOEF ? te[1] : 0.0;
                    double dd = te[2];
                    if (cmask != 0 && (uint64_t(s) & cmask) != op.cval) {
                        // a conditional operator that does not apply to this row
                        cr = 0.0;
                        ci = 0.0;
                        dd = 0.0;
                    }
                    dsum += dd;
                    if (smask != 0) {
                        // the fermion sign: flip the sign bits of the element
                        const int32_t sg = int32_t(parity_masked<W64>(s, smask) << 31);
                        cr = __hiloint2double(__double2hiint(cr) ^ sg, __double2loint(cr));
                        if constexpr (CCOEF) ci = __hiloint2double(__double2hiint(ci) ^ sg, __double2loint(ci));
                    }
                    int64_t idx;
                    bool live = valid;
                    if constexpr (SECTOR) {
                        // target high half (uniform over the tile): its first
                        // row, or -1 if no row of the sector has it (then every
                        // element of this operator is zero on this tile)
                        const uint64_t xm_hi = xmask >> bs.b_lo;
                        const uint64_t xm_lo = xmask & bs.mask_lo;
                        const int64_t base_hi = xm_hi ? jhi[hval ^ xm_hi] : hrow;
                        live = live && base_hi >= 0;
                        // low part: the row's own rank among its class when the
                        // operator leaves the low half alone, else the table;
                        // a table in global memory is read only by lanes whose
                        // element is nonzero (from LDS, the branch costs more
                        // than the reads it saves)
                        uint32_t part_lo = uint32_t(row - hrow);
                        if constexpr (TAB == 0) {
                            if (xm_lo) part_lo = jlo[(uint64_t(s) & bs.mask_lo) ^ xm_lo];
                        } else if constexpr (TAB == 3) {
                            if (xm_lo) {
                                const uint32_t l = uint32_t(uint64_t(s) & bs.mask_lo) ^ uint32_t(xm_lo);
                                // the two reads are independent: the class of b is
                                // counted here rather than read from T2p
                                const uint32_t b = l & ((1u << A.b2) - 1u);
                                const uint32_t cb = __builtin_amdgcn_readfirstlane(A.cls_pairs)
                                    ? __umul24(uint32_t(__popc(b & 0x55555555u)), uint32_t(A.w2)) + uint32_t(__popc(b & 0xAAAAAAAAu))
                                    : uint32_t(__popc(b));
                                part_lo = uint32_t(lt1[__umul24(l >> A.b2, uint32_t(A.n2)) + cb]) + (uint32_t(lt2[b]) & 1023u);
                            }
                        } else {
                            const bool nz = CCOEF ? (cr != 0.0 || ci != 0.0) : (cr != 0.0);
                            if (xm_lo && live && nz) part_lo = jlo[(uint64_t(s) & bs.mask_lo) ^ xm_lo];
                        }
                        idx = base_hi + int64_t(part_lo);
                    } else {
                        idx = int64_t(s ^ ST(xmask));
                    }
                    if constexpr (EXPORT) {
                        crk[k] = live ? cr : 0.0;
                        cik[k] = live ? ci : 0.0;
                    } else {
                        // a lane whose element is zero skips the gather and adds
                        // zero in its place (the accumulation selects on actk)
                        crk[k] = cr;
                        cik[k] = ci;
                        actk[k] = live && (CCOEF ? (cr != 0.0 || ci != 0.0) : (cr != 0.0));
                    }
                    ik[k] = idx;
                }
                if constexpr (SECTOR) {
                    // the four target indices are complete here (one wait for
                    // the rank loads), so the gathers below issue back to back
                    // instead of each waiting behind the previous one
#pragma unroll
                    for (int k = 0; k < 4; ++k) asm volatile("" : "+v"(ik[k]));
                }
                if constexpr (EXPORT) {
                    if (valid && sub == 0 && row >= A.ex.row0 && row < A.ex.row0 + A.ex.nrows) {
                        const size_t rb = size_t(row - A.ex.row0) * size_t(A.ex.n_slots);
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            if (o + k < A.ex.n_slots) {
                                A.ex.col[rb + o + k] = ik[k];
                                A.ex.cr[rb + o + k] = crk[k];
                                A.ex.ci[rb + o + k] = cik[k];
                            }
                    }
                    continue;
                }
                __builtin_amdgcn_s_setprio(2);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (actk[k]) load_lane<S, NE, LPR>(v, ik[k], sub, g[k]);
                __builtin_amdgcn_s_setprio(0);
#pragma unroll
                for (int k = 0; k < 4; ++k) accumulate<S, CPLX, CCOEF, VPL, true>(acc, g[k], actk[k], crk[k], cik[k]);
            }

            if constexpr (EXPORT) {
                if (valid && sub == 0 && row >= A.ex.row0 && row < A.ex.row0 + A.ex.nrows)
                    A.ex.diag[size_t(row - A.ex.row0) * size_t(A.ex.n_pass)] = dsum;
                continue;
            }
            // epilogue: u = a * H x + b * x + cy * y with x = sx * v
            double xr[NE], ur[NE];
            if (valid) {
                alignas(16) S vr[NE];
                load_lane<S, NE, LPR>(v, row, sub, vr);
                if (y) {
                    alignas(16) S yr[NE];
                    load_lane<S, NE, LPR>(y, row, sub, yr);
#pragma unroll
                    for (int b = 0; b < VPL; ++b)
#pragma unroll
                        for (int c = 0; c < NC; ++c) ur[NC * b + c] = cy[b] * double(yr[NC * b + c]);
                } else {
#pragma unroll
                    for (int e = 0; e < NE; ++e) ur[e] = 0.0;
                }
#pragma unroll
                for (int b = 0; b < VPL; ++b)
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        const int e = NC * b + c;
                        const double vv = double(vr[e]);
                        const double xv = sx[b] * vv;
                        const double hv = sx[b] * (acc[e] + dsum * vv);
                        acc[e] = hv;     // keep H x for the reductions
                        xr[e] = xv;      // keep x for the reductions
                        ur[e] += ca * hv + cb * xv;
                    }
                if (u) {
                    alignas(16) S us[NE];
#pragma unroll
                    for (int e = 0; e < NE; ++e) us[e] = S(ur[e]);
                    store_lane<S, NE, LPR>(u, row, sub, us);
                }
            } else {
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    acc[e] = 0.0;
                    xr[e] = 0.0;
                    ur[e] = 0.0;
                }
            }
            // per-row products of the four reductions, one quantity at a time
            wave_reduce_quantities<VPL, LPR, NC, NE>(xr, acc, ur, wq, lane);
        }
    }
    if constexpr (EXPORT) return;

    // block sums: TAB 3 reuses its dynamic LDS (at least this size) once
    // every wavefront is done with the tables, the others a static array
    double (*sh)[kNQ][64];
    if constexpr (TAB == 3) {
        __syncthreads();
        sh = reinterpret_cast<double (*)[kNQ][64]>(lds_dyn);
    } else {
        __shared__ double sh_s[kWavesPerBlock][kNQ][64];
        sh = sh_s;
    }
#pragma unroll
    for (int k = 0; k < kNQ; ++k) sh[wave][k][lane] = wq[k];
    __syncthreads();
    if (int(threadIdx.x) < kNQ * B) {
        const int k = threadIdx.x / B, b = threadIdx.x % B;
        int bsub = 0, bi = 0;
        vec_lane<S, NE, LPR, NC>(b, bsub, bi);
        const int L = (bi << (6 - LOGV)) | bsub;
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) acc += sh[w][k][L];
        A.partials[size_t(blk) * (kNQ * B) + threadIdx.x] = acc;
    }
}

template <typename S, bool CPLX, bool CCOEF, bool SECTOR, int B, int LPR, bool W64, int TAB, bool EXPORT>
__global__ __launch_bounds__(kBlock) void hv_kernel(HvArgs A) {
    hv_body<S, CPLX, CCOEF, SECTOR, B, LPR, W64, TAB, EXPORT>(A, int(blockIdx.x), int(gridDim.x));
}

// Several problems in one launch (uneven sector sizes): problem p owns the
// blocks begin[p] .. begin[p+1]-1 (multiples of 8, so block & 7 still
// names the XCD) and its own partials.
template <typename S, bool CPLX, bool CCOEF, bool SECTOR, int B, int LPR, bool W64, int TAB>
__global__ __launch_bounds__(kBlock) void hv_multi_kernel(const HvArgs* __restrict__ probs,
                                                          const int* __restrict__ begin, int n_probs) {
    int p = 0;
    for (int q = 1; q < n_probs; ++q)
        if (int(blockIdx.x) >= begin[q]) p = q;
    const HvArgs A = probs[p];
    hv_body<S, CPLX, CCOEF, SECTOR, B, LPR, W64, TAB>(A, int(blockIdx.x) - begin[p], begin[p + 1] - begin[p]);
}

// ---------------------------------------------------------------------------
// Block-staged sector product (Sec. 3.1 basis, Sec. 3.3 product).
//
// The rows of a sector basis are grouped by their high half h: block h is the
// contiguous index range [h_row[k], h_row[k+1]), ordered by the low half.  A
// workgroup owns one block at a time and stages its values in LDS, in chunks
// of at most `chunk` rows when the block is larger, then for every row and
// operator (the operator's flip mask decides the case, uniformly):
//   * the flip stays in the low half: the target is in the same block, at the
//     rank the two-level low-rank table gives (in LDS); its values come from
//     the staged chunk, or from memory when they lie in another chunk;
//   * the flip leaves the low half alone: the target is the row of the same
//     rank in block h ^ m (one scalar J_hi load per operator and block), so
//     the lanes of a wavefront read consecutive rows;
//   * the flip touches both halves: rank from the LDS table, values gathered
//     from block h ^ m_hi in memory.
// The two-level low-rank table splits the low half l = (a, b), b its low b2
// bits: rank(l) = T1[a][class(l)] + T2[b], where T2[b] is the rank of b among
// the b2-bit strings of its class and T1[a][c] counts the class-c low halves
// whose upper part is below a -- the split-table search of Sec. 3.1 applied
// once more inside the low half, small enough for LDS.
struct HvsArgs {
    BasisDev bs;
    const DevOp* ops;    // padded to n_ops (a multiple of 4)
    int n_ops;
    int b2;              // low bits of the low half ranked by T2
    const double* ptab;  // [n_ops][4][Re c, Im c, d, 0]
    const uint32_t* t1;  // [2^(b_lo - b2)][ncls]
    const uint16_t* t2;  // [2^b2]
    int ncls;            // classes of a low half
    int cls_pairs;       // 1: class = (set even bits, set odd bits) (fermions at fixed up and down counts)
    int nsl;             // cls_pairs: sites of the low half; class index = n_even * (nsl + 1) + n_odd
    int pad;
    int64_t chunk;       // rows staged in LDS at a time
    const void* v;
    void* u;
    const void* y;
    const double* cy;
    const double* sx;
    double a, b;
    const int* stop;
    double* partials;
};

constexpr int kBlockS = 512;   // threads of the block-staged sector kernel


// LDS row of a staged chunk -> registers (one lane holds a whole row)
template <typename S, int NE>
__device__ __forceinline__ void lds_row(const char* p, S (&out)[NE]) {
    constexpr int RB = NE * int(sizeof(S));
    constexpr int CB = RB >= 16 ? 16 : RB;
#pragma unroll
    for (int j = 0; j < RB / CB; ++j) copy_chunk<CB>(reinterpret_cast<char*>(out) + j * CB, p + j * CB);
}

template <typename S, bool CPLX, bool CCOEF, int B, bool W64>
__global__ __launch_bounds__(kBlockS) void hvs_kernel(HvsArgs A) {
    using ST = typename StateT<W64>::type;
    constexpr int NC = CPLX ? 2 : 1;
    constexpr int NE = B * NC;                 // scalars of a row; one lane per row
    constexpr int RB = NE * int(sizeof(S));    // row bytes
    constexpr int UB = RB >= 16 ? 16 : RB;     // staging unit (rows start on multiples of it)
    constexpr int NW = kBlockS / 64;
    constexpr int LOGV = Log2<B>::value;
    if (A.stop && *A.stop) return;
    const int tid = int(threadIdx.x);
    const int lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);
    const BasisDev& bs = A.bs;
    const S* __restrict__ v = static_cast<const S*>(A.v);
    S* __restrict__ u = static_cast<S*>(A.u);
    const S* __restrict__ y = static_cast<const S*>(A.y);
    const ConstOp* ops = (const ConstOp*)(A.ops);
    typedef const __attribute__((address_space(4))) int64_t ConstI64;
    const ConstI64* jhi = (const ConstI64*)(bs.j_hi);
    const int n_ops = A.n_ops;
    const int b2 = A.b2;
    const uint32_t mask2 = (1u << b2) - 1u;
    const int ncls = A.ncls, cpairs = A.cls_pairs, nsl = A.nsl;

    // LDS (hvs_lds_layout): pattern table | T1 | T2 | staged chunk and one zero
    // row, each part 16-byte aligned
    double* tab = lds_dyn;
    const size_t tab_b = size_t(n_ops) * 16 * sizeof(double);
    const size_t t1_n = (size_t(1) << (bs.b_lo - b2)) * size_t(ncls);
    uint32_t* t1 = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(lds_dyn) + tab_b);
    uint16_t* t2 = reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(t1) + (t1_n * 4 + 15) / 16 * 16);
    const size_t t2_b = ((size_t(1) << b2) * 2 + 15) / 16 * 16;
    char* blk = reinterpret_cast<char*>(t2) + t2_b;
    for (size_t i = tid; i < tab_b / 8; i += kBlockS) tab[i] = A.ptab[i];
    for (size_t i = tid; i < t1_n; i += kBlockS) t1[i] = A.t1[i];
    for (size_t i = tid; i < (size_t(1) << b2); i += kBlockS) t2[i] = A.t2[i];
    for (int i = tid; i < RB / 4; i += kBlockS) reinterpret_cast<uint32_t*>(blk + A.chunk * RB)[i] = 0u;
    __syncthreads();
    auto low_rank = [&](uint32_t l) -> uint32_t {
        return t1[(l >> b2) * uint32_t(ncls) + uint32_t(low_class(l, cpairs, nsl))] + uint32_t(t2[l & mask2]);
    };

    double sx[B], cy[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        sx[b] = A.sx ? A.sx[b] : 1.0;
        cy[b] = (A.y && A.cy) ? A.cy[b] : 0.0;
    }
    const double ca = A.a, cb = A.b;
    double wq[kNQ] = {0.0, 0.0, 0.0, 0.0};
    alignas(16) S g[4][NE];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < NE; ++e) g[k][e] = S(0);

    for (int64_t kb = blockIdx.x; kb < bs.n_high; kb += gridDim.x) {
        const int64_t hrow = bs.h_row[kb];
        const int64_t rows = bs.h_row[kb + 1] - hrow;
        const uint64_t hval = bs.h_val[kb];
        const ST hbits = ST(hval << bs.b_lo);
        const uint32_t lobase = bs.h_lobase[kb];
        for (int64_t c0 = 0; c0 < rows; c0 += A.chunk) {
            const int64_t cn = rows - c0 < A.chunk ? rows - c0 : A.chunk;
            __syncthreads();   // every read of the previous chunk is done
            {
                const char* src = reinterpret_cast<const char*>(v) + size_t(hrow + c0) * RB;
                const int64_t units = cn * (RB / UB);
                for (int64_t i = tid; i < units; i += kBlockS) copy_chunk<UB>(blk + i * UB, src + i * UB);
            }
            __syncthreads();
            for (int64_t t0 = int64_t(wave) * 64; t0 < cn; t0 += NW * 64) {
                const bool valid = t0 + lane < cn;
                const int64_t r = c0 + t0 + lane;            // rank within the block
                const uint32_t l = valid ? bs.lows[lobase + r] : 0u;
                const ST s = hbits | ST(l);
                double acc[NE];
#pragma unroll
                for (int e = 0; e < NE; ++e) acc[e] = 0.0;
                double dsum = 0.0;
                for (int o = 0; o < n_ops; o += 4) {
                    double crk[4], cik[4];
                    int64_t ik[4];     // chunk offset (LDS) or row index (memory)
                    bool lk[4];        // value in the staged chunk
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const ConstOp& op = ops[o + k];
                        const uint32_t bi = op.bi, bj = op.bj;
                        const uint64_t xmask = op.xmask, smask = op.smask;
                        const uint32_t pat = bit_at<W64>(s, bi) | (bit_at<W64>(s, bj) << 1);
                        const double* te = tab + ((o + k) * 4 + int(pat)) * 4;
                        double cr = te[0];
                        double ci = CCOEF ? te[1] : 0.0;
                        dsum += te[2];
                        if (smask != 0 && parity_masked<W64>(s, smask)) {
                            cr = -cr;
                            ci = -ci;
                        }
                        const uint64_t xm_hi = xmask >> bs.b_lo;
                        const uint32_t xm_lo = uint32_t(xmask & bs.mask_lo);
                        bool live = valid;
                        if (xm_hi == 0) {
                            // target in this block: rank from the LDS table
                            const int64_t rk = xm_lo ? int64_t(low_rank(l ^ xm_lo)) : r;
                            const int64_t rel = rk - c0;
                            lk[k] = rel >= 0 && rel < cn;
                            ik[k] = lk[k] ? rel : hrow + rk;
                        } else {
                            const int64_t base_hi = jhi[hval ^ xm_hi];
                            live = live && base_hi >= 0;
                            ik[k] = base_hi + (xm_lo ? int64_t(low_rank(l ^ xm_lo)) : r);
                            lk[k] = false;
                        }
                        crk[k] = live ? cr : 0.0;
                        cik[k] = live ? ci : 0.0;
                    }
                    // lanes whose element is zero read a zero row (after the chunk in
                    // LDS, or in memory)
                    bool actk[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        actk[k] = CCOEF ? (crk[k] != 0.0 || cik[k] != 0.0) : (crk[k] != 0.0);
                        if (lk[k]) lds_row<S, NE>(blk + (actk[k] ? ik[k] : A.chunk) * RB, g[k]);
                        else load_lane_at<S, NE, 1>(row_or_zero<S, NE, 1>(v, ik[k], actk[k]), 0, g[k]);
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) accumulate<S, CPLX, CCOEF, B>(acc, g[k], actk[k], crk[k], cik[k]);
                }
                // epilogue: u = a * H x + b * x + cy * y with x = sx * v (own row from the chunk)
                double xr[NE], ur[NE];
                if (valid) {
                    alignas(16) S vr[NE];
                    lds_row<S, NE>(blk + (t0 + lane) * RB, vr);
                    if (y) {
                        alignas(16) S yr[NE];
                        load_lane<S, NE, 1>(y, hrow + r, 0, yr);
#pragma unroll
                        for (int b = 0; b < B; ++b)
#pragma unroll
                            for (int c = 0; c < NC; ++c) ur[NC * b + c] = cy[b] * double(yr[NC * b + c]);
                    } else {
#pragma unroll
                        for (int e = 0; e < NE; ++e) ur[e] = 0.0;
                    }
#pragma unroll
                    for (int b = 0; b < B; ++b)
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            const int e = NC * b + c;
                            const double vv = double(vr[e]);
                            const double xv = sx[b] * vv;
                            const double hv = sx[b] * (acc[e] + dsum * vv);
                            acc[e] = hv;
                            xr[e] = xv;
                            ur[e] += ca * hv + cb * xv;
                        }
                    if (u) {
                        alignas(16) S us[NE];
#pragma unroll
                        for (int e = 0; e < NE; ++e) us[e] = S(ur[e]);
                        store_lane<S, NE, 1>(u, hrow + r, 0, us);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < NE; ++e) {
                        acc[e] = 0.0;
                        xr[e] = 0.0;
                        ur[e] = 0.0;
                    }
                }
                wave_reduce_quantities<B, 1, NC, NE>(xr, acc, ur, wq, lane);
            }
        }
    }
    // block sums: lane (b << (6 - LOGV)) of each wavefront holds vector b's sums
    __shared__ double sh[NW][kNQ][kMaxNvec];
    if ((lane & ((64 >> LOGV) - 1)) == 0) {
        const int b = lane >> (6 - LOGV);
#pragma unroll
        for (int k = 0; k < kNQ; ++k) sh[wave][k][b] = wq[k];
    }
    __syncthreads();
    if (tid < kNQ * B) {
        const int k = tid / B, b = tid % B;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += sh[w][k][b];
        A.partials[size_t(blockIdx.x) * (kNQ * B) + tid] = s;
    }
}

// ---------------------------------------------------------------------------
// Windowed full-space product (one pass of a pass plan).
//
// Rows are visited in the order of a bit permutation of the row index: the
// processing index q is scattered to the configuration s by perm[k] (q bit
// k -> configuration bit).  The low bits of q are the pass's window, so
// all partner rows s ^ xmask of the pass's operators lie within the block
// of rows currently in flight.  mode bit 0: first pass (no partial sum to
// read); bit 1: last pass (epilogue and reductions).  Partial sums of H v
// (unscaled) travel through u between passes.
//
// Staged schedule: the configuration bits of a later pass's window are in
// general scattered over the row index, so its window rows lie far apart
// in memory and compete for a few L2 sets.  There, the previous pass also
// writes each row of v it visits to `stage` at the row's processing index
// in the next pass (inv_next maps configuration bits to those index bits),
// and the next pass gathers from that copy at q ^ xmask', where xmask' is
// the flip mask in processing-index bits: its window is then one
// contiguous block.
struct HvwArgs {
    const void* kops;    // KOp<S> records of this pass, a multiple of 4
    int kop_begin;
    int kop_end;
    const int32_t* perm;
    int nbits;
    int mode;
    int64_t n_tiles;
    const void* v;       // gather source: v (row index s) or a staged copy (index q)
    int g_q;             // 1: v is a staged copy indexed by the processing index
    void* stage;         // nullptr, or the staged copy of v for the next pass
    const int32_t* inv_next;   // [64] configuration bit -> next pass's index bit
    void* u;
    const void* y;
    const double* cy;
    const double* sx;
    double a, b;
    const int* stop;
    double* partials;
    int pass;            // index of this pass (element export)
    ExportArgs ex;
};

// Payload of the element export: the row's configuration in the first four
// bytes of a lane's share, so the on-chip partner paths (LDS tile, lane
// exchange) move configurations instead of values.
template <typename S, int NE>
__device__ __forceinline__ void export_payload(uint32_t s, S (&x)[NE]) {
#pragma unroll
    for (int e = 0; e < NE; ++e) x[e] = S(0);
    __builtin_memcpy(&x[0], &s, 4);
}

template <typename S, int NE>
__device__ __forceinline__ uint32_t export_config(const S (&x)[NE]) {
    uint32_t s;
    __builtin_memcpy(&s, &x[0], 4);
    return s;
}

// EXPORT: the element export of this pass's decode (no memory gathers and no
// output): records the target configuration of every operator of the pass --
// for partners inside the tile the configuration travels through the same LDS
// tile or lane exchange that carries values in the product -- its signed
// element, and the pass's diagonal sum.
template <typename S, bool CPLX, bool CCOEF, int B, int LPR, bool NT, bool EXPORT = false>
__global__ __launch_bounds__(kBlock) void hvw_kernel(HvwArgs A) {
    constexpr int NC = CPLX ? 2 : 1;
    constexpr int VPL = B / LPR;
    constexpr int NE = VPL * NC;
    constexpr int RPW = 64 / LPR;
    constexpr int LOGV = Log2<VPL>::value;
    constexpr int LOGL = Log2<LPR>::value;
    constexpr int LOGR = 6 - LOGL;          // row bits held by one wavefront pass
    // the wavefront's tile of v in LDS (rows of at most 128 bytes, at most 4
    // lanes per row): partners anywhere in the tile are read from there;
    // otherwise only partners within the rows of one wavefront pass are
    // exchanged between lanes
    constexpr int TRB = LaneLayout<S, NE, LPR>::RB;
    constexpr bool TL = tile_in_lds(TRB, LPR);
    constexpr int LOGT = TL ? 6 : LOGR;
    static_assert(VPL * LPR == B, "LPR must divide B");
    if (A.stop && *A.stop) return;
    const bool first = (A.mode & 1) != 0, last = (A.mode & 2) != 0;

    const int lane = threadIdx.x & 63;
    const int sub = lane & (LPR - 1);
    const int rlane = lane >> LOGL;
    const int wave = wave_uniform(threadIdx.x >> 6);
    const S* __restrict__ v = static_cast<const S*>(A.v);
    S* __restrict__ u = static_cast<S*>(A.u);
    const S* __restrict__ y = static_cast<const S*>(A.y);
    typedef const __attribute__((address_space(4))) KOp<double> ConstKOp;
    const ConstKOp* kops = (const ConstKOp*)(A.kops);
    typedef const __attribute__((address_space(4))) int32_t ConstI32;
    const ConstI32* perm = (const ConstI32*)(A.perm);
    const ConstI32* inv_next = (const ConstI32*)(A.inv_next);
    S* __restrict__ stg = static_cast<S*>(A.stage);
    const bool gq = A.g_q != 0;
    // next-pass index bit of each of the six in-tile index bits
    uint32_t nlm[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) nlm[k] = stg ? (1u << inv_next[perm[k]]) : 0u;

    const int xcd = blockIdx.x & 7;
    const int waves_x = int(gridDim.x >> 3) * kWavesPerBlock;
    const int wl = int(blockIdx.x >> 3) * kWavesPerBlock + wave;
    const int64_t T = A.n_tiles;
    const int64_t Tx = (T + 7) >> 3;
    const int64_t t_begin = xcd * Tx;
    const int64_t t_end = (t_begin + Tx < T) ? t_begin + Tx : T;

    double wq[kNQ] = {0.0, 0.0, 0.0, 0.0};

    // pattern table of this pass's operators in LDS: entry (o, p) holds
    // {c[p], d[p]} (real coefficients) or {c[p], ci[p], d[p], 0}; each lane
    // reads the entry of its own row pattern p (at most four distinct
    // addresses per operator across the wavefront)
    constexpr int TE = CCOEF ? 4 : 2;
    const int n_ops = A.kop_end - A.kop_begin;
    for (int i = int(threadIdx.x); i < n_ops * 4; i += kBlock) {
        const ConstKOp& rec = kops[A.kop_begin + (i >> 2)];
        const int q = i & 3;
        const double c0 = rec.c[0], c1 = rec.c[1], c2 = rec.c[2], c3 = rec.c[3];
        const double d0 = rec.d[0], d1 = rec.d[1], d2 = rec.d[2], d3 = rec.d[3];
        lds_dyn[i * TE] = sel4(q, c0, c1, c2, c3);
        if constexpr (CCOEF) {
            const double e0 = rec.ci[0], e1 = rec.ci[1], e2 = rec.ci[2], e3 = rec.ci[3];
            lds_dyn[i * TE + 1] = sel4(q, e0, e1, e2, e3);
            lds_dyn[i * TE + 2] = sel4(q, d0, d1, d2, d3);
            lds_dyn[i * TE + 3] = 0.0;
        } else {
            lds_dyn[i * TE + 1] = sel4(q, d0, d1, d2, d3);
        }
    }
    // the wavefront's row tile: 64 rows and a zero row (row 64) that lanes
    // whose element is zero read instead of a partner
    char* tb = reinterpret_cast<char*>(lds_dyn) + size_t(n_ops) * 4 * TE * sizeof(double) + size_t(wave) * 65 * TRB;
    if constexpr (TL) {
        for (int i = lane; i < TRB / 4; i += 64) reinterpret_cast<uint32_t*>(tb + 64 * TRB)[i] = 0u;
    }
    __syncthreads();

    // gathered rows: a lane whose element is zero reads zeros (the zero row in
    // memory or in the LDS tile) or its own lane, so non-finite entries stay
    // with the rows they couple to
    alignas(16) S g[4][NE];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < NE; ++e) g[k][e] = S(0);
    // the lane's chunk of row 0 of v and of the zero row, and its chunk offset in a tile row
    const char* const vsub = reinterpret_cast<const char*>(v) + sub * LaneLayout<S, NE, LPR>::CB;
    const char* const zsub = reinterpret_cast<const char*>(kZeroRow) + sub * LaneLayout<S, NE, LPR>::CB;
    const uint32_t sub_cb = uint32_t(sub * LaneLayout<S, NE, LPR>::CB);

    for (int64_t tile = t_begin + wl; tile < t_end; tile += waves_x) {
        // configuration bits of the tile index, and their next-pass index bits (uniform)
        uint32_t s_tile = 0, qn_tile = 0;
        for (int k = 6; k < A.nbits; ++k)
            if ((tile >> (k - 6)) & 1) {
                const int c = perm[k];
                s_tile |= 1u << c;
                if (stg) qn_tile |= 1u << inv_next[c];
            }
        if constexpr (TL) {
            // the tile's rows into LDS (LDS accesses of a wavefront complete in
            // order, so the reads of the previous tile are done)
            alignas(16) S tv[LPR][NE];
#pragma unroll
            for (int pass = 0; pass < LPR; ++pass) {
                const int r = pass * RPW + rlane;
                uint32_t s = s_tile;
#pragma unroll
                for (int k = 0; k < 6; ++k)
                    if ((r >> k) & 1) s |= 1u << perm[k];
                const uint32_t base = gq ? ((uint32_t(tile) << 6) | uint32_t(r)) : s;
                if constexpr (EXPORT) export_payload<S, NE>(s, tv[pass]);
                else load_lane<S, NE, LPR>(v, int64_t(base), sub, tv[pass]);
            }
#pragma unroll
            for (int pass = 0; pass < LPR; ++pass) tile_put<S, NE, LPR>(tb, pass * RPW + rlane, sub, tv[pass]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
#pragma unroll 1
        for (int pass = 0; pass < LPR; ++pass) {
            const int r = pass * RPW + rlane;      // position within the 64-row tile
            uint32_t s = s_tile, qn = qn_tile;
#pragma unroll
            for (int k = 0; k < 6; ++k)
                if ((r >> k) & 1) {
                    s |= 1u << perm[k];
                    qn |= nlm[k];
                }
            const int64_t row = int64_t(s);
            // index of this row in the gather source
            const uint32_t base = gq ? ((uint32_t(tile) << 6) | uint32_t(r)) : s;

            // the row's own values first (from the LDS tile, or from memory;
            // without the tile, partners within this wavefront pass are
            // exchanged from them between lanes)
            alignas(16) S vr[NE];
            if constexpr (TL) tile_get<S, NE, LPR>(tb, r, sub, vr);
            else if constexpr (EXPORT) export_payload<S, NE>(s, vr);
            else load_lane<S, NE, LPR>(v, int64_t(base), sub, vr);
            const bool ex_row = EXPORT && sub == 0 && int64_t(s) >= A.ex.row0 && int64_t(s) < A.ex.row0 + A.ex.nrows;
            double acc[NE];
#pragma unroll
            for (int e = 0; e < NE; ++e) acc[e] = 0.0;
            double dsum = 0.0;
            // operators in groups of 4: decode all, issue every gather, then
            // accumulate (FP64 coefficients and sums), with the wave priority of
            // the single-pass kernel's phases
            for (int o = 0; o < n_ops; o += 4) {
                if constexpr (!EXPORT) __builtin_amdgcn_s_setprio(1);
                double crk[4], cik[4];
                uint32_t tk[4];
                uint32_t smk[4];   // sign masks (uniform)
                bool lk[4];   // partner on chip: in the LDS tile, or in this wavefront pass (uniform)
                int xa[4];
                int opk[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const ConstKOp& rec = kops[A.kop_begin + o + k];
                    const uint32_t xm = rec.xm, sm = rec.sm, bi = rec.bi, bj = rec.bj, lq = rec.lq;
                    opk[k] = EXPORT ? rec.op : -1;
                    lk[k] = (lq >> LOGT) == 0u;
                    // partner: tile row r ^ lq, or the byte address of its lane
                    xa[k] = TL ? int(lq & 63u) : (lane ^ int(lq << LOGL)) << 2;
                    const uint32_t pat = __builtin_amdgcn_ubfe(s, bi, 1u) | (__builtin_amdgcn_ubfe(s, bj, 1u) << 1);
                    const double* te = lds_dyn + ((o + k) * 4 + int(pat)) * TE;
                    double cr = te[0], ci = 0.0;
                    if constexpr (CCOEF) {
                        ci = te[1];
                        dsum += te[2];
                    } else {
                        dsum += te[1];
                    }
                    smk[k] = sm;
                    crk[k] = cr;
                    cik[k] = ci;
                    tk[k] = base ^ xm;
                }
                if (__builtin_expect((smk[0] | smk[1] | smk[2] | smk[3]) != 0u, 0)) {
                    // fermion signs: flip the sign bits where the parity is odd
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int32_t sg = int32_t((__popc(s & smk[k]) & 1u) << 31);
                        crk[k] = __hiloint2double(__double2hiint(crk[k]) ^ sg, __double2loint(crk[k]));
                        if constexpr (CCOEF) cik[k] = __hiloint2double(__double2hiint(cik[k]) ^ sg, __double2loint(cik[k]));
                    }
                }
                if constexpr (EXPORT) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        uint32_t t = tk[k];
                        if (lk[k]) {
                            // the partner row's payload through the on-chip path
                            if constexpr (TL) tile_get<S, NE, LPR>(tb, r ^ int(xa[k]), sub, g[k]);
                            else exchange_lane<S, NE>(vr, xa[k], g[k]);
                            t = export_config<S, NE>(g[k]);
                        } else if (gq) {
                            // staged copy: tk is the partner's processing index
                            uint32_t c = 0;
                            for (int b = 0; b < A.nbits; ++b)
                                if ((t >> b) & 1u) c |= 1u << perm[b];
                            t = c;
                        }
                        if (ex_row && opk[k] >= 0) {
                            const size_t at = size_t(int64_t(s) - A.ex.row0) * size_t(A.ex.n_slots) + size_t(opk[k]);
                            A.ex.col[at] = int64_t(t);
                            A.ex.cr[at] = crk[k];
                            A.ex.ci[at] = cik[k];
                        }
                    }
                    continue;
                }
                bool actk[4];
                __builtin_amdgcn_s_setprio(2);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    actk[k] = CCOEF ? (crk[k] != 0.0 || cik[k] != 0.0) : (crk[k] != 0.0);
                    if (lk[k]) {
                        if constexpr (TL) tile_get_off<S, NE, LPR>(tb, tile_off<S, NE, LPR>(actk[k] ? (r ^ int(xa[k])) : 64, sub_cb), g[k]);
                        else exchange_lane<S, NE>(vr, actk[k] ? xa[k] : (lane << 2), g[k]);
                    } else {
                        load_sub_at<S, NE, LPR>(actk[k] ? vsub + size_t(tk[k]) * LaneLayout<S, NE, LPR>::RB : zsub, g[k]);
                    }
                }
                __builtin_amdgcn_s_setprio(0);
#pragma unroll
                for (int k = 0; k < 4; ++k) accumulate<S, CPLX, CCOEF, VPL>(acc, g[k], actk[k], crk[k], cik[k]);
            }

            if constexpr (EXPORT) {
                if (ex_row) A.ex.diag[size_t(int64_t(s) - A.ex.row0) * size_t(A.ex.n_pass) + size_t(A.pass)] = dsum;
                continue;
            }
            if (stg) {
                if constexpr (NT) store_lane_nt<S, NE, LPR>(stg, int64_t(qn), sub, vr);
                else store_lane<S, NE, LPR>(stg, int64_t(qn), sub, vr);
            }
#pragma unroll
            for (int e = 0; e < NE; ++e) acc[e] += dsum * double(vr[e]);   // raw (unscaled) H v of this pass
            if (!first) {
                alignas(16) S pr[NE];
                if constexpr (NT) load_lane_nt<S, NE, LPR>(u, row, sub, pr);
                else load_lane<S, NE, LPR>(u, row, sub, pr);
#pragma unroll
                for (int e = 0; e < NE; ++e) acc[e] += double(pr[e]);
            }
            if (!last) {
                alignas(16) S ps[NE];
#pragma unroll
                for (int e = 0; e < NE; ++e) ps[e] = S(acc[e]);
                if constexpr (NT) store_lane_nt<S, NE, LPR>(u, row, sub, ps);
                else store_lane<S, NE, LPR>(u, row, sub, ps);
                continue;
            }
            double ur[NE], xr[NE];
            if (y) {
                alignas(16) S yr[NE];
                load_lane<S, NE, LPR>(y, row, sub, yr);
#pragma unroll
                for (int b = 0; b < VPL; ++b) {
                    const double c = A.cy ? A.cy[lane_vec<S, NE, LPR, NC>(sub, b)] : 0.0;
#pragma unroll
                    for (int c2 = 0; c2 < NC; ++c2) ur[NC * b + c2] = c * double(yr[NC * b + c2]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < NE; ++e) ur[e] = 0.0;
            }
            const double ca = A.a, cb = A.b;
#pragma unroll
            for (int b = 0; b < VPL; ++b) {
                const double sc = A.sx ? A.sx[lane_vec<S, NE, LPR, NC>(sub, b)] : 1.0;
#pragma unroll
                for (int c2 = 0; c2 < NC; ++c2) {
                    const int e = NC * b + c2;
                    const double xv = sc * double(vr[e]);
                    const double hv = sc * acc[e];
                    acc[e] = hv;
                    xr[e] = xv;
                    ur[e] += ca * hv + cb * xv;
                }
            }
            if (u) {
                alignas(16) S us[NE];
#pragma unroll
                for (int e = 0; e < NE; ++e) us[e] = S(ur[e]);
                if constexpr (NT) store_lane_nt<S, NE, LPR>(u, row, sub, us);
                else store_lane<S, NE, LPR>(u, row, sub, us);
            }
            wave_reduce_quantities<VPL, LPR, NC, NE>(xr, acc, ur, wq, lane);
        }
    }
    if (!last || EXPORT) return;
    __shared__ double sh[kWavesPerBlock][kNQ][64];
#pragma unroll
    for (int k = 0; k < kNQ; ++k) sh[wave][k][lane] = wq[k];
    __syncthreads();
    if (int(threadIdx.x) < kNQ * B) {
        const int k = threadIdx.x / B, b = threadIdx.x % B;
        int bsub = 0, bi = 0;
        vec_lane<S, NE, LPR, NC>(b, bsub, bi);
        const int L = (bi << (6 - LOGV)) | bsub;
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) acc += sh[w][k][L];
        A.partials[size_t(blockIdx.x) * (kNQ * B) + threadIdx.x] = acc;
    }
}

// ---- dense-block (CMA) product.  Stage c: for every block of D = 2^M rows
// that share the configuration bits outside cluster c, U_blk += H_c V_blk,
// where V_blk is D rows x RC real columns (the interleaved vectors, complex
// parts as separate columns; H_c is real).  A workgroup stages H_c in LDS
// once, then per block gathers the D rows through the cluster's bit
// positions into LDS and multiplies with 16x16x4 MFMA tiles (FP32 for FP32
// storage, FP64 for FP64 storage): wave w takes the 16-row tiles w, w+4, ...
// and every 16-column tile.  The stage result is added to u (written on the
// first stage), in the storage type.
struct CmaArgs {
    const void* v;
    void* u;
    const void* h;         // [D][D] dense partial Hamiltonian of this stage (S)
    const int32_t* bits;   // [64]: local bit -> configuration bit, then the block-index bits
    int nbits;
    int first;             // stage 0: write u instead of adding to it
    int last;              // last stage: apply a, b, the input scale and the reductions
    int64_t n_blocks;
    double a, b;
    const double* sx;      // [nvec] input scale or nullptr
    double* partials;      // last stage: [grid][kNQ * nvec] block sums, or nullptr
};

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <typename S>
struct MfmaAcc;
// Operand layouts (both): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].
// Result register r of lane l is D[row(l, r)][l % 16]; the row mapping
// differs between the FP32 and FP64 instructions (checked on gfx950).
template <>
struct MfmaAcc<float> {
    using type = f32x4_t;
    static __device__ __forceinline__ type step(float a, float b, type c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <>
struct MfmaAcc<double> {
    using type = f64x4_t;
    static __device__ __forceinline__ type step(double a, double b, type c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename S, int RC, int M>
struct CmaShape {
    static constexpr int D = 1 << M;
    static constexpr int NT = (RC + 15) / 16;                   // 16-column tiles
    static constexpr int RB = RC * int(sizeof(S));               // bytes of one row of the block
    static constexpr int CB = RB >= 16 ? 16 : RB;                // copy chunk
    static constexpr int CPR = RB / CB;                          // chunks per row
    static constexpr int EPC = CB / int(sizeof(S));              // scalars per chunk
    // V_blk row stride (scalars): 16-byte aligned, and for FP32 the four
    // 16-lane groups of an operand read land on different bank halves
    static constexpr int VLD = sizeof(S) == 4 ? (NT * 16 + ((NT & 1) ? 0 : 16)) : NT * 16 + 2;
    // output tile row stride: 16-byte aligned, rows 4 apart on other banks
    static constexpr int OLD = sizeof(S) == 4 ? ((RC + 3) / 4 * 4 + 4) : (RC + 1) / 2 * 2 + 2;
    static constexpr int TPW = (D / 16 + kWavesPerBlock - 1) / kWavesPerBlock;   // row tiles per wave
    static constexpr size_t lds_bytes = (size_t(D) * VLD + size_t(D) * OLD) * sizeof(S) + size_t(D) * 4;
};

template <int CB>
struct ChunkT;
template <>
struct ChunkT<16> {
    using type = uint4;
};
template <>
struct ChunkT<8> {
    using type = uint2;
};
template <>
struct ChunkT<4> {
    using type = uint32_t;
};

// Stage kernel.  Per block: the rows were gathered into V_blk (LDS) by the
// previous iteration; each wave multiplies its 16-row tiles of H_c (held in
// registers for the whole launch) by V_blk, writes the tile to the output
// tile in LDS; after a barrier the block adds the output tile to u row by
// row (16-byte accesses) while gathering the next block's rows.  The last
// stage also finishes the product there: with x = s v (the row's own values
// are in V_blk) and h the accumulated H v, it stores a h + b x and sums the
// four FP64 quantities per vector (a thread's chunk always holds the same
// vectors; wave shuffles, then a fixed-order block sum).
template <typename S, bool CPLX, int RC, int M>
__global__ __launch_bounds__(kBlock) void cma_kernel(CmaArgs A) {
    using Sh = CmaShape<S, RC, M>;
    constexpr int D = Sh::D, NT = Sh::NT, VLD = Sh::VLD, OLD = Sh::OLD, TPW = Sh::TPW;
    constexpr int CB = Sh::CB, CPR = Sh::CPR, EPC = Sh::EPC;
    using Chunk = typename ChunkT<CB>::type;
    static_assert(kBlock % CPR == 0, "chunks of a row divide the block");
    constexpr int RPI = kBlock / CPR;                            // rows per copy step
    constexpr int NC = CPLX ? 2 : 1;
    constexpr int B = RC / NC;                                   // vectors
    constexpr int VPT = EPC / NC;                                // vectors in a thread's chunk
    static_assert(VPT >= 1 && EPC % NC == 0, "a chunk holds whole elements");
    S* vs = reinterpret_cast<S*>(lds_dyn);
    S* os = vs + size_t(D) * VLD;
    uint32_t* lcfg = reinterpret_cast<uint32_t*>(os + size_t(D) * OLD);
    const S* __restrict__ v = static_cast<const S*>(A.v);
    S* __restrict__ u = static_cast<S*>(A.u);
    const S* __restrict__ h = static_cast<const S*>(A.h);
    typedef const __attribute__((address_space(4))) int32_t ConstI32;
    const ConstI32* bits = (const ConstI32*)(A.bits);
    const int tid = int(threadIdx.x);
    const int lane = tid & 63;
    const int wave = wave_uniform(tid >> 6);

    // the wave's A operands for the whole launch: lane holds
    // H_c[rt*16 + lane % 16][4k + lane / 16], k = 0 .. D/4 - 1
    S ha[TPW][D / 4];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int rt = wave + t * kWavesPerBlock;
#pragma unroll
        for (int k = 0; k < D / 4; ++k)
            ha[t][k] = rt < D / 16 ? h[size_t(rt * 16 + (lane & 15)) * D + 4 * k + (lane >> 4)] : S(0);
    }
    for (int r = tid; r < D; r += kBlock) {
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < M; ++j)
            if ((r >> j) & 1) c |= 1u << bits[j];
        lcfg[r] = c;
    }
    // padding columns of V_blk are read by the last column tile and never change
    if constexpr (NT * 16 > RC) {
        constexpr int PADC = NT * 16 - RC;
        for (int i = tid; i < D * PADC; i += kBlock) vs[(i / PADC) * VLD + RC + i % PADC] = S(0);
    }

    const int xcd = blockIdx.x & 7;
    const int64_t per_x = (A.n_blocks + 7) >> 3;
    const int64_t b_begin = xcd * per_x;
    const int64_t b_end = (b_begin + per_x < A.n_blocks) ? b_begin + per_x : A.n_blocks;
    const int64_t b_step = gridDim.x >> 3;
    const int c_row = tid / CPR, c_chunk = tid % CPR;
    double scl[VPT];
    double q[kNQ][VPT];
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
        scl[j] = (A.last && A.sx) ? A.sx[c_chunk * VPT + j] : 1.0;
#pragma unroll
        for (int k = 0; k < kNQ; ++k) q[k][j] = 0.0;
    }
    auto block_bits = [&](int64_t blk) {
        uint32_t sb = 0;
        for (int j = 0; j < A.nbits - M; ++j)
            if ((blk >> j) & 1) sb |= 1u << bits[M + j];
        return sb;
    };
    auto gather = [&](uint32_t sb) {
#pragma unroll 4
        for (int r0 = 0; r0 < D; r0 += RPI) {
            const int r = r0 + c_row;
            if (RPI <= D || r < D) {
                const Chunk w = *reinterpret_cast<const Chunk*>(v + size_t(sb | lcfg[r]) * RC + c_chunk * EPC);
                *reinterpret_cast<Chunk*>(vs + r * VLD + c_chunk * EPC) = w;
            }
        }
    };

    __syncthreads();   // lcfg ready
    int64_t blk = b_begin + (blockIdx.x >> 3);
    uint32_t sb = blk < b_end ? block_bits(blk) : 0u;
    if (blk < b_end) gather(sb);
    __syncthreads();
    for (; blk < b_end; blk += b_step) {
        // multiply: independent accumulators per row tile and column tile
        typename MfmaAcc<S>::type acc[TPW][NT];
#pragma unroll
        for (int t = 0; t < TPW; ++t)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[t][nt] = {S(0), S(0), S(0), S(0)};
        const S* vb = vs + (lane >> 4) * VLD + (lane & 15);
#pragma unroll
        for (int k = 0; k < D / 4; ++k) {
            S b[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) b[nt] = vb[4 * k * VLD + nt * 16];
#pragma unroll
            for (int t = 0; t < TPW; ++t)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[t][nt] = MfmaAcc<S>::step(ha[t][k], b[nt], acc[t][nt]);
        }
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const int rt = wave + t * kWavesPerBlock;
            if (rt >= D / 16) continue;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int col = nt * 16 + (lane & 15);
                if (col < RC) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) os[(rt * 16 + MfmaAcc<S>::row(lane, i)) * OLD + col] = acc[t][nt][i];
                }
            }
        }
        __syncthreads();   // output tile complete; V_blk free
        // add the output tile to u, and gather the next block
        const uint32_t sb_cur = sb;
        const int64_t nxt = blk + b_step;
        if (nxt < b_end) sb = block_bits(nxt);
#pragma unroll 2
        for (int r0 = 0; r0 < D; r0 += RPI) {
            const int r = r0 + c_row;
            if (RPI <= D || r < D) {
                S* dst = u + size_t(sb_cur | lcfg[r]) * RC + c_chunk * EPC;
                alignas(16) S o[EPC];
                *reinterpret_cast<Chunk*>(o) = *reinterpret_cast<const Chunk*>(os + r * OLD + c_chunk * EPC);
                if (!A.first) {
                    alignas(16) S p[EPC];
                    *reinterpret_cast<Chunk*>(p) = *reinterpret_cast<const Chunk*>(dst);
#pragma unroll
                    for (int e = 0; e < EPC; ++e) o[e] = S(o[e] + p[e]);
                }
                if (A.last) {
                    // the row's own values: this thread's chunk of V_blk (only this
                    // thread rewrites it, in the gather below)
                    alignas(16) S x[EPC];
                    *reinterpret_cast<Chunk*>(x) = *reinterpret_cast<const Chunk*>(vs + r * VLD + c_chunk * EPC);
#pragma unroll
                    for (int j = 0; j < VPT; ++j) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) {
                            const int e = j * NC + c;
                            const double hv = scl[j] * double(o[e]);
                            const double xv = scl[j] * double(x[e]);
                            const double ov = A.a * hv + A.b * xv;
                            o[e] = S(ov);
                            q[0][j] += xv * xv;
                            q[1][j] += xv * hv;
                            q[2][j] += hv * hv;
                            q[3][j] += ov * ov;
                        }
                    }
                }
                *reinterpret_cast<Chunk*>(dst) = *reinterpret_cast<const Chunk*>(o);
            }
        }
        if (nxt < b_end) gather(sb);
        __syncthreads();   // next V_blk in place; output tile free
    }
    if (!A.last || !A.partials) return;
    // lanes that share c_chunk hold the same vectors: reduce over the others
    __shared__ double red[kWavesPerBlock][kNQ][kMaxNvec];
#pragma unroll
    for (int k = 0; k < kNQ; ++k)
#pragma unroll
        for (int j = 0; j < VPT; ++j) {
            double t = q[k][j];
#pragma unroll
            for (int off = CPR; off < 64; off <<= 1) t += __shfl_xor(t, off, 64);
            if (lane < CPR) red[wave][k][lane * VPT + j] = t;
        }
    __syncthreads();
    if (tid < kNQ * B) {
        const int k = tid / B, vec = tid % B;
        double acc = 0.0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) acc += red[w][k][vec];
        A.partials[size_t(blockIdx.x) * (kNQ * B) + tid] = acc;
    }
}

// out[q] = sum over g of partials[g * nq + q], fixed order.  A non-finite
// sum sets `bit` in the problem's sticky flag word (if given).
__device__ __forceinline__ void reduce_body(const double* __restrict__ partials, int n_parts, int nq, int q,
                                            double* __restrict__ out, int32_t* flag, int32_t bit) {
    double s = 0.0;
    for (int g = threadIdx.x; g < n_parts; g += 256) s += partials[size_t(g) * nq + q];
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[q] = sh[0];
        if (flag && !isfinite(sh[0])) atomicOr(flag, bit);
    }
}

// one block per quantity q
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partials, int n_parts,
                                                              int nq, double* __restrict__ out,
                                                              const int* stop, int32_t* flag, int32_t bit) {
    if (stop && *stop) return;
    reduce_body(partials, n_parts, nq, int(blockIdx.x), out, flag, bit);
}

// several problems: block p * nq + q reduces quantity q of problem p
__global__ __launch_bounds__(256) void reduce_multi_kernel(const RedDesc* __restrict__ d, int nq) {
    const int p = int(blockIdx.x) / nq, q = int(blockIdx.x) % nq;
    const double* partials = d[p].partials;
    const int n_parts = d[p].n_parts;
    double* out = d[p].out;
    const int* stop = d[p].stop;
    if (stop && *stop) return;
    reduce_body(partials, n_parts, nq, q, out, d[p].flag, nq == 1 ? HPHI_NONFINITE_NORM : HPHI_NONFINITE_PRODUCT);
}

// ---- element lists from the records of an export: per row the diagonal (sum
// of the passes' diagonal parts, in pass order) if nonzero, then the nonzero
// off-diagonal elements in the order of the Hamiltonian's operator list
__global__ __launch_bounds__(256) void elements_compact_kernel(ExportArgs ex, const DevOp* __restrict__ ops, int cap,
                                                               int64_t* __restrict__ cols, double* __restrict__ re,
                                                               double* __restrict__ im, int32_t* __restrict__ term,
                                                               int32_t* __restrict__ counts) {
    const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (r >= ex.nrows) return;
    double dsum = 0.0;
    for (int p = 0; p < ex.n_pass; ++p) dsum += ex.diag[size_t(r) * ex.n_pass + p];
    const size_t out = size_t(r) * cap;
    int n = 0;
    if (dsum != 0.0) {
        if (n < cap) {
            cols[out + n] = ex.row0 + r;
            re[out + n] = dsum;
            im[out + n] = 0.0;
            term[out + n] = -1;
        }
        ++n;
    }
    const size_t rb = size_t(r) * ex.n_slots;
    for (int o = 0; o < ex.n_slots; ++o) {
        const double cr = ex.cr[rb + o], ci = ex.ci[rb + o];
        if (cr == 0.0 && ci == 0.0) continue;
        if (n < cap) {
            cols[out + n] = ex.col[rb + o];
            re[out + n] = cr;
            im[out + n] = ci;
            term[out + n] = ops[o].term;
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
        ok = int(__popcll(c)) == ta;
    } else if (sector == HPHI_SECTOR_NUP_NDN) {
        ok = int(__popcll(c & 0x5555555555555555ull)) == ta && int(__popcll(c & 0xAAAAAAAAAAAAAAAAull)) == tb;
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

// y += c2 * x, |y|^2; optionally acc += ecoef * x (FP64 accumulator);
// block blk of nblk, one partial per block
template <typename S>
__device__ __forceinline__ void update_body(S* __restrict__ y, const S* __restrict__ x, int64_t n,
                                            const double* __restrict__ c2p, double* __restrict__ acc,
                                            const double* __restrict__ ecp, double* __restrict__ partials,
                                            int blk, int nblk) {
    const double c2 = *c2p;
    const double ec = acc ? *ecp : 0.0;
    double s = 0.0;
    for (int64_t i = int64_t(blk) * 256 + threadIdx.x; i < n; i += int64_t(nblk) * 256) {
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
    if (threadIdx.x == 0) partials[blk] = sh[0];
}

template <typename S>
__global__ __launch_bounds__(256) void lanczos_update_kernel(S* __restrict__ y, const S* __restrict__ x, int64_t n,
                                                             const double* __restrict__ c2p,
                                                             double* __restrict__ acc,
                                                             const double* __restrict__ ecp,
                                                             double* __restrict__ partials, const int* stop) {
    if (stop && *stop) return;
    update_body<S>(y, x, n, c2p, acc, ecp, partials, int(blockIdx.x), int(gridDim.x));
}

// several problems: problem p owns blocks begin[p] .. begin[p+1]-1
template <typename S>
__global__ __launch_bounds__(256) void lanczos_update_multi_kernel(const UpdDesc* __restrict__ d,
                                                                   const int* __restrict__ begin, int n_probs) {
    int p = 0;
    for (int q = 1; q < n_probs; ++q)
        if (int(blockIdx.x) >= begin[q]) p = q;
    const UpdDesc D = d[p];
    if (D.stop && *D.stop) return;
    update_body<S>(static_cast<S*>(D.y), static_cast<const S*>(D.x), D.n, D.c2, D.acc, D.ec, D.partials,
                   int(blockIdx.x) - begin[p], begin[p + 1] - begin[p]);
}

// w = a x + b y over n FP64 scalars (w may alias x or y), |w|^2 partials per block
__global__ __launch_bounds__(256) void lincomb_kernel(double* w, const double* x, const double* y, int64_t n,
                                                      double a, double b, double* __restrict__ partials) {
    double s = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
        const double v = a * x[i] + b * y[i];
        w[i] = v;
        s += v * v;
    }
    __shared__ double sh[256];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (int(threadIdx.x) < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void fill_zero_kernel(uint32_t* __restrict__ p, int64_t n_words) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n_words; i += int64_t(gridDim.x) * 256) p[i] = 0u;
}

// <O> = Re<x|Ox> / <x|x> per vector, and <x|x>
__global__ void expect_kernel(const double* __restrict__ red, double* __restrict__ out, int nvec) {
    const int b = threadIdx.x;
    if (b >= nvec) return;
    const double xx = red[0 * nvec + b], xo = red[1 * nvec + b];
    out[b] = xo / xx;
    out[nvec + b] = xx;
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

// TPQ observables of a step inside a run: the step number lives on the
// device (graph replays advance it); the scale of the produced state goes
// to the slot of this step's parity, where the next step reads it.
__global__ void tpq_obs_run_kernel(const double* __restrict__ red, TpqRunState* st, double* __restrict__ obs_log,
                                   int nvec, double ns, double l) {
    const int b = threadIdx.x;
    const int j = st->j;
    if (b < nvec) {
        const double xx = red[0 * nvec + b], xh = red[1 * nvec + b], hh = red[2 * nvec + b],
                     uu = red[3 * nvec + b];
        const double uk = xh / xx / ns;
        double* o = obs_log + size_t(j) * 4 * nvec;
        o[0 * nvec + b] = uk;
        o[1 * nvec + b] = hh / xx / (ns * ns);
        o[2 * nvec + b] = (2.0 * double(st->k - 1) / ns) / (l - uk);
        const double s = 1.0 / sqrt(uu);
        o[3 * nvec + b] = s;
        st->scale[j & 1][b] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->j = j + 1;
        st->k = st->k + 1;
    }
}

__global__ void tpq_run_init_kernel(TpqRunState* st, int k0) {
    if (threadIdx.x == 0) {
        st->k = k0;
        st->j = 0;
    }
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

// The scalar steps of one recurrence (the caller has checked sc->stop):
// after the product, alpha_k and the update's coefficients; after the
// update, beta_{k+1}, the stop test and the next step's scales
__device__ void lz_after_hv_step(LzScalars* sc, const double* red, double* alpha, const double* evec) {
    const double a = red[1];          // Re<v_k|H v_k>, v_k = s_cur * X
    alpha[sc->k] = a;
    sc->c2 = -a * sc->s_cur;
    sc->ecoef = evec ? evec[sc->k] * sc->s_cur : 0.0;
}

__device__ void lz_after_update_step(LzScalars* sc, const double* red, double* beta, const double* alpha) {
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

// The product's kNQ sums of one recurrence, reduced by one block with the
// summation order of reduce_body (so they are bitwise those of
// reduce_partials_kernel); thread 0 writes them and the flag.
__device__ __forceinline__ void reduce_nq_body(const double* __restrict__ partials, int n_parts,
                                               double* __restrict__ out, int32_t* flag) {
    const int t = int(threadIdx.x);
    double s[kNQ];
#pragma unroll
    for (int q = 0; q < kNQ; ++q) s[q] = 0.0;
    for (int g = t; g < n_parts; g += 256)
#pragma unroll
        for (int q = 0; q < kNQ; ++q) s[q] += partials[size_t(g) * kNQ + q];
    __shared__ double sh[kNQ][256];
#pragma unroll
    for (int q = 0; q < kNQ; ++q) sh[q][t] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int q = 0; q < kNQ; ++q) sh[q][t] += sh[q][t + w];
        __syncthreads();
    }
    if (t == 0)
        for (int q = 0; q < kNQ; ++q) {
            out[q] = sh[q][0];
            if (flag && !isfinite(sh[q][0])) atomicOr(flag, HPHI_NONFINITE_PRODUCT);
        }
}

// One recurrence: the product's sums and the scalar step that reads them, in
// one launch (the step reads the sums thread 0 has just written)
__global__ __launch_bounds__(256) void reduce_lz_after_hv_kernel(const double* __restrict__ partials, int n_parts,
                                                                 double* __restrict__ out, int32_t* flag,
                                                                 LzScalars* sc, double* alpha, const double* evec) {
    if (sc->stop) return;
    reduce_nq_body(partials, n_parts, out, flag);
    if (threadIdx.x == 0) lz_after_hv_step(sc, out, alpha, evec);
}

// the update's |y|^2 and the scalar step that reads it, in one launch
__global__ __launch_bounds__(256) void reduce_lz_after_update_kernel(const double* __restrict__ partials, int n_parts,
                                                                     double* __restrict__ out, int32_t* flag,
                                                                     LzScalars* sc, double* beta, const double* alpha) {
    if (sc->stop) return;
    reduce_body(partials, n_parts, 1, 0, out, flag, HPHI_NONFINITE_NORM);
    if (threadIdx.x == 0) lz_after_update_step(sc, out, beta, alpha);
}

// the same for several recurrences: block p takes problem p (d[p]: its
// partials and sums; alpha/beta/evec: `stride` per problem)
__global__ __launch_bounds__(256) void reduce_lz_after_hv_multi_kernel(const RedDesc* __restrict__ d, LzScalars* scs,
                                                                       double* alphas, const double* evecs, int stride) {
    const int p = int(blockIdx.x);
    LzScalars* sc = scs + p;
    if (sc->stop) return;
    reduce_nq_body(d[p].partials, d[p].n_parts, d[p].out, d[p].flag);
    if (threadIdx.x == 0)
        lz_after_hv_step(sc, d[p].out, alphas + size_t(stride) * p, evecs ? evecs + size_t(stride) * p : nullptr);
}

__global__ __launch_bounds__(256) void reduce_lz_after_update_multi_kernel(const RedDesc* __restrict__ d,
                                                                           LzScalars* scs, double* betas,
                                                                           const double* alphas, int stride) {
    const int p = int(blockIdx.x);
    LzScalars* sc = scs + p;
    if (sc->stop) return;
    reduce_body(d[p].partials, d[p].n_parts, 1, 0, d[p].out, d[p].flag, HPHI_NONFINITE_NORM);
    if (threadIdx.x == 0)
        lz_after_update_step(sc, d[p].out, betas + size_t(stride) * p, alphas + size_t(stride) * p);
}

}  // namespace

// ------------------------------------------------------------------ launchers

// the product's sums (and, for one Lanczos recurrence, the scalar step that
// reads them)
static int launch_product_reduce(const hphi_ham* H, int n_parts, int B, const HvLaunch& L, hipStream_t st) {
    if (L.lz_sc) {
        if (B != 1) return set_error(HPHI_EINVAL, "Lanczos step fused with the reduction needs one vector");
        reduce_lz_after_hv_kernel<<<1, 256, 0, st>>>(H->d_partials, n_parts, L.reduce_out, H->d_flag, L.lz_sc,
                                                     L.lz_alpha, L.lz_evec);
    } else {
        reduce_partials_kernel<<<kNQ * B, 256, 0, st>>>(H->d_partials, n_parts, kNQ * B, L.reduce_out, L.stop,
                                                      H->d_flag, HPHI_NONFINITE_PRODUCT);
    }
    return check_hip(hipGetLastError(), "reduce launch");
}

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

// Persistent grid: the blocks that can be resident at once (capped by the
// schedule's blocks per CU), so the tiles in flight on an XCD form one
// contiguous front; a multiple of 8, capped by the work available.
template <typename Kernel>
static int occupancy_blocks(Kernel k) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kBlock, 0) != hipSuccess || nb < 1) nb = 1;
    return nb;
}

static int cu_count() {
    static const int n = [] {
        int dev = 0, ncu = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
            ncu = 256;
        return ncu;
    }();
    return n;
}

static int make_grid(int occ, const Schedule& sc, int64_t tiles) {
    int per_cu = occ;
    if (sc.blocks_per_cu > 0 && sc.blocks_per_cu < per_cu) per_cu = sc.blocks_per_cu;
    int64_t g = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t resident = int64_t(per_cu) * cu_count();
    if (g > resident) g = resident;
    if (g > kMaxGrid) g = kMaxGrid;
    g = ((g + 7) / 8) * 8;
    return int(g);
}

// LDS the single-pass product stages for this problem (0 = tables stay global)
static size_t hv_stage_bytes(const hphi_ham* H, bool sector) {
    size_t b = size_t(H->n_ops_pad) * 16 * sizeof(double);
    if (sector) {
        const int b_lo = H->basis->dev.b_lo;
        if (b_lo > 20) return kLdsStageBytes + 1;
        b += (size_t(1) << b_lo) * 4;
    }
    return b;
}

// resident blocks per CU once `lds` bytes of dynamic LDS are taken
static int occupancy_with_lds(int occ, size_t lds, size_t stat = 8 * 1024) {
    constexpr size_t kLdsPerCu = 160 * 1024;
    const int by_lds = int(kLdsPerCu / (lds + stat));
    return by_lds < occ ? (by_lds < 1 ? 1 : by_lds) : occ;
}

template <typename S, bool CPLX, bool CCOEF, bool SECTOR, int B, int LPR, bool W64, int TAB, bool EX>
static int launch_hv_g(const HvLaunch& L, const Schedule& sc, size_t lds, hipStream_t st) {
    const hphi_ham* H = L.ham;
    static const int occ = occupancy_blocks(hv_kernel<S, CPLX, CCOEF, SECTOR, B, LPR, W64, TAB, EX>);
    const int64_t tiles = EX ? L.ex->t1 - L.ex->t0 : H->basis->dev.n_tiles;
    const int grid = make_grid(occupancy_with_lds(occ, lds, TAB == 3 ? 0 : 8 * 1024), sc, tiles < 1 ? 1 : tiles);
    HvArgs A;
    A.bs = H->basis->dev;
    A.ops = H->d_ops;
    A.n_ops = H->n_ops_pad;
    A.ptab = H->d_ptab;
    A.v = L.v;
    A.u = L.u;
    A.y = L.y;
    A.cy = L.cy;
    A.sx = L.sx;
    A.a = L.a;
    A.b = L.b;
    A.stop = L.stop;
    A.partials = H->d_partials;
    if constexpr (EX) A.ex = *L.ex;
    if constexpr (TAB == 3) {
        const hphi_basis* Bs = H->basis;
        A.t1c = Bs->d_t1c;
        A.t2p = Bs->d_t2p;
        A.b2 = Bs->lr_b2;
        A.n2 = Bs->lr_n2;
        A.cls_pairs = Bs->lr_pairs;
        A.w2 = Bs->lr_b2 / 2 + 1;
    }
    hv_kernel<S, CPLX, CCOEF, SECTOR, B, LPR, W64, TAB, EX><<<grid, kBlock, lds, st>>>(A);
    int rc = check_hip(hipGetLastError(), "hv_kernel launch");
    if (rc) return rc;
    if (!EX && L.reduce_out) rc = launch_product_reduce(H, grid, B, L, st);
    return rc;
}

// Table placement: 0 = pattern table and low rank table in LDS, 1 = both read
// from global memory, 2 = pattern table in LDS and the (large) low rank
// table from global memory.
template <typename S, bool CPLX, bool CCOEF, bool SECTOR, int B, int LPR, bool W64, bool EX>
static int launch_hv_t(const HvLaunch& L, const Schedule& sc, hipStream_t st) {
    const size_t ptab = size_t(L.ham->n_ops_pad) * 16 * sizeof(double);
    if constexpr (!W64) {
        const size_t lds = hv_stage_bytes(L.ham, SECTOR);
        if (sc.stage_tables && lds <= kLdsStageBytes)
            return launch_hv_g<S, CPLX, CCOEF, SECTOR, B, LPR, W64, 0, EX>(L, sc, lds, st);
    }
    if constexpr (SECTOR && W64) {
        // the two-level low-rank table in LDS (16-bit entries) when it fits
        const hphi_basis* Bs = L.ham->basis;
        if (sc.stage_tables == 1 && Bs->d_t1c) {
            const size_t n1 = (size_t(1) << (Bs->b_lo - Bs->lr_b2)) * size_t(Bs->lr_n2);
            // at least the block-sum array, which this variant keeps in the same space
            const size_t lds = std::max(ptab + (n1 + 7) / 8 * 16 + (size_t(1) << Bs->lr_b2) * 2,
                                        size_t(kWavesPerBlock) * kNQ * 64 * sizeof(double));
            if (lds <= kLdsStageBytes) return launch_hv_g<S, CPLX, CCOEF, SECTOR, B, LPR, W64, 3, EX>(L, sc, lds, st);
        }
    }
    if constexpr (SECTOR) {
        if (sc.stage_tables && ptab <= kLdsStageBytes)
            return launch_hv_g<S, CPLX, CCOEF, SECTOR, B, LPR, W64, 2, EX>(L, sc, ptab, st);
    }
    return launch_hv_g<S, CPLX, CCOEF, SECTOR, B, LPR, W64, 1, EX>(L, sc, 0, st);
}

template <typename S, bool CPLX, bool CCOEF, bool SECTOR, int B, bool EX>
static int launch_hv_l(const HvLaunch& L, const Schedule& sc, hipStream_t st) {
    const bool w64 = L.ham->basis->nbits > 32;
    if (w64) {
        if constexpr (B <= 4) {
            if constexpr (B >= 2)
                if (sc.lpr == 2) return launch_hv_t<S, CPLX, CCOEF, SECTOR, B, 2, true, EX>(L, sc, st);
            if constexpr (B >= 4)
                if (sc.lpr == 4) return launch_hv_t<S, CPLX, CCOEF, SECTOR, B, 4, true, EX>(L, sc, st);
            return launch_hv_t<S, CPLX, CCOEF, SECTOR, B, 1, true, EX>(L, sc, st);
        }
        return set_error(HPHI_EINVAL, "nvec > 4 needs a space of at most 32 bits");
    }
    if constexpr (B >= 2) {
        switch (sc.lpr) {
            case 2: return launch_hv_t<S, CPLX, CCOEF, SECTOR, B, 2, false, EX>(L, sc, st);
            case 4:
                if constexpr (B >= 4) return launch_hv_t<S, CPLX, CCOEF, SECTOR, B, 4, false, EX>(L, sc, st);
                break;
            case 8:
                if constexpr (B >= 8) return launch_hv_t<S, CPLX, CCOEF, SECTOR, B, 8, false, EX>(L, sc, st);
                break;
        }
    }
    return launch_hv_t<S, CPLX, CCOEF, SECTOR, B, 1, false, EX>(L, sc, st);
}

template <typename S, bool CPLX, bool CCOEF, bool SECTOR, bool EX>
static int launch_hv_b(const HvLaunch& L, const Schedule& sc, hipStream_t st) {
    switch (L.nvec) {
        case 1: return launch_hv_l<S, CPLX, CCOEF, SECTOR, 1, EX>(L, sc, st);
        case 2: return launch_hv_l<S, CPLX, CCOEF, SECTOR, 2, EX>(L, sc, st);
        case 4: return launch_hv_l<S, CPLX, CCOEF, SECTOR, 4, EX>(L, sc, st);
        case 8: return launch_hv_l<S, CPLX, CCOEF, SECTOR, 8, EX>(L, sc, st);
        case 16: return launch_hv_l<S, CPLX, CCOEF, SECTOR, 16, EX>(L, sc, st);
    }
    return set_error(HPHI_EINVAL, "nvec must be 1, 2, 4, 8 or 16 (got %d)", L.nvec);
}

// ---- block-staged sector launches
// LDS bytes of the block-staged sector kernel for `chunk` staged rows
static size_t hvs_lds_layout(const hphi_ham* H, int row_bytes, int64_t chunk) {
    const hphi_basis* Bs = H->basis;
    const size_t tab = size_t(H->n_ops_pad) * 16 * sizeof(double);
    const size_t t1 = ((size_t(1) << (Bs->b_lo - Bs->lr_b2)) * size_t(Bs->lr_ncls) * 4 + 15) / 16 * 16;
    const size_t t2 = ((size_t(1) << Bs->lr_b2) * 2 + 15) / 16 * 16;
    return tab + t1 + t2 + size_t(chunk + 1) * size_t(row_bytes);
}

template <typename S, bool CPLX, bool CCOEF, int B, bool W64>
static int launch_hvs_t(const HvLaunch& L, int per_cu, hipStream_t st) {
    const hphi_ham* H = L.ham;
    const hphi_basis* Bs = H->basis;
    constexpr int RB = B * (CPLX ? 2 : 1) * int(sizeof(S));
    constexpr size_t kStatic = size_t(kBlockS / 64) * kNQ * kMaxNvec * sizeof(double);
    const size_t fixed = hvs_lds_layout(H, RB, 0);
    const size_t budget = size_t(160 * 1024) / size_t(per_cu);
    if (fixed + kStatic + 64 * size_t(RB) > budget) return 1;
    int64_t chunk = int64_t((budget - fixed - kStatic) / RB);
    if (chunk > Bs->max_block_rows) chunk = Bs->max_block_rows;
    // test hook: HPHI_SECTOR_CHUNK caps the staged rows (blocks then span several chunks)
    if (const char* e = std::getenv("HPHI_SECTOR_CHUNK")) {
        const int64_t cap = std::atoll(e);
        if (cap >= 1 && cap < chunk) chunk = cap;
    }
    const size_t lds = hvs_lds_layout(H, RB, chunk);
    int64_t grid = int64_t(per_cu) * cu_count();
    if (grid > Bs->dev.n_high) grid = Bs->dev.n_high;
    if (grid > kMaxGrid) grid = kMaxGrid;
    HvsArgs A;
    A.bs = Bs->dev;
    A.ops = H->d_ops;
    A.n_ops = H->n_ops_pad;
    A.b2 = Bs->lr_b2;
    A.ptab = H->d_ptab;
    A.t1 = Bs->d_t1;
    A.t2 = Bs->d_t2;
    A.ncls = Bs->lr_ncls;
    A.cls_pairs = Bs->lr_pairs;
    A.nsl = Bs->lr_nsl;
    A.pad = 0;
    A.chunk = chunk;
    A.v = L.v;
    A.u = L.u;
    A.y = L.y;
    A.cy = L.cy;
    A.sx = L.sx;
    A.a = L.a;
    A.b = L.b;
    A.stop = L.stop;
    A.partials = H->d_partials;
    hvs_kernel<S, CPLX, CCOEF, B, W64><<<int(grid), kBlockS, lds, st>>>(A);
    int rc = check_hip(hipGetLastError(), "hvs_kernel launch");
    if (rc) return rc;
    if (L.reduce_out) rc = launch_product_reduce(H, int(grid), B, L, st);
    return rc;
}

// the block-staged sector product when the schedule asks for it and its
// tables fit in LDS; 1 if not applicable
template <typename S, bool CPLX, bool CCOEF>
static int try_launch_hvs(const HvLaunch& L, const Schedule& sc, hipStream_t st) {
    const hphi_basis* Bs = L.ham->basis;
    if (Bs->dev.sector == 0 || !Bs->d_t1 || L.ex || L.nvec > 4 || L.ham->has_cond) return 1;
    const bool w64 = Bs->nbits > 32;
    if (sc.sector_blocks != 1) return 1;
    const int per_cu = sc.blocks_per_cu > 0 ? (sc.blocks_per_cu < 3 ? sc.blocks_per_cu : 3) : 2;
    auto go = [&](auto bconst) -> int {
        constexpr int B = decltype(bconst)::value;
        return w64 ? launch_hvs_t<S, CPLX, CCOEF, B, true>(L, per_cu, st)
                   : launch_hvs_t<S, CPLX, CCOEF, B, false>(L, per_cu, st);
    };
    switch (L.nvec) {
        case 1: return go(std::integral_constant<int, 1>{});
        case 2: return go(std::integral_constant<int, 2>{});
        case 4: return go(std::integral_constant<int, 4>{});
    }
    return 1;
}

// ---- windowed full-space launches
template <typename S, bool CPLX, bool CCOEF, int B, int LPR, bool NT, bool EX>
static int launch_hvw_t(const HvLaunch& L, const PassPlan* P, const Schedule& sc, bool staged, void* const* stage,
                        hipStream_t st) {
    const hphi_ham* H = L.ham;
    static const int occ = occupancy_blocks(hvw_kernel<S, CPLX, CCOEF, B, LPR, NT, EX>);
    // dynamic LDS: the pass's pattern table, then one row tile per wavefront
    constexpr int NE = (B / LPR) * (CPLX ? 2 : 1);
    constexpr int TRB = LaneLayout<S, NE, LPR>::RB;
    constexpr size_t tile_lds = tile_in_lds(TRB, LPR) ? size_t(kWavesPerBlock) * 65 * TRB : 0;
    auto lds_of = [&](int p) {
        return size_t(P->kop_begin[p + 1] - P->kop_begin[p]) * 4 * (CCOEF ? 4 : 2) * sizeof(double) + tile_lds;
    };
    size_t lds_max = 0;
    for (int p = 0; p < P->n_pass; ++p) lds_max = std::max(lds_max, lds_of(p));
    const int grid = make_grid(occupancy_with_lds(occ, lds_max), sc, H->basis->dev.n_tiles);
    HvwArgs A;
    A.nbits = H->basis->nbits;
    A.n_tiles = H->basis->dev.n_tiles;
    A.v = L.v;
    A.u = L.u;
    A.y = L.y;
    A.cy = L.cy;
    A.sx = L.sx;
    A.a = L.a;
    A.b = L.b;
    A.stop = L.stop;
    A.partials = H->d_partials;
    if constexpr (EX) {
        A.ex = *L.ex;
        if (P->n_pass > A.ex.n_pass) return set_error(HPHI_EINVAL, "element export: too many passes in the plan");
    } else {
        if (P->n_pass > 1 && !L.u) return set_error(HPHI_EINVAL, "multi-pass product needs an output buffer");
        if (staged && !stage[0]) return set_error(HPHI_EINVAL, "staged product without staging buffers");
    }
    for (int p = 0; p < P->n_pass; ++p) {
        const bool next = !EX && staged && p + 1 < P->n_pass;
        A.pass = p;
        A.kops = staged ? P->d_kopq : P->d_kop64;
        A.kop_begin = P->kop_begin[p];
        A.kop_end = P->kop_begin[p + 1];
        A.perm = P->d_perm + size_t(p) * 64;
        A.mode = (p == 0 ? 1 : 0) | (p == P->n_pass - 1 ? 2 : 0);
        A.v = (staged && p > 0 && !EX) ? stage[(p - 1) & 1] : L.v;
        A.g_q = (staged && p > 0) ? 1 : 0;
        A.stage = next ? stage[p & 1] : nullptr;
        A.inv_next = next ? P->d_inv + size_t(p + 1) * 64 : nullptr;
        hvw_kernel<S, CPLX, CCOEF, B, LPR, NT, EX><<<grid, kBlock, lds_of(p), st>>>(A);
        int rc = check_hip(hipGetLastError(), "hvw_kernel launch");
        if (rc) return rc;
    }
    if (!EX && L.reduce_out) return launch_product_reduce(H, grid, B, L, st);
    return HPHI_OK;
}

template <typename S, bool CPLX, bool CCOEF, int B, bool EX>
static int launch_hvw_b(const HvLaunch& L, const PassPlan* P, const Schedule& sc, bool staged, void* const* stage,
                        hipStream_t st) {
    if constexpr (B >= 8) {
        // streaming hints change no index or value: the export takes the plain variant
        if (sc.nt_streams && !EX) {
            switch (sc.lpr) {
                case 2: return launch_hvw_t<S, CPLX, CCOEF, B, 2, true, false>(L, P, sc, staged, stage, st);
                case 4: return launch_hvw_t<S, CPLX, CCOEF, B, 4, true, false>(L, P, sc, staged, stage, st);
                case 8: return launch_hvw_t<S, CPLX, CCOEF, B, 8, true, false>(L, P, sc, staged, stage, st);
            }
        }
        switch (sc.lpr) {
            case 2: return launch_hvw_t<S, CPLX, CCOEF, B, 2, false, EX>(L, P, sc, staged, stage, st);
            case 4: return launch_hvw_t<S, CPLX, CCOEF, B, 4, false, EX>(L, P, sc, staged, stage, st);
            case 8: return launch_hvw_t<S, CPLX, CCOEF, B, 8, false, EX>(L, P, sc, staged, stage, st);
        }
    }
    return launch_hvw_t<S, CPLX, CCOEF, B, 1, false, EX>(L, P, sc, staged, stage, st);
}

// windowed product when it applies (full space, <= 32 bits, no in-place
// extra input across several passes); returns 1 if not applicable
template <typename S, bool CPLX, bool CCOEF, bool EX>
static int try_launch_hvw(const HvLaunch& L, const Schedule& sc, hipStream_t st) {
    const hphi_basis* Bs = L.ham->basis;
    if (!sc.windowed || Bs->dev.sector != 0 || Bs->nbits > 32 || Bs->nbits < 6 || L.ham->has_cond) return 1;
    const int row_bytes = L.nvec * int(sizeof(S)) * (CPLX ? 2 : 1);
    const PassPlan* P = get_plan(L.ham, row_bytes, sc.window_kb, sc.max_passes, !L.no_alloc);
    if (!P) return 1;
    // several passes carry partial sums through u: they need a real output
    // buffer that is not also an input
    if (!EX && P->n_pass > 1 && (!L.u || L.y)) return 1;
    // the pattern table of a pass lives in LDS: at most kMaxPassOps operators,
    // and with the row tiles (rows of at most 128 bytes with the lanes per row
    // launch_hvw_b will use) and the kernel's static block-sum array within
    // the 160 KB of a workgroup
    const int lpr = (L.nvec >= 8 && (sc.lpr == 2 || sc.lpr == 4 || sc.lpr == 8)) ? sc.lpr : 1;
    const size_t tile_lds = tile_in_lds(row_bytes, lpr) ? size_t(kWavesPerBlock) * 65 * row_bytes : 0;
    constexpr size_t static_lds = size_t(kWavesPerBlock) * kNQ * 64 * sizeof(double);
    for (int p = 0; p < P->n_pass; ++p) {
        const int n = P->kop_begin[p + 1] - P->kop_begin[p];
        const size_t table = size_t(n) * 4 * (CCOEF ? 4 : 2) * sizeof(double);
        if (n > kMaxPassOps || table + tile_lds + static_lds > 160 * 1024) return 1;
    }
    bool staged = sc.windowed == 2 && P->n_pass > 1;
    void* stage[2] = {nullptr, nullptr};
    if (staged && !EX) {
        // staging buffers are allocated on first use; never inside a graph capture
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        (void)hipStreamIsCapturing(st, &cs);
        const size_t bytes = size_t(Bs->dim) * size_t(row_bytes);
        const int count = P->n_pass > 2 ? 2 : 1;
        bool have = true;
        for (int i = 0; i < count; ++i) have = have && L.ham->stage_bytes[i] >= bytes;
        if (((cs != hipStreamCaptureStatusNone || L.no_alloc) && !have) || get_stage_buffers(L.ham, bytes, count, stage))
            staged = false;
    }
    switch (L.nvec) {
        case 1: return launch_hvw_b<S, CPLX, CCOEF, 1, EX>(L, P, sc, staged, stage, st);
        case 2: return launch_hvw_b<S, CPLX, CCOEF, 2, EX>(L, P, sc, staged, stage, st);
        case 4: return launch_hvw_b<S, CPLX, CCOEF, 4, EX>(L, P, sc, staged, stage, st);
        case 8: return launch_hvw_b<S, CPLX, CCOEF, 8, EX>(L, P, sc, staged, stage, st);
        case 16: return launch_hvw_b<S, CPLX, CCOEF, 16, EX>(L, P, sc, staged, stage, st);
    }
    return 1;
}

template <typename S, bool CPLX, bool CCOEF, bool EX>
static int launch_hv_s2(const HvLaunch& L, hipStream_t st) {
    const Schedule sc = L.sched ? *L.sched : schedule_for(L.ham, L.nvec, L.dtype);
    const int w = try_launch_hvw<S, CPLX, CCOEF, EX>(L, sc, st);
    if (w != 1) return w;
    if constexpr (!EX) {
        const int b = try_launch_hvs<S, CPLX, CCOEF>(L, sc, st);
        if (b != 1) return b;
    }
    if (L.ham->basis->dev.sector != 0) return launch_hv_b<S, CPLX, CCOEF, true, EX>(L, sc, st);
    return launch_hv_b<S, CPLX, CCOEF, false, EX>(L, sc, st);
}

// the product, or (L.ex set) the element export through the same kernels and
// schedule; exports are instantiated for the complex storage types
template <typename S, bool CPLX, bool CCOEF>
static int launch_hv_s(const HvLaunch& L, hipStream_t st) {
    if (L.ex) {
        if constexpr (CPLX) return launch_hv_s2<S, CPLX, CCOEF, true>(L, st);
        return set_error(HPHI_EINVAL, "element export: use a complex storage type (C128 or C64)");
    }
    return launch_hv_s2<S, CPLX, CCOEF, false>(L, st);
}

// ---- dense-block product launch
template <typename S, bool CPLX, int RC, int M>
static int launch_cma_stages(const HvLaunch& L, const CmaPlan* P, hipStream_t st) {
    using Sh = CmaShape<S, RC, M>;
    const hphi_ham* H = L.ham;
    const size_t lds = Sh::lds_bytes;
    int dev = 0, max_lds = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        max_lds = 64 * 1024;
    if (lds > size_t(max_lds))
        return set_error(HPHI_EINVAL, "dense-block product: %d-bit clusters need %zu bytes of LDS", M, lds);
    static const int occ = occupancy_blocks(cma_kernel<S, CPLX, RC, M>);
    const int per_cu = occupancy_with_lds(occ, lds);
    CmaArgs A;
    A.v = L.v;
    A.u = L.u;
    A.nbits = H->basis->nbits;
    A.n_blocks = int64_t(1) << (A.nbits - M);
    A.a = L.a;
    A.b = L.b;
    A.sx = L.sx;
    A.partials = L.reduce_out ? H->d_partials : nullptr;
    int64_t g = int64_t(per_cu) * cu_count();
    if (g > A.n_blocks) g = A.n_blocks;
    g = ((g + 7) / 8) * 8;
    if (g > kMaxGrid) g = kMaxGrid;
    const size_t D2 = size_t(1) << (2 * M);
    for (int c = 0; c < P->n_stage; ++c) {
        A.h = std::is_same<S, float>::value ? static_cast<const void*>(P->d_hf + c * D2)
                                            : static_cast<const void*>(P->d_hd + c * D2);
        A.bits = P->d_bits + size_t(c) * 64;
        A.first = c == 0 ? 1 : 0;
        A.last = c == P->n_stage - 1 ? 1 : 0;
        cma_kernel<S, CPLX, RC, M><<<int(g), kBlock, lds, st>>>(A);
        const int rc = check_hip(hipGetLastError(), "cma_kernel launch");
        if (rc) return rc;
    }
    if (!L.reduce_out) return HPHI_OK;
    constexpr int B = RC / (CPLX ? 2 : 1);
    reduce_partials_kernel<<<kNQ * B, 256, 0, st>>>(H->d_partials, int(g), kNQ * B, L.reduce_out, nullptr, H->d_flag,
                                                      HPHI_NONFINITE_PRODUCT);
    return check_hip(hipGetLastError(), "reduce launch");
}

template <typename S, bool CPLX, int RC>
static int launch_cma_m(const HvLaunch& L, const CmaPlan* P, hipStream_t st) {
    switch (P->M) {
        case 4: return launch_cma_stages<S, CPLX, RC, 4>(L, P, st);
        case 5: return launch_cma_stages<S, CPLX, RC, 5>(L, P, st);
        case 6: return launch_cma_stages<S, CPLX, RC, 6>(L, P, st);
        case 7:
            if constexpr (sizeof(S) == 4) return launch_cma_stages<S, CPLX, RC, 7>(L, P, st);
            break;
    }
    return set_error(HPHI_EINVAL, "dense-block product: cluster_bits %d not supported for this dtype", P->M);
}

template <typename S, bool CPLX, int B>
static int launch_cma_b(const HvLaunch& L, const CmaPlan* P, hipStream_t st) {
    return launch_cma_m<S, CPLX, B * (CPLX ? 2 : 1)>(L, P, st);
}

template <typename S, bool CPLX>
static int launch_cma_s(const HvLaunch& L, const CmaPlan* P, hipStream_t st) {
    switch (L.nvec) {
        case 1: return launch_cma_b<S, CPLX, 1>(L, P, st);
        case 2: return launch_cma_b<S, CPLX, 2>(L, P, st);
        case 4: return launch_cma_b<S, CPLX, 4>(L, P, st);
        case 8: return launch_cma_b<S, CPLX, 8>(L, P, st);
        case 16: return launch_cma_b<S, CPLX, 16>(L, P, st);
    }
    return set_error(HPHI_EINVAL, "nvec must be 1, 2, 4, 8 or 16 (got %d)", L.nvec);
}

int launch_hv_cma(const HvLaunch& L, const CmaPlan* P, hipStream_t st) {
    switch (L.dtype) {
        case HPHI_F64: return launch_cma_s<double, false>(L, P, st);
        case HPHI_F32: return launch_cma_s<float, false>(L, P, st);
        case HPHI_C128: return launch_cma_s<double, true>(L, P, st);
        case HPHI_C64: return launch_cma_s<float, true>(L, P, st);
    }
    return set_error(HPHI_EINVAL, "bad dtype %d", L.dtype);
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

int launch_elements_compact(const hphi_ham* H, const ExportArgs& ex, int cap, int64_t* cols, double* re, double* im,
                            int32_t* term, int32_t* counts, hipStream_t st) {
    const int64_t blocks = (ex.nrows + 255) / 256;
    elements_compact_kernel<<<dim3(unsigned(blocks)), 256, 0, st>>>(ex, H->d_ops, cap, cols, re, im, term, counts);
    return check_hip(hipGetLastError(), "elements_compact launch");
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
                     int32_t* flag, hipStream_t st) {
    const int64_t ns = n * (dtype_complex(dtype) ? 2 : 1);
    if (grid <= 0) grid = stream_grid(ns);
    if (dtype == HPHI_F64 || dtype == HPHI_C128)
        copy_norm_kernel<double><<<grid, 256, 0, st>>>((const double*)src, (double*)dst, ns, partials);
    else
        copy_norm_kernel<float><<<grid, 256, 0, st>>>((const float*)src, (float*)dst, ns, partials);
    int rc = check_hip(hipGetLastError(), "copy_norm launch");
    if (rc) return rc;
    reduce_partials_kernel<<<1, 256, 0, st>>>(partials, grid, 1, red, nullptr, flag, HPHI_NONFINITE_NORM);
    return check_hip(hipGetLastError(), "reduce launch");
}

int launch_lanczos_update(void* y, const void* x, int64_t n, int dtype, const double* c2, void* acc,
                          const double* ecoef, double* partials, int grid, double* red, const int* stop,
                          int32_t* flag, hipStream_t st) {
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
    reduce_partials_kernel<<<1, 256, 0, st>>>(partials, grid, 1, red, stop, flag, HPHI_NONFINITE_NORM);
    return check_hip(hipGetLastError(), "reduce launch");
}

int launch_lanczos_update_lz(void* y, const void* x, int64_t n, int dtype, LzScalars* sc, void* acc,
                             double* partials, int grid, double* red, double* beta, const double* alpha,
                             int32_t* flag, hipStream_t st) {
    const int64_t ns = n * (dtype_complex(dtype) ? 2 : 1);
    if (grid <= 0) grid = stream_grid(ns);
    const int* stop = &sc->stop;
    if (dtype == HPHI_F64 || dtype == HPHI_C128)
        lanczos_update_kernel<double><<<grid, 256, 0, st>>>((double*)y, (const double*)x, ns, &sc->c2, (double*)acc,
                                                            &sc->ecoef, partials, stop);
    else
        lanczos_update_kernel<float><<<grid, 256, 0, st>>>((float*)y, (const float*)x, ns, &sc->c2, (double*)acc,
                                                           &sc->ecoef, partials, stop);
    int rc = check_hip(hipGetLastError(), "lanczos_update launch");
    if (rc) return rc;
    reduce_lz_after_update_kernel<<<1, 256, 0, st>>>(partials, grid, red, flag, sc, beta, alpha);
    return check_hip(hipGetLastError(), "reduce launch");
}

int launch_lincomb(double* w, const double* x, const double* y, int64_t n, double a, double b, double* partials,
                   double* norm2, hipStream_t st) {
    const int grid = stream_grid(n);
    lincomb_kernel<<<grid, 256, 0, st>>>(w, x, y, n, a, b, partials);
    int rc = check_hip(hipGetLastError(), "lincomb launch");
    if (rc || !norm2) return rc;
    reduce_partials_kernel<<<1, 256, 0, st>>>(partials, grid, 1, norm2, nullptr, nullptr, 0);
    return check_hip(hipGetLastError(), "reduce launch");
}

int launch_fill_zero(void* p, int64_t bytes, hipStream_t st) {
    const int64_t words = bytes / 4;
    fill_zero_kernel<<<stream_grid(words), 256, 0, st>>>((uint32_t*)p, words);
    return check_hip(hipGetLastError(), "fill_zero launch");
}

int launch_expect(const double* red, double* out, int nvec, hipStream_t st) {
    expect_kernel<<<1, 64, 0, st>>>(red, out, nvec);
    return check_hip(hipGetLastError(), "expect launch");
}

int launch_tpq_obs(const double* red, double* obs, int nvec, double n_sites, double l, int k, hipStream_t st) {
    tpq_obs_kernel<<<1, 64, 0, st>>>(red, obs, nvec, n_sites, l, k);
    return check_hip(hipGetLastError(), "tpq_obs launch");
}

// The allocation-free TPQ run keeps its state here: one per device, for the
// life of the process (272 bytes).  Host code never names it directly: the
// name is a host-side stand-in, so its device address is resolved per device.
static __device__ __align__(256) TpqRunState scratch;

int tpq_static_state(TpqRunState** out) {
    static std::mutex mu;
    static TpqRunState* addr[64] = {};
    int dev = 0;
    if (int rc = check_hip(hipGetDevice(&dev), "hphi_tpq_run_noalloc: current device")) return rc;
    if (dev < 0 || dev >= 64) return set_error(HPHI_EDEVICE, "hphi_tpq_run_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        if (int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hphi_tpq_run_noalloc: state address"))
            return rc;
        addr[dev] = static_cast<TpqRunState*>(p);
    }
    *out = addr[dev];
    return HPHI_OK;
}

int launch_tpq_run_init(TpqRunState* s, int k0, hipStream_t st) {
    tpq_run_init_kernel<<<1, 64, 0, st>>>(s, k0);
    return check_hip(hipGetLastError(), "tpq_run_init launch");
}

int launch_tpq_obs_run(const double* red, TpqRunState* s, double* obs_log, int nvec, double n_sites, double l,
                       hipStream_t st) {
    tpq_obs_run_kernel<<<1, 64, 0, st>>>(red, s, obs_log, nvec, n_sites, l);
    return check_hip(hipGetLastError(), "tpq_obs_run launch");
}

int launch_lz_init(LzScalars* sc, const double* red, double tol, int n_max, hipStream_t st) {
    lz_init_kernel<<<1, 1, 0, st>>>(sc, red, tol, n_max);
    return check_hip(hipGetLastError(), "lz_init launch");
}

// ---------------------------------------------------------------- batched

template <typename S, bool CPLX, bool CCOEF, bool SECTOR, bool W64, int TAB>
static int hv_multi_go(const MultiPlan& P, hipStream_t st) {
    hv_multi_kernel<S, CPLX, CCOEF, SECTOR, 1, 1, W64, TAB><<<P.grid, kBlock, P.lds, st>>>(
        static_cast<const HvArgs*>(P.d_args), P.d_begin, P.n);
    return check_hip(hipGetLastError(), "hv_multi launch");
}

template <typename S, bool CPLX, bool CCOEF>
static int hv_multi_s(const MultiPlan& P, hipStream_t st) {
    if (P.w64) {
        if (P.sector) return hv_multi_go<S, CPLX, CCOEF, true, true, 1>(P, st);
        return hv_multi_go<S, CPLX, CCOEF, false, true, 1>(P, st);
    }
    if (P.sector)
        return P.gtab ? hv_multi_go<S, CPLX, CCOEF, true, false, 1>(P, st)
                      : hv_multi_go<S, CPLX, CCOEF, true, false, 0>(P, st);
    return P.gtab ? hv_multi_go<S, CPLX, CCOEF, false, false, 1>(P, st)
                  : hv_multi_go<S, CPLX, CCOEF, false, false, 0>(P, st);
}

static int hv_multi_product(const MultiPlan& P, hipStream_t st) {
    switch (P.dtype) {
        case HPHI_F64: return hv_multi_s<double, false, false>(P, st);
        case HPHI_F32: return hv_multi_s<float, false, false>(P, st);
        case HPHI_C128: return P.cc ? hv_multi_s<double, true, true>(P, st) : hv_multi_s<double, true, false>(P, st);
        case HPHI_C64: return P.cc ? hv_multi_s<float, true, true>(P, st) : hv_multi_s<float, true, false>(P, st);
    }
    return set_error(HPHI_EINVAL, "bad dtype %d", P.dtype);
}

int hv_multi_launch(const MultiPlan& P, const LzMulti* lz, hipStream_t st) {
    int rc = hv_multi_product(P, st);
    if (rc) return rc;
    if (lz)
        reduce_lz_after_hv_multi_kernel<<<P.n, 256, 0, st>>>(P.d_red, lz->sc, lz->alpha, lz->evec, lz->stride);
    else
        reduce_multi_kernel<<<P.n * kNQ, 256, 0, st>>>(P.d_red, kNQ);
    return check_hip(hipGetLastError(), "reduce_multi launch");
}

int hv_multi_prepare(const HvLaunch* Ls, int n, MultiPlan* out) {
    if (n < 1 || !out) return set_error(HPHI_EINVAL, "hv_multi_prepare: no problems");
    MultiPlan P;
    P.n = n;
    P.dtype = Ls[0].dtype;
    P.cc = Ls[0].ham->is_complex;
    P.sector = Ls[0].ham->basis->dev.sector != 0;
    P.w64 = Ls[0].ham->basis->nbits > 32;
    size_t lds = 0;
    int64_t tiles_total = 0;
    for (int p = 0; p < n; ++p) {
        const HvLaunch& L = Ls[p];
        if (L.nvec != 1 || L.dtype != P.dtype || L.ham->is_complex != P.cc ||
            (L.ham->basis->dev.sector != 0) != P.sector || (L.ham->basis->nbits > 32) != P.w64)
            return set_error(HPHI_EINVAL, "hv_multi_prepare: problems differ in dtype, coefficients or space kind");
        const size_t b = hv_stage_bytes(L.ham, P.sector);
        if (b > lds) lds = b;
        tiles_total += L.ham->basis->dev.n_tiles;
    }
    const Schedule sc = schedule_for(Ls[0].ham, 1, P.dtype);
    P.gtab = P.w64 || !sc.stage_tables || lds > kLdsStageBytes;
    P.lds = P.gtab ? 0 : lds;
    // blocks: the grid is persistent, so it must fit the resident blocks;
    // every problem gets one group of 8 blocks and the rest is shared in
    // proportion to the tiles (largest remainders first), never more than
    // its tiles can use
    int occ = 1;
    if (P.gtab)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, hv_multi_kernel<double, false, false, true, 1, 1, false, true>, kBlock, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, hv_multi_kernel<double, false, false, true, 1, 1, false, false>, kBlock, 0);
    if (occ < 1) occ = 1;
    int per_cu = occupancy_with_lds(occ, P.lds);
    if (sc.blocks_per_cu > 0 && sc.blocks_per_cu < per_cu) per_cu = sc.blocks_per_cu;
    const int64_t groups = std::max<int64_t>(n, int64_t(per_cu) * cu_count() / 8);
    std::vector<int64_t> units(n, 1), cap(n);
    std::vector<double> frac(n, 0.0);
    int64_t left = groups - n;
    for (int p = 0; p < n; ++p) {
        const int64_t t = Ls[p].ham->basis->dev.n_tiles;
        cap[p] = std::max<int64_t>(1, ((t + kWavesPerBlock - 1) / kWavesPerBlock + 7) / 8);
        const double share = tiles_total > 0 ? double(groups - n) * double(t) / double(tiles_total) : 0.0;
        const int64_t whole = std::min<int64_t>(int64_t(share), cap[p] - 1);
        units[p] += whole;
        frac[p] = share - double(int64_t(share));
        left -= whole;
    }
    std::vector<int> order(n);
    for (int p = 0; p < n; ++p) order[p] = p;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return frac[a] > frac[b] || (frac[a] == frac[b] && a < b); });
    for (int k = 0; k < n && left > 0; ++k)
        if (units[order[k]] < cap[order[k]]) {
            ++units[order[k]];
            --left;
        }
    std::vector<int> begin(n + 1, 0);
    for (int p = 0; p < n; ++p) begin[p + 1] = begin[p] + int(units[p] * 8);
    P.grid = begin[n];
    // device memory: args | begin | partials | reductions
    const size_t a_bytes = size_t(n) * sizeof(HvArgs);
    const size_t b_off = (a_bytes + 255) / 256 * 256;
    const size_t p_off = b_off + (size_t(n + 1) * 4 + 255) / 256 * 256;
    const size_t r_off = p_off + size_t(P.grid) * kNQ * sizeof(double);
    const size_t total = r_off + size_t(n) * sizeof(RedDesc);
    char* mem = nullptr;
    if (int rc = dev_alloc((void**)&mem, total, "hv_multi_prepare")) return rc;
    std::vector<HvArgs> args(n);
    std::vector<RedDesc> red(n);
    double* partials = reinterpret_cast<double*>(mem + p_off);
    for (int p = 0; p < n; ++p) {
        const HvLaunch& L = Ls[p];
        HvArgs& A = args[p];
        A.bs = L.ham->basis->dev;
        A.ops = L.ham->d_ops;
        A.n_ops = L.ham->n_ops_pad;
        A.ptab = L.ham->d_ptab;
        A.v = L.v;
        A.u = L.u;
        A.y = L.y;
        A.cy = L.cy;
        A.sx = L.sx;
        A.a = L.a;
        A.b = L.b;
        A.stop = L.stop;
        A.partials = partials + size_t(begin[p]) * kNQ;
        red[p].partials = A.partials;
        red[p].n_parts = begin[p + 1] - begin[p];
        red[p].pad = 0;
        red[p].out = L.reduce_out;
        red[p].stop = L.stop;
        red[p].flag = L.ham->d_flag;
    }
    hipError_t e = hipMemcpy(mem, args.data(), a_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mem + b_off, begin.data(), size_t(n + 1) * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mem + r_off, red.data(), size_t(n) * sizeof(RedDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return check_hip(e, "hv_multi_prepare: upload");
    }
    P.mem = mem;
    P.d_args = mem;
    P.d_begin = reinterpret_cast<const int*>(mem + b_off);
    P.d_red = reinterpret_cast<const RedDesc*>(mem + r_off);
    *out = P;
    return HPHI_OK;
}

int upd_multi_prepare(const UpdDesc* descs, double* const* red_out, int n, int dtype, UpdPlan* out) {
    if (n < 1 || !out) return set_error(HPHI_EINVAL, "upd_multi_prepare: no problems");
    UpdPlan P;
    P.n = n;
    P.fp64 = dtype == HPHI_F64 || dtype == HPHI_C128;
    int64_t total = 0;
    for (int p = 0; p < n; ++p) total += descs[p].n;
    std::vector<int> begin(n + 1, 0);
    const int64_t target = 1024;   // blocks of the streaming kernel in all
    for (int p = 0; p < n; ++p) {
        int64_t nb = total > 0 ? (target * descs[p].n + total - 1) / total : 1;
        const int64_t useful = (descs[p].n + 255) / 256;
        if (nb > useful) nb = useful;
        if (nb < 1) nb = 1;
        begin[p + 1] = begin[p] + int(nb);
    }
    P.grid = begin[n];
    const size_t d_bytes = size_t(n) * sizeof(UpdDesc);
    const size_t b_off = (d_bytes + 255) / 256 * 256;
    const size_t p_off = b_off + (size_t(n + 1) * 4 + 255) / 256 * 256;
    const size_t r_off = p_off + size_t(P.grid) * sizeof(double);
    const size_t total_b = r_off + size_t(n) * sizeof(RedDesc);
    char* mem = nullptr;
    if (int rc = dev_alloc((void**)&mem, total_b, "upd_multi_prepare")) return rc;
    std::vector<UpdDesc> d(descs, descs + n);
    std::vector<RedDesc> red(n);
    double* partials = reinterpret_cast<double*>(mem + p_off);
    for (int p = 0; p < n; ++p) {
        d[p].partials = partials + begin[p];
        red[p].partials = d[p].partials;
        red[p].n_parts = begin[p + 1] - begin[p];
        red[p].pad = 0;
        red[p].out = red_out[p];
        red[p].stop = d[p].stop;
        red[p].flag = d[p].flag;
    }
    hipError_t e = hipMemcpy(mem, d.data(), d_bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mem + b_off, begin.data(), size_t(n + 1) * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mem + r_off, red.data(), size_t(n) * sizeof(RedDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return check_hip(e, "upd_multi_prepare: upload");
    }
    P.mem = mem;
    P.d_desc = reinterpret_cast<const UpdDesc*>(mem);
    P.d_begin = reinterpret_cast<const int*>(mem + b_off);
    P.d_red = reinterpret_cast<const RedDesc*>(mem + r_off);
    *out = P;
    return HPHI_OK;
}

int upd_multi_launch(const UpdPlan& P, const LzMulti* lz, hipStream_t st) {
    if (P.fp64)
        lanczos_update_multi_kernel<double><<<P.grid, 256, 0, st>>>(P.d_desc, P.d_begin, P.n);
    else
        lanczos_update_multi_kernel<float><<<P.grid, 256, 0, st>>>(P.d_desc, P.d_begin, P.n);
    int rc = check_hip(hipGetLastError(), "update_multi launch");
    if (rc) return rc;
    if (lz)
        reduce_lz_after_update_multi_kernel<<<P.n, 256, 0, st>>>(P.d_red, lz->sc, lz->beta, lz->alpha, lz->stride);
    else
        reduce_multi_kernel<<<P.n, 256, 0, st>>>(P.d_red, 1);
    return check_hip(hipGetLastError(), "reduce_multi launch");
}

}  // namespace hphi
