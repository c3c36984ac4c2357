// Hilbert space and split rank tables (Sec. 3.1: canonical restricted space,
// two-dimensional search, same-popcount successor).
#include <algorithm>
#include <cstdarg>
#include <cstring>
#include <new>

#include "hphi_internal.h"

using namespace hphi;

namespace {

// Next larger integer with the same number of set bits (the "next higher
// number with the same number of 1-bits" construction cited in Sec. 3.1).
inline uint64_t same_popcount_successor(uint64_t x) {
    uint64_t lowest = x & (~x + 1);
    uint64_t ripple = x + lowest;
    uint64_t ones = ((ripple ^ x) >> 2) / lowest;
    return ripple | ones;
}

inline int popc(uint64_t x) { return __builtin_popcountll(x); }

constexpr uint64_t kEven = 0x5555555555555555ull;
constexpr uint64_t kOdd = 0xAAAAAAAAAAAAAAAAull;

struct Charge {
    int sector;
    int lo_bits;
    // number of classes for the low half and class of a value
    int n_classes() const {
        if (sector == HPHI_SECTOR_NUP_NDN) return (lo_bits / 2 + 1) * (lo_bits / 2 + 1);
        return lo_bits + 1;
    }
    int cls_lo(uint64_t l) const {
        if (sector == HPHI_SECTOR_NUP_NDN) return popc(l & kEven) * (lo_bits / 2 + 1) + popc(l & kOdd);
        return popc(l);
    }
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

extern "C" int hphi_basis_build(const hphi_basis_desc* desc, hphi_basis** out) {
    if (!desc || !out) return set_error(HPHI_EINVAL, "hphi_basis_build: null argument");
    *out = nullptr;
    const hphi_basis_desc d = *desc;
    if (d.particle != HPHI_SPIN_HALF && d.particle != HPHI_FERMION)
        return set_error(HPHI_EINVAL, "hphi_basis_build: bad particle %d", d.particle);
    if (d.n_sites < 1) return set_error(HPHI_EINVAL, "hphi_basis_build: n_sites must be >= 1");
    const int nbits = d.particle == HPHI_SPIN_HALF ? d.n_sites : 2 * d.n_sites;
    if (nbits > 62) return set_error(HPHI_EINVAL, "hphi_basis_build: %d bits exceed 62", nbits);

    // target charge
    int tgt_a = 0, tgt_b = 0;
    switch (d.sector) {
        case HPHI_SECTOR_NONE:
            if (nbits > 40) return set_error(HPHI_EINVAL, "hphi_basis_build: full space limited to 40 bits");
            break;
        case HPHI_SECTOR_SZ:
            if (d.particle != HPHI_SPIN_HALF)
                return set_error(HPHI_EINVAL, "hphi_basis_build: SZ sector needs spins");
            if (d.two_sz < -d.n_sites || d.two_sz > d.n_sites || ((d.n_sites + d.two_sz) & 1))
                return set_error(HPHI_EINVAL, "hphi_basis_build: two_sz=%d impossible for %d sites",
                                 d.two_sz, d.n_sites);
            tgt_a = (d.n_sites + d.two_sz) / 2;
            break;
        case HPHI_SECTOR_NUP_NDN:
            if (d.particle != HPHI_FERMION)
                return set_error(HPHI_EINVAL, "hphi_basis_build: NUP_NDN sector needs fermions");
            if (d.n_up < 0 || d.n_up > d.n_sites || d.n_dn < 0 || d.n_dn > d.n_sites)
                return set_error(HPHI_EINVAL, "hphi_basis_build: n_up/n_dn out of range");
            tgt_a = d.n_up;
            tgt_b = d.n_dn;
            break;
        case HPHI_SECTOR_NTOT:
            if (d.particle != HPHI_FERMION)
                return set_error(HPHI_EINVAL, "hphi_basis_build: NTOT sector needs fermions");
            if (d.n_tot < 0 || d.n_tot > 2 * d.n_sites)
                return set_error(HPHI_EINVAL, "hphi_basis_build: n_tot out of range");
            tgt_a = d.n_tot;
            break;
        default:
            return set_error(HPHI_EINVAL, "hphi_basis_build: bad sector %d", d.sector);
    }

    hphi_basis* B = alloc_fails() ? nullptr : new (std::nothrow) hphi_basis();
    if (!B) return set_error(HPHI_ENOMEM, "hphi_basis_build: host allocation");
    B->desc = d;
    B->nbits = nbits;
    if (hipGetDevice(&B->device) != hipSuccess) {
        delete B;
        return set_error(HPHI_EDEVICE, "hphi_basis_build: no HIP device");
    }
    BasisDev& dv = B->dev;
    dv.nbits = nbits;

    if (d.sector == HPHI_SECTOR_NONE) {
        B->dim = int64_t(1) << nbits;
        dv.sector = 0;
        dv.dim = B->dim;
        dv.n_tiles = (B->dim + kTile - 1) / kTile;
        *out = B;
        return HPHI_OK;
    }

    int b_lo = d.split_bits;
    if (b_lo == 0) {
        b_lo = nbits / 2;
        if (d.particle == HPHI_FERMION) b_lo &= ~1;
        if (b_lo == 0) b_lo = d.particle == HPHI_FERMION ? 2 : 1;
    }
    if (b_lo < 1 || b_lo > nbits || (d.particle == HPHI_FERMION && (b_lo & 1))) {
        delete B;
        return set_error(HPHI_EINVAL, "hphi_basis_build: bad split_bits %d for %d bits", b_lo, nbits);
    }
    const int b_hi = nbits - b_lo;
    if (b_lo > 26 || b_hi > 26) {
        delete B;
        return set_error(HPHI_EINVAL, "hphi_basis_build: split tables above 2^26 entries");
    }
    B->b_lo = b_lo;
    B->b_hi = b_hi;
    Charge ch{d.sector, b_lo};
    const int ncls = ch.n_classes();
    const uint64_t n_lo = uint64_t(1) << b_lo, n_hi = uint64_t(1) << b_hi;

    // ---- low half: J_lo[l] = rank of l within its class; lows grouped by class
    std::vector<uint32_t> cls_count(ncls, 0), cls_off(ncls + 1, 0);
    B->j_lo.assign(n_lo, 0);
    std::vector<uint32_t> lows(n_lo);
    if (d.sector == HPHI_SECTOR_NUP_NDN) {
        for (uint64_t l = 0; l < n_lo; ++l) B->j_lo[l] = cls_count[ch.cls_lo(l)]++;
        for (int c = 0; c < ncls; ++c) cls_off[c + 1] = cls_off[c] + cls_count[c];
        for (uint64_t l = 0; l < n_lo; ++l) lows[cls_off[ch.cls_lo(l)] + B->j_lo[l]] = uint32_t(l);
    } else {
        // popcount classes: enumerate each class in ascending order by the
        // same-popcount successor
        uint32_t off = 0;
        for (int c = 0; c <= b_lo; ++c) {
            cls_off[c] = off;
            uint32_t r = 0;
            if (c == 0) {
                lows[off] = 0;
                B->j_lo[0] = 0;
                r = 1;
            } else {
                for (uint64_t x = (uint64_t(1) << c) - 1; x < n_lo; x = same_popcount_successor(x)) {
                    lows[off + r] = uint32_t(x);
                    B->j_lo[x] = r++;
                }
            }
            cls_count[c] = r;
            off += r;
        }
        cls_off[b_lo + 1] = off;
    }

    // ---- high half: valid highs, offsets, tiles
    B->j_hi.assign(n_hi, -1);
    std::vector<uint64_t> h_val;
    std::vector<int64_t> h_row, h_tile;
    std::vector<uint32_t> h_lobase;
    int64_t offset = 0, tiles = 0;
    const int hw = b_lo / 2 + 1;
    for (uint64_t h = 0; h < n_hi; ++h) {
        int need;
        if (d.sector == HPHI_SECTOR_NUP_NDN) {
            // high half starts at an even bit, so even/odd parity is preserved
            int nu = tgt_a - popc(h & kEven), nd = tgt_b - popc(h & kOdd);
            if (nu < 0 || nd < 0 || nu >= hw || nd >= hw) continue;
            need = nu * hw + nd;
        } else {
            need = tgt_a - popc(h);
            if (need < 0 || need > b_lo) continue;
        }
        const uint32_t cnt = cls_count[need];
        if (cnt == 0) continue;
        B->j_hi[h] = offset;
        h_val.push_back(h);
        h_row.push_back(offset);
        h_tile.push_back(tiles);
        h_lobase.push_back(cls_off[need]);
        offset += cnt;
        tiles += (cnt + kTile - 1) / kTile;
    }
    h_row.push_back(offset);
    h_tile.push_back(tiles);
    B->dim = offset;
    if (offset == 0) {
        delete B;
        return set_error(HPHI_EINVAL, "hphi_basis_build: empty sector");
    }

    // ---- device copy (one allocation)
    const size_t n_high = h_val.size();
    size_t sz_jlo = align256(n_lo * 4), sz_jhi = align256(n_hi * 8), sz_hv = align256(n_high * 8),
           sz_hr = align256((n_high + 1) * 8), sz_ht = align256((n_high + 1) * 8),
           sz_hb = align256(n_high * 4), sz_lows = align256(n_lo * 4);
    size_t total = sz_jlo + sz_jhi + sz_hv + sz_hr + sz_ht + sz_hb + sz_lows;
    char* base = nullptr;
    if (int rc = dev_alloc((void**)&base, total, "hphi_basis_build: rank tables")) {
        delete B;
        return rc;
    }
    B->dmem = base;
    char* p = base;
    auto put = [&](const void* src, size_t bytes, size_t stride) -> char* {
        char* at = p;
        if (bytes) (void)hipMemcpy(at, src, bytes, hipMemcpyHostToDevice);
        p += stride;
        return at;
    };
    dv.sector = d.sector;
    dv.b_lo = b_lo;
    dv.mask_lo = n_lo - 1;
    dv.dim = offset;
    dv.n_tiles = tiles;
    dv.n_high = int64_t(n_high);
    dv.j_lo = (const uint32_t*)put(B->j_lo.data(), n_lo * 4, sz_jlo);
    dv.j_hi = (const int64_t*)put(B->j_hi.data(), n_hi * 8, sz_jhi);
    dv.h_val = (const uint64_t*)put(h_val.data(), n_high * 8, sz_hv);
    dv.h_row = (const int64_t*)put(h_row.data(), (n_high + 1) * 8, sz_hr);
    dv.h_tile = (const int64_t*)put(h_tile.data(), (n_high + 1) * 8, sz_ht);
    dv.h_lobase = (const uint32_t*)put(h_lobase.data(), n_high * 4, sz_hb);
    dv.lows = (const uint32_t*)put(lows.data(), n_lo * 4, sz_lows);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(base);
        delete B;
        return check_hip(e, "hphi_basis_build: table upload");
    }
    for (size_t k = 0; k + 1 < h_row.size(); ++k)
        B->max_block_rows = std::max<int64_t>(B->max_block_rows, h_row[k + 1] - h_row[k]);
    B->h_row = std::move(h_row);
    B->h_tile = std::move(h_tile);

    // ---- two-level low-rank tables: the split search of the basis applied
    // once more inside the low half, l = (a, b) with b the low b2 bits:
    //   rank(l) = T1[a][class(l)] + T2[b]
    // T2[b] = rank of b among the b2-bit strings of its class, T1[a][c] = number
    // of class-c low halves whose upper part is below a.  b2 is even for
    // fermions, so both parts keep the even/odd (up/down) bit parity.
    {
        const bool pairs = d.sector == HPHI_SECTOR_NUP_NDN;
        int b2 = std::min(b_lo, 12);
        if (pairs) b2 &= ~1;
        const int b1 = b_lo - b2;
        const int w2 = b2 / 2 + 1;                  // class base of a b2-bit part (pairs)
        auto cls2 = [&](uint64_t x) { return pairs ? popc(x & kEven) * w2 + popc(x & kOdd) : popc(x); };
        const int n2 = pairs ? w2 * w2 : b2 + 1;
        std::vector<uint32_t> cnt2(n2, 0);
        std::vector<uint16_t> t2(size_t(1) << b2);
        for (uint64_t x = 0; x < (uint64_t(1) << b2); ++x) t2[x] = uint16_t(cnt2[cls2(x)]++);
        const size_t t1_n = (size_t(1) << b1) * size_t(ncls);
        const size_t bytes = t1_n * 4 + (((size_t(1) << b2) * 2 + 15) / 16 * 16);
        if (bytes <= 64 * 1024) {
            std::vector<uint32_t> t1(t1_n, 0), acc(ncls, 0);
            for (uint64_t a = 0; a < (uint64_t(1) << b1); ++a) {
                for (int c = 0; c < ncls; ++c) t1[a * ncls + c] = acc[c];
                // class-c low halves with upper part a: b completes the class
                const int ae = pairs ? popc(a & kEven) : 0, ao = pairs ? popc(a & kOdd) : 0, ap = popc(a);
                for (int c = 0; c < ncls; ++c) {
                    int need;
                    if (pairs) {
                        const int hw = b_lo / 2 + 1, ne = c / hw - ae, no = c % hw - ao;
                        if (ne < 0 || no < 0 || ne >= w2 || no >= w2) continue;
                        need = ne * w2 + no;
                    } else {
                        need = c - ap;
                        if (need < 0 || need > b2) continue;
                    }
                    acc[c] += cnt2[need];
                }
            }
            bool ok = true;
            for (uint64_t l = 0; l < n_lo && ok; ++l)
                ok = B->j_lo[l] == t1[(l >> b2) * ncls + uint64_t(ch.cls_lo(l))] + t2[l & ((uint64_t(1) << b2) - 1)];
            if (!ok) {
                hphi_basis_free(B);
                return set_error(HPHI_EDEVICE, "hphi_basis_build: internal error in the two-level rank tables");
            }
            char* p = nullptr;
            if (int rc = dev_alloc((void**)&p, bytes, "hphi_basis_build: two-level rank tables")) {
                hphi_basis_free(B);
                return rc;
            }
            B->d_t1 = reinterpret_cast<uint32_t*>(p);
            B->d_t2 = reinterpret_cast<uint16_t*>(p + t1_n * 4);
            hipError_t e2 = hipMemcpy(B->d_t1, t1.data(), t1_n * 4, hipMemcpyHostToDevice);
            if (e2 == hipSuccess) e2 = hipMemcpy(B->d_t2, t2.data(), t2.size() * 2, hipMemcpyHostToDevice);
            if (e2 != hipSuccess) {
                hphi_basis_free(B);
                return check_hip(e2, "hphi_basis_build: rank table upload");
            }
            B->lr_b2 = b2;
            B->lr_ncls = ncls;
            B->lr_pairs = pairs ? 1 : 0;
            B->lr_nsl = b_lo / 2;
            B->lr_bytes = bytes;

            // compact 16-bit form for the single-pass kernel: T2p[b] packs the
            // rank of b within its class (10 bits) with that class cb (6 bits),
            // and T1c[a][cb] = T1[a][class(a) + cb], so that
            //   rank(l) = T1c[a][T2p[b] >> 10] + (T2p[b] & 1023)
            // needs no class arithmetic on the device
            const uint32_t t1_max = *std::max_element(t1.begin(), t1.end());
            if (t1_max < 65536 && n2 <= 64 && b2 <= 12) {
                std::vector<uint16_t> t2p(size_t(1) << b2), t1c((size_t(1) << b1) * size_t(n2), 0);
                for (uint64_t x = 0; x < (uint64_t(1) << b2); ++x)
                    t2p[x] = uint16_t(uint32_t(t2[x]) | (uint32_t(cls2(x)) << 10));
                const int hw = b_lo / 2 + 1;
                for (uint64_t a = 0; a < (uint64_t(1) << b1); ++a)
                    for (int cb = 0; cb < n2; ++cb) {
                        int c;
                        if (pairs) {
                            const int ne = popc(a & kEven) + cb / w2, no = popc(a & kOdd) + cb % w2;
                            if (ne >= hw || no >= hw) continue;
                            c = ne * hw + no;
                        } else {
                            c = popc(a) + cb;
                            if (c >= ncls) continue;
                        }
                        t1c[a * n2 + cb] = uint16_t(t1[a * ncls + c]);
                    }
                bool okc = true;
                const uint64_t m2 = (uint64_t(1) << b2) - 1;
                for (uint64_t l = 0; l < n_lo && okc; ++l) {
                    const uint32_t p2 = t2p[l & m2];
                    okc = B->j_lo[l] == uint32_t(t1c[(l >> b2) * n2 + (p2 >> 10)]) + (p2 & 1023u);
                }
                if (!okc) {
                    hphi_basis_free(B);
                    return set_error(HPHI_EDEVICE, "hphi_basis_build: internal error in the compact rank tables");
                }
                const size_t c1 = (t1c.size() * 2 + 15) / 16 * 16;
                char* q = nullptr;
                if (int rc = dev_alloc((void**)&q, c1 + t2p.size() * 2, "hphi_basis_build: compact rank tables")) {
                    hphi_basis_free(B);
                    return rc;
                }
                B->d_t1c = reinterpret_cast<uint16_t*>(q);
                B->d_t2p = reinterpret_cast<uint16_t*>(q + c1);
                hipError_t e3 = hipMemcpy(B->d_t1c, t1c.data(), t1c.size() * 2, hipMemcpyHostToDevice);
                if (e3 == hipSuccess) e3 = hipMemcpy(B->d_t2p, t2p.data(), t2p.size() * 2, hipMemcpyHostToDevice);
                if (e3 != hipSuccess) {
                    hphi_basis_free(B);
                    return check_hip(e3, "hphi_basis_build: compact rank table upload");
                }
                B->lr_n2 = n2;
            }
        }
    }
    *out = B;
    return HPHI_OK;
}

extern "C" int hphi_basis_dim(const hphi_basis* b, int64_t* dim) {
    if (!b || !dim) return set_error(HPHI_EINVAL, "hphi_basis_dim: null argument");
    *dim = b->dim;
    return HPHI_OK;
}

extern "C" void hphi_basis_free(hphi_basis* b) {
    if (!b) return;
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->d_t1) (void)hipFree(b->d_t1);
    if (b->d_t1c) (void)hipFree(b->d_t1c);
    delete b;
}

extern "C" int hphi_basis_rank(const hphi_basis* b, const uint64_t* cfg, int64_t* idx, int64_t n,
                               void* stream) {
    if (!b || n < 0 || (n > 0 && (!cfg || !idx))) return set_error(HPHI_EINVAL, "hphi_basis_rank: bad argument");
    if (n == 0) return HPHI_OK;
    return launch_rank(b, cfg, idx, n, (hipStream_t)stream);
}

extern "C" int hphi_basis_unrank(const hphi_basis* b, const int64_t* idx, uint64_t* cfg, int64_t n,
                                 void* stream) {
    if (!b || n < 0 || (n > 0 && (!cfg || !idx))) return set_error(HPHI_EINVAL, "hphi_basis_unrank: bad argument");
    if (n == 0) return HPHI_OK;
    return launch_unrank(b, idx, cfg, n, (hipStream_t)stream);
}
