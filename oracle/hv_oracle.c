/*
 * hv_oracle.c -- plain C / OpenMP row-slice H.v of the CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py): used for full-size
 * sampled parity rows and for the CPU timing baseline.  It shares no code
 * with the HIP library.
 *
 * For each requested row configuration s it applies every term to |s>
 * literally, one single-site operator at a time (spin operators of
 * Appendix A.1 with S = 1/2; fermion operators with the Jordan-Wigner
 * parity of the occupied orbitals below, Sec. 3.3), and uses the
 * Hermiticity of each term:  u[s] = sum_t conj(<t|T|s>) v[t].
 * Indices: full space = the bit string; otherwise binary search in the
 * caller's ascending list of basis configurations.
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int32_t kind, i, j, reserved;
    double c[9];
} oterm;

enum { SPIN_BOND = 0, SPIN_FIELD = 1, HOP = 2, DENS = 3, NUM = 4, HUBBARD_U = 5 };

typedef struct {
    double complex c;
    uint64_t s;
} branch;

/* S^a on one site: a = 0 (x), 1 (y), 2 (z); bit 1 = up */
static branch spin_apply(int a, int site, branch in) {
    branch out = in;
    const uint64_t m = (uint64_t)1 << site;
    const int up = (in.s & m) != 0;
    if (a == 2) {
        out.c = in.c * (up ? 0.5 : -0.5);
    } else if (a == 0) {
        out.c = in.c * 0.5;
        out.s = in.s ^ m;
    } else {
        /* S^y = (S^+ - S^-)/(2i):  S^y|down> = -(i/2)|up>,  S^y|up> = (i/2)|down> */
        out.c = in.c * (up ? 0.5 * I : -0.5 * I);
        out.s = in.s ^ m;
    }
    return out;
}

static int parity_below(uint64_t s, int k) {
    int n = 0;
    for (int q = 0; q < k; ++q) n += (int)((s >> q) & 1);
    return n & 1;
}

static branch annihilate(int k, branch in) {
    branch out = in;
    const uint64_t m = (uint64_t)1 << k;
    if (!(in.s & m)) { out.c = 0; return out; }
    out.c = parity_below(in.s, k) ? -in.c : in.c;
    out.s = in.s & ~m;
    return out;
}

static branch create(int k, branch in) {
    branch out = in;
    const uint64_t m = (uint64_t)1 << k;
    if (in.s & m) { out.c = 0; return out; }
    out.c = parity_below(in.s, k) ? -in.c : in.c;
    out.s = in.s | m;
    return out;
}

/* Sector given by counts instead of a list: kind 0 = all bit strings,
 * 1 = n_a set bits, 2 = n_a set even bits (up) and n_b set odd bits (down). */
typedef struct {
    int32_t kind, nbits, n_a, n_b;
} osector;

static int64_t binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

/* index of t in the ascending list of its sector by counting (Sec. 3.1):
 * for each set bit, from the top, the sector configurations that agree with t
 * above it and have a 0 there; -1 if t is not in the sector */
static int64_t rank_count(uint64_t t, const osector* sec) {
    if (sec->kind == 0) return (int64_t)t;
    int na = sec->n_a, nb = sec->n_b;
    int64_t r = 0;
    for (int p = sec->nbits - 1; p >= 0; --p) {
        if (!((t >> p) & 1)) continue;
        if (sec->kind == 1) {
            r += binom(p, na);
            --na;
        } else {
            r += binom((p + 1) / 2, na) * binom(p / 2, nb);
            if (p % 2 == 0) --na; else --nb;
        }
    }
    if (na != 0 || (sec->kind == 2 && nb != 0)) return -1;
    if (sec->nbits < 64 && (t >> sec->nbits) != 0) return -1;
    return r;
}

static int64_t rank_of(uint64_t t, const uint64_t* states, int64_t dim) {
    if (!states) return (int64_t)t;
    int64_t lo = 0, hi = dim - 1;
    while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (states[mid] == t) return mid;
        if (states[mid] < t) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* apply one term to |s>; returns the number of branches written to out[] */
static int term_apply(const oterm* T, uint64_t s, branch* out) {
    int n = 0;
    branch b0 = {1.0, s};
    switch (T->kind) {
        case SPIN_BOND:
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    const double J = T->c[3 * a + b];
                    if (J == 0.0) continue;
                    branch r = spin_apply(a, T->i, spin_apply(b, T->j, b0));
                    r.c *= J;
                    out[n++] = r;
                }
            break;
        case SPIN_FIELD:
            for (int a = 0; a < 3; ++a) {
                if (T->c[a] == 0.0) continue;
                branch r = spin_apply(a, T->i, b0);
                r.c *= T->c[a];
                out[n++] = r;
            }
            break;
        case HOP: {
            const double complex t = T->c[0] + I * T->c[1];
            branch r1 = create(T->i, annihilate(T->j, b0));
            r1.c *= t;
            out[n++] = r1;
            branch r2 = create(T->j, annihilate(T->i, b0));
            r2.c *= conj(t);
            out[n++] = r2;
            break;
        }
        case DENS: {
            branch r = create(T->i, annihilate(T->i, create(T->j, annihilate(T->j, b0))));
            r.c *= T->c[0];
            out[n++] = r;
            break;
        }
        case NUM: {
            branch r = create(T->i, annihilate(T->i, b0));
            r.c *= T->c[0];
            out[n++] = r;
            break;
        }
        case HUBBARD_U: {
            const int up = 2 * T->i, dn = 2 * T->i + 1;
            branch r = create(up, annihilate(up, create(dn, annihilate(dn, b0))));
            r.c *= T->c[0];
            out[n++] = r;
            break;
        }
        default:
            break;
    }
    return n;
}

/* A term's element <t|T|s> is the sum of all its operator-product branches
 * that reach t (Sec. 3.3): merge branches with equal targets, so that
 * branches which cancel (e.g. the S+S+ parts of xx and yy exchange on an Sz
 * sector) never reach the ranking.  Returns the merged count. */
static int merge_branches(branch* br, int n) {
    int m = 0;
    for (int q = 0; q < n; ++q) {
        int k = 0;
        while (k < m && br[k].s != br[q].s) ++k;
        if (k < m) {
            br[k].c += br[q].c;
        } else {
            br[m++] = br[q];
        }
    }
    return m;
}

/*
 * u[r*nvec + b] = sum over terms and branches of conj(coef) * v[rank(t)*nvec + b]
 * for the row configurations rows[0..nrows).  v has dim*nvec complex entries.
 * Returns 0, or -1 if a reached configuration is not in the basis.
 */
int oracle_hv_rows(const oterm* terms, int nterms, const uint64_t* states, int64_t dim,
                   const uint64_t* rows, int64_t nrows, const double complex* v, int nvec,
                   double complex* u) {
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t r = 0; r < nrows; ++r) {
        branch br[16];
        double complex acc[64];
        for (int b = 0; b < nvec; ++b) acc[b] = 0;
        for (int k = 0; k < nterms; ++k) {
            const int n = merge_branches(br, term_apply(&terms[k], rows[r], br));
            for (int q = 0; q < n; ++q) {
                if (br[q].c == 0) continue;
                const int64_t t = rank_of(br[q].s, states, dim);
                if (t < 0) { bad = 1; continue; }
                const double complex cc = conj(br[q].c);
                for (int b = 0; b < nvec; ++b) acc[b] += cc * v[t * nvec + b];
            }
        }
        for (int b = 0; b < nvec; ++b) u[r * nvec + b] = acc[b];
    }
    return bad ? -1 : 0;
}

/* single-precision-input variant: v stored as complex float (the device layout of complex64) */
int oracle_hv_rows_c64(const oterm* terms, int nterms, const uint64_t* states, int64_t dim,
                       const uint64_t* rows, int64_t nrows, const float complex* v, int nvec,
                       double complex* u) {
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t r = 0; r < nrows; ++r) {
        branch br[16];
        double complex acc[64];
        for (int b = 0; b < nvec; ++b) acc[b] = 0;
        for (int k = 0; k < nterms; ++k) {
            const int n = merge_branches(br, term_apply(&terms[k], rows[r], br));
            for (int q = 0; q < n; ++q) {
                if (br[q].c == 0) continue;
                const int64_t t = rank_of(br[q].s, states, dim);
                if (t < 0) { bad = 1; continue; }
                const double complex cc = conj(br[q].c);
                for (int b = 0; b < nvec; ++b) acc[b] += cc * (double complex)v[t * nvec + b];
            }
        }
        for (int b = 0; b < nvec; ++b) u[r * nvec + b] = acc[b];
    }
    return bad ? -1 : 0;
}

/* as oracle_hv_rows, targets ranked by counting (no basis list needed) */
int oracle_hv_rows_counted(const oterm* terms, int nterms, const osector* sec, const uint64_t* rows, int64_t nrows,
                           const double complex* v, int nvec, double complex* u) {
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t r = 0; r < nrows; ++r) {
        branch br[16];
        double complex acc[64];
        for (int b = 0; b < nvec; ++b) acc[b] = 0;
        for (int k = 0; k < nterms; ++k) {
            const int n = merge_branches(br, term_apply(&terms[k], rows[r], br));
            for (int q = 0; q < n; ++q) {
                if (br[q].c == 0) continue;
                const int64_t t = rank_count(br[q].s, sec);
                if (t < 0) { bad = 1; continue; }
                const double complex cc = conj(br[q].c);
                for (int b = 0; b < nvec; ++b) acc[b] += cc * v[t * nvec + b];
            }
        }
        for (int b = 0; b < nvec; ++b) u[r * nvec + b] = acc[b];
    }
    return bad ? -1 : 0;
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): a counter-based stream,
 * element `index` of the stream started at `seed`, mapped to [-1, 1) with
 * 53 random bits.  Used where an input vector is too large for host memory:
 * v[t][b] is evaluated on demand from (seed, t * nvec + b). */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t index) {
    uint64_t z = seed + (index + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double splitmix_uniform(uint64_t seed, uint64_t index) {
    return (double)(oracle_splitmix64(seed, index) >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}

/* as oracle_hv_rows_counted, for a real vector v[t*nvec + b] that is not
 * stored but evaluated on demand (splitmix_uniform(seed, t*nvec + b));
 * u is real */
int oracle_hv_rows_counted_ondemand(const oterm* terms, int nterms, const osector* sec, const uint64_t* rows,
                                    int64_t nrows, uint64_t seed, int nvec, double* u) {
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t r = 0; r < nrows; ++r) {
        branch br[16];
        double acc[64];
        for (int b = 0; b < nvec; ++b) acc[b] = 0;
        for (int k = 0; k < nterms; ++k) {
            const int n = merge_branches(br, term_apply(&terms[k], rows[r], br));
            for (int q = 0; q < n; ++q) {
                if (br[q].c == 0) continue;
                const int64_t t = rank_count(br[q].s, sec);
                if (t < 0) { bad = 1; continue; }
                const double cr = creal(br[q].c);
                for (int b = 0; b < nvec; ++b)
                    acc[b] += cr * splitmix_uniform(seed, (uint64_t)t * (uint64_t)nvec + (uint64_t)b);
            }
        }
        for (int b = 0; b < nvec; ++b) u[r * nvec + b] = acc[b];
    }
    return bad ? -1 : 0;
}

/* the configuration of each rank (inverse of rank_count, greedy from the top bit) */
int oracle_unrank_counted(const osector* sec, const int64_t* idx, int64_t n, uint64_t* cfg) {
    for (int64_t k = 0; k < n; ++k) {
        int64_t r = idx[k];
        if (sec->kind == 0) {
            cfg[k] = (uint64_t)r;
            continue;
        }
        int na = sec->n_a, nb = sec->n_b;
        uint64_t s = 0;
        for (int p = sec->nbits - 1; p >= 0; --p) {
            const int64_t zero = sec->kind == 1 ? binom(p, na) : binom((p + 1) / 2, na) * binom(p / 2, nb);
            if (r >= zero) {
                r -= zero;
                s |= (uint64_t)1 << p;
                if (sec->kind == 1 || p % 2 == 0) --na; else --nb;
            }
        }
        if (r != 0) return -1;
        cfg[k] = s;
    }
    return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
