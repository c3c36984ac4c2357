// Pass plans of the windowed full-space product.
//
// Every off-diagonal operator gathers row s ^ xmask for row s.  When the
// flip bits of xmask all lie inside a window of W configuration bits, and
// the rows are processed so that the 2^W rows sharing the other bits are
// in flight together, the partner rows are served from L2 instead of being
// re-read from HBM.  The operators are covered by a few windows (greedily,
// deterministic); pass p processes rows in the order of its permutation
// (window bits lowest) and applies only its own operators, accumulating
// into the output.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <new>

#include "hphi_internal.h"

namespace hphi {
namespace {

constexpr int kMaxPasses = 4;

int log2_floor(uint64_t x) {
    int r = -1;
    while (x) {
        x >>= 1;
        ++r;
    }
    return r;
}

PassPlan* build_plan(const hphi_ham* H, int row_bytes, int window_kb, int max_passes) {
    const int nbits = H->basis->nbits;
    PassPlan* P = new (std::nothrow) PassPlan();
    if (!P) return nullptr;
    P->row_bytes = row_bytes;
    P->window_kb = window_kb;
    P->max_passes = max_passes;
    int w = log2_floor(uint64_t(window_kb) * 1024 / uint64_t(row_bytes));
    if (w < 6) w = 6;
    if (w > nbits || max_passes <= 1) w = nbits;
    // low bits that keep a 128-byte line inside consecutive rows
    int lb = 0;
    while ((row_bytes << lb) < 128 && lb < nbits) ++lb;
    if (lb > w) lb = w;
    P->wbits = w;

    const std::vector<DevOp>& ops = H->ops;
    const int n_ops = int(ops.size());
    std::vector<int> pass_of(n_ops, -1);
    std::vector<std::vector<int>> windows;   // bits per window (ordered)
    if (w >= nbits) {
        std::vector<int> all;
        for (int b = 0; b < nbits; ++b) all.push_back(b);
        windows.push_back(all);
        for (int o = 0; o < n_ops; ++o) pass_of[o] = 0;
    } else {
        std::vector<int> remaining;
        for (int o = 0; o < n_ops; ++o) {
            if (ops[o].xmask == 0) pass_of[o] = 0;   // diagonal-only: first pass
            else remaining.push_back(o);
        }
        while (!remaining.empty()) {
            if (int(windows.size()) == kMaxPasses) {
                delete P;
                return nullptr;
            }
            if (int(windows.size()) == max_passes) {
                // fold the rest back: each operator joins the pass whose window
                // holds most of its flip bits (its gathers then leave L2)
                for (int o : remaining) {
                    int best = 0, best_n = -1;
                    for (int p = 0; p < int(windows.size()); ++p) {
                        int n = 0;
                        for (int b : windows[p]) n += int((ops[o].xmask >> b) & 1);
                        if (n > best_n) {
                            best_n = n;
                            best = p;
                        }
                    }
                    pass_of[o] = best;
                }
                remaining.clear();
                break;
            }
            std::vector<char> in(nbits, 0);
            std::vector<int> order;
            for (int b = 0; b < lb; ++b) {
                in[b] = 1;
                order.push_back(b);
            }
            auto inside = [&](uint64_t m) {
                for (int b = 0; b < nbits; ++b)
                    if (((m >> b) & 1) && !in[b]) return false;
                return true;
            };
            while (int(order.size()) < w) {
                int best = -1;
                long best_score = -1;
                for (int c = 0; c < nbits; ++c) {
                    if (in[c]) continue;
                    in[c] = 1;
                    long gain = 0, touch = 0;
                    for (int o : remaining) {
                        const uint64_t m = ops[o].xmask;
                        if ((m >> c) & 1) ++touch;
                        if (((m >> c) & 1) && inside(m)) ++gain;
                    }
                    in[c] = 0;
                    const long score = gain * 1024 + touch;   // covered first, then reach
                    if (score > best_score) {
                        best_score = score;
                        best = c;
                    }
                }
                in[best] = 1;
                order.push_back(best);
            }
            std::vector<int> rest;
            const int p = int(windows.size());
            for (int o : remaining) {
                if (inside(ops[o].xmask)) pass_of[o] = p;
                else rest.push_back(o);
            }
            if (rest.size() == remaining.size()) {   // nothing covered: give up
                delete P;
                return nullptr;
            }
            remaining.swap(rest);
            // window bits: line bits first, then ascending
            std::sort(order.begin() + lb, order.end());
            windows.push_back(order);
        }
        if (windows.empty()) {
            std::vector<int> all;
            for (int b = 0; b < nbits; ++b) all.push_back(b);
            windows.push_back(all);
        }
    }
    P->n_pass = int(windows.size());
    P->perm.assign(size_t(P->n_pass) * 64, 0);
    for (int p = 0; p < P->n_pass; ++p) {
        std::vector<char> in(nbits, 0);
        int k = 0;
        for (int b : windows[p]) {
            P->perm[size_t(p) * 64 + k++] = b;
            in[b] = 1;
        }
        // next, the outside flip bits of the operators folded into this pass
        // (most frequent first): their partners are then one or two window
        // blocks away on the same XCD instead of anywhere in the space (the
        // top processing bits select the XCD)
        std::vector<int> cnt(nbits, 0);
        for (int o = 0; o < n_ops; ++o)
            if (pass_of[o] == p)
                for (int b = 0; b < nbits; ++b)
                    if (!in[b] && ((ops[o].xmask >> b) & 1)) ++cnt[b];
        std::vector<int> outside;
        for (int b = 0; b < nbits; ++b)
            if (cnt[b] > 0) outside.push_back(b);
        std::stable_sort(outside.begin(), outside.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
        for (int b : outside) {
            P->perm[size_t(p) * 64 + k++] = b;
            in[b] = 1;
        }
        for (int b = 0; b < nbits; ++b)
            if (!in[b]) P->perm[size_t(p) * 64 + k++] = b;
    }
    std::vector<DevOp> sorted;
    std::vector<int> sorted_idx;     // index of each sorted operator in the Hamiltonian's list
    P->op_begin.assign(P->n_pass + 1, 0);
    for (int p = 0; p < P->n_pass; ++p) {
        P->op_begin[p] = int(sorted.size());
        for (int o = 0; o < n_ops; ++o)
            if (pass_of[o] == p) {
                sorted.push_back(ops[o]);
                sorted_idx.push_back(o);
            }
    }
    P->op_begin[P->n_pass] = int(sorted.size());
    // compact records, padded per pass to a multiple of 4
    std::vector<KOp<double>> k64;
    P->kop_begin.assign(P->n_pass + 1, 0);
    for (int p = 0; p < P->n_pass; ++p) {
        P->kop_begin[p] = int(k64.size());
        for (int o = P->op_begin[p]; o < P->op_begin[p + 1]; ++o) {
            const DevOp& d = sorted[o];
            KOp<double> b{};
            b.op = sorted_idx[o];
            b.xm = d.has_off ? uint32_t(d.xmask) : 0u;
            b.sm = uint32_t(d.smask);
            b.bi = d.bi;
            b.bj = d.bj;
            for (int q = 0; q < 4; ++q) {
                b.c[q] = d.cr[q];
                b.ci[q] = d.ci[q];
                b.d[q] = d.d[q];
            }
            k64.push_back(b);
        }
        while (k64.size() % 4) {
            KOp<double> pad{};
            pad.op = -1;
            k64.push_back(pad);
        }
    }
    P->kop_begin[P->n_pass] = int(k64.size());
    if (k64.empty()) {
        KOp<double> pad{};
        pad.op = -1;
        k64.push_back(pad);
    }
    // inverse permutations, and the flip masks of passes after the first in
    // processing-index bits (a bit permutation commutes with XOR, so the
    // partner of processing index q is q ^ perm^-1(xmask))
    P->inv.assign(size_t(P->n_pass) * 64, 0);
    for (int p = 0; p < P->n_pass; ++p)
        for (int k = 0; k < nbits; ++k) P->inv[size_t(p) * 64 + P->perm[size_t(p) * 64 + k]] = k;
    // partners inside the 64-row tile, in processing-index bits
    for (int p = 0; p < P->n_pass; ++p)
        for (int o = P->kop_begin[p]; o < P->kop_begin[p + 1]; ++o) {
            uint32_t m = 0;
            for (int b = 0; b < nbits; ++b)
                if ((k64[o].xm >> b) & 1u) m |= 1u << P->inv[size_t(p) * 64 + b];
            k64[o].lq = (k64[o].xm != 0 && m < 64u) ? m : ~0u;
        }
    // within a pass, partners on chip first (ascending in-tile flip mask), then
    // the gathers from memory: an operator group then mixes the two kinds at
    // most once per pass, and a group of memory gathers never waits on the
    // loads of an earlier in-tile read into the same registers
    for (int p = 0; p < P->n_pass; ++p)
        std::stable_sort(k64.begin() + P->kop_begin[p], k64.begin() + P->kop_begin[p + 1],
                         [](const KOp<double>& a, const KOp<double>& b) { return a.lq < b.lq; });
    std::vector<KOp<double>> kq = k64;
    for (int p = 1; p < P->n_pass; ++p)
        for (int o = P->kop_begin[p]; o < P->kop_begin[p + 1]; ++o) {
            uint32_t m = 0;
            for (int b = 0; b < nbits; ++b)
                if ((kq[o].xm >> b) & 1u) m |= 1u << P->inv[size_t(p) * 64 + b];
            kq[o].xm = m;
        }
    const size_t kb = k64.size() * sizeof(KOp<double>);
    if (dev_alloc((void**)&P->d_kop64, kb, "pass plan")) {
        delete P;
        return nullptr;
    }
    if (dev_alloc((void**)&P->d_kopq, kb, "pass plan") || dev_alloc((void**)&P->d_inv, P->inv.size() * 4, "pass plan")) {
        (void)hipFree(P->d_kop64);
        if (P->d_kopq) (void)hipFree(P->d_kopq);
        delete P;
        return nullptr;
    }
    (void)hipMemcpy(P->d_kop64, k64.data(), kb, hipMemcpyHostToDevice);
    (void)hipMemcpy(P->d_kopq, kq.data(), kb, hipMemcpyHostToDevice);
    (void)hipMemcpy(P->d_inv, P->inv.data(), P->inv.size() * 4, hipMemcpyHostToDevice);
    const size_t ob = std::max<size_t>(1, sorted.size()) * sizeof(DevOp);
    if (dev_alloc((void**)&P->d_ops, ob, "pass plan") || dev_alloc((void**)&P->d_perm, P->perm.size() * 4, "pass plan")) {
        if (P->d_ops) (void)hipFree(P->d_ops);
        (void)hipFree(P->d_kop64);
        (void)hipFree(P->d_kopq);
        (void)hipFree(P->d_inv);
        delete P;
        return nullptr;
    }
    if (!sorted.empty()) (void)hipMemcpy(P->d_ops, sorted.data(), sorted.size() * sizeof(DevOp), hipMemcpyHostToDevice);
    (void)hipMemcpy(P->d_perm, P->perm.data(), P->perm.size() * 4, hipMemcpyHostToDevice);
    return P;
}

}  // namespace

const PassPlan* get_plan(const hphi_ham* ham, int row_bytes, int window_kb, int max_passes, bool may_build) {
    hphi_ham* H = const_cast<hphi_ham*>(ham);
    std::lock_guard<std::mutex> lock(H->plan_mu);
    for (PassPlan* p : H->plans)
        if (p->row_bytes == row_bytes && p->window_kb == window_kb && p->max_passes == max_passes)
            return p->n_pass > 0 ? p : nullptr;
    if (!may_build) return nullptr;
    PassPlan* p = build_plan(H, row_bytes, window_kb, max_passes);
    if (p && getenv("HPHI_DEBUG")) {
        fprintf(stderr, "[hphi] plan row_bytes=%d window_kb=%d window_bits=%d passes=%d ops/pass:", row_bytes,
                window_kb, p->wbits, p->n_pass);
        for (int q = 0; q < p->n_pass; ++q) fprintf(stderr, " %d", p->op_begin[q + 1] - p->op_begin[q]);
        fprintf(stderr, "\n");
        for (int q = 0; q < p->n_pass; ++q) {
            fprintf(stderr, "[hphi]   pass %d q-bit->config-bit:", q);
            for (int k = 0; k < H->basis->nbits; ++k) fprintf(stderr, " %d", p->perm[size_t(q) * 64 + k]);
            fprintf(stderr, "\n");
        }
    }
    if (!p) {
        p = new (std::nothrow) PassPlan();   // remember "no plan" for this key
        if (!p) return nullptr;
        p->row_bytes = row_bytes;
        p->window_kb = window_kb;
        p->max_passes = max_passes;
        p->n_pass = 0;
    }
    H->plans.push_back(p);
    return p->n_pass > 0 ? p : nullptr;
}

int get_stage_buffers(const hphi_ham* ham, size_t bytes, int count, void** out) {
    hphi_ham* H = const_cast<hphi_ham*>(ham);
    std::lock_guard<std::mutex> lock(H->plan_mu);
    for (int i = 0; i < count; ++i) {
        if (H->stage_bytes[i] < bytes) {
            if (H->d_stage[i]) (void)hipFree(H->d_stage[i]);
            H->d_stage[i] = nullptr;
            H->stage_bytes[i] = 0;
            if (dev_alloc(&H->d_stage[i], bytes, "staging buffer")) {
                H->d_stage[i] = nullptr;
                return 1;
            }
            H->stage_bytes[i] = bytes;
        }
        out[i] = H->d_stage[i];
    }
    return 0;
}

}  // namespace hphi
