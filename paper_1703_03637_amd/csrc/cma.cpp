// Dense-block plans of the product, after the continuous-memory-access
// method (Sec. 4.3): any sum of terms acting on M sites is a dense
// 2^M x 2^M matrix on the 2^M configurations of those sites, applied to
// every block of rows that agree on all other sites.  The paper brings each
// group of sites to the lowest bits by permuting the vector; here the
// product kernel gathers a block's rows through the cluster's bit
// positions instead, so the vector is never permuted.
//
// Plan: the operators are covered greedily by clusters of M bits (each
// cluster maximizes the operators it completes, then the operators it
// touches; deterministic); every operator joins the first cluster that
// holds all of its bits; the cluster's dense matrix is the sum of its
// operators' elements in the pull form u[r] += H_c[r][t] v[t].
#include <cstdio>
#include <cstdlib>
#include <new>

#include "hphi_internal.h"

namespace hphi {
namespace {

uint64_t support(const DevOp& o) {
    return (uint64_t(1) << o.bi) | (uint64_t(1) << o.bj) | (o.has_off ? o.xmask : 0);
}

CmaPlan* build_cma_plan(const hphi_ham* H, int M) {
    const int nbits = H->basis->nbits;
    const std::vector<DevOp>& ops = H->ops;
    const int n_ops = int(ops.size());
    CmaPlan* P = new (std::nothrow) CmaPlan();
    if (!P) return nullptr;
    P->M = M;
    std::vector<int> stage_of(n_ops, -1);
    std::vector<std::vector<int>> clusters;
    std::vector<int> remaining;
    for (int o = 0; o < n_ops; ++o) remaining.push_back(o);
    while (!remaining.empty()) {
        uint64_t in = 0;
        for (int n = 0; n < M; ++n) {
            int best = -1;
            long best_score = -1;
            for (int c = 0; c < nbits; ++c) {
                if ((in >> c) & 1) continue;
                const uint64_t T = in | (uint64_t(1) << c);
                long gain = 0, touch = 0;
                for (int o : remaining) {
                    const uint64_t m = support(ops[o]);
                    if (!((m >> c) & 1)) continue;
                    ++touch;
                    if ((m & ~T) == 0) ++gain;
                }
                const long score = gain * 1024 + touch;
                if (score > best_score) {
                    best_score = score;
                    best = c;
                }
            }
            in |= uint64_t(1) << best;
        }
        std::vector<int> rest;
        for (int o : remaining) {
            if ((support(ops[o]) & ~in) == 0) stage_of[o] = int(clusters.size());
            else rest.push_back(o);
        }
        if (rest.size() == remaining.size()) {
            delete P;
            return nullptr;
        }
        remaining.swap(rest);
        std::vector<int> bits;
        for (int b = 0; b < nbits; ++b)
            if ((in >> b) & 1) bits.push_back(b);
        clusters.push_back(bits);
    }
    if (clusters.empty()) {   // no operators: one cluster of the lowest bits (H = 0)
        std::vector<int> bits;
        for (int b = 0; b < M; ++b) bits.push_back(b);
        clusters.push_back(bits);
    }
    P->n_stage = int(clusters.size());
    P->bits.assign(size_t(P->n_stage) * 64, 0);
    P->n_ops.assign(P->n_stage, 0);
    const size_t D = size_t(1) << M;
    std::vector<double> hd(size_t(P->n_stage) * D * D, 0.0);
    for (int c = 0; c < P->n_stage; ++c) {
        int32_t* bl = &P->bits[size_t(c) * 64];
        int local[64];
        for (int b = 0; b < 64; ++b) local[b] = -1;
        int k = 0;
        for (int b : clusters[c]) {
            local[b] = k;
            bl[k++] = b;
        }
        for (int b = 0; b < nbits; ++b)
            if (local[b] < 0) bl[k++] = b;
        double* Hc = &hd[size_t(c) * D * D];
        for (int o = 0; o < n_ops; ++o) {
            if (stage_of[o] != c) continue;
            ++P->n_ops[c];
            const DevOp& op = ops[o];
            const int li = local[op.bi], lj = local[op.bj];
            uint32_t xm = 0;
            if (op.has_off)
                for (int b = 0; b < nbits; ++b)
                    if ((op.xmask >> b) & 1) xm |= 1u << local[b];
            for (uint32_t r = 0; r < D; ++r) {
                const int p = int((r >> li) & 1) | (int((r >> lj) & 1) << 1);
                Hc[size_t(r) * D + r] += op.d[p];
                if (op.has_off && xm != 0 && op.cr[p] != 0.0) Hc[size_t(r) * D + (r ^ xm)] += op.cr[p];
            }
        }
    }
    std::vector<float> hf(hd.size());
    for (size_t i = 0; i < hd.size(); ++i) hf[i] = float(hd[i]);
    if (dev_alloc((void**)&P->d_hd, hd.size() * sizeof(double), "dense-block plan") ||
        dev_alloc((void**)&P->d_hf, hf.size() * sizeof(float), "dense-block plan") ||
        dev_alloc((void**)&P->d_bits, P->bits.size() * sizeof(int32_t), "dense-block plan")) {
        if (P->d_hd) (void)hipFree(P->d_hd);
        if (P->d_hf) (void)hipFree(P->d_hf);
        delete P;
        return nullptr;
    }
    hipError_t e = hipMemcpy(P->d_hd, hd.data(), hd.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(P->d_hf, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(P->d_bits, P->bits.data(), P->bits.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(P->d_hd);
        (void)hipFree(P->d_hf);
        (void)hipFree(P->d_bits);
        delete P;
        return nullptr;
    }
    return P;
}

}  // namespace

int get_cma_plan(const hphi_ham* ham, int M, const CmaPlan** out) {
    hphi_ham* H = const_cast<hphi_ham*>(ham);
    const hphi_basis* B = H->basis;
    *out = nullptr;
    if (B->desc.particle != HPHI_SPIN_HALF || B->dev.sector != 0 || B->nbits < 6 || B->nbits > 32)
        return set_error(HPHI_EINVAL, "dense-block product: spin-1/2 full spaces of 6..32 sites only");
    if (H->is_complex) return set_error(HPHI_EDTYPE, "dense-block product: real matrix elements only");
    if (M < 4 || M > 7 || M > B->nbits)
        return set_error(HPHI_EINVAL, "dense-block product: cluster_bits must be in 4..7 and at most %d", B->nbits);
    for (const DevOp& o : H->ops) {
        uint64_t m = support(o);
        int c = 0;
        for (; m; m &= m - 1) ++c;
        if (c > M)
            return set_error(HPHI_EINVAL, "dense-block product: a term spans %d sites, more than cluster_bits = %d",
                             c, M);
    }
    std::lock_guard<std::mutex> lock(H->plan_mu);
    for (CmaPlan* p : H->cma_plans)
        if (p->M == M) {
            *out = p;
            return HPHI_OK;
        }
    CmaPlan* p = build_cma_plan(H, M);
    if (!p) return set_error(HPHI_ENOMEM, "dense-block product: plan construction failed");
    if (getenv("HPHI_DEBUG")) {
        fprintf(stderr, "[hphi] dense-block plan M=%d clusters=%d operators/cluster:", M, p->n_stage);
        for (int c = 0; c < p->n_stage; ++c) fprintf(stderr, " %d", p->n_ops[c]);
        fprintf(stderr, "\n");
    }
    H->cma_plans.push_back(p);
    *out = p;
    return HPHI_OK;
}

}  // namespace hphi
