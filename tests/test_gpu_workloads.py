"""GPU parity at the workloads' full sizes, in the launch configurations the
benchmark uses.

* 36-bit configurations (the kagome path) first on small sectors, checked
  completely against the oracle;
* the 24-site Kitaev-Heisenberg product with 16 complex64 vectors (tuned
  schedule, TPQ form u = -Hx/N + l x, FP64 reductions) against the C oracle
  over all 2^24 rows;
* the 4x3 Hubbard product (853,776 rows, FP64) against the C oracle;
* the 36-site kagome Sz = 0 sector (9,075,135,300 rows, FP32 storage):
  rank/unrank, element lists and product values on sampled rows, the oracle
  evaluating each row one by one through the combinatorial number system.
"""

import itertools

import numpy as np
import pytest
import torch

from synth import lattices as L
from synth.configs import BasisDesc, workload
from synth.vectors import device_uniform, uniform_vectors
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import c_oracle

pytestmark = pytest.mark.gpu

import paper_1703_03637_amd as hp  # noqa: E402


def _popcount_states(nbits, k):
    return np.array(sorted(sum(1 << b for b in c) for c in itertools.combinations(range(nbits), k)),
                    dtype=np.uint64)


def _elements(ham, row0, nrows, cap=128):
    cols, re, im, term, counts = (x.cpu().numpy() for x in hp.hphi_hv_elements(ham, row0, nrows, cap))
    assert counts.max() <= cap
    out = []
    for r in range(nrows):
        d = {}
        for k in range(counts[r]):
            key = (int(cols[r, k]), int(term[r, k]))
            assert key not in d
            d[key] = complex(re[r, k], im[r, k])
        out.append(d)
    return out


W64_CASES = {
    "kagome36_2sz34": (BasisDesc("spin", 36, "sz", two_sz=34), None),
    "kagome36_2sz32": (BasisDesc("spin", 36, "sz", two_sz=32), None),
    "hubbard18_1u1d": (BasisDesc("fermion", 18, "nupndn", n_up=1, n_dn=1), None),
}


def _w64_case(name):
    desc, _ = W64_CASES[name]
    if desc.particle == "spin":
        terms = [L.heisenberg_bond(i, j, 1.0) for (i, j) in L.kagome_bonds(3, 4)]
        k = (36 + desc.two_sz) // 2
        states = _popcount_states(36, k)
    else:
        terms = L.hubbard_terms(L.rect_bonds(6, 3), 18, t=1.0, U=8.0)
        ups = [1 << (2 * i) for i in range(18)]
        dns = [1 << (2 * i + 1) for i in range(18)]
        states = np.array(sorted(a | b for a in ups for b in dns), dtype=np.uint64)
    return desc, terms, states


@pytest.mark.parametrize("stage", [1, 2, 0])
@pytest.mark.parametrize("name", list(W64_CASES))
def test_w64_small_sectors_match_oracle(monkeypatch, name, stage):
    """36-bit configurations: rank/unrank, element lists (bit-exact) and FP64 products (1e-12), with
    the low rank from the two-level table in LDS (stage 1), from the full table through the caches
    (stage 2), and with every table in global memory (stage 0)."""
    monkeypatch.setenv("HPHI_STAGE_TABLES", str(stage))
    print(f"[gpu] w64 {name} stage={stage}", flush=True)
    desc, terms, states = _w64_case(name)
    basis = hp.hphi_basis_build(desc)
    assert basis.dim == len(states)
    ham = hp.hphi_ham_build(basis, terms)
    cfg = hp.hphi_basis_unrank(basis, torch.arange(basis.dim, device="cuda"))
    assert np.array_equal(cfg.cpu().numpy().astype(np.uint64), states)
    idx = hp.hphi_basis_rank(basis, torch.from_numpy(states.astype(np.int64)).cuda())
    assert np.array_equal(idx.cpu().numpy(), np.arange(basis.dim))
    gpu = _elements(ham, 0, basis.dim)
    ora = oh.row_elements(desc, terms, np.arange(basis.dim), basis_states=states)
    for r in range(basis.dim):
        o = {k: complex(v) for k, v in ora[r].items()}
        assert gpu[r].keys() == o.keys(), r
        for k in o:
            assert gpu[r][k] == o[k], (r, k)
    H = oh.sparse_h(desc, terms, basis_states=states)
    for nvec in (1, 2, 4):
        v = uniform_vectors(basis.dim, list(range(40, 40 + nvec)), True)
        vd = torch.from_numpy(v).cuda()
        if nvec == 1:
            vd = vd.reshape(-1)
        u = hp.hphi_hv(ham, vd).cpu().numpy().reshape(basis.dim, nvec)
        ref = H @ v
        bound = abs(H) @ np.abs(v)
        assert np.all(np.abs(u - ref) <= 1e-12 * bound + 1e-300)


@pytest.mark.parametrize("lpr", [2, 4])
@pytest.mark.parametrize("name", ["kagome36_2sz32", "hubbard18_1u1d"])
def test_w64_lanes_per_row(monkeypatch, name, lpr):
    """36-bit sector products with each row's 2 or 4 vectors split over lanes, FP64 and complex64."""
    monkeypatch.setenv("HPHI_LPR", str(lpr))
    print(f"[gpu] w64 lanes per row {name} lpr={lpr}", flush=True)
    desc, terms, states = _w64_case(name)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    H = oh.sparse_h(desc, terms, basis_states=states)
    for nvec in (2, 4):
        if lpr > nvec:
            continue
        v = uniform_vectors(basis.dim, list(range(50, 50 + nvec)), True)
        sx = torch.linspace(0.5, 1.5, nvec, dtype=torch.float64, device="cuda")
        for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 2e-6)):
            vd = torch.from_numpy(v).to(dt).cuda()
            red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
            u = hp.hphi_hv(ham, vd, in_scale=sx, reduce=red).cpu().numpy().astype(np.complex128)
            x = vd.cpu().numpy().astype(np.complex128) * sx.cpu().numpy()[None, :]
            ref = H @ x
            assert np.linalg.norm(u - ref) <= tol * np.linalg.norm(ref), (nvec, dt)
            red = red.cpu().numpy().reshape(4, nvec)
            for b in range(nvec):
                assert abs(red[1, b] - np.vdot(x[:, b], ref[:, b]).real) <= 10 * tol * np.linalg.norm(x[:, b]) * \
                    np.linalg.norm(ref[:, b]), (nvec, dt, b)


def _row_abs_sum_bound(terms, particle):
    """Upper bound on max_s sum_t |<s|H|t>|: each term's own maximum absolute row sum, from its
    dense matrix on the sites it touches (oracle)."""
    total = 0.0
    for t in terms:
        sites = sorted({t.i, t.j})
        relabel = {site: k for k, site in enumerate(sites)}
        t2 = t._replace(i=relabel[t.i], j=relabel[t.j])
        hd = oh.dense_h(BasisDesc(particle, len(sites)), [t2])
        total += float(np.abs(hd).sum(axis=1).max())
    return total


def test_kh_honeycomb24_full_product_matches_c_oracle():
    """All 2^24 rows of the batched TPQ product (16 complex64 vectors, tuned schedule)."""
    print("[gpu] kh_honeycomb24 full product vs C oracle", flush=True)
    w = workload("kh_honeycomb24")
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    dim, nvec, ns, l = basis.dim, w.nvec, w.basis.n_sites, w.tpq_l
    psi = device_uniform(dim, nvec, 911, True, torch.complex64)
    sched = hp.hphi_hv_tune(ham, psi)
    print(f"[gpu] schedule {sched}", flush=True)
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    u = hp.hphi_hv(ham, psi, a=-1.0 / ns, b=l, reduce=red).cpu().numpy()
    red = red.cpu().numpy().reshape(4, nvec)
    v = psi.cpu().numpy()
    del psi
    torch.cuda.empty_cache()
    hx = c_oracle.rows_hv(w.terms, np.arange(dim, dtype=np.uint64), v)
    # FP32 rounding of the FP64 result, plus (several passes) the FP32 rounding
    # of the partial row sum carried between passes, |P_s| <= (|H||v|)_s <= R |v|_max
    R = _row_abs_sum_bound(w.terms, "spin")
    for b in range(nvec):
        vb = v[:, b].astype(np.complex128)
        hb = hx[:, b]
        ref = -hb / ns + l * vb
        d = np.abs(u[:, b].astype(np.complex128) - ref)
        passes = sched["max_passes"] if sched["windowed"] else 1
        carry = 2.0 ** -24 * R * np.abs(vb).max() / ns if passes > 1 else 0.0
        bound = 2.0 ** -24 * np.abs(ref) * (1 + 1e-6) + carry + 1e-12 * (l * np.abs(vb) + np.abs(ref).max())
        if b == 0:
            print(f"[gpu] max |d|/bound = {float((d / bound).max()):.3f}, R = {R:.3f}", flush=True)
        assert np.all(d <= bound), b
        want = [np.vdot(vb, vb).real, np.vdot(vb, hb).real, np.vdot(hb, hb).real, np.vdot(ref, ref).real]
        scale = [want[0], np.linalg.norm(vb) * np.linalg.norm(hb), want[2], want[3]]
        # the reductions see H x with the carried partial rounded: |eps_s| <= c
        c = 2.0 ** -24 * R * np.abs(vb).max() if passes > 1 else 0.0
        carry_q = [0.0, c * np.abs(vb).sum(), 2 * c * np.abs(hb).sum() + dim * c * c,
                   2 * (c / ns) * np.abs(ref).sum() + dim * (c / ns) ** 2]
        for q in range(4):
            assert abs(red[q, b] - want[q]) <= 1e-11 * scale[q] + carry_q[q], (q, b, red[q, b], want[q])


def test_hubbard_4x3_full_product_matches_c_oracle():
    """All 853,776 rows of the FP64 Hubbard product (6 up + 6 down on the 4x3 open cluster)."""
    print("[gpu] hubbard_4x3 full product vs C oracle", flush=True)
    w = workload("hubbard_4x3")
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    states = ob.states(w.basis)
    assert basis.dim == len(states) == 853776
    vd = device_uniform(basis.dim, 1, 912, True, torch.complex128).reshape(-1).contiguous()
    u = hp.hphi_hv(ham, vd).cpu().numpy()
    v = vd.cpu().numpy()
    ref = c_oracle.rows_hv(w.terms, states, v, states=states)
    d = np.abs(u - ref)
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)
    assert d.max() <= 1e-12 * np.abs(ref).max() * 10


def test_kagome36_full_size_sampled_rows():
    """9,075,135,300 rows, FP32 storage (two vectors of 36 GB): sampled rows against the oracle's
    row-by-row evaluation; rank/unrank and element lists at random offsets and at the edges."""
    import math
    print("[gpu] kagome36 full size", flush=True)
    w = workload("kagome36_sz0")
    desc = w.basis
    basis = hp.hphi_basis_build(desc)
    dim = basis.dim
    assert dim == math.comb(36, 18)
    ham = hp.hphi_ham_build(basis, w.terms)
    rng = np.random.default_rng(913)
    rows = np.unique(np.concatenate([rng.integers(0, dim, 400), [0, 1, 2, dim - 3, dim - 2, dim - 1]]))
    cfg_ora = np.array([ob.cns_unrank(int(r), 18, 36) for r in rows], dtype=np.uint64)
    cfg = hp.hphi_basis_unrank(basis, torch.from_numpy(rows.astype(np.int64)).cuda()).cpu().numpy()
    assert np.array_equal(cfg.astype(np.uint64), cfg_ora)
    idx = hp.hphi_basis_rank(basis, torch.from_numpy(cfg_ora.astype(np.int64)).cuda()).cpu().numpy()
    assert np.array_equal(idx, rows)

    def cns_rank_arr(st):
        return np.array([ob.cns_rank(int(s)) for s in st], dtype=np.int64)

    # element lists of contiguous blocks (bit-exact indices, terms and values)
    for row0 in (0, int(rng.integers(0, dim - 64)), dim - 64):
        gpu = _elements(ham, row0, 64)
        st = np.array([ob.cns_unrank(row0 + k, 18, 36) for k in range(64)], dtype=np.uint64)
        ora = oh.row_elements_sampled(desc, w.terms, st, cns_rank_arr)
        for k in range(64):
            o = {kk: complex(vv) for kk, vv in ora[k].items()}
            assert gpu[k].keys() == o.keys(), (row0, k)
            for kk in o:
                assert gpu[k][kk] == o[kk]
    # the product on sampled rows (FP32 vectors, FP64 arithmetic)
    v = device_uniform(dim, 0, 914, False, torch.float32)
    u = torch.empty_like(v)
    hp.hphi_hv(ham, v, u)
    torch.cuda.synchronize()
    u_rows = u[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy().astype(np.float64)
    del u

    def v_of_state(st):
        ix = torch.from_numpy(cns_rank_arr(st)).cuda()
        return v[ix].cpu().numpy().astype(np.float64)

    ref = oh.rows_hv_sampled(desc, w.terms, cfg_ora, v_of_state).real
    # |H||v| per row from the same element lists
    bound = np.zeros(len(rows))
    for term in w.terms:
        for coef, tgt in oh.term_action(term, cfg_ora, desc.particle):
            nz = np.nonzero(coef != 0)[0]
            if nz.size:
                bound[nz] += np.abs(coef[nz]) * np.abs(v_of_state(tgt[nz]))
    d = np.abs(u_rows - ref)
    assert np.all(d <= 2.0 ** -24 * np.abs(ref) + 1e-12 * bound + 1e-30)
    del v
    torch.cuda.empty_cache()


def test_hubbard18_full_size_sampled_rows():
    """The paper's 18-site Hubbard cluster at half filling, Sz = 0 (2,363,904,400 rows, 36-bit
    interleaved fermion configurations): rank/unrank, element lists (bit-exact) and products on
    sampled rows -- complex128, and the 4-sample complex64 TPQ step -- against the oracle, which ranks
    every target by counting (no basis list)."""
    print("[gpu] hubbard18 full size", flush=True)
    w = workload("hubbard18_tpq")
    desc = w.basis
    basis = hp.hphi_basis_build(desc)
    dim = basis.dim
    assert dim == 2363904400
    ham = hp.hphi_ham_build(basis, w.terms)
    rng = np.random.default_rng(915)
    rows = np.unique(np.concatenate([rng.integers(0, dim, 200), [0, 1, dim - 2, dim - 1]]))
    cfg_ora = np.array([ob.sector_unrank(desc, int(r)) for r in rows], dtype=np.uint64)
    cfg = hp.hphi_basis_unrank(basis, torch.from_numpy(rows.astype(np.int64)).cuda()).cpu().numpy()
    assert np.array_equal(cfg.astype(np.uint64), cfg_ora)
    idx = hp.hphi_basis_rank(basis, torch.from_numpy(cfg_ora.astype(np.int64)).cuda()).cpu().numpy()
    assert np.array_equal(idx, rows)

    def rank_arr(st):
        return np.array([ob.sector_rank(desc, int(s)) for s in st], dtype=np.int64)

    for row0 in (0, int(rng.integers(0, dim - 64)), dim - 64):
        gpu = _elements(ham, row0, 64)
        st = np.array([ob.sector_unrank(desc, row0 + k) for k in range(64)], dtype=np.uint64)
        ora = oh.row_elements_sampled(desc, w.terms, st, rank_arr)
        for k in range(64):
            o = {kk: complex(vv) for kk, vv in ora[k].items()}
            assert gpu[k].keys() == o.keys(), (row0, k)
            for kk in o:
                assert gpu[k][kk] == o[kk]

    def sampled_check(vec, out, a, b, tol_store):
        def v_of_state(st):
            ix = torch.from_numpy(rank_arr(st)).cuda()
            return vec[ix].cpu().numpy().astype(np.complex128)
        hv = oh.rows_hv_sampled(desc, w.terms, cfg_ora, v_of_state)
        vr = v_of_state(cfg_ora)
        ref = a * hv + b * vr
        bound = np.zeros(hv.shape)
        for term in w.terms:
            for coef, tgt in oh.term_action(term, cfg_ora, desc.particle):
                nz = np.nonzero(coef != 0)[0]
                if nz.size:
                    vals = np.abs(v_of_state(tgt[nz]))
                    bound[nz] += np.abs(coef[nz])[:, None] * vals if vals.ndim == 2 else np.abs(coef[nz]) * vals
        got = out[torch.from_numpy(rows.astype(np.int64)).cuda()].cpu().numpy().astype(np.complex128)
        d = np.abs(got - ref)
        assert np.all(d <= tol_store * np.abs(ref) + 1e-12 * (abs(a) * bound + abs(b) * np.abs(vr)) + 1e-30)

    # complex128 product, one vector
    v = device_uniform(dim, 0, 916, True, torch.complex128)
    u = torch.empty_like(v)
    hp.hphi_hv(ham, v, u)
    torch.cuda.synchronize()
    sampled_check(v, u, 1.0, 0.0, 0.0)
    del v, u
    torch.cuda.empty_cache()
    # batched complex64 TPQ step, four samples
    ns, l = desc.n_sites, w.tpq_l
    psi = device_uniform(dim, 4, 917, True, torch.complex64)
    out = torch.empty_like(psi)
    obs = torch.empty(16, dtype=torch.float64, device="cuda")
    hp.hphi_tpq_step(ham, psi, out, l, 1, None, obs)
    torch.cuda.synchronize()
    sampled_check(psi, out, -1.0 / ns, l, 2.0 ** -24 * (1 + 1e-6))
    o = obs.cpu().numpy().reshape(4, 4)
    assert np.all(np.isfinite(o)) and np.all(np.abs(o[0]) < 8.5)
    del psi, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nvec", [1, 4])
@pytest.mark.parametrize("name", ["kagome36_2sz32", "hubbard18_1u1d"])
def test_w64_tuned_schedule_matches_oracle(name, nvec):
    """The autotuner on a 36-bit sector: every candidate it times (table modes 0, 1 and 2, resident
    blocks 0, 4 and 6, the block-staged kernel) runs on this basis, and the product under the pinned
    schedule matches the oracle (FP64, 1e-12 per element)."""
    print(f"[gpu] w64 tuned {name} nvec={nvec}", flush=True)
    desc, terms, states = _w64_case(name)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    v = uniform_vectors(basis.dim, list(range(70, 70 + nvec)), True)
    vd = torch.from_numpy(v).cuda()
    if nvec == 1:
        vd = vd.reshape(-1).contiguous()
    sched = hp.hphi_hv_tune(ham, vd)
    assert sched["us"] > 0
    if sched["sector_blocks"] == 0:
        assert sched["stage_tables"] in (0, 1, 2) and sched["blocks_per_cu"] in (0, 4, 6), sched
    u = hp.hphi_hv(ham, vd).cpu().numpy().reshape(basis.dim, nvec)
    H = oh.sparse_h(desc, terms, basis_states=states)
    ref = H @ v
    bound = abs(H) @ np.abs(v)
    assert np.all(np.abs(u - ref) <= 1e-12 * bound + 1e-300), sched
