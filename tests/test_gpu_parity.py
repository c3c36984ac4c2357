"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: element lists (indices, term ids, signs) bit-exact; FP64 H.v within
1e-12 relative, norm-wise and component-wise against |H||v|; FP32 storage
within a bound derived from FP32 rounding; reductions, Lanczos and TPQ
against the oracle's literal recurrences.
"""

import numpy as np
import pytest
import torch

from synth import lattices as L
from synth.configs import BasisDesc, workload, kh_honeycomb_terms
from synth.vectors import device_uniform, gaussian_vectors, uniform_vectors
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import solvers as osv

pytestmark = pytest.mark.gpu

import paper_1703_03637_amd as hp  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    print(f"[gpu] {torch.cuda.get_device_name(0)} lib={hp.LIB_PATH}", flush=True)


SMALL_CASES = {
    "spin_full_complex": (BasisDesc("spin", 7),
                          lambda: L.random_spin_terms(7, 10, 101, conserve_sz=False, fields=True, real=False)),
    "spin_full_real": (BasisDesc("spin", 8),
                       lambda: L.random_spin_terms(8, 12, 102, conserve_sz=False, fields=True, real=True)),
    "spin_sz_dm": (BasisDesc("spin", 10, "sz", two_sz=2),
                   lambda: L.random_spin_terms(10, 14, 103, conserve_sz=True, fields=True, real=False)),
    "spin_sz_split3": (BasisDesc("spin", 11, "sz", two_sz=-1, split_bits=3),
                       lambda: L.random_spin_terms(11, 15, 104, conserve_sz=True, real=True)),
    "ferm_nupndn": (BasisDesc("fermion", 5, "nupndn", n_up=2, n_dn=3),
                    lambda: L.random_fermion_terms(5, 12, 105, conserve_spin=True, real=False, n_dens=3,
                                                   with_mu=True)),
    "ferm_full": (BasisDesc("fermion", 3),
                  lambda: L.random_fermion_terms(3, 8, 106, conserve_spin=False, real=False, n_dens=2,
                                                 with_mu=True)),
    "ferm_ntot": (BasisDesc("fermion", 4, "ntot", n_tot=3),
                  lambda: L.random_fermion_terms(4, 10, 107, conserve_spin=False, real=True, n_dens=2)),
    "hubbard_3x3": (BasisDesc("fermion", 9, "nupndn", n_up=3, n_dn=4),
                    lambda: L.hubbard_terms(L.rect_bonds(3, 3), 9, t=1.0, U=8.0)),
    "kh_honeycomb12": (BasisDesc("spin", 12), lambda: kh_honeycomb_terms(lx=3, ly=2, random_dirs=False)),
    "ring4": (BasisDesc("spin", 4), lambda: [L.heisenberg_bond(i, j) for i, j in L.chain_bonds(4)]),
}


def _case(name):
    desc, mk = SMALL_CASES[name]
    terms = mk()
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    return desc, terms, basis, ham


def _gpu_elements(ham, rows0, nrows, cap=64):
    cols, re, im, term, counts = hp.hphi_hv_elements(ham, rows0, nrows, cap)
    cols, re, im, term, counts = (x.cpu().numpy() for x in (cols, re, im, term, counts))
    assert counts.max() <= cap
    out = []
    for r in range(nrows):
        d = {}
        for k in range(counts[r]):
            key = (int(cols[r, k]), int(term[r, k]))
            assert key not in d, "duplicate (col, term) from one row"
            d[key] = complex(re[r, k], im[r, k])
        out.append(d)
    return out


def _compare_elements(gpu, ora, exact_values, diag_tol=None):
    """Element lists per row: the off-diagonal (col, term) sets, signs and values; with diag_tol the
    diagonal (a sum of the operators' diagonal parts, term -1) is compared as a number within diag_tol
    (a multi-pass product sums it pass by pass, so it may differ in the last bits or vanish in one
    order and not the other)."""
    for r, (g, o) in enumerate(zip(gpu, ora)):
        if diag_tol is not None:
            g, o = dict(g), dict(o)
            gd, od = g.pop((r + _compare_elements.row0, -1), 0.0), o.pop((r + _compare_elements.row0, -1), 0.0)
            assert abs(gd - od) <= diag_tol, f"row {r}: diagonal {gd} vs {od}"
        assert g.keys() == o.keys(), f"row {r}: index/term sets differ"
        for key, val in o.items():
            gv = g[key]
            if exact_values:
                assert gv == val, f"row {r} {key}: {gv} != {val}"
            else:
                assert abs(gv - val) <= 4e-16 * max(1.0, abs(val)), f"row {r} {key}: {gv} vs {val}"
            # signs are integer data: bit-exact
            assert np.sign(gv.real) == np.sign(val.real) and np.sign(gv.imag) == np.sign(val.imag)


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_element_lists_match_oracle(name):
    print(f"[gpu] elements {name}", flush=True)
    desc, terms, basis, ham = _case(name)
    st = ob.states(desc)
    assert basis.dim == len(st)
    gpu = _gpu_elements(ham, 0, basis.dim)
    ora = oh.row_elements(desc, terms, np.arange(len(st)), st)
    ora = [ora[i] for i in range(len(st))]
    fermion = desc.particle == "fermion"
    # the diagonal is the sum of every operator's diagonal part (Sec. 3.3) in the
    # kernel's operator order (the windowed plan orders a pass's operators by their
    # in-tile flip mask): compared within a summation bound, the rest exactly
    scale = max(sum(abs(x) for x in t.c) for t in terms) * len(terms)
    _compare_elements(gpu, ora, exact_values=fermion, diag_tol=1e-15 * scale)


def test_element_lists_chain16_rows():
    w = workload("heis_chain16")
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    rows = [0, 1, 12345, 40000, 65535]
    for r in rows:
        g = _gpu_elements(ham, r, 1)[0]
        o = oh.row_elements_sampled(w.basis, w.terms, np.array([r], np.uint64), lambda x: x.astype(np.int64))[0]
        _compare_elements([g], [o], exact_values=True)


def test_element_lists_hubbard_4x3_sampled_rows():
    w = workload("hubbard_4x3")
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    st = ob.states(w.basis)
    assert basis.dim == len(st) == 853776
    rng = np.random.default_rng(5)
    rows = np.concatenate([[0, 1, len(st) - 1], rng.integers(0, len(st), 200)])
    ora = oh.row_elements_sampled(w.basis, w.terms, st[rows], lambda x: ob.rank(st, x))
    for r, o in zip(rows, ora):
        g = _gpu_elements(ham, int(r), 1)[0]
        _compare_elements([g], [o], exact_values=True)


def _export_lists(ham, nrows, nvec, dtype, cap=64):
    cols, re, im, term, counts = hp.hphi_hv_elements(ham, 0, nrows, cap, nvec=nvec, dtype=dtype)
    cols, re, im, term, counts = (x.cpu().numpy() for x in (cols, re, im, term, counts))
    assert counts.max() <= cap
    out = []
    for r in range(nrows):
        d = {}
        for k in range(counts[r]):
            key = (int(cols[r, k]), int(term[r, k]))
            assert key not in d, "duplicate (col, term) from one row"
            d[key] = complex(re[r, k], im[r, k])
        out.append(d)
    return out


EXPORT_LAYOUTS = [(1, torch.complex128, 0), (16, torch.complex64, 4), (16, torch.complex64, 8),
                  (8, torch.complex128, 2), (16, torch.complex128, 2), (4, torch.complex64, 1)]


@pytest.mark.parametrize("nvec,dtype,lpr", EXPORT_LAYOUTS)
@pytest.mark.parametrize("windowed,window_kb,passes", [(0, 2048, 1), (1, 2048, 1), (1, 1, 3), (1, 2, 2),
                                                       (2, 1, 3), (2, 2, 2)])
@pytest.mark.parametrize("name", ["kh_honeycomb12", "spin_full_complex", "spin_full_real", "ferm_full"])
def test_element_export_full_space_product_paths(monkeypatch, name, windowed, window_kb, passes, nvec, dtype, lpr):
    """Sec. 3.3 decode exported by the product kernels themselves on full spaces: the single-pass
    kernel and the windowed kernel with 1 to 3 passes, gathering from v or from staged copies (flip
    masks in processing-index bits), partners inside the 64-row tile read from the LDS tile (rows of
    at most 128 bytes, at most 4 lanes per row) or exchanged between lanes (8 lanes per row, or
    256-byte rows).  Index, term and sign lists bit-exact against the oracle."""
    print(f"[gpu] export {name} windowed={windowed} kb={window_kb} passes={passes} nvec={nvec} {dtype} lpr={lpr}",
          flush=True)
    for k, val in (("HPHI_WINDOWED", windowed), ("HPHI_L2_WINDOW_KB", window_kb), ("HPHI_PASSES", passes),
                   ("HPHI_LPR", lpr)):
        monkeypatch.setenv(k, str(val))
    desc, terms, basis, ham = _case(name)
    st = ob.states(desc)
    gpu = _export_lists(ham, basis.dim, nvec, dtype)
    ora = oh.row_elements(desc, terms, np.arange(len(st)), st)
    scale = max(sum(abs(x) for x in t.c) for t in terms) * len(terms)
    _compare_elements(gpu, [ora[i] for i in range(len(st))], exact_values=False, diag_tol=1e-15 * scale)


@pytest.mark.parametrize("nvec,dtype,lpr", [(1, torch.complex128, 0), (4, torch.complex64, 2),
                                            (4, torch.complex128, 4), (16, torch.complex64, 8),
                                            (2, torch.complex64, 1)])
@pytest.mark.parametrize("stage", [0, 1])
@pytest.mark.parametrize("name", ["spin_sz_dm", "spin_sz_split3", "ferm_nupndn", "ferm_ntot", "hubbard_3x3"])
def test_element_export_sector_product_paths(monkeypatch, name, stage, nvec, dtype, lpr):
    """The sector product's own decode (tile-uniform high-half rank, the row's own low rank when an
    operator leaves the low half alone, the low rank table in LDS or global memory, fermion parity)
    exported for every row: bit-exact against the oracle."""
    print(f"[gpu] export sector {name} stage={stage} nvec={nvec} {dtype} lpr={lpr}", flush=True)
    monkeypatch.setenv("HPHI_STAGE_TABLES", str(stage))
    monkeypatch.setenv("HPHI_LPR", str(lpr))
    desc, terms, basis, ham = _case(name)
    st = ob.states(desc)
    gpu = _export_lists(ham, basis.dim, nvec, dtype)
    ora = oh.row_elements(desc, terms, np.arange(len(st)), st)
    _compare_elements(gpu, [ora[i] for i in range(len(st))], exact_values=desc.particle == "fermion")


def test_element_export_row_windows_and_errors():
    """Row windows that start and end inside tiles and high halves give the rows of the full export;
    real storage types, too many rows and bad ranges are rejected."""
    desc, terms, basis, ham = _case("hubbard_3x3")
    full = _export_lists(ham, basis.dim, 1, torch.complex128)
    for r0, n in ((0, 1), (37, 100), (basis.dim - 70, 70), (63, 2), (1000, 1)):
        cols, re, im, term, counts = (x.cpu().numpy() for x in hp.hphi_hv_elements(ham, r0, n, 64))
        for r in range(n):
            got = {(int(cols[r, k]), int(term[r, k])): complex(re[r, k], im[r, k]) for k in range(counts[r])}
            assert got == full[r0 + r]
    for bad in (dict(nvec=3), dict(dtype=torch.float64)):
        with pytest.raises((hp.HphiError, KeyError)):
            hp.hphi_hv_elements(ham, 0, 4, 8, **bad)
    with pytest.raises(hp.HphiError):
        hp.hphi_hv_elements(ham, basis.dim - 1, 2, 8)


_compare_elements.row0 = 0


def _abs_bound(desc, terms, st, v):
    H = oh.sparse_h(desc, terms, st)
    Ha = abs(H)
    return Ha @ np.abs(v), H


def _to_dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("name", list(SMALL_CASES))
@pytest.mark.parametrize("nvec", [1, 4, 16])
def test_hv_fp64_matches_oracle(name, nvec):
    print(f"[gpu] hv fp64 {name} nvec={nvec}", flush=True)
    desc, terms, basis, ham = _case(name)
    st = ob.states(desc)
    cplx = ham.is_complex or nvec == 4
    v = uniform_vectors(len(st), list(range(7, 7 + nvec)), cplx)
    dt = torch.complex128 if cplx else torch.float64
    vd = _to_dev(v if cplx else v.real, dt)
    if nvec == 1:
        vd = vd.reshape(-1)
    u = hp.hphi_hv(ham, vd).cpu().numpy().reshape(len(st), nvec)
    bound, H = _abs_bound(desc, terms, st, v)
    ref = H @ v
    err = np.abs(u - ref)
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref) + 1e-300
    assert np.all(err <= 1e-12 * bound + 1e-300)


@pytest.mark.parametrize("name", ["spin_sz_dm", "ferm_nupndn", "kh_honeycomb12", "hubbard_3x3"])
@pytest.mark.parametrize("nvec", [1, 8])
def test_hv_fp32_storage(name, nvec):
    """FP32 storage: loads, coefficients and row sums in FP32; bound = 8 eps32 (|H||v|) per element."""
    desc, terms, basis, ham = _case(name)
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(20, 20 + nvec)), True)
    dt = torch.complex64
    if not ham.is_complex and nvec == 1:
        v = v.real.copy()
        dt = torch.float32
    vd = _to_dev(v, dt)
    if nvec == 1:
        vd = vd.reshape(-1)
    v32 = vd.cpu().numpy().astype(np.complex128).reshape(len(st), nvec)
    u = hp.hphi_hv(ham, vd).cpu().numpy().astype(np.complex128).reshape(len(st), nvec)
    bound, H = _abs_bound(desc, terms, st, v32)
    ref = H @ v32
    n_terms = max(8, len(terms))
    assert np.all(np.abs(u - ref) <= n_terms * 6e-8 * bound + 1e-30)


@pytest.mark.parametrize("nvec", [1, 2, 16])
def test_hv_epilogue_and_reductions(nvec):
    desc, terms, basis, ham = _case("spin_sz_dm")
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(30, 30 + nvec)), True)
    vd = _to_dev(v, torch.complex128)
    if nvec == 1:
        vd = vd.reshape(-1)
    scale = torch.tensor(np.linspace(0.5, 2.0, nvec), dtype=torch.float64, device="cuda")
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    a, b = -0.37, 1.25
    u = hp.hphi_hv(ham, vd, a=a, b=b, in_scale=scale, reduce=red).cpu().numpy().reshape(len(st), nvec)
    H = oh.sparse_h(desc, terms, st)
    x = v * scale.cpu().numpy()[None, :]
    hx = H @ x
    ref = a * hx + b * x
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)
    red = red.cpu().numpy().reshape(4, nvec)
    for bb in range(nvec):
        want = [np.vdot(x[:, bb], x[:, bb]).real, np.vdot(x[:, bb], hx[:, bb]).real,
                np.vdot(hx[:, bb], hx[:, bb]).real, np.vdot(ref[:, bb], ref[:, bb]).real]
        assert np.allclose(red[:, bb], want, rtol=1e-12, atol=0)
    # reduce-only mode (no output vector) gives the same sums
    red2 = torch.empty_like(torch.from_numpy(red.reshape(-1))).cuda()
    hp.hphi_hv(ham, vd, a=a, b=b, in_scale=scale, reduce=red2, write=False)
    assert np.array_equal(red2.cpu().numpy().reshape(4, nvec), red)


def test_batched_rows_bitwise_equal_single():
    """Interleaved batch: each vector's output equals its single-vector product bit for bit."""
    desc, terms, basis, ham = _case("kh_honeycomb12")
    v = uniform_vectors(basis.dim, list(range(40, 56)), True)
    vd = _to_dev(v, torch.complex64)
    ub = hp.hphi_hv(ham, vd).cpu()
    for bb in (0, 5, 15):
        us = hp.hphi_hv(ham, vd[:, bb].contiguous()).cpu()
        assert torch.equal(ub[:, bb], us)


@pytest.mark.parametrize("name", ["spin_sz_dm", "spin_sz_split3", "ferm_nupndn", "ferm_ntot", "hubbard_3x3"])
def test_rank_unrank_round_trip(name):
    desc, terms, basis, ham = _case(name)
    st = ob.states(desc)
    idx = torch.arange(basis.dim, dtype=torch.int64, device="cuda")
    cfg = hp.hphi_basis_unrank(basis, idx).cpu().numpy().astype(np.uint64)
    assert np.array_equal(cfg, st)
    r = hp.hphi_basis_rank(basis, torch.from_numpy(st.astype(np.int64)).cuda()).cpu().numpy()
    assert np.array_equal(r, np.arange(basis.dim))
    nb = ob.n_bits(desc)
    allst = np.arange(1 << nb, dtype=np.uint64)
    outside = allst[~ob.in_sector(desc, allst)][:500]
    r2 = hp.hphi_basis_rank(basis, torch.from_numpy(outside.astype(np.int64)).cuda()).cpu().numpy()
    assert np.all(r2 == -1)
    bad = hp.hphi_basis_unrank(basis, torch.tensor([-1, basis.dim], dtype=torch.int64, device="cuda")).cpu()
    assert np.all(bad.numpy().astype(np.uint64) == np.uint64(2 ** 64 - 1))


def test_error_paths():
    desc = BasisDesc("spin", 12, "sz", two_sz=0)
    basis = hp.hphi_basis_build(desc)
    with pytest.raises(hp.HphiError) as e:
        hp.hphi_ham_build(basis, kh_honeycomb_terms(lx=3, ly=2, random_dirs=False))
    assert e.value.code == -4      # ESECTOR: Kitaev pair flips leave the Sz sector
    with pytest.raises(hp.HphiError) as e:
        hp.hphi_ham_build(basis, [L.Term(L.SPIN_FIELD, 0, -1, (0.3, 0.0, 0.0))])
    assert e.value.code == -4
    with pytest.raises(hp.HphiError) as e:
        hp.hphi_ham_build(basis, [L.heisenberg_bond(0, 0)])
    assert e.value.code == -1
    with pytest.raises(hp.HphiError) as e:
        hp.hphi_ham_build(basis, [L.Term(L.HOP, 0, 1, (1.0, 0.0))])
    assert e.value.code == -1
    dm = [L.Term(L.SPIN_BOND, 0, 1, (1.0, 0.4, 0.0, -0.4, 1.0, 0.0, 0.0, 0.0, 1.0))]
    ham = hp.hphi_ham_build(basis, dm)
    assert ham.is_complex
    v = torch.zeros(basis.dim, dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HphiError) as e:
        hp.hphi_hv(ham, v)
    assert e.value.code == -5      # EDTYPE
    vc = torch.zeros(basis.dim, 3, dtype=torch.complex128, device="cuda")
    with pytest.raises(hp.HphiError) as e:
        hp.hphi_hv(ham, vc)
    assert e.value.code == -1      # nvec = 3
    import ctypes as C
    from paper_1703_03637_amd import _lib
    vv = torch.zeros(basis.dim, dtype=torch.complex128, device="cuda")
    rc = _lib.lib().hphi_hv(C.c_void_p(ham.handle), vv.data_ptr(), vv.data_ptr(), 1, _lib.HPHI_C128, None, None)
    assert rc == -1                # u aliases v


# ------------------------------------------------------------------ Lanczos

def _lanczos_case(wname, dtype=torch.complex128, n_iter=None, use_graph=True):
    w = workload(wname)
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    cplx = dtype.is_complex
    x0 = gaussian_vectors(basis.dim, w.seeds[:1], cplx)[:, 0]
    x0d = _to_dev(x0 if cplx else x0.real, dtype)
    res = hp.hphi_lanczos([ham], [x0d], n_iter or w.n_iter, use_graph=use_graph)[0]
    return w, basis, ham, x0d.cpu().numpy(), res


def test_lanczos_ring4_breakdown_at_dim():
    w, basis, ham, x0, res = _lanczos_case("heis_ring4", torch.float64, 16)
    assert res["n_done"] <= 16 and res["info"] == 1
    assert abs(res["e0_ritz"] - (-2.0)) < 1e-12
    assert abs(res["e0_refined"] - (-2.0)) < 1e-12


def test_lanczos_two_site_hubbard():
    w, basis, ham, x0, res = _lanczos_case("hubbard_2site", torch.float64, 4)
    assert abs(res["e0_ritz"] - (8 - np.sqrt(64 + 16)) / 2) < 1e-12


def test_lanczos_chain16_matches_oracle_and_bethe():
    w, basis, ham, x0, res = _lanczos_case("heis_chain16")
    H = oh.sparse_h(w.basis, w.terms)
    a, b = osv.lanczos(lambda v: H @ v, x0.astype(np.complex128), w.n_iter, basis.dim)
    assert np.allclose(res["alpha"][:30], a[:30], rtol=0, atol=1e-10)
    assert np.allclose(res["beta"][:30], b[:30], rtol=0, atol=1e-10)
    e_bethe = -7.142296360616757
    assert abs(res["e0_ritz"] - e_bethe) < 1e-10
    assert abs(res["e0_refined"] - e_bethe) < 1e-10
    assert res["residual"] < 1e-4


def test_lanczos_graph_replay_is_bitwise_identical():
    _, _, _, _, r1 = _lanczos_case("heis_chain12", n_iter=60, use_graph=True)
    _, _, _, _, r2 = _lanczos_case("heis_chain12", n_iter=60, use_graph=False)
    assert np.array_equal(r1["alpha"], r2["alpha"]) and np.array_equal(r1["beta"], r2["beta"])
    assert r1["e0_refined"] == r2["e0_refined"]


def test_lanczos_hubbard_3x3_vs_dense():
    desc, terms, basis, ham = _case("hubbard_3x3")
    H = oh.sparse_h(desc, terms)
    e = np.linalg.eigvalsh(H.toarray())
    x0 = gaussian_vectors(basis.dim, [77], False)[:, 0]
    res = hp.hphi_lanczos([ham], [_to_dev(x0, torch.float64)], 150)[0]
    assert abs(res["e0_ritz"] - e[0]) < 1e-10
    assert abs(res["e0_refined"] - e[0]) < 1e-10
    gap = e[1] - e[0]
    assert abs(res["e0_refined"] - e[0]) <= res["residual"] ** 2 / gap + 1e-11


def test_lanczos_fp32_storage_refined():
    """FP32 vectors, FP64 recurrence scalars: the FP64 Rayleigh quotient of the rebuilt vector."""
    w = workload("heis_chain12")
    basis = hp.hphi_basis_build(BasisDesc("spin", 12, "sz", two_sz=0))
    ham = hp.hphi_ham_build(basis, w.terms)
    H = oh.sparse_h(basis.desc, w.terms)
    e = np.linalg.eigvalsh(H.toarray())
    x0 = gaussian_vectors(basis.dim, [3], False)[:, 0]
    res = hp.hphi_lanczos([ham], [_to_dev(x0, torch.float32)], 120)[0]
    assert abs(res["e0_ritz"] - e[0]) < 1e-4
    assert abs(res["e0_refined"] - e[0]) / abs(e[0]) < 1e-8


def test_lanczos_multiple_problems():
    w = workload("heis_chain12")
    bases = [hp.hphi_basis_build(BasisDesc("spin", 12, "sz", two_sz=tz)) for tz in (0, 2, 10, 12)]
    hams = [hp.hphi_ham_build(b, w.terms) for b in bases]
    x0 = [_to_dev(gaussian_vectors(b.dim, [5 + k], False)[:, 0], torch.float64) for k, b in enumerate(bases)]
    res = hp.hphi_lanczos(hams, x0, 80)
    for b, r in zip(bases, res):
        H = oh.sparse_h(b.desc, w.terms)
        e0 = np.linalg.eigvalsh(H.toarray())[0]
        assert abs(r["e0_ritz"] - e0) < 1e-9
    assert res[-1]["n_done"] == 1 and res[-1]["info"] == 1
    assert abs(res[-1]["e0_ritz"] - 12 / 4) < 1e-14


# ---------------------------------------------------------------------- TPQ

@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
def test_tpq_trajectory_matches_oracle(dtype, tol):
    ns, l, steps, nvec = 12, 1.5, 40, 4
    desc, terms, basis, ham = _case("kh_honeycomb12")
    H = oh.sparse_h(desc, terms)
    psi0 = gaussian_vectors(basis.dim, [20, 21, 22, 23], True)
    a = _to_dev(psi0, dtype)
    bbuf = torch.empty_like(a)
    us = []
    scale = None
    for k in range(1, steps + 1):
        o = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
        hp.hphi_tpq_step(ham, a, bbuf, l, k, scale, o)
        us.append(o.cpu().numpy().reshape(4, nvec).copy())
        a, bbuf = bbuf, a
        scale = o[3 * nvec:4 * nvec]
    us = np.array(us)
    for bb in range(nvec):
        u_ref, h2_ref, _ = osv.tpq(lambda v: H @ v, psi0[:, bb], ns, l, steps)
        assert np.allclose(us[:, 0, bb], u_ref, rtol=0, atol=tol)
        assert np.allclose(us[:, 1, bb], h2_ref, rtol=0, atol=tol)
        assert np.allclose(us[:, 2, bb], osv.tpq_beta(u_ref, ns, l), rtol=0, atol=100 * tol)


@pytest.mark.parametrize("windowed,window_kb,passes", [(1, 1, 3), (1, 2, 2), (2, 1, 3), (1, 2048, 1)])
@pytest.mark.parametrize("nvec,dtype,lpr", [(1, torch.complex128, 0), (4, torch.complex64, 1), (4, torch.complex64, 4),
                                            (16, torch.complex64, 4), (8, torch.complex128, 2)])
def test_hv_windowed_fermion_signs(monkeypatch, windowed, window_kb, passes, nvec, dtype, lpr):
    """Fermion hopping on the full space of 6 orbitals (12 bits), Jordan-Wigner strings across the
    windows (Sec. 3.3): products through the windowed kernel with one to three passes, plain or
    staged, so that operator groups mix operators with and without sign masks, against the oracle's
    sparse H."""
    print(f"[gpu] windowed fermion signs windowed={windowed} kb={window_kb} passes={passes} nvec={nvec} "
          f"{dtype} lpr={lpr}", flush=True)
    for k, val in (("HPHI_WINDOWED", windowed), ("HPHI_L2_WINDOW_KB", window_kb), ("HPHI_PASSES", passes),
                   ("HPHI_LPR", lpr)):
        monkeypatch.setenv(k, str(val))
    desc = BasisDesc("fermion", 6)
    terms = L.random_fermion_terms(6, 20, 131, conserve_spin=False, real=False, n_dens=3, with_mu=True)
    assert any(t.kind == "hop" for t in terms)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(80, 80 + nvec)), True)
    vd = _to_dev(v, dtype)
    if nvec == 1:
        vd = vd.reshape(-1)
    vin = vd.cpu().numpy().astype(np.complex128).reshape(len(st), nvec)
    u = hp.hphi_hv(ham, vd).cpu().numpy().astype(np.complex128).reshape(len(st), nvec)
    bound, H = _abs_bound(desc, terms, st, vin)
    ref = H @ vin
    tol = 1e-12 if dtype == torch.complex128 else len(terms) * 6e-8
    assert np.all(np.abs(u - ref) <= tol * bound + 1e-300)


@pytest.mark.parametrize("staged", [1, 2])
@pytest.mark.parametrize("window_kb,nvec,passes", [(1, 1, 3), (2, 4, 2), (8, 16, 3), (8, 16, 2)])
def test_hv_windowed_multipass(monkeypatch, window_kb, nvec, passes, staged):
    """Small L2 windows force several passes (operators split by flip bits, bit-permuted row order);
    staged=2 makes every later pass gather from a copy of v written in its own row order."""
    print(f"[gpu] windowed multipass window_kb={window_kb} nvec={nvec} passes={passes} staged={staged}",
          flush=True)
    monkeypatch.setenv("HPHI_L2_WINDOW_KB", str(window_kb))
    monkeypatch.setenv("HPHI_PASSES", str(passes))
    monkeypatch.setenv("HPHI_WINDOWED", str(staged))
    desc = BasisDesc("spin", 12)
    terms = kh_honeycomb_terms(lx=3, ly=2, random_dirs=True, seed=9) + \
        L.random_spin_terms(12, 6, 9, conserve_sz=False, fields=True, real=True)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(60, 60 + nvec)), True)
    for dt, tol in ((torch.complex128, 1e-12), (torch.complex64, 3e-6)):
        vd = _to_dev(v, dt)
        if nvec == 1:
            vd = vd.reshape(-1)
        red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
        u = hp.hphi_hv(ham, vd, a=0.5, b=-0.25, reduce=red).cpu().numpy().astype(np.complex128)
        u = u.reshape(len(st), nvec)
        vin = vd.cpu().numpy().astype(np.complex128).reshape(len(st), nvec)
        H = oh.sparse_h(desc, terms, st)
        hx = H @ vin
        ref = 0.5 * hx - 0.25 * vin
        assert np.linalg.norm(u - ref) <= tol * np.linalg.norm(ref)
        red = red.cpu().numpy().reshape(4, nvec)
        for bb in range(nvec):
            assert abs(red[1, bb] - np.vdot(vin[:, bb], hx[:, bb]).real) <= 10 * tol * np.linalg.norm(hx[:, bb]) * np.linalg.norm(vin[:, bb])


@pytest.mark.parametrize("nvec,dt", [(16, torch.complex64), (1, torch.complex128)])
def test_autotuned_schedule_keeps_parity(nvec, dt):
    desc = BasisDesc("spin", 12)
    terms = kh_honeycomb_terms(lx=3, ly=2, random_dirs=True, seed=5)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(80, 80 + nvec)), True)
    vd = _to_dev(v, dt)
    if nvec == 1:
        vd = vd.reshape(-1)
    sched = hp.hphi_hv_tune(ham, vd)
    assert sched["windowed"] in (0, 1, 2) and sched["max_passes"] >= 1 and sched["us"] >= 0
    u = hp.hphi_hv(ham, vd).cpu().numpy().astype(np.complex128).reshape(len(st), nvec)
    vin = vd.cpu().numpy().astype(np.complex128).reshape(len(st), nvec)
    ref = oh.sparse_h(desc, terms, st) @ vin
    tol = 1e-12 if dt == torch.complex128 else 3e-6
    assert np.linalg.norm(u - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("window_kb", [1, 2048])
def test_hv_reduce_only_with_multipass_schedule(monkeypatch, window_kb):
    """Reduce-only calls (no output vector) must not take the multi-pass path, whatever the schedule."""
    monkeypatch.setenv("HPHI_L2_WINDOW_KB", str(window_kb))
    monkeypatch.setenv("HPHI_PASSES", "3")
    desc = BasisDesc("spin", 12)
    terms = kh_honeycomb_terms(lx=3, ly=2, random_dirs=True, seed=11)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    v = uniform_vectors(len(st), [90], True)[:, 0]
    vd = _to_dev(v, torch.complex128)
    red = torch.empty(4, dtype=torch.float64, device="cuda")
    hp.hphi_hv(ham, vd, a=1.0, b=-0.5, reduce=red, write=False)
    hx = oh.sparse_h(desc, terms, st) @ v
    want = [np.vdot(v, v).real, np.vdot(v, hx).real, np.vdot(hx, hx).real,
            np.linalg.norm(hx - 0.5 * v) ** 2]
    assert np.allclose(red.cpu().numpy(), want, rtol=1e-12, atol=0)
    # the written product (which may run several passes) gives the same sums
    red3 = torch.empty(4, dtype=torch.float64, device="cuda")
    u = hp.hphi_hv(ham, vd, a=1.0, b=-0.5, reduce=red3).cpu().numpy()
    assert np.linalg.norm(u - (hx - 0.5 * v)) <= 1e-12 * np.linalg.norm(hx - 0.5 * v)
    assert np.allclose(red3.cpu().numpy(), want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("lpr", [1, 2, 4, 8])
@pytest.mark.parametrize("case,windowed", [("spin_sz_dm", 0), ("kh_honeycomb12", 0), ("kh_honeycomb12", 1),
                                           ("spin_full_real", 2)])
@pytest.mark.parametrize("nvec", [2, 4, 8, 16])
def test_hv_lanes_per_row(monkeypatch, lpr, case, windowed, nvec):
    """Rows split over 1, 2, 4 or 8 lanes (interleaved 16-byte chunks): output, per-vector scales and
    per-vector reductions all land on the right vector, for every storage type."""
    print(f"[gpu] lanes per row lpr={lpr} case={case} windowed={windowed} nvec={nvec}", flush=True)
    monkeypatch.setenv("HPHI_LPR", str(lpr))
    monkeypatch.setenv("HPHI_WINDOWED", str(windowed))
    if windowed:
        monkeypatch.setenv("HPHI_L2_WINDOW_KB", "4")
        monkeypatch.setenv("HPHI_PASSES", "2")
    desc, terms, basis, ham = _case(case)
    st = ob.states(desc)
    H = oh.sparse_h(desc, terms, st)
    dts = [(torch.complex128, 1e-12), (torch.complex64, 3e-6)]
    if not ham.is_complex:
        dts += [(torch.float64, 1e-12), (torch.float32, 3e-6)]
    for dt, tol in dts:
        cplx = dt in (torch.complex128, torch.complex64)
        v = uniform_vectors(len(st), list(range(200, 200 + nvec)), cplx)
        vd = _to_dev(v if cplx else v.real, dt)
        vin = vd.cpu().numpy().astype(np.complex128)
        scale = np.linspace(0.5, 2.0, nvec)
        red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
        a, b = 0.75, -0.3
        u = hp.hphi_hv(ham, vd, a=a, b=b, in_scale=torch.tensor(scale, device="cuda"), reduce=red)
        u = u.cpu().numpy().astype(np.complex128)
        x = vin * scale[None, :]
        hx = H @ x
        ref = a * hx + b * x
        for k in range(nvec):
            assert np.linalg.norm(u[:, k] - ref[:, k]) <= tol * np.linalg.norm(ref[:, k]), (dt, k)
        red = red.cpu().numpy().reshape(4, nvec)
        for k in range(nvec):
            want = [np.vdot(x[:, k], x[:, k]).real, np.vdot(x[:, k], hx[:, k]).real,
                    np.vdot(hx[:, k], hx[:, k]).real, np.vdot(ref[:, k], ref[:, k]).real]
            scale_k = [abs(want[0]), np.linalg.norm(x[:, k]) * np.linalg.norm(hx[:, k]), abs(want[2]),
                       abs(want[3])]
            for q in range(4):
                assert abs(red[q, k] - want[q]) <= 10 * tol * scale_k[q] + 1e-300, (dt, q, k)


_TILE_PAIRS = [(0, 1), (1, 2), (2, 3), (0, 2), (1, 3), (0, 3),      # flips inside 16 rows
               (3, 4), (4, 5), (2, 4), (3, 5), (0, 5), (1, 4),      # inside a 64-row tile only
               (5, 6), (6, 7), (7, 8), (8, 9), (9, 10), (10, 11), (0, 11), (2, 9)]


@pytest.mark.parametrize("lpr", [1, 2, 4, 8])
@pytest.mark.parametrize("n_sites,windowed,passes", [(12, 1, 1), (12, 1, 2), (12, 2, 2), (7, 1, 1), (7, 2, 2)])
@pytest.mark.parametrize("dt,nvec", [(torch.complex64, 16), (torch.complex128, 8), (torch.complex128, 16),
                                     (torch.float32, 16), (torch.float64, 4)])
def test_hv_windowed_tile_partners(monkeypatch, lpr, n_sites, windowed, passes, dt, nvec):
    """Windowed product with partners in every place a row can find them: within the rows one
    wavefront pass holds (lane exchange), elsewhere in its 64-row tile (LDS tile for rows of at
    most 128 bytes and at most 4 lanes per row) and outside the tile (memory gathers); one window,
    and two passes with and without staged copies; 7 sites is two tiles."""
    print(f"[gpu] windowed tile partners lpr={lpr} n_sites={n_sites} windowed={windowed} passes={passes} "
          f"dt={dt} nvec={nvec}", flush=True)
    monkeypatch.setenv("HPHI_LPR", str(lpr))
    monkeypatch.setenv("HPHI_WINDOWED", str(windowed))
    monkeypatch.setenv("HPHI_PASSES", str(passes))
    monkeypatch.setenv("HPHI_L2_WINDOW_KB", "65536" if passes == 1 else "4")
    desc = BasisDesc("spin", n_sites)
    pairs = [(i, j) for (i, j) in _TILE_PAIRS if i < n_sites and j < n_sites]
    terms = [L.xxz_bond(i, j, 0.6 + 0.05 * k, -0.4 + 0.1 * k) for k, (i, j) in enumerate(pairs)]
    terms += L.random_spin_terms(n_sites, 4, 31, conserve_sz=False, fields=True, real=True)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    H = oh.sparse_h(desc, terms, st)
    cplx = dt in (torch.complex128, torch.complex64)
    tol = 1e-12 if dt in (torch.complex128, torch.float64) else 3e-6
    v = uniform_vectors(len(st), list(range(300, 300 + nvec)), cplx)
    vd = _to_dev(v if cplx else v.real, dt)
    vin = vd.cpu().numpy().astype(np.complex128)
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    a, b = 0.5, 0.25
    u = hp.hphi_hv(ham, vd, a=a, b=b, reduce=red).cpu().numpy().astype(np.complex128)
    hx = H @ vin
    ref = a * hx + b * vin
    for k in range(nvec):
        assert np.linalg.norm(u[:, k] - ref[:, k]) <= tol * np.linalg.norm(ref[:, k]), k
    red = red.cpu().numpy().reshape(4, nvec)
    for k in range(nvec):
        want = np.vdot(vin[:, k], hx[:, k]).real
        assert abs(red[1, k] - want) <= 10 * tol * np.linalg.norm(vin[:, k]) * np.linalg.norm(hx[:, k]), k


@pytest.mark.parametrize("lpr", [4, 8])
@pytest.mark.parametrize("dt,nvec", [(torch.complex64, 16), (torch.complex128, 8)])
def test_hv_windowed_pass_too_large_for_lds_falls_back(monkeypatch, dt, nvec, lpr):
    """990 operators with complex elements in one windowed pass: the pattern table (127 KB).  With
    4 lanes per row the row tiles of 128-byte rows (32 KB) and the kernel's block sums exceed a
    workgroup's LDS, so the product takes the single-pass kernel instead; with 8 lanes per row the
    windowed kernel keeps no row tile and the pass fits (table + block sums = 135 KB).  Both give the
    oracle's result."""
    print(f"[gpu] windowed pass near the LDS limit dt={dt} nvec={nvec} lpr={lpr}", flush=True)
    monkeypatch.setenv("HPHI_WINDOWED", "1")
    monkeypatch.setenv("HPHI_PASSES", "1")
    monkeypatch.setenv("HPHI_L2_WINDOW_KB", "65536")
    monkeypatch.setenv("HPHI_LPR", str(lpr))
    desc = BasisDesc("spin", 12)
    rng = np.random.default_rng(17)
    terms = [L.Term(L.SPIN_FIELD, k % 12, -1, tuple(float(x) for x in rng.uniform(-0.05, 0.05, 3))) for k in range(980)]
    terms += [L.heisenberg_bond(i, (i + 1) % 12, 1.0) for i in range(10)]
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    assert ham.is_complex
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(400, 400 + nvec)), True)
    vd = _to_dev(v, dt)
    u = hp.hphi_hv(ham, vd).cpu().numpy().astype(np.complex128)
    vin = vd.cpu().numpy().astype(np.complex128)
    ref = oh.sparse_h(desc, terms, st) @ vin
    tol = 1e-12 if dt == torch.complex128 else 3e-6
    assert np.linalg.norm(u - ref) <= tol * np.linalg.norm(ref)


# ------------------------------------------------------- batched Lanczos

def _tri12_sectors(dtype, n_iter, use_graph=True, seeds0=500):
    terms = [L.heisenberg_bond(i, j, 1.0) for (i, j) in L.triangular_bonds(4, 3)]
    descs = [BasisDesc("spin", 12, "sz", two_sz=2 * sz) for sz in range(7)]
    bases = [hp.hphi_basis_build(d) for d in descs]
    hams = [hp.hphi_ham_build(b, terms) for b in bases]
    x0 = [gaussian_vectors(b.dim, [seeds0 + k], False)[:, 0] for k, b in enumerate(bases)]
    x0d = [_to_dev(x, dtype) for x in x0]
    res = hp.hphi_lanczos(hams, x0d, n_iter, use_graph=use_graph)
    return terms, descs, [x.cpu().numpy() for x in x0d], res


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batched_lanczos_uneven_sectors_match_oracle(dtype):
    """All seven Sz sectors of a 12-site triangular torus (dims 924 down to 1) in one batched
    recurrence: alpha/beta against the oracle's literal Lanczos, ground energies against dense
    diagonalization, FP64 refinement for FP32 storage."""
    print(f"[gpu] batched lanczos tri12 dtype={dtype}", flush=True)
    terms, descs, x0, res = _tri12_sectors(dtype, 60)
    for d, x, r in zip(descs, x0, res):
        H = oh.sparse_h(d, terms)
        dim = H.shape[0]
        e = np.linalg.eigvalsh(H.toarray())
        a, b = osv.lanczos(lambda v: H @ v, x.astype(np.float64), min(60, dim), dim)
        # FP32 storage does not reach the FP64 breakdown threshold in tiny sectors:
        # compare the steps both recurrences took
        n = min(r["n_done"], len(a), 12)
        tol = 1e-10 if dtype == torch.float64 else 2e-5
        assert np.allclose(r["alpha"][:n], a[:n], rtol=0, atol=tol * max(1.0, np.abs(a[:n]).max())), d
        assert np.allclose(r["beta"][:n], b[:n], rtol=0, atol=tol * max(1.0, np.abs(b[:n]).max())), d
        if dim <= 60:
            assert r["info"] == 1 and r["n_done"] <= dim
        assert abs(r["e0_refined"] - e[0]) <= 1e-8 * max(1.0, abs(e[0])), (d, r["e0_refined"], e[0])
        if dtype == torch.float64:
            assert abs(r["e0_ritz"] - e[0]) <= 1e-10 * max(1.0, abs(e[0]))
    assert res[-1]["n_done"] == 1 and abs(res[-1]["e0_ritz"] - 36 * 0.25) < 1e-12


def test_batched_lanczos_graph_replay_is_bitwise_identical():
    _, _, _, r1 = _tri12_sectors(torch.float64, 40, use_graph=True)
    _, _, _, r2 = _tri12_sectors(torch.float64, 40, use_graph=False)
    for a, b in zip(r1, r2):
        assert np.array_equal(a["alpha"], b["alpha"]) and np.array_equal(a["beta"], b["beta"])
        assert a["e0_refined"] == b["e0_refined"]


def test_batched_lanczos_matches_one_problem_at_a_time():
    """The batched launch and single-problem calls run the same recurrence (same kernels, different
    launch shapes, so different summation orders): equal to rounding over the first steps (later
    steps amplify rounding once the ground state has converged), same refined energy."""
    terms, descs, x0, res = _tri12_sectors(torch.float64, 40)
    for d, x, r in zip(descs[:3], x0[:3], res[:3]):
        b = hp.hphi_basis_build(d)
        h = hp.hphi_ham_build(b, terms)
        r1 = hp.hphi_lanczos([h], [_to_dev(x, torch.float64)], 40)[0]
        assert r1["n_done"] == r["n_done"]
        assert np.allclose(r1["alpha"][:20], r["alpha"][:20], rtol=1e-10, atol=1e-10)
        assert np.allclose(r1["beta"][:20], r["beta"][:20], rtol=1e-10, atol=1e-10)
        # both Rayleigh quotients lie within O(residual^2) of the same eigenvalue
        assert abs(r1["e0_refined"] - r["e0_refined"]) <= 10 * max(r1["residual"], r["residual"]) ** 2 + 1e-11


def test_batched_lanczos_tri24_all_sectors_full_size():
    """The 24-site triangular torus, all 13 Sz sectors (dims 2,704,156 down to 1), FP32 storage, in
    one batched recurrence.  Sectors small enough for the oracle are checked against its sparse
    eigensolver; every sector's refinement must be self-consistent."""
    import scipy.sparse.linalg as sla
    print("[gpu] batched lanczos tri24 all sectors", flush=True)
    w = workload("tri24_allsz")
    descs = [w.basis] + list(w.extra_bases)
    bases = [hp.hphi_basis_build(d) for d in descs]
    hams = [hp.hphi_ham_build(b, w.terms) for b in bases]
    x0 = [device_uniform(b.dim, 1, w.seeds[k], False, torch.float32).reshape(-1).contiguous()
          for k, b in enumerate(bases)]
    res = hp.hphi_lanczos(hams, x0, 120)
    for d, b, r in zip(descs, bases, res):
        assert r["n_done"] == min(120, b.dim)
        assert r["variance"] >= -1e-9 and r["residual"] >= 0
        assert abs(r["e0_refined"] - r["e0_ritz"]) <= 1e-3 * max(1.0, abs(r["e0_ritz"]))
        if b.dim <= 12000:
            H = oh.sparse_h(d, w.terms)
            if b.dim <= 2100:
                e0 = np.linalg.eigvalsh(H.toarray())[0]
            else:
                e0 = sla.eigsh(H, k=1, which="SA", tol=1e-12)[0][0]
            assert abs(r["e0_refined"] - e0) <= 1e-8 * max(1.0, abs(e0)), (d, r["e0_refined"], e0)
    assert abs(res[-1]["e0_ritz"] - 72 * 0.25) < 1e-12


@pytest.mark.parametrize("name", ["spin_sz_dm", "spin_sz_split3", "ferm_nupndn", "ferm_ntot", "hubbard_3x3",
                                  "spin_full_complex"])
@pytest.mark.parametrize("stage", [0, 1])
@pytest.mark.parametrize("nvec", [1, 8])
def test_hv_table_placement(monkeypatch, name, stage, nvec):
    """Pattern and rank tables read from global memory (0) or staged in LDS (1): same FP64 product."""
    print(f"[gpu] table placement {name} stage={stage} nvec={nvec}", flush=True)
    monkeypatch.setenv("HPHI_STAGE_TABLES", str(stage))
    monkeypatch.setenv("HPHI_WINDOWED", "0")
    desc, terms, basis, ham = _case(name)
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(300, 300 + nvec)), True)
    vd = _to_dev(v, torch.complex128)
    if nvec == 1:
        vd = vd.reshape(-1)
    u = hp.hphi_hv(ham, vd).cpu().numpy().reshape(len(st), nvec)
    bound, H = _abs_bound(desc, terms, st, v)
    ref = H @ v
    assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref) + 1e-300
    assert np.all(np.abs(u - ref) <= 1e-12 * bound + 1e-300)


@pytest.mark.parametrize("stage", [0, 1])
def test_batched_lanczos_table_placement(monkeypatch, stage):
    monkeypatch.setenv("HPHI_STAGE_TABLES", str(stage))
    terms, descs, x0, res = _tri12_sectors(torch.float64, 60)
    for d, r in zip(descs, res):
        e0 = np.linalg.eigvalsh(oh.sparse_h(d, terms).toarray())[0]
        assert abs(r["e0_refined"] - e0) <= 1e-9 * max(1.0, abs(e0))


@pytest.mark.parametrize("staged,passes", [(1, 2), (2, 3)])
def test_streaming_hints_do_not_change_results(monkeypatch, staged, passes):
    """Non-temporal hints on the windowed kernel's streaming accesses change cache policy only:
    outputs and reductions are bitwise identical with and without them."""
    desc = BasisDesc("spin", 12)
    terms = kh_honeycomb_terms(lx=3, ly=2, random_dirs=True, seed=13)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(120, 136)), True)
    vd = _to_dev(v, torch.complex64)
    monkeypatch.setenv("HPHI_WINDOWED", str(staged))
    monkeypatch.setenv("HPHI_L2_WINDOW_KB", "16")
    monkeypatch.setenv("HPHI_PASSES", str(passes))
    outs = []
    for nt in (0, 1):
        monkeypatch.setenv("HPHI_NT_STREAMS", str(nt))
        red = torch.empty(64, dtype=torch.float64, device="cuda")
        u = hp.hphi_hv(ham, vd, a=0.5, b=0.25, reduce=red)
        outs.append((u.cpu().numpy(), red.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    ref = oh.sparse_h(desc, terms, st) @ vd.cpu().numpy().astype(np.complex128)
    ref = 0.5 * ref + 0.25 * vd.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(outs[1][0] - ref) <= 3e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("case", ["empty", "diagonal_only", "one_site", "two_site_full"])
@pytest.mark.parametrize("nvec", [1, 16])
def test_degenerate_hamiltonians_and_spaces(case, nvec):
    """No terms (H = 0), a diagonal-only H (Ising + fields along z), a one-site space (two rows, below
    one tile) and a two-site full space: outputs and reductions against the oracle."""
    if case == "empty":
        desc, terms = BasisDesc("spin", 8), []
    elif case == "diagonal_only":
        desc = BasisDesc("spin", 9, "sz", two_sz=1)
        terms = [L.Term(L.SPIN_BOND, i, (i + 1) % 9, (0, 0, 0, 0, 0, 0, 0, 0, 0.7 + 0.1 * i)) for i in range(9)] + \
            [L.Term(L.SPIN_FIELD, i, -1, (0.0, 0.0, 0.3 * i)) for i in range(9)]
    elif case == "one_site":
        desc, terms = BasisDesc("spin", 1), [L.Term(L.SPIN_FIELD, 0, -1, (0.5, 0.0, 0.25))]
    else:
        desc, terms = BasisDesc("spin", 2), [L.heisenberg_bond(0, 1, 1.3)]
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(140, 140 + nvec)), True)
    vd = _to_dev(v, torch.complex128)
    if nvec == 1:
        vd = vd.reshape(-1)
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    u = hp.hphi_hv(ham, vd, a=0.75, b=-0.5, reduce=red).cpu().numpy().reshape(len(st), nvec)
    if terms:
        H = oh.sparse_h(desc, terms, st)
        hx = H @ v
    else:
        hx = np.zeros_like(v)
    ref = 0.75 * hx - 0.5 * v
    assert np.allclose(u, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))
    red = red.cpu().numpy().reshape(4, nvec)
    for b in range(nvec):
        want = [np.vdot(v[:, b], v[:, b]).real, np.vdot(v[:, b], hx[:, b]).real,
                np.vdot(hx[:, b], hx[:, b]).real, np.vdot(ref[:, b], ref[:, b]).real]
        assert np.allclose(red[:, b], want, rtol=1e-12, atol=1e-14)
