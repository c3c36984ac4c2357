"""Dense-block variant of the product (the paper's continuous-memory-access
method, Sec. 4.3) through the C ABI against the oracle.

The variant covers the terms with clusters of M sites and multiplies every
2^M-row block by the cluster's dense partial Hamiltonian on the matrix
cores.  Its result is H v itself, so the oracle is the plain product (sparse
H from the term definitions, or the C oracle's row loop at full size).

Bars: FP64 storage within 1e-12 of the oracle (norm-wise); FP32 storage
within 3e-6 norm-wise, and element-wise within the bound of FP32 sums of
2^M products per cluster plus the rounding of the partial sums carried
between clusters.
"""

import numpy as np
import pytest
import torch

from synth import lattices as L
from synth.configs import BasisDesc, kh_honeycomb_terms, workload
from synth.vectors import device_uniform, uniform_vectors
from oracle import basis as ob
from oracle import c_oracle
from oracle import hamiltonian as oh

pytestmark = pytest.mark.gpu

import paper_1703_03637_amd as hp  # noqa: E402

CASES = {
    "kh_honeycomb12": (BasisDesc("spin", 12), lambda: kh_honeycomb_terms(lx=3, ly=2, random_dirs=True, seed=21)),
    "random_real10": (BasisDesc("spin", 10),
                      lambda: L.random_spin_terms(10, 14, 201, conserve_sz=False, fields=True, real=True)),
    "heisenberg_ring12": (BasisDesc("spin", 12), lambda: [L.heisenberg_bond(i, (i + 1) % 12, 1.0) for i in range(12)]),
}
DTYPES = {"f32": (torch.float32, 3e-6), "f64": (torch.float64, 1e-12),
          "c64": (torch.complex64, 3e-6), "c128": (torch.complex128, 1e-12)}


@pytest.mark.parametrize("m", [4, 6, 7])
@pytest.mark.parametrize("nvec", [1, 16])
@pytest.mark.parametrize("dt", list(DTYPES))
@pytest.mark.parametrize("case", list(CASES))
def test_cma_matches_oracle(case, dt, nvec, m):
    """Output, input scale, a/b and the four per-vector FP64 reductions, against the oracle.
    FP64 storage takes clusters of at most 6 bits: 7 is rejected before any launch."""
    torch_dt, tol = DTYPES[dt]
    print(f"[gpu] cma case={case} dt={dt} nvec={nvec} m={m}", flush=True)
    desc, mk = CASES[case]
    terms = mk()
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    cplx = dt.startswith("c")
    v = uniform_vectors(len(st), list(range(300, 300 + nvec)), cplx)
    vd = torch.from_numpy(v).to(torch_dt).cuda()
    if nvec == 1:
        vd = vd.reshape(-1)
    sx = torch.linspace(0.5, 1.5, nvec, dtype=torch.float64, device="cuda")
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    if m == 7 and torch_dt in (torch.float64, torch.complex128):
        with pytest.raises(hp.HphiError) as e:
            hp.hphi_hv_cma(ham, vd, cluster_bits=m, a=0.75, b=-0.5, in_scale=sx, reduce=red)
        assert e.value.code == -1
        return
    u = hp.hphi_hv_cma(ham, vd, cluster_bits=m, a=0.75, b=-0.5, in_scale=sx, reduce=red)
    u = u.cpu().numpy().astype(np.complex128).reshape(len(st), nvec)
    x = vd.cpu().numpy().astype(np.complex128).reshape(len(st), nvec) * sx.cpu().numpy()[None, :]
    hx = oh.sparse_h(desc, terms, st) @ x
    ref = 0.75 * hx - 0.5 * x
    assert np.linalg.norm(u - ref) <= tol * np.linalg.norm(ref)
    red = red.cpu().numpy().reshape(4, nvec)
    for b in range(nvec):
        nx, nh = np.linalg.norm(x[:, b]), np.linalg.norm(hx[:, b])
        assert abs(red[0, b] - nx ** 2) <= 10 * tol * nx ** 2
        assert abs(red[1, b] - np.vdot(x[:, b], hx[:, b]).real) <= 10 * tol * nx * nh
        assert abs(red[2, b] - nh ** 2) <= 10 * tol * nh ** 2
        assert abs(red[3, b] - np.linalg.norm(ref[:, b]) ** 2) <= 10 * tol * np.linalg.norm(ref[:, b]) ** 2


@pytest.mark.parametrize("nvec", [2, 4, 8])
@pytest.mark.parametrize("dt", ["f32", "c128"])
def test_cma_other_vector_counts(dt, nvec):
    """nvec 2, 4 and 8 (rows narrower than a 16-column tile, and 4- or 8-byte row copies)."""
    torch_dt, tol = DTYPES[dt]
    desc, mk = CASES["random_real10"]
    terms = mk()
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(330, 330 + nvec)), dt.startswith("c"))
    vd = torch.from_numpy(v).to(torch_dt).cuda()
    u = hp.hphi_hv_cma(ham, vd, cluster_bits=5, b=0.25).cpu().numpy().astype(np.complex128)
    x = vd.cpu().numpy().astype(np.complex128)
    ref = oh.sparse_h(desc, terms, st) @ x + 0.25 * x
    assert np.linalg.norm(u - ref) <= tol * np.linalg.norm(ref)


def test_cma_empty_and_diagonal_hamiltonians():
    """No terms (H = 0: one all-zero cluster) and a diagonal-only H (fields along z, Ising bonds)."""
    desc = BasisDesc("spin", 9)
    st = ob.states(desc)
    v = uniform_vectors(len(st), range(340, 344), True)
    vd = torch.from_numpy(v).cuda()
    diag = [L.Term(L.SPIN_BOND, i, (i + 1) % 9, (0, 0, 0, 0, 0, 0, 0, 0, 0.5 + 0.1 * i)) for i in range(9)] + \
        [L.Term(L.SPIN_FIELD, i, -1, (0.0, 0.0, 0.2 * i)) for i in range(9)]
    for terms in ([], diag):
        basis = hp.hphi_basis_build(desc)
        ham = hp.hphi_ham_build(basis, terms)
        red = torch.empty(16, dtype=torch.float64, device="cuda")
        u = hp.hphi_hv_cma(ham, vd, cluster_bits=4, a=2.0, b=-1.0, reduce=red).cpu().numpy()
        hx = oh.sparse_h(desc, terms, st) @ v if terms else np.zeros_like(v)
        ref = 2.0 * hx - v
        assert np.linalg.norm(u - ref) <= 1e-12 * np.linalg.norm(ref)
        assert np.allclose(red.cpu().numpy().reshape(4, 4)[1], [np.vdot(v[:, b], hx[:, b]).real for b in range(4)],
                           rtol=1e-12, atol=1e-12)


def test_cma_plan_covers_every_term():
    """The cluster cover: M distinct sites per cluster, every term inside one cluster, and the
    deterministic greedy gives the same cover on a second build."""
    w = workload("kh_honeycomb24")
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    for m in (4, 5, 6, 7):
        cl = hp.hphi_hv_cma_plan(ham, m)
        assert all(len(set(c)) == m and all(0 <= x < 24 for x in c) for c in cl)
        for t in w.terms:
            assert any(t.i in c and t.j in c for c in cl), (m, t.i, t.j)
        again = hp.hphi_hv_cma_plan(hp.hphi_ham_build(basis, w.terms), m)
        assert again == cl
    assert len(hp.hphi_hv_cma_plan(ham, 6)) == 8


def test_cma_equals_pull_product_in_fp64():
    """Both formulations of H v agree to rounding on the same FP64 input."""
    desc, mk = CASES["kh_honeycomb12"]
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, mk())
    v = torch.from_numpy(uniform_vectors(basis.dim, range(320, 324), True)).cuda()
    a = hp.hphi_hv(ham, v).cpu().numpy()
    b = hp.hphi_hv_cma(ham, v, cluster_bits=6).cpu().numpy()
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


def test_cma_rejects_what_it_does_not_cover():
    desc, mk = CASES["kh_honeycomb12"]
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, mk())
    v = torch.ones(basis.dim, 4, dtype=torch.complex128, device="cuda")
    for m in (3, 8):
        with pytest.raises(hp.HphiError):
            hp.hphi_hv_cma(ham, v, cluster_bits=m)
    with pytest.raises(hp.HphiError):
        hp.hphi_hv_cma(ham, v, cluster_bits=7)                  # FP64 storage: at most 6
    with pytest.raises(hp.HphiError):
        hp.hphi_hv_cma(ham, v.to(torch.complex64), cluster_bits=13)
    # complex matrix elements (a transverse y field)
    cham = hp.hphi_ham_build(basis, mk() + [L.Term(L.SPIN_FIELD, 0, -1, (0.0, 0.3, 0.0))])
    with pytest.raises(hp.HphiError) as e:
        hp.hphi_hv_cma(cham, v, cluster_bits=6)
    assert e.value.code == -5
    # Sz sector and fermion bases are outside the variant
    sz = BasisDesc("spin", 12, "sz", two_sz=0)
    sbasis = hp.hphi_basis_build(sz)
    sham = hp.hphi_ham_build(sbasis, [L.heisenberg_bond(i, (i + 1) % 12) for i in range(12)])
    with pytest.raises(hp.HphiError):
        hp.hphi_hv_cma(sham, torch.ones(sbasis.dim, dtype=torch.float64, device="cuda"), cluster_bits=6)
    fb = hp.hphi_basis_build(BasisDesc("fermion", 4))
    fham = hp.hphi_ham_build(fb, L.hubbard_terms(L.chain_bonds(4), 4, t=1.0, U=4.0))
    with pytest.raises(hp.HphiError):
        hp.hphi_hv_cma(fham, torch.ones(fb.dim, dtype=torch.float64, device="cuda"), cluster_bits=6)


def _row_abs_sum_bound(terms):
    """Upper bound on max_s sum_t |<s|H|t>|: each term's own maximum absolute row sum, from its
    dense matrix on the sites it touches (oracle)."""
    total = 0.0
    for t in terms:
        sites = sorted({t.i, t.j} - {-1})
        relabel = {site: k for k, site in enumerate(sites)}
        t2 = t._replace(i=relabel[t.i], j=relabel.get(t.j, -1))
        hd = oh.dense_h(BasisDesc("spin", len(sites)), [t2])
        total += float(np.abs(hd).sum(axis=1).max())
    return total


@pytest.mark.parametrize("m", [6])
def test_cma_kh_honeycomb24_sampled_rows_match_c_oracle(m):
    """The headline workload at full size (2^24 rows, 16 complex64 vectors) on 2^18 + 4096 sampled
    rows: element-wise within the FP32 bound of the dense blocks and the carried partial sums."""
    print(f"[gpu] cma kh_honeycomb24 m={m}", flush=True)
    w = workload("kh_honeycomb24")
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, w.terms)
    dim, nvec = basis.dim, w.nvec
    psi = device_uniform(dim, nvec, 913, True, torch.complex64)
    u = hp.hphi_hv_cma(ham, psi, cluster_bits=m).cpu().numpy()
    v = psi.cpu().numpy()
    del psi
    torch.cuda.empty_cache()
    rng = np.random.default_rng(914)
    rows = np.unique(np.concatenate([np.arange(4096), rng.integers(0, dim, 1 << 18)])).astype(np.uint64)
    hx = c_oracle.rows_hv(w.terms, rows, v)
    R = _row_abs_sum_bound(w.terms)
    n_clusters = len(w.terms)                      # at most one cluster per term
    carry = n_clusters * ((1 << m) + 2) * 2.0 ** -24 * R * np.abs(v).max()
    for b in range(nvec):
        ref = hx[:, b]
        d = np.abs(u[rows.astype(np.int64), b].astype(np.complex128) - ref)
        bound = 2.0 ** -24 * np.abs(ref) + carry + 1e-12
        assert np.all(d <= bound), (b, float((d / bound).max()))
    print(f"[gpu] max |d| = {float(d.max()):.3e}, bound floor {carry:.3e}", flush=True)
