"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values
printed in the paper (tests/golden/paper_examples.json), closed forms,
a Kronecker-product construction of the same operators, Bethe-ansatz
equations, and brute force on tiny inputs.
"""

import json
import os
import math
from math import comb

import numpy as np
import pytest

from synth import lattices as L
from synth.configs import BasisDesc, workload
from synth.vectors import gaussian_vectors, uniform_vectors
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import solvers as osv

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


# ----------------------------------------------------------------- paper examples

def test_four_ary_label():
    """Sec. 3.1: |0, up, down, updown> = [0123]_4 = 27 with up in the low bit of each site."""
    g = GOLD["four_ary_example"]
    # site 3 (leftmost) empty, site 2 up, site 1 down, site 0 doubly occupied
    occ = [(0, 0), (0, 1), (1, 1), (2, 0)]   # (site, sigma)
    st = np.array([0], dtype=np.uint64)
    for site, sigma in occ:
        c, st = oh.create(2 * site + sigma, st)
        assert abs(c[0]) == 1.0
    assert int(st[0]) == g["value"] == int(g["bits"], 2)
    digits = [(int(st[0]) >> (2 * s)) & 3 for s in range(4)]
    assert digits[::-1] == [0, 1, 2, 3]


def test_sz0_basis_n4():
    """Sec. 3.3: the Sz = 0 block of 4 sites is spanned by 3, 5, 6, 9, 10, 12 in this order."""
    g = GOLD["sz0_basis_n4"]
    st = ob.states(BasisDesc("spin", 4, "sz", two_sz=0))
    assert st.tolist() == g["states"]
    assert ob.rank(st, np.array(g["states"], np.uint64)).tolist() == list(range(6))


def test_xor_exchange_example():
    """Sec. 3.3: (S+_0 S-_1 + S-_0 S+_1)|1010> = |1001>, and |0011> -> 0."""
    g = GOLD["xor_exchange"]
    term = L.Term(L.SPIN_BOND, 0, 1, (2.0, 0, 0, 0, 2.0, 0, 0, 0, 0.0))  # 2(SxSx+SySy) = S+S- + S-S+
    for st, expect in ((g["state"], g["target"]), (g["forbidden_state"], None)):
        br = oh.term_branches(term, np.array([st], np.uint64), "spin")
        acc = {}
        for c, t in br:
            if c[0] != 0:
                acc[int(t[0])] = acc.get(int(t[0]), 0) + c[0]
        acc = {k: v for k, v in acc.items() if v != 0}
        if expect is None:
            assert acc == {}
        else:
            assert acc == {expect: 1.0}
            assert st ^ g["mask"] == expect


def test_paper_dimensions():
    g = GOLD["dimensions"]
    assert ob.dimension(BasisDesc("fermion", 18, "nupndn", n_up=9, n_dn=9)) == g["hubbard18_half_filling_sz0"]
    assert ob.dimension(BasisDesc("fermion", 13, "nupndn", n_up=6, n_dn=6)) == g["c13_6_squared"]
    assert ob.dimension(BasisDesc("fermion", 13, "nupndn", n_up=9, n_dn=9)) == g["c13_9_squared"]
    assert ob.dimension(BasisDesc("spin", 40)) == g["two_pow_40"]
    assert round(g["two_pow_40"] * 16 / 1e12, 1) == g["two_pow_40_complex128_TB"]


def test_workload_dimensions():
    assert ob.dimension(workload("hubbard_4x3").basis) == 853776
    assert ob.dimension(workload("kagome36_sz0").basis) == 9075135300
    w = workload("tri24_allsz")
    dims = [ob.dimension(b) for b in [w.basis] + w.extra_bases]
    assert dims[0] == 2704156 and dims[-1] == 1 and sum(dims) == 9740686


@pytest.mark.parametrize("desc", [
    BasisDesc("spin", 10, "sz", two_sz=2),
    BasisDesc("fermion", 5, "nupndn", n_up=2, n_dn=3),
    BasisDesc("fermion", 5, "ntot", n_tot=4),
])
def test_enumeration_matches_binomials(desc):
    st = ob.states(desc)
    assert len(st) == ob.dimension(desc)
    assert np.all(np.diff(st.astype(np.int64)) > 0)


def test_cns_rank_matches_enumeration():
    st = ob.states(BasisDesc("spin", 14, "sz", two_sz=2))   # popcount 8
    for r in [0, 1, 17, 500, len(st) - 1]:
        assert ob.cns_rank(int(st[r])) == r
        assert ob.cns_unrank(r, 8, 14) == int(st[r])
    # first and last of a 36-bit popcount-18 space
    assert ob.cns_rank((1 << 18) - 1) == 0
    assert ob.cns_rank(((1 << 18) - 1) << 18) == comb(36, 18) - 1


# ------------------------------------------------- Kronecker-product construction

def _kron_spin_h(n, terms):
    """H from 2x2 matrices and np.kron; site i is factor n-1-i (most significant left)."""
    sz = np.diag([-0.5, 0.5]).astype(complex)
    sp_ = np.array([[0, 0], [1, 0]], complex)     # <up|S+|down> = 1 (index 1 = up)
    sm = sp_.T.copy()
    sx = (sp_ + sm) / 2
    sy = (sp_ - sm) / 2j
    S = [sx, sy, sz]

    def site_op(op, i):
        m = np.array([[1.0]], complex)
        for k in range(n - 1, -1, -1):
            m = np.kron(m, op if k == i else np.eye(2))
        return m

    H = np.zeros((2 ** n, 2 ** n), complex)
    for t in terms:
        if t.kind == L.SPIN_BOND:
            for a in range(3):
                for b in range(3):
                    if t.c[3 * a + b]:
                        H += t.c[3 * a + b] * site_op(S[a], t.i) @ site_op(S[b], t.j)
        elif t.kind == L.SPIN_FIELD:
            for a in range(3):
                if t.c[a]:
                    H += t.c[a] * site_op(S[a], t.i)
    return H


def _kron_fermion_h(n_sites, terms):
    """H from Jordan-Wigner matrices: c_k = I..I (x) a (x) Z..Z with Z on orbitals below k."""
    no = 2 * n_sites
    a = np.array([[0, 1], [0, 0]], complex)        # a|1> = |0>
    Z = np.diag([1.0, -1.0]).astype(complex)

    def c(k):
        m = np.array([[1.0]], complex)
        for q in range(no - 1, -1, -1):
            m = np.kron(m, a if q == k else (Z if q < k else np.eye(2)))
        return m

    cs = [c(k) for k in range(no)]
    cd = [m.conj().T for m in cs]
    n_op = [cd[k] @ cs[k] for k in range(no)]
    H = np.zeros((2 ** no, 2 ** no), complex)
    for t in terms:
        if t.kind == L.HOP:
            tt = complex(t.c[0], t.c[1])
            H += tt * cd[t.i] @ cs[t.j] + np.conj(tt) * cd[t.j] @ cs[t.i]
        elif t.kind == L.DENS:
            H += t.c[0] * n_op[t.i] @ n_op[t.j]
        elif t.kind == L.NUM:
            H += t.c[0] * n_op[t.i]
        elif t.kind == L.HUBBARD_U:
            H += t.c[0] * n_op[2 * t.i] @ n_op[2 * t.i + 1]
        elif t.kind == L.GREEN2:
            tt = complex(t.c[0], t.c[1])
            T = cd[t.i] @ cs[t.j] @ cd[int(t.c[2])] @ cs[int(t.c[3])]
            H += tt * T + np.conj(tt) * T.conj().T
    return H


@pytest.mark.parametrize("seed,real,fields", [(1, True, False), (2, False, True), (3, True, True)])
def test_spin_h_matches_kron(seed, real, fields):
    n = 6
    terms = L.random_spin_terms(n, 9, seed, conserve_sz=False, fields=fields, real=real)
    H = oh.dense_h(BasisDesc("spin", n), terms)
    assert np.allclose(H, _kron_spin_h(n, terms), atol=1e-14, rtol=0)
    assert np.allclose(H, H.conj().T, atol=1e-15)


@pytest.mark.parametrize("seed,real", [(4, True), (5, False)])
def test_fermion_h_matches_jordan_wigner(seed, real):
    ns = 3
    terms = L.random_fermion_terms(ns, 8, seed, conserve_spin=False, real=real, n_dens=3,
                                   with_u=True, with_mu=True)
    H = oh.dense_h(BasisDesc("fermion", ns), terms)
    assert np.allclose(H, _kron_fermion_h(ns, terms), atol=1e-14, rtol=0)


def test_apply_h_matches_dense():
    desc = BasisDesc("fermion", 4, "nupndn", n_up=2, n_dn=1)
    terms = L.random_fermion_terms(4, 10, 7, conserve_spin=True, real=False, n_dens=2)
    H = oh.dense_h(desc, terms)
    v = uniform_vectors(H.shape[0], [1, 2, 3], True)
    assert np.allclose(oh.apply_h(desc, terms, v), H @ v, atol=1e-13)


def test_rows_sampled_matches_push():
    desc = BasisDesc("spin", 8, "sz", two_sz=0)
    terms = L.random_spin_terms(8, 12, 8, conserve_sz=True, real=False, fields=True)
    st = ob.states(desc)
    v = uniform_vectors(len(st), [5, 6], True)
    u = oh.apply_h(desc, terms, v)
    rows = np.array([0, 3, 17, len(st) - 1])
    us = oh.rows_hv_sampled(desc, terms, st[rows], lambda t: v[ob.rank(st, t)])
    assert np.allclose(us, u[rows], atol=1e-13)


# ------------------------------------------------------------------ closed forms

def test_ring4_ground_state():
    """4-site Heisenberg ring (Sec. 3.3 example Hamiltonian): E0 = -2J."""
    w = workload("heis_ring4")
    e = np.linalg.eigvalsh(oh.dense_h(w.basis, w.terms))
    assert abs(e[0] - (-2.0)) < 1e-13


def test_two_site_hubbard():
    """E0 = (U - sqrt(U^2 + 16 t^2))/2 for one up and one down electron."""
    for U in (0.0, 2.0, 8.0):
        terms = L.hubbard_terms([(0, 1)], 2, t=1.0, U=U)
        e = np.linalg.eigvalsh(oh.dense_h(BasisDesc("fermion", 2, "nupndn", n_up=1, n_dn=1), terms))
        assert abs(e[0] - (U - np.sqrt(U * U + 16)) / 2) < 1e-13


def _open_rect_levels(lx, ly, t=1.0):
    return np.sort([-2 * t * np.cos(np.pi * m / (lx + 1)) - 2 * t * np.cos(np.pi * n / (ly + 1))
                    for m in range(1, lx + 1) for n in range(1, ly + 1)])


@pytest.mark.parametrize("lx,ly,nup,ndn", [(3, 2, 2, 3), (3, 3, 3, 3)])
def test_free_fermions_open_rect(lx, ly, nup, ndn):
    """U = 0: E0 = sum of the lowest single-particle levels; sign-sensitive (hops jump over orbitals)."""
    n = lx * ly
    terms = L.hubbard_terms(L.rect_bonds(lx, ly), n, t=1.0, U=0.0)
    desc = BasisDesc("fermion", n, "nupndn", n_up=nup, n_dn=ndn)
    H = oh.sparse_h(desc, terms)
    x0 = gaussian_vectors(H.shape[0], [3], True)[:, 0]
    e0 = osv.lanczos_ground_state(lambda v: H @ v, x0, 120, H.shape[0], refine=False)["e0_ritz"]
    lev = _open_rect_levels(lx, ly)
    assert abs(e0 - (lev[:nup].sum() + lev[:ndn].sum())) < 1e-10


@pytest.mark.slow
def test_free_fermions_hubbard_4x3():
    """U = 0 limit of the 4x3 open cluster, 6 up + 6 down: E0 = 2 * (sum of 6 lowest levels)."""
    terms = L.hubbard_terms(L.rect_bonds(4, 3), 12, t=1.0, U=0.0)
    desc = BasisDesc("fermion", 12, "nupndn", n_up=6, n_dn=6)
    H = oh.sparse_h(desc, terms)
    x0 = gaussian_vectors(H.shape[0], [2], True)[:, 0]
    res = osv.lanczos_ground_state(lambda v: H @ v, x0, 150, H.shape[0], refine=False)
    lev = _open_rect_levels(4, 3)
    assert abs(res["e0_ritz"] - 2 * lev[:6].sum()) < 1e-9
    assert abs(2 * lev[:6].sum() - (-16.601126159491542)) < 1e-12


def test_one_electron_sector():
    """n_up = 1, n_dn = 0: spectrum = eigenvalues of the hopping matrix."""
    n = 5
    terms = L.random_fermion_terms(n, 8, 11, conserve_spin=True, real=False, with_u=True)
    desc = BasisDesc("fermion", n, "nupndn", n_up=1, n_dn=0)
    e = np.linalg.eigvalsh(oh.dense_h(desc, terms))
    T = np.zeros((n, n), complex)
    for t in terms:
        if t.kind == L.HOP and t.i % 2 == 0 and t.j % 2 == 0:
            tt = complex(*t.c)
            T[t.i // 2, t.j // 2] += tt
            T[t.j // 2, t.i // 2] += np.conj(tt)
    assert np.allclose(e, np.linalg.eigvalsh(T), atol=1e-13)


def test_one_magnon_sector():
    """Ferromagnet plus one flipped spin: diag(E_F - sum_j J_ij/2) + (J_ij/2) adjacency."""
    n = 8
    bonds = L.chain_bonds(n) + [(0, 4), (2, 6)]
    rng = np.random.default_rng(3)
    Js = rng.uniform(0.2, 1.5, len(bonds))
    terms = [L.heisenberg_bond(i, j, J) for (i, j), J in zip(bonds, Js)]
    desc = BasisDesc("spin", n, "sz", two_sz=-(n - 2))
    e = np.linalg.eigvalsh(oh.dense_h(desc, terms))
    EF = Js.sum() / 4
    M = np.diag(np.full(n, EF))
    for (i, j), J in zip(bonds, Js):
        M[i, i] -= J / 2
        M[j, j] -= J / 2
        M[i, j] += J / 2
        M[j, i] += J / 2
    assert np.allclose(e, np.linalg.eigvalsh(M), atol=1e-13)


def test_fully_polarized_triangular():
    """Sz = 12 sector of the 24-site triangular torus: one state, E = 72/4 = 18 exactly."""
    w = workload("tri24_allsz")
    desc = w.extra_bases[-1]
    st = np.array([(1 << 24) - 1], np.uint64)
    hv = oh.rows_hv_sampled(desc, w.terms, st, lambda t: np.where(t == st[0], 1.0, np.nan))
    assert hv[0] == 18.0


def test_traces_heisenberg_chain16():
    """Tr H = 0 and Tr H^2 / dim = (3/16) sum_b J_b^2 = 3 for the 16-site chain."""
    w = workload("heis_chain16")
    H = oh.sparse_h(w.basis, w.terms)
    assert abs(H.diagonal().sum()) < 1e-12
    tr2 = (abs(H.data) ** 2).sum() / H.shape[0]   # Tr H^2 = sum |H_ij|^2 (Hermitian)
    assert abs(tr2 - 3.0) < 1e-13


def test_trace_h2_general_bonds():
    """Tr H^2/dim = sum_b sum_ab (J^ab)^2 / 16 + sum_fields |h|^2/4 for distinct site pairs."""
    n = 7
    pairs = [(0, 1), (1, 2), (2, 5), (3, 6), (4, 0), (6, 2)]
    rng = np.random.default_rng(9)
    terms = [L.Term(L.SPIN_BOND, i, j, tuple(rng.uniform(-1, 1, 9))) for i, j in pairs]
    terms += [L.Term(L.SPIN_FIELD, i, -1, tuple(rng.uniform(-1, 1, 3))) for i in range(n)]
    H = oh.dense_h(BasisDesc("spin", n), terms)
    expect = sum((np.array(t.c) ** 2).sum() / (16 if t.kind == L.SPIN_BOND else 4) for t in terms)
    assert abs(np.trace(H @ H).real / H.shape[0] - expect) < 1e-12


def _bethe_ground_energy(N, J=1.0):
    """Antiferromagnetic periodic chain ground state from the Bethe equations (M = N/2).

    N arctan(2 l_j) = pi I_j + sum_k arctan(l_j - l_k), I_j = -(M-1)/2..(M-1)/2;
    E = N J/4 - J sum_j (1/2)/(l_j^2 + 1/4).
    """
    M = N // 2
    I = np.arange(M) - (M - 1) / 2
    lam = np.tan(np.pi * I / N) / 2
    for _ in range(2000):
        s = np.arctan(lam[:, None] - lam[None, :]).sum(axis=1)
        new = np.tan((np.pi * I + s) / N) / 2
        if np.max(abs(new - lam)) < 1e-15:
            lam = new
            break
        lam = 0.5 * lam + 0.5 * new
    return N * J / 4 - J * np.sum(0.5 / (lam ** 2 + 0.25))


def test_bethe_ansatz_chain16():
    """N = 16 periodic Heisenberg chain: oracle Lanczos E0 equals the Bethe-ansatz energy."""
    eb = _bethe_ground_energy(16)
    assert abs(eb - (-7.142296360616757)) < 1e-11
    assert abs(_bethe_ground_energy(4) - (-2.0)) < 1e-12
    w = workload("heis_chain16")
    H = oh.sparse_h(w.basis, w.terms)
    x0 = gaussian_vectors(H.shape[0], w.seeds, True)[:, 0]
    res = osv.lanczos_ground_state(lambda v: H @ v, x0, 200, H.shape[0])
    assert abs(res["e0_ritz"] - eb) < 1e-10
    assert abs(res["e0_refined"] - eb) < 1e-10
    assert res["residual"] < 1e-5


def test_sz_conservation_union_of_sectors():
    """[H, Sz] = 0: the full spectrum is the union of the sector spectra (N = 8)."""
    n = 8
    terms = L.random_spin_terms(n, 12, 21, conserve_sz=True, real=False, fields=True)
    full = np.linalg.eigvalsh(oh.dense_h(BasisDesc("spin", n), terms))
    parts = [np.linalg.eigvalsh(oh.dense_h(BasisDesc("spin", n, "sz", two_sz=tz), terms))
             for tz in range(-n, n + 1, 2)]
    assert np.allclose(np.sort(np.concatenate(parts)), full, atol=1e-12)


def test_nupndn_union_of_sectors():
    ns = 3
    terms = L.random_fermion_terms(ns, 6, 22, conserve_spin=True, real=False, n_dens=2, with_mu=True)
    full = np.linalg.eigvalsh(oh.dense_h(BasisDesc("fermion", ns), terms))
    parts = [np.linalg.eigvalsh(oh.dense_h(BasisDesc("fermion", ns, "nupndn", n_up=a, n_dn=b), terms))
             for a in range(ns + 1) for b in range(ns + 1)]
    assert np.allclose(np.sort(np.concatenate(parts)), full, atol=1e-12)


def test_sector_breaking_detected():
    desc = BasisDesc("spin", 6, "sz", two_sz=0)
    kitaev = workload("kh_honeycomb12").terms
    with pytest.raises(ValueError):
        oh.coo_elements(BasisDesc("spin", 12, "sz", two_sz=0), kitaev)
    assert oh.sector_preserving(desc, [L.heisenberg_bond(0, 1)])


# ------------------------------------------------------------------ solver pins

def test_lanczos_matches_dense_minimum():
    desc = BasisDesc("spin", 10)
    terms = L.random_spin_terms(10, 18, 31, conserve_sz=False, real=False, fields=True)
    H = oh.sparse_h(desc, terms)
    e = np.linalg.eigvalsh(H.toarray())
    x0 = gaussian_vectors(H.shape[0], [7], True)[:, 0]
    res = osv.lanczos_ground_state(lambda v: H @ v, x0, 150, H.shape[0])
    assert abs(res["e0_ritz"] - e[0]) < 1e-9
    assert abs(res["e0_refined"] - e[0]) < 1e-9
    # refinement bound |E_RQ - E0| <= |r|^2 / gap
    gap = e[1] - e[0]
    assert abs(res["e0_refined"] - e[0]) <= res["residual"] ** 2 / gap + 1e-12


def test_lanczos_shift_invariance():
    """Sec. 3.4: K(H) = K(H + aI): alpha shifts by a, beta is unchanged."""
    desc = BasisDesc("spin", 8)
    terms = L.random_spin_terms(8, 10, 32, conserve_sz=False)
    H = oh.sparse_h(desc, terms)
    x0 = gaussian_vectors(H.shape[0], [8], True)[:, 0]
    a1, b1 = osv.lanczos(lambda v: H @ v, x0, 30, H.shape[0])
    a2, b2 = osv.lanczos(lambda v: H @ v + 3.25 * v, x0, 30, H.shape[0])
    assert np.allclose(a2, a1 + 3.25, atol=1e-12)
    assert np.allclose(b2, b1, atol=1e-11)


def test_lanczos_breakdown_small_space():
    """dim-1 and tiny sectors: the recurrence stops at the dimension."""
    w = workload("tri24_allsz")
    desc = BasisDesc("spin", 6, "sz", two_sz=4)     # dim 6
    terms = [L.heisenberg_bond(i, j) for (i, j) in L.chain_bonds(6)]
    H = oh.sparse_h(desc, terms)
    x0 = gaussian_vectors(6, [1], False)[:, 0]
    a, b = osv.lanczos(lambda v: H @ v, x0, 50, 6)
    assert len(a) <= 6
    e0, _ = osv.tridiag_lowest(a, b)
    assert abs(e0 - np.linalg.eigvalsh(H.toarray())[0]) < 1e-12
    assert w.extra_bases[-1].two_sz == 24


def test_tpq_matches_spectral_closed_form():
    """Sec. 3.5: literal mTPQ trajectory equals sum_n (l - E_n/N)^k <n|psi0>|n> evaluated spectrally."""
    from synth.configs import kh_honeycomb_terms
    ns = 8
    terms = kh_honeycomb_terms(lx=2, ly=2, random_dirs=False)
    H = oh.dense_h(BasisDesc("spin", ns), terms)
    evals, evecs = np.linalg.eigh(H)
    psi0 = gaussian_vectors(H.shape[0], [20], True)[:, 0]
    psi0 = psi0 / np.linalg.norm(psi0)
    u, h2, _ = osv.tpq(lambda v: H @ v, psi0, ns, 1.5, 60)
    us, h2s = osv.tpq_spectral(evals, evecs, psi0, ns, 1.5, 60)
    assert np.allclose(u, us, atol=1e-13, rtol=0)
    assert np.allclose(h2, h2s, atol=1e-13, rtol=0)
    # k = 0 is the infinite-temperature estimate Tr H/(dim N_s) up to sampling noise
    assert abs(u[0] - np.trace(H).real / H.shape[0] / ns) < 5 / np.sqrt(H.shape[0])
    beta = osv.tpq_beta(u, ns, 1.5)
    assert beta[0] == 0 and np.all(np.diff(beta) > 0)


def test_row_elements_sampled_matches_push():
    """Row-wise elements from applying terms to |s> equal the column-wise push (Hermiticity)."""
    desc = BasisDesc("fermion", 4, "nupndn", n_up=2, n_dn=2)
    terms = L.random_fermion_terms(4, 9, 41, conserve_spin=True, real=False, n_dens=2, with_mu=True)
    st = ob.states(desc)
    rows = np.array([0, 5, 17, len(st) - 1])
    push = oh.row_elements(desc, terms, rows, st)
    pull = oh.row_elements_sampled(desc, terms, st[rows], lambda t: ob.rank(st, t))
    for k, r in enumerate(rows):
        assert push[int(r)].keys() == pull[k].keys()
        for key in push[int(r)]:
            assert abs(push[int(r)][key] - pull[k][key]) < 1e-15


# ------------------------------------------------------------ C row oracle

@pytest.mark.parametrize("seed,real", [(51, False), (52, True)])
def test_c_oracle_spin_matches_kron(seed, real):
    """C oracle rows against the Kronecker-product matrix (independent construction)."""
    from oracle import c_oracle
    n = 7
    terms = L.random_spin_terms(n, 11, seed, conserve_sz=False, fields=True, real=real)
    Hk = _kron_spin_h(n, terms)
    v = uniform_vectors(2 ** n, [1, 2, 3], True)
    rows = np.arange(2 ** n, dtype=np.uint64)
    u = c_oracle.rows_hv(terms, rows, v)
    assert np.allclose(u, Hk @ v, atol=1e-13, rtol=0)


def test_c_oracle_fermion_matches_jordan_wigner():
    from oracle import c_oracle
    ns = 3
    terms = L.random_fermion_terms(ns, 9, 53, conserve_spin=False, real=False, n_dens=3, with_mu=True)
    Hk = _kron_fermion_h(ns, terms)
    v = uniform_vectors(4 ** ns, [4, 5], True)
    u = c_oracle.rows_hv(terms, np.arange(4 ** ns, dtype=np.uint64), v)
    assert np.allclose(u, Hk @ v, atol=1e-13, rtol=0)


def test_c_oracle_sector_rows_match_python_oracle():
    from oracle import c_oracle
    desc = BasisDesc("fermion", 5, "nupndn", n_up=2, n_dn=2)
    terms = L.random_fermion_terms(5, 12, 54, conserve_spin=True, real=False, n_dens=2)
    st = ob.states(desc)
    v = uniform_vectors(len(st), [6], True)[:, 0]
    u = c_oracle.rows_hv(terms, st, v, states=st)
    assert np.allclose(u, oh.apply_h(desc, terms, v, st), atol=1e-13, rtol=0)


@pytest.mark.parametrize("desc", [BasisDesc("fermion", 5, "nupndn", n_up=2, n_dn=3),
                                  BasisDesc("fermion", 6, "nupndn", n_up=3, n_dn=3),
                                  BasisDesc("fermion", 6, "nupndn", n_up=1, n_dn=4),
                                  BasisDesc("fermion", 4, "ntot", n_tot=3),
                                  BasisDesc("spin", 10, "sz", two_sz=2),
                                  BasisDesc("spin", 7)])
def test_sector_rank_by_counting_matches_enumeration(desc):
    """Counting rank/unrank (no basis list) against the sorted brute-force enumeration."""
    st = ob.states(desc)
    assert [ob.sector_rank(desc, int(s)) for s in st] == list(range(len(st)))
    assert [ob.sector_unrank(desc, i) for i in range(len(st))] == [int(s) for s in st]


def test_sector_rank_agrees_with_cns_on_sz_sectors():
    d = BasisDesc("spin", 36, "sz", two_sz=0)
    rng = np.random.default_rng(1)
    for r in rng.integers(0, ob.dimension(d), 50):
        s = ob.cns_unrank(int(r), 18, 36)
        assert ob.sector_rank(d, s) == int(r) == ob.cns_rank(s)
        assert ob.sector_unrank(d, int(r)) == s


def test_sector_rank_endpoints_18_site_hubbard():
    """Half filling on 18 sites: the smallest and largest configurations take the first and last index."""
    d = BasisDesc("fermion", 18, "nupndn", n_up=9, n_dn=9)
    lo = sum(1 << (2 * i) for i in range(9)) | sum(1 << (2 * i + 1) for i in range(9))
    hi = sum(1 << (2 * i) for i in range(9, 18)) | sum(1 << (2 * i + 1) for i in range(9, 18))
    assert ob.sector_rank(d, lo) == 0 and ob.sector_rank(d, hi) == ob.dimension(d) - 1 == 2363904400 - 1
    assert ob.sector_unrank(d, 0) == lo and ob.sector_unrank(d, ob.dimension(d) - 1) == hi


@pytest.mark.parametrize("desc,terms", [
    (BasisDesc("fermion", 6, "nupndn", n_up=3, n_dn=2), L.hubbard_terms(L.rect_bonds(3, 2), 6, t=1.0, U=4.0)),
    (BasisDesc("spin", 10, "sz", two_sz=-2), L.random_spin_terms(10, 12, 31, conserve_sz=True, real=False)),
    (BasisDesc("fermion", 4, "ntot", n_tot=3), L.random_fermion_terms(4, 8, 32, conserve_spin=False, real=True)),
])
def test_c_oracle_counted_rank_matches_list_rank(desc, terms):
    """The C oracle's counting rank (no basis list) gives the same rows as its list-rank path, and its
    unrank inverts the enumeration."""
    from oracle import c_oracle
    st = ob.states(desc)
    v = uniform_vectors(len(st), [33, 34], True)
    a = c_oracle.rows_hv(terms, st, v, states=st)
    b = c_oracle.rows_hv_counted(desc, terms, st, v)
    assert np.array_equal(a, b)
    assert np.array_equal(c_oracle.unrank_counted(desc, np.arange(len(st))), st)
    ref = oh.sparse_h(desc, terms) @ v
    assert np.allclose(b, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


# ------------------------------------------------- TPQ temperature, variance, c64 rows

def _field_terms(n, h):
    return [L.Term(L.SPIN_FIELD, i, i, (0.0, 0.0, h)) for i in range(n)]


def _free_spin_energy(beta, h):
    """Canonical energy per site of free spins 1/2 in a field, H = h sum S^z: -(h/2) tanh(beta h/2)."""
    return -(h / 2.0) * np.tanh(beta * h / 2.0)


def test_tpq_beta_free_spins_match_canonical_ensemble():
    """Sec. 3.5: the mTPQ temperature beta_k = (2k/N_s)/(l - u_k).  For free spins in a field the
    canonical energy per site is -(h/2) tanh(beta h/2) in closed form; the literal TPQ energy u_k at
    the oracle's beta_k must match it up to the finite-size and sampling error, while a beta off by a
    factor of two misses by far more."""
    ns, h, l = 12, 1.0, 1.0
    desc = BasisDesc("spin", ns)
    H = oh.sparse_h(desc, _field_terms(ns, h))
    psi0 = gaussian_vectors(2 ** ns, [31], True)[:, 0]
    u, _, _ = osv.tpq(lambda x: H @ x, psi0, ns, l, 81)
    beta = osv.tpq_beta(u, ns, l)
    k = np.arange(1, 81)
    can = _free_spin_energy(beta[k], h)
    # absolute error on the energy scale h/2 = 0.5: finite size (about 0.01 for the exact ensemble
    # average at N_s = 12) plus the sampling error of one state of dimension 4096
    assert np.max(np.abs(u[k] - can)) < 0.04
    for wrong in (2.0, 0.5):
        bad = _free_spin_energy(wrong * beta[k], h)
        assert np.max(np.abs(u[k] - bad)) > 0.1
    # many spins: the ensemble-averaged mTPQ energy (closed form over the binomial spectrum,
    # weights (l - E/N)^(2k)) approaches the canonical energy at beta_k to O(1/N)
    n = 400
    m = np.arange(n + 1)
    E = h * (m - n / 2.0)
    logdeg = np.array([math.lgamma(n + 1) - math.lgamma(x + 1) - math.lgamma(n - x + 1) for x in m])
    for kk in (1, 10, 100, 400):
        lw = 2 * kk * np.log(l - E / n) + logdeg
        w = np.exp(lw - lw.max())
        uk = float((w * E).sum() / w.sum()) / n
        b = osv.tpq_beta(np.r_[np.zeros(kk), uk], n, l)[kk]
        assert abs(uk - _free_spin_energy(b, h)) <= 2e-3 * abs(uk)


def test_rayleigh_check_variance_and_residual():
    """App. A.3: the energy/variance check.  An exact eigenvector has zero variance and residual; an
    equal superposition of eigenvectors a and b has E = (E_a + E_b)/2, variance ((E_a - E_b)/2)^2 and
    residual |E_a - E_b|/2."""
    n = 6
    terms = L.random_spin_terms(n, 9, 61, conserve_sz=False, fields=True, real=False)
    Hd = oh.dense_h(BasisDesc("spin", n), terms)
    evals, evecs = np.linalg.eigh(Hd)
    apply = lambda x: Hd @ x
    for a in (0, 5, 40):
        e, var, res = osv.rayleigh_check(apply, evecs[:, a] * (0.3 - 1.1j))
        assert abs(e - evals[a]) < 1e-12 and abs(var) < 1e-12 and res < 1e-12
    for a, b in ((0, 1), (3, 50), (0, 63)):
        x = (evecs[:, a] * np.exp(0.7j) + evecs[:, b] * np.exp(-1.9j)) * 2.5
        e, var, res = osv.rayleigh_check(apply, x)
        half = (evals[a] - evals[b]) / 2
        assert abs(e - (evals[a] + evals[b]) / 2) < 1e-12
        assert abs(var - half * half) < 1e-11 * max(1.0, half * half)
        assert abs(res - abs(half)) < 1e-11


@pytest.mark.parametrize("sector", [False, True])
def test_c_oracle_c64_rows_equal_upcast_rows(sector):
    """The complex64-input C oracle reads each value, converts it exactly to complex128 and then does
    the same arithmetic as the complex128 rows, which are pinned against Kronecker and Jordan-Wigner
    matrices above: on the upcast input the two must agree bit for bit."""
    from oracle import c_oracle
    if sector:
        desc = BasisDesc("fermion", 5, "nupndn", n_up=2, n_dn=3)
        terms = L.random_fermion_terms(5, 12, 71, conserve_spin=True, real=False, n_dens=3, with_mu=True)
        st = ob.states(desc)
        rows, states = st, st
    else:
        terms = L.random_spin_terms(9, 14, 72, conserve_sz=False, fields=True, real=False)
        rows, states = np.arange(2 ** 9, dtype=np.uint64), None
    dim = len(rows)
    v = uniform_vectors(dim, [8, 9, 10, 11], True).astype(np.complex64)
    a = c_oracle.rows_hv(terms, rows, v, states=states)
    b = c_oracle.rows_hv(terms, rows, v.astype(np.complex128), states=states)
    assert np.array_equal(a, b)
    assert np.abs(a).max() > 0


def test_lowest_eigenvalue_matches_dense():
    """The sparse eigensolver step of the oracle against dense diagonalization (sectors of a
    12-site chain and a Hubbard cluster)."""
    for desc, terms in (
            (BasisDesc("spin", 12, "sz", two_sz=0), [L.heisenberg_bond(i, j) for i, j in L.chain_bonds(12)]),
            (BasisDesc("spin", 12, "sz", two_sz=10), [L.heisenberg_bond(i, j) for i, j in L.chain_bonds(12)]),
            (BasisDesc("fermion", 6, "nupndn", n_up=3, n_dn=3), L.hubbard_terms(L.rect_bonds(3, 2), 6, 1.0, 4.0))):
        H = oh.sparse_h(desc, terms)
        assert abs(osv.lowest_eigenvalue(H) - np.linalg.eigvalsh(H.toarray())[0]) < 1e-11


def test_golden_oracle_energies_pinned():
    """tests/golden/oracle_energies.json (written by make_oracle_energies.py from the oracle alone):
    its U = 0 Hubbard energy must equal the free-fermion closed form, the fully polarized tri24 sector
    72/4 exactly, the dimensions the binomials, and the sector energies must rise with Sz beyond
    Sz = 0 (the ground state of an antiferromagnet on a finite torus has the lowest total spin)."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_energies.json")))
    lv = sorted(-2 * math.cos(math.pi * m / 5) - 2 * math.cos(math.pi * n / 4) for m in range(1, 5)
                for n in range(1, 4))
    assert abs(g["hubbard_4x3_U0"]["e0"] - 2 * sum(lv[:6])) < 1e-10
    assert g["hubbard_4x3_U8"]["dim"] == comb(12, 6) ** 2
    assert g["hubbard_4x3_U0"]["e0"] < g["hubbard_4x3_U8"]["e0"] < 0
    tri = g["tri24"]
    assert sorted(int(k) for k in tri) == list(range(13))
    for sz in range(13):
        assert tri[str(sz)]["dim"] == comb(24, 12 + sz)
    assert tri["12"]["e0"] == 18.0
    e = [tri[str(sz)]["e0"] for sz in range(13)]
    assert all(a < b for a, b in zip(e, e[1:]))


def test_splitmix_stream_and_on_demand_rows():
    """The on-demand input vector of the C oracle (for spaces too large for host memory): its
    generator reproduces the published SplitMix64 outputs for seed 0, and rows computed with v
    evaluated on demand equal the counted-rank rows on the same vector stored explicitly."""
    from oracle import c_oracle
    sm = c_oracle.lib().oracle_splitmix64
    assert [sm(0, i) for i in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    desc = BasisDesc("spin", 12, "sz", two_sz=2)
    terms = [L.heisenberg_bond(i, j, 1.0) for i, j in L.kagome_bonds(2, 2)]
    st = ob.states(desc)
    nvec, seed = 3, 1234
    raw = np.array([sm(seed, i) for i in range(len(st) * nvec)], dtype=np.uint64)
    v = ((raw >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 * 2.0 - 1.0).reshape(len(st), nvec)
    a = c_oracle.rows_hv_counted_ondemand(desc, terms, st, seed, nvec)
    b = c_oracle.rows_hv_counted(desc, terms, st, v.astype(np.complex128))
    assert np.array_equal(a, b.real) and np.all(b.imag == 0)



GREEN2_QUADS = [(0, 2, 3, 5), (1, 4, 0, 2), (2, 2, 3, 3), (0, 3, 3, 0), (4, 1, 1, 4), (5, 5, 5, 5), (0, 1, 1, 0),
                (3, 0, 5, 3), (2, 5, 5, 1), (1, 0, 0, 1)]


@pytest.mark.parametrize("t", [1.0, 1j, 0.3 - 0.7j])
def test_green2_terms_match_jordan_wigner(t):
    """The two-body Green's-function observable t c+_a c_b c+_c c_d + h.c. applied operator by
    operator equals the product of Jordan-Wigner matrices, for distinct and repeated orbitals."""
    ns = 3
    for q in GREEN2_QUADS:
        term = L.green2_term(*q, t=t)
        H = oh.dense_h(BasisDesc("fermion", ns), [term])
        assert np.allclose(H, _kron_fermion_h(ns, [term]), atol=1e-14, rtol=0), q


def test_green2_special_cases():
    """c+_a c_a c+_b c_b = n_a n_b (a != b); c+_a c_b c+_b c_a = n_a (1 - n_b); with t = 1/2 the
    observable is exactly those densities."""
    desc = BasisDesc("fermion", 3)
    nn = oh.dense_h(desc, [L.Term(L.DENS, 1, 4, (1.0,))])
    assert np.array_equal(oh.dense_h(desc, [L.green2_term(1, 1, 4, 4, 0.5)]), nn)
    na = oh.dense_h(desc, [L.Term(L.NUM, 1, -1, (1.0,))])
    assert np.allclose(oh.dense_h(desc, [L.green2_term(1, 4, 4, 1, 0.5)]), na - nn, atol=0)
