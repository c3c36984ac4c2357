"""GPU tests of the fault surface: non-finite inputs, the non-finite flag
word of the fused reductions, degenerate start vectors, injected allocation
failures, and the Lanczos eigenvector written over the start vector.

Every case runs normal kernels on valid memory; faults are forced from the
host (a NaN or Inf placed in an input, the allocation hook), never on the GPU.
"""

import itertools

import numpy as np
import pytest
import torch

from synth import lattices as L
from synth.configs import BasisDesc, kh_honeycomb_terms
from synth.vectors import gaussian_vectors, uniform_vectors
from oracle import basis as ob
from oracle import hamiltonian as oh

pytestmark = pytest.mark.gpu

import paper_1703_03637_amd as hp  # noqa: E402
from paper_1703_03637_amd import _lib  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


# (space, terms, schedule env): single-pass full space and sector, windowed with the row tile in LDS
# (4 lanes per row) and with lane exchange (8 lanes per row), a fermion sector, a 34-bit sector
NONFINITE_CASES = {
    "full_single_pass": (BasisDesc("spin", 12), lambda: kh_honeycomb_terms(lx=3, ly=2, random_dirs=False),
                         {"HPHI_WINDOWED": "0"}),
    "full_windowed_tile": (BasisDesc("spin", 12), lambda: kh_honeycomb_terms(lx=3, ly=2, random_dirs=False),
                           {"HPHI_WINDOWED": "1", "HPHI_L2_WINDOW_KB": "8", "HPHI_PASSES": "2", "HPHI_LPR": "4"}),
    "full_windowed_lanes": (BasisDesc("spin", 12), lambda: kh_honeycomb_terms(lx=3, ly=2, random_dirs=False),
                            {"HPHI_WINDOWED": "1", "HPHI_L2_WINDOW_KB": "8", "HPHI_PASSES": "2", "HPHI_LPR": "8"}),
    "spin_sector": (BasisDesc("spin", 10, "sz", two_sz=2),
                    lambda: L.random_spin_terms(10, 14, 103, conserve_sz=True, fields=True, real=False), {}),
    "fermion_sector": (BasisDesc("fermion", 6, "nupndn", n_up=3, n_dn=2),
                       lambda: L.hubbard_terms(L.rect_bonds(3, 2), 6, t=1.0, U=4.0), {}),
    "spin_34bit_sector": (BasisDesc("spin", 34, "sz", two_sz=30),
                          lambda: [L.heisenberg_bond(i, j) for i, j in L.chain_bonds(34)], {}),
}


def _states(desc):
    """Basis states in ascending order (the oracle enumerates up to 28 bits; wider spin sectors with
    few down spins are listed from their down-spin positions)."""
    if desc.n_sites <= 28:
        return ob.states(desc)
    n_dn = (desc.n_sites - desc.two_sz) // 2
    full = (1 << desc.n_sites) - 1
    st = [full ^ sum(1 << b for b in c) for c in itertools.combinations(range(desc.n_sites), n_dn)]
    return np.array(sorted(st), dtype=np.uint64)


@pytest.mark.parametrize("nvec", [1, 16])
@pytest.mark.parametrize("name", list(NONFINITE_CASES))
def test_nonfinite_input_stays_with_the_rows_it_couples_to(monkeypatch, name, nvec):
    """One Inf and one NaN entry in v: rows that do not couple to them (H[s, t] = 0, s != t) stay
    finite and equal the oracle's product with those entries zeroed; the coupled rows are non-finite;
    the reductions set the product bit of the flag word, which clears on request."""
    desc, mk, env = NONFINITE_CASES[name]
    if desc.n_sites > 32 and nvec > 4:
        nvec = 4
    print(f"[gpu] non-finite input case={name} nvec={nvec}", flush=True)
    for k, val in env.items():
        monkeypatch.setenv(k, val)
    terms = mk()
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    st = _states(desc)
    dim = len(st)
    assert dim == basis.dim
    H = oh.sparse_h(desc, terms, st).tocsc()
    v = uniform_vectors(dim, list(range(900, 900 + nvec)), True)
    t_inf, t_nan = dim // 3, (2 * dim) // 3
    bad = v.copy()
    bad[t_inf, :] = np.inf
    bad[t_nan, 0] = np.nan
    vd = torch.from_numpy(bad.astype(np.complex64) if nvec == 16 else bad).cuda().contiguous()
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    hp.hphi_ham_nonfinite(ham, clear=True)
    u = hp.hphi_hv(ham, vd, reduce=red).cpu().numpy().astype(np.complex128)
    coupled = np.zeros(dim, bool)
    for t in (t_inf, t_nan):
        col = H[:, t]
        coupled[col.indices[col.data != 0]] = True
        coupled[t] = True
    clean = vd.cpu().numpy().astype(np.complex128)
    clean[t_inf, :] = 0
    clean[t_nan, 0] = 0
    ref = H @ clean
    assert np.isfinite(u[~coupled]).all(), "non-finite value reached an uncoupled row"
    tol = 1e-12 if nvec == 1 else 2e-6
    scale = np.abs(H) @ np.abs(clean)
    assert np.all(np.abs(u[~coupled] - ref[~coupled]) <= tol * (scale[~coupled] + 1e-300))
    assert not np.isfinite(u[t_inf]).any()
    assert hp.hphi_ham_nonfinite(ham, clear=True) & _lib.HPHI_NONFINITE_PRODUCT
    assert hp.hphi_ham_nonfinite(ham) == 0
    # a finite input leaves the word clear
    vd.copy_(torch.from_numpy(v.astype(np.complex64) if nvec == 16 else v))
    hp.hphi_hv(ham, vd, reduce=red)
    assert hp.hphi_ham_nonfinite(ham) == 0
    assert np.isfinite(red.cpu().numpy()).all()


def _chain_ham(n=10, sector=True):
    desc = BasisDesc("spin", n, "sz", two_sz=0) if sector else BasisDesc("spin", n)
    basis = hp.hphi_basis_build(desc)
    return desc, hp.hphi_ham_build(basis, [L.heisenberg_bond(i, j) for i, j in L.chain_bonds(n)])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_lanczos_zero_start_vector_is_rejected(dtype):
    print(f"[gpu] lanczos zero start dtype={dtype}", flush=True)
    _, ham = _chain_ham()
    x0 = torch.zeros(ham.dim, dtype=dtype, device="cuda")
    with pytest.raises(hp.HphiError) as ei:
        hp.hphi_lanczos([ham], [x0], 20)
    assert ei.value.code == _lib.HPHI_EINVAL and "zero start vector" in str(ei.value)


@pytest.mark.parametrize("batched", [False, True])
def test_lanczos_nonfinite_start_vector_is_reported(batched):
    print(f"[gpu] lanczos non-finite start batched={batched}", flush=True)
    _, ham = _chain_ham()
    _, ham2 = _chain_ham(10, sector=True)
    x0 = torch.from_numpy(gaussian_vectors(ham.dim, [5], False)[:, 0]).cuda()
    x0[7] = float("nan")
    hams, x0s = ([ham, ham2], [x0, x0.clone()]) if batched else ([ham], [x0])
    with pytest.raises(hp.HphiError) as ei:
        hp.hphi_lanczos(hams, x0s, 20)
    assert ei.value.code == _lib.HPHI_ENONFINITE
    # the next run on finite start vectors clears the word and succeeds
    for x in x0s:
        x[7] = 0.25
    res = hp.hphi_lanczos(hams, x0s, 20)
    assert np.isfinite(res[0]["e0_refined"])


@pytest.mark.parametrize("dtype", [torch.float64, torch.complex128])
def test_lanczos_eigenvector_over_start_vector(dtype):
    """x_out may be v0's buffer (FP64 storage): same alpha/beta, energies and eigenvector as with a
    separate x_out, and the start vector's buffer then holds the eigenvector."""
    print(f"[gpu] lanczos x_out over v0 dtype={dtype}", flush=True)
    desc, ham = _chain_ham(12)
    x0 = gaussian_vectors(ham.dim, [44], dtype.is_complex)[:, 0]
    a = torch.from_numpy(x0).cuda()
    r1 = hp.hphi_lanczos([ham], [a], 60)[0]
    b = torch.from_numpy(x0).cuda()
    r2 = hp.hphi_lanczos([ham], [b], 60, x_out=[b])[0]
    assert np.array_equal(r1["alpha"], r2["alpha"]) and np.array_equal(r1["beta"], r2["beta"])
    assert r1["e0_refined"] == r2["e0_refined"] and r1["residual"] == r2["residual"]
    assert torch.equal(r1["x"], b)


def test_injected_allocation_failures_return_enomem(monkeypatch):
    """Every allocation of a basis build, a Hamiltonian build and a batched Lanczos run fails in
    turn (the HPHI_FAIL_ALLOC hook): each call returns HPHI_ENOMEM cleanly, and afterwards the same
    calls succeed and give the same energies as a run without injection."""
    print("[gpu] injected allocation failures", flush=True)
    terms = [L.heisenberg_bond(i, j) for i, j in L.chain_bonds(10)]
    descs = [BasisDesc("spin", 10, "sz", two_sz=2 * s) for s in range(3)]
    x0 = [torch.from_numpy(gaussian_vectors(ob.dimension(d), [60 + k], False)[:, 0]).cuda()
          for k, d in enumerate(descs)]

    def run():
        bases = [hp.hphi_basis_build(d) for d in descs]
        hams = [hp.hphi_ham_build(b, terms) for b in bases]
        return [r["e0_refined"] for r in hp.hphi_lanczos(hams, x0, 30)]

    want = run()
    failures = 0
    for n in range(1, 400):
        monkeypatch.setenv("HPHI_FAIL_ALLOC", str(n))
        try:
            got = run()
        except hp.HphiError as e:
            assert e.code == _lib.HPHI_ENOMEM, str(e)
            failures += 1
            continue
        assert got == want
        break
    else:
        pytest.fail("allocations never ran out of injected failures")
    assert failures >= 5
    monkeypatch.delenv("HPHI_FAIL_ALLOC")
    assert run() == want
