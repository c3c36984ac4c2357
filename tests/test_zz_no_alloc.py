"""The allocation-free TPQ run (hphi_tpq_run_noalloc) against hphi_tpq_run.

Called through the C ABI twice in a row, the second time with a smaller
input; with the allocation hook armed (HPHI_FAIL_ALLOC=1 fails the first
allocation the library attempts), so any allocation would surface as
HPHI_ENOMEM.  Results must equal hphi_tpq_run's bit for bit when both use
the same pass plan, and to the parity bar (1e-12 for complex128) when the
allocation-free call runs first on a fresh Hamiltonian and must take the
single-pass kernel.
"""

import numpy as np
import pytest
import torch

from synth.configs import BasisDesc, kh_honeycomb_terms
from synth import lattices as L
from synth.vectors import gaussian_vectors

pytestmark = pytest.mark.gpu

import paper_1703_03637_amd as hp  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _ham(desc, terms):
    return hp.hphi_ham_build(hp.hphi_basis_build(desc), terms)


def _start(dim, nvec, dtype, seed):
    x = torch.from_numpy(gaussian_vectors(dim, list(range(seed, seed + nvec)), True)).to(dtype).cuda()
    return x if nvec > 1 else x.reshape(-1).contiguous()


def _reference(ham, psi, l, k0, n):
    a, b = psi.clone(), torch.empty_like(psi)
    log = hp.hphi_tpq_run(ham, a, b, l, k0, n).clone()
    return log, (a if n % 2 == 0 else b)


def _noalloc(ham, psi, l, k0, n, monkeypatch):
    nvec = 1 if psi.dim() == 1 else psi.shape[1]
    a, b = psi.clone(), torch.empty_like(psi)
    log = torch.empty((n, 4, nvec), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    monkeypatch.setenv("HPHI_FAIL_ALLOC", "1")
    try:
        hp.hphi_tpq_run_noalloc(ham, a, b, l, k0, n, log)
        torch.cuda.synchronize()
    finally:
        monkeypatch.delenv("HPHI_FAIL_ALLOC")
    return log, (a if n % 2 == 0 else b)


def test_noalloc_run_matches_tpq_run_twice(monkeypatch):
    print("[gpu] no-alloc TPQ run: two calls, the second smaller", flush=True)
    # first call: 12-site honeycomb, 16 complex64 samples, windowed plan built by the reference run
    ham1 = _ham(BasisDesc("spin", 12), kh_honeycomb_terms(lx=3, ly=2, random_dirs=False))
    psi1 = _start(ham1.dim, 16, torch.complex64, 20)
    ref_log, ref_state = _reference(ham1, psi1, 1.5, 1, 9)
    log, state = _noalloc(ham1, psi1, 1.5, 1, 9, monkeypatch)
    assert torch.equal(log, ref_log)
    assert torch.equal(state, ref_state)
    # second call, smaller: a 5-site Hubbard sector (10 orbitals, dim 100), one complex128 sample, k0 = 4
    desc = BasisDesc("fermion", 5, "nupndn", n_up=2, n_dn=2)
    ham2 = _ham(desc, L.hubbard_terms(L.chain_bonds(5), 5, t=1.0, U=4.0))
    psi2 = _start(ham2.dim, 1, torch.complex128, 40)
    assert ham2.dim * 1 * 16 < ham1.dim * 16 * 8
    ref_log, ref_state = _reference(ham2, psi2, 2.5, 4, 6)
    log, state = _noalloc(ham2, psi2, 2.5, 4, 6, monkeypatch)
    assert torch.equal(log, ref_log)
    assert torch.equal(state, ref_state)


def test_noalloc_run_on_fresh_ham_matches_to_parity(monkeypatch):
    """Called first on a fresh Hamiltonian, the run may not build a pass plan (that allocates), so
    it takes the single-pass kernel: same trajectory within the FP64 parity bar."""
    print("[gpu] no-alloc TPQ run on a fresh ham", flush=True)
    terms = kh_honeycomb_terms(lx=3, ly=2, random_dirs=False)
    ham_a = _ham(BasisDesc("spin", 12), terms)
    psi = _start(ham_a.dim, 4, torch.complex128, 60)
    log, state = _noalloc(ham_a, psi, 1.5, 1, 8, monkeypatch)
    ham_b = _ham(BasisDesc("spin", 12), terms)
    ref_log, ref_state = _reference(ham_b, psi, 1.5, 1, 8)
    assert np.allclose(log.cpu().numpy(), ref_log.cpu().numpy(), rtol=1e-12, atol=1e-13)
    assert (state - ref_state).abs().max().item() <= 1e-12 * ref_state.abs().max().item()


def test_noalloc_run_rejects_bad_arguments():
    ham = _ham(BasisDesc("spin", 8), [L.heisenberg_bond(i, j) for i, j in L.chain_bonds(8)])
    psi = _start(ham.dim, 2, torch.complex128, 80)
    log = torch.empty((4, 4, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HphiError):
        hp.hphi_tpq_run_noalloc(ham, psi, psi, 1.5, 1, 4, log)
    with pytest.raises(hp.HphiError):
        hp.hphi_tpq_run_noalloc(ham, psi, torch.empty_like(psi), 1.5, 0, 4, log)
