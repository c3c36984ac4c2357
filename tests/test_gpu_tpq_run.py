"""The multi-step TPQ run (hphi_tpq_run): graph-replayed steps with the step
index and normalizing scales on the device.

Checked against one hphi_tpq_step call per step (bitwise: same kernels,
same launch shapes) and against the oracle's literal mTPQ trajectory
(Sec. 3.5), including the temperature beta_k = (2k/N_s)/(l - u_k).
"""

import numpy as np
import pytest
import torch

from synth.configs import BasisDesc, kh_honeycomb_terms
from synth.vectors import gaussian_vectors
from oracle import hamiltonian as oh
from oracle import solvers as osv

pytestmark = pytest.mark.gpu

import paper_1703_03637_amd as hp  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _setup(nvec, dtype, seed0=20):
    desc = BasisDesc("spin", 12)
    terms = kh_honeycomb_terms(lx=3, ly=2, random_dirs=False)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    psi0 = gaussian_vectors(basis.dim, list(range(seed0, seed0 + nvec)), True)
    t = torch.from_numpy(psi0).to(dtype).cuda()
    return desc, terms, ham, psi0, (t if nvec > 1 else t.reshape(-1).contiguous())


def _stepwise(ham, psi, l, k0, n):
    a = psi.clone()
    b = torch.empty_like(a)
    nvec = 1 if a.dim() == 1 else a.shape[1]
    scale = None
    log = []
    for j in range(n):
        o = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
        hp.hphi_tpq_step(ham, a, b, l, k0 + j, scale, o)
        log.append(o.reshape(4, nvec))
        a, b = b, a
        scale = o[3 * nvec:]
    return torch.stack(log).cpu().numpy(), a


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("n_steps", [1, 2, 7, 30])
@pytest.mark.parametrize("nvec,dtype", [(16, torch.complex64), (1, torch.complex128), (4, torch.complex128)])
def test_tpq_run_equals_single_steps(nvec, dtype, n_steps, use_graph):
    print(f"[gpu] tpq_run vs steps nvec={nvec} dtype={dtype} n={n_steps} graph={use_graph}", flush=True)
    _, _, ham, _, psi = _setup(nvec, dtype)
    ref, ref_state = _stepwise(ham, psi, 1.5, 3, n_steps)
    a = psi.clone()
    b = torch.empty_like(a)
    log = hp.hphi_tpq_run(ham, a, b, 1.5, 3, n_steps, use_graph=use_graph).cpu().numpy()
    assert np.array_equal(log, ref)
    fin = a if n_steps % 2 == 0 else b
    assert torch.equal(fin, ref_state)


def test_tpq_run_in_scale_and_continuation():
    """Two runs of 10 steps, the second started from the first's final state and scale with
    k0 = 11, equal one run of 20 steps."""
    _, _, ham, _, psi = _setup(4, torch.complex128)
    a, b = psi.clone(), torch.empty_like(psi)
    whole = hp.hphi_tpq_run(ham, a, b, 1.5, 1, 20).cpu().numpy()
    c, d = psi.clone(), torch.empty_like(psi)
    first = hp.hphi_tpq_run(ham, c, d, 1.5, 1, 10)
    scale = first[9, 3].contiguous()
    second = hp.hphi_tpq_run(ham, c, d, 1.5, 11, 10, in_scale=scale).cpu().numpy()
    assert np.array_equal(np.concatenate([first.cpu().numpy(), second]), whole)


@pytest.mark.parametrize("dtype,tol", [(torch.complex128, 1e-12), (torch.complex64, 2e-6)])
def test_tpq_run_matches_oracle_trajectory(dtype, tol):
    ns, l, steps, nvec = 12, 1.5, 60, 4
    desc, terms, ham, psi0, psi = _setup(nvec, dtype)
    H = oh.sparse_h(desc, terms)
    start = psi.cpu().numpy().astype(np.complex128)
    a, b = psi.clone(), torch.empty_like(psi)
    log = hp.hphi_tpq_run(ham, a, b, l, 1, steps).cpu().numpy()
    for bb in range(nvec):
        u_ref, h2_ref, psi_ref = osv.tpq(lambda v: H @ v, start[:, bb], ns, l, steps)
        assert np.allclose(log[:, 0, bb], u_ref, rtol=0, atol=tol)
        assert np.allclose(log[:, 1, bb], h2_ref, rtol=0, atol=tol)
        assert np.allclose(log[:, 2, bb], osv.tpq_beta(u_ref, ns, l), rtol=0, atol=100 * tol)
        fin = (a if steps % 2 == 0 else b)[:, bb].cpu().numpy().astype(np.complex128) * log[-1, 3, bb]
        # psi_ref is psi_steps; fin is the same state up to the storage rounding
        assert np.linalg.norm(fin - psi_ref) <= 50 * tol


def test_tpq_run_rejects_bad_arguments():
    _, _, ham, _, psi = _setup(4, torch.complex128)
    with pytest.raises(hp.HphiError):
        hp.hphi_tpq_run(ham, psi, psi, 1.5, 1, 4)
    with pytest.raises(hp.HphiError):
        hp.hphi_tpq_run(ham, psi, torch.empty_like(psi), 1.5, 0, 4)
