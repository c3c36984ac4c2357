"""Full-size Lanczos configurations at parity with the oracle.

* 4x3 open Hubbard cluster (853,776 rows, complex128): at U = 0 the ground
  energy has a closed form (the sum of the 6 lowest one-body levels, twice);
  at U = 8 it is compared with the oracle's sparse eigensolver.
* 24-site triangular torus, all 13 Sz sectors in one batched FP32 recurrence
  of 200 steps: every refined energy against the oracle's FP64 value at
  |dE/E| <= 1e-8 (the mixed-precision gate).
* The energy/variance check of App. A.3: the GPU's variance and residual of
  its own eigenvector against the oracle's evaluation of the same vector.

Reference energies come from tests/golden/oracle_energies.json, written by
tests/golden/make_oracle_energies.py from oracle/ alone.
"""

import json
import math
import os

import numpy as np
import pytest
import torch

from synth import lattices as L
from synth.configs import BasisDesc, workload
from synth.vectors import device_uniform, gaussian_vectors
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import solvers as osv

pytestmark = pytest.mark.gpu

import paper_1703_03637_amd as hp  # noqa: E402

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_energies.json")))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


def _free_fermion_e0_4x3():
    """Sec. 5 Hubbard model at U = 0 on the 4x3 open cluster: one-body levels
    -2 cos(pi m/5) - 2 cos(pi n/4), m = 1..4, n = 1..3; 6 up + 6 down fill the 6 lowest twice."""
    lv = sorted(-2 * math.cos(math.pi * m / 5) - 2 * math.cos(math.pi * n / 4) for m in range(1, 5)
                for n in range(1, 4))
    return 2 * sum(lv[:6])


@pytest.mark.parametrize("U", [0.0, 8.0])
def test_hubbard_4x3_lanczos_full_size(U):
    print(f"[gpu] hubbard_4x3 lanczos U={U}", flush=True)
    w = workload("hubbard_4x3")
    terms = L.hubbard_terms(L.rect_bonds(4, 3, periodic=False), 12, t=1.0, U=U)
    basis = hp.hphi_basis_build(w.basis)
    ham = hp.hphi_ham_build(basis, terms)
    assert basis.dim == 853776
    x0 = device_uniform(basis.dim, 1, w.seeds[0], True, torch.complex128).reshape(-1).contiguous()
    r = hp.hphi_lanczos([ham], [x0], w.n_iter)[0]
    if U == 0.0:
        want = _free_fermion_e0_4x3()
        assert abs(want - (-16.601126159491542)) < 1e-12
    else:
        want = GOLD["hubbard_4x3_U8"]["e0"]
    print(f"[gpu]   E0 refined {r['e0_refined']!r} want {want!r} residual {r['residual']:.2e}", flush=True)
    assert abs(r["e0_refined"] - want) <= 1e-10 * abs(want)
    assert abs(r["e0_ritz"] - want) <= 1e-9 * abs(want)
    assert r["residual"] < 1e-4


def test_tri24_all_sectors_fp32_refined_match_oracle():
    """13 sectors Sz = 0..12 (dims 2,704,156 down to 1), FP32 vectors, FP64 alpha/beta, tridiagonal
    solve and Rayleigh-quotient refinement, 200 steps in one batched recurrence per step."""
    print("[gpu] tri24 all sectors vs oracle energies", flush=True)
    w = workload("tri24_allsz")
    descs = [w.basis] + list(w.extra_bases)
    bases = [hp.hphi_basis_build(d) for d in descs]
    hams = [hp.hphi_ham_build(b, w.terms) for b in bases]
    x0 = [device_uniform(b.dim, 1, w.seeds[k], False, torch.float32).reshape(-1).contiguous()
          for k, b in enumerate(bases)]
    res = hp.hphi_lanczos(hams, x0, w.n_iter)
    worst = 0.0
    for d, b, r in zip(descs, bases, res):
        g = GOLD["tri24"][str(d.two_sz // 2)]
        assert g["dim"] == b.dim
        rel = abs(r["e0_refined"] - g["e0"]) / max(1.0, abs(g["e0"]))
        worst = max(worst, rel)
        print(f"[gpu]   Sz={d.two_sz // 2} dim {b.dim} E0 {r['e0_refined']!r} oracle {g['e0']!r} rel {rel:.1e}",
              flush=True)
        assert rel <= 1e-8, (d.two_sz, r["e0_refined"], g["e0"])
    assert res[-1]["e0_refined"] == pytest.approx(18.0, abs=1e-12)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.complex128])
@pytest.mark.parametrize("case", ["hubbard_3x3", "chain14_full"])
def test_lanczos_variance_and_residual_match_oracle(dtype, case):
    """App. A.3: E = <x|H|x>/<x|x>, variance <H^2> - <H>^2 and residual |Hx - Ex|/|x| of the GPU's
    eigenvector x (a few steps short of convergence, so the variance is well above rounding),
    evaluated by the oracle on the same x."""
    if case == "hubbard_3x3":
        desc = BasisDesc("fermion", 9, "nupndn", n_up=3, n_dn=4)
        terms = L.hubbard_terms(L.rect_bonds(3, 3), 9, t=1.0, U=8.0)
    else:
        desc = BasisDesc("spin", 14)
        terms = [L.heisenberg_bond(i, j) for i, j in L.chain_bonds(14)]
    print(f"[gpu] lanczos variance vs oracle case={case} dtype={dtype}", flush=True)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    H = oh.sparse_h(desc, terms)
    x0 = gaussian_vectors(basis.dim, [77], dtype.is_complex)[:, 0]
    r = hp.hphi_lanczos([ham], [torch.from_numpy(x0).to(dtype).cuda()], 14)[0]
    x = r["x"].cpu().numpy()
    e, var, res = osv.rayleigh_check(lambda v: H @ v, x.astype(np.complex128))
    assert var > 1e-8, "the vector should be short of convergence"
    assert abs(r["e0_refined"] - e) <= 1e-12 * abs(e)
    assert abs(r["variance"] - var) <= 1e-12 * e * e
    assert abs(r["residual"] - res) <= 1e-9 * res
    assert abs(res * res - var) <= 1e-10 * e * e     # |Hx - Ex|^2/|x|^2 = <H^2> - E^2 for the RQ E
