"""The block-staged sector product (one high-half block of rows in LDS per
workgroup, two-level low-rank table in LDS): FP64 products against the
oracle on sector bases of spins and fermions, for every storage type,
1/2/4 vectors, 1..3 workgroups per CU and blocks split over several staged
chunks; Lanczos and TPQ through it; sampled rows of the 36-bit spaces.
"""

import numpy as np
import pytest
import torch

from synth import lattices as L
from synth.configs import BasisDesc, workload
from synth.vectors import uniform_vectors, gaussian_vectors
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import solvers as osv

pytestmark = pytest.mark.gpu

import paper_1703_03637_amd as hp  # noqa: E402

CASES = {
    "spin_sz_dm": (BasisDesc("spin", 10, "sz", two_sz=2),
                   lambda: L.random_spin_terms(10, 14, 103, conserve_sz=True, fields=True, real=False)),
    "spin_sz_split3": (BasisDesc("spin", 11, "sz", two_sz=-1, split_bits=3),
                       lambda: L.random_spin_terms(11, 15, 104, conserve_sz=True, real=True)),
    "tri12_sz0": (BasisDesc("spin", 12, "sz", two_sz=0),
                  lambda: [L.heisenberg_bond(i, j) for i, j in L.triangular_bonds(4, 3)]),
    "ferm_nupndn": (BasisDesc("fermion", 5, "nupndn", n_up=2, n_dn=3),
                    lambda: L.random_fermion_terms(5, 12, 105, conserve_spin=True, real=False, n_dens=3,
                                                   with_mu=True)),
    "ferm_ntot": (BasisDesc("fermion", 4, "ntot", n_tot=3),
                  lambda: L.random_fermion_terms(4, 10, 107, conserve_spin=False, real=True, n_dens=2)),
    "hubbard_3x3": (BasisDesc("fermion", 9, "nupndn", n_up=3, n_dn=4),
                    lambda: L.hubbard_terms(L.rect_bonds(3, 3), 9, t=1.0, U=8.0)),
}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"


@pytest.mark.parametrize("chunk", [0, 64])
@pytest.mark.parametrize("per_cu", [1, 3])
@pytest.mark.parametrize("nvec,dtype", [(1, torch.complex128), (1, torch.float64), (2, torch.complex64),
                                        (4, torch.complex128), (4, torch.float32)])
@pytest.mark.parametrize("name", list(CASES))
def test_sector_blocks_product_matches_oracle(monkeypatch, name, nvec, dtype, per_cu, chunk):
    desc, mk = CASES[name]
    terms = mk()
    print(f"[gpu] sector blocks {name} nvec={nvec} {dtype} per_cu={per_cu} chunk={chunk}", flush=True)
    monkeypatch.setenv("HPHI_SECTOR_BLOCKS", "1")
    monkeypatch.setenv("HPHI_BLOCKS_PER_CU", str(per_cu))
    if chunk:
        monkeypatch.setenv("HPHI_SECTOR_CHUNK", str(chunk))
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    if ham.is_complex and not dtype.is_complex:
        pytest.skip("complex elements need complex storage")
    st = ob.states(desc)
    v = uniform_vectors(len(st), list(range(500, 500 + nvec)), dtype.is_complex)
    vd = torch.from_numpy(v).to(dtype).cuda().contiguous()
    if nvec == 1:
        vd = vd.reshape(-1)
    red = torch.empty(4 * nvec, dtype=torch.float64, device="cuda")
    a, b = 0.75, -0.5
    u = hp.hphi_hv(ham, vd, a=a, b=b, reduce=red).cpu().numpy().reshape(len(st), nvec).astype(np.complex128)
    vin = vd.cpu().numpy().reshape(len(st), nvec).astype(np.complex128)
    H = oh.sparse_h(desc, terms, st)
    hx = H @ vin
    ref = a * hx + b * vin
    if dtype in (torch.complex128, torch.float64):
        bound = abs(a) * (abs(H) @ np.abs(vin)) + abs(b) * np.abs(vin)
        assert np.all(np.abs(u - ref) <= 1e-12 * bound + 1e-300)
    else:
        assert np.linalg.norm(u - ref) <= 1e-6 * np.linalg.norm(ref)
    r = red.cpu().numpy().reshape(4, nvec)
    for k in range(nvec):
        assert abs(r[0, k] - np.vdot(vin[:, k], vin[:, k]).real) <= 1e-12 * np.vdot(vin[:, k], vin[:, k]).real
        assert abs(r[1, k] - np.vdot(vin[:, k], hx[:, k]).real) <= 1e-11 * np.linalg.norm(vin[:, k]) * \
            np.linalg.norm(hx[:, k])


def test_sector_blocks_bitwise_reproducible_and_equal_to_lanczos(monkeypatch):
    """Two runs give identical bits; Lanczos through the block-staged kernel (with the previous
    vector as the extra input) reaches the dense ground state."""
    monkeypatch.setenv("HPHI_SECTOR_BLOCKS", "1")
    desc, mk = CASES["hubbard_3x3"]
    terms = mk()
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    v = torch.from_numpy(uniform_vectors(basis.dim, [7], True)[:, 0]).cuda()
    u1 = hp.hphi_hv(ham, v)
    u2 = hp.hphi_hv(ham, v)
    assert torch.equal(u1, u2)
    x0 = torch.from_numpy(gaussian_vectors(basis.dim, [8], False)[:, 0]).cuda()
    r = hp.hphi_lanczos([ham], [x0], 120)[0]
    e0 = np.linalg.eigvalsh(oh.sparse_h(desc, terms).toarray())[0]
    assert abs(r["e0_refined"] - e0) <= 1e-10 * abs(e0)


@pytest.mark.parametrize("name", ["kagome36_2sz32", "hubbard18_1u1d", "kagome36_2sz30"])
@pytest.mark.parametrize("nvec", [1, 4])
def test_sector_blocks_w64_small_sectors(monkeypatch, name, nvec):
    """36-bit sectors (the layout of the kagome and 18-site Hubbard workloads) with few particles,
    small enough for the oracle: the block-staged kernel against the oracle."""
    import itertools
    print(f"[gpu] sector blocks 36-bit {name} nvec={nvec}", flush=True)
    monkeypatch.setenv("HPHI_SECTOR_BLOCKS", "1")
    if name.startswith("kagome"):
        two_sz = int(name.split("sz")[1])
        desc = BasisDesc("spin", 36, "sz", two_sz=two_sz)
        terms = [L.heisenberg_bond(i, j) for i, j in L.kagome_bonds(3, 4)]
        n_dn = (36 - two_sz) // 2
        full = (1 << 36) - 1
        st = np.array(sorted(full ^ sum(1 << b for b in c) for c in itertools.combinations(range(36), n_dn)),
                      dtype=np.uint64)
    else:
        w = workload("hubbard18_tpq")
        desc = BasisDesc("fermion", 18, "nupndn", n_up=1, n_dn=1)
        terms = w.terms
        st = np.array(sorted((1 << (2 * a)) | (1 << (2 * b + 1)) for a in range(18) for b in range(18)),
                      dtype=np.uint64)
    basis = hp.hphi_basis_build(desc)
    ham = hp.hphi_ham_build(basis, terms)
    assert basis.dim == len(st)
    v = uniform_vectors(len(st), list(range(40, 40 + nvec)), True)
    vd = torch.from_numpy(v).cuda()
    if nvec == 1:
        vd = vd.reshape(-1).contiguous()
    u = hp.hphi_hv(ham, vd).cpu().numpy().reshape(len(st), nvec)
    H = oh.sparse_h(desc, terms, st)
    ref = H @ v
    bound = abs(H) @ np.abs(v)
    assert np.all(np.abs(u - ref) <= 1e-12 * bound + 1e-300)
