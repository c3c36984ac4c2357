"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every entry point that include/hphi.h
declares, and reject bad arguments before touching a device.
"""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hphi.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hphi_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1703_03637_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libhphi.so is not built (run __graft_entry__.build())")
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("hphi_basis_build", "hphi_hv", "hphi_lanczos", "hphi_tpq_step"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert missing == []


def test_version_and_error_string(lib):
    assert b"gfx950" in lib.hphi_version()
    assert isinstance(lib.hphi_last_error(), bytes)


def test_basis_build_rejects_bad_descriptors(lib):
    from paper_1703_03637_amd import _lib as L
    out = C.c_void_p()
    bad = [
        L.BasisDescC(7, 4, 0, 0, 0, 0, 0, 0),                    # bad particle
        L.BasisDescC(L.HPHI_SPIN_HALF, 0, 0, 0, 0, 0, 0, 0),     # no sites
        L.BasisDescC(L.HPHI_SPIN_HALF, 63, 1, 1, 0, 0, 0, 0),    # > 62 bits
        L.BasisDescC(L.HPHI_SPIN_HALF, 41, 0, 0, 0, 0, 0, 0),    # full space > 40 bits
        L.BasisDescC(L.HPHI_SPIN_HALF, 4, 1, 1, 0, 0, 0, 0),     # 2Sz parity
        L.BasisDescC(L.HPHI_SPIN_HALF, 4, 2, 0, 1, 1, 0, 0),     # fermion sector on spins
        L.BasisDescC(L.HPHI_FERMION, 4, 2, 0, 5, 1, 0, 0),       # n_up > n_sites
        L.BasisDescC(L.HPHI_FERMION, 4, 1, 0, 0, 0, 0, 0),       # SZ on fermions
        L.BasisDescC(L.HPHI_FERMION, 4, 3, 0, 0, 0, 9, 0),       # n_tot > 2N
        L.BasisDescC(L.HPHI_SPIN_HALF, 4, 9, 0, 0, 0, 0, 0),     # bad sector
    ]
    for d in bad:
        rc = lib.hphi_basis_build(C.byref(d), C.byref(out))
        assert rc == L.HPHI_EINVAL, (d.particle, d.n_sites, d.sector)
        assert out.value is None
        assert len(lib.hphi_last_error()) > 0
    assert lib.hphi_basis_build(None, C.byref(out)) == L.HPHI_EINVAL


def test_entry_points_reject_null_handles(lib):
    from paper_1703_03637_amd import _lib as L
    opts = L.HvOptsC(1.0, 0.0, None, None)
    assert lib.hphi_hv(None, None, None, 1, 0, C.byref(opts), None) == L.HPHI_EINVAL
    assert lib.hphi_tpq_step(None, None, None, 1, 0, 1.5, 1, None, None, None) == L.HPHI_EINVAL
    assert lib.hphi_hv_elements(None, 0, 1, 4, 1, L.HPHI_C128, None, None, None, None, None, None) == L.HPHI_EINVAL
    assert lib.hphi_basis_dim(None, None) == L.HPHI_EINVAL
    lo = L.LanczosOptsC(10, 0, 0, 0, 0.0)
    assert lib.hphi_lanczos(None, 1, C.byref(lo), None, None, None, None, None) == L.HPHI_EINVAL
    assert lib.hphi_expect(None, None, 1, 0, None, None) == L.HPHI_EINVAL
    co = L.CgOptsC(1e-6, 2, 100, 1e-12)
    cr = L.CgResultC()
    assert lib.hphi_cg_refine(None, None, 0, -1.0, C.byref(co), None, C.byref(cr), None) == L.HPHI_EINVAL
    assert lib.hphi_hv_tune(None, None, None, 16, 3, None, None) == L.HPHI_EINVAL
    assert lib.hphi_hv_cma(None, None, None, 16, 3, 6, C.byref(opts), None) == L.HPHI_EINVAL
    assert lib.hphi_hv_cma_plan(None, 6, None, None) == L.HPHI_EINVAL
    lib.hphi_basis_free(None)
    lib.hphi_ham_free(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1703_03637_amd import _lib as L
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(ImportError):
        L.lib()


def test_product_path_does_not_import_oracle():
    import subprocess, sys
    code = ("import sys; import paper_1703_03637_amd, paper_1703_03637_amd.binding; "
            "assert not any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules), 'oracle imported'")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_injected_allocation_failure_is_enomem(lib, monkeypatch):
    """The allocation hook (HPHI_FAIL_ALLOC=N fails the N-th allocation) turns the first allocation of
    a basis build into HPHI_ENOMEM before any device call, with a message."""
    from paper_1703_03637_amd import _lib as L
    desc = L.BasisDescC(L.HPHI_SPIN_HALF, 8, L.HPHI_SECTOR_SZ, 0, 0, 0, 0, 0)
    out = C.c_void_p()
    monkeypatch.setenv("HPHI_FAIL_ALLOC", "1")
    assert lib.hphi_basis_build(C.byref(desc), C.byref(out)) == L.HPHI_ENOMEM
    assert b"allocation" in lib.hphi_last_error()
    assert out.value is None


def test_nonfinite_query_rejects_null(lib):
    from paper_1703_03637_amd import _lib as L
    f = C.c_int32()
    assert lib.hphi_ham_nonfinite(None, C.byref(f), 0, None) == L.HPHI_EINVAL
