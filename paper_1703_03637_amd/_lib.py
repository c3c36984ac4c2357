"""ctypes declarations of libhphi.so (the C ABI in include/hphi.h).

Argument marshalling only; every computation happens in the HIP library.
Loading fails loudly if the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# HPHI_LIB names another build of the same library (experiments with kernel variants)
LIB_PATH = os.environ.get("HPHI_LIB") or os.path.join(HERE, "libhphi.so")

# status codes
HPHI_OK = 0
HPHI_EINVAL = -1
HPHI_ENOMEM = -2
HPHI_EDEVICE = -3
HPHI_ESECTOR = -4
HPHI_EDTYPE = -5
HPHI_ENONFINITE = -6
HPHI_NONFINITE_PRODUCT, HPHI_NONFINITE_NORM = 1, 2
HPHI_INFO_BREAKDOWN = 1
HPHI_INFO_MAXITER = 2

HPHI_SPIN_HALF, HPHI_FERMION = 0, 1
HPHI_SECTOR_NONE, HPHI_SECTOR_SZ, HPHI_SECTOR_NUP_NDN, HPHI_SECTOR_NTOT = 0, 1, 2, 3
HPHI_F64, HPHI_C128, HPHI_F32, HPHI_C64 = 0, 1, 2, 3
(HPHI_TERM_SPIN_BOND, HPHI_TERM_SPIN_FIELD, HPHI_TERM_HOP, HPHI_TERM_DENS, HPHI_TERM_NUM,
 HPHI_TERM_HUBBARD_U, HPHI_TERM_GREEN2) = range(7)


class BasisDescC(C.Structure):
    _fields_ = [("particle", C.c_int32), ("n_sites", C.c_int32), ("sector", C.c_int32),
                ("two_sz", C.c_int32), ("n_up", C.c_int32), ("n_dn", C.c_int32),
                ("n_tot", C.c_int32), ("split_bits", C.c_int32)]


class TermC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("reserved", C.c_int32),
                ("c", C.c_double * 9)]


class HvOptsC(C.Structure):
    _fields_ = [("a", C.c_double), ("b", C.c_double), ("in_scale", C.c_void_p), ("reduce", C.c_void_p)]


class LanczosOptsC(C.Structure):
    _fields_ = [("n_iter", C.c_int32), ("dtype", C.c_int32), ("refine", C.c_int32),
                ("use_graph", C.c_int32), ("breakdown_tol", C.c_double)]


class LanczosResultC(C.Structure):
    _fields_ = [("alpha", C.POINTER(C.c_double)), ("beta", C.POINTER(C.c_double)),
                ("n_done", C.c_int32), ("info", C.c_int32), ("e0_ritz", C.c_double),
                ("e0_refined", C.c_double), ("variance", C.c_double), ("residual", C.c_double)]


class CgOptsC(C.Structure):
    _fields_ = [("shift", C.c_double), ("n_inverse", C.c_int32), ("cg_max_iter", C.c_int32), ("cg_tol", C.c_double)]


class CgResultC(C.Structure):
    _fields_ = [("e_refined", C.c_double), ("variance", C.c_double), ("residual", C.c_double),
                ("cg_iters", C.c_int32), ("info", C.c_int32)]


class HphiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hphi error {code}: {msg}")
        self.code = code


_lib = None

_SIGS = {
    "hphi_basis_build": ([C.POINTER(BasisDescC), C.POINTER(C.c_void_p)], C.c_int),
    "hphi_basis_dim": ([C.c_void_p, C.POINTER(C.c_int64)], C.c_int),
    "hphi_basis_rank": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "hphi_basis_unrank": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
    "hphi_basis_free": ([C.c_void_p], None),
    "hphi_ham_build": ([C.c_void_p, C.POINTER(TermC), C.c_int64, C.POINTER(C.c_void_p)], C.c_int),
    "hphi_ham_is_complex": ([C.c_void_p, C.POINTER(C.c_int32)], C.c_int),
    "hphi_ham_nonfinite": ([C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.c_void_p], C.c_int),
    "hphi_ham_free": ([C.c_void_p], None),
    "hphi_hv": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.POINTER(HvOptsC),
                 C.c_void_p], C.c_int),
    "hphi_hv_tune": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "hphi_hv_cma": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.POINTER(HvOptsC),
                     C.c_void_p], C.c_int),
    "hphi_hv_cma_plan": ([C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_void_p], C.c_int),
    "hphi_hv_elements": ([C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_int64, C.c_int32, C.c_void_p,
                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hphi_lanczos": ([C.POINTER(C.c_void_p), C.c_int32, C.POINTER(LanczosOptsC),
                      C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                      C.POINTER(LanczosResultC), C.c_void_p], C.c_int),
    "hphi_tpq_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_double,
                       C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hphi_tpq_run": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                      C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p], C.c_int),
    "hphi_tpq_run_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                              C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "hphi_cg_refine": ([C.c_void_p, C.c_void_p, C.c_int32, C.c_double, C.POINTER(CgOptsC), C.c_void_p,
                        C.POINTER(CgResultC), C.c_void_p], C.c_int),
    "hphi_expect": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
    "hphi_last_error": ([], C.c_char_p),
    "hphi_version": ([], C.c_char_p),
}


def lib():
    """The loaded library; raises if libhphi.so is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1703_03637_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(rc: int, allow=(HPHI_OK,)) -> int:
    if rc in allow:
        return rc
    msg = lib().hphi_last_error().decode(errors="replace")
    raise HphiError(rc, msg)
