"""ctypes wrapper of the C row-slice oracle (hv_oracle.c).

Test infrastructure only.  rows_hv(desc, terms, rows, v, states=None)
evaluates u[s] = sum_t <s|H|t> v[t] for the given row configurations.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

from synth.lattices import SPIN_BOND, SPIN_FIELD, HOP, DENS, NUM, HUBBARD_U
from .build import LIB, build

_KIND = {SPIN_BOND: 0, SPIN_FIELD: 1, HOP: 2, DENS: 3, NUM: 4, HUBBARD_U: 5}


class _OTerm(C.Structure):
    _fields_ = [("kind", C.c_int32), ("i", C.c_int32), ("j", C.c_int32), ("reserved", C.c_int32),
                ("c", C.c_double * 9)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        for name in ("oracle_hv_rows", "oracle_hv_rows_c64"):
            fn = getattr(L, name)
            fn.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                           C.c_int, C.c_void_p]
            fn.restype = C.c_int
        L.oracle_hv_rows_counted.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                             C.c_int, C.c_void_p]
        L.oracle_hv_rows_counted.restype = C.c_int
        L.oracle_hv_rows_counted_ondemand.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_int64,
                                                       C.c_uint64, C.c_int, C.c_void_p]
        L.oracle_hv_rows_counted_ondemand.restype = C.c_int
        L.oracle_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_unrank_counted.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.oracle_unrank_counted.restype = C.c_int
        L.oracle_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _terms(terms):
    arr = (_OTerm * max(1, len(terms)))()
    for n, t in enumerate(terms):
        arr[n].kind = _KIND[t.kind]
        arr[n].i = t.i
        arr[n].j = t.j
        for k, x in enumerate(t.c):
            arr[n].c[k] = x
    return arr


def threads() -> int:
    return lib().oracle_max_threads()


def rows_hv(terms, rows: np.ndarray, v: np.ndarray, states: np.ndarray | None = None) -> np.ndarray:
    """u for the row configurations `rows`; v is (dim,) or (dim, nvec), complex128 or complex64."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    nvec = 1 if v.ndim == 1 else v.shape[1]
    if nvec > 64:
        raise ValueError("nvec <= 64")
    dim = v.shape[0]
    if v.dtype == np.complex64:
        fn = lib().oracle_hv_rows_c64
    else:
        v = v.astype(np.complex128, copy=False)
        fn = lib().oracle_hv_rows
    v = np.ascontiguousarray(v)
    u = np.zeros((len(rows), nvec), dtype=np.complex128)
    st = None if states is None else np.ascontiguousarray(states, dtype=np.uint64)
    arr = _terms(terms)
    rc = fn(arr, len(terms), None if st is None else st.ctypes.data, dim, rows.ctypes.data, len(rows),
            v.ctypes.data, nvec, u.ctypes.data)
    if rc != 0:
        raise ValueError("a term leaves the basis")
    return u if v.ndim == 2 else u[:, 0]


class _OSector(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nbits", C.c_int32), ("n_a", C.c_int32), ("n_b", C.c_int32)]


def _sector(desc):
    nb = desc.n_sites if desc.particle == "spin" else 2 * desc.n_sites
    if desc.sector == "none":
        return _OSector(0, nb, 0, 0)
    if desc.sector == "nupndn":
        return _OSector(2, nb, desc.n_up, desc.n_dn)
    if desc.particle == "spin":
        return _OSector(1, nb, (desc.n_sites + desc.two_sz) // 2, 0)
    return _OSector(1, nb, desc.n_tot, 0)


def rows_hv_counted(desc, terms, rows: np.ndarray, v: np.ndarray) -> np.ndarray:
    """As rows_hv, with targets ranked by counting within desc's sector (no
    basis list; v holds the whole vector, complex128)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    nvec = 1 if v.ndim == 1 else v.shape[1]
    if nvec > 64:
        raise ValueError("nvec <= 64")
    v = np.ascontiguousarray(v.astype(np.complex128, copy=False))
    u = np.zeros((len(rows), nvec), dtype=np.complex128)
    sec = _sector(desc)
    arr = _terms(terms)
    rc = lib().oracle_hv_rows_counted(arr, len(terms), C.byref(sec), rows.ctypes.data, len(rows), v.ctypes.data,
                                      nvec, u.ctypes.data)
    if rc != 0:
        raise ValueError("a term leaves the basis")
    return u if v.ndim == 2 else u[:, 0]


def unrank_counted(desc, idx: np.ndarray) -> np.ndarray:
    """Configurations of the given sector indices (counting, no basis list)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    cfg = np.zeros(len(idx), dtype=np.uint64)
    sec = _sector(desc)
    if lib().oracle_unrank_counted(C.byref(sec), idx.ctypes.data, len(idx), cfg.ctypes.data) != 0:
        raise ValueError("rank out of range")
    return cfg


def rows_hv_counted_ondemand(desc, terms, rows: np.ndarray, seed: int, nvec: int = 1) -> np.ndarray:
    """u for the given rows of desc's sector with a real input vector that is never stored:
    v[t, b] = splitmix_uniform(seed, t * nvec + b) is evaluated per target (real terms only).
    For sectors too large for host memory (the 36-site kagome Sz = 0 space)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    u = np.zeros((len(rows), nvec), dtype=np.float64)
    sec = _sector(desc)
    arr = _terms(terms)
    rc = lib().oracle_hv_rows_counted_ondemand(arr, len(terms), C.byref(sec), rows.ctypes.data, len(rows),
                                               C.c_uint64(seed), nvec, u.ctypes.data)
    if rc != 0:
        raise ValueError("a term leaves the basis")
    return u if nvec > 1 else u[:, 0]
