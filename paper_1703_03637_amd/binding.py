"""Python binding of the C ABI, one function per entry point, same names.

Only argument marshalling happens here: torch tensors provide device
memory and the current HIP stream; every step of the computation runs in
libhphi.so.  Vectors are torch tensors on the GPU of shape (dim,) or
(dim, nvec) (interleaved, C-contiguous) with dtype float64, complex128,
float32 or complex64.
"""

from __future__ import annotations

import ctypes as C
from typing import Iterable, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from ._lib import check

_PARTICLE = {"spin": L.HPHI_SPIN_HALF, "fermion": L.HPHI_FERMION}
_SECTOR = {"none": L.HPHI_SECTOR_NONE, "sz": L.HPHI_SECTOR_SZ, "nupndn": L.HPHI_SECTOR_NUP_NDN,
           "ntot": L.HPHI_SECTOR_NTOT}
_KIND = {"spin_bond": L.HPHI_TERM_SPIN_BOND, "spin_field": L.HPHI_TERM_SPIN_FIELD, "hop": L.HPHI_TERM_HOP,
         "dens": L.HPHI_TERM_DENS, "num": L.HPHI_TERM_NUM, "hubbard_u": L.HPHI_TERM_HUBBARD_U,
         "green2": L.HPHI_TERM_GREEN2}
_DTYPE = {torch.float64: L.HPHI_F64, torch.complex128: L.HPHI_C128, torch.float32: L.HPHI_F32,
          torch.complex64: L.HPHI_C64}
DTYPE_NAMES = {"f64": torch.float64, "c128": torch.complex128, "f32": torch.float32, "c64": torch.complex64}


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _dtype_code(t: torch.Tensor) -> int:
    try:
        return _DTYPE[t.dtype]
    except KeyError:
        raise ValueError(f"unsupported dtype {t.dtype}") from None


def version() -> str:
    return L.lib().hphi_version().decode()


# ------------------------------------------------------------------ basis

class Basis:
    """Owning handle of an hphi_basis."""

    def __init__(self, handle: int, desc):
        self.handle = handle
        self.desc = desc
        d = C.c_int64()
        check(L.lib().hphi_basis_dim(C.c_void_p(handle), C.byref(d)))
        self.dim = int(d.value)

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                L.lib().hphi_basis_free(C.c_void_p(self.handle))
            except Exception:      # interpreter shutdown: the process frees everything
                pass
            self.handle = None


def desc_to_c(desc) -> L.BasisDescC:
    return L.BasisDescC(_PARTICLE[desc.particle], desc.n_sites, _SECTOR[desc.sector], desc.two_sz,
                        desc.n_up, desc.n_dn, desc.n_tot, desc.split_bits)


def hphi_basis_build(desc) -> Basis:
    out = C.c_void_p()
    cdesc = desc_to_c(desc)
    check(L.lib().hphi_basis_build(C.byref(cdesc), C.byref(out)))
    return Basis(out.value, desc)


def hphi_basis_rank(basis: Basis, cfg: torch.Tensor) -> torch.Tensor:
    """cfg: int64 device tensor of bit strings (bit patterns of uint64)."""
    idx = torch.empty(cfg.shape, dtype=torch.int64, device=cfg.device)
    check(L.lib().hphi_basis_rank(C.c_void_p(basis.handle), _ptr(cfg), _ptr(idx), cfg.numel(), _stream()))
    return idx


def hphi_basis_unrank(basis: Basis, idx: torch.Tensor) -> torch.Tensor:
    cfg = torch.empty(idx.shape, dtype=torch.int64, device=idx.device)
    check(L.lib().hphi_basis_unrank(C.c_void_p(basis.handle), _ptr(idx), _ptr(cfg), idx.numel(), _stream()))
    return cfg


# ------------------------------------------------------------ Hamiltonian

class Ham:
    """Owning handle of an hphi_ham (keeps its basis alive)."""

    def __init__(self, handle: int, basis: Basis, n_terms: int):
        self.handle = handle
        self.basis = basis
        self.n_terms = n_terms
        flag = C.c_int32()
        check(L.lib().hphi_ham_is_complex(C.c_void_p(handle), C.byref(flag)))
        self.is_complex = bool(flag.value)

    @property
    def dim(self) -> int:
        return self.basis.dim

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                L.lib().hphi_ham_free(C.c_void_p(self.handle))
            except Exception:      # interpreter shutdown: the process frees everything
                pass
            self.handle = None


def terms_to_c(terms: Iterable) -> "C.Array":
    terms = list(terms)
    arr = (L.TermC * max(1, len(terms)))()
    for n, t in enumerate(terms):
        c = list(t.c) + [0.0] * (9 - len(t.c))
        arr[n].kind = _KIND[t.kind] if isinstance(t.kind, str) else int(t.kind)
        arr[n].i = int(t.i)
        arr[n].j = int(t.j)
        arr[n].reserved = 0
        for k in range(9):
            arr[n].c[k] = float(c[k])
    return arr, len(terms)


def hphi_ham_build(basis: Basis, terms) -> Ham:
    arr, n = terms_to_c(terms)
    out = C.c_void_p()
    check(L.lib().hphi_ham_build(C.c_void_p(basis.handle), arr, n, C.byref(out)))
    return Ham(out.value, basis, n)


def hphi_ham_nonfinite(ham: Ham, clear: bool = False) -> int:
    """The sticky non-finite flag word of ham's reductions (HPHI_NONFINITE_* bits); synchronizes."""
    f = C.c_int32(0)
    check(L.lib().hphi_ham_nonfinite(C.c_void_p(ham.handle), C.byref(f), int(bool(clear)), _stream()))
    return int(f.value)


# ------------------------------------------------------------------ H . v

def _nvec(v: torch.Tensor, dim: int) -> int:
    if v.dim() == 1:
        nv = 1
    elif v.dim() == 2:
        nv = v.shape[1]
    else:
        raise ValueError("vector must be (dim,) or (dim, nvec)")
    if v.shape[0] != dim:
        raise ValueError(f"vector has {v.shape[0]} rows, basis dimension is {dim}")
    return nv


def hphi_hv(ham: Ham, v: torch.Tensor, u: Optional[torch.Tensor] = None, *, a: float = 1.0, b: float = 0.0,
            in_scale: Optional[torch.Tensor] = None, reduce: Optional[torch.Tensor] = None,
            write: bool = True) -> Optional[torch.Tensor]:
    """u = a H (s v) + b (s v); optional reductions into `reduce` ([4*nvec] float64)."""
    nv = _nvec(v, ham.dim)
    if u is None and write:
        u = torch.empty_like(v)
    if u is not None and (u.shape != v.shape or u.dtype != v.dtype):
        raise ValueError("u must match v in shape and dtype")
    opts = L.HvOptsC(a, b, _ptr(in_scale), _ptr(reduce))
    check(L.lib().hphi_hv(C.c_void_p(ham.handle), _ptr(v), _ptr(u), nv, _dtype_code(v), C.byref(opts),
                          _stream()))
    return u


def hphi_hv_cma(ham: Ham, v: torch.Tensor, u: Optional[torch.Tensor] = None, *, cluster_bits: int = 6,
                a: float = 1.0, b: float = 0.0, in_scale: Optional[torch.Tensor] = None,
                reduce: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Dense-block variant of hphi_hv (clusters of cluster_bits sites, MFMA blocks); same options."""
    nv = _nvec(v, ham.dim)
    if u is None:
        u = torch.empty_like(v)
    if u.shape != v.shape or u.dtype != v.dtype:
        raise ValueError("u must match v in shape and dtype")
    opts = L.HvOptsC(a, b, _ptr(in_scale), _ptr(reduce))
    check(L.lib().hphi_hv_cma(C.c_void_p(ham.handle), _ptr(v), _ptr(u), nv, _dtype_code(v), int(cluster_bits),
                              C.byref(opts), _stream()))
    return u


def hphi_hv_cma_plan(ham: Ham, cluster_bits: int = 6) -> list:
    """The clusters (lists of sites) hphi_hv_cma uses for cluster_bits."""
    n = C.c_int32(0)
    check(L.lib().hphi_hv_cma_plan(C.c_void_p(ham.handle), int(cluster_bits), C.byref(n), None))
    sites = (C.c_int32 * (n.value * int(cluster_bits)))()
    check(L.lib().hphi_hv_cma_plan(C.c_void_p(ham.handle), int(cluster_bits), C.byref(n), sites))
    m = int(cluster_bits)
    return [list(sites[c * m:(c + 1) * m]) for c in range(n.value)]


def hphi_hv_tune(ham: Ham, v: torch.Tensor, u: Optional[torch.Tensor] = None) -> dict:
    """Autotune the product schedule for v's nvec and dtype; returns the chosen schedule."""
    nv = _nvec(v, ham.dim)
    if u is None:
        u = torch.empty_like(v)
    out = (C.c_int32 * 9)()
    check(L.lib().hphi_hv_tune(C.c_void_p(ham.handle), _ptr(v), _ptr(u), nv, _dtype_code(v), out, _stream()))
    keys = ("windowed", "window_kb", "max_passes", "lanes_per_row", "blocks_per_cu", "stage_tables", "nt_streams",
            "sector_blocks", "us")
    return dict(zip(keys, list(out)))


def hphi_hv_elements(ham: Ham, row0: int, nrows: int, cap: int, *, nvec: int = 1,
                     dtype: torch.dtype = torch.complex128):
    """Element lists of rows row0.. through the product kernels that hphi_hv runs for nvec vectors
    of `dtype` (complex128 or complex64): (cols, re, im, term, counts)."""
    dev = torch.device("cuda")
    cols = torch.empty(nrows * cap, dtype=torch.int64, device=dev)
    re = torch.empty(nrows * cap, dtype=torch.float64, device=dev)
    im = torch.empty(nrows * cap, dtype=torch.float64, device=dev)
    term = torch.empty(nrows * cap, dtype=torch.int32, device=dev)
    counts = torch.empty(nrows, dtype=torch.int32, device=dev)
    check(L.lib().hphi_hv_elements(C.c_void_p(ham.handle), row0, nrows, cap, int(nvec), _DTYPE[dtype], _ptr(cols),
                                   _ptr(re), _ptr(im), _ptr(term), _ptr(counts), _stream()))
    return (cols.view(nrows, cap), re.view(nrows, cap), im.view(nrows, cap), term.view(nrows, cap), counts)


# ---------------------------------------------------------------- Lanczos

def hphi_lanczos(hams: Sequence[Ham], v0: Sequence[torch.Tensor], n_iter: int, *, refine: bool = True,
                 use_graph: bool = True, breakdown_tol: float = 0.0, work=None, x_out=None):
    """Run hphi_lanczos over one or more problems; returns a list of result dicts."""
    hams = list(hams)
    v0 = list(v0)
    nh = len(hams)
    dtype = v0[0].dtype
    for h, v in zip(hams, v0):
        if v.dtype != dtype or _nvec(v, h.dim) != 1:
            raise ValueError("start vectors must share the storage dtype and be 1-D")
    if work is None:
        work = [torch.empty(2 * h.dim, dtype=dtype, device=v.device) for h, v in zip(hams, v0)]
    xdt = torch.complex128 if dtype.is_complex else torch.float64
    if refine and x_out is None:
        x_out = [torch.empty(h.dim, dtype=xdt, device=v.device) for h, v in zip(hams, v0)]
    alphas = [np.zeros(n_iter) for _ in range(nh)]
    betas = [np.zeros(n_iter) for _ in range(nh)]
    res = (L.LanczosResultC * nh)()
    for k in range(nh):
        res[k].alpha = alphas[k].ctypes.data_as(C.POINTER(C.c_double))
        res[k].beta = betas[k].ctypes.data_as(C.POINTER(C.c_double))
    opts = L.LanczosOptsC(n_iter, _DTYPE[dtype], int(refine), int(use_graph), breakdown_tol)
    H = (C.c_void_p * nh)(*[h.handle for h in hams])
    V = (C.c_void_p * nh)(*[_ptr(v) for v in v0])
    W = (C.c_void_p * nh)(*[_ptr(w) for w in work])
    X = (C.c_void_p * nh)(*[_ptr(x) for x in x_out]) if refine else None
    check(L.lib().hphi_lanczos(H, nh, C.byref(opts), V, W, X, res, _stream()))
    out = []
    for k in range(nh):
        n = res[k].n_done
        out.append(dict(alpha=alphas[k][:n].copy(), beta=betas[k][:n].copy(), n_done=n, info=res[k].info,
                        e0_ritz=res[k].e0_ritz, e0_refined=res[k].e0_refined, variance=res[k].variance,
                        residual=res[k].residual, x=(x_out[k] if refine else None)))
    return out


def hphi_cg_refine(ham: Ham, x: torch.Tensor, e_approx: float, *, shift: float = 1e-6, n_inverse: int = 2,
                   cg_max_iter: int = 1000, cg_tol: float = 1e-12, work=None) -> dict:
    """Inverse-iteration refinement of the FP64 eigenvector x in place (CG solves); returns E, variance,
    residual, CG iterations and info."""
    if x.dtype not in (torch.float64, torch.complex128) or _nvec(x, ham.dim) != 1:
        raise ValueError("x must be a 1-D float64 or complex128 vector")
    if work is None:
        work = torch.empty(3 * ham.dim, dtype=x.dtype, device=x.device)
    opts = L.CgOptsC(shift, n_inverse, cg_max_iter, cg_tol)
    res = L.CgResultC()
    check(L.lib().hphi_cg_refine(C.c_void_p(ham.handle), _ptr(x), _dtype_code(x), float(e_approx), C.byref(opts),
                                 _ptr(work), C.byref(res), _stream()), allow=(L.HPHI_OK,))
    return dict(e_refined=res.e_refined, variance=res.variance, residual=res.residual, cg_iters=res.cg_iters,
                info=res.info)


# ------------------------------------------------------------ observables

def hphi_expect(obs: Ham, psi: torch.Tensor) -> torch.Tensor:
    """<O> per state (FP64 device tensor [nvec]) for the observable `obs` (an Ham built from its terms)."""
    nv = _nvec(psi, obs.dim)
    out = torch.empty(2 * nv, dtype=torch.float64, device=psi.device)
    check(L.lib().hphi_expect(C.c_void_p(obs.handle), _ptr(psi), nv, _dtype_code(psi), _ptr(out), _stream()))
    return out[:nv]


# -------------------------------------------------------------------- TPQ

def hphi_tpq_step(ham: Ham, psi_in: torch.Tensor, psi_out: torch.Tensor, l: float, k: int,
                  in_scale: Optional[torch.Tensor], obs: torch.Tensor) -> None:
    nv = _nvec(psi_in, ham.dim)
    if psi_out.shape != psi_in.shape or psi_out.dtype != psi_in.dtype:
        raise ValueError("psi_out must match psi_in")
    if obs.dtype != torch.float64 or obs.numel() < 4 * nv:
        raise ValueError("obs must be float64 with 4*nvec entries")
    check(L.lib().hphi_tpq_step(C.c_void_p(ham.handle), _ptr(psi_in), _ptr(psi_out), nv, _dtype_code(psi_in),
                                float(l), int(k), _ptr(in_scale), _ptr(obs), _stream()))


def hphi_tpq_run(ham: Ham, psi_a: torch.Tensor, psi_b: torch.Tensor, l: float, k0: int, n_steps: int,
                 in_scale: Optional[torch.Tensor] = None, obs_log: Optional[torch.Tensor] = None,
                 use_graph: bool = True) -> torch.Tensor:
    """n_steps TPQ steps alternating between psi_a and psi_b; returns the observable log
    (float64 device tensor [n_steps, 4, nvec]).  The final state is in psi_a if n_steps is even."""
    nv = _nvec(psi_a, ham.dim)
    if psi_b.shape != psi_a.shape or psi_b.dtype != psi_a.dtype:
        raise ValueError("psi_b must match psi_a")
    if obs_log is None:
        obs_log = torch.empty((max(n_steps, 1), 4, nv), dtype=torch.float64, device=psi_a.device)
    if obs_log.dtype != torch.float64 or obs_log.numel() < 4 * nv * n_steps or not obs_log.is_contiguous():
        raise ValueError("obs_log must be contiguous float64 with n_steps*4*nvec entries")
    check(L.lib().hphi_tpq_run(C.c_void_p(ham.handle), _ptr(psi_a), _ptr(psi_b), nv, _dtype_code(psi_a), float(l),
                               int(k0), int(n_steps), _ptr(in_scale), _ptr(obs_log), int(bool(use_graph)),
                               _stream()))
    return obs_log


def hphi_tpq_run_noalloc(ham: Ham, psi_a: torch.Tensor, psi_b: torch.Tensor, l: float, k0: int, n_steps: int,
                         obs_log: torch.Tensor, in_scale: Optional[torch.Tensor] = None) -> torch.Tensor:
    """hphi_tpq_run without any device allocation (static device state; no graph, no synchronization):
    obs_log must be a preallocated contiguous float64 device tensor of n_steps*4*nvec entries."""
    nv = _nvec(psi_a, ham.dim)
    if psi_b.shape != psi_a.shape or psi_b.dtype != psi_a.dtype:
        raise ValueError("psi_b must match psi_a")
    if obs_log.dtype != torch.float64 or obs_log.numel() < 4 * nv * n_steps or not obs_log.is_contiguous():
        raise ValueError("obs_log must be contiguous float64 with n_steps*4*nvec entries")
    check(L.lib().hphi_tpq_run_noalloc(C.c_void_p(ham.handle), _ptr(psi_a), _ptr(psi_b), nv, _dtype_code(psi_a),
                                       float(l), int(k0), int(n_steps), _ptr(in_scale), _ptr(obs_log), _stream()))
    return obs_log
