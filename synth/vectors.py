"""Seeded random input vectors (host numpy, PCG64 via default_rng).

Batched vectors use the interleaved layout v[idx * nvec + b]; as a numpy
array that is shape (dim, nvec) in C order.  Values are raw draws: any
normalization is left to the consumer.
"""

from __future__ import annotations

import numpy as np


def gaussian_vectors(dim: int, seeds, complex_: bool, dtype=None) -> np.ndarray:
    """One column per seed, entries i.i.d. N(0,1) (real and imaginary parts independent)."""
    seeds = list(seeds)
    cdt = np.complex128 if complex_ else np.float64
    out = np.empty((dim, len(seeds)), dtype=cdt)
    for b, s in enumerate(seeds):
        rng = np.random.default_rng(s)
        if complex_:
            out[:, b].real = rng.standard_normal(dim)
            out[:, b].imag = rng.standard_normal(dim)
        else:
            out[:, b] = rng.standard_normal(dim)
    if dtype is not None:
        out = out.astype(dtype)
    return out


def uniform_vectors(dim: int, seeds, complex_: bool, dtype=None) -> np.ndarray:
    """One column per seed, entries uniform in [-1, 1) (real and imaginary parts independent)."""
    seeds = list(seeds)
    cdt = np.complex128 if complex_ else np.float64
    out = np.empty((dim, len(seeds)), dtype=cdt)
    for b, s in enumerate(seeds):
        rng = np.random.default_rng(s)
        if complex_:
            out[:, b].real = rng.uniform(-1.0, 1.0, dim)
            out[:, b].imag = rng.uniform(-1.0, 1.0, dim)
        else:
            out[:, b] = rng.uniform(-1.0, 1.0, dim)
    if dtype is not None:
        out = out.astype(dtype)
    return out


def device_uniform(dim: int, nvec: int, seed: int, complex_: bool, dtype, device="cuda"):
    """Seeded uniform [-1, 1) vectors drawn with torch's generator on the device.

    Shape (dim, nvec) (or (dim,) for nvec = 0), values rounded to `dtype`;
    used for full-size inputs where a host draw would dominate set-up time.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    shape = (dim, max(nvec, 1))
    real_dt = torch.float32 if dtype in (torch.float32, torch.complex64) else torch.float64
    # drawn in place: one allocation of the output size (full-size vectors
    # reach tens of GB)
    if complex_:
        x = torch.empty(shape + (2,), device=device, dtype=real_dt).uniform_(-1.0, 1.0, generator=g)
        out = torch.view_as_complex(x).to(dtype)
    else:
        out = torch.empty(shape, device=device, dtype=real_dt).uniform_(-1.0, 1.0, generator=g).to(dtype)
    return out.reshape(dim) if nvec == 0 else out.contiguous()
