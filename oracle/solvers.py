"""Oracle solvers: dense diagonalization, Lanczos, microcanonical TPQ.

All FP64.  Each routine takes the product as a callable apply(v) -> H v,
so it can sit on the sparse oracle matrix or on oracle.hamiltonian.apply_h.

Lanczos (Sec. 3.4, Lanczos recurrence; Appendix A.3):
    v_0 = x_0/|x_0|, beta_0 = 0, v_{-1} = 0
    alpha_k = (H v_k, v_k)
    w = H v_k - beta_k v_{k-1} - alpha_k v_k
    beta_{k+1} = |w|,  v_{k+1} = w / beta_{k+1}
with no reorthogonalization (two-vector scheme).  n steps give the
tridiagonal T_n with diagonal alpha_0..alpha_{n-1} and off-diagonal
beta_1..beta_{n-1}.  Reading of the unstated breakdown rule: the
recurrence stops at step k (T keeps size k+1) when k+1 equals the
dimension or beta_{k+1} <= tol * max(|alpha_k|, beta_k, 1).
The eigenvector is rebuilt by repeating the same recurrence and
accumulating x = sum_k e~_k v_k; the check quantities are
E = <x|H|x>/<x|x>, variance <H^2> - <H>^2 and residual |Hx - Ex|/|x|.

TPQ (Sec. 3.5, microcanonical TPQ state):
    psi_k = (l - H/N_s) psi_{k-1} / |(l - H/N_s) psi_{k-1}|
    u_k = <psi_k|H|psi_k>/N_s,  beta_k = (2k/N_s)/(l - u_k)
psi_0 is the normalized random start (k = 0).  Each step applies H to
psi_{k-1}, which yields u_{k-1} and <H^2>_{k-1} of the state before the
step, then forms psi_k.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def dense_spectrum(hmat: np.ndarray):
    """All eigenvalues/eigenvectors of a dense Hermitian matrix (LAPACK heevd)."""
    return np.linalg.eigh(hmat)


def lanczos(apply, x0: np.ndarray, n_iter: int, dim: int, tol: float = 1e-13):
    """Plain FP64 Lanczos.  Returns (alpha, beta) with beta[k] = beta_{k+1}."""
    v = x0.astype(np.complex128) / np.linalg.norm(x0)
    v_prev = np.zeros_like(v)
    beta_k = 0.0
    alpha, beta = [], []
    n = min(n_iter, dim)
    for k in range(n):
        h = apply(v)
        a = float(np.vdot(v, h).real)
        w = h - beta_k * v_prev - a * v
        b = float(np.linalg.norm(w))
        alpha.append(a)
        beta.append(b)
        if k + 1 >= n:
            break
        if b <= tol * max(abs(a), beta_k, 1.0):
            break
        v_prev, v = v, w / b
        beta_k = b
    return np.array(alpha), np.array(beta)


def tridiag_lowest(alpha: np.ndarray, beta: np.ndarray):
    """Lowest eigenpair of T_n (diagonal alpha, off-diagonal beta[:n-1])."""
    n = len(alpha)
    if n == 1:
        return float(alpha[0]), np.ones(1)
    w, vec = sla.eigh_tridiagonal(alpha, beta[: n - 1], select="i", select_range=(0, 0))
    return float(w[0]), vec[:, 0]


def tridiag_eigvals(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    n = len(alpha)
    if n == 1:
        return np.array(alpha, dtype=float)
    return sla.eigh_tridiagonal(alpha, beta[: n - 1], eigvals_only=True)


def lanczos_eigenvector(apply, x0: np.ndarray, alpha, beta, coeffs):
    """Second pass: regenerate v_k with the same recurrence, accumulate x = sum c_k v_k."""
    n = len(alpha)
    v = x0.astype(np.complex128) / np.linalg.norm(x0)
    v_prev = np.zeros_like(v)
    x = coeffs[0] * v
    beta_k = 0.0
    for k in range(n - 1):
        h = apply(v)
        w = h - beta_k * v_prev - alpha[k] * v
        v_prev, v = v, w / beta[k]
        beta_k = beta[k]
        x = x + coeffs[k + 1] * v
    return x


def rayleigh_check(apply, x: np.ndarray):
    """E = <x|Hx>/<x|x>, variance <H^2> - <H>^2 and residual |Hx - E x| / |x|."""
    hx = apply(x)
    xx = float(np.vdot(x, x).real)
    e = float(np.vdot(x, hx).real) / xx
    h2 = float(np.vdot(hx, hx).real) / xx
    res = float(np.linalg.norm(hx - e * x)) / np.sqrt(xx)
    return e, h2 - e * e, res


def lanczos_ground_state(apply, x0, n_iter, dim, tol=1e-13, refine=True):
    alpha, beta = lanczos(apply, x0, n_iter, dim, tol)
    e0, vec = tridiag_lowest(alpha, beta)
    out = {"alpha": alpha, "beta": beta, "e0_ritz": e0, "n": len(alpha)}
    if refine:
        x = lanczos_eigenvector(apply, x0, alpha, beta, vec)
        e, var, res = rayleigh_check(apply, x)
        out.update(e0_refined=e, variance=var, residual=res, x=x)
    return out


def tpq(apply, psi0: np.ndarray, n_sites: int, l: float, n_steps: int):
    """Literal mTPQ.  Returns u[k], h2[k] (= <H^2>/N_s^2) for k = 0..n_steps-1 and psi_{n_steps}."""
    psi = psi0.astype(np.complex128) / np.linalg.norm(psi0)
    u, h2 = [], []
    for _ in range(n_steps):
        h = apply(psi)
        u.append(float(np.vdot(psi, h).real) / n_sites)
        h2.append(float(np.vdot(h, h).real) / n_sites ** 2)
        phi = l * psi - h / n_sites
        psi = phi / np.linalg.norm(phi)
    return np.array(u), np.array(h2), psi


def tpq_beta(u: np.ndarray, n_sites: int, l: float) -> np.ndarray:
    k = np.arange(len(u))
    return (2.0 * k / n_sites) / (l - u)


def tpq_spectral(evals: np.ndarray, evecs: np.ndarray, psi0: np.ndarray, n_sites: int,
                 l: float, n_steps: int):
    """Closed form: psi_k ∝ sum_n (l - E_n/N_s)^k <n|psi_0> |n>.

    u_k = sum_n w_n E_n / (N_s sum_n w_n) with w_n = (l - E_n/N_s)^{2k} |<n|psi_0>|^2,
    evaluated in log space to avoid overflow.
    """
    c2 = np.abs(evecs.conj().T @ psi0) ** 2
    f = np.abs(l - evals / n_sites)
    logf = np.log(f)
    u, h2 = [], []
    for k in range(n_steps):
        lw = 2 * k * logf + np.log(np.maximum(c2, 1e-300))
        w = np.exp(lw - lw.max())
        u.append(float((w * evals).sum() / w.sum()) / n_sites)
        h2.append(float((w * evals ** 2).sum() / w.sum()) / n_sites ** 2)
    return np.array(u), np.array(h2)


def lowest_eigenvalue(hmat, tol: float = 1e-14) -> float:
    """Lowest eigenvalue of a sparse Hermitian matrix: ARPACK's implicitly restarted Lanczos
    (scipy.sparse.linalg.eigsh, smallest algebraic) used as one library step; dense eigh for
    matrices of dimension <= 64, where ARPACK needs more vectors than the dimension."""
    import scipy.sparse.linalg as spla
    n = hmat.shape[0]
    if n <= 64:
        return float(np.linalg.eigvalsh(hmat.toarray() if hasattr(hmat, "toarray") else hmat)[0])
    w = spla.eigsh(hmat, k=1, which="SA", tol=tol, return_eigenvectors=False, ncv=min(n - 1, 40),
                   v0=np.ones(n, dtype=hmat.dtype) / np.sqrt(n))
    return float(w[0])
