"""Oracle Hamiltonian: literal operator action on basis states.

Operators (all FP64 / complex128):

* Spin-1/2 (Appendix A.1 with S = 1/2; bit 1 = up, bit 0 = down):
  S^z = diag(-1/2, +1/2); S^+|down> = |up>, S^-|up> = |down>;
  S^x = (S^+ + S^-)/2 and S^y = (S^+ - S^-)/(2i).
  A bilinear coupling J^{ab} S_i^a S_j^b is applied as S_j^b first and
  S_i^a second, one (a, b) component at a time (Sec. 2.3, spin model).
* Fermions (Sec. 2.3 Hubbard model, Sec. 3.3 sign from bit parity):
  orbital k = 2*site + sigma, Jordan-Wigner order ascending in k:
      c_k |n>  = (-1)^{sum_{q<k} n_q} n_k     |n - e_k>
      c+_k |n> = (-1)^{sum_{q<k} n_q} (1-n_k) |n + e_k>
  and every product of operators is applied one operator at a time,
  right to left (no precomputed between-mask).

H.v is built column by column ("push"): each term is applied to every
basis state |t>, producing <s|T|t> for the states s it reaches, and
u[s] += <s|T|t> v[t].  Terms are read as given: a HOP term means
t c+_a c_b + conj(t) c+_b c_a, a SPIN_BOND term one undirected bond, a
GREEN2 term the two-body Green's-function observable of Sec. 2.2 (output
of the eigenvectors and TPQ states), t c+_a c_b c+_c c_d + its conjugate.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from synth.lattices import SPIN_BOND, SPIN_FIELD, HOP, DENS, NUM, HUBBARD_U, GREEN2
from . import basis as ob

ONE = np.uint64(1)

# ------------------------------------------------------------ single operators


def spin_op(alpha: str, site: int, st: np.ndarray):
    """Apply S^alpha on one site to each state: returns (coef, new_states)."""
    m = ONE << np.uint64(site)
    up = (st & m) != 0
    if alpha == "z":
        return np.where(up, 0.5, -0.5).astype(np.complex128), st.copy()
    flipped = st ^ m
    if alpha == "+":      # |down> -> |up>
        return np.where(up, 0.0, 1.0).astype(np.complex128), flipped
    if alpha == "-":      # |up> -> |down>
        return np.where(up, 1.0, 0.0).astype(np.complex128), flipped
    if alpha == "x":      # (S+ + S-)/2
        cp, _ = spin_op("+", site, st)
        cm, _ = spin_op("-", site, st)
        return (cp + cm) / 2.0, flipped
    if alpha == "y":      # (S+ - S-)/(2i)
        cp, _ = spin_op("+", site, st)
        cm, _ = spin_op("-", site, st)
        return (cp - cm) / 2j, flipped
    raise ValueError(alpha)


def _parity_below(k: int, st: np.ndarray) -> np.ndarray:
    """(-1)^{number of occupied orbitals q < k}."""
    below = (ONE << np.uint64(k)) - ONE
    return np.where(np.bitwise_count(st & below) % 2 == 0, 1.0, -1.0)


def annihilate(k: int, st: np.ndarray):
    m = ONE << np.uint64(k)
    occ = (st & m) != 0
    return (_parity_below(k, st) * occ).astype(np.complex128), st & ~m


def create(k: int, st: np.ndarray):
    m = ONE << np.uint64(k)
    occ = (st & m) != 0
    return (_parity_below(k, st) * (~occ)).astype(np.complex128), st | m


def apply_product(ops, st: np.ndarray):
    """Apply a product of single operators, given left to right as written."""
    coef = np.ones(st.shape, dtype=np.complex128)
    cur = st
    for fn in reversed(ops):
        c, cur = fn(cur)
        coef = coef * c
    return coef, cur


def term_branches(term, st: np.ndarray, particle: str):
    """All branches (coef, new_states) of one term applied to each state."""
    k = term.kind
    out = []
    if k == SPIN_BOND:
        if particle != "spin":
            raise ValueError("spin term on fermion basis")
        axes = "xyz"
        for a in range(3):
            for b in range(3):
                J = term.c[3 * a + b]
                if J == 0.0:
                    continue
                c, s2 = apply_product([lambda x, a=a: spin_op(axes[a], term.i, x),
                                       lambda x, b=b: spin_op(axes[b], term.j, x)], st)
                out.append((J * c, s2))
    elif k == SPIN_FIELD:
        if particle != "spin":
            raise ValueError("spin term on fermion basis")
        for a, ax in enumerate("xyz"):
            h = term.c[a]
            if h == 0.0:
                continue
            c, s2 = spin_op(ax, term.i, st)
            out.append((h * c, s2))
    elif k == HOP:
        if particle != "fermion":
            raise ValueError("fermion term on spin basis")
        t = complex(term.c[0], term.c[1])
        a, b = term.i, term.j
        c1, s1 = apply_product([lambda x: create(a, x), lambda x: annihilate(b, x)], st)
        out.append((t * c1, s1))
        c2, s2 = apply_product([lambda x: create(b, x), lambda x: annihilate(a, x)], st)
        out.append((np.conj(t) * c2, s2))
    elif k == GREEN2:
        # t c+_a c_b c+_c c_d + conj(t) c+_d c_c c+_b c_a, each applied one operator at a time
        if particle != "fermion":
            raise ValueError("fermion term on spin basis")
        t = complex(term.c[0], term.c[1])
        a, b, cc, d = term.i, term.j, int(term.c[2]), int(term.c[3])
        c1, s1 = apply_product([lambda x: create(a, x), lambda x: annihilate(b, x),
                                lambda x: create(cc, x), lambda x: annihilate(d, x)], st)
        out.append((t * c1, s1))
        c2, s2 = apply_product([lambda x: create(d, x), lambda x: annihilate(cc, x),
                                lambda x: create(b, x), lambda x: annihilate(a, x)], st)
        out.append((np.conj(t) * c2, s2))
    elif k in (DENS, NUM, HUBBARD_U):
        if particle != "fermion":
            raise ValueError("fermion term on spin basis")
        if k == DENS:
            orbs = (term.i, term.j)
        elif k == NUM:
            orbs = (term.i,)
        else:
            orbs = (2 * term.i, 2 * term.i + 1)
        ops = []
        for o in orbs:    # n_o = c+_o c_o, product over the listed orbitals
            ops += [lambda x, o=o: create(o, x), lambda x, o=o: annihilate(o, x)]
        c, s2 = apply_product(ops, st)
        out.append((term.c[0] * c, s2))
    else:
        raise ValueError(f"unknown term kind {k!r}")
    return out


def term_action(term, st: np.ndarray, particle: str):
    """T|s> for each state, branches merged by reached state.

    Branches of one term that reach the same configuration from the same
    source are summed (e.g. the S^x S^x and S^y S^y pieces of a pair flip
    cancel for an isotropic coupling), so a term is judged by its total
    element, not by its pieces.  Returns a list of (coef, new_states)
    with one entry per distinct flip pattern s XOR t.
    """
    acc = {}
    for coef, tgt in term_branches(term, st, particle):
        nz = coef != 0
        if not nz.any():
            continue
        d = tgt ^ st
        for dv in np.unique(d[nz]):
            sel = nz & (d == dv)
            if int(dv) not in acc:
                acc[int(dv)] = np.zeros(st.shape, np.complex128)
            acc[int(dv)][sel] += coef[sel]
    return [(c, st ^ np.uint64(dv)) for dv, c in sorted(acc.items())]


# ------------------------------------------------------------------- H as data


def coo_elements(desc, terms, basis_states=None):
    """All matrix elements as (row, col, term_id, value), pushed column-wise.

    Raises ValueError if any term maps a basis state outside the space.
    Exact-zero values are dropped.
    """
    if basis_states is None:
        basis_states = ob.states(desc)
    cols_all = np.arange(len(basis_states), dtype=np.int64)
    R, C, T, V = [], [], [], []
    for tid, term in enumerate(terms):
        for coef, tgt in term_action(term, basis_states, desc.particle):
            nz = coef != 0
            if not nz.any():
                continue
            rows = ob.rank(basis_states, tgt[nz])
            if (rows < 0).any():
                raise ValueError(f"term {tid} ({term.kind}) leaves the sector")
            R.append(rows)
            C.append(cols_all[nz])
            T.append(np.full(rows.shape, tid, dtype=np.int64))
            V.append(coef[nz])
    if not R:
        z = np.zeros(0, np.int64)
        return z, z, z, np.zeros(0, np.complex128)
    return np.concatenate(R), np.concatenate(C), np.concatenate(T), np.concatenate(V)


def sparse_h(desc, terms, basis_states=None) -> sp.csr_matrix:
    if basis_states is None:
        basis_states = ob.states(desc)
    n = len(basis_states)
    r, c, _, v = coo_elements(desc, terms, basis_states)
    return sp.csr_matrix((v, (r, c)), shape=(n, n))


def dense_h(desc, terms, basis_states=None) -> np.ndarray:
    return sparse_h(desc, terms, basis_states).toarray()


def apply_h(desc, terms, v: np.ndarray, basis_states=None) -> np.ndarray:
    """u = H v, pushed column by column, for v of shape (dim,) or (dim, nvec)."""
    if basis_states is None:
        basis_states = ob.states(desc)
    n = len(basis_states)
    v2 = v.reshape(n, -1).astype(np.complex128)
    u = np.zeros_like(v2)
    for tid, term in enumerate(terms):
        for coef, tgt in term_action(term, basis_states, desc.particle):
            nz = np.nonzero(coef != 0)[0]
            if nz.size == 0:
                continue
            rows = ob.rank(basis_states, tgt[nz])
            if (rows < 0).any():
                raise ValueError(f"term {tid} ({term.kind}) leaves the sector")
            for b in range(v2.shape[1]):
                w = coef[nz] * v2[nz, b]
                u[:, b] += (np.bincount(rows, weights=w.real, minlength=n)
                            + 1j * np.bincount(rows, weights=w.imag, minlength=n))
    return u.reshape(v.shape)


def row_elements(desc, terms, rows: np.ndarray, basis_states=None):
    """Elements of the given rows as a dict row -> {(col, term_id): value}.

    Column-wise push restricted to the requested rows; diagonal entries of
    all terms are summed into key (row, -1).
    """
    r, c, t, v = coo_elements(desc, terms, basis_states)
    want = set(int(x) for x in rows)
    out = {int(x): {} for x in rows}
    for rr, cc, tt, vv in zip(r, c, t, v):
        rr = int(rr)
        if rr not in want:
            continue
        key = (int(cc), -1) if cc == rr else (int(cc), int(tt))
        out[rr][key] = out[rr].get(key, 0.0) + vv
    for rr in out:
        out[rr] = {k: val for k, val in out[rr].items() if val != 0}
    return out


def rows_hv_sampled(desc, terms, row_states: np.ndarray, v_of_state):
    """u[s] for selected rows, without a full basis list.

    Uses Hermiticity: u[s] = sum_t conj(<t|H|s>) v[t]; each term is applied
    to |s> and the conjugated coefficient multiplies v at the reached
    state.  v_of_state maps an array of configurations to the vector
    values (shape (n,) or (n, nvec)); states outside the space must not
    be reached (the caller's sector check).
    """
    st = np.asarray(row_states, dtype=np.uint64)
    acc = None
    for term in terms:
        for coef, tgt in term_action(term, st, desc.particle):
            nz = np.nonzero(coef != 0)[0]
            vals = v_of_state(tgt[nz])
            if acc is None:
                acc = np.zeros((len(st),) + vals.shape[1:], dtype=np.complex128)
            cc = np.conj(coef[nz])
            acc[nz] += cc[:, None] * vals if vals.ndim == 2 else cc * vals
    return acc


def sector_preserving(desc, terms) -> bool:
    """True if every term keeps each basis state inside the space (brute force)."""
    try:
        coo_elements(desc, terms)
    except ValueError:
        return False
    return True


def row_elements_sampled(desc, terms, row_states: np.ndarray, rank_fn):
    """Elements of selected rows without a full basis list.

    By Hermiticity of each term, <s|T|t> = conj(<t|T|s>): each term is
    applied to |s> and the reached states t give the elements of row s.
    rank_fn maps configurations to indices.  Returns a list (one dict per
    row) of {(col, term_id): value}, diagonal parts summed under term -1.
    """
    st = np.asarray(row_states, dtype=np.uint64)
    own = rank_fn(st)
    out = [dict() for _ in range(len(st))]
    for tid, term in enumerate(terms):
        for coef, tgt in term_action(term, st, desc.particle):
            nz = np.nonzero(coef != 0)[0]
            if nz.size == 0:
                continue
            cols = rank_fn(tgt[nz])
            for k, c, val in zip(nz, cols, np.conj(coef[nz])):
                key = (int(c), -1) if int(c) == int(own[k]) else (int(c), tid)
                out[k][key] = out[k].get(key, 0.0) + val
    return [{k: v for k, v in d.items() if v != 0} for d in out]
