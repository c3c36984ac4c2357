"""Lattice bond lists and coupling terms (inputs only).

Term kinds follow the model families of the paper (Sec. 2.3, "Models"):
the generalized spin Hamiltonian (fields and bilinear couplings
J_ij^{ab} S_i^a S_j^b) and the Hubbard family (transfer t, on-site U,
inter-site V, chemical potential).  A term is a plain record; what it
means as an operator is decided separately by each consumer.

Site numbering is part of the input.  Every generator documents its
numbering rule; results are only comparable for the same numbering.

Fermion orbitals are numbered 2*site + sigma (sigma = 0 for up, 1 for
down), the interleaved bit layout of Sec. 3.1.
"""

from __future__ import annotations

from typing import NamedTuple, Tuple, List

import numpy as np

SPIN_BOND = "spin_bond"      # i, j sites; c = J[a][b] row-major, a,b in (x,y,z): sum_ab J^ab S_i^a S_j^b
SPIN_FIELD = "spin_field"    # i site; c = (hx, hy, hz): sum_a h^a S_i^a
HOP = "hop"                  # i=a, j=b orbitals; c = (Re t, Im t): t c+_a c_b + conj(t) c+_b c_a
DENS = "dens"                # i=a, j=b orbitals; c = (V,): V n_a n_b
NUM = "num"                  # i=a orbital; c = (mu,): mu n_a
HUBBARD_U = "hubbard_u"      # i site; c = (U,): U n_{i,up} n_{i,down}
GREEN2 = "green2"            # i=a, j=b orbitals; c = (Re t, Im t, c, d): t c+_a c_b c+_c c_d + h.c.

KINDS = (SPIN_BOND, SPIN_FIELD, HOP, DENS, NUM, HUBBARD_U, GREEN2)


class Term(NamedTuple):
    kind: str
    i: int
    j: int
    c: Tuple[float, ...]


# ---------------------------------------------------------------- spin terms

def heisenberg_bond(i: int, j: int, J: float = 1.0) -> Term:
    """J S_i . S_j  (isotropic exchange, one entry per undirected bond)."""
    c = (J, 0.0, 0.0,
         0.0, J, 0.0,
         0.0, 0.0, J)
    return Term(SPIN_BOND, i, j, c)


def kitaev_heisenberg_bond(i: int, j: int, gamma: int, K: float, J: float) -> Term:
    """J S_i . S_j + K S_i^gamma S_j^gamma on a gamma-link (gamma = 0,1,2 for x,y,z)."""
    m = [[J if a == b else 0.0 for b in range(3)] for a in range(3)]
    m[gamma][gamma] += K
    return Term(SPIN_BOND, i, j, tuple(m[a][b] for a in range(3) for b in range(3)))


def xxz_bond(i: int, j: int, Jxy: float, Jz: float) -> Term:
    c = (Jxy, 0.0, 0.0,
         0.0, Jxy, 0.0,
         0.0, 0.0, Jz)
    return Term(SPIN_BOND, i, j, c)


# ------------------------------------------------------------ bond geometry

def chain_bonds(n: int, periodic: bool = True) -> List[Tuple[int, int]]:
    """Chain: bonds (i, i+1); with PBC also (n-1, 0)."""
    bonds = [(i, i + 1) for i in range(n - 1)]
    if periodic and n > 2:
        bonds.append((n - 1, 0))
    return bonds


def rect_bonds(lx: int, ly: int, periodic: bool = False) -> List[Tuple[int, int]]:
    """Square lattice lx x ly; site i = x + lx*y; bonds to (x+1,y) and (x,y+1)."""
    bonds = []
    for y in range(ly):
        for x in range(lx):
            i = x + lx * y
            if x + 1 < lx:
                bonds.append((i, i + 1))
            elif periodic and lx > 2:
                bonds.append((i, y * lx))
            if y + 1 < ly:
                bonds.append((i, i + lx))
            elif periodic and ly > 2:
                bonds.append((i, x))
    return bonds


def honeycomb_links(lx: int = 3, ly: int = 4) -> List[Tuple[int, int, int]]:
    """Periodic honeycomb: cell c = x + lx*y, A = 2c, B = 2c+1.

    Links (site_a, site_b, label) with label 2 (z) for A(x,y)-B(x,y),
    0 (x) for A(x,y)-B(x-1,y) and 1 (y) for A(x,y)-B(x,y-1), all modulo
    the torus.  3*lx*ly links.
    """
    links = []
    for y in range(ly):
        for x in range(lx):
            a = 2 * (x + lx * y)
            links.append((a, 2 * (x + lx * y) + 1, 2))
            links.append((a, 2 * (((x - 1) % lx) + lx * y) + 1, 0))
            links.append((a, 2 * (x + lx * ((y - 1) % ly)) + 1, 1))
    return links


def triangular_bonds(lx: int = 6, ly: int = 4) -> List[Tuple[int, int]]:
    """Triangular torus: i = x + lx*y; bonds to (x+1,y), (x,y+1), (x-1,y+1)."""
    bonds = []
    for y in range(ly):
        for x in range(lx):
            i = x + lx * y
            bonds.append((i, ((x + 1) % lx) + lx * y))
            bonds.append((i, x + lx * ((y + 1) % ly)))
            bonds.append((i, ((x - 1) % lx) + lx * ((y + 1) % ly)))
    return bonds


def kagome_bonds(lx: int = 3, ly: int = 4) -> List[Tuple[int, int]]:
    """Kagome torus: cell c = x + lx*y, A = 3c, B = 3c+1, C = 3c+2.

    Up triangles A-B, A-C, B-C in each cell; down triangles
    A(x,y)-B(x-1,y), A(x,y)-C(x,y-1), B(x,y)-C(x+1,y-1), modulo the torus.
    """
    def s(x, y, k):
        return 3 * ((x % lx) + lx * (y % ly)) + k

    bonds = []
    for y in range(ly):
        for x in range(lx):
            a, b, c = s(x, y, 0), s(x, y, 1), s(x, y, 2)
            bonds += [(a, b), (a, c), (b, c)]
            bonds.append((a, s(x - 1, y, 1)))
            bonds.append((a, s(x, y - 1, 2)))
            bonds.append((b, s(x + 1, y - 1, 2)))
    return bonds


# --------------------------------------------------------- random term lists

def random_spin_terms(n_sites: int, n_bonds: int, seed: int, *, conserve_sz: bool,
                      fields: bool = False, real: bool = True) -> List[Term]:
    """Random bilinear spin couplings on random site pairs.

    conserve_sz restricts J^ab to the U(1)-symmetric form (Jxx = Jyy,
    Jxy = -Jyx, no xz/yz couplings); otherwise all nine entries are drawn.
    real=True keeps every matrix element real (no J^xy / J^yx and no h^y).
    """
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(n_bonds):
        i, j = rng.choice(n_sites, size=2, replace=False)
        if conserve_sz:
            jxy = rng.uniform(-1, 1)
            jz = rng.uniform(-1, 1)
            dm = 0.0 if real else rng.uniform(-1, 1)
            m = [[jxy, dm, 0.0], [-dm, jxy, 0.0], [0.0, 0.0, jz]]
        else:
            m = rng.uniform(-1, 1, size=(3, 3)).tolist()
            if real:
                m[0][1] = m[1][0] = 0.0
                m[1][2] = m[2][1] = 0.0
        terms.append(Term(SPIN_BOND, int(i), int(j),
                          tuple(float(m[a][b]) for a in range(3) for b in range(3))))
    if fields:
        for i in range(n_sites):
            hx, hy, hz = rng.uniform(-1, 1, size=3)
            if conserve_sz:
                hx = hy = 0.0
            if real:
                hy = 0.0
            terms.append(Term(SPIN_FIELD, i, -1, (float(hx), float(hy), float(hz))))
    return terms


def random_fermion_terms(n_sites: int, n_hops: int, seed: int, *, conserve_spin: bool,
                         real: bool = True, n_dens: int = 0, with_u: bool = True,
                         with_mu: bool = False) -> List[Term]:
    """Random hoppings between random orbitals (plus optional U, V, mu)."""
    rng = np.random.default_rng(seed)
    terms = []
    norb = 2 * n_sites
    for _ in range(n_hops):
        if conserve_spin:
            sigma = int(rng.integers(0, 2))
            si, sj = rng.choice(n_sites, size=2, replace=False)
            a, b = 2 * int(si) + sigma, 2 * int(sj) + sigma
        else:
            a, b = (int(x) for x in rng.choice(norb, size=2, replace=False))
        tre = float(rng.uniform(-1, 1))
        tim = 0.0 if real else float(rng.uniform(-1, 1))
        terms.append(Term(HOP, a, b, (tre, tim)))
    for _ in range(n_dens):
        a, b = (int(x) for x in rng.choice(norb, size=2, replace=False))
        terms.append(Term(DENS, a, b, (float(rng.uniform(-1, 1)),)))
    if with_u:
        for i in range(n_sites):
            terms.append(Term(HUBBARD_U, i, -1, (float(rng.uniform(0, 4)),)))
    if with_mu:
        for a in range(norb):
            terms.append(Term(NUM, a, -1, (float(rng.uniform(-1, 1)),)))
    return terms


def green2_term(a: int, b: int, c: int, d: int, t: complex = 1.0) -> Term:
    """The two-body Green's-function observable t c+_a c_b c+_c c_d + h.c. (orbitals 2*site+sigma):
    its expectation is 2 Re(t <c+_a c_b c+_c c_d>), so t = 1 and t = i give Re and -Im."""
    t = complex(t)
    return Term(GREEN2, a, b, (t.real, t.imag, float(c), float(d)))


def hubbard_terms(bonds, n_sites: int, t: float, U: float) -> List[Term]:
    """-t sum_<ij>,sigma (c+_is c_js + h.c.) + U sum_i n_iu n_id (one HOP term per bond and spin)."""
    terms = []
    for (i, j) in bonds:
        for sigma in (0, 1):
            terms.append(Term(HOP, 2 * i + sigma, 2 * j + sigma, (-t, 0.0)))
    if U != 0.0:
        for i in range(n_sites):
            terms.append(Term(HUBBARD_U, i, -1, (U,)))
    return terms


def square_supercell(a0: Tuple[int, int], a1: Tuple[int, int]):
    """Square-lattice supercell spanned by a0 = a0W e_W + a0L e_L and a1 (the
    lattice rule of Sec. 2.4 with unit vectors e_W = (1, 0), e_L = (0, 1)).

    Sites: the integer points with fractional coordinates in [0, 1) along
    (a0, a1), numbered in ascending (y, x).  Bonds: each site to its +x and +y
    neighbours, folded back by supercell translations; one entry per
    undirected bond.  Returns (n_sites, bonds, coords).
    """
    (ax, ay), (bx, by) = a0, a1
    det = ax * by - ay * bx
    if det == 0:
        raise ValueError("degenerate supercell")
    sgn = 1 if det > 0 else -1
    D = abs(det)

    def frac_num(x, y):
        # numerators of the fractional coordinates (times |det|)
        return (sgn * (x * by - y * bx), sgn * (ax * y - ay * x))

    xs = [0, ax, bx, ax + bx]
    ys = [0, ay, by, ay + by]
    pts = []
    for y in range(min(ys), max(ys) + 1):
        for x in range(min(xs), max(xs) + 1):
            f0, f1 = frac_num(x, y)
            if 0 <= f0 < D and 0 <= f1 < D:
                pts.append((x, y))
    pts.sort(key=lambda p: (p[1], p[0]))
    index = {p: k for k, p in enumerate(pts)}

    def fold(x, y):
        f0, f1 = frac_num(x, y)
        n0, n1 = f0 // D, f1 // D
        return (x - n0 * ax - n1 * bx, y - n0 * ay - n1 * by)

    bonds = []
    seen = set()
    for (x, y) in pts:
        i = index[(x, y)]
        for dx, dy in ((1, 0), (0, 1)):
            j = index[fold(x + dx, y + dy)]
            key = (min(i, j), max(i, j), dx)
            if i != j and key not in seen:
                seen.add(key)
                bonds.append((i, j))
    return len(pts), bonds, pts
