"""Named workloads: basis descriptor + term list + solver parameters + seeds.

The five production workloads are:

* ``heis_chain16``     Heisenberg chain N=16, PBC, J=1, full 2^16 space,
                       complex128, FP64 Lanczos 200 iterations, start seed 1.
* ``hubbard_4x3``      Hubbard 4x3 open cluster, t=1, U=8, 6 up + 6 down,
                       dim C(12,6)^2 = 853,776, complex128 FP64 Lanczos, seed 2.
* ``kh_honeycomb24``   Kitaev-Heisenberg honeycomb 24 sites PBC, K=-1, J=0.1,
                       link directions drawn per link, full 2^24 space,
                       microcanonical TPQ, 16 samples (seeds 300..315),
                       complex64 storage, l = 1.5 (intensive shift), 2000 steps.
* ``tri24_allsz``      Triangular J1 Heisenberg 6x4 torus, Sz = 0..12 sectors,
                       real FP32 storage, FP64 recurrences, seeds 400 + Sz.
* ``kagome36_sz0``     Kagome Heisenberg 36 sites PBC, Sz = 0,
                       dim C(36,18) = 9,075,135,300, real FP64 / FP32, seed 5.

Widening beyond them:

* ``hubbard18_tpq``    the paper's 18-site tilted square Hubbard cluster
                       (a0 = (3, 3), a1 = (-3, 3)), t = 1, U = 8, half filling,
                       Sz = 0: dim C(18,9)^2 = 2,363,904,400, split 18/18,
                       microcanonical TPQ, complex128 (one sample) or complex64
                       (four samples), l = 8.5 (above the largest energy per
                       site, <= U/2 + 4t), seeds 600...
* ``hubbard8_tpq``     the paper's 8-site cluster (a0 = (2, 2), a1 = (-2, 2)),
                       U = 8, half filling, Sz = 0 (dim 4,900), 20 samples.

plus small cases used by tests (4-site ring, two-site Hubbard, ...).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import lattices as L


@dataclass(frozen=True)
class BasisDesc:
    """Hilbert-space descriptor.

    particle: "spin" (one bit per site) or "fermion" (two bits per site,
    orbital 2*site + sigma).  sector: "none", "sz" (spins; two_sz = 2*Sz),
    "nupndn" (fermions; n_up, n_dn) or "ntot" (fermions; n_tot).
    """
    particle: str
    n_sites: int
    sector: str = "none"
    two_sz: int = 0
    n_up: int = 0
    n_dn: int = 0
    n_tot: int = 0
    split_bits: int = 0

    @property
    def n_bits(self) -> int:
        return self.n_sites if self.particle == "spin" else 2 * self.n_sites


@dataclass
class Workload:
    name: str
    basis: BasisDesc
    terms: List[L.Term]
    dtype: str                      # storage: "f64", "c128", "f32", "c64"
    method: str                     # "lanczos" or "tpq"
    n_iter: int = 0                 # Lanczos iterations or TPQ steps
    nvec: int = 1                   # batch (TPQ samples)
    seeds: List[int] = field(default_factory=list)
    tpq_l: float = 0.0
    extra_bases: List[BasisDesc] = field(default_factory=list)   # further sectors of one batched run
    note: str = ""


def _heis_chain(n=16, J=1.0):
    return [L.heisenberg_bond(i, j, J) for (i, j) in L.chain_bonds(n, True)]


def kh_directions(n_links: int = 36, seed: int = 3) -> np.ndarray:
    """Per-link Kitaev direction gamma in {0,1,2}, drawn uniformly in link order."""
    return np.random.default_rng(seed).integers(0, 3, size=n_links)


def kh_honeycomb_terms(K=-1.0, J=0.1, lx=3, ly=4, random_dirs=True, seed=3):
    links = L.honeycomb_links(lx, ly)
    if random_dirs:
        g = kh_directions(len(links), seed)
        return [L.kitaev_heisenberg_bond(a, b, int(g[n]), K, J) for n, (a, b, _) in enumerate(links)]
    return [L.kitaev_heisenberg_bond(a, b, lab, K, J) for (a, b, lab) in links]


def workload(name: str) -> Workload:
    if name == "heis_chain16":
        return Workload(name, BasisDesc("spin", 16), _heis_chain(16), "c128", "lanczos",
                        n_iter=200, seeds=[1])
    if name == "hubbard_4x3":
        terms = L.hubbard_terms(L.rect_bonds(4, 3, periodic=False), 12, t=1.0, U=8.0)
        return Workload(name, BasisDesc("fermion", 12, "nupndn", n_up=6, n_dn=6), terms,
                        "c128", "lanczos", n_iter=200, seeds=[2])
    if name == "kh_honeycomb24":
        return Workload(name, BasisDesc("spin", 24), kh_honeycomb_terms(), "c64", "tpq",
                        n_iter=2000, nvec=16, seeds=list(range(300, 316)), tpq_l=1.5)
    if name == "tri24_allsz":
        terms = [L.heisenberg_bond(i, j, 1.0) for (i, j) in L.triangular_bonds(6, 4)]
        bases = [BasisDesc("spin", 24, "sz", two_sz=2 * sz) for sz in range(13)]
        return Workload(name, bases[0], terms, "f32", "lanczos", n_iter=200,
                        seeds=[400 + sz for sz in range(13)], extra_bases=bases[1:])
    if name == "kagome36_sz0":
        terms = [L.heisenberg_bond(i, j, 1.0) for (i, j) in L.kagome_bonds(3, 4)]
        return Workload(name, BasisDesc("spin", 36, "sz", two_sz=0, split_bits=18), terms,
                        "f64", "lanczos", n_iter=100, seeds=[5])
    if name == "hubbard18_tpq":
        n, bonds, _ = L.square_supercell((3, 3), (-3, 3))
        terms = L.hubbard_terms(bonds, n, t=1.0, U=8.0)
        return Workload(name, BasisDesc("fermion", n, "nupndn", n_up=9, n_dn=9, split_bits=18), terms,
                        "c128", "tpq", n_iter=2000, nvec=1, seeds=[600, 601, 602, 603], tpq_l=8.5)
    if name == "hubbard8_tpq":
        n, bonds, _ = L.square_supercell((2, 2), (-2, 2))
        terms = L.hubbard_terms(bonds, n, t=1.0, U=8.0)
        return Workload(name, BasisDesc("fermion", n, "nupndn", n_up=4, n_dn=4), terms,
                        "c128", "tpq", n_iter=400, nvec=16, seeds=list(range(700, 720)), tpq_l=8.5)
    # ---- small cases
    if name == "heis_ring4":
        return Workload(name, BasisDesc("spin", 4), _heis_chain(4), "f64", "lanczos", n_iter=16, seeds=[11])
    if name == "hubbard_2site":
        terms = L.hubbard_terms([(0, 1)], 2, t=1.0, U=8.0)
        return Workload(name, BasisDesc("fermion", 2, "nupndn", n_up=1, n_dn=1), terms,
                        "f64", "lanczos", n_iter=4, seeds=[12])
    if name == "heis_chain12":
        return Workload(name, BasisDesc("spin", 12), _heis_chain(12), "c128", "lanczos", n_iter=120, seeds=[13])
    if name == "kh_honeycomb12":
        return Workload(name, BasisDesc("spin", 12), kh_honeycomb_terms(lx=3, ly=2, random_dirs=False),
                        "c128", "tpq", n_iter=50, nvec=4, seeds=[20, 21, 22, 23], tpq_l=1.5)
    raise KeyError(name)


WORKLOADS = ("heis_chain16", "hubbard_4x3", "kh_honeycomb24", "tri24_allsz", "kagome36_sz0")
