"""Seeded synthetic inputs shared by the product path and the CPU oracle.

This package only *describes* inputs: lattice bond lists written as
physical coupling terms, basis (sector) descriptors, and seeded random
vectors.  It holds none of the method's arithmetic (no operator algebra,
no rank tables, no matrix elements), so that the HIP path and the oracle
stay independent while consuming identical inputs.
"""

from .lattices import (  # noqa: F401
    Term,
    SPIN_BOND,
    SPIN_FIELD,
    HOP,
    DENS,
    NUM,
    HUBBARD_U,
    heisenberg_bond,
    kitaev_heisenberg_bond,
    chain_bonds,
    honeycomb_links,
    triangular_bonds,
    kagome_bonds,
    rect_bonds,
    random_spin_terms,
    random_fermion_terms,
)
from .configs import (  # noqa: F401
    BasisDesc,
    Workload,
    workload,
    WORKLOADS,
)
from .vectors import gaussian_vectors, uniform_vectors  # noqa: F401
