"""CPU oracle for the matrix-free H.v / Lanczos / TPQ hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, literal CPU
reference written from the paper (Kawamura et al., "Quantum Lattice
Model Solver HPhi", Sec. 3).  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import or execute it.  The
product library never calls it, shares no code with it, and must fail
loudly instead of falling back to it.

Everything is FP64 (complex128 where the Hamiltonian is complex).

Modules
-------
basis        sector enumeration by filtering and sorting, rank by binary
             search, combinatorial-number-system rank (Sec. 3.1).
hamiltonian  spin and fermion operators applied literally to basis
             states (Sec. 2.3 models, Sec. 3.3 product, Appendix A.1 spin
             operators), H.v by pushing columns, element lists, dense H.
solvers      dense diagonalization (Sec. 3.2), Lanczos with the second
             pass for the eigenvector and the energy/variance check
             (Sec. 3.4, Appendix A.3), microcanonical TPQ (Sec. 3.5) and
             its spectral closed form.
c_oracle     ctypes wrapper of hv_oracle.c, a plain C/OpenMP row-slice
             H.v used for full-size sampled checks and CPU timing.

Parity status: every function is pinned by tests under tests/ against
values the paper prints, closed forms or brute force; see the module
headers.
"""
