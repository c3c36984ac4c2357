"""Write tests/golden/oracle_energies.json: ground-state energies of the
full-size Lanczos workloads, computed by the CPU oracle only.

For each space: the oracle's sparse H (terms applied literally, pushed
column by column) and its lowest eigenvalue (oracle.solvers.lowest_eigenvalue).
  * hubbard_4x3: 4x3 open Hubbard cluster, t = 1, U = 8 (and U = 0), 6 up + 6 down
  * tri24: 6x4 triangular Heisenberg torus, J = 1, every sector Sz = 0 .. 12

Run from the repository root: python tests/golden/make_oracle_energies.py
(several minutes and about 12 GB of memory for the Sz = 0 sector).
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from synth import lattices as L  # noqa: E402
from synth.configs import workload  # noqa: E402
from oracle import hamiltonian as oh  # noqa: E402
from oracle import solvers as osv  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_energies.json")


def e0(desc, terms):
    t0 = time.time()
    H = oh.sparse_h(desc, terms)
    e = osv.lowest_eigenvalue(H)
    print(f"  dim {H.shape[0]} nnz {H.nnz}: E0 = {e!r} ({time.time() - t0:.0f} s)", flush=True)
    return e, int(H.shape[0])


def main():
    out = {"source": "oracle.hamiltonian.sparse_h + oracle.solvers.lowest_eigenvalue (tests/golden/"
                     "make_oracle_energies.py)"}
    w = workload("hubbard_4x3")
    print("hubbard_4x3 U=8", flush=True)
    e, d = e0(w.basis, w.terms)
    out["hubbard_4x3_U8"] = {"dim": d, "e0": e}
    print("hubbard_4x3 U=0", flush=True)
    e, d = e0(w.basis, L.hubbard_terms(L.rect_bonds(4, 3, periodic=False), 12, t=1.0, U=0.0))
    out["hubbard_4x3_U0"] = {"dim": d, "e0": e}
    w = workload("tri24_allsz")
    sec = {}
    for d in [w.basis] + list(w.extra_bases):
        print(f"tri24 Sz={d.two_sz // 2}", flush=True)
        e, dim = e0(d, w.terms)
        sec[str(d.two_sz // 2)] = {"dim": dim, "e0": e}
        json.dump(dict(out, tri24=sec), open(OUT, "w"), indent=1)
    out["tri24"] = sec
    json.dump(out, open(OUT, "w"), indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
