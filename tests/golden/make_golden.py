"""Writes tiny_bruteforce.json: spin-orbital brute-force values of term F
(Eq. expensive_term) and of F1..F8 (Table II) for one tiny seeded problem.
Calls only the oracle and the seeded generator."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dsrg_oracle as O  # noqa: E402
from paper_1603_00561_amd.workloads import make_problem  # noqa: E402


def main():
    shape, seed, s = (2, 2, 3, 10), 31, 0.5
    p = make_problem(*shape, s=s, seed=seed)
    B = O.full_symmetric_B(p.B_cv, p.B_ca, p.B_av)
    eri = np.einsum("Qpq,Qrs->pqrs", B, B)
    eps = np.concatenate([p.eps_c, p.eps_a, p.eps_v])
    r = O.brute_force_spinorbital(eri, p.nc, p.na, p.nv, eps, p.gamma1, p.s)
    out = dict(source="spin-orbital brute force of Eq. expensive_term and Table II",
               shape=list(shape), seed=seed, s=s,
               values={k: float(v) for k, v in r.items()})
    with open(os.path.join(HERE, "tiny_bruteforce.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
