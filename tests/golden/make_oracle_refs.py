"""Writes oracle_refs.json: the CPU oracle's energies (and, for the
gradient workloads, sampled gradient entries, full orbital-energy and s
gradients and the norms of the B gradients) on the seeded synthetic
workloads. Calls only the oracle and the seeded generator.

    python tests/golden/make_oracle_refs.py [cfg ...]
    python tests/golden/make_oracle_refs.py --active [cfg ...]

With --active only the pieces F4-F8 of term F are computed (key "F48_s<s>")
and merged into the existing entries; with --laplace the Laplace-factorized
Coulomb part of E_CCVV (key "laplace_nq<N>": the oracle's exponential-sum fit
t, w and its error, the per-term sums S_k, the factorized energy and the
exact Coulomb part).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dsrg_laplace as L  # noqa: E402
from oracle import dsrg_oracle as O  # noqa: E402
from paper_1603_00561_amd.workloads import CONFIGS, make_config  # noqa: E402

OUT = os.path.join(HERE, "oracle_refs.json")
GE = (1.0, 0.75, -0.5)        # upstream weights used by the gradient references
NSAMPLE = 64
# fixed seeds of the sampled gradient entries, one per block of B
SAMPLE_SEEDS = {"B_cv": 711, "B_ca": 712, "B_av": 713}


def sample_indices(shape, seed):
    rng = np.random.default_rng(seed)
    return [[int(rng.integers(0, n)) for n in shape] for _ in range(NSAMPLE)]


def run(name):
    c = CONFIGS[name]
    out = {}
    s_list = c.get("s_list", (c["s"],))
    for s in s_list:
        p = make_config(name, s=s)
        t = time.time()
        e = O.energy_terms(p, terms=c["terms"])
        out["E_s%g" % s] = list(e)
        out["t_energy_s%g" % s] = time.time() - t
        print(name, s, e, time.time() - t, flush=True)
    if c["grad"]:
        p = make_config(name)
        t = time.time()
        g = O.gradients(p, GE)
        gr = dict(gE=list(GE), t=time.time() - t)
        for k in ("B_cv", "B_ca", "B_av"):
            idx = sample_indices(g[k].shape, SAMPLE_SEEDS[k])
            gr[k] = dict(idx=idx, val=[float(g[k][tuple(i)]) for i in idx],
                         norm=float(np.linalg.norm(g[k])), absmax=float(np.abs(g[k]).max()),
                         dot_B=float(np.sum(g[k] * getattr(p, k))))
        for k in ("eps_c", "eps_a", "eps_v", "s"):
            gr[k] = [float(x) for x in g[k]]
        out["grad"] = gr
        print(name, "grad", time.time() - t, flush=True)
    return out


def run_active(name, entry):
    p = make_config(name)
    t = time.time()
    f = O.active_terms(p)
    entry["F48_s%g" % p.s] = list(f)
    entry["t_F48_s%g" % p.s] = time.time() - t
    print(name, "F4-F8", f, time.time() - t, flush=True)
    return entry


LAPLACE_NQ = 16


def run_laplace(name, entry):
    p = make_config(name)
    lo, hi = L.spectral_range(p.eps_c, p.eps_v)
    t0 = time.time()
    t, w, err = L.laplace_fit(p.s, lo, hi, LAPLACE_NQ)
    e_lt, S = L.coulomb_laplace(p.B_cv, p.eps_c, p.eps_v, t, w)
    t1 = time.time()
    e_j = L.coulomb_exact_pairs(p.B_cv, p.eps_c, p.eps_v, p.s)
    entry["laplace_nq%d" % LAPLACE_NQ] = dict(
        x_lo=lo, x_hi=hi, t=[float(x) for x in t], w=[float(x) for x in w], max_err=err,
        S=[float(x) for x in S], E_LT=e_lt, E_J=e_j, t_lt=t1 - t0, t_exact=time.time() - t1)
    print(name, "laplace", e_lt, e_j, err, time.time() - t0, flush=True)
    return entry


def main():
    args = sys.argv[1:]
    active = "--active" in args
    laplace = "--laplace" in args
    names = [a for a in args if a not in ("--active", "--laplace")] or list(CONFIGS)
    refs = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            refs = json.load(f)
    for n in names:
        if laplace:
            refs[n] = run_laplace(n, refs.get(n, {}))
        elif active:
            refs[n] = run_active(n, refs.get(n, {}))
        else:
            refs[n] = {**refs.get(n, {}), **run(n)}
        with open(OUT, "w") as f:
            json.dump(refs, f, indent=1)


if __name__ == "__main__":
    main()
