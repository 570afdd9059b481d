"""GPU parity of the error-free int8 slice path (precision "ozaki") against
the FP64 CPU oracle. Gate: |E_gpu - E_oracle| <= 1e-6 Eh per term."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import dsrg_oracle as O
from paper_1603_00561_amd.workloads import make_problem, make_config, make_near_degenerate

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GATE = 1e-6


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(p):
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in p.arrays()]


def gpu_E(p, **kw):
    print(f"[gpu-split] nc={p.nc} na={p.na} nv={p.nv} naux={p.naux} s={p.s} {kw}", flush=True)
    E = _b().energy(*_dev(p), p.s, precision="ozaki", **kw)
    torch.cuda.synchronize()
    return E.cpu().numpy()


def refs():
    with open(os.path.join(HERE, "golden", "oracle_refs.json")) as f:
        return json.load(f)


def check(Eg, Eo, gate=GATE):
    err = np.abs(np.asarray(Eg) - np.asarray(Eo))
    print("split |dE| per term:", err, "relative:", err / np.maximum(np.abs(Eo), 1e-300))
    assert np.all(err <= gate), (Eg, Eo, err)


@pytest.mark.parametrize("shape", [(5, 3, 150, 70), (3, 1, 64, 32), (4, 2, 65, 33),
                                   (2, 8, 130, 40), (1, 1, 1, 1), (7, 5, 33, 100),
                                   (3, 0, 90, 31), (6, 6, 200, 257)])
def test_small_shapes(shape):
    p = make_problem(*shape, s=0.5, seed=sum(shape) + 3)
    Eg = gpu_E(p)
    Eo = np.array(O.energy_terms(p))
    check(Eg, Eo)
    # far inside the gate at these magnitudes
    assert np.all(np.abs(Eg - Eo) <= 1e-10 * np.abs(Eo).max() + 1e-15)


def test_s_zero_and_special_gammas():
    p = make_problem(4, 3, 100, 40, s=0.0, seed=5)
    assert np.all(gpu_E(p) == 0.0)
    p = make_problem(4, 3, 100, 40, s=0.5, seed=6)
    p.gamma1 = 2.0 * np.eye(3)
    check(gpu_E(p), O.energy_terms(p))
    p.gamma1 = np.zeros((3, 3))
    Eg = gpu_E(p)
    assert Eg[1] == 0.0
    check(Eg, O.energy_terms(p))


def test_near_degenerate():
    p = make_near_degenerate(nc=4, na=3, nv=70, naux=40)
    check(gpu_E(p), O.energy_terms(p))


def test_bitwise_reproducible():
    p = make_problem(6, 2, 200, 64, seed=9)
    t = _dev(p)
    b = _b()
    E1 = b.energy(*t, p.s, precision="ozaki").cpu().numpy()
    E2 = b.energy(*t, p.s, precision="ozaki").cpu().numpy()
    assert np.array_equal(E1, E2)


def test_term_masks():
    p = make_problem(4, 3, 70, 20, seed=3)
    Eo = O.energy_terms(p)
    for mask, keep in (("ccvv", (0,)), ("cavv", (1,)), ("ccav", (2,))):
        Eg = gpu_E(p, terms=mask)
        for t in range(3):
            if t in keep:
                assert abs(Eg[t] - Eo[t]) <= GATE
            else:
                assert Eg[t] == 0.0


@pytest.mark.parametrize("name", ["cfg2", "cfg4", "cfg5"])
def test_full_size(name):
    r = refs()[name]
    p = make_config(name)
    check(gpu_E(p), r["E_s%g" % p.s])


def test_cfg3_all_s():
    r = refs()["cfg3"]
    for s in (0.1, 0.5, 1.0):
        p = make_config("cfg3", s=s)
        check(gpu_E(p), r["E_s%g" % s])


def _balanced_digits(v, n=4):
    """Round-to-nearest digits of v in (-1, 1]: 127 v = d0 + (d1 + (d2 + ...)/254)/254."""
    r, d = 127.0 * v, []
    for _ in range(n):
        s = np.rint(r)
        d.append(int(s))
        r = (r - s) * 254.0
    return d


def test_naux_limit_near_worst_case_level_sums():
    """naux = 33000, the largest contraction the slice path accepts, with every
    element of B equal to c = 2^-10 (126 + (126 + (126 + 126/254)/254)/254)/127.
    Every column then has scale 2^-10 and digits (126, 126, 126, 126), so the
    level-3 int32 sums of the off-diagonal integrals reach
    2 (126*126 + 126*126) * 33000 = 2.096e9, 97.6 % of 2^31: a wrapped sum
    would show as an O(1) relative error."""
    c = (126 + (126 + (126 + 126 / 254) / 254) / 254) / 127
    d = _balanced_digits(c)
    assert d == [126, 126, 126, 126]
    naux = 33000
    level3 = 2 * (d[0] * d[3] + d[1] * d[2]) * naux
    assert 0.97 * 2**31 < level3 < 2**31
    p = make_problem(2, 1, 40, naux, s=0.5, seed=33)
    v = c * 2.0**-10
    p.B_cv = np.full_like(p.B_cv, v)
    p.B_ca = np.full_like(p.B_ca, v)
    p.B_av = np.full_like(p.B_av, v)
    Eo = np.array(O.energy_terms(p))
    assert np.abs(Eo).max() > 0.1
    check(gpu_E(p), Eo)
    # the FP64 path on the same input, at its own gate (33000 equal terms per
    # integral: summation order alone moves the sums by ~1e-12 relative)
    E64 = _b().energy(*_dev(p), p.s).cpu().numpy()
    assert np.all(np.abs(E64 - Eo) <= 1e-10), (E64, Eo, np.abs(E64 - Eo))
