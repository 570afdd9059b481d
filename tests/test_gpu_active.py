"""GPU parity of dsrg_df_energy_active (the pieces F4-F8 of term F, Table II)
against the FP64 CPU oracle. Gate: |F_gpu - F_oracle| <= 1e-10 Eh per piece
(the FP64 bar), with the relative error printed."""
import copy
import json
import os

import numpy as np
import pytest
import torch

from oracle import dsrg_oracle as O
from paper_1603_00561_amd.workloads import make_problem, make_config, make_near_degenerate

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GATE = 1e-10


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def gpu_F(p, **kw):
    print(f"[gpu-active] nc={p.nc} na={p.na} nv={p.nv} naux={p.naux} s={p.s} {kw}", flush=True)
    F = _b().energy_active(_dev(p.B_cv), _dev(p.B_ca), _dev(p.B_av), _dev(p.B_aa),
                           _dev(p.eps_c), _dev(p.eps_a), _dev(p.eps_v), _dev(p.gamma1), p.s, **kw)
    torch.cuda.synchronize()
    return F.cpu().numpy()


def check(Fg, Fo, gate=GATE):
    Fo = np.asarray(Fo)
    err = np.abs(np.asarray(Fg) - Fo)
    print("F4..F8 |dF|:", err, "relative:", err / np.maximum(np.abs(Fo), 1e-300), flush=True)
    assert np.all(err <= gate), (Fg, Fo, err)


@pytest.mark.parametrize("shape", [(3, 2, 70, 20), (4, 3, 65, 33), (2, 1, 130, 9),
                                   (5, 6, 200, 40), (1, 8, 40, 8), (6, 4, 257, 31),
                                   (1, 1, 1, 1), (7, 5, 64, 16)])
def test_small_shapes(shape):
    # several 64-wide virtual panels with ragged tails, auxiliary counts off the
    # 16-row chunk, one orbital per space
    p = make_problem(*shape, s=0.5, seed=sum(shape) + 17)
    check(gpu_F(p), O.active_terms(p))


@pytest.mark.parametrize("na", list(range(1, 9)))
def test_every_active_size(na):
    p = make_problem(4, na, 90, 24, s=0.7, seed=60 + na)
    check(gpu_F(p), O.active_terms(p))


def test_no_active_orbitals_gives_zeros():
    p = make_problem(3, 0, 50, 10, seed=2)
    F = _b().energy_active(_dev(p.B_cv), None, None, None, _dev(p.eps_c), None,
                           _dev(p.eps_v), None, p.s)
    assert np.all(F.cpu().numpy() == 0.0)


def test_s_zero_and_density_limits():
    p = make_problem(4, 3, 80, 20, s=0.0, seed=5)
    assert np.all(gpu_F(p) == 0.0)
    p = make_problem(4, 3, 80, 20, s=0.5, seed=6)
    q = copy.deepcopy(p)
    q.gamma1 = np.zeros((3, 3))          # no active hole line: only F5 survives
    F = gpu_F(q)
    assert F[0] == 0.0 and F[2] == 0.0 and F[3] == 0.0 and F[4] == 0.0
    check(F, O.active_terms(q))
    q.gamma1 = 2.0 * np.eye(3)           # no active particle line: only F4 survives
    F = gpu_F(q)
    assert F[1] == 0.0 and F[2] == 0.0 and F[3] == 0.0 and F[4] == 0.0
    check(F, O.active_terms(q))


def test_near_degenerate_series_branch():
    p = make_near_degenerate(nc=4, na=3, nv=70, naux=40)
    check(gpu_F(p), O.active_terms(p))


def test_bitwise_reproducible_and_timing_option():
    p = make_problem(6, 4, 200, 64, seed=9)
    F1 = gpu_F(p)
    F2 = gpu_F(p, timing=True)
    assert np.array_equal(F1, F2)
    names = [n for n, _ in _b().kernel_times(64)]
    for k in ("act_f4", "act_f5", "act_f6", "act_f7", "act_f8", "finalize"):
        assert k in names, (k, names)


@pytest.mark.parametrize("name", ["cfg2", "cfg4", "cfg5"])
def test_full_size_against_oracle(name):
    """References from tests/golden/make_oracle_refs.py --active."""
    with open(os.path.join(HERE, "golden", "oracle_refs.json")) as f:
        r = json.load(f)[name]
    p = make_config(name)
    check(gpu_F(p), r["F48_s%g" % p.s])
