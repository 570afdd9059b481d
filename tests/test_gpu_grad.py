"""GPU parity of dsrg_df_energy_backward (FP64 path) against the CPU oracle's
analytic gradient, central finite differences and the gradient identities.

Gate: relative gradient error <= 1e-6; the FP64 path is held to
1e-9 relative (norm-wise and per entry against the largest entry)."""
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
KEYS = ("B_cv", "B_ca", "B_av", "eps_c", "eps_a", "eps_v", "s")
REL = 1e-9


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(p):
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in p.arrays()]


def gpu_grad(p, gE, **kw):
    print(f"[gpu-grad] nc={p.nc} na={p.na} nv={p.nv} naux={p.naux} s={p.s} gE={gE} {kw}",
          flush=True)
    g = _b().energy_backward(*_dev(p), p.s, torch.tensor(gE, dtype=torch.float64).cuda(), **kw)
    torch.cuda.synchronize()
    ren = {"dB_cv": "B_cv", "dB_ca": "B_ca", "dB_av": "B_av", "deps_c": "eps_c",
           "deps_a": "eps_a", "deps_v": "eps_v", "ds": "s", "E": "E"}
    return {ren[k]: v.cpu().numpy() for k, v in g.items()}


def compare(g, ref, rel=REL):
    for k in KEYS:
        a, r = np.asarray(g[k]).ravel(), np.asarray(ref[k]).ravel()
        scale = max(np.abs(r).max(), 1e-300) if r.size else 1.0
        err = np.abs(a - r).max() if r.size else 0.0
        assert err <= rel * scale, (k, err, scale)
        if r.size:
            nerr = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300)
            assert nerr <= rel, (k, nerr)


@pytest.mark.parametrize("shape,gE", [
    ((3, 2, 70, 20), (1.0, 1.0, 1.0)),
    ((4, 3, 30, 17), (1.0, 0.75, -0.5)),    # 32-wide CAVV tiles inside one 64-wide panel
    ((2, 1, 130, 9), (0.3, -1.0, 2.0)),
    ((5, 6, 65, 33), (1.0, 0.75, -0.5)),
    ((1, 8, 40, 8), (1.0, 1.0, 1.0)),
    ((3, 0, 100, 24), (1.0, 1.0, 1.0)),
    # adjoint products split over K (contraction nc 64 ceil(nv/64) >= 1024 with
    # few output tiles): four equal segments in the CCVV, CAVV and CCAV
    # products; then K = 1600 in segments 544 / 544 / 512 (a short last one)
    ((9, 2, 200, 300), (1.0, 0.75, -0.5)),
    ((5, 2, 300, 200), (1.0, 1.0, 1.0)),
])
def test_small_gradients_against_oracle(shape, gE):
    p = make_problem(*shape, s=0.5, seed=sum(shape) + 11)
    g = gpu_grad(p, gE)
    ref = O.gradients(p, gE)
    compare(g, ref)
    assert np.allclose(g["E"], O.energy_terms(p), rtol=0, atol=1e-12)


@pytest.mark.parametrize("terms", ["ccvv", "cavv", "ccav"])
def test_term_masks(terms):
    p = make_problem(4, 3, 90, 24, s=0.7, seed=5)
    gE = (1.0, 0.75, -0.5)
    g = gpu_grad(p, gE, terms=terms)
    keep = {"ccvv": 0, "cavv": 1, "ccav": 2}[terms]
    gE_m = tuple(v if t == keep else 0.0 for t, v in enumerate(gE))
    compare(g, O.gradients(p, gE_m))


def test_near_degenerate_series_branch():
    p = make_near_degenerate(nc=3, na=2, nv=40, naux=24)
    gE = (1.0, 1.0, 1.0)
    compare(gpu_grad(p, gE), O.gradients(p, gE), rel=1e-8)


def test_gradient_identities_at_cfg4():
    p = make_config("cfg4")
    g = gpu_grad(p, (1.0, 1.0, 1.0))
    E = g["E"].sum()
    hb = sum(float(np.sum(getattr(p, k) * g[k])) for k in ("B_cv", "B_ca", "B_av"))
    assert abs(hb - 4 * E) <= 1e-11 * abs(E)
    assert abs(g["eps_c"].sum() + g["eps_a"].sum() + g["eps_v"].sum()) <= 1e-11 * abs(E)
    sc = (p.eps_c @ g["eps_c"] + p.eps_a @ g["eps_a"] + p.eps_v @ g["eps_v"]
          - 2 * p.s * g["s"][0])
    assert abs(sc + E) <= 1e-11 * abs(E)


def _check_refs(name, g):
    r = json.load(open(os.path.join(HERE, "golden", "oracle_refs.json")))[name]["grad"]
    for k in ("B_cv", "B_ca", "B_av"):
        vals = np.array([g[k][tuple(i)] for i in r[k]["idx"]])
        err = np.abs(vals - np.array(r[k]["val"])).max()
        assert err <= REL * r[k]["absmax"], (k, err)
        nrm = np.linalg.norm(g[k])
        assert abs(nrm - r[k]["norm"]) <= REL * r[k]["norm"], (k, nrm, r[k]["norm"])
        assert abs(np.sum(g[k] * getattr(make_config(name), k)) - r[k]["dot_B"]) <= \
            REL * abs(r[k]["dot_B"]) + 1e-12
    for k in ("eps_c", "eps_a", "eps_v", "s"):
        ref = np.array(r[k])
        assert np.abs(g[k] - ref).max() <= REL * np.abs(ref).max(), k


@pytest.mark.parametrize("name", ["cfg4", "cfg5"])
def test_full_size_gradients_against_oracle(name):
    r = json.load(open(os.path.join(HERE, "golden", "oracle_refs.json")))[name]["grad"]
    p = make_config(name)
    g = gpu_grad(p, tuple(r["gE"]))
    _check_refs(name, g)


def test_cfg4_central_differences_50_entries():
    """Central differences (h = 1e-5) of the GPU energy on 50 seeded entries
    against the GPU gradient; tolerance 1e-6 |g| + 10 ulp(E) / h."""
    b = _b()
    p = make_config("cfg4")
    gE = (1.0, 0.75, -0.5)
    g = gpu_grad(p, gE)
    t = _dev(p)
    wv = torch.tensor(gE, dtype=torch.float64)

    def L(tt, s):
        return float((b.energy(*tt, s).cpu() * wv).sum())

    E0 = abs(L(t, p.s))
    tol_fd = 10 * np.spacing(E0) / 1e-5
    rng = np.random.default_rng(2024)
    h = 1e-5
    names = ("B_cv", "B_ca", "B_av", "eps_c", "eps_a", "eps_v")
    for n in range(50):
        k = names[n % len(names)]
        arr_i = names.index(k)
        shape = t[arr_i].shape
        idx = tuple(int(rng.integers(0, d)) for d in shape)
        tp = [x.clone() for x in t]
        tm = [x.clone() for x in t]
        tp[arr_i][idx] += h
        tm[arr_i][idx] -= h
        fd = (L(tp, p.s) - L(tm, p.s)) / (2 * h)
        an = g[k][idx]
        assert abs(fd - an) <= 1e-6 * abs(an) + tol_fd, (k, idx, fd, an)
    fd = (L(t, p.s + h) - L(t, p.s - h)) / (2 * h)
    assert abs(fd - g["s"][0]) <= 1e-6 * abs(g["s"][0]) + tol_fd


def test_autograd_function_matches_backward_entry_point():
    from paper_1603_00561_amd import autograd
    p = make_problem(4, 2, 80, 20, s=0.5, seed=12)
    t = [x.clone().requires_grad_(k not in ("gamma1",)) for x, k in
         zip(_dev(p), ("B_cv", "B_ca", "B_av", "eps_c", "eps_a", "eps_v", "gamma1"))]
    s = torch.tensor(p.s, dtype=torch.float64, device="cuda", requires_grad=True)
    E = autograd.energy(*t, s)
    w = torch.tensor([1.0, 0.75, -0.5], dtype=torch.float64, device="cuda")
    (E * w).sum().backward()
    ref = O.gradients(p, (1.0, 0.75, -0.5))
    got = {k: x.grad.cpu().numpy() for k, x in zip(("B_cv", "B_ca", "B_av", "eps_c", "eps_a",
                                                    "eps_v"), t[:6])}
    got["s"] = np.array([s.grad.item()])
    compare(got, ref)


@pytest.mark.parametrize("shape,budget", [
    ((7, 3, 100, 40), 2_400_000),     # CAVV-bound: blocks of 3, 3, 1 core orbitals
    ((7, 0, 100, 40), 600_000),       # CCVV only: blocks of 2, 2, 2, 1
    ((6, 2, 140, 70), 3_500_000),     # blocks of 2, 2, 2
    ((9, 2, 200, 300), 8_000_000),    # blocks of 3, 3, 3; the CCAV products split over K
])
def test_gradient_in_core_blocks(shape, budget):
    """A small bound on the gradient's adjoint-tile region splits the core
    orbitals into blocks (block pairs for CCVV, blocks for CAVV); every
    element against the oracle, and bitwise equal to itself run to run."""
    b = _b()
    old = b.set_gradient_block_bytes(budget)
    try:
        p = make_problem(*shape, s=0.5, seed=sum(shape) + 5)
        gE = (1.0, 0.75, -0.5)
        g = gpu_grad(p, gE)
        g2 = gpu_grad(p, gE)
    finally:
        b.set_gradient_block_bytes(old)
    compare(g, O.gradients(p, gE))
    assert np.allclose(g["E"], O.energy_terms(p), rtol=0, atol=1e-12)
    for k in ("B_cv", "B_ca", "B_av"):
        assert np.array_equal(g[k], g2[k]), k


def test_workspace_bound_and_block_count():
    """The gradient workspace at the quintuple-zeta-shaped size stays far
    below the nc^2 nv^2 doubles that all pair tiles would take."""
    b = _b()
    nc, na, nv, naux = 23, 6, 1100, 3000
    ws = b.workspace_size(nc, na, nv, naux, with_grad=True)
    all_tiles = 8 * (nc * 64 * 18) ** 2
    assert ws < 2.5e9 < all_tiles, (ws, all_tiles)
