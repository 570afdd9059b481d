"""HIP-graph capture of the entry points (torch.cuda.graph). The library only
enqueues kernels and device-to-device copies on the caller's stream (every
buffer it clears is cleared by a kernel, never by a memset node), so a captured
call replays. Each graph is replayed several times with eager calls on other
inputs (which overwrite the shared workspace) and synchronizations in between,
and every replay is compared with the eager result of the captured inputs:
bitwise wherever the reduction order is fixed (everything but the gradient's
dE/d eps and dE/ds, which are sums of FP64 atomics)."""
import numpy as np
import pytest
import torch

from paper_1603_00561_amd.workloads import make_fock_problem, make_problem

pytestmark = pytest.mark.gpu
REPLAYS = 3


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _capture(fn):
    """fn() enqueues the call and returns its output tensors; warm up on a
    side stream, then capture one call."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        outs = fn()
    torch.cuda.synchronize()
    return g, outs


def _replay_and_check(g, outs, ref, other, last_bits=()):
    """outs listed by index in last_bits are sums of FP64 atomics (their order
    varies run to run): compared to 1e-13 of their largest entry, the rest
    bitwise."""
    for k in range(REPLAYS):
        for o in outs:
            o.fill_(float("nan"))
        other()                      # eager work on other inputs, same workspace
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for n, (o, r) in enumerate(zip(outs, ref)):
            if n in last_bits:
                tol = 1e-13 * max(r.abs().max().item(), 1e-300)
                assert (o - r).abs().max().item() <= tol, (k, n, (o - r).abs().max().item())
            else:
                assert torch.equal(o, r), (k, n, (o - r).abs().max().item())
        print(f"[gpu-graph] replay {k} matches", flush=True)


@pytest.mark.parametrize("prec", ["fp64", "ozaki"])
def test_energy_replays(prec):
    print(f"[gpu-graph] energy {prec}", flush=True)
    b = _b()
    p = make_problem(6, 3, 150, 70, s=0.5, seed=21)
    q = make_problem(6, 3, 150, 70, s=0.3, seed=22)
    t, u = [_dev(x) for x in p.arrays()], [_dev(x) for x in q.arrays()]
    ws = torch.empty(b.workspace_size(p.nc, p.na, p.nv, p.naux, precision=prec),
                     dtype=torch.uint8, device="cuda")
    ref = [b.energy(*t, p.s, precision=prec, workspace=ws).clone()]
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    g, outs = _capture(lambda: [b.energy(*t, p.s, precision=prec, workspace=ws, out=out)])
    _replay_and_check(g, outs, ref, lambda: b.energy(*u, q.s, precision=prec, workspace=ws))


def test_energy_backward_replays():
    print("[gpu-graph] energy_backward fp64", flush=True)
    b = _b()
    p = make_problem(5, 2, 130, 60, s=0.5, seed=23)
    q = make_problem(5, 2, 130, 60, s=0.7, seed=24)
    t, u = [_dev(x) for x in p.arrays()], [_dev(x) for x in q.arrays()]
    gE = torch.tensor([1.0, -0.5, 0.25], dtype=torch.float64, device="cuda")
    ws = torch.empty(b.workspace_size(p.nc, p.na, p.nv, p.naux, with_grad=True),
                     dtype=torch.uint8, device="cuda")
    keys = ("dB_cv", "dB_ca", "dB_av", "deps_c", "deps_a", "deps_v", "ds", "E")
    r = b.energy_backward(*t, p.s, gE, workspace=ws)
    ref = [r[k].clone() for k in keys]

    def call():
        g = b.energy_backward(*t, p.s, gE, workspace=ws)
        return [g[k] for k in keys]
    g, outs = _capture(call)
    atomics = tuple(n for n, k in enumerate(keys) if k.startswith("deps") or k == "ds")
    _replay_and_check(g, outs, ref, lambda: b.energy_backward(*u, q.s, gE, workspace=ws),
                      last_bits=atomics)


def test_upstream_builds_replay():
    # DF factors, generalized Fock matrix and semicanonical rotation (the
    # last with its device-side convergence flag) captured in one graph
    print("[gpu-graph] factors + fock + semicanonicalize", flush=True)
    b = _b()
    f = make_fock_problem(2, 5, 3, 60, 90, seed=25)
    o = make_fock_problem(2, 5, 3, 60, 90, seed=26)
    ins = [_dev(x) for x in (f.ao3, f.J, f.C, f.h, f.gamma1)]
    oth = [_dev(x) for x in (o.ao3, o.J, o.C, o.h, o.gamma1)]
    shape = (f.nfrz, f.nc, f.na, f.nv)

    def chain(ao3, J, C, h, g1):
        B = b.df_factors(ao3, J, C, *shape)
        F = b.df_fock(ao3, J, C, h, g1, *shape)
        eps, U, Cs = b.semicanonicalize(F, *shape, C=C)
        return [B["B_cv"], B["B_ca"], B["B_av"], B["B_aa"], F, eps, U, Cs]

    ref = [x.clone() for x in chain(*ins)]
    g, outs = _capture(lambda: chain(*ins))
    _replay_and_check(g, outs, ref, lambda: chain(*oth))


def test_active_terms_replay():
    # F4-F8 (about twenty launches, no host wait inside the call)
    print("[gpu-graph] energy_active", flush=True)
    b = _b()
    p = make_problem(5, 3, 70, 40, seed=31)
    q = make_problem(5, 3, 70, 40, s=0.3, seed=32)
    keys = ("B_cv", "B_ca", "B_av", "B_aa", "eps_c", "eps_a", "eps_v", "gamma1")
    u = [_dev(getattr(p, k)) for k in keys]
    v = [_dev(getattr(q, k)) for k in keys]
    ws = torch.empty(b.active_workspace_size(p.nc, p.na, p.nv, p.naux), dtype=torch.uint8,
                     device="cuda")

    def call(t, s):
        F = torch.empty(5, dtype=torch.float64, device="cuda")
        b.energy_active(*t, s, out=F, workspace=ws)
        return [F]

    ref = [x.clone() for x in call(u, p.s)]
    g, outs = _capture(lambda: call(u, p.s))
    _replay_and_check(g, outs, ref, lambda: call(v, q.s))
