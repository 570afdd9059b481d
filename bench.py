"""Throughput of the DF-DSRG-MRPT2 F1-F3 hot path on one MI355X.

One step = one dsrg_df_energy call (panel packing, the CCVV, CAVV and CCAV
contraction kernels with their fused regulariser epilogues, and the final
reduction) on seeded synthetic inputs already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cfg2]
                    [--precision fp64] [--no-cpu-baseline]
                    [--grad | --active | --dfgen | --fock | --semican]

With --active a step is one dsrg_df_energy_active call instead (the pieces
F4-F8 of term F, FP64), measured the same way against its own algorithmic
work (the contractions over Q that form its integrals). With --dfgen a step
is one dsrg_df_factors call (the density-fitting factors B from AO
three-index integrals, FP64) for the config's orbital spaces; with --fock one
dsrg_df_fock call (the generalized Fock matrix of Eq. gen_fock from the same
DF integrals, FP64); with --semican one dsrg_df_semicanonicalize call (the
semicanonical rotation of that Fock matrix and C U, FP64).

Prints one JSON line. `value` is algorithmic TFLOP/s of the whole step:
F_alg = 2 naux [nc(nc+1)/2 nv^2 + nc na nv^2 + nc^2 na nv] (the contractions
the method must perform; epilogue exponentials are not counted) divided by
the measured time per step. `roofline` reports the dominant kernel (CCVV)
against the FP64 matrix-core peak, timed with HIP events on the stream it
runs on. `cpu_baseline` times the CPU oracle on a bounded sample of the same
workload on this host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "split_bf16": 2500.0, "ozaki": 5000.0}
PEAK_HBM_GBS = 8000.0


# int8 slice products per multiply-add of the slice path (four slices, levels <= 3)
SLICE_PRODUCTS = 10.0


def alg_flops(nc, na, nv, naux, terms=("ccvv", "cavv", "ccav")):
    f = {"ccvv": 2.0 * naux * (nc * (nc + 1) / 2) * nv * nv,
         "cavv": 2.0 * naux * nc * na * nv * nv,
         "ccav": 2.0 * naux * nc * nc * na * nv}
    return sum(f[t] for t in terms), f


def active_alg_flops(nc, na, nv, naux):
    """Contractions over Q that the pieces F4-F8 need: (xe|uf) for F4 over its
    distinct pairs x <= u ((xe|uf) = (uf|xe)), (mv|xe) and (me|xv) for F6,
    (ze|yv) for F7, (mv|ny) for F5, (mv|wy) for F8."""
    f = {"f4": 2.0 * naux * (na * (na + 1) / 2) * nv * nv,
         "f6": 2.0 * naux * 2 * nc * na * na * nv,
         "f7": 2.0 * naux * na ** 3 * nv,
         "f5": 2.0 * naux * nc * nc * na * na,
         "f8": 2.0 * naux * nc * na ** 3}
    return sum(f.values()), f


def cpu_baseline_active(p, budget_s=20.0):
    """The oracle's F4-F8 on the first nv_s virtual orbitals, nv_s sized to the
    budget from a 32-orbital probe (the work scales as nv^2)."""
    import copy
    from oracle import dsrg_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1

    def sub(nv_s):
        q = copy.copy(p)
        q.nv, q.B_cv, q.B_av, q.eps_v = nv_s, p.B_cv[:, :, :nv_s], p.B_av[:, :, :nv_s], p.eps_v[:nv_s]
        return q

    nv0 = min(p.nv, 32)
    t = time.perf_counter()
    O.active_terms(sub(nv0))
    t0 = max(time.perf_counter() - t, 1e-6)
    nv_s = int(min(p.nv, max(nv0, nv0 * (budget_s / t0) ** 0.5)))
    t = time.perf_counter()
    O.active_terms(sub(nv_s))
    dt = time.perf_counter() - t
    F, _ = active_alg_flops(p.nc, p.na, nv_s, p.naux)
    return {"value": F / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "seconds": round(dt, 3),
            "sample": f"F4-F8 over the first {nv_s}/{p.nv} virtual orbitals "
                      "(FP64 numpy/BLAS oracle, same inputs)"}


def dfgen_alg_flops(nao, naux, nc, na, nv):
    """The density-fitting build: the two MO-transform contractions (the
    short core | active index first), the Cholesky factor and inverse of the
    metric, and the triangular application."""
    npp, nq = nc + na, na + nv
    f = {"half1": 2.0 * naux * npp * nao * nao,
         "half2": 2.0 * naux * npp * nao * nq,
         "metric": 2.0 * naux ** 3 / 3.0,
         "apply": 1.0 * naux * naux * npp * nq}
    return sum(f.values()), f


def dfgen_alg_bytes(nao, naux, nc, na, nv):
    """HBM bytes each single-launch stage of the factor build must move: its
    operands read once and its result written once (FP64)."""
    npp, nq = nc + na, na + nv
    return {"half1": 8.0 * (naux * nao * nao + naux * npp * nao),
            "half2": 8.0 * (naux * npp * nao + naux * npp * nq),
            "apply": 8.0 * (naux * naux / 2.0 + 2.0 * naux * npp * nq)}


def kernel_table(binding, torch, call, n):
    """Average duration per launch of every kernel (HIP events), from n calls
    of call(True) made outside the timed region."""
    binding.kernel_times(1)
    for _ in range(n):
        call(True)
    torch.cuda.synchronize()
    per = {}
    for name, ms in binding.kernel_times(4096):
        per.setdefault(name, []).append(ms)
    return {k: float(np.mean(v)) for k, v in per.items()}


def timed_region(binding, torch, call, steps, names):
    """Wall time per call over `steps` calls of call(True), with HIP events
    around the named kernels only; returns (ms per call, average ms per launch
    of the named kernels)."""
    binding.kernel_times(1)
    binding.timing_filter(names)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            call(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = binding.kernel_times(4096)
    finally:
        binding.timing_filter(None)
    launches = [ms for name, ms in kt if name in names]
    return (t1 - t0) * 1e3 / steps, (float(np.mean(launches)) if launches else None)


def table_steps(args):
    return max(1, min(args.steps, 5))


def table_note(args):
    return ("every kernel timed with HIP events in %d calls outside the timed region, "
            "which records the roofline kernel alone" % table_steps(args))


def longest_stage(avg, stages):
    return max(stages, key=lambda k: avg.get(k, 0.0))


def stage_roofline(avg, stages, dom_ms=None):
    """Roofline of the longest single-launch stage: stages maps a timer name to
    its (algorithmic flops, algorithmic HBM bytes); the stage is priced against
    the FP64 matrix-core peak or the HBM peak, whichever its flops-to-bytes
    ratio puts it under. dom_ms: its launch time from the timed region."""
    dom = longest_stage(avg, stages)
    dom_ms = avg.get(dom) if dom_ms is None else dom_ms
    ops, nbytes = stages[dom]
    peak_f, peak_b = PEAK_TFLOPS["fp64"], PEAK_HBM_GBS
    if nbytes / (peak_b * 1e9) > ops / (peak_f * 1e12):
        ach = nbytes / (dom_ms * 1e-3) / 1e9 if dom_ms else None
        return {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": peak_b, "unit": "GB/s",
                "frac": (ach / peak_b) if ach else None, "avg_launch_ms": dom_ms,
                "bytes_per_launch": nbytes, "flops_per_launch": ops, "traffic": None}
    ach = ops / (dom_ms * 1e-3) / 1e12 if dom_ms else None
    return {"bound": "mfma", "kernel": dom, "achieved": ach, "peak": peak_f, "unit": "TFLOP/s",
            "frac": (ach / peak_f) if ach else None, "avg_launch_ms": dom_ms,
            "ops_per_launch": ops, "bytes_per_launch": nbytes, "traffic": None}


def fock_alg_work(nao, naux, nfrz, nc, na, nv):
    """Algorithmic flops and single-launch HBM bytes of the generalized Fock
    build: the two transforms of the occupied-row integrals, the metric factor
    and inverse, its triangular application, the Coulomb part (the contraction
    of the fitted density with (mu nu|P) and the AO-to-MO transform) and the
    exchange product over the auxiliary and occupied indices."""
    nmo = nfrz + nc + na + nv
    no = nfrz + nc + na
    f = {"half1": 2.0 * naux * no * nao * nao,
         "half2": 2.0 * naux * no * nao * nmo,
         "metric": 2.0 * naux ** 3 / 3.0,
         "apply": 1.0 * naux * naux * no * nmo,
         "coulomb": 2.0 * naux * nao * nao + 2.0 * nao * nao * nmo + 2.0 * nao * nmo * nmo,
         "exchange": 2.0 * naux * no * nmo * nmo}
    b = {"half1": 8.0 * (naux * nao * nao + naux * no * nao),
         "half2": 8.0 * (naux * no * nao + naux * no * nmo),
         "apply": 8.0 * (naux * naux / 2.0 + 2.0 * naux * no * nmo),
         "exchange": 8.0 * (2.0 * naux * no * nmo + nmo * nmo)}
    return sum(f.values()), f, b


def cpu_baseline_fock(g, budget_s=20.0, F_gpu=None):
    """The oracle's generalized Fock build on the whole workload (a few
    seconds at the configs' sizes; the budget is not needed), and the largest
    deviation of the device's F from it relative to max |F|."""
    from oracle import dsrg_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    t = time.perf_counter()
    ref = O.generalized_fock(g.ao3, g.J, g.C, g.h, g.gamma1, g.nfrz, g.nc, g.na)
    dt = time.perf_counter() - t
    F, _, _ = fock_alg_work(g.nao, g.naux, g.nfrz, g.nc, g.na, g.nv)
    out = {"value": F / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
           "seconds": round(dt, 3),
           "sample": f"the whole generalized Fock build (naux={g.naux}, nmo={g.C.shape[1]}; "
                     "FP64 numpy/BLAS oracle, same inputs)"}
    if F_gpu is not None:
        out["rel_err_vs_oracle"] = float(np.abs(F_gpu - ref).max() / np.abs(ref).max())
    return out


def semican_alg_work(nao, nfrz, nc, na, nv):
    """Conventional work of the semicanonical rotation: 9 n^3 per symmetric
    eigen-decomposition with eigenvectors (the usual count for reduction to
    tridiagonal form, the eigenvector iteration and the back-transformation;
    Jacobi does not have a fixed count of its own) for the core, active and
    virtual blocks, and 2 nao nmo^2 for C U."""
    nmo = nfrz + nc + na + nv
    return 9.0 * (nc ** 3 + na ** 3 + nv ** 3) + 2.0 * nao * nmo * nmo


def cpu_baseline_semican(F, shape, nao, eps_gpu=None, U_gpu=None):
    """The oracle's semicanonical rotation (numpy eigen-decompositions) of the
    same Fock matrix, and the device's largest deviations from it."""
    from oracle import dsrg_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    t = time.perf_counter()
    e_ref, U_ref = O.semicanonicalize(F, *shape)
    dt = time.perf_counter() - t
    out = {"value": semican_alg_work(nao, *shape) / dt / 1e12, "unit": "TFLOP/s",
           "cores": int(cores), "kind": "oracle", "seconds": round(dt, 4),
           "sample": "the whole rotation without C U (FP64 numpy/LAPACK oracle, same F)"}
    if eps_gpu is not None:
        out["eps_err_rel"] = float(np.abs(eps_gpu - e_ref).max() / np.abs(F).max())
        out["U_err"] = float(np.abs(U_gpu - U_ref).max())
    return out


def cpu_baseline_dfgen(g, budget_s=20.0, f_gpu=None):
    """The oracle's factor build on the first naux_s auxiliary functions,
    naux_s sized to the budget from a probe (the work is linear in naux for
    the transform, which dominates); when the sample is the whole problem, the
    largest deviation of the device's factors from it, relative to each
    block's max |B|."""
    from oracle import dsrg_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    n0 = min(g.naux, 16)
    t = time.perf_counter()
    O.df_factors(g.ao3[:n0], g.J[:n0, :n0], g.C, g.nfrz, g.nc, g.na, g.nv)
    t0 = max(time.perf_counter() - t, 1e-6)
    ns = int(min(g.naux, max(n0, n0 * budget_s / t0)))
    t = time.perf_counter()
    ref = O.df_factors(g.ao3[:ns], g.J[:ns, :ns], g.C, g.nfrz, g.nc, g.na, g.nv)
    dt = time.perf_counter() - t
    F, _ = dfgen_alg_flops(g.nao, ns, g.nc, g.na, g.nv)
    out = {"value": F / dt / 1e12, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
           "seconds": round(dt, 3),
           "sample": f"DF factor build over the first {ns}/{g.naux} auxiliary functions "
                     "(FP64 numpy/BLAS oracle, same inputs)"}
    if f_gpu is not None and ns == g.naux:
        out["rel_err_vs_oracle"] = {k: float(np.abs(f_gpu[k] - ref[k]).max() / np.abs(ref[k]).max())
                                    for k in ref if ref[k].size}
    return out


def cpu_baseline(p, budget_s=20.0):
    """Time the oracle on a bounded sample: whole terms while the budget
    allows, core pairs / core orbitals of the CCVV and CAVV loops otherwise."""
    import math
    from oracle import dsrg_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    flops_done, t_used, parts = 0.0, 0.0, []
    nc, na, nv, naux = p.nc, p.na, p.nv, p.naux
    # CCVV over the first core orbitals (pairs i <= j < nc_s)
    t = time.perf_counter()
    nc_s = nc
    while nc_s > 1 and (nc_s * (nc_s + 1) / 2) * 2.0 * naux * nv * nv / 40e9 > budget_s / 2:
        nc_s -= 1
    O.energy_ccvv(p.B_cv[:, :nc_s], p.eps_c[:nc_s], p.eps_v, p.s)
    dt = time.perf_counter() - t
    flops_done += 2.0 * naux * (nc_s * (nc_s + 1) / 2) * nv * nv
    t_used += dt
    parts.append(f"CCVV over core pairs of {nc_s}/{nc} core orbitals")
    if na > 0 and t_used < budget_s:
        # one core orbital first, to size the sample to the rest of the budget
        t = time.perf_counter()
        O.energy_cavv(p.B_cv[:, :1], p.B_av, p.eps_c[:1], p.eps_a, p.eps_v, p.gamma1, p.s)
        t1 = max(time.perf_counter() - t, 1e-6)
        m_s = max(1, min(nc, int((budget_s - t_used) / t1)))
        t = time.perf_counter()
        O.energy_cavv(p.B_cv[:, :m_s], p.B_av, p.eps_c[:m_s], p.eps_a, p.eps_v, p.gamma1, p.s)
        O.energy_ccav(p.B_cv[:, :m_s], p.B_ca[:, :m_s], p.eps_c[:m_s], p.eps_a, p.eps_v,
                      p.gamma1, p.s)
        dt = time.perf_counter() - t
        flops_done += 2.0 * naux * m_s * na * nv * nv + 2.0 * naux * m_s * m_s * na * nv
        t_used += dt
        parts.append(f"CAVV and CCAV over {m_s}/{nc} core orbitals")
    return {"value": flops_done / t_used / 1e12, "unit": "TFLOP/s", "cores": int(cores),
            "kind": "oracle", "seconds": round(t_used, 3),
            "sample": "; ".join(parts) + " (FP64 numpy/BLAS oracle, same inputs)"}


def kernel_source_sha(src):
    """sha256 over a kernel's .hip source followed by every header of the
    library source directory (sorted), so a change to shared tile code also
    marks the counters stale."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1603_00561_amd", "csrc")
    for f in [os.path.join(csrc, src)] + sorted(glob.glob(os.path.join(csrc, "*.h"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def load_traffic(kernel, workload):
    """HBM bytes per launch measured with rocprofv3 counters, if the summary
    for this kernel and workload was taken on the current kernel source."""
    f = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        d = json.load(fh)
    src = d.get("source", "")
    if not src or not os.path.exists(os.path.join(ROOT, "paper_1603_00561_amd", "csrc", src)):
        return None
    if kernel_source_sha(src) != d.get("source_sha256"):
        return None
    return d.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--grad", action="store_true",
                    help="time energy + gradient (dsrg_df_energy_backward) instead of energy")
    ap.add_argument("--active", action="store_true",
                    help="time the pieces F4-F8 of term F (dsrg_df_energy_active, FP64)")
    ap.add_argument("--dfgen", action="store_true",
                    help="time the density-fitting factor build (dsrg_df_factors, FP64) for the "
                         "orbital spaces of the config with 10 frozen core orbitals")
    ap.add_argument("--fock", action="store_true",
                    help="time the generalized Fock build (dsrg_df_fock, FP64) for the orbital "
                         "spaces of the config with 10 frozen core orbitals")
    ap.add_argument("--semican", action="store_true",
                    help="time the semicanonical rotation (dsrg_df_semicanonicalize, FP64) of the "
                         "generalized Fock matrix of the --fock workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 1 GiB elementwise copy first (known HBM bytes) so "
                         "hardware byte counters can be scaled")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only (the energy would shard over core pairs, "
              "but no multi-GPU path is built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1603_00561_amd import binding
    from paper_1603_00561_amd.workloads import make_config, CONFIGS

    if args.calibrate_copy:
        x = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        del x, y

    if args.dfgen:
        return bench_dfgen(args, binding, torch)
    if args.fock:
        return bench_fock(args, binding, torch)
    if args.semican:
        return bench_semican(args, binding, torch)
    p = make_config(args.config)
    if args.active:
        return bench_active(args, p, binding, torch)
    c = CONFIGS[args.config]
    terms = c["terms"]
    dev = torch.device("cuda:0")
    t_in = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in p.arrays()]
    nbytes = binding.workspace_size(p.nc, p.na, p.nv, p.naux, precision=args.precision,
                                    terms=list(terms))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    E = torch.empty(3, dtype=torch.float64, device=dev)

    gE = torch.tensor([1.0, 1.0, 1.0], dtype=torch.float64, device=dev)
    if args.grad:
        nbytes = binding.workspace_size(p.nc, p.na, p.nv, p.naux, precision=args.precision,
                                        terms=list(terms), with_grad=True)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        gout = {}

    def step(timing):
        if args.grad:
            g = binding.energy_backward(*t_in, p.s, gE, precision=args.precision,
                                        terms=list(terms), workspace=ws, timing=timing)
            E.copy_(g["E"])
            gout["g"] = g
        else:
            binding.energy(*t_in, p.s, precision=args.precision, terms=list(terms),
                           workspace=ws, out=E, timing=timing)

    # the kernel the roofline is taken on: the CCVV contraction, or with the
    # gradient the adjoint GEMM (2/3 of the work, several launches per step)
    if args.grad:
        if args.precision == "fp64":
            dom, unit, mult = "gemm_adj_fp64", "TFLOP/s", 1.0
            dom_names = ["gemm_adj_fp64", "gemm_adj_tb_fp64"]
        else:
            dom, unit, mult = "gemm_adj_i8", "TOP/s", SLICE_PRODUCTS
            dom_names = ["gemm_adj_i8"]
    elif args.precision == "fp64":
        dom, unit, mult = "ccvv_fp64", "TFLOP/s", 1.0
        dom_names = [dom]
    else:
        # int8 slices: SLICE_PRODUCTS exact int8 products per algorithmic multiply-add
        dom, unit, mult = "ccvv_i8", "TOP/s", SLICE_PRODUCTS
        dom_names = [dom]

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    binding.kernel_times(1)   # clear the record

    # timed region: HIP events around the roofline kernel's launches only (an
    # event pair around every kernel adds about 3 % to the energy step at
    # nc = 23, nv = 380, naux = 1100)
    binding.timing_filter(dom_names)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt_dom = binding.kernel_times(4096)
    finally:
        binding.timing_filter(None)
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    # every kernel, in a short pass after the timed region (the per-kernel table)
    for _ in range(max(1, min(args.steps, 5))):
        step(True)
    torch.cuda.synchronize()
    per_kernel = {}
    for name, ms in binding.kernel_times(4096):
        per_kernel.setdefault(name, []).append(ms)
    avg = {k: float(np.mean(v)) for k, v in per_kernel.items()}

    F, Fparts = alg_flops(p.nc, p.na, p.nv, p.naux, terms)
    if args.grad:
        # recompute (1x) plus the two adjoint contractions (2x) of every term
        F, Fparts = 3.0 * F, {k: 3.0 * v for k, v in Fparts.items()}
        Fparts = dict(Fparts)
        Fparts["ccvv"] = 2.0 / 3.0 * F
    value = F / (ms_per_step * 1e-3) / 1e12
    # per step: all launches of the roofline kernel in the timed region
    dom_ms = sum(ms for name, ms in kt_dom if name in dom_names) / args.steps if kt_dom else None
    if args.grad:
        avg[dom] = dom_ms   # the per-step total of its launches
    ach = mult * Fparts["ccvv"] / (dom_ms * 1e-3) / 1e12 if dom_ms else None
    peak = PEAK_TFLOPS[args.precision]
    roof = {"bound": "mfma", "kernel": dom, "achieved": ach, "peak": peak, "unit": unit,
            "frac": (ach / peak) if ach else None, "avg_launch_ms": dom_ms,
            "ops_per_launch": mult * Fparts["ccvv"],
            "algorithmic_tflops_per_launch": Fparts["ccvv"] / (dom_ms * 1e-3) / 1e12 if dom_ms else None,
            "traffic": load_traffic(dom, args.config)}

    Eg = E.cpu().numpy()
    err = None
    refs = os.path.join(ROOT, "tests", "golden", "oracle_refs.json")
    if os.path.exists(refs):
        r = json.load(open(refs)).get(args.config, {}).get("E_s%g" % p.s)
        if r is not None:
            err = [abs(float(a) - float(b)) for a, b in zip(Eg, r)]

    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "s_per_solve": ms_per_step * 1e-3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "i8 slices (int32 exact) + f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: nc={p.nc} na={p.na} nv={p.nv} naux={p.naux} "
                               f"s={p.s}, " + ("energy+gradient" if args.grad else "energy")
                               + " of " + "+".join(t.upper() for t in terms),
                   "precision": args.precision, "parallelism": "single-gpu"},
        "kernel_ms": avg,
        "kernel_ms_from": table_note(args),
        "E_terms": [float(x) for x in Eg],
        "abs_err_vs_oracle": err,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_budget)
    print(json.dumps(out))


def bench_active(args, p, binding, torch):
    """--active: one step = one dsrg_df_energy_active call (F4-F8, FP64)."""
    if args.precision != "fp64" or args.grad:
        print("bench.py: --active runs the FP64 energy only", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(p, k))).to(dev)
         for k in ("B_cv", "B_ca", "B_av", "B_aa", "eps_c", "eps_a", "eps_v", "gamma1")}
    F = torch.empty(5, dtype=torch.float64, device=dev)
    args_t = (t["B_cv"], t["B_ca"], t["B_av"], t["B_aa"], t["eps_c"], t["eps_a"], t["eps_v"],
              t["gamma1"], p.s)
    nbytes = binding.active_workspace_size(p.nc, p.na, p.nv, p.naux)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    call = lambda timing: binding.energy_active(*args_t, out=F, workspace=ws,  # noqa: E731
                                                timing=timing)
    for _ in range(args.warmup):
        call(False)
    torch.cuda.synchronize()
    avg = kernel_table(binding, torch, call, table_steps(args))
    dom = "cavv_fp64_x"   # the (xe|uf) producer of F4
    ms_per_step, dom_ms = timed_region(binding, torch, call, args.steps, [dom])
    Ftot, Fparts = active_alg_flops(p.nc, p.na, p.nv, p.naux)
    ach = Fparts["f4"] / (dom_ms * 1e-3) / 1e12 if dom_ms else None
    peak = PEAK_TFLOPS["fp64"]
    roof = {"bound": "mfma", "kernel": dom, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
            "frac": (ach / peak) if ach else None, "avg_launch_ms": dom_ms,
            "ops_per_launch": Fparts["f4"], "traffic": None}
    Fg = F.cpu().numpy()
    err = None
    refs = os.path.join(ROOT, "tests", "golden", "oracle_refs.json")
    if os.path.exists(refs):
        r = json.load(open(refs)).get(args.config, {}).get("F48_s%g" % p.s)
        if r is not None:
            err = [abs(float(a) - float(b)) for a, b in zip(Fg, r)]
    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": Ftot / (ms_per_step * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "s_per_solve": ms_per_step * 1e-3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: nc={p.nc} na={p.na} nv={p.nv} naux={p.naux} "
                               f"s={p.s}, energy of F4+F5+F6+F7+F8",
                   "precision": "fp64", "parallelism": "single-gpu"},
        "kernel_ms": avg,
        "kernel_ms_from": table_note(args),
        "F_terms": [float(x) for x in Fg],
        "abs_err_vs_oracle": err,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_active(p, args.cpu_budget)
    print(json.dumps(out))


def bench_dfgen(args, binding, torch):
    """--dfgen: one step = one dsrg_df_factors call (FP64)."""
    from paper_1603_00561_amd.workloads import CONFIGS, make_dfgen_problem
    if args.precision != "fp64" or args.grad or args.active:
        print("bench.py: --dfgen runs the FP64 factor build only", file=sys.stderr)
        sys.exit(2)
    c = CONFIGS[args.config]
    nfrz = 10
    g = make_dfgen_problem(nfrz, c["nc"], c["na"], c["nv"], c["naux"])
    dev = torch.device("cuda:0")
    ao3, J, C = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (g.ao3, g.J, g.C))
    nbytes = binding.df_factors_workspace_size(g.nao, g.C.shape[1], g.naux, g.nfrz, g.nc, g.na,
                                               g.nv)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    res = {}

    def call(timing):
        res["f"] = binding.df_factors(ao3, J, C, g.nfrz, g.nc, g.na, g.nv, workspace=ws,
                                      timing=timing)
    for _ in range(args.warmup):
        call(False)
    torch.cuda.synchronize()
    Ftot, Fparts = dfgen_alg_flops(g.nao, g.naux, g.nc, g.na, g.nv)
    Bparts = dfgen_alg_bytes(g.nao, g.naux, g.nc, g.na, g.nv)
    stages = {"df_half1": (Fparts["half1"], Bparts["half1"]),
              "df_half2": (Fparts["half2"], Bparts["half2"]),
              "df_metric_apply": (Fparts["apply"], Bparts["apply"])}
    avg = kernel_table(binding, torch, call, table_steps(args))
    ms_per_step, dom_ms = timed_region(binding, torch, call, args.steps,
                                       [longest_stage(avg, stages)])
    roof = stage_roofline(avg, stages, dom_ms)
    f = res["f"]
    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": Ftot / (ms_per_step * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "s_per_solve": ms_per_step * 1e-3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config} orbital spaces: nfrz={g.nfrz} nc={g.nc} na={g.na} "
                               f"nv={g.nv} nao={g.nao} naux={g.naux}, density-fitting factors",
                   "precision": "fp64", "parallelism": "single-gpu"},
        "kernel_ms": avg,
        "kernel_ms_from": table_note(args),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline_dfgen(g, args.cpu_budget, {k: v.cpu().numpy() for k, v in f.items()})
        if "rel_err_vs_oracle" in cb:
            out["rel_err_vs_oracle"] = cb.pop("rel_err_vs_oracle")
        out["cpu_baseline"] = cb
    print(json.dumps(out))



def bench_fock(args, binding, torch):
    """--fock: one step = one dsrg_df_fock call (FP64)."""
    from paper_1603_00561_amd.workloads import CONFIGS, make_fock_problem
    if args.precision != "fp64" or args.grad or args.active:
        print("bench.py: --fock runs the FP64 Fock build only", file=sys.stderr)
        sys.exit(2)
    c = CONFIGS[args.config]
    g = make_fock_problem(10, c["nc"], c["na"], c["nv"], c["naux"])
    dev = torch.device("cuda:0")
    ao3, J, C, h = (torch.from_numpy(np.ascontiguousarray(x)).to(dev)
                    for x in (g.ao3, g.J, g.C, g.h))
    g1 = torch.from_numpy(np.ascontiguousarray(g.gamma1)).to(dev) if g.na > 0 else None
    nmo = g.C.shape[1]
    nbytes = binding.df_fock_workspace_size(g.nao, nmo, g.naux, g.nfrz, g.nc, g.na, g.nv)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    call = lambda timing: binding.df_fock(ao3, J, C, h, g1, g.nfrz, g.nc, g.na, g.nv,  # noqa: E731
                                          workspace=ws, timing=timing)
    for _ in range(args.warmup):
        F = call(False)
    torch.cuda.synchronize()
    Ftot, Fp, Bp = fock_alg_work(g.nao, g.naux, g.nfrz, g.nc, g.na, g.nv)
    stages = {"fock_half1": (Fp["half1"], Bp["half1"]),
              "fock_half2": (Fp["half2"], Bp["half2"]),
              "fock_metric_apply": (Fp["apply"], Bp["apply"])}
    avg = kernel_table(binding, torch, call, table_steps(args))
    ms_per_step, dom_ms = timed_region(binding, torch, call, args.steps,
                                       [longest_stage(avg, stages)])
    roof = stage_roofline(avg, stages, dom_ms)
    F = call(False)
    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": Ftot / (ms_per_step * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "s_per_solve": ms_per_step * 1e-3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config} orbital spaces: nfrz={g.nfrz} nc={g.nc} na={g.na} "
                               f"nv={g.nv} nao={g.nao} naux={g.naux}, generalized Fock matrix",
                   "precision": "fp64", "parallelism": "single-gpu"},
        "kernel_ms": avg,
        "kernel_ms_from": table_note(args),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline_fock(g, args.cpu_budget, F.cpu().numpy())
        out["rel_err_vs_oracle"] = cb.pop("rel_err_vs_oracle")
        out["cpu_baseline"] = cb
    print(json.dumps(out))



def bench_semican(args, binding, torch):
    """--semican: one step = one dsrg_df_semicanonicalize call (FP64) on the
    generalized Fock matrix of the --fock workload, formed once on the GPU."""
    from paper_1603_00561_amd.workloads import CONFIGS, make_fock_problem
    if args.precision != "fp64" or args.grad or args.active:
        print("bench.py: --semican runs the FP64 rotation only", file=sys.stderr)
        sys.exit(2)
    c = CONFIGS[args.config]
    g = make_fock_problem(10, c["nc"], c["na"], c["nv"], c["naux"])
    dev = torch.device("cuda:0")
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    F = binding.df_fock(d(g.ao3), d(g.J), d(g.C), d(g.h), d(g.gamma1) if g.na else None, g.nfrz,
                        g.nc, g.na, g.nv)
    F = 0.5 * (F + F.T).contiguous()
    C = d(g.C)
    shape = (g.nfrz, g.nc, g.na, g.nv)
    nmo = g.C.shape[1]
    res = {}

    def call(timing):
        res["r"] = binding.semicanonicalize(F, *shape, C=C, timing=timing)
    for _ in range(args.warmup):
        call(False)
    torch.cuda.synchronize()
    avg = kernel_table(binding, torch, call, table_steps(args))
    dom = max(avg, key=avg.get)
    ms_per_step, dom_ms = timed_region(binding, torch, call, args.steps, [dom])
    eps, U, Cs = res["r"]
    work = semican_alg_work(g.nao, *shape)
    roof = {"bound": "latency", "kernel": dom, "avg_launch_ms": dom_ms,
            "note": "a chain of Jacobi rounds (three launches each); frac is the whole step's "
                    "conventional work rate against the FP64 matrix-core peak",
            "achieved": work / (ms_per_step * 1e-3) / 1e12, "peak": PEAK_TFLOPS["fp64"],
            "unit": "TFLOP/s", "frac": work / (ms_per_step * 1e-3) / 1e12 / PEAK_TFLOPS["fp64"],
            "traffic": None}
    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": work / (ms_per_step * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "s_per_solve": ms_per_step * 1e-3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config} orbital spaces: nfrz={g.nfrz} nc={g.nc} na={g.na} "
                               f"nv={g.nv} nao={g.nao}, semicanonical rotation of the generalized "
                               "Fock matrix", "precision": "fp64", "parallelism": "single-gpu"},
        "kernel_ms": avg,
        "kernel_ms_from": table_note(args),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline_semican(F.cpu().numpy(), shape, g.nao, eps.cpu().numpy(),
                                  U.cpu().numpy())
        out["eps_err_rel"] = cb.pop("eps_err_rel")
        out["U_err"] = cb.pop("U_err")
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
