"""Throughput of the DF-DSRG-MRPT2 F1-F3 hot path on one MI355X.

Default step: one dsrg_df_energy_backward call in FP64 on the largest
workload (nc=23, na=6, nv=1100, naux=3000, s=0.5: quintuple-zeta-shaped),
which recomputes the CCVV, CAVV and CCAV integral tiles, forms the three
energies and every gradient (dE/dB, dE/deps, dE/ds) through the adjoint
products, on seeded synthetic inputs already resident in HBM. The same
workload is then timed on the int8 slice path (energy + gradient, and the
energy alone for the CCVV slice kernel's rate) and reported under
"compare".

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cfg5]
                    [--precision fp64] [--energy] [--no-compare]
                    [--no-cpu-baseline]
                    [--active | --dfgen | --fock | --semican | --rest | --cd |
                     --laplace]

--energy times dsrg_df_energy alone. With --active a step is one
dsrg_df_energy_active call instead (the pieces F4-F8 of term F, FP64),
measured the same way against its own algorithmic work (the contractions
over Q that form its integrals). With --dfgen a step is one dsrg_df_factors
call (the density-fitting factors B from AO three-index integrals, FP64) for
the config's orbital spaces; with --fock one dsrg_df_fock call (the
generalized Fock matrix of Eq. gen_fock from the same DF integrals, FP64);
with --semican one dsrg_df_semicanonicalize call (the semicanonical rotation
of that Fock matrix and C U, FP64); with --rest one dsrg_df_energy_rest call
(the Table I terms A-E and G-K with the cumulants, FP64) for the config's
orbital spaces; with --cd one dsrg_df_cholesky call (the CD factors of an
s-Gaussian integral matrix of nao = 170 AO functions, the cc-pVDZ size of
C10H6, to the threshold 1e-5 Eh, FP64); with --laplace one
dsrg_df_coulomb_laplace call (the Coulomb part of E_CCVV factorized by a
16-term exponential sum of the renormalised denominator, FP64) for the
config, beside the direct CCVV energy kernel on the same inputs.

Prints one JSON line. `value` is algorithmic TFLOP/s of the whole step:
F_alg = 2 naux [nc(nc+1)/2 nv^2 + nc na nv^2 + nc^2 na nv] (the contractions
the method must perform; epilogue exponentials are not counted), times 3 for
energy + gradient, divided by the measured time per step. `roofline`
reports the dominant kernel (the adjoint products with the gradient, the
CCVV contraction for the energy) against the matrix-core peak of its
datatype, timed with HIP events on the stream it runs on. `cpu_baseline`
times the CPU oracle on a bounded sample of the same workload on this host,
on every BLAS thread and on one.
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
# upstream weights dL/dE_t of the timed gradient (those of the stored oracle
# gradient references, so the result can be checked against them)
BENCH_GE = (1.0, 0.75, -0.5)


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


def graph_replay_ms(torch, fn, steps):
    """Wall time per call when one call of fn (which only enqueues work on the
    current stream) is captured in a HIP graph (torch.cuda.CUDAGraph) and the
    graph is replayed `steps` times: the same kernels, without the host's
    per-launch work between them."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


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


def host_info():
    """CPU model, logical CPU count and the BLAS library numpy calls."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:  # pragma: no cover
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        for i in threadpool_info():
            if i.get("user_api") == "blas":
                blas = f"{i.get('internal_api')} {i.get('version')} ({i.get('threading_layer', '')})"
                break
    except Exception:  # pragma: no cover
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "blas": blas}


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()
                    if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def _sub_problem(p, nc_s):
    """The problem restricted to its first nc_s core orbitals (same active,
    virtual and auxiliary spaces)."""
    import copy
    q = copy.copy(p)
    q.nc = nc_s
    q.B_cv = np.ascontiguousarray(p.B_cv[:, :nc_s])
    q.B_ca = np.ascontiguousarray(p.B_ca[:, :nc_s])
    q.eps_c = p.eps_c[:nc_s]
    return q


def cpu_baseline(p, budget_s=20.0, grad=False):
    """Time the oracle on a bounded sample of the same workload: the problem
    restricted to its first nc_s core orbitals, nc_s sized from a one-orbital
    probe so the run takes about budget_s; energy (and, with grad, the
    analytic gradient) of all three terms. Run once on every BLAS thread and
    once on one thread (a smaller sample)."""
    from oracle import dsrg_oracle as O
    from threadpoolctl import threadpool_limits

    def work(nc_s):
        f, _ = alg_flops(nc_s, p.na, p.nv, p.naux)
        return 3.0 * f if grad else f

    def run(nc_s):
        q = _sub_problem(p, nc_s)
        t = time.perf_counter()
        O.energy_terms(q)
        if grad:
            O.gradients(q, (1.0, 1.0, 1.0))
        return time.perf_counter() - t

    def sample(budget):
        t1 = max(run(1), 1e-6)
        nc_s = 1
        while nc_s < p.nc and t1 * work(nc_s + 1) / work(1) <= budget:
            nc_s += 1
        dt = run(nc_s) if nc_s > 1 else t1
        return nc_s, dt

    what = "energy + gradient" if grad else "energy"
    nc_all, dt_all = sample(budget_s)
    cores = _blas_threads()
    with threadpool_limits(limits=1, user_api="blas"):
        nc_one, dt_one = sample(budget_s / 2)
    out = {"value": work(nc_all) / dt_all / 1e12, "unit": "TFLOP/s", "cores": int(cores),
           "kind": "oracle", "seconds": round(dt_all, 3),
           "sample": f"{what} of CCVV+CAVV+CCAV over the first {nc_all}/{p.nc} core orbitals "
                     "(all virtual, active and auxiliary functions; FP64 numpy/BLAS oracle, "
                     "same inputs)",
           "one_thread": {"value": work(nc_one) / dt_one / 1e12, "unit": "TFLOP/s", "cores": 1,
                          "seconds": round(dt_one, 3),
                          "sample": f"{what} over the first {nc_one}/{p.nc} core orbitals"}}
    out.update(host_info())
    return out


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


# launch shape of the matrix-core rate probe per kind: (workgroups, rounds);
# about 15-20 ms per launch at the quoted peaks
PROBE_LAUNCH = {"i8": (2048, 16384), "f64": (2048, 4096)}
PROBE_PEAK = {"i8": PEAK_TFLOPS["ozaki"], "f64": PEAK_TFLOPS["fp64"]}


def mfma_probe_rate(binding, torch, kind):
    """The matrix-core rate on register operands of full-entropy random bits
    (dsrg_df_mfma_probe: the operand statistics of the tile kernels without
    their memory traffic) and the shader clock it ran at. One warm-up launch,
    then one timed with events on the launch stream. The clock is the median
    over workgroups of shader cycles per constant-rate tick, times the tick
    rate (the counter's span over the launch divided by the event-timed
    length of the launch)."""
    nwg, iters = PROBE_LAUNCH[kind]
    dev = torch.device("cuda:0")
    stamps = torch.zeros(4 * nwg, dtype=torch.int64, device=dev)
    sink = torch.empty(512 * nwg, dtype=torch.int32 if kind == "i8" else torch.float64,
                       device=dev)
    binding.mfma_probe(kind, nwg, iters, stamps, sink)
    st = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    binding.mfma_probe(kind, nwg, iters, stamps, sink)
    e1.record(st)
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    s = stamps.view(nwg, 4).cpu().numpy()
    cyc, ticks = (s[:, 2] - s[:, 0]).astype(np.float64), (s[:, 3] - s[:, 1]).astype(np.float64)
    tick_hz = float(s[:, 3].max() - s[:, 1].min()) / (ms * 1e-3)
    ops = nwg * 8 * iters * 8 * binding.PROBE_OPS[kind]
    rate = ops / (ms * 1e-3) / 1e12
    return {"value": rate, "unit": "TOP/s" if kind == "i8" else "TFLOP/s",
            "clock_GHz": float(np.median(cyc / ticks)) * tick_hz / 1e9,
            "published_peak": PROBE_PEAK[kind], "frac_of_published": rate / PROBE_PEAK[kind],
            "launch": f"{nwg} workgroups x 8 waves x {iters} rounds of 8 products, {ms:.2f} ms"}


def roofline_kernel(precision, grad):
    """The kernel the roofline is taken on, the names its launches are timed
    under, its unit and the executed operations per algorithmic multiply-add.
    Energy: the CCVV contraction. Gradient: the adjoint products (2/3 of the
    work, several launches per step, summed per step)."""
    if grad:
        if precision == "fp64":
            return "gemm_adj_fp64", ["gemm_adj_fp64", "gemm_adj_tb_fp64"], "TFLOP/s", 1.0
        return "gemm_adj_i8", ["gemm_adj_i8"], "TOP/s", SLICE_PRODUCTS
    if precision == "fp64":
        return "ccvv_fp64", ["ccvv_fp64"], "TFLOP/s", 1.0
    return "ccvv_i8", ["ccvv_i8"], "TOP/s", SLICE_PRODUCTS


def run_energy_path(binding, torch, p, t_in, terms, precision, grad, steps, warmup, ntable):
    """Time `steps` calls of the energy (or energy + gradient) entry point
    after `warmup` untimed ones. HIP events surround the roofline kernel's
    launches only inside the timed region; every kernel is timed in ntable
    further calls for the per-kernel table. Returns the measurements and the
    last call's outputs (on the host)."""
    dev = t_in[0].device
    nbytes = binding.workspace_size(p.nc, p.na, p.nv, p.naux, precision=precision,
                                    terms=list(terms), with_grad=grad)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    E = torch.empty(3, dtype=torch.float64, device=dev)
    gE = torch.tensor(BENCH_GE, dtype=torch.float64, device=dev)
    out = {}

    def step(timing):
        if grad:
            g = binding.energy_backward(*t_in, p.s, gE, precision=precision, terms=list(terms),
                                        workspace=ws, timing=timing)
            E.copy_(g["E"])
            out["g"] = g
        else:
            binding.energy(*t_in, p.s, precision=precision, terms=list(terms), workspace=ws,
                           out=E, timing=timing)

    dom, dom_names, unit, mult = roofline_kernel(precision, grad)
    for _ in range(warmup):
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
        for _ in range(steps):
            step(True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt_dom = binding.kernel_times(1 << 16)
    finally:
        binding.timing_filter(None)
    ms_per_step = (t1 - t0) * 1e3 / steps
    # every kernel, in a short pass after the timed region (the per-kernel table)
    for _ in range(ntable):
        step(True)
    torch.cuda.synchronize()
    per_kernel = {}
    for name, ms in binding.kernel_times(1 << 16):
        per_kernel.setdefault(name, []).append(ms)
    avg = {k: float(np.mean(v)) for k, v in per_kernel.items()}
    launches = [ms for name, ms in kt_dom if name in dom_names]
    dom_ms = sum(launches) / steps if launches else None
    res = {"ms_per_step": ms_per_step, "dom": dom, "dom_names": dom_names, "unit": unit,
           "mult": mult, "dom_ms": dom_ms, "dom_launches_per_step": len(launches) / steps,
           "kernel_ms": avg, "workspace_bytes": int(nbytes),
           "E": E.cpu().numpy()}
    if grad:
        res["grad"] = {k: v.cpu().numpy() for k, v in out["g"].items()}
    del ws
    return res


def path_flops(p, terms, grad):
    """Algorithmic flops of one step and of the roofline kernel's share: the
    CCVV contraction for the energy; for energy + gradient the whole step is
    3 F_alg (recompute once, two adjoint contractions) and the adjoint
    products carry 2 F_alg."""
    F, parts = alg_flops(p.nc, p.na, p.nv, p.naux, terms)
    if grad:
        return 3.0 * F, 2.0 * F
    return F, parts["ccvv"]


def oracle_refs(config, s):
    refs = os.path.join(ROOT, "tests", "golden", "oracle_refs.json")
    if not os.path.exists(refs):
        return {}
    return json.load(open(refs)).get(config, {})


def energy_errors(config, s, E):
    r = oracle_refs(config, s).get("E_s%g" % s)
    if r is None:
        return None
    return [abs(float(a) - float(b)) for a, b in zip(E, r)]


def sampled_grad_error(config, g):
    """Largest deviation of the sampled dE/dB entries and of dE/deps, dE/ds from
    the oracle's (stored by the reference generator with the same upstream
    weights), relative to each output's largest oracle entry."""
    r = oracle_refs(config, None).get("grad")
    if r is None or list(r["gE"]) != list(BENCH_GE):
        return None
    ren = {"B_cv": "dB_cv", "B_ca": "dB_ca", "B_av": "dB_av", "eps_c": "deps_c",
           "eps_a": "deps_a", "eps_v": "deps_v", "s": "ds"}
    worst = 0.0
    for k in ("B_cv", "B_ca", "B_av"):
        vals = np.array([g[ren[k]][tuple(i)] for i in r[k]["idx"]])
        worst = max(worst, float(np.abs(vals - np.array(r[k]["val"])).max() / r[k]["absmax"]))
    for k in ("eps_c", "eps_a", "eps_v", "s"):
        ref = np.array(r[k])
        worst = max(worst, float(np.abs(g[ren[k]] - ref).max() / np.abs(ref).max()))
    return worst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cfg5")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--energy", action="store_true",
                    help="time the energy alone (dsrg_df_energy) instead of energy + gradient")
    ap.add_argument("--grad", action="store_true",
                    help="energy + gradient (the default; kept for older command lines)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the same workload in the other precision")
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
    ap.add_argument("--rest", action="store_true",
                    help="time the Table I terms A-E, G-K (dsrg_df_energy_rest, FP64) for the "
                         "orbital spaces of the config")
    ap.add_argument("--cd", action="store_true",
                    help="time the CD factor build (dsrg_df_cholesky, FP64) of the nao = 170 "
                         "s-Gaussian integral matrix to 1e-5 Eh")
    ap.add_argument("--laplace", action="store_true",
                    help="time the Laplace-factorized CCVV Coulomb part (dsrg_df_coulomb_laplace, "
                         "FP64) with a 16-term exponential sum")
    ap.add_argument("--cd-max-rank", type=int, default=0,
                    help="max_rank of the --cd call (default 6 nao)")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the matrix-core rate probe (dsrg_df_mfma_probe) after the "
                         "energy / gradient measurement")
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
    if args.rest:
        return bench_rest(args, binding, torch)
    if args.cd:
        return bench_cd(args, binding, torch)
    if args.laplace:
        return bench_laplace(args, binding, torch)
    p = make_config(args.config)
    if args.active:
        return bench_active(args, p, binding, torch)
    grad = not args.energy
    c = CONFIGS[args.config]
    terms = c["terms"]
    dev = torch.device("cuda:0")
    t_in = [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in p.arrays()]
    ntable = table_steps(args)

    r = run_energy_path(binding, torch, p, t_in, terms, args.precision, grad, args.steps,
                        args.warmup, ntable)
    F, Fdom = path_flops(p, terms, grad)
    value = F / (r["ms_per_step"] * 1e-3) / 1e12
    dom_ms = r["dom_ms"]
    ach = r["mult"] * Fdom / (dom_ms * 1e-3) / 1e12 if dom_ms else None
    peak = PEAK_TFLOPS[args.precision]
    if grad:
        r["kernel_ms"][r["dom"]] = dom_ms   # the per-step total of its launches
    roof = {"bound": "mfma", "kernel": r["dom"], "achieved": ach, "peak": peak, "unit": r["unit"],
            "frac": (ach / peak) if ach else None, "avg_launch_ms": dom_ms,
            "launches_per_step": r["dom_launches_per_step"],
            "ops_per_launch": r["mult"] * Fdom,
            "per_launch_note": ("the adjoint products of one step taken together: their "
                                "algorithmic flops (2 F_alg) over the summed duration of their "
                                "launches in the timed region") if grad else
                               "one launch: the CCVV contraction's algorithmic flops",
            "algorithmic_tflops_per_launch": Fdom / (dom_ms * 1e-3) / 1e12 if dom_ms else None,
            "traffic": load_traffic(r["dom"], args.config)}
    what = "energy+gradient" if grad else "energy"
    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": value, "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "s_per_solve": r["ms_per_step"] * 1e-3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "i8 slices (int32 exact) + f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: nc={p.nc} na={p.na} nv={p.nv} naux={p.naux} "
                               f"s={p.s}, {what} of " + "+".join(t.upper() for t in terms),
                   "precision": args.precision, "parallelism": "single-gpu"},
        "flops_per_step": F,
        "kernel_ms": r["kernel_ms"],
        "kernel_ms_from": table_note(args),
        "workspace_bytes": r["workspace_bytes"],
        "E_terms": [float(x) for x in r["E"]],
        "abs_err_vs_oracle": energy_errors(args.config, p.s, r["E"]),
        "roofline": roof,
    }
    if grad:
        out["grad_sampled_rel_err_vs_oracle"] = sampled_grad_error(args.config, r["grad"])

    if not args.no_compare:
        # the same workload in the other precision, and on slices the CCVV
        # energy kernel's rate against the int8 matrix-core peak
        other = "ozaki" if args.precision == "fp64" else "fp64"
        r2 = run_energy_path(binding, torch, p, t_in, terms, other, grad, args.steps,
                             args.warmup, 0)
        cmp_ = {"precision": other, "ms_per_step": r2["ms_per_step"],
                "value": F / (r2["ms_per_step"] * 1e-3) / 1e12, "unit": "TFLOP/s",
                "workspace_bytes": r2["workspace_bytes"],
                "E_terms": [float(x) for x in r2["E"]],
                "abs_err_vs_oracle": energy_errors(args.config, p.s, r2["E"])}
        split_ms = r2["ms_per_step"] if other == "ozaki" else r["ms_per_step"]
        fp64_ms = r["ms_per_step"] if other == "ozaki" else r2["ms_per_step"]
        cmp_["speedup_slices_over_fp64"] = fp64_ms / split_ms
        d_ms = r2["dom_ms"]
        if d_ms:
            a2 = r2["mult"] * Fdom / (d_ms * 1e-3) / 1e12
            cmp_["roofline"] = {"kernel": r2["dom"], "avg_launch_ms": d_ms, "achieved": a2,
                                "unit": r2["unit"], "peak": PEAK_TFLOPS[other],
                                "frac": a2 / PEAK_TFLOPS[other]}
        if grad:
            cmp_["grad_sampled_rel_err_vs_oracle"] = sampled_grad_error(args.config, r2["grad"])
        if "ozaki" in (args.precision, other):
            r3 = run_energy_path(binding, torch, p, t_in, terms, "ozaki", False, args.steps,
                                 args.warmup, 0)
            Fe, Fccvv = path_flops(p, terms, False)
            a3 = SLICE_PRODUCTS * Fccvv / (r3["dom_ms"] * 1e-3) / 1e12 if r3["dom_ms"] else None
            cmp_["slice_energy"] = {
                "ms_per_step": r3["ms_per_step"], "value": Fe / (r3["ms_per_step"] * 1e-3) / 1e12,
                "abs_err_vs_oracle": energy_errors(args.config, p.s, r3["E"]),
                "ccvv_i8": {"avg_launch_ms": r3["dom_ms"], "executed_TOPs": a3,
                            "peak": PEAK_TFLOPS["ozaki"],
                            "frac": (a3 / PEAK_TFLOPS["ozaki"]) if a3 else None}}
        out["compare"] = cmp_
    if not args.no_probe:
        # the sustained matrix-core rates of the run's box, beside the
        # published peaks the rooflines are priced against
        probe = {k: mfma_probe_rate(binding, torch, k) for k in ("f64", "i8")}
        out["mfma_probe"] = probe

        def sustained(roofline, kind):
            if roofline and roofline.get("achieved"):
                roofline["probe_rate"] = probe[kind]["value"]
                roofline["frac_of_probe_rate"] = roofline["achieved"] / probe[kind]["value"]
        sustained(roof, "f64" if args.precision == "fp64" else "i8")
        cmp_ = out.get("compare", {})
        sustained(cmp_.get("roofline"), "i8" if args.precision == "fp64" else "f64")
        ce = cmp_.get("slice_energy", {}).get("ccvv_i8")
        if ce and ce.get("executed_TOPs"):
            ce["frac_of_probe_rate"] = ce["executed_TOPs"] / probe["i8"]["value"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_budget, grad=grad)
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
        # the same call replayed from a HIP graph (about twenty launches a call)
        "graph_replay_ms_per_step": graph_replay_ms(torch, lambda: call(False), args.steps),
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
        # the same call replayed from a HIP graph (a few hundred launches a call)
        "graph_replay_ms_per_step": graph_replay_ms(torch, lambda: call(False), args.steps),
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline_semican(F.cpu().numpy(), shape, g.nao, eps.cpu().numpy(),
                                  U.cpu().numpy())
        out["eps_err_rel"] = cb.pop("eps_err_rel")
        out["U_err"] = cb.pop("U_err")
        out["cpu_baseline"] = cb
    print(json.dumps(out))



def rest_alg_work(nc, na, nv, naux):
    """Algorithmic flops and HBM bytes of the integral stage of the Table I
    terms: the seven products over the auxiliary index that form (pq|rs)
    with two or more active indices. The three Gram products (uv|wx),
    (mu|nv) and (xe|yf) are symmetric, so their unique entries, n (n + 1) / 2
    of them, count (the largest, (xe|yf), reads B_av twice and writes its
    na^2 nv^2 values)."""
    na2 = na * na
    prods = [(nc * nv, na2), (na * nv, na2), (nc * na, na2), (na * nv, nc * na)]
    grams = [na2, nc * na, na * nv]
    flops = (sum(2.0 * naux * m * n for m, n in prods)
             + sum(2.0 * naux * n * (n + 1) / 2 for n in grams))
    nbytes = (sum(8.0 * (naux * (m + n) + m * n) for m, n in prods)
              + sum(8.0 * (2 * naux * n + n * n) for n in grams))
    return flops, nbytes


def bench_rest(args, binding, torch):
    """--rest: one step = one dsrg_df_energy_rest call (Table I terms A-E,
    G-K, FP64) on make_rest_problem inputs of the config's orbital spaces."""
    from paper_1603_00561_amd.workloads import CONFIGS, make_rest_problem
    if args.precision != "fp64" or args.grad or args.active:
        print("bench.py: --rest runs the FP64 energy only", file=sys.stderr)
        sys.exit(2)
    c = CONFIGS[args.config]
    p = make_rest_problem(c["nc"], c["na"], c["nv"], c["naux"], s=c["s"])
    dev = torch.device("cuda:0")
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    l2, l3 = binding.cumulants(d(p.rdm1), d(p.rdm2), d(p.rdm3))
    t = [d(x) for x in (p.B_cv, p.B_ca, p.B_av, p.B_aa, p.eps_c, p.eps_a, p.eps_v, p.f_ca,
                        p.f_cv, p.f_av, p.rdm1)]
    nbytes = binding.rest_workspace_size(p.nc, p.na, p.nv, p.naux)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    res = {}

    def call(timing):
        res["T"] = binding.energy_rest(*t, l2, l3, p.s, workspace=ws, timing=timing)
    for _ in range(args.warmup):
        call(False)
    torch.cuda.synchronize()
    avg = kernel_table(binding, torch, call, table_steps(args))
    flops, nb = rest_alg_work(p.nc, p.na, p.nv, p.naux)
    stages = {"rest_integrals": (flops, nb)}
    ms_per_step, dom_ms = timed_region(binding, torch, call, args.steps, ["rest_integrals"])
    roof = stage_roofline(avg, stages, dom_ms)
    T = res["T"].cpu().numpy()
    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": flops / (ms_per_step * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "s_per_solve": ms_per_step * 1e-3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config} orbital spaces: nc={p.nc} na={p.na} nv={p.nv} "
                               f"naux={p.naux} s={p.s}, Table I terms A-E and G-K "
                               "(value counts the integral products only)",
                   "precision": "fp64", "parallelism": "single-gpu"},
        "terms": dict(zip(binding.REST_TERMS, [float(x) for x in T])),
        "kernel_ms": avg,
        "kernel_ms_from": table_note(args),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        from oracle import dsrg_table1 as OT
        cores = _blas_threads()
        t0 = time.perf_counter()
        ref = OT.rest_terms(p)
        dt = time.perf_counter() - t0
        refv = np.array([ref[k] for k in binding.REST_TERMS])
        out["abs_err_vs_oracle"] = [float(x) for x in np.abs(T - refv)]
        out["cpu_baseline"] = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores,
                               "kind": "oracle", "seconds": dt,
                               "sample": "the whole workload (spin-orbital blocked oracle, "
                                         "numpy on every BLAS thread)",
                               "host": host_info()}
    print(json.dumps(out))


def cd_alg_bytes(npair, rank):
    """Algorithmic HBM bytes of the rank step launches of the CD build: step k
    reads the k earlier vectors on every pair and the pivot's integral row,
    reads and writes the residual diagonal, and writes its vector unpacked
    (both triangles): (k + 5) npair doubles."""
    return 8.0 * npair * (rank * (rank - 1) / 2.0 + 5.0 * rank)


def bench_cd(args, binding, torch):
    """--cd: one step = one dsrg_df_cholesky call (FP64) on the s-Gaussian
    integral matrix of make_cd_problem (nao = 170) to the threshold 1e-5."""
    from paper_1603_00561_amd.workloads import make_cd_problem
    if args.precision != "fp64" or args.grad or args.active:
        print("bench.py: --cd runs the FP64 factor build only", file=sys.stderr)
        sys.exit(2)
    tol = 1e-5
    p = make_cd_problem()
    nao, npair = p.nao, p.M.shape[0]
    max_rank = args.cd_max_rank or 6 * nao
    dev = torch.device("cuda:0")
    M = torch.from_numpy(p.M).to(dev)
    ws = torch.empty(binding.cholesky_workspace_size(nao, max_rank, tol), dtype=torch.uint8,
                     device=dev)
    res = {}

    def call(timing):
        res["r"] = binding.cholesky(M, nao, tol, max_rank, workspace=ws, timing=timing,
                                    sync=False)
    for _ in range(args.warmup):
        call(False)
    torch.cuda.synchronize()
    avg = kernel_table(binding, torch, call, table_steps(args))
    ms_per_step, dom_ms = timed_region(binding, torch, call, args.steps, ["cd_step"])
    rank = int(res["r"]["rank_t"].item())
    dmax = float(res["r"]["dmax_t"].item())
    flops = 2.0 * npair * rank * (rank - 1) / 2.0      # the products against earlier vectors
    nbytes = cd_alg_bytes(npair, rank)
    ach = nbytes / (dom_ms * 1e-3) / 1e9 if dom_ms else None
    roof = {"bound": "hbm", "kernel": "cd_step", "achieved": ach, "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": (ach / PEAK_HBM_GBS) if ach else None,
            "avg_launch_ms": dom_ms,
            "note": "cd_step is the sequence of max_rank step launches of one call (one timer "
                    "pair around them); bytes are those of the rank steps that do work",
            "bytes_per_launch": nbytes, "traffic": None}
    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": flops / (ms_per_step * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "s_per_solve": ms_per_step * 1e-3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"CD of (mu nu|la si): nao={nao} (npair={npair}) s-Gaussian "
                               f"functions, threshold {tol:g} Eh, max_rank={max_rank}",
                   "precision": "fp64", "parallelism": "single-gpu"},
        "rank": rank, "dmax": dmax,
        "kernel_ms": avg,
        "kernel_ms_from": table_note(args),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        from oracle import dsrg_oracle as O
        from scipy.linalg import lapack
        cores = _blas_threads()
        t0 = time.perf_counter()
        L, piv, dm = O.pivoted_cholesky_steps(p.M, tol, max_rank)
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, pvt, lrank, _ = lapack.dpstrf(p.M.copy(), lower=1, tol=tol)
        dl = time.perf_counter() - t0
        out["pivots_equal_oracle"] = bool(
            np.array_equal(res["r"]["pivots_full"][:rank].cpu().numpy(), piv))
        out["cpu_baseline"] = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores,
                               "kind": "oracle", "seconds": dt, "rank": int(L.shape[1]),
                               "sample": "the whole workload (greedy pivoted Cholesky, one "
                                         "numpy vector update per earlier vector)",
                               "host": host_info()}
        out["cpu_lapack_dpstrf"] = {"seconds": dl, "rank": int(lrank), "cores": cores}
    print(json.dumps(out))



def bench_laplace(args, binding, torch):
    """--laplace: one step = one dsrg_df_coulomb_laplace call (FP64) with the
    library's 16-term fit for the config's orbital energies; the direct FP64
    CCVV energy (Coulomb and exchange, fifth order) is timed beside it."""
    from paper_1603_00561_amd.workloads import make_config
    if args.precision != "fp64" or args.grad or args.active:
        print("bench.py: --laplace runs FP64 only", file=sys.stderr)
        sys.exit(2)
    nq = 16
    p = make_config(args.config)
    dev = torch.device("cuda:0")
    d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)  # noqa: E731
    Bcv, ec, ev = d(p.B_cv), d(p.eps_c), d(p.eps_v)
    lo = 2.0 * (float(p.eps_v.min()) - float(p.eps_c.max()))
    hi = 2.0 * (float(p.eps_v.max()) - float(p.eps_c.min()))
    t, w, fit_err = binding.laplace_fit(p.s, lo, hi, nq)
    ws = torch.empty(binding.laplace_workspace_size(p.nc, p.nv, p.naux, nq), dtype=torch.uint8,
                     device=dev)
    res = {}

    def call(timing):
        res["r"] = binding.coulomb_laplace(Bcv, ec, ev, t, w, workspace=ws, timing=timing)
    for _ in range(args.warmup):
        call(False)
    torch.cuda.synchronize()
    # launches of the batched product per call (the terms run in batches)
    binding.kernel_times(1)
    call(True)
    torch.cuda.synchronize()
    gemm_launches = sum(1 for n, _ in binding.kernel_times(4096) if n == "lt_gemm")
    avg = kernel_table(binding, torch, call, table_steps(args))
    ms_per_step, dom_ms = timed_region(binding, torch, call, args.steps, ["lt_gemm"])
    E = float(res["r"][0].item())
    # Y_k is a symmetric Gram matrix: its naux (naux + 1) / 2 unique entries
    flops = 1.0 * p.naux * (p.naux + 1) * p.nc * p.nv * nq
    gemm_ms = dom_ms * gemm_launches if dom_ms else None
    ach = flops / (gemm_ms * 1e-3) / 1e12 if gemm_ms else None
    # the direct CCVV energy on the same inputs (Coulomb and exchange)
    t_in = {k: d(getattr(p, k)) for k in ("B_cv", "B_ca", "B_av", "eps_c", "eps_a", "eps_v",
                                          "gamma1")}

    def direct():
        return binding.energy(t_in["B_cv"], t_in["B_ca"], t_in["B_av"], t_in["eps_c"],
                              t_in["eps_a"], t_in["eps_v"], t_in["gamma1"], p.s, terms="ccvv")
    direct()
    torch.cuda.synchronize()
    nd = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(nd):
        Ed = direct()
    torch.cuda.synchronize()
    direct_ms = (time.perf_counter() - t0) * 1e3 / nd
    out = {
        "metric": "DF-DSRG-MRPT2 energy(+grad) TFLOP/s & s/solve, FP64 vs split-BF16 @1µEh",
        "value": flops / (ms_per_step * 1e-3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "s_per_solve": ms_per_step * 1e-3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: nc={p.nc} nv={p.nv} naux={p.naux} s={p.s}, "
                               f"Coulomb part of E_CCVV factorized with {nq} exponential-sum "
                               "terms", "precision": "fp64", "parallelism": "single-gpu"},
        "E_J_laplace": E, "fit_max_err": fit_err, "x_range": [lo, hi],
        "direct_ccvv_energy_ms": direct_ms, "E_CCVV_direct": float(Ed[0].item()),
        "kernel_ms": avg, "kernel_ms_from": table_note(args),
        "roofline": {"bound": "mfma", "kernel": "lt_gemm", "avg_launch_ms": dom_ms,
                     "launches_per_call": gemm_launches, "achieved": ach,
                     "peak": PEAK_TFLOPS["fp64"], "unit": "TFLOP/s",
                     "frac": (ach / PEAK_TFLOPS["fp64"]) if ach else None,
                     "flops_per_call": flops, "traffic": None},
    }
    ref_path = os.path.join(ROOT, "tests", "golden", "oracle_refs.json")
    if os.path.exists(ref_path):
        r = json.load(open(ref_path)).get(args.config, {}).get("laplace_nq16")
        if r is not None:
            out["rel_err_vs_exact_coulomb"] = abs(E - r["E_J"]) / abs(r["E_J"])
    if not args.no_cpu_baseline:
        from oracle import dsrg_laplace as L
        cores = _blas_threads()
        t0 = time.perf_counter()
        e_ref, _ = L.coulomb_laplace(p.B_cv, p.eps_c, p.eps_v, t, w)
        dt = time.perf_counter() - t0
        out["abs_err_vs_oracle"] = abs(E - e_ref)
        out["cpu_baseline"] = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cores,
                               "kind": "oracle", "seconds": dt,
                               "sample": "the whole workload (factorized form in numpy, BLAS "
                                         "on every thread)", "host": host_info()}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
