"""Thin Python binding of libdsrgdf (ctypes).

Argument marshalling only: every step of the computation runs in the HIP
library. PyTorch supplies device memory and the current stream. There is no
CPU fallback; if the library is missing this module raises on first use.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Union

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsrgdf.so")

DSRG_OK, DSRG_ERR_ARG, DSRG_ERR_UNSUPPORTED, DSRG_ERR_WORKSPACE, DSRG_ERR_HIP = range(5)
PRECISIONS = {"fp64": 0, "split_bf16": 1, "ozaki": 2}
TERM_BITS = {"ccvv": 1, "cavv": 2, "ccav": 4}
TERM_ALL = 7
OPT_ATOMIC_REDUCE = 0x100
OPT_KERNEL_TIMING = 0x200
OPT_CHECK_SIGNS = 0x400
MAX_ACTIVE = 8

EXPORTED = ("dsrg_df_workspace_size", "dsrg_df_energy", "dsrg_df_energy_noalloc",
            "dsrg_df_energy_backward",
            "dsrg_df_active_workspace_size", "dsrg_df_energy_active",
            "dsrg_df_factors_workspace_size", "dsrg_df_factors",
            "dsrg_df_fock_workspace_size", "dsrg_df_fock",
            "dsrg_df_semicanonicalize_workspace_size", "dsrg_df_semicanonicalize",
            "dsrg_df_last_error", "dsrg_df_kernel_times", "dsrg_df_timing_filter",
            "dsrg_df_set_gradient_block_bytes", "dsrg_df_gradient_block_bytes",
            "dsrg_df_rest_workspace_size", "dsrg_df_energy_rest", "dsrg_df_cumulants",
            "dsrg_df_cholesky_workspace_size", "dsrg_df_cholesky",
            "dsrg_df_laplace_fit", "dsrg_df_laplace_workspace_size", "dsrg_df_coulomb_laplace",
            "dsrg_df_sign_check", "dsrg_df_mfma_probe", "dsrg_df_version")


class DsrgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libdsrgdf status {status}: {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("nc", ctypes.c_int64), ("na", ctypes.c_int64), ("nv", ctypes.c_int64),
        ("naux", ctypes.c_int64),
        ("B_cv", ctypes.c_void_p), ("B_ca", ctypes.c_void_p), ("B_av", ctypes.c_void_p),
        ("eps_c", ctypes.c_void_p), ("eps_a", ctypes.c_void_p), ("eps_v", ctypes.c_void_p),
        ("gamma1", ctypes.c_void_p),
        ("s", ctypes.c_double),
    ]


class RestProblem(ctypes.Structure):
    _fields_ = [("base", Problem), ("B_aa", ctypes.c_void_p), ("f_ca", ctypes.c_void_p),
                ("f_cv", ctypes.c_void_p), ("f_av", ctypes.c_void_p), ("rdm1", ctypes.c_void_p),
                ("lambda2", ctypes.c_void_p), ("lambda3", ctypes.c_void_p)]


REST_TERMS = ("A", "B", "C", "D", "E", "G", "H", "I", "J", "K")


class DFGenProblem(ctypes.Structure):
    _fields_ = [
        ("nao", ctypes.c_int64), ("nmo", ctypes.c_int64), ("naux", ctypes.c_int64),
        ("nfrz", ctypes.c_int64), ("nc", ctypes.c_int64), ("na", ctypes.c_int64),
        ("nv", ctypes.c_int64),
        ("ao3", ctypes.c_void_p), ("J", ctypes.c_void_p), ("C", ctypes.c_void_p),
    ]


class CDProblem(ctypes.Structure):
    _fields_ = [("nao", ctypes.c_int64), ("M", ctypes.c_void_p), ("tol", ctypes.c_double),
                ("max_rank", ctypes.c_int64)]


class FockProblem(ctypes.Structure):
    _fields_ = [("df", DFGenProblem), ("h", ctypes.c_void_p), ("gamma1", ctypes.c_void_p)]


class SemicanProblem(ctypes.Structure):
    _fields_ = [
        ("nao", ctypes.c_int64), ("nmo", ctypes.c_int64), ("nfrz", ctypes.c_int64),
        ("nc", ctypes.c_int64), ("na", ctypes.c_int64), ("nv", ctypes.c_int64),
        ("F", ctypes.c_void_p), ("C", ctypes.c_void_p),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdsrgdf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libdsrgdf.so not found at {path}; build it first "
            "(python -m paper_1603_00561_amd.build)")
    lib = ctypes.CDLL(path)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    lib.dsrg_df_workspace_size.argtypes = [ctypes.POINTER(Problem), i32, i32, i32,
                                           ctypes.POINTER(sz)]
    lib.dsrg_df_workspace_size.restype = i32
    lib.dsrg_df_energy.argtypes = [ctypes.POINTER(Problem), i32, i32, vp, vp, sz, vp]
    lib.dsrg_df_energy.restype = i32
    lib.dsrg_df_energy_noalloc.argtypes = [ctypes.POINTER(Problem), i32, i32, vp, vp]
    lib.dsrg_df_energy_noalloc.restype = i32
    lib.dsrg_df_sign_check.argtypes = [ctypes.POINTER(ctypes.c_uint)]
    lib.dsrg_df_sign_check.restype = i32
    lib.dsrg_df_mfma_probe.argtypes = [i32, ctypes.c_int64, ctypes.c_int64, vp, vp, vp]
    lib.dsrg_df_mfma_probe.restype = i32
    lib.dsrg_df_energy_backward.argtypes = [ctypes.POINTER(Problem), i32, i32, vp,
                                            vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.dsrg_df_energy_backward.restype = i32
    lib.dsrg_df_active_workspace_size.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(sz)]
    lib.dsrg_df_active_workspace_size.restype = i32
    lib.dsrg_df_energy_active.argtypes = [ctypes.POINTER(Problem), vp, i32, vp, vp, sz, vp]
    lib.dsrg_df_energy_active.restype = i32
    lib.dsrg_df_factors_workspace_size.argtypes = [ctypes.POINTER(DFGenProblem),
                                                   ctypes.POINTER(sz)]
    lib.dsrg_df_factors_workspace_size.restype = i32
    lib.dsrg_df_factors.argtypes = [ctypes.POINTER(DFGenProblem), i32, vp, vp, vp, vp, vp, sz,
                                    vp]
    lib.dsrg_df_factors.restype = i32
    lib.dsrg_df_fock_workspace_size.argtypes = [ctypes.POINTER(FockProblem), ctypes.POINTER(sz)]
    lib.dsrg_df_fock_workspace_size.restype = i32
    lib.dsrg_df_fock.argtypes = [ctypes.POINTER(FockProblem), i32, vp, vp, sz, vp]
    lib.dsrg_df_fock.restype = i32
    lib.dsrg_df_semicanonicalize_workspace_size.argtypes = [ctypes.POINTER(SemicanProblem),
                                                            ctypes.POINTER(sz)]
    lib.dsrg_df_semicanonicalize_workspace_size.restype = i32
    lib.dsrg_df_semicanonicalize.argtypes = [ctypes.POINTER(SemicanProblem), i32, vp, vp, vp, vp,
                                             vp, sz, vp]
    lib.dsrg_df_semicanonicalize.restype = i32
    lib.dsrg_df_last_error.argtypes = []
    lib.dsrg_df_last_error.restype = ctypes.c_char_p
    lib.dsrg_df_kernel_times.argtypes = [ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_char_p), i32]
    lib.dsrg_df_kernel_times.restype = i32
    lib.dsrg_df_timing_filter.argtypes = [ctypes.c_char_p]
    lib.dsrg_df_timing_filter.restype = i32
    lib.dsrg_df_rest_workspace_size.argtypes = [ctypes.POINTER(RestProblem), ctypes.POINTER(sz)]
    lib.dsrg_df_rest_workspace_size.restype = i32
    lib.dsrg_df_energy_rest.argtypes = [ctypes.POINTER(RestProblem), i32, vp, vp, sz, vp]
    lib.dsrg_df_energy_rest.restype = i32
    lib.dsrg_df_cumulants.argtypes = [ctypes.c_int64, vp, vp, vp, vp, vp, vp]
    lib.dsrg_df_cumulants.restype = i32
    lib.dsrg_df_set_gradient_block_bytes.argtypes = [sz]
    lib.dsrg_df_set_gradient_block_bytes.restype = i32
    lib.dsrg_df_gradient_block_bytes.argtypes = []
    lib.dsrg_df_gradient_block_bytes.restype = sz
    lib.dsrg_df_cholesky_workspace_size.argtypes = [ctypes.POINTER(CDProblem),
                                                    ctypes.POINTER(sz)]
    lib.dsrg_df_cholesky_workspace_size.restype = i32
    lib.dsrg_df_cholesky.argtypes = [ctypes.POINTER(CDProblem), i32, vp, vp, vp, vp, vp, sz, vp]
    lib.dsrg_df_cholesky.restype = i32
    dp = ctypes.POINTER(ctypes.c_double)
    lib.dsrg_df_laplace_fit.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, i32,
                                        dp, dp, dp]
    lib.dsrg_df_laplace_fit.restype = i32
    lib.dsrg_df_laplace_workspace_size.argtypes = [ctypes.POINTER(Problem), i32,
                                                   ctypes.POINTER(sz)]
    lib.dsrg_df_laplace_workspace_size.restype = i32
    lib.dsrg_df_coulomb_laplace.argtypes = [ctypes.POINTER(Problem), i32, dp, dp, i32, vp, vp, vp,
                                            sz, vp]
    lib.dsrg_df_coulomb_laplace.restype = i32
    lib.dsrg_df_version.argtypes = []
    lib.dsrg_df_version.restype = i32
    _lib = lib
    return lib


def _check(status: int):
    if status != DSRG_OK:
        msg = load_library().dsrg_df_last_error().decode(errors="replace")
        raise DsrgError(status, msg)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def kernel_times(cap: int = 32):
    """[(kernel name, ms)] of the last call made with timing=True on this
    thread (waits for that work to finish)."""
    lib = load_library()
    ms = (ctypes.c_double * cap)()
    names = (ctypes.c_char_p * cap)()
    n = lib.dsrg_df_kernel_times(ms, names, cap)
    if n < 0:
        raise DsrgError(DSRG_ERR_HIP, "could not read kernel timing events")
    return [(names[k].decode(), ms[k]) for k in range(min(n, cap))]


def timing_filter(names: Optional[Sequence[str]] = None) -> None:
    """Record only the named kernels (names as kernel_times reports them) in
    later calls made with timing=True on this thread; None or () records
    every kernel again."""
    lib = load_library()
    arg = ",".join(names).encode() if names else None
    st = lib.dsrg_df_timing_filter(arg)
    if st != 0:
        raise DsrgError(st, lib.dsrg_df_last_error().decode())


def set_gradient_block_bytes(nbytes: int = 0) -> int:
    """Bound the gradient's per-block adjoint-tile region (0 = the default);
    returns the bound that was in force before."""
    lib = load_library()
    old = int(lib.dsrg_df_gradient_block_bytes())
    st = lib.dsrg_df_set_gradient_block_bytes(int(nbytes))
    if st != 0:
        raise DsrgError(st, lib.dsrg_df_last_error().decode())
    return old


def _terms_mask(terms: Union[str, int, Sequence[str]], atomic: bool, timing: bool = False) -> int:
    if isinstance(terms, int):
        m = terms
    elif terms == "all":
        m = TERM_ALL
    elif isinstance(terms, str):
        m = TERM_BITS[terms]
    else:
        m = 0
        for t in terms:
            m |= TERM_BITS[t]
    return m | (OPT_ATOMIC_REDUCE if atomic else 0) | (OPT_KERNEL_TIMING if timing else 0)


def _as_dev(t: Optional[torch.Tensor], name: str, shape, device) -> Optional[torch.Tensor]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on the GPU (got {t.device}); there is no CPU path")
    if t.dtype != torch.float64:
        raise ValueError(f"{name} must be float64 (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t.contiguous()


def make_problem_struct(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s):
    """Validate tensors and fill the C problem struct. Returns (struct, kept
    tensors) so the caller keeps the contiguous copies alive."""
    naux, nc, nv = B_cv.shape
    na = 0 if B_ca is None else B_ca.shape[2]
    dev = B_cv.device
    keep = [
        _as_dev(B_cv, "B_cv", (naux, nc, nv), dev),
        _as_dev(B_ca, "B_ca", (naux, nc, na), dev) if na else None,
        _as_dev(B_av, "B_av", (naux, na, nv), dev) if na else None,
        _as_dev(eps_c, "eps_c", (nc,), dev),
        _as_dev(eps_a, "eps_a", (na,), dev) if na else None,
        _as_dev(eps_v, "eps_v", (nv,), dev),
        _as_dev(gamma1, "gamma1", (na, na), dev) if na else None,
    ]
    p = Problem(nc, na, nv, naux, *[_ptr(t) for t in keep], float(s))
    return p, keep


def workspace_size(nc, na, nv, naux, precision="fp64", terms="all", with_grad=False,
                   atomic=False) -> int:
    lib = load_library()
    p = Problem(nc, na, nv, naux, None, None, None, None, None, None, None, 0.5)
    out = ctypes.c_size_t(0)
    _check(lib.dsrg_df_workspace_size(ctypes.byref(p), PRECISIONS[precision],
                                      _terms_mask(terms, atomic), int(bool(with_grad)),
                                      ctypes.byref(out)))
    return out.value


def active_workspace_size(nc, na, nv, naux) -> int:
    """Workspace bytes of dsrg_df_energy_active for these sizes."""
    lib = load_library()
    p = Problem(nc, na, nv, naux, None, None, None, None, None, None, None, 0.5)
    out = ctypes.c_size_t(0)
    _check(lib.dsrg_df_active_workspace_size(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _workspace(nbytes: int, device, workspace: Optional[torch.Tensor]) -> torch.Tensor:
    if workspace is not None:
        if workspace.device != device or workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError("workspace is too small or on the wrong device")
        return workspace
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def energy(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s, precision="fp64",
           terms="all", atomic=False, workspace: Optional[torch.Tensor] = None,
           timing: bool = False, out: Optional[torch.Tensor] = None,
           check_signs: bool = False) -> torch.Tensor:
    """E_CCVV, E_CAVV, E_CCAV (device tensor [3], float64) via dsrg_df_energy
    (check_signs: DSRG_OPT_CHECK_SIGNS, read with sign_check())."""
    lib = load_library()
    p, keep = make_problem_struct(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s)
    dev = B_cv.device
    mask = _terms_mask(terms, atomic, timing) | (OPT_CHECK_SIGNS if check_signs else 0)
    prec = PRECISIONS[precision]
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_workspace_size(ctypes.byref(p), prec, mask, 0, ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    E = torch.empty(3, dtype=torch.float64, device=dev) if out is None else out
    _check(lib.dsrg_df_energy(ctypes.byref(p), prec, mask, E.data_ptr(), ws.data_ptr(),
                              nbytes.value, _stream_handle(dev)))
    del keep
    return E


def energy_noalloc(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s, precision="fp64",
                   terms="all", atomic=False, out: Optional[torch.Tensor] = None,
                   check_signs: bool = False) -> torch.Tensor:
    """E_CCVV, E_CAVV, E_CCAV via dsrg_df_energy_noalloc (the library's static
    device scratch instead of a workspace; out, when given, is written in place)."""
    lib = load_library()
    p, keep = make_problem_struct(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s)
    dev = B_cv.device
    mask = _terms_mask(terms, atomic, False) | (OPT_CHECK_SIGNS if check_signs else 0)
    E = torch.empty(3, dtype=torch.float64, device=dev) if out is None else out
    _check(lib.dsrg_df_energy_noalloc(ctypes.byref(p), PRECISIONS[precision], mask, E.data_ptr(),
                                      _stream_handle(dev)))
    del keep
    return E


def sign_check() -> int:
    """The current device's sign check word via dsrg_df_sign_check (waits for
    the device; bit 0: a CCVV work item of a call with check_signs gave a
    positive or NaN contribution since the last read), then cleared."""
    lib = load_library()
    w = ctypes.c_uint(0)
    _check(lib.dsrg_df_sign_check(ctypes.byref(w)))
    return int(w.value)


PROBE_KINDS = {"i8": 0, "f64": 1}   # DSRG_PROBE_I8, DSRG_PROBE_F64
PROBE_OPS = {"i8": 65536, "f64": 2048}   # operations per matrix product


def mfma_probe(kind: str, nwg: int, iters: int, stamps: torch.Tensor, sink: torch.Tensor):
    """Enqueues the matrix-core rate probe (dsrg_df_mfma_probe) on the current
    stream of stamps' device: nwg workgroups of eight waves, iters rounds of
    eight products per wave (nwg * 8 * iters * 8 * PROBE_OPS[kind]
    operations). stamps: int64 [4 nwg] (per workgroup: cycle and constant-rate
    counters before, then after its products); sink: nwg * 512 int32 (i8) or
    float64 (f64) values."""
    lib = load_library()
    want = torch.int32 if kind == "i8" else torch.float64
    if stamps.dtype != torch.int64 or stamps.numel() < 4 * nwg or not stamps.is_cuda:
        raise ValueError("stamps must be a device int64 tensor of 4 nwg entries")
    if sink.dtype != want or sink.numel() < 512 * nwg or sink.device != stamps.device:
        raise ValueError("sink must be a device tensor of nwg * 512 entries of the kind's type")
    _check(lib.dsrg_df_mfma_probe(PROBE_KINDS[kind], nwg, iters, stamps.data_ptr(),
                                  sink.data_ptr(), _stream_handle(stamps.device)))


def cumulants(rdm1, rdm2, rdm3):
    """(lambda2, lambda3) device tensors from the active spin-orbital reduced
    density matrices (device float64 tensors [n]^2, [n]^4, [n]^6, n = 2 na)
    via dsrg_df_cumulants."""
    lib = load_library()
    n = rdm1.shape[0]
    dev = rdm1.device
    g1 = _as_dev(rdm1, "rdm1", (n, n), dev)
    g2 = _as_dev(rdm2, "rdm2", (n,) * 4, dev)
    g3 = _as_dev(rdm3, "rdm3", (n,) * 6, dev)
    l2 = torch.empty((n,) * 4, dtype=torch.float64, device=dev)
    l3 = torch.empty((n,) * 6, dtype=torch.float64, device=dev)
    _check(lib.dsrg_df_cumulants(n // 2, g1.data_ptr(), g2.data_ptr(), g3.data_ptr(),
                                 l2.data_ptr(), l3.data_ptr(), _stream_handle(dev)))
    return l2, l3


def rest_problem_struct(B_cv, B_ca, B_av, B_aa, eps_c, eps_a, eps_v, f_ca, f_cv, f_av, rdm1,
                        lambda2, lambda3, s):
    naux, nc, nv = B_cv.shape
    na = 0 if B_ca is None else B_ca.shape[2]
    dev = B_cv.device
    base, keep = make_problem_struct(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, None, s)
    n = 2 * na
    extra = [
        _as_dev(B_aa, "B_aa", (naux, na, na), dev) if na else None,
        _as_dev(f_ca, "f_ca", (nc, na), dev) if na else None,
        _as_dev(f_cv, "f_cv", (nc, nv), dev) if na else None,
        _as_dev(f_av, "f_av", (na, nv), dev) if na else None,
        _as_dev(rdm1, "rdm1", (n, n), dev) if na else None,
        _as_dev(lambda2, "lambda2", (n,) * 4, dev) if na else None,
        _as_dev(lambda3, "lambda3", (n,) * 6, dev) if na else None,
    ]
    return RestProblem(base, *[_ptr(t) for t in extra]), keep + extra


def energy_rest(B_cv, B_ca, B_av, B_aa, eps_c, eps_a, eps_v, f_ca, f_cv, f_av, rdm1, lambda2,
                lambda3, s, workspace: Optional[torch.Tensor] = None, timing: bool = False,
                out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Table I terms A, B, C, D, E, G, H, I, J, K (device tensor [10], float64)
    via dsrg_df_energy_rest."""
    lib = load_library()
    p, keep = rest_problem_struct(B_cv, B_ca, B_av, B_aa, eps_c, eps_a, eps_v, f_ca, f_cv, f_av,
                                  rdm1, lambda2, lambda3, s)
    dev = B_cv.device
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_rest_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    T = torch.empty(10, dtype=torch.float64, device=dev) if out is None else out
    _check(lib.dsrg_df_energy_rest(ctypes.byref(p), OPT_KERNEL_TIMING if timing else 0,
                                   T.data_ptr(), ws.data_ptr(), nbytes.value,
                                   _stream_handle(dev)))
    del keep
    return T


def rest_workspace_size(nc, na, nv, naux) -> int:
    lib = load_library()
    base = Problem(nc, na, nv, naux, None, None, None, None, None, None, None, 0.5)
    p = RestProblem(base, None, None, None, None, None, None, None)
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_rest_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)))
    return int(nbytes.value)


def energy_active(B_cv, B_ca, B_av, B_aa, eps_c, eps_a, eps_v, gamma1, s,
                  workspace: Optional[torch.Tensor] = None, timing: bool = False,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """F4..F8 of term F (device tensor [5], float64) via dsrg_df_energy_active."""
    lib = load_library()
    p, keep = make_problem_struct(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s)
    dev = B_cv.device
    na = int(p.na)
    baa = _as_dev(B_aa, "B_aa", (int(p.naux), na, na), dev) if na else None
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_active_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    F = torch.empty(5, dtype=torch.float64, device=dev) if out is None else out
    _check(lib.dsrg_df_energy_active(ctypes.byref(p), _ptr(baa),
                                     OPT_KERNEL_TIMING if timing else 0, F.data_ptr(),
                                     ws.data_ptr(), nbytes.value, _stream_handle(dev)))
    del keep, baa
    return F


def df_factors(ao3, J, C, nfrz, nc, na, nv, workspace: Optional[torch.Tensor] = None,
               timing: bool = False):
    """B_cv, B_ca, B_av, B_aa (device tensors, float64) via dsrg_df_factors
    from the AO three-index integrals ao3 [naux][nao][nao], the metric J
    [naux][naux] and the MO coefficients C [nao][nmo]. J = None: ao3 holds
    factors of the AO integrals already (CD vectors), no metric applied."""
    lib = load_library()
    naux, nao, _ = ao3.shape
    nmo = C.shape[1]
    dev = ao3.device
    keep = [_as_dev(ao3, "ao3", (naux, nao, nao), dev),
            None if J is None else _as_dev(J, "J", (naux, naux), dev),
            _as_dev(C, "C", (nao, nmo), dev)]
    p = DFGenProblem(nao, nmo, naux, nfrz, nc, na, nv, *[_ptr(t) for t in keep])
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_factors_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    out = {"B_cv": torch.empty(naux, nc, nv, dtype=torch.float64, device=dev),
           "B_ca": torch.empty(naux, nc, na, dtype=torch.float64, device=dev),
           "B_av": torch.empty(naux, na, nv, dtype=torch.float64, device=dev),
           "B_aa": torch.empty(naux, na, na, dtype=torch.float64, device=dev)}
    ptrs = [out[k].data_ptr() if (k == "B_cv" or na > 0) else None
            for k in ("B_cv", "B_ca", "B_av", "B_aa")]
    _check(lib.dsrg_df_factors(ctypes.byref(p), OPT_KERNEL_TIMING if timing else 0, *ptrs,
                               ws.data_ptr(), nbytes.value, _stream_handle(dev)))
    del keep
    return out


def df_fock(ao3, J, C, h, gamma1, nfrz, nc, na, nv, workspace: Optional[torch.Tensor] = None,
            timing: bool = False):
    """The generalized Fock matrix F [nmo][nmo] (device, float64) via
    dsrg_df_fock from ao3 [naux][nao][nao], J [naux][naux], C [nao][nmo], the
    MO one-electron integrals h [nmo][nmo] and the active 1-RDM gamma1 (J =
    None: ao3 holds CD vectors, no metric)."""
    lib = load_library()
    naux, nao, _ = ao3.shape
    nmo = C.shape[1]
    dev = ao3.device
    keep = [_as_dev(ao3, "ao3", (naux, nao, nao), dev),
            None if J is None else _as_dev(J, "J", (naux, naux), dev),
            _as_dev(C, "C", (nao, nmo), dev), _as_dev(h, "h", (nmo, nmo), dev)]
    g1 = _as_dev(gamma1, "gamma1", (na, na), dev) if na > 0 else None
    if g1 is not None:
        keep.append(g1)
    p = FockProblem(DFGenProblem(nao, nmo, naux, nfrz, nc, na, nv, *[_ptr(t) for t in keep[:3]]),
                    _ptr(keep[3]), None if g1 is None else _ptr(g1))
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_fock_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    F = torch.empty(nmo, nmo, dtype=torch.float64, device=dev)
    _check(lib.dsrg_df_fock(ctypes.byref(p), OPT_KERNEL_TIMING if timing else 0, F.data_ptr(),
                            ws.data_ptr(), nbytes.value, _stream_handle(dev)))
    del keep
    return F


def semicanonicalize(F, nfrz, nc, na, nv, C=None, workspace: Optional[torch.Tensor] = None,
                     timing: bool = False, info: Optional[torch.Tensor] = None):
    """(eps [nmo], U [nmo][nmo], Cs = C U or None) via dsrg_df_semicanonicalize
    from the generalized Fock matrix F [nmo][nmo] (device tensors, float64).
    info: optional device int32 tensor [1] that receives the convergence bit
    mask (0 = every block met the criterion) once the work has run."""
    lib = load_library()
    nmo = F.shape[0]
    dev = F.device
    Fd = _as_dev(F, "F", (nmo, nmo), dev)
    nao = C.shape[0] if C is not None else 0
    Cd = _as_dev(C, "C", (nao, nmo), dev) if C is not None else None
    p = SemicanProblem(nao, nmo, nfrz, nc, na, nv, _ptr(Fd), _ptr(Cd))
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_semicanonicalize_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    f64 = dict(dtype=torch.float64, device=dev)
    U = torch.empty(nmo, nmo, **f64)
    eps = torch.empty(nmo, **f64)
    Cs = torch.empty(nao, nmo, **f64) if Cd is not None else None
    if info is not None and (info.device != dev or info.dtype != torch.int32 or info.numel() < 1):
        raise ValueError("info must be an int32 tensor of at least one element on the device of F")
    _check(lib.dsrg_df_semicanonicalize(ctypes.byref(p), OPT_KERNEL_TIMING if timing else 0,
                                        U.data_ptr(), eps.data_ptr(), _ptr(Cs), _ptr(info),
                                        ws.data_ptr(), nbytes.value, _stream_handle(dev)))
    del Fd, Cd
    return eps, U, Cs


# stands for a metric in the size queries, which read no array
_SOME_METRIC = ctypes.c_void_p(256)


def df_fock_workspace_size(nao, nmo, naux, nfrz, nc, na, nv, metric: bool = True) -> int:
    lib = load_library()
    p = FockProblem(DFGenProblem(nao, nmo, naux, nfrz, nc, na, nv, None,
                                 _SOME_METRIC if metric else None, None), None, None)
    out = ctypes.c_size_t(0)
    _check(lib.dsrg_df_fock_workspace_size(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def df_factors_workspace_size(nao, nmo, naux, nfrz, nc, na, nv, metric: bool = True) -> int:
    lib = load_library()
    p = DFGenProblem(nao, nmo, naux, nfrz, nc, na, nv, None,
                     _SOME_METRIC if metric else None, None)
    out = ctypes.c_size_t(0)
    _check(lib.dsrg_df_factors_workspace_size(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def cholesky_workspace_size(nao: int, max_rank: int, tol: float = 0.0) -> int:
    lib = load_library()
    p = CDProblem(nao, None, tol, max_rank)
    out = ctypes.c_size_t(0)
    _check(lib.dsrg_df_cholesky_workspace_size(ctypes.byref(p), ctypes.byref(out)))
    return out.value


def cholesky(M, nao: int, tol: float, max_rank: int, workspace: Optional[torch.Tensor] = None,
             timing: bool = False, with_pivots: bool = True, sync: bool = True):
    """CD vectors of the AO integrals via dsrg_df_cholesky. M: [npair][npair]
    (mu nu|la si) over packed pairs (device, float64). Returns a dict with
    B [rank][nao][nao] (a view of the [max_rank] output; the whole output as
    "B_full"), rank, dmax (Python numbers, read after a stream sync unless
    sync=False, then the device tensors "rank_t", "dmax_t") and pivots
    [rank] (device int64)."""
    lib = load_library()
    npair = nao * (nao + 1) // 2
    dev = M.device
    Md = _as_dev(M, "M", (npair, npair), dev)
    p = CDProblem(nao, Md.data_ptr(), float(tol), int(max_rank))
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_cholesky_workspace_size(ctypes.byref(p), ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    B = torch.empty(max_rank, nao, nao, dtype=torch.float64, device=dev)
    rank_t = torch.empty(1, dtype=torch.int64, device=dev)
    dmax_t = torch.empty(1, dtype=torch.float64, device=dev)
    piv = torch.empty(max(max_rank, 1), dtype=torch.int64, device=dev) if with_pivots else None
    _check(lib.dsrg_df_cholesky(ctypes.byref(p), OPT_KERNEL_TIMING if timing else 0,
                                B.data_ptr() if max_rank > 0 else None, rank_t.data_ptr(),
                                dmax_t.data_ptr(), _ptr(piv), ws.data_ptr(), nbytes.value,
                                _stream_handle(dev)))
    out = {"B_full": B, "rank_t": rank_t, "dmax_t": dmax_t, "pivots_full": piv}
    if sync:
        torch.cuda.current_stream(dev).synchronize()
        r = int(rank_t.item())
        out.update(rank=r, dmax=float(dmax_t.item()), B=B[:r],
                   pivots=None if piv is None else piv[:r])
    del Md
    return out


def laplace_fit(s: float, x_lo: float, x_hi: float, nq: int):
    """(t [nq], w [nq], max_err) of the exponential sum via dsrg_df_laplace_fit
    (host computation, numpy float64 arrays)."""
    import numpy as np
    lib = load_library()
    t = np.zeros(nq)
    w = np.zeros(nq)
    err = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.dsrg_df_laplace_fit(float(s), float(x_lo), float(x_hi), int(nq),
                                   t.ctypes.data_as(dp), w.ctypes.data_as(dp), ctypes.byref(err)))
    return t, w, err.value


def laplace_workspace_size(nc, nv, naux, nq) -> int:
    lib = load_library()
    p = Problem(nc, 0, nv, naux, None, None, None, None, None, None, None, 0.5)
    out = ctypes.c_size_t(0)
    _check(lib.dsrg_df_laplace_workspace_size(ctypes.byref(p), int(nq), ctypes.byref(out)))
    return out.value


def coulomb_laplace(B_cv, eps_c, eps_v, t, w, workspace: Optional[torch.Tensor] = None,
                    timing: bool = False, with_terms: bool = True):
    """(E [1], S [nq] or None) device tensors via dsrg_df_coulomb_laplace: the
    factorized Coulomb part -2 sum_k w_k S_k of E_CCVV for the exponential
    sum (t, w) (host sequences)."""
    import numpy as np
    lib = load_library()
    naux, nc, nv = B_cv.shape
    dev = B_cv.device
    keep = [_as_dev(B_cv, "B_cv", (naux, nc, nv), dev), _as_dev(eps_c, "eps_c", (nc,), dev),
            _as_dev(eps_v, "eps_v", (nv,), dev)]
    p = Problem(nc, 0, nv, naux, _ptr(keep[0]), None, None, _ptr(keep[1]), None, _ptr(keep[2]),
                None, 0.5)
    th = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    wh = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    nq = len(th)
    if len(wh) != nq:
        raise ValueError("t and w differ in length")
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_laplace_workspace_size(ctypes.byref(p), nq, ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    E = torch.empty(1, dtype=torch.float64, device=dev)
    S = torch.empty(nq, dtype=torch.float64, device=dev) if with_terms else None
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib.dsrg_df_coulomb_laplace(ctypes.byref(p), nq, th.ctypes.data_as(dp),
                                       wh.ctypes.data_as(dp), OPT_KERNEL_TIMING if timing else 0,
                                       E.data_ptr(), _ptr(S), ws.data_ptr(), nbytes.value,
                                       _stream_handle(dev)))
    del keep
    return E, S


def energy_backward(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s, gE, precision="fp64",
                    terms="all", want_energy=True, workspace: Optional[torch.Tensor] = None,
                    timing: bool = False, check_signs: bool = False):
    """Gradient of sum_t gE[t] E_t via dsrg_df_energy_backward.

    Returns a dict with device tensors dB_cv, dB_ca, dB_av, deps_c, deps_a,
    deps_v, ds (shape [1]) and, if want_energy, E (shape [3])."""
    lib = load_library()
    p, keep = make_problem_struct(B_cv, B_ca, B_av, eps_c, eps_a, eps_v, gamma1, s)
    dev = B_cv.device
    gE = _as_dev(gE, "gE", (3,), dev)
    mask = _terms_mask(terms, False, timing) | (OPT_CHECK_SIGNS if check_signs else 0)
    prec = PRECISIONS[precision]
    nbytes = ctypes.c_size_t(0)
    _check(lib.dsrg_df_workspace_size(ctypes.byref(p), prec, mask, 1, ctypes.byref(nbytes)))
    ws = _workspace(nbytes.value, dev, workspace)
    naux, nc, nv = B_cv.shape
    na = p.na
    f64 = dict(dtype=torch.float64, device=dev)
    out = dict(dB_cv=torch.empty(naux, nc, nv, **f64),
               dB_ca=torch.empty(naux, nc, na, **f64),
               dB_av=torch.empty(naux, na, nv, **f64),
               deps_c=torch.empty(nc, **f64), deps_a=torch.empty(na, **f64),
               deps_v=torch.empty(nv, **f64), ds=torch.empty(1, **f64))
    E = torch.empty(3, **f64) if want_energy else None
    nz = lambda t: t.data_ptr() if t.numel() else None  # noqa: E731
    _check(lib.dsrg_df_energy_backward(
        ctypes.byref(p), prec, mask, gE.data_ptr(), out["dB_cv"].data_ptr(), nz(out["dB_ca"]),
        nz(out["dB_av"]), out["deps_c"].data_ptr(), nz(out["deps_a"]), out["deps_v"].data_ptr(),
        out["ds"].data_ptr(), None if E is None else E.data_ptr(), ws.data_ptr(), nbytes.value,
        _stream_handle(dev)))
    del keep
    if want_energy:
        out["E"] = E
    return out
