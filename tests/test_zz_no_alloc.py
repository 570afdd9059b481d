"""GPU parity of dsrg_df_energy_noalloc (the energy with the library's static
device scratch instead of a caller workspace) against dsrg_df_energy on the
same inputs: two calls in a row, the second on a smaller problem, in both
precisions; results must be bitwise equal (same kernels, same reduction
order) and, like dsrg_df_energy's, within 1e-10 Eh (FP64) or 1e-6 Eh
(slices) of the oracle."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import dsrg_oracle as O
from paper_1603_00561_amd.workloads import make_problem


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(p):
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in p.arrays()]


@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("ozaki", 1e-6)])
def test_noalloc_energy_matches_workspace_entry_point(precision, tol):
    b = _b()
    big = make_problem(9, 2, 200, 300, s=0.5, seed=71)
    small = make_problem(4, 3, 60, 30, s=0.7, seed=72)
    for p in (big, small, big):
        print(f"[gpu-noalloc] {precision} nc={p.nc} na={p.na} nv={p.nv} naux={p.naux}",
              flush=True)
        t = _dev(p)
        E_na = b.energy_noalloc(*t, p.s, precision=precision).cpu().numpy()
        E_ws = b.energy(*t, p.s, precision=precision).cpu().numpy()
        assert np.array_equal(E_na, E_ws), (E_na, E_ws)
        Eo = np.array(O.energy_terms(p))
        assert np.all(np.abs(E_na - Eo) <= tol), (E_na, Eo)


@pytest.mark.gpu
def test_noalloc_energy_on_a_side_stream_with_term_mask():
    b = _b()
    p = make_problem(5, 2, 130, 70, s=0.5, seed=73)
    t = _dev(p)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        E_na = b.energy_noalloc(*t, p.s, terms=("ccvv", "ccav"))
    st.synchronize()
    E_ws = b.energy(*t, p.s, terms=("ccvv", "ccav"))
    assert np.array_equal(E_na.cpu().numpy(), E_ws.cpu().numpy())
    assert E_na[1].item() == 0.0


def test_noalloc_validation_on_the_host():
    """Host-side refusals (no GPU needed: nothing is enqueued): a problem whose
    workspace exceeds the static array, the timing option, a missing output."""
    b = _b()
    lib = b.load_library()
    a = 0x10000
    big = b.Problem(23, 6, 1100, 3000, a, a, a, a, a, a, a, 0.5)
    E = ctypes.c_void_p(0x20000)
    assert lib.dsrg_df_energy_noalloc(ctypes.byref(big), 0, 7, E, None) == b.DSRG_ERR_UNSUPPORTED
    assert "static scratch" in lib.dsrg_df_last_error().decode()
    small = b.Problem(4, 2, 70, 33, a, a, a, a, a, a, a, 0.5)
    assert lib.dsrg_df_energy_noalloc(ctypes.byref(small), 0, 7 | b.OPT_KERNEL_TIMING, E,
                                      None) == b.DSRG_ERR_ARG
    assert lib.dsrg_df_energy_noalloc(ctypes.byref(small), 0, 7, None, None) == b.DSRG_ERR_ARG
    # the workspace the static array must hold for the triple-zeta-shaped energy
    out = ctypes.c_size_t(0)
    tz = b.Problem(23, 2, 380, 1100, a, a, a, a, a, a, a, 0.5)
    assert lib.dsrg_df_workspace_size(ctypes.byref(tz), 0, 7, 0, ctypes.byref(out)) == 0
    assert out.value <= 256 << 20
