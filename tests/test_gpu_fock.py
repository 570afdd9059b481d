"""GPU parity of dsrg_df_fock (the generalized Fock matrix of Eq. gen_fock
from the DF integrals) against the FP64 CPU oracle, element by element. Gate:
1e-11 of the largest |F| (FP64; the device applies J^{-1} through a Cholesky
factor and its triangular inverse, the oracle through a linear solve)."""
import numpy as np
import pytest
import torch

from oracle import dsrg_oracle as O
from paper_1603_00561_amd.workloads import make_fock_problem

pytestmark = pytest.mark.gpu
GATE = 1e-11


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def gpu_fock(g, **kw):
    print(f"[gpu-fock] nfrz={g.nfrz} nc={g.nc} na={g.na} nv={g.nv} naux={g.naux} nao={g.nao} {kw}",
          flush=True)
    F = _b().df_fock(_dev(g.ao3), _dev(g.J), _dev(g.C), _dev(g.h),
                     _dev(g.gamma1) if g.na > 0 else None, g.nfrz, g.nc, g.na, g.nv, **kw)
    torch.cuda.synchronize()
    return F.cpu().numpy()


def check(F, g):
    ref = O.generalized_fock(g.ao3, g.J, g.C, g.h, g.gamma1, g.nfrz, g.nc, g.na)
    err = np.abs(F - ref).max()
    scale = np.abs(ref).max()
    print("[gpu-fock] max |dF| / max |F|:", err / scale, flush=True)
    assert err <= GATE * scale, (err, scale)


@pytest.mark.parametrize("shape", [(1, 3, 2, 10, 20), (2, 5, 3, 40, 70), (0, 4, 0, 30, 33),
                                   (3, 8, 4, 130, 200), (1, 2, 1, 5, 65), (0, 1, 1, 1, 1),
                                   (4, 30, 5, 40, 50), (5, 40, 10, 20, 30), (10, 50, 8, 20, 40)])
def test_small_shapes(shape):
    # ragged GEMM tiles and metric leaves; no active orbitals; one orbital per
    # space; up to 32, 33..48, 49..64 and more than 64 occupied orbitals (the
    # forms of the first transform)
    g = make_fock_problem(*shape, seed=sum(shape) + 70)
    check(gpu_fock(g), g)


def test_active_limits():
    # Gamma = 2I: the active orbitals act as doubly occupied; Gamma = 0: empty
    g = make_fock_problem(2, 4, 3, 30, 40, seed=11)
    g.gamma1 = 2.0 * np.eye(3)
    F = gpu_fock(g)
    check(F, g)
    g.gamma1 = np.zeros((3, 3))
    check(gpu_fock(g), g)


def test_cfg2_sized_build():
    # the orbital spaces of the triple-zeta-shaped workload with 10 frozen core
    # orbitals: nao = nmo = 415, naux = 1100, 35 occupied orbitals
    g = make_fock_problem(10, 23, 2, 380, 1100, seed=1603)
    check(gpu_fock(g), g)


def test_reproducible_and_timing_option():
    g = make_fock_problem(2, 5, 3, 40, 70, seed=3)
    F1 = gpu_fock(g)
    F2 = gpu_fock(g, timing=True)
    assert np.array_equal(F1, F2)
    names = [n for n, _ in _b().kernel_times(64)]
    for k in ("fock_half1", "fock_half2", "fock_metric", "fock_metric_apply", "fock_coulomb",
              "fock_exchange"):
        assert k in names, (k, names)
