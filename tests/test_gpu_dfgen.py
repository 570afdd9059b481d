"""GPU parity of dsrg_df_factors (the density-fitting factors B of Eq.
int_fact from AO three-index integrals, the metric and the MO coefficients)
against the FP64 CPU oracle, element by element. Gate: 1e-11 of the largest
|B| per block (FP64 with a Cholesky factor and a triangular inverse of a
well-conditioned metric)."""
import numpy as np
import pytest
import torch

from oracle import dsrg_oracle as O
from paper_1603_00561_amd.workloads import make_dfgen_problem, make_problem

pytestmark = pytest.mark.gpu
GATE = 1e-11
KEYS = ("B_cv", "B_ca", "B_av", "B_aa")


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def gpu_factors(g, ao3=None, **kw):
    print(f"[gpu-dfgen] nfrz={g.nfrz} nc={g.nc} na={g.na} nv={g.nv} naux={g.naux} nao={g.nao} {kw}",
          flush=True)
    f = _b().df_factors(_dev(g.ao3 if ao3 is None else ao3), _dev(g.J), _dev(g.C), g.nfrz, g.nc,
                        g.na, g.nv, **kw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in f.items()}


def compare(f, ref):
    worst = {}
    for k in KEYS:
        if ref[k].size == 0:
            continue
        scale = np.abs(ref[k]).max()
        err = np.abs(f[k] - ref[k]).max()
        worst[k] = err / scale
        assert err <= GATE * scale, (k, err, scale)
    print("[gpu-dfgen] max error / max |B|:", worst, flush=True)


@pytest.mark.parametrize("shape", [(1, 3, 2, 10, 20), (2, 5, 3, 40, 70), (0, 4, 0, 30, 33),
                                   (3, 8, 4, 130, 200), (1, 2, 1, 5, 65), (2, 10, 6, 300, 300),
                                   (0, 1, 1, 1, 1), (1, 30, 5, 40, 50), (2, 33, 0, 20, 129)])
def test_small_shapes(shape):
    # GEMM tiles with ragged tails, metric leaves of 64 with ragged tails, na = 0,
    # one orbital per space; more than 32 core + active orbitals (the first
    # transform batched over P instead of folded into one product)
    g = make_dfgen_problem(*shape, seed=sum(shape) + 5)
    compare(gpu_factors(g), O.df_factors(g.ao3, g.J, g.C, g.nfrz, g.nc, g.na, g.nv))


def test_recovers_a_known_factor():
    g = make_dfgen_problem(2, 6, 3, 70, 150, seed=8)
    nmo = g.nfrz + g.nc + g.na + g.nv
    rng = np.random.default_rng(9)
    B0 = rng.standard_normal((g.naux, nmo, nmo)) * 0.05
    B0 = 0.5 * (B0 + B0.transpose(0, 2, 1))
    L0 = np.linalg.cholesky(g.J)
    ao3 = np.einsum("mp,Ppq,nq->Pmn", g.C, np.einsum("PQ,Qpq->Ppq", L0, B0), g.C,
                    optimize=True)
    f = gpu_factors(g, ao3=ao3)
    c, a, v = slice(2, 8), slice(8, 11), slice(11, 81)
    for k, (P, Q) in {"B_cv": (c, v), "B_ca": (c, a), "B_av": (a, v), "B_aa": (a, a)}.items():
        ref = B0[:, P, Q]
        assert np.abs(f[k] - ref).max() <= 1e-11 * np.abs(ref).max(), k


def test_energies_from_gpu_factors():
    # the chain: DF factors on the GPU feed the energy on the GPU; the same
    # chain on the oracle gives the same energies
    g = make_dfgen_problem(1, 4, 2, 60, 90, seed=12)
    f = gpu_factors(g)
    ref = O.df_factors(g.ao3, g.J, g.C, g.nfrz, g.nc, g.na, g.nv)
    p = make_problem(4, 2, 60, 90, s=0.5, seed=13)
    p.B_cv, p.B_ca, p.B_av = ref["B_cv"], ref["B_ca"], ref["B_av"]
    Eo = np.array(O.energy_terms(p))
    E = _b().energy(_dev(f["B_cv"]), _dev(f["B_ca"]), _dev(f["B_av"]), _dev(p.eps_c),
                    _dev(p.eps_a), _dev(p.eps_v), _dev(p.gamma1), p.s).cpu().numpy()
    assert np.all(np.abs(E - Eo) <= 1e-10), (E, Eo)


def test_cfg2_sized_build():
    # the orbital spaces of the triple-zeta-shaped workload with 10 frozen core
    # orbitals: nao = nmo = 415, naux = 1100
    g = make_dfgen_problem(10, 23, 2, 380, 1100, seed=1603)
    compare(gpu_factors(g), O.df_factors(g.ao3, g.J, g.C, g.nfrz, g.nc, g.na, g.nv))


def test_cfg3_orbital_spaces_large_tiles():
    # the orbital spaces of the larger triple-zeta-shaped workload (10 frozen,
    # 23 core, 2 active, 700 virtual: nao = nmo = 735) with 800 auxiliary
    # functions: the second transform (20000 x 702) and the triangular
    # application (800 x 17550) both take the 128 x 128 tile, as at the full
    # 2000 auxiliary functions, with ragged tails in every index
    g = make_dfgen_problem(10, 23, 2, 700, 800, seed=1603)
    compare(gpu_factors(g), O.df_factors(g.ao3, g.J, g.C, g.nfrz, g.nc, g.na, g.nv))


def test_reproducible_and_timing_option():
    g = make_dfgen_problem(2, 5, 3, 40, 70, seed=3)
    f1 = gpu_factors(g)
    f2 = gpu_factors(g, timing=True)
    for k in KEYS:
        assert np.array_equal(f1[k], f2[k]), k
    names = [n for n, _ in _b().kernel_times(64)]
    for k in ("df_half1", "df_half2", "df_metric", "df_metric_apply", "df_scatter"):
        assert k in names, (k, names)
