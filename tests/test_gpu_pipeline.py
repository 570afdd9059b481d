"""The whole chain on the GPU, every step through the C ABI: DF factors for
the occupied rows of the Fock build, the generalized Fock matrix (Eq.
gen_fock), the semicanonical rotation (section II.B), the DF factors in the
semicanonical basis, then F1-F3 and F4-F8 of term F (Table II); against the
same chain through the oracle. Gate: 1e-9 of |E| per piece (five FP64 steps,
the eigenvectors' sign convention shared)."""
import numpy as np
import pytest
import torch

from oracle import dsrg_oracle as O
from paper_1603_00561_amd.workloads import Problem, make_fock_problem

pytestmark = pytest.mark.gpu


def _b():
    from paper_1603_00561_amd import binding
    return binding


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def oracle_chain(g, s):
    F = O.generalized_fock(g.ao3, g.J, g.C, g.h, g.gamma1, g.nfrz, g.nc, g.na)
    eps, U = O.semicanonicalize(F, g.nfrz, g.nc, g.na, g.nv)
    f = O.df_factors(g.ao3, g.J, g.C @ U, g.nfrz, g.nc, g.na, g.nv)
    o = g.nfrz
    Ua = U[o + g.nc:o + g.nc + g.na, o + g.nc:o + g.nc + g.na]
    p = Problem(g.nc, g.na, g.nv, g.naux, f["B_cv"], f["B_ca"], f["B_av"],
                eps[o:o + g.nc], eps[o + g.nc:o + g.nc + g.na], eps[o + g.nc + g.na:],
                Ua.T @ g.gamma1 @ Ua, s, B_aa=f["B_aa"])
    return np.concatenate([O.energy_terms(p), O.active_terms(p)])


def gpu_chain(g, s):
    b = _b()
    ao3, J, C, h, g1 = (_dev(x) for x in (g.ao3, g.J, g.C, g.h, g.gamma1))
    F = b.df_fock(ao3, J, C, h, g1, g.nfrz, g.nc, g.na, g.nv)
    eps, U, Cs = b.semicanonicalize(F, g.nfrz, g.nc, g.na, g.nv, C=C)
    f = b.df_factors(ao3, J, Cs, g.nfrz, g.nc, g.na, g.nv)
    o, nc, na = g.nfrz, g.nc, g.na
    # the caller's share: the active density in the semicanonical basis,
    # U_a^T Gamma U_a (na x na, on the host)
    Ua = U.cpu().numpy()[o + nc:o + nc + na, o + nc:o + nc + na]
    ga = _dev(Ua.T @ g.gamma1 @ Ua)
    e_c, e_a, e_v = (eps[o:o + nc].contiguous(), eps[o + nc:o + nc + na].contiguous(),
                     eps[o + nc + na:o + nc + na + g.nv].contiguous())
    E = b.energy(f["B_cv"], f["B_ca"], f["B_av"], e_c, e_a, e_v, ga, s)
    Fa = b.energy_active(f["B_cv"], f["B_ca"], f["B_av"], f["B_aa"], e_c, e_a, e_v, ga, s)
    torch.cuda.synchronize()
    return np.concatenate([E.cpu().numpy(), Fa.cpu().numpy()])


@pytest.mark.parametrize("shape", [(1, 4, 2, 30, 48), (2, 6, 3, 70, 120), (0, 5, 0, 40, 60)])
def test_chain_matches_oracle_chain(shape):
    g = make_fock_problem(*shape, seed=sum(shape) + 90)
    print(f"[gpu-pipeline] nfrz={g.nfrz} nc={g.nc} na={g.na} nv={g.nv} naux={g.naux}", flush=True)
    Eg = gpu_chain(g, 0.5)
    Eo = oracle_chain(g, 0.5)
    print("[gpu-pipeline] F1..F8 gpu", Eg, "oracle", Eo, flush=True)
    err = np.abs(Eg - Eo)
    assert np.all(err <= 1e-9 * np.maximum(np.abs(Eo), 1e-300) + 1e-14), (Eg, Eo, err)
