"""Pins of the oracle's Cholesky-decomposition (CD) factors, section II.C.

The CD approach factors the AO two-electron integrals by a numerical
pivoted Cholesky decomposition stopped at a threshold. The oracle's
``pivoted_cholesky_steps`` is checked against what fixes it from outside:
LAPACK's pivoted Cholesky (dpstrf: same greedy rule, same stopping test),
the residual bound a PSD residual obeys, the exactness of the approximation
on the pivot rows, the exact rank of low-rank matrices, and the integrals and
Fock matrix that the factors must reproduce. The s-Gaussian integral
generator is checked against its closed-form special cases.
"""
import math

import numpy as np
import pytest
from scipy.linalg import lapack

from oracle import dsrg_oracle as O
from paper_1603_00561_amd.workloads import (make_cd_problem, make_psd_lowrank,
                                            s_gaussian_eri)


def _small_cd(seed=11, **kw):
    args = dict(n_heavy=3, n_light=2, per_heavy=6, per_light=3, nc=4, na=2, seed=seed)
    args.update(kw)
    return make_cd_problem(**args)


def _decaying_psd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    w = np.exp(-np.arange(n) / 4.0)
    return (Q * w) @ Q.T


# --- the integral generator ----------------------------------------------------
def test_s_gaussian_eri_closed_forms():
    # one normalized s function: (aa|aa) = 2 sqrt(alpha / pi) (self-repulsion
    # of a normalized Gaussian charge of exponent 2 alpha); two functions far
    # apart: (aa|bb) -> 1 / R (point charges)
    alpha = np.array([0.7, 1.3])
    R = 40.0
    centers = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, R]])
    M = s_gaussian_eri(centers, alpha)
    # packed pairs: (0,0)=0, (1,0)=1, (1,1)=2
    assert M[0, 0] == pytest.approx(2.0 * math.sqrt(0.7 / math.pi), rel=1e-14)
    assert M[2, 2] == pytest.approx(2.0 * math.sqrt(1.3 / math.pi), rel=1e-14)
    assert M[0, 2] == pytest.approx(1.0 / R, rel=1e-12)
    assert abs(M[1, 1]) < 1e-100          # overlap density of far-apart functions


def test_s_gaussian_eri_is_symmetric_psd():
    p = _small_cd()
    M = p.M
    assert np.array_equal(M, M.T)
    w = np.linalg.eigvalsh(M)
    assert w.min() >= -1e-12 * w.max()


# --- pivoted Cholesky against LAPACK dpstrf --------------------------------------
@pytest.mark.parametrize("case", ["random", "eri"])
@pytest.mark.parametrize("tol", [1e-5, 1e-9])
def test_pivoted_cholesky_matches_lapack_pstrf(case, tol):
    M = _decaying_psd(70, 3) if case == "random" else _small_cd().M
    L, piv, dmax = O.pivoted_cholesky_steps(M, tol)
    Lp, pvt, rank, info = lapack.dpstrf(M.copy(), lower=1, tol=tol)
    assert L.shape[1] == rank
    assert np.array_equal(piv, pvt[:rank] - 1)
    Ll = np.tril(Lp)[:, :rank]                    # M[piv][:, piv] = Ll Ll^T
    # column k divides a difference of O(max M) terms by sqrt(d_k), the pivot's
    # residual diagonal: rounding differences grow like eps max(M) / sqrt(d_k)
    dk = L[piv, np.arange(rank)] ** 2
    col_tol = 1e-14 * M.diagonal().max() / np.sqrt(dk)
    assert np.all(np.abs(L[pvt - 1] - Ll) <= col_tol[None, :])
    assert dmax <= tol


def test_residual_bounded_by_threshold():
    # the residual R = M - L L^T is PSD with diagonal <= tol, so every element
    # obeys |R_ij| <= sqrt(R_ii R_jj) <= tol
    M = _small_cd(seed=12).M
    for tol in (1e-3, 1e-5, 1e-8):
        L, piv, dmax = O.pivoted_cholesky_steps(M, tol)
        R = M - L @ L.T
        assert np.abs(np.diag(R)).max() <= tol * (1 + 1e-9) + 1e-13
        assert np.abs(R).max() <= tol * (1 + 1e-9) + 1e-13
        assert dmax == pytest.approx(np.diag(R).max(), rel=1e-6, abs=1e-13)
        assert len(piv) == len(set(piv.tolist()))


def test_exact_on_pivot_rows():
    # the pivoted Cholesky approximation reproduces M exactly on the rows (and
    # columns) it pivoted on: (M - L L^T)[piv, :] = 0 up to rounding
    M = _small_cd(seed=13).M
    L, piv, _ = O.pivoted_cholesky_steps(M, 1e-6)
    R = M - L @ L.T
    assert np.abs(R[piv]).max() <= 1e-12 * np.abs(M).max()
    assert np.abs(R[:, piv]).max() <= 1e-12 * np.abs(M).max()


def test_exact_rank_of_low_rank_matrices():
    for n, r in ((40, 7), (90, 31), (25, 25)):
        M = make_psd_lowrank(n, r, seed=n + r)
        L, piv, dmax = O.pivoted_cholesky_steps(M, 1e-10 * M.diagonal().max())
        assert L.shape[1] == r
        assert np.abs(L @ L.T - M).max() <= 1e-11 * np.abs(M).max()


def test_threshold_and_rank_cap_edges():
    M = _small_cd(seed=14).M
    L, piv, dmax = O.pivoted_cholesky_steps(M, M.diagonal().max())
    assert L.shape == (M.shape[0], 0) and len(piv) == 0
    assert dmax == M.diagonal().max()
    Lf, pf, _ = O.pivoted_cholesky_steps(M, 1e-7)
    for cap in (0, 1, 5, 17):
        Lc, pc, dc = O.pivoted_cholesky_steps(M, 1e-7, max_rank=cap)
        assert Lc.shape[1] == cap
        assert np.array_equal(pc, pf[:cap])
        assert np.array_equal(Lc, Lf[:, :cap])
        R = M - Lc @ Lc.T
        assert dc == pytest.approx(np.diag(R).max(), rel=1e-9, abs=1e-14)
    e = O.pivoted_cholesky_steps(np.zeros((0, 0)), 0.0)
    assert e[0].shape == (0, 0) and e[2] == 0.0


# --- the factors -------------------------------------------------------------------
def _unpack4(M, nao):
    # (mu nu|la si) from the packed-pair matrix
    mu, nu = np.tril_indices(nao)
    idx = np.zeros((nao, nao), dtype=np.int64)
    idx[mu, nu] = np.arange(len(mu))
    idx[nu, mu] = np.arange(len(mu))
    return M[np.ix_(idx.ravel(), idx.ravel())].reshape(nao, nao, nao, nao)


def test_cd_factors_reproduce_the_integrals():
    p = _small_cd(seed=15)
    eri = _unpack4(p.M, p.nao)
    B, piv, dmax = O.cd_factors(p.M, p.nao, 1e-5)
    assert np.array_equal(B, B.transpose(0, 2, 1))
    assert np.abs(np.einsum("Qmn,Qls->mnls", B, B) - eri).max() <= 1e-5 * (1 + 1e-9)
    B0, _, _ = O.cd_factors(p.M, p.nao, 0.0)
    assert np.abs(np.einsum("Qmn,Qls->mnls", B0, B0) - eri).max() <= 1e-12 * np.abs(eri).max()


def test_energies_from_cd_factors_equal_four_index_bruteforce():
    # zero threshold: the MO energies from the CD factors (df_factors with no
    # metric) equal the spin-orbital brute force over the MO integrals
    # C^T (mu nu|la si) C built directly from the four-index matrix
    p = make_cd_problem(n_heavy=2, n_light=1, per_heavy=3, per_light=2, nc=2, na=1, seed=16)
    nmo = p.nao
    B, _, _ = O.cd_factors(p.M, p.nao, 0.0)
    f = O.df_factors(B, None, p.C, p.nfrz, p.nc, p.na, p.nv)
    eri_mo = np.einsum("mnls,mp,nq,lr,st->pqrt", _unpack4(p.M, p.nao), p.C, p.C, p.C, p.C,
                       optimize=True)
    eps = np.concatenate([p.eps_c, p.eps_a, p.eps_v])
    r = O.brute_force_spinorbital(eri_mo, p.nc, p.na, p.nv, eps, p.gamma1, p.s)

    class Q:
        pass
    q = Q()
    q.B_cv, q.B_ca, q.B_av = f["B_cv"], f["B_ca"], f["B_av"]
    q.eps_c, q.eps_a, q.eps_v, q.gamma1, q.s = p.eps_c, p.eps_a, p.eps_v, p.gamma1, p.s
    e = O.energy_terms(q)
    for k, v in zip(("F1", "F2", "F3"), e):
        assert abs(r[k] - v) <= 1e-11 * abs(r["F"]), k
    assert nmo == p.nc + p.na + p.nv


def test_fock_from_cd_factors_equals_four_index_route():
    # generalized_fock with J = None against h + J[D] - K[D]/2 written with the
    # MO integrals from the four-index matrix
    p = _small_cd(seed=17, nfrz=1, nc=3, na=2)
    B, _, _ = O.cd_factors(p.M, p.nao, 0.0)
    rng = np.random.default_rng(18)
    G = rng.standard_normal((p.nao, p.nao))
    h = np.diag(rng.uniform(-5, -0.5, p.nao)) + 0.05 * (G + G.T)
    f = O.generalized_fock(B, None, p.C, h, p.gamma1, p.nfrz, p.nc, p.na)
    eri_mo = np.einsum("mnls,mp,nq,lr,st->pqrt", _unpack4(p.M, p.nao), p.C, p.C, p.C, p.C,
                       optimize=True)
    nd = p.nfrz + p.nc
    D = np.zeros((p.nao, p.nao))
    D[np.arange(nd), np.arange(nd)] = 2.0
    D[nd:nd + p.na, nd:nd + p.na] = p.gamma1
    ref = h + np.einsum("pqrs,rs->pq", eri_mo, D) - 0.5 * np.einsum("prqs,rs->pq", eri_mo, D)
    assert np.allclose(f, ref, rtol=0, atol=1e-11)
