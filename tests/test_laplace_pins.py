"""Pins of the oracle's Laplace-type factorization of the CCVV Coulomb part
(section VI outlook; the decomposition of the renormalised denominator is the
exponential-sum fit described in oracle/dsrg_laplace.py).

* the factorized sum -2 sum_k w_k ||Y_k||^2 equals the plain quadruple sum
  with the same exponential sum (the separation identity);
* the energy error is bounded by 2 sum (ia|jb)^2 times the largest fit error
  over the problem's x values;
* the fit is a least-squares solution (normal equations hold) and its error
  falls as terms are added, so the factorized energy converges to E_J;
* s = 0 gives zero weights and zero energy; s -> infinity fits 1/x, the
  plain MP2 denominator, whose Coulomb part is checked against a direct sum.
"""
import math

import numpy as np
import pytest

from oracle import dsrg_laplace as L
from paper_1603_00561_amd.workloads import make_problem


def _small(seed=3, nc=4, nv=9, naux=12):
    return make_problem(nc, 1, nv, naux, s=0.5, seed=seed)


def test_factorized_equals_plain_sum():
    p = _small()
    lo, hi = L.spectral_range(p.eps_c, p.eps_v)
    t, w, _ = L.laplace_fit(p.s, lo, hi, 10)
    e_fac, S = L.coulomb_laplace(p.B_cv, p.eps_c, p.eps_v, t, w)
    e_plain = L.coulomb_laplace_plain(p.B_cv, p.eps_c, p.eps_v, t, w)
    scale = 2.0 * float(np.abs(w) @ S)
    assert abs(e_fac - e_plain) <= 1e-13 * scale
    assert np.all(S > 0)


@pytest.mark.parametrize("s,nq", [(0.1, 6), (0.5, 8), (0.5, 14), (1.0, 10), (2.0, 12)])
def test_energy_error_within_fit_bound(s, nq):
    p = _small(seed=int(10 * s) + nq)
    lo, hi = L.spectral_range(p.eps_c, p.eps_v)
    t, w, err = L.laplace_fit(s, lo, hi, nq)
    e_exact = L.coulomb_exact(p.B_cv, p.eps_c, p.eps_v, s)
    e_lt, _ = L.coulomb_laplace(p.B_cv, p.eps_c, p.eps_v, t, w)
    V = np.einsum("Qia,Qjb->ijab", p.B_cv, p.B_cv)
    x = L._pair_x(p.eps_c, p.eps_v)
    fit_at_x = np.abs(sum(wk * np.exp(-tk * x) for tk, wk in zip(t, w)) - L.h_of_x(x, s))
    bound = 2.0 * float(np.sum(V * V * fit_at_x))
    assert abs(e_lt - e_exact) <= bound * (1 + 1e-9) + 1e-12 * abs(e_exact)
    assert fit_at_x.max() <= err * (1 + 1e-6) + 1e-15   # the check grid covers the x values


def test_fit_is_least_squares_and_converges():
    s, lo, hi = 0.5, 0.8, 14.0
    errs = []
    for nq in (4, 8, 12, 16, 20):
        t, w, err = L.laplace_fit(s, lo, hi, nq)
        errs.append(err)
        # normal equations at the sample points of the chosen exponent grid
        xs = np.geomspace(lo, hi, L.FIT_SAMPLES)
        A = np.exp(-np.outer(xs, t))
        g = A.T @ (A @ w - L.h_of_x(xs, s))
        assert np.abs(g).max() <= 1e-8 * np.abs(A.T @ L.h_of_x(xs, s)).max()
    assert errs[-1] < 1e-5 * L.h_of_x(np.geomspace(lo, hi, 100), s).max()
    assert errs[-1] < errs[2] < errs[0]
    p = _small(seed=9)
    lo2, hi2 = L.spectral_range(p.eps_c, p.eps_v)
    e_exact = L.coulomb_exact(p.B_cv, p.eps_c, p.eps_v, s)
    e20 = L.coulomb_laplace(p.B_cv, p.eps_c, p.eps_v, *L.laplace_fit(s, lo2, hi2, 20)[:2])[0]
    assert abs(e20 - e_exact) <= 1e-4 * abs(e_exact)


def test_zero_flow_parameter_gives_zero():
    p = _small(seed=5)
    lo, hi = L.spectral_range(p.eps_c, p.eps_v)
    t, w, err = L.laplace_fit(0.0, lo, hi, 8)
    assert np.all(w == 0.0) and err == 0.0
    assert L.coulomb_laplace(p.B_cv, p.eps_c, p.eps_v, t, w)[0] == 0.0


def test_large_flow_parameter_fits_the_mp2_denominator():
    # s -> infinity: h(x) = 1 / x, the MP2 Coulomb part 2 sum (ia|jb)^2 / Delta
    p = _small(seed=6)
    lo, hi = L.spectral_range(p.eps_c, p.eps_v)
    t, w, err = L.laplace_fit(1e8, lo, hi, 14)
    V = np.einsum("Qia,Qjb->ijab", p.B_cv, p.B_cv)
    D = -L._pair_x(p.eps_c, p.eps_v)
    e_mp2_j = 2.0 * math.fsum((V * V / D).ravel())
    e_lt = L.coulomb_laplace(p.B_cv, p.eps_c, p.eps_v, t, w)[0]
    assert err < 1e-6 / lo
    assert abs(e_lt - e_mp2_j) <= 2.0 * err * float(np.sum(V * V)) * (1 + 1e-9)


def test_h_is_the_ccvv_regulariser_and_the_exact_coulomb_part():
    # h(x) = -R(-x) with R of Eq. expensive as the term-F oracle evaluates it,
    # and E_J from the term-F oracle's per-pair integrals and regulariser
    from oracle import dsrg_oracle as O
    x = np.geomspace(1e-3, 30.0, 400)
    for s in (0.1, 0.5, 2.0):
        assert np.allclose(L.h_of_x(x, s), -O.reg_R(-x, s), rtol=1e-14, atol=0)
    p = _small(seed=8)
    e = 0.0
    for i in range(p.nc):
        for j in range(p.nc):
            K = p.B_cv[:, i, :].T @ p.B_cv[:, j, :]
            D = p.eps_c[i] + p.eps_c[j] - p.eps_v[:, None] - p.eps_v[None, :]
            e += 2.0 * float(np.sum(K * K * O.reg_R(D, p.s)))
    assert L.coulomb_exact(p.B_cv, p.eps_c, p.eps_v, p.s) == pytest.approx(e, rel=1e-13)


def test_pair_loop_equals_the_four_index_sum():
    p = _small(seed=12, nc=5, nv=7, naux=10)
    for s in (0.3, 1.5):
        assert L.coulomb_exact_pairs(p.B_cv, p.eps_c, p.eps_v, s) == pytest.approx(
            L.coulomb_exact(p.B_cv, p.eps_c, p.eps_v, s), rel=1e-13)
