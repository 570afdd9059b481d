"""CPU FP64 oracle for a Laplace-type factorization of the renormalised CCVV
denominator (the outlook of section VI).

TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
HIP path is checked against. Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import or run it; the product path never
does, and the two share no code.

The paper names the Laplace transformation of the energy denominators as the
way to lower the scaling, and notes that the DSRG denominators are
renormalised, which a decomposition has to handle. With x = -Delta =
e_a + e_b - e_i - e_j > 0 for core i, j and virtual a, b, the CCVV regulariser
of Eq. expensive is R(Delta) = -h(x) with h(x) = (1 - exp(-2 s x^2)) / x.
h is not a Laplace transform of a function (the Gaussian grows along the
imaginary axis), so no exact quadrature exists; on the interval [x_lo, x_hi]
that holds every x of a problem it is approximated by an exponential sum

    h(x) ~ sum_k w_k exp(-t_k x),

exponents on a geometric grid t_k from c1 / x_hi to c2 / x_lo and weights by
linear least squares on 600 logarithmically spaced points; (c1, c2) is the
pair of a fixed set whose fit has the smallest largest error on a 5000-point
check grid. Each term separates over the four orbital energies, so the
Coulomb part of E_CCVV,

    E_J = 2 sum_{ij,ab} (ia|jb)^2 R(Delta)
        ~ -2 sum_k w_k sum_{PQ} (Y_k)_{PQ}^2,
    Y_k[P][Q] = sum_{ia} B^P_ia B^Q_ia exp(-t_k (e_a - e_i)),

costs 2 naux^2 nc nv per term (fourth order) instead of the fifth-order pair
sum. The exchange part (ia|jb)(ib|ja) does not separate this way.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

FIT_C1 = (0.1, 0.3, 1.0)
FIT_C2 = (3.0, 10.0, 30.0)
FIT_SAMPLES = 600
FIT_CHECK = 5000


def h_of_x(x: np.ndarray, s: float) -> np.ndarray:
    """h(x) = (1 - exp(-2 s x^2)) / x = -R(-x) (Eq. expensive), x > 0."""
    x = np.asarray(x, dtype=np.float64)
    return -np.expm1(-2.0 * s * x * x) / x


def spectral_range(eps_c: np.ndarray, eps_v: np.ndarray) -> Tuple[float, float]:
    """Smallest and largest x = e_a + e_b - e_i - e_j over the CCVV quadruples."""
    lo = 2.0 * (float(np.min(eps_v)) - float(np.max(eps_c)))
    hi = 2.0 * (float(np.max(eps_v)) - float(np.min(eps_c)))
    return lo, hi


def _fit_once(s, x_lo, x_hi, nq, c1, c2):
    t = np.geomspace(c1 / x_hi, c2 / x_lo, nq) if nq > 1 else np.array([c1 / x_hi])
    xs = np.geomspace(x_lo, x_hi, FIT_SAMPLES)
    A = np.exp(-np.outer(xs, t))
    w, *_ = np.linalg.lstsq(A, h_of_x(xs, s), rcond=None)
    xc = np.geomspace(x_lo, x_hi, FIT_CHECK)
    err = float(np.max(np.abs(np.exp(-np.outer(xc, t)) @ w - h_of_x(xc, s))))
    return t, w, err


def laplace_fit(s: float, x_lo: float, x_hi: float, nq: int):
    """Exponents t [nq], weights w [nq] and the largest absolute error of the
    exponential sum on the check grid (see the module docstring). s = 0 gives
    h = 0: zero weights, error 0."""
    best = None
    for c1 in FIT_C1:
        for c2 in FIT_C2:
            t, w, err = _fit_once(s, x_lo, x_hi, nq, c1, c2)
            if best is None or err < best[2]:
                best = (t, w, err)
    return best


def _pair_x(eps_c, eps_v):
    # x[i, j, a, b] = e_a + e_b - e_i - e_j
    return (eps_v[None, None, :, None] + eps_v[None, None, None, :]
            - eps_c[:, None, None, None] - eps_c[None, :, None, None])


def coulomb_exact(B_cv, eps_c, eps_v, s) -> float:
    """E_J = 2 sum (ia|jb)^2 R(Delta) with the exact regulariser (small
    inputs: four-index intermediate)."""
    V = np.einsum("Qia,Qjb->ijab", B_cv, B_cv)
    x = _pair_x(eps_c, eps_v)
    return float(-2.0 * math.fsum((V * V * h_of_x(x, s)).ravel()))


def coulomb_exact_pairs(B_cv, eps_c, eps_v, s) -> float:
    """E_J = 2 sum (ia|jb)^2 R(Delta) pair by pair (any size): for i <= j the
    integrals K = B_i^T B_j, counted twice for i < j ((ia|jb)^2 and its
    regulariser are symmetric under (i, a) <-> (j, b))."""
    nc = B_cv.shape[1]
    parts = []
    for i in range(nc):
        for j in range(i, nc):
            K = B_cv[:, i, :].T @ B_cv[:, j, :]
            x = eps_v[:, None] + eps_v[None, :] - eps_c[i] - eps_c[j]
            v = -2.0 * math.fsum((K * K * h_of_x(x, s)).ravel())
            parts.append(v if i == j else 2.0 * v)
    return float(math.fsum(parts))


def coulomb_laplace_plain(B_cv, eps_c, eps_v, t, w) -> float:
    """-2 sum_k w_k sum (ia|jb)^2 exp(-t_k x), summed over the quadruples
    (small inputs)."""
    V = np.einsum("Qia,Qjb->ijab", B_cv, B_cv)
    x = _pair_x(eps_c, eps_v)
    hx = sum(wk * np.exp(-tk * x) for tk, wk in zip(t, w))
    return float(-2.0 * math.fsum((V * V * hx).ravel()))


def coulomb_laplace(B_cv, eps_c, eps_v, t, w) -> Tuple[float, np.ndarray]:
    """The factorized form -2 sum_k w_k ||Y_k||_F^2 and the per-term sums
    S_k = ||Y_k||_F^2 (fourth-order work per term)."""
    naux, nc, nv = B_cv.shape
    Bf = B_cv.reshape(naux, nc * nv)
    d = (eps_v[None, :] - eps_c[:, None]).ravel()          # e_a - e_i over (i, a)
    S = np.empty(len(t))
    for k, tk in enumerate(t):
        Y = (Bf * np.exp(-tk * d)[None, :]) @ Bf.T
        S[k] = math.fsum((Y * Y).ravel())
    return float(-2.0 * math.fsum(w * S)), S
