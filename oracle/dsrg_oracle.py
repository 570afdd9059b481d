"""CPU FP64 oracle for the DF-DSRG-MRPT2 terms F1 (CCVV), F2 (CAVV), F3 (CCAV).

TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
HIP path is checked against. Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import or run it; the product path never
does, and the two share no code (inputs come from the seeded generator
module, which holds no arithmetic of the method).

Notation (paper section II): core m,n (also i,j), active u,v,w, virtual
e,f (also a,b). Chemists' integrals come from the factorisation of Eq.
int_fact, (pq|rs) = sum_Q B^Q_pq B^Q_rs, with the three blocks that F1-F3
touch: B_cv[Q][m][e], B_ca[Q][m][u], B_av[Q][u][e]. Denominators are
Delta^{ab}_{ij} = e_i + e_j - e_a - e_b (section II.B, after Eq. T2amp).

Spin adaptation (a reading of the spin-orbital Table II; see the pinned
brute-force in ``brute_force_spinorbital``): restricted core and virtual
orbitals, spin-summed active density Gamma (spin-orbital gamma = Gamma/2 in
each spin block, eta = 1 - gamma), which gives

  E_CCVV = sum_{ij} sum_{ab} (ia|jb) [2 (ia|jb) - (ib|ja)] R(D^{ab}_{ij})
  E_CAVV = sum_{uv} Gamma_uv sum_m sum_{ef} (me|uf) S(D^{ef}_{mu})
                                       [2 (me|vf) - (mf|ve)] R1(D^{ef}_{mv})
  E_CCAV = sum_{uv} (2 delta_uv - Gamma_uv) sum_{mn} sum_e (me|nv) S(D^{ev}_{mn})
                                       [2 (me|nu) - (mu|ne)] R1(D^{eu}_{mn})

with R(D) = (1 - exp(-2 s D^2)) / D (Eq. expensive),
R1(D) = (1 - exp(-s D^2)) / D (Eq. T2amp), S(D) = 1 + exp(-s D^2)
(Eq. v_tilde). At D == 0 the regularisers take their limits R = R1 = 0.

The remaining pieces F4-F8 of Table II (two or more active indices) also
read the active-active block B_aa[Q][u][v]. With etab = 2 I - Gamma and
x, y, u, v, w, z active, the same spin summation gives

  F4 = 1/4 sum Gamma_xy Gamma_uv sum_{ef} (xe|uf) S(D^{ef}_{xu})
                                      [2 (ye|vf) - (yf|ve)] R1(D^{ef}_{yv})
  F5 = 1/4 sum etab_uv etab_xy sum_{mn} (mv|ny) S(D^{vy}_{mn})
                                      [2 (mu|nx) - (mx|nu)] R1(D^{ux}_{mn})
  F6 = sum Gamma_xy etab_uv sum_{me} S(D^{ve}_{mx}) R1(D^{ue}_{my})
       [K1 K1' + K2 K2' - (K1 K2' + K2 K1') / 2],
       K1 = (mv|xe), K2 = (me|xv), K1' = (mu|ye), K2' = (me|yu)
  F7 = 1/4 sum Gamma_yw Gamma_zx etab_uv sum_e (yv|ze) S(D^{ve}_{yz})
                                      [2 (wu|xe) - (we|xu)] R1(D^{ue}_{wx})
  F8 = 1/4 sum Gamma_wz etab_uv etab_xy sum_m (mv|wy) S(D^{vy}_{mw})
                                      [2 (mu|zx) - (mx|zu)] R1(D^{ux}_{mz})

(each pinned against ``brute_force_spinorbital``).

Upstream of the energies: ``df_factors`` builds the blocks of B from AO
three-index integrals, the metric and the MO coefficients, and
``generalized_fock`` the generalized Fock matrix of Eq. gen_fock over all
orbitals from the same DF integrals, and ``semicanonicalize`` the rotation to
semicanonical orbitals; ``pivoted_cholesky_steps`` and ``cd_factors`` give
the CD variant of the factors (section II.C), which ``df_factors`` and
``generalized_fock`` take with J = None (all pinned in the test-suite).

Regularisers use libm ``expm1``; every sum over many elements is a
``math.fsum``. Gradients are written out from the same formulas by the chain
rule, term by term, in separate plain code.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# regularisers (Eq. T2amp, Eq. v_tilde, Eq. expensive)
# ---------------------------------------------------------------------------
def _safe_div(num: np.ndarray, den: np.ndarray) -> np.ndarray:
    out = np.zeros(np.broadcast(num, den).shape)
    nz = den != 0.0
    np.divide(num, den, out=out, where=nz)
    return out


def reg_R(D: np.ndarray, s: float) -> np.ndarray:
    """(1 - exp(-2 s D^2)) / D, with value 0 at D = 0."""
    D = np.asarray(D, dtype=np.float64)
    return _safe_div(-np.expm1(-2.0 * s * D * D), D)


def reg_R1(D: np.ndarray, s: float) -> np.ndarray:
    """(1 - exp(-s D^2)) / D, the T2 renormalised denominator; 0 at D = 0."""
    D = np.asarray(D, dtype=np.float64)
    return _safe_div(-np.expm1(-s * D * D), D)


def reg_S(D: np.ndarray, s: float) -> np.ndarray:
    """1 + exp(-s D^2), the factor that turns v into v-tilde."""
    D = np.asarray(D, dtype=np.float64)
    return 1.0 + np.exp(-s * D * D)


def dreg_R(D, s):
    """dR/dD = 4 s exp(-2 s D^2) - R/D, with the limit 2 s at D = 0."""
    D = np.asarray(D, dtype=np.float64)
    e = np.exp(-2.0 * s * D * D)
    return np.where(D == 0.0, 2.0 * s, 4.0 * s * e - _safe_div(reg_R(D, s), D))


def dreg_R1(D, s):
    """dR1/dD = 2 s exp(-s D^2) - R1/D, with the limit s at D = 0."""
    D = np.asarray(D, dtype=np.float64)
    e = np.exp(-s * D * D)
    return np.where(D == 0.0, s, 2.0 * s * e - _safe_div(reg_R1(D, s), D))


def dreg_S(D, s):
    """dS/dD = -2 s D exp(-s D^2)."""
    D = np.asarray(D, dtype=np.float64)
    return -2.0 * s * D * np.exp(-s * D * D)


def sreg_R(D, s):
    """dR/ds = 2 D exp(-2 s D^2)."""
    D = np.asarray(D, dtype=np.float64)
    return 2.0 * D * np.exp(-2.0 * s * D * D)


def sreg_R1(D, s):
    """dR1/ds = D exp(-s D^2)."""
    D = np.asarray(D, dtype=np.float64)
    return D * np.exp(-s * D * D)


def sreg_S(D, s):
    """dS/ds = -D^2 exp(-s D^2)."""
    D = np.asarray(D, dtype=np.float64)
    return -D * D * np.exp(-s * D * D)


def _fsum(a: np.ndarray) -> float:
    return math.fsum(np.asarray(a, dtype=np.float64).ravel().tolist())


# ---------------------------------------------------------------------------
# energies
# ---------------------------------------------------------------------------
def ccvv_pair_energies(B_cv, eps_c, eps_v, s) -> np.ndarray:
    """Pair energies e_ij of F1 (Eq. expensive; the pair loop of section III).

    Returns the full nc x nc matrix e[i, j] = sum_ab (ia|jb)[2(ia|jb)-(ib|ja)]
    R(D^{ab}_{ij}) over ordered pairs, so that E_CCVV = sum_ij e[i, j].
    """
    naux, nc, nv = B_cv.shape
    e = np.zeros((nc, nc))
    for i in range(nc):
        Bi = np.ascontiguousarray(B_cv[:, i, :])
        for j in range(i, nc):
            Bj = np.ascontiguousarray(B_cv[:, j, :])
            K = Bi.T @ Bj                      # K[a, b] = (ia|jb)
            D = eps_c[i] + eps_c[j] - eps_v[:, None] - eps_v[None, :]
            val = _fsum(K * (2.0 * K - K.T) * reg_R(D, s))
            e[i, j] = val
            e[j, i] = val                      # (ji) term equals (ij) term
    return e


def energy_ccvv(B_cv, eps_c, eps_v, s) -> float:
    """F1 of Table II after spin summation."""
    if s == 0.0:
        return 0.0
    return math.fsum(ccvv_pair_energies(B_cv, eps_c, eps_v, s).ravel().tolist())


def energy_cavv(B_cv, B_av, eps_c, eps_a, eps_v, gamma1, s) -> float:
    """F2 of Table II after spin summation (spin-summed Gamma)."""
    naux, nc, nv = B_cv.shape
    na = B_av.shape[1]
    if na == 0 or s == 0.0:
        return 0.0
    parts = []
    for m in range(nc):
        Bm = np.ascontiguousarray(B_cv[:, m, :])
        X = [Bm.T @ np.ascontiguousarray(B_av[:, u, :]) for u in range(na)]  # X[u][e,f] = (me|uf)
        D = [eps_c[m] + eps_a[u] - eps_v[:, None] - eps_v[None, :] for u in range(na)]
        Y = [(2.0 * X[v] - X[v].T) * reg_R1(D[v], s) for v in range(na)]
        for u in range(na):
            Z = X[u] * reg_S(D[u], s)
            T = sum(gamma1[u, v] * Y[v] for v in range(na))
            parts.append(_fsum(Z * T))
    return math.fsum(parts)


def energy_ccav(B_cv, B_ca, eps_c, eps_a, eps_v, gamma1, s) -> float:
    """F3 of Table II after spin summation (eta-bar = 2 I - Gamma)."""
    naux, nc, nv = B_cv.shape
    na = B_ca.shape[2]
    if na == 0 or s == 0.0:
        return 0.0
    etab = 2.0 * np.eye(na) - gamma1
    # J[m][n][e, u] = (me|nu)
    J = np.empty((nc, nc, nv, na))
    for m in range(nc):
        Bm = np.ascontiguousarray(B_cv[:, m, :])
        for n in range(nc):
            J[m, n] = Bm.T @ np.ascontiguousarray(B_ca[:, n, :])
    parts = []
    for m in range(nc):
        for n in range(nc):
            D = eps_c[m] + eps_c[n] - eps_v[:, None] - eps_a[None, :]   # D[e, u]
            Z = J[m, n] * reg_S(D, s)                                  # (me|nv) S, column v
            W = (2.0 * J[m, n] - J[n, m]) * reg_R1(D, s)               # [2(me|nu)-(mu|ne)] R1, column u
            parts.append(_fsum(Z * (W @ etab)))                        # sum_uv etab_uv Z[:,v] W[:,u]
    return math.fsum(parts)


def energy_terms(p, terms=("ccvv", "cavv", "ccav")) -> Tuple[float, float, float]:
    """(E_CCVV, E_CAVV, E_CCAV) for a workloads.Problem-like object."""
    e1 = energy_ccvv(p.B_cv, p.eps_c, p.eps_v, p.s) if "ccvv" in terms else 0.0
    e2 = (energy_cavv(p.B_cv, p.B_av, p.eps_c, p.eps_a, p.eps_v, p.gamma1, p.s)
          if "cavv" in terms else 0.0)
    e3 = (energy_ccav(p.B_cv, p.B_ca, p.eps_c, p.eps_a, p.eps_v, p.gamma1, p.s)
          if "ccav" in terms else 0.0)
    return e1, e2, e3


# ---------------------------------------------------------------------------
# F4-F8 of Table II (spin-summed forms in the module docstring)
# ---------------------------------------------------------------------------
def energy_f4(B_av, eps_a, eps_v, gamma1, s) -> float:
    """F4: two active hole indices, two virtual particle indices."""
    naux, na, nv = B_av.shape
    if na == 0 or s == 0.0:
        return 0.0
    # X[x, u][e, f] = (xe|uf)
    X = np.einsum("Qxe,Quf->xuef", B_av, B_av)
    D = (eps_a[:, None, None, None] + eps_a[None, :, None, None]
         - eps_v[None, None, :, None] - eps_v[None, None, None, :])     # D^{ef}_{xu}
    Z = X * reg_S(D, s)                                                # (xe|uf) S
    W = (2.0 * X - X.transpose(0, 1, 3, 2)) * reg_R1(D, s)             # [2(ye|vf) - (yf|ve)] R1
    parts = []
    for x in range(na):
        for u in range(na):
            T = sum(gamma1[x, y] * gamma1[u, v] * W[y, v] for y in range(na) for v in range(na))
            parts.append(_fsum(Z[x, u] * T))
    return 0.25 * math.fsum(parts)


def energy_f5(B_ca, eps_c, eps_a, gamma1, s) -> float:
    """F5: two core hole indices, two active particle indices."""
    naux, nc, na = B_ca.shape
    if na == 0 or s == 0.0:
        return 0.0
    etab = 2.0 * np.eye(na) - gamma1
    parts = []
    for m in range(nc):
        for n in range(nc):
            K = B_ca[:, m, :].T @ B_ca[:, n, :]                    # K[v, y] = (mv|ny)
            D = eps_c[m] + eps_c[n] - eps_a[:, None] - eps_a[None, :]   # D^{vy}_{mn}
            Z = K * reg_S(D, s)
            W = (2.0 * K - K.T) * reg_R1(D, s)                     # W[u, x] = [2(mu|nx) - (mx|nu)] R1
            parts.append(_fsum(Z * (etab @ W @ etab)))             # sum etab_vu W_ux etab_xy
    return 0.25 * math.fsum(parts)


def energy_f6(B_cv, B_ca, B_av, B_aa, eps_c, eps_a, eps_v, gamma1, s) -> float:
    """F6: one core and one active hole index, one active and one virtual
    particle index."""
    naux, nc, nv = B_cv.shape
    na = B_ca.shape[2]
    if na == 0 or s == 0.0:
        return 0.0
    etab = 2.0 * np.eye(na) - gamma1
    parts = []
    for m in range(nc):
        K1 = np.einsum("Qv,Qxe->vxe", B_ca[:, m, :], B_av)        # (mv|xe)
        K2 = np.einsum("Qe,Qxv->vxe", B_cv[:, m, :], B_aa)        # (me|xv)
        D = (eps_c[m] + eps_a[None, :, None] - eps_a[:, None, None]
             - eps_v[None, None, :])                              # D^{ve}_{mx} at [v, x, e]
        S_, R1_ = reg_S(D, s), reg_R1(D, s)
        Z1, Z2 = K1 * S_, K2 * S_
        W1, W2 = K1 * R1_, K2 * R1_                               # at [u, y, e]
        # sum_{uy} etab_vu W[u, y] Gamma_yx, for each e
        M1 = np.einsum("vu,uye,yx->vxe", etab, W1, gamma1)
        M2 = np.einsum("vu,uye,yx->vxe", etab, W2, gamma1)
        parts.append(_fsum(Z1 * M1 + Z2 * M2 - 0.5 * (Z1 * M2 + Z2 * M1)))
    return math.fsum(parts)


def energy_f7(B_av, B_aa, eps_a, eps_v, gamma1, s) -> float:
    """F7: two active hole indices, one active and one virtual particle index."""
    naux, na, nv = B_av.shape
    if na == 0 or s == 0.0:
        return 0.0
    etab = 2.0 * np.eye(na) - gamma1
    C = np.einsum("Qyv,Qze->yvze", B_aa, B_av)                    # C[y, v, z, e] = (yv|ze)
    D = (eps_a[:, None, None, None] + eps_a[None, None, :, None]
         - eps_a[None, :, None, None] - eps_v[None, None, None, :])  # D^{ve}_{yz}
    Z = C * reg_S(D, s)
    W = (2.0 * C - C.transpose(2, 1, 0, 3)) * reg_R1(D, s)        # at [w, u, x, e]
    T = np.einsum("yw,vu,zx,wuxe->yvze", gamma1, etab, gamma1, W)
    return 0.25 * _fsum(Z * T)


def energy_f8(B_ca, B_aa, eps_c, eps_a, gamma1, s) -> float:
    """F8: one core and one active hole index, two active particle indices."""
    naux, nc, na = B_ca.shape
    if na == 0 or s == 0.0:
        return 0.0
    etab = 2.0 * np.eye(na) - gamma1
    parts = []
    for m in range(nc):
        E = np.einsum("Qv,Qwy->vwy", B_ca[:, m, :], B_aa)         # E[v, w, y] = (mv|wy)
        D = (eps_c[m] + eps_a[None, :, None] - eps_a[:, None, None]
             - eps_a[None, None, :])                              # D^{vy}_{mw}
        Z = E * reg_S(D, s)
        W = (2.0 * E - E.transpose(2, 1, 0)) * reg_R1(D, s)       # at [u, z, x]
        T = np.einsum("vu,wz,yx,uzx->vwy", etab, gamma1, etab, W)
        parts.append(_fsum(Z * T))
    return 0.25 * math.fsum(parts)


def active_terms(p) -> Tuple[float, float, float, float, float]:
    """(F4, F5, F6, F7, F8) for a workloads.Problem-like object with B_aa."""
    return (energy_f4(p.B_av, p.eps_a, p.eps_v, p.gamma1, p.s),
            energy_f5(p.B_ca, p.eps_c, p.eps_a, p.gamma1, p.s),
            energy_f6(p.B_cv, p.B_ca, p.B_av, p.B_aa, p.eps_c, p.eps_a, p.eps_v, p.gamma1, p.s),
            energy_f7(p.B_av, p.B_aa, p.eps_a, p.eps_v, p.gamma1, p.s),
            energy_f8(p.B_ca, p.B_aa, p.eps_c, p.eps_a, p.gamma1, p.s))


def closed_shell_df_mp2(B_cv, eps_c, eps_v) -> float:
    """Textbook closed-shell DF-MP2 correlation energy
    sum_ijab (ia|jb)[2(ia|jb) - (ib|ja)] / (e_i + e_j - e_a - e_b),
    written with one four-index tensor (the s -> infinity limit of F1)."""
    K = np.einsum("Qia,Qjb->iajb", B_cv, B_cv, optimize=True)
    D = (eps_c[:, None, None, None] - eps_v[None, :, None, None]
         + eps_c[None, None, :, None] - eps_v[None, None, None, :])
    return _fsum(K * (2.0 * K - K.transpose(0, 3, 2, 1)) / D)


# ---------------------------------------------------------------------------
# gradients: dE/dB, dE/deps, dE/ds of sum_t gE[t] * E_t
# ---------------------------------------------------------------------------
def gradients(p, gE=(1.0, 1.0, 1.0)) -> Dict[str, np.ndarray]:
    """Analytic gradient of gE[0] E_CCVV + gE[1] E_CAVV + gE[2] E_CCAV."""
    B_cv, B_ca, B_av = p.B_cv, p.B_ca, p.B_av
    eps_c, eps_a, eps_v, gam, s = p.eps_c, p.eps_a, p.eps_v, p.gamma1, p.s
    naux, nc, nv = B_cv.shape
    na = B_ca.shape[2]
    g = dict(B_cv=np.zeros_like(B_cv), B_ca=np.zeros_like(B_ca),
             B_av=np.zeros_like(B_av), eps_c=np.zeros(nc), eps_a=np.zeros(na),
             eps_v=np.zeros(nv), s=np.zeros(1))
    ds_parts = []
    # ---- F1 (CCVV): E = sum_ij sum_ab P R,  P = K (2K - K^T) ----
    if gE[0] != 0.0:
        w = gE[0]
        for i in range(nc):
            Bi = np.ascontiguousarray(B_cv[:, i, :])
            for j in range(nc):
                Bj = np.ascontiguousarray(B_cv[:, j, :])
                K = Bi.T @ Bj
                D = eps_c[i] + eps_c[j] - eps_v[:, None] - eps_v[None, :]
                R = reg_R(D, s)
                G = 2.0 * R * (2.0 * K - K.T)          # dE/dK^{ij}_{ab}
                # dE/dB_{Q,ia} = 2 sum_jb G^{ij}_{ab} B_{Q,jb}  (sum over ordered j)
                g["B_cv"][:, i, :] += w * 2.0 * (Bj @ G.T)
                P = K * (2.0 * K - K.T)
                dD = P * dreg_R(D, s)
                # D contains +e_i +e_j -e_a -e_b
                g["eps_c"][i] += w * _fsum(dD)
                g["eps_c"][j] += w * _fsum(dD)
                g["eps_v"] -= w * (dD.sum(axis=1) + dD.sum(axis=0))
                ds_parts.append(w * _fsum(P * sreg_R(D, s)))
    # ---- F2 (CAVV) ----
    if gE[1] != 0.0 and na > 0:
        w = gE[1]
        for m in range(nc):
            Bm = np.ascontiguousarray(B_cv[:, m, :])
            X = [Bm.T @ np.ascontiguousarray(B_av[:, u, :]) for u in range(na)]
            D = [eps_c[m] + eps_a[u] - eps_v[:, None] - eps_v[None, :] for u in range(na)]
            S = [reg_S(D[u], s) for u in range(na)]
            R1 = [reg_R1(D[u], s) for u in range(na)]
            Wt = [2.0 * X[u] - X[u].T for u in range(na)]
            Y = [Wt[u] * R1[u] for u in range(na)]
            Z = [X[u] * S[u] for u in range(na)]
            A = [sum(gam[u, v] * Y[v] for v in range(na)) for u in range(na)]   # dE/dS^{mu} = X A
            C = [sum(gam[u, v] * Z[u] for u in range(na)) for v in range(na)]   # dE/dR1^{mv} = W C
            for x in range(na):
                # dE/dX^{mx}_{ef}
                Gx = S[x] * A[x] + R1[x] * (2.0 * C[x] - C[x].T)
                g["B_cv"][:, m, :] += w * (np.ascontiguousarray(B_av[:, x, :]) @ Gx.T)
                g["B_av"][:, x, :] += w * (Bm @ Gx)
                dD = X[x] * A[x] * dreg_S(D[x], s) + Wt[x] * C[x] * dreg_R1(D[x], s)
                g["eps_c"][m] += w * _fsum(dD)
                g["eps_a"][x] += w * _fsum(dD)
                g["eps_v"] -= w * (dD.sum(axis=1) + dD.sum(axis=0))
                ds_parts.append(w * _fsum(X[x] * A[x] * sreg_S(D[x], s)
                                          + Wt[x] * C[x] * sreg_R1(D[x], s)))
    # ---- F3 (CCAV) ----
    if gE[2] != 0.0 and na > 0:
        w = gE[2]
        etab = 2.0 * np.eye(na) - gam
        J = np.empty((nc, nc, nv, na))
        for m in range(nc):
            Bm = np.ascontiguousarray(B_cv[:, m, :])
            for n in range(nc):
                J[m, n] = Bm.T @ np.ascontiguousarray(B_ca[:, n, :])
        Dmn = {}
        for m in range(nc):
            for n in range(nc):
                Dmn[m, n] = eps_c[m] + eps_c[n] - eps_v[:, None] - eps_a[None, :]
        C3 = {}
        for m in range(nc):
            for n in range(nc):
                Z3 = J[m, n] * reg_S(Dmn[m, n], s)
                C3[m, n] = Z3 @ etab                    # C3[e,u] = sum_v etab_uv Z3[e,v]
        for m in range(nc):
            for n in range(nc):
                D = Dmn[m, n]
                Sx, R1x = reg_S(D, s), reg_R1(D, s)
                Wt = 2.0 * J[m, n] - J[n, m]
                A3 = (Wt * R1x) @ etab                  # A3[e,v] = sum_u etab_uv W3[e,u]
                G3 = Sx * A3 + R1x * (2.0 * C3[m, n] - C3[n, m])   # dE/dJ^{mn}_{ew}
                g["B_cv"][:, m, :] += w * (np.ascontiguousarray(B_ca[:, n, :]) @ G3.T)
                g["B_ca"][:, n, :] += w * (np.ascontiguousarray(B_cv[:, m, :]) @ G3)
                dD = J[m, n] * A3 * dreg_S(D, s) + Wt * C3[m, n] * dreg_R1(D, s)
                g["eps_c"][m] += w * _fsum(dD)
                g["eps_c"][n] += w * _fsum(dD)
                g["eps_v"] -= w * dD.sum(axis=1)
                g["eps_a"] -= w * dD.sum(axis=0)
                ds_parts.append(w * _fsum(J[m, n] * A3 * sreg_S(D, s)
                                          + Wt * C3[m, n] * sreg_R1(D, s)))
    g["s"][0] = math.fsum(ds_parts)
    return g


# ---------------------------------------------------------------------------
# spin-orbital brute force (Eq. expensive_term and Table II, tiny inputs)
# ---------------------------------------------------------------------------
def full_symmetric_B(B_cv, B_ca, B_av, rng=None, B_cc=None, B_aa=None, B_vv=None):
    """Assemble a full B[Q][p][q] over spatial orbitals ordered C|A|V that is
    symmetric in p<->q and whose cv, ca, av blocks are the given ones. The
    remaining diagonal blocks (cc, aa, vv) are symmetric random unless given.
    """
    naux, nc, nv = B_cv.shape
    na = B_ca.shape[2]
    n = nc + na + nv
    C, A, V = slice(0, nc), slice(nc, nc + na), slice(nc + na, n)
    rng = np.random.default_rng(99) if rng is None else rng

    def sym(k):
        x = rng.standard_normal((naux, k, k)) * 0.05
        return 0.5 * (x + x.transpose(0, 2, 1))

    B = np.zeros((naux, n, n))
    B[:, C, C] = sym(nc) if B_cc is None else B_cc
    B[:, A, A] = sym(na) if B_aa is None else B_aa
    B[:, V, V] = sym(nv) if B_vv is None else B_vv
    B[:, C, V] = B_cv
    B[:, V, C] = B_cv.transpose(0, 2, 1)
    B[:, C, A] = B_ca
    B[:, A, C] = B_ca.transpose(0, 2, 1)
    B[:, A, V] = B_av
    B[:, V, A] = B_av.transpose(0, 2, 1)
    return B


def brute_force_spinorbital(eri, nc, na, nv, eps, gamma1, s):
    """Spin-orbital evaluation of term F (Eq. expensive_term) and of its
    eight pieces F1..F8 (Table II), from the full chemists' tensor
    eri[p,q,r,s] = (pq|rs) over spatial orbitals ordered C|A|V.

    Spin orbitals are (spatial, spin); <pq||rs> = <pq|rs> - <pq|sr> with
    <pq|rs> = (pr|qs) delta_spin. One-particle density: core 1, virtual 0,
    active Gamma/2 in each spin block; eta = 1 - gamma. First-order T2
    amplitudes t^{ij}_{ab} = v (1 - exp(-s D^2))/D for i,j in H = C+A and
    a,b in P = A+V with the all-active block removed (section II.A); the
    modified integrals carry 1 + exp(-s D^2) (Eq. v_tilde).

    Returns dict(F=..., F1..F8=...).
    """
    n = nc + na + nv
    ns = 2 * n
    sp = np.arange(ns) // 2           # spatial index
    sg = np.arange(ns) % 2            # spin
    same = (sg[:, None] == sg[None, :]).astype(float)
    # <pq|rs> = (pr|qs) d(sp,sr) d(sq,ss)
    phys = eri[np.ix_(sp, sp, sp, sp)].transpose(0, 2, 1, 3)     # [p,q,r,s] = (pr|qs)
    phys = phys * same[:, None, :, None] * same[None, :, None, :]
    v = phys - phys.transpose(0, 1, 3, 2)
    e = eps[sp]
    # spin-orbital index sets
    core = [p for p in range(ns) if sp[p] < nc]
    act = [p for p in range(ns) if nc <= sp[p] < nc + na]
    vir = [p for p in range(ns) if sp[p] >= nc + na]
    H = core + act
    P = act + vir
    # densities on the full spin-orbital space
    gam = np.zeros((ns, ns))
    for p in core:
        gam[p, p] = 1.0
    for p in act:
        for q in act:
            if sg[p] == sg[q]:
                gam[p, q] = 0.5 * gamma1[sp[p] - nc, sp[q] - nc]
    eta = np.eye(ns) - gam
    for p in core:
        eta[p, p] = 0.0
    # amplitudes t[i,j,a,b] (i,j in H; a,b in P) and modified integrals vt
    iH, iP = np.array(H), np.array(P)
    vHP = v[np.ix_(iH, iH, iP, iP)]
    Dl = (e[iH][:, None, None, None] + e[iH][None, :, None, None]
          - e[iP][None, None, :, None] - e[iP][None, None, None, :])
    t = vHP * reg_R1(Dl, s)
    vt = vHP * reg_S(Dl, s)
    isA_H = np.array([p in act for p in H])
    isA_P = np.array([p in act for p in P])
    allact = (isA_H[:, None, None, None] & isA_H[None, :, None, None]
              & isA_P[None, None, :, None] & isA_P[None, None, None, :])
    t[allact] = 0.0
    vt[allact] = 0.0
    gH = gam[np.ix_(iH, iH)]
    eP = eta[np.ix_(iP, iP)]
    # Eq. expensive_term: F = 1/4 vt[k,l,c,d] t[i,j,a,b] g[k,i] g[l,j] eta[a,c] eta[b,d]
    F = 0.25 * np.einsum("klcd,ijab,ki,lj,ac,bd->", vt, t, gH, gH, eP, eP, optimize=True)
    # Table II pieces, each with its own index ranges
    pos_H = {p: k for k, p in enumerate(H)}
    pos_P = {p: k for k, p in enumerate(P)}
    hc = [pos_H[p] for p in core]
    ha = [pos_H[p] for p in act]
    pa = [pos_P[p] for p in act]
    pv = [pos_P[p] for p in vir]
    gA = gam[np.ix_(act, act)]
    eA = eta[np.ix_(act, act)]

    def blk(x, i1, i2, i3, i4):
        return x[np.ix_(i1, i2, i3, i4)]

    F1 = 0.25 * np.einsum("mnef,mnef->", blk(vt, hc, hc, pv, pv), blk(t, hc, hc, pv, pv))
    F2 = 0.5 * np.einsum("muef,mvef,uv->", blk(vt, hc, ha, pv, pv), blk(t, hc, ha, pv, pv), gA)
    F3 = 0.5 * np.einsum("mnev,mneu,uv->", blk(vt, hc, hc, pv, pa), blk(t, hc, hc, pv, pa), eA)
    F4 = 0.25 * np.einsum("xuef,yvef,xy,uv->", blk(vt, ha, ha, pv, pv), blk(t, ha, ha, pv, pv), gA, gA)
    F5 = 0.25 * np.einsum("mnvy,mnux,uv,xy->", blk(vt, hc, hc, pa, pa), blk(t, hc, hc, pa, pa), eA, eA)
    F6 = np.einsum("mxve,myue,xy,uv->", blk(vt, hc, ha, pa, pv), blk(t, hc, ha, pa, pv), gA, eA)
    F7 = 0.5 * np.einsum("yzve,wxue,yw,zx,uv->", blk(vt, ha, ha, pa, pv), blk(t, ha, ha, pa, pv), gA, gA, eA)
    F8 = 0.5 * np.einsum("mwvy,mzux,wz,uv,xy->", blk(vt, hc, ha, pa, pa), blk(t, hc, ha, pa, pa), gA, eA, eA)
    return dict(F=F, F1=F1, F2=F2, F3=F3, F4=F4, F5=F5, F6=F6, F7=F7, F8=F8)


# ---------------------------------------------------------------------------
# density-fitting factors (Eq. int_fact, DF definition of section II.C)
# ---------------------------------------------------------------------------
def df_factors(ao3, J, C, nfrz, nc, na, nv) -> Dict[str, np.ndarray]:
    """B^Q_pq for the blocks the energy reads, from AO three-index integrals.

    (pq|P) = sum_{mu nu} C_{mu p} C_{nu q} (mu nu|P) (the MO three-index
    integrals), then B^Q_pq = sum_P [L^{-1}]_{QP} (pq|P) with J = L L^T the
    Cholesky factor of the metric: sum_Q B^Q_pq B^Q_rs = (pq|P) J^{-1} (P|rs),
    the DF integrals of Eq. int_fact (the symmetric J^{-1/2} of the paper gives
    the same factors up to an orthogonal rotation of Q). Returns B_cv, B_ca,
    B_av, B_aa in the [Q][p][q] layout of the energy kernels.

    J = None means ao3 already holds factors of the AO integrals (the CD
    vectors B^Q_{mu nu} of ``cd_factors``): no metric, B^Q_pq is their MO
    transform."""
    o_c = nfrz
    o_a = nfrz + nc
    o_v = nfrz + nc + na
    Cc, Ca, Cv = C[:, o_c:o_a], C[:, o_a:o_v], C[:, o_v:o_v + nv]
    if J is None:
        Linv = None
    else:
        L = np.linalg.cholesky(J)
        Linv = np.linalg.solve(L, np.eye(J.shape[0]))      # lower triangular L^{-1}

    def block(Cp, Cq):
        Y = np.einsum("Pmn,mp,nq->Ppq", ao3, Cp, Cq, optimize=True)   # (pq|P)
        if Linv is None:
            return Y
        return np.einsum("QP,Ppq->Qpq", Linv, Y, optimize=True)

    return {"B_cv": block(Cc, Cv), "B_ca": block(Cc, Ca), "B_av": block(Ca, Cv),
            "B_aa": block(Ca, Ca)}


def generalized_fock(ao3, J, C, h, gamma1, nfrz, nc, na) -> np.ndarray:
    """Generalized Fock matrix of Eq. gen_fock over all MOs, with the DF
    integrals (pq|rs) = sum_PQ (pq|P) [J^{-1}]_PQ (Q|rs) (Eq. int_fact, DF
    definition of section II.C, J^{-1} applied by a linear solve).

    In spin orbitals f_pq = h_pq + sum_rs <pr||qs> gamma_sr; with doubly
    occupied frozen + core orbitals and the spin-summed active density
    (gamma = Gamma / 2 per spin) this is f = h + J[D] - K[D] / 2 with the MO
    density D (2 on the doubly occupied diagonal, Gamma on the active block),
    J[D]_pq = sum_rs (pq|rs) D_rs and K[D]_pq = sum_rs (pr|qs) D_rs.
    J = None takes ao3 as CD factors (pq|rs) = sum_Q B^Q_pq B^Q_rs (no metric)."""
    nmo = C.shape[1]
    no = nfrz + nc + na
    naux = ao3.shape[0]
    D = np.zeros((no, no))
    D[np.arange(nfrz + nc), np.arange(nfrz + nc)] = 2.0
    D[nfrz + nc:, nfrz + nc:] = gamma1
    Y = np.einsum("Pmn,mp,nq->Ppq", ao3, C, C, optimize=True)          # (pq|P)
    Yo = np.ascontiguousarray(Y[:, :, :no])                               # (p r|P), r occupied
    if J is None:                                                         # CD factors: J = 1
        So = Yo
    else:
        So = np.linalg.solve(J, Yo.reshape(naux, -1)).reshape(Yo.shape)  # J^{-1} (P|q s)
    d = np.einsum("Prs,rs->P", So[:, :no, :], D)                          # sum_Q J^-1_PQ (Q|rs) D_rs
    Jm = np.einsum("Ppq,P->pq", Y, d)
    Km = np.einsum("Ppr,rs,Pqs->pq", Yo, D, So, optimize=True)
    return h + Jm - 0.5 * Km


def semicanonicalize(F, nfrz, nc, na, nv) -> Tuple[np.ndarray, np.ndarray]:
    """Semicanonical orbitals (section II.B): the rotation U that diagonalizes
    the core, active and virtual diagonal blocks of the generalized Fock matrix
    F, and the orbital energies eps = diag(U^T F U). Frozen core orbitals are
    left as they are (U = I there, eps = their diagonal of F). Within each
    block the eigenvalues ascend and every eigenvector has its component of
    largest magnitude positive. Returns (eps [nmo], U [nmo][nmo])."""
    nmo = F.shape[0]
    U = np.eye(nmo)
    eps = np.diag(F).copy()
    o = nfrz
    for n in (nc, na, nv):
        if n > 0:
            w, V = np.linalg.eigh(F[o:o + n, o:o + n])
            k = np.argmax(np.abs(V), axis=0)
            V = V * np.sign(V[k, np.arange(n)])[None, :]
            U[o:o + n, o:o + n] = V
            eps[o:o + n] = w
        o += n
    return eps, U


def pivoted_cholesky_steps(M: np.ndarray, tol: float = 0.0, max_rank=None):
    """Pivoted Cholesky of a symmetric positive semidefinite M ~= L L^T, the
    numerical decomposition that generates the CD factors (section II.C).

    Greedy: keep the diagonal d of the residual M - L L^T; at every step take
    the row p of the largest d (the first one on ties) and stop if d[p] <= tol
    (the CD threshold, which bounds every element of the PSD residual) or once
    max_rank vectors exist; otherwise the new vector is the residual's column
    p scaled by 1 / sqrt(d[p]): L[:, k] = (M[:, p] - sum_{j<k} L[:, j] L[p, j])
    / sqrt(d[p]), and d -= L[:, k]^2 with d[p] = 0.

    Returns (L [n][rank], pivots [rank], dmax) with dmax the largest remaining
    diagonal when it stopped (<= tol unless max_rank ended it)."""
    M = np.array(M, dtype=np.float64)
    n = M.shape[0]
    cap = n if max_rank is None else min(int(max_rank), n)
    d = np.diag(M).copy()
    cols, piv = [], []
    dmax = float(d.max()) if n else 0.0
    while True:
        p = int(np.argmax(d)) if n else 0
        dmax = float(d[p]) if n else 0.0
        if n == 0 or d[p] <= tol or len(cols) >= cap:
            break
        col = M[:, p].copy()
        for c in cols:
            col -= c * c[p]
        col /= math.sqrt(d[p])
        cols.append(col)
        piv.append(p)
        d -= col * col
        d[p] = 0.0
    L = np.array(cols).T if cols else np.zeros((n, 0))
    return L, np.array(piv, dtype=np.int64), dmax


def pivoted_cholesky(M: np.ndarray, tol: float = 0.0) -> np.ndarray:
    """The Cholesky vectors of ``pivoted_cholesky_steps`` alone, as an
    (n, rank) array."""
    return pivoted_cholesky_steps(M, tol)[0]


def cd_factors(M: np.ndarray, nao: int, tol: float, max_rank=None):
    """CD factors B^Q_{mu nu} of the AO two-electron integrals (CD approach of
    section II.C, Eq. int_fact with M terms fixed by the threshold).

    M is the integral matrix over packed AO pairs, M[(mu nu)][(la si)] =
    (mu nu|la si) with the pair index mu (mu + 1) / 2 + nu for mu >= nu. Its
    pivoted Cholesky vectors, unpacked symmetrically, are the factors:
    (mu nu|la si) ~= sum_Q B^Q_{mu nu} B^Q_{la si}. Returns (B [rank][nao][nao],
    pivots, dmax) as in ``pivoted_cholesky_steps``."""
    L, piv, dmax = pivoted_cholesky_steps(M, tol, max_rank)
    mu, nu = np.tril_indices(nao)          # row-major lower triangle: mu (mu+1)/2 + nu
    B = np.zeros((L.shape[1], nao, nao))
    B[:, mu, nu] = L.T
    B[:, nu, mu] = L.T
    return B, piv, dmax
