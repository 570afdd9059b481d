"""CPU FP64 oracle for the DSRG-MRPT2 second-order energy terms of Table I
other than F: A, B, C, D, E, G, H, I, J, K.

TEST INFRASTRUCTURE ONLY. This file is the slow, plain reference that the
HIP path is checked against. Only the test-suite, the package smoke check and
the benchmark's CPU-baseline leg may import or run it; the product path never
does, and the two share no code (inputs come from the seeded generator
module, which holds no arithmetic of the method).

Reading of the paper's tensors (pinned in the test-suite by a Fock-space
evaluation of <[H~, T]> (Eq. Esecond) with normal-ordered operators): a
tensor X_{p..}^{q..} is the coefficient of a+_p .. a_q .. (lower indices
created, upper annihilated); gamma_p^q = <a+_p a_q>, eta_p^q = delta_pq -
gamma_q^p; lambda_{xy}^{uv} and lambda_{xyz}^{uvw} are the two- and
three-body cumulants of section II.A. Spin orbitals: spatial orbital k with
spin s is 2k + s; the spaces are ordered core C | active A | virtual V,
holes H = C + A, particles P = A + V.

* First-order amplitudes (Eq. T2amp): t_{ab}^{ij} = <ab||ij> R1(D^{ij}_{ab})
  with D^{ij}_{ab} = e_i + e_j - e_a - e_b, R1(D) = (1 - exp(-s D^2)) / D,
  i, j in H, a, b in P, the all-active block excluded (section II.A).
* Eq. T1amp: t_a^i = [f_a^i + sum_{ux} D_u^x t_{ax}^{iu} gamma_x^u] R1(D_a^i),
  D_u^x = e_x - e_u, f_a^i the first-order (off-diagonal-block) Fock element.
* Eq. f_tilde: f~_a^i = f_a^i [1 + exp(-s D^2)] + [sum_{ux} D_u^x t_{ax}^{iu}
  gamma_x^u] exp(-s D^2), D = D_a^i; Eq. v_tilde: v~_{ab}^{ij} = v_{ab}^{ij}
  [1 + exp(-s (D^{ij}_{ab})^2)]. The de-excitation elements that Table I
  contracts are their transposes (Hermitian, real): f~_j^b = f~_b^j,
  v~_{kl}^{cd} = v~_{cd}^{kl}.
* Table I (Einstein summation over the index ranges above):
    A = f~_j^b t_a^i gamma_j^i eta_a^b
    B = 1/2 v~_{xy}^{ev} t_e^u lambda_{xy}^{uv}
    C = -1/2 v~_{my}^{uv} t_x^m lambda_{xy}^{uv}
    D = 1/2 f~_x^e t_{ey}^{uv} lambda_{xy}^{uv}
    E = -1/2 f~_m^v t_{xy}^{um} lambda_{xy}^{uv}
    F = 1/4 v~_{kl}^{cd} t_{ab}^{ij} gamma_k^i gamma_l^j eta_a^c eta_b^d
    G = 1/8 v~_{xy}^{cd} t_{ab}^{uv} eta_a^c eta_b^d lambda_{xy}^{uv}
    H = 1/8 v~_{kl}^{uv} t_{xy}^{ij} gamma_k^i gamma_l^j lambda_{xy}^{uv}
    I = v~_{jx}^{bu} t_{ay}^{iv} gamma_j^i eta_a^b lambda_{xy}^{uv}
    J = 1/4 v~_{mz}^{uv} t_{xy}^{mw} lambda_{xyz}^{uvw}
    K = 1/4 v~_{xy}^{we} t_{ez}^{uv} lambda_{xyz}^{uvw}

Integrals: (pq|rs) = sum_Q B^Q_pq B^Q_rs (Eq. int_fact); <pq||rs> =
(pr|qs) d(s_p, s_r) d(s_q, s_s) - (ps|qr) d(s_p, s_s) d(s_q, s_r) for
restricted orbitals. Only blocks with one index in P and one in H on each
side of a (..|..) enter, so B_cv, B_ca, B_av and B_aa suffice.

``table1_dense`` evaluates every term by brute force over all spin orbitals
(tiny inputs); ``rest_terms`` evaluates A-E and G-K from the spin-orbital
blocks the terms touch (W = <pu||hx> for h in H, x, u in A, p in P; the
core-core block <uv||mn>), and the virtual-virtual part of G from spatial
integrals after summing over the spins of the two virtual indices.
"""
from __future__ import annotations

import itertools
from typing import Dict

import numpy as np


# ---------------------------------------------------------------------------
# regularisers
# ---------------------------------------------------------------------------
def _R1(D, s):
    D = np.asarray(D, dtype=np.float64)
    out = np.zeros(D.shape)
    nz = D != 0.0
    out[nz] = -np.expm1(-s * D[nz] * D[nz]) / D[nz]
    return out


def _S(D, s):
    D = np.asarray(D, dtype=np.float64)
    return 1.0 + np.exp(-s * D * D)


def _E(D, s):
    D = np.asarray(D, dtype=np.float64)
    return np.exp(-s * D * D)


# ---------------------------------------------------------------------------
# cumulants (section II.A)
# ---------------------------------------------------------------------------
def cumulants(g1, g2, g3):
    """Two- and three-body cumulants from the reduced density matrices of one
    orbital set: g1[p,q] = <a+_p a_q>, g2[p,q,r,s] = <a+_p a+_q a_s a_r>,
    g3[p,q,r,s,t,u] = <a+_p a+_q a+_r a_u a_t a_s> (lower indices first).

    lambda2 = g2 - gamma ^ gamma (the antisymmetrized product over the upper
    labels); lambda3 = g3 - sum over the nine (lower, upper) pairs of
    (-1)^(pair positions) gamma lambda2(rest) - det(gamma gamma gamma)."""
    g1 = np.asarray(g1, dtype=np.float64)
    l2 = g2 - np.einsum("pr,qs->pqrs", g1, g1) + np.einsum("ps,qr->pqrs", g1, g1)
    up = "stu"
    ggg = np.zeros(g3.shape)
    for perm in itertools.permutations(range(3)):
        sign = 1.0
        p_ = list(perm)
        for i in range(3):
            for j in range(i + 1, 3):
                if p_[i] > p_[j]:
                    sign = -sign
        sub = "".join(up[k] for k in perm)
        ggg += sign * np.einsum(f"p{sub[0]},q{sub[1]},r{sub[2]}->pqrstu", g1, g1, g1)
    low = "pqr"
    gl = np.zeros(g3.shape)
    for i in range(3):
        for j in range(3):
            lo_rest = low[:i] + low[i + 1:]
            up_rest = up[:j] + up[j + 1:]
            gl += (-1.0) ** (i + j) * np.einsum(f"{low[i]}{up[j]},{lo_rest}{up_rest}->pqrstu",
                                                 g1, l2)
    l3 = g3 - ggg - gl
    return l2, l3


# ---------------------------------------------------------------------------
# spin-orbital setup (tiny inputs)
# ---------------------------------------------------------------------------
def _spin(n):
    return np.arange(2 * n) // 2, np.arange(2 * n) % 2


def full_B(p):
    """B[Q][p][q] over spatial orbitals C|A|V from the four blocks that enter
    (cc and vv left zero: no integral with two core or two virtual indices on
    one side of (..|..) occurs in A-K)."""
    naux, nc, nv = p.B_cv.shape
    na = p.na
    n = nc + na + nv
    C, A, V = slice(0, nc), slice(nc, nc + na), slice(nc + na, n)
    B = np.zeros((naux, n, n))
    B[:, C, V] = p.B_cv
    B[:, V, C] = p.B_cv.transpose(0, 2, 1)
    B[:, C, A] = p.B_ca
    B[:, A, C] = p.B_ca.transpose(0, 2, 1)
    B[:, A, V] = p.B_av
    B[:, V, A] = p.B_av.transpose(0, 2, 1)
    B[:, A, A] = p.B_aa
    return B


def fock_first_order(p):
    """First-order Fock matrix over spatial orbitals: the off-diagonal blocks
    (core-active, core-virtual, active-virtual) of the generalized Fock matrix
    in the semicanonical basis; the diagonal blocks are zero."""
    nc, na, nv = p.nc, p.na, p.nv
    n = nc + na + nv
    C, A, V = slice(0, nc), slice(nc, nc + na), slice(nc + na, n)
    f = np.zeros((n, n))
    f[C, A] = p.f_ca
    f[A, C] = p.f_ca.T
    f[C, V] = p.f_cv
    f[V, C] = p.f_cv.T
    f[A, V] = p.f_av
    f[V, A] = p.f_av.T
    return f


def spinorbital_densities(p):
    """gamma over all spin orbitals (core 1, active from the reference's
    one-body density, virtual 0), eta = 1 - gamma, and the cumulants placed
    on the active spin orbitals."""
    nc, na, nv = p.nc, p.na, p.nv
    n = 2 * (nc + na + nv)
    a0, a1 = 2 * nc, 2 * (nc + na)
    g = np.zeros((n, n))
    g[np.arange(a0), np.arange(a0)] = 1.0
    g[a0:a1, a0:a1] = p.rdm1
    eta = np.eye(n) - g
    l2a, l3a = cumulants(p.rdm1, p.rdm2, p.rdm3)
    l2 = np.zeros((n,) * 4)
    l3 = np.zeros((n,) * 6)
    A = np.arange(a0, a1)
    l2[np.ix_(A, A, A, A)] = l2a
    l3[np.ix_(A, A, A, A, A, A)] = l3a
    return g, eta, l2, l3


def t1_correction(t2, g, eps, act):
    """The one-body term of Eq. T1amp beside f_a^i: sum_{u,x in A}
    D_u^x t_{ax}^{iu} gamma_x^u with D_u^x = e_x - e_u, at [i][a], from
    t2[i,u,a,x] = t_{ax}^{iu}, gamma[x,u] = gamma_x^u and the spin-orbital
    energies eps (act: the active spin orbitals)."""
    corr = np.zeros(t2.shape[:1] + t2.shape[2:3])
    for u in act:
        for x in act:
            if g[x, u] != 0.0:
                corr += (eps[x] - eps[u]) * t2[:, u, :, x] * g[x, u]
    return corr


def amplitudes_dense(p):
    """t1[i,a] = t_a^i, f~[i,a] = f~_a^i (= f~_i^a), t2[i,j,a,b] = t_{ab}^{ij},
    v~[i,j,a,b] = v~_{ab}^{ij} over all spin orbitals (zero outside i, j in H
    and a, b in P, and on the all-active block)."""
    nc, na, nv = p.nc, p.na, p.nv
    ns = nc + na + nv
    n = 2 * ns
    sp_, sg = _spin(ns)
    B = full_B(p)
    eri = np.einsum("Qpq,Qrs->pqrs", B, B)
    same = (sg[:, None] == sg[None, :]).astype(float)
    phys = eri[np.ix_(sp_, sp_, sp_, sp_)].transpose(0, 2, 1, 3)   # <pq|rs> = (pr|qs)
    phys = phys * same[:, None, :, None] * same[None, :, None, :]
    v = phys - phys.transpose(0, 1, 3, 2)                          # v[p,q,r,s] = <pq||rs>
    eps = np.concatenate([p.eps_c, p.eps_a, p.eps_v])[sp_]
    isH = sp_ < nc + na
    isP = sp_ >= nc
    isA = isH & isP
    g, eta, l2, l3 = spinorbital_densities(p)
    # T2 (Eq. T2amp)
    D2 = eps[:, None, None, None] + eps[None, :, None, None] - eps[None, None, :, None] \
        - eps[None, None, None, :]
    m2 = isH[:, None, None, None] & isH[None, :, None, None] & isP[None, None, :, None] \
        & isP[None, None, None, :]
    m2 &= ~(isA[:, None, None, None] & isA[None, :, None, None] & isA[None, None, :, None]
            & isA[None, None, None, :])
    vHP = v.transpose(2, 3, 0, 1)                                 # <ab||ij> at [i,j,a,b]
    t2 = np.where(m2, vHP * _R1(D2, p.s), 0.0)
    vt = np.where(m2, vHP * _S(D2, p.s), 0.0)
    # T1 (Eq. T1amp) and f~ (Eq. f_tilde)
    f1 = fock_first_order(p)[np.ix_(sp_, sp_)] * same
    corr = t1_correction(t2, g, eps, np.nonzero(isA)[0])
    D1 = eps[:, None] - eps[None, :]
    m1 = isH[:, None] & isP[None, :] & ~(isA[:, None] & isA[None, :])
    num = f1.T + corr                                            # f_a^i at [i,a]
    t1 = np.where(m1, num * _R1(D1, p.s), 0.0)
    ft = np.where(m1, f1.T * _S(D1, p.s) + corr * _E(D1, p.s), 0.0)
    return dict(t1=t1, ft=ft, t2=t2, vt=vt, gamma=g, eta=eta, l2=l2, l3=l3)


def table1_dense(g, eta, l2, l3, ft, t1, vt, t2) -> Dict[str, float]:
    """Every term of Table I by direct summation over all spin orbitals."""
    es = dict(optimize=True)
    out = {}
    out["A"] = np.einsum("jb,ia,ji,ab->", ft, t1, g, eta, **es)
    out["B"] = 0.5 * np.einsum("xyev,ue,xyuv->", vt, t1, l2, **es)
    out["C"] = -0.5 * np.einsum("myuv,mx,xyuv->", vt, t1, l2, **es)
    out["D"] = 0.5 * np.einsum("xe,uvey,xyuv->", ft, t2, l2, **es)
    out["E"] = -0.5 * np.einsum("mv,umxy,xyuv->", ft, t2, l2, **es)
    out["F"] = 0.25 * np.einsum("klcd,ijab,ki,lj,ac,bd->", vt, t2, g, g, eta, eta, **es)
    out["G"] = 0.125 * np.einsum("xycd,uvab,ac,bd,xyuv->", vt, t2, eta, eta, l2, **es)
    out["H"] = 0.125 * np.einsum("kluv,ijxy,ki,lj,xyuv->", vt, t2, g, g, l2, **es)
    out["I"] = np.einsum("jxbu,ivay,ji,ab,xyuv->", vt, t2, g, eta, l2, **es)
    out["J"] = 0.25 * np.einsum("mzuv,mwxy,xyzuvw->", vt, t2, l3, **es)
    out["K"] = 0.25 * np.einsum("xywe,uvez,xyzuvw->", vt, t2, l3, **es)
    return {k: float(v) for k, v in out.items()}


def all_terms_dense(p) -> Dict[str, float]:
    """Table I A-K for a tiny problem (spin-orbital brute force)."""
    d = amplitudes_dense(p)
    return table1_dense(d["gamma"], d["eta"], d["l2"], d["l3"], d["ft"], d["t1"], d["vt"],
                        d["t2"])


# ---------------------------------------------------------------------------
# the same terms from the blocks they touch (realistic sizes)
# ---------------------------------------------------------------------------
REST_TERMS = ("A", "B", "C", "D", "E", "G", "H", "I", "J", "K")


def rest_terms(p) -> Dict[str, float]:
    """Table I terms A-E and G-K from spin-orbital blocks:
    W[h][x][p][u] = <pu||hx> (h in H, x, u in A, p in P), Wcc[m][n][u][v] =
    <uv||mn>, T1 over H x P, and the virtual-virtual part of G from spatial
    (ex|fy) after the sum over the virtual spins (G_VV = 1/2 sum_{xyuv}
    Lambda_{xyuv} M_{xyuv} with Lambda_{xyuv} = sum_{s,t} lambda_{x_s y_t}^{u_s v_t}
    and M_{xyuv} = sum_{ef} (ex|fy) S(D^{xy}_{ef}) (eu|fv) R1(D^{uv}_{ef}))."""
    nc, na, nv, s = p.nc, p.na, p.nv, p.s
    if na == 0:
        return {k: 0.0 for k in REST_TERMS}
    nH, nP = nc + na, na + nv
    # spatial B^Q_{ph} (p in P, h in H) and B^Q_{ux} (u, x in A)
    naux = p.B_cv.shape[0]
    Bph = np.zeros((naux, nP, nH))
    Bph[:, :na, :nc] = p.B_ca.transpose(0, 2, 1)
    Bph[:, :na, nc:] = p.B_aa
    Bph[:, na:, :nc] = p.B_cv.transpose(0, 2, 1)
    Bph[:, na:, nc:] = p.B_av.transpose(0, 2, 1)
    Baa = p.B_aa
    K1 = np.einsum("Qph,Qux->phux", Bph, Baa, optimize=True)          # (ph|ux)
    K2 = np.einsum("Qpx,Quh->pxuh", Bph[:, :, nc:], Bph[:, :na, :], optimize=True)   # (px|uh)
    eH = np.concatenate([p.eps_c, p.eps_a])
    eP = np.concatenate([p.eps_a, p.eps_v])
    eA = p.eps_a
    # spin-orbital index maps: h_so = 2 h + s
    sH, sA, sP = 2 * nH, 2 * na, 2 * nP

    def sp(n2):
        return np.arange(n2) // 2, np.arange(n2) % 2
    hs, hsg = sp(sH)
    xs, xsg = sp(sA)
    ps, psg = sp(sP)
    # W[h][x][p][u] = (ph|ux) d(sp,sh) d(su,sx) - (px|uh) d(sp,sx) d(su,sh)
    k1 = K1[np.ix_(ps, hs, xs, xs)].transpose(1, 3, 0, 2)              # [h][x][p][u] = (ph|ux)
    k2 = K2[np.ix_(ps, xs, xs, hs)].transpose(3, 1, 0, 2)              # [h][x][p][u] = (px|uh)
    d = lambda a, b: (a[:, None] == b[None, :]).astype(float)          # noqa: E731
    dph = d(hsg, psg)            # [h][p]
    dux = d(xsg, xsg)            # [x][u]
    dpx = d(xsg, psg)            # [x][p]
    duh = d(hsg, xsg)            # [h][u]
    W = k1 * dph[:, None, :, None] * dux[None, :, None, :] \
        - k2 * dpx[None, :, :, None] * duh[:, None, None, :]
    D = eH[hs][:, None, None, None] + eA[xs][None, :, None, None] - eP[ps][None, None, :, None] \
        - eA[xs][None, None, None, :]
    allact = (hs >= nc)[:, None, None, None] & (ps < na)[None, None, :, None]
    allact = np.broadcast_to(allact, W.shape)
    Wt = np.where(allact, 0.0, W * _R1(D, s))
    Wv = np.where(allact, 0.0, W * _S(D, s))
    # densities on the spin orbitals: gamma over H (core 1, active rdm1),
    # eta over P (active 1 - rdm1, virtual 1)
    g1 = p.rdm1
    l2, l3 = cumulants(p.rdm1, p.rdm2, p.rdm3)
    gH = np.zeros((sH, sH))
    gH[np.arange(2 * nc), np.arange(2 * nc)] = 1.0
    gH[2 * nc:, 2 * nc:] = g1
    eP_ = np.eye(sP)
    eP_[:sA, :sA] -= g1
    # T1 and f~ over H x P
    f1 = fock_first_order(p)
    n = nc + na + nv
    Hsp = np.arange(nH)
    Psp = np.arange(nc, n)
    fHP = f1[np.ix_(Hsp, Psp)][np.ix_(hs, ps)] * d(hsg, psg)          # f_a^i at [i][a]
    # sum_{u,x in A} (e_x - e_u) t[i,u,a,x] gamma[x,u]
    dE = eA[xs][None, :] - eA[xs][:, None]                            # [u][x] = e_x - e_u
    corr = np.einsum("iuax,xu,ux->ia", Wt, g1, dE, optimize=True)
    D1 = eH[hs][:, None] - eP[ps][None, :]
    m1 = ~((hs >= nc)[:, None] & (ps < na)[None, :])
    t1 = np.where(m1, (fHP + corr) * _R1(D1, s), 0.0)
    ft = np.where(m1, fHP * _S(D1, s) + corr * _E(D1, s), 0.0)
    out = {}
    c0 = 2 * nc              # first active spin orbital in H
    Ah, Ap, Vp = slice(c0, sH), slice(0, sA), slice(sA, sP)
    Ch = slice(0, c0)
    # A = f~[j,b] t1[i,a] gamma[j,i] eta[a,b]
    out["A"] = float(np.sum(ft * (gH @ t1 @ eP_)))
    # B = 1/2 v~[x,y,e,v] t1[u,e] lambda[x,y,u,v]
    out["B"] = 0.5 * float(np.einsum("xyev,ue,xyuv->", Wv[Ah, :, Vp, :], t1[Ah, Vp], l2,
                                     optimize=True))
    # C = -1/2 v~[m,y,u,v] t1[m,x] lambda[x,y,u,v]
    out["C"] = -0.5 * float(np.einsum("myuv,mx,xyuv->", Wv[Ch, :, Ap, :], t1[Ch, Ap], l2,
                                      optimize=True))
    # D = 1/2 f~[x,e] t2[u,v,e,y] lambda[x,y,u,v]
    out["D"] = 0.5 * float(np.einsum("xe,uvey,xyuv->", ft[Ah, Vp], Wt[Ah, :, Vp, :], l2,
                                     optimize=True))
    # E = -1/2 f~[m,v] t2[u,m,x,y] lambda[x,y,u,v], t2[u,m,x,y] = -W_t[m][u][x][y]
    out["E"] = 0.5 * float(np.einsum("mv,muxy,xyuv->", ft[Ch, Ap], Wt[Ch, :, Ap, :], l2,
                                     optimize=True))
    # G: virtual-virtual part from spatial integrals, virtual-active parts
    # (twice the VA part, the AV part being equal) from W
    X = np.einsum("Qxe,Quf->xuef", p.B_av, p.B_av, optimize=True)     # (xe|uf)
    Dxy = eA[:, None, None, None] + eA[None, :, None, None] - p.eps_v[None, None, :, None] \
        - p.eps_v[None, None, None, :]
    Z1 = (X * _S(Dxy, s)).reshape(na * na, -1)
    Z2 = (X * _R1(Dxy, s)).reshape(na * na, -1)
    M = (Z1 @ Z2.T).reshape(na, na, na, na)                           # M[x,y,u,v]
    Lam = np.einsum("xsytusvt->xyuv", l2.reshape(na, 2, na, 2, na, 2, na, 2))
    g_vv = 0.5 * float(np.sum(Lam * M))
    g_va = 0.25 * float(np.einsum("xyed,uveb,bd,xyuv->", Wv[Ah, :, Vp, :], Wt[Ah, :, Vp, :],
                                  np.eye(sA) - g1, l2, optimize=True))
    out["G"] = g_vv + g_va
    # H: core-core block and twice the core-active block
    Bca = p.B_ca
    Kcc = np.einsum("Qmu,Qnv->munv", Bca, Bca, optimize=True)          # (um|vn)
    cs, csg = sp(2 * nc)
    kcc1 = Kcc[np.ix_(cs, xs, cs, xs)].transpose(0, 2, 1, 3)           # [m][n][u][v] = (um|vn)
    kcc2 = Kcc[np.ix_(cs, xs, cs, xs)].transpose(0, 2, 3, 1)           # [m][n][u][v] = (un|vm)
    dmu = d(csg, xsg)
    Wcc = kcc1 * dmu[:, None, :, None] * dmu[None, :, None, :] \
        - kcc2 * dmu[None, :, :, None] * dmu[:, None, None, :]
    Dcc = p.eps_c[cs][:, None, None, None] + p.eps_c[cs][None, :, None, None] \
        - eA[xs][None, None, :, None] - eA[xs][None, None, None, :]
    h_cc = float(np.einsum("mnuv,mnxy,xyuv->", Wcc * _S(Dcc, s), Wcc * _R1(Dcc, s), l2,
                           optimize=True))
    h_ca = float(np.einsum("mluv,mjxy,lj,xyuv->", Wv[Ch, :, Ap, :], Wt[Ch, :, Ap, :], g1, l2,
                           optimize=True))
    out["H"] = 0.125 * (h_cc + 2.0 * h_ca)
    # I = v~[j,x,b,u] t2[i,v,a,y] gamma[j,i] eta[a,b] lambda[x,y,u,v]
    Tg = np.einsum("ji,ivay->jvay", gH, Wt, optimize=True)
    Tg = np.einsum("jvay,ab->jvby", Tg, eP_, optimize=True)
    out["I"] = float(np.einsum("jxbu,jvby,xyuv->", Wv, Tg, l2, optimize=True))
    # J = 1/4 v~[m,z,u,v] t2[m,w,x,y] lambda3[x,y,z,u,v,w]
    out["J"] = 0.25 * float(np.einsum("mzuv,mwxy,xyzuvw->", Wv[Ch, :, Ap, :], Wt[Ch, :, Ap, :],
                                      l3, optimize=True))
    # K = 1/4 v~[x,y,w,e] t2[u,v,e,z] lambda3, v~[x,y,w,e] = -W_v[x][y][e][w]
    out["K"] = -0.25 * float(np.einsum("xyew,uvez,xyzuvw->", Wv[Ah, :, Vp, :], Wt[Ah, :, Vp, :],
                                       l3, optimize=True))
    return out
