"""Seeded synthetic DF-DSRG-MRPT2 problems.

This module only draws random numbers; it holds none of the method's
arithmetic, so both the HIP path and the CPU oracle can take their inputs
from it.

The paper's timing study (section V.B, Table VIII) runs singlet
(2,3)-naphthyne with cc-pVXZ / cc-pVXZ-RI bases; neither the geometries nor
the bases are available here, so seeded synthetic tensors of the same block
shapes stand in for them:

* B^Q_pq blocks (the density-fitting / Cholesky factors of Eq. int_fact):
  N(0,1) * 0.05 * exp(-3 Q / naux), Q counted from 0, in the order
  B_cv [naux][nc][nv], B_ca [naux][nc][na], B_av [naux][na][nv].
* semicanonical orbital energies (diagonal generalized Fock, section II.B):
  core U[-2.0, -0.3], active U[-0.3, 0.1], virtual U[0.1, 5.0] Eh.
* spin-summed active 1-RDM Gamma = O diag(lam) O^T, O from the QR of a
  standard-normal matrix with diag(R) > 0, lam_k = 1 + (v_k - mean v) /
  max(1, max_k |v_k - mean v|), v ~ U[-1, 1]: eigenvalues in [0, 2], trace na.
* the active-active block B_aa [naux][na][na] (read only by the pieces F4-F8
  of term F): (G + G^T) / 2 with G ~ N(0,1) * 0.05 * exp(-3 Q / naux), so
  that it is symmetric in its two orbital indices like every block of B.

One ``numpy.random.default_rng(seed)`` per problem, drawn in exactly the
order listed above (B_aa last, so the other inputs do not depend on it).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

DEFAULT_SEED = 1603


@dataclass
class Problem:
    """One DF-DSRG-MRPT2 F1-F3 problem (host arrays, float64, C order)."""

    nc: int
    na: int
    nv: int
    naux: int
    B_cv: np.ndarray          # [naux][nc][nv]
    B_ca: np.ndarray          # [naux][nc][na]
    B_av: np.ndarray          # [naux][na][nv]
    eps_c: np.ndarray         # [nc]
    eps_a: np.ndarray         # [na]
    eps_v: np.ndarray         # [nv]
    gamma1: np.ndarray        # [na][na] spin-summed, symmetric
    s: float                  # flow parameter, Eh^-2
    name: str = "custom"
    seed: Optional[int] = None
    meta: dict = field(default_factory=dict)
    B_aa: Optional[np.ndarray] = None   # [naux][na][na], symmetric in (u, v)

    def arrays(self):
        return (self.B_cv, self.B_ca, self.B_av, self.eps_c, self.eps_a,
                self.eps_v, self.gamma1)

    def with_s(self, s: float) -> "Problem":
        return Problem(self.nc, self.na, self.nv, self.naux, self.B_cv,
                       self.B_ca, self.B_av, self.eps_c, self.eps_a,
                       self.eps_v, self.gamma1, float(s), self.name,
                       self.seed, dict(self.meta), self.B_aa)


# The five workload shapes: (nc, na, nv, naux, s, terms, gradient wanted).
# cfg1: small case the oracle finishes in seconds (CCVV only).
# cfg2: triple-zeta-shaped naphthyne, all three terms, FP64.
# cfg3: larger triple-zeta-like case, s in {0.1, 0.5, 1.0}, split precision.
# cfg4: energy + gradient case.
# cfg5: quintuple-zeta-shaped case, energy + gradient.
CONFIGS = {
    "cfg1": dict(nc=8, na=4, nv=40, naux=160, s=0.5, terms=("ccvv",), grad=False),
    "cfg2": dict(nc=23, na=2, nv=380, naux=1100, s=0.5,
                 terms=("ccvv", "cavv", "ccav"), grad=False),
    "cfg3": dict(nc=23, na=2, nv=700, naux=2000, s=0.5,
                 terms=("ccvv", "cavv", "ccav"), grad=False, s_list=(0.1, 0.5, 1.0)),
    "cfg4": dict(nc=16, na=4, nv=300, naux=900, s=0.5,
                 terms=("ccvv", "cavv", "ccav"), grad=True),
    "cfg5": dict(nc=23, na=6, nv=1100, naux=3000, s=0.5,
                 terms=("ccvv", "cavv", "ccav"), grad=True),
}


def _b_aa(rng: np.random.Generator, scale: np.ndarray, naux: int, na: int) -> np.ndarray:
    g = rng.standard_normal((naux, na, na)) * scale
    return 0.5 * (g + g.transpose(0, 2, 1))


def _gamma(rng: np.random.Generator, na: int) -> np.ndarray:
    if na == 0:
        return np.zeros((0, 0))
    g = rng.standard_normal((na, na))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    v = rng.uniform(-1.0, 1.0, size=na)
    dv = v - v.mean()
    lam = 1.0 + dv / max(1.0, float(np.max(np.abs(dv))))
    gam = (q * lam[None, :]) @ q.T
    return 0.5 * (gam + gam.T)


def make_problem(nc: int, na: int, nv: int, naux: int, s: float = 0.5,
                 seed: int = DEFAULT_SEED, name: str = "custom",
                 b_scale: float = 0.05, b_decay: float = 3.0) -> Problem:
    """Draw one seeded problem with the recipe in the module docstring."""
    rng = np.random.default_rng(seed)
    q = np.arange(naux, dtype=np.float64)
    scale = (b_scale * np.exp(-b_decay * q / max(naux, 1)))[:, None, None]
    B_cv = rng.standard_normal((naux, nc, nv)) * scale
    B_ca = rng.standard_normal((naux, nc, na)) * scale
    B_av = rng.standard_normal((naux, na, nv)) * scale
    eps_c = rng.uniform(-2.0, -0.3, size=nc)
    eps_a = rng.uniform(-0.3, 0.1, size=na)
    eps_v = rng.uniform(0.1, 5.0, size=nv)
    gamma1 = _gamma(rng, na)
    B_aa = _b_aa(rng, scale, naux, na)
    return Problem(nc, na, nv, naux, B_cv, B_ca, B_av, eps_c, eps_a, eps_v,
                   gamma1, float(s), name, seed, B_aa=B_aa)


def make_config(name: str, seed: int = DEFAULT_SEED, s: Optional[float] = None) -> Problem:
    c = CONFIGS[name]
    p = make_problem(c["nc"], c["na"], c["nv"], c["naux"],
                     c["s"] if s is None else s, seed=seed, name=name)
    p.meta = {k: v for k, v in c.items()}
    return p


def make_near_degenerate(nc: int = 3, na: int = 2, nv: int = 20, naux: int = 48,
                         seed: int = 7, s: float = 0.5) -> Problem:
    """A problem whose orbital energies put many denominators near zero
    (|Delta| down to ~1e-3 Eh), so that s*Delta^2 spans the small-argument
    regime of the regulariser. Core energies are drawn first, then every
    virtual and active energy is set to a random core-pair mean plus a small
    random offset."""
    rng = np.random.default_rng(seed)
    q = np.arange(naux, dtype=np.float64)
    scale = (0.05 * np.exp(-3.0 * q / naux))[:, None, None]
    B_cv = rng.standard_normal((naux, nc, nv)) * scale
    B_ca = rng.standard_normal((naux, nc, na)) * scale
    B_av = rng.standard_normal((naux, na, nv)) * scale
    eps_c = rng.uniform(-0.6, -0.3, size=nc)
    pick_v = rng.integers(0, nc, size=(nv, 2))
    off_v = rng.uniform(-2e-3, 2e-3, size=nv) * rng.choice([1e-3, 1e-1, 1.0], size=nv)
    eps_v = eps_c[pick_v].sum(axis=1) / 2.0 + off_v
    pick_a = rng.integers(0, nc, size=na)
    eps_a = eps_c[pick_a] + rng.uniform(-2e-3, 2e-3, size=na)
    gamma1 = _gamma(rng, na)
    B_aa = _b_aa(rng, scale, naux, na)
    return Problem(nc, na, nv, naux, B_cv, B_ca, B_av, eps_c, eps_a, eps_v,
                   gamma1, float(s), "near_degenerate", seed, B_aa=B_aa)


def _annihilators(n: int):
    """Annihilation operators a_p (p < n) on the 2^n-dimensional Fock space in
    the occupation-number basis (Jordan-Wigner signs), as sparse matrices."""
    import scipy.sparse as sp
    dim = 1 << n
    st = np.arange(dim)
    ops = []
    for p in range(n):
        cols = st[((st >> p) & 1) == 1]
        below = np.array([bin(int(c) & ((1 << p) - 1)).count("1") for c in cols], dtype=np.int64)
        vals = np.where(below % 2 == 1, -1.0, 1.0)
        ops.append(sp.csr_matrix((vals, (cols ^ (1 << p), cols)), shape=(dim, dim)))
    return ops


def cas_reference_rdms(rng: np.random.Generator, na: int, nel: int):
    """Reduced density matrices of a random singlet reference of nel (even)
    electrons in na active orbitals, over the spin orbitals 2u + s (s = 0
    alpha, 1 beta): a standard-normal vector over the determinants with equal
    alpha and beta counts, projected onto the kernel of the spin-raising
    operator sum_u a+_{u alpha} a_{u beta} (total spin 0) and normalized.
    Returns rdm1[p,q] = <a+_p a_q>, rdm2[p,q,r,s] = <a+_p a+_q a_s a_r> and
    rdm3[p,q,r,s,t,u] = <a+_p a+_q a+_r a_u a_t a_s>."""
    if nel % 2 or not 0 <= nel <= 2 * na:
        raise ValueError("a singlet needs an even electron count between 0 and 2 na")
    n = 2 * na
    if n == 0:
        return np.zeros((0, 0)), np.zeros((0,) * 4), np.zeros((0,) * 6)
    a = _annihilators(n)
    st = np.arange(1 << n)
    nal = np.array([bin(int(x) & int("01" * na, 2)).count("1") for x in st])
    nbe = np.array([bin(int(x)).count("1") for x in st]) - nal
    sector = np.nonzero((nal + nbe == nel) & (nal == nbe))[0]
    raised = np.nonzero((nal + nbe == nel) & (nal == nbe + 2))[0]
    psi_s = rng.standard_normal(len(sector))
    if len(raised):
        splus = sum(a[2 * u].T @ a[2 * u + 1] for u in range(na)).tocsr()
        S = splus[raised][:, sector].toarray()
        _, sv, vt = np.linalg.svd(S, full_matrices=True)
        null = vt[int(np.sum(sv > 1e-10 * sv.max())):]
        psi_s = null.T @ (null @ psi_s)
    psi = np.zeros(1 << n)
    psi[sector] = psi_s / np.linalg.norm(psi_s)
    V1 = np.array([a[x] @ psi for x in range(n)])
    V2 = np.array([a[y] @ V1[x] for x in range(n) for y in range(n)])
    V3 = np.array([a[z] @ V2[x * n + y] for x in range(n) for y in range(n) for z in range(n)])
    rdm1 = V1 @ V1.T
    rdm2 = (V2 @ V2.T).reshape((n,) * 4)
    rdm3 = (V3 @ V3.T).reshape((n,) * 6)
    return rdm1, rdm2, rdm3


def make_rest_problem(nc: int, na: int, nv: int, naux: int, s: float = 0.5,
                      seed: int = DEFAULT_SEED, nel: Optional[int] = None,
                      name: str = "custom") -> Problem:
    """Inputs of the Table I terms A-E and G-K: the problem of make_problem
    (same seed, same draws), then from default_rng([seed, 2]) the first-order
    Fock blocks f_ca [nc][na], f_cv [nc][nv], f_av [na][nv] ~ N(0,1) * 0.05
    (the off-diagonal blocks of the generalized Fock matrix in the
    semicanonical basis) and a random singlet reference of nel electrons
    (default na, half filling as in the paper's CAS(n,n)) in the active
    orbitals, whose spin-orbital density matrices rdm1, rdm2, rdm3 are stored
    and whose spin-summed one-body density replaces gamma1."""
    p = make_problem(nc, na, nv, naux, s=s, seed=seed, name=name)
    rng = np.random.default_rng([seed, 2])
    p.f_ca = rng.standard_normal((nc, na)) * 0.05
    p.f_cv = rng.standard_normal((nc, nv)) * 0.05
    p.f_av = rng.standard_normal((na, nv)) * 0.05
    nel = na if nel is None else nel
    p.rdm1, p.rdm2, p.rdm3 = cas_reference_rdms(rng, na, nel)
    p.gamma1 = np.ascontiguousarray(p.rdm1[0::2, 0::2] + p.rdm1[1::2, 1::2])
    return p


@dataclass
class DFGenProblem:
    """Inputs of the density-fitting factor build (Eq. int_fact and the DF
    definition of section II.C): AO three-index integrals (mu nu|P), the
    two-centre metric J and the MO coefficients, orbitals ordered frozen core |
    core | active | virtual (host arrays, float64, C order)."""

    nfrz: int
    nc: int
    na: int
    nv: int
    naux: int
    nao: int
    ao3: np.ndarray           # [naux][nao][nao], symmetric in (mu, nu)
    J: np.ndarray             # [naux][naux], symmetric positive definite
    C: np.ndarray             # [nao][nmo], nmo = nfrz + nc + na + nv
    seed: Optional[int] = None


@dataclass
class FockProblem(DFGenProblem):
    """Inputs of the generalized Fock build (Eq. gen_fock): the DF-build inputs
    plus the one-electron integrals h[nmo][nmo] in the MO basis (symmetric) and
    the spin-summed active 1-RDM gamma1[na][na]."""

    h: np.ndarray = None
    gamma1: np.ndarray = None


def make_fock_problem(nfrz: int, nc: int, na: int, nv: int, naux: int,
                      seed: int = DEFAULT_SEED) -> FockProblem:
    """The DF-build inputs of make_dfgen_problem (same seed, same draws), then
    h = diag(U[-5, -0.5]) + 0.05 (G + G^T) with G ~ N(0,1), then Gamma as in
    make_problem."""
    nmo = nfrz + nc + na + nv
    rng = np.random.default_rng(seed)
    ao3, J, C = _dfgen_draws(rng, nmo, naux)
    G = rng.standard_normal((nmo, nmo))
    h = np.diag(rng.uniform(-5.0, -0.5, size=nmo)) + 0.05 * (G + G.T)
    gamma1 = _gamma(rng, na)
    return FockProblem(nfrz, nc, na, nv, naux, nmo, np.ascontiguousarray(ao3),
                       np.ascontiguousarray(J), np.ascontiguousarray(C), seed,
                       np.ascontiguousarray(h), np.ascontiguousarray(gamma1))


def _dfgen_draws(rng: np.random.Generator, nmo: int, naux: int):
    nao = nmo
    q = np.arange(naux, dtype=np.float64)
    g = rng.standard_normal((naux, nao, nao)) * (0.05 * np.exp(-3.0 * q / naux))[:, None, None]
    ao3 = 0.5 * (g + g.transpose(0, 2, 1))
    L0 = np.tril(rng.standard_normal((naux, naux)) * (0.1 / np.sqrt(naux)), -1)
    L0 += np.diag(rng.uniform(1.0, 2.0, size=naux))
    J = L0 @ L0.T
    J = 0.5 * (J + J.T)
    m = rng.standard_normal((nao, nmo))
    Cq, r = np.linalg.qr(m)
    C = Cq * np.sign(np.diag(r))[None, :]
    return ao3, J, C


def make_dfgen_problem(nfrz: int, nc: int, na: int, nv: int, naux: int,
                       seed: int = DEFAULT_SEED) -> DFGenProblem:
    """Seeded synthetic DF-build inputs with nao = nmo: (mu nu|P) symmetric,
    N(0,1) * 0.05 * exp(-3 P / naux); J = L0 L0^T with L0 lower triangular,
    unit-order diagonal U[1, 2] and N(0,1) * 0.1 / sqrt(naux) below it (well
    conditioned); C orthogonal (QR of a standard-normal matrix, column signs
    fixed). Drawn in that order from one default_rng(seed)."""
    nmo = nfrz + nc + na + nv
    nao = nmo
    rng = np.random.default_rng(seed)
    ao3, J, C = _dfgen_draws(rng, nmo, naux)
    return DFGenProblem(nfrz, nc, na, nv, naux, nao, np.ascontiguousarray(ao3),
                        np.ascontiguousarray(J), np.ascontiguousarray(C), seed)



# ---------------------------------------------------------------------------
# Cholesky-decomposition inputs (CD approach of section II.C)
# ---------------------------------------------------------------------------
@dataclass
class CDProblem:
    """AO two-electron integrals for the CD factor build and the orbital data
    of an energy on top of it (host arrays, float64, C order).

    M[(mu nu)][(la si)] = (mu nu|la si) over packed AO pairs mu >= nu with the
    pair index mu (mu + 1) / 2 + nu; C [nao][nmo] orthogonal with nmo = nao,
    columns frozen core | core | active | virtual."""

    nao: int
    nfrz: int
    nc: int
    na: int
    nv: int
    M: np.ndarray
    centers: np.ndarray       # [nao][3] centre of each basis function (bohr)
    alphas: np.ndarray        # [nao] Gaussian exponents
    C: np.ndarray
    eps_c: np.ndarray
    eps_a: np.ndarray
    eps_v: np.ndarray
    gamma1: np.ndarray
    s: float
    seed: Optional[int] = None


def s_gaussian_eri(centers: np.ndarray, alphas: np.ndarray, rows: int = 256) -> np.ndarray:
    """Electron repulsion integrals (ab|cd) of normalized s-type Gaussians
    exp(-alpha |r - A|^2) (2 alpha / pi)^(3/4), over packed pairs a >= b, from
    the closed form for s functions: with p = a + b exponents, P the weighted
    centre and K_ab = exp(-alpha_a alpha_b / p |A - B|^2),
      (ab|cd) = N_a N_b N_c N_d K_ab K_cd 2 pi^(5/2) / (p q sqrt(p + q))
                F0(p q / (p + q) |P - Q|^2),
    F0(T) = sqrt(pi / T) erf(sqrt T) / 2 (F0(0) = 1). The matrix is symmetric
    positive semidefinite (a Coulomb metric over pair densities)."""
    from scipy.special import erf
    nao = len(alphas)
    mu, nu = np.tril_indices(nao)
    a, b = alphas[mu], alphas[nu]
    A, B = centers[mu], centers[nu]
    p = a + b
    P = (a[:, None] * A + b[:, None] * B) / p[:, None]
    K = np.exp(-a * b / p * ((A - B) ** 2).sum(1))
    pref = (2.0 * a / np.pi) ** 0.75 * (2.0 * b / np.pi) ** 0.75 * K
    npair = len(p)
    M = np.empty((npair, npair))
    for r0 in range(0, npair, rows):
        r1 = min(npair, r0 + rows)
        pp, qq = p[r0:r1, None], p[None, :]
        R2 = ((P[r0:r1, None, :] - P[None, :, :]) ** 2).sum(-1)
        T = pp * qq / (pp + qq) * R2
        st = np.sqrt(np.maximum(T, 1e-300))
        F0 = np.where(T < 1e-12, 1.0 - T / 3.0, 0.5 * np.sqrt(np.pi) * erf(st) / st)
        M[r0:r1] = (pref[r0:r1, None] * pref[None, :] * 2.0 * np.pi ** 2.5
                    / (pp * qq * np.sqrt(pp + qq)) * F0)
    return 0.5 * (M + M.T)


def make_cd_problem(n_heavy: int = 10, n_light: int = 6, per_heavy: int = 14,
                    per_light: int = 5, nfrz: int = 0, nc: int = 30, na: int = 2,
                    s: float = 0.5, seed: int = DEFAULT_SEED,
                    spacing: float = 2.6) -> CDProblem:
    """Seeded s-Gaussian "molecule" for the CD build. n_heavy + n_light atoms
    placed one by one uniformly in a flat box (half-widths 1.5, 1.0, 0.3 times
    spacing * sqrt(atoms)), a draw rejected while it comes closer than
    `spacing` bohr to an atom already placed; per_heavy even-tempered s
    functions 0.08 * 2.6^k on each heavy atom and per_light functions 0.12 *
    3^k on each light one, so nao = n_heavy per_heavy + n_light per_light
    (the default 170 is the cc-pVDZ size of C10H6). Then C orthogonal (QR of a
    standard-normal matrix, column signs fixed), orbital energies and Gamma as
    in make_problem, nv = nao - nfrz - nc - na. One default_rng(seed), drawn
    in that order."""
    rng = np.random.default_rng(seed)
    nat = n_heavy + n_light
    half = spacing * np.sqrt(nat) * np.array([1.5, 1.0, 0.3])
    pts = []
    while len(pts) < nat:
        x = rng.uniform(-1.0, 1.0, 3) * half
        if all(np.linalg.norm(x - q) > spacing for q in pts):
            pts.append(x)
    centers, alphas = [], []
    for i, x in enumerate(pts):
        heavy = i < n_heavy
        k, base, r = (per_heavy, 0.08, 2.6) if heavy else (per_light, 0.12, 3.0)
        for j in range(k):
            centers.append(x)
            alphas.append(base * r ** j)
    centers, alphas = np.array(centers), np.array(alphas)
    nao = len(alphas)
    nv = nao - nfrz - nc - na
    if nv < 1:
        raise ValueError("nao = %d leaves no virtual orbitals" % nao)
    M = s_gaussian_eri(centers, alphas)
    m = rng.standard_normal((nao, nao))
    Cq, r = np.linalg.qr(m)
    C = Cq * np.sign(np.diag(r))[None, :]
    eps_c = rng.uniform(-2.0, -0.3, size=nc)
    eps_a = rng.uniform(-0.3, 0.1, size=na)
    eps_v = rng.uniform(0.1, 5.0, size=nv)
    gamma1 = _gamma(rng, na)
    return CDProblem(nao, nfrz, nc, na, nv, np.ascontiguousarray(M), centers, alphas,
                     np.ascontiguousarray(C), eps_c, eps_a, eps_v, gamma1, float(s), seed)


def make_psd_lowrank(n: int, rank: int, seed: int = DEFAULT_SEED, decay: float = 4.0) -> np.ndarray:
    """Symmetric positive semidefinite n x n matrix of exact rank `rank`:
    G G^T with G [n][rank] ~ N(0,1) scaled by exp(-decay k / rank) in column k."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, rank)) * np.exp(-decay * np.arange(rank) / max(rank, 1))[None, :]
    M = G @ G.T
    return 0.5 * (M + M.T)
