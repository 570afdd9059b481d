/*
 * dsrg_df.h - C ABI of libdsrgdf, the MI355X (gfx950) library for the
 * density-fitted DSRG-MRPT2 energy terms F1 (CCVV), F2 (CAVV) and F3 (CCAV),
 * their gradients, the remaining pieces F4-F8 of term F, and the
 * density-fitting factors B themselves.
 *
 * What is computed (Hannon, Li, Evangelista, "An integral-factorized
 * implementation of the driven similarity renormalization group second-order
 * multireference perturbation theory"):
 *
 *   The three pieces of term F (Eq. expensive_term) that Table II names F1,
 *   F2 and F3, after spin summation over restricted core / virtual orbitals
 *   with a spin-summed active density Gamma:
 *
 *   E_CCVV = sum_{ij in C} sum_{ab in V} (ia|jb) [2(ia|jb) - (ib|ja)] R(D^{ab}_{ij})
 *   E_CAVV = sum_{uv} Gamma_uv sum_m sum_{ef} (me|uf) S(D^{ef}_{mu})
 *                                   [2(me|vf) - (mf|ve)] R1(D^{ef}_{mv})
 *   E_CCAV = sum_{uv} (2 delta_uv - Gamma_uv) sum_{mn} sum_e (me|nv) S(D^{ev}_{mn})
 *                                   [2(me|nu) - (mu|ne)] R1(D^{eu}_{mn})
 *
 *   with (pq|rs) = sum_Q B^Q_pq B^Q_rs (Eq. int_fact), the Moller-Plesset
 *   denominator D^{ab}_{ij} = e_i + e_j - e_a - e_b (section II.B), and the
 *   regularisers R(D) = (1 - exp(-2 s D^2))/D (Eq. expensive),
 *   R1(D) = (1 - exp(-s D^2))/D (Eq. T2amp), S(D) = 1 + exp(-s D^2)
 *   (Eq. v_tilde). No four-index tensor is ever stored (section III).
 *
 * Conventions shared by every entry point:
 *   - Every array pointer is HIP device memory owned by the caller, FP64,
 *     C (row-major) order, 8-byte aligned. Nothing is retained after return.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls only enqueue work on it: they never synchronise and never
 *     allocate device memory. The caller keeps inputs, outputs and the
 *     workspace alive until that work completes. (dsrg_df_factors and
 *     dsrg_df_fock run the metric factor on one internal stream per host
 *     thread and device, forked from `stream` and joined back to it with
 *     events before anything reads it: to the caller their work is ordered
 *     on `stream`, and capturing `stream` in a graph captures it.)
 *   - Outputs are overwritten, never accumulated into.
 *   - Every argument is validated on the host before anything is enqueued.
 *     On any error the call returns a non-zero status, enqueues nothing and
 *     leaves every output untouched; dsrg_df_last_error() then describes it.
 *     NaN or Inf inside B or the orbital energies is not checked; it
 *     propagates into the results.
 *   - Not re-entrant on one workspace: two calls that overlap in time must
 *     use different workspaces.
 */
#ifndef DSRG_DF_H
#define DSRG_DF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DSRG_OK = 0,
  DSRG_ERR_ARG = 1,          /* invalid argument (null, bad size, bad value)   */
  DSRG_ERR_UNSUPPORTED = 2,  /* valid but not supported (e.g. na too large)    */
  DSRG_ERR_WORKSPACE = 3,    /* workspace missing or smaller than required     */
  DSRG_ERR_HIP = 4           /* the HIP runtime refused a launch               */
} dsrg_status;

/* Arithmetic of the (pq|rs) contractions. Denominators, regularisers and
 * every energy accumulation are FP64 in all modes. */
typedef enum {
  DSRG_FP64 = 0,        /* FP64 matrix-core contractions                         */
  DSRG_SPLIT_BF16 = 1,  /* B = hi + lo in BF16, three products, FP32 accumulate  */
  DSRG_SPLIT_OZAKI = 2  /* error-free int8 slices of B, exact int32 accumulate   */
} dsrg_precision;
/* DSRG_SPLIT_BF16 returns DSRG_ERR_UNSUPPORTED (three BF16 products cannot
 * reach 1e-6 Eh on these sizes). DSRG_SPLIT_OZAKI splits every column of B
 * (a vector over the auxiliary index) into four int8 slices and keeps the
 * ten slice products of levels <= 3; its int32 sums are exact for naux <=
 * DSRG_DF_MAX_SLICE_NAUX (larger naux returns DSRG_ERR_UNSUPPORTED). Its
 * gradient splits the longer adjoint contractions into segments. */
#define DSRG_DF_MAX_SLICE_NAUX 33000

/* Term mask bits (argument `terms`). */
enum {
  DSRG_TERM_CCVV = 1,   /* F1 */
  DSRG_TERM_CAVV = 2,   /* F2 */
  DSRG_TERM_CCAV = 4,   /* F3 */
  DSRG_TERM_ALL = 7,
  /* Option bit: reduce tile partial energies with FP64 atomics into one slot
   * per term instead of one slot per workgroup. Results then depend on the
   * order in which workgroups finish (last-bit differences run to run). */
  DSRG_OPT_ATOMIC_REDUCE = 0x100,
  /* Option bit: record a HIP event pair around every kernel the call
   * enqueues, so dsrg_df_kernel_times() can report per-kernel durations. */
  DSRG_OPT_KERNEL_TIMING = 0x200,
  /* Option bit (dsrg_df_energy, dsrg_df_energy_noalloc,
   * dsrg_df_energy_backward): check that the contribution of every CCVV work
   * item (one tile of virtual pairs (a, b) of one core pair) is <= 0, as
   * Eq. expensive makes it when every denominator e_i + e_j - e_a - e_b is
   * negative (R(Delta) <= 0 and (ia|jb)^2 - (ia|jb)(ib|ja) + (ib|ja)^2 >= 0).
   * A positive or NaN contribution sets bit 0 of the device's sign check
   * word (dsrg_df_sign_check). The library does not require the orbital
   * energies to be ordered; this is how a caller can learn that they were
   * not. The results are the same with and without the bit. */
  DSRG_OPT_CHECK_SIGNS = 0x400
};

/* One problem. Orbitals are ordered core | active | virtual; only the three
 * off-diagonal blocks of B that F1-F3 touch are read, and B is taken to be
 * symmetric in its two orbital indices (real orbitals), so the transposed
 * blocks are never needed. */
typedef struct {
  int64_t nc;            /* correlated core orbitals, >= 1 (frozen core excluded)  */
  int64_t na;            /* active orbitals, >= 0                                  */
  int64_t nv;            /* virtual orbitals, >= 1                                 */
  int64_t naux;          /* auxiliary (DF) or Cholesky vectors M, >= 1             */
  const double *B_cv;    /* [naux][nc][nv]  B^Q_{me}                               */
  const double *B_ca;    /* [naux][nc][na]  B^Q_{mu}  (may be NULL when na == 0)   */
  const double *B_av;    /* [naux][na][nv]  B^Q_{ue}  (may be NULL when na == 0)   */
  const double *eps_c;   /* [nc] semicanonical core orbital energies, Eh           */
  const double *eps_a;   /* [na] semicanonical active orbital energies (NULL if 0) */
  const double *eps_v;   /* [nv] semicanonical virtual orbital energies            */
  const double *gamma1;  /* [na][na] spin-summed active 1-RDM, symmetric (NULL if 0)*/
  double s;              /* flow parameter, Eh^-2, finite and >= 0                 */
} dsrg_df_problem;

/* Largest na the CAVV and CCAV kernels are compiled for. */
#define DSRG_DF_MAX_ACTIVE 8

/* Bytes of device workspace that dsrg_df_energy (with_grad == 0) or
 * dsrg_df_energy_backward (with_grad != 0) needs for this problem,
 * precision and term mask. Reads only the sizes in *p (no pointer is
 * dereferenced). Returns DSRG_OK and stores the size in *bytes. */
dsrg_status dsrg_df_workspace_size(const dsrg_df_problem *p, int precision,
                                   int terms, int with_grad, size_t *bytes);

/* Energies of the selected terms (Table II F1, F2, F3).
 *   E_terms   device [3]: E_CCVV, E_CAVV, E_CCAV in Eh; unselected terms are 0.
 *   workspace device buffer of at least dsrg_df_workspace_size(...) bytes,
 *             256-byte aligned; its contents on entry do not matter.
 * The energies are exactly 0 for s == 0 and tend to the closed-shell DF-MP2
 * form of Eq. expensive as s grows. */
dsrg_status dsrg_df_energy(const dsrg_df_problem *p, int precision, int terms,
                           double *E_terms, void *workspace, size_t ws_bytes,
                           void *stream);

/* dsrg_df_energy without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). The workspace is the library's own
 * static device array of DSRG_DF_NOALLOC_SCRATCH_BYTES per GPU, which each
 * GPU the library runs on holds until the process ends; the call allocates
 * nothing (the array's device address is looked up once per device, on the
 * first call made with that device current).
 *   E_terms  device [3], as for dsrg_df_energy.
 * Problems whose workspace (dsrg_df_workspace_size with with_grad == 0)
 * exceeds the array return DSRG_ERR_UNSUPPORTED without enqueuing anything.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (on different streams or host threads) race and must not be
 * made; calls ordered on one stream are safe (each clears what it needs).
 * DSRG_OPT_KERNEL_TIMING is refused (DSRG_ERR_ARG). Otherwise as
 * dsrg_df_energy, with the same results. */
#define DSRG_DF_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
dsrg_status dsrg_df_energy_noalloc(const dsrg_df_problem *p, int precision, int terms,
                                   double *E_terms, void *stream);

/* Gradient of L = sum_t gE[t] * E_t with respect to every input that the
 * energy depends on (the adjoint of dsrg_df_energy; amplitudes are
 * recomputed, never stored).
 *   gE                   device [3]: dL/dE_CCVV, dL/dE_CAVV, dL/dE_CCAV
 *   dB_cv, dB_ca, dB_av  device, shapes as B_cv, B_ca, B_av (dB_ca, dB_av may be
 *                        NULL when na == 0)
 *   deps_c, deps_a, deps_v  device [nc], [na], [nv]
 *   ds                   device [1]
 *   E_terms              optional device [3] (NULL = not wanted): the energies
 * Terms outside `terms` contribute nothing. dB and the energies are bitwise
 * reproducible run to run; deps_* and ds are summed with FP64 atomics and
 * can differ in the last bits between runs. */
dsrg_status dsrg_df_energy_backward(const dsrg_df_problem *p, int precision, int terms,
                                    const double *gE,
                                    double *dB_cv, double *dB_ca, double *dB_av,
                                    double *deps_c, double *deps_a, double *deps_v,
                                    double *ds, double *E_terms,
                                    void *workspace, size_t ws_bytes, void *stream);

/* ---- The remaining pieces F4..F8 of term F (Table II) ----
 * The five pieces of Eq. expensive_term with two or more active indices,
 * after the same spin summation (etab = 2 I - Gamma; x, y, u, v, w, z active):
 *
 *   F4 = 1/4 sum Gamma_xy Gamma_uv sum_{ef} (xe|uf) S(D^{ef}_{xu}) [2(ye|vf) - (yf|ve)] R1(D^{ef}_{yv})
 *   F5 = 1/4 sum etab_uv etab_xy sum_{mn} (mv|ny) S(D^{vy}_{mn}) [2(mu|nx) - (mx|nu)] R1(D^{ux}_{mn})
 *   F6 = sum Gamma_xy etab_uv sum_{me} S(D^{ve}_{mx}) R1(D^{ue}_{my})
 *          [(mv|xe)(mu|ye) + (me|xv)(me|yu) - ((mv|xe)(me|yu) + (me|xv)(mu|ye))/2]
 *   F7 = 1/4 sum Gamma_yw Gamma_zx etab_uv sum_e (yv|ze) S(D^{ve}_{yz}) [2(wu|xe) - (we|xu)] R1(D^{ue}_{wx})
 *   F8 = 1/4 sum Gamma_wz etab_uv etab_xy sum_m (mv|wy) S(D^{vy}_{mw}) [2(mu|zx) - (mx|zu)] R1(D^{ux}_{mz})
 *
 * They read, besides the blocks of *p, the active-active block of B. FP64
 * only; na <= DSRG_DF_MAX_ACTIVE. */

/* Bytes of device workspace that dsrg_df_energy_active needs for *p (sizes
 * only, no pointer is dereferenced). */
dsrg_status dsrg_df_active_workspace_size(const dsrg_df_problem *p, size_t *bytes);

/* F4..F8 of the problem.
 *   B_aa      device [naux][na][na]  B^Q_{uv}, symmetric in u, v (may be NULL
 *             when na == 0)
 *   options   0 or DSRG_OPT_KERNEL_TIMING
 *   F_terms   device [5]: F4, F5, F6, F7, F8 in Eh (all 0 when na == 0)
 *   workspace device buffer of at least dsrg_df_active_workspace_size(...)
 *             bytes, 256-byte aligned; its contents on entry do not matter.
 * Every term is exactly 0 for s == 0. Errors as for dsrg_df_energy. */
dsrg_status dsrg_df_energy_active(const dsrg_df_problem *p, const double *B_aa, int options,
                                  double *F_terms, void *workspace, size_t ws_bytes,
                                  void *stream);

/* ---- The other terms of the second-order energy (Table I): A, B, C, D, E,
 * G, H, I, J, K ----
 * With X_{p..}^{q..} the coefficient of a+_p .. a_q .. (lower indices
 * created, upper annihilated), gamma_p^q = <a+_p a_q>, eta = 1 - gamma, the
 * two- and three-body cumulants lambda of section II.A, holes i, j, k, l in
 * C + A, particles a, b, c, d in A + V, core m, virtual e, active u..z, the
 * terms are, in spin orbitals (2k + s for spatial orbital k and spin s),
 *   A = f~_j^b t_a^i gamma_j^i eta_a^b
 *   B = 1/2 v~_{xy}^{ev} t_e^u lambda_{xy}^{uv}    C = -1/2 v~_{my}^{uv} t_x^m lambda_{xy}^{uv}
 *   D = 1/2 f~_x^e t_{ey}^{uv} lambda_{xy}^{uv}    E = -1/2 f~_m^v t_{xy}^{um} lambda_{xy}^{uv}
 *   G = 1/8 v~_{xy}^{cd} t_{ab}^{uv} eta_a^c eta_b^d lambda_{xy}^{uv}
 *   H = 1/8 v~_{kl}^{uv} t_{xy}^{ij} gamma_k^i gamma_l^j lambda_{xy}^{uv}
 *   I = v~_{jx}^{bu} t_{ay}^{iv} gamma_j^i eta_a^b lambda_{xy}^{uv}
 *   J = 1/4 v~_{mz}^{uv} t_{xy}^{mw} lambda_{xyz}^{uvw}   K = 1/4 v~_{xy}^{we} t_{ez}^{uv} lambda_{xyz}^{uvw}
 * with t_{ab}^{ij} = <ab||ij> R1(D^{ij}_{ab}) (Eq. T2amp), v~ = <ab||ij>
 * S(D^{ij}_{ab}) (Eq. v_tilde), t_a^i = [f_a^i + sum_ux D_u^x t_{ax}^{iu}
 * gamma_x^u] R1(D_a^i) (Eq. T1amp, D_u^x = e_x - e_u), f~_a^i = f_a^i S(D) +
 * [sum_ux D_u^x t_{ax}^{iu} gamma_x^u] exp(-s D^2) (Eq. f_tilde), the all-
 * active amplitudes excluded, restricted orbitals (<pq||rs> from (pq|rs) =
 * sum_Q B^Q_pq B^Q_rs). Term F is dsrg_df_energy plus dsrg_df_energy_active
 * (F1..F8). FP64. */
typedef struct {
  dsrg_df_problem base;     /* sizes, B_cv, B_ca, B_av, eps_c, eps_a, eps_v and s as for
                               dsrg_df_energy (gamma1 is not read)                        */
  const double *B_aa;       /* [naux][na][na] B^Q_{uv}, symmetric in u, v                  */
  const double *f_ca;       /* [nc][na] first-order Fock elements f_{mu}: the off-diagonal */
  const double *f_cv;       /* [nc][nv] blocks of the generalized Fock matrix in the       */
  const double *f_av;       /* [na][nv] semicanonical basis                                */
  const double *rdm1;       /* [2na][2na] active spin-orbital <a+_p a_q> (p = 2u + spin)   */
  const double *lambda2;    /* [2na]^4 lambda_{pq}^{rs} at [p][q][r][s]                    */
  const double *lambda3;    /* [2na]^6 lambda_{pqr}^{stu} at [p][q][r][s][t][u]            */
} dsrg_df_rest_problem;

/* Bytes of device workspace that dsrg_df_energy_rest needs (sizes only). */
dsrg_status dsrg_df_rest_workspace_size(const dsrg_df_rest_problem *p, size_t *bytes);

/* terms device [10]: A, B, C, D, E, G, H, I, J, K in Eh (all 0 when na == 0).
 * options 0 or DSRG_OPT_KERNEL_TIMING. na <= DSRG_DF_MAX_ACTIVE. Errors as
 * for dsrg_df_energy. */
dsrg_status dsrg_df_energy_rest(const dsrg_df_rest_problem *p, int options, double *terms,
                                void *workspace, size_t ws_bytes, void *stream);

/* Cumulants of section II.A from the active spin-orbital reduced density
 * matrices (2 na spin orbitals, device arrays):
 *   rdm1 [2na][2na] <a+_p a_q>, rdm2 [2na]^4 <a+_p a+_q a_s a_r> at [p][q][r][s],
 *   rdm3 [2na]^6 <a+_p a+_q a+_r a_u a_t a_s> at [p][q][r][s][t][u];
 *   lambda2 = rdm2 - rdm1 ^ rdm1, lambda3 = rdm3 - (antisymmetrized rdm1
 *   lambda2) - (antisymmetrized rdm1 rdm1 rdm1), written to lambda2 [2na]^4 and
 *   lambda3 [2na]^6 (device). 1 <= na <= DSRG_DF_MAX_ACTIVE. */
dsrg_status dsrg_df_cumulants(int64_t na, const double *rdm1, const double *rdm2,
                              const double *rdm3, double *lambda2, double *lambda3,
                              void *stream);

/* ---- Density-fitting factors (Eq. int_fact and the DF definition of
 * section II.C): B^Q_pq = sum_P [J^{-1/2}]_{QP} (pq|P) with the MO
 * three-index integrals (pq|P) = sum_{mu nu} C_{mu p} C_{nu q} (mu nu|P).
 * The factor of J^{-1} taken here is L^{-1} with J = L L^T (Cholesky): the
 * factors differ from the symmetric-root ones by an orthogonal rotation of
 * Q, so every (pq|rs) = sum_Q B^Q_pq B^Q_rs and every energy is the same. */
typedef struct {
  int64_t nao;           /* AO basis functions, >= 1                                */
  int64_t nmo;           /* molecular orbitals (columns of C), >= nfrz+nc+na+nv    */
  int64_t naux;          /* auxiliary basis functions, >= 1                         */
  int64_t nfrz, nc, na, nv; /* frozen core, correlated core, active, virtual MOs    */
  const double *ao3;     /* [naux][nao][nao] (mu nu|P) (symmetric in mu, nu by its
                            definition; the build does not rely on it)              */
  const double *J;       /* [naux][naux] two-centre metric, symmetric positive
                            definite (otherwise the factors contain NaN); or NULL:
                            ao3 then holds factors of the AO integrals already
                            (the CD vectors B^Q_{mu nu} of dsrg_df_cholesky, naux
                            of them) and no metric is applied                      */
  const double *C;       /* [nao][nmo] MO coefficients; columns ordered frozen core
                            | core | active | virtual (| any further orbitals)      */
} dsrg_dfgen_problem;

/* Bytes of device workspace that dsrg_df_factors needs (sizes only). */
dsrg_status dsrg_df_factors_workspace_size(const dsrg_dfgen_problem *p, size_t *bytes);

/* The blocks of B that the energies read, in the layout of dsrg_df_problem:
 *   B_cv [naux][nc][nv], B_ca [naux][nc][na], B_av [naux][na][nv],
 *   B_aa [naux][na][na] (device; the last three may be NULL when na == 0)
 *   options  0 or DSRG_OPT_KERNEL_TIMING
 * FP64 throughout. Errors as for dsrg_df_energy. */
dsrg_status dsrg_df_factors(const dsrg_dfgen_problem *p, int options, double *B_cv,
                            double *B_ca, double *B_av, double *B_aa, void *workspace,
                            size_t ws_bytes, void *stream);

/* ---- Cholesky-decomposition factors (CD approach of section II.C): a
 * pivoted Cholesky decomposition of the AO two-electron integrals stopped at
 * a threshold, (mu nu|la si) ~= sum_{Q < rank} B^Q_{mu nu} B^Q_{la si}.
 * Greedy pivoting: step k takes the pair p with the largest diagonal d of the
 * residual M - sum_{Q<k} L^Q L^Q^T (the smallest pair index on ties) and stops
 * if d_p <= tol; otherwise L^k = (M_{p .} - sum_{Q<k} L^Q L^Q_p) / sqrt(d_p).
 * The residual of a positive semidefinite M stays positive semidefinite, so
 * on convergence every integral is reproduced to within tol. */
#define DSRG_CD_MAX_NAO 16384
typedef struct {
  int64_t nao;        /* AO basis functions, 1 .. DSRG_CD_MAX_NAO; npair =
                         nao (nao + 1) / 2                                          */
  const double *M;    /* [npair][npair] (mu nu|la si) over packed pairs mu >= nu,
                         pair index mu (mu + 1) / 2 + nu (device); symmetric
                         positive semidefinite; only its diagonal and the pivot
                         rows are read                                              */
  double tol;         /* CD threshold >= 0 (Eh), e.g. 1e-5                          */
  int64_t max_rank;   /* most vectors, 0 .. npair; one kernel launch per vector is
                         enqueued, so keep it near the rank expected            */
} dsrg_cd_problem;

/* Bytes of device workspace that dsrg_df_cholesky needs (sizes only). */
dsrg_status dsrg_df_cholesky_workspace_size(const dsrg_cd_problem *p, size_t *bytes);

/* B [max_rank][nao][nao] (device): B^Q_{mu nu} = B^Q_{nu mu} for Q < rank,
 * zero for rank <= Q < max_rank (may be NULL when max_rank == 0).
 *   rank    device int64: vectors made; < max_rank means converged, == max_rank
 *           means converged only if *dmax <= tol
 *   dmax    device double: the largest residual diagonal when it stopped
 *   pivots  device int64 [max_rank] (or NULL): the pair index of each step
 *   options 0 or DSRG_OPT_KERNEL_TIMING
 * rank and dmax are written on the stream like every output: read them after
 * the stream has reached this call's end. FP64 throughout. Errors as for
 * dsrg_df_energy (nao too large: DSRG_ERR_UNSUPPORTED). */
dsrg_status dsrg_df_cholesky(const dsrg_cd_problem *p, int options, double *B, int64_t *rank,
                             double *dmax, int64_t *pivots, void *workspace, size_t ws_bytes,
                             void *stream);

/* ---- Laplace-type factorization of the CCVV Coulomb part (the outlook of
 * section VI: a decomposition of the renormalised denominators). With
 * x = e_a + e_b - e_i - e_j > 0 the regulariser of Eq. expensive is
 * R = -h(x), h(x) = (1 - exp(-2 s x^2)) / x; an exponential sum
 * h(x) ~ sum_k w_k exp(-t_k x) on an interval holding every x separates over
 * the four orbital energies, and the Coulomb part of E_CCVV,
 * E_J = 2 sum_{ij,ab} (ia|jb)^2 R(Delta), becomes
 *   E_J ~ -2 sum_k w_k S_k,  S_k = sum_PQ (Y_k)_PQ^2,
 *   Y_k[P][Q] = sum_{ia} B^P_ia B^Q_ia exp(-t_k (e_a - e_i)),
 * 2 naux^2 nc nv flops per term (fourth order) instead of the fifth-order
 * pair sum. The exchange part of E_CCVV does not separate this way and is
 * not computed here. */
#define DSRG_DF_MAX_LAPLACE_TERMS 64

/* The exponential sum (host, no device work): exponents t_k on a geometric
 * grid from c1 / x_hi to c2 / x_lo, weights by linear least squares on 600
 * logarithmically spaced points of [x_lo, x_hi]; (c1, c2) from {0.1, 0.3,
 * 1.0} x {3, 10, 30}, the pair whose fit has the smallest largest absolute
 * error max_err on 5000 such points. t, w: host arrays [nq], 1 <= nq <=
 * DSRG_DF_MAX_LAPLACE_TERMS; 0 < x_lo < x_hi (for a problem: x_lo = 2
 * (min e_v - max e_c), x_hi = 2 (max e_v - min e_c)); s >= 0 (s = 0: zero
 * weights). The weights alternate in sign for larger nq: their cancellation
 * costs up to about 1e6 of the FP64 rounding unit at nq = 20. */
dsrg_status dsrg_df_laplace_fit(double s, double x_lo, double x_hi, int nq, double *t, double *w,
                                double *max_err);

/* Bytes of device workspace that dsrg_df_coulomb_laplace needs (sizes only;
 * up to about 2 GiB of scaled factors and Y_k per batch of terms). */
dsrg_status dsrg_df_laplace_workspace_size(const dsrg_df_problem *p, int nq, size_t *bytes);

/* E [1] (device): -2 sum_k w_k S_k from B_cv, eps_c and eps_v of p (na, B_ca,
 * B_av, gamma1 and s are not read); S [nq] (device, or NULL): the S_k.
 * t, w: host arrays [nq] (t_k > 0), e.g. from dsrg_df_laplace_fit.
 * options 0 or DSRG_OPT_KERNEL_TIMING. FP64 throughout. Errors as for
 * dsrg_df_energy. */
dsrg_status dsrg_df_coulomb_laplace(const dsrg_df_problem *p, int nq, const double *t,
                                    const double *w, int options, double *E, double *S,
                                    void *workspace, size_t ws_bytes, void *stream);

/* ---- Generalized Fock matrix (Eq. gen_fock) over all MOs from the same DF
 * integrals (pq|rs) = sum_PQ (pq|P) [J^{-1}]_PQ (Q|rs):
 *   f_pq = h_pq + sum_{i in frozen+core} [2 (pq|ii) - (pi|qi)]
 *        + sum_{uv in active} Gamma_uv [(pq|uv) - (pu|qv) / 2]
 * (the spin-orbital f_pq = h_pq + sum_rs <pr||qs> gamma_sr with doubly
 * occupied frozen and core orbitals and the spin-summed active density
 * Gamma; spin-orbital gamma = Gamma / 2 in each spin block). */
typedef struct {
  dsrg_dfgen_problem df; /* sizes, ao3, J and C as for dsrg_df_factors; here the
                            symmetry of ao3 in mu, nu is relied on             */
  const double *h;       /* [nmo][nmo] one-electron integrals, MO basis          */
  const double *gamma1;  /* [na][na] spin-summed active 1-RDM (NULL if na == 0)  */
} dsrg_fock_problem;

/* Bytes of device workspace that dsrg_df_fock needs (sizes only). */
dsrg_status dsrg_df_fock_workspace_size(const dsrg_fock_problem *p, size_t *bytes);

/* F [nmo][nmo] (device): the generalized Fock matrix, FP64.
 *   options   0 or DSRG_OPT_KERNEL_TIMING
 *   workspace device buffer of at least dsrg_df_fock_workspace_size(...)
 *             bytes, 256-byte aligned; its contents on entry do not matter.
 * Errors as for dsrg_df_energy. */
dsrg_status dsrg_df_fock(const dsrg_fock_problem *p, int options, double *F, void *workspace,
                         size_t ws_bytes, void *stream);

/* ---- Semicanonical orbitals (section II.B): the orthogonal U that
 * diagonalizes the core, active and virtual diagonal blocks of a generalized
 * Fock matrix F, eps = diag(U^T F U), and optionally C U. U is block-diagonal
 * over frozen | core | active | virtual, the identity on the frozen core and
 * on any orbitals past the virtual space (whose eps are the diagonal of F); within each block the eigenvalues ascend and
 * each eigenvector has its component of largest magnitude positive. */
typedef struct {
  int64_t nao;              /* rows of C (ignored when C is NULL)               */
  int64_t nmo;              /* order of F, >= nfrz + nc + na + nv               */
  int64_t nfrz, nc, na, nv; /* frozen core, core, active, virtual orbitals      */
  const double *F;          /* [nmo][nmo] symmetric generalized Fock matrix    */
  const double *C;          /* [nao][nmo] MO coefficients, or NULL              */
} dsrg_semican_problem;

/* Bytes of device workspace that dsrg_df_semicanonicalize needs. */
dsrg_status dsrg_df_semicanonicalize_workspace_size(const dsrg_semican_problem *p,
                                                    size_t *bytes);

/* U [nmo][nmo], eps [nmo] and, when C and Cs are both given, Cs = C U
 * [nao][nmo] (device, FP64). Jacobi rotations to an off-diagonal norm below
 * 1e-14 of the block's norm, or 40 block sweeps at most (a random spectrum
 * takes about 8, one with large exactly degenerate multiplets converges
 * linearly and takes 20-25; blocks of up to 32 orbitals: 40 inner sweeps at
 * most). The launches of the sweeps after convergence return at once.
 *   info  optional device int [1] (NULL = not wanted, 4-byte aligned): once
 *         the call's work has run, the bit mask of the blocks whose
 *         off-diagonal norm never met the criterion (bit 0 core, bit 1
 *         active, bit 2 virtual; 0 = every block converged). Written by
 *         kernels on `stream`: read it after synchronising, the call itself
 *         never waits. U and eps are returned in either case.
 * Errors as for dsrg_df_energy. */
dsrg_status dsrg_df_semicanonicalize(const dsrg_semican_problem *p, int options, double *U,
                                     double *eps, double *Cs, int *info, void *workspace,
                                     size_t ws_bytes, void *stream);

/* The current device's sign check word (see DSRG_OPT_CHECK_SIGNS): waits for
 * every stream of the device to finish (hipDeviceSynchronize), stores the word
 * in *word (host; bit 0: some CCVV work item of a call made with the option
 * since the last read gave a positive or NaN contribution) and clears it.
 * DSRG_ERR_ARG if word is NULL, DSRG_ERR_HIP if a HIP call fails. */
dsrg_status dsrg_df_sign_check(unsigned *word);

/* Text of the last error raised on the calling thread ("" if none). Valid
 * until the next dsrg_df_* call on that thread. */
const char *dsrg_df_last_error(void);

/* Per-kernel device durations (milliseconds) recorded on this thread by the
 * calls that set DSRG_OPT_KERNEL_TIMING since the previous read (at most 512
 * kernels; later ones are not recorded). Waits for those kernels to finish,
 * writes at most `cap` entries to ms[] and, if names != NULL, a static name
 * per entry, clears the record and returns the number of kernels recorded
 * (-1 if an event could not be read). Entries are in launch order. */
int dsrg_df_kernel_times(double *ms, const char **names, int cap);

/* Restricts the kernels that DSRG_OPT_KERNEL_TIMING records on the calling
 * thread to those named in `names`, a comma-separated list of the names
 * dsrg_df_kernel_times() reports (e.g. "ccvv_fp64"); NULL or "" records every
 * kernel again. Fewer event pairs leave the timed calls closer to their
 * untimed cost. The list is copied; DSRG_ERR_ARG if it is 256 characters or
 * longer (the filter is then unchanged). */
dsrg_status dsrg_df_timing_filter(const char *names);

/* The gradient (dsrg_df_energy_backward) forms its adjoint tiles per block of
 * core orbitals: the CCVV tiles of one block pair (gb 64 ceil(nv/64))^2
 * doubles, or the CAVV integrals and adjoint rows of one block, in one
 * workspace region, never the tiles of all nc^2 core pairs at once (section
 * III: no four-index storage). gb is the largest number of core orbitals
 * whose region fits `bytes` (at least one orbital, so a bound below one
 * orbital's need is exceeded), balanced over the blocks. 0 restores the
 * default of 1 GiB. Process-wide; it changes what dsrg_df_workspace_size
 * reports for the gradient, so set it before querying the size (a call
 * whose workspace has become too small returns DSRG_ERR_WORKSPACE). Smaller
 * blocks trade memory for shorter adjoint products; the results differ from
 * those of other block sizes only by the order of FP64 additions.
 * DSRG_ERR_ARG for a bound above 2^50 bytes. */
dsrg_status dsrg_df_set_gradient_block_bytes(size_t bytes);
/* The bound in force. */
size_t dsrg_df_gradient_block_bytes(void);

/* Matrix-core rate probe: a measurement aid for the rooflines of the tile
 * kernels (its callers are benchmarks), not a step of the method. Enqueues
 * on `stream` one launch of nwg workgroups of eight waves (two per SIMD);
 * each wave takes `iters` rounds of eight matrix products on register
 * operands of full-entropy random bits, each product of a round taking
 * another A and another B operand (the operand statistics of the tile
 * kernels, without their memory traffic):
 *   DSRG_PROBE_I8:  v_mfma_i32_32x32x32_i8, 65536 int8 operations a product;
 *   DSRG_PROBE_F64: v_mfma_f64_16x16x4f64, 2048 flops a product.
 * Operations per launch: nwg * 8 * iters * 8 * (65536 or 2048).
 * stamps: device int64 [4 nwg]; for workgroup g, stamps[4g .. 4g+1] = the
 *   shader cycle counter and the constant-rate counter before its products
 *   and stamps[4g+2 .. 4g+3] the same after them, so the clock the products
 *   ran at is cycles / (ticks / hipDeviceAttributeWallClockRate).
 * sink: device buffer of nwg * 512 values (uint32 for DSRG_PROBE_I8, double
 *   for DSRG_PROBE_F64) into which each thread folds its accumulators, so
 *   that no product can be dropped as dead code.
 * DSRG_ERR_ARG for an unknown kind, nwg outside [1, 65536], iters outside
 * [1, 2^24], or a stamps or sink pointer that is NULL or not 8-byte aligned. */
#define DSRG_PROBE_I8 0
#define DSRG_PROBE_F64 1
dsrg_status dsrg_df_mfma_probe(int kind, int64_t nwg, int64_t iters, int64_t *stamps, void *sink,
                               void *stream);

/* Library version as major*10000 + minor*100 + patch. */
int dsrg_df_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DSRG_DF_H */
