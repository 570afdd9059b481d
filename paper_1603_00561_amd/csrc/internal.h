// Internal declarations shared by the host ABI layer and the HIP kernels of
// libdsrgdf. Not part of the public interface (include/dsrg_df.h is).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace dsrg {

// Width of one packed virtual-orbital panel (columns) and the auxiliary-index
// chunk that the contraction kernels stage through LDS per step.
constexpr int kPanel = 64;
constexpr int kChunk = 16;
// Term mask selecting all three terms.
constexpr int kAllTerms = 7;
// Column width of a packed active-orbital panel (na padded up to this).
constexpr int kActPanel = 16;
// Persistent workgroups of the int8 CCVV kernel, each with an FP64 slot of
// 512 lanes x 32 values for the first product of a two-product tile.
constexpr int kSlicePersistWG = 256;
constexpr int kPersistCU = 256;   // compute units the persistent FP64 CCVV grid is sized for
constexpr int64_t kSliceXsDoubles = 512 * 32;
// followed by eight per-XCD work counters (ints; cleared before each launch)
constexpr size_t kSliceCounterBytes = 64;

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
// typed views of a workspace section
inline double *ws_d(void *ws, size_t off) {
  return reinterpret_cast<double *>(static_cast<char *>(ws) + off);
}
inline int8_t *ws_b(void *ws, size_t off) {
  return reinterpret_cast<int8_t *>(static_cast<char *>(ws) + off);
}
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
// K segments of an adjoint product with a rows x ncols output (128 x 128
// tiles; `slots` workgroups run at once: two per CU for the FP64 product),
// each segment at least 512 long and at most nmax of them. An output with
// fewer than 1024 tiles takes enough segments for about 1024 workgroups; a
// larger one takes the count from 1 to 4 that best fills the last round of
// workgroups, ceil(tiles n / slots) / n rounds of the whole contraction, with
// 1.5 % per extra segment for writing and adding the partial products.
inline int64_t adj_segments(int64_t rows, int64_t ncols, int64_t K, int64_t slots = 512,
                            int64_t nmax = (int64_t)1 << 30) {
  const int64_t tiles = ceil_div(rows, 128) * ceil_div(ncols, 128);
  int64_t kmax = K / 512;
  if (kmax > nmax) kmax = nmax;
  if (kmax < 1) kmax = 1;
  if (tiles < 1024) {
    int64_t n = ceil_div(1024, tiles > 0 ? tiles : 1);
    if (n > kmax) n = kmax;
    return n < 1 ? 1 : n;
  }
  int64_t best = 1;
  double bcost = 1e300;
  for (int64_t n = 1; n <= 4 && n <= kmax; ++n) {
    const double cost = (double)ceil_div(tiles * n, slots) / (double)n * (1.0 + 0.015 * (double)(n - 1));
    if (cost < bcost * (1.0 - 1e-9)) {
      bcost = cost;
      best = n;
    }
  }
  return best;
}
// output columns of an adjoint product whose ncols columns come in groups of
// GP of which the first nvalid are kept
inline int64_t adj_out_cols(int64_t ncols, int64_t GP, int64_t nvalid) {
  const int64_t rem = ncols % GP;
  return (ncols / GP) * nvalid + (rem < nvalid ? rem : nvalid);
}
// columns of the FP64 adjoint products' tile space: with nvalid even, the valid
// columns of every group of GP side by side, else the padded index space
inline int64_t adj_fp64_cols(int64_t ncols, int64_t GP, int64_t nvalid) {
  return (nvalid % 2 == 0 && ncols % GP == 0) ? (ncols / GP) * nvalid : ncols;
}
// Segments of an FP64 adjoint product, their partial products bounded by
// kAdjPartBytes.
constexpr int64_t kAdjPartBytes = (int64_t)512 << 20;
inline int64_t adj_fp64_segments(int64_t rows, int64_t ncols, int64_t GP, int64_t nvalid,
                                 int64_t K) {
  const int64_t part = 8 * rows * adj_out_cols(ncols, GP, nvalid);
  const int64_t cap = part > 0 ? kAdjPartBytes / part : 1;
  return adj_segments(rows, adj_fp64_cols(ncols, GP, nvalid), K, 512, cap < 1 ? 1 : cap);
}
// contraction indices per exact int32 segment of the int8 adjoint products
// (|I_L| <= 4 127^2 kGemmSeg < 2^31)
constexpr int64_t kGemmSeg = 32768;
constexpr int64_t kQChunk = 32;   // contraction chunk of the int8 operand panels
// K segments of an int8 adjoint product (128 x 128 output tiles): at least
// enough for exact int32 sums, more when the output has too few tiles to
// fill the chip; they always run side by side (partial products summed in a
// fixed order). Returns the segment count and their length in chunks.
inline int64_t i8_segments(int64_t rows, int64_t ncols, int64_t K, int64_t &segc) {
  const int64_t nqc = ceil_div(K, kQChunk);
  // (the last-round rule of adj_segments is for the FP64 products; an int8
  // product with 1024 tiles or more keeps one segment unless exactness needs more)
  const int64_t tiles = ceil_div(rows, 128) * ceil_div(ncols, 128);
  const int64_t want = tiles < 1024 ? adj_segments(rows, ncols, K) : 1;
  const int64_t seg = kGemmSeg / kQChunk;
  segc = ceil_div(nqc, want);
  if (segc > seg) segc = seg;
  if (segc < 1) segc = 1;
  return ceil_div(nqc, segc);
}
// Bytes for the adjoint tiles of one block of core orbitals in the gradient:
// the CCVV tiles of a block pair and the CAVV integrals with their adjoint
// rows share one region, whose size bounds the core orbitals per block.
constexpr int64_t kGradBlockBytes = (int64_t)1 << 30;

// Everything the launchers need, derived once on the host from the problem.
struct Plan {
  int64_t nc, na, nv, naux;
  int64_t naux_p;   // naux rounded up to kChunk
  int64_t ntv;      // number of kPanel-wide virtual panels
  int64_t ntv_s;    // panels of the int8 slices (ntv rounded up to even: 128-wide tiles)
  int64_t xld;      // row length (doubles) of the CAVV integral batch
  double s;
  int precision;
  int terms;
  bool atomic_reduce;
  unsigned *chk = nullptr;   // CCVV sign check word (DSRG_OPT_CHECK_SIGNS), else nullptr
  bool with_grad;

  // work counts (workgroups) per term
  int64_t n_ccvv, n_cavv, n_ccav;
  int64_t ccav_cols; // padded (n, u) column count of the CCAV integral block

  // workspace layout (byte offsets, 256-aligned)
  size_t off_pcv, off_pav, off_pca;   // packed FP64 panels
  size_t off_j;                       // CCAV integrals (me|nu)
  size_t off_jscr = 0;                // their per-segment partial sums (energy path)
  bool ccav_split = false;            // the CCAV contraction is split over Q segments
  // int8 slice path
  int64_t nqc;                        // chunks of 32 auxiliary indices
  int64_t cavv_mb;                    // core orbitals per CAVV integral batch
  size_t off_s8c, off_s8a, off_sigc, off_siga, off_diag, off_xb, off_scr;
  size_t off_xs;                      // per-workgroup x slots of the int8 CCVV kernel, then its work counters
  size_t off_gs, off_g2, off_g3;      // adjoint tiles (gradient only): Gs and G2 of one
                                      // block of core orbitals (aliased with off_xb), G3 whole
  int64_t gb = 0, ngb = 0;            // gradient: core orbitals per block, number of blocks
  size_t off_gpart = 0;               // per-segment partial adjoint products (FP64 gradient)
  int64_t gpart_doubles = 0;          // their capacity; 0: products are not split
  // int8 adjoint products (slice-path gradient): operand slices and scales
  size_t off_SA1, off_SA2, off_SB, off_sigA1, off_sigA2, off_sigB, off_opmax;
  size_t off_ctr;                     // eight per-XCD work counters (ints)
  size_t off_slots;                   // per-workgroup partial energies
  size_t off_acc;                     // [4] atomic accumulators
  size_t total;

  int64_t slot_base[3];               // first slot of each term
};

struct Inputs {
  const double *B_cv, *B_ca, *B_av;
  const double *eps_c, *eps_a, *eps_v, *gamma1;
};

struct BwdOut {
  double *dB_cv, *dB_ca, *dB_av;
  double *deps_c, *deps_a, *deps_v, *ds;
  const double *gE;
};

// number of A<B tile pairs, and the closed-form counts of the CCVV work list
inline int64_t tri_off(int64_t n) { return n * (n - 1) / 2; }

// The pieces F4-F8 of term F (two or more active indices), FP64.
constexpr int64_t kActPairGrid = 2048;   // workgroups of the F4, F5, F6 element loops
struct ActivePlan {
  int64_t nc, na, nv, naux;
  int64_t naux_p, ntv, W;   // W = ntv kPanel: padded virtual row length
  double s;
  int64_t ncC, ncA;         // flattened (m, u) and (u, v) columns, padded to 16
  size_t off_pav, off_pcv, off_pca, off_rca, off_raa;   // packed operands
  size_t off_x;             // X[x][u][e][f] = (xe|uf)
  size_t off_ja1, off_ja2, off_jc1, off_jk, off_je;    // integral blocks with active indices
  size_t off_jpart;         // per-segment partial integral blocks (the largest of the five)
  size_t off_ctr, off_slots;
  int64_t slot_base[5], slot_count[5];
  size_t total;
};

struct ActiveInputs {
  const double *B_cv, *B_ca, *B_av, *B_aa;
  const double *eps_c, *eps_a, *eps_v, *gamma1;
};

// The density-fitting factor build (FP64).
struct DFPlan {
  int64_t nao, nmo, naux, nfrz, nc, na, nv;
  bool metric;   // false: ao3 holds factors already (CD vectors), no J applied
  size_t off_t, off_y, off_l, off_x, off_tmp, off_bf;
  size_t total;
};
struct DFInputs {
  const double *ao3, *J, *C;
};
struct DFOutputs {
  double *B_cv, *B_ca, *B_av, *B_aa;
};

// ---- Table I terms A-E, G-K (rest_terms.hip) ----
constexpr int kRestTerms = 10;     // A, B, C, D, E, G, H, I, J, K
constexpr int kRestKernels = 12;   // reduction kernels (G and H in two pieces each)
struct RestPlan {
  int64_t nc, na, nv, naux;
  double s;
  size_t off_pcv, off_pav, off_pca, off_paa, off_qvc, off_kcc, off_x, off_wt, off_wv, off_tcc,
      off_vcc, off_t1, off_ft, off_y, off_tp, off_lp, off_ci, off_ak, off_bk, off_y2, off_slots;
  int64_t grid[kRestKernels], slot[kRestKernels];   // workgroups and first slot per kernel
  size_t total;
};
struct RestInputs {
  const double *B_cv, *B_ca, *B_av, *B_aa, *eps_c, *eps_a, *eps_v, *f_ca, *f_cv, *f_av, *rdm1,
      *lambda2, *lambda3;
};
hipError_t launch_rest_terms(const RestPlan &pl, const RestInputs &in, void *ws, double *out,
                             hipStream_t st);
void rest_grids(int64_t nc, int64_t na, int64_t nv, int64_t *grid);
// lambda2, lambda3 from the spin-orbital RDMs of n active spin orbitals
hipError_t launch_cumulants(int n, const double *g1, const double *g2, const double *g3,
                            double *l2, double *l3, hipStream_t st);

// ---- the library's static device scratch (noalloc.hip) ----
// Capacity of the array behind dsrg_df_energy_noalloc (bytes, per device).
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
// Device address of the current device's array (looked up once per device).
hipError_t noalloc_scratch(void **ptr);

// ---- the CCVV sign check word of DSRG_OPT_CHECK_SIGNS (checks.hip) ----
// Device address of the current device's word (looked up once per device).
hipError_t sign_check_ptr(unsigned **ptr);
// Waits for the current device, copies its word to *word and clears it.
hipError_t sign_check_read(unsigned *word);
// matrix-core rate probe (probe.hip): kind 0 int8, 1 FP64
hipError_t launch_mfma_probe(int kind, int64_t nwg, int64_t iters, int64_t *stamps, void *sink,
                             hipStream_t st);

// ---- per-kernel timing (api.cpp); no-ops unless the call asked for it ----
void timer_begin(const char *name, hipStream_t st);
void timer_end(hipStream_t st);

// ---- launchers (fp64_kernels.hip) ----
hipError_t launch_pack_fp64(const Plan &pl, const Inputs &in, void *ws, hipStream_t st);
hipError_t launch_energy_fp64(const Plan &pl, const Inputs &in, void *ws, hipStream_t st);
hipError_t launch_finalize(const Plan &pl, void *ws, double *E_terms, hipStream_t st);
hipError_t launch_ccav_fp64(const Plan &pl, const Inputs &in, void *ws, hipStream_t st);
hipError_t launch_zero(double *p, int n, hipStream_t st);
// P[(r ntile + t)][Q][c] = B[Q][r][t width + c] (zero outside), rows Q padded to naux_p
hipError_t launch_pack_panels(const double *B, double *P, int64_t nrow, int64_t ncol,
                              int64_t naux, int64_t naux_p, int64_t ntile, int width,
                              hipStream_t st);
// X[ml][u][e][f] = sum_Q L^Q_{(m0+ml) e} R^Q_{u f} for ml < mb, u < nright, from
// 64-wide panels (row length ntv 64, nv valid); ctr: eight work counters,
// cleared here. tri (L = R, m0 = 0, mb = nright): only the blocks ml <= u are
// written.
hipError_t launch_x_fp64(const double *Pleft, const double *Pright, int nright, int ntv, int nv,
                         int64_t naux_p, int m0, int mb, int *ctr, double *Xb, bool tri,
                         hipStream_t st);
// Column blocks of 16 per workgroup of the J contraction: the largest of 4,
// 3, 2, 1 that divides the block count, so no workgroup reads past the end.
inline int j_column_blocks(int64_t ncols) {
  const int64_t nblk = ncols / 16;
  return (nblk % 4 == 0) ? 4 : (nblk % 3 == 0) ? 3 : (nblk % 2 == 0) ? 2 : 1;
}
// Auxiliary-index segments of a J contraction with a scratch buffer: enough
// to give about 1024 workgroups, each segment at least four 16-row chunks.
inline int64_t j_segments(int64_t npanels, int64_t ncols, int64_t naux_p) {
  const int64_t wgs = npanels * (ncols / (16 * j_column_blocks(ncols)));
  int64_t nseg = ceil_div(1024, wgs > 0 ? wgs : 1);
  const int64_t cap = naux_p / (4 * kChunk);
  if (nseg > cap) nseg = cap;
  return nseg < 1 ? 1 : nseg;
}
// J[panel 64 + r][c] = sum_Q Pleft[panel][Q][r] R[Q][c], R row-major [naux_p][ncols],
// ncols a multiple of 16. With scratch (j_segments(...) npanels 64 ncols doubles)
// the auxiliary range is split into segments whose partial J are summed in a
// fixed order; without it (nullptr) one pass.
hipError_t launch_j_fp64(const double *Pleft, int64_t npanels, const double *R, int64_t ncols,
                         int64_t naux_p, double *J, double *scratch, hipStream_t st);
// compensated sums of slot ranges: E[t] = sum of slots[base[t] .. base[t] + count[t])
hipError_t launch_finalize_terms(const double *slots, const int64_t *base, const int64_t *count,
                                 int nterms, double *E, hipStream_t st);
// ---- density-fitting factors (dfgen.hip) ----
hipError_t launch_df_factors(const DFPlan &pl, const DFInputs &in, const DFOutputs &o, void *ws,
                             hipStream_t st);
// ---- CD factors of the AO integrals (cholesky.hip) ----
struct CdState {   // done flag, rank and residual maximum at convergence
  int64_t done, rank;
  double dmax, pad;
};
struct CdPlan {
  int64_t nao, npair, max_rank;
  int64_t pstride;   // published maxima per parity (the most workgroups of a launch)
  double tol;
  size_t off_d, off_pv, off_pi, off_state;
  size_t total;
};
int cd_rows_per_block(int64_t npair);     // pair rows per workgroup of a step launch
int cd_threads_per_block(int64_t npair);  // its threads (a multiple of the rows)
hipError_t launch_cholesky(const CdPlan &pl, const double *M, double *B, int64_t *rank,
                           double *dmax, int64_t *pivots, void *ws, hipStream_t st);
// ---- semicanonical orbitals (semican.hip) ----
struct SemicanPlan {
  int64_t nao, nmo, nfrz, nc, na, nv;
  size_t off_a, off_a2, off_v, off_q, off_part, off_flag;
  size_t total;
};
int64_t semican_npad(int64_t n);   // order of the padded Jacobi matrix of an n-orbital block
constexpr int64_t kSemicanParts = 64;
hipError_t launch_semican(const SemicanPlan &pl, const double *F, const double *C, double *U,
                          double *eps, double *Cs, int *info, void *ws, hipStream_t st);
// C = alpha op(A) op(B) + beta C, row-major FP64 on the matrix cores (dfgen.hip)
hipError_t gemm_f64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                    const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                    double *C, int64_t ldc, hipStream_t st);
// C_z = A_z^T A_z (trans: A_z K x n) or A_z A_z^T (A_z n x K), row-major with
// leading dimension lda, for z < batch (A_z = A + z sa, C_z = C + z sc), on
// the tiles (r, c), r <= c, of the n x n result: the upper triangle in whole
// tiles, the tiles below it not written; *tile receives the tile size
// (dfgen.hip)
hipError_t gemm_f64_gram_upper(bool trans, int64_t n, int64_t K, const double *A, int64_t lda,
                               int64_t sa, double *C, int64_t ldc, int64_t sc, int64_t batch,
                               int64_t *tile, hipStream_t st);
// batch of products C_z = alpha op(A_z) op(B_z) + beta C_z, operands advanced
// by the strides sa, sb, sc (doubles) per batch index (dfgen.hip)
hipError_t gemm_f64_batched(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                            const double *A, int64_t lda, int64_t sa, const double *B,
                            int64_t ldb, int64_t sb, double beta, double *C, int64_t ldc,
                            int64_t sc, int64_t batch, hipStream_t st);
// ---- Laplace-type factorization of the CCVV Coulomb part (laplace.hip) ----
constexpr int kLtMaxTerms = 64;   // exponential-sum terms per call
struct LtPlan {
  int64_t nc, nv, naux;
  int nq, kb;       // terms, terms per batch
  int64_t nwg;      // sum-of-squares workgroups per term
  size_t off_bs, off_y, off_slots;
  size_t total;
};
hipError_t launch_coulomb_laplace(const LtPlan &pl, const double *B_cv, const double *eps_c,
                                  const double *eps_v, const double *t, const double *w,
                                  double *E, double *S, void *ws, hipStream_t st);
// host: exponential-sum fit of h(x) = (1 - exp(-2 s x^2)) / x on [x_lo, x_hi]
int laplace_fit(double s, double x_lo, double x_hi, int nq, double *t, double *w,
                double *max_err);
// ---- generalized Fock matrix (dfgen.hip) ----
struct FockPlan {
  int64_t nao, nmo, naux, nfrz, nc, na, nv;
  bool metric;      // as in DFPlan
  int64_t no, nd;   // occupied (frozen + core + active), doubly occupied (frozen + core)
  size_t off_t, off_y, off_l, off_x, off_w, off_bo, off_d, off_c, off_jao, off_tj, off_part;
  size_t total;
};
struct FockInputs {
  const double *ao3, *J, *C, *h, *gamma1;
};
hipError_t launch_df_fock(const FockPlan &pl, const FockInputs &in, double *F, void *ws,
                          hipStream_t st);
// ---- F4-F8 (active_terms.hip) ----
hipError_t launch_active_terms(const ActivePlan &pl, const ActiveInputs &in, void *ws,
                               double *F, hipStream_t st);
// ---- int8 slice path (split_kernels.hip) ----
hipError_t launch_energy_split(const Plan &pl, const Inputs &in, void *ws, hipStream_t st);
hipError_t launch_cavv_epi(const Plan &pl, const Inputs &in, void *ws, int m0, int mb,
                           hipStream_t st);
// (me|uf) integral batch Xb for core orbitals m0 .. m0+mb-1 from the slices
hipError_t launch_cavv_x_split(const Plan &pl, void *ws, int m0, int mb, hipStream_t st);
// FP64 integrals X^{mu}[e][f] = (me|uf) of core orbitals m0 .. m0+mb-1 into the batch buffer
hipError_t launch_cavv_x_fp64(const Plan &pl, void *ws, int m0, int mb, hipStream_t st);
// CAVV adjoint epilogue over one integral batch: G2 (rows of the batch's core
// orbitals only, (m - m0) 64 ntv + e), the CAVV energy slots and the
// orbital-energy / flow-parameter gradient parts
hipError_t launch_cavv_adj_epi(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                               int m0, int mb, hipStream_t st);
// int8 slices of B_cv (with the FP64 diagonal) and, if with_av, of B_av
hipError_t launch_slices(const Plan &pl, const Inputs &in, void *ws, bool with_av,
                         hipStream_t st);
// ---- adjoint (fp64_bwd.hip, split_bwd.hip) ----
hipError_t launch_zero_fill(double *p, int64_t n, hipStream_t st);
// gradients of eps and s cleared, FP64 panels packed, the CCAV adjoint tiles G3
hipError_t launch_adjoint_start_fp64(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                                     hipStream_t st);
// first energy slot of the CCVV block pair (I, J) with tiles_per_pair tile pairs per core pair
int64_t ccvv_block_slot(const Plan &pl, int64_t I, int64_t J, int64_t tiles_per_pair);
hipError_t launch_backward_fp64(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                                hipStream_t st);
hipError_t launch_backward_split(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                                 hipStream_t st);

}  // namespace dsrg
