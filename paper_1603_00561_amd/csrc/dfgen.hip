// Density-fitting factors B^Q_pq (Eq. int_fact and the DF definition of
// section II.C of the paper) on the FP64 matrix cores (gfx950):
//
//   (pq|P)  = sum_{mu nu} C_{mu p} C_{nu q} (mu nu|P)      MO three-index integrals
//   J       = L L^T                                         Cholesky factor of the metric
//   B^Q_pq  = sum_{P <= Q} [L^{-1}]_{QP} (pq|P)              so that B^T B = (pq|P) J^{-1} (P|rs)
//
// for p in core | active and q in active | virtual (the blocks B_cv, B_ca,
// B_av, B_aa that the energy reads). The symmetric J^{-1/2} of the paper gives
// the same factors up to an orthogonal rotation of Q, which leaves every
// (pq|rs) unchanged. Steps: T[P][p][nu] = C_{mu p} (mu nu|P) (batched over
// P, the short core | active index first), Y[(P p)][q] = T[(P p)][nu] C_{nu q}
// (one GEMM over all P and p), the Cholesky factor of J and its inverse by
// recursive blocking, B = L^{-1} Y (one GEMM whose contraction stops at the
// diagonal), and a scatter into the four output blocks.
#include <algorithm>

#include "common_device.h"
#include "internal.h"

namespace dsrg {

// ---------------------------------------------------------------------------
// C[b] = alpha op(A[b]) op(B[b]) + beta C[b] for b = blockIdx.z, row-major:
//   op(A)(m, k) = TA ? A[k lda + m] : A[m lda + k]
//   op(B)(k, n) = TB ? B[n ldb + k] : B[k ldb + n]
// One TM x TN tile per workgroup of WR x WC x KS waves, each wave owning a
// (TM / WR) x (TN / WC) block of 16 x 16 FP64 MFMA fragments and every KS-th
// group of four k of each chunk; K chunks of KC staged through registers into
// LDS, one barrier per chunk; with KS > 1 the KS partial tiles are summed
// through LDS in a fixed order at the end. Each operand is read along its
// contiguous index (as 16-byte pairs when both operands are aligned for it):
// an operand contiguous in k is staged as [row][k] rows of KC + 2 (two pads:
// the 16 x 4 fragment read then touches each bank pair at most twice), one
// contiguous in m or n as [k][row] rows whose odd rows have their 16-element
// halves swapped within groups of 32 (plain when the tile height is not a
// multiple of 32). Out-of-range elements read as zero. With ktri set the
// contraction of the row tile starting at m0 stops at k = m0 + TM (A lower
// triangular). Tiles are walked XCD by XCD (see the kernel). Shapes: 128 x 128
// (8 waves, K chunks of 32) for large products; 32 x 128, 48 x 128 and
// 64 x 128 (4 waves) for products of few rows, also with a batch folded into
// the columns; 64 x 64 (4 waves, K chunks of 32) and 32 x 32 with K split over
// 4 waves (K chunks of 64) to spread smaller ones over more SIMDs (one FP64
// MFMA wave needs about a microsecond per 32 x 32 x 32 block); long products
// with small outputs are also split over K across workgroups.
// ---------------------------------------------------------------------------
struct GemmGArgs {
  int64_t M, N, K;
  int64_t lda, ldb, ldc;
  int64_t sa, sb, sc;      // batch strides
  double alpha, beta;
  int ktri;
  // folded batch (FOLD kernels): column n is column n % nin of batch n / nin,
  // which adds (n / nin) * fb to its B offset and (n / nin) * fc to its C offset
  int64_t nin, fb, fc;
  int colfast;   // tile walk: column tiles fastest (A the larger operand)
  // split K (ktotal > 0): batch z contracts k in [z K, min((z + 1) K, ktotal)),
  // its operands advanced by the batch strides
  int64_t ktotal;
  // upper-triangle tiles (utiles > 0, square tiles, M = N): the grid runs
  // over the utiles (utiles + 1) / 2 tiles (r, c), r <= c, of a utiles x
  // utiles tile grid, row by row
  int64_t utiles;
};

template <int TM_, int TN_, int WR_, int WC_, int KC_, int KS_ = 1>
struct GTile {
  static constexpr int TM = TM_, TN = TN_, WR = WR_, WC = WC_, KC = KC_, KP = KC_ + 2;
  static constexpr int KS = KS_;                     // waves splitting each chunk's k
  static constexpr int WM = TM / WR, WN = TN / WC;   // wave block
  static constexpr int FP = WM / 16, FQ = WN / 16;   // fragments per wave
  static constexpr int NT = 64 * WR * WC * KS;       // threads
  static constexpr int JA = TM * KC / NT, JB = TN * KC / NT;
  static_assert(WM % 16 == 0 && WN % 16 == 0 && KC % 4 == 0, "whole fragments");
  static_assert(TM * KC % NT == 0 && TN * KC % NT == 0, "chunk split evenly");
  static_assert(TM % 16 == 0 && TN % 16 == 0, "whole 16-row fragments");
  static_assert(KC % (4 * KS) == 0, "k groups split evenly over the waves");
  static_assert((KS - 1) * 64 * FP * FQ * 4 <= 2 * TM * KP, "reduction fits the A stage");
};
using GBig = GTile<128, 128, 2, 4, 32>;
using GMid = GTile<64, 64, 2, 2, 32>;
using GThin = GTile<32, 128, 1, 4, 16>;
using GSplit = GTile<32, 32, 1, 1, 64, 4>;
using GThin48 = GTile<48, 128, 1, 4, 16>;   // folded products of 33..48 rows
using GThin64 = GTile<64, 128, 1, 4, 16>;   // folded products of 49..64 rows

// half swap of the k-major layout: odd k rows exchange their 16-element
// halves within each group of 32; rows of R not a multiple of 32 are stored
// plainly
template <int R>
__device__ __forceinline__ int gswz(int k) { return (R % 32 == 0) ? ((k & 1) << 4) : 0; }

// element j of thread t's share of an R x KC operand chunk: (row, k) and the
// LDS index; KFAST: the operand is contiguous in k
template <bool KFAST, int R, int NT, int KC>
__device__ __forceinline__ void chunk_slot(int t, int j, int &row, int &k, int &lidx) {
  const int e = t + NT * j;
  if (KFAST) {
    row = e / KC;
    k = e % KC;
    lidx = row * (KC + 2) + k;
  } else {
    k = e / R;
    row = e % R;
    lidx = k * R + (row ^ gswz<R>(k));
  }
}

template <bool KFAST, int R, int KC>
__device__ __forceinline__ double frag(const double *L, int row, int k) {
  return KFAST ? L[row * (KC + 2) + k] : L[k * R + (row ^ gswz<R>(k))];
}

// pair j (two neighbours along the contiguous index) of thread t's share of
// an R x KC operand chunk: the first element's (row, k) and LDS index
template <bool KFAST, int R, int NT, int KC>
__device__ __forceinline__ void pair_slot(int t, int j, int &row, int &k, int &lidx) {
  const int e = t + NT * j;
  if (KFAST) {
    row = e / (KC / 2);
    k = 2 * (e % (KC / 2));
    lidx = row * (KC + 2) + k;
  } else {
    k = e / (R / 2);
    row = 2 * (e % (R / 2));
    lidx = k * R + (row ^ gswz<R>(k));
  }
}

// PAIR: operands read and staged as 16-byte pairs along their contiguous
// index (the host checks that both operands' base pointers, leading
// dimensions, batch strides and contiguous extents are even, so every pair is
// aligned and lies wholly inside or outside the operand)
template <bool TA, bool TB, class G, bool FOLD = false, bool PAIR = false>
__global__ __launch_bounds__(G::NT) void gemm_g_kernel(const double *__restrict__ A,
                                                      const double *__restrict__ B, GemmGArgs a,
                                                      double *__restrict__ C) {
  static_assert(!FOLD || (!TB && G::NT % G::TN == 0), "folded B: n-contiguous, one column per thread");
  static_assert(!(FOLD && PAIR), "folded products read single elements");
  static_assert(!PAIR || (G::JA % 2 == 0 && G::JB % 2 == 0), "whole pairs per thread");
  constexpr bool AK = !TA, BK = TB;   // operands contiguous in k
  constexpr int TM = G::TM, TN = G::TN, NT = G::NT, KC = G::KC;
  __shared__ __align__(16) double sA[2][TM * G::KP];
  __shared__ __align__(16) double sB[2][TN * G::KP];
  // XCD-aware tile order: the hardware deals workgroup id (x fastest) to XCD
  // id % 8; XCD k takes a contiguous range of tiles, walked so that the
  // workgroups reading one tile of the larger operand run side by side (row
  // tiles fastest when B is the larger, column tiles fastest when A is): they
  // share that XCD's L2 and the tile leaves HBM about once
  const int64_t nx = gridDim.x, ny = gridDim.y, per = nx * ny;
  const int64_t id = blockIdx.x + nx * blockIdx.y, xcd = id % 8;
  const int64_t tl = xcd * (per / 8) + std::min<int64_t>(xcd, per % 8) + id / 8;
  int64_t m0, n0;
  if (a.utiles > 0) {
    // row r of the upper triangle starts at tile r T - r (r - 1) / 2
    const int64_t T = a.utiles;
    const double b2 = 2.0 * (double)T + 1.0;
    int64_t r = (int64_t)((b2 - sqrt(b2 * b2 - 8.0 * (double)tl)) * 0.5);
    auto start = [&](int64_t q) { return q * T - q * (q - 1) / 2; };
    while (r > 0 && start(r) > tl) --r;
    while (r + 1 < T && start(r + 1) <= tl) ++r;
    m0 = r * TM;
    n0 = (r + tl - start(r)) * TN;
  } else {
    m0 = (a.colfast ? tl / ny : tl % nx) * TM;
    n0 = (a.colfast ? tl % ny : tl / nx) * TN;
  }
  A += (int64_t)blockIdx.z * a.sa;
  B += (int64_t)blockIdx.z * a.sb;
  C += (int64_t)blockIdx.z * a.sc;
  const int64_t Kb = a.ktotal > 0 ? std::min(a.K, a.ktotal - (int64_t)blockIdx.z * a.K) : a.K;
  const int64_t K = a.ktri ? std::min(Kb, m0 + TM) : Kb;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int ks = wave / (G::WR * G::WC), wrc = wave % (G::WR * G::WC);
  const int wr = wrc / G::WC, wc = wrc % G::WC;
  const int cl = lane & 15, kl = lane >> 4;
  d4 acc[G::FP][G::FQ];
#pragma unroll
  for (int p = 0; p < G::FP; ++p)
#pragma unroll
    for (int q = 0; q < G::FQ; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};

  double ra[G::JA], rb[G::JB];
  int64_t bcol = -1;   // FOLD: this thread's B column offset (-1 past N)
  if constexpr (FOLD) {
    const int64_t n = n0 + t % G::TN;
    if (n < a.N) bcol = n + (n / a.nin) * a.fb;
  }
  auto gload = [&](int64_t k0) {
    if constexpr (PAIR) {
#pragma unroll
      for (int j = 0; j < G::JA / 2; ++j) {
        int row, k, li;
        pair_slot<AK, TM, NT, KC>(t, j, row, k, li);
        const int64_t m = m0 + row, ka = k0 + k;
        d2v v = {0.0, 0.0};
        if (ka < K && m < a.M)
          v = *reinterpret_cast<const d2v *>(TA ? A + ka * a.lda + m : A + m * a.lda + ka);
        ra[2 * j] = v[0];
        ra[2 * j + 1] = v[1];
      }
#pragma unroll
      for (int j = 0; j < G::JB / 2; ++j) {
        int row, k, li;
        pair_slot<BK, TN, NT, KC>(t, j, row, k, li);
        const int64_t n = n0 + row, kb = k0 + k;
        d2v v = {0.0, 0.0};
        if (kb < K && n < a.N)
          v = *reinterpret_cast<const d2v *>(TB ? B + n * a.ldb + kb : B + kb * a.ldb + n);
        rb[2 * j] = v[0];
        rb[2 * j + 1] = v[1];
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < G::JA; ++j) {
      int row, k, li;
      chunk_slot<AK, TM, NT, KC>(t, j, row, k, li);
      const int64_t m = m0 + row, ka = k0 + k;
      ra[j] = (ka < K && m < a.M) ? (TA ? A[ka * a.lda + m] : A[m * a.lda + ka]) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < G::JB; ++j) {
      int row, k, li;
      chunk_slot<BK, TN, NT, KC>(t, j, row, k, li);
      const int64_t n = n0 + row, kb = k0 + k;
      if constexpr (FOLD)
        rb[j] = (kb < K && bcol >= 0) ? B[kb * a.ldb + bcol] : 0.0;
      else
        rb[j] = (kb < K && n < a.N) ? (TB ? B[n * a.ldb + kb] : B[kb * a.ldb + n]) : 0.0;
    }
  };
  auto sstore = [&](int b) {
    if constexpr (PAIR) {
#pragma unroll
      for (int j = 0; j < G::JA / 2; ++j) {
        int row, k, li;
        pair_slot<AK, TM, NT, KC>(t, j, row, k, li);
        *reinterpret_cast<d2v *>(&sA[b][li]) = d2v{ra[2 * j], ra[2 * j + 1]};
      }
#pragma unroll
      for (int j = 0; j < G::JB / 2; ++j) {
        int row, k, li;
        pair_slot<BK, TN, NT, KC>(t, j, row, k, li);
        *reinterpret_cast<d2v *>(&sB[b][li]) = d2v{rb[2 * j], rb[2 * j + 1]};
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < G::JA; ++j) {
      int row, k, li;
      chunk_slot<AK, TM, NT, KC>(t, j, row, k, li);
      sA[b][li] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < G::JB; ++j) {
      int row, k, li;
      chunk_slot<BK, TN, NT, KC>(t, j, row, k, li);
      sB[b][li] = rb[j];
    }
  };

  if (K > 0) {
    gload(0);
    sstore(0);
    if (K > KC) gload(KC);
  }
  __syncthreads();
  int b = 0;
  for (int64_t k0 = 0; k0 < K; k0 += KC) {
    const double *LA = sA[b], *LB = sB[b];
#pragma unroll
    for (int kg = 0; kg < KC / (4 * G::KS); ++kg) {
      const int k = (kg * G::KS + ks) * 4 + kl;
      double fa[G::FP], fb[G::FQ];
#pragma unroll
      for (int p = 0; p < G::FP; ++p) fa[p] = frag<AK, TM, KC>(LA, G::WM * wr + 16 * p + cl, k);
#pragma unroll
      for (int q = 0; q < G::FQ; ++q) fb[q] = frag<BK, TN, KC>(LB, G::WN * wc + 16 * q + cl, k);
#pragma unroll
      for (int p = 0; p < G::FP; ++p)
#pragma unroll
        for (int q = 0; q < G::FQ; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[p], fb[q], acc[p][q], 0, 0, 0);
    }
    if (k0 + KC < K) {
      sstore(b ^ 1);
      if (k0 + 2 * KC < K) gload(k0 + 2 * KC);
    }
    __syncthreads();
    b ^= 1;
  }
  if constexpr (G::KS > 1) {
    double *red = &sA[0][0];
    constexpr int NV = G::FP * G::FQ * 4;
    if (ks > 0) {
#pragma unroll
      for (int p = 0; p < G::FP; ++p)
#pragma unroll
        for (int q = 0; q < G::FQ; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            red[((ks - 1) * NV + (p * G::FQ + q) * 4 + r) * 64 + lane] = acc[p][q][r];
    }
    __syncthreads();
    if (ks > 0) return;
    for (int w = 1; w < G::KS; ++w)
#pragma unroll
      for (int p = 0; p < G::FP; ++p)
#pragma unroll
        for (int q = 0; q < G::FQ; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            acc[p][q][r] += red[((w - 1) * NV + (p * G::FQ + q) * 4 + r) * 64 + lane];
  }
#pragma unroll
  for (int q = 0; q < G::FQ; ++q) {
    const int64_t n = n0 + G::WN * wc + 16 * q + cl;
    if (n >= a.N) continue;
    const int64_t cn = FOLD ? n + (n / a.nin) * a.fc : n;
#pragma unroll
    for (int p = 0; p < G::FP; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + G::WM * wr + 16 * p + 4 * r + kl;
        if (m >= a.M) continue;
        double *dst = C + m * a.ldc + cn;
        const double v = a.alpha * acc[p][q][r];
        *dst = (a.beta != 0.0) ? v + a.beta * *dst : v;
      }
  }
}

template <class G, bool PAIR>
static void gemm_g_launch_p(bool ta, bool tb, const GemmGArgs &a, int64_t batch, const double *A,
                            const double *B, double *C, hipStream_t st) {
  const dim3 grid((unsigned)ceil_div(a.M, G::TM), (unsigned)ceil_div(a.N, G::TN), (unsigned)batch);
  const dim3 block(G::NT);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_g_kernel<false, false, G, false, PAIR>), grid, block, 0, st, A, B, a, C);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_g_kernel<true, false, G, false, PAIR>), grid, block, 0, st, A, B, a, C);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_g_kernel<false, true, G, false, PAIR>), grid, block, 0, st, A, B, a, C);
  else
    hipLaunchKernelGGL((gemm_g_kernel<true, true, G, false, PAIR>), grid, block, 0, st, A, B, a, C);
}

// pairs when both operands allow them: 16-byte-aligned bases, even leading
// dimensions and batch strides, and an even extent along each contiguous
// index (k for row-major A and transposed B, m for transposed A, n for B)
static bool pairs_fit(bool ta, bool tb, const GemmGArgs &a, const double *A, const double *B) {
  const bool aligned = ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0);
  const bool even = a.lda % 2 == 0 && a.ldb % 2 == 0 && a.sa % 2 == 0 && a.sb % 2 == 0;
  const bool ext = (ta ? a.M : a.K) % 2 == 0 && (tb ? a.K : a.N) % 2 == 0;
  return aligned && even && ext;
}

template <class G>
static void gemm_g_launch(bool ta, bool tb, const GemmGArgs &a, int64_t batch, const double *A,
                          const double *B, double *C, hipStream_t st) {
  if (pairs_fit(ta, tb, a, A, B))
    gemm_g_launch_p<G, true>(ta, tb, a, batch, A, B, C, st);
  else
    gemm_g_launch_p<G, false>(ta, tb, a, batch, A, B, C, st);
}

// tile shape: 32 x 128 for at most 32 rows when that gives a tile per CU,
// else 128 x 128 when that gives three or more tiles per CU, else 64 x 64 when that
// gives a tile per CU, else 32 x 32 with K split over four waves
static hipError_t gemm_g(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                         const double *A, int64_t lda, int64_t sa, const double *B, int64_t ldb,
                         int64_t sb, double beta, double *C, int64_t ldc, int64_t sc,
                         int64_t batch, bool ktri, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  GemmGArgs a{M, N, K, lda, ldb, ldc, sa, sb, sc, alpha, beta, ktri ? 1 : 0, 0, 0, 0, M > N ? 1 : 0,
              0, 0};
  auto tiles = [&](int tm, int tn) { return ceil_div(M, tm) * ceil_div(N, tn) * batch; };
  if (M <= GThin::TM && tiles(GThin::TM, GThin::TN) >= 256)
    gemm_g_launch<GThin>(ta, tb, a, batch, A, B, C, st);
  else if (tiles(GBig::TM, GBig::TN) >= 768)
    gemm_g_launch<GBig>(ta, tb, a, batch, A, B, C, st);
  else if (tiles(GMid::TM, GMid::TN) >= 256)
    gemm_g_launch<GMid>(ta, tb, a, batch, A, B, C, st);
  else
    gemm_g_launch<GSplit>(ta, tb, a, batch, A, B, C, st);
  return hipGetLastError();
}

hipError_t gemm_f64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                    const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
                    double *C, int64_t ldc, hipStream_t st) {
  return gemm_g(ta, tb, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1, false, st);
}

template <class G>
static void gram_launch(bool trans, const GemmGArgs &a, int64_t batch, const double *A, double *C,
                        hipStream_t st) {
  const dim3 grid((unsigned)(a.utiles * (a.utiles + 1) / 2), 1, (unsigned)batch);
  const bool pr = pairs_fit(trans, !trans, a, A, A);
  if (trans && pr)
    hipLaunchKernelGGL((gemm_g_kernel<true, false, G, false, true>), grid, dim3(G::NT), 0, st, A, A,
                       a, C);
  else if (trans)
    hipLaunchKernelGGL((gemm_g_kernel<true, false, G, false, false>), grid, dim3(G::NT), 0, st, A,
                       A, a, C);
  else if (pr)
    hipLaunchKernelGGL((gemm_g_kernel<false, true, G, false, true>), grid, dim3(G::NT), 0, st, A, A,
                       a, C);
  else
    hipLaunchKernelGGL((gemm_g_kernel<false, true, G, false, false>), grid, dim3(G::NT), 0, st, A,
                       A, a, C);
}

hipError_t gemm_f64_gram_upper(bool trans, int64_t n, int64_t K, const double *A, int64_t lda,
                               int64_t sa, double *C, int64_t ldc, int64_t sc, int64_t batch,
                               int64_t *tile, hipStream_t st) {
  *tile = 0;
  if (n <= 0 || batch <= 0) return hipSuccess;
  GemmGArgs a{n, n, K, lda, lda, ldc, sa, sa, sc, 1.0, 0.0, 0, 0, 0, 0, 0, 0, 0};
  auto utiles = [&](int t) { return ceil_div(n, t) * (ceil_div(n, t) + 1) / 2 * batch; };
  // 128 x 128 tiles when they give three or more per CU, else 64 x 64
  if (utiles(GBig::TM) >= 768) {
    a.utiles = ceil_div(n, GBig::TM);
    *tile = GBig::TM;
    gram_launch<GBig>(trans, a, batch, A, C, st);
  } else {
    a.utiles = ceil_div(n, GMid::TM);
    *tile = GMid::TM;
    gram_launch<GMid>(trans, a, batch, A, C, st);
  }
  return hipGetLastError();
}

hipError_t gemm_f64_batched(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                            const double *A, int64_t lda, int64_t sa, const double *B,
                            int64_t ldb, int64_t sb, double beta, double *C, int64_t ldc,
                            int64_t sc, int64_t batch, hipStream_t st) {
  return gemm_g(ta, tb, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, batch, false,
                st);
}

// C = sum_{s < nseg} P[s] with P[s] = op(A) op(B) over the s-th of nseg
// contiguous ranges of K (one launch, the segments as its batch index; the
// partial products land in part[nseg][M][N]); then C = alpha sum_s P[s] +
// beta C, the segments added in order. For products whose output is too small
// to fill the chip on its own.
__global__ __launch_bounds__(256) void sum_parts_kernel(const double *__restrict__ part,
                                                        int64_t nseg, int64_t n, double alpha,
                                                        double beta, double *__restrict__ C) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int64_t s = 0; s < nseg; ++s) v += part[s * n + e];
    C[e] = alpha * v + (beta != 0.0 ? beta * C[e] : 0.0);
  }
}

static hipError_t gemm_g_splitk(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                                const double *A, int64_t lda, const double *B, int64_t ldb,
                                double beta, double *C, double *part, int64_t nseg,
                                hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  nseg = std::max<int64_t>(1, std::min(nseg, K));
  const int64_t kseg = ceil_div(K, nseg);
  nseg = ceil_div(K, kseg);
  GemmGArgs a{M, N, kseg, lda, ldb, N, (ta ? kseg * lda : kseg), (tb ? kseg : kseg * ldb), M * N,
              1.0, 0.0, 0, 0, 0, 0, M > N ? 1 : 0, K, 0};
  auto tiles = [&](int tm, int tn) { return ceil_div(M, tm) * ceil_div(N, tn) * nseg; };
  if (tiles(GBig::TM, GBig::TN) >= 768)
    gemm_g_launch<GBig>(ta, tb, a, nseg, A, B, part, st);
  else if (tiles(GMid::TM, GMid::TN) >= 256)
    gemm_g_launch<GMid>(ta, tb, a, nseg, A, B, part, st);
  else
    gemm_g_launch<GSplit>(ta, tb, a, nseg, A, B, part, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_parts_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(M * N, 256), 4096)),
                     dim3(256), 0, st, part, nseg, M * N, alpha, beta, C);
  return hipGetLastError();
}

// segments of a long contraction with a small output: enough 64 x 64 tiles
// for about eight per CU, each segment at least 1024 long, at most
// kMaxSegments (the partial buffer holds that many products)
constexpr int64_t kMaxSegments = 32;
static int64_t splitk_segments(int64_t M, int64_t N, int64_t K) {
  const int64_t t = ceil_div(M, 64) * ceil_div(N, 64);
  return std::max<int64_t>(1, std::min({ceil_div(2048, t), K / 1024, kMaxSegments}));
}

// C = alpha op(A) B over a batch folded into the columns: B[b] (ldb, batch
// stride sb) holds columns [b nin, (b + 1) nin) and C[b] (ldc, stride sc)
// takes them; at most 32 rows, so the 32 x 128 tile runs over nbatch * nin
// columns with no per-batch ragged tile (32, 48 or 64 rows per tile, the
// smallest that holds M); folded_fits says whether a product has that form.
static bool folded_fits(int64_t M, int64_t nin, int64_t nbatch) {
  return M <= GThin64::TM && ceil_div(nin * nbatch, GThin::TN) <= 65535;
}

template <class G>
static void folded_launch(bool ta, const GemmGArgs &a, const double *A, const double *B,
                          double *C, hipStream_t st) {
  const dim3 grid(1, (unsigned)ceil_div(a.N, G::TN), 1);
  if (ta)
    hipLaunchKernelGGL((gemm_g_kernel<true, false, G, true>), grid, dim3(G::NT), 0, st, A, B, a,
                       C);
  else
    hipLaunchKernelGGL((gemm_g_kernel<false, false, G, true>), grid, dim3(G::NT), 0, st, A, B, a,
                       C);
}

static hipError_t gemm_g_folded(bool ta, int64_t M, int64_t nin, int64_t K, double alpha,
                                const double *A, int64_t lda, const double *B, int64_t ldb,
                                int64_t sb, double *C, int64_t ldc, int64_t sc, int64_t nbatch,
                                hipStream_t st) {
  const int64_t N = nin * nbatch;
  if (M <= 0 || N <= 0) return hipSuccess;
  if (!folded_fits(M, nin, nbatch)) return hipErrorInvalidValue;
  GemmGArgs a{M, N, K, lda, ldb, ldc, 0, 0, 0, alpha, 0.0, 0, nin, sb - nin, sc - nin, 0, 0, 0};
  if (M <= GThin::TM)
    folded_launch<GThin>(ta, a, A, B, C, st);
  else if (M <= GThin48::TM)
    folded_launch<GThin48>(ta, a, A, B, C, st);
  else
    folded_launch<GThin64>(ta, a, A, B, C, st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cholesky factor and inverse of the metric, J = L L^T, X = L^{-1}, by
// recursive 2 x 2 blocking (split at a multiple of kDB):
//   (L11, X11) of J11;  L21 = J21 X11^T;  J22 -= L21 L21^T;  (L22, X22) of J22;
//   X21 = -X22 (L21 X11)
// so the large GEMMs sit at the top of the recursion; leaves of at most kDB
// rows are factored and inverted by one workgroup each. Only the lower triangle of
// the working copy of J is read, and the copy is overwritten; X is written
// lower triangular (the caller clears it). A metric that is not positive
// definite gives NaN (square root of a negative pivot).
// ---------------------------------------------------------------------------
constexpr int kDB = 64;

// leaf: the nb x nb diagonal block at (r0, r0) of the working matrix A (its
// lower triangle) is factored, L L^T, and inverted in one sweep over the
// columns, two at a time (j, j + 1): the 2 x 2 pivot block gives d1 = sqrt(a_jj),
// l = a_{j+1,j} / d1 and d2 = sqrt(a_{j+1,j+1} - l^2); columns j and j + 1 of L
// are a_ij / d1 and (a_{i,j+1} - L_ij l) / d2, and the trailing matrix loses
// their rank-2 product. In the same step forward substitution on L X = I
// (b starting as the identity) takes rows j and j + 1 of X, b_j / d1 and
// (b_{j+1} - l X_j) / d2, and removes L_ij X_j + L_{i,j+1} X_{j+1} from the rows
// below. L itself is never stored. 256 threads; thread (ty, tx) holds in
// registers the elements (ty + 16 a, tx + 16 b), a, b < 4, of the trailing
// matrix and of b; rows and columns past nb hold the identity (so an odd last
// column pairs with an identity one). One barrier per two columns: the
// threads holding columns j, j + 1 and rows j, j + 1 of b publish them
// unscaled to LDS (double-buffered), and every thread forms the pivot block
// and the scaled columns and rows it needs from there.
constexpr int kLeafT = 256;

__global__ __launch_bounds__(kLeafT) void chol_inv_leaf_kernel(const double *__restrict__ A,
                                                               double *__restrict__ X, int64_t ld,
                                                               int64_t r0, int nb) {
  __shared__ double col[2][2][kDB], row[2][2][kDB];   // [buffer][column j / j + 1][index]
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
  double e[4][4], x[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ty + 16 * a, l = tx + 16 * b;
      double v = (i == l) ? 1.0 : 0.0;
      if (i < nb && l < nb) v = (l <= i) ? A[(r0 + i) * ld + r0 + l] : A[(r0 + l) * ld + r0 + i];
      e[a][b] = v;
      x[a][b] = (i == l) ? 1.0 : 0.0;
    }
  for (int j = 0; j < nb; j += 2) {
    const int bf = (j >> 1) & 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {   // columns j, j + 1 and rows j, j + 1 of b, as they stand
      const int jj = j + h, jb = jj >> 4, jr = jj & 15;   // jb is the same in every thread
      if (tx == jr) {
        switch (jb) {
#define DSRG_LEAF_COL(B)                                                    \
  case B:                                                                   \
    _Pragma("unroll") for (int a = 0; a < 4; ++a) col[bf][h][ty + 16 * a] = e[a][B]; \
    break;
          DSRG_LEAF_COL(0)
          DSRG_LEAF_COL(1)
          DSRG_LEAF_COL(2)
          DSRG_LEAF_COL(3)
#undef DSRG_LEAF_COL
        }
      }
      if (ty == jr) {
        switch (jb) {
#define DSRG_LEAF_ROW(A)                                                    \
  case A:                                                                   \
    _Pragma("unroll") for (int b = 0; b < 4; ++b) row[bf][h][tx + 16 * b] = x[A][b]; \
    break;
          DSRG_LEAF_ROW(0)
          DSRG_LEAF_ROW(1)
          DSRG_LEAF_ROW(2)
          DSRG_LEAF_ROW(3)
#undef DSRG_LEAF_ROW
        }
      }
    }
    __syncthreads();
    // only the reciprocals of the pivots are used: with the pivot block
    // [[p, q], [q, r]], rd1 = 1 / sqrt(p), l = q rd1 and
    // rd2 = 1 / sqrt(r - l^2) = p rd1 / sqrt(p r - q^2); the two inverse
    // square roots do not wait for each other
    const double pp = col[bf][0][j], pq = col[bf][0][j + 1], pr = col[bf][1][j + 1];
    const double rd1 = rsqrt(pp);
    const double rdet = rsqrt(fma(pp, pr, -pq * pq));
    const double l10 = pq * rd1;
    const double rd2 = (pp * rd1) * rdet;
    double ci0[4], ci1[4], cl0[4], cl1[4], rx0[4], sc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = ty + 16 * a;
      const double L0 = col[bf][0][i] * rd1;
      ci0[a] = (i > j) ? L0 : 0.0;
      ci1[a] = (i > j + 1) ? (col[bf][1][i] - L0 * l10) * rd2 : 0.0;
      // rows j and j + 1 of b become rows of X: b_j / d1 and (b_{j+1} - l X_j) / d2
      sc[a] = (i == j) ? rd1 : ((i == j + 1) ? rd2 : 1.0);
    }
    // columns l <= j + 1 of the trailing matrix are finished and never read
    // again, so the column factors need no mask
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int l = tx + 16 * b;
      const double L0 = col[bf][0][l] * rd1;
      cl0[b] = L0;
      cl1[b] = (col[bf][1][l] - L0 * l10) * rd2;
      rx0[b] = row[bf][0][l] * rd1;
    }
    double rx1[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) rx1[b] = fma(-l10, rx0[b], row[bf][1][tx + 16 * b]) * rd2;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        e[a][b] = fma(-ci1[a], cl1[b], fma(-ci0[a], cl0[b], e[a][b]));
        x[a][b] = fma(-ci1[a], rx1[b], fma(-ci0[a], rx0[b], x[a][b])) * sc[a];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ty + 16 * a, l = tx + 16 * b;
      if (i < nb && l < nb) X[(r0 + i) * ld + r0 + l] = x[a][b];
    }
}

// (L, X) of the block [r0, r0 + n) of the working matrix A (leading dimension
// ld). W has A's shape: the L21 block of each split is written there at its
// own position (disjoint from every other split's), and A's J21 block, no
// longer needed once L21 is formed, takes the product L21 X11.
static hipError_t chol_inv(double *A, double *X, double *W, int64_t ld, int64_t r0, int64_t n,
                           hipStream_t st) {
  hipError_t e;
  if (n <= kDB) {
    hipLaunchKernelGGL(chol_inv_leaf_kernel, dim3(1), dim3(kLeafT), 0, st, A, X, ld, r0, (int)n);
    return hipGetLastError();
  }
  const int64_t n1 = round_up(ceil_div(n, 2), kDB), n2 = n - n1;
  if ((e = chol_inv(A, X, W, ld, r0, n1, st)) != hipSuccess) return e;
  const int64_t o21 = (r0 + n1) * ld + r0, o22 = (r0 + n1) * ld + r0 + n1, o11 = r0 * ld + r0;
  // L21 = J21 X11^T
  if ((e = gemm_g(false, true, n2, n1, n1, 1.0, A + o21, ld, 0, X + o11, ld, 0, 0.0, W + o21, ld,
                  0, 1, false, st)) != hipSuccess)
    return e;
  // J22 -= L21 L21^T
  if ((e = gemm_g(false, true, n2, n2, n1, -1.0, W + o21, ld, 0, W + o21, ld, 0, 1.0, A + o22, ld,
                  0, 1, false, st)) != hipSuccess)
    return e;
  if ((e = chol_inv(A, X, W, ld, r0 + n1, n2, st)) != hipSuccess) return e;
  // X21 = -X22 (L21 X11)
  if ((e = gemm_g(false, false, n2, n1, n1, 1.0, W + o21, ld, 0, X + o11, ld, 0, 0.0, A + o21, ld,
                  0, 1, false, st)) != hipSuccess)
    return e;
  return gemm_g(false, false, n2, n1, n2, -1.0, X + o22, ld, 0, A + o21, ld, 0, 0.0, X + o21, ld,
                0, 1, false, st);
}

// ---------------------------------------------------------------------------
// scatter of B[Q][p][q] (p in core | active, q in active | virtual) into the
// four output blocks
// ---------------------------------------------------------------------------
struct ScatterArgs {
  int64_t naux, nc, na, nv;
};

__global__ __launch_bounds__(256) void df_scatter_kernel(const double *__restrict__ Bf,
                                                         ScatterArgs a, double *__restrict__ B_cv,
                                                         double *__restrict__ B_ca,
                                                         double *__restrict__ B_av,
                                                         double *__restrict__ B_aa) {
  const int64_t np = a.nc + a.na, nq = a.na + a.nv;
  const int64_t total = a.naux * np * nq;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t q = e % nq, p = (e / nq) % np, Q = e / (np * nq);
    const double v = Bf[e];
    if (p < a.nc) {
      if (q >= a.na)
        B_cv[(Q * a.nc + p) * a.nv + (q - a.na)] = v;
      else
        B_ca[(Q * a.nc + p) * a.na + q] = v;
    } else {
      const int64_t u = p - a.nc;
      if (q >= a.na)
        B_av[(Q * a.na + u) * a.nv + (q - a.na)] = v;
      else
        B_aa[(Q * a.na + u) * a.na + q] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// The metric factor depends on J alone, so the builds run it on a second
// stream beside the two MO transforms: a latency-bound chain of small
// launches next to two chip-filling products. One side stream (non-blocking,
// default priority) and a fork / join event pair per host thread and device,
// made on first use; the caller's stream waits for the join before anything
// reads the factor, so the call still enqueues only on the caller's stream as
// far as the caller can tell (and can be captured in a graph).
// ---------------------------------------------------------------------------
struct SideStream {
  int device = -1;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
thread_local SideStream g_side;

static hipError_t side_stream(SideStream *&out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  SideStream &ss = g_side;
  if (ss.device != dev) {
    if (ss.s) {   // made on another device: that device's objects are dropped
      (void)hipEventDestroy(ss.fork);
      (void)hipEventDestroy(ss.join);
      (void)hipStreamDestroy(ss.s);
      ss = SideStream{};
    }
    if ((e = hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&ss.join, hipEventDisableTiming)) != hipSuccess) return e;
    ss.device = dev;
  }
  out = &ss;
  return hipSuccess;
}

// Cholesky factor of J (in the copy Lm) and its inverse X = L^{-1} on the side
// stream, after everything already enqueued on st; st waits for it only at
// the join (side_join)
static hipError_t metric_forked(const char *name, const double *J, double *Lm, double *X,
                                double *W, int64_t naux, hipStream_t st, SideStream *&ss) {
  hipError_t e = side_stream(ss);
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(ss->fork, st)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(ss->s, ss->fork, 0)) != hipSuccess) return e;
  timer_begin(name, ss->s);
  if ((e = hipMemcpyAsync(Lm, J, sizeof(double) * naux * naux, hipMemcpyDeviceToDevice,
                          ss->s)) != hipSuccess)
    return e;
  if ((e = launch_zero_fill(X, naux * naux, ss->s)) != hipSuccess) return e;
  if ((e = chol_inv(Lm, X, W, naux, 0, naux, ss->s)) != hipSuccess) return e;
  timer_end(ss->s);
  return hipEventRecord(ss->join, ss->s);
}

static hipError_t side_join(const SideStream *ss, hipStream_t st) {
  return hipStreamWaitEvent(st, ss->join, 0);
}

hipError_t launch_df_factors(const DFPlan &pl, const DFInputs &in, const DFOutputs &o, void *ws,
                             hipStream_t st) {
  hipError_t e;
  const int64_t nao = pl.nao, nmo = pl.nmo, naux = pl.naux;
  const int64_t np = pl.nc + pl.na, nq = pl.na + pl.nv;
  const int64_t oc = pl.nfrz, oa = pl.nfrz + pl.nc;
  double *T = ws_d(ws, pl.off_t), *Y = ws_d(ws, pl.off_y), *Lm = ws_d(ws, pl.off_l);
  double *X = ws_d(ws, pl.off_x), *W = ws_d(ws, pl.off_tmp), *Bf = ws_d(ws, pl.off_bf);
  // the metric factor and inverse, beside the transforms (disjoint buffers:
  // Lm, X, W there; T, Y here); none for factors that need no metric
  SideStream *ss = nullptr;
  if (pl.metric &&
      (e = metric_forked("df_metric", in.J, Lm, X, W, naux, st, ss)) != hipSuccess)
    return e;
  // T[P][p][nu] = sum_mu C[mu][oc + p] (mu nu|P), batched over P: the small
  // (core | active) index first, so the second step contracts nao over
  // naux np rows instead of naux nao
  timer_begin("df_half1", st);
  if (folded_fits(np, nao, naux))
    e = gemm_g_folded(true, np, nao, nao, 1.0, in.C + oc, nmo, in.ao3, nao, nao * nao, T, nao,
                      np * nao, naux, st);
  else
    e = gemm_g(true, false, np, nao, nao, 1.0, in.C + oc, nmo, 0, in.ao3, nao, nao * nao, 0.0, T,
               nao, np * nao, naux, false, st);
  timer_end(st);
  if (e != hipSuccess) return e;
  // Y[(P p)][q] = sum_nu T[(P p)][nu] C[nu][oa + q], one GEMM over all P and p
  timer_begin("df_half2", st);
  e = gemm_g(false, false, naux * np, nq, nao, 1.0, T, nao, 0, in.C + oa, nmo, 0, 0.0, Y, nq, 0,
             1, false, st);
  timer_end(st);
  if (e != hipSuccess) return e;
  if (pl.metric) {
    if ((e = side_join(ss, st)) != hipSuccess) return e;
    // B[Q][(p q)] = sum_{P <= Q} X[Q][P] Y[P][(p q)]
    timer_begin("df_metric_apply", st);
    e = gemm_g(false, false, naux, np * nq, naux, 1.0, X, naux, 0, Y, np * nq, 0, 0.0, Bf,
               np * nq, 0, 1, true, st);
    timer_end(st);
    if (e != hipSuccess) return e;
  } else {
    Bf = Y;   // the transformed factors are B already
  }
  ScatterArgs sa{naux, pl.nc, pl.na, pl.nv};
  const int64_t total = naux * np * nq;
  timer_begin("df_scatter", st);
  hipLaunchKernelGGL(df_scatter_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 65536)),
                     dim3(256), 0, st, Bf, sa, o.B_cv, o.B_ca, o.B_av, o.B_aa);
  timer_end(st);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Generalized Fock matrix (Eq. gen_fock) from the DF integrals. With o the
// frozen + core + active orbitals, B^Q_mq (m in o, q all) the DF factors of
// (m q|P) (as in the factor build, L^{-1} of the metric applied) and the MO
// density D (2 on the frozen + core diagonal, Gamma on the active block):
//   Coulomb:  d^Q = sum_rs D_rs B^Q_rs, c = X^T d (X = L^{-1}),
//             J_AO = sum_P c_P (mu nu|P), J_MO = C^T J_AO C
//   exchange: K/2 = sum_{Q, m} B^Q_mp Bh^Q_mq with Bh^Q_iq = B^Q_iq for the
//             doubly occupied i and Bh^Q_uq = (1/2) sum_v Gamma_uv B^Q_vq
//   F = h + J_MO - K/2
// The first transform contracts the occupied index on the left of (mu nu|P),
// so (m q|P) = (q m|P) rests on the symmetry of the AO integrals in mu, nu.
// ---------------------------------------------------------------------------

// d^Q = 2 sum_{i < nd} B^Q_ii + sum_{uv} Gamma_uv B^Q_{nd+u, nd+v}, one thread per Q
__global__ __launch_bounds__(256) void fock_density_kernel(const double *__restrict__ Bo,
                                                           const double *__restrict__ gamma1,
                                                           int64_t naux, int64_t no, int64_t nmo,
                                                           int64_t nd, int64_t na,
                                                           double *__restrict__ d) {
  for (int64_t Q = (int64_t)blockIdx.x * 256 + threadIdx.x; Q < naux;
       Q += (int64_t)gridDim.x * 256) {
    const double *b = Bo + Q * no * nmo;
    double s = 0.0;
    for (int64_t i = 0; i < nd; ++i) s += 2.0 * b[i * nmo + i];
    for (int64_t u = 0; u < na; ++u)
      for (int64_t v = 0; v < na; ++v) s += gamma1[u * na + v] * b[(nd + u) * nmo + nd + v];
    d[Q] = s;
  }
}

// Bh^Q_mq: B^Q_mq for m < nd, (1/2) sum_v Gamma_{m-nd, v} B^Q_{nd+v, q} for the
// active rows; one thread per element
__global__ __launch_bounds__(256) void fock_exchange_rhs_kernel(const double *__restrict__ Bo,
                                                                const double *__restrict__ gamma1,
                                                                int64_t naux, int64_t no,
                                                                int64_t nmo, int64_t nd,
                                                                int64_t na,
                                                                double *__restrict__ Bh) {
  const int64_t total = naux * no * nmo;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t q = e % nmo, m = (e / nmo) % no, Q = e / (no * nmo);
    double v;
    if (m < nd) {
      v = Bo[e];
    } else {
      const double *b = Bo + (Q * no + nd) * nmo + q;
      const double *g = gamma1 + (m - nd) * na;
      v = 0.0;
      for (int64_t w = 0; w < na; ++w) v += g[w] * b[w * nmo];
      v *= 0.5;
    }
    Bh[e] = v;
  }
}

hipError_t launch_df_fock(const FockPlan &pl, const FockInputs &in, double *F, void *ws,
                          hipStream_t st) {
  hipError_t e;
  const int64_t nao = pl.nao, nmo = pl.nmo, naux = pl.naux, no = pl.no, nd = pl.nd, na = pl.na;
  double *T = ws_d(ws, pl.off_t), *Y = ws_d(ws, pl.off_y), *Lm = ws_d(ws, pl.off_l);
  double *X = ws_d(ws, pl.off_x), *W = ws_d(ws, pl.off_w), *Bo = ws_d(ws, pl.off_bo);
  double *dv = ws_d(ws, pl.off_d), *cv = ws_d(ws, pl.off_c), *Jao = ws_d(ws, pl.off_jao);
  double *Tj = ws_d(ws, pl.off_tj), *Part = ws_d(ws, pl.off_part);
  // the metric factor and inverse, beside the transforms (Lm, X, W there;
  // T, Y here); none for factors that need no metric
  SideStream *ss = nullptr;
  if (pl.metric &&
      (e = metric_forked("fock_metric", in.J, Lm, X, W, naux, st, ss)) != hipSuccess)
    return e;
  // T[P][m][nu] = sum_mu C[mu][m] (mu nu|P), m occupied
  timer_begin("fock_half1", st);
  if (folded_fits(no, nao, naux))
    e = gemm_g_folded(true, no, nao, nao, 1.0, in.C, nmo, in.ao3, nao, nao * nao, T, nao,
                      no * nao, naux, st);
  else
    e = gemm_g(true, false, no, nao, nao, 1.0, in.C, nmo, 0, in.ao3, nao, nao * nao, 0.0, T, nao,
               no * nao, naux, false, st);
  timer_end(st);
  if (e != hipSuccess) return e;
  // Y[(P m)][q] = sum_nu T[(P m)][nu] C[nu][q], q over all MOs (straight into
  // B when there is no metric)
  timer_begin("fock_half2", st);
  e = gemm_g(false, false, naux * no, nmo, nao, 1.0, T, nao, 0, in.C, nmo, 0, 0.0,
             pl.metric ? Y : Bo, nmo, 0, 1, false, st);
  timer_end(st);
  if (e != hipSuccess) return e;
  if (pl.metric) {
    if ((e = side_join(ss, st)) != hipSuccess) return e;
    // B[Q][(m q)] = sum_{P <= Q} X[Q][P] Y[P][(m q)]
    timer_begin("fock_metric_apply", st);
    e = gemm_g(false, false, naux, no * nmo, naux, 1.0, X, naux, 0, Y, no * nmo, 0, 0.0, Bo,
               no * nmo, 0, 1, true, st);
    timer_end(st);
    if (e != hipSuccess) return e;
  }
  // Coulomb part, through the AO basis (c = X^T d, or d itself with no metric)
  timer_begin("fock_coulomb", st);
  hipLaunchKernelGGL(fock_density_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(naux, 256), 1024)),
                     dim3(256), 0, st, Bo, in.gamma1, naux, no, nmo, nd, na, dv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (pl.metric) {
    if ((e = gemm_g(true, false, naux, 1, naux, 1.0, X, naux, 0, dv, 1, 0, 0.0, cv, 1, 0, 1,
                    false, st)) != hipSuccess)
      return e;
  } else {
    cv = dv;
  }
  if ((e = gemm_g(false, false, 1, nao * nao, naux, 1.0, cv, naux, 0, in.ao3, nao * nao, 0, 0.0,
                  Jao, nao * nao, 0, 1, false, st)) != hipSuccess)
    return e;
  if ((e = gemm_g(false, false, nao, nmo, nao, 1.0, Jao, nao, 0, in.C, nmo, 0, 0.0, Tj, nmo, 0, 1,
                  false, st)) != hipSuccess)
    return e;
  // F = h, then F += C^T (J_AO C)
  if ((e = hipMemcpyAsync(F, in.h, sizeof(double) * nmo * nmo, hipMemcpyDeviceToDevice, st)) !=
      hipSuccess)
    return e;
  if ((e = gemm_g(true, false, nmo, nmo, nao, 1.0, in.C, nmo, 0, Tj, nmo, 0, 1.0, F, nmo, 0, 1,
                  false, st)) != hipSuccess)
    return e;
  timer_end(st);
  // exchange part: F -= sum_{(Q m)} B[(Q m)][p] Bh[(Q m)][q]
  timer_begin("fock_exchange", st);
  double *Bh = Y;   // Y is no longer needed
  const int64_t total = naux * no * nmo;
  hipLaunchKernelGGL(fock_exchange_rhs_kernel,
                     dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 65536)), dim3(256), 0,
                     st, Bo, in.gamma1, naux, no, nmo, nd, na, Bh);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  e = gemm_g_splitk(true, false, nmo, nmo, naux * no, -1.0, Bo, nmo, Bh, nmo, 1.0, F, Part,
                    splitk_segments(nmo, nmo, naux * no), st);
  timer_end(st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace dsrg
