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
// (pq|rs) unchanged. Steps: T[(P mu)][q] = (mu nu|P) C_{nu q} (one GEMM over
// all P and mu), Y[P][p][q] = C_{mu p} T[P][mu][q] (batched over P), the
// blocked Cholesky factor of J and its blocked inverse, B = L^{-1} Y (one GEMM
// whose contraction stops at the diagonal), and a scatter into the four
// output blocks.
#include <algorithm>

#include "common_device.h"
#include "internal.h"

namespace dsrg {

// ---------------------------------------------------------------------------
// C[b] = alpha op(A[b]) op(B[b]) + beta C[b] for b = blockIdx.z, row-major:
//   op(A)(m, k) = TA ? A[k lda + m] : A[m lda + k]
//   op(B)(k, n) = TB ? B[n ldb + k] : B[k ldb + n]
// 128 x 128 tile per workgroup of 8 waves (two per SIMD), wave w owning rows
// 64 (w >> 2) .. +63 and columns 32 (w & 3) .. +31; K chunks of 16 staged
// through registers into LDS ([k][m] and [k][n] rows of 128, odd rows with
// their 16-column halves swapped), one barrier per chunk. Out-of-range
// elements read as zero. With ktri set the contraction of row tile t stops
// at k = 128 (t + 1) (A lower triangular).
// ---------------------------------------------------------------------------
struct GemmGArgs {
  int64_t M, N, K;
  int64_t lda, ldb, ldc;
  int64_t sa, sb, sc;      // batch strides
  double alpha, beta;
  int ktri;
};

constexpr int kGG = 128, kGGK = 16, kGGThreads = 512;

__device__ __forceinline__ int gswz(int k) { return (k & 1) << 4; }

template <bool TA, bool TB>
__global__ __launch_bounds__(kGGThreads) void gemm_g_kernel(const double *__restrict__ A,
                                                          const double *__restrict__ B,
                                                          GemmGArgs a, double *__restrict__ C) {
  __shared__ double sA[2][kGGK * kGG];
  __shared__ double sB[2][kGGK * kGG];
  const int64_t m0 = (int64_t)blockIdx.x * kGG, n0 = (int64_t)blockIdx.y * kGG;
  A += (int64_t)blockIdx.z * a.sa;
  B += (int64_t)blockIdx.z * a.sb;
  C += (int64_t)blockIdx.z * a.sc;
  const int64_t K = a.ktri ? std::min(a.K, m0 + kGG) : a.K;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int cl = lane & 15, kl = lane >> 4;
  d4 acc[4][2];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = d4{0.0, 0.0, 0.0, 0.0};

  // chunk element e = t + 512 j (j < 4): row k = e / 128, column c = e % 128
  double ra[4], rb[4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = t + kGGThreads * j;
      const int64_t k = k0 + e / kGG;
      const int64_t m = m0 + e % kGG, n = n0 + e % kGG;
      double va = 0.0, vb = 0.0;
      if (k < K) {
        if (m < a.M) va = TA ? A[k * a.lda + m] : A[m * a.lda + k];
        if (n < a.N) vb = TB ? B[n * a.ldb + k] : B[k * a.ldb + n];
      }
      ra[j] = va;
      rb[j] = vb;
    }
  };
  auto sstore = [&](int b) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = t + kGGThreads * j;
      const int k = e / kGG, c = e % kGG;
      sA[b][k * kGG + (c ^ gswz(k))] = ra[j];
      sB[b][k * kGG + (c ^ gswz(k))] = rb[j];
    }
  };

  if (K > 0) {
    gload(0);
    sstore(0);
    if (K > kGGK) gload(kGGK);
  }
  __syncthreads();
  int b = 0;
  for (int64_t k0 = 0; k0 < K; k0 += kGGK) {
    const double *LA = sA[b], *LB = sB[b];
#pragma unroll
    for (int kk = 0; kk < kGGK / 4; ++kk) {
      const int k = kk * 4 + kl;
      double fa[4], fb[2];
#pragma unroll
      for (int p = 0; p < 4; ++p) fa[p] = LA[k * kGG + ((64 * wr + 16 * p + cl) ^ gswz(k))];
#pragma unroll
      for (int q = 0; q < 2; ++q) fb[q] = LB[k * kGG + ((32 * wc + 16 * q + cl) ^ gswz(k))];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[p], fb[q], acc[p][q], 0, 0, 0);
    }
    if (k0 + kGGK < K) {
      sstore(b ^ 1);
      if (k0 + 2 * kGGK < K) gload(k0 + 2 * kGGK);
    }
    __syncthreads();
    b ^= 1;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int64_t n = n0 + 32 * wc + 16 * q + cl;
    if (n >= a.N) continue;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + 64 * wr + 16 * p + 4 * r + kl;
        if (m >= a.M) continue;
        double *dst = C + m * a.ldc + n;
        const double v = a.alpha * acc[p][q][r];
        *dst = (a.beta != 0.0) ? v + a.beta * *dst : v;
      }
  }
}

static hipError_t gemm_g(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                         const double *A, int64_t lda, int64_t sa, const double *B, int64_t ldb,
                         int64_t sb, double beta, double *C, int64_t ldc, int64_t sc,
                         int64_t batch, bool ktri, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  GemmGArgs a{M, N, K, lda, ldb, ldc, sa, sb, sc, alpha, beta, ktri ? 1 : 0};
  const dim3 grid((unsigned)ceil_div(M, kGG), (unsigned)ceil_div(N, kGG), (unsigned)batch);
  if (!ta && !tb)
    hipLaunchKernelGGL((gemm_g_kernel<false, false>), grid, dim3(kGGThreads), 0, st, A, B, a, C);
  else if (ta && !tb)
    hipLaunchKernelGGL((gemm_g_kernel<true, false>), grid, dim3(kGGThreads), 0, st, A, B, a, C);
  else if (!ta && tb)
    hipLaunchKernelGGL((gemm_g_kernel<false, true>), grid, dim3(kGGThreads), 0, st, A, B, a, C);
  else
    hipLaunchKernelGGL((gemm_g_kernel<true, true>), grid, dim3(kGGThreads), 0, st, A, B, a, C);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Blocked Cholesky J = L L^T in place (lower triangle; the strict upper
// triangle of each diagonal block is cleared), block width kDB. A metric that
// is not positive definite gives NaN in L (square root of a negative pivot).
// ---------------------------------------------------------------------------
constexpr int kDB = 64;

// factor the nb x nb diagonal block at (k0, k0) (one workgroup)
__global__ __launch_bounds__(256) void potrf_diag_kernel(double *__restrict__ Am, int64_t lda,
                                                         int64_t k0, int nb) {
  __shared__ double a[kDB][kDB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    a[i][j] = Am[(k0 + i) * lda + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (threadIdx.x == 0) a[j][j] = sqrt(a[j][j]);
    __syncthreads();
    const double d = a[j][j];
    for (int i = j + 1 + threadIdx.x; i < nb; i += 256) a[i][j] /= d;
    __syncthreads();
    // trailing a[i][l] -= a[i][j] a[l][j] for j < l <= i
    const int w = nb - j - 1;
    for (int e = threadIdx.x; e < w * w; e += 256) {
      const int i = j + 1 + e / w, l = j + 1 + e % w;
      if (l <= i) a[i][l] -= a[i][j] * a[l][j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    Am[(k0 + i) * lda + k0 + j] = (j <= i) ? a[i][j] : 0.0;
  }
}

// rows i in [k0 + nb, n): L[i][k0 .. k0+nb) = A[i][k0 .. k0+nb) L_kk^{-T}
__global__ __launch_bounds__(256) void trsm_panel_kernel(double *__restrict__ Am, int64_t lda,
                                                         int64_t k0, int nb, int64_t n) {
  __shared__ double l[kDB][kDB + 1];
  for (int e = threadIdx.x; e < nb * nb; e += 256) {
    const int i = e / nb, j = e % nb;
    l[i][j] = Am[(k0 + i) * lda + k0 + j];
  }
  __syncthreads();
  const int64_t i = k0 + nb + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double *row = Am + i * lda + k0;
  double x[kDB];
#pragma unroll
  for (int j = 0; j < kDB; ++j) {
    if (j < nb) {
      double v = row[j];
      for (int c = 0; c < j; ++c) v -= x[c] * l[j][c];
      x[j] = v / l[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < kDB; ++j)
    if (j < nb) row[j] = x[j];
}

// inverse of each lower-triangular diagonal block of L into X (block b per
// workgroup; thread c solves column c of L_bb X_bb = I)
__global__ __launch_bounds__(64) void trinv_diag_kernel(const double *__restrict__ L,
                                                        double *__restrict__ X, int64_t ld,
                                                        int64_t n) {
  __shared__ double l[kDB][kDB + 1];
  const int64_t k0 = (int64_t)blockIdx.x * kDB;
  const int nb = (int)std::min<int64_t>(kDB, n - k0);
  for (int e = threadIdx.x; e < nb * nb; e += 64) {
    const int i = e / nb, j = e % nb;
    l[i][j] = L[(k0 + i) * ld + k0 + j];
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c >= nb) return;
  double x[kDB];
#pragma unroll
  for (int r = 0; r < kDB; ++r) {
    if (r < nb) {
      double v = (r == c) ? 1.0 : 0.0;
      if (r < c) {
        v = 0.0;
      } else {
        for (int q = c; q < r; ++q) v -= l[r][q] * x[q];
        v /= l[r][r];
      }
      x[r] = v;
    }
  }
#pragma unroll
  for (int r = 0; r < kDB; ++r)
    if (r < nb) X[(k0 + r) * ld + k0 + c] = x[r];
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
hipError_t launch_df_factors(const DFPlan &pl, const DFInputs &in, const DFOutputs &o, void *ws,
                             hipStream_t st) {
  hipError_t e;
  const int64_t nao = pl.nao, nmo = pl.nmo, naux = pl.naux;
  const int64_t np = pl.nc + pl.na, nq = pl.na + pl.nv;
  const int64_t oc = pl.nfrz, oa = pl.nfrz + pl.nc;
  double *T = ws_d(ws, pl.off_t), *Y = ws_d(ws, pl.off_y), *Lm = ws_d(ws, pl.off_l);
  double *X = ws_d(ws, pl.off_x), *Tmp = ws_d(ws, pl.off_tmp), *Bf = ws_d(ws, pl.off_bf);
  // T[(P mu)][q] = sum_nu (mu nu|P) C[nu][oa + q]
  timer_begin("df_half1", st);
  e = gemm_g(false, false, naux * nao, nq, nao, 1.0, in.ao3, nao, 0, in.C + oa, nmo, 0, 0.0, T,
             nq, 0, 1, false, st);
  timer_end(st);
  if (e != hipSuccess) return e;
  // Y[P][p][q] = sum_mu C[mu][oc + p] T[P][mu][q]
  timer_begin("df_half2", st);
  e = gemm_g(true, false, np, nq, nao, 1.0, in.C + oc, nmo, 0, T, nq, nao * nq, 0.0, Y, nq,
             np * nq, naux, false, st);
  timer_end(st);
  if (e != hipSuccess) return e;
  // Cholesky factor of J (copy into L), then X = L^{-1}
  timer_begin("df_metric", st);
  if ((e = hipMemcpyAsync(Lm, in.J, sizeof(double) * naux * naux, hipMemcpyDeviceToDevice, st)) !=
      hipSuccess)
    return e;
  for (int64_t k0 = 0; k0 < naux; k0 += kDB) {
    const int nb = (int)std::min<int64_t>(kDB, naux - k0);
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, Lm, naux, k0, nb);
    const int64_t rest = naux - k0 - nb;
    if (rest > 0) {
      hipLaunchKernelGGL(trsm_panel_kernel, dim3((unsigned)ceil_div(rest, 256)), dim3(256), 0, st,
                         Lm, naux, k0, nb, naux);
      // trailing J[i][j] -= L[i][panel] L[j][panel]^T for i, j >= k0 + nb
      double *Lp = Lm + (k0 + nb) * naux + k0;
      e = gemm_g(false, true, rest, rest, nb, -1.0, Lp, naux, 0, Lp, naux, 0, 1.0,
                 Lm + (k0 + nb) * naux + k0 + nb, naux, 0, 1, false, st);
      if (e != hipSuccess) return e;
    }
  }
  // X: clear, diagonal block inverses, then block rows
  //   X[i, 0:i] = -X_ii (L[i, 0:i] X[0:i, 0:i])
  if ((e = launch_zero_fill(X, naux * naux, st)) != hipSuccess) return e;
  const int64_t nblk = ceil_div(naux, kDB);
  hipLaunchKernelGGL(trinv_diag_kernel, dim3((unsigned)nblk), dim3(64), 0, st, Lm, X, naux, naux);
  for (int64_t i = 1; i < nblk; ++i) {
    const int64_t r0 = i * kDB, nr = std::min<int64_t>(kDB, naux - r0);
    e = gemm_g(false, false, nr, r0, r0, 1.0, Lm + r0 * naux, naux, 0, X, naux, 0, 0.0, Tmp, naux,
               0, 1, false, st);
    if (e != hipSuccess) return e;
    e = gemm_g(false, false, nr, r0, nr, -1.0, X + r0 * naux + r0, naux, 0, Tmp, naux, 0, 0.0,
               X + r0 * naux, naux, 0, 1, false, st);
    if (e != hipSuccess) return e;
  }
  timer_end(st);
  // B[Q][(p q)] = sum_{P <= Q} X[Q][P] Y[P][(p q)]
  timer_begin("df_metric_apply", st);
  e = gemm_g(false, false, naux, np * nq, naux, 1.0, X, naux, 0, Y, np * nq, 0, 0.0, Bf, np * nq,
             0, 1, true, st);
  timer_end(st);
  if (e != hipSuccess) return e;
  ScatterArgs sa{naux, pl.nc, pl.na, pl.nv};
  const int64_t total = naux * np * nq;
  timer_begin("df_scatter", st);
  hipLaunchKernelGGL(df_scatter_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 65536)),
                     dim3(256), 0, st, Bf, sa, o.B_cv, o.B_ca, o.B_av, o.B_aa);
  timer_end(st);
  return hipGetLastError();
}

}  // namespace dsrg
