// Laplace-type factorization of the Coulomb part of the CCVV energy (the
// outlook of section VI: a decomposition of the renormalised denominator).
//
// With x = e_a + e_b - e_i - e_j > 0, the CCVV regulariser of Eq. expensive
// is R(Delta) = -h(x), h(x) = (1 - exp(-2 s x^2)) / x. On the interval that
// holds every x of a problem, h is approximated by an exponential sum
// sum_k w_k exp(-t_k x) (laplace_fit below). Each term separates over the four
// orbital energies, so the Coulomb part E_J = 2 sum (ia|jb)^2 R(Delta) becomes
//   E_J ~ -2 sum_k w_k S_k,   S_k = sum_{PQ} (Y_k)_{PQ}^2,
//   Y_k = (B D_k) B^T over the (i, a) index, D_k = diag(exp(-t_k (e_a - e_i))),
// a product of 2 naux^2 nc nv flops per term instead of the fifth-order pair
// sum. D_k is positive, so Y_k = C_k C_k^T with C_k = B D_k^{1/2} is a
// symmetric Gram matrix and only its upper triangle is formed (half the
// flops). Per batch of terms: one scaling kernel writes C_k, one batched FP64
// matrix-core product forms the tiles (r, c), r <= c, of the Y_k, one kernel
// reduces their squares into per-workgroup slots (tiles above the diagonal
// tiles counted twice); a last kernel adds the slots of each term in a fixed
// order and combines the terms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common_device.h"
#include "internal.h"

namespace dsrg {

// ---------------------------------------------------------------------------
// host: the exponential-sum fit
// ---------------------------------------------------------------------------
namespace {

constexpr int kFitSamples = 600, kFitCheck = 5000;
const double kFitC1[3] = {0.1, 0.3, 1.0};
const double kFitC2[3] = {3.0, 10.0, 30.0};

double h_of_x(double x, double s) { return -std::expm1(-2.0 * s * x * x) / x; }

// n points from a to b, evenly spaced in log
void geom(double a, double b, int n, std::vector<double> &out) {
  out.resize(n);
  if (n == 1) {
    out[0] = a;
    return;
  }
  const double la = std::log(a), lb = std::log(b);
  for (int i = 0; i < n; ++i) out[i] = std::exp(la + (lb - la) * i / (n - 1));
  out[0] = a;
  out[n - 1] = b;
}

// min ||A w - y|| for A (m x n, column-major, m >= n): columns scaled to unit
// norm, Householder QR, back substitution; a column whose diagonal of R falls
// below 1e-15 of the largest is dropped (weight 0)
void lstsq(std::vector<double> A, std::vector<double> y, int m, int n, double *w) {
  std::vector<double> scale(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double nn = 0.0;
    for (int i = 0; i < m; ++i) nn += A[(size_t)j * m + i] * A[(size_t)j * m + i];
    scale[j] = nn > 0.0 ? 1.0 / std::sqrt(nn) : 0.0;
    for (int i = 0; i < m; ++i) A[(size_t)j * m + i] *= scale[j];
  }
  std::vector<double> rdiag(n, 0.0), v(m);
  for (int j = 0; j < n; ++j) {
    double *a = &A[(size_t)j * m];
    double nn = 0.0;
    for (int i = j; i < m; ++i) nn += a[i] * a[i];
    const double norm = std::sqrt(nn);
    if (norm == 0.0) continue;
    const double alpha = a[j] > 0.0 ? -norm : norm;
    for (int i = j; i < m; ++i) v[i] = a[i];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < m; ++i) vv += v[i] * v[i];
    rdiag[j] = alpha;
    if (vv == 0.0) continue;
    for (int c = j; c < n; ++c) {
      double *ac = &A[(size_t)c * m];
      double d = 0.0;
      for (int i = j; i < m; ++i) d += v[i] * ac[i];
      const double f = 2.0 * d / vv;
      for (int i = j; i < m; ++i) ac[i] -= f * v[i];
    }
    double d = 0.0;
    for (int i = j; i < m; ++i) d += v[i] * y[i];
    const double f = 2.0 * d / vv;
    for (int i = j; i < m; ++i) y[i] -= f * v[i];
  }
  double rmax = 0.0;
  for (int j = 0; j < n; ++j) rmax = std::max(rmax, std::fabs(A[(size_t)j * m + j]));
  for (int j = n - 1; j >= 0; --j) {
    const double r = A[(size_t)j * m + j];
    if (std::fabs(r) <= 1e-15 * rmax || rmax == 0.0) {
      w[j] = 0.0;
      continue;
    }
    double acc = y[j];
    for (int c = j + 1; c < n; ++c) acc -= A[(size_t)c * m + j] * w[c];
    w[j] = acc / r;
  }
  for (int j = 0; j < n; ++j) w[j] *= scale[j];
}

}  // namespace

int laplace_fit(double s, double x_lo, double x_hi, int nq, double *t, double *w,
                double *max_err) {
  std::vector<double> xs, xc, tt(nq), ww(nq), ys(kFitSamples), hc(kFitCheck);
  geom(x_lo, x_hi, kFitSamples, xs);
  geom(x_lo, x_hi, kFitCheck, xc);
  for (int i = 0; i < kFitSamples; ++i) ys[i] = h_of_x(xs[i], s);
  for (int i = 0; i < kFitCheck; ++i) hc[i] = h_of_x(xc[i], s);
  double best = -1.0;
  for (double c1 : kFitC1)
    for (double c2 : kFitC2) {
      std::vector<double> tk;
      if (nq > 1)
        geom(c1 / x_hi, c2 / x_lo, nq, tk);
      else
        tk.assign(1, c1 / x_hi);
      std::vector<double> A((size_t)kFitSamples * nq);
      for (int j = 0; j < nq; ++j)
        for (int i = 0; i < kFitSamples; ++i) A[(size_t)j * kFitSamples + i] = std::exp(-tk[j] * xs[i]);
      lstsq(A, ys, kFitSamples, nq, ww.data());
      double err = 0.0;
      for (int i = 0; i < kFitCheck; ++i) {
        double f = 0.0;
        for (int j = 0; j < nq; ++j) f += ww[j] * std::exp(-tk[j] * xc[i]);
        err = std::max(err, std::fabs(f - hc[i]));
      }
      if (best < 0.0 || err < best) {
        best = err;
        for (int j = 0; j < nq; ++j) {
          t[j] = tk[j];
          w[j] = ww[j];
        }
      }
    }
  *max_err = best;
  return 0;
}

// ---------------------------------------------------------------------------
// device
// ---------------------------------------------------------------------------
namespace {

struct LtTerms {
  double t[kLtMaxTerms], w[kLtMaxTerms];
};

// Bs[kk][Q][(i, a)] = B[Q][i][a] exp(-t_{k0 + kk} (e_a - e_i) / 2) for kk < kb
__global__ __launch_bounds__(256) void lt_scale_kernel(const double *__restrict__ B,
                                                       const double *__restrict__ eps_c,
                                                       const double *__restrict__ eps_v,
                                                       LtTerms T, int k0, int kb, int64_t naux,
                                                       int64_t nc, int64_t nv,
                                                       double *__restrict__ Bs) {
  const int64_t per = naux * nc * nv, total = per * kb;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t kk = e / per, r = e % per;
    const int64_t a = r % nv, i = (r / nv) % nc;
    Bs[e] = B[r] * exp(-0.5 * T.t[k0 + kk] * (eps_v[a] - eps_c[i]));
  }
}

// slots[(k0 + kk) nwg + blockIdx.x] = this workgroup's share of ||Y[kk]||_F^2
// from the upper tiles of the symmetric Y[kk] (tile size tile): rows P =
// blockIdx.x, + nwg, ..., columns from the start of P's diagonal tile, the
// diagonal tile once and the tiles right of it twice (grid nwg x kb, fixed
// order)
__global__ __launch_bounds__(256) void lt_sumsq_kernel(const double *__restrict__ Y, int64_t n,
                                                       int64_t tile, int k0, int64_t nwg,
                                                       double *__restrict__ slots) {
  __shared__ double red[4];
  const double *y = Y + (int64_t)blockIdx.y * n * n;
  double acc = 0.0;
  for (int64_t P = blockIdx.x; P < n; P += nwg) {
    const int64_t q0 = (P / tile) * tile, q1 = q0 + tile;
    for (int64_t Q = q0 + threadIdx.x; Q < n; Q += 256) {
      const double v = y[P * n + Q];
      acc = fma(Q < q1 ? v : 2.0 * v, v, acc);
    }
  }
  const double t = block_sum(acc, red);
  if (threadIdx.x == 0) slots[(int64_t)(k0 + blockIdx.y) * nwg + blockIdx.x] = t;
}

// E[0] = -2 sum_k w_k S_k and, if S is given, S[k] = sum of the slots of term k
__global__ __launch_bounds__(256) void lt_finalize_kernel(const double *__restrict__ slots,
                                                          int64_t nwg, int nq, LtTerms T,
                                                          double *E, double *S) {
  __shared__ double red[4];
  __shared__ double sk[kLtMaxTerms];
  for (int k = 0; k < nq; ++k) {
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nwg; b += 256) acc += slots[(int64_t)k * nwg + b];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) sk[k] = t;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // Neumaier sum of the weighted terms
    double sum = 0.0, c = 0.0;
    for (int k = 0; k < nq; ++k) {
      const double v = T.w[k] * sk[k];
      const double tt = sum + v;
      c += (std::fabs(sum) >= std::fabs(v)) ? (sum - tt) + v : (v - tt) + sum;
      sum = tt;
      if (S) S[k] = sk[k];
    }
    E[0] = -2.0 * (sum + c);
  }
}

}  // namespace

hipError_t launch_coulomb_laplace(const LtPlan &pl, const double *B_cv, const double *eps_c,
                                  const double *eps_v, const double *t, const double *w,
                                  double *E, double *S, void *ws, hipStream_t st) {
  hipError_t e;
  LtTerms T;
  for (int k = 0; k < kLtMaxTerms; ++k) {
    T.t[k] = k < pl.nq ? t[k] : 0.0;
    T.w[k] = k < pl.nq ? w[k] : 0.0;
  }
  double *Bs = ws_d(ws, pl.off_bs), *Y = ws_d(ws, pl.off_y), *slots = ws_d(ws, pl.off_slots);
  const int64_t ncnv = pl.nc * pl.nv, n2 = pl.naux * pl.naux;
  for (int k0 = 0; k0 < pl.nq; k0 += pl.kb) {
    const int kb = std::min(pl.kb, pl.nq - k0);
    const int64_t total = (int64_t)kb * pl.naux * ncnv;
    timer_begin("lt_scale", st);
    hipLaunchKernelGGL(lt_scale_kernel,
                       dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 65536)), dim3(256),
                       0, st, B_cv, eps_c, eps_v, T, k0, kb, pl.naux, pl.nc, pl.nv, Bs);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    timer_begin("lt_gemm", st);
    int64_t tile = 0;
    e = gemm_f64_gram_upper(false, pl.naux, ncnv, Bs, ncnv, pl.naux * ncnv, Y, pl.naux, n2, kb,
                            &tile, st);
    timer_end(st);
    if (e != hipSuccess) return e;
    timer_begin("lt_sumsq", st);
    hipLaunchKernelGGL(lt_sumsq_kernel, dim3((unsigned)pl.nwg, (unsigned)kb), dim3(256), 0, st, Y,
                       pl.naux, tile, k0, pl.nwg, slots);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  timer_begin("lt_finalize", st);
  hipLaunchKernelGGL(lt_finalize_kernel, dim3(1), dim3(256), 0, st, slots, pl.nwg, pl.nq, T, E,
                     S);
  timer_end(st);
  return hipGetLastError();
}

}  // namespace dsrg
