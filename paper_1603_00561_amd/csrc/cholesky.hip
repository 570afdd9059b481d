// Cholesky-decomposition (CD) factors of the AO two-electron integrals, the
// CD approach of section II.C: a numerical pivoted Cholesky decomposition of
// the integral matrix over packed AO pairs,
//   M[(mu nu)][(la si)] = (mu nu|la si),  pair index mu (mu + 1) / 2 + nu, mu >= nu,
// stopped once the largest diagonal of the residual M - sum_Q L^Q L^Q^T is at
// most the CD threshold (which bounds every element of the PSD residual, so
// the threshold is the error of Eq. int_fact with M = rank terms).
//
// Greedy pivoting: step k takes the pair p of the largest residual diagonal d
// (the smallest index on ties) and forms the Cholesky vector
//   L^k_i = (M_{p i} - sum_{j<k} L^j_i L^j_p) / sqrt(d_p),   d_i -= (L^k_i)^2, d_p = 0.
// The vectors are written unpacked and symmetric as B^Q_{mu nu} = B^Q_{nu mu}
// = L^Q_{(mu nu)}, the three-index layout the factor build transforms.
//
// GPU shape: one launch per Cholesky vector (the pivot of step k + 1 depends
// on every element of vector k). Each launch streams the k earlier vectors
// once (a matrix-vector product against the pivot's row, HBM-bound), with the
// pair rows spread over the workgroups and the earlier vectors over the
// waves of a workgroup. Every workgroup publishes the maximum of the updated
// diagonal over its rows (double-buffered by step parity); the next launch
// starts with every workgroup reducing those maxima itself, in workgroup
// order, to the same pivot (no atomics, no inter-workgroup waits). Launches
// past convergence return at once (a done flag in the workspace). Every sum
// runs in a fixed order, so results repeat bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace dsrg {

namespace {

constexpr int kCdT = 256;     // threads per workgroup of the init and finish kernels
constexpr int kCdLp = 2048;   // pivot-row values of the earlier vectors staged per LDS chunk
constexpr int kCdU = 8;       // earlier vectors loaded back to back per thread

struct CdArgs {
  const double *M;   // [N][N] integrals over packed pairs
  double *B;         // [max_rank][nao][nao] vectors, unpacked
  double *d;         // [N] residual diagonal
  double *part_v;    // [2][pstride] per-workgroup maxima of d, by step parity
  int64_t *part_i;   // [2][pstride] their pair indices
  CdState *state;
  int64_t *pivots;   // [max_rank] or nullptr
  int64_t nao, npair, pstride;
  double tol;
};

// (mu, nu) with mu >= nu of packed pair index i = mu (mu + 1) / 2 + nu
__device__ inline void pair_of(int64_t i, int64_t &mu, int64_t &nu) {
  int64_t m = (int64_t)((sqrt(8.0 * (double)i + 1.0) - 1.0) * 0.5);
  while ((m + 1) * (m + 2) / 2 <= i) ++m;
  while (m * (m + 1) / 2 > i) --m;
  mu = m;
  nu = i - m * (m + 1) / 2;
}

// (v1, i1) replaces (v2, i2) as the maximum: larger value, or equal value and
// smaller index; a NaN never does
__device__ inline bool beats(double v1, int64_t i1, double v2, int64_t i2) {
  return v1 > v2 || (v1 == v2 && i1 < i2);
}

// d - c^2 with the product rounded on its own (no fused multiply-add), as a
// plain evaluation of the update does it
__device__ inline double sub_square(double d, double c) {
#pragma clang fp contract(off)
  return d - c * c;
}

// Workgroup argmax of (v, i) over all T threads, returned to every thread:
// a butterfly over the 64 lanes of each wave (the order is total, so every
// lane ends with the same maximum), then the T / 64 wave maxima in order. A
// NaN value takes no part (it is never a maximum).
template <int T>
__device__ inline void block_argmax(double &v, int64_t &i, double *sv, int64_t *si) {
  if (!(v == v)) {
    v = -INFINITY;
    i = INT64_MAX;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const int64_t oi = __shfl_xor(i, off);
    if (beats(ov, oi, v, i)) {
      v = ov;
      i = oi;
    }
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();   // earlier readers of sv / si are done
  if ((threadIdx.x & 63) == 0) {
    sv[w] = v;
    si[w] = i;
  }
  __syncthreads();
  v = sv[0];
  i = si[0];
#pragma unroll
  for (int q = 1; q < T / 64; ++q)
    if (beats(sv[q], si[q], v, i)) {
      v = sv[q];
      i = si[q];
    }
}

// The pivot of the next step: the maximum over the n maxima that the
// previous launch published at parity `par`, reduced by every workgroup to
// the same (value, index) (the order of the comparisons is fixed).
template <int T>
__device__ inline void reduce_published(const CdArgs &a, int par, int64_t n, double &v,
                                        int64_t &i, double *sv, int64_t *si) {
  const double *pv = a.part_v + par * a.pstride;
  const int64_t *pi = a.part_i + par * a.pstride;
  double bv = -INFINITY;
  int64_t bi = INT64_MAX;
  for (int64_t b = threadIdx.x; b < n; b += T) {
    const double w = pv[b];
    const int64_t j = pi[b];
    if (beats(w, j, bv, bi)) {
      bv = w;
      bi = j;
    }
  }
  block_argmax<T>(bv, bi, sv, si);
  v = bv;
  i = bi;
}

// publish this workgroup's maximum (v, i) at parity `par`
template <int T>
__device__ inline void publish(const CdArgs &a, int par, double v, int64_t i, double *sv,
                               int64_t *si) {
  block_argmax<T>(v, i, sv, si);
  if (threadIdx.x == 0) {
    a.part_v[par * a.pstride + blockIdx.x] = v;
    a.part_i[par * a.pstride + blockIdx.x] = i;
  }
}

// d = diag(M), its maxima published at parity 0; one thread per pair
__global__ __launch_bounds__(kCdT) void cd_init_kernel(CdArgs a) {
  __shared__ double sv[kCdT];
  __shared__ int64_t si[kCdT];
  const int64_t i = (int64_t)blockIdx.x * kCdT + threadIdx.x;
  double v = -INFINITY;
  int64_t vi = INT64_MAX;
  if (i < a.npair) {
    v = a.M[i * a.npair + i];
    vi = i;
    a.d[i] = v;
  }
  publish<kCdT>(a, 0, v, vi, sv, si);
}

// Cholesky vector k: R pair rows per workgroup of T threads, G = T / R
// groups of earlier vectors per row (vector j in group j mod G, summed in
// increasing j within a group, then over the groups in order); nprev maxima
// published by the previous launch
template <int R, int T>
__global__ __launch_bounds__(T) void cd_step_kernel(CdArgs a, int64_t k, int64_t nprev) {
  constexpr int G = T / R;
  __shared__ double lp[kCdLp];
  __shared__ double sv[T];
  __shared__ int64_t si[T];
  if (a.state->done) return;
  const int64_t nao = a.nao, nao2 = a.nao * a.nao, N = a.npair;
  const int t = threadIdx.x, r = t % R, g = t / R;
  const int64_t i = (int64_t)blockIdx.x * R + r;
  const bool valid = i < N;
  const bool owner = g == 0 && valid;   // the thread that finishes row i
  int64_t mu = 0, nu = 0;
  if (valid) pair_of(i, mu, nu);
  const int64_t ioff = mu * nao + nu;
  // loads that do not depend on the pivot go out before its reduction: the
  // residual diagonal of row i and the first round of earlier-vector values
  const double d_i = owner ? a.d[i] : 0.0;
  const int cn0 = (int)(k < kCdLp ? k : kCdLp);
  double x0[kCdU];
#pragma unroll
  for (int u = 0; u < kCdU; ++u) {
    const int jj = g + u * G;
    x0[u] = (valid && jj < cn0) ? a.B[(int64_t)jj * nao2 + ioff] : 0.0;
  }
  double dmax;
  int64_t p;
  reduce_published<T>(a, (int)(k & 1), nprev, dmax, p, sv, si);
  if (!(dmax > a.tol)) {   // converged (or nothing left): rank = k
    if (blockIdx.x == 0 && t == 0) {
      a.state->done = 1;
      a.state->rank = k;
      a.state->dmax = dmax;
    }
    return;
  }
  int64_t pm, pn;
  pair_of(p, pm, pn);
  const int64_t poff = pm * nao + pn;
  const double m_pi = owner ? a.M[p * N + i] : 0.0;   // issued beside the pivot-row staging
  double acc = 0.0;
  for (int64_t c0 = 0; c0 < k; c0 += kCdLp) {
    const int cn = (int)((k - c0) < kCdLp ? (k - c0) : kCdLp);
    __syncthreads();
    for (int j = t; j < cn; j += T) lp[j] = a.B[(c0 + j) * nao2 + poff];
    __syncthreads();
    if (valid) {
      // rounds of kCdU loads, the last one predicated (no serial tail)
      const double *Lc = a.B + c0 * nao2 + ioff;
      for (int j = g; j < cn; j += kCdU * G) {
        double x[kCdU], w[kCdU];
        const bool first = c0 == 0 && j == g;
#pragma unroll
        for (int u = 0; u < kCdU; ++u) {
          const int jj = j + u * G;
          x[u] = first ? x0[u] : (jj < cn ? Lc[(int64_t)jj * nao2] : 0.0);
          w[u] = jj < cn ? lp[jj] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kCdU; ++u) acc = fma(x[u], w[u], acc);
      }
    }
  }
  __syncthreads();
  sv[t] = acc;
  __syncthreads();
  double cand = -INFINITY;
  int64_t ci = INT64_MAX;
  if (owner) {
    double sum = 0.0;
    for (int q = 0; q < G; ++q) sum += sv[r + q * R];
    const double col = (m_pi - sum) / sqrt(dmax);
    double *Bk = a.B + k * nao2;
    Bk[mu * nao + nu] = col;
    Bk[nu * nao + mu] = col;
    const double dn = (i == p) ? 0.0 : sub_square(d_i, col);
    a.d[i] = dn;
    cand = dn;
    ci = i;
  }
  if (blockIdx.x == 0 && t == 0 && a.pivots) a.pivots[k] = p;
  publish<T>(a, (int)((k + 1) & 1), cand, ci, sv, si);
}

// rank and final residual maximum (one workgroup, after the last step)
__global__ __launch_bounds__(kCdT) void cd_finish_kernel(CdArgs a, int64_t max_rank,
                                                         int64_t nlast, int64_t *rank,
                                                         double *dmax) {
  __shared__ double sv[kCdT];
  __shared__ int64_t si[kCdT];
  if (a.state->done) {
    if (threadIdx.x == 0) {
      *rank = a.state->rank;
      *dmax = a.state->dmax;
    }
    return;
  }
  double v;
  int64_t i;
  reduce_published<kCdT>(a, (int)(max_rank & 1), nlast, v, i, sv, si);
  if (threadIdx.x == 0) {
    *rank = max_rank;
    *dmax = v;
  }
}

}  // namespace

int cd_rows_per_block(int64_t npair) {
  // few, wide workgroups: the fixed cost of a step (the reduction of the
  // published maxima, the pivot-row staging) grows with their number
  return npair >= 64 * 64 ? 64 : 16;
}

int cd_threads_per_block(int64_t npair) {
  (void)npair;
  return 256;
}

hipError_t launch_cholesky(const CdPlan &pl, const double *M, double *B, int64_t *rank,
                           double *dmax, int64_t *pivots, void *ws, hipStream_t st) {
  hipError_t e;
  CdArgs a;
  a.M = M;
  a.B = B;
  a.d = ws_d(ws, pl.off_d);
  a.part_v = ws_d(ws, pl.off_pv);
  a.part_i = reinterpret_cast<int64_t *>(static_cast<char *>(ws) + pl.off_pi);
  a.state = reinterpret_cast<CdState *>(static_cast<char *>(ws) + pl.off_state);
  a.pivots = pivots;
  a.nao = pl.nao;
  a.npair = pl.npair;
  a.pstride = pl.pstride;
  a.tol = pl.tol;
  // vectors past the rank stay zero; the done flag cleared
  timer_begin("cd_init", st);
  if ((e = launch_zero_fill(B, pl.max_rank * pl.nao * pl.nao, st)) != hipSuccess) return e;
  if ((e = launch_zero_fill(reinterpret_cast<double *>(a.state),
                            (int64_t)(sizeof(CdState) / sizeof(double)), st)) != hipSuccess)
    return e;
  const int64_t ninit = ceil_div(pl.npair, kCdT);
  hipLaunchKernelGGL(cd_init_kernel, dim3((unsigned)ninit), dim3(kCdT), 0, st, a);
  timer_end(st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int R = cd_rows_per_block(pl.npair), T = cd_threads_per_block(pl.npair);
  const int64_t nblk = ceil_div(pl.npair, R);
  const dim3 grid((unsigned)nblk);
  auto step = [&](int64_t k, int64_t nprev) {
    if (R == 128)
      hipLaunchKernelGGL((cd_step_kernel<128, 256>), grid, dim3(T), 0, st, a, k, nprev);
    else if (R == 64 && T == 512)
      hipLaunchKernelGGL((cd_step_kernel<64, 512>), grid, dim3(T), 0, st, a, k, nprev);
    else if (R == 64)
      hipLaunchKernelGGL((cd_step_kernel<64, 256>), grid, dim3(T), 0, st, a, k, nprev);
    else if (R == 32)
      hipLaunchKernelGGL((cd_step_kernel<32, 256>), grid, dim3(T), 0, st, a, k, nprev);
    else
      hipLaunchKernelGGL((cd_step_kernel<16, 256>), grid, dim3(T), 0, st, a, k, nprev);
  };
  timer_begin("cd_step", st);
  for (int64_t k = 0; k < pl.max_rank; ++k) {
    step(k, k == 0 ? ninit : nblk);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  timer_end(st);
  hipLaunchKernelGGL(cd_finish_kernel, dim3(1), dim3(kCdT), 0, st, a, pl.max_rank,
                     pl.max_rank == 0 ? ninit : nblk, rank, dmax);
  return hipGetLastError();
}

}  // namespace dsrg
