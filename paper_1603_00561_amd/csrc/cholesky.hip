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
// waves of a workgroup. The argmax of the updated diagonal is reduced in the
// same launch: every workgroup publishes its local maximum, and the last
// workgroup to arrive (an atomic ticket, no waiting) reduces them and leaves
// the next pivot for the following launch. Launches past convergence return
// at once (a done flag in the workspace). Every sum runs in a fixed order, so
// results repeat bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace dsrg {

namespace {

constexpr int kCdT = 256;     // threads per workgroup
constexpr int kCdLp = 2048;   // pivot-row values of the earlier vectors staged per LDS chunk

struct CdArgs {
  const double *M;   // [N][N] integrals over packed pairs
  double *B;         // [max_rank][nao][nao] vectors, unpacked
  double *d;         // [N] residual diagonal
  double *part_v;    // [nblk] per-workgroup maxima of d
  int64_t *part_i;   // [nblk] their pair indices
  CdSel *sel;        // [2] pivot for the next step, by step parity
  CdState *state;
  int64_t *pivots;   // [max_rank] or nullptr
  int64_t nao, npair;
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

// Workgroup argmax of (v, i) over all threads into thread 0's return value.
__device__ inline void block_argmax(double &v, int64_t &i, double *sv, int64_t *si) {
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = i;
  __syncthreads();
  for (int h = kCdT / 2; h > 0; h >>= 1) {
    if (t < h && beats(sv[t + h], si[t + h], sv[t], si[t])) {
      sv[t] = sv[t + h];
      si[t] = si[t + h];
    }
    __syncthreads();
  }
  v = sv[0];
  i = si[0];
}

// Publish this workgroup's maximum; the last workgroup of the launch to
// arrive reduces all of them (in index order of the workgroups, so the
// result does not depend on arrival order) into sel_out and rearms the
// ticket. Called by every thread of every workgroup.
__device__ void publish_max(const CdArgs &a, double v, int64_t i, CdSel *sel_out, double *sv,
                            int64_t *si) {
  __shared__ int s_last;
  const int t = threadIdx.x;
  const unsigned nblk = gridDim.x;
  block_argmax(v, i, sv, si);
  if (t == 0) {
    a.part_v[blockIdx.x] = v;
    a.part_i[blockIdx.x] = i;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned ticket =
        __hip_atomic_fetch_add(&a.state->ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (ticket == nblk - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  double bv = -INFINITY;
  int64_t bi = INT64_MAX;
  for (unsigned b = t; b < nblk; b += kCdT) {
    const double w = a.part_v[b];
    const int64_t j = a.part_i[b];
    if (beats(w, j, bv, bi)) {
      bv = w;
      bi = j;
    }
  }
  __syncthreads();
  block_argmax(bv, bi, sv, si);
  if (t == 0) {
    sel_out->dmax = bv;
    sel_out->p = bi;
    a.state->ticket = 0;
  }
}

// d = diag(M) and the first pivot; one thread per pair
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
  publish_max(a, v, vi, &a.sel[0], sv, si);
}

// Cholesky vector k: R pair rows per workgroup, 256 / R groups of earlier
// vectors per row
template <int R>
__global__ __launch_bounds__(kCdT) void cd_step_kernel(CdArgs a, int64_t k) {
  constexpr int G = kCdT / R;
  __shared__ double lp[kCdLp];
  __shared__ double sv[kCdT];
  __shared__ int64_t si[kCdT];
  if (a.state->done) return;
  const CdSel s = a.sel[k & 1];
  if (!(s.dmax > a.tol)) {   // converged (or nothing left): rank = k
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.state->done = 1;
      a.state->rank = k;
      a.state->dmax = s.dmax;
    }
    return;
  }
  const int64_t nao = a.nao, nao2 = a.nao * a.nao, N = a.npair;
  const int64_t p = s.p;
  int64_t pm, pn;
  pair_of(p, pm, pn);
  const int64_t poff = pm * nao + pn;
  const int t = threadIdx.x, r = t % R, g = t / R;
  const int64_t i = (int64_t)blockIdx.x * R + r;
  const bool valid = i < N;
  int64_t mu = 0, nu = 0;
  if (valid) pair_of(i, mu, nu);
  const int64_t ioff = mu * nao + nu;
  double acc = 0.0;
  for (int64_t c0 = 0; c0 < k; c0 += kCdLp) {
    const int cn = (int)((k - c0) < kCdLp ? (k - c0) : kCdLp);
    __syncthreads();
    for (int j = t; j < cn; j += kCdT) lp[j] = a.B[(c0 + j) * nao2 + poff];
    __syncthreads();
    if (valid) {
      const double *Lc = a.B + c0 * nao2 + ioff;
      int j = g;
      for (; j + 3 * G < cn; j += 4 * G) {
        const double x0 = Lc[(int64_t)j * nao2];
        const double x1 = Lc[(int64_t)(j + G) * nao2];
        const double x2 = Lc[(int64_t)(j + 2 * G) * nao2];
        const double x3 = Lc[(int64_t)(j + 3 * G) * nao2];
        acc = fma(x0, lp[j], acc);
        acc = fma(x1, lp[j + G], acc);
        acc = fma(x2, lp[j + 2 * G], acc);
        acc = fma(x3, lp[j + 3 * G], acc);
      }
      for (; j < cn; j += G) acc = fma(Lc[(int64_t)j * nao2], lp[j], acc);
    }
  }
  __syncthreads();
  sv[t] = acc;
  __syncthreads();
  double cand = -INFINITY;
  int64_t ci = INT64_MAX;
  if (g == 0 && valid) {
    double sum = 0.0;
    for (int q = 0; q < G; ++q) sum += sv[r + q * R];
    const double col = (a.M[p * N + i] - sum) / sqrt(s.dmax);
    double *Bk = a.B + k * nao2;
    Bk[mu * nao + nu] = col;
    Bk[nu * nao + mu] = col;
    const double dn = (i == p) ? 0.0 : sub_square(a.d[i], col);
    a.d[i] = dn;
    cand = dn;
    ci = i;
  }
  if (blockIdx.x == 0 && t == 0 && a.pivots) a.pivots[k] = p;
  __syncthreads();
  publish_max(a, cand, ci, &a.sel[(k + 1) & 1], sv, si);
}

// rank and final residual maximum (a single thread, after the last step)
__global__ void cd_finish_kernel(CdArgs a, int64_t max_rank, int64_t *rank, double *dmax) {
  if (a.state->done) {
    *rank = a.state->rank;
    *dmax = a.state->dmax;
  } else {
    *rank = max_rank;
    *dmax = a.sel[max_rank & 1].dmax;
  }
}

}  // namespace

int cd_rows_per_block(int64_t npair) {
  // the most pair rows per workgroup that still leave about 512 workgroups
  if (ceil_div(npair, 64) >= 512) return 64;
  if (ceil_div(npair, 32) >= 512) return 32;
  return 16;
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
  a.sel = reinterpret_cast<CdSel *>(static_cast<char *>(ws) + pl.off_sel);
  a.state = reinterpret_cast<CdState *>(static_cast<char *>(ws) + pl.off_state);
  a.pivots = pivots;
  a.nao = pl.nao;
  a.npair = pl.npair;
  a.tol = pl.tol;
  // vectors past the rank stay zero; ticket, done flag and selection cleared
  timer_begin("cd_init", st);
  if ((e = launch_zero_fill(B, pl.max_rank * pl.nao * pl.nao, st)) != hipSuccess) return e;
  if ((e = launch_zero_fill(reinterpret_cast<double *>(a.sel),
                            (int64_t)((pl.off_end - pl.off_sel) / sizeof(double)), st)) !=
      hipSuccess)
    return e;
  hipLaunchKernelGGL(cd_init_kernel, dim3((unsigned)ceil_div(pl.npair, kCdT)), dim3(kCdT), 0, st,
                     a);
  timer_end(st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int R = cd_rows_per_block(pl.npair);
  const dim3 grid((unsigned)ceil_div(pl.npair, R));
  timer_begin("cd_step", st);
  for (int64_t k = 0; k < pl.max_rank; ++k) {
    if (R == 64)
      hipLaunchKernelGGL(cd_step_kernel<64>, grid, dim3(kCdT), 0, st, a, k);
    else if (R == 32)
      hipLaunchKernelGGL(cd_step_kernel<32>, grid, dim3(kCdT), 0, st, a, k);
    else
      hipLaunchKernelGGL(cd_step_kernel<16>, grid, dim3(kCdT), 0, st, a, k);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  timer_end(st);
  hipLaunchKernelGGL(cd_finish_kernel, dim3(1), dim3(1), 0, st, a, pl.max_rank, rank, dmax);
  return hipGetLastError();
}

}  // namespace dsrg
