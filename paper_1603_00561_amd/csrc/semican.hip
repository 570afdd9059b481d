// Semicanonical orbitals (section II.B): the rotation U that diagonalizes
// the core, active and virtual diagonal blocks of the generalized Fock matrix,
// the orbital energies eps on the diagonal of U^T F U, and the rotated
// coefficients C U. Frozen core orbitals keep U = I and their diagonal of F.
//
// Each block is diagonalized by two-sided block Jacobi (gfx950, FP64): the
// block, zero-padded to a multiple of 64, is cut into 32-wide blocks; a sweep
// runs the circle-method rounds over those blocks, and a round (i) solves
// every disjoint pair of blocks approximately, as one parallel Jacobi sweep
// over its 64 x 64 submatrix in LDS (one workgroup per pair, 32 disjoint
// rotations at a time), and (ii) applies each pair's 64 x 64 rotation to the
// pair's columns of the whole matrix and of the eigenvector matrix, then to
// the pair's rows. Padded rows and columns never couple (their off-diagonal
// entries stay exactly zero), so they keep their unit eigenvectors. After
// each sweep the off-diagonal norm is compared with the whole norm (partial
// sums over 64 workgroups, added in order) and a device flag is set when
// their ratio is below 1e-15; the launches of the
// remaining sweeps (at most kMaxSweeps in all) then return at once, so
// nothing waits on the host. Blocks of at most 64 orbitals are solved in one
// workgroup with inner sweeps repeated to the same criterion. The eigenvalues
// are finally ranked (ascending) and each eigenvector signed so that its
// component of largest magnitude is positive.
#include <algorithm>

#include "common_device.h"
#include "internal.h"

namespace dsrg {

constexpr int kJB = 32;             // Jacobi block width
constexpr int kJP = 2 * kJB;        // pair submatrix order
constexpr int kJP1 = kJP + 1;       // LDS row pitch
constexpr int kJT = 256;            // threads per workgroup
constexpr int kMaxSweeps = 15;      // block Jacobi sweeps at most
constexpr int kSmallSweeps = 40;    // inner sweeps at most for blocks of <= 64
constexpr double kJacTol2 = 1e-30;  // (off-diagonal / whole)^2 at convergence

// pair k of round r of the circle method over np (even) players
__device__ __forceinline__ void circle_pair(int np, int r, int k, int &i, int &j) {
  const int m = np - 1;
  if (k == 0) {
    i = r % m;
    j = m;
  } else {
    i = (r + k) % m;
    j = (r - k + m) % m;
  }
}

// rotation (c, s) in the (p, q) plane that zeroes the (p, q) entry of a
// symmetric matrix under S -> J^T S J, J = [[c, s], [-s, c]] on (p, q)
__device__ __forceinline__ void jac_rot(double spp, double sqq, double spq, double &c,
                                        double &s) {
  if (spq == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double tau = (sqq - spp) / (2.0 * spq);
  const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

struct JacLds {
  double S[kJP][kJP1];
  double Q[kJP][kJP1];
  double c[kJP / 2], s[kJP / 2];
  int p[kJP / 2], q[kJP / 2];
  double red[kJT];
};

// one parallel Jacobi sweep over the 64 x 64 symmetric S, the rotations
// accumulated into Q (Q <- Q J)
__device__ void jac_inner_sweep(JacLds &L) {
  const int t = threadIdx.x;
  for (int ri = 0; ri < kJP - 1; ++ri) {
    if (t < kJP / 2) {
      int p, q;
      circle_pair(kJP, ri, t, p, q);
      double c, s;
      jac_rot(L.S[p][p], L.S[q][q], L.S[p][q], c, s);
      L.p[t] = p;
      L.q[t] = q;
      L.c[t] = c;
      L.s[t] = s;
    }
    __syncthreads();
    // columns of S and of Q
    for (int e = t; e < 2 * (kJP / 2) * kJP; e += kJT) {
      const int k = (e / kJP) % (kJP / 2), a = e % kJP;
      double(*M)[kJP1] = (e < (kJP / 2) * kJP) ? L.S : L.Q;
      const int p = L.p[k], q = L.q[k];
      const double c = L.c[k], s = L.s[k];
      const double x = M[a][p], y = M[a][q];
      M[a][p] = c * x - s * y;
      M[a][q] = s * x + c * y;
    }
    __syncthreads();
    // rows of S
    for (int e = t; e < (kJP / 2) * kJP; e += kJT) {
      const int k = e / kJP, b = e % kJP;
      const int p = L.p[k], q = L.q[k];
      const double c = L.c[k], s = L.s[k];
      const double x = L.S[p][b], y = L.S[q][b];
      L.S[p][b] = c * x - s * y;
      L.S[q][b] = s * x + c * y;
    }
    __syncthreads();
  }
}

// A [npad][npad] = the n x n block of F at (o, o), zero-padded; V = I
__global__ __launch_bounds__(256) void jac_load_kernel(const double *__restrict__ F, int64_t nmo,
                                                       int64_t o, int64_t n, int64_t npad,
                                                       double *__restrict__ A,
                                                       double *__restrict__ V) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < npad * npad;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / npad, j = e % npad;
    A[e] = (i < n && j < n) ? F[(o + i) * nmo + o + j] : 0.0;
    V[e] = (i == j) ? 1.0 : 0.0;
  }
}

__global__ void jac_reset_kernel(int *done) {
  if (threadIdx.x == 0) *done = 0;
}

// global index of row a (0..63) of the pair (I, J)
__device__ __forceinline__ int64_t pair_index(int I, int J, int a) {
  return a < kJB ? (int64_t)I * kJB + a : (int64_t)J * kJB + (a - kJB);
}

// one workgroup per pair of round r: one inner sweep on the pair's submatrix,
// the accumulated 64 x 64 rotation written to Qout[pair]
__global__ __launch_bounds__(kJT) void jac_pair_kernel(const double *__restrict__ A, int64_t npad,
                                                       int nb, int r, double *__restrict__ Qout,
                                                       const int *__restrict__ done) {
  if (*done) return;
  __shared__ JacLds L;
  int I, J;
  circle_pair(nb, r, blockIdx.x, I, J);
  const int t = threadIdx.x;
  for (int e = t; e < kJP * kJP; e += kJT) {
    const int a = e / kJP, b = e % kJP;
    L.S[a][b] = A[pair_index(I, J, a) * npad + pair_index(I, J, b)];
    L.Q[a][b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  jac_inner_sweep(L);
  double *Qo = Qout + (int64_t)blockIdx.x * kJP * kJP;
  for (int e = t; e < kJP * kJP; e += kJT) Qo[e] = L.Q[e / kJP][e % kJP];
}

// columns of the pairs of round r: M[:, pair] <- M[:, pair] Q for M = A
// (blockIdx.z = 0) and M = V (1); one workgroup per 64-row tile and pair
__global__ __launch_bounds__(kJT) void jac_cols_kernel(double *__restrict__ A,
                                                       double *__restrict__ V, int64_t npad,
                                                       int nb, int r, const double *__restrict__ Qall,
                                                       const int *__restrict__ done) {
  if (*done) return;
  __shared__ double X[kJP][kJP1], Qs[kJP][kJP1];
  int I, J;
  circle_pair(nb, r, blockIdx.y, I, J);
  double *M = blockIdx.z ? V : A;
  const int64_t r0 = (int64_t)blockIdx.x * kJP;
  const double *Qp = Qall + (int64_t)blockIdx.y * kJP * kJP;
  const int t = threadIdx.x;
  for (int e = t; e < kJP * kJP; e += kJT) {
    const int a = e / kJP, b = e % kJP;
    X[a][b] = M[(r0 + a) * npad + pair_index(I, J, b)];
    Qs[a][b] = Qp[e];
  }
  __syncthreads();
  // X and Qs live in LDS and the results go to global memory, so each
  // result is stored as soon as it is formed
  for (int j = 0; j < kJP * kJP / kJT; ++j) {
    const int e = t + kJT * j, a = e / kJP, c = e % kJP;
    double v = 0.0;
#pragma unroll 16
    for (int b = 0; b < kJP; ++b) v = fma(X[a][b], Qs[b][c], v);
    M[(r0 + a) * npad + pair_index(I, J, c)] = v;
  }
}

// rows of the pairs of round r: A[pair, :] <- Q^T A[pair, :]; one workgroup
// per 64-column tile and pair
__global__ __launch_bounds__(kJT) void jac_rows_kernel(double *__restrict__ A, int64_t npad,
                                                       int nb, int r, const double *__restrict__ Qall,
                                                       const int *__restrict__ done) {
  if (*done) return;
  __shared__ double X[kJP][kJP1], Qs[kJP][kJP1];
  int I, J;
  circle_pair(nb, r, blockIdx.y, I, J);
  const int64_t c0 = (int64_t)blockIdx.x * kJP;
  const double *Qp = Qall + (int64_t)blockIdx.y * kJP * kJP;
  const int t = threadIdx.x;
  for (int e = t; e < kJP * kJP; e += kJT) {
    const int a = e / kJP, b = e % kJP;
    X[a][b] = A[pair_index(I, J, a) * npad + c0 + b];
    Qs[a][b] = Qp[e];
  }
  __syncthreads();
  for (int j = 0; j < kJP * kJP / kJT; ++j) {
    const int e = t + kJT * j, a = e / kJP, c = e % kJP;
    double v = 0.0;
#pragma unroll 16
    for (int b = 0; b < kJP; ++b) v = fma(Qs[b][a], X[b][c], v);
    A[pair_index(I, J, a) * npad + c0 + c] = v;
  }
}

// fixed-order sum over the workgroup (kJT threads)
__device__ double jac_block_sum(double v, double *red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int w = kJT / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

// convergence check, in two launches: kJacParts workgroups each sum the
// squared off-diagonal and all squared entries of a strided share of the rows
// into part[2 * wg]; one workgroup adds the partial sums in order and sets
// done = (off <= tol2 * all)
constexpr int kJacParts = (int)kSemicanParts;

__global__ __launch_bounds__(kJT) void jac_check_part_kernel(const double *__restrict__ A,
                                                             int64_t npad,
                                                             double *__restrict__ part,
                                                             const int *__restrict__ done) {
  if (*done) return;
  __shared__ double red[kJT];
  double off = 0.0, tot = 0.0;
  for (int64_t i = blockIdx.x; i < npad; i += kJacParts)
    for (int64_t j = threadIdx.x; j < npad; j += kJT) {
      const double v = A[i * npad + j] * A[i * npad + j];
      tot += v;
      if (i != j) off += v;
    }
  off = jac_block_sum(off, red);
  tot = jac_block_sum(tot, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = off;
    part[2 * blockIdx.x + 1] = tot;
  }
}

__global__ void jac_check_final_kernel(const double *__restrict__ part, int *__restrict__ done) {
  if (threadIdx.x != 0 || *done) return;
  double off = 0.0, tot = 0.0;
  for (int k = 0; k < kJacParts; ++k) {
    off += part[2 * k];
    tot += part[2 * k + 1];
  }
  if (off <= kJacTol2 * tot) *done = 1;
}

// blocks of at most 64 (npad == 64): inner sweeps in one workgroup until the
// same criterion holds (at most kSmallSweeps), then A and V written back
__global__ __launch_bounds__(kJT) void jac_small_kernel(double *__restrict__ A,
                                                        double *__restrict__ V) {
  __shared__ JacLds L;
  const int t = threadIdx.x;
  for (int e = t; e < kJP * kJP; e += kJT) {
    L.S[e / kJP][e % kJP] = A[e];
    L.Q[e / kJP][e % kJP] = (e / kJP == e % kJP) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sw = 0; sw < kSmallSweeps; ++sw) {
    double off = 0.0, tot = 0.0;
    for (int e = t; e < kJP * kJP; e += kJT) {
      const double v = L.S[e / kJP][e % kJP] * L.S[e / kJP][e % kJP];
      tot += v;
      if (e / kJP != e % kJP) off += v;
    }
    off = jac_block_sum(off, L.red);
    tot = jac_block_sum(tot, L.red);
    if (off <= kJacTol2 * tot) break;   // the same value in every thread
    jac_inner_sweep(L);
  }
  for (int e = t; e < kJP * kJP; e += kJT) {
    A[e] = L.S[e / kJP][e % kJP];
    V[e] = L.Q[e / kJP][e % kJP];
  }
}

// U = 0 with the frozen block the identity; eps = diag(F) (the rotated blocks
// are overwritten later)
__global__ __launch_bounds__(256) void semican_init_kernel(const double *__restrict__ F,
                                                           int64_t nmo, int64_t nfrz,
                                                           double *__restrict__ U,
                                                           double *__restrict__ eps) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nmo * nmo;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / nmo, j = e % nmo;
    U[e] = (i == j && i < nfrz) ? 1.0 : 0.0;
    if (i == j) eps[i] = F[e];
  }
}

// eigenvalue i goes to position rank(i) of the block (ascending, ties by
// index); its eigenvector, signed so that its largest component (the first
// such) is positive, to column o + rank(i) of U
__global__ __launch_bounds__(256) void jac_finalize_kernel(const double *__restrict__ A,
                                                           const double *__restrict__ V,
                                                           int64_t npad, int64_t n, int64_t o,
                                                           int64_t nmo, double *__restrict__ U,
                                                           double *__restrict__ eps) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const double lam = A[i * npad + i];
    int64_t rank = 0;
    for (int64_t j = 0; j < n; ++j) {
      const double mu = A[j * npad + j];
      rank += (mu < lam || (mu == lam && j < i)) ? 1 : 0;
    }
    double best = -1.0, sg = 1.0;
    for (int64_t r = 0; r < n; ++r) {
      const double v = V[r * npad + i];
      if (fabs(v) > best) {
        best = fabs(v);
        sg = v < 0.0 ? -1.0 : 1.0;
      }
    }
    eps[o + rank] = lam;
    for (int64_t r = 0; r < n; ++r) U[(o + r) * nmo + o + rank] = sg * V[r * npad + i];
  }
}

int64_t semican_npad(int64_t n) { return std::max<int64_t>(kJP, round_up(n, kJP)); }

hipError_t launch_semican(const SemicanPlan &pl, const double *F, const double *C, double *U,
                          double *eps, double *Cs, void *ws, hipStream_t st) {
  hipError_t e;
  const int64_t nmo = pl.nmo;
  double *A = ws_d(ws, pl.off_a), *V = ws_d(ws, pl.off_v), *Qb = ws_d(ws, pl.off_q);
  double *Pt = ws_d(ws, pl.off_part);
  int *done = reinterpret_cast<int *>(static_cast<char *>(ws) + pl.off_flag);
  hipLaunchKernelGGL(semican_init_kernel,
                     dim3((unsigned)std::min<int64_t>(ceil_div(nmo * nmo, 256), 4096)), dim3(256),
                     0, st, F, nmo, pl.nfrz, U, eps);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const char *names[3] = {"semican_core", "semican_active", "semican_virtual"};
  const int64_t sizes[3] = {pl.nc, pl.na, pl.nv};
  int64_t o = pl.nfrz;
  for (int b = 0; b < 3; ++b) {
    const int64_t n = sizes[b];
    if (n == 0) continue;
    const int64_t npad = semican_npad(n);
    const int nb = (int)(npad / kJB);
    timer_begin(names[b], st);
    hipLaunchKernelGGL(jac_load_kernel,
                       dim3((unsigned)std::min<int64_t>(ceil_div(npad * npad, 256), 4096)),
                       dim3(256), 0, st, F, nmo, o, n, npad, A, V);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (npad == kJP) {
      hipLaunchKernelGGL(jac_small_kernel, dim3(1), dim3(kJT), 0, st, A, V);
    } else {
      hipLaunchKernelGGL(jac_reset_kernel, dim3(1), dim3(64), 0, st, done);
      const int npairs = nb / 2;
      const unsigned tiles = (unsigned)(npad / kJP);
      for (int sw = 0; sw < kMaxSweeps; ++sw) {
        for (int r = 0; r < nb - 1; ++r) {
          hipLaunchKernelGGL(jac_pair_kernel, dim3(npairs), dim3(kJT), 0, st, A, npad, nb, r, Qb,
                             done);
          hipLaunchKernelGGL(jac_cols_kernel, dim3(tiles, npairs, 2), dim3(kJT), 0, st, A, V,
                             npad, nb, r, Qb, done);
          hipLaunchKernelGGL(jac_rows_kernel, dim3(tiles, npairs), dim3(kJT), 0, st, A, npad, nb,
                             r, Qb, done);
        }
        hipLaunchKernelGGL(jac_check_part_kernel, dim3(kJacParts), dim3(kJT), 0, st, A, npad,
                           Pt, done);
        hipLaunchKernelGGL(jac_check_final_kernel, dim3(1), dim3(64), 0, st, Pt, done);
      }
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(jac_finalize_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, A,
                       V, npad, n, o, nmo, U, eps);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    timer_end(st);
    o += n;
  }
  if (C && Cs) {
    timer_begin("semican_rotate", st);
    e = gemm_f64(false, false, pl.nao, nmo, nmo, 1.0, C, nmo, U, nmo, 0.0, Cs, nmo, st);
    timer_end(st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace dsrg
