// Semicanonical orbitals (section II.B): the rotation U that diagonalizes
// the core, active and virtual diagonal blocks of the generalized Fock matrix,
// the orbital energies eps on the diagonal of U^T F U, and the rotated
// coefficients C U. Frozen core orbitals keep U = I and their diagonal of F.
//
// Each block is diagonalized by two-sided block Jacobi (gfx950, FP64): the
// block, zero-padded to a multiple of 32, is cut into 16-wide blocks; a sweep
// runs the circle-method rounds over those blocks, and a round (i) solves
// every disjoint pair of blocks approximately, as one parallel Jacobi sweep
// over its 32 x 32 submatrix in LDS (one workgroup per pair, 16 disjoint
// rotations at a time, each thread taking one 2 x 2 block through both
// sides), and (ii) forms
// every block of the new matrix as Q_P^T A_PP' Q_P' from the old one (a second
// buffer, so the update is fully parallel) and rotates the pair's columns of
// the eigenvector matrix, both in one launch. Padded rows and columns never couple (their off-diagonal
// entries stay exactly zero), so they keep their unit eigenvectors. After
// each sweep the off-diagonal norm is compared with the whole norm (partial
// sums over 64 workgroups, added in order) and a device flag is set when
// their ratio is below 1e-14, recording which of the two matrix buffers holds
// the converged matrix; the launches of the remaining sweeps (at most
// kMaxSweeps in all: spectra with large exactly degenerate multiplets converge
// only linearly, about 20-25 sweeps at 150-380 orbitals) then return at once,
// so nothing waits on the host, and
// the final ordering reads the buffer the flag names. Blocks of at most
// 32 orbitals are solved in one
// workgroup with inner sweeps repeated to the same criterion. The eigenvalues
// are finally ranked (ascending) and each eigenvector signed so that its
// component of largest magnitude is positive.
#include <algorithm>

#include "common_device.h"
#include "internal.h"

namespace dsrg {

constexpr int kJB = 16;             // Jacobi block width
constexpr int kJP = 2 * kJB;        // pair submatrix order
constexpr int kJP1 = kJP + 1;       // LDS row pitch
constexpr int kJT = 256;            // threads per workgroup
constexpr int kMaxSweeps = 40;      // block Jacobi sweeps at most (degenerate spectra need ~25)
constexpr int kSmallSweeps = 40;    // inner sweeps at most for blocks of <= kJP
constexpr double kJacTol2 = 1e-28;  // (off-diagonal / whole)^2 at convergence

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
// symmetric matrix under S -> J^T S J, J = [[c, s], [-s, c]] on (p, q): the
// smaller of the two angles, tan = sgn |e| / (|d| + r) with d = s_qq - s_pp,
// e = 2 s_pq, r = sqrt(d^2 + e^2) and sgn the sign of d e.
// Since (|d| + r)^2 + e^2 = 2 r (|d| + r), both c = (|d| + r) w and
// |s| = |e| w follow from w = 1 / sqrt(2 r (|d| + r)): two inverse square
// roots and no division on the dependent chain. The rotation does not change
// when d and e are scaled by one factor, so both are first scaled by a power
// of two to bring the larger into [1/2, 1) and d^2 + e^2 into [1/4, 2).
// Branch-free, so that a thread's two rotations are scheduled together.
__device__ __forceinline__ void jac_rot(double spp, double sqq, double spq, double &c,
                                        double &s) {
  const double d0 = sqq - spp, e0 = 2.0 * spq;
  int k;
  (void)frexp(fmax(fabs(d0), fabs(e0)), &k);
  const double d = ldexp(d0, -k), e = ldexp(e0, -k);
  const double q2 = d * d + e * e;
  const double r = q2 * rsqrt(q2);
  const double u = fabs(d) + r;
  const double w = rsqrt(2.0 * r * u);
  const double se = copysign(fabs(e), d * e);   // sgn |e| (d = 0: either sign zeroes the entry)
  const bool zero = (spq == 0.0);
  c = zero ? 1.0 : u * w;
  s = zero ? 0.0 : se * w;
}

struct JacLds {
  double S[2][kJP][kJP1];   // submatrix, read from one buffer and written to the other
  double Q[kJP][kJP1];      // accumulated rotation
  double red[kJT];
};

// one parallel Jacobi sweep over the symmetric submatrix in S[cur],
// accumulating Q <- Q J; returns the buffer that holds the rotated matrix. In
// a round the kJP / 2 disjoint rotations split the indices into pairs, so the
// 2 x 2 blocks {p_a, q_a} x {p_b, q_b} partition S: thread (a, b) forms the
// rotations a and b itself from the diagonal and pivot entries of the
// current buffer, takes block (a, b) through J_a^T (.) J_b into the other
// buffer, and the rows a, a + kJP / 2 of Q at columns p_b, q_b (which no
// other thread touches in this round) through J_b in place. One barrier per
// round: nothing a thread writes is read by another thread before it.
__device__ int jac_inner_sweep(JacLds &L, int cur) {
  const int t = threadIdx.x;
  static_assert((kJP / 2) * (kJP / 2) == kJT, "one 2 x 2 block of S per thread");
  const int ka = t / (kJP / 2), kb = t % (kJP / 2);
#pragma unroll 1   // a rolled loop keeps the kernel within the instruction cache
  for (int ri = 0; ri < kJP - 1; ++ri) {
    const double (*S)[kJP1] = L.S[cur];
    double (*T)[kJP1] = L.S[cur ^ 1];
    int pa, qa, pb, qb;
    circle_pair(kJP, ri, ka, pa, qa);
    circle_pair(kJP, ri, kb, pb, qb);
    const double m00 = S[pa][pb], m01 = S[pa][qb], m10 = S[qa][pb], m11 = S[qa][qb];
    double ca, sa, cb, sb;   // two independent chains
    jac_rot(S[pa][pa], S[qa][qa], S[pa][qa], ca, sa);
    jac_rot(S[pb][pb], S[qb][qb], S[pb][qb], cb, sb);
    // rows: new p = c p - s q, new q = s p + c q
    const double t00 = ca * m00 - sa * m10, t01 = ca * m01 - sa * m11;
    const double t10 = sa * m00 + ca * m10, t11 = sa * m01 + ca * m11;
    // columns likewise
    T[pa][pb] = t00 * cb - t01 * sb;
    T[pa][qb] = t00 * sb + t01 * cb;
    T[qa][pb] = t10 * cb - t11 * sb;
    T[qa][qb] = t10 * sb + t11 * cb;
#pragma unroll
    for (int a = ka; a < kJP; a += kJP / 2) {
      const double x = L.Q[a][pb], y = L.Q[a][qb];
      L.Q[a][pb] = cb * x - sb * y;
      L.Q[a][qb] = sb * x + cb * y;
    }
    __syncthreads();
    cur ^= 1;
  }
  return cur;
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

// convergence status: info = 0 before the first block (a kernel, not a
// memset, so the call can be captured in a graph)
__global__ void jac_info_clear_kernel(int *info) {
  if (threadIdx.x == 0) *info = 0;
}

// after the sweeps of a block: its bit of info set when the criterion was
// never met (the flag is still clear)
__global__ void jac_info_kernel(const int *__restrict__ done, int *__restrict__ info, int bit) {
  if (threadIdx.x == 0 && *done == 0) atomicOr(info, bit);
}

// global index of row a (0..kJP-1) of the pair (I, J)
__device__ __forceinline__ int64_t pair_index(int I, int J, int a) {
  return a < kJB ? (int64_t)I * kJB + a : (int64_t)J * kJB + (a - kJB);
}

// one workgroup per pair of round r: one inner sweep on the pair's submatrix,
// the accumulated kJP x kJP rotation written to Qout[pair]
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
    L.S[0][a][b] = A[pair_index(I, J, a) * npad + pair_index(I, J, b)];
    L.Q[a][b] = (a == b) ? 1.0 : 0.0;
  }
  __syncthreads();
  (void)jac_inner_sweep(L, 0);
  double *Qo = Qout + (int64_t)blockIdx.x * kJP * kJP;
  for (int e = t; e < kJP * kJP; e += kJT) Qo[e] = L.Q[e / kJP][e % kJP];
}

// one launch per round for both updates: workgroups (x, y < npairs) form
// Anew[P, P'] = Q_P^T Aold[P, P'] Q_P' for the pairs P = x, P' = y of round r
// (the pairs cover every block, so Anew is written whole); workgroups
// (x, y >= npairs) rotate the eigenvector columns of pair x in the kJP-row
// tile y - npairs, V[rows, P] <- V[rows, P] Q_P. Nothing once converged.
__global__ __launch_bounds__(kJT) void jac_update_kernel(const double *__restrict__ Aold,
                                                         double *__restrict__ Anew,
                                                         double *__restrict__ V, int64_t npad,
                                                         int nb, int r,
                                                         const double *__restrict__ Qall,
                                                         const int *__restrict__ done) {
  __shared__ double X[kJP][kJP1], Y[kJP][kJP1], Qa[kJP][kJP1], Qb[kJP][kJP1];
  const int npairs = nb / 2;
  const int t = threadIdx.x;
  const int a0 = t / (kJP / 2), b0 = t % (kJP / 2), h = kJP / 2;
  int I, J;
  circle_pair(nb, r, blockIdx.x, I, J);
  const double *QP = Qall + (int64_t)blockIdx.x * kJP * kJP;
  if (*done) return;   // converged: the flag names the buffer that holds the matrix
  if ((int)blockIdx.y >= npairs) {   // eigenvector columns
    const int64_t r0 = (int64_t)(blockIdx.y - npairs) * kJP;
    for (int e = t; e < kJP * kJP; e += kJT) {
      const int a = e / kJP, b = e % kJP;
      X[a][b] = V[(r0 + a) * npad + pair_index(I, J, b)];
      Qa[a][b] = QP[e];
    }
    __syncthreads();
    // X and Qa live in LDS and the results go to global memory; each thread
    // a 2 x 2 block of outputs
    double z00 = 0.0, z01 = 0.0, z10 = 0.0, z11 = 0.0;
#pragma unroll 8
    for (int k = 0; k < kJP; ++k) {
      const double x0 = X[a0][k], x1 = X[a0 + h][k], q0 = Qa[k][b0], q1 = Qa[k][b0 + h];
      z00 = fma(x0, q0, z00);
      z01 = fma(x0, q1, z01);
      z10 = fma(x1, q0, z10);
      z11 = fma(x1, q1, z11);
    }
    V[(r0 + a0) * npad + pair_index(I, J, b0)] = z00;
    V[(r0 + a0) * npad + pair_index(I, J, b0 + h)] = z01;
    V[(r0 + a0 + h) * npad + pair_index(I, J, b0)] = z10;
    V[(r0 + a0 + h) * npad + pair_index(I, J, b0 + h)] = z11;
    return;
  }
  int K, M;
  circle_pair(nb, r, blockIdx.y, K, M);
  const double *QQ = Qall + (int64_t)blockIdx.y * kJP * kJP;
  for (int e = t; e < kJP * kJP; e += kJT) {
    const int a = e / kJP, b = e % kJP;
    X[a][b] = Aold[pair_index(I, J, a) * npad + pair_index(K, M, b)];
    Qa[a][b] = QP[e];
    Qb[a][b] = QQ[e];
  }
  __syncthreads();
  {   // Y = Q_P^T X
    double y00 = 0.0, y01 = 0.0, y10 = 0.0, y11 = 0.0;
#pragma unroll 8
    for (int k = 0; k < kJP; ++k) {
      const double q0 = Qa[k][a0], q1 = Qa[k][a0 + h], x0 = X[k][b0], x1 = X[k][b0 + h];
      y00 = fma(q0, x0, y00);
      y01 = fma(q0, x1, y01);
      y10 = fma(q1, x0, y10);
      y11 = fma(q1, x1, y11);
    }
    Y[a0][b0] = y00;
    Y[a0][b0 + h] = y01;
    Y[a0 + h][b0] = y10;
    Y[a0 + h][b0 + h] = y11;
  }
  __syncthreads();
  {   // Anew = Y Q_P'
    double z00 = 0.0, z01 = 0.0, z10 = 0.0, z11 = 0.0;
#pragma unroll 8
    for (int k = 0; k < kJP; ++k) {
      const double y0 = Y[a0][k], y1 = Y[a0 + h][k], q0 = Qb[k][b0], q1 = Qb[k][b0 + h];
      z00 = fma(y0, q0, z00);
      z01 = fma(y0, q1, z01);
      z10 = fma(y1, q0, z10);
      z11 = fma(y1, q1, z11);
    }
    const int64_t r0 = pair_index(I, J, a0) * npad, r1 = pair_index(I, J, a0 + h) * npad;
    const int64_t c0 = pair_index(K, M, b0), c1 = pair_index(K, M, b0 + h);
    Anew[r0 + c0] = z00;
    Anew[r0 + c1] = z01;
    Anew[r1 + c0] = z10;
    Anew[r1 + c1] = z11;
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
// done = 1 + which (the index of the buffer checked) when off <= tol2 * all
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

__global__ void jac_check_final_kernel(const double *__restrict__ part, int which,
                                       int *__restrict__ done) {
  if (threadIdx.x != 0 || *done) return;
  double off = 0.0, tot = 0.0;
  for (int k = 0; k < kJacParts; ++k) {
    off += part[2 * k];
    tot += part[2 * k + 1];
  }
  if (off <= kJacTol2 * tot) *done = 1 + which;
}

// blocks of at most kJP orbitals (npad == kJP): inner sweeps in one workgroup
// until the same criterion holds (at most kSmallSweeps), then A and V written
// back
__global__ __launch_bounds__(kJT) void jac_small_kernel(double *__restrict__ A,
                                                        double *__restrict__ V,
                                                        int *__restrict__ info, int bit) {
  __shared__ JacLds L;
  const int t = threadIdx.x;
  for (int e = t; e < kJP * kJP; e += kJT) {
    L.S[0][e / kJP][e % kJP] = A[e];
    L.Q[e / kJP][e % kJP] = (e / kJP == e % kJP) ? 1.0 : 0.0;
  }
  __syncthreads();
  int cur = 0;
  bool conv = false;
  for (int sw = 0; sw <= kSmallSweeps; ++sw) {
    double off = 0.0, tot = 0.0;
    for (int e = t; e < kJP * kJP; e += kJT) {
      const double v = L.S[cur][e / kJP][e % kJP] * L.S[cur][e / kJP][e % kJP];
      tot += v;
      if (e / kJP != e % kJP) off += v;
    }
    off = jac_block_sum(off, L.red);
    tot = jac_block_sum(tot, L.red);
    if (off <= kJacTol2 * tot) {   // the same value in every thread
      conv = true;
      break;
    }
    if (sw == kSmallSweeps) break;
    cur = jac_inner_sweep(L, cur);
  }
  if (t == 0 && !conv && info) atomicOr(info, bit);
  for (int e = t; e < kJP * kJP; e += kJT) {
    A[e] = L.S[cur][e / kJP][e % kJP];
    V[e] = L.Q[e / kJP][e % kJP];
  }
}

// U = 0 with the identity on the orbitals that are not rotated (the frozen
// core, i < nfrz, and any beyond the virtual space, i >= nrot); eps = diag(F)
// (the rotated blocks are overwritten later)
__global__ __launch_bounds__(256) void semican_init_kernel(const double *__restrict__ F,
                                                           int64_t nmo, int64_t nfrz, int64_t nrot,
                                                           double *__restrict__ U,
                                                           double *__restrict__ eps) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < nmo * nmo;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / nmo, j = e % nmo;
    U[e] = (i == j && (i < nfrz || i >= nrot)) ? 1.0 : 0.0;
    if (i == j) eps[i] = F[e];
  }
}

// eigenvalue i (one workgroup each) goes to position rank(i) of the block
// (ascending, ties by index); its eigenvector, signed so that its largest
// component (the first such) is positive, to column o + rank(i) of U. The
// matrix is read from buffer A1 if the convergence flag (when given) names
// it, else from buffer cur when the flag is absent or unset.
__global__ __launch_bounds__(kJT) void jac_finalize_kernel(const double *__restrict__ A0,
                                                           const double *__restrict__ A1,
                                                           int cur, const int *__restrict__ done,
                                                           const double *__restrict__ V,
                                                           int64_t npad, int64_t n, int64_t o,
                                                           int64_t nmo, double *__restrict__ U,
                                                           double *__restrict__ eps) {
  __shared__ double red[kJT];
  __shared__ double bv[kJT];
  __shared__ int64_t bi[kJT];
  const int t = threadIdx.x;
  const int64_t i = blockIdx.x;
  const int flag = done ? *done : 0;
  const double *__restrict__ A = (flag ? flag == 2 : cur == 1) ? A1 : A0;
  const double lam = A[i * npad + i];
  double cnt = 0.0, best = -1.0;
  int64_t bidx = 0;
  for (int64_t j = t; j < n; j += kJT) {
    const double mu = A[j * npad + j];
    cnt += (mu < lam || (mu == lam && j < i)) ? 1.0 : 0.0;
    const double v = fabs(V[j * npad + i]);
    if (v > best) {   // j ascends within the thread: the first largest is kept
      best = v;
      bidx = j;
    }
  }
  const int64_t rank = (int64_t)jac_block_sum(cnt, red);
  bv[t] = best;
  bi[t] = bidx;
  __syncthreads();
  for (int w = kJT / 2; w > 0; w >>= 1) {   // largest |v|, the smallest index among equals
    if (t < w && (bv[t + w] > bv[t] || (bv[t + w] == bv[t] && bi[t + w] < bi[t]))) {
      bv[t] = bv[t + w];
      bi[t] = bi[t + w];
    }
    __syncthreads();
  }
  const double sg = V[bi[0] * npad + i] < 0.0 ? -1.0 : 1.0;
  if (t == 0) eps[o + rank] = lam;
  for (int64_t r = t; r < n; r += kJT) U[(o + r) * nmo + o + rank] = sg * V[r * npad + i];
}

int64_t semican_npad(int64_t n) { return std::max<int64_t>(kJP, round_up(n, kJP)); }

hipError_t launch_semican(const SemicanPlan &pl, const double *F, const double *C, double *U,
                          double *eps, double *Cs, int *info, void *ws, hipStream_t st) {
  hipError_t e;
  const int64_t nmo = pl.nmo;
  double *Ab[2] = {ws_d(ws, pl.off_a), ws_d(ws, pl.off_a2)};
  double *V = ws_d(ws, pl.off_v), *Qb = ws_d(ws, pl.off_q);
  double *Pt = ws_d(ws, pl.off_part);
  int *done = reinterpret_cast<int *>(static_cast<char *>(ws) + pl.off_flag);
  hipLaunchKernelGGL(semican_init_kernel,
                     dim3((unsigned)std::min<int64_t>(ceil_div(nmo * nmo, 256), 4096)), dim3(256),
                     0, st, F, nmo, pl.nfrz, pl.nfrz + pl.nc + pl.na + pl.nv, U, eps);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (info) {
    hipLaunchKernelGGL(jac_info_clear_kernel, dim3(1), dim3(64), 0, st, info);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const char *names[3] = {"semican_core", "semican_active", "semican_virtual"};
  const int64_t sizes[3] = {pl.nc, pl.na, pl.nv};
  int64_t o = pl.nfrz;
  for (int blk = 0; blk < 3; ++blk) {
    const int64_t n = sizes[blk];
    if (n == 0) continue;
    const int64_t npad = semican_npad(n);
    const int nb = (int)(npad / kJB);
    timer_begin(names[blk], st);
    int cur = 0;
    hipLaunchKernelGGL(jac_load_kernel,
                       dim3((unsigned)std::min<int64_t>(ceil_div(npad * npad, 256), 4096)),
                       dim3(256), 0, st, F, nmo, o, n, npad, Ab[0], V);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (npad == kJP) {
      hipLaunchKernelGGL(jac_small_kernel, dim3(1), dim3(kJT), 0, st, Ab[0], V, info, 1 << blk);
    } else {
      hipLaunchKernelGGL(jac_reset_kernel, dim3(1), dim3(64), 0, st, done);
      const int npairs = nb / 2;
      const unsigned tiles = (unsigned)(npad / kJP);
      for (int sw = 0; sw < kMaxSweeps; ++sw) {
        for (int r = 0; r < nb - 1; ++r) {
          hipLaunchKernelGGL(jac_pair_kernel, dim3(npairs), dim3(kJT), 0, st, Ab[cur], npad, nb,
                             r, Qb, done);
          hipLaunchKernelGGL(jac_update_kernel, dim3(npairs, npairs + tiles), dim3(kJT), 0, st,
                             Ab[cur], Ab[cur ^ 1], V, npad, nb, r, Qb, done);
          cur ^= 1;
        }
        hipLaunchKernelGGL(jac_check_part_kernel, dim3(kJacParts), dim3(kJT), 0, st, Ab[cur],
                           npad, Pt, done);
        hipLaunchKernelGGL(jac_check_final_kernel, dim3(1), dim3(64), 0, st, Pt, cur, done);
      }
      if (info) hipLaunchKernelGGL(jac_info_kernel, dim3(1), dim3(64), 0, st, done, info, 1 << blk);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(jac_finalize_kernel, dim3((unsigned)n), dim3(kJT), 0, st, Ab[0], Ab[1],
                       cur, npad == kJP ? nullptr : done, V, npad, n, o, nmo, U, eps);
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
