// FP64 adjoint path of libdsrgdf: gradients of L = sum_t gE[t] E_t with
// respect to B, the orbital energies and s.
//
// Step 1 (adjoint tiles): the (pq|rs) tiles are recomputed exactly as in the
// forward kernels (never stored from the forward) and the epilogue writes
// the adjoint tiles dL/d(pq|rs) to the workspace, accumulating dL/deps and
// dL/ds on the way:
//   Gs[(j,b)][(i,a)] = 2 dL/d(ia|jb)          (CCVV, symmetric N x N)
//   G2[(m,e)][(w,f)] = dL/d(me|wf)            (CAVV)
//   G3[(m,e)][(n,w)] = dL/d(me|nw)            (CCAV)
// with N = nc * ntv * 64 padded core-virtual rows. The CAVV integrals are
// formed in batches of core orbitals by the forward producer and G2 is written
// by the adjoint epilogue shared with the slice path. Step 2 (adjoint GEMMs):
// dB^Q_{pq} = sum over the contracted index pair of B^Q times the adjoint
// tile (the chain rule through Eq. int_fact):
//   dB_cv = Pcv . Gs + Pav . G2^T + Pca . G3^T,  dB_av = Pcv . G2,  dB_ca = Pcv . G3.
#include "fp64_tiles.h"

namespace dsrg {

__global__ void zero_fill_kernel(double *p, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
    p[k] = 0.0;
}

static hipError_t zero_fill(double *p, int64_t n, hipStream_t st) {
  if (!p || n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// Write a 64 x 64 tile held in LDS (T[r][c], row stride 65) transposed into a
// row-major global matrix: dst[c * ld + r] = T[r][c]; a wave instruction
// writes 128-byte pieces of four rows c (lane: 16 consecutive r of one of four
// consecutive c), not one row's 512 bytes.
__device__ __forceinline__ void store_transposed64(const double (*T)[kPanel + 1], double *dst,
                                                   int64_t ld) {
  for (int k = threadIdx.x; k < kPanel * kPanel; k += kThreads) {
    const int lane = k & 63, wv = k >> 6;
    const int c = 4 * (wv >> 2) + (lane >> 4), r = 16 * (wv & 3) + (lane & 15);
    dst[(int64_t)c * ld + r] = T[r][c];
  }
}

struct GradOut {
  double *deps_c, *deps_a, *deps_v, *ds;
  const double *gE;
};

// ---------------------------------------------------------------------------
// CCVV adjoint tiles. For element (a,b) of work item (i,j,A,B):
// x = (ia|jb), y = (ib|ja), P = w (x^2 - x y + y^2) (all ordered terms the
// item covers), and dL/dD = gE0 P R'(D) feeds eps_i, eps_j (+) and eps_a,
// eps_b (-); dL/ds += gE0 P dR/ds. Adjoint values
//   g1 = 2 dL/d(ia|jb) = 4 gE0 R (2x - y),  g2 = 2 dL/d(ib|ja) = 4 gE0 R (2y - x)
// go to Gs[(i,a)][(j,b)] = Gs[(j,b)][(i,a)] = g1 and
// Gs[(j,a)][(i,b)] = Gs[(i,b)][(j,a)] = g2 (the blocks each class owns).
// ---------------------------------------------------------------------------
struct CcvvAdjArgs {
  int nc, nv, ntv;
  int64_t naux_p;
  double s;
  int64_t slot_base;   // first energy slot of this block pair
  // block pair of core orbitals: rows of the G block are (i, a) for i in
  // [r0, r0 + nr), columns (j, b) for j in [c0, c0 + ncb); r0 == c0 is a
  // diagonal block (pairs i <= j inside it, both orientations stored), else
  // r0 + nr <= c0 (pairs i in the row block, j in the column block, only the
  // entries whose row orbital is in the row block stored)
  int r0, nr, c0, ncb;
  int64_t ld;   // row length of the G block (ncb 64 ntv)
  unsigned *chk;   // sign check word (nullptr: off)
};

// pair p of a block pair -> (i, j), i <= j
__device__ __forceinline__ void block_pair(const CcvvAdjArgs &a, int64_t p, int &i, int &j) {
  if (a.r0 == a.c0) {
    int il, jl;
    decode_pair_le(p, a.nr, il, jl);
    i = a.r0 + il;
    j = a.r0 + jl;
  } else {
    i = a.r0 + (int)(p / a.ncb);
    j = a.c0 + (int)(p % a.ncb);
  }
}

__global__ __launch_bounds__(256, 3) void ccvv_adj_fp64_kernel(
    const double *__restrict__ Pcv, const double *__restrict__ eps_c,
    const double *__restrict__ eps_v, CcvvAdjArgs a, GradOut g, double *__restrict__ Gs,
    double *slots) {
  constexpr int W = kPanel;
  __shared__ double lds[kCcvvLds];
  __shared__ double rsum[W], csum[W];
  const int64_t npair = (a.r0 == a.c0) ? (int64_t)a.nr * (a.nr + 1) / 2 : (int64_t)a.nr * a.ncb;
  const PairTile pt = decode_pairtile(blockIdx.x, npair, a.ntv);
  if (pt.item < 0) return;
  CcvvWork c;
  block_pair(a, pt.p, c.i, c.j);
  c.A = pt.A;
  c.B = pt.B;
  c.cls = (c.i == c.j) ? (c.A == c.B ? 3 : 2) : (c.A == c.B ? 1 : 0);
  const bool diag = a.r0 == a.c0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int cl = lane & 15, kl = lane >> 4;
  d4 ax[2][2], ay[2][2];
  ccvv_compute(Pcv, Pcv, a.naux_p, a.ntv, a.nv, c, lds, ax, ay, wr, wc, cl, kl);
  if (threadIdx.x < W) {
    rsum[threadIdx.x] = 0.0;
    csum[threadIdx.x] = 0.0;
  }
  __syncthreads();

  const double gE0 = g.gE[0];
  const double w = (c.cls == 0) ? 4.0 : (c.cls == 3 ? 1.0 : 2.0);
  const double eij = eps_c[c.i] + eps_c[c.j];
  double eb[2];
  int bcol[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    bcol[q] = c.B * W + 32 * wc + 16 * q + cl;
    eb[q] = bcol[q] < a.nv ? eps_v[bcol[q]] : 0.0;
  }
  double e_part = 0.0, d_part = 0.0, s_part = 0.0, csl[2] = {0.0, 0.0};
  double g1[2][2][4], g2[2][2][4];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ar = 32 * wr + 16 * p + 4 * r + kl;
      const int arow = c.A * W + ar;
      const double ea = arow < a.nv ? eps_v[arow] : 0.0;
      double rs = 0.0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        g1[p][q][r] = 0.0;
        g2[p][q][r] = 0.0;
        if (arow >= a.nv || bcol[q] >= a.nv) continue;
        double R, dRD, dRs;
        reg_R_grad(eij - (ea + eb[q]), a.s, R, dRD, dRs);
        const double x = ax[p][q][r], y = ay[p][q][r];
        const double P = w * (x * x - x * y + y * y);
        e_part += R * P;
        const double dd = P * dRD;
        d_part += dd;
        rs += dd;
        csl[q] += dd;
        s_part += P * dRs;
        g1[p][q][r] = 4.0 * gE0 * R * (2.0 * x - y);
        g2[p][q][r] = 4.0 * gE0 * R * (2.0 * y - x);
      }
      if (rs != 0.0) atomicAdd(&rsum[ar], rs);
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q)
    if (csl[q] != 0.0) atomicAdd(&csum[32 * wc + 16 * q + cl], csl[q]);

  // G block entries: row (x, a) at (x - r0) 64 ntv + a, column (y, b) at
  // (y - c0) 64 ntv + b. Natural orientation: G[(i,A)][(j,B)] = g1 and, in a
  // diagonal block, G[(j,A)][(i,B)] = g2 (classes 0, 1); transposed (classes
  // 0 and 2, through LDS): G[(j,B)][(i,A)] = g1^T in a diagonal block and
  // G[(i,B)][(j,A)] = g2^T (class 0). An off-diagonal block keeps only the
  // entries with row orbital i: the others are their transposes, which the
  // adjoint products read from the same block.
  const int64_t WT = (int64_t)a.ntv * W;
  const int64_t rowI = (int64_t)(c.i - a.r0) * WT, colJ = (int64_t)(c.j - a.c0) * WT;
  const int64_t rowJ = (int64_t)(c.j - a.r0) * WT, colI = (int64_t)(c.i - a.c0) * WT;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t ra = c.A * W + 32 * wr + 16 * p + 4 * r + kl;
        const int64_t cb = c.B * W + 32 * wc + 16 * q + cl;
        Gs[(rowI + ra) * a.ld + colJ + cb] = g1[p][q][r];
        if (diag && (c.cls == 0 || c.cls == 1)) Gs[(rowJ + ra) * a.ld + colI + cb] = g2[p][q][r];
      }
  if ((diag && c.cls == 2) || c.cls == 0) {
    double (*T)[W + 1] = reinterpret_cast<double (*)[W + 1]>(lds);
    if (diag) {
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            T[32 * wr + 16 * p + 4 * r + kl][32 * wc + 16 * q + cl] = g1[p][q][r];
      __syncthreads();
      store_transposed64(T, Gs + (rowJ + c.B * W) * a.ld + colI + c.A * W, a.ld);
      __syncthreads();
    }
    if (c.cls == 0) {
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            T[32 * wr + 16 * p + 4 * r + kl][32 * wc + 16 * q + cl] = g2[p][q][r];
      __syncthreads();
      store_transposed64(T, Gs + (rowI + c.B * W) * a.ld + colJ + c.A * W, a.ld);
    }
  }
  __syncthreads();
  if (threadIdx.x < W) {
    const int t = threadIdx.x;
    if (c.A * W + t < a.nv) atomicAdd(&g.deps_v[c.A * W + t], -gE0 * rsum[t]);
    if (c.B * W + t < a.nv) atomicAdd(&g.deps_v[c.B * W + t], -gE0 * csum[t]);
  }
  const double tE = block_sum(e_part, lds);
  __syncthreads();
  const double tD = block_sum(d_part, lds);
  __syncthreads();
  const double tS = block_sum(s_part, lds);
  check_nonpositive(tE, a.chk);
  if (threadIdx.x == 0) {
    slots[a.slot_base + pt.item] = tE;
    atomicAdd(&g.deps_c[c.i], gE0 * tD);
    atomicAdd(&g.deps_c[c.j], gE0 * tD);
    atomicAdd(g.ds, gE0 * tS);
  }
}

// ---------------------------------------------------------------------------
// CCAV adjoint tiles for (m <= n, 64-row tile T), from the integrals
// J[(m,e)][(n,u)] = (me|nu) formed beforehand by one product over the inputs
// (nc nv rows of nc na). Per e and active w, with x_u = (me|nu),
// y_u = (ne|mu), etab = 2I - Gamma:
//   A_w = sum_u etab_uw R1_u (2x_u - y_u),  A'_w = sum_u etab_uw R1_u (2y_u - x_u)
//   C_w = sum_v etab_wv S_v x_v,            C'_w = sum_v etab_wv S_v y_v
//   dL/d(me|nw) = gE2 [S_w A_w  + R1_w (2C_w  - C'_w)]  -> G3[(m,e)][(n,w)]
//   dL/d(ne|mw) = gE2 [S_w A'_w + R1_w (2C'_w - C_w )]  -> G3[(n,e)][(m,w)]
//   dE/dD^{ew}_{mn} = x_w A_w S'_w + (2x_w - y_w) C_w R1'_w (+ the (n,m) mirror)
// weight 1/2 for m = n. Columns w >= na and padded rows are written as 0.
// ---------------------------------------------------------------------------
struct CcavAdjArgs {
  int nc, na, nv, ntv;
  double s;
  int64_t slot_base;
  int64_t N3;   // row length of G3 = nc * 16
};

template <int NA>
__global__ __launch_bounds__(256) void ccav_adj_fp64_kernel(
    const double *__restrict__ J, const double *__restrict__ eps_c,
    const double *__restrict__ eps_a, const double *__restrict__ eps_v,
    const double *__restrict__ gamma1, CcavAdjArgs a, GradOut g, double *__restrict__ G3,
    double *slots) {
  constexpr int W = kPanel, WA = kActPanel;
  __shared__ double lds[4];
  __shared__ double xs[2][kPanel][kActPanel + 1];
  __shared__ double asum[NA];
  int m, n;
  decode_pair_le(blockIdx.x / a.ntv, a.nc, m, n);
  const int T = (int)(blockIdx.x % a.ntv);
  if (threadIdx.x < NA) asum[threadIdx.x] = 0.0;
  // x_u = (me|nu) into xs[0], y_u = (ne|mu) into xs[1], for the tile's 64 e
  const int64_t ldj = (int64_t)a.nc * NA;
  for (int k = threadIdx.x; k < 2 * W * NA; k += 256) {
    const int which = k / (W * NA), el = (k / NA) % W, u = k % NA;
    const int e = T * W + el;
    const int p = which ? n : m, q = which ? m : n;
    xs[which][el][u] = (e < a.nv) ? J[((int64_t)p * a.nv + e) * ldj + (int64_t)q * NA + u] : 0.0;
  }
  __syncthreads();
  const double gE2 = g.gE[2];
  const double wgt = (m == n) ? 0.5 : 1.0;
  double e_part = 0.0, d_part = 0.0, s_part = 0.0;
  if (threadIdx.x < W) {
    const int el = threadIdx.x;
    const int e = T * W + el;
    const bool ok = e < a.nv;
    double gmn[WA], gnm[WA];
#pragma unroll
    for (int w = 0; w < WA; ++w) gmn[w] = gnm[w] = 0.0;
    if (ok) {
      const double base = eps_c[m] + eps_c[n] - eps_v[e];
      double S[NA], R1[NA], dS[NA], dR1[NA], sS[NA], sR1[NA], xv[NA], yv[NA], eb[NA][NA];
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        reg_S_R1_grad(base - eps_a[u], a.s, S[u], R1[u], dS[u], dR1[u], sS[u], sR1[u]);
        xv[u] = xs[0][el][u];
        yv[u] = xs[1][el][u];
#pragma unroll
        for (int v = 0; v < NA; ++v) eb[u][v] = (u == v ? 2.0 : 0.0) - gamma1[u * NA + v];
      }
#pragma unroll
      for (int w = 0; w < NA; ++w) {
        double Aw = 0.0, Ap = 0.0, Cw = 0.0, Cp = 0.0;
#pragma unroll
        for (int u = 0; u < NA; ++u) {
          Aw += eb[u][w] * R1[u] * (2.0 * xv[u] - yv[u]);
          Ap += eb[u][w] * R1[u] * (2.0 * yv[u] - xv[u]);
          Cw += eb[w][u] * S[u] * xv[u];
          Cp += eb[w][u] * S[u] * yv[u];
        }
        gmn[w] = gE2 * (S[w] * Aw + R1[w] * (2.0 * Cw - Cp));
        gnm[w] = gE2 * (S[w] * Ap + R1[w] * (2.0 * Cp - Cw));
        e_part += wgt * S[w] * (xv[w] * Aw + yv[w] * Ap);
        const double dd = wgt * (xv[w] * Aw * dS[w] + (2.0 * xv[w] - yv[w]) * Cw * dR1[w] +
                                 yv[w] * Ap * dS[w] + (2.0 * yv[w] - xv[w]) * Cp * dR1[w]);
        s_part += wgt * (xv[w] * Aw * sS[w] + (2.0 * xv[w] - yv[w]) * Cw * sR1[w] +
                         yv[w] * Ap * sS[w] + (2.0 * yv[w] - xv[w]) * Cp * sR1[w]);
        d_part += dd;
        atomicAdd(&asum[w], dd);
      }
    }
    double *rm = G3 + ((int64_t)m * a.ntv * W + e) * a.N3 + (int64_t)n * WA;
    double *rn = G3 + ((int64_t)n * a.ntv * W + e) * a.N3 + (int64_t)m * WA;
#pragma unroll
    for (int w = 0; w < WA; w += 2) *reinterpret_cast<d2v *>(rm + w) = d2v{gmn[w], gmn[w + 1]};
    if (m != n) {
#pragma unroll
      for (int w = 0; w < WA; w += 2) *reinterpret_cast<d2v *>(rn + w) = d2v{gnm[w], gnm[w + 1]};
    }
    if (ok) {
      double dsum = 0.0;
      // d_part accumulated above equals this thread's sum over w
      dsum = d_part;
      atomicAdd(&g.deps_v[e], -gE2 * dsum);
    }
  }
  __syncthreads();
  if (threadIdx.x < NA) atomicAdd(&g.deps_a[threadIdx.x], -gE2 * asum[threadIdx.x]);
  const double tE = block_sum(e_part, lds);
  __syncthreads();
  const double tD = block_sum(d_part, lds);
  __syncthreads();
  const double tS = block_sum(s_part, lds);
  if (threadIdx.x == 0) {
    slots[a.slot_base + blockIdx.x] = tE;
    atomicAdd(&g.deps_c[m], gE2 * tD);
    atomicAdd(&g.deps_c[n], gE2 * tD);
    atomicAdd(g.ds, gE2 * tS);
  }
}

// ---------------------------------------------------------------------------
// Adjoint GEMM: C[Q][n] (+)= sum_k A[Q][k] Bm[k][n], with
//   A[Q][k]  = Apan[k / PW][Q][k % PW]   (packed panels, Q rows < naux_p)
//   Bm[k][n] = TB ? G[g(n) * ldg + k] : G[k * ldg + g(n)]
//   g(n)     = (n / nvalid) * GP + n % nvalid when compact (the valid columns
//              of every group of GP, side by side), else g(n) = n with the
//              output column (n / GP) * nvalid + n % GP for n % GP < nvalid
// The contraction index runs over groups of kgrp of which the first kval are
// valid (a core orbital's virtual panels): chunks wholly past kval hold only
// the panels' zero padding and are skipped.
// 128 x 128 output tile per workgroup of 8 waves (two per SIMD: the FP64
// matrix cores need a second wave to issue back to back), wave w owning rows
// 64 (w >> 2) .. +63 and columns 32 (w & 3) .. +31; K chunks of 16 staged
// through registers and double-buffered in LDS, one barrier per chunk.
// ---------------------------------------------------------------------------
struct GemmArgs {
  int64_t naux, naux_p;   // rows of C / rows stored per panel
  int64_t K;              // contraction length (multiple of 16)
  int PW;                 // panel width of A (16 or 64)
  int64_t Ncols;          // columns of Bm (compact: valid columns only)
  int64_t ldg;
  int64_t GP, nvalid, ldc;
  int accumulate;
  int compact;
  int64_t kgrp, kval;     // contraction groups and their valid chunks (multiple of kGK)
  int64_t kseg;      // contraction indices per segment (blockIdx.z), a multiple of kGK
  int64_t zstride;   // doubles between the outputs of two segments
};

constexpr int kGT = 128, kGK = 16, kGA = kGK + 1, kGThreads = 512;

// A contraction chunk: its first index k and that index's place in its group.
struct AdjChunk {
  int64_t k;
  int64_t in;
  // the first chunk at or after this one that holds a valid index
  __device__ __forceinline__ void settle(const GemmArgs &a) {
    if (in >= a.kval) {
      k += a.kgrp - in;
      in = 0;
    }
  }
  __device__ __forceinline__ AdjChunk next(const GemmArgs &a) const {
    AdjChunk c{k + kGK, in + kGK};
    c.settle(a);
    return c;
  }
};

// The 16 x 128 chunk of G[k][n] (k-major form) as 1024 double2 pieces: piece
// idx (thread t + 512 h) holds row adj_row(idx), columns 2 adj_c2(idx) .. +1.
// A wave's 64 pieces are 64-byte pieces of all 16 rows (four lanes a row),
// not one row of 1 KB: a wave instruction then spans 16 rows of G, as the
// n-major form's spans 8 (cfg5 energy + gradient 166.4 -> 161.6 ms; 8 rows of
// 128 bytes: 164.0 ms).
__device__ __forceinline__ int adj_row(int idx) { return (idx & 63) >> 2; }
__device__ __forceinline__ int adj_c2(int idx) { return 4 * (idx >> 6) + (idx & 3); }

template <bool TB>
__global__ __launch_bounds__(kGThreads, 4) void gemm_adj_fp64_kernel(const double *__restrict__ Apan,
                                                                  const double *__restrict__ G,
                                                                  GemmArgs a,
                                                                  double *__restrict__ C) {
  __shared__ double sA[2][kGT * kGA];
  // Bm chunk: k-major 16 x 128 (half-swapped odd rows) for G, n-major
  // 128 x (16 + 1) like sA for G^T (rows stored as loaded, no transpose)
  __shared__ double sB[2][TB ? kGT * kGA : kGK * kGT];
  const int64_t Q0 = (int64_t)blockIdx.x * kGT, n0 = (int64_t)blockIdx.y * kGT;
  // this workgroup's segment of the contraction, [kb, ke)
  const int64_t kb = (int64_t)blockIdx.z * a.kseg;
  const int64_t ke = (kb + a.kseg < a.K) ? kb + a.kseg : a.K;
  // the G column (!TB) or row (TB) each thread loads is the same in every chunk
  auto gcol = [&](int64_t n) { return a.compact ? (n / a.nvalid) * a.GP + n % a.nvalid : n; };
  C += (int64_t)blockIdx.z * a.zstride;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int cl = lane & 15, kl = lane >> 4;

  d4 acc[4][2];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = zero4();

  // a chunk is 128 x 16 of A and 16 x 128 of Bm: 1024 double2 each, two per thread
  d2v ra[2], rb[2];
  int64_t goff[2];
  bool gok[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int idx = t + h * kGThreads;
    // !TB: columns n, n + 1 (nvalid even when compact: one group)
    const int64_t n = TB ? n0 + (idx >> 3) : n0 + 2 * adj_c2(idx);
    gok[h] = n < a.Ncols;
    goff[h] = gcol(n);
  }
  auto gload = [&](int64_t k0) {
    const int64_t pan = k0 / a.PW, c0 = k0 % a.PW;
    const double *Ab = Apan + pan * a.naux_p * a.PW + c0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = t + h * kGThreads;       // 128 rows x 8 double2
      const int row = idx >> 3, c2 = idx & 7;
      const int64_t Q = Q0 + row;
      ra[h] = (Q < a.naux_p) ? *reinterpret_cast<const d2v *>(Ab + Q * a.PW + 2 * c2)
                             : d2v{0.0, 0.0};
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = t + h * kGThreads;
      if constexpr (!TB) {
        const int row = adj_row(idx), c2 = adj_c2(idx);   // 16 rows x 64 double2
        rb[h] = gok[h] ? *reinterpret_cast<const d2v *>(G + (k0 + row) * a.ldg + goff[h])
                       : d2v{0.0, 0.0};
      } else {
        const int c2 = idx & 7;                    // 128 n-rows x 8 double2
        rb[h] = gok[h] ? *reinterpret_cast<const d2v *>(G + goff[h] * a.ldg + k0 + 2 * c2)
                       : d2v{0.0, 0.0};
      }
    }
  };
  auto sstore = [&](int b) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = t + h * kGThreads;
      const int row = idx >> 3, c2 = idx & 7;
      sA[b][row * kGA + 2 * c2] = ra[h][0];
      sA[b][row * kGA + 2 * c2 + 1] = ra[h][1];
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = t + h * kGThreads;
      if constexpr (!TB) {
        const int row = adj_row(idx), c2 = adj_c2(idx);
        *reinterpret_cast<d2v *>(&sB[b][row * kGT + ((2 * c2) ^ swz(row))]) = rb[h];
      } else {
        const int nr = idx >> 3, c2 = idx & 7;
        sB[b][nr * kGA + 2 * c2] = rb[h][0];
        sB[b][nr * kGA + 2 * c2 + 1] = rb[h][1];
      }
    }
  };

  // chunks c0 (in LDS), c1 (in registers) and c2 (next to load)
  AdjChunk c0{kb, kb % a.kgrp};
  c0.settle(a);
  AdjChunk c1 = c0.next(a), c2 = c1.next(a);
  if (c0.k < ke) {
    gload(c0.k);
    sstore(0);
    if (c1.k < ke) gload(c1.k);
  }
  __syncthreads();
  int b = 0;
  for (; c0.k < ke; c0 = c1, c1 = c2, c2 = c2.next(a)) {
    const double *LA = sA[b], *LB = sB[b];
#pragma unroll
    for (int kk = 0; kk < kGK / 4; ++kk) {
      const int k = kk * 4 + kl;
      double fa[4], fb[2];
#pragma unroll
      for (int p = 0; p < 4; ++p) fa[p] = LA[(64 * wr + 16 * p + cl) * kGA + k];
#pragma unroll
      for (int q = 0; q < 2; ++q)
        fb[q] = TB ? LB[(32 * wc + 16 * q + cl) * kGA + k]
                   : LB[k * kGT + ((32 * wc + 16 * q + cl) ^ swz(k))];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[p][q] = mfma64(fa[p], fb[q], acc[p][q]);
    }
    if (c1.k < ke) {
      sstore(b ^ 1);
      if (c2.k < ke) gload(c2.k);
    }
    __syncthreads();
    b ^= 1;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int64_t n = n0 + 32 * wc + 16 * q + cl;
    if (n >= a.Ncols) continue;
    const int64_t grp = n / a.GP, cc = n % a.GP;
    if (!a.compact && cc >= a.nvalid) continue;
    const int64_t col = a.compact ? n : grp * a.nvalid + cc;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t Q = Q0 + 64 * wr + 16 * p + 4 * r + kl;
        if (Q >= a.naux) continue;
        double *dst = C + Q * a.ldc + col;
        *dst = a.accumulate ? (*dst + acc[p][q][r]) : acc[p][q][r];
      }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// C[Q][col] (+)= sum over the segments z = 0 .. nseg-1 of P[z][Q][col], in that
// order, for Q < rows, col < ncol
__global__ __launch_bounds__(256) void adj_sum_kernel(const double *__restrict__ P, int nseg,
                                                      int64_t rows, int64_t ncol,
                                                      int64_t zstride, double *__restrict__ C,
                                                      int64_t ldc, int accumulate) {
  const int64_t n = rows * ncol;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    double v = P[i];
    for (int z = 1; z < nseg; ++z) v += P[z * zstride + i];
    double *dst = C + (i / ncol) * ldc + i % ncol;
    *dst = accumulate ? *dst + v : v;
  }
}

// the same sum for the int8 adjoint products (split_bwd.hip)
hipError_t launch_adj_sum(const double *P, int nseg, int64_t rows, int64_t ncol, int64_t zstride,
                          double *C, int64_t ldc, bool accumulate, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>(ceil_div(rows * ncol, 256), 4096);
  hipLaunchKernelGGL(adj_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, st, P, nseg, rows,
                     ncol, zstride, C, ldc, accumulate ? 1 : 0);
  return hipGetLastError();
}

// C (+)= A Bm with A the packed panels (K = npan PW) and Bm = G (TB: G^T). A
// product with too few 128 x 128 output tiles for the chip is split over K
// (adj_segments) when the plan holds room for the partial products, which
// adj_sum_kernel then adds in a fixed order.
template <bool TB>
static hipError_t gemm(const Plan &pl, void *ws, const double *Apan, int PW, int64_t npan,
                       const double *G, int64_t Ncols, int64_t ldg, int64_t GP, int64_t nvalid,
                       double *C, int64_t ldc, bool accumulate, hipStream_t st) {
  GemmArgs a;
  a.naux = pl.naux;
  a.naux_p = pl.naux_p;
  a.K = npan * PW;
  a.PW = PW;
  a.compact = (nvalid % 2 == 0 && Ncols % GP == 0) ? 1 : 0;
  a.Ncols = adj_fp64_cols(Ncols, GP, nvalid);
  a.ldg = ldg;
  a.GP = GP;
  a.nvalid = nvalid;
  a.ldc = ldc;
  a.accumulate = accumulate ? 1 : 0;
  // a core orbital's virtual panels (PW 64) hold nv valid columns of ntv 64;
  // the active panels (PW 16) are one chunk each
  a.kgrp = (PW == kPanel) ? pl.ntv * kPanel : PW;
  a.kval = (PW == kPanel) ? round_up(pl.nv, kGK) : PW;
  a.kseg = a.K;
  a.zstride = 0;
  const int64_t ncol = adj_out_cols(Ncols, GP, nvalid);
  int64_t nseg = adj_fp64_segments(pl.naux, Ncols, GP, nvalid, a.K);
  if (nseg > 1) {
    a.kseg = round_up(ceil_div(a.K, nseg), kGK);
    nseg = ceil_div(a.K, a.kseg);
  }
  const bool split = nseg > 1 && pl.gpart_doubles > 0 && nseg * pl.naux * ncol <= pl.gpart_doubles;
  double *out = C;
  if (split) {
    out = ws_d(ws, pl.off_gpart);
    a.ldc = ncol;
    a.accumulate = 0;
    a.zstride = pl.naux * ncol;
  } else {
    a.kseg = a.K;
    nseg = 1;
  }
  const dim3 grid((unsigned)ceil_div(pl.naux, kGT), (unsigned)ceil_div(a.Ncols, kGT),
                  (unsigned)nseg);
  timer_begin(TB ? "gemm_adj_tb_fp64" : "gemm_adj_fp64", st);
  hipLaunchKernelGGL(gemm_adj_fp64_kernel<TB>, grid, dim3(kGThreads), 0, st, Apan, G, a, out);
  if (split) {
    const int64_t blocks = std::min<int64_t>(ceil_div(pl.naux * ncol, 256), 4096);
    hipLaunchKernelGGL(adj_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, st, out, (int)nseg,
                       pl.naux, ncol, a.zstride, C, ldc, accumulate ? 1 : 0);
  }
  timer_end(st);
  return hipGetLastError();
}

template <int NA>
static hipError_t launch_adj_act(const Plan &pl, const Inputs &in, const GradOut &g, void *ws,
                                 int mask, hipStream_t st) {
  double *slots = ws_d(ws, pl.off_slots);
  if ((pl.terms & mask & 4)) {
    CcavAdjArgs a;
    a.nc = (int)pl.nc;
    a.na = (int)pl.na;
    a.nv = (int)pl.nv;
    a.ntv = (int)pl.ntv;
    a.s = pl.s;
    a.slot_base = pl.slot_base[2];
    a.N3 = pl.nc * kActPanel;
    double *J = ws_d(ws, pl.off_j);
    timer_begin("ccav_adj_fp64", st);
    // J[(m,e)][(n,u)] = sum_Q B^Q_me B^Q_nu: B_cv and B_ca as stored, [Q][(m,e)]
    // and [Q][(n,u)]
    hipError_t e = gemm_f64(true, false, pl.nc * pl.nv, pl.nc * pl.na, pl.naux, 1.0, in.B_cv,
                            pl.nc * pl.nv, in.B_ca, pl.nc * pl.na, 0.0, J, pl.nc * pl.na, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((ccav_adj_fp64_kernel<NA>), dim3((unsigned)pl.n_ccav), dim3(256), 0, st, J,
                       in.eps_c, in.eps_a, in.eps_v, in.gamma1, a, g, ws_d(ws, pl.off_g3), slots);
    timer_end(st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_zero_fill(double *p, int64_t n, hipStream_t st) { return zero_fill(p, n, st); }

// Gradients of eps and s cleared, the FP64 panels packed (FP64 path), and the
// CCAV adjoint tiles G3 (whole: nc 64 ntv rows of nc 16) with their energies
// and eps / s parts.
hipError_t launch_adjoint_start_fp64(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                                     hipStream_t st) {
  hipError_t e;
  GradOut g{o.deps_c, o.deps_a, o.deps_v, o.ds, o.gE};
  if ((e = zero_fill(o.deps_c, pl.nc, st)) != hipSuccess) return e;
  if ((e = zero_fill(o.deps_a, pl.na, st)) != hipSuccess) return e;
  if ((e = zero_fill(o.deps_v, pl.nv, st)) != hipSuccess) return e;
  if ((e = zero_fill(o.ds, 1, st)) != hipSuccess) return e;
  // the FP64 panels feed the FP64 path's adjoint tiles and products (the
  // slice path reads its operands from the inputs and its slices)
  if (pl.precision == 0 && (e = launch_pack_fp64(pl, in, ws, st)) != hipSuccess) return e;
  if ((pl.terms & 4) && pl.na > 0) {
    switch (pl.na) {
      case 1: e = launch_adj_act<1>(pl, in, g, ws, 4, st); break;
      case 2: e = launch_adj_act<2>(pl, in, g, ws, 4, st); break;
      case 3: e = launch_adj_act<3>(pl, in, g, ws, 4, st); break;
      case 4: e = launch_adj_act<4>(pl, in, g, ws, 4, st); break;
      case 5: e = launch_adj_act<5>(pl, in, g, ws, 4, st); break;
      case 6: e = launch_adj_act<6>(pl, in, g, ws, 4, st); break;
      case 7: e = launch_adj_act<7>(pl, in, g, ws, 4, st); break;
      case 8: e = launch_adj_act<8>(pl, in, g, ws, 4, st); break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// First energy slot of the CCVV block pair (I, J), I <= J: the pairs of the
// block pairs before it in the order (0,0), (0,1), .., (0,ngb-1), (1,1), ..
// times the tile pairs per core pair.
int64_t ccvv_block_slot(const Plan &pl, int64_t I, int64_t J, int64_t tiles_per_pair) {
  int64_t pairs = 0;
  for (int64_t a = 0; a <= I; ++a)
    for (int64_t b = a; b < pl.ngb; ++b) {
      if (a == I && b == J) return pl.slot_base[0] + pairs * tiles_per_pair;
      const int64_t na_ = std::min(pl.gb, pl.nc - a * pl.gb);
      const int64_t nb_ = std::min(pl.gb, pl.nc - b * pl.gb);
      pairs += (a == b) ? na_ * (na_ + 1) / 2 : na_ * nb_;
    }
  return -1;
}

// CCVV adjoint tiles of the core-orbital block pair (I, J) into the G block
// (FP64 integrals), with their energies and eps / s parts.
static hipError_t ccvv_adj_block_fp64(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                                      int64_t I, int64_t J, hipStream_t st) {
  GradOut g{o.deps_c, o.deps_a, o.deps_v, o.ds, o.gE};
  CcvvAdjArgs a;
  a.nc = (int)pl.nc;
  a.nv = (int)pl.nv;
  a.ntv = (int)pl.ntv;
  a.naux_p = pl.naux_p;
  a.s = pl.s;
  a.r0 = (int)(I * pl.gb);
  a.nr = (int)std::min(pl.gb, pl.nc - I * pl.gb);
  a.c0 = (int)(J * pl.gb);
  a.ncb = (int)std::min(pl.gb, pl.nc - J * pl.gb);
  a.ld = (int64_t)a.ncb * pl.ntv * kPanel;
  a.chk = pl.chk;
  const int64_t T = pl.ntv * (pl.ntv + 1) / 2;
  a.slot_base = ccvv_block_slot(pl, I, J, T);
  const int64_t npair = (I == J) ? (int64_t)a.nr * (a.nr + 1) / 2 : (int64_t)a.nr * a.ncb;
  timer_begin("ccvv_adj_fp64", st);
  hipLaunchKernelGGL(ccvv_adj_fp64_kernel, dim3((unsigned)pairtile_grid(npair, pl.ntv)), dim3(256),
                     0, st, ws_d(ws, pl.off_pcv), in.eps_c, in.eps_v, a, g, ws_d(ws, pl.off_gs),
                     ws_d(ws, pl.off_slots));
  timer_end(st);
  return hipGetLastError();
}

// dB_cv = the adjoint products of the CCVV, CAVV and CCAV tiles (FP64): per
// core block I the CAVV rows G2_I (dB_cv[I] += B_av G2_I^T, dB_av += B_cv[I]
// G2_I), per block pair (I, J) the CCVV block G_IJ (dB_cv[J] += B_cv[I] G_IJ
// and, off the diagonal, dB_cv[I] += B_cv[J] G_IJ^T), then the CCAV tiles G3
// (dB_cv += B_ca G3^T, dB_ca = B_cv G3). Every output element is first
// written, then accumulated in a fixed order.
hipError_t launch_backward_fp64(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                                hipStream_t st) {
  hipError_t e;
  if ((e = launch_adjoint_start_fp64(pl, in, o, ws, st)) != hipSuccess) return e;
  const bool cavv = (pl.terms & 2) && pl.na > 0, ccav = (pl.terms & 4) && pl.na > 0;
  const int64_t W = pl.ntv * kPanel;
  const int64_t Np = pl.nc * W, N2 = pl.na * W;
  const int64_t ldcv = pl.nc * pl.nv;
  const int64_t pstride = pl.ntv * pl.naux_p * kPanel;   // doubles per core orbital of Pcv
  const double *Pcv = ws_d(ws, pl.off_pcv);
  bool written = false;   // dB_cv holds a first product in every block
  auto blk = [&](int64_t I, int64_t &b0, int64_t &nb) {
    b0 = I * pl.gb;
    nb = std::min(pl.gb, pl.nc - b0);
  };
  if (cavv) {
    double *G2 = ws_d(ws, pl.off_g2);
    for (int64_t I = 0; I < pl.ngb; ++I) {
      int64_t m0, mb;
      blk(I, m0, mb);
      // padding rows of G2 are read by the products, never written by the epilogue
      if ((e = zero_fill(G2, mb * W * N2, st)) != hipSuccess) return e;
      if ((e = launch_cavv_x_fp64(pl, ws, (int)m0, (int)mb, st)) != hipSuccess) return e;
      if ((e = launch_cavv_adj_epi(pl, in, o, ws, (int)m0, (int)mb, st)) != hipSuccess) return e;
      e = gemm<true>(pl, ws, ws_d(ws, pl.off_pav), kPanel, pl.na * pl.ntv, G2, mb * W, N2, W,
                     pl.nv, o.dB_cv + m0 * pl.nv, ldcv, false, st);
      if (e != hipSuccess) return e;
      e = gemm<false>(pl, ws, Pcv + m0 * pstride, kPanel, mb * pl.ntv, G2, N2, N2, W, pl.nv,
                      o.dB_av, pl.na * pl.nv, I > 0, st);
      if (e != hipSuccess) return e;
    }
    written = true;
  } else if (o.dB_av) {
    if ((e = zero_fill(o.dB_av, pl.naux * pl.na * pl.nv, st)) != hipSuccess) return e;
  }
  if (pl.terms & 1) {
    const double *G = ws_d(ws, pl.off_gs);
    for (int64_t I = 0; I < pl.ngb; ++I)
      for (int64_t J = I; J < pl.ngb; ++J) {
        int64_t i0, ni, j0, nj;
        blk(I, i0, ni);
        blk(J, j0, nj);
        if ((e = ccvv_adj_block_fp64(pl, in, o, ws, I, J, st)) != hipSuccess) return e;
        // dB_cv[(j,b)] (+)= sum_(i,a) B_cv[(i,a)] G[(i,a)][(j,b)]; block J is
        // first written by the pair (0, J). A diagonal block holds both
        // orientations (the same values), so its product may take either
        // form; the one that reads G by rows of the output index (128 rows x
        // 16 contraction values per chunk) is the faster (cfg5 energy +
        // gradient 161.6 against 162.4 ms).
        const int64_t ldgs = nj * W;
        e = (I == J) ? gemm<true>(pl, ws, Pcv + i0 * pstride, kPanel, ni * pl.ntv, G, nj * W,
                                  ldgs, W, pl.nv, o.dB_cv + j0 * pl.nv, ldcv, written || I > 0,
                                  st)
                     : gemm<false>(pl, ws, Pcv + i0 * pstride, kPanel, ni * pl.ntv, G, nj * W,
                                   ldgs, W, pl.nv, o.dB_cv + j0 * pl.nv, ldcv,
                                   written || I > 0, st);
        if (e != hipSuccess) return e;
        if (J > I) {
          // dB_cv[(i,a)] += sum_(j,b) B_cv[(j,b)] G[(i,a)][(j,b)]
          e = gemm<true>(pl, ws, Pcv + j0 * pstride, kPanel, nj * pl.ntv, G, ni * W, ldgs, W,
                         pl.nv, o.dB_cv + i0 * pl.nv, ldcv, true, st);
          if (e != hipSuccess) return e;
        }
      }
    written = true;
  }
  if (ccav) {
    const int64_t N3 = pl.nc * kActPanel;
    e = gemm<true>(pl, ws, ws_d(ws, pl.off_pca), kActPanel, pl.nc, ws_d(ws, pl.off_g3), Np, N3,
                   W, pl.nv, o.dB_cv, ldcv, written, st);
    if (e != hipSuccess) return e;
    written = true;
    e = gemm<false>(pl, ws, Pcv, kPanel, pl.nc * pl.ntv, ws_d(ws, pl.off_g3), N3, N3, kActPanel,
                    pl.na, o.dB_ca, pl.nc * pl.na, false, st);
    if (e != hipSuccess) return e;
  } else if (o.dB_ca) {
    if ((e = zero_fill(o.dB_ca, pl.naux * pl.nc * pl.na, st)) != hipSuccess) return e;
  }
  if (!written) {
    if ((e = zero_fill(o.dB_cv, pl.naux * ldcv, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dsrg
