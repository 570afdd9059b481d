// FP64 forward path of libdsrgdf: panel packing, the CCVV / CAVV / CCAV
// pair-tiled contractions with fused regulariser epilogues, and the final
// reduction of the partial energies (gfx950, FP64 matrix cores).
//
// Every contraction is K = L^T R over the auxiliary index Q (Eq. int_fact),
// with L and R packed panels [Q][64 columns]; the (pq|rs) tiles live only in
// registers and are reduced into energies in the same kernel (section III:
// no four-index storage).
#include <algorithm>

#include "fp64_tiles.h"

namespace dsrg {

// ---------------------------------------------------------------------------
// Packing: P[(r * ntile + t)][Q][c] = B[Q][r][t * width + c], zero outside
// (Q >= naux or column >= ncol). Rows Q are padded to naux_p.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_panels_kernel(
    const double *__restrict__ B, double *__restrict__ P, int64_t nrow, int64_t ncol,
    int64_t naux, int64_t naux_p, int64_t ntile, int width) {
  const int64_t total = nrow * ntile * naux_p * width;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * 256) {
    const int c = (int)(idx % width);
    int64_t rest = idx / width;
    const int64_t q = rest % naux_p;
    rest /= naux_p;
    const int64_t t = rest % ntile;
    const int64_t r = rest / ntile;
    const int64_t col = t * width + c;
    double v = 0.0;
    if (q < naux && col < ncol) v = B[(q * nrow + r) * ncol + col];
    P[idx] = v;
  }
}

// ---------------------------------------------------------------------------
// CCVV (F1). Work items (core pair i <= j, virtual tile pair A <= B) in the
// order of decode_ccvv_list, taken by a persistent grid from per-XCD
// counters (two-product items first); the tile contributes
// weight * R(D) (x^2 - x y + y^2) with x = (ia|jb), y = (ib|ja) and weight
// 4, 2, 2, 1 for (i<j, A<B), (i<j, A=B), (i=j, A<B), (i=j, A=B).
// ---------------------------------------------------------------------------
struct CcvvArgs {
  int nc, nv, ntv;
  int64_t naux_p;
  double s;
  int64_t n0, n1, n2;      // sizes of the first three work classes
  int64_t slot_base;
  int atomic_mode;
  unsigned *chk;           // sign check word (nullptr: off)
};

__device__ __forceinline__ double ccvv_weight(int cls) {
  return (cls == 0) ? 4.0 : (cls == 3 ? 1.0 : 2.0);
}

__global__ __launch_bounds__(256, 3) void ccvv_fp64_kernel(const double *__restrict__ Pcv,
                                                        const double *__restrict__ eps_c,
                                                        const double *__restrict__ eps_v,
                                                        CcvvArgs a, int *ctr, double *slots,
                                                        double *acc) {
  constexpr int W = kPanel;
  __shared__ double lds[kCcvvLds];
  __shared__ int next;
  const int x = blockIdx.x % 8;   // the XCD this workgroup runs on
  CcvvWork c;
  int64_t slot;
  for (;;) {
  __syncthreads();   // the previous item is done with the LDS
  if (threadIdx.x == 0) next = atomicAdd(ctr + x, 1);
  __syncthreads();
  if (!decode_ccvv_list(next, x, a.nc, a.ntv, c, slot)) break;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int cl = lane & 15, kl = lane >> 4;
  d4 ax[2][2], ay[2][2];
  ccvv_compute(Pcv, Pcv, a.naux_p, a.ntv, a.nv, c, lds, ax, ay, wr, wc, cl, kl);

  const double eij = eps_c[c.i] + eps_c[c.j];
  double eb[2];
  int bcol[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    bcol[q] = c.B * W + 32 * wc + 16 * q + cl;
    eb[q] = bcol[q] < a.nv ? eps_v[bcol[q]] : 0.0;
  }
  double part = 0.0;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int arow = c.A * W + 32 * wr + 16 * p + 4 * r + kl;
      if (arow >= a.nv) continue;
      const double ea = eps_v[arow];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (bcol[q] >= a.nv) continue;
        const double R = reg_R(eij - (ea + eb[q]), a.s);
        const double x = ax[p][q][r], y = ay[p][q][r];
        part += R * (x * x - x * y + y * y);
      }
    }
  }
  const double t = block_sum(part, lds) * ccvv_weight(c.cls);
  check_nonpositive(t, a.chk);
  emit_partial(t, slots, a.slot_base + slot, acc, a.atomic_mode);
  }
}

// ---------------------------------------------------------------------------
// CAVV (F2), step 1 in FP64: for core orbitals m0 .. m0+mb-1 and active u, the
// integrals X^{mu}[e][f] = (me|uf) of every virtual tile pair A <= B (the CCVV
// tile machinery with pair (m, u), left panels B_cv, right panels B_av) are
// written to Xb[(m - m0)][u][e][f]: block [A,B] from x and block [B,A] from
// y = X^{mu}[B,A]^T. A persistent grid takes the items of decode_pair_list
// from per-XCD counters. Step 2 (cavv_epi_kernel) forms the energy. With
// tri set (the same panels on both sides), only the pairs m <= u are formed.
// ---------------------------------------------------------------------------
struct CavvXArgs64 {
  int na, ntv, nv;
  int64_t naux_p;
  int m0, mb;
  int tri;   // left and right panels are the same orbitals: only the pairs ml <= u
};

__global__ __launch_bounds__(256, 3) void cavv_fp64_x_kernel(const double *__restrict__ Pcv,
                                                          const double *__restrict__ Pav,
                                                          CavvXArgs64 a, int *ctr,
                                                          double *__restrict__ Xb) {
  constexpr int W = kPanel;
  __shared__ double lds[kCcvvLds];
  __shared__ int next;
  const int xcd = blockIdx.x % 8;
  for (;;) {
  __syncthreads();   // the previous item is done with the LDS
  if (threadIdx.x == 0) next = atomicAdd(ctr + xcd, 1);
  __syncthreads();
  int64_t pp;
  CcvvWork c;
  const int64_t npairs = a.tri ? (int64_t)a.na * (a.na + 1) / 2 : (int64_t)a.mb * a.na;
  if (!decode_pair_list(next, xcd, npairs, a.ntv, pp, c.A, c.B)) break;
  int ml, u;
  if (a.tri) {
    decode_pair_le(pp, a.na, ml, u);
  } else {
    ml = (int)(pp / a.na);
    u = (int)(pp % a.na);
  }
  c.i = a.m0 + ml;
  c.j = u;
  c.cls = (c.A == c.B) ? 2 : 0;   // y is needed only off the diagonal
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int cl = lane & 15, kl = lane >> 4;
  d4 ax[2][2], ay[2][2];
  ccvv_compute(Pcv, Pav, a.naux_p, a.ntv, a.nv, c, lds, ax, ay, wr, wc, cl, kl);
  const int64_t ld = (int64_t)a.ntv * W;
  double *X = Xb + ((int64_t)ml * a.na + u) * ld * ld;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        X[(int64_t)(c.A * W + 32 * wr + 16 * p + 4 * r + kl) * ld + c.B * W + 32 * wc + 16 * q +
          cl] = ax[p][q][r];
  if (c.A != c.B) {
    double (*T)[W + 1] = reinterpret_cast<double (*)[W + 1]>(lds);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          T[32 * wr + 16 * p + 4 * r + kl][32 * wc + 16 * q + cl] = ay[p][q][r];
    __syncthreads();
    for (int k = threadIdx.x; k < W * W; k += kThreads) {
      const int fr = k / W, ec = k % W;
      X[(int64_t)(c.B * W + fr) * ld + c.A * W + ec] = T[ec][fr];
    }
  }
  }
}

// ---------------------------------------------------------------------------
// CCAV (F3), two steps. (1) J[(m,e)][(n,u)] = (me|nu) = sum_Q B^Q_me B^Q_nu as
// one FP64 matrix-core GEMM over all core-virtual rows (m, e) and all
// core-active columns (n, u) (the B_ca block flattened, padded to a multiple
// of 16 columns); J holds nc^2 nv na values, the size of the integrals with
// one active index. (2) per (m <= n, e):
//   sum_uv etab_uv S(D^{ev}_{mn}) R1(D^{eu}_{mn}) [x_v (2x_u - y_u) + y_v (2y_u - x_u)]
// with x_u = (me|nu), y_u = (ne|mu), etab = 2I - Gamma: covers (m,n) and
// (n,m); weight 1 for m < n and 1/2 for m = n.
// ---------------------------------------------------------------------------
struct CcavJArgs {
  int64_t naux_p;
  int64_t ncols;     // padded column count of J (multiple of 16)
  int64_t qseg;      // auxiliary rows per segment (blockIdx.z), a multiple of 16
  int64_t jstride;   // doubles between the outputs of two segments
};

template <int NB>   // column blocks of 16 per workgroup
__global__ __launch_bounds__(256) void ccav_j_fp64_kernel(const double *__restrict__ Pcv,
                                                          const double *__restrict__ Pca2,
                                                          CcavJArgs a, double *__restrict__ J) {
  constexpr int W = kPanel, WB = 16 * NB, KC = 16;
  __shared__ double lv[2 * KC * W];
  __shared__ double lb[2 * KC * WB];
  const int64_t panel = blockIdx.x;                 // (m, T) panel index
  const int64_t c0 = (int64_t)blockIdx.y * WB;      // first column of this workgroup
  const int64_t qb = (int64_t)blockIdx.z * a.qseg;  // first auxiliary row of this segment
  const int64_t nq = (a.naux_p - qb < a.qseg) ? a.naux_p - qb : a.qseg;
  const double *srcv[1] = {Pcv + panel * a.naux_p * W + qb * W};
  const double *srcb[1] = {Pca2 + qb * a.ncols + c0};
  J += (int64_t)blockIdx.z * a.jstride;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, kl = lane >> 4;
  d4 acc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) acc[q] = zero4();
  Stage<1, W, KC> sv;
  Stage<1, WB, KC> sb;
  sv.load(srcv, W, 0);
  sb.load(srcb, a.ncols, 0);
  sv.store(lv);
  sb.store(lb);
  if (nq > KC) {
    sv.load(srcv, W, KC);
    sb.load(srcb, a.ncols, KC);
  }
  __syncthreads();
  int b = 0;
  for (int64_t q0 = 0; q0 < nq; q0 += KC) {
    const double *LV = lv + b * (KC * W), *LB = lb + b * (KC * WB);
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int k = kk * 4 + kl;
      const double fa = LV[k * W + lcol<W>(16 * wave + cl, k)];
#pragma unroll
      for (int q = 0; q < NB; ++q) acc[q] = mfma64(fa, LB[k * WB + lcol<WB>(16 * q + cl, k)], acc[q]);
    }
    if (q0 + KC < nq) {
      sv.store(lv + (b ^ 1) * (KC * W));
      sb.store(lb + (b ^ 1) * (KC * WB));
      if (q0 + 2 * KC < nq) {
        sv.load(srcv, W, q0 + 2 * KC);
        sb.load(srcb, a.ncols, q0 + 2 * KC);
      }
    }
    __syncthreads();
    b ^= 1;
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int64_t col = c0 + 16 * q + cl;
    if (col >= a.ncols) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = panel * W + 16 * wave + 4 * r + kl;
      J[row * a.ncols + col] = acc[q][r];
    }
  }
}

struct CcavEpiArgs {
  int nc, na, nv, ntv;
  int64_t ncols;
  double s;
  int echunks;       // blocks of 256 virtual orbitals per core pair
  int64_t slot_base;
  int atomic_mode;
};

template <int NA>
__global__ __launch_bounds__(256) void ccav_epi_fp64_kernel(
    const double *__restrict__ J, const double *__restrict__ eps_c,
    const double *__restrict__ eps_a, const double *__restrict__ eps_v,
    const double *__restrict__ gamma1, CcavEpiArgs a, double *slots, double *acc) {
  __shared__ double red[4];
  int m, n;
  decode_pair_le(blockIdx.x / a.echunks, a.nc, m, n);
  const int e = (int)(blockIdx.x % a.echunks) * 256 + threadIdx.x;
  double part = 0.0;
  if (e < a.nv) {
    const double *xr = J + ((int64_t)m * a.ntv * kPanel + e) * a.ncols + (int64_t)n * NA;
    const double *yr = J + ((int64_t)n * a.ntv * kPanel + e) * a.ncols + (int64_t)m * NA;
    const double base = eps_c[m] + eps_c[n] - eps_v[e];
    double S[NA], R1[NA], xv[NA], yv[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      reg_S_R1(base - eps_a[u], a.s, S[u], R1[u]);
      xv[u] = xr[u];
      yv[u] = yr[u];
    }
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      double sx = 0.0, sy = 0.0;
#pragma unroll
      for (int v = 0; v < NA; ++v) {
        const double eb = (u == v ? 2.0 : 0.0) - gamma1[u * NA + v];
        sx += eb * S[v] * xv[v];
        sy += eb * S[v] * yv[v];
      }
      part += R1[u] * ((2.0 * xv[u] - yv[u]) * sx + (2.0 * yv[u] - xv[u]) * sy);
    }
  }
  const double t = block_sum(part, red) * ((m == n) ? 0.5 : 1.0);
  emit_partial(t, slots, a.slot_base + blockIdx.x, acc, a.atomic_mode);
}

// ---------------------------------------------------------------------------
// Final reduction: one workgroup per term; compensated (Neumaier) sums of
// the per-workgroup slots in a fixed order, or a copy of the atomic
// accumulator. Unselected terms are written as 0.
// ---------------------------------------------------------------------------
constexpr int kFinTerms = 12;
struct FinArgs {
  int64_t base[kFinTerms], count[kFinTerms];
  int selected[kFinTerms];
  int atomic_mode;
};

__device__ __forceinline__ void two_sum_acc(double &s, double &c, double v) {
  const double t = s + v;
  if (fabs(s) >= fabs(v))
    c += (s - t) + v;
  else
    c += (v - t) + s;
  s = t;
}

__global__ __launch_bounds__(256) void finalize_kernel(const double *__restrict__ slots,
                                                       const double *__restrict__ acc,
                                                       FinArgs a, double *E) {
  __shared__ double ss[256], sc[256];
  const int t = blockIdx.x;
  if (!a.selected[t]) {
    if (threadIdx.x == 0) E[t] = 0.0;
    return;
  }
  if (a.atomic_mode) {
    if (threadIdx.x == 0) E[t] = acc[t];
    return;
  }
  double s = 0.0, c = 0.0;
  for (int64_t k = threadIdx.x; k < a.count[t]; k += 256) two_sum_acc(s, c, slots[a.base[t] + k]);
  ss[threadIdx.x] = s;
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      double s1 = ss[threadIdx.x], c1 = sc[threadIdx.x] + sc[threadIdx.x + h];
      two_sum_acc(s1, c1, ss[threadIdx.x + h]);
      ss[threadIdx.x] = s1;
      sc[threadIdx.x] = c1;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) E[t] = ss[0] + sc[0];
}

__global__ void zero_kernel(double *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static hipError_t pack_one(const double *B, double *P, int64_t nrow, int64_t ncol, int64_t naux,
                           int64_t naux_p, int64_t ntile, int width, hipStream_t st) {
  const int64_t total = nrow * ntile * naux_p * width;
  if (total == 0) return hipSuccess;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  timer_begin("pack_fp64", st);
  hipLaunchKernelGGL(pack_panels_kernel, dim3((unsigned)blocks), dim3(256), 0, st, B, P, nrow,
                     ncol, naux, naux_p, ntile, width);
  timer_end(st);
  return hipGetLastError();
}

hipError_t launch_pack_panels(const double *B, double *P, int64_t nrow, int64_t ncol,
                              int64_t naux, int64_t naux_p, int64_t ntile, int width,
                              hipStream_t st) {
  return pack_one(B, P, nrow, ncol, naux, naux_p, ntile, width, st);
}

hipError_t launch_pack_fp64(const Plan &pl, const Inputs &in, void *ws, hipStream_t st) {
  hipError_t e = pack_one(in.B_cv, ws_d(ws, pl.off_pcv), pl.nc, pl.nv, pl.naux, pl.naux_p,
                          pl.ntv, kPanel, st);
  if (e != hipSuccess) return e;
  if (pl.na > 0 && (pl.terms & 2) && pl.precision == 0) {
    e = pack_one(in.B_av, ws_d(ws, pl.off_pav), pl.na, pl.nv, pl.naux, pl.naux_p, pl.ntv,
                 kPanel, st);
    if (e != hipSuccess) return e;
  }
  if (pl.na > 0 && (pl.terms & 4)) {
    if (pl.with_grad)
      e = pack_one(in.B_ca, ws_d(ws, pl.off_pca), pl.nc, pl.na, pl.naux, pl.naux_p, 1,
                   kActPanel, st);
    else   // flattened (n,u) columns, padded to ccav_cols
      e = pack_one(in.B_ca, ws_d(ws, pl.off_pca), 1, pl.nc * pl.na, pl.naux, pl.naux_p, 1,
                   (int)pl.ccav_cols, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// out[i] = sum over segments z = 0 .. nseg-1 of part[z stride + i], in that order
__global__ __launch_bounds__(256) void sum_segments_kernel(const double *__restrict__ part,
                                                           int nseg, int64_t n, int64_t stride,
                                                           double *__restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    double v = part[i];
    for (int z = 1; z < nseg; ++z) v += part[z * stride + i];
    out[i] = v;
  }
}

hipError_t launch_j_fp64(const double *Pleft, int64_t npanels, const double *R, int64_t ncols,
                         int64_t naux_p, double *J, double *scratch, hipStream_t st) {
  if (ncols % 16 != 0 || naux_p % kChunk != 0) return hipErrorInvalidValue;
  CcavJArgs ja;
  ja.naux_p = naux_p;
  ja.ncols = ncols;
  ja.qseg = round_up(ceil_div(naux_p, scratch ? j_segments(npanels, ncols, naux_p) : 1), kChunk);
  // every segment starts inside the auxiliary range (and holds >= one chunk)
  const int nseg = (int)ceil_div(naux_p, ja.qseg);
  ja.jstride = npanels * kPanel * ncols;
  const int NBsel = j_column_blocks(ncols);
  const dim3 gj((unsigned)npanels, (unsigned)(ncols / (16 * NBsel)), (unsigned)nseg);
  double *out = nseg > 1 ? scratch : J;
  timer_begin("ccav_j_fp64", st);
  switch (NBsel) {
    case 1: hipLaunchKernelGGL(ccav_j_fp64_kernel<1>, gj, dim3(256), 0, st, Pleft, R, ja, out); break;
    case 2: hipLaunchKernelGGL(ccav_j_fp64_kernel<2>, gj, dim3(256), 0, st, Pleft, R, ja, out); break;
    case 3: hipLaunchKernelGGL(ccav_j_fp64_kernel<3>, gj, dim3(256), 0, st, Pleft, R, ja, out); break;
    default: hipLaunchKernelGGL(ccav_j_fp64_kernel<4>, gj, dim3(256), 0, st, Pleft, R, ja, out); break;
  }
  if (nseg > 1) {
    const int64_t n = ja.jstride;
    const int64_t blocks = std::min<int64_t>(ceil_div(n, 256), 4096);
    hipLaunchKernelGGL(sum_segments_kernel, dim3((unsigned)blocks), dim3(256), 0, st, scratch,
                       nseg, n, ja.jstride, J);
  }
  timer_end(st);
  return hipGetLastError();
}

template <int NA>
static hipError_t launch_ccav_na(const Plan &pl, const Inputs &in, void *ws, hipStream_t st,
                                 double *slots, double *acc) {
  hipError_t e = launch_j_fp64(ws_d(ws, pl.off_pcv), pl.nc * pl.ntv, ws_d(ws, pl.off_pca),
                               pl.ccav_cols, pl.naux_p, ws_d(ws, pl.off_j),
                               pl.ccav_split ? ws_d(ws, pl.off_jscr) : nullptr, st);
  if (e != hipSuccess) return e;
  CcavEpiArgs a;
  a.nc = (int)pl.nc;
  a.na = (int)pl.na;
  a.nv = (int)pl.nv;
  a.ntv = (int)pl.ntv;
  a.ncols = pl.ccav_cols;
  a.s = pl.s;
  a.echunks = (int)ceil_div(pl.nv, 256);
  a.slot_base = pl.slot_base[2];
  a.atomic_mode = pl.atomic_reduce ? 1 : 0;
  timer_begin("ccav_epi_fp64", st);
  hipLaunchKernelGGL((ccav_epi_fp64_kernel<NA>), dim3((unsigned)pl.n_ccav), dim3(256), 0, st,
                     ws_d(ws, pl.off_j), in.eps_c, in.eps_a, in.eps_v, in.gamma1, a, slots,
                     acc + 2);
  timer_end(st);
  return hipGetLastError();
}

#define DSRG_NA_SWITCH(FN, ...)                 \
  switch (pl.na) {                              \
    case 1: return FN<1>(__VA_ARGS__);          \
    case 2: return FN<2>(__VA_ARGS__);          \
    case 3: return FN<3>(__VA_ARGS__);          \
    case 4: return FN<4>(__VA_ARGS__);          \
    case 5: return FN<5>(__VA_ARGS__);          \
    case 6: return FN<6>(__VA_ARGS__);          \
    case 7: return FN<7>(__VA_ARGS__);          \
    case 8: return FN<8>(__VA_ARGS__);          \
    default: return hipErrorInvalidValue;       \
  }

hipError_t launch_x_fp64(const double *Pleft, const double *Pright, int nright, int ntv, int nv,
                         int64_t naux_p, int m0, int mb, int *ctr, double *Xb, bool tri,
                         hipStream_t st) {
  if (tri && (m0 != 0 || mb != nright || Pleft != Pright)) return hipErrorInvalidValue;
  CavvXArgs64 xa;
  xa.na = nright;
  xa.ntv = ntv;
  xa.nv = nv;
  xa.naux_p = naux_p;
  xa.m0 = m0;
  xa.mb = mb;
  xa.tri = tri ? 1 : 0;
  const int64_t npairs = tri ? (int64_t)nright * (nright + 1) / 2 : (int64_t)mb * nright;
  const int64_t items = pairtile_grid(npairs, ntv);
  const int64_t grid = items < 4 * kPersistCU ? items : 4 * kPersistCU;   // multiples of 8
  hipError_t e = launch_zero(reinterpret_cast<double *>(ctr), 4, st);
  if (e != hipSuccess) return e;
  timer_begin("cavv_fp64_x", st);
  hipLaunchKernelGGL(cavv_fp64_x_kernel, dim3((unsigned)grid), dim3(256), 0, st, Pleft, Pright,
                     xa, ctr, Xb);
  timer_end(st);
  return hipGetLastError();
}

hipError_t launch_cavv_x_fp64(const Plan &pl, void *ws, int m0, int mb, hipStream_t st) {
  return launch_x_fp64(ws_d(ws, pl.off_pcv), ws_d(ws, pl.off_pav), (int)pl.na, (int)pl.ntv,
                       (int)pl.nv, pl.naux_p, m0, mb, reinterpret_cast<int *>(ws_d(ws, pl.off_ctr)),
                       ws_d(ws, pl.off_xb), false, st);
}

static hipError_t launch_cavv(const Plan &pl, const Inputs &in, void *ws, hipStream_t st,
                              double *, double *) {
  for (int64_t m0 = 0; m0 < pl.nc; m0 += pl.cavv_mb) {
    const int mb = (int)((pl.nc - m0) < pl.cavv_mb ? (pl.nc - m0) : pl.cavv_mb);
    hipError_t e = launch_cavv_x_fp64(pl, ws, (int)m0, mb, st);
    if (e != hipSuccess) return e;
    if ((e = launch_cavv_epi(pl, in, ws, (int)m0, mb, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}
static hipError_t launch_ccav(const Plan &pl, const Inputs &in, void *ws, hipStream_t st,
                              double *slots, double *acc) {
  DSRG_NA_SWITCH(launch_ccav_na, pl, in, ws, st, slots, acc)
}

hipError_t launch_ccav_fp64(const Plan &pl, const Inputs &in, void *ws, hipStream_t st) {
  return launch_ccav(pl, in, ws, st, ws_d(ws, pl.off_slots), ws_d(ws, pl.off_acc));
}

hipError_t launch_zero(double *p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_energy_fp64(const Plan &pl, const Inputs &in, void *ws, hipStream_t st) {
  double *slots = ws_d(ws, pl.off_slots);
  double *acc = ws_d(ws, pl.off_acc);
  hipError_t e;
  if (pl.atomic_reduce) {
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(64), 0, st, acc, 4);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_pack_fp64(pl, in, ws, st)) != hipSuccess) return e;
  if (pl.terms & 1) {
    CcvvArgs a;
    a.nc = (int)pl.nc;
    a.nv = (int)pl.nv;
    a.ntv = (int)pl.ntv;
    a.naux_p = pl.naux_p;
    a.s = pl.s;
    const int64_t npo = tri_off(pl.nc), ntpo = tri_off(pl.ntv);
    a.n0 = npo * ntpo;
    a.n1 = npo * pl.ntv;
    a.n2 = pl.nc * ntpo;
    a.slot_base = pl.slot_base[0];
    a.atomic_mode = pl.atomic_reduce ? 1 : 0;
    a.chk = pl.chk;
    // persistent: two workgroups per CU (64 KiB of LDS each), items from
    // per-XCD counters
    const int64_t items = pairtile_grid(pl.nc * (pl.nc + 1) / 2, pl.ntv);
    const int64_t grid = items < 4 * kPersistCU ? items : 4 * kPersistCU;   // multiples of 8
    int *ctr = reinterpret_cast<int *>(ws_d(ws, pl.off_ctr));
    if ((e = launch_zero(ws_d(ws, pl.off_ctr), 4, st)) != hipSuccess) return e;
    timer_begin("ccvv_fp64", st);
    hipLaunchKernelGGL(ccvv_fp64_kernel, dim3((unsigned)grid), dim3(256), 0, st,
                       ws_d(ws, pl.off_pcv), in.eps_c, in.eps_v, a, ctr, slots, acc + 0);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((pl.terms & 2) && pl.na > 0) {
    if ((e = launch_cavv(pl, in, ws, st, slots, acc)) != hipSuccess) return e;
  }
  if ((pl.terms & 4) && pl.na > 0) {
    if ((e = launch_ccav(pl, in, ws, st, slots, acc)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_finalize(const Plan &pl, void *ws, double *E_terms, hipStream_t st) {
  FinArgs f = {};
  const int64_t counts[3] = {pl.n_ccvv, pl.n_cavv, pl.n_ccav};
  for (int t = 0; t < 3; ++t) {
    f.base[t] = pl.slot_base[t];
    f.count[t] = counts[t];
    f.selected[t] = ((pl.terms >> t) & 1) && (t == 0 || pl.na > 0);
  }
  f.atomic_mode = pl.atomic_reduce ? 1 : 0;
  timer_begin("finalize", st);
  hipLaunchKernelGGL(finalize_kernel, dim3(3), dim3(256), 0, st, ws_d(ws, pl.off_slots),
                     ws_d(ws, pl.off_acc), f, E_terms);
  timer_end(st);
  return hipGetLastError();
}

hipError_t launch_finalize_terms(const double *slots, const int64_t *base, const int64_t *count,
                                 int nterms, double *E, hipStream_t st) {
  if (nterms < 1 || nterms > kFinTerms) return hipErrorInvalidValue;
  FinArgs f = {};
  for (int t = 0; t < nterms; ++t) {
    f.base[t] = base[t];
    f.count[t] = count[t];
    f.selected[t] = 1;
  }
  timer_begin("finalize", st);
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)nterms), dim3(256), 0, st, slots, nullptr, f,
                     E);
  timer_end(st);
  return hipGetLastError();
}

}  // namespace dsrg
