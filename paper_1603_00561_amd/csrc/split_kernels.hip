// Error-free int8 slice path (DSRG_SPLIT_OZAKI) of libdsrgdf (gfx950).
//
// Each column of B (one core or active orbital p and one virtual orbital e,
// a vector over the auxiliary index Q) is scaled by a power of two sigma with
// |B^Q_pe| < sigma and split into four round-to-nearest int8 slices,
//   B^Q_pe = sigma (s0 / 127 + s1 / (127 254) + s2 / (127 254^2)
//                   + s3 / (127 254^3) + r),
// |s_k| <= 127, |r| <= 1 / (2 127 254^3) (the splitting of Ozaki, Ogita,
// Oishi and Rump, "Error-free transformations of matrix multiplication by
// using fast routines of matrix multiplication", 2012, with an integer base
// that fills the int8 range). A contraction over Q becomes
//   (pe|qf) = sigma_pe sigma_qf sum_L I_L / (127^2 254^L),
//   I_L = sum_{k+l=L} sum_Q s_k s_l,
// kept for levels L <= 3 (ten slice products). Every I_L is an exact int32
// sum on the int8 matrix cores (|I_L| <= 4 * 127^2 * naux < 2^31 for naux <=
// 33000), so the only error left is the dropped levels and the residual r;
// the FP64 recombination rounds once per level. The self-pair diagonal
// (ia|ia) = sum_Q (B^Q_ia)^2, whose dropped terms all have one sign, is taken
// in FP64 instead.
#include "int8_tiles.h"

namespace dsrg {

// Column maxima and sums of squares in kScaleGroups slices of the auxiliary
// range (partials), then an in-order combine per column (deterministic).
constexpr int kScaleGroups = 32;

__global__ __launch_bounds__(256) void slice_scale_partial_kernel(
    const double *__restrict__ B, int64_t nrow, int64_t nv, int64_t naux, int64_t ntv,
    double *__restrict__ pmax, double *__restrict__ psum) {
  const int64_t ncol = nrow * ntv * kPanel;
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;   // (p, e) flattened
  const int g = blockIdx.y;
  if (col >= ncol) return;
  const int64_t p = col / (ntv * kPanel), e = col % (ntv * kPanel);
  double mx = 0.0, d = 0.0;
  if (e < nv) {
    const int64_t q0 = naux * g / kScaleGroups, q1 = naux * (g + 1) / kScaleGroups;
    const double *src = B + p * nv + e;
    for (int64_t q = q0; q < q1; ++q) {
      const double v = src[q * nrow * nv];
      mx = fmax(mx, fabs(v));
      d = fma(v, v, d);
    }
  }
  pmax[g * ncol + col] = mx;
  psum[g * ncol + col] = d;
}

__global__ __launch_bounds__(256) void slice_scale_final_kernel(const double *__restrict__ pmax,
                                                                const double *__restrict__ psum,
                                                                int64_t ncol,
                                                                double *__restrict__ sig,
                                                                double *__restrict__ diag) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= ncol) return;
  double mx = 0.0, d = 0.0;
  for (int g = 0; g < kScaleGroups; ++g) {
    mx = fmax(mx, pmax[g * ncol + col]);
    d += psum[g * ncol + col];
  }
  int ex = 0;
  if (mx > 0.0) (void)frexp(mx, &ex);     // mx < 2^ex
  sig[col] = (mx > 0.0) ? ldexp(1.0, ex) : 1.0;
  if (diag) diag[col] = d;
}

__global__ __launch_bounds__(256) void slice_pack_kernel(const double *__restrict__ B,
                                                         int64_t nrow, int64_t nv,
                                                         int64_t naux, int64_t ntv,
                                                         int64_t nqc,
                                                         const double *__restrict__ sig,
                                                         int8_t *__restrict__ S8) {
  // one thread per (column, chunk of 32 auxiliary indices)
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t ncol = nrow * ntv * kPanel;
  if (id >= ncol * nqc) return;
  const int64_t col = id % ncol, qc = id / ncol;   // consecutive threads: consecutive columns
  const int64_t p = col / (ntv * kPanel), e = col % (ntv * kPanel);
  const int64_t t = e / kPanel;
  const int c = (int)(e % kPanel);
  const double inv = 1.0 / sig[col];              // exact: sig is a power of two
  int8_t buf[kSlices][kQC];
#pragma unroll
  for (int j = 0; j < kQC; ++j) {
    const int64_t q = qc * kQC + j;
    double x = 0.0;
    if (e < nv && q < naux) x = B[(q * nrow + p) * nv + e] * inv * 127.0;
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const double r = rint(x);
      buf[s][j] = (int8_t)(int)r;
      x = (x - r) * 254.0;
    }
  }
  int8_t *dst = S8 + ((p * ntv + t) * nqc + qc) * (int64_t)kSlicePanelChunk;
  const int sw = (c >> 3) & 1;
#pragma unroll
  for (int s = 0; s < kSlices; ++s) {
    i4v *o = reinterpret_cast<i4v *>(dst + (s * kPanel + c) * kQC);
    const i4v *h = reinterpret_cast<const i4v *>(buf[s]);
    o[sw] = h[0];
    o[sw ^ 1] = h[1];
  }
}

// ---------------------------------------------------------------------------
// CCVV on slices. Work items are (core pair i <= j, 128-tile pair A <= B)
// in the order of decode_ccvv_list; classes 0: i<j, A<B (x and y = K^{ji}[A,B]),
// 1: i<j, A=B (y = x^T), 2: i=j, A<B and 3: i=j, A=B (y = x). The grid is
// persistent (kSlicePersistWG workgroups, a multiple of 8, each taking the
// next item of its XCD's list from that XCD's counter in ctr, which must be
// zero at launch); a class-0 item parks x in its workgroup's FP64 slot xs
// while y is formed. The self-pair diagonal (i = j, a = b) uses the FP64 sum
// of squares.
// ---------------------------------------------------------------------------
struct CcvvI8Args {
  int nc, nv, ntv_s;
  int64_t nqc;
  double s;
  int64_t slot_base;
  int atomic_mode;
  unsigned *chk;   // sign check word (nullptr: off)
};

__global__ __launch_bounds__(512) void ccvv_i8_kernel(const int8_t *__restrict__ S8,
                                                      const double *__restrict__ sig,
                                                      const double *__restrict__ diag,
                                                      const double *__restrict__ eps_c,
                                                      const double *__restrict__ eps_v,
                                                      CcvvI8Args a, double *__restrict__ xs,
                                                      int *ctr, double *slots, double *acc) {
  __shared__ __attribute__((aligned(16))) int8_t lds[kI8LdsRing];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int nt = a.ntv_s / 2;   // 128-wide tiles
  const int64_t ldv = (int64_t)a.ntv_s * kPanel;   // sigma / diagonal row length
  double *xw = xs + (int64_t)blockIdx.x * kSliceXsDoubles + threadIdx.x;
  const int x = blockIdx.x % 8;   // the XCD this workgroup runs on
  scalar_here(S8);
  scalar_here(sig);
  scalar_here(diag);
  scalar_here(eps_c);
  scalar_here(eps_v);
  scalar_here(xs);
  scalar_here(ctr);
  scalar_here(slots);
  scalar_here(acc);
  scalar_here(a.nc);
  scalar_here(a.nv);
  scalar_here(a.ntv_s);
  scalar_here(a.nqc);
  scalar_here(a.s);
  scalar_here(a.slot_base);
  scalar_here(a.atomic_mode);
  CcvvWork c;
  int64_t slot;
  // the next item of this XCD's list comes from its work counter, so the
  // items in flight on an XCD are always consecutive ones (shared panels)
  int *next = reinterpret_cast<int *>(lds + kI8LdsRing - sizeof(int));
  for (;;) {
    __syncthreads();   // the previous item is done with the LDS
    if (threadIdx.x == 0) *next = atomicAdd(ctr + x, 1);
    __syncthreads();
    const int64_t kk = *next;
    if (!decode_ccvv_list(kk, x, a.nc, nt, c, slot)) break;
    double v[kI8Out];
    ccvv_i8_item(S8, sig, c, a.nqc, a.ntv_s, lds, xw, wr, wc, lane, v);
    double (*T)[kI8Tile + 1] = reinterpret_cast<double (*)[kI8Tile + 1]>(lds);
    if (c.cls == 1) {
      // y = x^T through LDS (the ring is free after the last barrier)
#pragma unroll
      for (int q = 0; q < kI8Blocks; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) T[i8_row(wr, q, lane, r)][i8_col(wc, q, lane)] = v[q * 16 + r];
      __syncthreads();
    }
    double part = 0.0;
    const double eij = eps_c[c.i] + eps_c[c.j];
#pragma unroll
    for (int q = 0; q < kI8Blocks; ++q) {
      const int bcol = c.B * kI8Tile + i8_col(wc, q, lane);
      if (bcol >= a.nv) continue;
      const double eb = eps_v[bcol];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int arow = c.A * kI8Tile + i8_row(wr, q, lane, r);
        if (arow >= a.nv) continue;
        double xv, yv;
        if (c.cls == 0) {
          xv = xw[(q * 16 + r) * kI8Threads];
          yv = v[q * 16 + r];
        } else if (c.cls == 1) {
          xv = v[q * 16 + r];
          yv = T[i8_col(wc, q, lane)][i8_row(wr, q, lane, r)];
        } else {
          xv = yv = v[q * 16 + r];
          if (c.cls == 3 && arow == bcol) xv = yv = diag[c.i * ldv + arow];
        }
        const double R = reg_R(eij - (eps_v[arow] + eb), a.s);
        part += R * (xv * xv - xv * yv + yv * yv);
      }
    }
    if (c.cls == 1) __syncthreads();   // T is read before the reduction reuses the LDS
    const double w = (c.cls == 0) ? 4.0 : (c.cls == 3 ? 1.0 : 2.0);
    const double t = block_sum_n<8>(part, reinterpret_cast<double *>(lds)) * w;
    check_nonpositive(t, a.chk);
    emit_partial(t, slots, a.slot_base + slot, acc, a.atomic_mode);
  }
}

// ---------------------------------------------------------------------------
// CAVV on slices, step 1: for core orbitals m0 .. m0+mb-1 and all active u,
// the FP64 integrals X^{mu}[e][f] = (me|uf) = sum_Q B^Q_me B^Q_uf are written
// to Xb[(m - m0)][u][e][f] (row length xld = 128 ntv_s / 2). One workgroup per
// (pair (m, u), 128-tile pair (A, B)) over the full tile grid; pairs are dealt
// round-robin over the XCDs and tiles walked in 4 x 4 blocks.
// ---------------------------------------------------------------------------
struct CavvXArgs {
  int na, ntv_s;
  int64_t nqc;
  int m0, mb;
};

__device__ __forceinline__ void decode_tile_full_blocked(int64_t t, int nt, int &A, int &B) {
  const int nb = (nt + kTileBlock - 1) / kTileBlock;
  const int64_t row = (int64_t)kTileBlock * nt;   // tiles in one band of kTileBlock rows
  const int ba = (int)(t / row);
  int64_t rest = t % row;
  const int ha = (ba == nb - 1) ? nt - ba * kTileBlock : kTileBlock;   // band height
  const int bb = (int)(rest / ((int64_t)ha * kTileBlock));
  const int64_t in = rest % ((int64_t)ha * kTileBlock);
  const int wb = (bb == nb - 1) ? nt - bb * kTileBlock : kTileBlock;  // block width
  A = ba * kTileBlock + (int)(in / wb);
  B = bb * kTileBlock + (int)(in % wb);
}

inline int64_t fulltile_grid(int64_t P, int64_t nt) { return 8 * ((P + 7) / 8) * nt * nt; }

__global__ __launch_bounds__(512) void cavv_i8_x_kernel(const int8_t *__restrict__ S8c,
                                                        const int8_t *__restrict__ S8a,
                                                        const double *__restrict__ sigc,
                                                        const double *__restrict__ siga,
                                                        CavvXArgs a, double *__restrict__ Xb) {
  __shared__ __attribute__((aligned(16))) int8_t lds[kI8LdsRing];
  const int nt = a.ntv_s / 2;
  const int64_t T = (int64_t)nt * nt;
  const int64_t xcd = blockIdx.x % 8, kk = blockIdx.x / 8;
  const int64_t p = (kk / T) * 8 + xcd;
  if (p >= (int64_t)a.mb * a.na) return;
  int A, B;
  decode_tile_full_blocked(kk % T, nt, A, B);
  const int u = (int)(p % a.na), ml = (int)(p / a.na), m = a.m0 + ml;
  scalar_here(S8c);
  scalar_here(S8a);
  scalar_here(sigc);
  scalar_here(siga);
  scalar_here(Xb);
  scalar_here(a.nqc);
  scalar_here(a.ntv_s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int64_t ps = a.nqc * (int64_t)kSlicePanelChunk;
  const int8_t *r0 = slice_panel(S8c, m, 2 * A, a.ntv_s, a.nqc);
  const int8_t *c0 = slice_panel(S8a, u, 2 * B, a.ntv_s, a.nqc);
  i16v ac[kI8Blocks][kSlices];
  i8_tile_product(r0, r0 + ps, c0, c0 + ps, (int)a.nqc, lds, ac, wr, wc, lane);
  const int64_t ld = (int64_t)a.ntv_s * kPanel;
  double *X = Xb + ((int64_t)ml * a.na + u) * ld * ld + (int64_t)A * kI8Tile * ld + B * kI8Tile;
#pragma unroll
  for (int q = 0; q < kI8Blocks; ++q) {
    double x[16];
    i8_block_values(ac[q], sigc + m * ld + A * kI8Tile, siga + u * ld + B * kI8Tile, wr, wc, q,
                    lane, x);
#pragma unroll
    for (int r = 0; r < 16; ++r)
      X[(int64_t)i8_row(wr, q, lane, r) * ld + i8_col(wc, q, lane)] = x[r];
  }
}

// CAVV step 2 (both precisions). With X_u = (me|uf) = X^{mu}[e][f] and
// X'_u = (mf|ue) = X^{mu}[f][e], the energy is the sum over (m, e, f) of
//   sum_uv Gamma_uv [S(D_mu) X_u] [R1(D_mv) (2 X_v - X'_v)],
// D_mu = eps_m + eps_u - eps_e - eps_f. One workgroup per (m, 16-block pair
// E <= F): blocks X^{mu}[E][F] and X^{mu}[F][E] of every u are staged in LDS;
// thread (e, f) takes element (e, f) of E x F and, when E < F, element (f, e)
// of F x E, so every integral is read from memory once.
constexpr int kEpiT = 16;

struct CavvEpiArgs {
  int nv, nt16;
  int64_t ld;
  double s;
  int m0;
  int64_t slot_base;
  int atomic_mode;
};

template <int NA>
__device__ __forceinline__ double cavv_epi_element(const double (&Xu)[NA], const double (&Xp)[NA],
                                                   const double (&G)[NA][NA],
                                                   const double (&ea)[NA], double base,
                                                   double s) {
  double Sx[NA], W[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    double S, R1;
    reg_S_R1(base + ea[u], s, S, R1);
    Sx[u] = S * Xu[u];
    W[u] = R1 * (2.0 * Xu[u] - Xp[u]);
  }
  double part = 0.0;
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    double t = 0.0;
#pragma unroll
    for (int v = 0; v < NA; ++v) t += G[u][v] * W[v];
    part += Sx[u] * t;
  }
  return part;
}

template <int NA>
__global__ __launch_bounds__(256) void cavv_epi_kernel(const double *__restrict__ Xb,
                                                       const double *__restrict__ eps_c,
                                                       const double *__restrict__ eps_a,
                                                       const double *__restrict__ eps_v,
                                                       const double *__restrict__ gamma1,
                                                       CavvEpiArgs a, double *slots,
                                                       double *acc) {
  __shared__ double Xs[NA][2][kEpiT][kEpiT + 1];
  __shared__ double red[4];
  const int64_t T = (int64_t)a.nt16 * (a.nt16 + 1) / 2;
  const int ml = (int)(blockIdx.x / T);
  int E, F;
  decode_pair_le(blockIdx.x % T, a.nt16, E, F);
  const int e = threadIdx.x >> 4, f = threadIdx.x & 15;
  const int64_t ld = a.ld;
  const double *X = Xb + (int64_t)ml * NA * ld * ld;
  const int e0 = E * kEpiT, f0 = F * kEpiT;
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const double *Xu = X + (int64_t)u * ld * ld;
    Xs[u][0][e][f] = Xu[(int64_t)(e0 + e) * ld + f0 + f];
    Xs[u][1][e][f] = Xu[(int64_t)(f0 + e) * ld + e0 + f];
  }
  double G[NA][NA], ea[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    ea[u] = eps_a[u];
#pragma unroll
    for (int v = 0; v < NA; ++v) G[u][v] = gamma1[u * NA + v];
  }
  const double em = eps_c[a.m0 + ml];
  __syncthreads();
  double part = 0.0;
  double Xu[NA], Xp[NA];
  if (e0 + e < a.nv && f0 + f < a.nv) {
    // element (e0 + e, f0 + f)
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      Xu[u] = Xs[u][0][e][f];
      Xp[u] = Xs[u][1][f][e];
    }
    part += cavv_epi_element<NA>(Xu, Xp, G, ea, em - (eps_v[e0 + e] + eps_v[f0 + f]), a.s);
  }
  if (E != F && f0 + e < a.nv && e0 + f < a.nv) {
    // element (f0 + e, e0 + f)
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      Xu[u] = Xs[u][1][e][f];
      Xp[u] = Xs[u][0][f][e];
    }
    part += cavv_epi_element<NA>(Xu, Xp, G, ea, em - (eps_v[f0 + e] + eps_v[e0 + f]), a.s);
  }
  const double t = block_sum(part, red);
  emit_partial(t, slots, a.slot_base + blockIdx.x, acc, a.atomic_mode);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static hipError_t slice_one(const double *B, int64_t nrow, const Plan &pl, double *sig,
                            double *diag, int8_t *S8, double *scratch, hipStream_t st) {
  const int64_t ncol = nrow * pl.ntv_s * kPanel;
  double *pmax = scratch, *psum = scratch + kScaleGroups * ncol;
  timer_begin("slice_scale", st);
  hipLaunchKernelGGL(slice_scale_partial_kernel, dim3((unsigned)ceil_div(ncol, 256), kScaleGroups),
                     dim3(256), 0, st, B, nrow, pl.nv, pl.naux, pl.ntv_s, pmax, psum);
  hipLaunchKernelGGL(slice_scale_final_kernel, dim3((unsigned)ceil_div(ncol, 256)), dim3(256), 0,
                     st, pmax, psum, ncol, sig, diag);
  timer_end(st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  timer_begin("slice_pack", st);
  hipLaunchKernelGGL(slice_pack_kernel, dim3((unsigned)ceil_div(ncol * pl.nqc, 256)), dim3(256),
                     0, st, B, nrow, pl.nv, pl.naux, pl.ntv_s, pl.nqc, sig, S8);
  timer_end(st);
  return hipGetLastError();
}

hipError_t launch_slices(const Plan &pl, const Inputs &in, void *ws, bool with_av,
                         hipStream_t st) {
  hipError_t e = slice_one(in.B_cv, pl.nc, pl, ws_d(ws, pl.off_sigc), ws_d(ws, pl.off_diag),
                           ws_b(ws, pl.off_s8c), ws_d(ws, pl.off_scr), st);
  if (e != hipSuccess || !with_av) return e;
  return slice_one(in.B_av, pl.na, pl, ws_d(ws, pl.off_siga), nullptr, ws_b(ws, pl.off_s8a),
                   ws_d(ws, pl.off_scr), st);
}

template <int NA>
static hipError_t cavv_epi_na(const Plan &pl, const Inputs &in, void *ws, int m0, int mb,
                              hipStream_t st) {
  CavvEpiArgs a;
  a.nv = (int)pl.nv;
  a.nt16 = (int)ceil_div(pl.nv, kEpiT);
  a.ld = pl.xld;
  a.s = pl.s;
  a.m0 = m0;
  const int64_t T = (int64_t)a.nt16 * (a.nt16 + 1) / 2;
  a.slot_base = pl.slot_base[1] + (int64_t)m0 * T;
  a.atomic_mode = pl.atomic_reduce ? 1 : 0;
  timer_begin("cavv_epi", st);
  hipLaunchKernelGGL((cavv_epi_kernel<NA>), dim3((unsigned)(mb * T)), dim3(256), 0, st,
                     ws_d(ws, pl.off_xb), in.eps_c, in.eps_a, in.eps_v, in.gamma1, a,
                     ws_d(ws, pl.off_slots), ws_d(ws, pl.off_acc) + 1);
  timer_end(st);
  return hipGetLastError();
}

hipError_t launch_cavv_epi(const Plan &pl, const Inputs &in, void *ws, int m0, int mb,
                           hipStream_t st) {
  switch (pl.na) {
    case 1: return cavv_epi_na<1>(pl, in, ws, m0, mb, st);
    case 2: return cavv_epi_na<2>(pl, in, ws, m0, mb, st);
    case 3: return cavv_epi_na<3>(pl, in, ws, m0, mb, st);
    case 4: return cavv_epi_na<4>(pl, in, ws, m0, mb, st);
    case 5: return cavv_epi_na<5>(pl, in, ws, m0, mb, st);
    case 6: return cavv_epi_na<6>(pl, in, ws, m0, mb, st);
    case 7: return cavv_epi_na<7>(pl, in, ws, m0, mb, st);
    case 8: return cavv_epi_na<8>(pl, in, ws, m0, mb, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_cavv_x_split(const Plan &pl, void *ws, int m0, int mb, hipStream_t st) {
  CavvXArgs xa;
  xa.na = (int)pl.na;
  xa.ntv_s = (int)pl.ntv_s;
  xa.nqc = pl.nqc;
  xa.m0 = m0;
  xa.mb = mb;
  timer_begin("cavv_i8_x", st);
  hipLaunchKernelGGL(cavv_i8_x_kernel,
                     dim3((unsigned)fulltile_grid((int64_t)mb * pl.na, pl.ntv_s / 2)),
                     dim3(kI8Threads), 0, st, ws_b(ws, pl.off_s8c), ws_b(ws, pl.off_s8a),
                     ws_d(ws, pl.off_sigc), ws_d(ws, pl.off_siga), xa, ws_d(ws, pl.off_xb));
  timer_end(st);
  return hipGetLastError();
}

hipError_t launch_energy_split(const Plan &pl, const Inputs &in, void *ws, hipStream_t st) {
  hipError_t e;
  double *slots = ws_d(ws, pl.off_slots), *acc = ws_d(ws, pl.off_acc);
  if (pl.atomic_reduce) {
    if ((e = launch_zero(acc, 4, st)) != hipSuccess) return e;
  }
  // slices of B_cv (with the FP64 diagonal) and, for CAVV, of B_av
  if ((e = slice_one(in.B_cv, pl.nc, pl, ws_d(ws, pl.off_sigc), ws_d(ws, pl.off_diag),
                     ws_b(ws, pl.off_s8c), ws_d(ws, pl.off_scr), st)) != hipSuccess)
    return e;
  const bool cavv = (pl.terms & 2) && pl.na > 0, ccav = (pl.terms & 4) && pl.na > 0;
  if (cavv) {
    if ((e = slice_one(in.B_av, pl.na, pl, ws_d(ws, pl.off_siga), nullptr,
                       ws_b(ws, pl.off_s8a), ws_d(ws, pl.off_scr), st)) != hipSuccess)
      return e;
  }
  if (pl.terms & 1) {
    CcvvI8Args a;
    a.nc = (int)pl.nc;
    a.nv = (int)pl.nv;
    a.ntv_s = (int)pl.ntv_s;
    a.nqc = pl.nqc;
    a.s = pl.s;
    a.slot_base = pl.slot_base[0];
    a.atomic_mode = pl.atomic_reduce ? 1 : 0;
    a.chk = pl.chk;
    const int64_t items = pairtile_grid(pl.nc * (pl.nc + 1) / 2, pl.ntv_s / 2);
    const int64_t grid = items < kSlicePersistWG ? items : kSlicePersistWG;   // multiples of 8
    double *xs = ws_d(ws, pl.off_xs);
    int *ctr = reinterpret_cast<int *>(xs + (size_t)kSlicePersistWG * kSliceXsDoubles);
    if ((e = launch_zero(reinterpret_cast<double *>(ctr), 4, st)) != hipSuccess) return e;
    timer_begin("ccvv_i8", st);
    hipLaunchKernelGGL(ccvv_i8_kernel, dim3((unsigned)grid), dim3(kI8Threads), 0, st,
                       ws_b(ws, pl.off_s8c), ws_d(ws, pl.off_sigc), ws_d(ws, pl.off_diag),
                       in.eps_c, in.eps_v, a, xs, ctr, slots, acc + 0);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (cavv) {
    for (int64_t m0 = 0; m0 < pl.nc; m0 += pl.cavv_mb) {
      const int mb = (int)((pl.nc - m0) < pl.cavv_mb ? (pl.nc - m0) : pl.cavv_mb);
      if ((e = launch_cavv_x_split(pl, ws, (int)m0, mb, st)) != hipSuccess) return e;
      e = launch_cavv_epi(pl, in, ws, (int)m0, mb, st);
      if (e != hipSuccess) return e;
    }
  }
  if (ccav) {
    // the CCAV contraction is small: FP64 panels and the FP64 two-step kernels
    if ((e = launch_pack_fp64(pl, in, ws, st)) != hipSuccess) return e;
    if ((e = launch_ccav_fp64(pl, in, ws, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dsrg
