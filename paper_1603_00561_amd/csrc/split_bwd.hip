// Backward pass of the int8 slice path (DSRG_SPLIT_OZAKI) of libdsrgdf
// (gfx950): the adjoint contractions dE/dB = B G on the int8 matrix cores.
//
// The adjoint tiles G (Gs for CCVV, G2 for CAVV, G3 for CCAV) are formed in
// FP64 (CCAV) or from the slice-path integrals (CCVV, CAVV); each product
// C[Q][n] = sum_k B^Q_k G[k][n] is then taken on error-free int8 slices:
// both operands are split per row (Q for B, the output index n for G) into
// four scaled slices (the scheme of the forward slice path), the ten slice
// products of levels L <= 3 are exact int32 sums over segments of at most
// kGemmSeg contraction indices (|I_L| <= 4 * 127^2 * kGemmSeg < 2^31), and
// the levels are recombined in FP64, segment sums added in FP64.
#include "int8_tiles.h"

namespace dsrg {

// An FP64 operand seen as rows r (the index kept by the product) and a
// contraction index k, both in padded index spaces made of blocks: element
// (r, k) is base[(r / rblk) ldrb + (r % rblk) ldr + (k / kblk) ldkb +
// (k % kblk) ldk], and zero when r >= rlim, k >= klim, r % rblk >= rval or
// k % kblk >= kval.
struct OpMap {
  const double *base;
  int64_t rblk, rval, ldrb, ldr, rlim;
  int64_t kblk, kval, ldkb, ldk, klim;
};

// Row r of the map: returns its base pointer (or nullptr when the row is
// padding); k is walked by op_next with a running (block, offset) pair.
__device__ __forceinline__ const double *op_row(const OpMap &m, int64_t r) {
  if (r >= m.rlim) return nullptr;
  const int64_t rb = r / m.rblk, re = r % m.rblk;
  if (re >= m.rval) return nullptr;
  return m.base + rb * m.ldrb + re * m.ldr;
}

struct KWalk {
  int64_t k, kb, ke;
};

__device__ __forceinline__ KWalk kwalk_start(const OpMap &m, int64_t k) {
  return KWalk{k, k / m.kblk, k % m.kblk};
}

__device__ __forceinline__ double op_next(const OpMap &m, const double *row, KWalk &w) {
  double v = 0.0;
  if (row && w.k < m.klim && w.ke < m.kval) v = row[w.kb * m.ldkb + w.ke * m.ldk];
  ++w.k;
  if (++w.ke == m.kblk) {
    w.ke = 0;
    ++w.kb;
  }
  return v;
}

constexpr int kOpScaleGroups = 32;

// max_k |op(r, k)| over kOpScaleGroups ranges of k, one thread per row.
__global__ __launch_bounds__(256) void op_scale_partial_kernel(OpMap m, int64_t R, int64_t K,
                                                               double *__restrict__ pmax) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (r >= R) return;
  const int64_t k0 = K * g / kOpScaleGroups, k1 = K * (g + 1) / kOpScaleGroups;
  const double *row = op_row(m, r);
  double mx = 0.0;
  if (row) {
    KWalk w = kwalk_start(m, k0);
    for (int64_t k = k0; k < k1; ++k) mx = fmax(mx, fabs(op_next(m, row, w)));
  }
  pmax[g * R + r] = mx;
}

// The same partial maxima for operands whose contraction index is contiguous
// in memory (ldk = 1): one wave per row, lanes striding over k, so every
// load instruction reads 64 consecutive elements.
__global__ __launch_bounds__(256) void op_scale_rows_kernel(OpMap m, int64_t R, int64_t K,
                                                            double *__restrict__ pmax) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, g = blockIdx.y;
  if (r >= R) return;
  const int64_t k0 = K * g / kOpScaleGroups, k1 = K * (g + 1) / kOpScaleGroups;
  const double *row = op_row(m, r);
  double mx = 0.0;
  if (row) {
    int64_t k = k0 + lane, kb = k / m.kblk, ke = k % m.kblk;
    for (; k < k1 && k < m.klim; k += 64) {
      if (ke < m.kval) mx = fmax(mx, fabs(row[kb * m.ldkb + ke * m.ldk]));
      ke += 64;
      while (ke >= m.kblk) {
        ke -= m.kblk;
        ++kb;
      }
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) pmax[g * R + r] = mx;
}

// sigma[r] = the smallest power of two above the row maximum (1 for zero rows)
__global__ __launch_bounds__(256) void op_scale_final_kernel(const double *__restrict__ pmax,
                                                             int64_t R,
                                                             double *__restrict__ sig) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  double mx = 0.0;
  for (int g = 0; g < kOpScaleGroups; ++g) mx = fmax(mx, pmax[g * R + r]);
  int ex = 0;
  if (mx > 0.0) (void)frexp(mx, &ex);   // mx < 2^ex
  sig[r] = (mx > 0.0) ? ldexp(1.0, ex) : 1.0;
}

// Row and column maxima of |G| over an R x C block of an adjoint-tile array,
// for the operands of the two products that read it (rows of one, columns of
// the other): row r at base + (r / rblk) ldrb + (r % rblk) ldr, column c at
// + (c / cblk) ldcb + c % cblk. One 64 x 64 tile per workgroup, one pass over
// the block; the tile maxima are merged with integer atomic maxima of the
// values' bit patterns, which order nonnegative doubles as their values
// (rmax and cmax cleared to zero before; either may be nullptr).
struct MaxView {
  const double *base;
  int64_t R, C;
  int64_t rblk, ldrb, ldr;
  int64_t cblk, ldcb;
};

__global__ __launch_bounds__(256) void op_maxima_kernel(MaxView v, unsigned long long *rmax,
                                                        unsigned long long *cmax) {
  __shared__ double cs[4][64];
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t c = c0 + lane;
  const bool cok = c < v.C;
  const double *col = v.base + (cok ? (c / v.cblk) * v.ldcb + c % v.cblk : 0);
  double cm = 0.0;
  // 64-row tiles blockIdx.y, blockIdx.y + gridDim.y, ...
  for (int64_t r0 = (int64_t)blockIdx.y * 64; r0 < v.R; r0 += (int64_t)gridDim.y * 64) {
    for (int i = 0; i < 16; ++i) {
      const int64_t r = r0 + g * 16 + i;   // the same for the whole wave
      if (r >= v.R) break;
      const double x = cok ? fabs(col[(r / v.rblk) * v.ldrb + (r % v.rblk) * v.ldr]) : 0.0;
      cm = fmax(cm, x);
      if (rmax) {
        double m = x;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        if (lane == 0) atomicMax(rmax + r, (unsigned long long)__double_as_longlong(m));
      }
    }
  }
  cs[g][lane] = cm;
  __syncthreads();
  if (threadIdx.x < 64 && cok && cmax) {
    const double m = fmax(fmax(cs[0][lane], cs[1][lane]), fmax(cs[2][lane], cs[3][lane]));
    atomicMax(cmax + c, (unsigned long long)__double_as_longlong(m));
  }
}

// sig[r] = the smallest power of two above the maximum m[r] (bit pattern of a
// nonnegative double) for r < Rv, 1 for zero maxima and padding rows r < R
__global__ __launch_bounds__(256) void op_sigma_kernel(const unsigned long long *__restrict__ m,
                                                       int64_t Rv, int64_t R,
                                                       double *__restrict__ sig) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= R) return;
  const double mx = r < Rv ? __longlong_as_double((long long)m[r]) : 0.0;
  int ex = 0;
  if (mx > 0.0) (void)frexp(mx, &ex);   // mx < 2^ex
  sig[r] = (mx > 0.0) ? ldexp(1.0, ex) : 1.0;
}

// Slices of rows r in the panel layout of the forward path: panel r / 64,
// chunk qc of 32 contraction indices, slice s, column r % 64 (halves swapped
// when (r >> 3) & 1). One thread per (row, chunk); consecutive threads take
// consecutive rows.
__global__ __launch_bounds__(256) void op_pack_kernel(OpMap m, int64_t R, int64_t nqc,
                                                      const double *__restrict__ sig,
                                                      int8_t *__restrict__ S8) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= R * nqc) return;
  const int64_t r = id % R, qc = id / R;
  const double inv = 1.0 / sig[r];   // exact: a power of two
  const double *row = op_row(m, r);
  KWalk w = kwalk_start(m, qc * kQC);
  int8_t buf[kSlices][kQC];
#pragma unroll
  for (int j = 0; j < kQC; ++j) {
    double x = op_next(m, row, w) * inv * 127.0;
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const double t = rint(x);
      buf[s][j] = (int8_t)(int)t;
      x = (x - t) * 254.0;
    }
  }
  const int c = (int)(r % kPanel);
  int8_t *dst = S8 + ((r / kPanel) * nqc + qc) * (int64_t)kSlicePanelChunk;
  const int sw = (c >> 3) & 1;
#pragma unroll
  for (int s = 0; s < kSlices; ++s) {
    i4v *o = reinterpret_cast<i4v *>(dst + (s * kPanel + c) * kQC);
    const i4v *hh = reinterpret_cast<const i4v *>(buf[s]);
    o[sw] = hh[0];
    o[sw ^ 1] = hh[1];
  }
}

// The same slices for maps whose contraction index is contiguous in memory
// (ldk = 1) in blocks of whole chunks (kblk a multiple of 32): one workgroup
// per (64-row panel, chunk), chunks fastest; thread t takes row t / 4 and the
// eight contraction indices 8 (t % 4) .. +7, so four threads read a row's 256
// contiguous bytes (the one-thread-per-row kernel above reads 64 rows per load
// instruction) and write their eight bytes of each slice in place.
__global__ __launch_bounds__(256) void op_pack_rows_kernel(OpMap m, int64_t nqc,
                                                           const double *__restrict__ sig,
                                                           int8_t *__restrict__ S8) {
  const int64_t qc = blockIdx.x % nqc, pan = blockIdx.x / nqc;
  const int c = threadIdx.x >> 2, part = threadIdx.x & 3;
  const int64_t r = pan * kPanel + c;
  const double inv = 1.0 / sig[r];   // exact: a power of two
  const double *row = op_row(m, r);
  const int64_t k0 = qc * kQC + 8 * part;
  const int64_t kb = k0 / m.kblk, ke = k0 % m.kblk;
  uint64_t packed[kSlices] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double x = 0.0;
    if (row && ke + j < m.kval && k0 + j < m.klim) x = row[kb * m.ldkb + ke + j];
    x *= inv * 127.0;
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const double t = rint(x);
      packed[s] |= (uint64_t)(uint8_t)(int8_t)(int)t << (8 * j);
      x = (x - t) * 254.0;
    }
  }
  const int sw = (c >> 3) & 1;
  int8_t *dst = S8 + (pan * nqc + qc) * (int64_t)kSlicePanelChunk +
                (((part >> 1) ^ sw) << 4) + ((part & 1) << 3);
#pragma unroll
  for (int s = 0; s < kSlices; ++s)
    *reinterpret_cast<uint64_t *>(dst + (s * kPanel + c) * kQC) = packed[s];
}

static void launch_op_pack(const OpMap &m, int64_t R, int64_t nqc, const double *sig, int8_t *S8,
                           hipStream_t st) {
  if (m.ldk == 1 && m.kblk % kQC == 0 && R % kPanel == 0 && (R / kPanel) * nqc < ((int64_t)1 << 31))
    hipLaunchKernelGGL(op_pack_rows_kernel, dim3((unsigned)((R / kPanel) * nqc)), dim3(256), 0,
                       st, m, nqc, sig, S8);
  else
    hipLaunchKernelGGL(op_pack_kernel, dim3((unsigned)ceil_div(R * nqc, 256)), dim3(256), 0, st,
                       m, R, nqc, sig, S8);
}

// C[Q][n] (=|+=) sum_k A[Q][k] B[n][k] on slices, one 128 x 128 tile per
// workgroup (A tiles fastest, so the workgroups of one XCD share A panels).
// Output column n is written at (n / GP) nvalid + n % GP and skipped when
// n % GP >= nvalid (padding of the column blocks).
struct I8GemmArgs {
  int64_t tA;                 // 128-row tiles of A
  int64_t nqc;                // 32-wide contraction chunks of the product (and of B's panels)
  int64_t nqcA, qcA;          // chunks of A's panels, and A's chunk of contraction index 0
  int64_t segc, zstride;      // segment blockIdx.y: chunks [y segc, (y + 1) segc) (the last
                              // one may be shorter), output at y zstride
  int64_t M;                  // valid rows of A
  int64_t Ncols, GP, nvalid;  // padded output columns, their block width, valid per block
  int64_t ldc;
  int accumulate;
};

__global__ __launch_bounds__(512) void i8_gemm_kernel(const int8_t *__restrict__ SA,
                                                      const double *__restrict__ sigA,
                                                      const int8_t *__restrict__ SB,
                                                      const double *__restrict__ sigB,
                                                      I8GemmArgs a, double *__restrict__ C) {
  __shared__ __attribute__((aligned(16))) int8_t lds[kI8LdsRing];
  scalar_here(SA);
  scalar_here(sigA);
  scalar_here(SB);
  scalar_here(sigB);
  scalar_here(C);
  scalar_here(a.nqc);
  const int64_t ta = blockIdx.x % a.tA, tb = blockIdx.x / a.tA;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int64_t psA = a.nqcA * (int64_t)kSlicePanelChunk, psB = a.nqc * (int64_t)kSlicePanelChunk;
  const int64_t qc0 = (int64_t)blockIdx.y * a.segc;
  const int64_t nsg = (a.nqc - qc0 < a.segc) ? a.nqc - qc0 : a.segc;
  C += (int64_t)blockIdx.y * a.zstride;
  const int8_t *r0 = SA + 2 * ta * psA + (a.qcA + qc0) * (int64_t)kSlicePanelChunk;
  const int8_t *c0 = SB + 2 * tb * psB + qc0 * (int64_t)kSlicePanelChunk;
  i16v ac[kI8Blocks][kSlices];
  i8_tile_product(r0, r0 + psA, c0, c0 + psB, (int)nsg, lds, ac, wr, wc, lane);
#pragma unroll
  for (int q = 0; q < kI8Blocks; ++q) {
    double v[16];
    i8_block_values(ac[q], sigA + ta * kI8Tile, sigB + tb * kI8Tile, wr, wc, q, lane, v);
    const int64_t n = tb * kI8Tile + i8_col(wc, q, lane);
    const int64_t nb = n / a.GP, ne = n % a.GP;
    if (n >= a.Ncols || ne >= a.nvalid) continue;
    double *Cn = C + nb * a.nvalid + ne;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t Q = ta * kI8Tile + i8_row(wr, q, lane, r);
      if (Q >= a.M) continue;
      double *d = Cn + Q * a.ldc;
      *d = a.accumulate ? *d + v[r] : v[r];
    }
  }
}


// ---------------------------------------------------------------------------
// CCVV adjoint tiles on slices. Same work list, integrals and persistent grid
// as the forward slice kernel; per element (a, b) of item (i, j, A, B), with
// x = (ia|jb), y = (ib|ja), class weight w and P = w (x^2 - x y + y^2):
//   E += R P,  dL/dD = gE0 P R'(D) -> eps_i, eps_j (+), eps_a, eps_b (-),
//   dL/ds += gE0 P dR/ds,
//   g1 = 4 gE0 R (2x - y) -> Gs[(i,a)][(j,b)] and (classes 0, 2) Gs[(j,b)][(i,a)],
//   g2 = 4 gE0 R (2y - x) -> Gs[(j,a)][(i,b)] (classes 0, 1) and (class 0)
//   Gs[(i,b)][(j,a)],
// so every element of the symmetric Gs (row (p, e) = p W + e, W = 64 ntv) with
// e < nv is written once; the transposed blocks go through LDS. Padding
// columns of Gs are never written (the operand packer masks them).
// ---------------------------------------------------------------------------
struct CcvvAdjI8Args {
  int nc, nv, ntv_s;
  int64_t nqc;
  double s;
  int64_t slot_base;   // first energy slot of this block pair
  int64_t W, ld;       // G block: padded virtual orbitals per core orbital, row length
  // block pair of core orbitals (as for the FP64 adjoint tiles): rows (i, a)
  // for i in [r0, r0 + nr), columns (j, b) for j in [c0, c0 + ncb); r0 == c0
  // is a diagonal block, else only entries with row orbital i are stored
  int r0, nr, c0, ncb;
  unsigned *chk;   // sign check word (nullptr: off)
};

// dst[c ld + r] = T[r][c] for r < rvalid, c < cvalid; a wave instruction
// writes 128-byte pieces of four rows c of dst (lane: 16 consecutive r of one
// of four consecutive c), not one row's 512 bytes
__device__ __forceinline__ void store_transposed128(const double (*T)[kI8Tile + 1], double *dst,
                                                    int64_t ld, int rvalid, int cvalid) {
  for (int k = threadIdx.x; k < kI8Tile * kI8Tile; k += kI8Threads) {
    const int lane = k & 63, wv = k >> 6;
    const int c = 4 * (wv >> 3) + (lane >> 4), r = 16 * (wv & 7) + (lane & 15);
    if (r < rvalid && c < cvalid) dst[(int64_t)c * ld + r] = T[r][c];
  }
}

__global__ __launch_bounds__(512) void ccvv_adj_i8_kernel(
    const int8_t *__restrict__ S8, const double *__restrict__ sig,
    const double *__restrict__ diag, const double *__restrict__ eps_c,
    const double *__restrict__ eps_v, CcvvAdjI8Args a, double *__restrict__ xs, int *ctr,
    double *deps_c, double *deps_v, double *ds, const double *__restrict__ gE,
    double *__restrict__ Gs, double *slots) {
  __shared__ __attribute__((aligned(16))) int8_t lds[kI8LdsRing];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int nt = a.ntv_s / 2;
  const int64_t ldv = (int64_t)a.ntv_s * kPanel;
  double *xw = xs + (int64_t)blockIdx.x * kSliceXsDoubles + threadIdx.x;
  const int x = blockIdx.x % 8;
  scalar_here(S8);
  scalar_here(sig);
  scalar_here(diag);
  scalar_here(eps_c);
  scalar_here(eps_v);
  scalar_here(xs);
  scalar_here(ctr);
  scalar_here(Gs);
  scalar_here(slots);
  scalar_here(a.nqc);
  scalar_here(a.ntv_s);
  scalar_here(a.s);
  scalar_here(a.W);
  scalar_here(a.ld);
  double (*T)[kI8Tile + 1] = reinterpret_cast<double (*)[kI8Tile + 1]>(lds);
  double *rsum = reinterpret_cast<double *>(lds) + kI8Tile * (kI8Tile + 1);
  double *csum = rsum + kI8Tile;
  double *red = reinterpret_cast<double *>(lds);
  int *next = reinterpret_cast<int *>(lds + kI8LdsRing - sizeof(int));
  static_assert((kI8Tile * (kI8Tile + 3)) * sizeof(double) + sizeof(int) <= kI8LdsRing, "LDS");
  CcvvWork c;
  int64_t slot;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) *next = atomicAdd(ctr + x, 1);
    __syncthreads();
    const int64_t kk = *next;
    if (!decode_ccvv_block_list(kk, x, a.r0, a.nr, a.c0, a.ncb, nt, c, slot)) break;
    double v[kI8Out];
    ccvv_i8_item(S8, sig, c, a.nqc, a.ntv_s, lds, xw, wr, wc, lane, v);
    if (c.cls == 1) {
#pragma unroll
      for (int q = 0; q < kI8Blocks; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) T[i8_row(wr, q, lane, r)][i8_col(wc, q, lane)] = v[q * 16 + r];
    }
    if (threadIdx.x < 2 * kI8Tile) rsum[threadIdx.x] = 0.0;   // rsum and csum
    __syncthreads();
    const double gE0 = gE[0];
    const double w = (c.cls == 0) ? 4.0 : (c.cls == 3 ? 1.0 : 2.0);
    const double eij = eps_c[c.i] + eps_c[c.j];
    // G block rows (x, a) at (x - r0) W + a, columns (y, b) at (y - c0) W + b
    const bool dblk = a.r0 == a.c0;   // a diagonal block
    const int64_t rowI = (int64_t)(c.i - a.r0) * a.W, colJ = (int64_t)(c.j - a.c0) * a.W;
    const int64_t rowJ = (int64_t)(c.j - a.r0) * a.W, colI = (int64_t)(c.i - a.c0) * a.W;
    double e_part = 0.0, d_part = 0.0, s_part = 0.0;
    double g1v[kI8Out], g2v[kI8Out];
#pragma unroll
    for (int q = 0; q < kI8Blocks; ++q) {
      const int cl = i8_col(wc, q, lane);
      const int bcol = c.B * kI8Tile + cl;
      const bool bok = bcol < a.nv;
      const double eb = bok ? eps_v[bcol] : 0.0;
      double cs = 0.0;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rl = i8_row(wr, q, lane, r);
        const int arow = c.A * kI8Tile + rl;
        g1v[q * 16 + r] = 0.0;
        g2v[q * 16 + r] = 0.0;
        if (!bok || arow >= a.nv) continue;
        double xv, yv;
        if (c.cls == 0) {
          xv = xw[(q * 16 + r) * kI8Threads];
          yv = v[q * 16 + r];
        } else if (c.cls == 1) {
          xv = v[q * 16 + r];
          yv = T[cl][rl];
        } else {
          xv = yv = v[q * 16 + r];
          if (c.cls == 3 && arow == bcol) xv = yv = diag[c.i * ldv + arow];
        }
        double R, dRD, dRs;
        reg_R_grad(eij - (eps_v[arow] + eb), a.s, R, dRD, dRs);
        const double P = w * (xv * xv - xv * yv + yv * yv);
        e_part += R * P;
        const double dd = P * dRD;
        d_part += dd;
        cs += dd;
        atomicAdd(&rsum[rl], dd);
        s_part += P * dRs;
        const double g1 = 4.0 * gE0 * R * (2.0 * xv - yv);
        const double g2 = 4.0 * gE0 * R * (2.0 * yv - xv);
        g1v[q * 16 + r] = g1;
        g2v[q * 16 + r] = g2;
        Gs[(rowI + arow) * a.ld + colJ + bcol] = g1;
        if (dblk && c.cls <= 1) Gs[(rowJ + arow) * a.ld + colI + bcol] = g2;
      }
      if (cs != 0.0) atomicAdd(&csum[cl], cs);
    }
    const int rvalid = min(kI8Tile, a.nv - c.A * kI8Tile);
    const int cvalid = min(kI8Tile, a.nv - c.B * kI8Tile);
    if (c.cls == 0 || (dblk && c.cls == 2)) {
      // transposed blocks: (diagonal block) G[(j,B)][(i,A)] = g1^T, then
      // (class 0) G[(i,B)][(j,A)] = g2^T
      __syncthreads();   // class 1 has read T
      if (dblk) {
#pragma unroll
        for (int q = 0; q < kI8Blocks; ++q)
#pragma unroll
          for (int r = 0; r < 16; ++r)
            T[i8_row(wr, q, lane, r)][i8_col(wc, q, lane)] = g1v[q * 16 + r];
        __syncthreads();
        store_transposed128(T, Gs + (rowJ + c.B * kI8Tile) * a.ld + colI + c.A * kI8Tile, a.ld,
                            rvalid, cvalid);
        __syncthreads();
      }
      if (c.cls == 0) {
#pragma unroll
        for (int q = 0; q < kI8Blocks; ++q)
#pragma unroll
          for (int r = 0; r < 16; ++r)
            T[i8_row(wr, q, lane, r)][i8_col(wc, q, lane)] = g2v[q * 16 + r];
        __syncthreads();
        store_transposed128(T, Gs + (rowI + c.B * kI8Tile) * a.ld + colJ + c.A * kI8Tile, a.ld,
                            rvalid, cvalid);
      }
    }
    __syncthreads();
    if (threadIdx.x < kI8Tile) {
      const int t = threadIdx.x;
      if (t < rvalid) atomicAdd(&deps_v[c.A * kI8Tile + t], -gE0 * rsum[t]);
      if (t < cvalid) atomicAdd(&deps_v[c.B * kI8Tile + t], -gE0 * csum[t]);
    }
    const double tE = block_sum_n<8>(e_part, red);
    __syncthreads();
    const double tD = block_sum_n<8>(d_part, red);
    __syncthreads();
    const double tS = block_sum_n<8>(s_part, red);
    check_nonpositive(tE, a.chk);
    if (threadIdx.x == 0) {
      slots[a.slot_base + slot] = tE;
      atomicAdd(&deps_c[c.i], gE0 * tD);
      atomicAdd(&deps_c[c.j], gE0 * tD);
      atomicAdd(ds, gE0 * tS);
    }
  }
}

// ---------------------------------------------------------------------------
// CAVV adjoint tiles from a batch of integrals X^{mu}[e][f] = (me|uf) (the
// slice-path producer). One workgroup per (m, 16-block pair E <= F); thread
// (e, f) of E x F takes the element pair (e, f), (f, e). With X_u = (me|uf),
// Y_u = (mf|ue), S_u, R1_u at D^{mu}_{ef} (symmetric in e, f):
//   A_w  = sum_v Gamma_wv R1_v (2X_v - Y_v),  A'_w = sum_v Gamma_wv R1_v (2Y_v - X_v)
//   C_w  = sum_u Gamma_uw S_u X_u,            C'_w = sum_u Gamma_uw S_u Y_u
//   E   += S_w (X_w A_w + Y_w A'_w)
//   dL/d(me|wf) = gE1 [S_w A_w  + R1_w (2C_w  - C'_w)]   -> G2[(m,e)][(w,f)]
//   dL/d(mf|we) = gE1 [S_w A'_w + R1_w (2C'_w - C_w )]   -> G2[(m,f)][(w,e)]
//   dE/dD^{mw}_{ef} = X_w A_w S'_w + (2X_w - Y_w) C_w R1'_w + (the same with
//   X <-> Y, A <-> A', C <-> C')
// Diagonal block pairs (E = F) visit each pair twice: weight 1/2 in the sums,
// and only the first G2 entry is written (the mirrored thread writes the other).
// ---------------------------------------------------------------------------
constexpr int kAdjT = 16;

struct CavvAdjEpiArgs {
  int nv, nt16;
  int64_t ld;      // row length of the integral batch
  double s;
  int m0;
  int64_t W, N2;   // G2: padded virtual orbitals per orbital, row length
  int64_t slot_base;
};

template <int NA>
__global__ __launch_bounds__(256) void cavv_adj_epi_kernel(
    const double *__restrict__ Xb, const double *__restrict__ eps_c,
    const double *__restrict__ eps_a, const double *__restrict__ eps_v,
    const double *__restrict__ gamma1, CavvAdjEpiArgs a, double *deps_c, double *deps_a,
    double *deps_v, double *ds, const double *__restrict__ gE, double *__restrict__ G2,
    double *slots) {
  __shared__ double Xs[NA][2][kAdjT][kAdjT + 1];
  __shared__ double csw[4][kAdjT], red[4][NA + 3];
  const int64_t T = (int64_t)a.nt16 * (a.nt16 + 1) / 2;
  const int ml = (int)(blockIdx.x / T);
  int E, F;
  decode_pair_le(blockIdx.x % T, a.nt16, E, F);
  const int el = threadIdx.x >> 4, fl = threadIdx.x & 15;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t ld = a.ld;
  const double *X = Xb + (int64_t)ml * NA * ld * ld;
  const int e0 = E * kAdjT, f0 = F * kAdjT;
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const double *Xu = X + (int64_t)u * ld * ld;
    Xs[u][0][el][fl] = Xu[(int64_t)(e0 + el) * ld + f0 + fl];
    Xs[u][1][el][fl] = Xu[(int64_t)(f0 + el) * ld + e0 + fl];
  }
  double Gm[NA][NA], ea[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    ea[u] = eps_a[u];
#pragma unroll
    for (int v = 0; v < NA; ++v) Gm[u][v] = gamma1[u * NA + v];
  }
  const int m = a.m0 + ml;
  const double em = eps_c[m];
  const double gE1 = gE[1];
  const double wgt = (E == F) ? 0.5 : 1.0;
  __syncthreads();
  const int e = e0 + el, f = f0 + fl;
  const bool ok = e < a.nv && f < a.nv;
  // per-thread sums: energy, eps (total and per active w) and s parts; the
  // transposed adjoint values go out through LDS after the loads are done
  double e_part = 0.0, d_part = 0.0, s_part = 0.0, ddw[NA], gt[NA];
#pragma unroll
  for (int w = 0; w < NA; ++w) ddw[w] = gt[w] = 0.0;
  if (ok) {
    double Xv[NA], Yv[NA], S[NA], R1[NA], dS[NA], dR1[NA], sS[NA], sR1[NA];
    const double base = em - (eps_v[e] + eps_v[f]);
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      Xv[u] = Xs[u][0][el][fl];
      Yv[u] = Xs[u][1][fl][el];
      reg_S_R1_grad(base + ea[u], a.s, S[u], R1[u], dS[u], dR1[u], sS[u], sR1[u]);
    }
    double Av[NA], Ap[NA], Cv[NA], Cp[NA];
#pragma unroll
    for (int w = 0; w < NA; ++w) {
      double sa = 0.0, sp = 0.0, ca = 0.0, cp = 0.0;
#pragma unroll
      for (int v = 0; v < NA; ++v) {
        sa += Gm[w][v] * R1[v] * (2.0 * Xv[v] - Yv[v]);
        sp += Gm[w][v] * R1[v] * (2.0 * Yv[v] - Xv[v]);
        ca += Gm[v][w] * S[v] * Xv[v];
        cp += Gm[v][w] * S[v] * Yv[v];
      }
      Av[w] = sa;
      Ap[w] = sp;
      Cv[w] = ca;
      Cp[w] = cp;
    }
    // rows of the batch's core orbitals: (m - m0) W + e
    double *Gn = G2 + ((int64_t)ml * a.W + e) * a.N2 + f;   // + w W
#pragma unroll
    for (int w = 0; w < NA; ++w) {
      const double Wv = 2.0 * Xv[w] - Yv[w], Wp = 2.0 * Yv[w] - Xv[w];
      Gn[(int64_t)w * a.W] = gE1 * (S[w] * Av[w] + R1[w] * (2.0 * Cv[w] - Cp[w]));
      gt[w] = gE1 * (S[w] * Ap[w] + R1[w] * (2.0 * Cp[w] - Cv[w]));
      e_part += wgt * S[w] * (Xv[w] * Av[w] + Yv[w] * Ap[w]);
      const double dd = wgt * (Xv[w] * Av[w] * dS[w] + Wv * Cv[w] * dR1[w] +
                               Yv[w] * Ap[w] * dS[w] + Wp * Cp[w] * dR1[w]);
      s_part += wgt * (Xv[w] * Av[w] * sS[w] + Wv * Cv[w] * sR1[w] + Yv[w] * Ap[w] * sS[w] +
                       Wp * Cp[w] * sR1[w]);
      d_part += dd;
      ddw[w] = dd;
    }
  }
  // row sums (over f: the 16 lanes of one e) and column sums (over e: lanes
  // fl, fl + 16, fl + 32, fl + 48 of each wave, then the four waves), in a
  // fixed order
  double rsum = d_part, csum = d_part;
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) rsum += __shfl_xor(rsum, o, 64);
  csum += __shfl_xor(csum, 16, 64);
  csum += __shfl_xor(csum, 32, 64);
  // workgroup sums of the energy, eps and s parts and of each w's eps part
  double v3[NA + 3];
  v3[0] = e_part;
  v3[1] = d_part;
  v3[2] = s_part;
#pragma unroll
  for (int w = 0; w < NA; ++w) v3[3 + w] = ddw[w];
#pragma unroll
  for (int k = 0; k < NA + 3; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v3[k] += __shfl_xor(v3[k], o, 64);
  if (lane < kAdjT) csw[wave][lane] = csum;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NA + 3; ++k) red[wave][k] = v3[k];
  }
  if (fl == 0 && e < a.nv) atomicAdd(&deps_v[e], -gE1 * rsum);
  __syncthreads();   // every thread has read Xs, csw and red are complete
  if (E != F) {
#pragma unroll
    for (int w = 0; w < NA; ++w) Xs[w][0][fl][el] = gt[w];
  }
  if (threadIdx.x < kAdjT) {
    const int t = threadIdx.x;
    const double c = (csw[0][t] + csw[1][t]) + (csw[2][t] + csw[3][t]);
    if (f0 + t < a.nv) atomicAdd(&deps_v[f0 + t], -gE1 * c);
  }
  if (threadIdx.x < NA) {
    const int w = threadIdx.x;
    atomicAdd(&deps_a[w], gE1 * ((red[0][3 + w] + red[1][3 + w]) + (red[2][3 + w] + red[3][3 + w])));
  }
  if (threadIdx.x == 0) {
    const double tE = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    const double tD = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    const double tS = (red[0][2] + red[1][2]) + (red[2][2] + red[3][2]);
    slots[a.slot_base + blockIdx.x] = tE;
    atomicAdd(&deps_c[m], gE1 * tD);
    atomicAdd(ds, gE1 * tS);
  }
  if (E != F) {
    // G2[(m - m0) W + f][w W + e]: rows f, the 16 e of a row from 16 threads
    __syncthreads();
    const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    if (f0 + r < a.nv && e0 + c < a.nv) {
      double *Gt = G2 + ((int64_t)ml * a.W + f0 + r) * a.N2 + e0 + c;
#pragma unroll
      for (int w = 0; w < NA; ++w) Gt[(int64_t)w * a.W] = Xs[w][0][r][c];
    }
  }
}

template <int NA>
static hipError_t cavv_adj_epi_na(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                                  int m0, int mb, hipStream_t st) {
  CavvAdjEpiArgs a;
  a.nv = (int)pl.nv;
  a.nt16 = (int)ceil_div(pl.nv, kAdjT);
  a.ld = pl.xld;
  a.s = pl.s;
  a.m0 = m0;
  a.W = pl.ntv * kPanel;
  a.N2 = pl.na * a.W;
  const int64_t T = (int64_t)a.nt16 * (a.nt16 + 1) / 2;
  a.slot_base = pl.slot_base[1] + (int64_t)m0 * T;
  timer_begin("cavv_adj_epi", st);
  hipLaunchKernelGGL((cavv_adj_epi_kernel<NA>), dim3((unsigned)(mb * T)), dim3(256), 0, st,
                     ws_d(ws, pl.off_xb), in.eps_c, in.eps_a, in.eps_v, in.gamma1, a, o.deps_c,
                     o.deps_a, o.deps_v, o.ds, o.gE, ws_d(ws, pl.off_g2),
                     ws_d(ws, pl.off_slots));
  timer_end(st);
  return hipGetLastError();
}

hipError_t launch_cavv_adj_epi(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                               int m0, int mb, hipStream_t st) {
  switch (pl.na) {
    case 1: return cavv_adj_epi_na<1>(pl, in, o, ws, m0, mb, st);
    case 2: return cavv_adj_epi_na<2>(pl, in, o, ws, m0, mb, st);
    case 3: return cavv_adj_epi_na<3>(pl, in, o, ws, m0, mb, st);
    case 4: return cavv_adj_epi_na<4>(pl, in, o, ws, m0, mb, st);
    case 5: return cavv_adj_epi_na<5>(pl, in, o, ws, m0, mb, st);
    case 6: return cavv_adj_epi_na<6>(pl, in, o, ws, m0, mb, st);
    case 7: return cavv_adj_epi_na<7>(pl, in, o, ws, m0, mb, st);
    case 8: return cavv_adj_epi_na<8>(pl, in, o, ws, m0, mb, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static OpMap op_map(const double *base, int64_t rblk, int64_t rval, int64_t ldrb, int64_t ldr,
                    int64_t rlim, int64_t kblk, int64_t kval, int64_t ldkb, int64_t ldk,
                    int64_t klim) {
  OpMap m;
  m.base = base;
  m.rblk = rblk;
  m.rval = rval;
  m.ldrb = ldrb;
  m.ldr = ldr;
  m.rlim = rlim;
  m.kblk = kblk;
  m.kval = kval;
  m.ldkb = ldkb;
  m.ldk = ldk;
  m.klim = klim;
  return m;
}

// Scales and slices of an operand with R rows (a multiple of 128) and K
// contraction indices (a multiple of 32).
static hipError_t pack_operand(const OpMap &m, int64_t R, int64_t K, double *sig,
                               double *pmax, int8_t *S8, hipStream_t st) {
  timer_begin("op_pack", st);
  if (m.ldk == 1)
    hipLaunchKernelGGL(op_scale_rows_kernel, dim3((unsigned)ceil_div(R, 4), kOpScaleGroups),
                       dim3(256), 0, st, m, R, K, pmax);
  else
    hipLaunchKernelGGL(op_scale_partial_kernel, dim3((unsigned)ceil_div(R, 256), kOpScaleGroups),
                       dim3(256), 0, st, m, R, K, pmax);
  hipLaunchKernelGGL(op_scale_final_kernel, dim3((unsigned)ceil_div(R, 256)), dim3(256), 0, st,
                     pmax, R, sig);
  launch_op_pack(m, R, K / kQC, sig, S8, st);
  timer_end(st);
  return hipGetLastError();
}

// The maxima of an adjoint-tile block for both of its operands (one pass),
// into rmax [R] and cmax [C] (uint64 bit patterns in the pmax buffer).
static hipError_t block_maxima(const MaxView &v, double *rmax, double *cmax, hipStream_t st) {
  timer_begin("op_pack", st);
  hipError_t e;
  if (rmax && (e = launch_zero_fill(rmax, v.R, st)) != hipSuccess) return e;
  if (cmax && (e = launch_zero_fill(cmax, v.C, st)) != hipSuccess) return e;
  const int64_t ry = std::min<int64_t>(ceil_div(v.R, 64), 32768);
  hipLaunchKernelGGL(op_maxima_kernel, dim3((unsigned)ceil_div(v.C, 64), (unsigned)ry),
                     dim3(256), 0, st, v, reinterpret_cast<unsigned long long *>(rmax),
                     reinterpret_cast<unsigned long long *>(cmax));
  timer_end(st);
  return hipGetLastError();
}

// Slices of an operand with R rows (a multiple of 128, Rv of them valid) and
// K contraction indices whose row maxima are in m (block_maxima).
static hipError_t pack_with_maxima(const OpMap &om, int64_t Rv, int64_t R, int64_t K,
                                   const double *m, double *sig, int8_t *S8, hipStream_t st) {
  timer_begin("op_pack", st);
  hipLaunchKernelGGL(op_sigma_kernel, dim3((unsigned)ceil_div(R, 256)), dim3(256), 0, st,
                     reinterpret_cast<const unsigned long long *>(m), Rv, R, sig);
  launch_op_pack(om, R, K / kQC, sig, S8, st);
  timer_end(st);
  return hipGetLastError();
}

static MaxView max_view(const double *base, int64_t R, int64_t rblk, int64_t ldrb, int64_t ldr,
                        int64_t C, int64_t cblk, int64_t ldcb) {
  MaxView v;
  v.base = base;
  v.R = R;
  v.C = C;
  v.rblk = rblk;
  v.ldrb = ldrb;
  v.ldr = ldr;
  v.cblk = cblk;
  v.ldcb = ldcb;
  return v;
}

hipError_t launch_adj_sum(const double *P, int nseg, int64_t rows, int64_t ncol, int64_t zstride,
                          double *C, int64_t ldc, bool accumulate, hipStream_t st);

// C (+)= the exact int8 product of A (row panels SA, chunk stride nqcA, the
// product's contraction starting at A's chunk qcA) and B (SB, K / 32 chunks),
// over K in segments (i8_segments: at most kGemmSeg long for exact int32
// sums, more when the output has too few tiles for the chip). With one
// segment the product goes to C directly; with several they run side by side
// (blockIdx.y) into partial products in part, which launch_adj_sum adds in a
// fixed order.
static hipError_t i8_gemm(const int8_t *SA, const double *sigA, int64_t RA, int64_t nqcA,
                          int64_t qcA, const int8_t *SB, const double *sigB, int64_t RB,
                          int64_t K, int64_t M, int64_t Ncols, int64_t GP, int64_t nvalid,
                          double *C, int64_t ldc, bool accumulate, double *part,
                          int64_t part_doubles, hipStream_t st) {
  I8GemmArgs a;
  a.tA = RA / kI8Tile;
  a.nqc = K / kQC;
  a.nqcA = nqcA;
  a.qcA = qcA;
  a.M = M;
  a.Ncols = Ncols;
  a.GP = GP;
  a.nvalid = nvalid;
  a.ldc = ldc;
  a.zstride = 0;
  const int64_t grid = a.tA * (RB / kI8Tile);
  int64_t segc = 0;
  const int64_t nz = i8_segments(M, Ncols, K, segc);
  const int64_t ncol = adj_out_cols(Ncols, GP, nvalid);
  a.segc = segc;
  timer_begin("gemm_adj_i8", st);
  hipError_t e;
  if (nz == 1) {
    a.accumulate = accumulate ? 1 : 0;
    hipLaunchKernelGGL(i8_gemm_kernel, dim3((unsigned)grid), dim3(kI8Threads), 0, st, SA, sigA,
                       SB, sigB, a, C);
    e = hipGetLastError();
  } else if (part && nz * M * ncol <= part_doubles) {
    a.ldc = ncol;
    a.accumulate = 0;
    a.zstride = M * ncol;
    hipLaunchKernelGGL(i8_gemm_kernel, dim3((unsigned)grid, (unsigned)nz), dim3(kI8Threads), 0,
                       st, SA, sigA, SB, sigB, a, part);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_adj_sum(part, (int)nz, M, ncol, a.zstride, C, ldc, accumulate, st);
  } else {
    e = hipErrorInvalidValue;   // the plan sizes part for every product it makes
  }
  timer_end(st);
  return e;
}

hipError_t launch_backward_split(const Plan &pl, const Inputs &in, const BwdOut &o, void *ws,
                                 hipStream_t st) {
  hipError_t e;
  double *part = pl.gpart_doubles > 0 ? ws_d(ws, pl.off_gpart) : nullptr;   // split products
  const bool cavv = (pl.terms & 2) && pl.na > 0, ccav = (pl.terms & 4) && pl.na > 0;
  // gradients of eps and s cleared, G3 (with its eps / s parts) from the FP64
  // adjoint tiles
  if ((e = launch_adjoint_start_fp64(pl, in, o, ws, st)) != hipSuccess) return e;
  if ((e = launch_slices(pl, in, ws, cavv, st)) != hipSuccess) return e;
  // Memory: G rows and columns over (orbital, virtual) in groups of W = 64 ntv.
  // Products: a contraction over (orbital, virtual) runs over Wk = nv rounded
  // up to 32 per orbital (whole chunks, a block of orbitals a contiguous range
  // of them), and operand rows over (orbital, virtual) hold the nv valid ones
  // side by side, so the outputs are written densely.
  const int64_t W = pl.ntv * kPanel;
  const int64_t nv = pl.nv, Wk = round_up(pl.nv, kQC);
  const int64_t N2 = pl.na * W, N3 = pl.nc * kActPanel;
  const int64_t Npk = pl.nc * Wk, N2k = pl.na * Wk;
  const int64_t N3p = round_up(N3, kQC);
  const int64_t RA = round_up(pl.naux, kI8Tile);
  const int64_t big = (int64_t)1 << 40;
  double *pmax = ws_d(ws, pl.off_opmax);
  // maxima of an adjoint-tile block for its two operands (bit patterns in pmax,
  // which holds 32 max(RA, rbmax) doubles)
  const int64_t rbmax = std::max(round_up(pl.nc * pl.nv, kI8Tile),
                                 std::max(round_up(pl.na * pl.nv, kI8Tile),
                                          round_up(pl.nc * pl.na, kI8Tile)));
  double *rmx = pmax, *cmx = pmax + rbmax;
  double *sigA1 = ws_d(ws, pl.off_sigA1), *sigA2 = ws_d(ws, pl.off_sigA2);
  double *sigB = ws_d(ws, pl.off_sigB);
  int8_t *SA1 = ws_b(ws, pl.off_SA1), *SA2 = ws_b(ws, pl.off_SA2), *SB = ws_b(ws, pl.off_SB);
  const double *G3 = ws_d(ws, pl.off_g3);
  const int64_t ldcv = pl.nc * pl.nv;
  const int64_t nqcp = Npk / kQC;                // chunks of A1
  auto blk = [&](int64_t I, int64_t &b0, int64_t &nb) {
    b0 = I * pl.gb;
    nb = std::min(pl.gb, pl.nc - b0);
  };

  // A1 = B_cv with rows Q and contraction index (m, e)
  const OpMap Acv = op_map(in.B_cv, big, pl.naux, 0, ldcv, pl.naux, Wk, nv, nv, 1, Npk);
  if ((e = pack_operand(Acv, RA, Npk, sigA1, pmax, SA1, st)) != hipSuccess) return e;

  bool written = false;   // dB_cv holds a first product in every block
  if (cavv) {
    // A2 = B_av with contraction index (w, f)
    const OpMap Aav = op_map(in.B_av, big, pl.naux, 0, pl.na * nv, pl.naux, Wk, nv, nv, 1, N2k);
    if ((e = pack_operand(Aav, RA, N2k, sigA2, pmax, SA2, st)) != hipSuccess) return e;
    const double *G2 = ws_d(ws, pl.off_g2);
    for (int64_t I = 0; I < pl.ngb; ++I) {
      int64_t m0, mb;
      blk(I, m0, mb);
      // G2 rows of this block and the CAVV eps / s parts from slice-path integrals
      if ((e = launch_cavv_x_split(pl, ws, (int)m0, (int)mb, st)) != hipSuccess) return e;
      if ((e = launch_cavv_adj_epi(pl, in, o, ws, (int)m0, (int)mb, st)) != hipSuccess) return e;
      // dB_cv[Q][(m,e)] (+)= sum_(w,f) B_av[Q][(w,f)] G2[(m,e)][(w,f)], m in the block
      const int64_t RB = round_up(mb * nv, kI8Tile);
      const OpMap B2t = op_map(G2, nv, nv, W * N2, N2, mb * nv, Wk, nv, W, 1, N2k);
      if ((e = block_maxima(max_view(G2, mb * nv, nv, W * N2, N2, pl.na * nv, nv, W), rmx, cmx,
                            st)) != hipSuccess)
        return e;
      if ((e = pack_with_maxima(B2t, mb * nv, RB, N2k, rmx, sigB, SB, st)) != hipSuccess) return e;
      if ((e = i8_gemm(SA2, sigA2, RA, N2k / kQC, 0, SB, sigB, RB, N2k, pl.naux, mb * nv, nv, nv,
                       o.dB_cv + m0 * nv, ldcv, false, part, pl.gpart_doubles, st)) != hipSuccess)
        return e;
      // dB_av[Q][(w,f)] (+)= sum_(m,e) B_cv[Q][(m,e)] G2[(m,e)][(w,f)], m in the block
      const int64_t RB2 = round_up(pl.na * nv, kI8Tile);
      const OpMap B2 = op_map(G2, nv, nv, W, 1, pl.na * nv, Wk, nv, W * N2, N2, mb * Wk);
      if ((e = pack_with_maxima(B2, pl.na * nv, RB2, mb * Wk, cmx, sigB, SB, st)) != hipSuccess)
        return e;
      if ((e = i8_gemm(SA1, sigA1, RA, nqcp, m0 * Wk / kQC, SB, sigB, RB2, mb * Wk, pl.naux,
                       pl.na * nv, nv, nv, o.dB_av, pl.na * nv, I > 0, part, pl.gpart_doubles,
                       st)) != hipSuccess)
        return e;
    }
    written = true;
  } else if (o.dB_av) {
    if ((e = launch_zero_fill(o.dB_av, pl.naux * pl.na * pl.nv, st)) != hipSuccess) return e;
  }
  if (pl.terms & 1) {
    double *G = ws_d(ws, pl.off_gs);
    const int64_t T = (pl.ntv_s / 2) * (pl.ntv_s / 2 + 1) / 2;
    double *xs = ws_d(ws, pl.off_xs);
    int *ctr = reinterpret_cast<int *>(xs + (size_t)kSlicePersistWG * kSliceXsDoubles);
    for (int64_t I = 0; I < pl.ngb; ++I)
      for (int64_t J = I; J < pl.ngb; ++J) {
        int64_t i0, ni, j0, nj;
        blk(I, i0, ni);
        blk(J, j0, nj);
        // the block's adjoint tiles and its CCVV eps / s parts from slice-path integrals
        CcvvAdjI8Args a;
        a.nc = (int)pl.nc;
        a.nv = (int)pl.nv;
        a.ntv_s = (int)pl.ntv_s;
        a.nqc = pl.nqc;
        a.s = pl.s;
        a.slot_base = ccvv_block_slot(pl, I, J, T);
        a.W = W;
        a.ld = nj * W;
        a.r0 = (int)i0;
        a.nr = (int)ni;
        a.c0 = (int)j0;
        a.ncb = (int)nj;
        a.chk = pl.chk;
        const int64_t npair = (I == J) ? ni * (ni + 1) / 2 : ni * nj;
        const int64_t items = pairtile_grid(npair, pl.ntv_s / 2);
        const int64_t grid = items < kSlicePersistWG ? items : kSlicePersistWG;
        if ((e = launch_zero(reinterpret_cast<double *>(ctr), 4, st)) != hipSuccess) return e;
        timer_begin("ccvv_adj_i8", st);
        hipLaunchKernelGGL(ccvv_adj_i8_kernel, dim3((unsigned)grid), dim3(kI8Threads), 0, st,
                           ws_b(ws, pl.off_s8c), ws_d(ws, pl.off_sigc), ws_d(ws, pl.off_diag),
                           in.eps_c, in.eps_v, a, xs, ctr, o.deps_c, o.deps_v, o.ds, o.gE, G,
                           ws_d(ws, pl.off_slots));
        timer_end(st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t ld = nj * W;   // row length of the G block
        // dB_cv[Q][(j,b)] (+)= sum_(i,a) B_cv[Q][(i,a)] G[(i,a)][(j,b)]; block J is
        // first written by the pair (0, J)
        const int64_t RBj = round_up(nj * nv, kI8Tile);
        const OpMap Bn = op_map(G, nv, nv, W, 1, nj * nv, Wk, nv, W * ld, ld, ni * Wk);
        // Bn reads the block's columns, Bt (off the diagonal) its rows
        if ((e = block_maxima(max_view(G, ni * nv, nv, W * ld, ld, nj * nv, nv, W),
                              J > I ? rmx : nullptr, cmx, st)) != hipSuccess)
          return e;
        if ((e = pack_with_maxima(Bn, nj * nv, RBj, ni * Wk, cmx, sigB, SB, st)) != hipSuccess)
          return e;
        if ((e = i8_gemm(SA1, sigA1, RA, nqcp, i0 * Wk / kQC, SB, sigB, RBj, ni * Wk, pl.naux,
                         nj * nv, nv, nv, o.dB_cv + j0 * nv, ldcv, written || I > 0, part,
                         pl.gpart_doubles, st)) != hipSuccess)
          return e;
        if (J > I) {
          // dB_cv[Q][(i,a)] += sum_(j,b) B_cv[Q][(j,b)] G[(i,a)][(j,b)]
          const int64_t RBi = round_up(ni * nv, kI8Tile);
          const OpMap Bt = op_map(G, nv, nv, W * ld, ld, ni * nv, Wk, nv, W, 1, nj * Wk);
          if ((e = pack_with_maxima(Bt, ni * nv, RBi, nj * Wk, rmx, sigB, SB, st)) != hipSuccess)
            return e;
          if ((e = i8_gemm(SA1, sigA1, RA, nqcp, j0 * Wk / kQC, SB, sigB, RBi, nj * Wk, pl.naux,
                           ni * nv, nv, nv, o.dB_cv + i0 * nv, ldcv, true, part,
                           pl.gpart_doubles, st)) != hipSuccess)
            return e;
        }
      }
    written = true;
  }
  if (ccav) {
    // dB_cv[Q][(m,e)] += sum_(n,u) B_ca[Q][(n,u)] G3[(m,e)][(n,u)]
    const OpMap Aca = op_map(in.B_ca, big, pl.naux, 0, pl.nc * pl.na, pl.naux, kActPanel, pl.na,
                             pl.na, 1, N3);
    if ((e = pack_operand(Aca, RA, N3p, sigA2, pmax, SA2, st)) != hipSuccess) return e;
    const int64_t RB = round_up(pl.nc * nv, kI8Tile);
    const OpMap B3t = op_map(G3, nv, nv, W * N3, N3, pl.nc * nv, kActPanel, pl.na, kActPanel, 1,
                             N3);
    if ((e = block_maxima(max_view(G3, pl.nc * nv, nv, W * N3, N3, pl.nc * pl.na, pl.na,
                                   kActPanel),
                          rmx, cmx, st)) != hipSuccess)
      return e;
    if ((e = pack_with_maxima(B3t, pl.nc * nv, RB, N3p, rmx, sigB, SB, st)) != hipSuccess)
      return e;
    if ((e = i8_gemm(SA2, sigA2, RA, N3p / kQC, 0, SB, sigB, RB, N3p, pl.naux, pl.nc * nv, nv, nv,
                     o.dB_cv, ldcv, written, part, pl.gpart_doubles, st)) != hipSuccess)
      return e;
    written = true;
    // dB_ca[Q][(n,u)] = sum_(m,e) B_cv[Q][(m,e)] G3[(m,e)][(n,u)]
    const int64_t n3v = pl.nc * pl.na;
    const int64_t RB3 = round_up(n3v, kI8Tile);
    const OpMap B3 = op_map(G3, pl.na, pl.na, kActPanel, 1, n3v, Wk, nv, W * N3, N3, Npk);
    if ((e = pack_with_maxima(B3, n3v, RB3, Npk, cmx, sigB, SB, st)) != hipSuccess) return e;
    if ((e = i8_gemm(SA1, sigA1, RA, nqcp, 0, SB, sigB, RB3, Npk, pl.naux, n3v, pl.na, pl.na,
                     o.dB_ca, n3v, false, part, pl.gpart_doubles, st)) != hipSuccess)
      return e;
  } else if (o.dB_ca) {
    if ((e = launch_zero_fill(o.dB_ca, pl.naux * pl.nc * pl.na, st)) != hipSuccess) return e;
  }
  if (!written) {
    if ((e = launch_zero_fill(o.dB_cv, pl.naux * ldcv, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dsrg
