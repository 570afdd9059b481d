// Error-free int8 slice path (DSRG_SPLIT_OZAKI) of libdsrgdf (gfx950).
//
// Each column of B (one core or active orbital p and one virtual orbital e,
// a vector over the auxiliary index Q) is scaled by a power of two sigma with
// |B^Q_pe| < sigma and split into five round-to-nearest int8 slices,
//   B^Q_pe = sigma (s0 2^-6 + s1 2^-13 + s2 2^-20 + s3 2^-27 + s4 2^-34) + r,
// |s_k| <= 64, |r| <= sigma 2^-35 (the splitting of Ozaki, Ogita, Oishi and
// Rump, "Error-free transformations of matrix multiplication by using fast
// routines of matrix multiplication", 2012). A contraction over Q becomes
//   (pe|qf) = sigma_pe sigma_qf sum_L 2^(-12-7L) I_L,  I_L = sum_{k+l=L} sum_Q s_k s_l,
// kept for levels L <= 4 (15 slice products). Every I_L is an exact int32
// sum on the int8 matrix cores (|I_L| <= 5 * 4096 * naux < 2^31 for
// naux <= 100000), so the only error left is the dropped levels and the
// residual r. The self-pair diagonal (ia|ia) = sum_Q (B^Q_ia)^2, whose
// dropped terms all have one sign, is taken in FP64 instead.
#include "fp64_tiles.h"

namespace dsrg {

typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

static inline double *ws_d(void *ws, size_t off) {
  return reinterpret_cast<double *>(static_cast<char *>(ws) + off);
}
static inline int8_t *ws_b(void *ws, size_t off) {
  return reinterpret_cast<int8_t *>(static_cast<char *>(ws) + off);
}

// v_mfma_i32_32x32x32_i8: lane l supplies 16 bytes of row l % 32 of A (and of
// column l % 32 of B) for the k-range 16 (l / 32) .. +15; result register r
// of lane l holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
__device__ __forceinline__ i16v mfma_i8(i4v a, i4v b, i16v c) {
  return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Slicing. Slice panels: S8[(p * ntv + t)][qc][s][c][32 bytes] for a 64-column
// virtual panel t of orbital p, chunk qc of 32 auxiliary indices, slice s,
// column c; the two 16-byte halves of column c are swapped when (c >> 3) & 1
// (bank-conflict-free fragment reads). sig[(p * ntv * 64) + e] = sigma.
// ---------------------------------------------------------------------------
constexpr int kSlices = 5;
constexpr int kQC = 32;                                  // auxiliary indices per chunk
constexpr int kSlicePanelChunk = kSlices * kPanel * kQC; // bytes per (panel, chunk)

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
    if (e < nv && q < naux) x = B[(q * nrow + p) * nv + e] * inv * 64.0;
#pragma unroll
    for (int s = 0; s < kSlices; ++s) {
      const double r = rint(x);
      buf[s][j] = (int8_t)(int)r;
      x = (x - r) * 128.0;
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
// Pair tile on int8 slices, eight waves (two per SIMD) per workgroup.
// x = L0^T R0 and y = L1^T R1 over all auxiliary chunks for 64 x 64 tiles.
// Waves 0-3 (group 0) own the four 32 x 32 quadrants of x, waves 4-7 (group
// 1) those of y; each wave keeps its own five level accumulators. When only
// x is needed, group 1 takes every second auxiliary chunk of x instead and
// its exact int32 partial sums are added to group 0's at the end. A stage is
// four 10 KB panel-chunks (L0, R0, L1, R1 of one chunk, or L0, R0 of two
// chunks), double-buffered in LDS with one barrier per stage.
// ---------------------------------------------------------------------------
constexpr int kI8Threads = 512;
constexpr int kI8Lds = 2 * 4 * kSlicePanelChunk;   // bytes: two stages of four panel-chunks

struct I8Stage {
  static constexpr int PER = 4 * (kSlicePanelChunk / 16) / kI8Threads;   // 16-byte pieces
  static_assert(4 * (kSlicePanelChunk / 16) % kI8Threads == 0, "stage must split evenly");
  i4v r[PER];
  __device__ __forceinline__ void load(const int8_t *s0, const int8_t *s1, const int8_t *s2,
                                       const int8_t *s3) {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = threadIdx.x + k * kI8Threads;
      const int p = idx / (kSlicePanelChunk / 16), off = idx % (kSlicePanelChunk / 16);
      // select, not index: keeps the panel pointers in registers
      const int8_t *base = (p == 0) ? s0 : (p == 1) ? s1 : (p == 2) ? s2 : s3;
      r[k] = reinterpret_cast<const i4v *>(base)[off];
    }
  }
  __device__ __forceinline__ void store(int8_t *lds) const {
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int idx = threadIdx.x + k * kI8Threads;
      reinterpret_cast<i4v *>(lds)[idx] = r[k];
    }
  }
};

__device__ __forceinline__ i4v frag_i8(const int8_t *panel, int s, int row, int h) {
  const int off = (s * kPanel + row) * kQC + (((h ^ (row >> 3)) & 1) << 4);
  return *reinterpret_cast<const i4v *>(panel + off);
}

// 15 products of one 32 x 32 block into 5 level accumulators, ordered so that
// consecutive products go to different accumulators.
__device__ __forceinline__ void level_products(const i4v (&a)[kSlices], const i4v (&b)[kSlices],
                                               i16v (&acc)[kSlices]) {
#pragma unroll
  for (int k = 0; k < kSlices; ++k)
#pragma unroll
    for (int L = k; L < kSlices; ++L) acc[L] = mfma_i8(a[k], b[L - k], acc[L]);
}

// Asynchronous variant: chunks are copied global -> LDS directly
// (global_load_lds, 16 bytes per lane, no register staging) into a ring of
// kI8Ring stage buffers, kI8Ring - 1 stages ahead of the compute.
constexpr int kI8Ring = 4;
constexpr int kI8LdsRing = kI8Ring * 4 * kSlicePanelChunk;   // 160 KB

__device__ __forceinline__ void i8_issue_stage(const int8_t *s0, const int8_t *s1,
                                               const int8_t *s2, const int8_t *s3,
                                               int8_t *dst) {
  constexpr int PIECES = kSlicePanelChunk / 16;   // per panel-chunk
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 4 * PIECES / kI8Threads; ++k) {
    const int base = wave * 64 + k * kI8Threads;   // first piece of this wave (multiple of 64)
    const int p = base / PIECES, off = base % PIECES + lane;
    const int8_t *src = (p == 0) ? s0 : (p == 1) ? s1 : (p == 2) ? s2 : s3;
    __builtin_amdgcn_global_load_lds(
        reinterpret_cast<const void *>(src + off * 16),
        (__attribute__((address_space(3))) void *)(dst + base * 16), 16, 0, 0);
  }
}

template <bool NEED_Y>
__device__ __forceinline__ void i8_tiles_async(const int8_t *const *P, int64_t nqc, int8_t *lds,
                                               i16v (&acc)[kSlices], int g, int wr, int wc,
                                               int lane) {
  constexpr int64_t CH = kSlicePanelChunk;
  constexpr int BUF = 4 * kSlicePanelChunk;
  constexpr int STEP = NEED_Y ? 1 : 2;
  const int64_t nst = nqc / STEP;   // nqc is even
  const int row = lane & 31, h = lane >> 5;
  auto issue = [&](int64_t s) {
    const int64_t c0 = s * STEP;
    int8_t *dst = lds + (int)(s % kI8Ring) * BUF;
    if constexpr (NEED_Y)
      i8_issue_stage(P[0] + c0 * CH, P[1] + c0 * CH, P[2] + c0 * CH, P[3] + c0 * CH, dst);
    else
      i8_issue_stage(P[0] + c0 * CH, P[1] + c0 * CH, P[0] + (c0 + 1) * CH, P[1] + (c0 + 1) * CH,
                     dst);
  };
  for (int64_t s = 0; s < kI8Ring - 1 && s < nst; ++s) issue(s);
  __builtin_amdgcn_s_waitcnt(0xF70);   // vmcnt(0): stage 0 (and the others issued) landed
  __builtin_amdgcn_s_barrier();
  for (int64_t s = 0; s < nst; ++s) {
    const int8_t *L = lds + (int)(s % kI8Ring) * BUF + 2 * g * CH;
    i4v fa[kSlices], fb[kSlices];
#pragma unroll
    for (int k = 0; k < kSlices; ++k) {
      fa[k] = frag_i8(L, k, 32 * wr + row, h);
      fb[k] = frag_i8(L + CH, k, 32 * wc + row, h);
    }
    level_products(fa, fb, acc);
    // the ring slot of stage s + kI8Ring - 1 was last read in stage s - 1,
    // which every wave finished before the barrier that ended it
    if (s + kI8Ring - 1 < nst) {
      issue(s + kI8Ring - 1);
      // at most two later stages (10 copies per thread) may still be in flight
      __builtin_amdgcn_s_waitcnt(0xF7A);   // vmcnt(10)
    } else {
      __builtin_amdgcn_s_waitcnt(0xF70);   // vmcnt(0)
    }
    __builtin_amdgcn_s_barrier();
  }
}

template <bool NEED_Y>
__device__ __forceinline__ void i8_tiles(const int8_t *const *P, int64_t nqc, int8_t *lds,
                                         i16v (&acc)[kSlices], int g, int wr, int wc, int lane) {
  constexpr int64_t CH = kSlicePanelChunk;
  constexpr int BUF = 4 * kSlicePanelChunk;
  constexpr int STEP = NEED_Y ? 1 : 2;
  const int64_t nst = nqc / STEP;   // nqc is even
  const int row = lane & 31, h = lane >> 5;
  I8Stage st;
  auto fetch = [&](int64_t s) {
    const int64_t c0 = s * STEP;
    if constexpr (NEED_Y)
      st.load(P[0] + c0 * CH, P[1] + c0 * CH, P[2] + c0 * CH, P[3] + c0 * CH);
    else
      st.load(P[0] + c0 * CH, P[1] + c0 * CH, P[0] + (c0 + 1) * CH, P[1] + (c0 + 1) * CH);
  };
  fetch(0);
  st.store(lds);
  if (nst > 1) fetch(1);
  __syncthreads();
  int b = 0;
  for (int64_t s = 0; s < nst; ++s) {
    const int8_t *L = lds + b * BUF + 2 * g * CH;
    i4v fa[kSlices], fb[kSlices];
#pragma unroll
    for (int k = 0; k < kSlices; ++k) {
      fa[k] = frag_i8(L, k, 32 * wr + row, h);
      fb[k] = frag_i8(L + CH, k, 32 * wc + row, h);
    }
    level_products(fa, fb, acc);
    if (s + 1 < nst) {
      st.store(lds + (b ^ 1) * BUF);
      if (s + 2 < nst) fetch(s + 2);
    }
    __syncthreads();
    b ^= 1;
  }
}

// sum_L 2^(-12-7L) I_L, smallest level first
__device__ __forceinline__ double level_value(const i16v (&acc)[kSlices], int r) {
  double v = 0.0;
#pragma unroll
  for (int L = kSlices - 1; L >= 0; --L) v += ldexp((double)acc[L][r], -12 - 7 * L);
  return v;
}

// Row / column of result register r of this lane inside the 64 x 64 tile.
__device__ __forceinline__ int i8_row(int wr, int lane, int r) {
  return 32 * wr + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}
__device__ __forceinline__ int i8_col(int wc, int lane) { return 32 * wc + (lane & 31); }

// One pair-tile work item (classes as decode_ccvv) on slices. On return the
// group-0 waves hold x and y (FP64) of their quadrant (class 1: y = x^T,
// classes 2, 3: y = x); for class 0, T = lds viewed as double[64][65] still
// holds y[row][col] (it is not written after the last barrier).
__device__ __forceinline__ void i8_pair_compute(const int8_t *S8L, const int8_t *S8R,
                                                const double *sigL, const double *sigR,
                                                int64_t nqc, int ntv, int pi, int pj, int A,
                                                int B, int cls, int8_t *lds, double (&x)[16],
                                                double (&y)[16], int g, int wr, int wc,
                                                int lane) {
  const int64_t ps = nqc * (int64_t)kSlicePanelChunk;
  const int8_t *P[4] = {S8L + (int64_t)(pi * ntv + A) * ps, S8R + (int64_t)(pj * ntv + B) * ps,
                        S8R + (int64_t)(pj * ntv + A) * ps, S8L + (int64_t)(pi * ntv + B) * ps};
  i16v acc[kSlices];
#pragma unroll
  for (int L = 0; L < kSlices; ++L) acc[L] = i16v{};
  if (cls == 0)
    i8_tiles_async<true>(P, nqc, lds, acc, g, wr, wc, lane);
  else
    i8_tiles_async<false>(P, nqc, lds, acc, g, wr, wc, lane);
  const int wq = 2 * wr + wc;
  // group 1 holds the odd-chunk half of x when only x is needed: add it in
  int *Ti = reinterpret_cast<int *>(lds);   // [4][5][16][64] ints = 80 KB
  if (cls != 0 && g == 1) {
#pragma unroll
    for (int L = 0; L < kSlices; ++L)
#pragma unroll
      for (int r = 0; r < 16; ++r) Ti[((wq * kSlices + L) * 16 + r) * 64 + lane] = acc[L][r];
  }
  __syncthreads();
  if (cls != 0 && g == 0) {
#pragma unroll
    for (int L = 0; L < kSlices; ++L)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[L][r] += Ti[((wq * kSlices + L) * 16 + r) * 64 + lane];
  }
  __syncthreads();
  const int cb = i8_col(wc, lane);
  double (*T)[kPanel + 1] = reinterpret_cast<double (*)[kPanel + 1]>(lds);
  if (g == 0) {
    const double sB = sigR[(int64_t)pj * ntv * kPanel + B * kPanel + cb];
#pragma unroll
    for (int r = 0; r < 16; ++r)
      x[r] = sigL[(int64_t)pi * ntv * kPanel + A * kPanel + i8_row(wr, lane, r)] * sB *
             level_value(acc, r);
    if (cls == 1) {
#pragma unroll
      for (int r = 0; r < 16; ++r) T[i8_row(wr, lane, r)][cb] = x[r];
    }
  } else if (cls == 0) {
    const double sB = sigL[(int64_t)pi * ntv * kPanel + B * kPanel + cb];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ra = i8_row(wr, lane, r);
      T[ra][cb] = sigR[(int64_t)pj * ntv * kPanel + A * kPanel + ra] * sB * level_value(acc, r);
    }
  }
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int ra = i8_row(wr, lane, r);
      y[r] = (cls == 0) ? T[ra][cb] : (cls == 1) ? T[cb][ra] : x[r];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// CCVV on slices: same work list and epilogue as the FP64 kernel; the
// self-pair diagonal (i = j, a = b) uses the FP64 sum of squares.
// ---------------------------------------------------------------------------
struct CcvvI8Args {
  int nc, nv, ntv;
  int64_t nqc;
  double s;
  int64_t slot_base;
  int atomic_mode;
};

__global__ __launch_bounds__(512) void ccvv_i8_kernel(const int8_t *__restrict__ S8,
                                                      const double *__restrict__ sig,
                                                      const double *__restrict__ diag,
                                                      const double *__restrict__ eps_c,
                                                      const double *__restrict__ eps_v,
                                                      CcvvI8Args a, double *slots, double *acc) {
  __shared__ __attribute__((aligned(16))) int8_t lds[kI8LdsRing];
  const PairTile pt = decode_pairtile(blockIdx.x, (int64_t)a.nc * (a.nc + 1) / 2, a.ntv);
  if (pt.item < 0) return;
  const CcvvWork c = ccvv_work_from(pt, a.nc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = wave >> 2, wr = (wave >> 1) & 1, wc = wave & 1;
  double x[16], y[16];
  i8_pair_compute(S8, S8, sig, sig, a.nqc, a.ntv, c.i, c.j, c.A, c.B, c.cls, lds, x, y, g, wr,
                  wc, lane);
  double part = 0.0;
  if (g == 0) {
    const int bcol = c.B * kPanel + i8_col(wc, lane);
    const double eb = bcol < a.nv ? eps_v[bcol] : 0.0;
    const double eij = eps_c[c.i] + eps_c[c.j];
    if (bcol < a.nv) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int arow = c.A * kPanel + i8_row(wr, lane, r);
        if (arow >= a.nv) continue;
        double xv = x[r], yv = y[r];
        if (c.cls == 3 && arow == bcol) xv = yv = diag[(int64_t)c.i * a.ntv * kPanel + arow];
        const double R = reg_R(eij - (eps_v[arow] + eb), a.s);
        part += R * (xv * xv - xv * yv + yv * yv);
      }
    }
  }
  const double w = (c.cls == 0) ? 4.0 : (c.cls == 3 ? 1.0 : 2.0);
  const double t = block_sum_n<8>(part, reinterpret_cast<double *>(lds)) * w;
  emit_partial(t, slots, a.slot_base + pt.item, acc, a.atomic_mode);
}

// ---------------------------------------------------------------------------
// CAVV on slices, step 1: for core orbitals m0 .. m0+mb-1, all active u and
// virtual tile pairs A <= B, the FP64 integrals X^{mu}[e][f] = (me|uf) are
// written to Xb[(m - m0)][u][e][f] (row length ntv*64): block [A,B] from x and
// block [B,A] from y = X^{mu}[B,A]^T.
// ---------------------------------------------------------------------------
struct CavvXArgs {
  int na, nv, ntv;
  int64_t nqc;
  int m0, mb;
};

__global__ __launch_bounds__(512) void cavv_i8_x_kernel(const int8_t *__restrict__ S8c,
                                                        const int8_t *__restrict__ S8a,
                                                        const double *__restrict__ sigc,
                                                        const double *__restrict__ siga,
                                                        CavvXArgs a, double *__restrict__ Xb) {
  __shared__ __attribute__((aligned(16))) int8_t lds[kI8LdsRing];
  const PairTile pt = decode_pairtile(blockIdx.x, (int64_t)a.mb * a.na, a.ntv);
  if (pt.item < 0) return;
  const int u = (int)(pt.p % a.na), ml = (int)(pt.p / a.na);
  const int A = pt.A, B = pt.B;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = wave >> 2, wr = (wave >> 1) & 1, wc = wave & 1;
  double x[16], y[16];
  // pair (m, u): left panels from B_cv (m), right panels from B_av (u)
  i8_pair_compute(S8c, S8a, sigc, siga, a.nqc, a.ntv, a.m0 + ml, u, A, B, (A == B) ? 2 : 0,
                  lds, x, y, g, wr, wc, lane);
  const int64_t ld = (int64_t)a.ntv * kPanel;
  double *X = Xb + ((int64_t)ml * a.na + u) * ld * ld;
  if (g == 0) {
    const int cb = i8_col(wc, lane);
#pragma unroll
    for (int r = 0; r < 16; ++r)
      X[(int64_t)(A * kPanel + i8_row(wr, lane, r)) * ld + B * kPanel + cb] = x[r];
  }
  if (A != B) {
    // X^{mu}[f][e] for f in B, e in A equals y[e][f], still in LDS as T[e][f]
    const double (*T)[kPanel + 1] = reinterpret_cast<const double (*)[kPanel + 1]>(lds);
    for (int k = threadIdx.x; k < kPanel * kPanel; k += kI8Threads) {
      const int fr = k / kPanel, ec = k % kPanel;
      X[(int64_t)(B * kPanel + fr) * ld + A * kPanel + ec] = T[ec][fr];
    }
  }
}

// CAVV step 2: per (m, e, f), with X_u = (me|uf), X'_u = (mf|ue):
//   sum_uv Gamma_uv S(D_mu) R1(D_mv) X_u (2 X_v - X'_v), summed over all (e, f).
// One workgroup per (m, 64-row block of e, 256 columns f); X'_u is read from
// the mirrored rows through L2.
struct CavvEpiArgs {
  int na, nv, ntv;
  double s;
  int m0;
  int fchunks;
  int64_t slot_base;
  int atomic_mode;
};

template <int NA>
__global__ __launch_bounds__(256) void cavv_epi_kernel(const double *__restrict__ Xb,
                                                       const double *__restrict__ eps_c,
                                                       const double *__restrict__ eps_a,
                                                       const double *__restrict__ eps_v,
                                                       const double *__restrict__ gamma1,
                                                       CavvEpiArgs a, double *slots,
                                                       double *acc) {
  __shared__ double red[4];
  const int64_t ld = (int64_t)a.ntv * kPanel;
  const int64_t w = blockIdx.x;
  const int fch = (int)(w % a.fchunks);
  const int64_t rest = w / a.fchunks;
  const int eb = (int)(rest % a.ntv), ml = (int)(rest / a.ntv);
  const int f = fch * 256 + threadIdx.x;
  const double *X = Xb + (int64_t)ml * NA * ld * ld;
  double G[NA][NA], ea[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    ea[u] = eps_a[u];
#pragma unroll
    for (int v = 0; v < NA; ++v) G[u][v] = gamma1[u * NA + v];
  }
  const double em = eps_c[a.m0 + ml];
  double part = 0.0;
  if (f < a.nv) {
    const double ef = eps_v[f];
    for (int el = 0; el < kPanel; ++el) {
      const int e = eb * kPanel + el;
      if (e >= a.nv) break;
      const double base = em - (eps_v[e] + ef);
      double S[NA], R1[NA], Xv[NA], W[NA];
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        reg_S_R1(base + ea[u], a.s, S[u], R1[u]);
        Xv[u] = X[((int64_t)u * ld + e) * ld + f];
        W[u] = R1[u] * (2.0 * Xv[u] - X[((int64_t)u * ld + f) * ld + e]);
      }
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        double t = 0.0;
#pragma unroll
        for (int v = 0; v < NA; ++v) t += G[u][v] * W[v];
        part += S[u] * Xv[u] * t;
      }
    }
  }
  const double t = block_sum(part, red);
  emit_partial(t, slots, a.slot_base + blockIdx.x, acc, a.atomic_mode);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static hipError_t slice_one(const double *B, int64_t nrow, const Plan &pl, double *sig,
                            double *diag, int8_t *S8, double *scratch, hipStream_t st) {
  const int64_t ncol = nrow * pl.ntv * kPanel;
  double *pmax = scratch, *psum = scratch + kScaleGroups * ncol;
  timer_begin("slice_scale", st);
  hipLaunchKernelGGL(slice_scale_partial_kernel, dim3((unsigned)ceil_div(ncol, 256), kScaleGroups),
                     dim3(256), 0, st, B, nrow, pl.nv, pl.naux, pl.ntv, pmax, psum);
  hipLaunchKernelGGL(slice_scale_final_kernel, dim3((unsigned)ceil_div(ncol, 256)), dim3(256), 0,
                     st, pmax, psum, ncol, sig, diag);
  timer_end(st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  timer_begin("slice_pack", st);
  hipLaunchKernelGGL(slice_pack_kernel, dim3((unsigned)ceil_div(ncol * pl.nqc, 256)), dim3(256),
                     0, st, B, nrow, pl.nv, pl.naux, pl.ntv, pl.nqc, sig, S8);
  timer_end(st);
  return hipGetLastError();
}

template <int NA>
static hipError_t cavv_epi_na(const Plan &pl, const Inputs &in, void *ws, int m0, int mb,
                              hipStream_t st) {
  CavvEpiArgs a;
  a.na = (int)pl.na;
  a.nv = (int)pl.nv;
  a.ntv = (int)pl.ntv;
  a.s = pl.s;
  a.m0 = m0;
  a.fchunks = (int)ceil_div(pl.nv, 256);
  a.slot_base = pl.slot_base[1] + (int64_t)m0 * pl.ntv * a.fchunks;
  a.atomic_mode = pl.atomic_reduce ? 1 : 0;
  const int64_t nblk = (int64_t)mb * pl.ntv * a.fchunks;
  timer_begin("cavv_epi", st);
  hipLaunchKernelGGL((cavv_epi_kernel<NA>), dim3((unsigned)nblk), dim3(256), 0, st,
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
    a.ntv = (int)pl.ntv;
    a.nqc = pl.nqc;
    a.s = pl.s;
    a.slot_base = pl.slot_base[0];
    a.atomic_mode = pl.atomic_reduce ? 1 : 0;
    timer_begin("ccvv_i8", st);
    hipLaunchKernelGGL(ccvv_i8_kernel, dim3((unsigned)pairtile_grid(pl.nc * (pl.nc + 1) / 2, pl.ntv)), dim3(kI8Threads), 0, st,
                       ws_b(ws, pl.off_s8c), ws_d(ws, pl.off_sigc), ws_d(ws, pl.off_diag),
                       in.eps_c, in.eps_v, a, slots, acc + 0);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (cavv) {
    for (int64_t m0 = 0; m0 < pl.nc; m0 += pl.cavv_mb) {
      const int mb = (int)((pl.nc - m0) < pl.cavv_mb ? (pl.nc - m0) : pl.cavv_mb);
      CavvXArgs xa;
      xa.na = (int)pl.na;
      xa.nv = (int)pl.nv;
      xa.ntv = (int)pl.ntv;
      xa.nqc = pl.nqc;
      xa.m0 = (int)m0;
      xa.mb = mb;
      timer_begin("cavv_i8_x", st);
      hipLaunchKernelGGL(cavv_i8_x_kernel, dim3((unsigned)pairtile_grid((int64_t)mb * pl.na, pl.ntv)), dim3(kI8Threads), 0, st,
                         ws_b(ws, pl.off_s8c), ws_b(ws, pl.off_s8a), ws_d(ws, pl.off_sigc),
                         ws_d(ws, pl.off_siga), xa, ws_d(ws, pl.off_xb));
      timer_end(st);
      if ((e = hipGetLastError()) != hipSuccess) return e;
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
