// Int8 slice tiles shared by the slice-path kernels of libdsrgdf (gfx950):
// the slice panel layout, the pipelined 128 x 128 int8 tile product on the
// matrix cores and the FP64 recombination of its level sums.
#pragma once

#include "fp64_tiles.h"

namespace dsrg {

typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i16v __attribute__((ext_vector_type(16)));

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
constexpr int kSlices = 4;
constexpr int kQC = 32;                                  // auxiliary indices per chunk
constexpr int kSlicePanelChunk = kSlices * kPanel * kQC; // bytes per (panel, chunk)

// ---------------------------------------------------------------------------
// Int8 tile product, eight waves (two per SIMD) per workgroup.
// K[a][b] = sum_Q L^Q_a R^Q_b for a 128 x 128 output tile: rows from two
// 64-column slice panels (r0, r1), columns from two more (c0, c1). Wave w
// owns rows 64 (w >> 2) .. +63 (two 32-row blocks q = 0, 1) and columns
// 32 (w & 3) .. +31, with four int32 level accumulators per block (128
// registers). A stage is one 32-index auxiliary chunk of the four panels
// (4 x 8 KB); stages are copied global -> LDS directly (global_load_lds,
// 16 bytes per lane) into a ring of five, four stages ahead of the matrix
// cores.
// ---------------------------------------------------------------------------
constexpr int kI8Threads = 512;
constexpr int kI8Tile = 128;
constexpr int kI8Ring = 5;
constexpr int kI8Stage = 4 * kSlicePanelChunk;       // 32 KB
constexpr int kI8LdsRing = kI8Ring * kI8Stage;       // 160 KB
constexpr int kI8Blocks = 2;                         // 32 x 32 blocks per wave
constexpr int kI8Out = kI8Blocks * 16;               // outputs per lane
static_assert(kI8Threads * kI8Out == kSliceXsDoubles, "x slot size");
constexpr int kI8CopiesPerStage = 4 * (kSlicePanelChunk / 16) / kI8Threads;   // 4

__device__ __forceinline__ i4v frag_i8(const int8_t *panel, int s, int row, int h) {
  const int off = (s * kPanel + row) * kQC + (((h ^ (row >> 3)) & 1) << 4);
  return *reinterpret_cast<const i4v *>(panel + off);
}

// Copy one stage (four panel-chunks, in order s0..s3) into the LDS ring slot
// dst: one instruction per panel-chunk, wave w moving its 64 consecutive
// 16-byte pieces w * 1 KB .. +1 KB, so source base and LDS address are
// wave-uniform (scalar registers) with no per-copy selection.
__device__ __forceinline__ void i8_issue_stage(const int8_t *s0, const int8_t *s1,
                                               const int8_t *s2, const int8_t *s3,
                                               int8_t *dst) {
  static_assert(kSlicePanelChunk == kI8Threads * 16 && kI8CopiesPerStage == 4,
                "one copy instruction per panel-chunk");
  const int woff = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 1024;
  const uint32_t voff = (threadIdx.x & 63) * 16;
  const int8_t *src[4] = {s0, s1, s2, s3};
#pragma unroll
  for (int k = 0; k < 4; ++k)
    __builtin_amdgcn_global_load_lds(
        reinterpret_cast<const void *>(src[k] + woff + voff),
        (__attribute__((address_space(3))) void *)(dst + k * kSlicePanelChunk + woff), 16, 0,
        0);
}

// Ties a scalar value (a kernel argument) to this point: its scalar load
// completes before the K-loop, so no scalar load is in flight there and the
// loop's LDS waits can count outstanding reads instead of draining them.
template <class T>
__device__ __forceinline__ void scalar_here(const T &v) {
  asm volatile("" ::"s"(v));
}

// The K loop of one tile product through the LDS ring: rows from the slice
// panels (Ra, Rb), columns from (Ca, Cb), stages s = 0 .. nqc-1 of 32
// auxiliary indices each (a panel's chunks are consecutive).
//
// Products of one stage are taken in four rounds: round r multiplies row
// slice r with column slices 0 .. 3-r into the levels r .. 3, so two products
// into one accumulator are at least four instructions apart, and after round
// r the fragments of row slice r and column slice 3-r are dead: the next
// stage's copies of exactly those are read into them at once. The LDS reads
// of a stage thus overlap the matrix products of the previous one, which
// needs the next stage in LDS one stage earlier than the products do.
struct I8Stream {
  const int8_t *Ra, *Rb, *Ca, *Cb;   // next stage to copy
  int nqc;
  int8_t *lds;
  int wr, wc, row, h, cr;
  i4v fa[kI8Blocks][kSlices], fb[kSlices];

  __device__ __forceinline__ I8Stream(const int8_t *ra, const int8_t *rb, const int8_t *ca,
                                      const int8_t *cb, int nqc_, int8_t *lds_, int wr_,
                                      int wc_, int lane)
      : Ra(ra), Rb(rb), Ca(ca), Cb(cb), nqc(nqc_), lds(lds_), wr(wr_), wc(wc_),
        row(lane & 31), h(lane >> 5), cr(32 * (wc_ & 1) + (lane & 31)) {}

  // copies the next stage into the ring slot at byte offset slot
  __device__ __forceinline__ void issue(int slot) {
    i8_issue_stage(Ra, Rb, Ca, Cb, lds + slot);
    Ra += kSlicePanelChunk;
    Rb += kSlicePanelChunk;
    Ca += kSlicePanelChunk;
    Cb += kSlicePanelChunk;
  }
  static __device__ __forceinline__ int next_slot(int slot) {
    return slot + kI8Stage == kI8LdsRing ? 0 : slot + kI8Stage;
  }
  // fragments consumed in round r: row slice r, column slice 3 - r
  __device__ __forceinline__ void read_round(int slot, int r) {
    const int8_t *Lr = lds + slot + wr * kSlicePanelChunk;
    const int8_t *Lc = lds + slot + (2 + (wc >> 1)) * kSlicePanelChunk;
#pragma unroll
    for (int q = 0; q < kI8Blocks; ++q) fa[q][r] = frag_i8(Lr, r, 32 * q + row, h);
    fb[kSlices - 1 - r] = frag_i8(Lc, kSlices - 1 - r, cr, h);
  }

  __device__ __forceinline__ void run(i16v (&acc)[kI8Blocks][kSlices]) {
    int wslot = 0;
    for (int s = 0; s < kI8Ring - 1 && s < nqc; ++s) {
      issue(wslot);
      wslot += kI8Stage;
    }
    wait_vm<0>();
    ring_barrier();
    // same order as the reads inside the loop, so that the LDS counter
    // state entering the loop matches the one carried around it
#pragma unroll
    for (int r = 0; r < kSlices; ++r) {
      read_round(0, r);
      __builtin_amdgcn_sched_barrier(0);
    }
    int rslot = 0;
    for (int s = 0; s < nqc; ++s) {
      // the slot of stage s + 4 held stage s - 1, whose fragments were read
      // during stage s - 2 and consumed before the barrier that ended stage s - 1
      const bool more = s + kI8Ring - 1 < nqc;
      if (more) {
        issue(wslot);
        wslot = next_slot(wslot);
      }
      // fragments of stage s + 1 (a stale slot after the last stage: never used)
      const int nslot = next_slot(rslot);
#pragma unroll
      for (int r = 0; r < kSlices; ++r) {
#pragma unroll
        for (int Lv = kSlices - 1; Lv >= r; --Lv)
#pragma unroll
          for (int q = 0; q < kI8Blocks; ++q)
            acc[q][Lv] = mfma_i8(fa[q][r], fb[Lv - r], acc[q][Lv]);
        __builtin_amdgcn_sched_barrier(0);
        read_round(nslot, r);
        __builtin_amdgcn_sched_barrier(0);
      }
      // stage s + 2 must have landed (its fragments are read during stage
      // s + 1); stages s + 3 and s + 4 may still be in flight
      if (more)
        wait_vm<(kI8Ring - 3) * kI8CopiesPerStage>();
      else
        wait_vm<0>();
      ring_barrier();
      rslot = nslot;
    }
  }
};

__device__ __forceinline__ void i8_clear(i16v (&acc)[kI8Blocks][kSlices]) {
#pragma unroll
  for (int q = 0; q < kI8Blocks; ++q)
#pragma unroll
    for (int L = 0; L < kSlices; ++L) acc[q][L] = i16v{};
}

// One tile product: rows from panels (r0, r1), columns from (c0, c1).
__device__ __forceinline__ void i8_tile_product(const int8_t *r0, const int8_t *r1,
                                                const int8_t *c0, const int8_t *c1, int nqc,
                                                int8_t *lds, i16v (&acc)[kI8Blocks][kSlices],
                                                int wr, int wc, int lane) {
  I8Stream st(r0, r1, c0, c1, nqc, lds, wr, wc, lane);
  i8_clear(acc);
  st.run(acc);
}

// sum_L w_L I_L with w_L = 1 / (127^2 254^L), smallest level first (Horner)
__device__ __forceinline__ double level_value(const i16v (&acc)[kSlices], int r) {
  double v = (double)acc[kSlices - 1][r];
#pragma unroll
  for (int L = kSlices - 2; L >= 0; --L) v = v * (1.0 / 254.0) + (double)acc[L][r];
  return v * (1.0 / 16129.0);
}

// Row / column inside the 128 x 128 tile of output r of block q of this lane.
__device__ __forceinline__ int i8_row(int wr, int q, int lane, int r) {
  return 64 * wr + 32 * q + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}
__device__ __forceinline__ int i8_col(int wc, int q, int lane) {
  (void)q;
  return 32 * wc + (lane & 31);
}

// FP64 values of block q: v[r] = sig_row[row] sig_col[col] K[row][col].
__device__ __forceinline__ void i8_block_values(const i16v (&acc)[kSlices], const double *sig_row,
                                                const double *sig_col, int wr, int wc, int q,
                                                int lane, double (&v)[16]) {
  const double sc = sig_col[i8_col(wc, q, lane)];
#pragma unroll
  for (int r = 0; r < 16; ++r)
    v[r] = sig_row[i8_row(wr, q, lane, r)] * sc * level_value(acc, r);
}

// Slice panel t (64 columns) of orbital p; sigma of its first column.
__device__ __forceinline__ const int8_t *slice_panel(const int8_t *S8, int64_t p, int64_t t,
                                                     int64_t ntv_s, int64_t nqc) {
  return S8 + (p * ntv_s + t) * nqc * (int64_t)kSlicePanelChunk;
}

// Integrals of one CCVV slice item (the work list of decode_ccvv_list). Pass 0
// forms x = K^{ij}[A,B] (rows from i's A panels, columns from j's B panels);
// a class-0 item parks x in its workgroup slot xw (lane-private layout
// xw[(q 16 + r) 512]) and takes pass 1, y[a][b] = (ja|ib). On return v holds
// the FP64 values of the last product (class 0: y, else x); the level
// accumulators are dead, so the epilogue has the registers to itself.
__device__ __forceinline__ void ccvv_i8_item(const int8_t *S8, const double *sig,
                                             const CcvvWork &c, int64_t nqc, int ntv_s,
                                             int8_t *lds, double *xw, int wr, int wc, int lane,
                                             double (&v)[kI8Out]) {
  const int64_t ldv = (int64_t)ntv_s * kPanel;
  const double *sri = sig + c.i * ldv + c.A * kI8Tile, *scj = sig + c.j * ldv + c.B * kI8Tile;
  const double *srj = sig + c.j * ldv + c.A * kI8Tile, *sci = sig + c.i * ldv + c.B * kI8Tile;
  const int64_t ps = nqc * (int64_t)kSlicePanelChunk;
  i16v ac[kI8Blocks][kSlices];
  const int npass = (c.cls == 0) ? 2 : 1;
  for (int pass = 0; pass < npass; ++pass) {
    const int8_t *r0 = slice_panel(S8, pass ? c.j : c.i, 2 * c.A, ntv_s, nqc);
    const int8_t *c0 = slice_panel(S8, pass ? c.i : c.j, 2 * c.B, ntv_s, nqc);
    i8_tile_product(r0, r0 + ps, c0, c0 + ps, (int)nqc, lds, ac, wr, wc, lane);
    if (pass + 1 < npass) {
#pragma unroll
      for (int q = 0; q < kI8Blocks; ++q) {
        double t[16];
        i8_block_values(ac[q], sri, scj, wr, wc, q, lane, t);
#pragma unroll
        for (int r = 0; r < 16; ++r) xw[(q * 16 + r) * kI8Threads] = t[r];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kI8Blocks; ++q) {
    double t[16];
    if (c.cls == 0)
      i8_block_values(ac[q], srj, sci, wr, wc, q, lane, t);
    else
      i8_block_values(ac[q], sri, scj, wr, wc, q, lane, t);
#pragma unroll
    for (int r = 0; r < 16; ++r) v[q * 16 + r] = t[r];
  }
}

}  // namespace dsrg
