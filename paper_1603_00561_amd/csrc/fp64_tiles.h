// FP64 tile machinery shared by the forward and adjoint kernels: staging of
// packed panel chunks through LDS, the double-buffered K loop over the
// auxiliary index, and the FP64 matrix-core fragment helpers (gfx950).
#pragma once

#include "common_device.h"
#include "internal.h"

namespace dsrg {

// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// result register r of lane l holds D[4 r + l / 16][l % 16] (rows interleaved
// by four, unlike the FP32-output shapes).
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ d4 zero4() { return d4{0.0, 0.0, 0.0, 0.0}; }

// LDS rows of W doubles hold one auxiliary index each. For W a multiple of
// 32, the 16-column halves of odd rows are swapped (column c of row k lives at c ^ swz(k)), so the two
// rows that one 32-lane half of a fragment read touches land in different
// bank halves without padding.
__device__ __forceinline__ int swz(int k) { return (k & 1) << 4; }

// NP panel chunks of KC rows x W doubles, global row stride ld, copied
// global -> registers -> LDS by all 256 threads with 16-byte accesses.
template <int NP, int W, int KC>
struct Stage {
  static constexpr int N2 = KC * W / 2;                         // double2 per chunk
  static constexpr int PER = (N2 + kThreads - 1) / kThreads;    // per thread
  d2v r[NP][PER];

  __device__ __forceinline__ void load(const double *const *src, int64_t ld, int64_t q0) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = threadIdx.x + k * kThreads;
        if (N2 % kThreads == 0 || idx < N2) {
          const int row = idx / (W / 2);
          const int c2 = idx % (W / 2);
          r[p][k] = *reinterpret_cast<const d2v *>(src[p] + (q0 + row) * ld + 2 * c2);
        }
      }
    }
  }
  // buf: NP consecutive [KC][W] blocks
  __device__ __forceinline__ void store(double *buf) const {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = threadIdx.x + k * kThreads;
        if (N2 % kThreads == 0 || idx < N2) {
          const int row = idx / (W / 2);
          const int c2 = idx % (W / 2);
          const int col = (W % 32 == 0) ? ((2 * c2) ^ swz(row)) : 2 * c2;
          *reinterpret_cast<d2v *>(&buf[(p * KC + row) * W + col]) = r[p][k];
        }
      }
    }
  }
};

// Column of row k in an LDS panel of width W (matches Stage::store).
template <int W>
__device__ __forceinline__ int lcol(int c, int k) {
  return (W % 32 == 0) ? (c ^ swz(k)) : c;
}

// Double-buffered K loop: lds holds 2 * NP * KC * W doubles. compute(L) is
// called once per chunk with L = the NP staged [KC][W] panels. While it
// runs, chunk c+1 waits in registers and is then written to the other
// buffer, and chunk c+2 is fetched; one barrier per chunk. Ends on a barrier.
template <int NP, int W, int KC, typename F>
__device__ __forceinline__ void kloop(const double *const *src, int64_t ld, int64_t naux_p,
                                      double *lds, F &&compute) {
  static_assert(kChunk % KC == 0, "chunks must tile naux_p, a multiple of kChunk");
  constexpr int BUF = NP * KC * W;
  Stage<NP, W, KC> st;
  st.load(src, ld, 0);
  st.store(lds);
  if (naux_p > KC) st.load(src, ld, KC);
  __syncthreads();
  int b = 0;
  for (int64_t q0 = 0; q0 < naux_p; q0 += KC) {
    compute(static_cast<const double *>(lds + b * BUF));
    if (q0 + KC < naux_p) {
      st.store(lds + (b ^ 1) * BUF);
      if (q0 + 2 * KC < naux_p) st.load(src, ld, q0 + 2 * KC);
    }
    __syncthreads();
    b ^= 1;
  }
}

// ---------------------------------------------------------------------------
// CCVV tile pair: x = K^{ij}[A,B] = B_iA^T B_jB, y = K^{ji}[A,B] = B_jA^T B_iB
// on a 64 x 64 tile, each wave owning a 32 x 32 quadrant (wr, wc).
// src = {B_iA, B_jB, B_jA, B_iB} packed panels.
// ---------------------------------------------------------------------------
struct CcvvWork {
  int i, j, A, B, cls;   // cls 0: i<j,A<B  1: i<j,A=B  2: i=j,A<B  3: i=j,A=B
};

__device__ __forceinline__ CcvvWork decode_ccvv(int64_t w, int nc, int ntv, int64_t n0,
                                                int64_t n1, int64_t n2) {
  CcvvWork c;
  const int64_t ntp_lt = (int64_t)ntv * (ntv - 1) / 2;
  if (w < n0) {
    decode_pair_lt(w / ntp_lt, nc, c.i, c.j);
    decode_pair_lt(w % ntp_lt, ntv, c.A, c.B);
    c.cls = 0;
  } else if ((w -= n0) < n1) {
    decode_pair_lt(w / ntv, nc, c.i, c.j);
    c.A = c.B = (int)(w % ntv);
    c.cls = 1;
  } else if ((w -= n1) < n2) {
    c.i = c.j = (int)(w / ntp_lt);
    decode_pair_lt(w % ntp_lt, ntv, c.A, c.B);
    c.cls = 2;
  } else {
    w -= n2;
    c.i = c.j = (int)(w / ntv);
    c.A = c.B = (int)(w % ntv);
    c.cls = 3;
  }
  return c;
}

// Pair-tile schedule. Items are (pair p, virtual tile pair A <= B) for P pairs
// and T = ntv (ntv + 1) / 2 tile pairs. Workgroup b runs on XCD b % 8 (the
// hardware deals workgroups round-robin over the eight XCDs); pairs are
// dealt to XCDs round-robin too, so the eight XCDs work on eight consecutive
// pairs at a time (sharing one core orbital), and each XCD walks the tile
// pairs of its pair in 4 x 4 blocks so that concurrent workgroups share
// panels in its L2. Item id = p * T + t (its slot); grid = 8 ceil(P/8) T.
constexpr int kTileBlock = 4;

__device__ __forceinline__ void decode_tile_blocked(int64_t t, int ntv, int &A, int &B) {
  const int nb = (ntv + kTileBlock - 1) / kTileBlock;
  for (int ba = 0; ba < nb; ++ba) {
    const int na_ = (ba == nb - 1) ? ntv - ba * kTileBlock : kTileBlock;
    for (int bb = ba; bb < nb; ++bb) {
      const int nb_ = (bb == nb - 1) ? ntv - bb * kTileBlock : kTileBlock;
      const int64_t size = (ba == bb) ? (int64_t)na_ * (na_ + 1) / 2 : (int64_t)na_ * nb_;
      if (t < size) {
        int a0, b0;
        if (ba == bb) {
          decode_pair_le(t, na_, a0, b0);
        } else {
          a0 = (int)(t / nb_);
          b0 = (int)(t % nb_);
        }
        A = ba * kTileBlock + a0;
        B = bb * kTileBlock + b0;
        return;
      }
      t -= size;
    }
  }
  A = B = 0;   // not reached for t < T
}

struct PairTile {
  int64_t item;   // p * T + t, or -1 when this workgroup has no item
  int64_t p;
  int A, B;
};

__device__ __forceinline__ PairTile decode_pairtile(int64_t bid, int64_t P, int ntv) {
  const int64_t T = (int64_t)ntv * (ntv + 1) / 2;
  const int64_t x = bid % 8, k = bid / 8;
  const int64_t lp = k / T, t = k % T;
  PairTile r;
  r.p = lp * 8 + x;
  if (r.p >= P) {
    r.item = -1;
    r.A = r.B = 0;
    return r;
  }
  r.item = r.p * T + t;
  decode_tile_blocked(t, ntv, r.A, r.B);
  return r;
}

__host__ __device__ inline int64_t pairtile_grid(int64_t P, int64_t ntv) {
  return 8 * ((P + 7) / 8) * (ntv * (ntv + 1) / 2);
}

__device__ __forceinline__ CcvvWork ccvv_work_from(const PairTile &pt, int nc) {
  CcvvWork c;
  decode_pair_le(pt.p, nc, c.i, c.j);
  c.A = pt.A;
  c.B = pt.B;
  c.cls = (c.i == c.j) ? (c.A == c.B ? 3 : 2) : (c.A == c.B ? 1 : 0);
  return c;
}

// Blocked walk (kTileBlock x kTileBlock blocks) over the strictly ordered
// tile pairs A < B of nt tiles.
__device__ __forceinline__ void decode_tile_blocked_lt(int64_t t, int nt, int &A, int &B) {
  const int nb = (nt + kTileBlock - 1) / kTileBlock;
  for (int ba = 0; ba < nb; ++ba) {
    const int na_ = (ba == nb - 1) ? nt - ba * kTileBlock : kTileBlock;
    for (int bb = ba; bb < nb; ++bb) {
      const int nb_ = (bb == nb - 1) ? nt - bb * kTileBlock : kTileBlock;
      const int64_t size = (ba == bb) ? (int64_t)na_ * (na_ - 1) / 2 : (int64_t)na_ * nb_;
      if (t < size) {
        int a0, b0;
        if (ba == bb) {
          decode_pair_lt(t, na_, a0, b0);
        } else {
          a0 = (int)(t / nb_);
          b0 = (int)(t % nb_);
        }
        A = ba * kTileBlock + a0;
        B = bb * kTileBlock + b0;
        return;
      }
      t -= size;
    }
  }
  A = B = 0;   // not reached for t < nt (nt - 1) / 2
}

// Work list of the persistent CCVV kernels (nt tiles per orbital) on XCD x (pairs p = x mod 8; pairs
// 0 .. P0-1 are the i < j pairs in order, P0 + i the self pairs), item kk:
// first every class-0 item (two products each) of its i < j pairs, then the
// single-product items (class 1 of its i < j pairs, classes 2 and 3 of its
// self pairs). The workgroups of one XCD take consecutive items, so each
// round holds items of equal cost that share panels and stay in step along
// the auxiliary index. slot = p T + (index of A <= B). Returns false past
// the end of the list.
__device__ __forceinline__ bool decode_ccvv_list(int64_t kk, int x, int nc, int nt, CcvvWork &c,
                                               int64_t &slot) {
  const int64_t P0 = (int64_t)nc * (nc - 1) / 2;
  const int64_t T0 = (int64_t)nt * (nt - 1) / 2, T = (int64_t)nt * (nt + 1) / 2;
  const int64_t nlt = (P0 > x) ? (P0 - x + 7) / 8 : 0;
  const int64_t first_eq = P0 + ((x - P0 % 8) + 8) % 8;   // first self pair on this XCD
  const int64_t neq = (first_eq < P0 + nc) ? (P0 + nc - first_eq + 7) / 8 : 0;
  int64_t p;
  if (kk < nlt * T0) {
    p = 8 * (kk / T0) + x;
    decode_tile_blocked_lt(kk % T0, nt, c.A, c.B);
    c.cls = 0;
  } else if ((kk -= nlt * T0) < nlt * nt) {
    p = 8 * (kk / nt) + x;
    c.A = c.B = (int)(kk % nt);
    c.cls = 1;
  } else if ((kk -= nlt * nt) < neq * T) {
    p = first_eq + 8 * (kk / T);
    decode_tile_blocked(kk % T, nt, c.A, c.B);
    c.cls = (c.A == c.B) ? 3 : 2;
  } else {
    return false;
  }
  if (p < P0) {
    decode_pair_lt(p, nc, c.i, c.j);
  } else {
    c.i = c.j = (int)(p - P0);
  }
  slot = p * T + (int64_t)c.A * nt - (int64_t)c.A * (c.A - 1) / 2 + (c.B - c.A);
  return true;
}


// The same work list over the core pairs of one block pair of core orbitals
// (rows r0 .. r0+nr-1, columns c0 .. c0+ncb-1): a diagonal block (r0 == c0)
// has the i < j pairs inside it and its self pairs, an off-diagonal block
// (r0 + nr <= c0) the nr ncb pairs i < j across. slot counts from the block
// pair's first item.
__device__ __forceinline__ bool decode_ccvv_block_list(int64_t kk, int x, int r0, int nr, int c0,
                                                       int ncb, int nt, CcvvWork &c,
                                                       int64_t &slot) {
  const bool diag = r0 == c0;
  const int64_t P0 = diag ? (int64_t)nr * (nr - 1) / 2 : (int64_t)nr * ncb;
  const int64_t nself = diag ? nr : 0;
  const int64_t T0 = (int64_t)nt * (nt - 1) / 2, T = (int64_t)nt * (nt + 1) / 2;
  const int64_t nlt = (P0 > x) ? (P0 - x + 7) / 8 : 0;
  const int64_t first_eq = P0 + ((x - P0 % 8) + 8) % 8;   // first self pair on this XCD
  const int64_t neq = (first_eq < P0 + nself) ? (P0 + nself - first_eq + 7) / 8 : 0;
  int64_t p;
  if (kk < nlt * T0) {
    p = 8 * (kk / T0) + x;
    decode_tile_blocked_lt(kk % T0, nt, c.A, c.B);
    c.cls = 0;
  } else if ((kk -= nlt * T0) < nlt * nt) {
    p = 8 * (kk / nt) + x;
    c.A = c.B = (int)(kk % nt);
    c.cls = 1;
  } else if ((kk -= nlt * nt) < neq * T) {
    p = first_eq + 8 * (kk / T);
    decode_tile_blocked(kk % T, nt, c.A, c.B);
    c.cls = (c.A == c.B) ? 3 : 2;
  } else {
    return false;
  }
  if (p < P0) {
    if (diag) {
      int il, jl;
      decode_pair_lt(p, nr, il, jl);
      c.i = r0 + il;
      c.j = r0 + jl;
    } else {
      c.i = r0 + (int)(p / ncb);
      c.j = c0 + (int)(p % ncb);
    }
  } else {
    c.i = c.j = r0 + (int)(p - P0);
  }
  slot = p * T + (int64_t)c.A * nt - (int64_t)c.A * (c.A - 1) / 2 + (c.B - c.A);
  return true;
}

// Work list of a persistent producer over P pairs (all distinct) and tile
// pairs A <= B of nt tiles, on XCD x (pairs p = x mod 8): first the A < B
// items (two products) of its pairs, then the A = B items. Returns false past
// the end of the list.
__device__ __forceinline__ bool decode_pair_list(int64_t kk, int x, int64_t P, int nt,
                                                 int64_t &p, int &A, int &B) {
  const int64_t T0 = (int64_t)nt * (nt - 1) / 2;
  const int64_t np = (P > x) ? (P - x + 7) / 8 : 0;
  if (kk < np * T0) {
    p = 8 * (kk / T0) + x;
    decode_tile_blocked_lt(kk % T0, nt, A, B);
    return true;
  }
  kk -= np * T0;
  if (kk < np * nt) {
    p = 8 * (kk / nt) + x;
    A = B = (int)(kk % nt);
    return true;
  }
  return false;
}

// Workgroup barrier that does not drain the vector-memory counter (a ring of
// direct global -> LDS copies waits for its copies explicitly); the empty asm
// keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void ring_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// s_waitcnt with only the vector-memory count (expcnt, lgkmcnt not waited)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// CCVV / CAVV tile K loop: chunks of kCcvvKC auxiliary indices of up to four
// 64-column panels are copied global -> LDS directly (global_load_lds, 16
// bytes per lane: a panel chunk of 8 rows x 512 B is one copy per thread, each
// wave moving its 1 KB quarter) into a ring of kCcvvRing slots, two chunks
// ahead of the matrix cores, with one barrier per chunk and no staging
// registers. LDS rows are stored as in memory (row k of panel p of a slot at
// (p kCcvvKC + k) 64): a fragment read takes 16 consecutive doubles of a row
// per 16 lanes.
constexpr int kCcvvKC = 8;
constexpr int kCcvvRing = 3;
constexpr int kCcvvStage = 4 * kCcvvKC * kPanel;   // doubles per slot
// the ring, or a 64 x 65 transpose tile
constexpr int kCcvvLds = (kCcvvRing * kCcvvStage > kPanel * (kPanel + 1))
                             ? kCcvvRing * kCcvvStage
                             : kPanel * (kPanel + 1);   // doubles
static_assert(kChunk % kCcvvKC == 0, "chunks must tile naux_p, a multiple of kChunk");

// One 16-byte global -> LDS copy per lane: lane l of the wave writes LDS
// bytes lds + 16 l .. +15 (lds wave-uniform). Written out rather than through
// the builtin, which makes the compiler drain every outstanding copy before
// any LDS read it cannot prove disjoint, i.e. before each chunk of the ring;
// the ring's own vector-memory waits and barriers order the copies and the
// reads. No register receives data (the copy writes LDS only), and the
// compiler's own vector-memory waits stay conservative: untracked copies can
// only make them wait longer.
__device__ __forceinline__ void lds_copy16(const void *g, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(g), "s"(lds)
               : "memory", "m0");
}

// copies chunk q0 of the NP panels src[] into the ring slot at lds
template <int NP>
__device__ __forceinline__ void ccvv_issue(const double *const *src, int64_t q0, double *slot) {
  static_assert(kCcvvKC * kPanel * 8 == kThreads * 16, "a panel chunk is one copy per thread");
  const int woff = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * 1024;
  const uint32_t voff = (threadIdx.x & 63) * 16;
  const uint32_t base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) char *)slot;
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    const char *g = reinterpret_cast<const char *>(src[p] + q0 * kPanel) + woff + voff;
    lds_copy16(g, __builtin_amdgcn_readfirstlane(base + p * kCcvvKC * kPanel * 8 + woff));
  }
}

// Computes ax (and ay for class 0); classes 1-3 derive ay afterwards. EDGE:
// a tile whose rows (ra of 64) or columns (rb of 64) run past nv, the last
// virtual panel; a wave then multiplies only its 16 x 16 blocks that hold a
// valid row and column (bit p of pm, bit q of qm; the others stay zero, as
// the zero padding would have left them). Ends on a barrier (LDS free).
template <bool NEED_Y, bool EDGE>
__device__ __forceinline__ void ccvv_tiles(const double *const *src, int64_t naux_p,
                                           double *lds, d4 (&ax)[2][2], d4 (&ay)[2][2],
                                           int wr, int wc, int cl, int kl, int pm, int qm) {
  constexpr int W = kPanel, KC = kCcvvKC, R = kCcvvRing;
  constexpr int NP = NEED_Y ? 4 : 2;
  const int64_t nst = naux_p / KC;
  for (int s = 0; s < R - 1 && s < nst; ++s) ccvv_issue<NP>(src, (int64_t)s * KC, lds + s * kCcvvStage);
  int slot = 0;
  for (int64_t s = 0; s < nst; ++s) {
    // chunk s has landed (this wave's copies; the barrier: everyone's), and
    // every wave is done with chunk s - 1, whose slot takes chunk s + R - 1
    if (s + 1 < nst)
      wait_vm<(R - 2) * NP>();
    else
      wait_vm<0>();
    ring_barrier();
    if (s + R - 1 < nst) {
      const int ns = (slot + R - 1) % R;
      ccvv_issue<NP>(src, (s + R - 1) * KC, lds + ns * kCcvvStage);
    }
    const double *L = lds + slot * kCcvvStage;
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int k = kk * 4 + kl;
      double fa[2], fb[2], ga[2], gb[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) fa[p] = L[(0 * KC + k) * W + 32 * wr + 16 * p + cl];
#pragma unroll
      for (int q = 0; q < 2; ++q) fb[q] = L[(1 * KC + k) * W + 32 * wc + 16 * q + cl];
      if constexpr (NEED_Y) {
#pragma unroll
        for (int p = 0; p < 2; ++p) ga[p] = L[(2 * KC + k) * W + 32 * wr + 16 * p + cl];
#pragma unroll
        for (int q = 0; q < 2; ++q) gb[q] = L[(3 * KC + k) * W + 32 * wc + 16 * q + cl];
      }
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (EDGE && !((pm >> p) & (qm >> q) & 1)) continue;
          ax[p][q] = mfma64(fa[p], fb[q], ax[p][q]);
          if constexpr (NEED_Y) ay[p][q] = mfma64(ga[p], gb[q], ay[p][q]);
        }
    }
    slot = (slot + 1 == R) ? 0 : slot + 1;
  }
  __syncthreads();
}

// Full x, y for one CCVV work item (x^T through LDS for class 1, y = x for
// classes 2 and 3). Leaves LDS free (ends on a barrier).
// PL holds the panels of orbital c.i, PR those of orbital c.j (both Pcv for
// CCVV; Pcv and Pav for the CAVV integrals (me|uf)).
__device__ __forceinline__ void ccvv_compute(const double *PL, const double *PR, int64_t naux_p,
                                             int ntv, int nv, const CcvvWork &c, double *lds,
                                             d4 (&ax)[2][2], d4 (&ay)[2][2], int wr, int wc,
                                             int cl, int kl) {
  constexpr int W = kPanel;
  const int64_t pstride = naux_p * W;
  const double *src[4] = {PL + (int64_t)(c.i * ntv + c.A) * pstride,
                          PR + (int64_t)(c.j * ntv + c.B) * pstride,
                          PR + (int64_t)(c.j * ntv + c.A) * pstride,
                          PL + (int64_t)(c.i * ntv + c.B) * pstride};
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ax[p][q] = zero4();
      ay[p][q] = zero4();
    }
  // valid rows / columns of the tile, and this wave's 16-blocks that hold any
  const int ra = nv - W * c.A, rb = nv - W * c.B;
  if (ra >= W && rb >= W) {
    if (c.cls == 0)
      ccvv_tiles<true, false>(src, naux_p, lds, ax, ay, wr, wc, cl, kl, 3, 3);
    else
      ccvv_tiles<false, false>(src, naux_p, lds, ax, ay, wr, wc, cl, kl, 3, 3);
  } else {
    // wave-uniform (wr, wc are): scalar branches around the matrix products
    const int pm = __builtin_amdgcn_readfirstlane((32 * wr < ra ? 1 : 0) | (32 * wr + 16 < ra ? 2 : 0));
    const int qm = __builtin_amdgcn_readfirstlane((32 * wc < rb ? 1 : 0) | (32 * wc + 16 < rb ? 2 : 0));
    if (c.cls == 0)
      ccvv_tiles<true, true>(src, naux_p, lds, ax, ay, wr, wc, cl, kl, pm, qm);
    else
      ccvv_tiles<false, true>(src, naux_p, lds, ax, ay, wr, wc, cl, kl, pm, qm);
  }
  if (c.cls == 1) {
    double (*T)[W + 1] = reinterpret_cast<double (*)[W + 1]>(lds);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          T[32 * wr + 16 * p + 4 * r + kl][32 * wc + 16 * q + cl] = ax[p][q][r];
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          ay[p][q][r] = T[32 * wc + 16 * q + cl][32 * wr + 16 * p + 4 * r + kl];
    __syncthreads();
  } else if (c.cls != 0) {
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int q = 0; q < 2; ++q) ay[p][q] = ax[p][q];
  }
}

// ---------------------------------------------------------------------------
// CAVV tiles for one (m, A <= B): X_u = B_mA^T B_uB, Y_u = B_uA^T B_mB for all
// u < NA on TW x TW tiles (TW = 32 or 64), each wave owning a quadrant.
// ---------------------------------------------------------------------------
template <int NA, int TW>
struct CavvCfg {
  static constexpr int NP = 2 + 2 * NA;
  static constexpr int HB = TW / 32;
  static constexpr int HW = TW / 2;
  // chunk length keeps both LDS buffers within 96 KB
  static constexpr int KC = (2 * NP * 16 * TW * 8 <= 98304) ? 16 : ((2 * NP * 8 * TW * 8 <= 98304) ? 8 : 4);
  static constexpr int LDS = 2 * NP * KC * TW;   // doubles
};

struct CavvWork {
  int m, A, B;
  bool diag;
};

__device__ __forceinline__ CavvWork decode_cavv(int64_t w, int ntw, int64_t n0) {
  CavvWork c;
  const int64_t ntp_lt = (int64_t)ntw * (ntw - 1) / 2;
  if (w < n0) {
    c.m = (int)(w / ntp_lt);
    decode_pair_lt(w % ntp_lt, ntw, c.A, c.B);
    c.diag = false;
  } else {
    w -= n0;
    c.m = (int)(w / ntw);
    c.A = c.B = (int)(w % ntw);
    c.diag = true;
  }
  return c;
}

template <int NA, int TW>
__device__ __forceinline__ void cavv_compute(const double *Pcv, const double *Pav,
                                             int64_t naux_p, int ntv, const CavvWork &c,
                                             double *lds, d4 (&X)[NA][TW / 32][TW / 32],
                                             d4 (&Y)[NA][TW / 32][TW / 32], int wr, int wc,
                                             int cl, int kl) {
  using C = CavvCfg<NA, TW>;
  constexpr int KC = C::KC, HB = C::HB, HW = C::HW, NP = C::NP;
  const int64_t pstride = naux_p * kPanel;
  const int pA = (c.A * TW) / kPanel, oA = (c.A * TW) % kPanel;
  const int pB = (c.B * TW) / kPanel, oB = (c.B * TW) % kPanel;
  const double *src[NP];
  src[0] = Pcv + (int64_t)(c.m * ntv + pA) * pstride + oA;
  src[1] = Pcv + (int64_t)(c.m * ntv + pB) * pstride + oB;
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    src[2 + u] = Pav + (int64_t)(u * ntv + pA) * pstride + oA;
    src[2 + NA + u] = Pav + (int64_t)(u * ntv + pB) * pstride + oB;
  }
#pragma unroll
  for (int u = 0; u < NA; ++u)
#pragma unroll
    for (int p = 0; p < HB; ++p)
#pragma unroll
      for (int q = 0; q < HB; ++q) {
        X[u][p][q] = zero4();
        Y[u][p][q] = zero4();
      }
  kloop<NP, TW, KC>(src, kPanel, naux_p, lds, [&](const double *L) {
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int k = kk * 4 + kl;
      double am[HB], bm[HB];
#pragma unroll
      for (int p = 0; p < HB; ++p) am[p] = L[(0 * KC + k) * TW + lcol<TW>(HW * wr + 16 * p + cl, k)];
#pragma unroll
      for (int q = 0; q < HB; ++q) bm[q] = L[(1 * KC + k) * TW + lcol<TW>(HW * wc + 16 * q + cl, k)];
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        double au[HB], bu[HB];
#pragma unroll
        for (int p = 0; p < HB; ++p)
          au[p] = L[((2 + u) * KC + k) * TW + lcol<TW>(HW * wr + 16 * p + cl, k)];
#pragma unroll
        for (int q = 0; q < HB; ++q)
          bu[q] = L[((2 + NA + u) * KC + k) * TW + lcol<TW>(HW * wc + 16 * q + cl, k)];
#pragma unroll
        for (int p = 0; p < HB; ++p)
#pragma unroll
          for (int q = 0; q < HB; ++q) {
            X[u][p][q] = mfma64(am[p], bu[q], X[u][p][q]);
            Y[u][p][q] = mfma64(au[p], bm[q], Y[u][p][q]);
          }
      }
    }
  });
}

}  // namespace dsrg
