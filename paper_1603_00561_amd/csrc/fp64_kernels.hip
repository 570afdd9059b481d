// FP64 forward path of libdsrgdf: panel packing, the CCVV / CAVV / CCAV
// pair-tiled contractions with fused regulariser epilogues, and the final
// reduction of the partial energies (gfx950, FP64 matrix cores).
//
// Every contraction is K = L^T R over the auxiliary index Q (Eq. int_fact),
// with L and R packed panels [Q][64 columns]; the (pq|rs) tiles live only in
// registers and are reduced into energies in the same kernel (section III:
// no four-index storage).
#include "common_device.h"
#include "internal.h"

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
// Staging of NP panel chunks (KC rows of W doubles each, row stride ld in
// global memory) through registers into LDS rows of length LDW.
// ---------------------------------------------------------------------------
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
  template <int LDW>
  __device__ __forceinline__ void store(double (*lds)[KC][LDW]) const {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int idx = threadIdx.x + k * kThreads;
        if (N2 % kThreads == 0 || idx < N2) {
          const int row = idx / (W / 2);
          const int c2 = idx % (W / 2);
          *reinterpret_cast<d2v *>(&lds[p][row][2 * c2]) = r[p][k];
        }
      }
    }
  }
};

// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// result register r of lane l holds D[4 r + l / 16][l % 16] (rows interleaved
// by four, unlike the FP32-output shapes).
__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// CCVV (F1). One workgroup per (core pair i <= j, virtual tile pair A <= B).
// x = K^{ij}[A,B] = B_iA^T B_jB and y = K^{ji}[A,B] = B_jA^T B_iB, so that
// y[a][b] = (ib|ja) sits in the same registers as x[a][b] = (ia|jb).
// Work order: (i<j, A<B), (i<j, A=B), (i=j, A<B), (i=j, A=B); the energy
// weight c of c R (x^2 - x y + y^2) is 4, 2, 2, 1 respectively.
// ---------------------------------------------------------------------------
struct CcvvArgs {
  int nc, nv, ntv;
  int64_t naux_p;
  double s;
  int64_t n0, n1, n2;      // sizes of the first three work classes
  int64_t slot_base;
  int atomic_mode;
};

template <int KC>
__global__ __launch_bounds__(256) void ccvv_fp64_kernel(const double *__restrict__ Pcv,
                                                        const double *__restrict__ eps_c,
                                                        const double *__restrict__ eps_v,
                                                        CcvvArgs a, double *slots,
                                                        double *acc) {
  constexpr int W = kPanel, LDW = W + kPadV;
  __shared__ double lds[4][KC][LDW];
  __shared__ double red[4];

  // ---- decode the work item ----
  int64_t w = blockIdx.x;
  int i, j, A, B;
  double weight;
  const int64_t ntp_lt = (int64_t)a.ntv * (a.ntv - 1) / 2;
  if (w < a.n0) {
    decode_pair_lt(w / ntp_lt, a.nc, i, j);
    decode_pair_lt(w % ntp_lt, a.ntv, A, B);
    weight = 4.0;
  } else if ((w -= a.n0) < a.n1) {
    decode_pair_lt(w / a.ntv, a.nc, i, j);
    A = B = (int)(w % a.ntv);
    weight = 2.0;
  } else if ((w -= a.n1) < a.n2) {
    i = j = (int)(w / ntp_lt);
    decode_pair_lt(w % ntp_lt, a.ntv, A, B);
    weight = 2.0;
  } else {
    w -= a.n2;
    i = j = (int)(w / a.ntv);
    A = B = (int)(w % a.ntv);
    weight = 1.0;
  }
  const bool need_y = (i != j);
  const int64_t pstride = a.naux_p * W;
  const double *src[4] = {Pcv + (int64_t)(i * a.ntv + A) * pstride,
                          Pcv + (int64_t)(j * a.ntv + B) * pstride,
                          Pcv + (int64_t)(j * a.ntv + A) * pstride,
                          Pcv + (int64_t)(i * a.ntv + B) * pstride};

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int cl = lane & 15, kl = lane >> 4;

  d4 ax[2][2], ay[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      ax[p][q] = d4{0.0, 0.0, 0.0, 0.0};
      ay[p][q] = d4{0.0, 0.0, 0.0, 0.0};
    }

  Stage<4, W, KC> st;
  st.load(src, W, 0);
  for (int64_t q0 = 0; q0 < a.naux_p; q0 += KC) {
    __syncthreads();
    st.template store<LDW>(lds);
    __syncthreads();
    if (q0 + KC < a.naux_p) st.load(src, W, q0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int k = kk * 4 + kl;
      double fa[2], fb[2];
#pragma unroll
      for (int p = 0; p < 2; ++p) fa[p] = lds[0][k][32 * wr + 16 * p + cl];
#pragma unroll
      for (int q = 0; q < 2; ++q) fb[q] = lds[1][k][32 * wc + 16 * q + cl];
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) ax[p][q] = mfma64(fa[p], fb[q], ax[p][q]);
      if (need_y) {
#pragma unroll
        for (int p = 0; p < 2; ++p) fa[p] = lds[2][k][32 * wr + 16 * p + cl];
#pragma unroll
        for (int q = 0; q < 2; ++q) fb[q] = lds[3][k][32 * wc + 16 * q + cl];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) ay[p][q] = mfma64(fa[p], fb[q], ay[p][q]);
      }
    }
  }

  // ---- epilogue: c R(D) (x^2 - x y + y^2) ----
  const double eij = eps_c[i] + eps_c[j];
  double eb[2];
  int bcol[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    bcol[q] = B * W + 32 * wc + 16 * q + cl;
    eb[q] = bcol[q] < a.nv ? eps_v[bcol[q]] : 0.0;
  }
  double part = 0.0;
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int arow = A * W + 32 * wr + 16 * p + 4 * r + kl;
      if (arow >= a.nv) continue;
      const double ea = eps_v[arow];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (bcol[q] >= a.nv) continue;
        const double D = eij - ea - eb[q];
        const double R = reg_R(D, a.s);
        const double x = ax[p][q][r];
        const double y = need_y ? ay[p][q][r] : x;
        part += R * (x * x - x * y + y * y);
      }
    }
  }
  const double t = block_sum(part, red) * weight;
  emit_partial(t, slots, a.slot_base + blockIdx.x, acc, a.atomic_mode);
}

// ---------------------------------------------------------------------------
// CAVV (F2). One workgroup per (core m, virtual tile pair A <= B) with tiles
// of TW columns. For every active u: X_u[e][f] = (me|uf) = B_mA^T B_uB and
// Y_u[e][f] = (mf|ue) = B_uA^T B_mB. The epilogue forms, per (e,f),
//   sum_uv Gamma_uv S(D_mu) R1(D_mv) [X_u (2X_v - Y_v) + Y_u (2Y_v - X_v)]
// which covers (e,f) and (f,e); weight 1 for A<B and 1/2 for A=B.
// ---------------------------------------------------------------------------
struct CavvArgs {
  int nc, na, nv, ntv, ntw;
  int64_t naux_p;
  double s;
  int64_t n0;              // number of A<B work items
  int64_t slot_base;
  int atomic_mode;
};

template <int NA, int TW, int KC>
__global__ __launch_bounds__(256) void cavv_fp64_kernel(
    const double *__restrict__ Pcv, const double *__restrict__ Pav,
    const double *__restrict__ eps_c, const double *__restrict__ eps_a,
    const double *__restrict__ eps_v, const double *__restrict__ gamma1, CavvArgs a,
    double *slots, double *acc) {
  constexpr int NP = 2 + 2 * NA;
  constexpr int LDW = TW + kPadV;
  constexpr int HB = TW / 32;   // 16-row blocks per wave side
  __shared__ double lds[NP][KC][LDW];
  __shared__ double red[4];

  int64_t w = blockIdx.x;
  int m, A, B;
  double weight;
  const int64_t ntp_lt = (int64_t)a.ntw * (a.ntw - 1) / 2;
  if (w < a.n0) {
    m = (int)(w / ntp_lt);
    decode_pair_lt(w % ntp_lt, a.ntw, A, B);
    weight = 1.0;
  } else {
    w -= a.n0;
    m = (int)(w / a.ntw);
    A = B = (int)(w % a.ntw);
    weight = 0.5;
  }
  const int64_t pstride = a.naux_p * kPanel;
  const int pA = (A * TW) / kPanel, oA = (A * TW) % kPanel;
  const int pB = (B * TW) / kPanel, oB = (B * TW) % kPanel;
  const double *src[NP];
  src[0] = Pcv + (int64_t)(m * a.ntv + pA) * pstride + oA;
  src[1] = Pcv + (int64_t)(m * a.ntv + pB) * pstride + oB;
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    src[2 + u] = Pav + (int64_t)(u * a.ntv + pA) * pstride + oA;
    src[2 + NA + u] = Pav + (int64_t)(u * a.ntv + pB) * pstride + oB;
  }

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int cl = lane & 15, kl = lane >> 4;
  constexpr int HW = TW / 2;

  d4 X[NA][HB][HB], Y[NA][HB][HB];
#pragma unroll
  for (int u = 0; u < NA; ++u)
#pragma unroll
    for (int p = 0; p < HB; ++p)
#pragma unroll
      for (int q = 0; q < HB; ++q) {
        X[u][p][q] = d4{0.0, 0.0, 0.0, 0.0};
        Y[u][p][q] = d4{0.0, 0.0, 0.0, 0.0};
      }

  Stage<NP, TW, KC> st;
  st.load(src, kPanel, 0);
  for (int64_t q0 = 0; q0 < a.naux_p; q0 += KC) {
    __syncthreads();
    st.template store<LDW>(lds);
    __syncthreads();
    if (q0 + KC < a.naux_p) st.load(src, kPanel, q0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int k = kk * 4 + kl;
      double am[HB], bm[HB];
#pragma unroll
      for (int p = 0; p < HB; ++p) am[p] = lds[0][k][HW * wr + 16 * p + cl];
#pragma unroll
      for (int q = 0; q < HB; ++q) bm[q] = lds[1][k][HW * wc + 16 * q + cl];
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        double au[HB], bu[HB];
#pragma unroll
        for (int p = 0; p < HB; ++p) au[p] = lds[2 + u][k][HW * wr + 16 * p + cl];
#pragma unroll
        for (int q = 0; q < HB; ++q) bu[q] = lds[2 + NA + u][k][HW * wc + 16 * q + cl];
#pragma unroll
        for (int p = 0; p < HB; ++p)
#pragma unroll
          for (int q = 0; q < HB; ++q) {
            X[u][p][q] = mfma64(am[p], bu[q], X[u][p][q]);
            Y[u][p][q] = mfma64(au[p], bm[q], Y[u][p][q]);
          }
      }
    }
  }

  // ---- epilogue ----
  double G[NA][NA], ea[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    ea[u] = eps_a[u];
#pragma unroll
    for (int v = 0; v < NA; ++v) G[u][v] = gamma1[u * NA + v];
  }
  const double em = eps_c[m];
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < HB; ++q) {
    const int f = B * TW + HW * wc + 16 * q + cl;
    if (f >= a.nv) continue;
    const double ef = eps_v[f];
#pragma unroll
    for (int p = 0; p < HB; ++p) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int e = A * TW + HW * wr + 16 * p + 4 * r + kl;
        if (e >= a.nv) continue;
        const double base = em - eps_v[e] - ef;
        double S[NA], R1[NA];
#pragma unroll
        for (int u = 0; u < NA; ++u) reg_S_R1(base + ea[u], a.s, S[u], R1[u]);
        double Wv[NA], Wp[NA];
#pragma unroll
        for (int v = 0; v < NA; ++v) {
          const double xv = X[v][p][q][r], yv = Y[v][p][q][r];
          Wv[v] = R1[v] * (2.0 * xv - yv);
          Wp[v] = R1[v] * (2.0 * yv - xv);
        }
        double val = 0.0;
#pragma unroll
        for (int u = 0; u < NA; ++u) {
          double tw = 0.0, tp = 0.0;
#pragma unroll
          for (int v = 0; v < NA; ++v) {
            tw += G[u][v] * Wv[v];
            tp += G[u][v] * Wp[v];
          }
          val += S[u] * (X[u][p][q][r] * tw + Y[u][p][q][r] * tp);
        }
        part += val;
      }
    }
  }
  const double t = block_sum(part, red) * weight;
  emit_partial(t, slots, a.slot_base + blockIdx.x, acc, a.atomic_mode);
}

// ---------------------------------------------------------------------------
// CCAV (F3). One workgroup per (core pair m <= n, 64-wide virtual tile T).
// x[e][u] = (me|nu) = B_mT^T B_n(act), y[e][u] = (ne|mu) = B_nT^T B_m(act).
// Per e: sum_uv etab_uv S(D^{ev}_{mn}) R1(D^{eu}_{mn})
//        [x_v (2 x_u - y_u) + y_v (2 y_u - x_u)],  etab = 2I - Gamma,
// which covers (m,n) and (n,m); weight 1 for m<n and 1/2 for m=n.
// ---------------------------------------------------------------------------
struct CcavArgs {
  int nc, na, nv, ntv;
  int64_t naux_p;
  double s;
  int64_t slot_base;
  int atomic_mode;
};

template <int NA, int KC>
__global__ __launch_bounds__(256) void ccav_fp64_kernel(
    const double *__restrict__ Pcv, const double *__restrict__ Pca,
    const double *__restrict__ eps_c, const double *__restrict__ eps_a,
    const double *__restrict__ eps_v, const double *__restrict__ gamma1, CcavArgs a,
    double *slots, double *acc) {
  constexpr int W = kPanel, LDW = W + kPadV, WA = kActPanel;
  __shared__ double lv[2][KC][LDW];
  __shared__ double la[2][KC][WA];
  __shared__ double xs[2][W][WA + 1];
  __shared__ double red[4];

  const int64_t w = blockIdx.x;
  int m, n;
  decode_pair_le(w / a.ntv, a.nc, m, n);
  const int T = (int)(w % a.ntv);
  const double weight = (m == n) ? 0.5 : 1.0;
  const int64_t pstride = a.naux_p * W;
  const double *srcv[2] = {Pcv + (int64_t)(m * a.ntv + T) * pstride,
                           Pcv + (int64_t)(n * a.ntv + T) * pstride};
  const double *srca[2] = {Pca + (int64_t)n * a.naux_p * WA, Pca + (int64_t)m * a.naux_p * WA};

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, kl = lane >> 4;
  d4 x = {0.0, 0.0, 0.0, 0.0}, y = {0.0, 0.0, 0.0, 0.0};

  Stage<2, W, KC> sv;
  Stage<2, WA, KC> sa;
  sv.load(srcv, W, 0);
  sa.load(srca, WA, 0);
  for (int64_t q0 = 0; q0 < a.naux_p; q0 += KC) {
    __syncthreads();
    sv.template store<LDW>(lv);
    sa.template store<WA>(la);
    __syncthreads();
    if (q0 + KC < a.naux_p) {
      sv.load(srcv, W, q0 + KC);
      sa.load(srca, WA, q0 + KC);
    }
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const int k = kk * 4 + kl;
      x = mfma64(lv[0][k][16 * wave + cl], la[0][k][cl], x);
      y = mfma64(lv[1][k][16 * wave + cl], la[1][k][cl], y);
    }
  }
  // stage the two 64 x 16 tiles through LDS so one thread sees a whole row
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    xs[0][16 * wave + 4 * r + kl][cl] = x[r];
    xs[1][16 * wave + 4 * r + kl][cl] = y[r];
  }
  __syncthreads();
  double part = 0.0;
  if (threadIdx.x < W) {
    const int e = T * W + threadIdx.x;
    if (e < a.nv) {
      const double base = eps_c[m] + eps_c[n] - eps_v[e];
      double S[NA], R1[NA], xv[NA], yv[NA];
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        reg_S_R1(base - eps_a[u], a.s, S[u], R1[u]);
        xv[u] = xs[0][threadIdx.x][u];
        yv[u] = xs[1][threadIdx.x][u];
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
  }
  const double t = block_sum(part, red) * weight;
  emit_partial(t, slots, a.slot_base + blockIdx.x, acc, a.atomic_mode);
}

// ---------------------------------------------------------------------------
// Final reduction: one workgroup per term; compensated (Neumaier) sums of
// the per-workgroup slots in a fixed order, or a copy of the atomic
// accumulator. Unselected terms are written as 0.
// ---------------------------------------------------------------------------
struct FinArgs {
  int64_t base[3], count[3];
  int selected[3];
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
static inline double *ws_d(void *ws, size_t off) {
  return reinterpret_cast<double *>(static_cast<char *>(ws) + off);
}

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

hipError_t launch_pack_fp64(const Plan &pl, const Inputs &in, void *ws, hipStream_t st) {
  hipError_t e = pack_one(in.B_cv, ws_d(ws, pl.off_pcv), pl.nc, pl.nv, pl.naux, pl.naux_p,
                          pl.ntv, kPanel, st);
  if (e != hipSuccess) return e;
  if (pl.na > 0 && (pl.terms & 2)) {
    e = pack_one(in.B_av, ws_d(ws, pl.off_pav), pl.na, pl.nv, pl.naux, pl.naux_p, pl.ntv,
                 kPanel, st);
    if (e != hipSuccess) return e;
  }
  if (pl.na > 0 && (pl.terms & 4)) {
    e = pack_one(in.B_ca, ws_d(ws, pl.off_pca), pl.nc, pl.na, pl.naux, pl.naux_p, 1,
                 kActPanel, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int NA>
static hipError_t launch_cavv_na(const Plan &pl, const Inputs &in, void *ws, hipStream_t st,
                                 double *slots, double *acc) {
  CavvArgs a;
  a.nc = (int)pl.nc;
  a.na = (int)pl.na;
  a.nv = (int)pl.nv;
  a.ntv = (int)pl.ntv;
  a.ntw = (int)ceil_div(pl.nv, pl.cavv_tile);
  a.naux_p = pl.naux_p;
  a.s = pl.s;
  a.n0 = pl.nc * tri_off(a.ntw);
  a.slot_base = pl.slot_base[1];
  a.atomic_mode = pl.atomic_reduce ? 1 : 0;
  const dim3 grid((unsigned)pl.n_cavv), block(256);
  if constexpr (NA <= 2) {
    if (pl.cavv_tile == 64) {
      timer_begin("cavv_fp64", st);
      hipLaunchKernelGGL((cavv_fp64_kernel<NA, 64, 16>), grid, block, 0, st,
                         ws_d(ws, pl.off_pcv), ws_d(ws, pl.off_pav), in.eps_c, in.eps_a,
                         in.eps_v, in.gamma1, a, slots, acc + 1);
      timer_end(st);
      return hipGetLastError();
    }
  }
  {
    constexpr int KC = (NA <= 4) ? 16 : 8;
    timer_begin("cavv_fp64", st);
    hipLaunchKernelGGL((cavv_fp64_kernel<NA, 32, KC>), grid, block, 0, st,
                       ws_d(ws, pl.off_pcv), ws_d(ws, pl.off_pav), in.eps_c, in.eps_a, in.eps_v,
                       in.gamma1, a, slots, acc + 1);
    timer_end(st);
  }
  return hipGetLastError();
}

template <int NA>
static hipError_t launch_ccav_na(const Plan &pl, const Inputs &in, void *ws, hipStream_t st,
                                 double *slots, double *acc) {
  CcavArgs a;
  a.nc = (int)pl.nc;
  a.na = (int)pl.na;
  a.nv = (int)pl.nv;
  a.ntv = (int)pl.ntv;
  a.naux_p = pl.naux_p;
  a.s = pl.s;
  a.slot_base = pl.slot_base[2];
  a.atomic_mode = pl.atomic_reduce ? 1 : 0;
  timer_begin("ccav_fp64", st);
  hipLaunchKernelGGL((ccav_fp64_kernel<NA, kChunk>), dim3((unsigned)pl.n_ccav), dim3(256), 0,
                     st, ws_d(ws, pl.off_pcv), ws_d(ws, pl.off_pca), in.eps_c, in.eps_a,
                     in.eps_v, in.gamma1, a, slots, acc + 2);
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

static hipError_t launch_cavv(const Plan &pl, const Inputs &in, void *ws, hipStream_t st,
                              double *slots, double *acc) {
  DSRG_NA_SWITCH(launch_cavv_na, pl, in, ws, st, slots, acc)
}
static hipError_t launch_ccav(const Plan &pl, const Inputs &in, void *ws, hipStream_t st,
                              double *slots, double *acc) {
  DSRG_NA_SWITCH(launch_ccav_na, pl, in, ws, st, slots, acc)
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
    timer_begin("ccvv_fp64", st);
    hipLaunchKernelGGL(ccvv_fp64_kernel<kChunk>, dim3((unsigned)pl.n_ccvv), dim3(256), 0, st,
                       ws_d(ws, pl.off_pcv), in.eps_c, in.eps_v, a, slots, acc + 0);
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
  FinArgs f;
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

}  // namespace dsrg
