// Device-side helpers shared by the HIP kernels of libdsrgdf (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;   // every contraction kernel runs 4 waves of 64
constexpr int kPadV = 16;       // LDS row padding (doubles) for virtual panels

// ---------------------------------------------------------------------------
// Regularisers. x = s D^2.
// R(D)  = (1 - exp(-2x)) / D            F1 pair weight (Eq. expensive)
// R1(D) = (1 - exp(-x)) / D             T2 renormalised denominator (Eq. T2amp)
// S(D)  = 1 + exp(-x)                   v -> v-tilde factor (Eq. v_tilde)
// For x < 1e-3 the Maclaurin series in x (section II.B analysis) is used,
// truncated after x^4 (x^5 for S); the dropped terms are below 1e-16
// relative there. For exponents beyond 37.5, exp(-.) < 2^-54 and
// 1 -/+ exp(-.) rounds to exactly 1, so the exponential is skipped.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double reg_R(double D, double s) {
  const double x = s * D * D;
  if (x < 1e-3) {
    return 2.0 * s * D *
           (1.0 + x * (-1.0 + x * (2.0 / 3.0 + x * (-1.0 / 3.0 + x * (2.0 / 15.0)))));
  }
  const double y = 2.0 * x;
  if (y > 37.5) return 1.0 / D;
  return -expm1(-y) / D;
}

__device__ __forceinline__ void reg_S_R1(double D, double s, double &S, double &R1) {
  const double x = s * D * D;
  if (x < 1e-3) {
    R1 = s * D * (1.0 + x * (-0.5 + x * (1.0 / 6.0 + x * (-1.0 / 24.0 + x * (1.0 / 120.0)))));
    S = 2.0 + x * (-1.0 + x * (0.5 + x * (-1.0 / 6.0 + x * (1.0 / 24.0 + x * (-1.0 / 120.0)))));
    return;
  }
  if (x > 37.5) {
    S = 1.0;
    R1 = 1.0 / D;
    return;
  }
  const double em = expm1(-x);
  S = 2.0 + em;
  R1 = -em / D;
}

// Regularisers with their derivatives for the adjoint kernels.
// dR/dD = 4 s e^{-2x} - R/D, dR/ds = 2 D e^{-2x}; series for x < 1e-3:
// dR/dD = 2s[1 - 3x + 10/3 x^2 - 7/3 x^3 + 6/5 x^4].
__device__ __forceinline__ void reg_R_grad(double D, double s, double &R, double &dD,
                                           double &ds) {
  const double x = s * D * D;
  const double e2 = exp(-2.0 * x);
  ds = 2.0 * D * e2;
  if (x < 1e-3) {
    R = 2.0 * s * D *
        (1.0 + x * (-1.0 + x * (2.0 / 3.0 + x * (-1.0 / 3.0 + x * (2.0 / 15.0)))));
    dD = 2.0 * s * (1.0 + x * (-3.0 + x * (10.0 / 3.0 + x * (-7.0 / 3.0 + x * (6.0 / 5.0)))));
    return;
  }
  R = -expm1(-2.0 * x) / D;
  dD = 4.0 * s * e2 - R / D;
}

// S, R1 with dS/dD = -2 s D e^{-x}, dR1/dD = 2 s e^{-x} - R1/D,
// dS/ds = -D^2 e^{-x}, dR1/ds = D e^{-x}; series for x < 1e-3:
// dR1/dD = s[1 - 3/2 x + 5/6 x^2 - 7/24 x^3 + 3/40 x^4].
__device__ __forceinline__ void reg_S_R1_grad(double D, double s, double &S, double &R1,
                                              double &dS, double &dR1, double &sS,
                                              double &sR1) {
  const double x = s * D * D;
  const double e1 = exp(-x);
  dS = -2.0 * s * D * e1;
  sS = -D * D * e1;
  sR1 = D * e1;
  if (x < 1e-3) {
    R1 = s * D * (1.0 + x * (-0.5 + x * (1.0 / 6.0 + x * (-1.0 / 24.0 + x * (1.0 / 120.0)))));
    S = 2.0 + x * (-1.0 + x * (0.5 + x * (-1.0 / 6.0 + x * (1.0 / 24.0 + x * (-1.0 / 120.0)))));
    dR1 = s * (1.0 + x * (-1.5 + x * (5.0 / 6.0 + x * (-7.0 / 24.0 + x * (3.0 / 40.0)))));
    return;
  }
  const double em = expm1(-x);
  S = 2.0 + em;
  R1 = -em / D;
  dR1 = 2.0 * s * e1 - R1 / D;
}

// Sum over the 256 threads of a workgroup in a fixed order; the result is
// valid in thread 0. `red` is a __shared__ double[4].
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = (red[0] + red[1]) + (red[2] + red[3]);
  return t;
}

// Same for NW waves (blockDim = 64 NW); `red` is a __shared__ double[NW].
template <int NW>
__device__ __forceinline__ double block_sum_n(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NW; ++k) t += red[k];
  }
  return t;
}

// Deliver one workgroup's partial energy: its own slot (deterministic
// reduction) or an FP64 atomic into the term accumulator.
// Sign check of a CCVV work item's contribution (Eq. expensive): with every
// denominator Delta = e_i + e_j - e_a - e_b negative, R(Delta) <= 0 and
// x^2 - x y + y^2 >= 0, so each term and their sum are <= 0 in any rounding.
// A positive or NaN sum sets bit 0 of *chk (nullptr: not checked).
__device__ __forceinline__ void check_nonpositive(double t, unsigned *chk) {
  if (chk && threadIdx.x == 0 && !(t <= 0.0)) atomicOr(chk, 1u);
}

__device__ __forceinline__ void emit_partial(double t, double *slots, int64_t slot,
                                             double *acc, int atomic_mode) {
  if (threadIdx.x == 0) {
    if (atomic_mode)
      atomicAdd(acc, t);
    else
      slots[slot] = t;
  }
}

// Decode the k-th strictly-ordered pair (p < q) of n items, row-major.
__device__ __forceinline__ void decode_pair_lt(int64_t k, int n, int &p, int &q) {
  int r = 0;
  int64_t rowlen = n - 1;
  while (k >= rowlen) {
    k -= rowlen;
    ++r;
    --rowlen;
  }
  p = r;
  q = r + 1 + (int)k;
}

// Decode the k-th pair (p <= q) of n items, row-major.
__device__ __forceinline__ void decode_pair_le(int64_t k, int n, int &p, int &q) {
  int r = 0;
  int64_t rowlen = n;
  while (k >= rowlen) {
    k -= rowlen;
    ++r;
    --rowlen;
  }
  p = r;
  q = r + (int)k;
}

}  // namespace dsrg
