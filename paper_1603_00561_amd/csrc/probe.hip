// Matrix-core rate probe of libdsrgdf (gfx950): a measurement aid for the
// rooflines of the tile kernels, not a step of the method. Each wave takes
// `iters` rounds of independent matrix products on register operands of
// full-entropy random bits that change from one product to the next (a ring
// of eight A and eight B operands), the operand statistics of the slice and
// FP64 tile kernels without their memory traffic. Thread 0 of every
// workgroup stamps the shader cycle counter and the constant-rate counter
// before and after the workgroup's products, so the caller can read the
// clock the products ran at beside the rate.
#include "int8_tiles.h"

namespace dsrg {

constexpr int kProbeThreads = 512;   // eight waves, two per SIMD
constexpr int kProbeRing = 8;        // distinct operands per input

// splitmix64 finalizer (Steele, Lea and Flood, 2014): operand bits from an index
__device__ __forceinline__ uint64_t probe_mix(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ void probe_stamp(int64_t *stamps, int which) {
  if (threadIdx.x == 0) {
    const long long w = wall_clock64(), c = clock64();
    stamps[4 * (int64_t)blockIdx.x + 2 * which] = c;
    stamps[4 * (int64_t)blockIdx.x + 2 * which + 1] = w;
  }
}

// four accumulators of v_mfma_i32_32x32x32_i8 per wave and round
__global__ __launch_bounds__(kProbeThreads) void probe_i8_kernel(int64_t iters,
                                                                 int64_t *__restrict__ stamps,
                                                                 uint32_t *__restrict__ sink) {
  const uint64_t id = (uint64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  i4v a[kProbeRing], b[kProbeRing];
#pragma unroll
  for (int k = 0; k < kProbeRing; ++k)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      a[k][e] = (int)probe_mix(id * 64 + k * 8 + e);
      b[k][e] = (int)probe_mix(id * 64 + k * 8 + 4 + e);
    }
  i16v acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) acc[k] = i16v{};
  __syncthreads();
  probe_stamp(stamps, 0);
  for (int64_t it = 0; it < iters; ++it) {
    // two rounds of four products: every product of the eight takes another A and B
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[m & 3] = mfma_i8(a[m], b[(3 * m + 1) & 7], acc[m & 3]);
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += (uint32_t)acc[k][e];
  sink[id] = s;
  __syncthreads();
  probe_stamp(stamps, 1);
}

// eight accumulators of v_mfma_f64_16x16x4f64 per wave and round; operands
// uniform in [-1, 1) with full 53-bit mantissas
__global__ __launch_bounds__(kProbeThreads) void probe_f64_kernel(int64_t iters,
                                                                  int64_t *__restrict__ stamps,
                                                                  double *__restrict__ sink) {
  const uint64_t id = (uint64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  double a[kProbeRing], b[kProbeRing];
#pragma unroll
  for (int k = 0; k < kProbeRing; ++k) {
    a[k] = (double)(probe_mix(id * 16 + k) >> 11) * 0x1.0p-52 - 1.0;
    b[k] = (double)(probe_mix(id * 16 + 8 + k) >> 11) * 0x1.0p-52 - 1.0;
  }
  d4 acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
  __syncthreads();
  probe_stamp(stamps, 0);
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[m] = mfma64(a[m], b[(3 * m + 1) & 7], acc[m]);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  sink[id] = s;
  __syncthreads();
  probe_stamp(stamps, 1);
}

hipError_t launch_mfma_probe(int kind, int64_t nwg, int64_t iters, int64_t *stamps, void *sink,
                             hipStream_t st) {
  if (kind == 0)
    hipLaunchKernelGGL(probe_i8_kernel, dim3((unsigned)nwg), dim3(kProbeThreads), 0, st, iters,
                       stamps, static_cast<uint32_t *>(sink));
  else
    hipLaunchKernelGGL(probe_f64_kernel, dim3((unsigned)nwg), dim3(kProbeThreads), 0, st, iters,
                       stamps, static_cast<double *>(sink));
  return hipGetLastError();
}

}  // namespace dsrg
