// The pieces F4-F8 of term F (Table II of the paper): every piece with two
// or more active indices, in FP64, after spin summation over restricted core
// and virtual orbitals with the spin-summed active density Gamma and
// etab = 2 I - Gamma (x, y, u, v, w, z active):
//
//   F4 = 1/4 sum Gamma_xy Gamma_uv sum_{ef} (xe|uf) S(D^{ef}_{xu}) [2 (ye|vf) - (yf|ve)] R1(D^{ef}_{yv})
//   F5 = 1/4 sum etab_uv etab_xy sum_{mn} (mv|ny) S(D^{vy}_{mn}) [2 (mu|nx) - (mx|nu)] R1(D^{ux}_{mn})
//   F6 = sum Gamma_xy etab_uv sum_{me} S(D^{ve}_{mx}) R1(D^{ue}_{my})
//          [K1 K1' + K2 K2' - (K1 K2' + K2 K1') / 2],
//        K1 = (mv|xe), K2 = (me|xv), K1' = (mu|ye), K2' = (me|yu)
//   F7 = 1/4 sum Gamma_yw Gamma_zx etab_uv sum_e (yv|ze) S(D^{ve}_{yz}) [2 (wu|xe) - (we|xu)] R1(D^{ue}_{wx})
//   F8 = 1/4 sum Gamma_wz etab_uv etab_xy sum_m (mv|wy) S(D^{vy}_{mw}) [2 (mu|zx) - (mx|zu)] R1(D^{ux}_{mz})
//
// Integrals (Eq. int_fact) come from the FP64 matrix-core producers: the
// (xe|uf) tiles of the CAVV integral producer with the active panels on both
// sides (pairs x <= u only: (xe|uf) = (uf|xe)), and the contractions over Q
// of packed panels with the flattened
// active blocks (B_ca, B_aa) for everything with at most one virtual index.
// Each piece is then a small contraction over active indices per element
// (e f, m n, m e, e or m), done with one wave (pair pieces) or one workgroup
// (three-index pieces) per element, one FP64 partial energy per workgroup
// and a compensated final sum.
#include "common_device.h"
#include "internal.h"

namespace dsrg {

constexpr int kActWaves = 4;   // elements in flight per workgroup of the pair pieces
// The pair pieces run at most kActPairGrid workgroups; each takes elements
// blockIdx.x 4 + wave + k gridDim.x 4 (a fixed assignment, so the slot sums
// are deterministic).

template <int NA>
__device__ __forceinline__ void load_densities(const double *gamma1, double *G, double *H) {
  for (int k = threadIdx.x; k < NA * NA; k += blockDim.x) {
    const double g = gamma1[k];
    G[k] = g;
    H[k] = ((k / NA) == (k % NA) ? 2.0 : 0.0) - g;
  }
}

// Lane l < NA NA of a wave owns entry (p, q) = (l / NA, l % NA) of an
// na x na matrix W (value w) and of Z (value z). Returns, in every lane,
// z (L W Rm)[p][q] (0 in the other lanes). W is staged in the wave's LDS row
// lw; every thread of the workgroup must call this (it holds barriers).
template <int NA>
__device__ __forceinline__ double sandwich(double z, double w, const double *L,
                                           const double *Rm, double *lw, int lane) {
  if (lane < NA * NA) lw[lane] = w;
  __syncthreads();
  double t = 0.0;
  if (lane < NA * NA) {
    const int p = lane / NA, q = lane % NA;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      double r = 0.0;
#pragma unroll
      for (int b = 0; b < NA; ++b) r += lw[a * NA + b] * Rm[b * NA + q];
      t += L[p * NA + a] * r;
    }
  }
  __syncthreads();   // lw is reused by the next call
  return z * t;
}

// ---------------------------------------------------------------------------
// F4 and F5: element (r, c) of a ncol-wide grid, entry (p, q) at
// A[r rs + c cs + p sp + q sq]; D_pq = bsign (eps_rc[r] + eps_rc[c] -
// eps_a[p] - eps_a[q]); z = A_pq S(D_pq), w = (2 A_pq - A_qp) R1(D_pq);
// the element contributes 1/4 sum z (M W M), M = Gamma (F4) or etab (F5).
//   F4: element (e, f), A_pq = X^{pq}_{ef} = (pe|qf), bsign = -1, M = Gamma
//   F5: element (m, n), A_vy = (mv|ny), bsign = +1, M = etab
// Both satisfy A_pq(r, c) = A_qp(c, r); with tri set only the blocks p <= q
// are stored and the others are read through that symmetry.
// ---------------------------------------------------------------------------
struct ActPairArgs {
  int64_t count, ncol;
  int64_t rs, cs, sp, sq;
  double bsign, s;
  int use_eta, tri;
  int64_t slot_base;
};

__device__ __forceinline__ double pair_entry(const double *A, const ActPairArgs &a, int64_t r,
                                             int64_t c, int p, int q) {
  if (a.tri && p > q) return A[c * a.rs + r * a.cs + q * a.sp + p * a.sq];
  return A[r * a.rs + c * a.cs + p * a.sp + q * a.sq];
}

template <int NA>
__global__ __launch_bounds__(256) void act_pair_kernel(const double *__restrict__ A,
                                                       const double *__restrict__ eps_rc,
                                                       const double *__restrict__ eps_a,
                                                       const double *__restrict__ gamma1,
                                                       ActPairArgs a, double *__restrict__ slots) {
  __shared__ double G[NA * NA], H[NA * NA], lw[kActWaves][NA * NA], red[4];
  load_densities<NA>(gamma1, G, H);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t stride = (int64_t)gridDim.x * kActWaves;
  const double *M = a.use_eta ? H : G;
  double v = 0.0;
  __syncthreads();   // densities
  // the loop bound is the same for every wave of the workgroup (barriers inside)
  for (int64_t e0 = (int64_t)blockIdx.x * kActWaves; e0 < a.count; e0 += stride) {
    const int64_t el = e0 + wave;
    double z = 0.0, w = 0.0;
    if (el < a.count && lane < NA * NA) {
      const int64_t r = el / a.ncol, c = el % a.ncol;
      const int p = lane / NA, q = lane % NA;
      const double x = pair_entry(A, a, r, c, p, q), xt = pair_entry(A, a, r, c, q, p);
      const double D = a.bsign * ((eps_rc[r] + eps_rc[c]) - (eps_a[p] + eps_a[q]));
      double S, R1;
      reg_S_R1(D, a.s, S, R1);
      z = x * S;
      w = (2.0 * x - xt) * R1;
    }
    v += sandwich<NA>(z, w, M, M, lw[wave], lane);
  }
  const double t = block_sum(v, red);
  if (threadIdx.x == 0) slots[a.slot_base + blockIdx.x] = 0.25 * t;
}

// ---------------------------------------------------------------------------
// F6: element (m, e); lane (v, x): K1 = (mv|xe) from J1[(x W + e)][(m, v)],
// K2 = (me|xv) from J2[(m W + e)][(x, v)], D = eps_m + eps_x - eps_v - eps_e;
// z1,2 = K1,2 S(D), P = (K1 - K2/2) R1(D), Q = (K2 - K1/2) R1(D); the element
// contributes sum z1 (etab P Gamma) + z2 (etab Q Gamma).
// ---------------------------------------------------------------------------
struct ActF6Args {
  int64_t count, nv, W, ld1, ld2;
  double s;
  int64_t slot_base;
};

template <int NA>
__global__ __launch_bounds__(256) void act_f6_kernel(const double *__restrict__ J1,
                                                     const double *__restrict__ J2,
                                                     const double *__restrict__ eps_c,
                                                     const double *__restrict__ eps_a,
                                                     const double *__restrict__ eps_v,
                                                     const double *__restrict__ gamma1,
                                                     ActF6Args a, double *__restrict__ slots) {
  __shared__ double G[NA * NA], H[NA * NA], lw[kActWaves][NA * NA], red[4];
  load_densities<NA>(gamma1, G, H);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t stride = (int64_t)gridDim.x * kActWaves;
  double v = 0.0;
  __syncthreads();   // densities
  for (int64_t e0 = (int64_t)blockIdx.x * kActWaves; e0 < a.count; e0 += stride) {
    const int64_t el = e0 + wave;
    double z1 = 0.0, z2 = 0.0, wp = 0.0, wq = 0.0;
    if (el < a.count && lane < NA * NA) {
      const int64_t m = el / a.nv, e = el % a.nv;
      const int vi = lane / NA, x = lane % NA;
      const double k1 = J1[((int64_t)x * a.W + e) * a.ld1 + m * NA + vi];
      const double k2 = J2[(m * a.W + e) * a.ld2 + (int64_t)x * NA + vi];
      const double D = (eps_c[m] + eps_a[x]) - (eps_a[vi] + eps_v[e]);
      double S, R1;
      reg_S_R1(D, a.s, S, R1);
      z1 = k1 * S;
      z2 = k2 * S;
      wp = (k1 - 0.5 * k2) * R1;
      wq = (k2 - 0.5 * k1) * R1;
    }
    v += sandwich<NA>(z1, wp, H, G, lw[wave], lane);
    v += sandwich<NA>(z2, wq, H, G, lw[wave], lane);
  }
  const double t = block_sum(v, red);
  if (threadIdx.x == 0) slots[a.slot_base + blockIdx.x] = t;
}

// ---------------------------------------------------------------------------
// F7 and F8: one workgroup per element el; entry (i, j, k) at
// A[el es + i si + j sj + k sk]; D_ijk = sign (eps_a[i] - eps_a[j] + eps_a[k]
// - eps_el[el]); z = A_ijk S(D), w = (2 A_ijk - A_kji) R1(D); the element
// contributes 1/4 sum z (Mo x Mm x Mo) w, the three modes transformed by the
// outer, middle and outer density.
//   F7: element e, A_yvz = (yv|ze), sign +1, Mo = Gamma, Mm = etab
//   F8: element m, A_vwy = (mv|wy), sign -1, Mo = etab, Mm = Gamma
// ---------------------------------------------------------------------------
struct ActTriArgs {
  int64_t es, si, sj, sk;
  double sign, s;
  int outer_eta;
  int64_t slot_base;
};

template <int NA>
__global__ __launch_bounds__(256) void act_tri_kernel(const double *__restrict__ A,
                                                      const double *__restrict__ eps_el,
                                                      const double *__restrict__ eps_a,
                                                      const double *__restrict__ gamma1,
                                                      ActTriArgs a, double *__restrict__ slots) {
  constexpr int N2 = NA * NA, N3 = NA * NA * NA, PER = (N3 + 255) / 256;
  __shared__ double G[N2], H[N2], W0[N3], W1[N3], red[4];
  load_densities<NA>(gamma1, G, H);
  const int64_t el = blockIdx.x;
  const double *Ae = A + el * a.es;
  const double ee = eps_el[el];
  double z[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + 256 * k;
    z[k] = 0.0;
    if (t < N3) {
      const int i = t / N2, j = (t / NA) % NA, kk = t % NA;
      const double x = Ae[i * a.si + j * a.sj + kk * a.sk];
      const double xs = Ae[kk * a.si + j * a.sj + i * a.sk];
      const double D = a.sign * ((eps_a[i] + eps_a[kk]) - (eps_a[j] + ee));
      double S, R1;
      reg_S_R1(D, a.s, S, R1);
      z[k] = x * S;
      W0[t] = (2.0 * x - xs) * R1;
    }
  }
  __syncthreads();
  const double *Mo = a.outer_eta ? H : G, *Mm = a.outer_eta ? G : H;
  // W1[a'][b'][c] = sum_c' W0[a'][b'][c'] Mo[c'][c]
  for (int t = threadIdx.x; t < N3; t += 256) {
    const int ab = t / NA, c = t % NA;
    double r = 0.0;
#pragma unroll
    for (int cp = 0; cp < NA; ++cp) r += W0[ab * NA + cp] * Mo[cp * NA + c];
    W1[t] = r;
  }
  __syncthreads();
  // W0[a'][b][c] = sum_b' Mm[b][b'] W1[a'][b'][c]
  for (int t = threadIdx.x; t < N3; t += 256) {
    const int ap = t / N2, b = (t / NA) % NA, c = t % NA;
    double r = 0.0;
#pragma unroll
    for (int bp = 0; bp < NA; ++bp) r += Mm[b * NA + bp] * W1[ap * N2 + bp * NA + c];
    W0[t] = r;
  }
  __syncthreads();
  // T[a][b][c] = sum_a' Mo[a][a'] W0[a'][b][c], dotted with z
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x + 256 * k;
    if (t < N3) {
      const int ai = t / N2, bc = t % N2;
      double r = 0.0;
#pragma unroll
      for (int ap = 0; ap < NA; ++ap) r += Mo[ai * NA + ap] * W0[ap * N2 + bc];
      v += z[k] * r;
    }
  }
  const double t = block_sum(v, red);
  if (threadIdx.x == 0) slots[a.slot_base + blockIdx.x] = 0.25 * t;
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
template <int NA>
static hipError_t launch_active_na(const ActivePlan &pl, const ActiveInputs &in, void *ws,
                                   hipStream_t st) {
  double *slots = ws_d(ws, pl.off_slots);
  hipError_t e;
  {  // F4 over (e, f)
    ActPairArgs a;
    a.count = pl.nv * pl.nv;
    a.ncol = pl.nv;
    a.rs = pl.W;
    a.cs = 1;
    a.sq = pl.W * pl.W;
    a.sp = NA * a.sq;
    a.bsign = -1.0;
    a.s = pl.s;
    a.use_eta = 0;
    a.tri = 1;
    a.slot_base = pl.slot_base[0];
    timer_begin("act_f4", st);
    hipLaunchKernelGGL(act_pair_kernel<NA>, dim3((unsigned)pl.slot_count[0]), dim3(256), 0, st,
                       ws_d(ws, pl.off_x), in.eps_v, in.eps_a, in.gamma1, a, slots);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {  // F5 over (m, n)
    ActPairArgs a;
    a.count = pl.nc * pl.nc;
    a.ncol = pl.nc;
    a.rs = (int64_t)kPanel * pl.ncC;
    a.cs = NA;
    a.sp = pl.ncC;
    a.sq = 1;
    a.bsign = 1.0;
    a.s = pl.s;
    a.use_eta = 1;
    a.tri = 0;
    a.slot_base = pl.slot_base[1];
    timer_begin("act_f5", st);
    hipLaunchKernelGGL(act_pair_kernel<NA>, dim3((unsigned)pl.slot_count[1]), dim3(256), 0, st,
                       ws_d(ws, pl.off_jk), in.eps_c, in.eps_a, in.gamma1, a, slots);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {  // F6 over (m, e)
    ActF6Args a;
    a.count = pl.nc * pl.nv;
    a.nv = pl.nv;
    a.W = pl.W;
    a.ld1 = pl.ncC;
    a.ld2 = pl.ncA;
    a.s = pl.s;
    a.slot_base = pl.slot_base[2];
    timer_begin("act_f6", st);
    hipLaunchKernelGGL(act_f6_kernel<NA>, dim3((unsigned)pl.slot_count[2]), dim3(256), 0, st,
                       ws_d(ws, pl.off_ja1), ws_d(ws, pl.off_ja2), in.eps_c, in.eps_a, in.eps_v,
                       in.gamma1, a, slots);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {  // F7 over e: A_yvz = (yv|ze) = C[(z W + e)][(y, v)]
    ActTriArgs a;
    a.es = pl.ncA;
    a.si = NA;
    a.sj = 1;
    a.sk = pl.W * pl.ncA;
    a.sign = 1.0;
    a.s = pl.s;
    a.outer_eta = 0;
    a.slot_base = pl.slot_base[3];
    timer_begin("act_f7", st);
    hipLaunchKernelGGL(act_tri_kernel<NA>, dim3((unsigned)pl.slot_count[3]), dim3(256), 0, st,
                       ws_d(ws, pl.off_jc1), in.eps_v, in.eps_a, in.gamma1, a, slots);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  {  // F8 over m: A_vwy = (mv|wy) = E[(m 64 + v)][(w, y)]
    ActTriArgs a;
    a.es = (int64_t)kPanel * pl.ncA;
    a.si = pl.ncA;
    a.sj = NA;
    a.sk = 1;
    a.sign = -1.0;
    a.s = pl.s;
    a.outer_eta = 1;
    a.slot_base = pl.slot_base[4];
    timer_begin("act_f8", st);
    hipLaunchKernelGGL(act_tri_kernel<NA>, dim3((unsigned)pl.slot_count[4]), dim3(256), 0, st,
                       ws_d(ws, pl.off_je), in.eps_c, in.eps_a, in.gamma1, a, slots);
    timer_end(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_active_terms(const ActivePlan &pl, const ActiveInputs &in, void *ws,
                               double *F, hipStream_t st) {
  if (pl.na == 0) return launch_zero(F, 5, st);
  hipError_t e;
  // packed operands: virtual panels of B_av and B_cv, 64-wide panels of B_ca
  // (one per core orbital), and B_ca, B_aa flattened over their orbital pairs
  double *Pav = ws_d(ws, pl.off_pav), *Pcv = ws_d(ws, pl.off_pcv), *Pca = ws_d(ws, pl.off_pca);
  double *Rca = ws_d(ws, pl.off_rca), *Raa = ws_d(ws, pl.off_raa);
  if ((e = launch_pack_panels(in.B_av, Pav, pl.na, pl.nv, pl.naux, pl.naux_p, pl.ntv, kPanel,
                              st)) != hipSuccess)
    return e;
  if ((e = launch_pack_panels(in.B_cv, Pcv, pl.nc, pl.nv, pl.naux, pl.naux_p, pl.ntv, kPanel,
                              st)) != hipSuccess)
    return e;
  if ((e = launch_pack_panels(in.B_ca, Pca, pl.nc, pl.na, pl.naux, pl.naux_p, 1, kPanel, st)) !=
      hipSuccess)
    return e;
  if ((e = launch_pack_panels(in.B_ca, Rca, 1, pl.nc * pl.na, pl.naux, pl.naux_p, 1,
                              (int)pl.ncC, st)) != hipSuccess)
    return e;
  if ((e = launch_pack_panels(in.B_aa, Raa, 1, pl.na * pl.na, pl.naux, pl.naux_p, 1,
                              (int)pl.ncA, st)) != hipSuccess)
    return e;
  // integrals: X[x][u][e][f] = (xe|uf); (xe|mv); (me|xv); (ze|yv); (mv|ny); (mv|wy)
  if ((e = launch_x_fp64(Pav, Pav, (int)pl.na, (int)pl.ntv, (int)pl.nv, pl.naux_p, 0, (int)pl.na,
                         reinterpret_cast<int *>(ws_d(ws, pl.off_ctr)), ws_d(ws, pl.off_x), true,
                         st)) != hipSuccess)
    return e;
  double *jp = ws_d(ws, pl.off_jpart);
  if ((e = launch_j_fp64(Pav, pl.na * pl.ntv, Rca, pl.ncC, pl.naux_p, ws_d(ws, pl.off_ja1), jp,
                         st)) != hipSuccess)
    return e;
  if ((e = launch_j_fp64(Pcv, pl.nc * pl.ntv, Raa, pl.ncA, pl.naux_p, ws_d(ws, pl.off_ja2), jp,
                         st)) != hipSuccess)
    return e;
  if ((e = launch_j_fp64(Pav, pl.na * pl.ntv, Raa, pl.ncA, pl.naux_p, ws_d(ws, pl.off_jc1), jp,
                         st)) != hipSuccess)
    return e;
  if ((e = launch_j_fp64(Pca, pl.nc, Rca, pl.ncC, pl.naux_p, ws_d(ws, pl.off_jk), jp, st)) !=
      hipSuccess)
    return e;
  if ((e = launch_j_fp64(Pca, pl.nc, Raa, pl.ncA, pl.naux_p, ws_d(ws, pl.off_je), jp, st)) !=
      hipSuccess)
    return e;
  switch (pl.na) {
    case 1: e = launch_active_na<1>(pl, in, ws, st); break;
    case 2: e = launch_active_na<2>(pl, in, ws, st); break;
    case 3: e = launch_active_na<3>(pl, in, ws, st); break;
    case 4: e = launch_active_na<4>(pl, in, ws, st); break;
    case 5: e = launch_active_na<5>(pl, in, ws, st); break;
    case 6: e = launch_active_na<6>(pl, in, ws, st); break;
    case 7: e = launch_active_na<7>(pl, in, ws, st); break;
    case 8: e = launch_active_na<8>(pl, in, ws, st); break;
    default: e = hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  return launch_finalize_terms(ws_d(ws, pl.off_slots), pl.slot_base, pl.slot_count, 5, F, st);
}

}  // namespace dsrg
