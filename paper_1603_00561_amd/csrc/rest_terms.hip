// The DSRG-MRPT2 second-order energy terms of Table I other than F: A, B, C,
// D, E (one-body pieces and the two-body cumulant with f-tilde / T1), G, H,
// I (two-body cumulant with v-tilde and T2), J, K (three-body cumulant), in
// spin orbitals over restricted orbitals, FP64 (gfx950).
//
// Index reading: X_{p..}^{q..} multiplies a+_p .. a_q .. (lower created,
// upper annihilated); gamma_p^q = <a+_p a_q>, eta = 1 - gamma; spin orbital
// 2k + s of spatial orbital k; holes H = C + A, particles P = A + V.
//
// Steps:
//  1. DF integrals with one index pair in P x H and the other in A x A, and
//     (ex|uh), (mu|nv), (xe|yf), as FP64 matrix-core GEMMs over the
//     auxiliary index straight from the B blocks (Eq. int_fact).
//  2. The spin-orbital block W[h][x][p][u] = <pu||hx> (h in H, x, u in A,
//     p in P), with t = W R1(D) (Eq. T2amp) and v-tilde = W S(D) (Eq.
//     v_tilde), D = e_h + e_x - e_p - e_u, zero on the all-active block; the
//     core-core block <uv||mn> the same way.
//  3. T1 and f-tilde over H x P (Eq. T1amp, Eq. f_tilde).
//  4. One reduction kernel per term (per piece for G and H), each workgroup
//     writing its partial sum, with the term's prefactor, to its own slot;
//     the slots of each term are added in a fixed order at the end.
// The virtual-virtual part of G is taken from spatial integrals after the
// sum over the spins of the two virtual indices:
//   G_VV = 1/2 sum_{xyuv} L(x,y,u,v) M(x,y,u,v), L = sum_{s,t} lambda_{x_s y_t}^{u_s v_t},
//   M(x,y,u,v) = sum_{ef} (ex|fy) S(D^{xy}_{ef}) (eu|fv) R1(D^{uv}_{ef}).
#include <algorithm>

#include "../../include/dsrg_df.h"
#include "common_device.h"
#include "internal.h"

namespace dsrg {

namespace {

constexpr int kRT = 256;          // threads per workgroup of the element kernels
constexpr int64_t kRGrid = 2048;  // workgroups at most per reduction kernel

struct RestDims {
  int nc, na, nv;
  int sC, sA, sV, sH, sP;   // spin-orbital counts
  double s;
};

__device__ __forceinline__ double eH(const RestDims &d, const double *ec, const double *ea,
                                     int hs) {
  return hs < d.nc ? ec[hs] : ea[hs - d.nc];
}
__device__ __forceinline__ double eP(const RestDims &d, const double *ea, const double *ev,
                                     int ps) {
  return ps < d.na ? ea[ps] : ev[ps - d.na];
}

int64_t grid_for(int64_t n) { return std::max<int64_t>(1, std::min(ceil_div(n, kRT), kRGrid)); }

}  // namespace

// ---------------------------------------------------------------------------
// Cumulants (section II.A) from the spin-orbital reduced density matrices of
// the active space (n spin orbitals): lambda2 = g2 - g1 ^ g1, lambda3 = g3 -
// sum over (lower, upper) position pairs (i, j) of (-1)^(i+j) g1 lambda2(rest)
// - det(g1 g1 g1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kRT) void cumulant2_kernel(int n, const double *__restrict__ g1,
                                                        const double *__restrict__ g2,
                                                        double *__restrict__ l2) {
  const int64_t N = (int64_t)n * n * n * n;
  for (int64_t k = (int64_t)blockIdx.x * kRT + threadIdx.x; k < N; k += (int64_t)gridDim.x * kRT) {
    const int s = (int)(k % n), r = (int)((k / n) % n), q = (int)((k / n / n) % n),
              p = (int)(k / n / n / n);
    l2[k] = g2[k] - g1[p * n + r] * g1[q * n + s] + g1[p * n + s] * g1[q * n + r];
  }
}

__global__ __launch_bounds__(kRT) void cumulant3_kernel(int n, const double *__restrict__ g1,
                                                        const double *__restrict__ l2,
                                                        const double *__restrict__ g3,
                                                        double *__restrict__ l3) {
  const int64_t n2 = (int64_t)n * n, n3 = n2 * n, N = n3 * n3;
  // permutations of three upper positions with their signs
  constexpr int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  constexpr double psign[6] = {1.0, -1.0, -1.0, 1.0, 1.0, -1.0};
  for (int64_t k = (int64_t)blockIdx.x * kRT + threadIdx.x; k < N; k += (int64_t)gridDim.x * kRT) {
    int lo[3], up[3];
    int64_t t = k;
    for (int i = 2; i >= 0; --i) {
      up[i] = (int)(t % n);
      t /= n;
    }
    for (int i = 2; i >= 0; --i) {
      lo[i] = (int)(t % n);
      t /= n;
    }
    double v = g3[k];
    for (int q = 0; q < 6; ++q)
      v -= psign[q] * g1[lo[0] * n + up[perm[q][0]]] * g1[lo[1] * n + up[perm[q][1]]] *
           g1[lo[2] * n + up[perm[q][2]]];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int l0 = lo[i == 0 ? 1 : 0], l1 = lo[i == 2 ? 1 : 2];
        const int u0 = up[j == 0 ? 1 : 0], u1 = up[j == 2 ? 1 : 2];
        const double sg = ((i + j) & 1) ? -1.0 : 1.0;
        v -= sg * g1[lo[i] * n + up[j]] * l2[((int64_t)(l0 * n + l1) * n + u0) * n + u1];
      }
    l3[k] = v;
  }
}

hipError_t launch_cumulants(int n, const double *g1, const double *g2, const double *g3,
                            double *l2, double *l3, hipStream_t st) {
  const int64_t n4 = (int64_t)n * n * n * n, n6 = n4 * n * n;
  timer_begin("cumulants", st);
  hipLaunchKernelGGL(cumulant2_kernel, dim3((unsigned)grid_for(n4)), dim3(kRT), 0, st, n, g1, g2,
                     l2);
  hipLaunchKernelGGL(cumulant3_kernel, dim3((unsigned)grid_for(n6)), dim3(kRT), 0, st, n, g1, l2,
                     g3, l3);
  timer_end(st);
  return hipGetLastError();
}

namespace {

// Spatial integral blocks (row-major, from the GEMMs of step 1).
struct RestInts {
  const double *Pcv;   // [h in C][e][u][x] = (eh|ux)
  const double *Pav;   // [h in A][e][u][x] = (eh|ux)
  const double *Pca;   // [h in C][w][u][x] = (wh|ux)
  const double *Paa;   // [h in A][w][u][x] = (wh|ux)
  const double *Qvc;   // [x][e][h in C][u] = (ex|uh)
  const double *Kcc;   // [m][u][n][v] = (mu|nv)
};

// (ph|ux) for p in P, h in H (spatial indices within P and H), u, x in A
__device__ __forceinline__ double K1(const RestDims &d, const RestInts &I, int p, int h, int u,
                                     int x) {
  const int na = d.na, nc = d.nc, nv = d.nv;
  const int64_t ux = (int64_t)u * na + x;
  if (p < na) {
    if (h < nc) return I.Pca[((int64_t)h * na + p) * na * na + ux];
    return I.Paa[((int64_t)(h - nc) * na + p) * na * na + ux];
  }
  const int e = p - na;
  if (h < nc) return I.Pcv[((int64_t)h * nv + e) * na * na + ux];
  return I.Pav[((int64_t)(h - nc) * nv + e) * na * na + ux];
}

// (px|uh) for p in P, x, u in A, h in H
__device__ __forceinline__ double K2(const RestDims &d, const RestInts &I, int p, int x, int u,
                                     int h) {
  const int na = d.na, nc = d.nc, nv = d.nv;
  if (p < na) {   // (wx|uh) = (uh|wx)
    if (h < nc) return I.Pca[((int64_t)h * na + u) * na * na + (int64_t)p * na + x];
    return I.Paa[((int64_t)(h - nc) * na + u) * na * na + (int64_t)p * na + x];
  }
  const int e = p - na;
  if (h < nc) return I.Qvc[(((int64_t)x * nv + e) * nc + h) * na + u];
  return I.Pav[((int64_t)x * nv + e) * na * na + (int64_t)u * na + (h - nc)];   // (ex|uh') = (eh'..)
}

}  // namespace

// W[h][x][p][u] = <pu||hx>; Wt = W R1(D), Wv = W S(D); zero on the all-active block
__global__ __launch_bounds__(kRT) void rest_w_kernel(RestDims d, RestInts I,
                                                     const double *__restrict__ ec,
                                                     const double *__restrict__ ea,
                                                     const double *__restrict__ ev,
                                                     double *__restrict__ Wt,
                                                     double *__restrict__ Wv) {
  const int64_t N = (int64_t)d.sH * d.sA * d.sP * d.sA;
  for (int64_t k = (int64_t)blockIdx.x * kRT + threadIdx.x; k < N; k += (int64_t)gridDim.x * kRT) {
    const int u = (int)(k % d.sA);
    int64_t t = k / d.sA;
    const int p = (int)(t % d.sP);
    t /= d.sP;
    const int x = (int)(t % d.sA), h = (int)(t / d.sA);
    const int hs = h >> 1, xs = x >> 1, ps = p >> 1, us = u >> 1;
    const int hg = h & 1, xg = x & 1, pg = p & 1, ug = u & 1;
    double w = 0.0;
    if (!(hs >= d.nc && ps < d.na)) {
      if (pg == hg && ug == xg) w += K1(d, I, ps, hs, us, xs);
      if (pg == xg && ug == hg) w -= K2(d, I, ps, xs, us, hs);
    }
    double S = 0.0, R1 = 0.0;
    if (w != 0.0) {
      const double D = eH(d, ec, ea, hs) + ea[xs] - eP(d, ea, ev, ps) - ea[us];
      reg_S_R1(D, d.s, S, R1);
    }
    Wt[k] = w * R1;
    Wv[k] = w * S;
  }
}

// core-core block: Wcc[m][n][u][v] = <uv||mn>, t and v-tilde
__global__ __launch_bounds__(kRT) void rest_wcc_kernel(RestDims d, const double *__restrict__ Kcc,
                                                       const double *__restrict__ ec,
                                                       const double *__restrict__ ea,
                                                       double *__restrict__ Tcc,
                                                       double *__restrict__ Vcc) {
  const int64_t N = (int64_t)d.sC * d.sC * d.sA * d.sA;
  const int na = d.na, nc = d.nc;
  for (int64_t k = (int64_t)blockIdx.x * kRT + threadIdx.x; k < N; k += (int64_t)gridDim.x * kRT) {
    const int v = (int)(k % d.sA), u = (int)((k / d.sA) % d.sA);
    const int n = (int)((k / d.sA / d.sA) % d.sC), m = (int)(k / d.sA / d.sA / d.sC);
    const int ms = m >> 1, ns = n >> 1, us = u >> 1, vs = v >> 1;
    const int mg = m & 1, ng = n & 1, ug = u & 1, vg = v & 1;
    double w = 0.0;
    const int64_t ld = (int64_t)nc * na;
    if (ug == mg && vg == ng) w += Kcc[((int64_t)ms * na + us) * ld + (int64_t)ns * na + vs];
    if (ug == ng && vg == mg) w -= Kcc[((int64_t)ns * na + us) * ld + (int64_t)ms * na + vs];
    double S = 0.0, R1 = 0.0;
    if (w != 0.0) reg_S_R1(ec[ms] + ec[ns] - ea[us] - ea[vs], d.s, S, R1);
    Tcc[k] = w * R1;
    Vcc[k] = w * S;
  }
}

// T1 and f-tilde over H x P: t1 = [f + c] R1(D), f~ = f S(D) + c (S(D) - 1)
// with c = sum_{u,x in A} (e_x - e_u) t[i][u][a][x] gamma[x][u], D = e_i - e_a
__global__ __launch_bounds__(kRT) void rest_t1_kernel(RestDims d, const double *__restrict__ Wt,
                                                      const double *__restrict__ g1,
                                                      const double *__restrict__ f_ca,
                                                      const double *__restrict__ f_cv,
                                                      const double *__restrict__ f_av,
                                                      const double *__restrict__ ec,
                                                      const double *__restrict__ ea,
                                                      const double *__restrict__ ev,
                                                      double *__restrict__ t1,
                                                      double *__restrict__ ft) {
  const int64_t N = (int64_t)d.sH * d.sP;
  for (int64_t k = (int64_t)blockIdx.x * kRT + threadIdx.x; k < N; k += (int64_t)gridDim.x * kRT) {
    const int i = (int)(k / d.sP), a = (int)(k % d.sP);
    const int is = i >> 1, as = a >> 1;
    double tv = 0.0, fv = 0.0;
    if (!(is >= d.nc && as < d.na)) {
      double f = 0.0;
      if ((i & 1) == (a & 1)) {
        if (is < d.nc)
          f = as < d.na ? f_ca[(int64_t)is * d.na + as] : f_cv[(int64_t)is * d.nv + (as - d.na)];
        else
          f = f_av[(int64_t)(is - d.nc) * d.nv + (as - d.na)];
      }
      double c = 0.0;
      for (int u = 0; u < d.sA; ++u)
        for (int x = 0; x < d.sA; ++x) {
          const double g = g1[x * d.sA + u];
          if (g == 0.0) continue;
          c += (ea[x >> 1] - ea[u >> 1]) *
               Wt[(((int64_t)i * d.sA + u) * d.sP + a) * d.sA + x] * g;
        }
      double S, R1;
      reg_S_R1(eH(d, ec, ea, is) - eP(d, ea, ev, as), d.s, S, R1);
      tv = (f + c) * R1;
      fv = f * S + c * (S - 1.0);
    }
    t1[k] = tv;
    ft[k] = fv;
  }
}

// ---------------------------------------------------------------------------
// reductions: every kernel sums its elements grid-stride, multiplies by the
// term's prefactor and writes one slot per workgroup
// ---------------------------------------------------------------------------
#define REST_LOOP(N) \
  for (int64_t k = (int64_t)blockIdx.x * kRT + threadIdx.x; k < (N); k += (int64_t)gridDim.x * kRT)

__device__ __forceinline__ void rest_emit(double v, double pref, double *slots) {
  __shared__ double red[4];
  const double t = block_sum(v, red);
  if (threadIdx.x == 0) slots[blockIdx.x] = pref * t;
}

// W index
__device__ __forceinline__ int64_t widx(const RestDims &d, int h, int x, int p, int u) {
  return (((int64_t)h * d.sA + x) * d.sP + p) * d.sA + u;
}
__device__ __forceinline__ double l2at(const double *l2, int n, int x, int y, int u, int v) {
  return l2[(((int64_t)x * n + y) * n + u) * n + v];
}

// A = f~[j][b] (gamma_H t1 eta_P)[j][b]
__global__ __launch_bounds__(kRT) void rest_a_kernel(RestDims d, const double *__restrict__ t1,
                                                     const double *__restrict__ ft,
                                                     const double *__restrict__ g1,
                                                     double *slots) {
  double acc = 0.0;
  REST_LOOP((int64_t)d.sH * d.sP) {
    const int j = (int)(k / d.sP), b = (int)(k % d.sP);
    const double fjb = ft[k];
    if (fjb == 0.0) continue;
    const bool ja = j >= d.sC, ba = b < d.sA;
    double x2 = 0.0;
    const int i0 = ja ? d.sC : j, i1 = ja ? d.sH : j + 1;
    const int a0 = ba ? 0 : b, a1 = ba ? d.sA : b + 1;
    for (int i = i0; i < i1; ++i) {
      const double gji = ja ? g1[(j - d.sC) * d.sA + (i - d.sC)] : 1.0;
      if (gji == 0.0) continue;
      for (int a = a0; a < a1; ++a) {
        const double eab = ba ? ((a == b ? 1.0 : 0.0) - g1[a * d.sA + b]) : 1.0;
        x2 += gji * t1[(int64_t)i * d.sP + a] * eab;
      }
    }
    acc += fjb * x2;
  }
  rest_emit(acc, 1.0, slots);
}

// B = 1/2 v~[x,y,e,v] t1[u,e] lambda2[x,y,u,v]
__global__ __launch_bounds__(kRT) void rest_b_kernel(RestDims d, const double *__restrict__ Wv,
                                                     const double *__restrict__ t1,
                                                     const double *__restrict__ l2,
                                                     double *slots) {
  const int n = d.sA;
  double acc = 0.0;
  REST_LOOP((int64_t)n * n * d.sV * n) {
    const int v = (int)(k % n), e = (int)((k / n) % d.sV);
    const int y = (int)((k / n / d.sV) % n), x = (int)(k / n / d.sV / n);
    const double w = Wv[widx(d, d.sC + x, y, d.sA + e, v)];
    if (w == 0.0) continue;
    double c = 0.0;
    for (int u = 0; u < n; ++u) c += t1[(int64_t)(d.sC + u) * d.sP + d.sA + e] * l2at(l2, n, x, y, u, v);
    acc += w * c;
  }
  rest_emit(acc, 0.5, slots);
}

// C = -1/2 v~[m,y,u,v] t1[m,x] lambda2[x,y,u,v]
__global__ __launch_bounds__(kRT) void rest_c_kernel(RestDims d, const double *__restrict__ Wv,
                                                     const double *__restrict__ t1,
                                                     const double *__restrict__ l2,
                                                     double *slots) {
  const int n = d.sA;
  double acc = 0.0;
  REST_LOOP((int64_t)d.sC * n * n * n) {
    const int v = (int)(k % n), u = (int)((k / n) % n), y = (int)((k / n / n) % n);
    const int m = (int)(k / n / n / n);
    const double w = Wv[widx(d, m, y, u, v)];
    if (w == 0.0) continue;
    double c = 0.0;
    for (int x = 0; x < n; ++x) c += t1[(int64_t)m * d.sP + x] * l2at(l2, n, x, y, u, v);
    acc += w * c;
  }
  rest_emit(acc, -0.5, slots);
}

// D = 1/2 f~[x,e] t2[u,v,e,y] lambda2[x,y,u,v]
__global__ __launch_bounds__(kRT) void rest_d_kernel(RestDims d, const double *__restrict__ Wt,
                                                     const double *__restrict__ ft,
                                                     const double *__restrict__ l2,
                                                     double *slots) {
  const int n = d.sA;
  double acc = 0.0;
  REST_LOOP((int64_t)n * n * d.sV * n) {
    const int y = (int)(k % n), e = (int)((k / n) % d.sV);
    const int v = (int)((k / n / d.sV) % n), u = (int)(k / n / d.sV / n);
    const double w = Wt[widx(d, d.sC + u, v, d.sA + e, y)];
    if (w == 0.0) continue;
    double c = 0.0;
    for (int x = 0; x < n; ++x) c += ft[(int64_t)(d.sC + x) * d.sP + d.sA + e] * l2at(l2, n, x, y, u, v);
    acc += w * c;
  }
  rest_emit(acc, 0.5, slots);
}

// E = -1/2 f~[m,v] t2[u,m,x,y] lambda2 = 1/2 f~[m,v] t2[m,u,x,y] lambda2[x,y,u,v]
__global__ __launch_bounds__(kRT) void rest_e_kernel(RestDims d, const double *__restrict__ Wt,
                                                     const double *__restrict__ ft,
                                                     const double *__restrict__ l2,
                                                     double *slots) {
  const int n = d.sA;
  double acc = 0.0;
  REST_LOOP((int64_t)d.sC * n * n * n) {
    const int y = (int)(k % n), x = (int)((k / n) % n), u = (int)((k / n / n) % n);
    const int m = (int)(k / n / n / n);
    const double w = Wt[widx(d, m, u, x, y)];
    if (w == 0.0) continue;
    double c = 0.0;
    for (int v = 0; v < n; ++v) c += ft[(int64_t)m * d.sP + v] * l2at(l2, n, x, y, u, v);
    acc += w * c;
  }
  rest_emit(acc, 0.5, slots);
}

// G, virtual-active part: Y[u][v][e][d] = sum_b t2[u,v,e,b] eta[b][d], then
// 1/4 v~[x,y,e,d] sum_{uv} lambda2[x,y,u,v] Y[u][v][e][d] (twice the VA part)
__global__ __launch_bounds__(kRT) void rest_gva_y_kernel(RestDims d, const double *__restrict__ Wt,
                                                         const double *__restrict__ g1,
                                                         double *__restrict__ Y) {
  const int n = d.sA;
  REST_LOOP((int64_t)n * n * d.sV * n) {
    const int dd = (int)(k % n), e = (int)((k / n) % d.sV);
    const int v = (int)((k / n / d.sV) % n), u = (int)(k / n / d.sV / n);
    double c = 0.0;
    for (int b = 0; b < n; ++b)
      c += Wt[widx(d, d.sC + u, v, d.sA + e, b)] * ((b == dd ? 1.0 : 0.0) - g1[b * n + dd]);
    Y[k] = c;
  }
}

__global__ __launch_bounds__(kRT) void rest_gva_kernel(RestDims d, const double *__restrict__ Wv,
                                                       const double *__restrict__ Y,
                                                       const double *__restrict__ l2,
                                                       double *slots) {
  const int n = d.sA;
  double acc = 0.0;
  REST_LOOP((int64_t)n * n * d.sV * n) {
    const int dd = (int)(k % n), e = (int)((k / n) % d.sV);
    const int y = (int)((k / n / d.sV) % n), x = (int)(k / n / d.sV / n);
    const double w = Wv[widx(d, d.sC + x, y, d.sA + e, dd)];
    if (w == 0.0) continue;
    double c = 0.0;
    for (int u = 0; u < n; ++u)
      for (int v = 0; v < n; ++v)
        c += l2at(l2, n, x, y, u, v) * Y[(((int64_t)u * n + v) * d.sV + e) * n + dd];
    acc += w * c;
  }
  rest_emit(acc, 0.25, slots);
}

// G, virtual-virtual part: M(x,y,u,v) = sum_{e,f} Z1[(e,f)][xy] Z2[(e,f)][uv]
// with Z1 = (xe|yf) S(D^{xy}_{ef}) and Z2 = (ue|vf) R1(D^{uv}_{ef}), from
// X[(x,e)][(y,f)] = (xe|yf). A workgroup takes items of one e and 64 f: it
// forms the item's Z1 and Z2 in LDS (the regularisers once per element), then
// accumulates 4 x 4 register tiles of M, one per thread, with the 64 f split
// over groups of threads when the tiles do not fill the workgroup. At the end
// the groups' tiles are summed in group order and the slot receives
// 1/2 sum Lambda(x,y,u,v) M_partial(x,y,u,v).
constexpr int kGvvF = 64;
constexpr int kMaxNa = DSRG_DF_MAX_ACTIVE;
constexpr int kMaxNp = kMaxNa * kMaxNa;   // active pairs (x, y)
constexpr int kGvvT = 4;                  // register tile edge

__global__ __launch_bounds__(kRT) void rest_gvv_kernel(RestDims d, const double *__restrict__ X,
                                                       const double *__restrict__ ea,
                                                       const double *__restrict__ ev,
                                                       const double *__restrict__ l2,
                                                       double *slots) {
  __shared__ double z1[kGvvF][kMaxNp + 1];
  __shared__ double z2[kGvvF][kMaxNp + 1];
  const int na = d.na, nv = d.nv, np = na * na;
  const int nt = (np + kGvvT - 1) / kGvvT;   // tiles per edge of M
  const int ntiles = nt * nt;                // <= 256 (np <= 64)
  const int ngroups = kRT / ntiles;          // >= 1
  const int tid = threadIdx.x, grp = tid / ntiles, tile = tid % ntiles;
  const bool active = grp < ngroups;
  const int ta = (tile / nt) * kGvvT, tb = (tile % nt) * kGvvT;
  const int64_t ld = (int64_t)na * nv;   // row length of X
  double acc[kGvvT][kGvvT];
#pragma unroll
  for (int a = 0; a < kGvvT; ++a)
#pragma unroll
    for (int b = 0; b < kGvvT; ++b) acc[a][b] = 0.0;
  // pad columns of the tiles past np stay zero
  for (int q = tid; q < kGvvF * (kMaxNp + 1); q += kRT) {
    (&z1[0][0])[q] = 0.0;
    (&z2[0][0])[q] = 0.0;
  }
  const int nfc = (nv + kGvvF - 1) / kGvvF;
  for (int64_t item = blockIdx.x; item < (int64_t)nv * nfc; item += gridDim.x) {
    const int e = (int)(item / nfc), f0 = (int)(item % nfc) * kGvvF;
    __syncthreads();
    for (int q = tid; q < np * kGvvF; q += kRT) {
      const int xy = q / kGvvF, fl = q % kGvvF, f = f0 + fl;
      double a = 0.0, b = 0.0;
      if (f < nv) {
        const int x = xy / na, y = xy % na;
        const double xv = X[((int64_t)x * nv + e) * ld + (int64_t)y * nv + f];
        double S, R1;
        reg_S_R1(ea[x] + ea[y] - ev[e] - ev[f], d.s, S, R1);
        a = xv * S;
        b = xv * R1;
      }
      z1[fl][xy] = a;
      z2[fl][xy] = b;
    }
    __syncthreads();
    if (active) {
      for (int fl = grp; fl < kGvvF; fl += ngroups) {
        double za[kGvvT], zb[kGvvT];
#pragma unroll
        for (int a = 0; a < kGvvT; ++a) za[a] = z1[fl][ta + a];
#pragma unroll
        for (int b = 0; b < kGvvT; ++b) zb[b] = z2[fl][tb + b];
#pragma unroll
        for (int a = 0; a < kGvvT; ++a)
#pragma unroll
          for (int b = 0; b < kGvvT; ++b) acc[a][b] = fma(za[a], zb[b], acc[a][b]);
      }
    }
  }
  // the groups' tiles, summed in group order by the threads of group 0
  __syncthreads();
  double *red = &z1[0][0];   // ngroups * ntiles * 16 <= 4096 doubles
  if (active) {
#pragma unroll
    for (int a = 0; a < kGvvT; ++a)
#pragma unroll
      for (int b = 0; b < kGvvT; ++b)
        red[((int64_t)grp * ntiles + tile) * kGvvT * kGvvT + a * kGvvT + b] = acc[a][b];
  }
  __syncthreads();
  double part = 0.0;
  const int n = d.sA;
  if (tid < ntiles) {
    for (int a = 0; a < kGvvT; ++a)
      for (int b = 0; b < kGvvT; ++b) {
        const int xy = ta + a, uv = tb + b;
        if (xy >= np || uv >= np) continue;
        double m = 0.0;
        for (int gq = 0; gq < ngroups; ++gq)
          m += red[((int64_t)gq * ntiles + tid) * kGvvT * kGvvT + a * kGvvT + b];
        const int x = xy / na, y = xy % na, u = uv / na, v = uv % na;
        double L = 0.0;
        for (int s1 = 0; s1 < 2; ++s1)
          for (int s2 = 0; s2 < 2; ++s2)
            L += l2at(l2, n, 2 * x + s1, 2 * y + s2, 2 * u + s1, 2 * v + s2);
        part += L * m;
      }
  }
  rest_emit(part, 0.5, slots);
}

// H, core-core part: 1/8 v~cc[m,n,u,v] sum_{xy} tcc[m,n,x,y] lambda2[x,y,u,v]
__global__ __launch_bounds__(kRT) void rest_hcc_kernel(RestDims d, const double *__restrict__ Tcc,
                                                       const double *__restrict__ Vcc,
                                                       const double *__restrict__ l2,
                                                       double *slots) {
  const int n = d.sA;
  double acc = 0.0;
  REST_LOOP((int64_t)d.sC * d.sC * n * n) {
    const double w = Vcc[k];
    if (w == 0.0) continue;
    const int v = (int)(k % n), u = (int)((k / n) % n);
    const int64_t mn = k / n / n;
    double c = 0.0;
    for (int x = 0; x < n; ++x)
      for (int y = 0; y < n; ++y) c += Tcc[(mn * n + x) * n + y] * l2at(l2, n, x, y, u, v);
    acc += w * c;
  }
  rest_emit(acc, 0.125, slots);
}

// H, core-active part (twice): 1/4 v~[m,l,u,v] sum_{j,x,y} t2[m,j,x,y] gamma[l][j] lambda2[x,y,u,v]
__global__ __launch_bounds__(kRT) void rest_hca_kernel(RestDims d, const double *__restrict__ Wt,
                                                       const double *__restrict__ Wv,
                                                       const double *__restrict__ g1,
                                                       const double *__restrict__ l2,
                                                       double *slots) {
  const int n = d.sA;
  double acc = 0.0;
  REST_LOOP((int64_t)d.sC * n * n * n) {
    const int v = (int)(k % n), u = (int)((k / n) % n), l = (int)((k / n / n) % n);
    const int m = (int)(k / n / n / n);
    const double w = Wv[widx(d, m, l, u, v)];
    if (w == 0.0) continue;
    double c = 0.0;
    for (int j = 0; j < n; ++j) {
      const double g = g1[l * n + j];
      if (g == 0.0) continue;
      double cj = 0.0;
      for (int x = 0; x < n; ++x)
        for (int y = 0; y < n; ++y) cj += Wt[widx(d, m, j, x, y)] * l2at(l2, n, x, y, u, v);
      c += g * cj;
    }
    acc += w * c;
  }
  rest_emit(acc, 0.25, slots);
}

// I, in three steps: Tp[(j,b)][(v,y)] = sum_{i, a} gamma_H[j][i] eta_P[a][b]
// t2[i,v,a,y]; then the product C[(j,b)][(x,u)] = sum_{(v,y)} Tp[(j,b)][(v,y)]
// Lp[(v,y)][(x,u)] with Lp[(v,y)][(x,u)] = lambda2[x,y,u,v] (a GEMM over the
// n^2 active spin-orbital pairs); then sum v~[j,x,b,u] C[(j,b)][(x,u)]
__global__ __launch_bounds__(kRT) void rest_i_tp_kernel(RestDims d, const double *__restrict__ Wt,
                                                        const double *__restrict__ g1,
                                                        double *__restrict__ Tp) {
  const int n = d.sA;
  REST_LOOP((int64_t)d.sH * d.sP * n * n) {
    const int y = (int)(k % n);
    int64_t t = k / n;
    const int v = (int)(t % n);
    t /= n;
    const int b = (int)(t % d.sP), j = (int)(t / d.sP);
    const bool ja = j >= d.sC, ba = b < d.sA;
    const int i0 = ja ? d.sC : j, i1 = ja ? d.sH : j + 1;
    const int a0 = ba ? 0 : b, a1 = ba ? d.sA : b + 1;
    double c = 0.0;
    for (int i = i0; i < i1; ++i) {
      const double gji = ja ? g1[(j - d.sC) * n + (i - d.sC)] : 1.0;
      if (gji == 0.0) continue;
      for (int a = a0; a < a1; ++a) {
        const double eab = ba ? ((a == b ? 1.0 : 0.0) - g1[a * n + b]) : 1.0;
        c += gji * eab * Wt[widx(d, i, v, a, y)];
      }
    }
    Tp[k] = c;
  }
}

// Lp[(v,y)][(x,u)] = lambda2[x,y,u,v]
__global__ __launch_bounds__(kRT) void rest_i_lam_kernel(RestDims d, const double *__restrict__ l2,
                                                         double *__restrict__ Lp) {
  const int n = d.sA;
  REST_LOOP((int64_t)n * n * n * n) {
    const int u = (int)(k % n), x = (int)((k / n) % n), y = (int)((k / n / n) % n);
    const int v = (int)(k / n / n / n);
    Lp[k] = l2at(l2, n, x, y, u, v);
  }
}

__global__ __launch_bounds__(kRT) void rest_i_kernel(RestDims d, const double *__restrict__ Wv,
                                                     const double *__restrict__ C,
                                                     double *slots) {
  const int n = d.sA;
  double acc = 0.0;
  REST_LOOP((int64_t)d.sH * n * d.sP * n) {
    const int u = (int)(k % n);
    int64_t t = k / n;
    const int b = (int)(t % d.sP);
    t /= d.sP;
    const int x = (int)(t % n), j = (int)(t / n);
    acc += Wv[k] * C[(((int64_t)j * d.sP + b) * n + x) * n + u];
  }
  rest_emit(acc, 1.0, slots);
}

// J = 1/4 v~[m,z,u,v] t2[m,w,x,y] lambda3[x,y,z,u,v,w]
__global__ __launch_bounds__(kRT) void rest_j_kernel(RestDims d, const double *__restrict__ Wt,
                                                     const double *__restrict__ Wv,
                                                     const double *__restrict__ l3,
                                                     double *slots) {
  const int n = d.sA;
  const int64_t n2 = (int64_t)n * n, n3 = n2 * n;
  double acc = 0.0;
  REST_LOOP((int64_t)d.sC * n3) {
    const int v = (int)(k % n), u = (int)((k / n) % n), z = (int)((k / n2) % n);
    const int m = (int)(k / n3);
    const double wv = Wv[widx(d, m, z, u, v)];
    if (wv == 0.0) continue;
    double c = 0.0;
    for (int w = 0; w < n; ++w)
      for (int x = 0; x < n; ++x)
        for (int y = 0; y < n; ++y)
          c += Wt[widx(d, m, w, x, y)] *
               l3[(((((int64_t)x * n + y) * n + z) * n + u) * n + v) * n + w];
    acc += wv * c;
  }
  rest_emit(acc, 0.25, slots);
}

// K: Ak[(x,y,w)][e] = v~[x,y,e,w], Bk[e][(u,v,z)] = t2[u,v,e,z] (e virtual),
// Y2 = Ak Bk (GEMM), then -1/4 Y2[(x,y,w)][(u,v,z)] lambda3[x,y,z,u,v,w]
__global__ __launch_bounds__(kRT) void rest_k_pack_kernel(RestDims d, const double *__restrict__ Wt,
                                                          const double *__restrict__ Wv,
                                                          double *__restrict__ Ak,
                                                          double *__restrict__ Bk) {
  const int n = d.sA;
  const int64_t n3 = (int64_t)n * n * n;
  REST_LOOP(n3 * d.sV) {
    // Ak row-major [(x,y,w)][e]; Bk row-major [e][(u,v,z)]
    const int e = (int)(k % d.sV);
    const int64_t r = k / d.sV;
    const int w = (int)(r % n), y = (int)((r / n) % n), x = (int)(r / n / n);
    Ak[k] = Wv[widx(d, d.sC + x, y, d.sA + e, w)];
    const int64_t k2 = k;   // reuse the same index space for Bk: (e, u, v, z)
    const int z = (int)(k2 % n), v = (int)((k2 / n) % n), u = (int)((k2 / n / n) % n);
    const int e2 = (int)(k2 / n3);
    Bk[k2] = Wt[widx(d, d.sC + u, v, d.sA + e2, z)];
  }
}

__global__ __launch_bounds__(kRT) void rest_k_kernel(RestDims d, const double *__restrict__ Y2,
                                                     const double *__restrict__ l3,
                                                     double *slots) {
  const int n = d.sA;
  const int64_t n3 = (int64_t)n * n * n;
  double acc = 0.0;
  REST_LOOP(n3 * n3) {
    const int64_t r = k / n3, c = k % n3;
    const int w = (int)(r % n), y = (int)((r / n) % n), x = (int)(r / n / n);
    const int z = (int)(c % n), v = (int)((c / n) % n), u = (int)(c / n / n);
    acc += Y2[k] * l3[(((((int64_t)x * n + y) * n + z) * n + u) * n + v) * n + w];
  }
  rest_emit(acc, -0.25, slots);
}

__global__ void rest_zero_kernel(double *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

// X[i][j] = X[j][i] for the entries below the strip diagonal blocks (row i in
// the strip of rows [r0, r1), column j < r0), 32 x 32 tiles through LDS so
// that reads and writes are both coalesced; grid (column tiles, row tiles)
// over the whole matrix, tiles with nothing to copy return at once
__global__ __launch_bounds__(256) void rest_mirror_kernel(double *X, int64_t n, int64_t strip) {
  __shared__ double tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
  // strips are a multiple of 32 wide, so every row of a tile has the same
  // strip start
  const int64_t rstart = (i0 / strip) * strip;
  if (j0 >= rstart) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t sj = j0 + r, si = i0 + tx;   // source X[sj][si] (upper part)
    if (sj < n && si < n) tile[r][tx] = X[sj * n + si];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = i0 + r, j = j0 + tx;
    if (i < n && j < n && j < rstart) X[i * n + j] = tile[tx][r];
  }
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
hipError_t launch_rest_terms(const RestPlan &pl, const RestInputs &in, void *ws, double *out,
                             hipStream_t st) {
  hipError_t e;
  if (pl.na == 0) {
    hipLaunchKernelGGL(rest_zero_kernel, dim3(1), dim3(64), 0, st, out, kRestTerms);
    return hipGetLastError();
  }
  RestDims d;
  d.nc = (int)pl.nc;
  d.na = (int)pl.na;
  d.nv = (int)pl.nv;
  d.sC = 2 * d.nc;
  d.sA = 2 * d.na;
  d.sV = 2 * d.nv;
  d.sH = d.sC + d.sA;
  d.sP = d.sA + d.sV;
  d.s = pl.s;
  const int64_t nc = pl.nc, na = pl.na, nv = pl.nv, naux = pl.naux, na2 = na * na;
  double *Pcv = ws_d(ws, pl.off_pcv), *Pav = ws_d(ws, pl.off_pav), *Pca = ws_d(ws, pl.off_pca),
         *Paa = ws_d(ws, pl.off_paa), *Qvc = ws_d(ws, pl.off_qvc), *Kcc = ws_d(ws, pl.off_kcc);
  double *X = ws_d(ws, pl.off_x);
  double *Wt = ws_d(ws, pl.off_wt), *Wv = ws_d(ws, pl.off_wv);
  double *Tcc = ws_d(ws, pl.off_tcc), *Vcc = ws_d(ws, pl.off_vcc);
  double *t1 = ws_d(ws, pl.off_t1), *ft = ws_d(ws, pl.off_ft);
  double *Y = ws_d(ws, pl.off_y), *Tp = ws_d(ws, pl.off_tp), *Lp = ws_d(ws, pl.off_lp),
         *Ci = ws_d(ws, pl.off_ci);
  double *Ak = ws_d(ws, pl.off_ak), *Bk = ws_d(ws, pl.off_bk), *Y2 = ws_d(ws, pl.off_y2);
  double *slots = ws_d(ws, pl.off_slots);

  // 1. integrals: C = A^T B over the auxiliary index
  timer_begin("rest_integrals", st);
  struct G {
    const double *A;
    int64_t M;
    const double *B;
    int64_t N;
    double *C;
  } gs[6] = {{in.B_cv, nc * nv, in.B_aa, na2, Pcv},      {in.B_av, na * nv, in.B_aa, na2, Pav},
             {in.B_ca, nc * na, in.B_aa, na2, Pca},      {in.B_aa, na2, in.B_aa, na2, Paa},
             {in.B_av, na * nv, in.B_ca, nc * na, Qvc},  {in.B_ca, nc * na, in.B_ca, nc * na, Kcc}};
  for (const G &g : gs) {
    if ((e = gemm_f64(true, false, g.M, g.N, naux, 1.0, g.A, g.M, g.B, g.N, 0.0, g.C, g.N, st)) !=
        hipSuccess)
      return e;
  }
  // X = (xe|yf) = B_av^T B_av is symmetric: the tiles of its upper triangle,
  // then the rest mirrored
  {
    const int64_t n = na * nv;
    int64_t strip = 0;
    if ((e = gemm_f64_gram_upper(true, n, naux, in.B_av, n, 0, X, n, 0, 1, &strip, st)) !=
        hipSuccess)
      return e;
    if (strip > 0 && strip < n) {
      hipLaunchKernelGGL(rest_mirror_kernel,
                         dim3((unsigned)ceil_div(n, 32), (unsigned)ceil_div(n, 32)), dim3(256), 0,
                         st, X, n, strip);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  timer_end(st);
  RestInts I{Pcv, Pav, Pca, Paa, Qvc, Kcc};

  // 2. spin-orbital blocks, 3. T1 and f-tilde
  const int64_t nW = (int64_t)d.sH * d.sA * d.sP * d.sA;
  timer_begin("rest_amplitudes", st);
  hipLaunchKernelGGL(rest_w_kernel, dim3((unsigned)grid_for(nW)), dim3(kRT), 0, st, d, I,
                     in.eps_c, in.eps_a, in.eps_v, Wt, Wv);
  const int64_t nCC = (int64_t)d.sC * d.sC * d.sA * d.sA;
  hipLaunchKernelGGL(rest_wcc_kernel, dim3((unsigned)grid_for(nCC)), dim3(kRT), 0, st, d, Kcc,
                     in.eps_c, in.eps_a, Tcc, Vcc);
  hipLaunchKernelGGL(rest_t1_kernel, dim3((unsigned)grid_for((int64_t)d.sH * d.sP)), dim3(kRT), 0,
                     st, d, Wt, in.rdm1, in.f_ca, in.f_cv, in.f_av, in.eps_c, in.eps_a, in.eps_v,
                     t1, ft);
  timer_end(st);
  if ((e = hipGetLastError()) != hipSuccess) return e;

  // 4. terms
  const double *l2 = in.lambda2, *l3 = in.lambda3, *g1 = in.rdm1;
  const int64_t *gr = pl.grid;
  const int64_t *sb = pl.slot;
  timer_begin("rest_terms", st);
  hipLaunchKernelGGL(rest_a_kernel, dim3((unsigned)gr[0]), dim3(kRT), 0, st, d, t1, ft, g1, slots + sb[0]);
  hipLaunchKernelGGL(rest_b_kernel, dim3((unsigned)gr[1]), dim3(kRT), 0, st, d, Wv, t1, l2, slots + sb[1]);
  hipLaunchKernelGGL(rest_c_kernel, dim3((unsigned)gr[2]), dim3(kRT), 0, st, d, Wv, t1, l2, slots + sb[2]);
  hipLaunchKernelGGL(rest_d_kernel, dim3((unsigned)gr[3]), dim3(kRT), 0, st, d, Wt, ft, l2, slots + sb[3]);
  hipLaunchKernelGGL(rest_e_kernel, dim3((unsigned)gr[4]), dim3(kRT), 0, st, d, Wt, ft, l2, slots + sb[4]);
  hipLaunchKernelGGL(rest_gvv_kernel, dim3((unsigned)gr[5]), dim3(kRT), 0, st, d, X, in.eps_a,
                     in.eps_v, l2, slots + sb[5]);
  const int64_t nY = (int64_t)d.sA * d.sA * d.sV * d.sA;
  hipLaunchKernelGGL(rest_gva_y_kernel, dim3((unsigned)grid_for(nY)), dim3(kRT), 0, st, d, Wt, g1, Y);
  hipLaunchKernelGGL(rest_gva_kernel, dim3((unsigned)gr[6]), dim3(kRT), 0, st, d, Wv, Y, l2, slots + sb[6]);
  hipLaunchKernelGGL(rest_hcc_kernel, dim3((unsigned)gr[7]), dim3(kRT), 0, st, d, Tcc, Vcc, l2, slots + sb[7]);
  hipLaunchKernelGGL(rest_hca_kernel, dim3((unsigned)gr[8]), dim3(kRT), 0, st, d, Wt, Wv, g1, l2, slots + sb[8]);
  hipLaunchKernelGGL(rest_i_tp_kernel, dim3((unsigned)grid_for(nW)), dim3(kRT), 0, st, d, Wt, g1, Tp);
  const int64_t nA2 = (int64_t)d.sA * d.sA;
  hipLaunchKernelGGL(rest_i_lam_kernel, dim3((unsigned)grid_for(nA2 * nA2)), dim3(kRT), 0, st, d, l2,
                     Lp);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = gemm_f64(false, false, (int64_t)d.sH * d.sP, nA2, nA2, 1.0, Tp, nA2, Lp, nA2, 0.0, Ci,
                    nA2, st)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(rest_i_kernel, dim3((unsigned)gr[9]), dim3(kRT), 0, st, d, Wv, Ci, slots + sb[9]);
  hipLaunchKernelGGL(rest_j_kernel, dim3((unsigned)gr[10]), dim3(kRT), 0, st, d, Wt, Wv, l3, slots + sb[10]);
  const int64_t n3 = (int64_t)d.sA * d.sA * d.sA;
  hipLaunchKernelGGL(rest_k_pack_kernel, dim3((unsigned)grid_for(n3 * d.sV)), dim3(kRT), 0, st, d, Wt, Wv, Ak, Bk);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = gemm_f64(false, false, n3, n3, d.sV, 1.0, Ak, d.sV, Bk, n3, 0.0, Y2, n3, st)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(rest_k_kernel, dim3((unsigned)gr[11]), dim3(kRT), 0, st, d, Y2, l3, slots + sb[11]);
  timer_end(st);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // slot ranges per output term: A, B, C, D, E, G (VV then VA), H (cc then
  // ca), I, J, K
  int64_t base[kRestTerms], count[kRestTerms];
  const int map[kRestTerms][2] = {{0, 0}, {1, 1}, {2, 2}, {3, 3}, {4, 4},
                                  {5, 6}, {7, 8}, {9, 9}, {10, 10}, {11, 11}};
  for (int t = 0; t < kRestTerms; ++t) {
    base[t] = sb[map[t][0]];
    count[t] = sb[map[t][1]] + gr[map[t][1]] - sb[map[t][0]];
  }
  return launch_finalize_terms(slots, base, count, kRestTerms, out, st);
}

// grid sizes of the twelve reduction kernels (see launch_rest_terms)
void rest_grids(int64_t nc, int64_t na, int64_t nv, int64_t *grid) {
  const int64_t sC = 2 * nc, sA = 2 * na, sV = 2 * nv, sH = sC + sA, sP = sA + sV;
  const int64_t n3 = sA * sA * sA;
  const int64_t sizes[kRestKernels] = {sH * sP,          sA * sA * sV * sA, sC * sA * sA * sA,
                                       sA * sA * sV * sA, sC * sA * sA * sA, 0,
                                       sA * sA * sV * sA, sC * sC * sA * sA, sC * sA * sA * sA,
                                       sH * sA * sP * sA, sC * sA * sA * sA, n3 * n3};
  for (int k = 0; k < kRestKernels; ++k) grid[k] = grid_for(sizes[k]);
  const int64_t nfc = ceil_div(nv, kGvvF);
  grid[5] = std::max<int64_t>(1, std::min<int64_t>(nv * nfc, 1024));
}

}  // namespace dsrg
