// Host-only driver for the AddressSanitizer / UndefinedBehaviorSanitizer run
// of the C ABI layer (tests/test_abi_sanitizers.py builds it with g++, the
// ABI translation unit instrumented, against the library's other objects).
// Every call below is answered on the host: workspace sizes over a grid of
// problem sizes (the plan arithmetic, including sizes at the documented
// limits), and each entry point's argument validation. No device is needed
// and none is touched. Exit status 0 and "checks passed" on success.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dsrg_df.h"

namespace {

int g_checks = 0, g_fail = 0;

void check(bool ok, const char *what, int line) {
  ++g_checks;
  if (!ok) {
    ++g_fail;
    std::fprintf(stderr, "FAILED line %d: %s (last error: %s)\n", line, what,
                 dsrg_df_last_error());
  }
}
#define CHECK(x) check((x), #x, __LINE__)

// aligned, non-null stand-ins for device addresses: never dereferenced, every
// call that receives them fails validation or only sizes
const double *fake(uintptr_t a = 0x10000) { return reinterpret_cast<const double *>(a); }
double *fakew(uintptr_t a = 0x20000) { return reinterpret_cast<double *>(a); }
void *fakews() { return reinterpret_cast<void *>(0x40000); }

dsrg_df_problem prob(int64_t nc, int64_t na, int64_t nv, int64_t naux, double s = 0.5) {
  dsrg_df_problem p;
  p.nc = nc;
  p.na = na;
  p.nv = nv;
  p.naux = naux;
  p.B_cv = p.B_ca = p.B_av = p.eps_c = p.eps_a = p.eps_v = p.gamma1 = fake();
  p.s = s;
  return p;
}

void workspace_grid() {
  const int64_t ncs[] = {1, 2, 7, 23, 64, 300};
  const int64_t nas[] = {0, 1, 3, 6, 8};
  const int64_t nvs[] = {1, 2, 63, 64, 65, 1100, 4097};
  const int64_t nauxs[] = {1, 17, 3000, 33000};
  for (int64_t nc : ncs)
    for (int64_t na : nas)
      for (int64_t nv : nvs)
        for (int64_t naux : nauxs)
          for (int prec : {0, 2})
            for (int terms = 1; terms <= 7; ++terms)
              for (int grad = 0; grad <= 1; ++grad) {
                dsrg_df_problem p = prob(nc, na, nv, naux);
                size_t b = 0;
                const dsrg_status st = dsrg_df_workspace_size(&p, prec, terms, grad, &b);
                CHECK(st == DSRG_OK && b > 0);
              }
  // rest, active, Laplace and CD sizes over a smaller grid
  for (int64_t nc : ncs)
    for (int64_t na : {1, 4, 8})
      for (int64_t nv : {1, 65, 1100}) {
        dsrg_df_problem p = prob(nc, na, nv, 300);
        size_t b = 0;
        CHECK(dsrg_df_active_workspace_size(&p, &b) == DSRG_OK && b > 0);
        dsrg_df_rest_problem r;
        std::memset(&r, 0, sizeof(r));
        r.base = p;
        b = 0;
        CHECK(dsrg_df_rest_workspace_size(&r, &b) == DSRG_OK && b > 0);
        for (int nq : {1, 16, DSRG_DF_MAX_LAPLACE_TERMS}) {
          b = 0;
          CHECK(dsrg_df_laplace_workspace_size(&p, nq, &b) == DSRG_OK && b > 0);
        }
      }
  for (int64_t nao : {1, 2, 170, 1000, DSRG_CD_MAX_NAO}) {
    dsrg_cd_problem c;
    c.nao = nao;
    c.M = fake();
    c.tol = 1e-5;
    c.max_rank = nao * (nao + 1) / 2;
    size_t b = 0;
    CHECK(dsrg_df_cholesky_workspace_size(&c, &b) == DSRG_OK && b > 0);
  }
}

// sizes at and beyond the documented limits: either a size or a clean
// refusal, never an overflowing computation
void limits() {
  const int64_t big[][4] = {{1 << 20, 8, 1 << 24, 1 << 24}, {1 << 20, 0, 1 << 24, 1},
                            {1, 0, 1 << 24, 1 << 24},       {(1 << 20) + 1, 0, 64, 64},
                            {64, 0, (1 << 24) + 1, 64},     {64, 0, 64, (1 << 24) + 1},
                            {INT64_MAX, 0, 1, 1},           {1, 0, INT64_MAX, 1}};
  for (const auto &d : big)
    for (int prec : {0, 2})
      for (int grad = 0; grad <= 1; ++grad) {
        dsrg_df_problem p = prob(d[0], d[1], d[2], d[3]);
        size_t b = 0;
        const dsrg_status st = dsrg_df_workspace_size(&p, prec, 7, grad, &b);
        CHECK(st == DSRG_OK || st == DSRG_ERR_UNSUPPORTED || st == DSRG_ERR_ARG);
        if (st == DSRG_OK) CHECK(b > 0);
      }
  dsrg_cd_problem c;
  c.nao = DSRG_CD_MAX_NAO + 1;
  c.M = fake();
  c.tol = 1e-5;
  c.max_rank = 10;
  size_t b = 0;
  CHECK(dsrg_df_cholesky_workspace_size(&c, &b) != DSRG_OK);
  c.nao = INT64_MAX;
  CHECK(dsrg_df_cholesky_workspace_size(&c, &b) != DSRG_OK);
  dsrg_df_problem p = prob(1 << 20, 8, 1 << 24, 1 << 24);
  CHECK(dsrg_df_laplace_workspace_size(&p, DSRG_DF_MAX_LAPLACE_TERMS, &b) != DSRG_ERR_HIP);
  CHECK(dsrg_df_active_workspace_size(&p, &b) != DSRG_ERR_HIP);
  dsrg_df_rest_problem r;
  std::memset(&r, 0, sizeof(r));
  r.base = p;
  CHECK(dsrg_df_rest_workspace_size(&r, &b) != DSRG_ERR_HIP);
  r.base = prob(INT64_MAX / 2, 8, INT64_MAX / 2, INT64_MAX / 2);
  CHECK(dsrg_df_rest_workspace_size(&r, &b) != DSRG_OK);
  // factor build, Fock matrix and rotation at huge sizes
  const int64_t hs[][3] = {{1 << 20, 1 << 20, 1 << 20}, {INT64_MAX / 4, 4, 4},
                           {4, INT64_MAX / 4, 4},       {4, 4, INT64_MAX / 4}};
  for (const auto &h : hs) {
    dsrg_dfgen_problem d;
    d.nao = h[0];
    d.naux = h[2];
    d.nfrz = 0;
    d.nc = 1;
    d.na = 1;
    d.nv = h[1] > 2 ? h[1] - 2 : 1;
    d.nmo = d.nc + d.na + d.nv;
    d.ao3 = d.J = d.C = fake();
    const dsrg_status st = dsrg_df_factors_workspace_size(&d, &b);
    CHECK(st == DSRG_OK || st == DSRG_ERR_UNSUPPORTED || st == DSRG_ERR_ARG);
    dsrg_fock_problem f;
    f.df = d;
    f.h = f.gamma1 = fake();
    const dsrg_status sf = dsrg_df_fock_workspace_size(&f, &b);
    CHECK(sf == DSRG_OK || sf == DSRG_ERR_UNSUPPORTED || sf == DSRG_ERR_ARG);
    dsrg_semican_problem sp;
    sp.nao = h[0];
    sp.nmo = d.nmo;
    sp.nfrz = 0;
    sp.nc = 1;
    sp.na = 1;
    sp.nv = d.nv;
    sp.F = sp.C = fake();
    const dsrg_status ss = dsrg_df_semicanonicalize_workspace_size(&sp, &b);
    CHECK(ss == DSRG_OK || ss == DSRG_ERR_UNSUPPORTED || ss == DSRG_ERR_ARG);
  }
  c.nao = DSRG_CD_MAX_NAO;
  c.max_rank = INT64_MAX;
  CHECK(dsrg_df_cholesky_workspace_size(&c, &b) == DSRG_ERR_ARG);
}

void energy_validation() {
  dsrg_df_problem p = prob(4, 2, 70, 33);
  double *E = fakew();
  size_t need = 0;
  CHECK(dsrg_df_workspace_size(&p, 0, 7, 0, &need) == DSRG_OK);
  // invalid sizes and scalars
  const int64_t bad[][4] = {{0, 2, 70, 33}, {4, -1, 70, 33}, {4, 2, 0, 33}, {4, 2, 70, 0}};
  for (const auto &d : bad) {
    dsrg_df_problem q = prob(d[0], d[1], d[2], d[3]);
    CHECK(dsrg_df_energy(&q, 0, 7, E, fakews(), need, nullptr) == DSRG_ERR_ARG);
    CHECK(std::strlen(dsrg_df_last_error()) > 0);
  }
  for (double s : {-1.0, (double)NAN, (double)INFINITY}) {
    dsrg_df_problem q = prob(4, 2, 70, 33, s);
    CHECK(dsrg_df_energy(&q, 0, 7, E, fakews(), need, nullptr) == DSRG_ERR_ARG);
  }
  dsrg_df_problem q = prob(4, DSRG_DF_MAX_ACTIVE + 1, 70, 33);
  CHECK(dsrg_df_energy(&q, 0, 7, E, fakews(), 1ull << 40, nullptr) == DSRG_ERR_UNSUPPORTED);
  q = prob(4, 2, 70, DSRG_DF_MAX_SLICE_NAUX + 1);
  CHECK(dsrg_df_energy(&q, DSRG_SPLIT_OZAKI, 7, E, fakews(), 1ull << 40, nullptr) ==
        DSRG_ERR_UNSUPPORTED);
  CHECK(dsrg_df_energy(&p, DSRG_SPLIT_BF16, 7, E, fakews(), need, nullptr) ==
        DSRG_ERR_UNSUPPORTED);
  // precision, term mask, pointers, workspace
  CHECK(dsrg_df_energy(&p, 7, 7, E, fakews(), need, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy(&p, 0, 0, E, fakews(), need, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy(&p, 0, 0x1000, E, fakews(), need, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy(nullptr, 0, 7, E, fakews(), need, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy(&p, 0, 7, nullptr, fakews(), need, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy(&p, 0, 7, fakew(0x20004), fakews(), need, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy(&p, 0, 7, E, nullptr, need, nullptr) == DSRG_ERR_WORKSPACE);
  CHECK(dsrg_df_energy(&p, 0, 7, E, fakews(), need - 1, nullptr) == DSRG_ERR_WORKSPACE);
  CHECK(dsrg_df_energy(&p, 0, 7, E, reinterpret_cast<void *>(0x40010), need, nullptr) ==
        DSRG_ERR_WORKSPACE);
  q = p;
  q.B_cv = nullptr;
  CHECK(dsrg_df_energy(&q, 0, 7, E, fakews(), need, nullptr) == DSRG_ERR_ARG);
  q = p;
  q.eps_v = reinterpret_cast<const double *>(0x10004);
  CHECK(dsrg_df_energy(&q, 0, 7, E, fakews(), need, nullptr) == DSRG_ERR_ARG);
  // the allocation-free variant and the gradient
  CHECK(dsrg_df_energy_noalloc(&p, 0, 7 | DSRG_OPT_KERNEL_TIMING, E, nullptr) == DSRG_ERR_ARG);
  q = prob(23, 6, 1100, 3000);
  CHECK(dsrg_df_energy_noalloc(&q, 0, 7, E, nullptr) == DSRG_ERR_UNSUPPORTED);
  double *g = fakew(0x30000);
  size_t gneed = 0;
  CHECK(dsrg_df_workspace_size(&p, 0, 7, 1, &gneed) == DSRG_OK && gneed > need);
  CHECK(dsrg_df_energy_backward(&p, 0, 7, nullptr, g, g, g, g, g, g, g, E, fakews(), gneed,
                                nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy_backward(&p, 0, 7, g, nullptr, g, g, g, g, g, g, E, fakews(), gneed,
                                nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy_backward(&p, 0, 7, g, g, g, g, g, g, g, g, E, fakews(), gneed - 8,
                                nullptr) == DSRG_ERR_WORKSPACE);
  CHECK(dsrg_df_sign_check(nullptr) == DSRG_ERR_ARG);
  int64_t *st = reinterpret_cast<int64_t *>(0x10000);
  void *sk = reinterpret_cast<void *>(0x20000);
  CHECK(dsrg_df_mfma_probe(2, 256, 16, st, sk, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_mfma_probe(0, 0, 16, st, sk, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_mfma_probe(1, 65537, 16, st, sk, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_mfma_probe(0, 256, 0, st, sk, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_mfma_probe(0, 256, (int64_t(1) << 24) + 1, st, sk, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_mfma_probe(1, 256, 16, nullptr, sk, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_mfma_probe(1, 256, 16, st + 0, reinterpret_cast<char *>(sk) + 4, nullptr) ==
        DSRG_ERR_ARG);
}

void other_entry_points() {
  size_t b = 0;
  dsrg_df_problem p = prob(4, 2, 70, 33);
  // F4-F8
  CHECK(dsrg_df_active_workspace_size(nullptr, &b) == DSRG_ERR_ARG);
  CHECK(dsrg_df_energy_active(&p, nullptr, 0, fakew(), fakews(), 1ull << 40, nullptr) ==
        DSRG_ERR_ARG);
  // Table I terms
  dsrg_df_rest_problem r;
  std::memset(&r, 0, sizeof(r));
  r.base = p;
  CHECK(dsrg_df_energy_rest(&r, 0, fakew(), fakews(), 1ull << 40, nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_cumulants(0, fake(), fake(), fake(), fakew(), fakew(), nullptr) == DSRG_ERR_ARG);
  CHECK(dsrg_df_cumulants(DSRG_DF_MAX_ACTIVE + 1, fake(), fake(), fake(), fakew(), fakew(),
                          nullptr) != DSRG_OK);
  // DF factors and the Fock matrix
  dsrg_dfgen_problem d;
  d.nao = 20;
  d.nmo = 20;
  d.naux = 50;
  d.nfrz = 1;
  d.nc = 3;
  d.na = 2;
  d.nv = 14;
  d.ao3 = d.J = d.C = fake();
  CHECK(dsrg_df_factors_workspace_size(&d, &b) == DSRG_OK && b > 0);
  dsrg_dfgen_problem e = d;
  e.nv = 15;   // nfrz + nc + na + nv > nmo
  CHECK(dsrg_df_factors_workspace_size(&e, &b) == DSRG_ERR_ARG);
  e = d;
  e.J = nullptr;
  CHECK(dsrg_df_factors_workspace_size(&e, &b) == DSRG_OK && b > 0);
  CHECK(dsrg_df_factors(&d, 0, nullptr, fakew(), fakew(), fakew(), fakews(), 1ull << 40,
                        nullptr) == DSRG_ERR_ARG);
  dsrg_fock_problem f;
  f.df = d;
  f.h = f.gamma1 = fake();
  CHECK(dsrg_df_fock_workspace_size(&f, &b) == DSRG_OK && b > 0);
  CHECK(dsrg_df_fock(&f, 0, nullptr, fakews(), 1ull << 40, nullptr) == DSRG_ERR_ARG);
  // semicanonical rotation
  dsrg_semican_problem sp;
  sp.nao = 20;
  sp.nmo = 20;
  sp.nfrz = 1;
  sp.nc = 3;
  sp.na = 2;
  sp.nv = 14;
  sp.F = fake();
  sp.C = nullptr;
  CHECK(dsrg_df_semicanonicalize_workspace_size(&sp, &b) == DSRG_OK && b > 0);
  sp.nv = 15;   // nfrz + nc + na + nv > nmo
  CHECK(dsrg_df_semicanonicalize_workspace_size(&sp, &b) == DSRG_ERR_ARG);
  // CD
  dsrg_cd_problem c;
  c.nao = 10;
  c.M = fake();
  c.tol = 1e-5;
  c.max_rank = 56;   // > npair = 55
  CHECK(dsrg_df_cholesky_workspace_size(&c, &b) == DSRG_ERR_ARG);
  c.max_rank = 20;
  c.tol = -1.0;
  CHECK(dsrg_df_cholesky_workspace_size(&c, &b) == DSRG_ERR_ARG);
  // Laplace fit (host): valid, then invalid ranges and counts
  double t[DSRG_DF_MAX_LAPLACE_TERMS], w[DSRG_DF_MAX_LAPLACE_TERMS], err = -1.0;
  CHECK(dsrg_df_laplace_fit(0.5, 0.8, 12.0, 12, t, w, &err) == DSRG_OK && err >= 0.0 &&
        err < 1e-3);
  CHECK(dsrg_df_laplace_fit(0.5, 0.0, 12.0, 12, t, w, &err) == DSRG_ERR_ARG);
  CHECK(dsrg_df_laplace_fit(0.5, 2.0, 1.0, 12, t, w, &err) == DSRG_ERR_ARG);
  CHECK(dsrg_df_laplace_fit(0.5, 0.8, 12.0, 0, t, w, &err) == DSRG_ERR_ARG);
  CHECK(dsrg_df_laplace_fit(0.5, 0.8, 12.0, DSRG_DF_MAX_LAPLACE_TERMS + 1, t, w, &err) !=
        DSRG_OK);
  CHECK(dsrg_df_laplace_fit(-1.0, 0.8, 12.0, 12, t, w, &err) == DSRG_ERR_ARG);
  CHECK(dsrg_df_laplace_fit(0.5, 0.8, 12.0, 12, nullptr, w, &err) == DSRG_ERR_ARG);
  // timing and the gradient block bound
  std::vector<char> longname(300, 'a');
  longname.back() = 0;
  CHECK(dsrg_df_timing_filter(longname.data()) == DSRG_ERR_ARG);
  CHECK(dsrg_df_timing_filter("ccvv_fp64,gemm_adj_fp64") == DSRG_OK);
  CHECK(dsrg_df_timing_filter(nullptr) == DSRG_OK);
  double ms[4];
  const char *names[4];
  CHECK(dsrg_df_kernel_times(ms, names, 4) == 0);
  const size_t old = dsrg_df_gradient_block_bytes();
  CHECK(dsrg_df_set_gradient_block_bytes((size_t)1 << 51) == DSRG_ERR_ARG);
  CHECK(dsrg_df_set_gradient_block_bytes(1000) == DSRG_OK);
  dsrg_df_problem q = prob(7, 3, 100, 40);
  CHECK(dsrg_df_workspace_size(&q, 0, 7, 1, &b) == DSRG_OK && b > 0);
  CHECK(dsrg_df_set_gradient_block_bytes(0) == DSRG_OK);
  CHECK(dsrg_df_gradient_block_bytes() == old);
  CHECK(dsrg_df_version() >= 100);
}

}  // namespace

int main() {
  workspace_grid();
  limits();
  energy_validation();
  other_entry_points();
  std::printf("%d checks, %d failed\n", g_checks, g_fail);
  if (g_fail == 0) std::printf("checks passed\n");
  return g_fail == 0 ? 0 : 1;
}
