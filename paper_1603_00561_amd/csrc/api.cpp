// Host side of the libdsrgdf C ABI: argument validation, workspace planning
// and kernel launches. Nothing here allocates device memory or waits on the
// device; every error is found before the first launch.
#include <math.h>
#include <cmath>
#include <stdarg.h>
#include <stdio.h>
#include <algorithm>
#include <atomic>
#include <string.h>

#include "../../include/dsrg_df.h"
#include "internal.h"

namespace {

thread_local char g_err[512] = "";

static_assert(DSRG_DF_NOALLOC_SCRATCH_BYTES == dsrg::kNoAllocScratchBytes,
              "the header states the static scratch size");

// bound on the gradient's per-block adjoint-tile region (process-wide)
std::atomic<int64_t> g_grad_block_bytes{dsrg::kGradBlockBytes};

dsrg_status fail(dsrg_status code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

// ---- per-kernel timing: one table per host thread ----
// Calls that set DSRG_OPT_KERNEL_TIMING append an event pair per kernel
// (only the kernels the filter names, when one is set);
// dsrg_df_kernel_times() reads and clears the table.
struct TimerTable {
  static constexpr int kMax = 512;
  static constexpr int kFilter = 256;
  hipEvent_t ev[2 * kMax] = {};
  const char *name[kMax] = {};
  int n = 0;          // kernels recorded since the last read
  int created = 0;    // events created so far
  int device = -1;
  bool active = false;
  bool skip = false;  // the kernel between timer_begin and timer_end is not recorded
  char filter[kFilter] = {};   // comma-separated kernel names; empty: every kernel
};

// name is one of the comma-separated entries of list
bool in_list(const char *list, const char *name) {
  const size_t len = strlen(name);
  for (const char *p = list; *p;) {
    const char *q = strchr(p, ',');
    const size_t n = q ? (size_t)(q - p) : strlen(p);
    if (n == len && strncmp(p, name, n) == 0) return true;
    if (!q) break;
    p = q + 1;
  }
  return false;
}
thread_local TimerTable g_timer;

void timer_reset(bool on) {
  g_timer.active = false;
  if (!on) return;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  if (g_timer.device != dev) {
    for (int k = 0; k < g_timer.created; ++k) (void)hipEventDestroy(g_timer.ev[k]);
    g_timer.created = 0;
    g_timer.n = 0;
    g_timer.device = dev;
  }
  g_timer.active = true;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

// Validate sizes, scalar arguments and the option bits; fill the plan.
dsrg_status make_plan(const dsrg_df_problem *p, int precision, int terms, int with_grad,
                      dsrg::Plan &pl) {
  using namespace dsrg;
  if (!p) return fail(DSRG_ERR_ARG, "problem pointer is NULL");
  if (p->nc < 1) return fail(DSRG_ERR_ARG, "nc must be >= 1 (got %lld)", (long long)p->nc);
  if (p->nv < 1) return fail(DSRG_ERR_ARG, "nv must be >= 1 (got %lld)", (long long)p->nv);
  if (p->naux < 1) return fail(DSRG_ERR_ARG, "naux must be >= 1 (got %lld)", (long long)p->naux);
  if (p->na < 0) return fail(DSRG_ERR_ARG, "na must be >= 0 (got %lld)", (long long)p->na);
  if (!(p->s >= 0.0) || !isfinite(p->s))
    return fail(DSRG_ERR_ARG, "s must be finite and >= 0 (got %g)", p->s);
  if (precision != DSRG_FP64 && precision != DSRG_SPLIT_BF16 && precision != DSRG_SPLIT_OZAKI)
    return fail(DSRG_ERR_ARG, "unknown precision %d", precision);
  const int term_bits = terms & DSRG_TERM_ALL;
  if (term_bits == 0) return fail(DSRG_ERR_ARG, "term mask selects no term (0x%x)", terms);
  if (terms & ~(DSRG_TERM_ALL | DSRG_OPT_ATOMIC_REDUCE | DSRG_OPT_KERNEL_TIMING |
                DSRG_OPT_CHECK_SIGNS))
    return fail(DSRG_ERR_ARG, "unknown bits in term mask 0x%x", terms);
  const bool need_act = p->na > 0 && (term_bits & (DSRG_TERM_CAVV | DSRG_TERM_CCAV));
  if (need_act && p->na > DSRG_DF_MAX_ACTIVE)
    return fail(DSRG_ERR_UNSUPPORTED, "na = %lld exceeds the compiled maximum %d",
                (long long)p->na, DSRG_DF_MAX_ACTIVE);
  // index ranges used by the kernels (int for orbital indices, int64 offsets)
  if (p->nc > (1 << 20) || p->nv > (1 << 24) || p->naux > (1 << 24))
    return fail(DSRG_ERR_UNSUPPORTED, "dimensions too large (nc %lld, nv %lld, naux %lld)",
                (long long)p->nc, (long long)p->nv, (long long)p->naux);
  if (precision == DSRG_SPLIT_BF16)
    return fail(DSRG_ERR_UNSUPPORTED,
                "precision %d is not implemented (three BF16 products cannot reach 1e-6 Eh)",
                precision);
  if (precision == DSRG_SPLIT_OZAKI && p->naux > DSRG_DF_MAX_SLICE_NAUX)
    return fail(DSRG_ERR_UNSUPPORTED,
                "naux = %lld exceeds %d, beyond which int32 slice sums could overflow",
                (long long)p->naux, DSRG_DF_MAX_SLICE_NAUX);

  pl.nc = p->nc;
  pl.na = p->na;
  pl.nv = p->nv;
  pl.naux = p->naux;
  pl.s = p->s;
  pl.precision = precision;
  pl.terms = term_bits;
  pl.atomic_reduce = (terms & DSRG_OPT_ATOMIC_REDUCE) != 0;
  pl.with_grad = with_grad != 0;
  pl.naux_p = round_up(pl.naux, kChunk);
  pl.ntv = ceil_div(pl.nv, kPanel);
  pl.ntv_s = (precision == DSRG_SPLIT_OZAKI) ? round_up(pl.ntv, 2) : pl.ntv;
  pl.xld = pl.ntv_s * kPanel;
  {
    // every count and byte size formed below is at most one of these
    // products (panels and slices, the adjoint tiles of all core pairs, the
    // CAVV integrals, the work lists, the CCAV integrals with up to 1024
    // auxiliary segments): refuse a problem for which one of them would not
    // fit in 62 bits, so that the int64 and size_t sums here never overflow
    const double nc = (double)pl.nc, na = (double)pl.na, W = (double)pl.xld,
                 q = (double)pl.naux_p;
    const double big = std::max({8.0 * (nc + na) * W * q, 8.0 * (nc * W) * (nc * W),
                                 8.0 * nc * na * W * W, (nc * nc) * (W * W),
                                 8.0 * 1024.0 * (nc * W) * (nc * na + 16.0)});
    if (!(big < 0x1p62))
      return fail(DSRG_ERR_UNSUPPORTED,
                  "problem too large (nc %lld, na %lld, nv %lld, naux %lld): its workspace "
                  "sizes would not fit in 64 bits",
                  (long long)pl.nc, (long long)pl.na, (long long)pl.nv, (long long)pl.naux);
  }

  const int64_t npo = tri_off(pl.nc), ntpo = tri_off(pl.ntv);
  // one slot per (core pair, tile pair): 64-wide tiles in FP64, 128-wide on slices
  const int64_t nt2 = pl.ntv_s / 2;
  pl.n_ccvv = !(term_bits & DSRG_TERM_CCVV) ? 0
              : (precision == DSRG_SPLIT_OZAKI)
                  ? (pl.nc * (pl.nc + 1) / 2) * (nt2 * (nt2 + 1) / 2)
                  : (npo * ntpo + npo * pl.ntv + pl.nc * ntpo + pl.nc * pl.ntv);
  const bool split = precision == DSRG_SPLIT_OZAKI;
  const bool has_cavv = (term_bits & DSRG_TERM_CAVV) && pl.na > 0;
  const bool has_ccav = (term_bits & DSRG_TERM_CCAV) && pl.na > 0;
  pl.nqc = ceil_div(pl.naux, 32);
  // CAVV energy: batches of (me|uf) integrals of at most 4 GiB (one batch up
  // to nc = 23, na = 6, nv = 1100 and beyond)
  const bool xbatch = has_cavv;
  const int64_t Wg = pl.ntv * kPanel;   // padded virtual orbitals per orbital (FP64 tiles)
  if (xbatch) {
    const int64_t per_m = pl.na * pl.xld * pl.xld * 8;
    pl.cavv_mb = ((int64_t)4 << 30) / per_m;
    if (pl.cavv_mb < 1) pl.cavv_mb = 1;
    if (pl.cavv_mb > pl.nc) pl.cavv_mb = pl.nc;
  } else {
    pl.cavv_mb = 0;
  }
  // Gradient: the adjoint tiles are formed per block of gb core orbitals (the
  // CCVV tiles of one block pair, the CAVV integrals and adjoint rows of one
  // block) in one region of at most kGradBlockBytes, so the workspace holds
  // O(gb^2 nv^2 + gb na nv^2) values, never the nc^2 nv^2 of all pairs.
  size_t gblk_bytes = 0;
  if (pl.with_grad) {
    const bool ccvv = (term_bits & DSRG_TERM_CCVV) != 0;
    auto need = [&](int64_t b) {
      size_t n = 0;
      if (ccvv) n = sizeof(double) * (size_t)(b * Wg) * (size_t)(b * Wg);
      if (has_cavv) {
        const size_t xb = sizeof(double) * (size_t)(b * pl.na) * (size_t)pl.xld * (size_t)pl.xld;
        const size_t g2 = sizeof(double) * (size_t)(b * Wg) * (size_t)(pl.na * Wg);
        n = std::max(n, align256(xb) + g2);
      }
      return n;
    };
    const size_t budget = (size_t)g_grad_block_bytes.load();
    int64_t b = pl.nc;
    while (b > 1 && need(b) > budget) --b;
    pl.ngb = ceil_div(pl.nc, b);
    pl.gb = ceil_div(pl.nc, pl.ngb);   // balanced blocks, the last one no larger
    gblk_bytes = need(pl.gb);
    if (has_cavv) pl.cavv_mb = pl.gb;
  }
  pl.n_cavv = has_cavv ? pl.nc * (ceil_div(pl.nv, 16) * (ceil_div(pl.nv, 16) + 1) / 2) : 0;
  pl.ccav_cols = round_up(pl.nc * pl.na, 16);
  // forward: one slot per (m <= n, 256 virtual orbitals); adjoint: per (m <= n, 64-tile)
  pl.n_ccav = has_ccav
                  ? (pl.nc * (pl.nc + 1) / 2) * (pl.with_grad ? pl.ntv : ceil_div(pl.nv, 256))
                  : 0;
  const int64_t maxgrid = ((int64_t)1 << 31) - 1;
  if (pl.n_ccvv > maxgrid || pl.n_cavv > maxgrid || pl.n_ccav > maxgrid)
    return fail(DSRG_ERR_UNSUPPORTED, "work list exceeds one launch grid");

  size_t off = 0;
  // FP64 panels: every FP64 kernel; in the slice path only the forward CCAV
  // product (the gradient's CCAV integrals come from one product over the
  // inputs, and its other adjoint tiles from the slices)
  const bool fp64_tiles = !split;
  pl.off_pcv = off;
  if (fp64_tiles || (has_ccav && !pl.with_grad))
    off = align256(off + sizeof(double) * (size_t)(pl.nc * pl.ntv * pl.naux_p * kPanel));
  pl.off_pav = off;
  if (!split && has_cavv)
    off = align256(off + sizeof(double) * (size_t)(pl.na * pl.ntv * pl.naux_p * kPanel));
  pl.off_pca = off;
  pl.off_j = off;
  if (has_ccav) {
    if (pl.with_grad) {
      // B_ca panels of the FP64 adjoint products
      if (!split) off = align256(off + sizeof(double) * (size_t)(pl.nc * pl.naux_p * kActPanel));
      // the CCAV integrals J[(m,e)][(n,u)] of the adjoint tiles
      pl.off_j = off;
      off = align256(off + sizeof(double) * (size_t)(pl.nc * pl.nv) * (size_t)(pl.nc * pl.na));
    } else {
      off = align256(off + sizeof(double) * (size_t)(pl.naux_p * pl.ccav_cols));
      pl.off_j = off;
      off = align256(off + sizeof(double) *
                               (size_t)(pl.nc * pl.ntv * kPanel) * (size_t)pl.ccav_cols);
      // with few 64-row panels (nc ntv of them) the contraction is split over
      // auxiliary segments, summed in a fixed order, to fill the chip
      const int64_t nseg = j_segments(pl.nc * pl.ntv, pl.ccav_cols, pl.naux_p);
      if (nseg > 1) {
        pl.ccav_split = true;
        pl.off_jscr = off;
        off = align256(off + sizeof(double) * (size_t)nseg *
                                 (size_t)(pl.nc * pl.ntv * kPanel) * (size_t)pl.ccav_cols);
      }
    }
  }
  pl.off_s8c = pl.off_s8a = pl.off_sigc = pl.off_siga = pl.off_diag = pl.off_xb = pl.off_scr =
      off;
  if (split) {
    const size_t chunk = 5 * kPanel * 32;   // bytes per (panel, 32 auxiliary indices)
    const size_t colc = (size_t)(pl.nc * pl.ntv_s * kPanel), cola = (size_t)(pl.na * pl.ntv_s * kPanel);
    pl.off_s8c = off;
    off = align256(off + chunk * (size_t)(pl.nc * pl.ntv_s * pl.nqc));
    pl.off_sigc = off;
    off = align256(off + sizeof(double) * colc);
    pl.off_diag = off;
    off = align256(off + sizeof(double) * colc);
    pl.off_scr = off;
    off = align256(off + sizeof(double) * 2 * 32 * (colc > cola ? colc : cola));
    if (has_cavv) {
      pl.off_s8a = off;
      off = align256(off + chunk * (size_t)(pl.na * pl.ntv_s * pl.nqc));
      pl.off_siga = off;
      off = align256(off + sizeof(double) * cola);
    }
  }
  if (xbatch && !pl.with_grad) {
    pl.off_xb = off;
    off = align256(off + sizeof(double) * (size_t)(pl.cavv_mb * pl.na) * (size_t)pl.xld *
                             (size_t)pl.xld);
  }
  pl.off_xs = off;
  if (split && (term_bits & DSRG_TERM_CCVV))
    off = align256(off + sizeof(double) * (size_t)(kSlicePersistWG * kSliceXsDoubles) +
                   kSliceCounterBytes);
  pl.off_gs = pl.off_g2 = pl.off_g3 = off;
  if (pl.with_grad) {
    // one region: the CCVV tiles of a block pair (off_gs), or the CAVV
    // integral batch (off_xb) followed by the adjoint rows G2 of the block
    // (off_g2); the phases run one after the other on the stream
    pl.off_gs = pl.off_xb = off;
    pl.off_g2 = off;
    if (xbatch)
      pl.off_g2 = align256(off + sizeof(double) * (size_t)(pl.gb * pl.na) * (size_t)pl.xld *
                                     (size_t)pl.xld);
    off = align256(off + gblk_bytes);
    const int64_t Np = pl.nc * Wg;
    if (pl.na > 0 && (term_bits & DSRG_TERM_CCAV)) {
      pl.off_g3 = off;
      off = align256(off + sizeof(double) * (size_t)Np * (size_t)(pl.nc * kActPanel));
    }
    {
      // adjoint products with too few output tiles are split over K into
      // segments (partial products summed in a fixed order); on slices every
      // product longer than one exact int32 segment is split too: room for
      // the largest. Shapes (ncols, GP, nvalid, K) as the products take them,
      // for the full-size and the last (smaller) core block.
      const int64_t gp = Wg, n2 = pl.na * Wg, n3 = pl.nc * kActPanel;
      const int64_t wk = round_up(pl.nv, kQChunk);
      const int64_t n3p = round_up(n3, kQChunk);
      const int64_t blast = pl.nc - (pl.ngb - 1) * pl.gb;
      int64_t most = 0;
      // (Kk: the int8 product's contraction length, which runs over wk per
      // orbital; its output columns are the valid ones side by side)
      auto consider = [&](int64_t ncols, int64_t GPc, int64_t nvalid, int64_t K, int64_t Kk) {
        if (ncols <= 0 || K <= 0) return;
        int64_t nseg = adj_fp64_segments(pl.naux, ncols, GPc, nvalid, K);
        const int64_t ncol = adj_out_cols(ncols, GPc, nvalid);
        if (split) {
          int64_t segc = 0;
          nseg = i8_segments(pl.naux, ncol, Kk, segc);
        }
        if (nseg > 1) most = std::max(most, nseg * pl.naux * ncol);
      };
      for (const int64_t bi : {pl.gb, blast})
        for (const int64_t bj : {pl.gb, blast}) {
          if (term_bits & DSRG_TERM_CCVV) consider(bj * gp, gp, pl.nv, bi * gp, bi * wk);
          if (has_cavv) {
            consider(bi * gp, gp, pl.nv, n2, pl.na * wk);
            consider(n2, gp, pl.nv, bi * gp, bi * wk);
          }
        }
      if (has_ccav) {
        consider(Np, gp, pl.nv, n3, n3p);
        consider(n3, kActPanel, pl.na, Np, pl.nc * wk);
      }
      if (most > 0) {
        pl.off_gpart = off;
        pl.gpart_doubles = most;
        off = align256(off + sizeof(double) * (size_t)most);
      }
    }
  }
  pl.off_SA1 = pl.off_SA2 = pl.off_SB = pl.off_sigA1 = pl.off_sigA2 = pl.off_sigB =
      pl.off_opmax = off;
  if (split && pl.with_grad) {
    // operand slices of the int8 adjoint products (5 bytes per element) and
    // their row scales; the G operands share one buffer, used in turn. A
    // contraction over (orbital, virtual) runs over Wk = nv rounded up to 32
    // per orbital, and operand rows over (orbital, virtual) hold the nv valid
    // ones side by side.
    const size_t Wk = (size_t)round_up(pl.nv, 32), nv = (size_t)pl.nv;
    const size_t Np = (size_t)pl.nc * Wk, N2 = (size_t)pl.na * Wk,
                 N3 = (size_t)(pl.nc * pl.na);
    const size_t N3p = (size_t)round_up(pl.nc * kActPanel, 32);
    const size_t RA = (size_t)round_up(pl.naux, 128);
    const size_t gb = (size_t)pl.gb;
    auto r128 = [](size_t n) { return (size_t)round_up((int64_t)n, 128); };
    const bool act = pl.na > 0 && (term_bits & (DSRG_TERM_CAVV | DSRG_TERM_CCAV));
    size_t sb = 0, rbmax = 0;
    if (term_bits & DSRG_TERM_CCVV) sb = std::max(sb, r128(gb * nv) * gb * Wk);
    if (pl.na > 0 && (term_bits & DSRG_TERM_CAVV))
      sb = std::max(sb, std::max(r128(gb * nv) * N2, r128(pl.na * nv) * gb * Wk));
    if (pl.na > 0 && (term_bits & DSRG_TERM_CCAV))
      sb = std::max(sb, std::max(r128(pl.nc * nv) * N3p, r128(N3) * Np));
    rbmax = std::max(r128(pl.nc * nv), std::max(r128(pl.na * nv), r128(N3)));
    pl.off_SA1 = off;
    off = align256(off + 5 * RA * Np);
    pl.off_SA2 = off;
    if (act) off = align256(off + 5 * RA * std::max(N2, N3p));
    pl.off_SB = off;
    off = align256(off + 5 * sb);
    pl.off_sigA1 = off;
    off = align256(off + sizeof(double) * RA);
    pl.off_sigA2 = off;
    off = align256(off + sizeof(double) * RA);
    pl.off_sigB = off;
    off = align256(off + sizeof(double) * rbmax);
    pl.off_opmax = off;
    off = align256(off + sizeof(double) * 32 * std::max(RA, rbmax));
  }
  pl.off_ctr = off;
  off = align256(off + 64);
  pl.off_slots = off;
  pl.slot_base[0] = 0;
  pl.slot_base[1] = pl.n_ccvv;
  pl.slot_base[2] = pl.n_ccvv + pl.n_cavv;
  off = align256(off + sizeof(double) * (size_t)(pl.n_ccvv + pl.n_cavv + pl.n_ccav + 1));
  pl.off_acc = off;
  off = align256(off + sizeof(double) * 4);
  pl.total = off;
  return DSRG_OK;
}

dsrg_status check_inputs(const dsrg_df_problem *p, const dsrg::Plan &pl) {
  if (!p->B_cv || !aligned8(p->B_cv)) return fail(DSRG_ERR_ARG, "B_cv is NULL or misaligned");
  if (!p->eps_c || !aligned8(p->eps_c)) return fail(DSRG_ERR_ARG, "eps_c is NULL or misaligned");
  if (!p->eps_v || !aligned8(p->eps_v)) return fail(DSRG_ERR_ARG, "eps_v is NULL or misaligned");
  const bool cavv = pl.na > 0 && (pl.terms & DSRG_TERM_CAVV);
  const bool ccav = pl.na > 0 && (pl.terms & DSRG_TERM_CCAV);
  if (cavv && (!p->B_av || !aligned8(p->B_av)))
    return fail(DSRG_ERR_ARG, "B_av is NULL or misaligned");
  if (ccav && (!p->B_ca || !aligned8(p->B_ca)))
    return fail(DSRG_ERR_ARG, "B_ca is NULL or misaligned");
  if ((cavv || ccav) && (!p->eps_a || !aligned8(p->eps_a)))
    return fail(DSRG_ERR_ARG, "eps_a is NULL or misaligned");
  if ((cavv || ccav) && (!p->gamma1 || !aligned8(p->gamma1)))
    return fail(DSRG_ERR_ARG, "gamma1 is NULL or misaligned");
  return DSRG_OK;
}

dsrg_status check_workspace(const dsrg::Plan &pl, void *ws, size_t ws_bytes) {
  if (ws_bytes < pl.total)
    return fail(DSRG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, pl.total);
  if (!ws) return fail(DSRG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) & 255u)
    return fail(DSRG_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  return DSRG_OK;
}

// Plan of the F4-F8 entry point (FP64): sizes, validation of the scalars and
// the workspace layout.
dsrg_status make_active_plan(const dsrg_df_problem *p, dsrg::ActivePlan &pl) {
  using namespace dsrg;
  if (!p) return fail(DSRG_ERR_ARG, "problem pointer is NULL");
  if (p->nc < 1) return fail(DSRG_ERR_ARG, "nc must be >= 1 (got %lld)", (long long)p->nc);
  if (p->nv < 1) return fail(DSRG_ERR_ARG, "nv must be >= 1 (got %lld)", (long long)p->nv);
  if (p->naux < 1) return fail(DSRG_ERR_ARG, "naux must be >= 1 (got %lld)", (long long)p->naux);
  if (p->na < 0) return fail(DSRG_ERR_ARG, "na must be >= 0 (got %lld)", (long long)p->na);
  if (!(p->s >= 0.0) || !isfinite(p->s))
    return fail(DSRG_ERR_ARG, "s must be finite and >= 0 (got %g)", p->s);
  if (p->na > DSRG_DF_MAX_ACTIVE)
    return fail(DSRG_ERR_UNSUPPORTED, "na = %lld exceeds the compiled maximum %d",
                (long long)p->na, DSRG_DF_MAX_ACTIVE);
  if (p->nc > (1 << 20) || p->nv > (1 << 24) || p->naux > (1 << 24))
    return fail(DSRG_ERR_UNSUPPORTED, "dimensions too large (nc %lld, nv %lld, naux %lld)",
                (long long)p->nc, (long long)p->nv, (long long)p->naux);
  pl.nc = p->nc;
  pl.na = p->na;
  pl.nv = p->nv;
  pl.naux = p->naux;
  pl.s = p->s;
  pl.naux_p = round_up(pl.naux, kChunk);
  pl.ntv = ceil_div(pl.nv, kPanel);
  pl.W = pl.ntv * kPanel;
  pl.ncC = round_up(pl.nc * pl.na, 16);
  pl.ncA = round_up(pl.na * pl.na, 16);
  // F4, F5, F6: at most kActPairGrid workgroups of four waves (elements
  // (e f), (m n), (m e) taken grid-stride); F7, F8: one workgroup per e, m
  auto pair_grid = [&](int64_t n) { return std::min(ceil_div(n, 4), kActPairGrid); };
  const int64_t nslot[5] = {pair_grid(pl.nv * pl.nv), pair_grid(pl.nc * pl.nc),
                            pair_grid(pl.nc * pl.nv), pl.nv, pl.nc};
  const int64_t maxgrid = ((int64_t)1 << 31) - 1;
  int64_t base = 0;
  for (int t = 0; t < 5; ++t) {
    if (nslot[t] > maxgrid) return fail(DSRG_ERR_UNSUPPORTED, "work list exceeds one launch grid");
    pl.slot_base[t] = base;
    pl.slot_count[t] = pl.na > 0 ? nslot[t] : 0;
    base += pl.slot_count[t];
  }
  size_t off = 0;
  auto take = [&](size_t doubles) {
    const size_t at = off;
    off = align256(off + sizeof(double) * doubles);
    return at;
  };
  const size_t na = (size_t)pl.na, nc = (size_t)pl.nc, W = (size_t)pl.W;
  const size_t np = (size_t)pl.naux_p, ntv = (size_t)pl.ntv;
  if (pl.na > 0) {
    pl.off_pav = take(na * ntv * np * kPanel);
    pl.off_pcv = take(nc * ntv * np * kPanel);
    pl.off_pca = take(nc * np * kPanel);
    pl.off_rca = take(np * (size_t)pl.ncC);
    pl.off_raa = take(np * (size_t)pl.ncA);
    pl.off_x = take(na * na * W * W);
    pl.off_ja1 = take(na * W * (size_t)pl.ncC);
    pl.off_ja2 = take(nc * W * (size_t)pl.ncA);
    pl.off_jc1 = take(na * W * (size_t)pl.ncA);
    pl.off_jk = take(nc * kPanel * (size_t)pl.ncC);
    pl.off_je = take(nc * kPanel * (size_t)pl.ncA);
    // scratch of the segmented integral blocks: the largest segments x block
    const int64_t jb[5][2] = {{pl.na * pl.ntv, pl.ncC}, {pl.nc * pl.ntv, pl.ncA},
                              {pl.na * pl.ntv, pl.ncA}, {pl.nc, pl.ncC}, {pl.nc, pl.ncA}};
    size_t jpart = 0;
    for (const auto &b : jb)
      jpart = std::max(jpart, (size_t)(j_segments(b[0], b[1], pl.naux_p) * b[0] * kPanel * b[1]));
    pl.off_jpart = take(jpart);
    pl.off_ctr = off;
    off = align256(off + 64);
  } else {
    pl.off_pav = pl.off_pcv = pl.off_pca = pl.off_rca = pl.off_raa = pl.off_x = pl.off_ja1 =
        pl.off_ja2 = pl.off_jc1 = pl.off_jk = pl.off_je = pl.off_jpart = pl.off_ctr = off;
  }
  pl.off_slots = take((size_t)base + 1);
  pl.total = off;
  return DSRG_OK;
}

// Plan of the density-fitting factor build: validation of the sizes and the
// workspace layout.
dsrg_status make_df_plan(const dsrg_dfgen_problem *p, dsrg::DFPlan &pl) {
  using namespace dsrg;
  if (!p) return fail(DSRG_ERR_ARG, "problem pointer is NULL");
  if (p->nao < 1 || p->naux < 1 || p->nc < 1 || p->nv < 1 || p->na < 0 || p->nfrz < 0)
    return fail(DSRG_ERR_ARG, "sizes must satisfy nao, naux, nc, nv >= 1 and na, nfrz >= 0");
  if (p->nmo < p->nfrz + p->nc + p->na + p->nv)
    return fail(DSRG_ERR_ARG, "nmo = %lld is smaller than nfrz + nc + na + nv",
                (long long)p->nmo);
  if (p->nao > (1 << 20) || p->naux > (1 << 20) || p->nmo > (1 << 20))
    return fail(DSRG_ERR_UNSUPPORTED, "dimensions too large");
  pl.nao = p->nao;
  pl.nmo = p->nmo;
  pl.naux = p->naux;
  pl.nfrz = p->nfrz;
  pl.nc = p->nc;
  pl.na = p->na;
  pl.nv = p->nv;
  const size_t np = (size_t)(pl.nc + pl.na), nq = (size_t)(pl.na + pl.nv);
  const size_t nx = (size_t)pl.naux;
  size_t off = 0;
  auto take = [&](size_t doubles) {
    const size_t at = off;
    off = align256(off + sizeof(double) * doubles);
    return at;
  };
  pl.metric = p->J != nullptr;
  pl.off_t = take(nx * np * (size_t)pl.nao);
  pl.off_y = take(nx * np * nq);
  if (pl.metric) {
    pl.off_l = take(nx * nx);
    pl.off_x = take(nx * nx);
    pl.off_tmp = take(nx * nx);   // L21 blocks of the recursive metric factor, at their positions
    pl.off_bf = take(nx * np * nq);
  } else {
    pl.off_l = pl.off_x = pl.off_tmp = pl.off_bf = off;
  }
  pl.total = off;
  return DSRG_OK;
}

}  // namespace

namespace dsrg {
void timer_begin(const char *name, hipStream_t st) {
  TimerTable &t = g_timer;
  t.skip = t.active && t.filter[0] != '\0' && !in_list(t.filter, name);
  if (!t.active || t.skip || t.n >= TimerTable::kMax) return;
  while (t.created < 2 * (t.n + 1)) {
    if (hipEventCreate(&t.ev[t.created]) != hipSuccess) {
      t.active = false;
      return;
    }
    ++t.created;
  }
  t.name[t.n] = name;
  (void)hipEventRecord(t.ev[2 * t.n], st);
}
void timer_end(hipStream_t st) {
  TimerTable &t = g_timer;
  if (t.skip) {
    t.skip = false;
    return;
  }
  if (!t.active || t.n >= TimerTable::kMax) return;
  (void)hipEventRecord(t.ev[2 * t.n + 1], st);
  ++t.n;
}
}  // namespace dsrg

// DSRG_OPT_CHECK_SIGNS: the current device's sign check word for the kernels
static dsrg_status sign_check_setup(int terms, dsrg::Plan &pl) {
  pl.chk = nullptr;
  if (!(terms & DSRG_OPT_CHECK_SIGNS)) return DSRG_OK;
  hipError_t e = dsrg::sign_check_ptr(&pl.chk);
  if (e != hipSuccess)
    return fail(DSRG_ERR_HIP, "sign check word lookup failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

extern "C" {

dsrg_status dsrg_df_sign_check(unsigned *word) {
  g_err[0] = 0;
  if (!word) return fail(DSRG_ERR_ARG, "word pointer is NULL");
  hipError_t e = dsrg::sign_check_read(word);
  if (e != hipSuccess)
    return fail(DSRG_ERR_HIP, "sign check word read failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

dsrg_status dsrg_df_mfma_probe(int kind, int64_t nwg, int64_t iters, int64_t *stamps, void *sink,
                               void *stream) {
  g_err[0] = 0;
  if (kind != DSRG_PROBE_I8 && kind != DSRG_PROBE_F64)
    return fail(DSRG_ERR_ARG, "unknown probe kind %d", kind);
  if (nwg < 1 || nwg > 65536) return fail(DSRG_ERR_ARG, "nwg = %lld outside [1, 65536]", (long long)nwg);
  if (iters < 1 || iters > (int64_t(1) << 24))
    return fail(DSRG_ERR_ARG, "iters = %lld outside [1, 2^24]", (long long)iters);
  if (!stamps || !sink) return fail(DSRG_ERR_ARG, "stamps or sink is NULL");
  if ((reinterpret_cast<uintptr_t>(stamps) | reinterpret_cast<uintptr_t>(sink)) & 7)
    return fail(DSRG_ERR_ARG, "stamps or sink is not 8-byte aligned");
  hipError_t e = dsrg::launch_mfma_probe(kind, nwg, iters, stamps, sink,
                                         reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "probe launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

dsrg_status dsrg_df_workspace_size(const dsrg_df_problem *p, int precision, int terms,
                                   int with_grad, size_t *bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(DSRG_ERR_ARG, "bytes pointer is NULL");
  dsrg::Plan pl;
  dsrg_status st = make_plan(p, precision, terms, with_grad, pl);
  if (st != DSRG_OK) return st;
  *bytes = pl.total;
  return DSRG_OK;
}

dsrg_status dsrg_df_energy(const dsrg_df_problem *p, int precision, int terms, double *E_terms,
                           void *workspace, size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  dsrg::Plan pl;
  dsrg_status st = make_plan(p, precision, terms, 0, pl);
  if (st != DSRG_OK) return st;
  if ((st = check_inputs(p, pl)) != DSRG_OK) return st;
  if (!E_terms || !aligned8(E_terms)) return fail(DSRG_ERR_ARG, "E_terms is NULL or misaligned");
  if ((st = check_workspace(pl, workspace, ws_bytes)) != DSRG_OK) return st;
  if ((st = sign_check_setup(terms, pl)) != DSRG_OK) return st;

  dsrg::Inputs in{p->B_cv, p->B_ca, p->B_av, p->eps_c, p->eps_a, p->eps_v, p->gamma1};
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((terms & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = (precision == DSRG_SPLIT_OZAKI) ? dsrg::launch_energy_split(pl, in, workspace, hs)
                                                 : dsrg::launch_energy_fp64(pl, in, workspace, hs);
  if (e == hipSuccess) e = dsrg::launch_finalize(pl, workspace, E_terms, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

dsrg_status dsrg_df_energy_noalloc(const dsrg_df_problem *p, int precision, int terms,
                                   double *E_terms, void *stream) {
  g_err[0] = 0;
  if (terms & DSRG_OPT_KERNEL_TIMING)
    return fail(DSRG_ERR_ARG, "DSRG_OPT_KERNEL_TIMING is not available without allocation");
  dsrg::Plan pl;
  dsrg_status st = make_plan(p, precision, terms, 0, pl);
  if (st != DSRG_OK) return st;
  if ((st = check_inputs(p, pl)) != DSRG_OK) return st;
  if (!E_terms || !aligned8(E_terms)) return fail(DSRG_ERR_ARG, "E_terms is NULL or misaligned");
  if (pl.total > dsrg::kNoAllocScratchBytes)
    return fail(DSRG_ERR_UNSUPPORTED,
                "problem needs %zu bytes of workspace, more than the %zu of the static scratch "
                "(use dsrg_df_energy with a workspace)",
                pl.total, dsrg::kNoAllocScratchBytes);
  if ((st = sign_check_setup(terms, pl)) != DSRG_OK) return st;
  void *ws = nullptr;
  hipError_t e = dsrg::noalloc_scratch(&ws);
  if (e != hipSuccess)
    return fail(DSRG_ERR_HIP, "static scratch lookup failed: %s", hipGetErrorString(e));
  dsrg::Inputs in{p->B_cv, p->B_ca, p->B_av, p->eps_c, p->eps_a, p->eps_v, p->gamma1};
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset(false);
  e = (precision == DSRG_SPLIT_OZAKI) ? dsrg::launch_energy_split(pl, in, ws, hs)
                                      : dsrg::launch_energy_fp64(pl, in, ws, hs);
  if (e == hipSuccess) e = dsrg::launch_finalize(pl, ws, E_terms, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

dsrg_status dsrg_df_energy_backward(const dsrg_df_problem *p, int precision, int terms,
                                    const double *gE, double *dB_cv, double *dB_ca,
                                    double *dB_av, double *deps_c, double *deps_a,
                                    double *deps_v, double *ds, double *E_terms,
                                    void *workspace, size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  dsrg::Plan pl;
  dsrg_status st = make_plan(p, precision, terms, 1, pl);
  if (st != DSRG_OK) return st;
  if ((st = check_inputs(p, pl)) != DSRG_OK) return st;
  if (!gE || !aligned8(gE)) return fail(DSRG_ERR_ARG, "gE is NULL or misaligned");
  if (!dB_cv || !aligned8(dB_cv)) return fail(DSRG_ERR_ARG, "dB_cv is NULL or misaligned");
  if (!deps_c || !aligned8(deps_c)) return fail(DSRG_ERR_ARG, "deps_c is NULL or misaligned");
  if (!deps_v || !aligned8(deps_v)) return fail(DSRG_ERR_ARG, "deps_v is NULL or misaligned");
  if (!ds || !aligned8(ds)) return fail(DSRG_ERR_ARG, "ds is NULL or misaligned");
  if (pl.na > 0) {
    if (!dB_ca || !aligned8(dB_ca)) return fail(DSRG_ERR_ARG, "dB_ca is NULL or misaligned");
    if (!dB_av || !aligned8(dB_av)) return fail(DSRG_ERR_ARG, "dB_av is NULL or misaligned");
    if (!deps_a || !aligned8(deps_a)) return fail(DSRG_ERR_ARG, "deps_a is NULL or misaligned");
  }
  if (E_terms && !aligned8(E_terms)) return fail(DSRG_ERR_ARG, "E_terms is misaligned");
  if ((st = check_workspace(pl, workspace, ws_bytes)) != DSRG_OK) return st;

  if ((st = sign_check_setup(terms, pl)) != DSRG_OK) return st;
  pl.atomic_reduce = false;   // the adjoint kernels always fill per-workgroup slots
  dsrg::Inputs in{p->B_cv, p->B_ca, p->B_av, p->eps_c, p->eps_a, p->eps_v, p->gamma1};
  dsrg::BwdOut o{dB_cv, pl.na > 0 ? dB_ca : nullptr, pl.na > 0 ? dB_av : nullptr,
                 deps_c, pl.na > 0 ? deps_a : nullptr, deps_v, ds, gE};
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((terms & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = (precision == DSRG_SPLIT_OZAKI)
                     ? dsrg::launch_backward_split(pl, in, o, workspace, hs)
                     : dsrg::launch_backward_fp64(pl, in, o, workspace, hs);
  if (e == hipSuccess && E_terms) e = dsrg::launch_finalize(pl, workspace, E_terms, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

dsrg_status dsrg_df_active_workspace_size(const dsrg_df_problem *p, size_t *bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(DSRG_ERR_ARG, "bytes pointer is NULL");
  dsrg::ActivePlan pl;
  dsrg_status st = make_active_plan(p, pl);
  if (st != DSRG_OK) return st;
  *bytes = pl.total;
  return DSRG_OK;
}

dsrg_status dsrg_df_energy_active(const dsrg_df_problem *p, const double *B_aa, int options,
                                  double *F_terms, void *workspace, size_t ws_bytes,
                                  void *stream) {
  g_err[0] = 0;
  dsrg::ActivePlan pl;
  dsrg_status st = make_active_plan(p, pl);
  if (st != DSRG_OK) return st;
  if (options & ~DSRG_OPT_KERNEL_TIMING)
    return fail(DSRG_ERR_ARG, "unknown option bits 0x%x", options);
  if (!F_terms || !aligned8(F_terms)) return fail(DSRG_ERR_ARG, "F_terms is NULL or misaligned");
  if (pl.na > 0) {
    const struct {
      const double *ptr;
      const char *name;
    } need[] = {{p->B_cv, "B_cv"},   {p->B_ca, "B_ca"},   {p->B_av, "B_av"},
                {B_aa, "B_aa"},      {p->eps_c, "eps_c"}, {p->eps_a, "eps_a"},
                {p->eps_v, "eps_v"}, {p->gamma1, "gamma1"}};
    for (const auto &n : need)
      if (!n.ptr || !aligned8(n.ptr)) return fail(DSRG_ERR_ARG, "%s is NULL or misaligned", n.name);
  }
  if (ws_bytes < pl.total)
    return fail(DSRG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, pl.total);
  if (!workspace) return fail(DSRG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u)
    return fail(DSRG_ERR_WORKSPACE, "workspace is not 256-byte aligned");

  dsrg::ActiveInputs in{p->B_cv, p->B_ca, p->B_av, B_aa, p->eps_c, p->eps_a, p->eps_v,
                        p->gamma1};
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((options & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = dsrg::launch_active_terms(pl, in, workspace, F_terms, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

dsrg_status dsrg_df_factors_workspace_size(const dsrg_dfgen_problem *p, size_t *bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(DSRG_ERR_ARG, "bytes pointer is NULL");
  dsrg::DFPlan pl;
  dsrg_status st = make_df_plan(p, pl);
  if (st != DSRG_OK) return st;
  *bytes = pl.total;
  return DSRG_OK;
}

dsrg_status dsrg_df_factors(const dsrg_dfgen_problem *p, int options, double *B_cv,
                            double *B_ca, double *B_av, double *B_aa, void *workspace,
                            size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  dsrg::DFPlan pl;
  dsrg_status st = make_df_plan(p, pl);
  if (st != DSRG_OK) return st;
  if (options & ~DSRG_OPT_KERNEL_TIMING)
    return fail(DSRG_ERR_ARG, "unknown option bits 0x%x", options);
  const struct {
    const void *ptr;
    const char *name;
    bool need;
  } chk[] = {{p->ao3, "ao3", true},     {p->J, "J", false},         {p->C, "C", true},
             {B_cv, "B_cv", true},       {B_ca, "B_ca", pl.na > 0}, {B_av, "B_av", pl.na > 0},
             {B_aa, "B_aa", pl.na > 0}};
  for (const auto &c : chk)
    if ((c.need && !c.ptr) || (c.ptr && !aligned8(c.ptr)))
      return fail(DSRG_ERR_ARG, "%s is NULL or misaligned", c.name);
  if (ws_bytes < pl.total)
    return fail(DSRG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, pl.total);
  if (!workspace) return fail(DSRG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u)
    return fail(DSRG_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  dsrg::DFInputs in{p->ao3, p->J, p->C};
  dsrg::DFOutputs o{B_cv, B_ca, B_av, B_aa};
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((options & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = dsrg::launch_df_factors(pl, in, o, workspace, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

namespace {
dsrg_status make_fock_plan(const dsrg_fock_problem *p, dsrg::FockPlan &pl) {
  if (!p) return fail(DSRG_ERR_ARG, "problem pointer is NULL");
  dsrg::DFPlan dp;
  dsrg_status st = make_df_plan(&p->df, dp);
  if (st != DSRG_OK) return st;
  pl.nao = dp.nao;
  pl.nmo = dp.nmo;
  pl.naux = dp.naux;
  pl.nfrz = dp.nfrz;
  pl.nc = dp.nc;
  pl.na = dp.na;
  pl.nv = dp.nv;
  pl.nd = pl.nfrz + pl.nc;
  pl.no = pl.nd + pl.na;
  const size_t nx = (size_t)pl.naux, no = (size_t)pl.no, nmo = (size_t)pl.nmo,
               nao = (size_t)pl.nao;
  size_t off = 0;
  auto take = [&](size_t doubles) {
    const size_t at = off;
    off = align256(off + sizeof(double) * doubles);
    return at;
  };
  pl.metric = dp.metric;
  pl.off_t = take(nx * no * nao);
  pl.off_y = take(nx * no * nmo);   // later the right operand of the exchange product
  if (pl.metric) {
    pl.off_l = take(nx * nx);
    pl.off_x = take(nx * nx);
    pl.off_w = take(nx * nx);
  } else {
    pl.off_l = pl.off_x = pl.off_w = off;
  }
  pl.off_bo = take(nx * no * nmo);
  pl.off_d = take(nx);
  pl.off_c = take(nx);
  pl.off_jao = take(nao * nao);
  pl.off_tj = take(nao * nmo);
  pl.off_part = take(32 * nmo * nmo);   // split-K partial products of the exchange part (32 at most)
  pl.total = off;
  return DSRG_OK;
}
}  // namespace

dsrg_status dsrg_df_fock_workspace_size(const dsrg_fock_problem *p, size_t *bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(DSRG_ERR_ARG, "bytes pointer is NULL");
  dsrg::FockPlan pl;
  dsrg_status st = make_fock_plan(p, pl);
  if (st != DSRG_OK) return st;
  *bytes = pl.total;
  return DSRG_OK;
}

dsrg_status dsrg_df_fock(const dsrg_fock_problem *p, int options, double *F, void *workspace,
                         size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  dsrg::FockPlan pl;
  dsrg_status st = make_fock_plan(p, pl);
  if (st != DSRG_OK) return st;
  if (options & ~DSRG_OPT_KERNEL_TIMING)
    return fail(DSRG_ERR_ARG, "unknown option bits 0x%x", options);
  const struct {
    const void *ptr;
    const char *name;
    bool need;
  } chk[] = {{p->df.ao3, "ao3", true}, {p->df.J, "J", false}, {p->df.C, "C", true},
             {p->h, "h", true},        {p->gamma1, "gamma1", pl.na > 0}, {F, "F", true}};
  for (const auto &c : chk)
    if ((c.need && !c.ptr) || (c.ptr && !aligned8(c.ptr)))
      return fail(DSRG_ERR_ARG, "%s is NULL or misaligned", c.name);
  if (ws_bytes < pl.total)
    return fail(DSRG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, pl.total);
  if (!workspace) return fail(DSRG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u)
    return fail(DSRG_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  dsrg::FockInputs in{p->df.ao3, p->df.J, p->df.C, p->h, p->gamma1};
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((options & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = dsrg::launch_df_fock(pl, in, F, workspace, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

namespace {
dsrg_status make_semican_plan(const dsrg_semican_problem *p, dsrg::SemicanPlan &pl) {
  if (!p) return fail(DSRG_ERR_ARG, "problem pointer is NULL");
  if (p->nmo < 1 || p->nfrz < 0 || p->nc < 0 || p->na < 0 || p->nv < 0 || p->nao < 0)
    return fail(DSRG_ERR_ARG, "sizes must satisfy nmo >= 1 and nao, nfrz, nc, na, nv >= 0");
  if (p->nmo < p->nfrz + p->nc + p->na + p->nv)
    return fail(DSRG_ERR_ARG, "nmo = %lld is smaller than nfrz + nc + na + nv",
                (long long)p->nmo);
  if (p->nmo > (1 << 16)) return fail(DSRG_ERR_UNSUPPORTED, "nmo too large");
  pl.nao = p->nao;
  pl.nmo = p->nmo;
  pl.nfrz = p->nfrz;
  pl.nc = p->nc;
  pl.na = p->na;
  pl.nv = p->nv;
  const size_t np = (size_t)dsrg::semican_npad(std::max({p->nc, p->na, p->nv, (int64_t)1}));
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  pl.off_a = take(sizeof(double) * np * np);
  pl.off_a2 = take(sizeof(double) * np * np);   // the matrix of the next Jacobi round
  pl.off_v = take(sizeof(double) * np * np);
  pl.off_q = take(sizeof(double) * (np / 32) * 32 * 32);   // one 32 x 32 rotation per pair
  pl.off_part = take(sizeof(double) * 2 * dsrg::kSemicanParts);
  pl.off_flag = take(sizeof(int));
  pl.total = off;
  return DSRG_OK;
}
}  // namespace

dsrg_status dsrg_df_semicanonicalize_workspace_size(const dsrg_semican_problem *p,
                                                    size_t *bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(DSRG_ERR_ARG, "bytes pointer is NULL");
  dsrg::SemicanPlan pl;
  dsrg_status st = make_semican_plan(p, pl);
  if (st != DSRG_OK) return st;
  *bytes = pl.total;
  return DSRG_OK;
}

dsrg_status dsrg_df_semicanonicalize(const dsrg_semican_problem *p, int options, double *U,
                                     double *eps, double *Cs, int *info, void *workspace,
                                     size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  dsrg::SemicanPlan pl;
  dsrg_status st = make_semican_plan(p, pl);
  if (st != DSRG_OK) return st;
  if (options & ~DSRG_OPT_KERNEL_TIMING)
    return fail(DSRG_ERR_ARG, "unknown option bits 0x%x", options);
  if (!p->F || !aligned8(p->F)) return fail(DSRG_ERR_ARG, "F is NULL or misaligned");
  if (!U || !aligned8(U)) return fail(DSRG_ERR_ARG, "U is NULL or misaligned");
  if (!eps || !aligned8(eps)) return fail(DSRG_ERR_ARG, "eps is NULL or misaligned");
  if ((Cs != nullptr) != (p->C != nullptr))
    return fail(DSRG_ERR_ARG, "C and Cs must be given together");
  if (Cs && (!aligned8(Cs) || !aligned8(p->C) || p->nao < 1))
    return fail(DSRG_ERR_ARG, "C or Cs misaligned, or nao < 1 with C given");
  if (info && (reinterpret_cast<uintptr_t>(info) & 3u))
    return fail(DSRG_ERR_ARG, "info is misaligned");
  if (ws_bytes < pl.total)
    return fail(DSRG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, pl.total);
  if (!workspace) return fail(DSRG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u)
    return fail(DSRG_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((options & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = dsrg::launch_semican(pl, p->F, p->C, U, eps, Cs, info, workspace, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

namespace {
dsrg_status make_rest_plan(const dsrg_df_rest_problem *rp, dsrg::RestPlan &pl) {
  using namespace dsrg;
  if (!rp) return fail(DSRG_ERR_ARG, "problem pointer is NULL");
  const dsrg_df_problem *p = &rp->base;
  if (p->nc < 1 || p->nv < 1 || p->naux < 1 || p->na < 0)
    return fail(DSRG_ERR_ARG, "sizes must satisfy nc, nv, naux >= 1 and na >= 0");
  if (!(p->s >= 0.0) || !isfinite(p->s))
    return fail(DSRG_ERR_ARG, "s must be finite and >= 0 (got %g)", p->s);
  if (p->na > DSRG_DF_MAX_ACTIVE)
    return fail(DSRG_ERR_UNSUPPORTED, "na = %lld exceeds the compiled maximum %d",
                (long long)p->na, DSRG_DF_MAX_ACTIVE);
  if (p->nc > (1 << 16) || p->nv > (1 << 20) || p->naux > (1 << 24))
    return fail(DSRG_ERR_UNSUPPORTED, "dimensions too large");
  pl.nc = p->nc;
  pl.na = p->na;
  pl.nv = p->nv;
  pl.naux = p->naux;
  pl.s = p->s;
  const size_t nc = (size_t)pl.nc, na = (size_t)pl.na, nv = (size_t)pl.nv;
  const size_t sC = 2 * nc, sA = 2 * na, sV = 2 * nv, sH = sC + sA, sP = sA + sV;
  size_t off = 0;
  auto take = [&](size_t doubles) {
    const size_t at = off;
    off = align256(off + sizeof(double) * std::max<size_t>(doubles, 1));
    return at;
  };
  if (pl.na > 0) {
    pl.off_pcv = take(nc * nv * na * na);
    pl.off_pav = take(na * nv * na * na);
    pl.off_pca = take(nc * na * na * na);
    pl.off_paa = take(na * na * na * na);
    pl.off_qvc = take(na * nv * nc * na);
    pl.off_kcc = take(nc * na * nc * na);
    pl.off_x = take(na * nv * na * nv);
    pl.off_wt = take(sH * sA * sP * sA);
    pl.off_wv = take(sH * sA * sP * sA);
    pl.off_tcc = take(sC * sC * sA * sA);
    pl.off_vcc = take(sC * sC * sA * sA);
    pl.off_t1 = take(sH * sP);
    pl.off_ft = take(sH * sP);
    pl.off_y = take(sA * sA * sV * sA);
    pl.off_tp = take(sH * sA * sP * sA);
    pl.off_lp = take(sA * sA * sA * sA);
    pl.off_ci = take(sH * sP * sA * sA);
    pl.off_ak = take(sA * sA * sA * sV);
    pl.off_bk = take(sA * sA * sA * sV);
    pl.off_y2 = take(sA * sA * sA * sA * sA * sA);
    rest_grids(pl.nc, pl.na, pl.nv, pl.grid);
    int64_t nslot = 0;
    for (int k = 0; k < kRestKernels; ++k) {
      pl.slot[k] = nslot;
      nslot += pl.grid[k];
    }
    pl.off_slots = take((size_t)nslot);
  } else {
    pl.off_pcv = pl.off_pav = pl.off_pca = pl.off_paa = pl.off_qvc = pl.off_kcc = pl.off_x =
        pl.off_wt = pl.off_wv = pl.off_tcc = pl.off_vcc = pl.off_t1 = pl.off_ft = pl.off_y =
            pl.off_tp = pl.off_lp = pl.off_ci = pl.off_ak = pl.off_bk = pl.off_y2 =
                pl.off_slots = 0;
    off = 256;
  }
  pl.total = off;
  return DSRG_OK;
}
}  // namespace

dsrg_status dsrg_df_rest_workspace_size(const dsrg_df_rest_problem *p, size_t *bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(DSRG_ERR_ARG, "bytes pointer is NULL");
  dsrg::RestPlan pl;
  dsrg_status st = make_rest_plan(p, pl);
  if (st != DSRG_OK) return st;
  *bytes = pl.total;
  return DSRG_OK;
}

dsrg_status dsrg_df_energy_rest(const dsrg_df_rest_problem *p, int options, double *terms,
                                void *workspace, size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  dsrg::RestPlan pl;
  dsrg_status st = make_rest_plan(p, pl);
  if (st != DSRG_OK) return st;
  if (options & ~DSRG_OPT_KERNEL_TIMING)
    return fail(DSRG_ERR_ARG, "unknown option bits 0x%x", options);
  if (!terms || !aligned8(terms)) return fail(DSRG_ERR_ARG, "terms is NULL or misaligned");
  if (pl.na > 0) {
    const struct {
      const double *ptr;
      const char *name;
    } need[] = {{p->base.B_cv, "B_cv"}, {p->base.B_ca, "B_ca"}, {p->base.B_av, "B_av"},
                {p->B_aa, "B_aa"},      {p->base.eps_c, "eps_c"}, {p->base.eps_a, "eps_a"},
                {p->base.eps_v, "eps_v"}, {p->f_ca, "f_ca"},  {p->f_cv, "f_cv"},
                {p->f_av, "f_av"},      {p->rdm1, "rdm1"},    {p->lambda2, "lambda2"},
                {p->lambda3, "lambda3"}};
    for (const auto &n : need)
      if (!n.ptr || !aligned8(n.ptr)) return fail(DSRG_ERR_ARG, "%s is NULL or misaligned", n.name);
  }
  if (ws_bytes < pl.total)
    return fail(DSRG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, pl.total);
  if (!workspace) return fail(DSRG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u)
    return fail(DSRG_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  dsrg::RestInputs in{p->base.B_cv, p->base.B_ca, p->base.B_av, p->B_aa, p->base.eps_c,
                      p->base.eps_a, p->base.eps_v, p->f_ca, p->f_cv, p->f_av, p->rdm1,
                      p->lambda2, p->lambda3};
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((options & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = dsrg::launch_rest_terms(pl, in, workspace, terms, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

dsrg_status dsrg_df_cumulants(int64_t na, const double *rdm1, const double *rdm2,
                              const double *rdm3, double *lambda2, double *lambda3,
                              void *stream) {
  g_err[0] = 0;
  if (na < 1) return fail(DSRG_ERR_ARG, "na must be >= 1 (got %lld)", (long long)na);
  if (na > DSRG_DF_MAX_ACTIVE)
    return fail(DSRG_ERR_UNSUPPORTED, "na = %lld exceeds the compiled maximum %d", (long long)na,
                DSRG_DF_MAX_ACTIVE);
  const struct {
    const void *ptr;
    const char *name;
  } need[] = {{rdm1, "rdm1"}, {rdm2, "rdm2"}, {rdm3, "rdm3"}, {lambda2, "lambda2"},
              {lambda3, "lambda3"}};
  for (const auto &n : need)
    if (!n.ptr || !aligned8(n.ptr)) return fail(DSRG_ERR_ARG, "%s is NULL or misaligned", n.name);
  hipError_t e = dsrg::launch_cumulants((int)(2 * na), rdm1, rdm2, rdm3, lambda2, lambda3,
                                        reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

namespace {
// Plan of the CD factor build: validation and the workspace layout.
dsrg_status make_cd_plan(const dsrg_cd_problem *p, dsrg::CdPlan &pl) {
  using namespace dsrg;
  if (!p) return fail(DSRG_ERR_ARG, "problem pointer is NULL");
  if (p->nao < 1) return fail(DSRG_ERR_ARG, "nao must be >= 1 (got %lld)", (long long)p->nao);
  if (p->nao > DSRG_CD_MAX_NAO)
    return fail(DSRG_ERR_UNSUPPORTED, "nao = %lld exceeds %d", (long long)p->nao,
                DSRG_CD_MAX_NAO);
  if (!(p->tol >= 0.0) || !std::isfinite(p->tol))
    return fail(DSRG_ERR_ARG, "tol must be finite and >= 0");
  pl.nao = p->nao;
  pl.npair = p->nao * (p->nao + 1) / 2;
  if (p->max_rank < 0 || p->max_rank > pl.npair)
    return fail(DSRG_ERR_ARG, "max_rank = %lld is outside [0, %lld]", (long long)p->max_rank,
                (long long)pl.npair);
  pl.max_rank = p->max_rank;
  pl.tol = p->tol;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align256(off + bytes);
    return at;
  };
  // the most workgroups of any launch: the init kernel's one per 256 pairs or
  // a step's one per cd_rows_per_block pairs
  pl.pstride = std::max(ceil_div(pl.npair, 256), ceil_div(pl.npair, cd_rows_per_block(pl.npair)));
  pl.off_d = take(sizeof(double) * (size_t)pl.npair);
  pl.off_pv = take(sizeof(double) * 2 * (size_t)pl.pstride);
  pl.off_pi = take(sizeof(int64_t) * 2 * (size_t)pl.pstride);
  pl.off_state = take(sizeof(CdState));
  pl.total = off;
  return DSRG_OK;
}
}  // namespace

dsrg_status dsrg_df_cholesky_workspace_size(const dsrg_cd_problem *p, size_t *bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(DSRG_ERR_ARG, "bytes pointer is NULL");
  dsrg::CdPlan pl;
  dsrg_status st = make_cd_plan(p, pl);
  if (st != DSRG_OK) return st;
  *bytes = pl.total;
  return DSRG_OK;
}

dsrg_status dsrg_df_cholesky(const dsrg_cd_problem *p, int options, double *B, int64_t *rank,
                             double *dmax, int64_t *pivots, void *workspace, size_t ws_bytes,
                             void *stream) {
  g_err[0] = 0;
  dsrg::CdPlan pl;
  dsrg_status st = make_cd_plan(p, pl);
  if (st != DSRG_OK) return st;
  if (options & ~DSRG_OPT_KERNEL_TIMING)
    return fail(DSRG_ERR_ARG, "unknown option bits 0x%x", options);
  const struct {
    const void *ptr;
    const char *name;
    bool need;
  } chk[] = {{p->M, "M", true},       {B, "B", pl.max_rank > 0}, {rank, "rank", true},
             {dmax, "dmax", true},    {pivots, "pivots", false}};
  for (const auto &c : chk)
    if ((c.need && !c.ptr) || (c.ptr && !aligned8(c.ptr)))
      return fail(DSRG_ERR_ARG, "%s is NULL or misaligned", c.name);
  if (ws_bytes < pl.total)
    return fail(DSRG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, pl.total);
  if (!workspace) return fail(DSRG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u)
    return fail(DSRG_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((options & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = dsrg::launch_cholesky(pl, p->M, B, rank, dmax, pivots, workspace, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

static_assert(dsrg::kLtMaxTerms == DSRG_DF_MAX_LAPLACE_TERMS, "the header states the term limit");

namespace {
// Plan of the Laplace-factorized Coulomb part: validation and workspace.
dsrg_status make_lt_plan(const dsrg_df_problem *p, int nq, dsrg::LtPlan &pl) {
  using namespace dsrg;
  if (!p) return fail(DSRG_ERR_ARG, "problem pointer is NULL");
  if (p->nc < 1 || p->nv < 1 || p->naux < 1)
    return fail(DSRG_ERR_ARG, "sizes must satisfy nc, nv, naux >= 1");
  if (nq < 1 || nq > kLtMaxTerms)
    return fail(DSRG_ERR_ARG, "nq = %d is outside [1, %d]", nq, kLtMaxTerms);
  // B D_k and Y_k of one term, in bytes, must fit in 62 bits (the sizes below)
  const double nc = (double)p->nc, nv = (double)p->nv, naux = (double)p->naux;
  if (!(8.0 * naux * (nc * nv + naux) < 0x1p62))
    return fail(DSRG_ERR_UNSUPPORTED, "problem too large (nc %lld, nv %lld, naux %lld)",
                (long long)p->nc, (long long)p->nv, (long long)p->naux);
  pl.nc = p->nc;
  pl.nv = p->nv;
  pl.naux = p->naux;
  pl.nq = nq;
  const int64_t per_term = pl.naux * pl.nc * pl.nv + pl.naux * pl.naux;   // B D_k and Y_k
  int64_t kb = (((int64_t)2 << 30) / 8) / std::max<int64_t>(per_term, 1);
  pl.kb = (int)std::max<int64_t>(1, std::min<int64_t>(kb, nq));
  pl.nwg = std::max<int64_t>(1, std::min<int64_t>(1024, ceil_div(pl.naux * pl.naux, 256)));
  size_t off = 0;
  auto take = [&](size_t doubles) {
    const size_t at = off;
    off = align256(off + sizeof(double) * doubles);
    return at;
  };
  pl.off_bs = take((size_t)pl.kb * (size_t)(pl.naux * pl.nc * pl.nv));
  pl.off_y = take((size_t)pl.kb * (size_t)(pl.naux * pl.naux));
  pl.off_slots = take((size_t)nq * (size_t)pl.nwg);
  pl.total = off;
  return DSRG_OK;
}
}  // namespace

dsrg_status dsrg_df_laplace_fit(double s, double x_lo, double x_hi, int nq, double *t, double *w,
                                double *max_err) {
  g_err[0] = 0;
  if (!(s >= 0.0) || !std::isfinite(s)) return fail(DSRG_ERR_ARG, "s must be finite and >= 0");
  if (!(x_lo > 0.0) || !(x_hi > x_lo) || !std::isfinite(x_hi))
    return fail(DSRG_ERR_ARG, "need 0 < x_lo < x_hi, finite");
  if (nq < 1 || nq > dsrg::kLtMaxTerms)
    return fail(DSRG_ERR_ARG, "nq = %d is outside [1, %d]", nq, dsrg::kLtMaxTerms);
  if (!t || !w || !max_err) return fail(DSRG_ERR_ARG, "t, w and max_err must not be NULL");
  dsrg::laplace_fit(s, x_lo, x_hi, nq, t, w, max_err);
  return DSRG_OK;
}

dsrg_status dsrg_df_laplace_workspace_size(const dsrg_df_problem *p, int nq, size_t *bytes) {
  g_err[0] = 0;
  if (!bytes) return fail(DSRG_ERR_ARG, "bytes pointer is NULL");
  dsrg::LtPlan pl;
  dsrg_status st = make_lt_plan(p, nq, pl);
  if (st != DSRG_OK) return st;
  *bytes = pl.total;
  return DSRG_OK;
}

dsrg_status dsrg_df_coulomb_laplace(const dsrg_df_problem *p, int nq, const double *t,
                                    const double *w, int options, double *E, double *S,
                                    void *workspace, size_t ws_bytes, void *stream) {
  g_err[0] = 0;
  dsrg::LtPlan pl;
  dsrg_status st = make_lt_plan(p, nq, pl);
  if (st != DSRG_OK) return st;
  if (options & ~DSRG_OPT_KERNEL_TIMING)
    return fail(DSRG_ERR_ARG, "unknown option bits 0x%x", options);
  if (!t || !w) return fail(DSRG_ERR_ARG, "t and w (host arrays) must not be NULL");
  for (int k = 0; k < nq; ++k)
    if (!(t[k] > 0.0) || !std::isfinite(t[k]) || !std::isfinite(w[k]))
      return fail(DSRG_ERR_ARG, "term %d: t must be finite and > 0, w finite", k);
  const struct {
    const void *ptr;
    const char *name;
    bool need;
  } chk[] = {{p->B_cv, "B_cv", true}, {p->eps_c, "eps_c", true}, {p->eps_v, "eps_v", true},
             {E, "E", true},          {S, "S", false}};
  for (const auto &c : chk)
    if ((c.need && !c.ptr) || (c.ptr && !aligned8(c.ptr)))
      return fail(DSRG_ERR_ARG, "%s is NULL or misaligned", c.name);
  if (ws_bytes < pl.total)
    return fail(DSRG_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                ws_bytes, pl.total);
  if (!workspace) return fail(DSRG_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) & 255u)
    return fail(DSRG_ERR_WORKSPACE, "workspace is not 256-byte aligned");
  hipStream_t hs = reinterpret_cast<hipStream_t>(stream);
  timer_reset((options & DSRG_OPT_KERNEL_TIMING) != 0);
  hipError_t e = dsrg::launch_coulomb_laplace(pl, p->B_cv, p->eps_c, p->eps_v, t, w, E, S,
                                              workspace, hs);
  if (e != hipSuccess) return fail(DSRG_ERR_HIP, "HIP launch failed: %s", hipGetErrorString(e));
  return DSRG_OK;
}

const char *dsrg_df_last_error(void) { return g_err; }

int dsrg_df_kernel_times(double *ms, const char **names, int cap) {
  TimerTable &t = g_timer;
  const int n = t.n;
  t.n = 0;
  for (int k = 0; k < n && k < cap; ++k) {
    if (hipEventSynchronize(t.ev[2 * k + 1]) != hipSuccess) return -1;
    float f = 0.0f;
    if (hipEventElapsedTime(&f, t.ev[2 * k], t.ev[2 * k + 1]) != hipSuccess) return -1;
    if (ms) ms[k] = (double)f;
    if (names) names[k] = t.name[k];
  }
  return n;
}

dsrg_status dsrg_df_timing_filter(const char *names) {
  g_err[0] = '\0';
  TimerTable &t = g_timer;
  if (!names) {
    t.filter[0] = '\0';
    return DSRG_OK;
  }
  if (strlen(names) >= sizeof(t.filter))
    return fail(DSRG_ERR_ARG, "timing filter longer than %d characters",
                (int)sizeof(t.filter) - 1);
  strcpy(t.filter, names);
  return DSRG_OK;
}

dsrg_status dsrg_df_set_gradient_block_bytes(size_t bytes) {
  g_err[0] = '\0';
  if (bytes > ((size_t)1 << 50)) return fail(DSRG_ERR_ARG, "bound of %zu bytes is too large", bytes);
  g_grad_block_bytes.store(bytes == 0 ? dsrg::kGradBlockBytes : (int64_t)bytes);
  return DSRG_OK;
}

size_t dsrg_df_gradient_block_bytes(void) { return (size_t)g_grad_block_bytes.load(); }

int dsrg_df_version(void) { return 200; }

}  // extern "C"
