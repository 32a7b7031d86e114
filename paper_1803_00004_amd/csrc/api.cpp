// C ABI of the library (declared in include/bf.h): plan lifetime, workspace
// sizing, argument validation and kernel launches.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <numeric>
#include <vector>

#include "bf.h"
#include "bf_internal.h"

namespace {

constexpr int kMaxSide = 32768;

bool ranges_overlap(const void *a, size_t na, const void *b, size_t nb) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + nb && b0 < a0 + na;
}

// Launch shapes chosen by bf_autotune, per image-size class (256-pixel
// buckets of H and W) and plan shape.  Only plans whose results do not depend
// on the tiling are tuned (every tap in a quadruplet: q fixed by the box).
struct TuneKey {
  int hb, wb, radius, n_terms, n_images, n_quads, u8;
  bool operator<(const TuneKey &o) const {
    return std::tie(hb, wb, radius, n_terms, n_images, n_quads, u8) <
           std::tie(o.hb, o.wb, o.radius, o.n_terms, o.n_images, o.n_quads, o.u8);
  }
};
struct TuneVal {
  int tile, kb_single, ka_one;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tuned;

TuneKey tune_key(const bf_plan_s *p, int H, int W) {
  const bf::DevTables &h = p->host_tables;
  return TuneKey{(H + 255) / 256, (W + 255) / 256, p->fit.radius, h.n_terms, h.n_images, h.n_quads, h.in_u8};
}

bool tunable(const bf_plan_s *p) {
  return p->tile == 0 && !p->host_tables.direct && !p->host_tables.range_box && !p->host_tables.reduced;
}

bf::Geometry geometry_with(const bf_plan_s *p, int H, int W, int tile_override, int kb_single,
                           int ka_one) {
  int tile = 0, q = 0;
  // an untuned image of a lattice-kernel plan gets a table tile of whole lattice tiles
  const bf::DevTables &ht = p->host_tables;
  const bool tables = !ht.direct && !ht.range_box && !ht.reduced;
  const int row_unit = tables && bf::lookup_kernel_for(ht, kb_single) == 3 ? bf::lattice_rows(ht) : 0;
  bf::choose_tiling(H, W, p->fit.radius, p->host_tables.n_terms, tile_override ? tile_override : p->tile,
                    p->gmax, row_unit, &tile, &q);
  // a direct plan keeps no tables: an empty workspace
  const bool no_tables = p->host_tables.direct || p->host_tables.range_box || p->host_tables.reduced;
  bf::Geometry g = bf::make_geometry(H, W, tile, p->fit.radius, no_tables ? 0 : p->host_tables.n_images, q);
  if (p->host_tables.reduced) g.bytes = bf::reduced_workspace_bytes(p->host_tables, H, W);  // FP16 term images
  g.kb_single = kb_single;
  g.ka_one = ka_one;
  return g;
}

bf::Geometry geometry_of(const bf_plan_s *p, int H, int W) {
  if (tunable(p)) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(tune_key(p, H, W));
    if (it != g_tuned.end())
      return geometry_with(p, H, W, it->second.tile, it->second.kb_single, it->second.ka_one);
  }
  return geometry_with(p, H, W, 0, 0, 0);
}

// Pre-computed tables are laid out by the untuned heuristic tiling of the
// plan that builds them, so a later call finds them where they were written.
bf::Geometry precompute_geometry(const bf_plan_s *p, int H, int W) { return geometry_with(p, H, W, 0, 0, 0); }

bf_status_t check_image(const bf_plan_s *p, const void *I, const float *out, int H, int W) {
  if (!p || !I || !out) return BF_ERR_INVALID_ARG;
  if (p->flags & BF_FLAG_HOST_ONLY) return BF_ERR_INVALID_ARG;
  if (H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return BF_ERR_INVALID_ARG;
  const size_t n = (size_t)H * W;
  const size_t in_bytes = n * (p->in_dtype == BF_IN_U8 ? 1 : 4);
  if (ranges_overlap(I, in_bytes, out, n * 4)) return BF_ERR_INVALID_ARG;
  return BF_OK;
}

// Fit, compile and upload a plan of the given kernels (both creation calls).
bf_status_t create_plan(const bf::KernelSpec &kern, int radius, bf_terms_t N, const bf_plan_opts_t *opts,
                        bf_plan_t *plan);

}  // namespace

extern "C" {

bf_status_t bf_plan_create(bf_plan_t *plan, bf_kernel_t K_s, bf_kernel_t K_r, double sigma_s,
                           double sigma_r, int radius, bf_terms_t N, const bf_plan_opts_t *opts) {
  if (!plan) return BF_ERR_INVALID_ARG;
  *plan = nullptr;
  auto known = [](bf_kernel_t k) { return k == BF_KERNEL_GAUSSIAN || k == BF_KERNEL_EXPONENTIAL; };
  if (!known(K_s) || !known(K_r)) {
    if ((int)K_s < 0 || (int)K_r < 0) return BF_ERR_INVALID_ARG;
    return BF_ERR_UNSUPPORTED;
  }
  bf::KernelSpec kern;
  kern.kind_s = (int)K_s;
  kern.kind_r = (int)K_r;
  kern.sigma_s = sigma_s;
  kern.sigma_r = sigma_r;
  return create_plan(kern, radius, N, opts, plan);
}

bf_status_t bf_plan_create_tabulated(bf_plan_t *plan, const double *K_s, int radius, const double *K_r,
                                     int n_r, double step_r, bf_terms_t N, const bf_plan_opts_t *opts) {
  if (!plan) return BF_ERR_INVALID_ARG;
  *plan = nullptr;
  if (!K_s || !K_r || radius < 1) return BF_ERR_INVALID_ARG;
  bf::KernelSpec kern;
  kern.ks = K_s;
  kern.kr = K_r;
  kern.kr_n = n_r;
  kern.kr_step = step_r;
  return create_plan(kern, radius, N, opts, plan);
}

}  // extern "C"

namespace {

bf_status_t create_plan(const bf::KernelSpec &kern, int radius, bf_terms_t N, const bf_plan_opts_t *opts,
                        bf_plan_t *plan) {
  bf_plan_opts_t o{};
  if (opts) o = *opts;
  if (o.in_dtype != BF_IN_F32 && o.in_dtype != BF_IN_U8) return BF_ERR_INVALID_ARG;
  if (o.precision != BF_PREC_PLAIN && o.precision != BF_PREC_REDUCED) return BF_ERR_INVALID_ARG;
  const double eps = o.eps == 0.0 ? 0.01 : o.eps;
  const double span = o.span == 0.0 ? 1.0 : o.span;
  if (!(span > 0) || !std::isfinite(span) || radius < 0) return BF_ERR_INVALID_ARG;
  if (o.tile != 0 && (o.tile < 64 || o.tile > 1024 || o.tile % 64 != 0)) return BF_ERR_INVALID_ARG;

  bf_plan_s *p = new (std::nothrow) bf_plan_s();
  if (!p) return BF_ERR_OUT_OF_MEMORY;
  // the paper's own 8-bit regime: series on [-T_r, T_r] (span 0) and the range box
  const bool range_box = (o.flags & BF_FLAG_RANGE_BOX) != 0;
  // 8-bit input, the default regime with the range terms folded per output level
  const bool level_fold = (o.flags & BF_FLAG_LEVEL_FOLD) != 0;
  if ((range_box || level_fold) && (o.flags & (BF_FLAG_DIRECT | BF_FLAG_DIRECT_AUTO))) {
    delete p;
    return BF_ERR_INVALID_ARG;
  }
  if (range_box && level_fold) {
    delete p;
    return BF_ERR_INVALID_ARG;
  }
  if ((range_box || level_fold) && o.in_dtype != BF_IN_U8) {
    delete p;
    return BF_ERR_UNSUPPORTED;
  }
  const bool reduced = o.precision == BF_PREC_REDUCED;
  if (reduced && (o.flags & (BF_FLAG_DIRECT | BF_FLAG_DIRECT_AUTO | BF_FLAG_RANGE_BOX | BF_FLAG_LEVEL_FOLD))) {
    delete p;
    return BF_ERR_INVALID_ARG;
  }
  const bool tabulated = kern.ks || kern.kr;
  if (tabulated && (o.flags & BF_FLAG_DIRECT)) {  // direct summation evaluates analytic kernels only
    delete p;
    return BF_ERR_UNSUPPORTED;
  }
  bf_status_t st = bf::fit_plan(kern, radius, N, eps, range_box ? 0.0 : span, &p->fit);
  if (st != BF_OK) {
    delete p;
    return st;
  }
  const bf::Fit &f = p->fit;
  if ((int)f.row_off.size() > bf::kMaxTapAxis || (int)f.col_off.size() > bf::kMaxTapAxis) {
    delete p;
    return BF_ERR_UNSUPPORTED;
  }
  p->in_dtype = o.in_dtype;
  p->precision = o.precision;
  p->flags = o.flags;
  p->tile = o.tile;
  if (64 + 2 * f.radius + 1 > 768 || (p->tile && p->tile + 2 * f.radius + 1 > 768)) {
    delete p;  // a table row must fit three 256-column chunks
    return BF_ERR_UNSUPPORTED;
  }
  const double gmax = o.in_dtype == BF_IN_U8 ? 1.0 : std::max(1.0, span);
  p->gmax = gmax;

  bf::DevTables &t = p->host_tables;
  std::memset(&t, 0, sizeof t);
  t.n_terms = (int)f.k.size();
  const int nt = (int)f.tap_w.size();
  if (nt > bf::kMaxTaps) {
    delete p;
    return BF_ERR_UNSUPPORTED;
  }
  t.tap_dy_min = t.tap_dx_min = 1 << 30;
  t.tap_dy_max = t.tap_dx_max = -(1 << 30);
  for (int i = 0; i < nt; ++i) {
    t.tap_dy_min = std::min(t.tap_dy_min, f.tap_dy[i]);
    t.tap_dy_max = std::max(t.tap_dy_max, f.tap_dy[i]);
    t.tap_dx_min = std::min(t.tap_dx_min, f.tap_dx[i]);
    t.tap_dx_max = std::max(t.tap_dx_max, f.tap_dx[i]);
  }
  // quadruplets for the LDS tile kernel: region of 64 + (dx_max - dx_min) columns
  t.lds_pitch = bf::lds_pitch_for(64 + t.tap_dx_max - t.tap_dx_min);
  {
    auto weight_at = [&](int dy, int dx, double *w) {
      for (int i = 0; i < nt; ++i)
        if (f.tap_dy[i] == dy && f.tap_dx[i] == dx) {
          *w = f.tap_w[i];
          return true;
        }
      return false;
    };
    std::vector<char> used(nt, 0);
    for (int i = 0; i < nt; ++i) {
      const int dy = f.tap_dy[i], dx = f.tap_dx[i];
      if (used[i] || dy < 1 || dx < 1) continue;  // representative has dy >= 1, dx >= 1
      double wb, wc, wd;
      const double wa = f.tap_w[i];
      // the expansion is symmetric under u -> -u on each axis, so the four
      // taps carry +-w up to the rounding of the fit; 1e-12 relative admits
      // exactly that
      const double tol = 1e-12 * std::fabs(wa);
      if (weight_at(1 - dy, dx, &wb) && weight_at(dy, 1 - dx, &wc) && weight_at(1 - dy, 1 - dx, &wd) &&
          std::fabs(wb + wa) <= tol && std::fabs(wc + wa) <= tol && std::fabs(wd - wa) <= tol) {
        const int q = t.n_quads++;
        t.quad_dy[q] = dy;
        t.quad_dx[q] = dx;
        t.quad_w[q] = (float)(0.25 * ((wa + wd) - (wb + wc)));
        for (int j = 0; j < nt; ++j) {
          const int ey = f.tap_dy[j], ex = f.tap_dx[j];
          if ((ey == dy || ey == 1 - dy) && (ex == dx || ex == 1 - dx)) used[j] = 1;
        }
      }
    }
    // quadruplets in (dy, dx) order: every lookup kernel sums a pixel's box
    // sums in this order, so they agree bit for bit
    {
      std::vector<int> ord(t.n_quads);
      for (int q = 0; q < t.n_quads; ++q) ord[q] = q;
      std::sort(ord.begin(), ord.end(), [&](int a, int b) {
        return t.quad_dy[a] != t.quad_dy[b] ? t.quad_dy[a] < t.quad_dy[b] : t.quad_dx[a] < t.quad_dx[b];
      });
      int dy[bf::kMaxQuads], dx[bf::kMaxQuads];
      float w[bf::kMaxQuads];
      for (int q = 0; q < t.n_quads; ++q) {
        dy[q] = t.quad_dy[ord[q]];
        dx[q] = t.quad_dx[ord[q]];
        w[q] = t.quad_w[ord[q]];
      }
      for (int q = 0; q < t.n_quads; ++q) {
        t.quad_dy[q] = dy[q];
        t.quad_dx[q] = dx[q];
        t.quad_w[q] = w[q];
      }
    }
    // Every expansion of a kernel that is even in dy and in dx (all kernels
    // the plans take: each Haar level group is symmetric on both axes) pairs
    // all of its taps; a tap left over would need raw table values, which
    // wrap, so such a plan is refused.
    for (int i = 0; i < nt; ++i)
      if (!used[i]) {
        delete p;
        return BF_ERR_UNSUPPORTED;
      }
  }
  // the quadruplets' row lattice (lattice lookup kernel): distinct dy in an
  // arithmetic progression of step s; a step above 16 is split into d equal
  // steps with empty rows between
  {
    std::vector<int> dys, dxs;
    for (int q = 0; q < t.n_quads; ++q) {
      dys.push_back(t.quad_dy[q]);
      dxs.push_back(t.quad_dx[q]);
    }
    std::sort(dys.begin(), dys.end());
    dys.erase(std::unique(dys.begin(), dys.end()), dys.end());
    std::sort(dxs.begin(), dxs.end());
    dxs.erase(std::unique(dxs.begin(), dxs.end()), dxs.end());
    bool ok = dys.size() >= 2 && dxs.size() <= 4;
    int step = ok ? dys[1] - dys[0] : 0;
    for (size_t j = 1; ok && j < dys.size(); ++j) ok = dys[j] - dys[j - 1] == step;
    int d = 1;
    while (ok && step / d > 16) {
      ++d;
      while (step % d) ++d;
    }
    const int m = ok ? (int)(dys.size() - 1) * d + 1 : 0;
    if (ok && m <= 4 && step / d >= 1) {
      t.lat_s = step / d;
      t.lat_m = m;
      t.lat_dy0 = dys[0];
      t.lat_n = dxs.size() <= 2 ? 2 : 4;
      for (int i = 0; i < 4; ++i) t.lat_dx[i] = dxs[std::min<size_t>(i, dxs.size() - 1)];
      for (int q = 0; q < t.n_quads; ++q) {
        const int j = (t.quad_dy[q] - t.lat_dy0) / t.lat_s;
        const int i = (int)(std::find(dxs.begin(), dxs.end(), t.quad_dx[q]) - dxs.begin());
        t.lat_w[4 * j + i] = t.quad_w[q];
        t.lat_mask |= 1 << (4 * j + i);
      }
      const int rw = 64 + t.tap_dx_max - t.tap_dx_min;
      t.lat_pitch = rw <= 128 ? 128 : rw <= 192 ? 192 : 0;
      t.lat_g = std::max(1, 16 / t.lat_s);
      while (t.lat_g > 1 && bf::lattice_lds_bytes(t) > 160 * 1024) --t.lat_g;
      t.lat = t.lat_pitch > 0 && bf::lattice_lds_bytes(t) <= 160 * 1024;
    }
  }
  int slot = 0;
  for (int i = 0; i < t.n_terms; ++i) {
    double fk = f.k[i] / (2.0 * f.T);
    if (o.in_dtype == BF_IN_U8) fk /= 255.0;
    t.f_hi[i] = (float)fk;
    t.f_lo[i] = (float)(fk - (double)t.f_hi[i]);
    t.a[i] = (float)f.a[i];
    t.k_is_zero[i] = f.k[i] == 0;
    t.slot[i] = slot;
    const int nparts = f.k[i] == 0 ? 1 : 4;
    for (int q = 0; q < nparts; ++q) {
      t.slot_term[slot + q] = i;
      t.slot_part[slot + q] = f.k[i] == 0 ? 4 : q;
      t.slot_fhi[slot + q] = t.f_hi[i];
      t.slot_flo[slot + q] = t.f_lo[i];
      t.slot_a[slot + q] = t.a[i];
    }
    slot += nparts;
  }
  t.n_images = slot;
  t.gmax = (float)gmax;
  t.den_floor = (float)(1e-7 * f.sum_abs_K);
  t.in_u8 = o.in_dtype == BF_IN_U8;

  // direct summation: on request, or where its cost model is lower
  // Cost model in vector operations per pixel, fitted to MI355X timings of
  // both paths at 1920 x 1080: direct 8.5 (2r + 1)^2; expansion
  // (1700 + n_images (85 + 10 quadruplets)) (1 + r / 120).
  if (reduced) {
    t.reduced = 1;
    if (bf::reduced_tile(t) == 0 || t.n_quads > 12) {
      delete p;
      return BF_ERR_UNSUPPORTED;
    }
  }
  if (range_box || level_fold) {
    if (f.radius > bf::kMaxRangeBoxRadius) {
      delete p;
      return BF_ERR_UNSUPPORTED;
    }
    // the same kernel: level_fold opens the level window to every difference,
    // which is the default regime's filter (T = max(T_r, span))
    t.range_box = 1;
    t.level_fold = level_fold;
    t.direct_r = f.radius;
    t.box_zr = level_fold ? 255 : (int)std::min(255.0, std::floor(255.0 * f.T_r));
    // the range terms folded per level difference d = L - z (8-bit input)
    double wmax = 0.0;
    for (int d = -255; d <= 255; ++d) {
      double w = 0.0;
      if (std::abs(d) <= t.box_zr)
        for (size_t i = 0; i < f.k.size(); ++i) w += f.a[i] * std::cos(f.omega[i] * (d / 255.0));
      t.box_w[d + 255] = (float)w;
      wmax = std::max(wmax, std::fabs((double)t.box_w[d + 255]));
    }
    // slab values |W(d) z / 255| <= wmax are stored as round(v 2^q), computed
    // in FP32; every box of a quadruplet lies inside the (2r+1)^2 window, so q
    // is the largest shift (<= 24) with
    // (2r + 1)^2 (wmax 2^q (1 + 2^-20) + 1) <= 2^31 - 1
    const double area = (double)(2 * f.radius + 1) * (2 * f.radius + 1);
    int q = 24;
    while (q > 0 && area * (wmax * std::ldexp(1.0, q) * (1.0 + std::ldexp(1.0, -20)) + 1.0) > 2147483647.0) --q;
    t.box_scale = std::ldexp(1.0f, q);
  }
  bool direct = (o.flags & BF_FLAG_DIRECT) != 0;
  if (!direct && !tabulated && (o.flags & BF_FLAG_DIRECT_AUTO) && f.radius <= bf::kMaxDirectRadius) {
    const double e = (double)(2 * f.radius + 1) * (2 * f.radius + 1);
    const double expansion = (1700.0 + t.n_images * (85.0 + 10.0 * t.n_quads)) * (1.0 + f.radius / 120.0);
    direct = 8.5 * e < expansion;
  }
  if (direct && f.radius > bf::kMaxDirectRadius) {
    delete p;
    return BF_ERR_UNSUPPORTED;
  }
  std::vector<float> ks;
  if (direct) {
    const int r = f.radius, K = 2 * r + 1;
    ks.resize((size_t)K * K);
    for (int dy = -r; dy <= r; ++dy)
      for (int dx = -r; dx <= r; ++dx)
        ks[(size_t)(dy + r) * K + dx + r] =
            (float)(kern.kind_s == BF_KERNEL_EXPONENTIAL
                        ? std::exp(-std::sqrt((double)(dx * dx + dy * dy)) / kern.sigma_s)
                        : std::exp(-(dx * dx + dy * dy) / (2.0 * kern.sigma_s * kern.sigma_s)));
    t.direct = 1;
    t.direct_r = r;
    // K_r(d) = 2^(c d^2) (Gaussian) or 2^(c |d|) (exponential)
    const double log2e = 1.4426950408889634;
    t.direct_abs = kern.kind_r == BF_KERNEL_EXPONENTIAL;
    const double sr = kern.sigma_r;
    double c = t.direct_abs ? -log2e / sr : -log2e / (2.0 * sr * sr);
    if (o.in_dtype == BF_IN_U8) c /= t.direct_abs ? 255.0 : 255.0 * 255.0;  // differences in bytes
    t.direct_c = (float)c;
  }

  if (!(p->flags & BF_FLAG_HOST_ONLY)) {
    if (hipGetDevice(&p->device) != hipSuccess) {
      delete p;
      return BF_ERR_DEVICE;
    }
    if (direct) {
      void *k = nullptr;
      if (hipMalloc(&k, ks.size() * sizeof(float)) != hipSuccess) {
        delete p;
        return BF_ERR_OUT_OF_MEMORY;
      }
      p->dev_direct_ks = static_cast<float *>(k);
      if (hipMemcpy(k, ks.data(), ks.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        bf_plan_destroy(p);
        return BF_ERR_DEVICE;
      }
      t.direct_ks = p->dev_direct_ks;
    }
    void *d = nullptr;
    if (hipMalloc(&d, sizeof(bf::DevTables)) != hipSuccess) {
      bf_plan_destroy(p);
      return BF_ERR_OUT_OF_MEMORY;
    }
    if (hipMemcpy(d, &t, sizeof t, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(d);
      delete p;
      return BF_ERR_DEVICE;
    }
    p->dev_tables = static_cast<bf::DevTables *>(d);
  }
  *plan = p;
  return BF_OK;
}

}  // namespace

extern "C" {

bf_status_t bf_plan_destroy(bf_plan_t plan) {
  if (!plan) return BF_OK;
  if (plan->dev_tables) (void)hipFree(plan->dev_tables);
  if (plan->dev_direct_ks) (void)hipFree(plan->dev_direct_ks);
  if (plan->own_ws) (void)hipFree(plan->own_ws);
  delete plan;
  return BF_OK;
}

bf_status_t bf_workspace_size(bf_plan_t plan, int H, int W, size_t *bytes) {
  if (!plan || !bytes || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return BF_ERR_INVALID_ARG;
  *bytes = geometry_of(plan, H, W).bytes;
  return BF_OK;
}

bf_status_t bf_filter_parts(bf_plan_t plan, const void *I, float *out, float *num, float *den,
                            int H, int W, void *ws, size_t ws_bytes, void *stream) {
  bf_status_t st = check_image(plan, I, out, H, W);
  if (st != BF_OK) return st;
  const bf::Geometry g = geometry_of(plan, H, W);
  if ((!ws && g.bytes) || ws_bytes < g.bytes) return BF_ERR_INVALID_ARG;
  const size_t px = (size_t)H * W, in_bytes = px * (plan->in_dtype == BF_IN_U8 ? 1 : 4);
  if (ranges_overlap(ws, g.bytes, I, in_bytes) || ranges_overlap(ws, g.bytes, out, px * 4))
    return BF_ERR_INVALID_ARG;
  return bf::launch_filter(plan->dev_tables, plan->host_tables, g, I, out, num, den,
                           static_cast<int32_t *>(ws), stream);
}

bf_status_t bf_filter_ws(bf_plan_t plan, const void *I, float *out, int H, int W, void *ws,
                         size_t ws_bytes, void *stream) {
  return bf_filter_parts(plan, I, out, nullptr, nullptr, H, W, ws, ws_bytes, stream);
}

bf_status_t bf_filter(bf_plan_t plan, const void *I, float *out, int H, int W, void *stream) {
  bf_status_t st = check_image(plan, I, out, H, W);
  if (st != BF_OK) return st;
  const bf::Geometry g = geometry_of(plan, H, W);
  if (plan->own_ws_bytes < g.bytes) {
    // the old workspace may still be read by queued work, on any stream
    if (plan->own_ws) {
      if (hipDeviceSynchronize() != hipSuccess) return BF_ERR_DEVICE;
      (void)hipFree(plan->own_ws);
      plan->own_ws = nullptr;
      plan->own_ws_bytes = 0;
    }
    void *d = nullptr;
    if (hipMalloc(&d, g.bytes) != hipSuccess) return BF_ERR_OUT_OF_MEMORY;
    plan->own_ws = d;
    plan->own_ws_bytes = g.bytes;
  }
  return bf::launch_filter(plan->dev_tables, plan->host_tables, g, I, out, nullptr, nullptr,
                           static_cast<int32_t *>(plan->own_ws), stream);
}

bf_status_t bf_filter_noalloc(bf_plan_t plan, const void *I, float *out, int H, int W, void *stream) {
  bf_status_t st = check_image(plan, I, out, H, W);
  if (st != BF_OK) return st;
  const bf::Geometry g = geometry_of(plan, H, W);
  if (g.bytes > bf::kScratchBytes) return BF_ERR_INVALID_ARG;
  void *ws = nullptr;
  st = bf::scratch_workspace(&ws);
  if (st != BF_OK) return st;
  return bf::launch_filter(plan->dev_tables, plan->host_tables, g, I, out, nullptr, nullptr,
                           static_cast<int32_t *>(ws), stream);
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

bf_status_t bf_batch_workspace_size(const bf_plan_t *plans, int n, const int *H, const int *W,
                                    size_t *bytes) {
  if (!plans || !H || !W || !bytes || n < 0) return BF_ERR_INVALID_ARG;
  size_t need = bf::kBatchHeadBytes;
  for (int i = 0; i < n; ++i) {
    size_t b = 0;
    bf_status_t st = bf_workspace_size(plans[i], H[i], W[i], &b);
    if (st != BF_OK) return st;
    need += align256(b);
  }
  *bytes = need;
  return BF_OK;
}

bf_status_t bf_filter_batch(const bf_plan_t *plans, int n, const void *const *I, float *const *out,
                            const int *H, const int *W, void *ws, size_t ws_bytes, void *stream) {
  if (!plans || !I || !out || !H || !W || n < 0) return BF_ERR_INVALID_ARG;
  if (n == 0) return BF_OK;
  if (!ws) return BF_ERR_INVALID_ARG;
  std::vector<bf::BatchItem> items(n);
  size_t off = bf::kBatchHeadBytes;
  for (int i = 0; i < n; ++i) {
    bf_status_t st = check_image(plans[i], I[i], out[i], H[i], W[i]);
    if (st != BF_OK) return st;
    bf::BatchItem &it = items[i];
    it.dev = plans[i]->dev_tables;
    it.host = &plans[i]->host_tables;
    it.g = geometry_of(plans[i], H[i], W[i]);
    it.I = I[i];
    it.out = out[i];
    it.ws = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + off);
    off += align256(it.g.bytes);
  }
  if (ws_bytes < off) return BF_ERR_INVALID_ARG;
  // no output may overlap another output, any input or the workspace (the
  // lookup launch reads every input while it writes every output)
  auto in_bytes = [&](int i) {
    return (size_t)H[i] * W[i] * (plans[i]->in_dtype == BF_IN_U8 ? 1 : 4);
  };
  for (int i = 0; i < n; ++i) {
    const size_t oi = (size_t)H[i] * W[i] * 4;
    if (ranges_overlap(out[i], oi, ws, off) || ranges_overlap(I[i], in_bytes(i), ws, off))
      return BF_ERR_INVALID_ARG;
    for (int j = 0; j < n; ++j) {
      if (j > i && ranges_overlap(out[i], oi, out[j], (size_t)H[j] * W[j] * 4)) return BF_ERR_INVALID_ARG;
      if (j != i && ranges_overlap(out[i], oi, I[j], in_bytes(j))) return BF_ERR_INVALID_ARG;
    }
  }
  return bf::launch_batch(items.data(), n, static_cast<uint32_t *>(ws), stream);
}

bf_status_t bf_batch_set_fused(int fused) {
  if (fused != 0 && fused != 1) return BF_ERR_INVALID_ARG;
  bf::set_fused_batch(fused);
  return BF_OK;
}

bf_status_t bf_autotune(bf_plan_t plan, int H, int W, int reps, void *stream, int *tile_out) {
  if (!plan || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return BF_ERR_INVALID_ARG;
  if (plan->flags & BF_FLAG_HOST_ONLY) return BF_ERR_INVALID_ARG;
  if (!tunable(plan)) {
    if (tile_out) *tile_out = geometry_of(plan, H, W).tile;
    return BF_OK;
  }
  reps = std::max(reps, 3);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bf::DevTables &h = plan->host_tables;
  const int r = plan->fit.radius;
  struct Cand {
    int tile, single, one;
  };
  std::vector<Cand> cands;
  // the general tiles, and for a lattice plan the tiles that hold whole lattice tiles
  std::vector<int> tiles = {64, 128, 256, 512};
  if (bf::lattice_eligible(h)) {
    const int l = std::lcm(64, bf::lattice_rows(h));
    for (int c = l; c <= 576; c += l)
      if (std::find(tiles.begin(), tiles.end(), c) == tiles.end()) tiles.push_back(c);
  }
  for (int t : tiles) {
    if (t + 2 * r + 1 > 1024) continue;
    if ((t > 64 && (t / 2) >= std::max(H, W))) continue;  // one tile already covers the image
    for (int one = 0; one < 3; ++one) {
      // the default lookup kernel, and each other one the plan can use
      const int dflt = bf::lookup_kernel_for(h, 0);
      cands.push_back({t, 0, one});
      if (bf::kb_tile_eligible(h) && dflt != 2) cands.push_back({t, 1, one});
      if (bf::lattice_eligible(h) && dflt != 3) cands.push_back({t, 2, one});
    }
  }
  if (cands.empty()) cands.push_back({64, 0, 0});
  size_t ws_bytes = 0;
  for (const Cand &c : cands)
    ws_bytes = std::max(ws_bytes, geometry_with(plan, H, W, c.tile, c.single, c.one).bytes);
  const size_t in_bytes = (size_t)H * W * (plan->in_dtype == BF_IN_U8 ? 1 : 4);
  void *I = nullptr, *out = nullptr, *ws = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bf_status_t st = BF_OK;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (I) (void)hipFree(I);
    if (out) (void)hipFree(out);
    if (ws) (void)hipFree(ws);
  };
  if (hipMalloc(&I, in_bytes) != hipSuccess || hipMalloc(&out, (size_t)H * W * 4) != hipSuccess ||
      hipMalloc(&ws, ws_bytes) != hipSuccess) {
    cleanup();
    return BF_ERR_OUT_OF_MEMORY;
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipMemsetAsync(I, plan->in_dtype == BF_IN_U8 ? 0x80 : 0x3E, in_bytes, s) != hipSuccess) {
    cleanup();
    return BF_ERR_DEVICE;
  }
  std::vector<float> times;
  times.reserve(cands.size());
  for (const Cand &c : cands) {
    const bf::Geometry g = geometry_with(plan, H, W, c.tile, c.single, c.one);
    st = bf::launch_filter(plan->dev_tables, h, g, I, static_cast<float *>(out), nullptr, nullptr,
                           static_cast<int32_t *>(ws), s);
    if (st != BF_OK) break;
    if (hipEventRecord(e0, s) != hipSuccess) st = BF_ERR_DEVICE;
    for (int i = 0; i < reps && st == BF_OK; ++i)
      st = bf::launch_filter(plan->dev_tables, h, g, I, static_cast<float *>(out), nullptr, nullptr,
                             static_cast<int32_t *>(ws), s);
    float ms = 0;
    if (st != BF_OK || hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      if (st == BF_OK) st = BF_ERR_DEVICE;
      break;
    }
    times.push_back(ms);
  }
  if (st == BF_OK && hipStreamSynchronize(s) != hipSuccess) st = BF_ERR_DEVICE;
  cleanup();
  if (st != BF_OK) return st;
  // the fastest shape; among those within 1% of it (timing noise), the one
  // with the smallest workspace
  const float fastest = *std::min_element(times.begin(), times.end());
  Cand best = cands[0];
  size_t best_bytes = SIZE_MAX;
  for (size_t i = 0; i < cands.size(); ++i) {
    if (times[i] > 1.01f * fastest) continue;
    const size_t b = geometry_with(plan, H, W, cands[i].tile, cands[i].single, cands[i].one).bytes;
    if (b < best_bytes) {
      best_bytes = b;
      best = cands[i];
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[tune_key(plan, H, W)] = TuneVal{best.tile, best.single, best.one};
  }
  if (tile_out) *tile_out = best.tile;
  return BF_OK;
}

bf_status_t bf_tuning_set(bf_plan_t plan, int H, int W, int tile, int kb_single, int ka_one) {
  if (!plan || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return BF_ERR_INVALID_ARG;
  if (tile < 64 || tile % 64 || tile + 2 * plan->fit.radius + 1 > 1024 || kb_single < 0 || kb_single > 2 ||
      ka_one < 0 || ka_one > 2)
    return BF_ERR_INVALID_ARG;
  if (!tunable(plan)) return BF_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned[tune_key(plan, H, W)] = TuneVal{tile, kb_single, ka_one};
  return BF_OK;
}

bf_status_t bf_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tuned.clear();
  return BF_OK;
}

// ---------------------------------------------------------------------------
// Pre-computed tables (Case 1 of Sec. V-C): the term tables of an image built
// once under one plan serve later plans whose terms they contain.
// ---------------------------------------------------------------------------

bf_status_t bf_precompute_size(bf_plan_t tables_plan, int H, int W, size_t *bytes) {
  if (!tables_plan || !bytes || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return BF_ERR_INVALID_ARG;
  *bytes = precompute_geometry(tables_plan, H, W).bytes;
  return BF_OK;
}

bf_status_t bf_precompute(bf_plan_t tables_plan, const void *I, int H, int W, void *ws, size_t ws_bytes,
                          void *stream) {
  if (!tables_plan || !I || !ws || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return BF_ERR_INVALID_ARG;
  if (tables_plan->host_tables.direct || tables_plan->host_tables.range_box || tables_plan->host_tables.reduced)
    return BF_ERR_UNSUPPORTED;
  if (tables_plan->flags & BF_FLAG_HOST_ONLY) return BF_ERR_INVALID_ARG;
  const bf::Geometry g = precompute_geometry(tables_plan, H, W);
  const size_t in_bytes = (size_t)H * W * (tables_plan->in_dtype == BF_IN_U8 ? 1 : 4);
  if (ws_bytes < g.bytes || ranges_overlap(ws, g.bytes, I, in_bytes)) return BF_ERR_INVALID_ARG;
  return bf::launch_tables(tables_plan->dev_tables, tables_plan->host_tables, g, I,
                           static_cast<int32_t *>(ws), stream);
}

bf_status_t bf_precomputed_compatible(bf_plan_t tables_plan, bf_plan_t plan) {
  if (!tables_plan || !plan) return BF_ERR_INVALID_ARG;
  if (tables_plan->host_tables.direct || plan->host_tables.direct || tables_plan->host_tables.range_box ||
      plan->host_tables.range_box || tables_plan->host_tables.reduced || plan->host_tables.reduced)
    return BF_ERR_UNSUPPORTED;
  const bf::DevTables &a = tables_plan->host_tables, &b = plan->host_tables;
  if (tables_plan->in_dtype != plan->in_dtype) return BF_ERR_INVALID_ARG;
  if (plan->fit.radius > tables_plan->fit.radius) return BF_ERR_INVALID_ARG;  // halo too small
  if (b.n_terms > a.n_terms) return BF_ERR_INVALID_ARG;
  for (int i = 0; i < b.n_terms; ++i)  // the same terms, in the same table slots
    if (plan->fit.k[i] != tables_plan->fit.k[i] || b.f_hi[i] != a.f_hi[i] || b.f_lo[i] != a.f_lo[i] ||
        b.slot[i] != a.slot[i])
      return BF_ERR_INVALID_ARG;
  return BF_OK;
}

bf_status_t bf_filter_precomputed(bf_plan_t tables_plan, bf_plan_t plan, const void *I, float *out, int H,
                                  int W, const void *ws, size_t ws_bytes, void *stream) {
  bf_status_t st = bf_precomputed_compatible(tables_plan, plan);
  if (st != BF_OK) return st;
  st = check_image(plan, I, out, H, W);
  if (st != BF_OK) return st;
  const bf::Geometry g = precompute_geometry(tables_plan, H, W);
  if (!ws || ws_bytes < g.bytes || ranges_overlap(ws, g.bytes, out, (size_t)H * W * 4)) return BF_ERR_INVALID_ARG;
  return bf::launch_lookup(plan->dev_tables, plan->host_tables, g, I, out, nullptr, nullptr,
                           static_cast<const int32_t *>(ws), stream);
}

bf_status_t bf_plan_query(bf_plan_t plan, bf_plan_info_t *info) {
  if (!plan || !info) return BF_ERR_INVALID_ARG;
  const bf::Fit &f = plan->fit;
  info->radius = f.radius;
  info->n_range = (int)f.k.size();
  info->n_spatial = (int)f.group_lx.size();
  info->n_taps = (int)f.tap_w.size();
  info->n_tap_rows = (int)f.row_off.size();
  info->n_tap_cols = (int)f.col_off.size();
  info->n_images = plan->host_tables.n_images;
  info->tile = plan->tile;
  info->n_quads = plan->host_tables.n_quads;
  info->lookup_kernel = bf::lookup_kernel_kind(plan->host_tables);
  info->direct = plan->host_tables.direct;
  info->range_box = plan->host_tables.range_box && !plan->host_tables.level_fold;
  info->level_fold = plan->host_tables.level_fold;
  info->box_levels = plan->host_tables.range_box ? plan->host_tables.box_zr : -1;
  info->box_tile = plan->host_tables.range_box ? bf::rangebox_tile(plan->host_tables) : 0;
  info->reduced = plan->host_tables.reduced;
  info->n_single = 0;
  info->lds_pitch = bf::lookup_kernel_kind(plan->host_tables) ? plan->host_tables.lds_pitch : 0;
  info->lds_double_buffered = bf::kb_tile_eligible(plan->host_tables) && bf::kb_double_buffered(plan->host_tables);
  info->lattice = bf::lattice_eligible(plan->host_tables);
  info->lattice_step = info->lattice ? plan->host_tables.lat_s : 0;
  info->default_lookup = bf::lookup_kernel_for(plan->host_tables, 0);
  if (plan->host_tables.range_box) {
    info->sat_shift = (int)std::lround(std::log2((double)plan->host_tables.box_scale));
  } else {  // q depends on r and gmax only
    int tile = 0, q = 0;
    bf::choose_tiling(64, 64, f.radius, plan->host_tables.n_terms, 64, plan->gmax, 0, &tile, &q);
    info->sat_shift = q;
  }
  info->T_s = f.T_s;
  info->T_r = f.T_r;
  info->T = f.T;
  info->den_floor = 1e-7 * f.sum_abs_K;  // the kernels compare against its FP32 rounding
  return BF_OK;
}

bf_status_t bf_image_geometry(bf_plan_t plan, int H, int W, int *tile, int *sat_shift,
                              size_t *ws_bytes) {
  if (!plan || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return BF_ERR_INVALID_ARG;
  const bf::Geometry g = geometry_of(plan, H, W);
  if (tile) *tile = g.tile;
  if (sat_shift) *sat_shift = g.sat_shift;
  if (ws_bytes) *ws_bytes = g.bytes;
  return BF_OK;
}

bf_status_t bf_image_lookup_kernel(bf_plan_t plan, int H, int W, int *kind) {
  if (!plan || !kind || H < 1 || W < 1 || H > kMaxSide || W > kMaxSide) return BF_ERR_INVALID_ARG;
  const bf::DevTables &h = plan->host_tables;
  if (h.direct || h.range_box || h.level_fold || h.reduced) {
    *kind = -1;
    return BF_OK;
  }
  *kind = bf::lookup_kernel_for(h, geometry_of(plan, H, W).kb_single);
  return BF_OK;
}

bf_status_t bf_plan_range_terms(bf_plan_t plan, int *k, double *a, double *omega, int capacity) {
  if (!plan || !k || !a || !omega || capacity < (int)plan->fit.k.size()) return BF_ERR_INVALID_ARG;
  for (size_t i = 0; i < plan->fit.k.size(); ++i) {
    k[i] = plan->fit.k[i];
    a[i] = plan->fit.a[i];
    omega[i] = plan->fit.omega[i];
  }
  return BF_OK;
}

bf_status_t bf_plan_spatial_kernel(bf_plan_t plan, double *K, int capacity) {
  if (!plan || !K || capacity < (int)plan->fit.K.size()) return BF_ERR_INVALID_ARG;
  std::copy(plan->fit.K.begin(), plan->fit.K.end(), K);
  return BF_OK;
}

bf_status_t bf_plan_taps(bf_plan_t plan, int *dy, int *dx, double *w, int capacity) {
  if (!plan || !dy || !dx || !w || capacity < (int)plan->fit.tap_w.size()) return BF_ERR_INVALID_ARG;
  for (size_t i = 0; i < plan->fit.tap_w.size(); ++i) {
    dy[i] = plan->fit.tap_dy[i];
    dx[i] = plan->fit.tap_dx[i];
    w[i] = plan->fit.tap_w[i];
  }
  return BF_OK;
}

bf_status_t bf_plan_spatial_groups(bf_plan_t plan, int *level_x, int *level_y, int capacity) {
  if (!plan || !level_x || !level_y || capacity < (int)plan->fit.group_lx.size())
    return BF_ERR_INVALID_ARG;
  for (size_t i = 0; i < plan->fit.group_lx.size(); ++i) {
    level_x[i] = plan->fit.group_lx[i];
    level_y[i] = plan->fit.group_ly[i];
  }
  return BF_OK;
}

const char *bf_status_string(bf_status_t s) {
  switch (s) {
    case BF_OK: return "BF_OK";
    case BF_ERR_INVALID_ARG: return "BF_ERR_INVALID_ARG";
    case BF_ERR_OUT_OF_MEMORY: return "BF_ERR_OUT_OF_MEMORY";
    case BF_ERR_DEVICE: return "BF_ERR_DEVICE";
    case BF_ERR_UNSUPPORTED: return "BF_ERR_UNSUPPORTED";
  }
  return "BF_ERR_UNKNOWN";
}

const char *bf_version(void) { return "bf-mi355x 0.1 (gfx950)"; }

}  // extern "C"
