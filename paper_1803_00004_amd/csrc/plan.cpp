// Host-side FP64 fit of the two kernel expansions and compilation of the
// spatial expansion into summed-area-table taps.
//
//  * Spatial: best N-term approximation of the truncated Gaussian K_s on 2-D
//    Haar functions (Sec. III-C Eqs. Haar_scaling / Haar_mother / Haar_set,
//    2-D coefficients of Eq. Haar_2D_coefficients, selection of Eq.
//    Haar_N_terms).  The kernel is selected in level groups (all functions of
//    one level pair) ranked by L2 energy, point-sampled on the integer grid
//    with half-open intervals, T_s = r + 1/2.
//  * Taps: the sampled kernel is piecewise constant on rectangles (App. A,
//    Table VI); its mixed second differences give the corners at which the
//    four-reference box sums of Eq. sum_sat_sum_region_2D read the table.
//    Other kernels (Secs. I, IV-B and VI: the expansion takes any symmetric
//    kernel): the radial exponential exp(-||d|| / sigma_s), which is not
//    separable, and tabulated kernels get their 2-D coefficients from
//    integrals over the finest Haar cells -- by quadrature for the exponential,
//    as exact overlap sums for a table (constant on unit squares).
//  * Range: best N-term truncated cosine approximation (Sec. III-B, Eq.
//    1D_truncated_cos; Sec. IV-C, Eq. trigonometric_N_terms), coefficients by
//    composite Gauss-Legendre quadrature (in closed form for a table, linear
//    between samples), the N largest |a_k| among the first
//    20N (App. B), on [-T, T] with T = max(T_r, span) so that every intensity
//    difference lies inside the series interval.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "bf_internal.h"

namespace bf {
namespace {

constexpr double kPi = 3.14159265358979323846;

// Integral of exp(-t^2 / 2 sigma^2) over [a, b].
double gauss_int(double a, double b, double sigma) {
  const double s = sigma * std::sqrt(2.0);
  return sigma * std::sqrt(kPi / 2.0) * (std::erf(b / s) - std::erf(a / s));
}

struct Haar {
  int level;  // -1 = phi
  int k;
  double lo, mid, hi;
  double sample(double d) const {
    if (level < 0) return (d >= lo && d < hi) ? 1.0 : 0.0;
    if (d >= lo && d < mid) return 1.0;
    if (d >= mid && d < hi) return -1.0;
    return 0.0;
  }
};

std::vector<Haar> haar_family(double T, int J) {
  std::vector<Haar> f;
  f.push_back({-1, 0, -T, 0.0, T});
  f.push_back({0, 0, -T, 0.0, T});
  for (int j = 1; j <= J; ++j) {
    const int half = 1 << (j - 1);
    const double s = std::ldexp(1.0, -j);
    for (int k = -half; k <= half; ++k) {
      if (k == 0) continue;
      const double Z = (k > 0 ? 1.0 : -1.0) * (2.0 * std::abs(k) - 1.0) * T;
      f.push_back({j, k, s * (Z - T), s * Z, s * (Z + T)});
    }
  }
  return f;
}

double round_sig12(double x) {
  if (x == 0.0) return 0.0;
  char buf[64];
  std::snprintf(buf, sizeof buf, "%.11e", x);
  return std::strtod(buf, nullptr);
}

// n-point Gauss-Legendre nodes/weights on [-1, 1] (Newton on P_n).
void gauss_legendre(int n, std::vector<double> *x, std::vector<double> *w) {
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int m = 2; m <= n; ++m) {
        const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int m = 2; m <= n; ++m) {
      const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    (*x)[i] = z;
    (*w)[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Kernel profiles by kind (bf_kernel_t): 0 Gaussian, 1 exponential.
double range_profile(int kind, double t, double sigma) {
  return kind == BF_KERNEL_EXPONENTIAL ? std::exp(-std::fabs(t) / sigma)
                                       : std::exp(-t * t / (2.0 * sigma * sigma));
}
double spatial_profile(int kind, double x, double y, double sigma) {
  return kind == BF_KERNEL_EXPONENTIAL ? std::exp(-std::sqrt(x * x + y * y) / sigma)
                                       : std::exp(-(x * x + y * y) / (2.0 * sigma * sigma));
}
// K^{-1}(eps) of the 1-D profile (Sec. IV-A).
double kernel_inverse(int kind, double sigma, double eps) {
  return kind == BF_KERNEL_EXPONENTIAL ? sigma * std::log(1.0 / eps)
                                       : sigma * std::sqrt(2.0 * std::log(1.0 / eps));
}

// Integrals of K_s over the cells [x0, x0 + h) x [y0, y0 + h) of the quadrant
// x, y >= 0 of a grid with corner at the origin: Q[jy * n + ix], n cells per
// axis.  The cell at the origin holds the kernel's only non-smooth point
// (radial kernels) in its corner; there the square is split along its
// diagonal and each triangle mapped onto the unit square with the Jacobian
// vanishing at the corner (x = h s, y = h s t), which makes the integrand
// smooth.  Elsewhere: 2 x 2 panels of 10 x 10 Gauss-Legendre nodes per cell.
void quadrant_cell_integrals(int kind, double sigma, double h, int n, std::vector<double> *Q) {
  std::vector<double> gx, gw, cx, cw;
  gauss_legendre(10, &gx, &gw);
  for (int p = 0; p < 2; ++p)
    for (int i = 0; i < 10; ++i) {
      cx.push_back(0.25 * h * (gx[i] + 1.0) + 0.5 * h * p);  // node offset inside a cell
      cw.push_back(0.25 * h * gw[i]);
    }
  Q->assign((size_t)n * n, 0.0);
  for (int jy = 0; jy < n; ++jy)
    for (int ix = 0; ix < n; ++ix) {
      if (ix == 0 && jy == 0) continue;
      double s = 0.0;
      for (size_t a = 0; a < cx.size(); ++a) {
        double row = 0.0;
        for (size_t b = 0; b < cx.size(); ++b)
          row += cw[b] * spatial_profile(kind, ix * h + cx[b], jy * h + cx[a], sigma);
        s += cw[a] * row;
      }
      (*Q)[(size_t)jy * n + ix] = s;
    }
  std::vector<double> dx, dw;
  gauss_legendre(24, &dx, &dw);
  double s = 0.0;
  for (size_t a = 0; a < dx.size(); ++a) {
    const double u = 0.5 * (dx[a] + 1.0), wu = 0.5 * dw[a];  // radial-like coordinate
    for (size_t b = 0; b < dx.size(); ++b) {
      const double v = 0.5 * (dx[b] + 1.0), wv = 0.5 * dw[b];
      const double jac = h * h * u;
      s += wu * wv * jac * (spatial_profile(kind, h * u, h * u * v, sigma) +   // y <= x
                            spatial_profile(kind, h * u * v, h * u, sigma));   // x <= y
    }
  }
  (*Q)[0] = s;
}

// Cells of the quadrant (as above) for a tabulated K_s: weight ks(dy, dx) on
// the unit square [dx - 1/2, dx + 1/2) x [dy - 1/2, dy + 1/2).  A cell's
// integral is the sum over the squares it meets of weight times overlap
// area; the cell side h = (2r + 1) / 2^(J+1) and the square edges are exact
// binary fractions, so every overlap length is exact.
void tabulated_quadrant_cells(const double *ks, int r, double h, int n, std::vector<double> *Q) {
  const int K = 2 * r + 1;
  struct Span { int d; double len; };
  std::vector<std::vector<Span>> ov(n);  // per cell: offsets d >= 0 met, with the overlap length
  for (int i = 0; i < n; ++i) {
    const double lo = i * h, hi = (i + 1) * h;
    for (int d = std::max(0, (int)std::floor(lo - 0.5)); d <= r && d - 0.5 < hi; ++d) {
      const double len = std::min(hi, d + 0.5) - std::max(lo, d - 0.5);
      if (len > 0) ov[i].push_back({d, len});
    }
  }
  Q->assign((size_t)n * n, 0.0);
  for (int jy = 0; jy < n; ++jy)
    for (int ix = 0; ix < n; ++ix) {
      double s = 0.0;
      for (const Span &a : ov[jy]) {
        double row = 0.0;
        for (const Span &b : ov[ix]) row += b.len * ks[(size_t)(a.d + r) * K + b.d + r];
        s += a.len * row;
      }
      (*Q)[(size_t)jy * n + ix] = s;
    }
}

// Checks of a tabulated kernel: finite, non-negative weights, a positive
// centre, and a spatial table even in dy and in dx (bitwise).
bool valid_tables(const KernelSpec &k, int radius) {
  if (k.ks) {
    const int K = 2 * radius + 1;
    const double *t = k.ks;
    for (int i = 0; i < K * K; ++i)
      if (!std::isfinite(t[i]) || t[i] < 0) return false;
    if (!(t[(size_t)radius * K + radius] > 0)) return false;
    for (int y = 0; y < K; ++y)
      for (int x = 0; x < K; ++x) {
        const double v = t[(size_t)y * K + x];
        if (v != t[(size_t)(K - 1 - y) * K + x] || v != t[(size_t)y * K + K - 1 - x]) return false;
      }
  }
  if (k.kr) {
    if (k.kr_n < 2 || k.kr_n > kMaxRangeSamples || !(k.kr_step > 0) || !std::isfinite(k.kr_step)) return false;
    for (int i = 0; i < k.kr_n; ++i)
      if (!std::isfinite(k.kr[i]) || k.kr[i] < 0) return false;
    if (!(k.kr[0] > 0)) return false;
  }
  return true;
}

// a_j (j < M) of the even function equal on [0, T] to the linear interpolant
// of v_i = K_r(i s) and zero past t_{n-1} <= T.  On a piece [t_i, t_i + s]
// with slope beta_i, integration by parts gives
// [f sin(w t) / w + beta_i cos(w t) / w^2]; the first part telescopes over the
// pieces to v_{n-1} sin(w t_{n-1}) / w (sin 0 = 0), and each cosine
// difference is -2 sin(w (t_i + s/2)) sin(w s / 2).
void table_cosine_coefficients(const double *v, int n, double s, double T, int M, std::vector<double> *a) {
  a->assign(M, 0.0);
  double area = 0.0;
  for (int i = 0; i + 1 < n; ++i) area += 0.5 * (v[i] + v[i + 1]) * s;
  (*a)[0] = area / T;
  const double tl = (n - 1) * s;
  for (int j = 1; j < M; ++j) {
    const double w = kPi * j / T;
    double acc = 0.0;
    for (int i = 0; i + 1 < n; ++i) acc += (v[i + 1] - v[i]) / s * std::sin(w * (i * s + 0.5 * s));
    const double integral = v[n - 1] * std::sin(w * tl) / w - 2.0 * std::sin(0.5 * w * s) * acc / (w * w);
    (*a)[j] = 2.0 * integral / T;
  }
}

// a_j (j < M) of an analytic K_r on [-T, T] by composite 16-point
// Gauss-Legendre quadrature: 4 panels per period of the highest frequency, at
// least 256.
void kernel_cosine_coefficients(int kind, double sigma, double T, int M, std::vector<double> *a) {
  const int panels = std::max(256, 4 * M);
  std::vector<double> gx, gw;
  gauss_legendre(16, &gx, &gw);
  std::vector<double> t, fw;
  t.reserve((size_t)panels * 16);
  fw.reserve((size_t)panels * 16);
  const double h = 2.0 * T / panels;
  for (int p = 0; p < panels; ++p) {
    const double lo = -T + p * h;
    for (int i = 0; i < 16; ++i) {
      const double tt = lo + 0.5 * h * (gx[i] + 1.0);
      t.push_back(tt);
      fw.push_back(0.5 * h * gw[i] * range_profile(kind, tt, sigma));
    }
  }
  a->assign(M, 0.0);
  for (int j = 0; j < M; ++j) {
    double s = 0.0;
    const double w = kPi * j / T;
    for (size_t i = 0; i < t.size(); ++i) s += std::cos(w * t[i]) * fw[i];
    (*a)[j] = (j == 0 ? 0.5 : 1.0) * s / T;
  }
}

}  // namespace

bf_status_t fit_plan(const KernelSpec &kern, int radius, bf_terms_t N, double eps, double span, Fit *out) {
  const int kind_s = kern.ks ? -1 : kern.kind_s, kind_r = kern.kr ? -1 : kern.kind_r;
  const double sigma_s = kern.sigma_s, sigma_r = kern.sigma_r;
  if ((!kern.ks && (!(sigma_s > 0) || !std::isfinite(sigma_s))) ||
      (!kern.kr && (!(sigma_r > 0) || !std::isfinite(sigma_r))) || !(eps > 0 && eps < 1) || !(span >= 0) ||
      !std::isfinite(span))
    return BF_ERR_INVALID_ARG;
  if (radius == 0 && !kern.ks) radius = (int)std::ceil(kernel_inverse(kind_s, sigma_s, eps));
  if (radius < 1 || radius > 1024) return BF_ERR_INVALID_ARG;
  // the cell integrals of a non-separable kernel cost O((2^J)^2) evaluations
  if (kind_s != BF_KERNEL_GAUSSIAN && radius > kMaxCellFitRadius) return BF_ERR_UNSUPPORTED;
  if (!valid_tables(kern, radius)) return BF_ERR_INVALID_ARG;
  if (N.n_range < 1 || N.n_range > kMaxTerms) return BF_ERR_INVALID_ARG;

  Fit f;
  f.radius = radius;
  f.eps = eps;
  f.span = span;

  // ---------------- spatial ----------------
  const double T = radius + 0.5;
  f.T_s = T;
  const int J = (int)std::floor(std::log2(T));
  const int n_levels = J + 2;  // phi, 0..J
  if (N.n_spatial < 1 || N.n_spatial > n_levels * n_levels) return BF_ERR_INVALID_ARG;
  const std::vector<Haar> fam = haar_family(T, J);
  struct Group { double e; int lx, ly; };
  std::vector<Group> groups;
  auto rank_groups = [&]() {
    std::sort(groups.begin(), groups.end(), [](const Group &a, const Group &b) {
      if (a.e != b.e) return a.e > b.e;
      if (a.lx + a.ly != b.lx + b.ly) return a.lx + a.ly < b.lx + b.ly;
      return a.lx < b.lx;
    });
  };
  const int ks = 2 * radius + 1;
  f.K.assign((size_t)ks * ks, 0.0);
  if (kind_s == BF_KERNEL_GAUSSIAN) {
    // separable: 2-D coefficients are products of 1-D ones (closed form)
    std::vector<double> c(fam.size());
    std::vector<double> e1(n_levels, 0.0);  // index level + 1
    for (size_t i = 0; i < fam.size(); ++i) {
      const Haar &h = fam[i];
      if (h.level < 0)
        c[i] = gauss_int(h.lo, h.hi, sigma_s) / (2.0 * T);
      else
        c[i] = std::ldexp(1.0, h.level) *
               (gauss_int(h.lo, h.mid, sigma_s) - gauss_int(h.mid, h.hi, sigma_s)) / (2.0 * T);
      e1[h.level + 1] += c[i] * c[i] * (h.hi - h.lo);
    }
    for (int lx = -1; lx <= J; ++lx)
      for (int ly = -1; ly <= J; ++ly)
        groups.push_back({round_sig12(e1[lx + 1] * e1[ly + 1]), lx, ly});
    rank_groups();
    // u_l(d) = sum_{b in level l} c_b b(d), d in [-r, r]
    std::vector<double> u((size_t)n_levels * ks, 0.0);
    for (size_t i = 0; i < fam.size(); ++i)
      for (int d = -radius; d <= radius; ++d)
        u[(size_t)(fam[i].level + 1) * ks + d + radius] += c[i] * fam[i].sample((double)d);
    for (int g = 0; g < N.n_spatial; ++g) {
      const int lx = groups[g].lx, ly = groups[g].ly;
      f.group_lx.push_back(lx);
      f.group_ly.push_back(ly);
      const double *ux = &u[(size_t)(lx + 1) * ks], *uy = &u[(size_t)(ly + 1) * ks];
      for (int iy = 0; iy < ks; ++iy)
        for (int ix = 0; ix < ks; ++ix) f.K[(size_t)iy * ks + ix] += uy[iy] * ux[ix];
    }
  } else {
    // Not separable.  Every Haar function up to level J is constant on the
    // n = 2^(J+1) finest cells of [-T, T): it is +-1 on one or two aligned
    // blocks of n / 2^e cells (e = 0 for phi, level + 1 for psi), so
    // <K, h_a(x) h_b(y)> is a signed sum of block sums of the cell-integral
    // matrix.  The block sums of every (e_x, e_y) come from pairwise sums of
    // the finer ones (positive terms: no cancellation, and mirrored blocks get
    // bitwise equal sums, so the symmetric taps pair exactly).
    // c_ab = <K, h_a h_b> / (|h_a|^2 |h_b|^2).
    const int n = 1 << (J + 1), n2 = n / 2, E = J + 2;  // block exponents e = 0 .. J + 1
    const double h = 2.0 * T / n;
    std::vector<double> Q;
    if (kern.ks)  // kernel even in x and in y
      tabulated_quadrant_cells(kern.ks, radius, h, n2, &Q);
    else
      quadrant_cell_integrals(kind_s, sigma_s, h, n2, &Q);
    // X[ex]: n rows x 2^ex column blocks; B[ex][ey]: 2^ey x 2^ex blocks
    std::vector<std::vector<double>> X(E);
    X[E - 1].resize((size_t)n * n);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const int qi = i >= n2 ? i - n2 : n2 - 1 - i, qj = j >= n2 ? j - n2 : n2 - 1 - j;
        X[E - 1][(size_t)j * n + i] = Q[(size_t)qj * n2 + qi];
      }
    for (int ex = E - 2; ex >= 0; --ex) {
      const int w = 1 << ex;
      X[ex].resize((size_t)n * w);
      for (int j = 0; j < n; ++j)
        for (int c = 0; c < w; ++c)
          X[ex][(size_t)j * w + c] = X[ex + 1][(size_t)j * 2 * w + 2 * c] + X[ex + 1][(size_t)j * 2 * w + 2 * c + 1];
    }
    std::vector<std::vector<double>> B((size_t)E * E);
    for (int ex = 0; ex < E; ++ex) {
      const int w = 1 << ex;
      B[(size_t)ex * E + E - 1] = X[ex];
      for (int ey = E - 2; ey >= 0; --ey) {
        const int hgt = 1 << ey;
        const std::vector<double> &fine = B[(size_t)ex * E + ey + 1];
        std::vector<double> &out = B[(size_t)ex * E + ey];
        out.resize((size_t)hgt * w);
        for (int r = 0; r < hgt; ++r)
          for (int c = 0; c < w; ++c) out[(size_t)r * w + c] = fine[(size_t)2 * r * w + c] + fine[(size_t)(2 * r + 1) * w + c];
      }
    }
    struct Piece { int e, blk; double sign; };
    auto pieces = [&](const Haar &f, Piece *pc) {  // returns the count
      if (f.level < 0) {
        pc[0] = {0, 0, 1.0};
        return 1;
      }
      const int e = f.level + 1;
      const int blk = (int)std::lround((f.lo + T) / h) / (n >> e);
      pc[0] = {e, blk, 1.0};
      pc[1] = {e, blk + 1, -1.0};
      return 2;
    };
    const size_t nf = fam.size();
    std::vector<double> C(nf * nf);  // C[b * nf + a]: h_a in x, h_b in y
    std::vector<double> e2((size_t)n_levels * n_levels, 0.0);
    for (size_t b = 0; b < nf; ++b)
      for (size_t a = 0; a < nf; ++a) {
        const Haar &fa = fam[a], &fb = fam[b];
        Piece pa[2], pb[2];
        const int na_p = pieces(fa, pa), nb_p = pieces(fb, pb);
        double ip = 0.0;
        for (int u = 0; u < nb_p; ++u)
          for (int v = 0; v < na_p; ++v) {
            const std::vector<double> &blk = B[(size_t)pa[v].e * E + pb[u].e];
            ip += pb[u].sign * pa[v].sign * blk[(size_t)pb[u].blk * (1 << pa[v].e) + pa[v].blk];
          }
        const double na = fa.hi - fa.lo, nb = fb.hi - fb.lo;
        const double cab = ip / (na * nb);
        C[b * nf + a] = cab;
        e2[(size_t)(fa.level + 1) * n_levels + fb.level + 1] += cab * cab * na * nb;
      }
    // energies of groups that vanish by symmetry are quadrature noise: below
    // 1e-12 of the largest they are zero, and the level rule orders them
    const double floor_e = 1e-12 * *std::max_element(e2.begin(), e2.end());
    for (int lx = -1; lx <= J; ++lx)
      for (int ly = -1; ly <= J; ++ly) {
        const double e = e2[(size_t)(lx + 1) * n_levels + ly + 1];
        groups.push_back({e > floor_e ? round_sig12(e) : 0.0, lx, ly});
      }
    rank_groups();
    // K(dy, dx) += sum_{a in lx} h_a(dx) sum_{b in ly} c_ab h_b(dy)
    std::vector<double> col(ks);
    for (int g = 0; g < N.n_spatial; ++g) {
      const int lx = groups[g].lx, ly = groups[g].ly;
      f.group_lx.push_back(lx);
      f.group_ly.push_back(ly);
      for (size_t a = 0; a < nf; ++a) {
        if (fam[a].level != lx) continue;
        std::fill(col.begin(), col.end(), 0.0);
        for (size_t b = 0; b < nf; ++b) {
          if (fam[b].level != ly) continue;
          for (int d = -radius; d <= radius; ++d) col[d + radius] += C[b * nf + a] * fam[b].sample((double)d);
        }
        for (int dx = -radius; dx <= radius; ++dx) {
          const double hx = fam[a].sample((double)dx);
          if (hx == 0.0) continue;
          for (int iy = 0; iy < ks; ++iy) f.K[(size_t)iy * ks + dx + radius] += hx * col[iy];
        }
      }
    }
  }
  double kmax = 0;
  f.sum_abs_K = 0;
  for (double v : f.K) {
    kmax = std::max(kmax, std::fabs(v));
    f.sum_abs_K += std::fabs(v);
  }
  // Taps.  corr(p) = sum_q K(p - q) g(q) = sum_u D(u) S_incl(p - u) with
  // D(u) = K(u) - K(u - e_y) - K(u - e_x) + K(u - e_y - e_x), u in [-r, r+1]^2
  // (K zero outside the window) and S_incl(Y, X) = S(Y + 1, X + 1) for the
  // exclusive table S; so the tap offset is (1 - u_y, 1 - u_x).
  auto Kat = [&](int dy, int dx) -> double {
    if (dy < -radius || dy > radius || dx < -radius || dx > radius) return 0.0;
    return f.K[(size_t)(dy + radius) * ks + dx + radius];
  };
  std::vector<int> rows, cols;
  for (int uy = -radius; uy <= radius + 1; ++uy)
    for (int ux = -radius; ux <= radius + 1; ++ux) {
      const double D = Kat(uy, ux) - Kat(uy - 1, ux) - Kat(uy, ux - 1) + Kat(uy - 1, ux - 1);
      if (std::fabs(D) <= 1e-14 * kmax) continue;
      f.tap_dy.push_back(1 - uy);
      f.tap_dx.push_back(1 - ux);
      f.tap_w.push_back(D);
      rows.push_back(1 - uy);
      cols.push_back(1 - ux);
    }
  std::sort(rows.begin(), rows.end());
  rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
  std::sort(cols.begin(), cols.end());
  cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  f.row_off = rows;
  f.col_off = cols;
  f.tap_grid.assign(rows.size() * cols.size(), 0.0);
  for (size_t t = 0; t < f.tap_w.size(); ++t) {
    const size_t i = std::lower_bound(rows.begin(), rows.end(), f.tap_dy[t]) - rows.begin();
    const size_t j = std::lower_bound(cols.begin(), cols.end(), f.tap_dx[t]) - cols.begin();
    f.tap_grid[i * cols.size() + j] = f.tap_w[t];
  }

  // ---------------- range ----------------
  f.T_r = kern.kr ? (kern.kr_n - 1) * kern.kr_step : kernel_inverse(kind_r, sigma_r, eps);
  f.T = std::max(f.T_r, span);
  const int M = std::max(20 * N.n_range, 2);
  std::vector<double> a;
  if (kern.kr)
    table_cosine_coefficients(kern.kr, kern.kr_n, kern.kr_step, f.T, M, &a);
  else
    kernel_cosine_coefficients(kind_r, sigma_r, f.T, M, &a);
  double amax = 0;
  for (double v : a) amax = std::max(amax, std::fabs(v));
  std::vector<double> q(M);
  for (int j = 0; j < M; ++j) q[j] = amax > 0 ? std::nearbyint(std::fabs(a[j]) / (1e-13 * amax)) : 0;
  std::vector<int> order(M);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (q[x] != q[y]) return q[x] > q[y];
    return x < y;
  });
  std::vector<int> sel(order.begin(), order.begin() + N.n_range);
  std::sort(sel.begin(), sel.end());
  for (int kk : sel) {
    f.k.push_back(kk);
    f.a.push_back(a[kk]);
    f.omega.push_back(kPi * kk / f.T);
  }
  *out = std::move(f);
  return BF_OK;
}

}  // namespace bf
