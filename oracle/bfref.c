/*
 * FP64 CPU oracle for the bilateral filter (TEST INFRASTRUCTURE ONLY).
 *
 * Plain, slow loops in double precision.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg load this library; the GPU library never
 * does, and the two share no code or headers.
 *
 *   T1  ref_true_bf        Eq. BF with Gaussian K_s on the square window
 *                          [-r, r]^2 and Gaussian K_r (the filter being
 *                          approximated).
 *   T2  ref_expanded_brute Eq. BF with both kernels replaced by their N-term
 *                          expansions, summed pixel by pixel.
 *   T3  ref_expanded_box   the same quantity through the shift identity of the
 *                          cosine terms (Eq. 1D_N_terms; the range box is
 *                          identically one because the series interval covers
 *                          every intensity difference) and 2-D box sums read
 *                          from FP64 summed-area tables (Eqs. sum_sat_2D,
 *                          sum_sat_recurrence_2D, sum_sat_sum_region_2D) over
 *                          the rectangles of the Haar box representation
 *                          (App. A, Eq. 2D_box_N_terms).
 *
 *   T4  ref_expanded_rangebox  the paper's own regime for 8-bit images:
 *                          the range series on [-T_r, T_r] times the range box
 *                          (Eq. trigonometric_N_terms with its box factor,
 *                          Eq. 1D_box_N_terms), summed pixel by pixel; the box
 *                          keeps q when |Z(p) - Z(q)| <= 255 T_r in levels.
 *
 * Conventions shared by all of them: the weight of source pixel q for output p
 * is K_s(p - q) K_r(I(p) - I(q)); only in-image q contribute (borders);
 * out = num / den when den > den_floor, else out = I(p).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Kernels: kind 0 Gaussian exp(-x^2 / 2 sigma^2); kind 1 exponential
 * exp(-|x| / sigma), radial in space (exp(-||d|| / sigma), not separable). */
static inline double ks_weight(int kind, double d2, double sigma) {
  return kind == 1 ? exp(-sqrt(d2) / sigma) : exp(-d2 / (2.0 * sigma * sigma));
}
static inline double kr_weight(int kind, double t, double sigma) {
  return kind == 1 ? exp(-fabs(t) / sigma) : exp(-t * t / (2.0 * sigma * sigma));
}

/* T1: true bilateral filter at the listed pixels (all pixels if ys == NULL). */
void ref_true_bf(const double *I, int H, int W, int r, double sigma_s, double sigma_r, int kind_s,
                 int kind_r, const int *ys, const int *xs, long npix, double den_floor, double *out) {
  long n = ys ? npix : (long)H * W;
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < n; ++i) {
    int py = ys ? ys[i] : (int)(i / W), px = ys ? xs[i] : (int)(i % W);
    double Ip = I[(long)py * W + px], num = 0.0, den = 0.0;
    for (int dy = -r; dy <= r; ++dy) {
      int qy = py - dy;
      if (qy < 0 || qy >= H) continue;
      for (int dx = -r; dx <= r; ++dx) {
        int qx = px - dx;
        if (qx < 0 || qx >= W) continue;
        double Iq = I[(long)qy * W + qx], t = Ip - Iq;
        double w = ks_weight(kind_s, (double)(dx * dx + dy * dy), sigma_s) * kr_weight(kind_r, t, sigma_r);
        num += w * Iq;
        den += w;
      }
    }
    out[i] = den > den_floor ? num / den : Ip;
  }
}

/* T1 with tabulated kernels: ks holds (2r+1)^2 spatial weights,
 * ks[(dy + r)(2r+1) + dx + r]; the range weight of a difference t is the
 * linear interpolant of kr[i] at |t| = i step, zero past (n - 1) step. */
static inline double kr_table(const double *kr, int n, double step, double t) {
  const double u = fabs(t) / step;
  if (u > (double)(n - 1)) return 0.0;
  int i = (int)floor(u);
  if (i >= n - 1) return kr[n - 1];
  return kr[i] + (u - i) * (kr[i + 1] - kr[i]);
}

void ref_true_bf_tab(const double *I, int H, int W, int r, const double *ks, const double *kr, int kr_n,
                     double kr_step, const int *ys, const int *xs, long npix, double den_floor, double *out) {
  long n = ys ? npix : (long)H * W;
  const int K = 2 * r + 1;
#pragma omp parallel for schedule(dynamic, 64)
  for (long i = 0; i < n; ++i) {
    int py = ys ? ys[i] : (int)(i / W), px = ys ? xs[i] : (int)(i % W);
    double Ip = I[(long)py * W + px], num = 0.0, den = 0.0;
    for (int dy = -r; dy <= r; ++dy) {
      int qy = py - dy;
      if (qy < 0 || qy >= H) continue;
      for (int dx = -r; dx <= r; ++dx) {
        int qx = px - dx;
        if (qx < 0 || qx >= W) continue;
        double Iq = I[(long)qy * W + qx];
        double w = ks[(dy + r) * K + dx + r] * kr_table(kr, kr_n, kr_step, Ip - Iq);
        num += w * Iq;
        den += w;
      }
    }
    out[i] = den > den_floor ? num / den : Ip;
  }
}

/* T2: expanded form by brute force.  Ks is the (2r+1)^2 sampled spatial
 * expansion, Ks[(dy + r)(2r+1) + dx + r] = K~_s(dy, dx); the range expansion is
 * K~_r(t) = sum_k a[k] cos(omega[k] t).  num/den may be NULL. */
void ref_expanded_brute(const double *I, int H, int W, int r, const double *Ks, int nterms,
                        const double *a, const double *omega, const int *ys, const int *xs,
                        long npix, double den_floor, double *out, double *num_out,
                        double *den_out) {
  const int ks = 2 * r + 1;
  long n = ys ? npix : (long)H * W;
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < n; ++i) {
    int py = ys ? ys[i] : (int)(i / W), px = ys ? xs[i] : (int)(i % W);
    double Ip = I[(long)py * W + px], num = 0.0, den = 0.0;
    for (int dy = -r; dy <= r; ++dy) {
      int qy = py - dy;
      if (qy < 0 || qy >= H) continue;
      for (int dx = -r; dx <= r; ++dx) {
        int qx = px - dx;
        if (qx < 0 || qx >= W) continue;
        double ws = Ks[(dy + r) * ks + (dx + r)];
        if (ws == 0.0) continue;
        double Iq = I[(long)qy * W + qx], t = Ip - Iq, kr = 0.0;
        for (int k = 0; k < nterms; ++k) kr += a[k] * cos(omega[k] * t);
        num += ws * kr * Iq;
        den += ws * kr;
      }
    }
    out[i] = den > den_floor ? num / den : Ip;
    if (num_out) num_out[i] = num;
    if (den_out) den_out[i] = den;
  }
}

/* Exclusive FP64 summed-area table: S[(y)(W+1) + x] = sum_{y'<y, x'<x} g. */
static void sat_fp64(const double *g, int H, int W, double *S) {
  for (int x = 0; x <= W; ++x) S[x] = 0.0;
  for (int y = 1; y <= H; ++y) {
    double run = 0.0;  /* c(x, y): running sum along the row */
    S[(long)y * (W + 1)] = 0.0;
    for (int x = 1; x <= W; ++x) {
      run += g[(long)(y - 1) * W + (x - 1)];
      S[(long)y * (W + 1) + x] = S[(long)(y - 1) * (W + 1) + x] + run;
    }
  }
}

/* Sum of g over rows [y0, y1] x cols [x0, x1] (inclusive, clipped to the image). */
static inline double box_sum(const double *S, int H, int W, int y0, int y1, int x0, int x1) {
  y0 = clampi(y0, 0, H);
  x0 = clampi(x0, 0, W);
  y1 = clampi(y1 + 1, 0, H);
  x1 = clampi(x1 + 1, 0, W);
  if (y1 <= y0 || x1 <= x0) return 0.0;
  const long w1 = W + 1;
  return S[(long)y1 * w1 + x1] - S[(long)y0 * w1 + x1] - S[(long)y1 * w1 + x0] +
         S[(long)y0 * w1 + x0];
}

/* corr(p) = sum_q K~_s(p - q) g(q), K~_s = sum over rectangles of w on offsets
 * e = p - q with ey in [rect0, rect1], ex in [rect2, rect3]. */
static void correlate_rects(const double *S, int H, int W, const double *rects, int nrect,
                            double *corr) {
#pragma omp parallel for schedule(static)
  for (int py = 0; py < H; ++py) {
    for (int px = 0; px < W; ++px) {
      double acc = 0.0;
      for (int j = 0; j < nrect; ++j) {
        const double *R = rects + 5 * j;
        int ey0 = (int)R[0], ey1 = (int)R[1], ex0 = (int)R[2], ex1 = (int)R[3];
        acc += R[4] * box_sum(S, H, W, py - ey1, py - ey0, px - ex1, px - ex0);
      }
      corr[(long)py * W + px] = acc;
    }
  }
}

/* T3: shift-decomposed expanded form over the whole image. */
int ref_expanded_box(const double *I, int H, int W, const double *rects, int nrect, int nterms,
                     const double *a, const double *omega, double den_floor, double *out,
                     double *num_out, double *den_out) {
  const long n = (long)H * W;
  double *num = (double *)calloc(n, sizeof(double)), *den = (double *)calloc(n, sizeof(double));
  double *g = (double *)malloc(n * sizeof(double)), *c = (double *)malloc(n * sizeof(double));
  double *s = (double *)malloc(n * sizeof(double)), *corr = (double *)malloc(n * sizeof(double));
  double *S = (double *)malloc((long)(H + 1) * (W + 1) * sizeof(double));
  if (!num || !den || !g || !c || !s || !corr || !S) {
    free(num); free(den); free(g); free(c); free(s); free(corr); free(S);
    return -1;
  }
  for (int k = 0; k < nterms; ++k) {
    for (long i = 0; i < n; ++i) {
      c[i] = cos(omega[k] * I[i]);
      s[i] = sin(omega[k] * I[i]);
    }
    /* numerator: a_k [C(p) (K ⋆ C I)(p) + S(p) (K ⋆ S I)(p)] */
    for (int part = 0; part < 4; ++part) {
      const double *mod = (part == 0 || part == 2) ? c : s;
      for (long i = 0; i < n; ++i) g[i] = part < 2 ? mod[i] * I[i] : mod[i];
      sat_fp64(g, H, W, S);
      correlate_rects(S, H, W, rects, nrect, corr);
      double *acc = part < 2 ? num : den;
      for (long i = 0; i < n; ++i) acc[i] += a[k] * mod[i] * corr[i];
    }
  }
  for (long i = 0; i < n; ++i) {
    out[i] = den[i] > den_floor ? num[i] / den[i] : I[i];
    if (num_out) num_out[i] = num[i];
    if (den_out) den_out[i] = den[i];
  }
  free(num); free(den); free(g); free(c); free(s); free(corr); free(S);
  return 0;
}

/* Box sums of one image for a list of rectangles, exported for tests. */
int ref_correlate_rects(const double *g, int H, int W, const double *rects, int nrect,
                        double *corr) {
  double *S = (double *)malloc((long)(H + 1) * (W + 1) * sizeof(double));
  if (!S) return -1;
  sat_fp64(g, H, W, S);
  correlate_rects(S, H, W, rects, nrect, corr);
  free(S);
  return 0;
}

/* T4: the expanded form with the range box, 8-bit levels Z (I = Z / 255).
 * zr = 255 T_r: source q counts for output p when |Z(p) - Z(q)| <= zr. */
void ref_expanded_rangebox(const uint8_t *Z, int H, int W, int r, const double *Ks, int nterms,
                           const double *a, const double *omega, double zr, const int *ys,
                           const int *xs, long npix, double den_floor, double *out,
                           double *num_out, double *den_out) {
  const int ks = 2 * r + 1;
  long n = ys ? npix : (long)H * W;
#pragma omp parallel for schedule(dynamic, 16)
  for (long i = 0; i < n; ++i) {
    int py = ys ? ys[i] : (int)(i / W), px = ys ? xs[i] : (int)(i % W);
    const int zp = Z[(long)py * W + px];
    double Ip = zp / 255.0, num = 0.0, den = 0.0;
    for (int dy = -r; dy <= r; ++dy) {
      int qy = py - dy;
      if (qy < 0 || qy >= H) continue;
      for (int dx = -r; dx <= r; ++dx) {
        int qx = px - dx;
        if (qx < 0 || qx >= W) continue;
        const int zq = Z[(long)qy * W + qx];
        if (fabs((double)(zp - zq)) > zr) continue; /* outside the range box */
        double ws = Ks[(dy + r) * ks + (dx + r)];
        if (ws == 0.0) continue;
        double Iq = zq / 255.0, t = Ip - Iq, kr = 0.0;
        for (int k = 0; k < nterms; ++k) kr += a[k] * cos(omega[k] * t);
        num += ws * kr * Iq;
        den += ws * kr;
      }
    }
    out[i] = den > den_floor ? num / den : Ip;
    if (num_out) num_out[i] = num;
    if (den_out) den_out[i] = den;
  }
}
