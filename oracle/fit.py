"""FP64 reference fit of the two kernel expansions (TEST INFRASTRUCTURE ONLY).

This package is the oracle that the GPU library is checked against.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it; the
library never does, and the two share no code.

It computes, in double precision and straight from the paper's definitions:

* the Haar expansion of the truncated spatial kernel (Sec. III-C, Eqs.
  Haar_scaling / Haar_mother / Haar_set, Haar_decomposition and the 2-D
  coefficients of Eq. Haar_2D_coefficients), its best N-term selection
  (Sec. III-A, Eq. N_term; Sec. IV-B, Eq. Haar_N_terms) and the box form of
  each selected 2-D Haar function (App. A, Table VI);
* for a kernel that is not separable (the radial exponential), the same 2-D
  coefficients from numerical integrals of K_s over the finest Haar cells;
* tabulated kernels (the method takes arbitrary kernels, Secs. I, IV-B and VI):
  a spatial table of weights on the integer offsets, taken as constant on the
  unit square around each offset, whose cell integrals are exact overlap sums;
  a range table of samples on a uniform grid, taken as linear between samples
  and zero past the last, whose cosine coefficients are exact integrals of each
  linear piece;
* the truncated-cosine expansion of the range kernel (Sec. III-B, Eq.
  1D_truncated_cos; Sec. IV-C, Eq. trigonometric_N_terms) with its best N-term
  selection out of the first 20N coefficients (App. B, Table VII).

Readings where the paper is silent or ambiguous (each is listed in the design doc):

* truncation: T_s = r + 1/2 for a window radius r, so that no integer offset
  falls on +-T_s; T = max(T_r, span) for the range series, so the range box of
  Eq. 1D_N_terms is identically one on every intensity difference;
* N_s counts Haar *level groups* (lx, ly): all functions phi or psi_{j,.} of
  one level in x times all of one level in y; groups are ranked by L2 energy;
* range coefficients are ranked by raw |a_k| (this reproduces Table VII),
  a_0 included in the candidate pool;
* Haar functions are point-sampled at integer offsets on half-open intervals
  [lo, hi); coefficients are the continuous integrals;
* ties: energies rounded to 12 significant digits, then smaller lx+ly, then
  smaller lx (phi counts as -1); |a_k| rounded to 1e-13 * max|a|, then smaller k.
"""
import math

import numpy as np

PHI = -1  # level index used for the scaling function phi


# ----------------------------------------------------------------------------
# Gaussian kernels (Sec. I: G_sigma(x) = exp(-x^2 / 2 sigma^2))
# ----------------------------------------------------------------------------
def gaussian(x, sigma):
    x = np.asarray(x, dtype=np.float64)
    return np.exp(-x * x / (2.0 * sigma * sigma))


def gaussian_integral(a, b, sigma):
    """Integral of exp(-t^2 / 2 sigma^2) over [a, b] (closed form with erf)."""
    s = sigma * math.sqrt(2.0)
    return sigma * math.sqrt(math.pi / 2.0) * (math.erf(b / s) - math.erf(a / s))


def truncation_radius(sigma, eps=0.01, kind="gaussian"):
    """T = K^{-1}(eps) (Sec. IV-A): sigma sqrt(2 ln(1/eps)) for the Gaussian,
    sigma ln(1/eps) for the exponential exp(-|x| / sigma)."""
    if kind == "exponential":
        return sigma * math.log(1.0 / eps)
    return sigma * math.sqrt(2.0 * math.log(1.0 / eps))


# ----------------------------------------------------------------------------
# Other kernels (the method takes arbitrary kernels, Secs. I, IV-B and VI): the
# exponential exp(-|x| / sigma) in range and the radially symmetric, not
# separable exp(-||(x, y)|| / sigma) in space.
# ----------------------------------------------------------------------------
KINDS = ("gaussian", "exponential")


def range_kernel(kind, sigma):
    if kind == "gaussian":
        return lambda t: gaussian(t, sigma)
    if kind == "exponential":
        return lambda t: np.exp(-np.abs(np.asarray(t, dtype=np.float64)) / sigma)
    raise ValueError(kind)


def spatial_kernel_2d(kind, sigma):
    """K_s(x, y) as a function of the offset (vectorised)."""
    if kind == "gaussian":
        return lambda x, y: np.exp(-(x * x + y * y) / (2.0 * sigma * sigma))
    if kind == "exponential":
        return lambda x, y: np.exp(-np.sqrt(x * x + y * y) / sigma)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# 1-D Haar functions on [-T, T) (Sec. III-C, Eqs. Haar_scaling, Haar_mother,
# Haar_set; support intervals as in App. A)
# ----------------------------------------------------------------------------
class Haar1D:
    """One 1-D Haar function: +1 on [lo, mid), -1 on [mid, hi); phi is +1 on [lo, hi)."""

    __slots__ = ("level", "k", "lo", "mid", "hi")

    def __init__(self, level, k, lo, mid, hi):
        self.level, self.k, self.lo, self.mid, self.hi = level, k, lo, mid, hi

    def intervals(self):
        """[(lo, hi, sign)] pieces on which the function is constant and nonzero."""
        if self.level == PHI:
            return [(self.lo, self.hi, 1.0)]
        return [(self.lo, self.mid, 1.0), (self.mid, self.hi, -1.0)]

    def sample(self, d):
        """Point samples at (integer) offsets d, half-open intervals."""
        d = np.asarray(d, dtype=np.float64)
        out = np.zeros(d.shape)
        for lo, hi, s in self.intervals():
            out += s * ((d >= lo) & (d < hi))
        return out

    def norm2(self):
        """Squared L2 norm: support width (phi: 2T; psi_{j,k}: 2T / 2^j)."""
        return self.hi - self.lo

    def __repr__(self):
        name = "phi" if self.level == PHI else "psi_%d,%d" % (self.level, self.k)
        return "%s[%g,%s,%g)" % (name, self.lo, "" if self.mid is None else "%g" % self.mid, self.hi)


def haar_family(T, J):
    """phi, psi_{0,0} and psi_{j,k}, j = 1..J, k in {+-1, ..., +-2^{j-1}}.

    psi_{j,k}(x) = psi_{0,0}(2^j x - Z_k) with Z_k = sign(k)(2|k|-1) T, so psi_{j,k}
    is +1 on [2^-j (Z_k - T), 2^-j Z_k) and -1 on [2^-j Z_k, 2^-j (Z_k + T))."""
    fam = [Haar1D(PHI, 0, -T, None, T), Haar1D(0, 0, -T, 0.0, T)]
    for j in range(1, J + 1):
        ks = list(range(-2 ** (j - 1), 0)) + list(range(1, 2 ** (j - 1) + 1))
        for k in ks:
            Z = math.copysign(2 * abs(k) - 1, k) * T
            s = 2.0 ** (-j)
            fam.append(Haar1D(j, k, s * (Z - T), s * Z, s * (Z + T)))
    return fam


def haar_coefficient(f, sigma, T):
    """Coefficient of Eq. Haar_decomposition for the Gaussian g = G_sigma:
    c_0 = (1/2T) int g phi, c_{jk} = (2^j / 2T) int g psi_{j,k}."""
    if f.level == PHI:
        return gaussian_integral(f.lo, f.hi, sigma) / (2.0 * T)
    return (2.0 ** f.level) * (gaussian_integral(f.lo, f.mid, sigma)
                               - gaussian_integral(f.mid, f.hi, sigma)) / (2.0 * T)


def max_level(T):
    """Finest level J such that a half-cell T / 2^J is at least one pixel wide."""
    return int(math.floor(math.log2(T)))


# ----------------------------------------------------------------------------
# Spatial fit: best N-term over 2-D Haar level groups (Eq. Haar_N_terms)
# ----------------------------------------------------------------------------
class SpatialFit:
    pass


def _round_sig(x, digits=12):
    if x == 0.0:
        return 0.0
    return float("%.*e" % (digits - 1, x))


def spatial_fit(sigma_s, radius, n_spatial):
    """Best N_s-group Haar approximation of the Gaussian K_s(||x||) = g(x) g(y) on
    [-T_s, T_s)^2, T_s = radius + 1/2.  The 2-D coefficients are products of 1-D
    ones (Eq. Haar_2D_coefficients for a separable kernel)."""
    T = radius + 0.5
    J = max_level(T)
    fam = haar_family(T, J)
    coef = [haar_coefficient(f, sigma_s, T) for f in fam]
    levels = [PHI] + list(range(0, J + 1))
    # per-level 1-D energy sum c_b^2 ||b||^2; a group's energy is the product
    e1 = {l: 0.0 for l in levels}
    for f, c in zip(fam, coef):
        e1[f.level] += c * c * f.norm2()
    groups = []
    for lx in levels:
        for ly in levels:
            groups.append((_round_sig(e1[lx] * e1[ly]), lx, ly))
    n_groups = len(groups)
    if not (1 <= n_spatial <= n_groups):
        raise ValueError("n_spatial must be in [1, %d]" % n_groups)
    groups.sort(key=lambda g: (-g[0], g[1] + g[2], g[1]))
    sel = [(lx, ly) for _, lx, ly in groups[:n_spatial]]

    d = np.arange(-radius, radius + 1)
    u = {}
    for l in levels:
        u[l] = sum(c * f.sample(d) for f, c in zip(fam, coef) if f.level == l)
    K = np.zeros((2 * radius + 1, 2 * radius + 1))  # K[dy + r, dx + r]
    for lx, ly in sel:
        K += np.outer(u[ly], u[lx])

    out = SpatialFit()
    out.sigma, out.radius, out.T, out.J = sigma_s, radius, T, J
    out.family, out.coef = fam, coef
    out.level_energy = e1
    out.groups_ranked = groups
    out.selected = sel
    out.u = u
    out.K = K
    return out


def _square_integral(kernel2d, x0, y0, h, sub, x, w):
    """Tensor Gauss-Legendre over [x0, x0 + h) x [y0, y0 + h), sub x sub panels."""
    e = np.linspace(0.0, h, sub + 1)
    lo, hi = e[:-1, None], e[1:, None]
    t = (0.5 * (hi - lo) * x[None, :] + 0.5 * (hi + lo)).ravel()
    wt = (0.5 * (hi - lo) * w[None, :]).ravel()
    return wt @ kernel2d((x0 + t)[None, :], (y0 + t)[:, None]) @ wt


def cell_integrals(kernel2d, T, n_cells, sub=4, nodes=12, grading=24):
    """M[j, i] = integral of K(x, y) over the finest cell (x in cell i, y in
    cell j) of the grid of n_cells equal cells on [-T, T) per axis, by
    composite tensor Gauss-Legendre (sub x sub panels of nodes^2 points per
    cell).  The offset origin is a corner of four cells, and there radial
    kernels have their only non-smooth point: those cells are split toward the
    origin into squares of halving size (each L-shaped ring as three squares
    that keep their distance from the corner), the last tiny corner square
    taken as its area times K at its centre."""
    x, w = np.polynomial.legendre.leggauss(nodes)
    h = 2.0 * T / n_cells
    edges = -T + h * np.arange(n_cells)
    M = np.empty((n_cells, n_cells))
    for j in range(n_cells):
        for i in range(n_cells):
            x0, y0 = edges[i], edges[j]
            sx = 1.0 if abs(x0) < 1e-9 * h else (-1.0 if abs(x0 + h) < 1e-9 * h else 0.0)
            sy = 1.0 if abs(y0) < 1e-9 * h else (-1.0 if abs(y0 + h) < 1e-9 * h else 0.0)
            if sx == 0.0 or sy == 0.0:
                M[j, i] = _square_integral(kernel2d, x0, y0, h, sub, x, w)
                continue
            # mirror onto the quadrant cell [0, h)^2 with its corner at the origin
            k = lambda X, Y: kernel2d(sx * X, sy * Y)
            total, s = 0.0, h
            for _ in range(grading):
                q = 0.5 * s
                total += (_square_integral(k, q, 0.0, q, 1, x, w) + _square_integral(k, 0.0, q, q, 1, x, w)
                          + _square_integral(k, q, q, q, 1, x, w))
                s = q
            total += s * s * float(k(np.array(0.5 * s), np.array(0.5 * s)))
            M[j, i] = total
    return M


def tabulated_cell_integrals(table, n_cells):
    """Cell integrals (as cell_integrals) of the tabulated spatial kernel: the
    weight table[dy + r, dx + r] on the unit square [dx - 1/2, dx + 1/2) x
    [dy - 1/2, dy + 1/2) around each integer offset, zero outside [-T, T)^2
    with T = r + 1/2.  A cell's integral is the sum of the weights times the
    areas of overlap, A_y table A_x^T with A[i, d] the length of cell i's
    interval inside offset d's."""
    table = np.asarray(table, dtype=np.float64)
    radius = (table.shape[0] - 1) // 2
    T = radius + 0.5
    h = 2.0 * T / n_cells
    lo = -T + h * np.arange(n_cells)
    d = np.arange(-radius, radius + 1)
    A = np.clip(np.minimum(lo[:, None] + h, d[None, :] + 0.5) - np.maximum(lo[:, None], d[None, :] - 0.5),
                0.0, None)
    return A @ table @ A.T


def spatial_fit_2d(kernel2d, radius, n_spatial, cells=None):
    """Best N_s-group Haar approximation of an arbitrary K_s on
    [-T_s, T_s)^2 (Eq. Haar_2D_coefficients without separability): every 2-D
    coefficient c_ab = <K, h_a(x) h_b(y)> / (||h_a||^2 ||h_b||^2) is a signed sum
    of integrals of K over the finest cells (every Haar function up to level J
    is constant on them).  cells: a function of the cell count giving those
    integrals (default: quadrature of kernel2d)."""
    T = radius + 0.5
    J = max_level(T)
    fam = haar_family(T, J)
    n_cells = 2 ** (J + 1)
    M = cell_integrals(kernel2d, T, n_cells) if cells is None else cells(n_cells)
    centers = -T + (2.0 * T / n_cells) * (np.arange(n_cells) + 0.5)
    Hm = np.array([f.sample(centers) for f in fam])        # functions x cells, +-1 / 0
    norms = np.array([f.norm2() for f in fam])
    C = (Hm @ M @ Hm.T) / np.outer(norms, norms)           # C[b, a]: h_b in y, h_a in x
    levels = [PHI] + list(range(0, J + 1))
    lev = np.array([f.level for f in fam])
    energy = {}
    for lx in levels:
        for ly in levels:
            sb, sa = lev == ly, lev == lx
            energy[lx, ly] = float(((C[np.ix_(sb, sa)] ** 2) * np.outer(norms[sb], norms[sa])).sum())
    # groups whose coefficients vanish by symmetry hold only quadrature noise:
    # below 1e-12 of the largest energy they count as zero (ties then fall to
    # the level rule, as for the closed-form separable coefficients)
    floor = 1e-12 * max(energy.values())
    groups = [(_round_sig(e) if e > floor else 0.0, lx, ly) for (lx, ly), e in energy.items()]
    if not (1 <= n_spatial <= len(groups)):
        raise ValueError("n_spatial must be in [1, %d]" % len(groups))
    groups.sort(key=lambda g: (-g[0], g[1] + g[2], g[1]))
    sel = [(lx, ly) for _, lx, ly in groups[:n_spatial]]
    d = np.arange(-radius, radius + 1)
    S = np.array([f.sample(d) for f in fam])               # functions x offsets
    K = np.zeros((2 * radius + 1, 2 * radius + 1))
    for lx, ly in sel:
        sb, sa = lev == ly, lev == lx
        K += S[sb].T @ C[np.ix_(sb, sa)] @ S[sa]
    out = SpatialFit()
    out.sigma, out.radius, out.T, out.J = None, radius, T, J
    out.family, out.coef2 = fam, C
    out.cells = M
    out.groups_ranked = groups
    out.selected = sel
    out.K = K
    return out


def spatial_fit_table(table, n_spatial):
    """spatial_fit_2d of a tabulated K_s, (2r + 1) x (2r + 1) weights indexed
    [dy + r, dx + r]; the table must be even in dy and in dx."""
    table = np.asarray(table, dtype=np.float64)
    K = table.shape[0]
    if table.ndim != 2 or table.shape[1] != K or K % 2 != 1 or K < 3:
        raise ValueError("spatial table must be (2r + 1) x (2r + 1), r >= 1")
    if not (np.array_equal(table, table[::-1, :]) and np.array_equal(table, table[:, ::-1])):
        raise ValueError("spatial table must be even in dy and in dx")
    return spatial_fit_2d(None, (K - 1) // 2, n_spatial, cells=lambda n: tabulated_cell_integrals(table, n))


def spatial_rectangles(fit):
    """The selected expansion written as weighted rectangles in offset space
    (App. A: phi*psi = B1 - B2, psi*psi = B1 - B2 + B3 - B4; Eq. 2D_box_N_terms).

    Returns an array of rows (ey_lo, ey_hi, ex_lo, ex_hi, w): K~_s(e) is the sum of
    w over rectangles with ey_lo <= e_y <= ey_hi and ex_lo <= e_x <= ex_hi
    (integer offsets, inclusive; the half-open real interval [lo, hi) holds the
    integers ceil(lo) .. ceil(hi) - 1)."""
    rows = []
    by_level = {}
    C = getattr(fit, "coef2", None)
    for i, f in enumerate(fit.family):
        by_level.setdefault(f.level, []).append((i, f))
    for lx, ly in fit.selected:
        for ia, fx in by_level[lx]:
            for ib, fy in by_level[ly]:
                # separable kernels: product of 1-D coefficients; otherwise the 2-D one
                w = fit.coef[ia] * fit.coef[ib] if C is None else C[ib, ia]
                if w == 0.0:
                    continue
                for xlo, xhi, sx in fx.intervals():
                    for ylo, yhi, sy in fy.intervals():
                        rows.append((math.ceil(ylo), math.ceil(yhi) - 1,
                                     math.ceil(xlo), math.ceil(xhi) - 1, w * sx * sy))
    return np.array(rows, dtype=np.float64).reshape(-1, 5)


# ----------------------------------------------------------------------------
# Range fit: truncated cosine series (Eq. 1D_truncated_cos, Eq.
# trigonometric_N_terms) with the candidate pool of App. B
# ----------------------------------------------------------------------------
class RangeFit:
    pass


def _gauss_legendre_panels(a, b, panels, nodes=16):
    x, w = np.polynomial.legendre.leggauss(nodes)
    edges = np.linspace(a, b, panels + 1)
    lo, hi = edges[:-1, None], edges[1:, None]
    t = (0.5 * (hi - lo) * x[None, :] + 0.5 * (hi + lo)).ravel()
    wt = (0.5 * (hi - lo) * w[None, :]).ravel()
    return t, wt


def cosine_coefficients(kernel, T, M):
    """a_0 = (1/2T) int_{-T}^{T} f, a_j = (1/T) int_{-T}^{T} f(x) cos(pi j x / T) dx,
    j < M, by composite 16-point Gauss-Legendre quadrature (4 panels per period
    of the highest frequency, at least 256)."""
    panels = max(256, 4 * M)
    t, wt = _gauss_legendre_panels(-T, T, panels)
    fw = kernel(t) * wt
    a = np.empty(M)
    for j0 in range(0, M, 64):
        js = np.arange(j0, min(M, j0 + 64))
        a[js] = np.cos(np.pi * js[:, None] * t[None, :] / T) @ fw / T
    a[0] *= 0.5
    return a


def select_largest(a, n):
    """Indices of the n largest |a_k| (ties broken toward smaller k after rounding
    |a_k| to an absolute grid of 1e-13 * max|a|), returned in increasing k."""
    mag = np.abs(a)
    q = np.rint(mag / (1e-13 * mag.max())) if mag.max() > 0 else mag
    order = sorted(range(len(a)), key=lambda k: (-q[k], k))
    return sorted(order[:n])


def range_fit(sigma_r, n_range, eps=0.01, span=1.0, kernel=None):
    """Best N_r-term cosine approximation of K_r on [-T, T], T = max(T_r, span).

    The approximated function on [-T, T] is K_r itself (untruncated there); with
    span = 0 this is the paper's own regime T = T_r.  Returns the selected
    (k, a_k, omega_k = pi k / T)."""
    if not (1 <= n_range <= 64):
        raise ValueError("n_range must be in [1, 64]")
    kind = "gaussian"
    if kernel is None:
        kernel = lambda t: gaussian(t, sigma_r)
    elif isinstance(kernel, str):
        kind, kernel = kernel, range_kernel(kernel, sigma_r)
    T_r = truncation_radius(sigma_r, eps, kind)
    T = max(T_r, span)
    M = max(20 * n_range, 2)
    a = cosine_coefficients(kernel, T, M)
    ks = select_largest(a, n_range)
    out = RangeFit()
    out.sigma, out.T_r, out.T, out.M = sigma_r, T_r, T, M
    out.a_all = a
    out.k = np.array(ks, dtype=np.int64)
    out.a = a[ks]
    out.omega = np.pi * out.k / T
    return out


def piecewise_linear_cosine_coefficients(values, step, T, M):
    """a_j (as cosine_coefficients) of the even function equal on [0, T] to the
    linear interpolant of values[i] at t_i = i step and to zero past the last
    sample (which must lie in [0, T]).  Exact per linear piece: with
    f(t) = v0 + beta (t - t0) on [t0, t1],
        int f(t) cos(w t) dt = [f(t) sin(w t) / w + beta cos(w t) / w^2]_{t0}^{t1},
    the cosine difference written as -2 sin(w (t0 + t1) / 2) sin(w (t1 - t0) / 2)."""
    v = np.asarray(values, dtype=np.float64)
    n = len(v)
    t0 = step * np.arange(n - 1)
    t1 = step * np.arange(1, n)
    v0, v1 = v[:-1], v[1:]
    beta = (v1 - v0) / (t1 - t0)
    a = np.empty(M)
    a[0] = float(np.sum(0.5 * (v0 + v1) * (t1 - t0))) / T          # (1 / 2T) int_{-T}^{T} f
    for j in range(1, M):
        w = math.pi * j / T
        seg = ((v1 * np.sin(w * t1) - v0 * np.sin(w * t0)) / w
               - 2.0 * beta * np.sin(0.5 * w * (t0 + t1)) * np.sin(0.5 * w * (t1 - t0)) / (w * w))
        a[j] = 2.0 * float(np.sum(seg)) / T                         # (1 / T) int_{-T}^{T} f cos
    return a


def range_fit_table(values, step, n_range, span=1.0):
    """range_fit of a tabulated K_r: samples values[i] = K_r(i step), linear
    between samples, zero past T_r = (n - 1) step; T = max(T_r, span)."""
    v = np.asarray(values, dtype=np.float64)
    if not (1 <= n_range <= 64):
        raise ValueError("n_range must be in [1, 64]")
    if v.ndim != 1 or len(v) < 2 or not step > 0:
        raise ValueError("range table needs >= 2 samples and a positive step")
    T_r = (len(v) - 1) * step
    T = max(T_r, span)
    M = max(20 * n_range, 2)
    a = piecewise_linear_cosine_coefficients(v, step, T, M)
    ks = select_largest(a, n_range)
    out = RangeFit()
    out.sigma, out.T_r, out.T, out.M = None, T_r, T, M
    out.a_all = a
    out.k = np.array(ks, dtype=np.int64)
    out.a = a[ks]
    out.omega = np.pi * out.k / T
    return out


def range_kernel_approx(fit, t):
    t = np.asarray(t, dtype=np.float64)
    return sum(a * np.cos(w * t) for a, w in zip(fit.a, fit.omega))


def first_m_containing(a, n):
    """Table VII's M(N): the smallest M such that the first M coefficients hold the
    N largest ones (raw-magnitude ranking)."""
    return max(select_largest(a, n)) + 1
