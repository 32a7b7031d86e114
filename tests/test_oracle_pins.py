"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: each compares it with a printed
value of the paper (Table VII, the Sec. V-A worked example), with an identity
the paper states (App. A box representation, Parseval for a best N-term
approximation, the cosine shift identity), with an independent numerical
route (adaptive quadrature, scipy's complex error function, scipy's 2-D
correlation, a pure-Python double loop) or with an invariant of Eq. BF
(constant images, sigma_r -> infinity, convergence as N grows).  The last
section plants mistakes in the oracle and checks that some pin fails.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, signal, special

import oracle
import synth
from oracle import fit as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return rows


# ---------------------------------------------------------------------------
# Range expansion (Sec. III-B, Eq. 1D_truncated_cos; App. B)
# ---------------------------------------------------------------------------
def test_table7_range_row():
    """App. B, Table VII: G_40 on [-T_r, T_r] (eps = 0.01) gives M(N) = 2,2,3,...,8
    under raw-magnitude ranking with a_0 in the pool."""
    rows = _golden("table7_range_row.txt")
    fit = F.range_fit(40.0, 8, eps=0.01, span=0.0)
    assert abs(fit.T - 40.0 * math.sqrt(2 * math.log(100.0))) < 1e-12
    for n, m in rows:
        assert F.first_m_containing(fit.a_all, int(n)) == int(m)


def _cos_coef_closed_form(sigma, T, k):
    """a_k of a Gaussian on [-T, T] through the complex error function:
    int_{-T}^{T} e^{-t^2/2s^2} cos(w t) dt = Re{ e^{-w^2 s^2/2} s sqrt(pi/2)
    [erf((T - i w s^2)/(s sqrt2)) - erf((-T - i w s^2)/(s sqrt2))] }."""
    w = math.pi * k / T
    z1 = (T - 1j * w * sigma * sigma) / (sigma * math.sqrt(2))
    z0 = (-T - 1j * w * sigma * sigma) / (sigma * math.sqrt(2))
    with np.errstate(all="ignore"):  # exp underflow times erf overflow at large k
        val = (math.exp(-0.5 * (w * sigma) ** 2) * sigma * math.sqrt(math.pi / 2)
               * (special.erf(z1) - special.erf(z0))).real
    return val / (2 * T) if k == 0 else val / T


@pytest.mark.parametrize("sigma,T", [(0.3, 1.0), (0.2, 1.0), (1.0, 3.0), (40.0, 121.39417)])
def test_cosine_coefficients_closed_form(sigma, T):
    a = F.cosine_coefficients(lambda t: F.gaussian(t, sigma), T, 40)
    checked = 0
    for k in range(0, 40):
        ref = _cos_coef_closed_form(sigma, T, k)
        if not np.isfinite(ref):
            continue
        checked += 1
        assert abs(a[k] - ref) < 1e-13, (k, a[k], ref)
    assert checked >= 10


@pytest.mark.parametrize("sigma", [0.05, 0.1])
def test_cosine_coefficients_wide_interval(sigma):
    """For T >> sigma the interval barely truncates the Gaussian, so
    a_k -> sigma sqrt(2 pi) / T exp(-(pi k sigma / T)^2 / 2) (its Fourier transform)."""
    T = 1.0
    a = F.cosine_coefficients(lambda t: F.gaussian(t, sigma), T, 200)
    k = np.arange(200)
    ref = sigma * math.sqrt(2 * math.pi) / T * np.exp(-0.5 * (math.pi * k * sigma / T) ** 2)
    ref[0] *= 0.5
    assert np.abs(a - ref).max() < 1e-13


def test_cosine_parseval_and_convergence():
    """||f||^2 = 2T a_0^2 + T sum a_k^2 on [-T, T]; the best-N error is ||f||^2 minus
    the kept energy (Sec. III-A), so it never grows with N."""
    sigma, T = 0.1, 1.0
    a = F.cosine_coefficients(lambda t: F.gaussian(t, sigma), T, 400)
    norm2 = integrate.quad(lambda t: math.exp(-t * t / sigma ** 2), -T, T, epsabs=1e-14)[0]
    energy = 2 * T * a[0] ** 2 + T * np.sum(a[1:] ** 2)
    assert abs(energy - norm2) < 1e-12
    t = np.linspace(-T, T, 4001)
    errs = []
    for n in (2, 4, 8, 16, 24):
        fit = F.range_fit(sigma, n)
        errs.append(np.sqrt(np.mean((F.range_kernel_approx(fit, t) - F.gaussian(t, sigma)) ** 2)))
    assert all(e1 >= e2 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-6


def test_range_selection_candidates_and_ties():
    """a_0 is a candidate (Table VII needs it); at sigma_r = 0.1, T = 1 the kept
    terms are k = 0..N-1; coefficients beyond the double-precision noise floor tie
    and the tie goes to smaller k."""
    for n in (8, 16, 32):
        fit = F.range_fit(0.1, n)
        assert fit.k.tolist() == list(range(n))
    assert F.select_largest(np.array([1.0, 0.5, 0.5, 1e-20, 0.0]), 3) == [0, 1, 2]
    assert F.select_largest(np.array([0.2, 1.0, 0.3]), 1) == [1]


# ---------------------------------------------------------------------------
# Spatial expansion (Sec. III-C, Eqs. Haar_scaling .. Haar_2D_coefficients)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sigma,T", [(1.0, 3.0), (3.0, 9.5), (16.0, 48.5)])
def test_haar_coefficients_by_quadrature(sigma, T):
    """c_0 = (1/2T) int g phi and c_jk = (2^j/2T) int g psi_jk against adaptive
    quadrature of the sampled function definitions."""
    fam = F.haar_family(T, F.max_level(T))
    for f in fam:
        c = F.haar_coefficient(f, sigma, T)
        val = 0.0
        for lo, hi, s in f.intervals():
            val += s * integrate.quad(lambda x: math.exp(-x * x / (2 * sigma * sigma)), lo, hi,
                                      epsabs=1e-15, epsrel=1e-13)[0]
        scale = 1.0 if f.level == F.PHI else 2.0 ** f.level
        assert abs(c - scale * val / (2 * T)) < 1e-13, f


def test_haar_family_shapes():
    """psi_{j,k}(x) = psi_00(2^j x - Z_k), Z_k = sign(k)(2|k|-1)T: check the supports
    against the paper's worked list for T = 2 (Fig. Haar_1D) and the orthogonality
    of the family on a fine grid."""
    T = 2.0
    fam = {(f.level, f.k): f for f in F.haar_family(T, 2)}
    x = np.linspace(-T, T, 64001)[:-1] + T / 64000
    psi00 = lambda u: np.where((u >= -T) & (u < 0), 1.0, 0.0) - np.where((u >= 0) & (u < T), 1.0, 0.0)
    shifts = {(1, -1): (2, -T), (1, 1): (2, T), (2, -1): (4, -T), (2, 1): (4, T),
              (2, -2): (4, -3 * T), (2, 2): (4, 3 * T)}
    for (j, k), (mul, z) in shifts.items():
        assert np.array_equal(fam[(j, k)].sample(x), psi00(mul * x - z)), (j, k)
    B = np.array([f.sample(x) for f in fam.values()])
    G = B @ B.T * (2 * T / len(x))
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-9)
    assert np.allclose(np.diag(G), [f.norm2() for f in fam.values()], atol=1e-9)


@pytest.mark.parametrize("sigma,T", [(1.0, 3.0), (5.0, 15.5)])
def test_haar_expansion_reproduces_cell_averages(sigma, T):
    """The Haar expansion through level J is the orthogonal projection onto
    functions constant on the 2^{J+1} cells of width T/2^J: its value on a cell
    is the cell average of g (independent quadrature)."""
    J = 3
    fam = F.haar_family(T, J)
    coef = [F.haar_coefficient(f, sigma, T) for f in fam]
    ncell = 2 ** (J + 1)
    w = 2 * T / ncell
    for i in range(ncell):
        lo = -T + i * w
        mid = lo + 0.5 * w
        approx = sum(c * f.sample(np.array([mid]))[0] for f, c in zip(fam, coef))
        avg = integrate.quad(lambda x: math.exp(-x * x / (2 * sigma * sigma)), lo, lo + w,
                             epsabs=1e-15)[0] / w
        assert abs(approx - avg) < 1e-12, (i, approx, avg)


def test_haar_parseval_levels():
    """Sum of level energies -> ||g||^2 on [-T, T] as J grows (Parseval), and the
    closed-form value of ||exp(-x^2/2)||^2 on [-3, 3] = sqrt(pi) erf(3)."""
    sigma, T = 1.0, 3.0
    norm2 = math.sqrt(math.pi) * math.erf(3.0)
    for J, tol in ((3, 0.02), (10, 1e-6)):
        fam = F.haar_family(T, J)
        e = sum(F.haar_coefficient(f, sigma, T) ** 2 * f.norm2() for f in fam)
        assert e <= norm2 + 1e-12
        assert norm2 - e < tol


def test_box_representation_app_a():
    """App. A: phi psi_{j,k} = B1 - B2 and psi psi = B1 - B2 + B3 - B4 with
    A1 = [2^-j (Z_k - T), 2^-j Z_k), A2 = [2^-j Z_k, 2^-j (Z_k + T)), pointwise on
    the integer grid; and the rectangle list reproduces the sampled kernel."""
    r = 12
    T = r + 0.5
    d = np.arange(-r, r + 1)
    for f in F.haar_family(T, F.max_level(T)):
        if f.level == F.PHI:
            continue
        Z = math.copysign(2 * abs(f.k) - 1, f.k) * T if f.level > 0 else 0.0
        s = 2.0 ** (-f.level)
        a1 = (d >= s * (Z - T)) & (d < s * Z)
        a2 = (d >= s * Z) & (d < s * (Z + T))
        assert np.array_equal(f.sample(d), a1.astype(float) - a2.astype(float))
    for ss, rr, ns in ((3.0, 9, 4), (8.0, 24, 6), (4.0, 12, 9)):
        fit = F.spatial_fit(ss, rr, ns)
        K = np.zeros_like(fit.K)
        for ey0, ey1, ex0, ex1, w in F.spatial_rectangles(fit):
            K[int(ey0) + rr:int(ey1) + rr + 1, int(ex0) + rr:int(ex1) + rr + 1] += w
        assert np.abs(K - fit.K).max() < 1e-15


def test_worked_example_three_boxes():
    """Sec. V-A: f1 + f2 + f3 (groups phi phi, phi psi_1, psi_1 phi: five Haar
    functions) equals three centred boxes 2T x 2T, 2T x T, T x 2T."""
    (n_haar, n_box, *dims), = _golden("worked_example_boxes.txt")
    r = 10
    T = r + 0.5
    fit = F.spatial_fit(3.0, r, 3)
    assert fit.selected == [(F.PHI, F.PHI), (F.PHI, 1), (1, F.PHI)]
    nfun = sum(1 for f in fit.family if f.level in (F.PHI, 1))
    assert nfun * 2 - 1 == n_haar  # phi shared by the three groups: 1 + 2 + 2
    d = np.arange(-r, r + 1)
    boxes = []
    for i in range(int(n_box)):
        h, w = dims[2 * i] * T, dims[2 * i + 1] * T
        by = (d >= -h / 2) & (d < h / 2)
        bx = (d >= -w / 2) & (d < w / 2)
        boxes.append(np.outer(by, bx).astype(float).ravel())
    A = np.array(boxes).T
    coef, *_ = np.linalg.lstsq(A, fit.K.ravel(), rcond=None)
    assert np.abs(A @ coef - fit.K.ravel()).max() < 1e-14


def test_spatial_groups_symmetric_and_energy_ordered():
    """Selected groups of the five workloads: symmetric kernels (Eq. BF asks for
    symmetric K_s), kernel L2 error non-increasing in N_s."""
    for ss, r in ((3.0, 9), (8.0, 24), (16.0, 48)):
        d = np.arange(-r, r + 1)
        G = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2 * ss * ss))
        prev = np.inf
        for ns in range(1, 10):
            K = F.spatial_fit(ss, r, ns).K
            if ns in (4, 6, 8):
                assert np.allclose(K, K.T, atol=1e-15) and np.allclose(K, K[::-1], atol=1e-15)
            err = np.sqrt(np.sum((K - G) ** 2))
            assert err <= prev + 1e-9
            prev = err


# ---------------------------------------------------------------------------
# The filters T1, T2, T3
# ---------------------------------------------------------------------------
def _py_true_bf(I, ss, r, sr):
    H, W = I.shape
    out = np.zeros_like(I)
    for py in range(H):
        for px in range(W):
            num = den = 0.0
            for qy in range(max(0, py - r), min(H, py + r + 1)):
                for qx in range(max(0, px - r), min(W, px + r + 1)):
                    w = math.exp(-((py - qy) ** 2 + (px - qx) ** 2) / (2 * ss * ss)) * \
                        math.exp(-(I[py, px] - I[qy, qx]) ** 2 / (2 * sr * sr))
                    num += w * I[qy, qx]
                    den += w
            out[py, px] = num / den
    return out


def _py_expanded(I, plan):
    """Eq. BF with both expansions, written as a plain quadruple loop; the spatial
    weight of q for output p is K~_s(p - q)."""
    H, W = I.shape
    r = plan.radius
    out = np.zeros_like(I)
    for py in range(H):
        for px in range(W):
            num = den = 0.0
            for qy in range(max(0, py - r), min(H, py + r + 1)):
                for qx in range(max(0, px - r), min(W, px + r + 1)):
                    ws = plan.Ks[py - qy + r, px - qx + r]
                    kr = sum(a * math.cos(w * (I[py, px] - I[qy, qx]))
                             for a, w in zip(plan.a, plan.omega))
                    num += ws * kr * I[qy, qx]
                    den += ws * kr
            out[py, px] = num / den
    return out


def test_true_bf_brute_force_tiny():
    I = synth.gen_image(7, 9, 2, 0.05, 11).astype(np.float64)
    ref = _py_true_bf(I, 1.5, 2, 0.2)
    assert np.abs(oracle.true_bf(I, 1.5, 2, 0.2) - ref).max() < 1e-14


def test_expanded_brute_force_tiny():
    I = synth.gen_image(8, 7, 2, 0.05, 12).astype(np.float64)
    plan = oracle.make_plan(1.5, 3, 4, 0.2, 8)
    ref = _py_expanded(I, plan)
    assert np.abs(oracle.expanded_brute(I, plan) - ref).max() < 1e-13
    assert np.abs(oracle.expanded_box(I, plan) - ref).max() < 1e-12


@pytest.mark.parametrize("H,W,ss,r,ns,sr,nr", [
    (40, 56, 2.0, 6, 4, 0.1, 16), (64, 64, 3.0, 9, 4, 0.1, 8), (33, 47, 4.0, 12, 6, 0.2, 8),
    (5, 60, 3.0, 9, 8, 0.05, 32), (60, 3, 2.0, 6, 5, 0.3, 8), (1, 1, 3.0, 9, 4, 0.1, 8),
    (9, 11, 8.0, 24, 6, 0.1, 16)])
def test_shift_identity_T2_equals_T3(H, W, ss, r, ns, sr, nr):
    """Eq. 1D_N_terms: the cosine shift identity plus box sums reach the expanded
    form exactly (up to rounding): T2 == T3 within 1e-12, incl. images smaller
    than the window and the 1 x 1 image."""
    I = synth.gen_image(H, W, 3, 0.03, H * 131 + W)
    plan = oracle.make_plan(ss, r, ns, sr, nr)
    o2, n2, d2 = oracle.expanded_brute(I, plan, return_parts=True)
    o3, n3, d3 = oracle.expanded_box(I, plan, return_parts=True)
    assert np.abs(o2 - o3).max() < 1e-12
    assert np.abs(n2 - n3).max() < 1e-10 * max(1.0, np.abs(n2).max())
    if H == W == 1:
        assert abs(o3[0, 0] - float(I[0, 0])) < 1e-12


def test_constant_image_is_unchanged():
    """Eq. BF is a weighted average: a constant image maps to itself (T1, T2, T3)."""
    Z = np.full((23, 31), 0.37)
    plan = oracle.make_plan(3.0, 9, 4, 0.1, 8)
    for out in (oracle.true_bf(Z, 3.0, 9, 0.1), oracle.expanded_brute(Z, plan),
                oracle.expanded_box(Z, plan)):
        assert np.abs(out - 0.37).max() < 1e-14


def test_sigma_r_infinity_is_spatial_filter():
    """sigma_r -> infinity: the range expansion is constant on every intensity
    difference in [-1, 1] and the filter is the normalised spatial filter
    (K~_s * I) / (K~_s * 1) (scipy)."""
    I = synth.gen_image(48, 40, 4, 0.02, 5).astype(np.float64)
    plan = oracle.make_plan(3.0, 9, 4, 1e6, 4)
    kr = F.range_kernel_approx(plan.range, np.linspace(-1.0, 1.0, 101))
    assert np.ptp(kr) < 1e-9 * abs(kr[50]) and abs(kr[50] - 1.0) < 1e-3
    K = plan.Ks[::-1, ::-1]  # correlate2d(x, K') = sum_q K'(q - p) x(q); K~_s(p - q) needs the flip
    num = signal.correlate2d(I, K, mode="same", boundary="fill")
    den = signal.correlate2d(np.ones_like(I), K, mode="same", boundary="fill")
    assert np.abs(oracle.expanded_box(I, plan) - num / den).max() < 1e-12


def test_correlation_orientation_asymmetric_kernel():
    """corr(p) = sum_q K(p - q) g(q) with an asymmetric rectangle kernel against
    scipy's 2-D convolution (which is exactly that sum)."""
    rng = np.random.default_rng(3)
    g = rng.standard_normal((21, 17))
    rects = np.array([[-3, 1, 0, 4, 0.7], [2, 3, -2, -1, -1.3], [0, 0, 0, 0, 0.25]])
    K = np.zeros((7, 9))  # offsets ey in [-3, 3], ex in [-4, 4]
    for ey0, ey1, ex0, ex1, w in rects:
        K[int(ey0) + 3:int(ey1) + 4, int(ex0) + 4:int(ex1) + 5] += w
    ref = signal.convolve2d(g, K, mode="same", boundary="fill")
    assert np.abs(oracle.correlate_rects(g, rects) - ref).max() < 1e-12


def test_expansion_converges_to_true_bf():
    """Error of the expanded filter against the true bilateral filter falls as the
    number of range terms grows (reported by the benchmark, asserted loosely)."""
    I = synth.gen_image(64, 64, 5, 0.02, 21)
    ref = oracle.true_bf(I, 3.0, 9, 0.1)
    errs = []
    for nr in (4, 8, 12, 16):
        plan = oracle.make_plan(3.0, 9, 6, 0.1, nr)
        errs.append(np.abs(oracle.expanded_box(I, plan) - ref).mean())
    assert errs[0] > errs[1] > errs[-1]


def test_uint8_input_is_scaled():
    Iu = synth.gen_image_u8(20, 24, 3, 0.02, 4)
    plan = oracle.make_plan(2.0, 6, 4, 0.1, 8)
    a = oracle.expanded_box(Iu, plan)
    b = oracle.expanded_box(Iu.astype(np.float64) / 255.0, plan)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Planted mistakes: each must make at least one pin above fail
# ---------------------------------------------------------------------------
def test_planted_mistakes_are_caught(monkeypatch):
    # (1) a_0 without its 1/2 factor: Table VII changes
    orig = F.cosine_coefficients

    def no_half(kernel, T, M):
        a = orig(kernel, T, M)
        a[0] *= 2.0
        return a
    monkeypatch.setattr(F, "cosine_coefficients", no_half)
    fit = F.range_fit(40.0, 8, eps=0.01, span=0.0)
    assert [F.first_m_containing(fit.a_all, n) for n in range(1, 9)] != [2, 2, 3, 4, 5, 6, 7, 8]
    monkeypatch.undo()

    # (2) psi coefficient without 2^j: cell averages no longer reproduced
    fam = F.haar_family(3.0, 3)
    bad = [F.gaussian_integral(f.lo, f.hi, 1.0) / 6.0 if f.level == F.PHI else
           (F.gaussian_integral(f.lo, f.mid, 1.0) - F.gaussian_integral(f.mid, f.hi, 1.0)) / 6.0
           for f in fam]
    mid = np.array([-3.0 + 0.75 * 0.5])
    approx = sum(c * f.sample(mid)[0] for f, c in zip(fam, bad))
    avg = integrate.quad(lambda x: math.exp(-x * x / 2), -3.0, -2.25)[0] / 0.75
    assert abs(approx - avg) > 1e-3

    # (3) a dropped sine term in the shift identity: T2 != T3
    I = synth.gen_image(20, 20, 3, 0.03, 8)
    plan = oracle.make_plan(2.0, 6, 4, 0.1, 8)
    t2 = oracle.expanded_brute(I, plan)
    cos_only = np.zeros_like(t2)
    num = den = 0.0
    Iu = I.astype(np.float64)
    num = np.zeros_like(Iu)
    den = np.zeros_like(Iu)
    for a, w in zip(plan.a, plan.omega):
        c = np.cos(w * Iu)
        num += a * c * oracle.correlate_rects(c * Iu, plan.rects)
        den += a * c * oracle.correlate_rects(c, plan.rects)
    cos_only = num / den
    assert np.abs(cos_only - t2).max() > 1e-3


# ---------------------------------------------------------------------------
# Other kernels: the exponential in range, the radial exponential in space
# (not separable; 2-D coefficients from integrals over the finest cells)
# ---------------------------------------------------------------------------
def _anisotropic(a, b):
    return lambda x, y: np.exp(-x * x / (2 * a * a) - y * y / (2 * b * b))


@pytest.mark.parametrize("ss,r,ns", [(3.0, 9, 4), (5.0, 15, 6), (2.0, 6, 9)])
def test_cell_fit_reproduces_separable_gaussian(ss, r, ns):
    """The generic 2-D cell path applied to the Gaussian must give the closed-form
    separable fit (products of erf-based 1-D coefficients)."""
    a = oracle.spatial_fit(ss, r, ns)
    b = oracle.spatial_fit_2d(oracle.spatial_kernel_2d("gaussian", ss), r, ns)
    assert a.selected == b.selected
    assert np.abs(a.K - b.K).max() < 1e-12
    ra, rb = oracle.spatial_rectangles(a), oracle.spatial_rectangles(b)
    assert ra.shape == rb.shape and np.abs(ra - rb).max() < 1e-12


def test_cell_fit_orientation_anisotropic():
    """exp(-x^2/2a^2 - y^2/2b^2) with a != b: C[b, a] is the product of the
    y-coefficient (sigma b) and the x-coefficient (sigma a); a transposed
    operand anywhere swaps them."""
    r, sa, sb = 9, 1.5, 4.0
    fit = oracle.spatial_fit_2d(_anisotropic(sa, sb), r, 6)
    T = r + 0.5
    cx = np.array([oracle.haar_coefficient(f, sa, T) for f in fit.family])
    cy = np.array([oracle.haar_coefficient(f, sb, T) for f in fit.family])
    assert np.abs(fit.coef2 - np.outer(cy, cx)).max() < 1e-13
    # the sampled expansion is wider along y than along x
    K = fit.K
    assert K[r + 6, r] > K[r, r + 6]


@pytest.mark.parametrize("cells", [(8, 8), (7, 8), (0, 0), (8, 11), (3, 15), (12, 5)])
def test_cell_integrals_by_adaptive_quadrature(cells):
    """Cell integrals of the radial exponential (cusp at the origin, a cell
    corner) against scipy's adaptive dblquad."""
    ss, T = 3.0, 9.5
    n = 16
    M = oracle.cell_integrals(oracle.spatial_kernel_2d("exponential", ss), T, n)
    h = 2 * T / n
    j, i = cells
    ylo, xlo = -T + h * j, -T + h * i
    ref, _ = integrate.dblquad(lambda y, x: math.exp(-math.hypot(x, y) / ss), xlo, xlo + h, ylo, ylo + h,
                               epsabs=1e-14, epsrel=1e-13)
    assert abs(M[j, i] - ref) <= 1e-12 * ref


def test_cell_fit_full_expansion_is_cell_average():
    """With every level group kept the Haar basis is complete on the finest
    cells: the expansion at an offset is the average of K over its cell.
    Asymmetric kernel, so index, sign and transpose mistakes show."""
    r = 6
    k = lambda x, y: np.exp(-((x - 0.7) ** 2) / 8.0 - ((y + 1.3) ** 2) / 3.0 - 0.1 * x * y)
    T = r + 0.5
    J = oracle.fit.max_level(T)
    fit = oracle.spatial_fit_2d(k, r, (J + 2) ** 2)
    n = 2 ** (J + 1)
    h = 2 * T / n
    M = oracle.cell_integrals(k, T, n)
    d = np.arange(-r, r + 1)
    cell = np.floor((d + T) / h).astype(int)
    expect = M[np.ix_(cell, cell)] / (h * h)       # [dy, dx]
    assert np.abs(fit.K - expect).max() < 1e-12


def test_cell_fit_parseval_energy():
    """Sum of every group's energy = squared L2 norm of the cell-average
    projection, sum of M^2 / h^2 (Parseval on the orthogonal Haar basis)."""
    r = 9
    T = r + 0.5
    J = oracle.fit.max_level(T)
    fit = oracle.spatial_fit_2d(oracle.spatial_kernel_2d("exponential", 2.5), r, 1)
    n = 2 ** (J + 1)
    h = 2 * T / n
    total = sum(e for e, _, _ in fit.groups_ranked)
    assert abs(total - (fit.cells ** 2).sum() / (h * h)) < 1e-9 * total


@pytest.mark.parametrize("sigma,span", [(0.1, 1.0), (0.3, 1.0), (0.05, 0.0)])
def test_exponential_range_coefficients_closed_form(sigma, span):
    """a_j of exp(-|t|/sigma) on [-T, T]: (2/T)(alpha - alpha e^{-alpha T}(-1)^j) /
    (alpha^2 + (pi j / T)^2), a_0 = (1 - e^{-alpha T}) / (alpha T), alpha = 1/sigma;
    T = max(sigma ln(1/eps), span)."""
    fit = oracle.range_fit(sigma, 8, eps=0.01, span=span, kernel="exponential")
    assert abs(fit.T_r - sigma * math.log(100.0)) < 1e-15
    T, al = fit.T, 1.0 / sigma
    j = np.arange(fit.M)
    w = np.pi * j / T
    cf = (2 / T) * (al - np.exp(-al * T) * al * (-1.0) ** j) / (al * al + w * w)
    cf[0] = (1 - math.exp(-al * T)) / (al * T)
    assert np.abs(cf - fit.a_all).max() < 1e-12 * cf[0]


def _py_true_bf_kinds(I, ss, r, sr):
    """Eq. BF with exp(-||d|| / ss) and exp(-|t| / sr), plain loops."""
    H, W = I.shape
    out = np.zeros_like(I)
    for py in range(H):
        for px in range(W):
            num = den = 0.0
            for qy in range(max(0, py - r), min(H, py + r + 1)):
                for qx in range(max(0, px - r), min(W, px + r + 1)):
                    w = math.exp(-math.hypot(py - qy, px - qx) / ss) * math.exp(-abs(I[py, px] - I[qy, qx]) / sr)
                    num += w * I[qy, qx]
                    den += w
            out[py, px] = num / den
    return out


def test_true_bf_exponential_kinds_brute_force_tiny():
    I = synth.gen_image(7, 9, 2, 0.05, 13).astype(np.float64)
    ref = _py_true_bf_kinds(I, 1.5, 3, 0.2)
    got = oracle.true_bf(I, 1.5, 3, 0.2, kind_s="exponential", kind_r="exponential")
    assert np.abs(got - ref).max() < 1e-14


def test_exponential_expansion_converges_to_true_bf():
    """More range terms and all spatial groups: the expanded filter approaches
    Eq. BF with the exponential kernels (the error shrinks)."""
    I = synth.gen_image(32, 32, 3, 0.02, 21)
    r = 7
    ref = oracle.true_bf(I, 2.0, r, 0.2, kind_s="exponential", kind_r="exponential")
    errs = []
    for ns, nr in ((2, 4), (6, 12), (16, 40)):
        p = oracle.make_plan(2.0, r, ns, 0.2, nr, kind_s="exponential", kind_r="exponential")
        errs.append(np.abs(oracle.expanded_box(I, p) - ref).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.02


def test_exponential_plan_T2_equals_T3():
    """Shift identity and box sums hold for any kernel pair."""
    I = synth.gen_image(33, 41, 3, 0.03, 5)
    p = oracle.make_plan(2.5, 8, 6, 0.15, 12, kind_s="exponential", kind_r="exponential")
    assert np.abs(oracle.expanded_brute(I, p) - oracle.expanded_box(I, p)).max() < 1e-11


# ---------------------------------------------------------------------------
# The paper's own regime for 8-bit images: T = T_r and the range box
# (T4 direct sum, T5 dimension promotion with 3-D summed-area tables)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("H,W,ss,r,ns,sr,nr,seed", [
    (23, 31, 2.0, 6, 4, 0.1, 5, 4), (17, 12, 1.5, 4, 6, 0.05, 8, 5), (20, 26, 3.0, 9, 4, 0.2, 3, 6),
    (1, 1, 2.0, 6, 4, 0.1, 5, 7), (3, 40, 2.0, 6, 5, 0.08, 5, 8)])
def test_rangebox_direct_sum_equals_3d_tables(H, W, ss, r, ns, sr, nr, seed):
    """T4 (the definition summed pixel by pixel) and T5 (auxiliary volumes over
    256 levels and 3-D summed-area tables, Eqs. sat_sum_3D_1/2) agree."""
    Z = synth.gen_image_u8(H, W, 3, 0.03, seed)
    p = oracle.make_plan(ss, r, ns, sr, nr, span=0.0)
    assert p.range.T == p.range.T_r
    a, na, da = oracle.expanded_rangebox(Z, p, return_parts=True)
    b, nb, db = oracle.expanded_sat3d(Z, p, return_parts=True)
    assert np.abs(na - nb).max() < 1e-12 and np.abs(da - db).max() < 1e-12
    assert np.abs(a - b).max() < 1e-12


def test_rangebox_wide_box_is_the_plain_expansion():
    """With 255 T_r >= 255 every level difference is inside the box: T4 = T2."""
    Z = synth.gen_image_u8(24, 28, 3, 0.03, 9)
    p = oracle.make_plan(2.0, 6, 4, 0.45, 8, span=0.0)
    assert oracle.box_levels(p) >= 255
    assert np.abs(oracle.expanded_rangebox(Z, p) - oracle.expanded_brute(Z, p)).max() < 1e-15


def _range_exact_with_box(Z, p, sr):
    """Eq. BF with the plan's K~_s, the exact Gaussian K_r and the range box."""
    H, W = Z.shape
    I = Z / 255.0
    r = p.radius
    zr = oracle.box_levels(p)
    out = np.zeros((H, W))
    for py in range(H):
        for px in range(W):
            y0, y1, x0, x1 = max(0, py - r), min(H, py + r + 1), max(0, px - r), min(W, px + r + 1)
            q = I[y0:y1, x0:x1]
            dz = np.abs(Z[y0:y1, x0:x1].astype(int) - int(Z[py, px]))
            ks = p.Ks[r + py - y1 + 1:r + py - y0 + 1, r + px - x1 + 1:r + px - x0 + 1][::-1, ::-1]
            w = ks * np.exp(-(I[py, px] - q) ** 2 / (2 * sr * sr)) * (dz <= zr)
            out[py, px] = (w * q).sum() / w.sum()
    return out


def test_rangebox_converges_in_range_terms():
    """Range series on [-T_r, T_r]: few terms suffice in this regime (Sec. VI:
    five terms; the kernel error at N = 5 is 3.8e-3) and the filter converges
    to Eq. BF with the exact range kernel inside the box."""
    Z = synth.gen_image_u8(24, 28, 3, 0.03, 9)
    sr = 0.1
    errs = []
    for nr in (2, 3, 5, 16):
        p = oracle.make_plan(2.0, 6, 4, sr, nr, span=0.0)
        errs.append(np.abs(oracle.expanded_rangebox(Z, p) - _range_exact_with_box(Z, p, sr)).max())
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[2] < 2e-4
    p = oracle.make_plan(2.0, 6, 4, sr, 5, span=0.0)
    t = np.linspace(-p.range.T_r, p.range.T_r, 4001)
    kerr = np.abs(oracle.range_kernel_approx(p.range, t) - np.exp(-t * t / (2 * sr * sr))).max()
    assert 3.0e-3 < kerr < 4.0e-3


def test_rangebox_constant_image_is_unchanged():
    Z = np.full((9, 13), 77, dtype=np.uint8)
    p = oracle.make_plan(2.0, 6, 4, 0.1, 5, span=0.0)
    assert np.abs(oracle.expanded_rangebox(Z, p) - 77 / 255.0).max() < 1e-14


# ---------------------------------------------------------------------------
# Tabulated kernels (arbitrary kernels, Secs. I, IV-B and VI): a spatial table
# constant on unit squares, a range table linear between samples
# ---------------------------------------------------------------------------
def _even_table(r, seed):
    g = np.random.default_rng(seed).uniform(0.05, 1.0, (r + 1, r + 1))
    q = np.concatenate([g[:0:-1], g])              # rows -r .. r from |dy|
    return np.concatenate([q[:, :0:-1], q], axis=1)


def _fine_grid(table, n_cells, sub):
    """The tabulated kernel sampled at the midpoints of a grid of step h / sub
    (h = 2T / n_cells): every pixel edge and every cell edge is a grid line
    when sub = 2r + 1, so midpoint sums of one cell are its exact integral."""
    r = (table.shape[0] - 1) // 2
    T = r + 0.5
    step = 2.0 * T / (n_cells * sub)
    mids = -T + step * (np.arange(n_cells * sub) + 0.5)
    idx = np.floor(mids + 0.5).astype(int) + r      # the offset whose unit square holds the midpoint
    return table[np.ix_(idx, idx)] * step * step


@pytest.mark.parametrize("r,seed", [(1, 0), (5, 1), (9, 2), (12, 3)])
def test_tabulated_cell_integrals_match_fine_grid(r, seed):
    """Exact overlap sums against midpoint sums on a grid fine enough to be
    exact for a function constant on unit squares."""
    table = _even_table(r, seed)
    n = 2 ** (F.max_level(r + 0.5) + 1)
    sub = 2 * r + 1
    fine = _fine_grid(table, n, sub).reshape(n, sub, n, sub).sum(axis=(1, 3))
    M = F.tabulated_cell_integrals(table, n)
    assert np.abs(M - fine).max() <= 1e-13 * table.sum()
    assert abs(M.sum() - table.sum()) <= 1e-12 * table.sum()      # each unit square has area 1


@pytest.mark.parametrize("r,seed", [(5, 4), (9, 5)])
def test_tabulated_full_expansion_is_the_cell_average(r, seed):
    """With every level group kept the Haar expansion is the projection onto
    functions constant on the finest cells: K~_s at an offset is the mean of
    the kernel over the cell holding it (half-open cells, by brute force)."""
    table = _even_table(r, seed)
    T = r + 0.5
    J = F.max_level(T)
    n = 2 ** (J + 1)
    fit = F.spatial_fit_table(table, (J + 2) ** 2)
    h = 2.0 * T / n
    sub = 2 * r + 1
    fine = _fine_grid(table, n, sub).reshape(n, sub, n, sub).sum(axis=(1, 3)) / (h * h)
    cell = np.floor((np.arange(-r, r + 1) + T) / h).astype(int)
    assert np.abs(fit.K - fine[np.ix_(cell, cell)]).max() <= 1e-12 * table.max()


def test_tabulated_spatial_table_must_be_even():
    t = _even_table(3, 6)
    t[0, 1] += 0.1
    with pytest.raises(ValueError):
        F.spatial_fit_table(t, 4)


@pytest.mark.parametrize("w,T", [(0.3, 1.0), (0.05, 1.0), (1.0, 1.0), (0.2, 2.5)])
def test_piecewise_linear_coefficients_of_a_tent(w, T):
    """Two samples (1, 0) at step w are the tent max(0, 1 - |t| / w), whose
    Fourier cosine integral is 2 (1 - cos(omega w)) / (omega^2 w)."""
    M = 200
    a = F.piecewise_linear_cosine_coefficients([1.0, 0.0], w, T, M)
    j = np.arange(1, M)
    om = np.pi * j / T
    ref = 2.0 * (1.0 - np.cos(om * w)) / (om * om * w) / T
    assert abs(a[0] - 0.5 * w / T) <= 1e-15
    assert np.abs(a[1:] - ref).max() <= 1e-14


def test_piecewise_linear_coefficients_match_adaptive_quadrature():
    """A random table against QUADPACK's cosine-weighted quadrature (QAWO) of
    np.interp on each linear piece."""
    rng = np.random.default_rng(7)
    v = rng.uniform(0.0, 1.0, 13)
    step, T, M = 0.06, 1.0, 60
    a = F.piecewise_linear_cosine_coefficients(v, step, T, M)
    tk = step * np.arange(len(v))
    f = lambda t: np.interp(t, tk, v)
    for j in range(M):
        om = np.pi * j / T
        s = sum(integrate.quad(f, tk[i], tk[i + 1], weight="cos", wvar=om, epsabs=1e-15, epsrel=1e-13)[0]
                for i in range(len(v) - 1))
        ref = s / T if j == 0 else 2.0 * s / T
        assert abs(a[j] - ref) <= 1e-13, j


def test_table_range_fit_converges_to_the_gaussian_fit():
    """Samples of the Gaussian range kernel at step 1e-4 over [0, 1] give the
    closed-form Gaussian fit's coefficients up to the interpolation error
    (step^2 max|K''| / 8 = 5e-7 at sigma_r = 0.05)."""
    sr = 0.05
    step = 1e-4
    t = step * np.arange(10001)
    tab = F.range_fit_table(F.gaussian(t, sr), step, 16, span=1.0)
    ref = F.range_fit(sr, 16, span=1.0)
    assert tab.T == ref.T == 1.0
    assert tab.k.tolist() == ref.k.tolist()
    assert np.abs(tab.a - ref.a).max() <= 1e-6


def test_tabulated_true_bf_equals_gaussian_true_bf_at_the_knots():
    """On 8-bit images every intensity difference is a multiple of 1/255, so a
    range table sampled at those levels and a spatial table sampled at the
    integer offsets reproduce T1 with the Gaussian kernels."""
    I = (synth.gen_image(23, 19, 4, 0.08, 11) * 255).round().clip(0, 255).astype(np.uint8)
    r, ss, sr = 4, 2.0, 0.1
    d = np.arange(-r, r + 1)
    ks = np.exp(-(d[:, None] ** 2 + d[None, :] ** 2) / (2 * ss * ss))
    kr = np.exp(-(np.arange(256) / 255.0) ** 2 / (2 * sr * sr))
    a = oracle.true_bf_tab(I, ks, kr, 1.0 / 255.0)
    b = oracle.true_bf(I, ss, r, sr)
    assert np.abs(a - b).max() <= 1e-12


def test_tabulated_true_bf_interpolates_linearly():
    """A tent range table (samples 1, 0.5, 0 at step w / 2) is linear on its
    pieces, so T1 with it is Eq. BF with max(0, 1 - |t| / w), summed here by a
    pure-Python double loop."""
    I = synth.gen_image(9, 11, 3, 0.1, 12).astype(np.float64)
    r, w = 2, 0.3
    ks = _even_table(r, 8)
    got = oracle.true_bf_tab(I, ks, [1.0, 0.5, 0.0], w / 2)
    H, W = I.shape
    for y in range(H):
        for x in range(W):
            num = den = 0.0
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    qy, qx = y - dy, x - dx
                    if 0 <= qy < H and 0 <= qx < W:
                        wt = ks[dy + r, dx + r] * max(0.0, 1.0 - abs(I[y, x] - I[qy, qx]) / w)
                        num += wt * I[qy, qx]
                        den += wt
            assert abs(got[y, x] - num / den) <= 1e-13


def test_tabulated_plan_through_the_filters():
    """A plan of two tables: T2 (direct sum) and T3 (box sums) agree, and with
    every term kept the expansion approaches T1 with the tables."""
    r = 6
    ks = _even_table(r, 9)
    kr = np.array([1.0, 0.9, 0.6, 0.35, 0.15, 0.05, 0.0])
    I = synth.gen_image(30, 27, 4, 0.05, 13).astype(np.float64)
    p = oracle.make_table_plan(ks, kr, 0.04, 4, 12)
    t2 = oracle.expanded_brute(I, p)
    t3 = oracle.expanded_box(I, p)
    assert np.abs(t2 - t3).max() <= 1e-10
    full = oracle.make_table_plan(ks, kr, 0.04, (F.max_level(r + 0.5) + 2) ** 2, 64)
    t1 = oracle.true_bf_tab(I, ks, kr, 0.04)
    # the full spatial expansion averages the table over cells of side h in [1, 2)
    assert np.abs(oracle.expanded_box(I, full) - t1).max() < 0.05
    # a box kernel is phi(x) phi(y) itself: one group reproduces it exactly,
    # and what is left is the range series' truncation error
    box = np.ones_like(ks)
    p1 = oracle.make_table_plan(box, kr, 0.04, 1, 64)
    assert p1.spatial.selected == [(F.PHI, F.PHI)] and np.abs(p1.Ks - 1.0).max() <= 1e-14
    assert np.abs(oracle.expanded_box(I, p1) - oracle.true_bf_tab(I, box, kr, 0.04)).max() < 1e-3


def test_planted_mistake_in_the_spatial_table_is_caught():
    """Unit squares anchored at the offset instead of centred on it: the
    fine-grid pin tells the two apart."""
    r = 5
    table = _even_table(r, 10)
    n = 2 ** (F.max_level(r + 0.5) + 1)
    T, h = r + 0.5, (2 * r + 1.0) / n
    lo = -T + h * np.arange(n)
    d = np.arange(-r, r + 1)
    A = np.clip(np.minimum(lo[:, None] + h, d[None, :] + 1.0) - np.maximum(lo[:, None], d[None, :] * 1.0), 0, None)
    shifted = A @ table @ A.T
    fine = _fine_grid(table, n, 2 * r + 1).reshape(n, 2 * r + 1, n, 2 * r + 1).sum(axis=(1, 3))
    assert np.abs(shifted - fine).max() > 1e-3
