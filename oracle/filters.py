"""Python front end of the FP64 oracle filters (TEST INFRASTRUCTURE ONLY).

T1 true_bf         : Eq. BF with the exact kernels (Gaussian or exponential),
                     square window [-r, r]^2; true_bf_tab with tabulated kernels.
T2 expanded_brute  : Eq. BF with the N-term expansions of both kernels, direct sum.
T3 expanded_box    : the same through the cosine shift identity (Eq. 1D_N_terms)
                     and FP64 summed-area-table box sums of the Haar rectangles
                     (Eqs. sum_sat_2D .. sum_sat_sum_region_2D, App. A).
T4 expanded_rangebox : the paper's own regime for 8-bit images: range series on
                     [-T_r, T_r] (T = T_r) times the range box |Z(p) - Z(q)| <=
                     255 T_r (Eq. 1D_box_N_terms), direct sum.
T5 expanded_sat3d  : the same quantity the paper's way: auxiliary volumes
                     F(y, z) = G(y) delta_{Z(y)}(z) over the 256 levels, 3-D
                     summed-area tables (Eqs. sat_sum_3D_1/2, sat_sum_1D) and
                     cube sums per Haar rectangle (Eq. numerator_2D_box_N_terms);
                     numpy, small images only.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build
from .fit import (spatial_fit, spatial_fit_2d, spatial_fit_table, spatial_kernel_2d, spatial_rectangles,
                  range_fit, range_fit_table)

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        lib.ref_true_bf.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_int, _ip, _ip, ctypes.c_long,
                                    ctypes.c_double, _dp]
        lib.ref_true_bf_tab.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, ctypes.c_int,
                                        ctypes.c_double, _ip, _ip, ctypes.c_long, ctypes.c_double, _dp]
        lib.ref_expanded_rangebox.argtypes = [ctypes.POINTER(ctypes.c_uint8), ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, _dp, ctypes.c_int, _dp, _dp, ctypes.c_double,
                                              _ip, _ip, ctypes.c_long, ctypes.c_double, _dp, _dp, _dp]
        lib.ref_expanded_brute.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp,
                                           ctypes.c_int, _dp, _dp, _ip, _ip, ctypes.c_long,
                                           ctypes.c_double, _dp, _dp, _dp]
        lib.ref_expanded_box.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                         ctypes.c_int, _dp, _dp, ctypes.c_double, _dp, _dp, _dp]
        lib.ref_expanded_box.restype = ctypes.c_int
        lib.ref_correlate_rects.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _dp]
        lib.ref_correlate_rects.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, ptr=_dp):
    return a.ctypes.data_as(ptr) if a is not None else None


def to_unit(I):
    """Intensities in [0, 1]: uint8 input is divided by 255 (float input as is)."""
    I = np.asarray(I)
    if I.dtype == np.uint8:
        return I.astype(np.float64) / 255.0
    return I.astype(np.float64)


class Plan:
    """Both kernel expansions for one parameter set."""

    def __init__(self, sigma_s, radius, n_spatial, sigma_r, n_range, eps=0.01, span=1.0,
                 kind_s="gaussian", kind_r="gaussian", tables=None):
        """tables = (spatial weights (2r+1) x (2r+1), range samples, range step):
        both kernels tabulated (sigma_s, sigma_r, kind_s, kind_r, eps unused;
        radius must match the spatial table)."""
        self.sigma_s, self.radius, self.sigma_r = sigma_s, radius, sigma_r
        self.kind_s, self.kind_r = kind_s, kind_r
        self.tables = tables
        if tables is not None:
            ks, kr, step = tables
            self.kind_s = self.kind_r = "tabulated"
            self.spatial = spatial_fit_table(ks, n_spatial)
            assert self.spatial.radius == radius
            self.range = range_fit_table(kr, step, n_range, span=span)
        elif kind_s == "gaussian":
            self.spatial = spatial_fit(sigma_s, radius, n_spatial)
        else:
            self.spatial = spatial_fit_2d(spatial_kernel_2d(kind_s, sigma_s), radius, n_spatial)
        if tables is None:
            self.range = range_fit(sigma_r, n_range, eps=eps, span=span, kernel=kind_r)
        self.Ks = np.ascontiguousarray(self.spatial.K, dtype=np.float64)
        self.rects = np.ascontiguousarray(spatial_rectangles(self.spatial), dtype=np.float64)
        self.a = np.ascontiguousarray(self.range.a, dtype=np.float64)
        self.omega = np.ascontiguousarray(self.range.omega, dtype=np.float64)
        # A11 guard: den below 1e-7 * sum|K~_s| falls back to I(p)
        self.den_floor = 1e-7 * float(np.abs(self.Ks).sum())


def make_plan(sigma_s, radius, n_spatial, sigma_r, n_range, **kw):
    return Plan(sigma_s, radius, n_spatial, sigma_r, n_range, **kw)


def make_table_plan(ks, kr, kr_step, n_spatial, n_range, span=1.0):
    """Plan of two tabulated kernels (see Plan)."""
    ks = np.asarray(ks, dtype=np.float64)
    return Plan(None, (ks.shape[0] - 1) // 2, n_spatial, None, n_range, span=span, tables=(ks, kr, kr_step))


def _pixels(H, W, ys, xs):
    if ys is None:
        return None, None, H * W
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    assert ys.shape == xs.shape and ys.ndim == 1
    assert ys.min() >= 0 and ys.max() < H and xs.min() >= 0 and xs.max() < W
    return ys, xs, len(ys)


_KIND = {"gaussian": 0, "exponential": 1}


def true_bf(I, sigma_s, radius, sigma_r, ys=None, xs=None, den_floor=0.0, kind_s="gaussian",
            kind_r="gaussian"):
    """T1 at all pixels (H x W result) or at the listed pixels (1-D result)."""
    I = np.ascontiguousarray(to_unit(I))
    H, W = I.shape
    ys, xs, n = _pixels(H, W, ys, xs)
    out = np.empty(n)
    _load().ref_true_bf(_p(I), H, W, int(radius), float(sigma_s), float(sigma_r), _KIND[kind_s],
                        _KIND[kind_r], _p(ys, _ip), _p(xs, _ip), n, float(den_floor), _p(out))
    return out.reshape(H, W) if ys is None else out


def true_bf_tab(I, ks, kr, kr_step, ys=None, xs=None, den_floor=0.0):
    """T1 with tabulated kernels: spatial weights ks[dy + r, dx + r], range
    weight the linear interpolant of kr[i] at |t| = i kr_step, zero past the
    last sample."""
    I = np.ascontiguousarray(to_unit(I))
    H, W = I.shape
    ks = np.ascontiguousarray(ks, dtype=np.float64)
    kr = np.ascontiguousarray(kr, dtype=np.float64)
    ys, xs, n = _pixels(H, W, ys, xs)
    out = np.empty(n)
    _load().ref_true_bf_tab(_p(I), H, W, (ks.shape[0] - 1) // 2, _p(ks), _p(kr), len(kr), float(kr_step),
                            _p(ys, _ip), _p(xs, _ip), n, float(den_floor), _p(out))
    return out.reshape(H, W) if ys is None else out


def expanded_brute(I, plan, ys=None, xs=None, return_parts=False):
    """T2 at all pixels (H x W) or at the listed pixels (1-D)."""
    I = np.ascontiguousarray(to_unit(I))
    H, W = I.shape
    ys, xs, n = _pixels(H, W, ys, xs)
    out, num, den = np.empty(n), np.empty(n), np.empty(n)
    _load().ref_expanded_brute(_p(I), H, W, int(plan.radius), _p(plan.Ks), len(plan.a),
                               _p(plan.a), _p(plan.omega), _p(ys, _ip), _p(xs, _ip), n,
                               plan.den_floor, _p(out), _p(num), _p(den))
    shp = (H, W) if ys is None else (n,)
    if return_parts:
        return out.reshape(shp), num.reshape(shp), den.reshape(shp)
    return out.reshape(shp)


def expanded_box(I, plan, return_parts=False):
    """T3 over the whole image."""
    I = np.ascontiguousarray(to_unit(I))
    H, W = I.shape
    out, num, den = np.empty((H, W)), np.empty((H, W)), np.empty((H, W))
    rc = _load().ref_expanded_box(_p(I), H, W, _p(plan.rects), len(plan.rects), len(plan.a),
                                  _p(plan.a), _p(plan.omega), plan.den_floor, _p(out), _p(num),
                                  _p(den))
    if rc != 0:
        raise MemoryError("oracle T3 allocation failed")
    if return_parts:
        return out, num, den
    return out


def correlate_rects(g, rects):
    """sum_q K(p - q) g(q) for K given as weighted rectangles, via an FP64 SAT."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    rects = np.ascontiguousarray(rects, dtype=np.float64)
    H, W = g.shape
    out = np.empty((H, W))
    if _load().ref_correlate_rects(_p(g), H, W, _p(rects), len(rects), _p(out)) != 0:
        raise MemoryError("oracle allocation failed")
    return out


def _levels(I):
    Z = np.asarray(I)
    if Z.dtype != np.uint8:
        raise TypeError("the range-box regime is defined for 8-bit images")
    return np.ascontiguousarray(Z)


def box_levels(plan):
    """255 T_r: the range box half-width in 8-bit levels (a level difference d
    is inside the box when |d| <= 255 T_r)."""
    return 255.0 * plan.range.T_r


def expanded_rangebox(Z, plan, ys=None, xs=None, return_parts=False):
    """T4 for an 8-bit image Z.  The plan must put the range series on
    [-T_r, T_r] (span = 0)."""
    Z = _levels(Z)
    if abs(plan.range.T - plan.range.T_r) > 0:
        raise ValueError("the range-box regime takes T = T_r (make the plan with span=0)")
    H, W = Z.shape
    ys, xs, n = _pixels(H, W, ys, xs)
    out, num, den = np.empty(n), np.empty(n), np.empty(n)
    _load().ref_expanded_rangebox(Z.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), H, W,
                                  int(plan.radius), _p(plan.Ks), len(plan.a), _p(plan.a),
                                  _p(plan.omega), box_levels(plan), _p(ys, _ip), _p(xs, _ip), n,
                                  plan.den_floor, _p(out), _p(num), _p(den))
    shp = (H, W) if ys is None else (n,)
    if return_parts:
        return out.reshape(shp), num.reshape(shp), den.reshape(shp)
    return out.reshape(shp)


def expanded_sat3d(Z, plan, return_parts=False):
    """T5: T4 computed with the paper's dimension promotion and 3-D summed-area
    tables (small images: four H x W x 256 volumes per range term)."""
    Z = _levels(Z).astype(np.int64)
    H, W = Z.shape
    I = Z / 255.0
    zr = int(math.floor(box_levels(plan)))
    zlo = np.clip(Z - zr, 0, 255)
    zhi = np.clip(Z + zr, 0, 255) + 1          # exclusive
    yy, xx = np.mgrid[0:H, 0:W]
    num = np.zeros((H, W))
    den = np.zeros((H, W))

    def sat3(G):
        F = np.zeros((H + 1, W + 1, 257))
        F[yy + 1, xx + 1, Z + 1] = G           # F(y, z) = G(y) delta_{Z(y)}(z)
        return F.cumsum(0).cumsum(1).cumsum(2)

    def cube(S, y0, y1, x0, x1, z0, z1):       # sum over [y0, y1) x [x0, x1) x [z0, z1)
        s = 0.0
        for Y, sy in ((y1, 1), (y0, -1)):
            for X, sx in ((x1, 1), (x0, -1)):
                s = s + sy * sx * (S[Y, X, z1] - S[Y, X, z0])
        return s

    def correlate_cube(S):
        acc = np.zeros((H, W))
        for ey0, ey1, ex0, ex1, w in plan.rects:
            # sources q = p - e with e in the rectangle, clipped to the image
            y0 = np.clip(yy - int(ey1), 0, H)
            y1 = np.clip(yy - int(ey0) + 1, 0, H)
            x0 = np.clip(xx - int(ex1), 0, W)
            x1 = np.clip(xx - int(ex0) + 1, 0, W)
            ok = (y1 > y0) & (x1 > x0)
            acc += w * np.where(ok, cube(S, y0, np.maximum(y1, y0), x0, np.maximum(x1, x0), zlo, zhi), 0.0)
        return acc

    for a, om in zip(plan.a, plan.omega):
        c, s_ = np.cos(om * I), np.sin(om * I)
        num += a * (c * correlate_cube(sat3(c * I)) + s_ * correlate_cube(sat3(s_ * I)))
        den += a * (c * correlate_cube(sat3(c)) + s_ * correlate_cube(sat3(s_)))
    out = np.where(den > plan.den_floor, num / np.where(den == 0, 1, den), I)
    if return_parts:
        return out, num, den
    return out
