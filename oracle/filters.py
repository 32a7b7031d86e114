"""Python front end of the FP64 oracle filters (TEST INFRASTRUCTURE ONLY).

T1 true_bf         : Eq. BF with the exact kernels (Gaussian or exponential),
                     square window [-r, r]^2.
T2 expanded_brute  : Eq. BF with the N-term expansions of both kernels, direct sum.
T3 expanded_box    : the same through the cosine shift identity (Eq. 1D_N_terms)
                     and FP64 summed-area-table box sums of the Haar rectangles
                     (Eqs. sum_sat_2D .. sum_sat_sum_region_2D, App. A).
"""
import ctypes
import os

import numpy as np

from . import build as _build
from .fit import spatial_fit, spatial_fit_2d, spatial_kernel_2d, spatial_rectangles, range_fit

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
                 kind_s="gaussian", kind_r="gaussian"):
        self.sigma_s, self.radius, self.sigma_r = sigma_s, radius, sigma_r
        self.kind_s, self.kind_r = kind_s, kind_r
        if kind_s == "gaussian":
            self.spatial = spatial_fit(sigma_s, radius, n_spatial)
        else:
            self.spatial = spatial_fit_2d(spatial_kernel_2d(kind_s, sigma_s), radius, n_spatial)
        self.range = range_fit(sigma_r, n_range, eps=eps, span=span, kernel=kind_r)
        self.Ks = np.ascontiguousarray(self.spatial.K, dtype=np.float64)
        self.rects = np.ascontiguousarray(spatial_rectangles(self.spatial), dtype=np.float64)
        self.a = np.ascontiguousarray(self.range.a, dtype=np.float64)
        self.omega = np.ascontiguousarray(self.range.omega, dtype=np.float64)
        # A11 guard: den below 1e-7 * sum|K~_s| falls back to I(p)
        self.den_floor = 1e-7 * float(np.abs(self.Ks).sum())


def make_plan(sigma_s, radius, n_spatial, sigma_r, n_range, **kw):
    return Plan(sigma_s, radius, n_spatial, sigma_r, n_range, **kw)


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
