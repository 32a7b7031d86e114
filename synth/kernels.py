"""Kernel tables used as inputs of tabulated plans: sampled shapes other than
the Gaussian, as a user of arbitrary kernels would pass them.  These are the
kernels' definitions only (no arithmetic of the filtering method)."""
import numpy as np


def _offsets(r):
    d = np.arange(-r, r + 1, dtype=np.float64)
    return d[:, None] ** 2 + d[None, :] ** 2


def cauchy_spatial(r, s):
    """1 / (1 + ||d||^2 / s^2) on the (2r+1)^2 offsets: radial, heavy-tailed,
    not separable."""
    return 1.0 / (1.0 + _offsets(r) / (s * s))


def gaussian_spatial(r, s):
    """exp(-||d||^2 / 2 s^2) on the (2r+1)^2 offsets."""
    return np.exp(-_offsets(r) / (2.0 * s * s))


def tukey_range(c, step):
    """Tukey's biweight (1 - (t / c)^2)^2 on [0, c], sampled at multiples of
    step (c a multiple of step)."""
    t = step * np.arange(int(round(c / step)) + 1)
    return (1.0 - (t / c) ** 2) ** 2


def cauchy_range(s, step, n):
    """1 / (1 + t^2 / s^2) at t = i step, i < n."""
    t = step * np.arange(n)
    return 1.0 / (1.0 + (t / s) ** 2)
