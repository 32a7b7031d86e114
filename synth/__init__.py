"""Seeded synthetic inputs shared by the tests, the oracle runs and the benchmark.

This module holds no arithmetic of the filtering method: it only draws images
(and request streams) from a seeded PCG64 generator.  The paper evaluates on
natural photographs (Lena, Barbara, Boat, an HDR scene) that are not available
here; these fields stand in for them: smooth multi-octave gradient noise for
the low-frequency content, straight step edges for the structures a bilateral
filter must preserve, and Gaussian sensor noise.  kernels.py holds sampled
kernel shapes for the plans of tabulated kernels.
"""
from .images import gen_image, gen_image_u8, config_image
from .stream import gen_stream
from . import kernels

__all__ = ["gen_image", "gen_image_u8", "config_image", "gen_stream", "kernels"]
