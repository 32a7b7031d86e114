"""Host-side tests of the library (no GPU): symbols, plan tables against the
oracle's independently computed tables, the tap convention, argument checks."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_1803_00004_amd import bf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CONFIGS = [(3.0, 9, 4, 0.1, 8), (8.0, 24, 6, 0.1, 16), (16.0, 48, 8, 0.05, 32),
           (2.0, 6, 4, 0.3, 8), (4.0, 12, 4, 0.2, 8), (3.0, 10, 3, 0.1, 5), (2.0, 6, 9, 0.05, 32)]


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "bf.h")).read()
    declared = set(re.findall(r"^\s*(?:bf_status_t|const char \*)\s*(bf_\w+)\s*\(", hdr, re.M))
    assert {"bf_plan_create", "bf_filter", "bf_filter_batch"} <= declared
    L = bf.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared <= set(bf.EXPORTED)
    assert bf.lib().bf_version().decode().startswith("bf-mi355x")


def test_binding_declares_every_argument_type():
    """Every entry point has its ctypes argument types: a size_t passed as a
    plain Python int would be cut to a C int (workspaces above 2 GiB)."""
    L = bf.lib()
    missing = [n for n in bf.EXPORTED if getattr(L, n).argtypes is None]
    assert not missing, missing
    # a size above 2^32 reaches the library intact: the bound check sees it
    p = bf.Plan(3.0, 0.1, 9, 8, 4, host_only=True)
    big = (1 << 33) + 5
    assert L.bf_filter_precomputed(p.handle, p.handle, ctypes.c_void_p(0x10000), ctypes.c_void_p(0x90000), 16, 16,
                                   ctypes.c_void_p(1 << 40), big, None) == bf.BF_ERR_INVALID_ARG  # host-only plan


@pytest.mark.parametrize("ss,r,ns,sr,nr", CONFIGS)
def test_plan_tables_match_oracle(ss, r, ns, sr, nr):
    p = bf.Plan(ss, sr, r, nr, ns, host_only=True)
    o = oracle.make_plan(ss, r, ns, sr, nr)
    assert p.spatial_groups() == o.spatial.selected
    assert np.abs(p.spatial_kernel() - o.Ks).max() <= 1e-13
    k, a, w = p.range_terms()
    assert k.tolist() == o.range.k.tolist()
    assert np.abs(a - o.a).max() <= 1e-13
    assert np.abs(w - o.omega).max() <= 1e-13
    info = p.info
    assert info.n_images == sum(1 if kk == 0 else 4 for kk in k)
    assert abs(info.T - o.range.T) < 1e-15 and abs(info.T_s - (r + 0.5)) < 1e-15
    assert abs(info.den_floor - o.den_floor) <= 1e-12 * o.den_floor


def test_config_tap_counts():
    """Tap counts of the three workloads' spatial expansions: 16 / 32 / 48."""
    for (ss, r, ns), P in zip([(3.0, 9, 4), (8.0, 24, 6), (16.0, 48, 8)], [16, 32, 48]):
        assert bf.Plan(ss, 0.1, r, 8, ns, host_only=True).info.n_taps == P


def _excl_sat(g):
    H, W = g.shape
    S = np.zeros((H + 1, W + 1))
    S[1:, 1:] = np.cumsum(np.cumsum(g, axis=0), axis=1)
    return S


@pytest.mark.parametrize("ss,r,ns,sr,nr", CONFIGS[:5])
def test_taps_reproduce_oracle_correlation(ss, r, ns, sr, nr):
    """corr(p) = sum_i w_i S(clamp(p + d_i)) over the plan's taps equals the
    oracle's rectangle correlation, with a global table and with the
    tile-relative tables the kernels build (origin max(y0 - r, 0))."""
    p = bf.Plan(ss, sr, r, nr, ns, host_only=True)
    o = oracle.make_plan(ss, r, ns, sr, nr)
    dy, dx, w = p.taps()
    assert dy.min() >= -r and dy.max() <= r + 1 and dx.min() >= -r and dx.max() <= r + 1
    H, W = 70, 83
    g = synth.gen_image(H, W, 4, 0.05, 17).astype(np.float64) - 0.3
    ref = oracle.correlate_rects(g, o.rects)
    S = _excl_sat(g)
    ys, xs = np.mgrid[0:H, 0:W]
    corr = np.zeros((H, W))
    for a, b, c in zip(dy, dx, w):
        corr += c * S[np.clip(ys + a, 0, H), np.clip(xs + b, 0, W)]
    assert np.abs(corr - ref).max() < 1e-10
    tile = 32
    for ty in range(0, H, tile):
        for tx in range(0, W, tile):
            y1, x1 = min(H, ty + tile), min(W, tx + tile)
            oy, ox = max(ty - r, 0), max(tx - r, 0)
            ye, xe = min(y1 + r, H), min(x1 + r, W)
            St = _excl_sat(g[oy:ye, ox:xe])
            yy, xx = np.mgrid[ty:y1, tx:x1]
            c2 = np.zeros(yy.shape)
            for a, b, c in zip(dy, dx, w):
                c2 += c * St[np.clip(yy + a, 0, H) - oy, np.clip(xx + b, 0, W) - ox]
            assert np.abs(c2 - ref[ty:y1, tx:x1]).max() < 1e-10


def test_tiling_keeps_boxes_in_int32():
    """Every box difference the kernels form stays inside int32: with all taps
    in symmetric quadruplets q is the largest shift (<= 24) with
    (2r + 1)^2 (gmax 2^q + 1) <= 2^31 - 1, the same for every image and tile;
    the tile is a multiple of 64, fixed when the plan fixes it, and a pure
    function of the image size."""
    for ss, r, ns, sr, nr in CONFIGS:
        for fixed in (0, 128, 256):
            p = bf.Plan(ss, sr, r, nr, ns, tile=fixed, host_only=True)
            info = p.info
            assert info.n_single == 0 and 4 * info.n_quads == info.n_taps
            B = (2 * r + 1) ** 2
            q0 = info.sat_shift
            assert B * (2.0 ** q0 + 1) <= 2 ** 31 - 1
            assert B * (2.0 ** (q0 + 1) + 1) > 2 ** 31 - 1 or q0 == 24
            for H, W in ((1, 1), (256, 256), (1080, 1920), (4096, 4096), (37, 3000)):
                tile, q, nbytes = p.geometry(H, W)
                assert tile % 64 == 0 and (fixed == 0 or tile == fixed)
                assert q == q0
                assert nbytes == p.workspace_size(H, W) and p.geometry(H, W) == (tile, q, nbytes)


def test_lookup_kernel_choice_and_lattice_tiles():
    """Which lookup kernel an untuned image runs: the double-buffered LDS tile
    kernel where two regions fit (r <= 32), the lattice kernel for plans of
    more than 8 quadruplets on a row lattice (r = 48, N_s = 8: 96-row lattice
    tiles, table tiles of 576 rows at 4096^2 and whole lattice tiles on every
    image), else the LDS tile kernel; a tuned choice wins; plans without
    tables have none."""
    cfg3 = bf.Plan(16.0, 0.05, 48, 32, 8, host_only=True)
    assert cfg3.info.lattice == 1 and cfg3.info.lattice_step == 12 and cfg3.info.n_quads == 12
    assert cfg3.info.default_lookup == 3 and cfg3.lookup_kernel(4096, 4096) == 3
    for H, W in ((4096, 4096), (1080, 1920), (300, 517), (1, 1), (32768, 48)):
        tile = cfg3.geometry(H, W)[0]
        assert tile % 64 == 0 and tile % 96 == 0 and tile <= 576, (H, W, tile)
    assert cfg3.geometry(4096, 4096)[0] == 576
    try:
        cfg3.set_tuning(4096, 4096, 512, 1, 0)
        assert cfg3.lookup_kernel(4096, 4096) == 2 and cfg3.geometry(4096, 4096)[0] == 512
        assert cfg3.lookup_kernel(1080, 1920) == 3  # another size bucket keeps the default
    finally:
        bf.lib().bf_autotune_clear()
    four = bf.Plan(16.0, 0.1, 48, 8, 4, host_only=True)  # 4 quadruplets: the overlap-staged tile kernel
    assert four.info.lattice == 1 and four.info.n_quads == 4 and four.lookup_kernel(4096, 4096) == 2
    assert bf.Plan(8.0, 0.1, 24, 16, 4, host_only=True).lookup_kernel(1080, 1920) == 1
    assert bf.Plan(23.3, 0.1, 70, 8, 4, host_only=True).lookup_kernel(300, 300) == 0
    assert bf.Plan(3.0, 0.1, 9, 8, 4, host_only=True, direct=True).lookup_kernel(64, 64) == -1
    with pytest.raises(bf.BFError):
        cfg3.lookup_kernel(0, 5)
    # table-kernel wave forms 0, 1, 2 (a range term, a table, a cosine or sine pair); nothing else
    try:
        for ka_one in (0, 1, 2):
            cfg3.set_tuning(4096, 4096, 576, 2, ka_one)
        for bad in (-1, 3):
            with pytest.raises(bf.BFError):
                cfg3.set_tuning(4096, 4096, 576, 2, bad)
    finally:
        bf.lib().bf_autotune_clear()


def test_symmetric_taps_pair_into_quadruplets():
    """The expansion is symmetric on each axis, so every tap (dy, dx) has
    partners (1-dy, dx), (dy, 1-dx), (1-dy, 1-dx) with weights -w, -w, w up to
    rounding of the fit: all taps group into quadruplets."""
    for ss, r, ns, sr, nr in CONFIGS:
        p = bf.Plan(ss, sr, r, nr, ns, host_only=True)
        dy, dx, w = p.taps()
        d = {(a, b): c for a, b, c in zip(dy.tolist(), dx.tolist(), w.tolist())}
        for (a, b), c in d.items():
            assert abs(d[(1 - a, b)] + c) <= 1e-12 * abs(c)
            assert abs(d[(a, 1 - b)] + c) <= 1e-12 * abs(c)
            assert abs(d[(1 - a, 1 - b)] - c) <= 1e-12 * abs(c)
        assert p.info.n_quads * 4 == len(d)


@pytest.mark.parametrize("kw", [dict(sigma_s=0.0, sigma_r=0.1), dict(sigma_s=3.0, sigma_r=-1.0),
                                dict(sigma_s=float("nan"), sigma_r=0.1),
                                dict(sigma_s=3.0, sigma_r=0.1, n_range=0),
                                dict(sigma_s=3.0, sigma_r=0.1, n_range=65),
                                dict(sigma_s=3.0, sigma_r=0.1, n_spatial=0),
                                dict(sigma_s=3.0, sigma_r=0.1, radius=9, n_spatial=26),
                                dict(sigma_s=3.0, sigma_r=0.1, radius=-1),
                                dict(sigma_s=3.0, sigma_r=0.1, tile=100)])
def test_invalid_plan_arguments(kw):
    kw.setdefault("radius", 9)
    with pytest.raises(bf.BFError) as e:
        bf.Plan(host_only=True, **kw)
    assert e.value.status == bf.BF_ERR_INVALID_ARG


def test_default_radius_and_unsupported():
    p = bf.Plan(3.0, 0.1, 0, 8, 4, host_only=True)
    assert p.info.radius == int(np.ceil(3.0 * np.sqrt(2 * np.log(100))))
    p = bf.Plan(3.0, 0.1, 0, 8, 4, host_only=True, kernel_s="exponential")
    assert p.info.radius == int(np.ceil(3.0 * np.log(100)))
    p = bf.Plan(3.0, 0.1, 9, 8, 4, host_only=True, kernel_r="exponential")
    assert abs(p.info.T_r - 0.1 * np.log(100)) < 1e-15
    h = ctypes.c_void_p()
    st = bf.lib().bf_plan_create(ctypes.byref(h), 2, 0, 3.0, 0.1, 9, bf._Terms(8, 4), None)
    assert st == bf.BF_ERR_UNSUPPORTED
    st = bf.lib().bf_plan_create(ctypes.byref(h), 0, 7, 3.0, 0.1, 9, bf._Terms(8, 4), None)
    assert st == bf.BF_ERR_UNSUPPORTED
    st = bf.lib().bf_plan_create(ctypes.byref(h), -1, 0, 3.0, 0.1, 9, bf._Terms(8, 4), None)
    assert st == bf.BF_ERR_INVALID_ARG
    # the cell fit of a non-separable K_s is bounded in radius
    st = bf.lib().bf_plan_create(ctypes.byref(h), 1, 0, 3.0, 0.1, 600, bf._Terms(8, 4), None)
    assert st == bf.BF_ERR_UNSUPPORTED


KIND_CASES = [("exponential", "gaussian", 3.0, 9, 4, 0.1, 8), ("exponential", "exponential", 2.0, 8, 6, 0.15, 10),
              ("gaussian", "exponential", 3.0, 9, 4, 0.1, 8), ("exponential", "exponential", 5.0, 23, 9, 0.1, 16),
              ("exponential", "gaussian", 1.0, 3, 9, 0.3, 4)]


@pytest.mark.parametrize("ks,kr,ss,r,ns,sr,nr", KIND_CASES)
def test_kernel_kinds_match_oracle(ks, kr, ss, r, ns, sr, nr):
    """The library's fit of the exponential kernels (its own quadrature of the
    cell integrals, prefix-table block sums) against the oracle's; the cell
    integrals agree to the two quadratures' errors, near FP64 rounding)."""
    p = bf.Plan(ss, sr, r, nr, ns, host_only=True, kernel_s=ks, kernel_r=kr)
    o = oracle.make_plan(ss, r, ns, sr, nr, kind_s=ks, kind_r=kr)
    assert p.spatial_groups() == o.spatial.selected
    assert np.abs(p.spatial_kernel() - o.Ks).max() <= 1e-12 * np.abs(o.Ks).max()
    k, a, w = p.range_terms()
    assert k.tolist() == o.range.k.tolist()
    assert np.abs(a - o.a).max() <= 1e-13
    assert np.abs(w - o.omega).max() <= 1e-13
    info = p.info
    assert abs(info.T - o.range.T) < 1e-15
    # both kernels are symmetric: every tap pairs into a quadruplet
    assert info.n_single == 0 and 4 * info.n_quads == info.n_taps
    # the taps reproduce the oracle's rectangle correlation
    dy, dx, tw = p.taps()
    g = synth.gen_image(40, 37, 4, 0.05, 3).astype(np.float64) - 0.3
    S = _excl_sat(g)
    ys, xs = np.mgrid[0:40, 0:37]
    corr = np.zeros(g.shape)
    for a_, b_, c_ in zip(dy, dx, tw):
        corr += c_ * S[np.clip(ys + a_, 0, 40), np.clip(xs + b_, 0, 37)]
    ref = oracle.correlate_rects(g, o.rects)
    assert np.abs(corr - ref).max() < 1e-7


def test_filter_rejects_bad_calls_without_touching_the_device():
    p = bf.Plan(3.0, 0.1, 9, 8, 4, host_only=True)
    L = bf.lib()
    buf_in, buf_out = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x90000)
    assert L.bf_filter(p.handle, buf_in, buf_out, 16, 16, None) == bf.BF_ERR_INVALID_ARG  # host-only plan
    assert L.bf_filter(None, buf_in, buf_out, 16, 16, None) == bf.BF_ERR_INVALID_ARG
    assert L.bf_workspace_size(p.handle, 0, 5, ctypes.byref(ctypes.c_size_t())) == bf.BF_ERR_INVALID_ARG
    assert L.bf_workspace_size(p.handle, 40000, 5, ctypes.byref(ctypes.c_size_t())) == bf.BF_ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert L.bf_workspace_size(p.handle, 1080, 1920, ctypes.byref(n)) == bf.BF_OK and n.value > 0
    assert L.bf_autotune(p.handle, 64, 64, 3, None, None) == bf.BF_ERR_INVALID_ARG  # host-only plan
    assert L.bf_plan_destroy(None) == bf.BF_OK
    assert bf.status_string(bf.BF_ERR_DEVICE) == "BF_ERR_DEVICE"


def test_batch_workspace_is_the_sum_of_aligned_parts():
    """A batch keeps every image's tables in its own 256-byte aligned region
    after 256 bytes of work-queue heads."""
    ps = [bf.Plan(3.0, 0.1, 9, 8, 4, host_only=True), bf.Plan(8.0, 0.2, 24, 8, 6, host_only=True)]
    shapes = [(300, 200), (1080, 1920), (1, 1)]
    plans = [ps[0], ps[1], ps[0]]
    total = bf.batch_workspace_size(plans, shapes)
    parts = [p.workspace_size(h, w) for p, (h, w) in zip(plans, shapes)]
    assert total == 1024 + sum((b + 255) // 256 * 256 for b in parts)  # 1024: the lookup work-queue heads


def test_precomputed_tables_compatibility():
    """Tables built under one plan serve plans with the same input type, a
    radius no larger, no lone taps, and range terms equal to the first terms
    of the tables' (same k, same T)."""
    t = bf.Plan(16.0, 0.05, 48, 32, 4, host_only=True)
    for ss in (2.0, 4.0, 8.0, 16.0):
        for sr, nr in ((0.05, 32), (0.1, 16), (0.2, 8), (0.3, 8)):
            assert bf.precomputed_compatible(t, bf.Plan(ss, sr, int(3 * ss), nr, 4, host_only=True)) == bf.BF_OK
    assert bf.precomputed_compatible(t, bf.Plan(20.0, 0.1, 60, 16, 4, host_only=True)) == bf.BF_ERR_INVALID_ARG
    small = bf.Plan(8.0, 0.1, 24, 8, 4, host_only=True)
    assert bf.precomputed_compatible(small, bf.Plan(8.0, 0.1, 24, 16, 4, host_only=True)) == bf.BF_ERR_INVALID_ARG
    # T = max(T_r, 1) grows past 1 for sigma_r = 0.5: other frequencies
    assert bf.precomputed_compatible(t, bf.Plan(8.0, 0.5, 24, 8, 4, host_only=True)) == bf.BF_ERR_INVALID_ARG
    assert bf.precomputed_compatible(t, bf.Plan(8.0, 0.1, 24, 8, 4, dtype="u8", host_only=True)) == bf.BF_ERR_INVALID_ARG


def test_direct_summation_choice():
    """Direct summation on request (radius <= 32) and, with the automatic
    flag, only where its cost model beats the expansion: small windows with
    many range terms."""
    assert bf.Plan(3.0, 0.1, 9, 8, 4, host_only=True, direct=True).info.direct == 1
    assert bf.Plan(3.0, 0.1, 9, 8, 4, host_only=True).info.direct == 0
    assert bf.Plan(2.0, 0.05, 6, 32, 4, host_only=True, direct="auto").info.direct == 1
    assert bf.Plan(8.0, 0.1, 24, 16, 6, host_only=True, direct="auto").info.direct == 0
    assert bf.Plan(16.0, 0.05, 48, 32, 8, host_only=True, direct="auto").info.direct == 0
    with pytest.raises(bf.BFError) as e:
        bf.Plan(12.0, 0.1, 36, 8, 4, host_only=True, direct=True)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    p = bf.Plan(2.0, 0.1, 6, 8, 4, host_only=True, direct=True)
    assert p.workspace_size(500, 700) == 0


def test_range_box_plan_rules():
    """BF_FLAG_RANGE_BOX: 8-bit input only, T = T_r whatever span, radius <= 48,
    not with the direct flags; no workspace, no pre-computed tables."""
    p = bf.Plan(3.0, 0.1, 9, 5, 4, dtype="u8", range_box=True, span=2.0, host_only=True)
    assert p.info.range_box == 1 and abs(p.info.T - p.info.T_r) < 1e-15
    assert p.info.box_levels == int(np.floor(255 * 0.1 * np.sqrt(2 * np.log(100))))
    assert p.workspace_size(1080, 1920) == 0
    assert p.info.box_tile == 64
    assert bf.Plan(16.0, 0.1, 48, 5, 4, dtype="u8", range_box=True, host_only=True).info.box_tile == 32
    wide = bf.Plan(3.0, 0.5, 9, 5, 4, dtype="u8", range_box=True, host_only=True)
    assert wide.info.box_levels == 255
    with pytest.raises(bf.BFError) as e:
        bf.Plan(3.0, 0.1, 9, 5, 4, dtype="f32", range_box=True, host_only=True)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.Plan(20.0, 0.1, 60, 5, 4, dtype="u8", range_box=True, host_only=True)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    with pytest.raises(bf.BFError) as e:
        bf.Plan(3.0, 0.1, 9, 5, 4, dtype="u8", range_box=True, direct=True, host_only=True)
    assert e.value.status == bf.BF_ERR_INVALID_ARG
    o = oracle.make_plan(3.0, 9, 4, 0.1, 5, span=0.0)
    k, a, w = p.range_terms()
    assert k.tolist() == o.range.k.tolist() and np.abs(a - o.a).max() < 1e-13


def test_reduced_precision_plan_rules():
    """BF_PREC_REDUCED: FP16 term images as workspace (n_images H W 2 bytes),
    not with the direct or range-box flags, radius <= 48."""
    p = bf.Plan(3.0, 0.1, 9, 8, 4, precision="reduced", host_only=True)
    assert p.info.reduced == 1
    assert p.workspace_size(1080, 1920) == (p.info.n_images * 1080 * 1920 * 2 + 255) // 256 * 256
    assert bf.Plan(3.0, 0.1, 9, 8, 4, host_only=True).info.reduced == 0
    with pytest.raises(bf.BFError) as e:
        bf.Plan(3.0, 0.1, 9, 8, 4, precision="reduced", direct=True, host_only=True)
    assert e.value.status == bf.BF_ERR_INVALID_ARG
    with pytest.raises(bf.BFError) as e:
        bf.Plan(3.0, 0.1, 9, 8, 4, dtype="u8", precision="reduced", range_box=True, host_only=True)
    assert e.value.status == bf.BF_ERR_INVALID_ARG
    with pytest.raises(bf.BFError) as e:
        bf.Plan(20.0, 0.1, 60, 8, 4, precision="reduced", host_only=True)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED


def test_level_fold_plan_rules():
    """BF_FLAG_LEVEL_FOLD: 8-bit input only, the default regime's series
    (T = max(T_r, span)), window open to every level difference."""
    p = bf.Plan(3.0, 0.1, 9, 8, 4, dtype="u8", level_fold=True, host_only=True)
    assert p.info.level_fold == 1 and p.info.range_box == 0 and p.info.box_levels == 255
    assert abs(p.info.T - 1.0) < 1e-15 and p.workspace_size(1080, 1920) == 0
    with pytest.raises(bf.BFError) as e:
        bf.Plan(3.0, 0.1, 9, 8, 4, dtype="f32", level_fold=True, host_only=True)
    assert e.value.status == bf.BF_ERR_UNSUPPORTED
    for kw in (dict(range_box=True), dict(direct=True), dict(precision="reduced")):
        with pytest.raises(bf.BFError) as e:
            bf.Plan(3.0, 0.1, 9, 8, 4, dtype="u8", level_fold=True, host_only=True, **kw)
        assert e.value.status == bf.BF_ERR_INVALID_ARG


def _table_cases():
    K = synth.kernels
    return [
        (K.cauchy_spatial(9, 3.0), K.tukey_range(0.2, 1 / 255.0), 1 / 255.0, 6, 8),
        (K.gaussian_spatial(24, 8.0), K.cauchy_range(0.05, 0.005, 201), 0.005, 6, 16),
        (K.cauchy_spatial(48, 10.0), K.tukey_range(0.3, 0.01), 0.01, 8, 32),
        (K.cauchy_spatial(3, 1.0), K.cauchy_range(0.1, 0.01, 101), 0.01, 4, 8),
    ]


@pytest.mark.parametrize("case", range(4))
def test_tabulated_kernels_match_oracle(case):
    """Tabulated kernels: the library's exact cell sums and closed-form cosine
    coefficients against the oracle's (exact overlap matrices, per-piece
    integrals), and the compiled taps against the oracle's rectangles."""
    ks, kr, step, ns, nr = _table_cases()[case]
    p = bf.Plan.tabulated(ks, kr, step, n_range=nr, n_spatial=ns, host_only=True)
    o = oracle.make_table_plan(ks, kr, step, ns, nr)
    assert p.spatial_groups() == o.spatial.selected
    assert np.abs(p.spatial_kernel() - o.Ks).max() <= 1e-13 * np.abs(o.Ks).max()
    k, a, w = p.range_terms()
    assert k.tolist() == o.range.k.tolist()
    assert np.abs(a - o.a).max() <= 1e-13
    assert np.abs(w - o.omega).max() <= 1e-12
    info = p.info
    assert info.T_r == o.range.T_r and info.T == o.range.T
    assert info.radius == (ks.shape[0] - 1) // 2
    assert info.n_single == 0 and 4 * info.n_quads == info.n_taps
    dy, dx, tw = p.taps()
    g = synth.gen_image(40, 37, 4, 0.05, 3).astype(np.float64) - 0.3
    S = _excl_sat(g)
    ys, xs = np.mgrid[0:40, 0:37]
    corr = np.zeros(g.shape)
    for a_, b_, c_ in zip(dy, dx, tw):
        corr += c_ * S[np.clip(ys + a_, 0, 40), np.clip(xs + b_, 0, 37)]
    assert np.abs(corr - oracle.correlate_rects(g, o.rects)).max() < 1e-7


def test_tabulated_plan_rules():
    """Table checks, and which flags a tabulated plan takes."""
    K = synth.kernels
    ks, kr = K.cauchy_spatial(6, 2.0), K.tukey_range(0.2, 0.01)
    L = bf.lib()
    dp = ctypes.POINTER(ctypes.c_double)

    def create(ks_, kr_, step, flags=bf.BF_FLAG_HOST_ONLY, dtype=0, precision=0, n=(8, 4)):
        h = ctypes.c_void_p()
        ks_ = np.ascontiguousarray(ks_, dtype=np.float64)
        kr_ = np.ascontiguousarray(kr_, dtype=np.float64)
        opts = bf._Opts(dtype, precision, 0.0, 0.0, 0, flags)
        st = L.bf_plan_create_tabulated(ctypes.byref(h), ks_.ctypes.data_as(dp), (ks_.shape[0] - 1) // 2,
                                        kr_.ctypes.data_as(dp), len(kr_), step, bf._Terms(*n), ctypes.byref(opts))
        if st == bf.BF_OK:
            L.bf_plan_destroy(h)
        return st

    assert create(ks, kr, 0.01) == bf.BF_OK
    bad = ks.copy()
    bad[0, 1] *= 1.5                                   # not even in dx
    assert create(bad, kr, 0.01) == bf.BF_ERR_INVALID_ARG
    bad = ks.copy()
    bad[0, 0] = bad[0, -1] = bad[-1, 0] = bad[-1, -1] = -0.1
    assert create(bad, kr, 0.01) == bf.BF_ERR_INVALID_ARG
    bad = ks.copy()
    bad[6, 6] = 0.0                                    # centre
    assert create(bad, kr, 0.01) == bf.BF_ERR_INVALID_ARG
    bad = ks.copy()
    bad[3, 3] = bad[3, 9] = bad[9, 3] = bad[9, 9] = np.nan
    assert create(bad, kr, 0.01) == bf.BF_ERR_INVALID_ARG
    assert create(ks, kr[:1], 0.01) == bf.BF_ERR_INVALID_ARG
    assert create(ks, kr, 0.0) == bf.BF_ERR_INVALID_ARG
    assert create(ks, kr, np.inf) == bf.BF_ERR_INVALID_ARG
    assert create(ks, np.concatenate([[0.0], kr[1:]]), 0.01) == bf.BF_ERR_INVALID_ARG
    assert create(ks, np.full(20000, 0.5), 1e-4) == bf.BF_ERR_INVALID_ARG   # above 16385 samples
    assert create(ks, kr, 0.01, n=(0, 4)) == bf.BF_ERR_INVALID_ARG
    h = ctypes.c_void_p()
    assert L.bf_plan_create_tabulated(ctypes.byref(h), None, 6, kr.ctypes.data_as(dp), len(kr), 0.01,
                                      bf._Terms(8, 4), None) == bf.BF_ERR_INVALID_ARG
    # direct summation evaluates analytic kernels only; the automatic choice never takes it
    assert create(ks, kr, 0.01, flags=bf.BF_FLAG_HOST_ONLY | bf.BF_FLAG_DIRECT) == bf.BF_ERR_UNSUPPORTED
    p = bf.Plan.tabulated(ks, kr, 0.01, n_range=32, n_spatial=4, host_only=True, direct="auto")
    assert p.info.direct == 0
    # a rough table keeps energy in fine Haar levels: at r = 19 (levels up to
    # 4) more tap offsets per axis than the kernels take
    rough = np.random.default_rng(1).uniform(0.1, 1.0, (20, 20))
    rough = np.concatenate([rough[:0:-1], rough])
    rough = np.concatenate([rough[:, :0:-1], rough], axis=1)
    assert create(rough, kr, 0.01, n=(8, 6)) == bf.BF_ERR_UNSUPPORTED
    # at r = 9 (levels up to 3) the same roughness gives 16 offsets per axis,
    # 64 quadruplets: the per-pixel lookup kernel takes them
    p = bf.Plan.tabulated(rough[10:29, 10:29], kr, 0.01, n_range=8, n_spatial=6, host_only=True)
    assert p.info.n_taps == 256 and p.info.n_quads == 64 and p.info.lookup_kernel == 0
    # the other regimes take tables
    p = bf.Plan.tabulated(ks, K.tukey_range(0.2, 1 / 255.0), 1 / 255.0, n_range=5, n_spatial=4, dtype="u8",
                          range_box=True, host_only=True)
    assert p.info.range_box == 1 and p.info.T == p.info.T_r == 51 / 255.0
    p = bf.Plan.tabulated(ks, kr, 0.01, n_range=8, n_spatial=4, dtype="u8", level_fold=True, host_only=True)
    assert p.info.level_fold == 1 and p.info.T == 1.0
    p = bf.Plan.tabulated(ks, kr, 0.01, n_range=8, n_spatial=4, precision="reduced", host_only=True)
    assert p.info.reduced == 1


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: a multi-GPU request exits with a message
    before anything touches a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_empty_batch_is_a_no_op():
    """A batch of no images: the workspace is the queue heads alone and the
    call succeeds without touching a device; a negative count is an error."""
    L = bf.lib()
    vp = ctypes.c_void_p
    plans = (vp * 1)()
    hw = (ctypes.c_int * 1)()
    size = ctypes.c_size_t()
    assert L.bf_batch_workspace_size(plans, 0, hw, hw, ctypes.byref(size)) == bf.BF_OK
    assert size.value == 1024  # the lookup work-queue heads only
    ptrs = (vp * 1)()
    assert L.bf_filter_batch(plans, 0, ptrs, ptrs, hw, hw, None, 0, None) == bf.BF_OK
    assert L.bf_filter_batch(plans, -1, ptrs, ptrs, hw, hw, None, 0, None) == bf.BF_ERR_INVALID_ARG


@pytest.mark.parametrize("span,step,n", [(2.0, 0.01, 31), (5.0, 0.05, 61), (1.0, 1 / 255.0, 256)])
def test_tabulated_range_fit_with_wider_series_interval(span, step, n):
    """The range table's coefficients when the series interval T = max(T_r,
    span) extends past the table (zero there) or the table covers every level
    difference of 8-bit data: library against oracle."""
    ks = synth.kernels.cauchy_spatial(6, 2.0)
    kr = synth.kernels.cauchy_range(0.1, step, n)
    p = bf.Plan.tabulated(ks, kr, step, n_range=24, n_spatial=4, span=span, host_only=True)
    o = oracle.make_table_plan(ks, kr, step, 4, 24, span=span)
    k, a, w = p.range_terms()
    assert p.info.T == o.range.T == max((n - 1) * step, span)
    assert k.tolist() == o.range.k.tolist()
    assert np.abs(a - o.a).max() <= 1e-13
    assert np.abs(w - o.omega).max() <= 1e-12
