"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerance: max-abs 1e-4 on [0, 1] intensities against the expanded form
(oracle T3 on whole images, T2 on sampled pixels at 4096^2).  The plain path
keeps exact int32 tables and FP32 tap sums, so its error is far below that;
the tests also assert a tighter 5e-5 to catch regressions early.
"""
import numpy as np
import pytest

import oracle
import synth
from synth.images import CONFIGS

pytestmark = pytest.mark.gpu

TOL = 1e-4
TIGHT = 5e-5


@pytest.fixture(scope="module")
def torch_dev(gpu):
    import torch
    return torch


def _bf():
    from paper_1803_00004_amd import bf
    return bf


def _run(torch, plan, I, **kw):
    bf = _bf()
    dev = torch.from_numpy(np.ascontiguousarray(I)).cuda()
    out = bf.filter(plan, dev, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _plans(ss, r, ns, sr, nr, dtype="f32", tile=0):
    bf = _bf()
    return bf.Plan(ss, sr, r, nr, ns, dtype=dtype, tile=tile), oracle.make_plan(ss, r, ns, sr, nr)


def _report(name, err):
    print("[parity] %s max-abs %.3e" % (name, err), flush=True)


def test_cfg1_full_image(torch_dev):
    c = CONFIGS["cfg1_256"]
    I = synth.config_image("cfg1_256")
    gp, op = _plans(c["sigma_s"], c["radius"], c["n_spatial"], c["sigma_r"], c["n_range"])
    out = _run(torch_dev, gp, I)
    ref = oracle.expanded_box(I, op)
    err = np.abs(out - ref).max()
    _report("cfg1 256^2 vs T3", err)
    true_err = np.abs(out - oracle.true_bf(I, c["sigma_s"], c["radius"], c["sigma_r"])).max()
    _report("cfg1 256^2 vs true BF (reported)", true_err)
    assert err <= TIGHT


@pytest.mark.parametrize("H,W,tile,ss,r,ns,sr,nr", [
    (300, 700, 128, 3.0, 9, 4, 0.1, 8),     # several tiles, ragged tails
    (197, 263, 64, 4.0, 12, 6, 0.2, 8),     # ragged, tile smaller than 2r+1 halo
    (130, 129, 64, 2.0, 6, 4, 0.3, 8),
    (7, 13, 0, 3.0, 9, 4, 0.1, 8),          # image smaller than the window
    (1, 1, 0, 3.0, 9, 4, 0.1, 8),
    (1, 77, 0, 2.0, 6, 4, 0.1, 8),
    (77, 1, 0, 2.0, 6, 4, 0.1, 8),
    (64, 64, 0, 3.0, 10, 3, 0.1, 5),        # odd N_s: asymmetric-free but 3 groups
    (96, 80, 64, 2.0, 6, 9, 0.05, 32),      # many groups / terms
])
def test_shapes_vs_oracle(torch_dev, H, W, tile, ss, r, ns, sr, nr):
    I = synth.gen_image(H, W, 5, 0.03, H * 1000 + W)
    gp, op = _plans(ss, r, ns, sr, nr, tile=tile)
    out = _run(torch_dev, gp, I)
    ref = oracle.expanded_box(I, op)
    err = np.abs(out - ref).max()
    _report("%dx%d tile %d r %d" % (H, W, gp.geometry(H, W)[0], r), err)
    assert err <= TIGHT


# Radii whose staged region (64 + 2r + 1 columns) selects each single-buffered
# pitch class of the LDS tile lookup kernel, with 4, 8 and 12 quadruplets:
# (H, W, sigma_s, r, N_s, sigma_r, N_r, pitch, quadruplets).
WIDE_CASES = [
    (300, 500, 13.0, 40, 6, 0.1, 16, 160, 8),
    (301, 499, 15.0, 45, 8, 0.1, 8, 160, 12),
    (290, 470, 17.0, 52, 4, 0.2, 8, 176, 4),
    (310, 520, 20.0, 60, 6, 0.2, 8, 192, 8),
    (257, 333, 21.0, 63, 8, 0.3, 8, 192, 12),
]


@pytest.mark.parametrize("H,W,ss,r,ns,sr,nr,pitch,nq", WIDE_CASES)
def test_wide_regions_vs_oracle(torch_dev, H, W, ss, r, ns, sr, nr, pitch, nq):
    """Every pitch class of the LDS tile kernel for regions wider than 128
    columns (overlap-staged at pitch 160 and, up to 164 region rows, 176;
    single-buffered beyond) against T3 on whole images."""
    I = synth.gen_image(H, W, 7, 0.03, 7 * r + H)
    gp, op = _plans(ss, r, ns, sr, nr)
    info = gp.info
    assert (info.lookup_kernel, info.lds_pitch, info.lds_double_buffered, info.n_quads) == (1, pitch, 0, nq)
    out = _run(torch_dev, gp, I)
    ref = oracle.expanded_box(I, op)
    err = np.abs(out - ref).max()
    _report("%dx%d r %d pitch %d quads %d" % (H, W, r, pitch, nq), err)
    assert err <= TIGHT


@pytest.mark.parametrize("ss,r,ns,pitch", [(16.0, 48, 8, 176), (13.0, 40, 6, 160)])
@pytest.mark.parametrize("H,W", [(1, 1), (1, 200), (200, 1), (63, 65), (129, 70), (64, 64), (65, 257)])
def test_overlap_staging_small_and_ragged(torch_dev, ss, r, ns, pitch, H, W):
    """The overlap-staged lookup (both layouts, register and direct rows) on
    images smaller than the window, single rows and columns and ragged tile
    edges, against T3 on the whole image."""
    I = synth.gen_image(H, W, 3, 0.03, 11 * H + W)
    gp, op = _plans(ss, r, ns, 0.1, 8)
    assert gp.info.lds_pitch == pitch and gp.info.lds_double_buffered == 0
    # the LDS tile kernel pinned (the default of the 12-quadruplet plan is the
    # lattice kernel, which must give the same bits)
    default = _run(torch_dev, gp, I)
    gp.set_tuning(H, W, gp.geometry(H, W)[0], 1, 0)
    out = _run(torch_dev, gp, I)
    _bf().lib().bf_autotune_clear()
    ref = oracle.expanded_box(I, op)
    err = np.abs(out - ref).max()
    _report("overlap %dx%d r %d" % (H, W, r), err)
    assert err <= TIGHT
    assert np.array_equal(out, default)


def test_wide_regions_in_one_batch(torch_dev):
    """All pitch classes (and a double-buffered plan) in one batch: each output
    is bitwise its single-image result."""
    import torch
    bf = _bf()
    plans, imgs = [], []
    for (H, W, ss, r, ns, sr, nr, _, _) in WIDE_CASES + [(200, 260, 3.0, 9, 4, 0.1, 8, 128, 4)]:
        plans.append(bf.Plan(ss, sr, r, nr, ns))
        imgs.append(torch.from_numpy(synth.gen_image(H, W, 5, 0.03, 11 * r)).cuda())
    singles = [bf.filter(p, I).clone() for p, I in zip(plans, imgs)]
    outs = bf.filter_batch(plans, imgs)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(outs, singles)):
        assert torch.equal(a, b), i


# Plans whose quadruplet rows lie on a lattice, with the step s, the rows M
# (after splitting steps above 16) and the LDS pitch of the lattice kernel:
# (H, W, sigma_s, r, N_s, sigma_r, N_r, dtype, table tile, s).
LATTICE_CASES = [
    (300, 517, 16.0, 48, 8, 0.05, 32, "f32", 512, 12),   # M 4, N 4, pitch 192 (the 12 boxes of N_s = 8)
    (211, 333, 16.0, 48, 8, 0.05, 32, "u8", 384, 12),    # the same boxes, 8-bit input, whole lattice tiles
    (333, 290, 16.0, 48, 4, 0.1, 8, "u8", 128, 12),      # step 24 split in two (M 3); tiles clip at 128
    (261, 389, 8.0, 24, 6, 0.1, 16, "f32", 64, 6),       # two groups of 6 waves, 64-row table tiles
    (200, 300, 3.0, 9, 4, 0.1, 8, "u8", 64, 5),          # M 2, N 2, three groups
    (130, 129, 2.0, 6, 4, 0.3, 8, "f32", 64, 3),         # five groups of 3 waves
    (310, 520, 13.0, 40, 6, 0.2, 8, "f32", 320, 10),     # pitch 192, step 10, 80-row lattice tiles
    (7, 13, 16.0, 48, 8, 0.05, 32, "f32", 64, 12),       # image smaller than the window
    (1, 1, 13.0, 40, 6, 0.1, 16, "f32", 64, 10),
]


@pytest.mark.parametrize("H,W,ss,r,ns,sr,nr,dt,tile,step", LATTICE_CASES)
def test_lattice_kernel_vs_oracle(torch_dev, H, W, ss, r, ns, sr, nr, dt, tile, step):
    """The lattice lookup kernel against T3, and bitwise against the LDS tile
    kernel on the same tables (both sum each pixel's boxes in (dy, dx)
    order)."""
    import torch
    bf = _bf()
    I = synth.gen_image_u8(H, W, 5, 0.03, H + r) if dt == "u8" else synth.gen_image(H, W, 5, 0.03, H + r)
    gp, op = bf.Plan(ss, sr, r, nr, ns, dtype=dt), oracle.make_plan(ss, r, ns, sr, nr)
    assert gp.info.lattice == 1 and gp.info.lattice_step == step
    dev = torch.from_numpy(np.ascontiguousarray(I)).cuda()
    gp.set_tuning(H, W, tile, 2, 0)
    lat = bf.filter(gp, dev).clone()
    ref = oracle.expanded_box(I, op)
    err = np.abs(lat.cpu().numpy().astype(np.float64) - ref).max()
    _report("lattice %dx%d r %d s %d tile %d %s" % (H, W, r, step, tile, dt), err)
    assert err <= TIGHT
    gp.set_tuning(H, W, tile, 1, 1)  # LDS tile kernel, single-buffered (one table per table-kernel wave)
    other = bf.filter(gp, dev)
    torch.cuda.synchronize()
    assert torch.equal(lat, other)
    bf.lib().bf_autotune_clear()


def test_lattice_plans_in_one_batch(torch_dev):
    """Lattice plans of several classes (pitch, rows, columns) beside LDS tile
    and per-pixel plans in one batch: each output is bitwise its single-image
    result."""
    import torch
    bf = _bf()
    specs = [(300, 517, 16.0, 48, 8, 0.05, 32), (333, 290, 16.0, 48, 4, 0.1, 8), (310, 520, 20.0, 60, 6, 0.2, 8),
             (257, 301, 13.0, 40, 6, 0.1, 16), (200, 260, 3.0, 9, 4, 0.1, 8), (150, 170, 15.0, 45, 8, 0.1, 8),
             (120, 90, 23.3, 70, 4, 0.1, 8)]
    plans, imgs = [], []
    for H, W, ss, r, ns, sr, nr in specs:
        plans.append(bf.Plan(ss, sr, r, nr, ns))
        imgs.append(torch.from_numpy(synth.gen_image(H, W, 5, 0.03, 3 * r + H)).cuda())
    kinds = sorted(set(p.info.default_lookup for p in plans))
    assert kinds == [0, 1, 2, 3], kinds
    # the first plan (12 boxes) keeps the lattice kernel as its untuned default (one launch of its own in
    # the batch); every other plan that can use the lattice kernel is tuned to it (the persistent form)
    assert plans[0].info.default_lookup == 3
    for p, (H, W, *_) in list(zip(plans, specs))[1:]:
        if p.info.lattice:
            p.set_tuning(H, W, p.geometry(H, W)[0], 2, 0)
    singles = [bf.filter(p, I).clone() for p, I in zip(plans, imgs)]
    outs = bf.filter_batch(plans, imgs)
    torch.cuda.synchronize()
    bf.lib().bf_autotune_clear()
    for i, (a, b) in enumerate(zip(outs, singles)):
        assert torch.equal(a, b), i


def test_u8_input(torch_dev):
    Iu = synth.gen_image_u8(200, 300, 8, 0.03, 9)
    gp, op = _plans(3.0, 9, 4, 0.1, 8, dtype="u8", tile=128)
    out = _run(torch_dev, gp, Iu)
    ref = oracle.expanded_box(Iu, op)
    err = np.abs(out - ref).max()
    _report("u8 200x300", err)
    assert err <= TIGHT


def test_numerator_denominator(torch_dev):
    import torch
    bf = _bf()
    I = synth.gen_image(150, 170, 5, 0.03, 3)
    gp, op = _plans(4.0, 12, 6, 0.1, 16, tile=64)
    dev = torch.from_numpy(I).cuda()
    num = torch.empty_like(dev)
    den = torch.empty_like(dev)
    out = bf.filter(gp, dev, num=num, den=den)
    torch.cuda.synchronize()
    o3, n3, d3 = oracle.expanded_box(I, op, return_parts=True)
    assert np.abs(den.cpu().numpy() - d3).max() <= 1e-6 * np.abs(d3).max()
    assert np.abs(num.cpu().numpy() - n3).max() <= 1e-6 * np.abs(d3).max()
    assert np.abs(out.cpu().numpy() - o3).max() <= TIGHT


def test_constant_image(torch_dev):
    I = np.full((90, 110), 0.37, dtype=np.float32)
    gp, _ = _plans(3.0, 9, 4, 0.1, 8, tile=64)
    out = _run(torch_dev, gp, I)
    assert np.abs(out - 0.37).max() <= 1e-6


def test_sigma_r_infinity_is_spatial_filter(torch_dev):
    from scipy import signal
    I = synth.gen_image(120, 90, 4, 0.02, 5)
    gp, op = _plans(3.0, 9, 4, 1e6, 4, tile=64)
    out = _run(torch_dev, gp, I)
    K = op.Ks[::-1, ::-1]
    Id = I.astype(np.float64)
    ref = signal.correlate2d(Id, K, mode="same") / signal.correlate2d(np.ones_like(Id), K, mode="same")
    assert np.abs(out - ref).max() <= TIGHT


def test_determinism_and_batch_equals_single(torch_dev):
    import torch
    bf = _bf()
    specs = [(3.0, 9, 4, 0.1, 8, 140, 210), (4.0, 12, 4, 0.2, 8, 300, 90), (2.0, 6, 4, 0.05, 32, 64, 64)]
    plans, imgs, singles = [], [], []
    for ss, r, ns, sr, nr, H, W in specs:
        p = bf.Plan(ss, sr, r, nr, ns)
        I = torch.from_numpy(synth.gen_image(H, W, 4, 0.03, H + W)).cuda()
        a = bf.filter(p, I)
        b = bf.filter(p, I)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        plans.append(p)
        imgs.append(I)
        singles.append(a.clone())
    outs = bf.filter_batch(plans, imgs)
    torch.cuda.synchronize()
    for o, s in zip(outs, singles):
        assert torch.equal(o, s)


def _mixed_batch(torch, n=26, seed=5):
    """n requests with their own plans, sizes and input types: f32 and u8,
    ragged shapes, a 1x1 image and a plan whose staged region is too wide
    for LDS (per-pixel lookup kernel)."""
    bf = _bf()
    rng = np.random.default_rng(seed)
    plans, imgs, specs = [], [], []
    cache = {}
    for i in range(n):
        ss = float(rng.choice([2.0, 3.0, 4.0, 8.0]))
        sr = float(rng.choice([0.05, 0.1, 0.2, 0.3]))
        nr = int(min(32, max(8, np.ceil(1.6 / sr))))
        ns = int(rng.choice([4, 6]))
        r = int(3 * ss)
        dtype = "u8" if i % 7 == 3 else "f32"
        H, W = int(rng.integers(40, 330)), int(rng.integers(40, 330))
        if i == 5:
            H = W = 1
        if i == 11:
            ss, r, ns, H, W = 24.0, 70, 4, 200, 180
        key = (ss, r, ns, sr, nr, dtype)
        if key not in cache:
            cache[key] = bf.Plan(ss, sr, r, nr, ns, dtype=dtype)
        plans.append(cache[key])
        specs.append(key)
        if dtype == "u8":
            imgs.append(torch.from_numpy(synth.gen_image_u8(H, W, 4, 0.03, 100 + i)).cuda())
        else:
            imgs.append(torch.from_numpy(synth.gen_image(H, W, 4, 0.03, 100 + i)).cuda())
    return plans, imgs, specs


def test_mixed_batch_is_bitwise_single(torch_dev):
    """More requests than one launch takes (two groups), both input types,
    both lookup kernels: every output equals its single-image call bit for
    bit, and one of them is checked against the oracle."""
    import torch
    bf = _bf()
    plans, imgs, specs = _mixed_batch(torch)
    assert any(p.info.radius == 70 for p in plans)
    singles = [bf.filter(p, I).clone() for p, I in zip(plans, imgs)]
    outs = bf.filter_batch(plans, imgs)
    torch.cuda.synchronize()
    for i, (o, s) in enumerate(zip(outs, singles)):
        assert torch.equal(o, s), i
    j = next(i for i, p in enumerate(plans) if p.info.radius == 70)
    ss, r, ns, sr, nr, _ = specs[j]
    ref = oracle.expanded_box(imgs[j].cpu().numpy(), oracle.make_plan(ss, r, ns, sr, nr))
    err = np.abs(outs[j].cpu().numpy() - ref).max()
    _report("batch member r=70 (per-pixel kernel)", err)
    assert err <= TIGHT


def _fused_group(torch, dtype, seed):
    """A batch group the fused launch takes: double-buffered lookups (radius
    6, 12, 24) beside overlap-staged ones (radius 48, pitch 176), 4 and 6
    spatial terms, ragged sizes over several table tiles and a 1x1 image."""
    bf = _bf()
    rng = np.random.default_rng(seed)
    plans, imgs = [], []
    for i, (ss, ns, nr, sr) in enumerate([(2.0, 4, 8, 0.2), (16.0, 4, 16, 0.1), (8.0, 6, 16, 0.1),
                                          (4.0, 4, 32, 0.05), (16.0, 4, 8, 0.3), (2.0, 6, 8, 0.2)]):
        H, W = (1, 1) if i == 5 else (int(rng.integers(40, 700)), int(rng.integers(40, 700)))
        plans.append(bf.Plan(ss, sr, int(3 * ss), nr, ns, dtype=dtype))
        if dtype == "u8":
            imgs.append(torch.from_numpy(synth.gen_image_u8(H, W, 6, 0.03, seed + i)).cuda())
        else:
            imgs.append(torch.from_numpy(synth.gen_image(H, W, 6, 0.03, seed + i)).cuda())
    return plans, imgs


@pytest.mark.parametrize("dtype", ["f32", "u8"])
def test_fused_batch_is_bitwise_single(torch_dev, dtype):
    """bf_batch_set_fused(1): the group runs as one persistent launch whose
    lookups wait on per-table-tile ready counters; every output equals its
    single-image call bit for bit, twice in a row with new inputs (the
    counters are reset per launch), no wait runs out (the workspace's error
    word stays 0), and one member is checked against the oracle."""
    import torch
    bf = _bf()
    plans, imgs = _fused_group(torch, dtype, 40 if dtype == "f32" else 60)
    shapes = [tuple(I.shape) for I in imgs]
    ws = torch.zeros(bf.batch_workspace_size(plans, shapes), dtype=torch.uint8, device="cuda")
    bf.set_batch_fused(True)
    try:
        for rep in range(2):
            if rep:
                imgs = [I.flip(0).contiguous() for I in imgs]
            singles = [bf.filter(p, I).clone() for p, I in zip(plans, imgs)]
            outs = bf.filter_batch(plans, imgs, ws=ws)
            torch.cuda.synchronize()
            for i, (o, s1) in enumerate(zip(outs, singles)):
                assert torch.equal(o, s1), (rep, i)
            assert int(ws[36:40].view(torch.int32).item()) == 0
    finally:
        bf.set_batch_fused(False)
    j = 1  # radius 48, overlap-staged lookup
    p = plans[j]
    ref = oracle.expanded_box(imgs[j].cpu().numpy(), oracle.make_plan(16.0, 48, 4, 0.1, 16))
    err = np.abs(outs[j].cpu().numpy() - ref).max()
    _report("fused batch member r=48 %s" % dtype, err)
    assert err <= TIGHT


def test_fused_batch_graph_replays(torch_dev):
    """The fused launch (with its counter reset) captured in a graph and
    replayed with new inputs, eager work between the replays: every replay
    equals the single-image calls on its inputs."""
    import torch
    bf = _bf()
    plans, imgs = _fused_group(torch, "f32", 80)
    static_in = [I.clone() for I in imgs]
    outs = [torch.empty(I.shape, dtype=torch.float32, device="cuda") for I in imgs]
    shapes = [tuple(I.shape) for I in imgs]
    ws = torch.zeros(bf.batch_workspace_size(plans, shapes), dtype=torch.uint8, device="cuda")
    bf.set_batch_fused(True)
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            bf.filter_batch(plans, static_in, outs=outs, ws=ws)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            bf.filter_batch(plans, static_in, outs=outs, ws=ws)
        torch.cuda.synchronize()
        for rep in range(3):
            for j, I in enumerate(static_in):
                I.copy_(torch.from_numpy(synth.gen_image(I.shape[0], I.shape[1], 4, 0.03, 700 + 10 * rep + j)))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            eager = [bf.filter(p, I) for p, I in zip(plans, static_in)]
            torch.cuda.synchronize()
            for j in range(len(plans)):
                assert torch.equal(outs[j], eager[j]), (rep, j)
            assert int(ws[36:40].view(torch.int32).item()) == 0
    finally:
        bf.set_batch_fused(False)


def test_batch_graph_replays(torch_dev):
    """A batch captured once in a graph and replayed with new inputs, with
    eager work in between: every replay equals the eager single-image calls
    on the inputs of that replay."""
    import torch
    bf = _bf()
    plans, imgs, _ = _mixed_batch(torch, n=6, seed=8)
    static_in = [I.clone() for I in imgs]
    outs = [torch.empty(I.shape, dtype=torch.float32, device="cuda") for I in imgs]
    shapes = [tuple(I.shape) for I in imgs]
    ws = torch.empty(bf.batch_workspace_size(plans, shapes), dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bf.filter_batch(plans, static_in, outs=outs, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bf.filter_batch(plans, static_in, outs=outs, ws=ws)
    torch.cuda.synchronize()
    for rep in range(4):
        for j, I in enumerate(static_in):
            if I.dtype == torch.uint8:
                I.copy_(torch.from_numpy(synth.gen_image_u8(I.shape[0], I.shape[1], 4, 0.03, 900 + 10 * rep + j)))
            else:
                I.copy_(torch.from_numpy(synth.gen_image(I.shape[0], I.shape[1], 4, 0.03, 900 + 10 * rep + j)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eager = [bf.filter(p, I) for p, I in zip(plans, static_in)]  # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for j in range(len(plans)):
            assert torch.equal(outs[j], eager[j]), (rep, j)
        assert torch.isfinite(junk)


def test_cfg2_full_image(torch_dev):
    c = CONFIGS["cfg2_1080p"]
    I = synth.config_image("cfg2_1080p")
    gp, op = _plans(c["sigma_s"], c["radius"], c["n_spatial"], c["sigma_r"], c["n_range"])
    out = _run(torch_dev, gp, I)
    ref = oracle.expanded_box(I, op)
    err = np.abs(out - ref).max()
    _report("cfg2 1920x1080 vs T3", err)
    assert err <= TIGHT


def _sample_pixels(H, W, n, seed):
    rng = np.random.default_rng(seed)
    ys = rng.integers(0, H, n)
    xs = rng.integers(0, W, n)
    edge_y = [0, 0, H - 1, H - 1, 1, H - 2, H // 2, 48, H - 49, 511, 512, 575, 576, 671, 672]
    edge_x = [0, W - 1, 0, W - 1, W // 2, 1, W - 1, 47, 512, W - 2, 513, 576, 575, 672, 671]
    return np.concatenate([ys, edge_y]).astype(np.int32), np.concatenate([xs, edge_x]).astype(np.int32)


@pytest.mark.parametrize("name", ["cfg3_4096", "cfg5_4096_u8"])
def test_4096_sampled(torch_dev, name):
    """4096^2 in the launch shape an untuned call takes (the lattice lookup
    kernel on 576-row table tiles), sampled against T2 with borders, tile and
    lattice-tile seams; and bitwise against the LDS tile kernel pinned on
    512-row table tiles."""
    c = CONFIGS[name]
    I = synth.config_image(name)
    gp, op = _plans(c["sigma_s"], c["radius"], c["n_spatial"], c["sigma_r"], c["n_range"], dtype=c["dtype"])
    assert gp.info.default_lookup == 3 and gp.geometry(4096, 4096)[0] == 576
    out = _run(torch_dev, gp, I)
    gp.set_tuning(4096, 4096, 512, 1, 0)
    try:
        assert np.array_equal(_run(torch_dev, gp, I), out)
    finally:
        _bf().lib().bf_autotune_clear()
    ys, xs = _sample_pixels(4096, 4096, 1500, 7)
    ref = oracle.expanded_brute(I, op, ys, xs)
    err = np.abs(out[ys, xs] - ref).max()
    _report("%s sampled vs T2" % name, err)
    assert np.isfinite(out).all()
    assert out.min() >= -1e-3 and out.max() <= 1.0 + 1e-3
    assert err <= TIGHT


@pytest.mark.parametrize("H,W,dtype", [(64, 32768, "f32"), (32768, 64, "f32"), (48, 32768, "u8")])
def test_maximum_sizes_sampled(torch_dev, H, W, dtype):
    """The largest image side (32768) on thin images, both orientations and
    both input types: sampled pixels, borders and tile seams included, against
    T2."""
    bf = _bf()
    ss, r, ns, sr, nr = (8.0, 24, 6, 0.1, 16) if dtype == "f32" else (16.0, 48, 8, 0.05, 32)
    I = synth.gen_image_u8(H, W, 20, 0.03, 5) if dtype == "u8" else synth.gen_image(H, W, 20, 0.03, 5)
    p = bf.Plan(ss, sr, r, nr, ns, dtype=dtype)
    try:
        out = _run(torch_dev, p, I)
    finally:
        p.close()  # the plan's workspace
    rng = np.random.default_rng(17)
    ys = np.concatenate([rng.integers(0, H, 1024), [0, H - 1, 0, H - 1, H // 2, min(H - 1, 511), min(H - 1, 512)]])
    xs = np.concatenate([rng.integers(0, W, 1024), [0, W - 1, W - 1, 0, W // 2, min(W - 1, 512), min(W - 1, 511)]])
    ys, xs = ys.astype(np.int32), xs.astype(np.int32)
    ref = oracle.expanded_brute(I, oracle.make_plan(ss, r, ns, sr, nr), ys, xs)
    err = np.abs(out[ys, xs] - ref).max()
    _report("%dx%d %s sampled vs T2" % (H, W, dtype), err)
    assert np.isfinite(out).all()
    assert err <= TIGHT


def test_argument_errors_on_device(torch_dev):
    import ctypes
    import torch
    bf = _bf()
    p = bf.Plan(3.0, 0.1, 9, 8, 4)
    I = torch.rand(64, 64, device="cuda")
    out = torch.empty_like(I)
    need = p.workspace_size(64, 64)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    L = bf.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.bf_filter_ws(p.handle, ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                          64, 64, ctypes.c_void_p(ws.data_ptr()), need - 1, s) == bf.BF_ERR_INVALID_ARG
    assert L.bf_filter(p.handle, ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(I.data_ptr() + 64),
                       64, 64, s) == bf.BF_ERR_INVALID_ARG
    assert L.bf_filter_ws(p.handle, ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                          64, 64, ctypes.c_void_p(ws.data_ptr()), need, s) == bf.BF_OK
    # a workspace overlapping the output is rejected
    big = torch.empty(need + 64 * 64 * 4, dtype=torch.uint8, device="cuda")
    assert L.bf_filter_ws(p.handle, ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(big.data_ptr()),
                          64, 64, ctypes.c_void_p(big.data_ptr() + 256), need, s) == bf.BF_ERR_INVALID_ARG
    torch.cuda.synchronize()
    # batch: an output over another request's input, or over the workspace, is rejected
    I2 = torch.rand(64, 64, device="cuda")
    outs = [torch.empty_like(I), torch.empty_like(I)]
    shapes = [(64, 64), (64, 64)]
    bws = torch.empty(bf.batch_workspace_size([p, p], shapes), dtype=torch.uint8, device="cuda")
    hp = (ctypes.c_void_p * 2)(p.handle.value, p.handle.value)
    hs = (ctypes.c_int * 2)(64, 64)

    def batch(ip, op, wsp):
        return L.bf_filter_batch(hp, 2, (ctypes.c_void_p * 2)(*ip), (ctypes.c_void_p * 2)(*op), hs, hs,
                                 ctypes.c_void_p(wsp), bws.numel(), s)
    assert batch([I.data_ptr(), I2.data_ptr()], [outs[0].data_ptr(), I2.data_ptr()],
                 bws.data_ptr()) == bf.BF_ERR_INVALID_ARG
    assert batch([I.data_ptr(), I2.data_ptr()], [outs[0].data_ptr(), I.data_ptr()],
                 bws.data_ptr()) == bf.BF_ERR_INVALID_ARG
    assert batch([I.data_ptr(), I2.data_ptr()], [outs[0].data_ptr(), bws.data_ptr() + 1024],
                 bws.data_ptr()) == bf.BF_ERR_INVALID_ARG
    assert batch([I.data_ptr(), I2.data_ptr()], [outs[0].data_ptr(), outs[1].data_ptr()],
                 bws.data_ptr()) == bf.BF_OK
    torch.cuda.synchronize()


def test_served_results_equal_alone(torch_dev):
    """A short served stream (Poisson arrivals, mixed sizes and sigmas)
    through the native request loop: every request completes, and each
    result is bitwise the single-image result, whatever it was batched and
    overlapped with."""
    import torch
    bf = _bf()
    from paper_1803_00004_amd import serve
    reqs = synth.gen_stream(n=40, rate_hz=20000.0, seed=14, hw_lo=48, hw_hi=400)
    plans = serve.make_plans(reqs)
    imgs = [torch.from_numpy(serve._gen_one(r)).cuda() for r in reqs]
    outs = [torch.full(I.shape, -1.0, device="cuda") for I in imgs]
    srv = bf.Server(hbm_budget=2 << 30, max_batch=6, n_streams=2)
    done, makespan = serve.run_open_loop(srv, reqs, plans, imgs, outs)
    st = srv.stats()
    srv.close()
    assert sorted(done) == list(range(len(reqs)))
    assert all(c.status == bf.BF_OK for c in done.values())
    assert st.batches < len(reqs)
    alone = [torch.empty_like(o) for o in outs]
    serve.run_plain(reqs, plans, imgs, alone)
    for i in range(len(reqs)):
        assert torch.equal(outs[i], alone[i]), i
    lat = serve.latency_summary(reqs, done)
    print("[served] 40 requests: batches %d, peak in flight %d batches / %d requests, p50 %.2f ms, p99 %.2f ms"
          % (st.batches, st.peak_batches_in_flight, st.peak_requests_in_flight, lat["p50_ms"], lat["p99_ms"]))
    r0 = reqs[3]
    ref = oracle.expanded_box(imgs[3].cpu().numpy(), oracle.make_plan(r0["sigma_s"], r0["radius"], r0["n_spatial"],
                                                                      r0["sigma_r"], r0["n_range"]))
    assert np.abs(outs[3].cpu().numpy() - ref).max() <= TIGHT


def test_tiling_and_autotuning_do_not_change_results(torch_dev):
    """With every tap in a quadruplet the kernels only form exact int32 box
    sums, so the table tile, the lookup kernel's buffering and the
    autotuner's choice leave every output bit unchanged."""
    import torch
    bf = _bf()
    I = torch.from_numpy(synth.gen_image(333, 517, 6, 0.03, 77)).cuda()
    ref = None
    for tile in (64, 128, 256, 512):
        p = bf.Plan(8.0, 0.1, 24, 16, 6, tile=tile)
        o = bf.filter(p, I)
        torch.cuda.synchronize()
        if ref is None:
            ref = o.clone()
        assert torch.equal(o, ref), tile
    p = bf.Plan(8.0, 0.1, 24, 16, 6)
    before = bf.filter(p, I).clone()
    # every launch shape the tuner may pick, pinned by hand
    for tile in (64, 128, 256, 512):
        for kb_single in (0, 1):
            for ka_one in (0, 1, 2):  # a range term, a table, a cosine or sine pair per table wave
                p.set_tuning(333, 517, tile, kb_single, ka_one)
                o = bf.filter(p, I)
                torch.cuda.synchronize()
                assert torch.equal(o, ref), (tile, kb_single, ka_one)
    # the three table-wave forms on 8-bit input (its k = 0 table is the bytes) agree too
    Iu = torch.from_numpy(synth.gen_image_u8(333, 517, 6, 0.03, 79)).cuda()
    pu = bf.Plan(8.0, 0.1, 24, 16, 6, dtype="u8")
    outs_u8 = []
    for ka_one in (0, 1, 2):
        pu.set_tuning(333, 517, 128, 0, ka_one)
        outs_u8.append(bf.filter(pu, Iu).clone())
    torch.cuda.synchronize()
    assert torch.equal(outs_u8[0], outs_u8[1]) and torch.equal(outs_u8[0], outs_u8[2])
    # and in a batch (one table-kernel launch for both images)
    I2 = torch.from_numpy(synth.gen_image(333, 517, 6, 0.03, 78)).cuda()
    p.set_tuning(333, 517, 256, 1, 1)
    outs = bf.filter_batch([p, p], [I, I2])
    torch.cuda.synchronize()
    assert torch.equal(outs[0], ref)
    bf.lib().bf_autotune_clear()
    t = p.autotune(333, 517, reps=3)
    after = bf.filter(p, I)
    torch.cuda.synchronize()
    print("[autotune] 333x517 r=24: tile %d" % t)
    assert t in (64, 128, 256, 512)
    assert torch.equal(before, ref) and torch.equal(after, ref)
    bf.lib().bf_autotune_clear()


def test_precomputed_tables_refilter(torch_dev):
    """Tables built once under one plan serve later filters of the same image
    under other plans (other sigma_s, sigma_r, fewer terms): each result
    matches the oracle for its own plan and the direct filter within 1e-6."""
    import torch
    bf = _bf()
    I_host = synth.gen_image(333, 517, 6, 0.03, 91)
    I = torch.from_numpy(I_host).cuda()
    tp = bf.Plan(8.0, 0.1, 24, 16, 6)
    ws = bf.precompute(tp, I)
    for ss, r, ns, sr, nr, ks, kr in [(8.0, 24, 6, 0.1, 16, "gaussian", "gaussian"),
                                      (4.0, 12, 4, 0.2, 8, "gaussian", "gaussian"),
                                      (2.0, 6, 4, 0.05, 16, "gaussian", "gaussian"),
                                      (6.0, 18, 6, 0.3, 8, "gaussian", "gaussian"),
                                      (3.0, 14, 6, 0.1, 12, "exponential", "exponential")]:
        # the tables hold C.I, S.I, C, S at omega_k = pi k / T: any kernel pair
        # whose series has the same T and a prefix of k reuses them
        p = bf.Plan(ss, sr, r, nr, ns, kernel_s=ks, kernel_r=kr)
        assert bf.precomputed_compatible(tp, p) == bf.BF_OK
        o = bf.filter_precomputed(tp, p, I, ws)
        d = bf.filter(p, I)
        torch.cuda.synchronize()
        ref = oracle.expanded_box(I_host, oracle.make_plan(ss, r, ns, sr, nr, kind_s=ks, kind_r=kr))
        err = np.abs(o.cpu().numpy() - ref).max()
        _report("refilter %s/%s sigma_s %g r %d N %d/%d from precomputed tables" % (ks, kr, ss, r, nr, ns), err)
        assert err <= TIGHT
        assert (o - d).abs().max().item() <= 1e-6


@pytest.mark.parametrize("H,W,ks,kr,ss,r,ns,sr,nr,dtype", [
    (300, 517, "exponential", "exponential", 3.0, 14, 6, 0.1, 12, "f32"),   # default exp radius
    (197, 263, "exponential", "gaussian", 2.0, 8, 4, 0.1, 8, "u8"),
    (130, 129, "gaussian", "exponential", 4.0, 12, 4, 0.2, 16, "f32"),
    (64, 700, "exponential", "exponential", 8.0, 37, 9, 0.05, 24, "u8"),
    (5, 33, "exponential", "exponential", 2.0, 8, 6, 0.15, 10, "f32"),   # image smaller than the window
])
def test_exponential_kernels_vs_oracle(torch_dev, H, W, ks, kr, ss, r, ns, sr, nr, dtype):
    """Other kernel shapes change only the fitted coefficients: the same
    kernels filter them, against the oracle's T3 for the same kernel pair."""
    bf = _bf()
    I = synth.gen_image_u8(H, W, 5, 0.03, H * 3 + W) if dtype == "u8" else synth.gen_image(H, W, 5, 0.03, H * 3 + W)
    p = bf.Plan(ss, sr, r, nr, ns, dtype=dtype, kernel_s=ks, kernel_r=kr)
    o = oracle.make_plan(ss, r, ns, sr, nr, kind_s=ks, kind_r=kr)
    out = _run(torch_dev, p, I)
    ref = oracle.expanded_box(I, o)
    err = np.abs(out - ref).max()
    _report("K_s %s K_r %s %dx%d r %d %s vs T3" % (ks, kr, H, W, r, dtype), err)
    true_err = np.abs(out - oracle.true_bf(I, ss, r, sr, kind_s=ks, kind_r=kr)).max()
    _report("  same vs true BF (reported)", true_err)
    assert err <= TIGHT


@pytest.mark.parametrize("H,W,ks,kr,ss,r,sr,dtype", [
    (197, 263, "exponential", "exponential", 2.0, 9, 0.1, "f32"),
    (130, 129, "gaussian", "exponential", 3.0, 9, 0.2, "u8"),
    (77, 64, "exponential", "gaussian", 4.0, 18, 0.05, "f32"),
])
def test_direct_summation_exponential_vs_true_bf(torch_dev, H, W, ks, kr, ss, r, sr, dtype):
    bf = _bf()
    I = synth.gen_image_u8(H, W, 4, 0.03, H + 5 * W) if dtype == "u8" else synth.gen_image(H, W, 4, 0.03, H + 5 * W)
    p = bf.Plan(ss, sr, r, 8, 4, dtype=dtype, direct=True, kernel_s=ks, kernel_r=kr)
    assert p.info.direct == 1
    out = _run(torch_dev, p, I)
    ref = oracle.true_bf(I, ss, r, sr, kind_s=ks, kind_r=kr)
    err = np.abs(out - ref).max()
    _report("direct K_s %s K_r %s %dx%d r %d %s vs T1" % (ks, kr, H, W, r, dtype), err)
    assert err <= TIGHT


@pytest.mark.parametrize("H,W,ss,r,sr,dtype", [
    (197, 263, 2.0, 6, 0.1, "f32"),   # ragged, several blocks, borders
    (5, 300, 3.0, 9, 0.05, "f32"),    # image shorter than the window
    (130, 129, 4.0, 12, 0.2, "u8"),
    (64, 64, 8.0, 24, 0.3, "f32"),
    (1, 1, 2.0, 6, 0.1, "f32"),
])
def test_direct_summation_vs_true_bf(torch_dev, H, W, ss, r, sr, dtype):
    """Direct summation is Eq. BF with the exact kernels: the oracle's T1."""
    bf = _bf()
    I = synth.gen_image_u8(H, W, 4, 0.03, H + 7 * W) if dtype == "u8" else synth.gen_image(H, W, 4, 0.03, H + 7 * W)
    p = bf.Plan(ss, sr, r, 8, 4, dtype=dtype, direct=True)
    assert p.info.direct == 1
    out = _run(torch_dev, p, I)
    ref = oracle.true_bf(I, ss, r, sr)
    err = np.abs(out - ref).max()
    _report("direct %dx%d r %d %s vs T1" % (H, W, r, dtype), err)
    assert err <= TIGHT


def test_direct_plans_in_batches(torch_dev):
    """Requests without term tables in a batch beside expansion requests:
    direct summation of several radii, both input types and both range kernel
    kinds (one launch per input type and kind, with the largest window's
    LDS), range-box and level-fold requests of both output-tile sizes (one
    launch per tile size), reduced-precision requests of both input types (a
    pair of launches per type), 1x1 images: bitwise the single-image results."""
    import torch
    bf = _bf()
    pd = bf.Plan(2.0, 0.05, 6, 32, 4, direct="auto")
    pd9 = bf.Plan(3.0, 0.1, 9, 8, 4, direct=True)
    pu = bf.Plan(2.0, 0.1, 6, 8, 4, dtype="u8", direct=True)
    pue = bf.Plan(2.0, 0.1, 9, 8, 4, dtype="u8", direct=True, kernel_s="exponential", kernel_r="exponential")
    pe = bf.Plan(4.0, 0.1, 12, 16, 4)
    assert pd.info.direct == 1 and pe.info.direct == 0
    # range-box and level-fold requests (8-bit) share launches per output-tile size too
    pz = bf.Plan(3.0, 0.1, 9, 5, 4, dtype="u8", range_box=True)
    pz48 = bf.Plan(16.0, 0.1, 48, 5, 4, dtype="u8", range_box=True)
    pf = bf.Plan(8.0, 0.1, 24, 16, 6, dtype="u8", level_fold=True)
    assert pz.info.box_tile == 64 and pz48.info.box_tile == 32
    # reduced-precision requests: one pair of launches per input type
    pr = bf.Plan(3.0, 0.1, 9, 8, 4, precision="reduced")
    pru = bf.Plan(8.0, 0.1, 24, 16, 6, dtype="u8", precision="reduced")
    specs = [(pd, 120, 333), (pe, 77, 64), (pd, 256, 256), (pd9, 1, 1), (pu, 90, 130), (pd9, 200, 70),
             (pue, 64, 65), (pu, 3, 500), (pz, 150, 170), (pz48, 70, 90), (pf, 130, 129), (pz, 1, 1),
             (pz48, 300, 40), (pr, 100, 170), (pru, 140, 90), (pr, 1, 1), (pru, 33, 270)]
    u8 = (pu, pue, pz, pz48, pf, pru)
    plans, imgs = [], []
    for p, h, w in specs:
        plans.append(p)
        if any(p is q for q in u8):
            imgs.append(torch.from_numpy(synth.gen_image_u8(h, w, 4, 0.03, h * w)).cuda())
        else:
            imgs.append(torch.from_numpy(synth.gen_image(h, w, 4, 0.03, h * w)).cuda())
    singles = [bf.filter(p, I).clone() for p, I in zip(plans, imgs)]
    outs = bf.filter_batch(plans, imgs)
    torch.cuda.synchronize()
    for i, (o, s) in enumerate(zip(outs, singles)):
        assert torch.equal(o, s), i


@pytest.mark.parametrize("H,W,ss,r,ns,sr,nr", [
    (300, 517, 2.0, 6, 4, 0.1, 5),     # several tiles, ragged tails
    (197, 263, 3.0, 9, 6, 0.05, 8),
    (130, 129, 8.0, 24, 6, 0.1, 5),
    (70, 90, 16.0, 48, 8, 0.2, 3),
    (150, 170, 10.0, 30, 6, 0.1, 5),   # largest radius of the 64 x 64 output tiles
    (64, 64, 16.0, 48, 4, 0.1, 5),     # largest radius of the regime (32 x 32 output tiles)
    (77, 61, 2.0, 6, 4, 0.1, 24),      # many range terms: same cost
    (5, 40, 2.0, 6, 4, 0.1, 5),        # image shorter than the window
    (1, 1, 2.0, 6, 4, 0.1, 5),
])
def test_range_box_regime_vs_oracle(torch_dev, H, W, ss, r, ns, sr, nr):
    """The paper's own 8-bit regime (T = T_r, range box) against the oracle's
    direct sum T4."""
    bf = _bf()
    Z = synth.gen_image_u8(H, W, 5, 0.03, H * 7 + W)
    p = bf.Plan(ss, sr, r, nr, ns, dtype="u8", range_box=True)
    o = oracle.make_plan(ss, r, ns, sr, nr, span=0.0)
    assert p.info.range_box == 1 and p.info.box_levels == int(np.floor(oracle.box_levels(o)))
    assert abs(p.info.T - o.range.T_r) < 1e-15
    out = _run(torch_dev, p, Z)
    ref = oracle.expanded_rangebox(Z, o)
    err = np.abs(out - ref).max()
    _report("range box %dx%d r %d N %d zr %d vs T4" % (H, W, r, nr, p.info.box_levels), err)
    assert err <= TIGHT


def test_range_box_1080p_sampled(torch_dev):
    """1920 x 1080 8-bit image, sigma_s 8 (r 24), sigma_r 0.1, five range terms:
    2048 sampled pixels (borders, tile seams) against T4."""
    bf = _bf()
    H, W = 1080, 1920
    Z = synth.gen_image_u8(H, W, 40, 0.03, 2)
    p = bf.Plan(8.0, 0.1, 24, 5, 6, dtype="u8", range_box=True)
    o = oracle.make_plan(8.0, 24, 6, 0.1, 5, span=0.0)
    out = _run(torch_dev, p, Z)
    rng = np.random.default_rng(5)
    ys = np.concatenate([rng.integers(0, H, 1536), [0, H - 1, 31, 32, 0, H - 1], rng.integers(0, H, 506)])
    xs = np.concatenate([rng.integers(0, W, 1536), [0, W - 1, 32, 31, W - 1, 0], rng.integers(0, W, 506)])
    ref = oracle.expanded_rangebox(Z, o, ys=ys, xs=xs)
    err = np.abs(out[ys, xs] - ref).max()
    _report("range box 1080p sampled vs T4", err)
    assert err <= TIGHT


def test_range_box_in_batches(torch_dev):
    """Range-box requests mixed with expansion requests in one batch: bitwise
    the single-image results."""
    import torch
    bf = _bf()
    pz = bf.Plan(3.0, 0.1, 9, 5, 4, dtype="u8", range_box=True)
    pe = bf.Plan(3.0, 0.1, 9, 16, 4, dtype="u8")
    imgs = [torch.from_numpy(synth.gen_image_u8(h, w, 4, 0.03, h + w)).cuda() for h, w in ((120, 333), (77, 64), (256, 256))]
    plans = [pz, pe, pz]
    singles = [bf.filter(p, I).clone() for p, I in zip(plans, imgs)]
    outs = bf.filter_batch(plans, imgs)
    torch.cuda.synchronize()
    for o, s in zip(outs, singles):
        assert torch.equal(o, s)


def test_served_mixed_plan_kinds(torch_dev):
    """The request loop with every kind of plan in one queue: Gaussian,
    exponential and tabulated expansions, direct summation (both range kinds),
    the 8-bit range-box regime and the level fold, on 8-bit images of mixed
    sizes.  Each result is bitwise the single-image result."""
    import torch
    bf = _bf()
    K = synth.kernels
    tab = (K.cauchy_spatial(9, 3.0), K.tukey_range(0.2, 1 / 255.0), 1 / 255.0)
    plans = [bf.Plan(3.0, 0.1, 9, 8, 4, dtype="u8"),
             bf.Plan(3.0, 0.1, 14, 12, 6, dtype="u8", kernel_s="exponential", kernel_r="exponential"),
             bf.Plan(2.0, 0.1, 6, 8, 4, dtype="u8", direct=True),
             bf.Plan(2.0, 0.1, 9, 8, 4, dtype="u8", direct=True, kernel_s="exponential", kernel_r="exponential"),
             bf.Plan(8.0, 0.1, 24, 5, 6, dtype="u8", range_box=True),
             bf.Plan(3.0, 0.1, 9, 5, 4, dtype="u8", range_box=True),
             bf.Plan.tabulated(*tab, n_range=8, n_spatial=6, dtype="u8"),
             bf.Plan(3.0, 0.1, 9, 16, 4, dtype="u8", level_fold=True)]
    rng = np.random.default_rng(31)
    sizes = [(int(rng.integers(40, 300)), int(rng.integers(40, 300))) for _ in range(24)]
    imgs = [torch.from_numpy(synth.gen_image_u8(h, w, 4, 0.03, 100 + i)).cuda() for i, (h, w) in enumerate(sizes)]
    which = [i % len(plans) for i in range(len(imgs))]
    outs = [torch.full(I.shape, -1.0, device="cuda") for I in imgs]
    torch.cuda.synchronize()  # the server's streams do not wait for the fills and copies above
    srv = bf.Server(hbm_budget=1 << 30, max_batch=5, n_streams=2)
    for i, I in enumerate(imgs):
        srv.submit(plans[which[i]], I, outs[i], tag=i, now=0.0)
    import time
    done = {}
    t0 = time.perf_counter()
    while len(done) < len(imgs) and time.perf_counter() - t0 < 60.0:
        for c in srv.poll(time.perf_counter() - t0):
            done[c.tag] = c
    srv.close()
    assert len(done) == len(imgs)
    assert all(c.status == bf.BF_OK for c in done.values())
    for i, I in enumerate(imgs):
        alone = bf.filter(plans[which[i]], I)
        torch.cuda.synchronize()
        assert torch.equal(outs[i], alone), (i, which[i])
    # one request of each kind against its oracle
    Z = imgs[4].cpu().numpy()
    ref = oracle.expanded_rangebox(Z, oracle.make_plan(8.0, 24, 6, 0.1, 5, span=0.0))
    assert np.abs(outs[4].cpu().numpy() - ref).max() <= TIGHT
    Z = imgs[1].cpu().numpy()
    ref = oracle.expanded_box(Z, oracle.make_plan(3.0, 14, 6, 0.1, 12, kind_s="exponential", kind_r="exponential"))
    assert np.abs(outs[1].cpu().numpy() - ref).max() <= TIGHT
    Z = imgs[6].cpu().numpy()
    ref = oracle.expanded_box(Z, oracle.make_table_plan(*tab, 6, 8))
    assert np.abs(outs[6].cpu().numpy() - ref).max() <= TIGHT
    Z = imgs[7].cpu().numpy()
    ref = oracle.expanded_box(Z, oracle.make_plan(3.0, 9, 4, 0.1, 16))
    assert np.abs(outs[7].cpu().numpy() - ref).max() <= TIGHT


@pytest.mark.parametrize("H,W,ss,r,ns,sr,nr,dtype", [
    (300, 517, 3.0, 9, 4, 0.1, 8, "f32"),     # several tiles, ragged tails
    (197, 263, 4.0, 12, 6, 0.2, 8, "u8"),
    (1080 // 4, 1920 // 4, 8.0, 24, 6, 0.1, 16, "f32"),
    (130, 129, 16.0, 48, 8, 0.05, 32, "f32"),  # the largest region of the path (12 quadruplets)
    (7, 13, 3.0, 9, 4, 0.1, 8, "f32"),         # image smaller than the window
    (1, 1, 3.0, 9, 4, 0.1, 8, "u8"),
])
def test_reduced_precision_vs_oracle(torch_dev, H, W, ss, r, ns, sr, nr, dtype):
    """FP16 term images, tables built in LDS: within the reduced bar 1e-3 of
    the oracle's T3 (FP16 rounding of the term values, a few 1e-5)."""
    bf = _bf()
    I = synth.gen_image_u8(H, W, 5, 0.03, H + W) if dtype == "u8" else synth.gen_image(H, W, 5, 0.03, H + W)
    p = bf.Plan(ss, sr, r, nr, ns, dtype=dtype, precision="reduced")
    assert p.info.reduced == 1
    out = _run(torch_dev, p, I)
    ref = oracle.expanded_box(I, oracle.make_plan(ss, r, ns, sr, nr))
    err = np.abs(out - ref).max()
    _report("reduced %dx%d r %d N %d %s vs T3" % (H, W, r, nr, dtype), err)
    assert err <= 1e-3
    assert err <= 2e-4  # the FP16 bound in practice; the 1e-3 bar leaves room


def test_reduced_precision_in_batches(torch_dev):
    import torch
    bf = _bf()
    pr = bf.Plan(3.0, 0.1, 9, 8, 4, precision="reduced")
    pe = bf.Plan(3.0, 0.1, 9, 8, 4)
    imgs = [torch.from_numpy(synth.gen_image(h, w, 4, 0.03, h * w)).cuda() for h, w in ((120, 333), (77, 64), (256, 256))]
    plans = [pr, pe, pr]
    singles = [bf.filter(p, I).clone() for p, I in zip(plans, imgs)]
    outs = bf.filter_batch(plans, imgs)
    torch.cuda.synchronize()
    for o, s in zip(outs, singles):
        assert torch.equal(o, s)


@pytest.mark.parametrize("mode", ["range_box", "reduced"])
def test_exponential_kernels_in_the_other_paths(torch_dev, mode):
    """The exponential kernel pair through the range-box regime (against T4)
    and the reduced-precision path (against T3)."""
    bf = _bf()
    H, W = 150, 211
    Z = synth.gen_image_u8(H, W, 5, 0.03, 41)
    kw = dict(kind_s="exponential", kind_r="exponential")
    if mode == "range_box":
        p = bf.Plan(3.0, 0.1, 14, 6, 6, dtype="u8", range_box=True, kernel_s="exponential", kernel_r="exponential")
        ref = oracle.expanded_rangebox(Z, oracle.make_plan(3.0, 14, 6, 0.1, 6, span=0.0, **kw))
        bar = TIGHT
    else:
        p = bf.Plan(3.0, 0.1, 14, 12, 6, dtype="u8", precision="reduced", kernel_s="exponential",
                    kernel_r="exponential")
        ref = oracle.expanded_box(Z, oracle.make_plan(3.0, 14, 6, 0.1, 12, **kw))
        bar = 1e-3
    out = _run(torch_dev, p, Z)
    err = np.abs(out - ref).max()
    _report("exponential kernels, %s, %dx%d" % (mode, H, W), err)
    assert err <= bar


@pytest.mark.parametrize("name", ["cfg2_1080p", "cfg3_4096", "cfg5_4096_u8"])
def test_reduced_precision_full_size(torch_dev, name):
    """The reduced-precision path at the workloads' own sizes: 1080p against
    T3 on the whole image, 4096^2 against T2 on sampled pixels (borders, tile
    seams), within the reduced bar 1e-3."""
    bf = _bf()
    c = CONFIGS[name]
    I = synth.config_image(name)
    p = bf.Plan(c["sigma_s"], c["sigma_r"], c["radius"], c["n_range"], c["n_spatial"], dtype=c["dtype"],
                precision="reduced")
    out = _run(torch_dev, p, I)
    op = oracle.make_plan(c["sigma_s"], c["radius"], c["n_spatial"], c["sigma_r"], c["n_range"])
    if c["H"] * c["W"] <= 4 * 1024 * 1024:
        err = np.abs(out - oracle.expanded_box(I, op)).max()
    else:
        ys, xs = _sample_pixels(c["H"], c["W"], 1500, 9)
        err = np.abs(out[ys, xs] - oracle.expanded_brute(I, op, ys, xs)).max()
    _report("reduced %s vs oracle" % name, err)
    assert err <= 1e-3


def test_graph_replays_of_every_plan_kind(torch_dev):
    """A batch holding every plan kind (expansion, direct summation with the
    exponential range kernel, range-box regime, reduced precision, tabulated
    kernels, level fold), captured once in a graph and replayed on new inputs
    with eager work in between: every replay equals the eager single-image
    calls."""
    import torch
    bf = _bf()
    K = synth.kernels
    plans = [bf.Plan(3.0, 0.1, 9, 8, 4, dtype="u8"),
             bf.Plan(2.0, 0.1, 9, 8, 4, dtype="u8", direct=True, kernel_r="exponential"),
             bf.Plan(8.0, 0.1, 24, 5, 6, dtype="u8", range_box=True),
             bf.Plan(3.0, 0.1, 9, 8, 4, dtype="u8", precision="reduced"),
             bf.Plan.tabulated(K.cauchy_spatial(9, 3.0), K.tukey_range(0.2, 1 / 255.0), 1 / 255.0, n_range=8,
                               n_spatial=6, dtype="u8"),
             bf.Plan(3.0, 0.1, 9, 16, 4, dtype="u8", level_fold=True)]
    shapes = [(97, 150), (64, 77), (130, 129), (111, 96), (80, 201), (150, 70)]
    static_in = [torch.from_numpy(synth.gen_image_u8(h, w, 4, 0.03, 300 + i)).cuda() for i, (h, w) in enumerate(shapes)]
    outs = [torch.empty(I.shape, dtype=torch.float32, device="cuda") for I in static_in]
    ws = torch.empty(bf.batch_workspace_size(plans, shapes), dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bf.filter_batch(plans, static_in, outs=outs, ws=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bf.filter_batch(plans, static_in, outs=outs, ws=ws)
    torch.cuda.synchronize()
    for rep in range(3):
        for j, I in enumerate(static_in):
            I.copy_(torch.from_numpy(synth.gen_image_u8(I.shape[0], I.shape[1], 4, 0.03, 700 + 10 * rep + j)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eager = [bf.filter(p, I) for p, I in zip(plans, static_in)]
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        for j in range(len(plans)):
            assert torch.equal(outs[j], eager[j]), (rep, j)
        assert torch.isfinite(junk)


@pytest.mark.parametrize("H,W,ss,r,ns,sr,nr", [
    (300, 517, 3.0, 9, 4, 0.1, 8),
    (197, 263, 8.0, 24, 6, 0.1, 16),
    (130, 129, 16.0, 48, 8, 0.05, 32),
    (5, 40, 2.0, 6, 4, 0.1, 8),
    (1, 1, 2.0, 6, 4, 0.1, 8),
])
def test_level_fold_vs_oracle(torch_dev, H, W, ss, r, ns, sr, nr):
    """8-bit input with the range terms folded per output level: the default
    regime's filter (T = max(T_r, span)), against the oracle's T3."""
    bf = _bf()
    Z = synth.gen_image_u8(H, W, 5, 0.03, 3 * H + W)
    p = bf.Plan(ss, sr, r, nr, ns, dtype="u8", level_fold=True)
    assert p.info.level_fold == 1 and p.info.range_box == 0
    out = _run(torch_dev, p, Z)
    ref = oracle.expanded_box(Z, oracle.make_plan(ss, r, ns, sr, nr))
    err = np.abs(out - ref).max()
    _report("level fold %dx%d r %d N %d vs T3" % (H, W, r, nr), err)
    assert err <= TIGHT


def test_level_fold_4096_sampled(torch_dev):
    bf = _bf()
    c = CONFIGS["cfg5_4096_u8"]
    Z = synth.config_image("cfg5_4096_u8")
    p = bf.Plan(c["sigma_s"], c["sigma_r"], c["radius"], c["n_range"], c["n_spatial"], dtype="u8", level_fold=True)
    out = _run(torch_dev, p, Z)
    op = oracle.make_plan(c["sigma_s"], c["radius"], c["n_spatial"], c["sigma_r"], c["n_range"])
    ys, xs = _sample_pixels(4096, 4096, 1500, 11)
    err = np.abs(out[ys, xs] - oracle.expanded_brute(Z, op, ys, xs)).max()
    _report("level fold cfg5 sampled vs T2", err)
    assert err <= TIGHT


def _table_cases():
    K = synth.kernels
    return {
        "cauchy r9 tukey u8": (300, 517, K.cauchy_spatial(9, 3.0), K.tukey_range(0.2, 1 / 255.0), 1 / 255.0, 6, 8, "u8"),
        "gauss r24 cauchy f32": (197, 263, K.gaussian_spatial(24, 8.0), K.cauchy_range(0.05, 0.005, 201), 0.005, 6,
                                 16, "f32"),
        "cauchy r48 tukey f32": (130, 129, K.cauchy_spatial(48, 10.0), K.tukey_range(0.3, 0.01), 0.01, 8, 32, "f32"),
        "cauchy r3 cauchy f32": (5, 33, K.cauchy_spatial(3, 1.0), K.cauchy_range(0.1, 0.01, 101), 0.01, 4, 8, "f32"),
        "cauchy r24 tukey 1080p f32": (1080, 1920, K.cauchy_spatial(24, 8.0), K.tukey_range(0.3, 0.005), 0.005, 6,
                                       16, "f32"),
    }


@pytest.mark.parametrize("name", ["cauchy r9 tukey u8", "gauss r24 cauchy f32", "cauchy r48 tukey f32",
                                  "cauchy r3 cauchy f32", "cauchy r24 tukey 1080p f32"])
def test_tabulated_kernels_vs_oracle(torch_dev, name):
    """Tabulated kernels change only the fitted coefficients: the same kernels
    filter them, against the oracle's T3 for the same tables."""
    bf = _bf()
    H, W, ks, kr, step, ns, nr, dtype = _table_cases()[name]
    I = synth.gen_image_u8(H, W, 5, 0.03, H + 5 * W) if dtype == "u8" else synth.gen_image(H, W, 5, 0.03, H + 5 * W)
    p = bf.Plan.tabulated(ks, kr, step, n_range=nr, n_spatial=ns, dtype=dtype)
    o = oracle.make_table_plan(ks, kr, step, ns, nr)
    out = _run(torch_dev, p, I)
    err = np.abs(out - oracle.expanded_box(I, o)).max()
    _report("tabulated %s %dx%d vs T3" % (name, H, W), err)
    _report("  same vs true BF with the tables (reported)",
            np.abs(out - oracle.true_bf_tab(I, ks, kr, step)).max())
    assert err <= TIGHT


@pytest.mark.parametrize("mode", ["range_box", "level_fold", "reduced", "batch"])
def test_tabulated_kernels_in_the_other_paths(torch_dev, mode):
    """A tabulated kernel pair through the range-box regime (against T4), the
    level fold and the reduced-precision path (against T3), and a batch mixed
    with Gaussian plans (bitwise the single-image results)."""
    import torch
    bf = _bf()
    K = synth.kernels
    H, W = 150, 211
    Z = synth.gen_image_u8(H, W, 5, 0.03, 43)
    ks, kr, step = K.cauchy_spatial(12, 4.0), K.tukey_range(0.2, 1 / 255.0), 1 / 255.0
    if mode == "batch":
        pt = bf.Plan.tabulated(ks, kr, step, n_range=12, n_spatial=6, dtype="u8")
        pg = bf.Plan(3.0, 0.1, 9, 8, 4, dtype="u8")
        imgs = [torch.from_numpy(synth.gen_image_u8(h, w, 4, 0.03, h * w)).cuda() for h, w in ((120, 333), (77, 64),
                                                                                               (256, 256))]
        plans = [pt, pg, pt]
        singles = [bf.filter(p, I).clone() for p, I in zip(plans, imgs)]
        outs = bf.filter_batch(plans, imgs)
        torch.cuda.synchronize()
        for o, s in zip(outs, singles):
            assert torch.equal(o, s)
        return
    if mode == "range_box":
        p = bf.Plan.tabulated(ks, kr, step, n_range=5, n_spatial=6, dtype="u8", range_box=True)
        ref = oracle.expanded_rangebox(Z, oracle.make_table_plan(ks, kr, step, 6, 5, span=0.0))
        bar = TIGHT
    elif mode == "level_fold":
        p = bf.Plan.tabulated(ks, kr, step, n_range=12, n_spatial=6, dtype="u8", level_fold=True)
        ref = oracle.expanded_box(Z, oracle.make_table_plan(ks, kr, step, 6, 12))
        bar = TIGHT
    else:
        p = bf.Plan.tabulated(ks, kr, step, n_range=12, n_spatial=6, dtype="u8", precision="reduced")
        ref = oracle.expanded_box(Z, oracle.make_table_plan(ks, kr, step, 6, 12))
        bar = 1e-3
    out = _run(torch_dev, p, Z)
    err = np.abs(out - ref).max()
    _report("tabulated kernels, %s, %dx%d" % (mode, H, W), err)
    assert err <= bar
