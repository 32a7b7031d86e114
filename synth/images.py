"""Seeded gray-level test images in [0, 1] (float32) or uint8."""
import numpy as np


def _fade(t):
    # quintic smoothstep 6t^5 - 15t^4 + 10t^3 of classic gradient noise
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _gradient_noise(H, W, cell, rng):
    """One octave of 2-D gradient noise on a lattice of `cell` pixels."""
    ny = int(np.ceil(H / cell)) + 2
    nx = int(np.ceil(W / cell)) + 2
    ang = rng.uniform(0.0, 2.0 * np.pi, size=(ny, nx))
    gy, gx = np.sin(ang), np.cos(ang)
    out = np.empty((H, W), dtype=np.float64)
    xs = np.arange(W, dtype=np.float64) / cell
    x0 = np.floor(xs).astype(np.int64)
    fx = xs - x0
    ux = _fade(fx)
    # blocks of rows keep temporaries at O(block * W) for 4096-wide images
    for ya in range(0, H, 256):
        yb = min(H, ya + 256)
        ys = np.arange(ya, yb, dtype=np.float64)[:, None] / cell
        y0 = np.floor(ys).astype(np.int64)
        fy = ys - y0
        uy = _fade(fy)
        g00 = gy[y0, x0] * fy + gx[y0, x0] * fx
        g01 = gy[y0, x0 + 1] * fy + gx[y0, x0 + 1] * (fx - 1.0)
        g10 = gy[y0 + 1, x0] * (fy - 1.0) + gx[y0 + 1, x0] * fx
        g11 = gy[y0 + 1, x0 + 1] * (fy - 1.0) + gx[y0 + 1, x0 + 1] * (fx - 1.0)
        top = g00 + ux * (g01 - g00)
        bot = g10 + ux * (g11 - g10)
        out[ya:yb] = top + uy * (bot - top)
    return out


def gen_image(H, W, edges, noise_sd, seed):
    """Float32 image in [0, 1]: 4 octaves of gradient noise plus `edges` random
    straight step edges of height U(-0.2, 0.2), the sum rescaled to [0.1, 0.9],
    then N(0, noise_sd^2) noise, clipped to [0, 1]."""
    H, W = int(H), int(W)
    rng = np.random.default_rng(seed)
    base = max(H, W) / 4.0
    field = np.zeros((H, W), dtype=np.float64)
    for o in range(4):
        cell = max(base / (2 ** o), 2.0)
        field += (0.5 ** o) * _gradient_noise(H, W, cell, rng)
    lo, hi = field.min(), field.max()
    field = (field - lo) / (hi - lo if hi > lo else 1.0)
    # step edges: pixel (y, x) gets delta where (x - px) cos(th) + (y - py) sin(th) > 0;
    # per row that is a half-line in x, accumulated in a difference array
    diff = np.zeros((H, W + 1), dtype=np.float64)
    yv = np.arange(H, dtype=np.float64)
    rows = np.arange(H)
    for _ in range(int(edges)):
        py, px = rng.uniform(0, H), rng.uniform(0, W)
        th = rng.uniform(0.0, np.pi)
        d = rng.uniform(-0.2, 0.2)
        cx, sy = np.cos(th), np.sin(th)
        if abs(cx) < 1e-12:
            on = (yv - py) * sy > 0
            diff[on, 0] += d
            diff[on, W] -= d
            continue
        thr = px - (yv - py) * sy / cx  # boundary x on each row
        if cx > 0:  # x > thr
            start = np.clip(np.floor(thr).astype(np.int64) + 1, 0, W)
            np.add.at(diff, (rows, start), d)
            diff[:, W] -= d
        else:       # x < thr
            stop = np.clip(np.ceil(thr).astype(np.int64), 0, W)
            diff[:, 0] += d
            np.add.at(diff, (rows, stop), -d)
    field += np.cumsum(diff, axis=1)[:, :W]
    lo, hi = field.min(), field.max()
    field = 0.1 + 0.8 * (field - lo) / (hi - lo if hi > lo else 1.0)
    field += rng.normal(0.0, noise_sd, size=(H, W))
    return np.clip(field, 0.0, 1.0).astype(np.float32)


def gen_image_u8(H, W, edges, noise_sd, seed):
    """uint8 variant: round(255 * gen_image(...))."""
    return np.rint(gen_image(H, W, edges, noise_sd, seed).astype(np.float64) * 255.0).astype(np.uint8)


# The workloads: image recipe and filter parameters.
CONFIGS = {
    "cfg1_256": dict(H=256, W=256, edges=6, noise=0.02, seed=1, sigma_s=3.0, radius=9,
                     sigma_r=0.1, n_range=8, n_spatial=4, dtype="f32"),
    "cfg2_1080p": dict(H=1080, W=1920, edges=40, noise=0.03, seed=2, sigma_s=8.0, radius=24,
                       sigma_r=0.1, n_range=16, n_spatial=6, dtype="f32"),
    "cfg3_4096": dict(H=4096, W=4096, edges=150, noise=0.03, seed=3, sigma_s=16.0, radius=48,
                      sigma_r=0.05, n_range=32, n_spatial=8, dtype="f32"),
    "cfg5_4096_u8": dict(H=4096, W=4096, edges=150, noise=0.03, seed=3, sigma_s=16.0, radius=48,
                         sigma_r=0.05, n_range=32, n_spatial=8, dtype="u8"),
    # the paper's own 8-bit regime: series on [-T_r, T_r] with the range box, five terms
    "cfg6_1080p_u8_box": dict(H=1080, W=1920, edges=40, noise=0.03, seed=2, sigma_s=8.0, radius=24,
                              sigma_r=0.1, n_range=5, n_spatial=6, dtype="u8", range_box=True),
}


def config_image(name):
    c = CONFIGS[name]
    if c["dtype"] == "u8":
        return gen_image_u8(c["H"], c["W"], c["edges"], c["noise"], c["seed"])
    return gen_image(c["H"], c["W"], c["edges"], c["noise"], c["seed"])
