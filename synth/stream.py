"""Seeded served-request stream: Poisson arrivals, mixed sizes and sigmas."""
import math
import numpy as np


def gen_stream(n=512, rate_hz=2000.0, seed=4, hw_lo=128, hw_hi=2048):
    """Request descriptors (no pixels): arrival time, H, W, generator recipe and
    filter parameters.  Range-term count follows N_r = clamp(ceil(1.6 / sigma_r), 8, 32),
    the number of cosine terms a [0, 1] span needs at that sigma_r."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        H = int(rng.integers(hw_lo, hw_hi + 1))
        W = int(rng.integers(hw_lo, hw_hi + 1))
        ss = float(rng.choice([2.0, 4.0, 8.0, 16.0]))
        sr = float(rng.choice([0.05, 0.1, 0.2, 0.3]))
        nr = int(min(32, max(8, math.ceil(1.6 / sr))))
        edges = int(round(6 + 144 * H * W / 4096.0 ** 2))
        reqs.append(dict(id=i, t_arrive=float(t[i]), H=H, W=W, edges=edges, noise=0.03,
                         seed=1000 + i, sigma_s=ss, radius=int(3 * ss), sigma_r=sr,
                         n_range=nr, n_spatial=4))
    return reqs
