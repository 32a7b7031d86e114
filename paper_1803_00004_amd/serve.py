"""Driver of the library's request loop (bf_server_*) for a served stream.

Requests arrive open-loop at their own times (wall clock); the native loop
queues them, admits them by workspace footprint and launches batches on its
streams.  This module only paces arrivals, holds the tensors and collects the
completions; every scheduling decision is made in the library.
"""
import multiprocessing as mp
import os
import time

import numpy as np

from . import bf


def _gen_one(r):
    import synth
    return synth.gen_image(r["H"], r["W"], r["edges"], r["noise"], r["seed"])


def generate_images(reqs, workers=None):
    """Host images of the requests (numpy float32), generated in a pool of
    forked workers.  Call before the process touches the GPU."""
    workers = workers or min(16, os.cpu_count() or 1)
    if workers <= 1 or len(reqs) < 4:
        return [_gen_one(r) for r in reqs]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_gen_one, reqs, chunksize=max(1, len(reqs) // (4 * workers)))


def plan_key(r):
    return (r["sigma_s"], r["radius"], r["n_spatial"], r["sigma_r"], r["n_range"])


def make_plans(reqs):
    plans = {}
    for r in reqs:
        k = plan_key(r)
        if k not in plans:
            plans[k] = bf.Plan(r["sigma_s"], r["sigma_r"], r["radius"], r["n_range"], r["n_spatial"])
    return plans


def _inputs_ready():
    """The server's streams wait for no other stream: whatever produced the
    inputs, or may still write the outputs, must be finished before submit."""
    import torch
    torch.cuda.synchronize()


def run_open_loop(srv, reqs, plans, imgs, outs, t_scale=1.0):
    """Submit request i at t_arrive[i] * t_scale after the start; poll until
    every request completes.  Returns (completions by tag, makespan s)."""
    _inputs_ready()
    n = len(reqs)
    done = {}
    t0 = time.perf_counter()
    i = 0
    while len(done) < n:
        now = time.perf_counter() - t0
        while i < n and reqs[i]["t_arrive"] * t_scale <= now:
            srv.submit(plans[plan_key(reqs[i])], imgs[i], outs[i], tag=i, now=now)
            i += 1
        for c in srv.poll(now):
            done[c.tag] = c
    return done, time.perf_counter() - t0


def run_closed_loop(srv, reqs, plans, imgs, outs):
    """Every request submitted at once; returns the makespan in seconds."""
    _inputs_ready()
    done = {}
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        srv.submit(plans[plan_key(r)], imgs[i], outs[i], tag=i, now=0.0)
    while len(done) < len(reqs):
        for c in srv.poll(time.perf_counter() - t0):
            done[c.tag] = c
    return done, time.perf_counter() - t0


def run_plain(reqs, plans, imgs, outs, stream=None):
    """The same requests one at a time with bf_filter on one stream."""
    import torch
    ws = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, r in enumerate(reqs):
        p = plans[plan_key(r)]
        need = p.workspace_size(r["H"], r["W"])
        if need > ws.get("n", 0):
            torch.cuda.synchronize()
            ws["t"] = torch.empty(need, dtype=torch.uint8, device=imgs[i].device)
            ws["n"] = need
        bf.filter(p, imgs[i], out=outs[i], ws=ws["t"], stream=stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def latency_summary(reqs, done, t_scale=1.0):
    lat = np.array([done[i].t_done - reqs[i]["t_arrive"] * t_scale for i in range(len(reqs))])
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}
