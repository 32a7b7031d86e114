"""Benchmark of the N-term bilateral filter on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu] [--no-served]

Default (no --workload): the headline line.  Its value is the 4096 x 4096
FP32 workload (sigma_s 16, r 48, sigma_r 0.05, N_r 32, N_s 8): a step is one
bf_filter call on one image already resident in HBM -- term modulation +
summed-area tables (kernel 0) and tap lookup, accumulation and normalisation
(kernel 1).  Beside it, in the same JSON line: the HBM roofline of the
dominant kernel from algorithmic bytes, the measured device-copy bandwidth,
one pass of the 512-request served stream (p50/p99 latency, open- and
closed-loop Mpix/s, results bitwise equal alone), and the FP64 oracle (T3)
timed on the host on all cores and on one core.

--workload selects a single workload instead:
  cfg1_256, cfg2_1080p, cfg3_4096, cfg5_4096_u8  one image per step, as above;
  cfg6_1080p_u8_box  the paper's own 8-bit regime (range series on [-T_r,
      T_r] with the range box, BF_FLAG_RANGE_BOX): one kernel per image; its
      roofline counts the integer adds of the level-slab tables it builds;
  cfg4_served  the served stream alone.

The plan (FP64 host fit) is built once per parameter set, timed separately
and reported as plan_ms.  Prints ONE JSON line; diagnostics go to stderr.
"""
import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s at fixed max-abs err vs FP64 oracle; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector
CPU_SECONDS = 10.0         # oracle work timed for the CPU baseline (each leg)
INT32_PEAK_TOPS = 39.3     # 256 CUs x 64 lanes x 2.4 GHz, one 32-bit add per lane per clock
HEADLINE = "cfg3_4096"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    p = os.path.join(ROOT, "paper_1803_00004_amd", "csrc", "kernels.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def recorded_traffic(workload, kernel):
    """HBM bytes per launch from committed rocprofv3 --pmc summaries, only if
    they were taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    try:
        rec = json.load(open(p))
    except ValueError:
        return None
    for r in rec.get("entries", []):
        if r.get("workload") == workload and r.get("kernel") == kernel and \
                r.get("kernels_hip_sha256_16") == kernel_source_hash():
            return r.get("hbm_bytes_per_launch")
    return None


def hbm_roofline(kernel, bytes_per_launch, kernel_ms, flops_per_launch=None):
    """HBM roofline of one kernel: algorithmic bytes per launch over its
    average launch time, against the 8 TB/s peak; its FP32 arithmetic against
    the FP32 vector peak beside it."""
    t = kernel_ms * 1e-3
    a = bytes_per_launch / t / 1e9
    roof = {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS,
            "kernel": kernel, "kernel_ms": kernel_ms, "algorithmic_bytes": bytes_per_launch}
    if flops_per_launch:
        tf = flops_per_launch / t / 1e12
        roof["fp32"] = {"achieved_tflops": tf, "peak_tflops": FP32_PEAK_TFLOPS, "frac": tf / FP32_PEAK_TFLOPS}
    return roof


def cpu_host():
    """Host CPU model and the cores this process may use."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return model, nproc


def device_copy_gbs(torch, dev, mib=1024, reps=10):
    """Achievable HBM bandwidth: a device-to-device copy of mib MiB (bytes read
    plus bytes written, over the time of reps copies)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def served_run(args, reqs, host_imgs, with_oracle):
    """One pass of the served stream through the request loop: open loop
    (Poisson arrivals), closed loop (all queued at once) and one at a time,
    each into its own outputs.  Returns the result fields."""
    import torch
    from paper_1803_00004_amd import bf, serve

    n = len(reqs)
    fused = bool(getattr(args, "fused_batch", False))
    bf.set_batch_fused(fused)  # process-wide: every batch of the server
    t0 = time.perf_counter()
    plans = serve.make_plans(reqs)
    plan_ms = (time.perf_counter() - t0) * 1e3
    dev = torch.device("cuda:0")
    imgs = [torch.from_numpy(I).to(dev) for I in host_imgs]
    outs_open = [torch.empty(I.shape, dtype=torch.float32, device=dev) for I in imgs]
    outs_closed = [torch.empty(I.shape, dtype=torch.float32, device=dev) for I in imgs]
    alone = [torch.empty(I.shape, dtype=torch.float32, device=dev) for I in imgs]
    px = np.array([r["H"] * r["W"] for r in reqs], dtype=np.float64)
    budget = 48 << 30
    max_batch = int(getattr(args, "served_max_batch", 16))
    n_streams = int(getattr(args, "served_streams", 2))
    srv = bf.Server(hbm_budget=budget, max_batch=max_batch, n_streams=n_streams)
    log("[served] %d plans in %.0f ms; %.1f Mpx in total; warm-up" % (len(plans), plan_ms, px.sum() / 1e6))
    for _ in range(max(1, args.warmup)):
        serve.run_closed_loop(srv, reqs[:32], plans, imgs[:32], outs_closed[:32])
    serve.run_plain(reqs[:32], plans, imgs[:32], alone[:32])

    bf.profile_enable(True)
    bf.profile_read()
    done, makespan = serve.run_open_loop(srv, reqs, plans, imgs, outs_open)
    kms, klaunch = bf.profile_read()
    bf.profile_enable(False)
    st = srv.stats()
    lat = serve.latency_summary(reqs, done)
    thr_open = px.sum() / makespan / 1e6
    log("[served] open loop: makespan %.1f ms, %.1f Mpix/s, p50 %.2f ms, p99 %.2f ms, %d batches"
        % (makespan * 1e3, thr_open, lat["p50_ms"], lat["p99_ms"], st.batches))
    _, mk_closed = serve.run_closed_loop(srv, reqs, plans, imgs, outs_closed)
    thr_closed = px.sum() / mk_closed / 1e6
    t_plain = serve.run_plain(reqs, plans, imgs, alone)
    thr_plain = px.sum() / t_plain / 1e6
    torch.cuda.synchronize()
    n_equal_open = sum(bool(torch.equal(outs_open[i], alone[i])) for i in range(n))
    n_equal_closed = sum(bool(torch.equal(outs_closed[i], alone[i])) for i in range(n))
    log("[served] closed loop %.1f Mpix/s; one at a time %.1f Mpix/s; bitwise equal alone: open loop %d/%d, "
        "closed loop %d/%d" % (thr_closed, thr_plain, n_equal_open, n, n_equal_closed, n))
    # the oracle check reads the open-loop outputs before anything else writes
    # them
    err = None
    if with_oracle:
        import oracle
        rng = np.random.default_rng(21)
        errs = []
        for i in range(32):
            r = reqs[i]
            op = oracle.make_plan(r["sigma_s"], r["radius"], r["n_spatial"], r["sigma_r"], r["n_range"])
            ys = rng.integers(0, r["H"], 64).astype(np.int32)
            xs = rng.integers(0, r["W"], 64).astype(np.int32)
            ref = oracle.expanded_brute(host_imgs[i], op, ys, xs)
            errs.append(float(np.abs(outs_open[i].cpu().numpy()[ys, xs] - ref).max()))
        err = max(errs)
        log("[served] open-loop outputs: max-abs err vs oracle T2 (32 requests x 64 px) %.3e" % err)
    # the same stream with direct summation where it is cheaper (small
    # windows: those requests get the exact bilateral filter), in their own
    # outputs
    auto_plans = {k: bf.Plan(k[0], k[3], k[1], k[4], k[2], direct="auto") for k in plans}
    n_direct = sum(1 for r in reqs if auto_plans[serve.plan_key(r)].info.direct)
    outs_auto = outs_closed
    serve.run_closed_loop(srv, reqs[:32], auto_plans, imgs[:32], outs_auto[:32])
    done_a, mk_a = serve.run_open_loop(srv, reqs, auto_plans, imgs, outs_auto)
    lat_a = serve.latency_summary(reqs, done_a)
    _, mk_ac = serve.run_closed_loop(srv, reqs, auto_plans, imgs, outs_auto)
    log("[served] with direct summation for %d small-window requests: open loop %.1f Mpix/s p50 %.2f ms p99 %.2f ms; "
        "closed loop %.1f Mpix/s" % (n_direct, px.sum() / mk_a / 1e6, lat_a["p50_ms"], lat_a["p99_ms"],
                                     px.sum() / mk_ac / 1e6))
    srv.close()
    del imgs, outs_open, outs_closed, alone
    torch.cuda.empty_cache()

    kb_b = 0.0
    for r in reqs:
        info = plans[serve.plan_key(r)].info
        kb_b += r["H"] * r["W"] * (4 * info.n_images + 8)
    fields = {
        "workload": "cfg4_served: 512 requests, Poisson 2000/s, H, W ~ U{128..2048}, sigma_s in {2,4,8,16} "
                    "(r = 3 sigma_s), sigma_r in {0.05,0.1,0.2,0.3}, N_r = clamp(ceil(1.6/sigma_r), 8, 32), N_s = 4",
        "p50_ms": round(lat["p50_ms"], 3), "p99_ms": round(lat["p99_ms"], 3),
        "mean_ms": round(lat["mean_ms"], 3), "makespan_ms": round(makespan * 1e3, 2),
        "open_loop_mpix_s": round(thr_open, 2), "closed_loop_batched_mpix_s": round(thr_closed, 2),
        "one_at_a_time_mpix_s": round(thr_plain, 2), "batches": int(st.batches),
        "peak_batches_in_flight": st.peak_batches_in_flight,
        "peak_requests_in_flight": st.peak_requests_in_flight,
        "peak_workspace_bytes": int(st.peak_arena_bytes),
        "hbm_budget_bytes": budget, "max_batch": max_batch, "streams": n_streams,
        "batch_size_hist": {str(k): int(st.batch_size_hist[k]) for k in range(65) if st.batch_size_hist[k]},
        "results_bitwise_equal_alone": "%d/%d" % (n_equal_open, n),
        "closed_loop_bitwise_equal_alone": "%d/%d" % (n_equal_closed, n),
        "max_abs_err_vs_oracle": err,
        "oracle_sample": "T2 (FP64 direct sum of the expanded form) at 64 random pixels of each of the first "
                         "32 requests, on the open-loop outputs",
        "plan_ms": round(plan_ms, 1),
        "fused_batch": fused,
        "kernel_ms_total_open_loop": {"tables": round(kms[0], 3), "lookup": round(kms[1], 3)},
        "lookup_hbm_gbs_open_loop": round(kb_b / max(kms[1], 1e-9) / 1e6, 1),
        "with_direct_auto": {"requests_direct": n_direct,
                             "open_loop_mpix_s": round(px.sum() / mk_a / 1e6, 2),
                             "p50_ms": round(lat_a["p50_ms"], 3), "p99_ms": round(lat_a["p99_ms"], 3),
                             "closed_loop_mpix_s": round(px.sum() / mk_ac / 1e6, 2)},
    }
    return fields, thr_open, makespan


def served(args):
    """--workload cfg4_served: the served stream alone."""
    import synth
    from paper_1803_00004_amd import serve

    reqs = synth.gen_stream()
    t0 = time.perf_counter()
    host_imgs = serve.generate_images(reqs)  # before the GPU is touched (forked pool)
    log("[served] %d request images generated in %.1f s" % (len(reqs), time.perf_counter() - t0))
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fields, thr_open, makespan = served_run(args, reqs, host_imgs, not args.no_cpu)
    result = {
        "metric": METRIC, "value": round(thr_open, 2), "unit": "Mpix/s", "n_gpus": 1,
        "steps": 1, "warmup": args.warmup, "ms_per_step": round(makespan * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32+f32",
        "data": "synthetic (seeded gradient noise + step edges + Gaussian noise per request)",
        "config": {"workload": fields["workload"]},
        "served": fields,
        "roofline": None,
    }
    print(json.dumps(result), flush=True)


def oracle_one_core(workload):
    """Child-process mode (OMP_NUM_THREADS=1): time the oracle on one core and
    print one JSON line -- T3 on sub-images of the workload's image (T4 on
    sampled pixels for the range-box workload)."""
    import oracle
    import synth
    from synth.images import CONFIGS
    c = CONFIGS[workload]
    I_host = synth.config_image(workload)
    H, W, r = c["H"], c["W"], c["radius"]
    rng = np.random.default_rng(13)
    done, dt, reps = 0, 0.0, 0
    if c.get("range_box", False):
        op = oracle.make_plan(c["sigma_s"], r, c["n_spatial"], c["sigma_r"], c["n_range"], span=0.0)
        n = 16384
        while reps == 0 or (dt < CPU_SECONDS and reps < 64):
            ys, xs = rng.integers(0, H, n).astype(np.int32), rng.integers(0, W, n).astype(np.int32)
            t0 = time.perf_counter()
            oracle.expanded_rangebox(I_host, op, ys, xs)
            dt += time.perf_counter() - t0
            done += n
            reps += 1
        sample = "%d random pixels, oracle T4 (FP64 direct sum with the range box)" % done
    else:
        op = oracle.make_plan(c["sigma_s"], r, c["n_spatial"], c["sigma_r"], c["n_range"])
        h, w = min(H, 32 + 2 * r), min(W, 512)
        while reps == 0 or (dt < CPU_SECONDS and reps < 64):
            y0, x0 = int(rng.integers(0, H - h + 1)), int(rng.integers(0, W - w + 1))
            sub = np.ascontiguousarray(I_host[y0:y0 + h, x0:x0 + w])
            t0 = time.perf_counter()
            oracle.expanded_box(sub, op)
            dt += time.perf_counter() - t0
            done += h * w
            reps += 1
        sample = "%d sub-images of %dx%d, oracle T3 (FP64 shift identity + box sums)" % (reps, w, h)
    print(json.dumps({"mpix_s": done / dt / 1e6, "seconds": dt, "pixels": done, "sample": sample}))


def one_core_baseline(workload):
    """The oracle on one host core, timed in a child process started before
    this process touches the GPU."""
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-core", workload],
                       env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        log("[bench] one-core oracle failed: %s" % r.stderr[-500:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def oracle_all_cores(I_host, c, out_host):
    """The oracle T3 on all host cores, about CPU_SECONDS of it, and the
    max-abs error of the GPU output against it.  Images up to 4 Mpx: the whole
    image, repeated.  Larger: bands of 64 + 2r rows at the top, the middle and
    the bottom of the image; a band row at least r rows from a cut band edge
    sees only band pixels, so there T3 of the band equals T3 of the image and
    the error is taken on those rows."""
    import oracle
    H, W, r = c["H"], c["W"], c["radius"]
    op = oracle.make_plan(c["sigma_s"], r, c["n_spatial"], c["sigma_r"], c["n_range"])
    err, done, cpu_s, reps, rows = 0.0, 0, 0.0, 0, 0
    if H * W <= 4 * 1024 * 1024:
        while reps == 0 or (cpu_s < CPU_SECONDS and reps < 64):
            t0 = time.perf_counter()
            ref = oracle.expanded_box(I_host, op)
            cpu_s += time.perf_counter() - t0
            reps += 1
            done += H * W
        err = float(np.abs(out_host - ref).max())
        rows = H
        sample = "full %dx%d image x %d, oracle T3 (FP64 shift identity + box sums)" % (W, H, reps)
    else:
        h = 64 + 2 * r
        starts = [0, (H - h) // 2, H - h]
        while reps == 0 or (cpu_s < CPU_SECONDS and reps < 8):
            y0 = starts[reps % len(starts)]
            band = np.ascontiguousarray(I_host[y0:y0 + h])
            t0 = time.perf_counter()
            ref = oracle.expanded_box(band, op)
            cpu_s += time.perf_counter() - t0
            lo = 0 if y0 == 0 else r
            hi = h if y0 + h == H else h - r
            err = max(err, float(np.abs(out_host[y0 + lo:y0 + hi] - ref[lo:hi]).max()))
            rows += hi - lo
            reps += 1
            done += h * W
        sample = ("%d bands of %dx%d (top, middle, bottom), oracle T3 (FP64 shift identity + box sums); error "
                  "over %d exact rows" % (reps, W, h, rows))
    return err, done / cpu_s / 1e6, cpu_s, sample, rows * W


def slab_table_adds(Z, plan_info, tile):
    """Algorithmic integer adds of the range-box kernel on image Z: for every
    tile x tile output tile, two slab tables (numerator, denominator) per distinct
    output level, each (region rows + 1) x (region columns + 1) entries built
    with two adds (row and column recurrences of Eq. sum_sat_recurrence_2D)."""
    H, W = Z.shape
    dy_lo, dy_hi = plan_info["tap_dy_min"], plan_info["tap_dy_max"]
    dx_lo, dx_hi = plan_info["tap_dx_min"], plan_info["tap_dx_max"]
    adds = 0
    for ty in range(0, H, tile):
        rs = min(max(ty + tile - 1 + dy_hi, 0), H) - min(max(ty + dy_lo, 0), H)
        for tx in range(0, W, tile):
            rc = min(max(tx + tile - 1 + dx_hi, 0), W) - min(max(tx + dx_lo, 0), W)
            levels = len(np.unique(Z[ty:ty + tile, tx:tx + tile]))
            adds += levels * 2 * 2 * (rs + 1) * (rc + 1)
    return adds


def range_box(args):
    import torch
    import synth
    from synth.images import CONFIGS
    from paper_1803_00004_amd import bf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = args.workload
    c = CONFIGS[w]
    H, W = c["H"], c["W"]
    Z = synth.config_image(w)
    one_core = None
    if not args.no_cpu:
        log("[bench] oracle T4 on sampled pixels, one core (child process)")
        one_core = one_core_baseline(w)
    t0 = time.perf_counter()
    plan = bf.Plan(c["sigma_s"], c["sigma_r"], c["radius"], c["n_range"], c["n_spatial"], dtype="u8",
                   range_box=True)
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info
    log("[bench] plan %.1f ms: %s" % (plan_ms, info.as_dict()))
    dy, dx, _ = plan.taps()
    taps = {"tap_dy_min": int(dy.min()), "tap_dy_max": int(dy.max()), "tap_dx_min": int(dx.min()),
            "tap_dx_max": int(dx.max())}
    dev = torch.device("cuda:0")
    I = torch.from_numpy(Z).to(dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        bf.filter(plan, I, out=out, stream=stream)
    torch.cuda.synchronize()
    bf.profile_enable(True)
    bf.profile_read()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(args.steps):
        bf.filter(plan, I, out=out, stream=stream)
    end.record(stream)
    torch.cuda.synchronize()
    ms_per_step = start.elapsed_time(end) / args.steps
    kms, kl = bf.profile_read()
    bf.profile_enable(False)
    k_ms = kms[1] / max(1, kl[1])
    mpix = H * W / (ms_per_step * 1e-3) / 1e6
    adds = slab_table_adds(Z, taps, info.box_tile)
    tops = adds / (k_ms * 1e-3) / 1e12
    log("[bench] %.4f ms/step  %.1f Mpix/s  kz_rangebox %.4f ms, %.3g table adds (%.2f TOP/s)"
        % (ms_per_step, mpix, k_ms, adds, tops))
    result = {
        "metric": METRIC, "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i32+f32", "data": "synthetic (seeded gradient noise + step edges + Gaussian noise)",
        "config": {"workload": "%s: %dx%d u8, Gaussian sigma_s=%g r=%d, sigma_r=%g, N_r=%d, N_s=%d, "
                               "T = T_r with the range box (level window +-%d)"
                               % (w, W, H, c["sigma_s"], c["radius"], c["sigma_r"], c["n_range"],
                                  c["n_spatial"], info.box_levels),
                   "H": H, "W": W, "box_levels": info.box_levels, "sat_shift": info.sat_shift,
                   "output_tile": info.box_tile},
        "plan_ms": round(plan_ms, 2),
        "kernel_ms": {"kz_rangebox": round(k_ms, 5)},
        "roofline": {"bound": "alu", "achieved": tops, "peak": INT32_PEAK_TOPS, "unit": "TOP/s",
                     "frac": tops / INT32_PEAK_TOPS, "traffic": None, "kernel": "kz_rangebox",
                     "kernel_ms": k_ms, "algorithmic_adds": adds},
    }
    if not args.no_cpu:
        import oracle
        op = oracle.make_plan(c["sigma_s"], c["radius"], c["n_spatial"], c["sigma_r"], c["n_range"], span=0.0)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        n = 262144  # about 2 s of 16 host cores per batch; batches for ~CPU_SECONDS
        rng = np.random.default_rng(11)
        log("[bench] oracle T4 on sampled pixels (%d threads), batches of %d for ~%.0f s" % (threads, n, CPU_SECONDS))
        out_host = out.cpu().numpy().astype(np.float64)
        err, done, cpu_s = 0.0, 0, 0.0
        while done == 0 or (cpu_s < CPU_SECONDS and done < 64 * n):
            ys, xs = rng.integers(0, H, n).astype(np.int32), rng.integers(0, W, n).astype(np.int32)
            t0 = time.perf_counter()
            ref = oracle.expanded_rangebox(Z, op, ys, xs)
            cpu_s += time.perf_counter() - t0
            err = max(err, float(np.abs(out_host[ys, xs] - ref).max()))
            done += n
        n = done
        t1 = oracle.true_bf(Z, c["sigma_s"], c["radius"], c["sigma_r"], ys[:4096], xs[:4096])
        result["max_abs_err_vs_oracle"] = err
        result["max_abs_err_vs_true_bf_4096px"] = float(np.abs(out_host[ys[:4096], xs[:4096]] - t1).max())
        result["cpu_baseline"] = {"value": round(n / cpu_s / 1e6, 4), "unit": "Mpix/s", "cores": threads,
                                  "kind": "oracle", "seconds": round(cpu_s, 2),
                                  "sample": "%d random pixels of the %dx%d image, oracle T4 (FP64 direct sum "
                                            "with the range box)" % (n, W, H)}
        model, nproc = cpu_host()
        result["cpu_baseline"].update({"cpu_model": model, "nproc": nproc})
        if one_core:
            result["cpu_baseline"]["one_core"] = {
                "value": round(one_core["mpix_s"], 5), "unit": "Mpix/s", "cores": 1,
                "sample": one_core["sample"], "seconds": round(one_core["seconds"], 2)}
        log("[bench] max-abs err vs oracle T4 %.3e" % err)
    print(json.dumps(result), flush=True)


def single_image(args, workload, pre=None):
    """One image per step (cfg1, cfg2, cfg3, cfg5): returns the result dict.
    `pre` holds what was prepared before the GPU was touched (image, one-core
    oracle leg)."""
    import torch
    import synth
    from synth.images import CONFIGS
    from paper_1803_00004_amd import bf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    c = CONFIGS[workload]
    H, W = c["H"], c["W"]
    I_host = pre["image"] if pre else synth.config_image(workload)
    one_core = pre.get("one_core") if pre else None

    t0 = time.perf_counter()
    reduced = args.precision == "reduced"
    fold = args.level_fold
    if fold and c["dtype"] != "u8":
        raise SystemExit("--level-fold needs an 8-bit workload")
    plan = bf.Plan(c["sigma_s"], c["sigma_r"], c["radius"], c["n_range"], c["n_spatial"],
                   dtype=c["dtype"], precision=args.precision, level_fold=fold)
    plan_ms = (time.perf_counter() - t0) * 1e3
    info = plan.info
    log("[bench] plan %.1f ms: %s" % (plan_ms, info.as_dict()))

    dev = torch.device("cuda:0")
    I = torch.from_numpy(I_host).to(dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    tuned = None
    if not args.no_tune and not reduced and not fold:
        t0 = time.perf_counter()
        tuned = plan.autotune(H, W, reps=5, stream=stream)
        log("[bench] autotuner: table tile %d (%.0f ms)" % (tuned, (time.perf_counter() - t0) * 1e3))
    tile, q, ws_bytes = plan.geometry(H, W)
    ws = bf.workspace(plan, H, W, dev)

    for _ in range(args.warmup):
        bf.filter(plan, I, out=out, ws=ws, stream=stream)
    torch.cuda.synchronize()
    if args.calib_copy > 0:
        n = args.calib_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] calibration copy: %d MiB read + %d MiB written" % (args.calib_copy, args.calib_copy))
        del a, b

    bf.profile_enable(True)
    bf.profile_read()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(args.steps):
        bf.filter(plan, I, out=out, ws=ws, stream=stream)
    end.record(stream)
    torch.cuda.synchronize()
    elapsed_ms = start.elapsed_time(end)
    kms, klaunch = bf.profile_read()
    bf.profile_enable(False)
    ms_per_step = elapsed_ms / args.steps
    mpix = H * W / (ms_per_step * 1e-3) / 1e6
    k_avg = [kms[i] / max(1, klaunch[i]) for i in range(2)]
    log("[bench] %.4f ms/step  %.1f Mpix/s  kernels: tables %.4f ms, lookup %.4f ms"
        % (ms_per_step, mpix, k_avg[0], k_avg[1]))
    out_host = out.cpu().numpy().astype(np.float64)

    # re-filtering the same image from tables pre-computed once (lookup only)
    refilter_ms = None
    if not reduced and not fold:
        del ws
        tables = bf.precompute(plan, I, stream=stream)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            bf.filter_precomputed(plan, plan, I, tables, out=out, stream=stream)
        end.record(stream)
        torch.cuda.synchronize()
        refilter_ms = start.elapsed_time(end) / args.steps
        del tables
        log("[bench] re-filter from pre-computed tables: %.4f ms (%.1f Mpix/s)"
            % (refilter_ms, H * W / (refilter_ms * 1e-3) / 1e6))
    del I, out
    torch.cuda.empty_cache()

    # roofline of the dominant kernel, from algorithmic work per launch
    px = H * W
    in_b = 1 if c["dtype"] == "u8" else 4
    n_img = info.n_images
    vb = 2 if reduced else 4                       # bytes per stored term value (FP16 images / int32 tables)
    ka_bytes = px * (vb * n_img + in_b)            # write every term image or table once, read I
    kb_bytes = px * (vb * n_img + in_b + 4)        # read every one once, read I, write out
    kb_flops = px * 2.0 * n_img * info.n_quads      # one FP32 FMA per quadruplet box per table
    lk = plan.lookup_kernel(H, W)  # the lookup kernel the timed calls ran (tuned or default)
    kb_name = "kr_tile" if reduced else "kz_rangebox" if fold else (
        "kl_tile" if lk == 3 else "kb_tile" if lk in (1, 2) else "kb_lookup")
    ka_name = "kr_modulate" if reduced else "ka_sat"
    if fold:
        # one kernel: integer adds of the level-slab tables it builds
        dy, dx, _ = plan.taps()
        adds = slab_table_adds(I_host, {"tap_dy_min": int(dy.min()), "tap_dy_max": int(dy.max()),
                                        "tap_dx_min": int(dx.min()), "tap_dx_max": int(dx.max())}, info.box_tile)
        tops = adds / (k_avg[1] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": tops, "peak": INT32_PEAK_TOPS, "unit": "TOP/s",
                "frac": tops / INT32_PEAK_TOPS, "kernel": "kz_rangebox", "kernel_ms": k_avg[1],
                "algorithmic_adds": adds, "traffic": None}
    else:
        dom = 1 if k_avg[1] >= k_avg[0] else 0
        if dom == 1:
            roof = hbm_roofline(kb_name, kb_bytes, k_avg[1], kb_flops)
        else:
            roof = hbm_roofline(ka_name, ka_bytes, k_avg[0])
        roof["traffic"] = recorded_traffic(workload, roof["kernel"])
        roof["other_kernel"] = hbm_roofline(ka_name, ka_bytes, k_avg[0]) if dom == 1 else \
            hbm_roofline(kb_name, kb_bytes, k_avg[1], kb_flops)
        roof["other_kernel"]["traffic"] = recorded_traffic(workload, roof["other_kernel"]["kernel"])
    # the whole path against HBM: every table written once and read once, I
    # read twice, out written once (8 n_img + 2 in_b + 4 bytes per pixel)
    path_bytes = px * (in_b + 4) if fold else px * (2 * vb * n_img + 2 * in_b + 4)
    path_gbs = path_bytes / (ms_per_step * 1e-3) / 1e9

    result = {
        "metric": METRIC, "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16+i32+f32" if reduced else "i32+f32",
        "data": "synthetic (seeded gradient noise + step edges + Gaussian noise)",
        "config": {"workload": "%s: %dx%d %s, Gaussian sigma_s=%g r=%d, sigma_r=%g, N_r=%d, N_s=%d%s"
                   % (workload, W, H, c["dtype"], c["sigma_s"], c["radius"], c["sigma_r"],
                      c["n_range"], c["n_spatial"], ", reduced precision (FP16 term images)" if reduced else
                      ", range terms folded per output level" if fold else ""),
                   "precision": args.precision, "level_fold": fold,
                   "H": H, "W": W, "table_tile": tile, "autotuned": tuned is not None, "sat_shift": q,
                   "n_images": n_img, "n_quads": info.n_quads, "workspace_bytes": ws_bytes},
        "plan_ms": round(plan_ms, 2),
        "kernel_ms": {kb_name: round(k_avg[1], 5)} if fold else {ka_name: round(k_avg[0], 5),
                                                                 kb_name: round(k_avg[1], 5)},
        "roofline": roof,
        "path_hbm": {"algorithmic_bytes_per_px": path_bytes // px, "achieved_gbs": round(path_gbs, 1),
                     "frac_of_peak": round(path_gbs / HBM_PEAK_GBS, 4)},
        "refilter_from_precomputed": None if refilter_ms is None else {
            "ms": round(refilter_ms, 5), "mpix_s": round(H * W / (refilter_ms * 1e-3) / 1e6, 2)},
    }

    if not args.no_cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        log("[bench] oracle T3 on %d threads for ~%.0f s" % (threads, CPU_SECONDS))
        err, cpu_mpix, cpu_s, sample, n_err = oracle_all_cores(I_host, c, out_host)
        rng = np.random.default_rng(12)
        ys, xs = rng.integers(0, H, 4096).astype(np.int32), rng.integers(0, W, 4096).astype(np.int32)
        t1 = oracle.true_bf(I_host, c["sigma_s"], c["radius"], c["sigma_r"], ys, xs)
        result["max_abs_err_vs_oracle"] = err
        result["max_abs_err_pixels"] = n_err
        result["max_abs_err_vs_true_bf_4096px"] = float(np.abs(out_host[ys, xs] - t1).max())
        model, nproc = cpu_host()
        result["cpu_baseline"] = {"value": round(cpu_mpix, 5), "unit": "Mpix/s", "cores": threads,
                                  "kind": "oracle", "sample": sample, "seconds": round(cpu_s, 2),
                                  "cpu_model": model, "nproc": nproc}
        if one_core:
            result["cpu_baseline"]["one_core"] = {
                "value": round(one_core["mpix_s"], 5), "unit": "Mpix/s", "cores": 1,
                "sample": one_core["sample"], "seconds": round(one_core["seconds"], 2)}
        log("[bench] max-abs err vs oracle %.3e over %d px; oracle %.4f Mpix/s" % (err, n_err, cpu_mpix))
    return result


def headline(args):
    """The default line: the 4096^2 workload, with the served stream, the
    device-copy bandwidth and the CPU oracle legs beside it."""
    import synth
    from paper_1803_00004_amd import serve
    pre = {}
    if not args.no_cpu:
        log("[bench] oracle T3 on sub-images, one core (child process)")
        pre["one_core"] = one_core_baseline(HEADLINE)
    log("[bench] generating %s" % HEADLINE)
    pre["image"] = synth.config_image(HEADLINE)
    reqs = host_imgs = None
    if not args.no_served:
        reqs = synth.gen_stream()
        t0 = time.perf_counter()
        host_imgs = serve.generate_images(reqs)  # forked pool, before the GPU is touched
        log("[served] %d request images generated in %.1f s" % (len(reqs), time.perf_counter() - t0))
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    copy_gbs = device_copy_gbs(torch, dev)
    log("[bench] device copy %.0f GB/s (read + write)" % copy_gbs)
    result = single_image(args, HEADLINE, pre)
    result["device_copy_gbs"] = round(copy_gbs, 1)
    result["roofline"]["achievable_copy_gbs"] = round(copy_gbs, 1)
    if reqs is not None:
        fields, _, _ = served_run(args, reqs, host_imgs, not args.no_cpu)
        result["served"] = fields
    print(json.dumps(result), flush=True)


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--oracle-one-core":
        return oracle_one_core(sys.argv[2])
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=None,
                    choices=["cfg1_256", "cfg2_1080p", "cfg3_4096", "cfg4_served", "cfg5_4096_u8",
                             "cfg6_1080p_u8_box"],
                    help="one workload alone (default: the 4096^2 headline with the served stream beside it)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs (no error check)")
    ap.add_argument("--no-served", action="store_true", help="headline without the served stream")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (heuristic tiling)")
    ap.add_argument("--served-streams", type=int, default=2, help="served stream: the request loop's streams")
    ap.add_argument("--served-max-batch", type=int, default=16, help="served stream: largest batch")
    ap.add_argument("--fused-batch", action="store_true",
                    help="served stream: each eligible batch as one fused launch (bf_batch_set_fused; "
                         "its time is all counted as lookup)")
    ap.add_argument("--precision", choices=["plain", "reduced"], default="plain",
                    help="reduced: FP16 term images, tables built in LDS (single-image workloads)")
    ap.add_argument("--level-fold", action="store_true",
                    help="8-bit workloads: range terms folded per output level (BF_FLAG_LEVEL_FOLD)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="also run one device copy of MIB MiB (a reference kernel of known "
                         "traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (served requests "
              "would shard across GPUs by request, and one large image into row bands with an r-row "
              "halo, without collectives).", file=sys.stderr)
        sys.exit(2)

    if args.workload is None:
        return headline(args)
    if args.workload == "cfg4_served":
        return served(args)
    if args.workload == "cfg6_1080p_u8_box":
        return range_box(args)
    import synth
    pre = {}
    if not args.no_cpu:
        log("[bench] oracle one core (child process)")
        pre["one_core"] = one_core_baseline(args.workload)
    log("[bench] generating %s" % args.workload)
    pre["image"] = synth.config_image(args.workload)
    print(json.dumps(single_image(args, args.workload, pre)), flush=True)


if __name__ == "__main__":
    main()
