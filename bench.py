"""Benchmark of the N-term bilateral filter on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu]

Single-image workloads: a step is one bf_filter call on one image already
resident in HBM: term modulation + summed-area tables (kernel 0) and tap
lookup, accumulation and normalisation (kernel 1).  The plan (FP64 host fit)
is built once per parameter set, timed separately and reported as plan_ms.

cfg6_1080p_u8_box: the paper's own 8-bit regime (range series on [-T_r,
T_r] with the range box, BF_FLAG_RANGE_BOX): one kernel per image; its
roofline counts the integer adds of the level-slab tables it builds.

cfg4_served: one pass of the 512-request served stream through the
library's request loop (open loop, Poisson arrivals); value is pixels served
per second over the makespan, with p50/p99 latency, and beside it the same
requests all queued at once (batched, closed loop) and one at a time with
bf_filter.

Prints ONE JSON line; diagnostics go to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s at fixed max-abs err vs FP64 oracle; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6    # MI355X FP64 vector
CPU_SECONDS = 10.0         # oracle work timed for the CPU baseline (each leg)
INT32_PEAK_TOPS = 39.3     # 256 CUs x 64 lanes x 2.4 GHz, one 32-bit add per lane per clock


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


def kb_roofline(kms, klaunch, ka_bytes, kb_bytes, kb_flops, kb_name, ka_name="ka_sat"):
    """Roofline of the dominant kernel from per-kernel times (ms summed over
    the timed launches) and algorithmic work summed over the same launches."""
    names = [ka_name, kb_name]
    dom = 0 if kms[0] >= kms[1] else 1
    t = kms[dom] * 1e-3
    if dom == 0:
        a = ka_bytes / t / 1e9
        roof = {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS}
    else:
        gbs = kb_bytes / t / 1e9
        tfl = kb_flops / t / 1e12
        if gbs / HBM_PEAK_GBS >= tfl / FP64_PEAK_TFLOPS:
            roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
        else:
            roof = {"bound": "alu", "achieved": tfl, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tfl / FP64_PEAK_TFLOPS}
    roof["kernel"] = names[dom]
    roof["kernel_ms"] = kms[dom] / max(1, klaunch[dom])
    return roof, dom


def served(args):
    import synth
    from paper_1803_00004_amd import serve

    reqs = synth.gen_stream()
    n = len(reqs)
    t0 = time.perf_counter()
    host_imgs = serve.generate_images(reqs)  # before the GPU is touched (forked pool)
    log("[served] %d request images generated in %.1f s" % (n, time.perf_counter() - t0))

    import torch
    from paper_1803_00004_amd import bf
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.perf_counter()
    plans = serve.make_plans(reqs)
    plan_ms = (time.perf_counter() - t0) * 1e3
    dev = torch.device("cuda:0")
    imgs = [torch.from_numpy(I).to(dev) for I in host_imgs]
    outs = [torch.empty(I.shape, dtype=torch.float32, device=dev) for I in imgs]
    alone = [torch.empty(I.shape, dtype=torch.float32, device=dev) for I in imgs]
    px = np.array([r["H"] * r["W"] for r in reqs], dtype=np.float64)
    budget, max_batch, n_streams = 48 << 30, 16, 2
    srv = bf.Server(hbm_budget=budget, max_batch=max_batch, n_streams=n_streams)
    log("[served] %d plans in %.0f ms; %.1f Mpx in total; warm-up" % (len(plans), plan_ms, px.sum() / 1e6))
    for _ in range(max(1, args.warmup)):
        serve.run_closed_loop(srv, reqs[:32], plans, imgs[:32], outs[:32])
    serve.run_plain(reqs[:32], plans, imgs[:32], alone[:32])

    bf.profile_enable(True)
    bf.profile_read()
    done, makespan = serve.run_open_loop(srv, reqs, plans, imgs, outs)
    kms, klaunch = bf.profile_read()
    bf.profile_enable(False)
    st = srv.stats()
    lat = serve.latency_summary(reqs, done)
    thr_open = px.sum() / makespan / 1e6
    log("[served] open loop: makespan %.1f ms, %.1f Mpix/s, p50 %.2f ms, p99 %.2f ms, %d batches"
        % (makespan * 1e3, thr_open, lat["p50_ms"], lat["p99_ms"], st.batches))
    _, mk_closed = serve.run_closed_loop(srv, reqs, plans, imgs, outs)
    thr_closed = px.sum() / mk_closed / 1e6
    t_plain = serve.run_plain(reqs, plans, imgs, alone)
    thr_plain = px.sum() / t_plain / 1e6
    torch.cuda.synchronize()
    n_equal = sum(bool(torch.equal(outs[i], alone[i])) for i in range(n))
    log("[served] closed loop %.1f Mpix/s; one at a time %.1f Mpix/s; %d/%d results bitwise equal alone"
        % (thr_closed, thr_plain, n_equal, n))
    # the same stream with direct summation where it is cheaper (small
    # windows: those requests get the exact bilateral filter)
    auto_plans = {k: bf.Plan(k[0], k[3], k[1], k[4], k[2], direct="auto") for k in plans}
    n_direct = sum(1 for r in reqs if auto_plans[serve.plan_key(r)].info.direct)
    serve.run_closed_loop(srv, reqs[:32], auto_plans, imgs[:32], outs[:32])
    done_a, mk_a = serve.run_open_loop(srv, reqs, auto_plans, imgs, outs)
    lat_a = serve.latency_summary(reqs, done_a)
    _, mk_ac = serve.run_closed_loop(srv, reqs, auto_plans, imgs, outs)
    log("[served] with direct summation for %d small-window requests: open loop %.1f Mpix/s p50 %.2f ms p99 %.2f ms; "
        "closed loop %.1f Mpix/s" % (n_direct, px.sum() / mk_a / 1e6, lat_a["p50_ms"], lat_a["p99_ms"], px.sum() / mk_ac / 1e6))
    srv.close()

    ka_b = kb_b = kb_f = 0.0
    for r in reqs:
        info = plans[serve.plan_key(r)].info
        p = r["H"] * r["W"]
        ka_b += p * (4 * info.n_images + 4)
        kb_b += p * (4 * info.n_images + 8)
        kb_f += p * 2.0 * info.n_images * info.n_taps
    roof, _ = kb_roofline(kms, klaunch, ka_b, kb_b, kb_f, "kb_tile")
    roof["traffic"] = None
    result = {
        "metric": METRIC, "value": round(thr_open, 2), "unit": "Mpix/s", "n_gpus": 1,
        "steps": 1, "warmup": args.warmup, "ms_per_step": round(makespan * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32+f64",
        "data": "synthetic (seeded gradient noise + step edges + Gaussian noise per request)",
        "config": {"workload": "cfg4_served: 512 requests, Poisson 2000/s, H, W ~ U{128..2048}, "
                               "sigma_s in {2,4,8,16} (r = 3 sigma_s), sigma_r in {0.05,0.1,0.2,0.3}, "
                               "N_r = clamp(ceil(1.6/sigma_r), 8, 32), N_s = 4",
                   "hbm_budget_bytes": budget, "max_batch": max_batch, "streams": n_streams},
        "served": {"p50_ms": round(lat["p50_ms"], 3), "p99_ms": round(lat["p99_ms"], 3),
                   "mean_ms": round(lat["mean_ms"], 3), "makespan_ms": round(makespan * 1e3, 2),
                   "open_loop_mpix_s": round(thr_open, 2), "closed_loop_batched_mpix_s": round(thr_closed, 2),
                   "one_at_a_time_mpix_s": round(thr_plain, 2), "batches": int(st.batches),
                   "peak_batches_in_flight": st.peak_batches_in_flight,
                   "peak_requests_in_flight": st.peak_requests_in_flight,
                   "peak_workspace_bytes": int(st.peak_arena_bytes),
                   "batch_size_hist": {str(k): int(st.batch_size_hist[k]) for k in range(65) if st.batch_size_hist[k]},
                   "results_bitwise_equal_alone": "%d/%d" % (n_equal, n),
                   "with_direct_auto": {"requests_direct": n_direct,
                                        "open_loop_mpix_s": round(px.sum() / mk_a / 1e6, 2),
                                        "p50_ms": round(lat_a["p50_ms"], 3), "p99_ms": round(lat_a["p99_ms"], 3),
                                        "closed_loop_mpix_s": round(px.sum() / mk_ac / 1e6, 2)}},
        "plan_ms": round(plan_ms, 1),
        "kernel_ms_total": {"ka_sat": round(kms[0], 3), "kb_lookup": round(kms[1], 3)},
        "roofline": roof,
    }
    if not args.no_cpu:
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        rng = np.random.default_rng(21)
        errs, n_px, cpu_s = [], 0, 0.0
        for i in range(32):
            r = reqs[i]
            op = oracle.make_plan(r["sigma_s"], r["radius"], r["n_spatial"], r["sigma_r"], r["n_range"])
            ys = rng.integers(0, r["H"], 64).astype(np.int32)
            xs = rng.integers(0, r["W"], 64).astype(np.int32)
            t1 = time.perf_counter()
            ref = oracle.expanded_brute(host_imgs[i], op, ys, xs)
            cpu_s += time.perf_counter() - t1
            n_px += 64
            errs.append(float(np.abs(outs[i].cpu().numpy()[ys, xs] - ref).max()))
        result["max_abs_err_vs_oracle"] = max(errs)
        result["cpu_baseline"] = {"value": round(n_px / cpu_s / 1e6, 5), "unit": "Mpix/s", "cores": threads,
                                  "kind": "oracle", "seconds": round(cpu_s, 2),
                                  "sample": "64 random pixels of each of the first 32 requests, oracle T2 "
                                            "(FP64 direct sum of the expanded form)"}
        log("[served] max-abs err vs oracle (32 requests x 64 px) %.3e" % max(errs))
    print(json.dumps(result), flush=True)


def oracle_one_core(workload, n):
    """Child-process mode (OMP_NUM_THREADS=1): time oracle T2 on n sampled
    pixels of the workload's image and print one JSON line."""
    import oracle
    import synth
    from synth.images import CONFIGS
    c = CONFIGS[workload]
    I_host = synth.config_image(workload)
    box = c.get("range_box", False)
    op = oracle.make_plan(c["sigma_s"], c["radius"], c["n_spatial"], c["sigma_r"], c["n_range"],
                          **({"span": 0.0} if box else {}))
    rng = np.random.default_rng(13)
    done, dt = 0, 0.0
    while done == 0 or (dt < CPU_SECONDS and done < 64 * n):  # batches of n pixels for ~CPU_SECONDS
        ys = rng.integers(0, c["H"], n).astype(np.int32)
        xs = rng.integers(0, c["W"], n).astype(np.int32)
        t0 = time.perf_counter()
        (oracle.expanded_rangebox if box else oracle.expanded_brute)(I_host, op, ys, xs)
        dt += time.perf_counter() - t0
        done += n
    print(json.dumps({"mpix_s": done / dt / 1e6, "seconds": dt, "pixels": done}))


def one_core_baseline(workload, n):
    """The oracle on one host core, timed in a child process started before
    this process touches the GPU."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-core", workload, str(n)],
                       env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        log("[bench] one-core oracle failed: %s" % r.stderr[-500:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


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
        log("[bench] oracle T4 on 16384 sampled pixels, one core (child process)")
        one_core = one_core_baseline(w, 16384)
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
        "dtype": "i32+f64", "data": "synthetic (seeded gradient noise + step edges + Gaussian noise)",
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
        if one_core:
            result["cpu_baseline"]["one_core"] = {
                "value": round(one_core["mpix_s"], 5), "unit": "Mpix/s", "cores": 1,
                "sample": "%d random pixels, oracle T4" % one_core["pixels"],
                "seconds": round(one_core["seconds"], 2)}
        log("[bench] max-abs err vs oracle T4 %.3e" % err)
    print(json.dumps(result), flush=True)


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--oracle-one-core":
        return oracle_one_core(sys.argv[2], int(sys.argv[3]))
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg2_1080p",
                    choices=["cfg1_256", "cfg2_1080p", "cfg3_4096", "cfg4_served", "cfg5_4096_u8",
                             "cfg6_1080p_u8_box"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (no error check)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (heuristic tiling)")
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

    if args.workload == "cfg4_served":
        return served(args)
    if args.workload == "cfg6_1080p_u8_box":
        return range_box(args)

    import torch
    import synth
    from synth.images import CONFIGS
    from paper_1803_00004_amd import bf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    c = CONFIGS[args.workload]
    H, W = c["H"], c["W"]
    log("[bench] generating %s %dx%d" % (args.workload, H, W))
    I_host = synth.config_image(args.workload)

    one_core = None
    if not args.no_cpu:
        n1 = 1024 if c["H"] * c["W"] > 4 * 1024 * 1024 else 4096  # a few seconds of one core
        log("[bench] oracle T2 on %d sampled pixels, one core (child process)" % n1)
        one_core = one_core_baseline(args.workload, n1)

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

    # re-filtering the same image from tables pre-computed once (lookup only)
    refilter_ms = None
    if not reduced and not fold:
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

    # roofline of the dominant kernel, from algorithmic work per launch
    px = H * W
    in_b = 1 if c["dtype"] == "u8" else 4
    n_img = info.n_images
    vb = 2 if reduced else 4                       # bytes per stored term value (FP16 images / int32 tables)
    ka_bytes = px * (vb * n_img + in_b)            # write every term image or table once, read I
    kb_bytes = px * (vb * n_img + in_b + 4)        # read every one once, read I, write out
    kb_flops = px * 2.0 * n_img * info.n_taps      # one FP64 FMA per tap per table
    kb_name = "kr_tile" if reduced else "kz_rangebox" if fold else (
        "kb_tile" if info.lookup_kernel == 1 else "kb_lookup")
    roof_names = ["kr_modulate" if reduced else "ka_sat", kb_name]
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
        roof, dom = kb_roofline(k_avg, [1, 1], ka_bytes, kb_bytes, kb_flops, kb_name, roof_names[0])
        roof["traffic"] = recorded_traffic(args.workload, roof["kernel"])
    # the whole path against HBM: every table written once and read once, I
    # read twice, out written once (8 n_img + 2 in_b + 4 bytes per pixel)
    path_bytes = px * (in_b + 4) if fold else px * (2 * vb * n_img + 2 * in_b + 4)
    path_gbs = path_bytes / (ms_per_step * 1e-3) / 1e9

    result = {
        "metric": METRIC, "value": round(mpix, 2), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16+i32+f64" if reduced else "i32+f64",
        "data": "synthetic (seeded gradient noise + step edges + Gaussian noise)",
        "config": {"workload": "%s: %dx%d %s, Gaussian sigma_s=%g r=%d, sigma_r=%g, N_r=%d, N_s=%d%s"
                   % (args.workload, W, H, c["dtype"], c["sigma_s"], c["radius"], c["sigma_r"],
                      c["n_range"], c["n_spatial"], ", reduced precision (FP16 term images)" if reduced else
                      ", range terms folded per output level" if fold else ""),
                   "precision": args.precision, "level_fold": fold,
                   "H": H, "W": W, "table_tile": tile, "autotuned": tuned is not None, "sat_shift": q,
                   "n_images": n_img, "n_taps": info.n_taps, "workspace_bytes": ws_bytes},
        "plan_ms": round(plan_ms, 2),
        "kernel_ms": {kb_name: round(k_avg[1], 5)} if fold else {roof_names[0]: round(k_avg[0], 5),
                                                                 kb_name: round(k_avg[1], 5)},
        "roofline": roof,
        "path_hbm": {"algorithmic_bytes_per_px": path_bytes // px, "achieved_gbs": round(path_gbs, 1),
                     "frac_of_peak": round(path_gbs / HBM_PEAK_GBS, 4)},
        "refilter_from_precomputed": None if refilter_ms is None else {
            "ms": round(refilter_ms, 5), "mpix_s": round(H * W / (refilter_ms * 1e-3) / 1e6, 2)},
    }

    if not args.no_cpu:
        import oracle
        out_host = out.cpu().numpy().astype(np.float64)
        op = oracle.make_plan(c["sigma_s"], c["radius"], c["n_spatial"], c["sigma_r"], c["n_range"])
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        # the oracle is run again until about CPU_SECONDS of work have been timed
        if px <= 4 * 1024 * 1024:
            log("[bench] oracle T3 on the full image (%d threads), repeated for ~%.0f s" % (threads, CPU_SECONDS))
            reps, cpu_s = 0, 0.0
            while reps == 0 or (cpu_s < CPU_SECONDS and reps < 64):
                t0 = time.perf_counter()
                ref = oracle.expanded_box(I_host, op)
                cpu_s += time.perf_counter() - t0
                reps += 1
            err = float(np.abs(out_host - ref).max())
            sample = "full %dx%d image x %d, oracle T3 (FP64 shift identity + box sums)" % (W, H, reps)
            cpu_mpix = reps * px / cpu_s / 1e6
        else:
            n = 2048
            rng = np.random.default_rng(11)
            log("[bench] oracle T2 on sampled pixels (%d threads), batches of %d for ~%.0f s" % (threads, n, CPU_SECONDS))
            err, done, cpu_s = 0.0, 0, 0.0
            while done == 0 or (cpu_s < CPU_SECONDS and done < 64 * n):
                ys, xs = rng.integers(0, H, n).astype(np.int32), rng.integers(0, W, n).astype(np.int32)
                t0 = time.perf_counter()
                ref = oracle.expanded_brute(I_host, op, ys, xs)
                cpu_s += time.perf_counter() - t0
                err = max(err, float(np.abs(out_host[ys, xs] - ref).max()))
                done += n
            sample = "%d random pixels of the %dx%d image, oracle T2 (FP64 direct sum)" % (done, W, H)
            cpu_mpix = done / cpu_s / 1e6
        rng = np.random.default_rng(12)
        ys, xs = rng.integers(0, H, 4096).astype(np.int32), rng.integers(0, W, 4096).astype(np.int32)
        t1 = oracle.true_bf(I_host, c["sigma_s"], c["radius"], c["sigma_r"], ys, xs)
        result["max_abs_err_vs_oracle"] = err
        result["max_abs_err_vs_true_bf_4096px"] = float(np.abs(out_host[ys, xs] - t1).max())
        result["cpu_baseline"] = {"value": round(cpu_mpix, 4), "unit": "Mpix/s", "cores": threads,
                                  "kind": "oracle", "sample": sample, "seconds": round(cpu_s, 2)}
        if one_core:
            result["cpu_baseline"]["one_core"] = {
                "value": round(one_core["mpix_s"], 5), "unit": "Mpix/s", "cores": 1,
                "sample": "%d random pixels, oracle T2 (FP64 direct sum)" % one_core["pixels"],
                "seconds": round(one_core["seconds"], 2)}
        log("[bench] max-abs err vs oracle %.3e; oracle %.3f Mpix/s" % (err, cpu_mpix))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
