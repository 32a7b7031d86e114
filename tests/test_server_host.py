"""The serving loop's queue, admission and batching logic, on the CPU: the
server's dry run executes no device work and completes a batch when the
caller's clock passes launch time + pixels / rate."""
import numpy as np
import pytest

import synth
from paper_1803_00004_amd import bf

FAKE_I, FAKE_O = 0x1000, 0x2000


def _plans():
    return {ss: bf.Plan(ss, 0.1, int(3 * ss), 8, 4, host_only=True) for ss in (2.0, 4.0, 8.0, 16.0)}


def _drain(srv, now, dt=1e-4, limit=100000):
    out = []
    for _ in range(limit):
        out += srv.poll(now)
        q, f = srv.pending()
        if q == 0 and f == 0:
            return out, now
        now += dt
    raise AssertionError("server did not drain")


def test_every_request_completes_once_in_fifo_batches():
    plans = _plans()
    srv = bf.Server(hbm_budget=8 << 30, max_batch=5, n_streams=2, dry_run=True, dry_rate=2e9)
    rng = np.random.default_rng(1)
    n = 60
    for i in range(n):
        p = plans[float(rng.choice([2.0, 4.0, 8.0, 16.0]))]
        srv.submit(p, FAKE_I, FAKE_O, tag=i, now=0.0, H=int(rng.integers(64, 700)), W=int(rng.integers(64, 700)))
    done, _ = _drain(srv, 0.0)
    assert sorted(c.tag for c in done) == list(range(n))
    assert all(c.status == bf.BF_OK for c in done)
    batch = {c.tag: c.batch for c in done}
    # the queue head is never overtaken: batch numbers follow submission order
    assert all(batch[i] <= batch[i + 1] for i in range(n - 1))
    st = srv.stats()
    assert st.completed == n and st.submitted == n
    assert sum(st.batch_size_hist[k] * k for k in range(65)) == n
    assert all(st.batch_size_hist[k] == 0 for k in range(6, 65))
    assert st.peak_batches_in_flight <= 2


HEADS = 1024  # a batch's work-queue heads (bf_batch_workspace_size of an empty batch)


def test_admission_keeps_the_arena_budget():
    plans = _plans()
    p = plans[16.0]
    one = (p.workspace_size(1500, 1500) + 255) // 256 * 256
    budget = HEADS + 2 * one + 1000  # room for two such requests at once, not three
    srv = bf.Server(hbm_budget=budget, max_batch=8, n_streams=4, dry_run=True, dry_rate=1e9)
    for i in range(7):
        srv.submit(p, FAKE_I, FAKE_O, tag=i, now=0.0, H=1500, W=1500)
    done, _ = _drain(srv, 0.0)
    st = srv.stats()
    assert st.completed == 7
    assert st.peak_arena_bytes <= st.arena_bytes
    assert st.peak_requests_in_flight <= 2
    assert max(c.batch_size for c in done) <= 2


def test_oversized_request_fails_alone_and_does_not_block():
    plans = _plans()
    small = (plans[2.0].workspace_size(100, 100) + 255) // 256 * 256
    srv = bf.Server(hbm_budget=HEADS + 4 * small, max_batch=8, n_streams=2, dry_run=True)
    srv.submit(plans[16.0], FAKE_I, FAKE_O, tag=0, now=0.0, H=2048, W=2048)
    for i in range(1, 4):
        srv.submit(plans[2.0], FAKE_I, FAKE_O, tag=i, now=0.0, H=100, W=100)
    done, _ = _drain(srv, 0.0)
    st = {c.tag: c.status for c in done}
    assert st[0] == bf.BF_ERR_OUT_OF_MEMORY
    assert all(st[i] == bf.BF_OK for i in (1, 2, 3))


def test_continuous_batching_overlaps_new_arrivals():
    """A request that arrives while a batch runs starts at once on the free
    stream; it does not wait for the running batch."""
    p = _plans()[4.0]
    rate = 1e8
    srv = bf.Server(hbm_budget=8 << 30, max_batch=4, n_streams=2, dry_run=True, dry_rate=rate)
    srv.submit(p, FAKE_I, FAKE_O, tag=0, now=0.0, H=2000, W=2000)  # 40 ms
    srv.submit(p, FAKE_I, FAKE_O, tag=1, now=0.005, H=200, W=200)  # arrives while 0 runs
    done = srv.poll(0.0061)
    assert [c.tag for c in done] == [1]
    assert abs(done[0].t_launch - 0.005) < 1e-12
    rest, _ = _drain(srv, 0.0062)
    assert [c.tag for c in rest] == [0]
    assert srv.stats().peak_batches_in_flight == 2


def test_single_stream_serialises_batches():
    p = _plans()[2.0]
    rate = 1e8
    srv = bf.Server(max_batch=2, n_streams=1, dry_run=True, dry_rate=rate)
    for i in range(4):
        srv.submit(p, FAKE_I, FAKE_O, tag=i, now=0.0, H=1000, W=1000)  # 10 ms each
    done, _ = _drain(srv, 0.0, dt=1e-3)
    launch = {c.tag: c.t_launch for c in done}
    # work-conserving: the first request starts alone at once; the next two
    # share the batch launched when the stream frees (10 ms), the last one
    # follows that batch (20 ms later)
    assert launch[0] == 0.0
    assert abs(launch[1] - 0.01) < 1.5e-3 and launch[1] == launch[2]
    assert abs(launch[3] - 0.03) < 2.5e-3
    assert srv.stats().peak_batches_in_flight == 1


def test_served_stream_schedule_dry_run():
    """The 512-request served stream (Poisson arrivals, mixed sizes and
    sigmas) through the real admission logic with its real workspace sizes."""
    reqs = synth.gen_stream()
    assert len(reqs) == 512
    plans = {}
    for r in reqs:
        key = (r["sigma_s"], r["radius"], r["n_spatial"], r["sigma_r"], r["n_range"])
        if key not in plans:
            plans[key] = bf.Plan(r["sigma_s"], r["sigma_r"], r["radius"], r["n_range"], r["n_spatial"],
                                 host_only=True)
    assert len(plans) == 16
    srv = bf.Server(hbm_budget=48 << 30, max_batch=16, n_streams=2, dry_run=True, dry_rate=1.5e9)
    done, i, now = [], 0, 0.0
    while len(done) < len(reqs):
        while i < len(reqs) and reqs[i]["t_arrive"] <= now:
            r = reqs[i]
            key = (r["sigma_s"], r["radius"], r["n_spatial"], r["sigma_r"], r["n_range"])
            srv.submit(plans[key], FAKE_I, FAKE_O, tag=i, now=now, H=r["H"], W=r["W"])
            i += 1
        done += srv.poll(now)
        now += 2e-5
    assert sorted(c.tag for c in done) == list(range(512))
    st = srv.stats()
    assert st.peak_arena_bytes <= st.arena_bytes
    assert st.batches < 512  # requests were batched
    lat = np.array([c.t_done - reqs[c.tag]["t_arrive"] for c in done])
    assert (lat >= 0).all()


def test_server_argument_errors():
    with pytest.raises(bf.BFError):
        bf.Server(n_streams=9, dry_run=True)
    srv = bf.Server(dry_run=True)
    p = _plans()[2.0]
    with pytest.raises(bf.BFError):
        srv.submit(p, FAKE_I, FAKE_O, tag=0, now=0.0, H=0, W=10)
    with pytest.raises(bf.BFError):
        srv.submit(p, 0, FAKE_O, tag=0, now=0.0, H=10, W=10)
