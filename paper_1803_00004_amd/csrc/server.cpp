// Serving loop over bf_filter_batch: FIFO queue, HBM-footprint admission
// from a workspace arena, continuous batching over several streams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <vector>

#include "bf.h"
#include "bf_internal.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct Request {
  unsigned long long tag;
  bf_plan_t plan;
  const void *I;
  float *out;
  int H, W;
  size_t ws;  // aligned workspace bytes of this image in a batch
};

struct Batch {
  int id = -1;
  int stream = -1;
  size_t off = 0, bytes = 0;
  std::vector<Request> reqs;
  bf_status_t status = BF_OK;
  double t_launch = 0, t_sim_done = 0;
  hipEvent_t ev = nullptr;
};

// First-fit allocator over [0, cap) with coalescing free list.
struct Arena {
  size_t cap = 0;
  std::vector<std::pair<size_t, size_t>> free_;  // (offset, length), sorted by offset
  void reset(size_t c) {
    cap = c;
    free_.assign(1, {0, c});
  }
  size_t largest() const {
    size_t m = 0;
    for (auto &f : free_) m = std::max(m, f.second);
    return m;
  }
  bool alloc(size_t n, size_t *off) {
    for (size_t i = 0; i < free_.size(); ++i)
      if (free_[i].second >= n) {
        *off = free_[i].first;
        free_[i].first += n;
        free_[i].second -= n;
        if (free_[i].second == 0) free_.erase(free_.begin() + i);
        return true;
      }
    return false;
  }
  void release(size_t off, size_t n) {
    auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (size_t)0));
    it = free_.insert(it, {off, n});
    size_t i = it - free_.begin();
    if (i + 1 < free_.size() && free_[i].first + free_[i].second == free_[i + 1].first) {
      free_[i].second += free_[i + 1].second;
      free_.erase(free_.begin() + i + 1);
    }
    if (i > 0 && free_[i - 1].first + free_[i - 1].second == free_[i].first) {
      free_[i - 1].second += free_[i].second;
      free_.erase(free_.begin() + i);
    }
  }
  size_t used() const {
    size_t f = 0;
    for (auto &x : free_) f += x.second;
    return cap - f;
  }
};

}  // namespace

struct bf_server_s {
  bf_server_opts_t o{};
  bool dry = false;
  void *arena_mem = nullptr;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<int> stream_busy;
  std::vector<double> stream_sim_free;  // dry run: when each stream's last batch ends
  std::deque<Request> queue;
  std::vector<Batch> inflight;
  std::deque<bf_completion_t> done;
  bf_server_stats_t st{};
  int next_batch = 0;
  int inflight_requests = 0;
};

namespace {

void finish(bf_server_s *s, Batch &b, double now) {
  for (const Request &r : b.reqs) {
    bf_completion_t c{};
    c.tag = r.tag;
    c.status = b.status;
    c.batch = b.id;
    c.batch_size = (int)b.reqs.size();
    c.t_launch = b.t_launch;
    c.t_done = now;
    s->done.push_back(c);
  }
  s->st.completed += (long long)b.reqs.size();
  s->inflight_requests -= (int)b.reqs.size();
  if (b.bytes) s->arena.release(b.off, b.bytes);
  if (b.stream >= 0) s->stream_busy[b.stream] = 0;
  if (b.ev) (void)hipEventDestroy(b.ev);
  b.ev = nullptr;
}

bf_status_t launch(bf_server_s *s, Batch &b) {
  if (s->dry) return BF_OK;
  const int n = (int)b.reqs.size();
  std::vector<bf_plan_t> plans(n);
  std::vector<const void *> I(n);
  std::vector<float *> out(n);
  std::vector<int> H(n), W(n);
  for (int i = 0; i < n; ++i) {
    plans[i] = b.reqs[i].plan;
    I[i] = b.reqs[i].I;
    out[i] = b.reqs[i].out;
    H[i] = b.reqs[i].H;
    W[i] = b.reqs[i].W;
  }
  hipStream_t st = s->streams[b.stream];
  bf_status_t r = bf_filter_batch(plans.data(), n, I.data(), out.data(), H.data(), W.data(),
                                  static_cast<char *>(s->arena_mem) + b.off, b.bytes, st);
  if (r != BF_OK) return r;
  if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) return BF_ERR_DEVICE;
  if (hipEventRecord(b.ev, st) != hipSuccess) return BF_ERR_DEVICE;
  return BF_OK;
}

// Launch batches while a stream is free and the queue head fits.
void schedule(bf_server_s *s, double now) {
  for (;;) {
    if (s->queue.empty()) return;
    int stream = -1;
    for (int i = 0; i < (int)s->stream_busy.size(); ++i)
      if (!s->stream_busy[i]) {
        stream = i;
        break;
      }
    if (stream < 0) return;
    // requests that can never fit complete with an error
    const Request &h = s->queue.front();
    if (bf::kBatchHeadBytes + h.ws > s->arena.cap) {
      Batch b;
      b.id = -1;
      b.status = BF_ERR_OUT_OF_MEMORY;
      b.reqs.push_back(h);
      s->queue.pop_front();
      s->inflight_requests += 1;
      finish(s, b, now);
      continue;
    }
    const size_t room = s->arena.largest();
    size_t need = bf::kBatchHeadBytes;  // the batch's work-queue heads
    size_t take = 0;
    for (const Request &r : s->queue) {
      if ((int)take >= s->o.max_batch || need + r.ws > room) break;
      need += r.ws;
      ++take;
    }
    if (take == 0) return;  // wait for memory (the head is never overtaken)
    Batch b;
    b.id = s->next_batch++;
    b.stream = stream;
    b.bytes = need;
    if (!s->arena.alloc(need, &b.off)) return;
    for (size_t i = 0; i < take; ++i) {
      b.reqs.push_back(s->queue.front());
      s->queue.pop_front();
    }
    b.t_launch = now;
    s->stream_busy[stream] = 1;
    s->inflight_requests += (int)take;
    s->st.batches += 1;
    s->st.batch_size_hist[std::min<size_t>(take, 64)] += 1;
    s->st.peak_arena_bytes = std::max(s->st.peak_arena_bytes, s->arena.used());
    s->st.peak_requests_in_flight = std::max(s->st.peak_requests_in_flight, s->inflight_requests);
    if (s->dry) {
      double px = 0;
      for (const Request &r : b.reqs) px += (double)r.H * r.W;
      const double start = std::max(now, s->stream_sim_free[stream]);
      b.t_sim_done = start + px / s->o.dry_rate;
      s->stream_sim_free[stream] = b.t_sim_done;
    }
    b.status = launch(s, b);
    s->inflight.push_back(std::move(b));
    s->st.peak_batches_in_flight = std::max(s->st.peak_batches_in_flight, (int)s->inflight.size());
    if (s->inflight.back().status != BF_OK) {
      // part of the batch may be enqueued: let it drain before its arena
      // region is handed to another batch
      Batch f = std::move(s->inflight.back());
      s->inflight.pop_back();
      if (!s->dry) (void)hipStreamSynchronize(s->streams[f.stream]);
      finish(s, f, now);
    }
  }
}

// Retire every batch that has finished.
void retire(bf_server_s *s, double now) {
  for (size_t i = 0; i < s->inflight.size();) {
    Batch &b = s->inflight[i];
    bool fin;
    if (s->dry) {
      fin = now >= b.t_sim_done;
    } else {
      const hipError_t q = hipEventQuery(b.ev);
      fin = q != hipErrorNotReady;
      if (fin && q != hipSuccess) b.status = BF_ERR_DEVICE;
    }
    if (fin) {
      finish(s, b, now);
      s->inflight.erase(s->inflight.begin() + i);
    } else {
      ++i;
    }
  }
}

}  // namespace

extern "C" {

bf_status_t bf_server_create(bf_server_t *server, const bf_server_opts_t *opts) {
  if (!server) return BF_ERR_INVALID_ARG;
  *server = nullptr;
  bf_server_opts_t o{};
  if (opts) o = *opts;
  if (o.hbm_budget == 0) o.hbm_budget = (size_t)16 << 30;
  if (o.max_batch == 0) o.max_batch = 32;
  if (o.n_streams == 0) o.n_streams = 2;
  if (o.dry_rate <= 0) o.dry_rate = 1e9;
  if (o.max_batch < 1 || o.n_streams < 1 || o.n_streams > 8 || o.hbm_budget < 2 * kAlign)
    return BF_ERR_INVALID_ARG;
  auto *s = new bf_server_s;
  s->o = o;
  s->dry = (o.flags & BF_SERVER_DRY_RUN) != 0;
  s->arena.reset(o.hbm_budget / kAlign * kAlign);
  s->stream_busy.assign(o.n_streams, 0);
  s->stream_sim_free.assign(o.n_streams, 0.0);
  s->st.arena_bytes = s->arena.cap;
  if (!s->dry) {
    if (hipMalloc(&s->arena_mem, s->arena.cap) != hipSuccess) {
      delete s;
      return BF_ERR_OUT_OF_MEMORY;
    }
    for (int i = 0; i < o.n_streams; ++i) {
      hipStream_t st = nullptr;
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        bf_server_destroy(s);
        return BF_ERR_DEVICE;
      }
      s->streams.push_back(st);
    }
  }
  *server = s;
  return BF_OK;
}

bf_status_t bf_server_destroy(bf_server_t s) {
  if (!s) return BF_OK;
  for (Batch &b : s->inflight)
    if (b.ev) {
      (void)hipEventSynchronize(b.ev);
      (void)hipEventDestroy(b.ev);
    }
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  delete s;
  return BF_OK;
}

bf_status_t bf_server_submit(bf_server_t s, bf_plan_t plan, const void *I, float *out, int H, int W,
                             unsigned long long tag, double now) {
  if (!s || !plan || !I || !out) return BF_ERR_INVALID_ARG;
  size_t ws = 0;
  bf_status_t st = bf_workspace_size(plan, H, W, &ws);
  if (st != BF_OK) return st;
  if (!s->dry) {
    if (plan->flags & BF_FLAG_HOST_ONLY) return BF_ERR_INVALID_ARG;
    // the request's own input and output must not overlap (requests that
    // overlap each other are rejected with their whole batch)
    const uintptr_t i0 = (uintptr_t)I, o0 = (uintptr_t)out;
    const size_t px = (size_t)H * W, ib = px * (plan->in_dtype == BF_IN_U8 ? 1 : 4);
    if (i0 < o0 + px * 4 && o0 < i0 + ib) return BF_ERR_INVALID_ARG;
  }
  Request r;
  r.tag = tag;
  r.plan = plan;
  r.I = I;
  r.out = out;
  r.H = H;
  r.W = W;
  r.ws = align_up(ws);
  s->queue.push_back(r);
  s->st.submitted += 1;
  schedule(s, now);
  return BF_OK;
}

bf_status_t bf_server_poll(bf_server_t s, double now, bf_completion_t *done, int capacity, int *n_done) {
  if (!s || !n_done || capacity < 0 || (capacity > 0 && !done)) return BF_ERR_INVALID_ARG;
  retire(s, now);
  schedule(s, now);
  int n = 0;
  while (n < capacity && !s->done.empty()) {
    done[n++] = s->done.front();
    s->done.pop_front();
  }
  *n_done = n;
  return BF_OK;
}

bf_status_t bf_server_pending(bf_server_t s, int *queued, int *in_flight) {
  if (!s) return BF_ERR_INVALID_ARG;
  if (queued) *queued = (int)s->queue.size();
  if (in_flight) *in_flight = s->inflight_requests;
  return BF_OK;
}

bf_status_t bf_server_stats(bf_server_t s, bf_server_stats_t *stats) {
  if (!s || !stats) return BF_ERR_INVALID_ARG;
  *stats = s->st;
  return BF_OK;
}

}  // extern "C"
