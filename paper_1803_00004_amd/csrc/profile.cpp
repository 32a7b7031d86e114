// Optional per-kernel HIP-event timing (bf_profile_enable / bf_profile_read).
#include <hip/hip_runtime_api.h>

#include <vector>

#include "bf.h"
#include "bf_internal.h"

namespace {

struct Mark {
  hipEvent_t begin, end;
  int kernel;
};

bool g_on = false;
std::vector<Mark> g_marks;       // recorded pairs, read by bf_profile_read
std::vector<hipEvent_t> g_pool;  // free events
hipEvent_t g_open[2] = {nullptr, nullptr};

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

namespace bf {

void profile_mark(int kernel, int begin, void *stream) {
  if (!g_on) return;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (begin) {
    g_open[kernel] = take();
    if (g_open[kernel]) (void)hipEventRecord(g_open[kernel], s);
  } else if (g_open[kernel]) {
    hipEvent_t e = take();
    if (e) {
      (void)hipEventRecord(e, s);
      g_marks.push_back({g_open[kernel], e, kernel});
    }
    g_open[kernel] = nullptr;
  }
}

}  // namespace bf

extern "C" {

bf_status_t bf_profile_enable(int on) {
  g_on = on != 0;
  return BF_OK;
}

bf_status_t bf_profile_read(double ms[2], int launches[2]) {
  if (!ms || !launches) return BF_ERR_INVALID_ARG;
  ms[0] = ms[1] = 0.0;
  launches[0] = launches[1] = 0;
  bf_status_t st = BF_OK;
  for (const Mark &m : g_marks) {
    float t = 0.f;
    if (hipEventSynchronize(m.end) != hipSuccess || hipEventElapsedTime(&t, m.begin, m.end) != hipSuccess)
      st = BF_ERR_DEVICE;
    ms[m.kernel] += t;
    launches[m.kernel] += 1;
    g_pool.push_back(m.begin);
    g_pool.push_back(m.end);
  }
  g_marks.clear();
  return st;
}

}  // extern "C"
