// Host-only parts of the C ABI: status strings and the profiling hook.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "ff.h"

namespace ff {

namespace {
std::mutex g_prof_mu;
std::atomic<int> g_prof_class{0};   // read without the lock on every launch
int g_prof_max = 0;
std::vector<hipEvent_t> g_prof_start, g_prof_stop;
int g_prof_open = 0;       // launches started
int g_prof_done = 0;       // launches closed
bool g_prof_err = false;   // an event record failed: ff_profile_end reports it

void destroy_events() {
  for (auto e : g_prof_start)
    if (e) (void)hipEventDestroy(e);
  for (auto e : g_prof_stop)
    if (e) (void)hipEventDestroy(e);
  g_prof_start.clear();
  g_prof_stop.clear();
}
}  // namespace

void prof_mark(int kernel_class, hipStream_t stream, bool start) {
  if (kernel_class != g_prof_class.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (kernel_class != g_prof_class.load(std::memory_order_relaxed)) return;
  if (start) {
    if (g_prof_open >= g_prof_max) return;
    if (hipEventRecord(g_prof_start[g_prof_open++], stream) != hipSuccess) g_prof_err = true;
  } else {
    if (g_prof_done >= g_prof_open) return;
    if (hipEventRecord(g_prof_stop[g_prof_done++], stream) != hipSuccess) g_prof_err = true;
  }
}

}  // namespace ff

extern "C" {

ff_status ff_profile_begin(int32_t kernel_class, int32_t max_launches) {
  using namespace ff;
  if (kernel_class < 1 || kernel_class > 20 || max_launches < 1 || max_launches > 1 << 20) return FF_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_class = 0;
  destroy_events();
  g_prof_start.assign(max_launches, nullptr);
  g_prof_stop.assign(max_launches, nullptr);
  for (int i = 0; i < max_launches; ++i)
    if (hipEventCreate(&g_prof_start[i]) != hipSuccess || hipEventCreate(&g_prof_stop[i]) != hipSuccess) {
      destroy_events();
      return FF_ERR_HIP;
    }
  g_prof_max = max_launches;
  g_prof_open = g_prof_done = 0;
  g_prof_err = false;
  g_prof_class = kernel_class;
  return FF_OK;
}

ff_status ff_profile_end_each(double* total_ms, int32_t* launches, double* each_ms, int32_t max_each) {
  using namespace ff;
  if (!total_ms || !launches || max_each < 0 || (max_each > 0 && !each_ms)) return FF_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_class = 0;
  double t = 0.0;
  const int n = g_prof_done;
  ff_status st = g_prof_err ? FF_ERR_HIP : FF_OK;
  for (int i = 0; i < n && st == FF_OK; ++i) {
    float ms = 0.f;
    if (hipEventSynchronize(g_prof_stop[i]) != hipSuccess ||
        hipEventElapsedTime(&ms, g_prof_start[i], g_prof_stop[i]) != hipSuccess)
      st = FF_ERR_HIP;
    t += ms;
    if (i < max_each) each_ms[i] = ms;
  }
  destroy_events();
  g_prof_open = g_prof_done = 0;
  g_prof_err = false;
  *total_ms = t;
  *launches = n;
  return st;
}

ff_status ff_profile_end(double* total_ms, int32_t* launches) {
  return ff_profile_end_each(total_ms, launches, nullptr, 0);
}

const char* ff_status_string(ff_status s) {
  switch (s) {
    case FF_OK: return "ok";
    case FF_ERR_ARG: return "invalid argument";
    case FF_ERR_SIZE: return "image too large";
    case FF_ERR_WORKSPACE: return "workspace or descriptor buffer too small";
    case FF_ERR_UNSUPPORTED: return "unsupported";
    case FF_ERR_HIP: return "HIP runtime error";
    case FF_ERR_DEVICE: return "device watchdog fired";
  }
  return "unknown status";
}

}  // extern "C"
