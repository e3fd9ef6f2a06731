// Host-only parts of the C ABI: status strings and the profiling hook.
#include <hip/hip_runtime_api.h>

#include <mutex>
#include <vector>

#include "ff.h"

namespace ff {

namespace {
std::mutex g_prof_mu;
int g_prof_class = 0;
int g_prof_max = 0;
std::vector<hipEvent_t> g_prof_start, g_prof_stop;
int g_prof_open = 0;   // launches started
int g_prof_done = 0;   // launches closed
}  // namespace

void prof_mark(int kernel_class, hipStream_t stream, bool start) {
  if (g_prof_class == 0 || kernel_class != g_prof_class) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (kernel_class != g_prof_class) return;
  if (start) {
    if (g_prof_open >= g_prof_max) return;
    hipEventRecord(g_prof_start[g_prof_open++], stream);
  } else {
    if (g_prof_done >= g_prof_open) return;
    hipEventRecord(g_prof_stop[g_prof_done++], stream);
  }
}

}  // namespace ff

extern "C" {

ff_status ff_profile_begin(int32_t kernel_class, int32_t max_launches) {
  using namespace ff;
  if (kernel_class < 1 || kernel_class > 9 || max_launches < 1 || max_launches > 1 << 20) return FF_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto e : g_prof_start) hipEventDestroy(e);
  for (auto e : g_prof_stop) hipEventDestroy(e);
  g_prof_start.assign(max_launches, nullptr);
  g_prof_stop.assign(max_launches, nullptr);
  for (int i = 0; i < max_launches; ++i)
    if (hipEventCreate(&g_prof_start[i]) != hipSuccess || hipEventCreate(&g_prof_stop[i]) != hipSuccess)
      return FF_ERR_HIP;
  g_prof_max = max_launches;
  g_prof_open = g_prof_done = 0;
  g_prof_class = kernel_class;
  return FF_OK;
}

ff_status ff_profile_end(double* total_ms, int32_t* launches) {
  using namespace ff;
  if (!total_ms || !launches) return FF_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double t = 0.0;
  const int n = g_prof_done;
  for (int i = 0; i < n; ++i) {
    if (hipEventSynchronize(g_prof_stop[i]) != hipSuccess) return FF_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_prof_start[i], g_prof_stop[i]) != hipSuccess) return FF_ERR_HIP;
    t += ms;
  }
  for (auto e : g_prof_start) hipEventDestroy(e);
  for (auto e : g_prof_stop) hipEventDestroy(e);
  g_prof_start.clear();
  g_prof_stop.clear();
  g_prof_class = 0;
  g_prof_open = g_prof_done = 0;
  *total_ms = t;
  *launches = n;
  return FF_OK;
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
