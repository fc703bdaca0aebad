// Error reporting, version, option defaults and stats read-back of libfg.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>

#include "fg_common.h"

static thread_local char g_err[512] = "no error";

fg_status fg_set_error(fg_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

extern "C" const char* fg_last_error(void) { return g_err; }

extern "C" const char* fg_version(void) { return "0.1.0"; }

fg_device_props fg_props(int device) {
  static std::mutex mu;
  static fg_device_props cache[64];
  static bool have[64] = {false};
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0 || device >= 64) return fg_device_props{0, 0, 0};
  if (!have[device]) {
    fg_device_props p{0, 0, 0};
    hipDeviceGetAttribute(&p.cus, hipDeviceAttributeMultiprocessorCount, device);
    hipDeviceGetAttribute(&p.coop, hipDeviceAttributeCooperativeLaunch, device);
    hipDeviceGetAttribute(&p.clock_khz, hipDeviceAttributeWallClockRate, device);
    cache[device] = p;
    have[device] = true;
  }
  return cache[device];
}

extern "C" void fg_bfs_opts_default(fg_bfs_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->mode = FG_MODE_DO;
  o->do_a_num = 1;
  o->do_a_den = 100;
  o->do_b_num = 1;
  o->do_b_den = 10;
}

extern "C" fg_status fg_stats_read(const fg_run_stats* dev_stats, fg_run_stats* host,
                                   void* stream) {
  if (!dev_stats || !host) return fg_set_error(FG_EINVAL, "fg_stats_read: NULL pointer");
  hipStream_t s = (hipStream_t)stream;
  FG_HIP_TRY(hipMemcpyAsync(host, dev_stats, sizeof(fg_run_stats), hipMemcpyDeviceToHost, s));
  FG_HIP_TRY(hipStreamSynchronize(s));
  return FG_OK;
}
