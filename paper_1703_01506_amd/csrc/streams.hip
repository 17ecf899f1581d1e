// A second stream per device for work that overlaps the caller's stream:
// created on first use (never while the caller's stream is being captured),
// default priority, never destroyed.  Every event is recorded and waited on
// under the device's lock, so concurrent callers cannot swap each other's
// dependencies.
#include "rpt_internal.h"

namespace rpt {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_side_init;
SideStream g_side[kMaxDevices];
}  // namespace

SideStream* side_stream(hipStream_t s) {
  int dev = 0;
  if (hipStreamGetDevice(s, &dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_side_init);
  SideStream& sd = g_side[dev];
  if (sd.ok) return &sd;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return nullptr;
  if (cur != dev && hipSetDevice(dev) != hipSuccess) return nullptr;
  bool good = hipStreamCreateWithFlags(&sd.st, hipStreamNonBlocking) == hipSuccess;
  for (hipEvent_t* ev : {&sd.fork, &sd.mid, &sd.join, &sd.step})
    good = good && hipEventCreateWithFlags(ev, hipEventDisableTiming) == hipSuccess;
  if (cur != dev) (void)hipSetDevice(cur);
  if (!good) {
    (void)hipGetLastError();
    return nullptr;
  }
  sd.ok = true;
  return &sd;
}

rpt_status stream_wait(SideStream* sd, hipEvent_t ev, hipStream_t from, hipStream_t to) {
  std::lock_guard<std::mutex> lk(sd->mu);
  hipError_t e = hipEventRecord(ev, from);
  if (e == hipSuccess) e = hipStreamWaitEvent(to, ev, 0);
  if (e != hipSuccess) {
    set_hip_error(e);
    return RPT_ERR_HIP;
  }
  return RPT_OK;
}

}  // namespace rpt
