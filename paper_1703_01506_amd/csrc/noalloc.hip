// rpt_reorth_noalloc: the orthonormalisation of rpt_reorth for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).  Its workspace is a file-scope
// device array of fixed size instead of a caller-provided buffer; the kernels
// are rpt_reorth's own.
#include "rpt_internal.h"

namespace rpt {
namespace {

// The largest workspace one Cholesky-QR pass needs (reorth_bytes): the Gram
// partials of at most 768 workgroups whatever v is (36 lower 16 x 16 tiles
// of rank 128 each), the FP64 Gram matrix and the BF16 hi/lo factor of rank
// 128.
constexpr size_t kScratchBytes = static_cast<size_t>(768) * 36 * 256 * sizeof(float) +
                                 static_cast<size_t>(128) * 128 * sizeof(double) +
                                 2 * static_cast<size_t>(128) * 128 * sizeof(uint16_t);

// One copy per GPU the library runs on, held until the process ends.  In host
// code this name is only a handle: its device address comes from
// hipGetSymbolAddress (kept per device below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the device of `stream`, looked up once
// per device with that device current.
rpt_status scratch_address(hipStream_t stream, void** out) {
  int dev = 0;
  hipError_t e = hipStreamGetDevice(stream, &dev);
  if (e != hipSuccess) {
    set_hip_error(e);
    return RPT_ERR_HIP;
  }
  if (dev < 0 || dev >= kMaxDevices) return RPT_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    int cur = 0;
    e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) {
      set_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol);
      return RPT_ERR_HIP;
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return RPT_OK;
}

}  // namespace
}  // namespace rpt

using namespace rpt;

extern "C" {

size_t rpt_reorth_noalloc_capacity(void) { return kScratchBytes; }

rpt_status rpt_reorth_noalloc(float* U, int64_t v, int32_t r, int32_t* info, void* stream) {
  if (!U || v < 1 || r < 1 || r > 128 || v < r) return RPT_ERR_INVALID_ARG;
  if (reorth_bytes(v, r) > kScratchBytes) return RPT_ERR_UNSUPPORTED;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* ws = nullptr;
  RPT_TRY(scratch_address(s, &ws));
  RPT_TRY(reorth_launch(U, v, r, info, ws, s));
  return reorth_launch(U, v, r, info, ws, s);
}

}  // extern "C"
