// Issue rates of the VALU instruction classes that the reconstruction's noise
// generator uses, measured on the whole chip: eight independent chains per
// lane, eight waves per SIMD, so that throughput and not latency is timed.
// The result is the SIMD cycles per wave64 instruction at a given clock.  It
// backs the ALU roofline of the generator (a diagnostic, not on any path).
#include "rpt_internal.h"

namespace rpt {
namespace {

constexpr int kProbeBlocksPerCU = 8;  // 8 workgroups of 4 waves: 8 waves per SIMD

template <int MODE>
__global__ __launch_bounds__(kBlock) void issue_rate_kernel(float* out, int iters) {
  float a[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = threadIdx.x * 1e-3f + 1.0f + q;
  for (int i = 0; i < iters; ++i) {
    if (MODE == 0) {  // FP32 add
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] += 1.0001f;
    } else if (MODE == 1) {  // v_log_f32
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = __builtin_amdgcn_logf(a[q]);
    } else if (MODE == 2) {  // v_sin_f32
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = __builtin_amdgcn_sinf(a[q]);
    } else if (MODE == 3) {  // v_bitop3_b32 (three-input XOR, one scalar operand)
      unsigned u[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) u[q] = __float_as_uint(a[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        unsigned r;
        asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(u[q]), "v"(u[(q + 1) & 7]), "s"(0x9E3779B9u));
        u[q] = r;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = __uint_as_float(u[q]);
    } else {  // v_mad_u64_u32 then v_xor_b32 of its halves
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const uint64_t pr = static_cast<uint64_t>(0xD2511F53u) * __float_as_uint(a[q]);
        a[q] = __uint_as_float(static_cast<unsigned>(pr) ^ static_cast<unsigned>(pr >> 32));
      }
    }
  }
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < 8; ++q) s += a[q];
  out[static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x] = s;
}

}  // namespace
}  // namespace rpt

using namespace rpt;

extern "C" {

size_t rpt_issue_rates_workspace(int32_t compute_units) {
  if (compute_units < 1) return 0;
  return static_cast<size_t>(compute_units) * kProbeBlocksPerCU * kBlock * sizeof(float);
}

rpt_status rpt_issue_rates(int32_t compute_units, double clock_ghz, int32_t iters, double* cycles_out, void* ws,
                           size_t ws_bytes, void* stream) {
  if (compute_units < 1 || clock_ghz <= 0.0 || iters < 1 || !cycles_out || !ws ||
      ws_bytes < rpt_issue_rates_workspace(compute_units))
    return RPT_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned blocks = static_cast<unsigned>(compute_units) * kProbeBlocksPerCU;
  const double waves_per_simd = blocks * 4.0 / (compute_units * 4.0);
  void* const fns[5] = {reinterpret_cast<void*>(&issue_rate_kernel<0>), reinterpret_cast<void*>(&issue_rate_kernel<1>),
                        reinterpret_cast<void*>(&issue_rate_kernel<2>), reinterpret_cast<void*>(&issue_rate_kernel<3>),
                        reinterpret_cast<void*>(&issue_rate_kernel<4>)};
  const double instr[5] = {8, 8, 8, 8, 16};  // per loop iteration
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rpt_status st = RPT_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = RPT_ERR_HIP;
  float* out = static_cast<float*>(ws);
  for (int m = 0; m < 5 && st == RPT_OK; ++m) {
    void* args[] = {&out, &iters};
    float ms = 0.0f;
    if (hipLaunchKernel(fns[m], dim3(blocks), dim3(kBlock), args, 0, s) != hipSuccess ||  // warm-up
        hipEventRecord(e0, s) != hipSuccess ||
        hipLaunchKernel(fns[m], dim3(blocks), dim3(kBlock), args, 0, s) != hipSuccess ||
        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = RPT_ERR_HIP;
      break;
    }
    cycles_out[m] = ms * 1e-3 * clock_ghz * 1e9 / (waves_per_simd * iters * instr[m]);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return st;
}

}  // extern "C"
