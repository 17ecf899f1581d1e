// C ABI of librpt: argument validation, workspace carving and launch order.
// Every entry point enqueues on the caller's stream and never synchronises.
#include "rpt_internal.h"

namespace rpt {

static thread_local int g_last_hip_error = 0;
void set_hip_error(hipError_t e) { g_last_hip_error = static_cast<int>(e); }

namespace {

bool ws_ok(const void* ws, size_t have, size_t need) {
  if (need == 0) return true;
  return ws != nullptr && (reinterpret_cast<uintptr_t>(ws) & 255u) == 0 && have >= need;
}

bool design_ok(int64_t v, int32_t n, int64_t ldx, int32_t n1) {
  return v >= 1 && n >= 4 && n <= 128 && ldx >= n && n1 >= 2 && n1 <= n - 2;
}

int naive_flags(int prec, bool unbal) {
  if (prec == RPT_SPLIT_BF16) return kPrepSplit;
  return kPrepF32 | (unbal ? kPrepUnbal : 0);
}

}  // namespace
}  // namespace rpt

using namespace rpt;

extern "C" {

const char* rpt_status_string(int status) {
  switch (status) {
    case RPT_OK: return "ok";
    case RPT_ERR_INVALID_ARG: return "invalid argument";
    case RPT_ERR_UNDERDETERMINED: return "sampled set smaller than the rank";
    case RPT_ERR_NOT_SPD: return "sampled Gram matrix not positive definite";
    case RPT_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case RPT_ERR_HIP: return "HIP launch failed";
    case RPT_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

int rpt_last_hip_error(void) { return g_last_hip_error; }

int rpt_version(void) { return 100; }

size_t rpt_naive_workspace(int64_t v, int32_t n, int64_t L, int prec) {
  if (v < 1 || n < 4 || L < 0) return 0;
  Carver c(nullptr);
  prep_carve(c, v, n, n / 2, naive_flags(prec, false) | (prec == RPT_FP32 ? kPrepUnbal : 0));
  return c.off + naive_bytes(v, n, L, prec);
}

rpt_status rpt_naive_maxnull(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* labels,
                             int64_t L, int tail, int prec, float* max_out, float* T_out, void* ws, size_t ws_bytes,
                             void* stream) {
  if (!design_ok(v, n, ldx, n1) || L < 0) return RPT_ERR_INVALID_ARG;
  if (tail != RPT_TAIL_SIGNED && tail != RPT_TAIL_ABS) return RPT_ERR_INVALID_ARG;
  if (prec != RPT_FP32 && prec != RPT_SPLIT_BF16) return RPT_ERR_INVALID_ARG;
  if (L > 0 && (!X || !labels || (!max_out && !T_out))) return RPT_ERR_INVALID_ARG;
  const bool unbal = 2 * n1 != n;
  if (unbal && prec != RPT_FP32) return RPT_ERR_UNSUPPORTED;
  if (!ws_ok(ws, ws_bytes, rpt_naive_workspace(v, n, L, prec))) return RPT_ERR_WORKSPACE;
  if (L == 0) return RPT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int flags = naive_flags(prec, unbal);
  Carver c(ws);
  PrepX p = prep_carve(c, v, n, n1, flags);
  const NaivePlan pl = naive_plan(v, L, n, prec, T_out != nullptr);
  float* partial = c.take<float>(static_cast<size_t>(pl.nc) * L);
  RPT_TRY(prep_launch(p, X, ldx, tail, flags, s));
  return naive_launch(p, pl, labels, L, tail, prec, partial, T_out, max_out, s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// entry points whose kernels are added in later files; kept as explicit
// UNSUPPORTED stubs until then so that the exported symbol set matches rpt.h
extern "C" {
__attribute__((weak)) size_t rpt_sampled_tstat_workspace(int64_t, int32_t) { return 0; }
__attribute__((weak)) rpt_status rpt_sampled_tstat(const float*, int64_t, int32_t, int64_t, int32_t, const uint8_t*,
                                                   int64_t, const int32_t*, int32_t, float*, void*, size_t, void*) {
  return RPT_ERR_UNSUPPORTED;
}
__attribute__((weak)) size_t rpt_complete_workspace(int64_t, int32_t) { return 0; }
__attribute__((weak)) rpt_status rpt_complete(const float*, int64_t, int32_t, const int32_t*, int32_t, const float*,
                                              int64_t, float*, float*, int32_t*, void*, size_t, void*) {
  return RPT_ERR_UNSUPPORTED;
}
__attribute__((weak)) size_t rpt_train_workspace(int64_t, int32_t, int32_t, int32_t, int32_t, int) { return 0; }
__attribute__((weak)) rpt_status rpt_train_subspace(const float*, int64_t, int32_t, int64_t, int32_t, const uint8_t*,
                                                    int32_t, const float*, int32_t, const int32_t*, int32_t, int32_t,
                                                    int32_t, float, const int32_t*, uint64_t, int, int, float*,
                                                    float*, float*, float*, int32_t*, void*, size_t, void*) {
  return RPT_ERR_UNSUPPORTED;
}
__attribute__((weak)) size_t rpt_recover_workspace(int64_t, int32_t, int64_t, int32_t, int32_t) { return 0; }
__attribute__((weak)) rpt_status rpt_recover_maxnull(const float*, int64_t, int32_t, int64_t, int32_t, const uint8_t*,
                                                     int64_t, int64_t, const float*, int32_t, const float*,
                                                     const int32_t*, int32_t, uint64_t, float*, float*, int32_t*,
                                                     void*, size_t, void*) {
  return RPT_ERR_UNSUPPORTED;
}
__attribute__((weak)) size_t rpt_reorth_workspace(int64_t, int32_t) { return 0; }
__attribute__((weak)) rpt_status rpt_reorth(float*, int64_t, int32_t, int32_t*, void*, size_t, void*) {
  return RPT_ERR_UNSUPPORTED;
}
__attribute__((weak)) rpt_status rpt_masked_loss_fwd(const float*, int64_t, int32_t, const float*, int32_t,
                                                     const int64_t*, const int32_t*, const float*, int64_t, double*,
                                                     float*, void*) {
  return RPT_ERR_UNSUPPORTED;
}
__attribute__((weak)) rpt_status rpt_masked_loss_bwd(const float*, int64_t, int32_t, const float*, int32_t,
                                                     const int64_t*, const int32_t*, const float*, int64_t, float*,
                                                     float*, void*) {
  return RPT_ERR_UNSUPPORTED;
}
}  // extern "C"
