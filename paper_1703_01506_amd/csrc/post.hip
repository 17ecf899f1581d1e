// Inference on the observed labelling from a max-null distribution (Sec. 2,
// Sec. 5.5, Eq. 4):
//   observed t map   t_k for the labelling with group 1 = subjects 0..n1-1
//   FWER threshold   the ascending order statistic m_(L - floor(alpha L))
//   corrected p      p_k = #{i : m_i >= t_k} / L
//   rejection counts v1, v2 (voxels with p <= alpha under two max nulls) and
//                    vc (both), the inputs of the resampling risk of Eq. 4.
// Counting is exact (FP32 comparisons of FP32 values); the max null is staged
// through LDS in tiles so every thread compares against it at LDS speed.
#include "rpt_internal.h"

namespace rpt {

namespace {

constexpr int kTile = 4096;  // maxima per LDS tile

struct ObservedArgs {
  int64_t v;
  const float* rows;
  int ldn;
  const float2* cst;
  const float2* cstg;
  int n, n1;
  float fs, tm;
  float* t;
};

// One thread per voxel, same contrast and statistic as the sampled kernel.
__global__ __launch_bounds__(kBlock) void observed_kernel(ObservedArgs a) {
  const int64_t vox = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (vox >= a.v) return;
  const float* row = a.rows + vox * a.ldn;
  float s1 = 0.0f, q1 = 0.0f;
  const bool unbal = 2 * a.n1 != a.n;
  for (int j = 0; j < a.n1; ++j) {
    s1 += row[j];
    if (unbal) q1 = fmaf(row[j], row[j], q1);
  }
  float t;
  if (!unbal) {
    const float2 c2 = a.cst[vox];
    t = t_from_u_f(fmaf(s1, c2.x, c2.y), a.fs, a.tm);
  } else {
    const int n1 = a.n1, n2 = a.n - a.n1;
    const float2 sq = a.cstg[vox];
    const float S2 = sq.x - s1, Q2 = sq.y - q1;
    const float m1 = s1 / n1, m2 = S2 / n2;
    const float v1 = fmaxf((q1 - s1 * m1) / (n1 - 1), 0.0f), v2 = fmaxf((Q2 - S2 * m2) / (n2 - 1), 0.0f);
    const float den2 = v1 / n1 + v2 / n2;
    t = den2 > 0.0f ? (m1 - m2) * rsqrtf(den2) : 0.0f;
  }
  a.t[vox] = t;
}

// #{i : m_i >= x} for every thread's x, with the maxima staged in LDS
__device__ __forceinline__ int64_t count_ge(const float* h, int64_t L, float x, bool active, float* tile) {
  int64_t c = 0;
  for (int64_t b0 = 0; b0 < L; b0 += kTile) {
    const int nb = static_cast<int>(L - b0 < kTile ? L - b0 : kTile);
    __syncthreads();
    for (int q = threadIdx.x; q < nb; q += kBlock) tile[q] = h[b0 + q];
    __syncthreads();
    if (active) {
      int cc = 0;
      for (int q = 0; q < nb; ++q) cc += tile[q] >= x ? 1 : 0;
      c += cc;
    }
  }
  return c;
}

__global__ __launch_bounds__(kBlock) void pvalue_kernel(const float* __restrict__ h, int64_t L,
                                                       const float* __restrict__ t, int64_t v, float* p) {
  __shared__ float tile[kTile];
  const int64_t vox = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const bool active = vox < v;
  const float x = active ? t[vox] : 0.0f;
  const int64_t c = count_ge(h, L, x, active, tile);
  if (active) p[vox] = static_cast<float>(static_cast<double>(c) / static_cast<double>(L));
}

// candidate i is the answer when #{m < m_i} <= R < #{m <= m_i}
__global__ __launch_bounds__(kBlock) void select_kernel(const float* __restrict__ h, int64_t L, int64_t R,
                                                       float* out) {
  __shared__ float tile[kTile];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const bool active = i < L;
  const float x = active ? h[i] : 0.0f;
  int64_t lt = 0, le = 0;
  for (int64_t b0 = 0; b0 < L; b0 += kTile) {
    const int nb = static_cast<int>(L - b0 < kTile ? L - b0 : kTile);
    __syncthreads();
    for (int q = threadIdx.x; q < nb; q += kBlock) tile[q] = h[b0 + q];
    __syncthreads();
    if (active) {
      int a = 0, b = 0;
      for (int q = 0; q < nb; ++q) {
        a += tile[q] < x ? 1 : 0;
        b += tile[q] <= x ? 1 : 0;
      }
      lt += a;
      le += b;
    }
  }
  if (active && lt <= R && R < le) *out = x;  // ties write the same value
}

__global__ __launch_bounds__(kBlock) void reject_kernel(const float* __restrict__ h1, int64_t L1,
                                                       const float* __restrict__ h2, int64_t L2,
                                                       const float* __restrict__ t, int64_t v, double alpha,
                                                       unsigned long long* counts) {
  __shared__ float tile[kTile];
  __shared__ unsigned long long red[3];
  const int64_t vox = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const bool active = vox < v;
  const float x = active ? t[vox] : 0.0f;
  if (threadIdx.x < 3) red[threadIdx.x] = 0;
  const int64_t c1 = count_ge(h1, L1, x, active, tile);
  const int64_t c2 = count_ge(h2, L2, x, active, tile);
  const bool r1 = active && static_cast<double>(c1) / static_cast<double>(L1) <= alpha;
  const bool r2 = active && static_cast<double>(c2) / static_cast<double>(L2) <= alpha;
  // per-wave ballots, one atomic per wave and count
  const unsigned long long b1 = __ballot(r1), b2 = __ballot(r2), b12 = __ballot(r1 && r2);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&red[0], static_cast<unsigned long long>(__popcll(b1)));
    atomicAdd(&red[1], static_cast<unsigned long long>(__popcll(b2)));
    atomicAdd(&red[2], static_cast<unsigned long long>(__popcll(b12)));
  }
  __syncthreads();
  if (threadIdx.x < 3 && red[threadIdx.x]) atomicAdd(&counts[threadIdx.x], red[threadIdx.x]);
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0;
}

}  // namespace

}  // namespace rpt

extern "C" {

size_t rpt_observed_tstat_workspace(int64_t v, int32_t n) {
  if (v < 1 || n < 4) return 0;
  rpt::Carver c(nullptr);
  rpt::prep_carve(c, v, n, n / 2, rpt::kPrepRows | rpt::kPrepUnbal);
  return c.off;
}

rpt_status rpt_observed_tstat(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, float* t_out, void* ws,
                              size_t ws_bytes, void* stream) {
  using namespace rpt;
  if (v < 1 || n < 4 || n > 512 || ldx < n || n1 < 2 || n1 > n - 2 || !X || !t_out) return RPT_ERR_INVALID_ARG;
  const size_t need = rpt_observed_tstat_workspace(v, n);
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255)) return RPT_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Carver c(ws);
  const int flags = kPrepRows | kPrepUnbal;
  PrepX p = prep_carve(c, v, n, n1, flags);
  RPT_TRY(prep_launch(p, X, ldx, RPT_TAIL_SIGNED, flags, s));
  ObservedArgs a;
  a.v = v;
  a.rows = p.rows;
  a.ldn = p.ldn;
  a.cst = p.cst;
  a.cstg = p.cstg;
  a.n = n;
  a.n1 = n1;
  stat_consts(p, &a.fs, &a.tm);
  a.t = t_out;
  RPT_STAGE("observed_t", s);
  hipLaunchKernelGGL(observed_kernel, dim3(static_cast<unsigned>(ceil_div(v, kBlock))), dim3(kBlock), 0, s, a);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status rpt_fwer_threshold(const float* maxima, int64_t L, double alpha, float* thr_out, void* stream) {
  using namespace rpt;
  if (L < 1 || !(alpha >= 0.0 && alpha < 1.0) || !maxima || !thr_out) return RPT_ERR_INVALID_ARG;
  const int64_t R = L - static_cast<int64_t>(floor(alpha * static_cast<double>(L))) - 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(select_kernel, dim3(static_cast<unsigned>(ceil_div(L, kBlock))), dim3(kBlock), 0, s, maxima,
                     L, R, thr_out);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status rpt_corrected_pvalues(const float* maxima, int64_t L, const float* t, int64_t v, float* p_out,
                                 void* stream) {
  using namespace rpt;
  if (L < 1 || v < 0 || !maxima || (v > 0 && (!t || !p_out))) return RPT_ERR_INVALID_ARG;
  if (v == 0) return RPT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(pvalue_kernel, dim3(static_cast<unsigned>(ceil_div(v, kBlock))), dim3(kBlock), 0, s, maxima, L,
                     t, v, p_out);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status rpt_rejection_counts(const float* maxima1, int64_t L1, const float* maxima2, int64_t L2, const float* t,
                                int64_t v, double alpha, int64_t* counts_out, void* stream) {
  using namespace rpt;
  if (L1 < 1 || L2 < 1 || v < 0 || !maxima1 || !maxima2 || !counts_out || (v > 0 && !t) ||
      !(alpha >= 0.0 && alpha < 1.0))
    return RPT_ERR_INVALID_ARG;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counts_out);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, s, cnt, 3);
  RPT_CHECK_LAUNCH();
  if (v == 0) return RPT_OK;
  hipLaunchKernelGGL(reject_kernel, dim3(static_cast<unsigned>(ceil_div(v, kBlock))), dim3(kBlock), 0, s, maxima1,
                     L1, maxima2, L2, t, v, alpha, cnt);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // extern "C"
