// K2 -- the test() step of RapidPT recovery (Alg. 2) on the sampled voxels:
// y[i, q] = t statistic of voxel omega[i, q] under relabelling i (sampled
// sets of k voxels per relabelling, or uneven sets in CSR form).
//
// One workgroup per relabelling: the group-1 indicator goes to LDS, each thread
// takes sampled rows, reads the standardised row (prep.hip, 16-byte aligned)
// with 16-byte loads and forms the group-1 sum (and sum of squares for
// unbalanced designs) in FP32.  The balanced statistic uses the same scaled
// contrast u as NaivePT; unbalanced designs evaluate Eq. 2 directly.
#include "rpt_internal.h"

namespace rpt {

namespace {

struct SampledArgs {
  int64_t v;
  const float* rows;
  int ldn;
  const float2* cst;
  const float2* cstg;
  const uint8_t* labels;
  int n, n1;
  const int32_t* omega;
  int k;
  const int64_t* optr;  // CSR offsets of uneven sampled sets (nullptr: k per row)
  float* y;
  float fs, tm;
};

__global__ __launch_bounds__(kBlock) void sampled_kernel(SampledArgs a) {
  __shared__ float lab[kBlock];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  for (int j = tid; j < a.ldn; j += kBlock) lab[j] = (j < a.n && a.labels[i * a.n + j]) ? 1.0f : 0.0f;
  __syncthreads();
  const bool unbal = 2 * a.n1 != a.n;
  const int n1 = a.n1, n2 = a.n - a.n1;
  const int64_t base = a.optr ? a.optr[i] : i * a.k;
  const int ki = a.optr ? static_cast<int>(a.optr[i + 1] - base) : a.k;
  for (int q = tid; q < ki; q += kBlock) {
    const int64_t vox = a.omega[base + q];
    if (vox < 0 || vox >= a.v) {  // out-of-range index: no statistic
      a.y[base + q] = NAN;
      continue;
    }
    const f32x4* row = reinterpret_cast<const f32x4*>(a.rows + vox * a.ldn);
    float s1 = 0.0f, q1 = 0.0f;
    for (int j4 = 0; j4 < a.ldn / 4; ++j4) {
      const f32x4 x = row[j4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float l = lab[4 * j4 + e];
        s1 = fmaf(x[e], l, s1);
        if (unbal) q1 = fmaf(x[e] * x[e], l, q1);
      }
    }
    float t;
    if (!unbal) {
      const float2 c2 = a.cst[vox];
      t = t_from_u_f(fmaf(s1, c2.x, c2.y), a.fs, a.tm);
    } else {
      const float2 sq = a.cstg[vox];
      const float S2 = sq.x - s1, Q2 = sq.y - q1;
      const float m1 = s1 / n1, m2 = S2 / n2;
      const float v1 = fmaxf((q1 - s1 * m1) / (n1 - 1), 0.0f), v2 = fmaxf((Q2 - S2 * m2) / (n2 - 1), 0.0f);
      const float den2 = v1 / n1 + v2 / n2;
      t = den2 > 0.0f ? (m1 - m2) * rsqrtf(den2) : 0.0f;
    }
    a.y[base + q] = t;
  }
}

}  // namespace

rpt_status sampled_launch(const PrepX& p, const uint8_t* labels, int64_t L, const int32_t* omega, int k,
                          const float* Tsrc, float* y, hipStream_t s, const int64_t* optr) {
  (void)Tsrc;
  if (L == 0 || (k == 0 && !optr)) return RPT_OK;
  if (p.ldn > kBlock) return RPT_ERR_UNSUPPORTED;
  SampledArgs a;
  a.v = p.v;
  a.rows = p.rows;
  a.ldn = p.ldn;
  a.cst = p.cst;
  a.cstg = p.cstg;
  a.labels = labels;
  a.n = p.n;
  a.n1 = p.n1;
  a.omega = omega;
  a.k = k;
  a.optr = optr;
  a.y = y;
  const int m = p.n / 2;
  a.fs = static_cast<float>(2.0 * sqrt((m - 1.0) / m));
  a.tm = static_cast<float>(2.0 / m);
  RPT_STAGE("sampled_t", s);
  hipLaunchKernelGGL(sampled_kernel, dim3(static_cast<unsigned>(L)), dim3(kBlock), 0, s, a);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace rpt
