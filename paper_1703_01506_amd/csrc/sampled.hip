// K2 -- the test() step of RapidPT recovery (Alg. 2) on the sampled voxels:
// y[i, q] = t statistic of voxel omega[i, q] under relabelling i (sampled
// sets of k voxels per relabelling, or uneven sets in CSR form).
//
// One workgroup per relabelling: the group-1 indicator goes to LDS; 32 lanes
// share one sampled row (prep.hip's standardised row, 16-byte aligned), each
// reading 16 consecutive bytes of every 512-byte piece of it, so a row costs
// its own cache lines once; four rows per lane group are in flight at a time.  The group-1 sum
// (and sum of squares for unbalanced designs) is reduced across the 32 lanes
// in FP32.  The balanced statistic uses the same scaled contrast u as
// NaivePT; unbalanced designs evaluate Eq. 2 directly.
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

constexpr int kRowLanes = 32;  // lanes sharing one sampled row
constexpr int kRowsInFlight = 4;
constexpr int kLabMax = 4 * kRowLanes * 4;  // rows of up to 512 subjects (four 16-byte pieces per lane)

__device__ __forceinline__ float t_of(const SampledArgs& a, int64_t vox, float s1, float q1) {
  if (2 * a.n1 == a.n) {
    const float2 c2 = a.cst[vox];
    return t_from_u_f(fmaf(s1, c2.x, c2.y), a.fs, a.tm);
  }
  const int n1 = a.n1, n2 = a.n - a.n1;
  const float2 sq = a.cstg[vox];
  const float S2 = sq.x - s1, Q2 = sq.y - q1;
  const float m1 = s1 / n1, m2 = S2 / n2;
  const float v1 = fmaxf((q1 - s1 * m1) / (n1 - 1), 0.0f), v2 = fmaxf((Q2 - S2 * m2) / (n2 - 1), 0.0f);
  const float den2 = v1 / n1 + v2 / n2;
  return den2 > 0.0f ? (m1 - m2) * rsqrtf(den2) : 0.0f;
}

// NCH 16-byte pieces per lane: one for rows of up to 128 subjects, four up to 512
template <int NCH>
__global__ __launch_bounds__(kBlock) void sampled_kernel(SampledArgs a) {
  constexpr int kRowChunks = NCH;
  __shared__ __align__(16) float lab[kLabMax];
  const int64_t i = blockIdx.x;
  const int tid = threadIdx.x;
  for (int j = tid; j < a.ldn; j += kBlock) lab[j] = (j < a.n && a.labels[i * a.n + j]) ? 1.0f : 0.0f;
  __syncthreads();
  const bool unbal = 2 * a.n1 != a.n;
  const int64_t base = a.optr ? a.optr[i] : i * a.k;
  const int ki = a.optr ? static_cast<int>(a.optr[i + 1] - base) : a.k;
  const int gl = tid & (kRowLanes - 1);  // lane within the row group
  const int grp = tid / kRowLanes;       // row group of the workgroup
  constexpr int kGroups = kBlock / kRowLanes;
  f32x4 l4[kRowChunks];
  bool on[kRowChunks];
#pragma unroll
  for (int cc = 0; cc < kRowChunks; ++cc) {
    on[cc] = 4 * (gl + kRowLanes * cc) < a.ldn;
    l4[cc] = on[cc] ? *reinterpret_cast<const f32x4*>(lab + 4 * (gl + kRowLanes * cc)) : f32x4{0.f, 0.f, 0.f, 0.f};
  }
  for (int q0 = 0; q0 < ki; q0 += kGroups * kRowsInFlight) {
    int64_t vox[kRowsInFlight];
    f32x4 x[kRowsInFlight][kRowChunks];
#pragma unroll
    for (int e = 0; e < kRowsInFlight; ++e) {
      const int q = q0 + e * kGroups + grp;
      vox[e] = q < ki ? a.omega[base + q] : -1;
      const bool ok = vox[e] >= 0 && vox[e] < a.v;
#pragma unroll
      for (int cc = 0; cc < kRowChunks; ++cc)
        x[e][cc] = (ok && on[cc])
                       ? *reinterpret_cast<const f32x4*>(a.rows + vox[e] * a.ldn + 4 * (gl + kRowLanes * cc))
                       : f32x4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int e = 0; e < kRowsInFlight; ++e) {
      float s1 = 0.0f, q1 = 0.0f;
#pragma unroll
      for (int cc = 0; cc < kRowChunks; ++cc)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          s1 = fmaf(x[e][cc][c], l4[cc][c], s1);
          if (unbal) q1 = fmaf(x[e][cc][c] * x[e][cc][c], l4[cc][c], q1);
        }
#pragma unroll
      for (int off = kRowLanes / 2; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off, kRowLanes);
        if (unbal) q1 += __shfl_xor(q1, off, kRowLanes);
      }
      const int q = q0 + e * kGroups + grp;
      if (gl == 0 && q < ki)
        a.y[base + q] = (vox[e] < 0 || vox[e] >= a.v) ? 0.0f : t_of(a, vox[e], s1, q1);  // out of range: 0
    }
  }
}

}  // namespace

rpt_status sampled_launch(const PrepX& p, const uint8_t* labels, int64_t L, const int32_t* omega, int k,
                          const float* Tsrc, float* y, hipStream_t s, const int64_t* optr) {
  (void)Tsrc;
  if (L == 0 || (k == 0 && !optr)) return RPT_OK;
  if (p.ldn > kLabMax) return RPT_ERR_UNSUPPORTED;
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
  stat_consts(p, &a.fs, &a.tm);
  RPT_STAGE("sampled_t", s);
  if (p.ldn <= 4 * kRowLanes)
    hipLaunchKernelGGL(sampled_kernel<1>, dim3(static_cast<unsigned>(L)), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(sampled_kernel<4>, dim3(static_cast<unsigned>(L)), dim3(kBlock), 0, s, a);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace rpt
