// K0 -- per-voxel preparation of X for the matrix-core contractions.
//
// The t statistic of Eq. 2 is unchanged by a per-voxel affine map with a
// positive scale, so every voxel row is first centred and scaled to unit
// variance in FP64.  This keeps FP32/BF16 group sums free of the cancellation
// that raw grey-matter values (mean >> spread) would cause.
//
// For a balanced design (n1 = n2 = m) the statistic of relabelling i at voxel k
// depends on the group-1 sum a = sum_{j in G1} x_kj only through
//     u = (a - S_k / 2) / sqrt(Qc_k),
// with S_k the row sum and Qc_k the centred sum of squares of the stored row:
// the between-group sum of squares is 2 d^2 / m with d = a - S/2, hence
//     t = 2 u sqrt((m-1)/m) / sqrt(1 - 2 u^2 / m),
// a single increasing function of u shared by all voxels.  The contraction
// epilogue therefore needs one FMA per element, u = a * rinv_k + c_k, and the
// column maximum of t is t(max u).  The constants are computed from the values
// the contraction actually multiplies (hi + lo for the split path), in FP64.
//
// Layouts written (vpad = v rounded up to 32; padding voxels are zero and get
// epilogue constants that can never win a maximum):
//   kb16  [ks][vpad][2][16] bf16  hi(x_{16s+e}) then lo(x_{16s+e}), 0 past n
//   kb32  [ks][vpad][2][4] f32 subject 8s+2q+h at [s][k][h][q]
//   rows  [vpad][ldn] f32      standardised rows, for the sampled statistics
//   cst   [vpad] (rinv, -S/2 * rinv)       cstg [vpad] (S, Q)
#include "rpt_internal.h"

namespace rpt {

namespace {

__global__ void prep_kernel(const float* __restrict__ X, int64_t v, int n, int64_t ldx, PrepX p, int tail,
                            int flags) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= p.vpad) return;
  const bool split = (flags & kPrepSplit) != 0;
  if (k >= v) {
    if (p.kb16) {
      for (int s = 0; s < p.ksteps; ++s) {
        u32x4* d = reinterpret_cast<u32x4*>(p.kb16 + (static_cast<size_t>(s) * p.vpad + k) * 32);
        d[0] = u32x4{0, 0, 0, 0};
        d[1] = u32x4{0, 0, 0, 0};
        d[2] = u32x4{0, 0, 0, 0};
        d[3] = u32x4{0, 0, 0, 0};
      }
    }
    if (p.kb32) {
      for (int s = 0; s < p.ksteps; ++s) {
        f32x4* d = reinterpret_cast<f32x4*>(p.kb32 + (static_cast<size_t>(s) * p.vpad + k) * 8);
        d[0] = f32x4{0, 0, 0, 0};
        d[1] = f32x4{0, 0, 0, 0};
        if (p.kb32sq) {
          f32x4* d2 = reinterpret_cast<f32x4*>(p.kb32sq + (static_cast<size_t>(s) * p.vpad + k) * 8);
          d2[0] = f32x4{0, 0, 0, 0};
          d2[1] = f32x4{0, 0, 0, 0};
        }
      }
    }
    if (p.rows)
      for (int j = 0; j < p.ldn; ++j) p.rows[k * p.ldn + j] = 0.0f;
    if (p.cst) p.cst[k] = make_float2(0.0f, tail == RPT_TAIL_ABS ? 0.0f : -INFINITY);
    if (p.cstg) p.cstg[k] = make_float2(0.0f, 0.0f);
    return;
  }
  const float* x = X + k * ldx;
  double s0 = 0.0;
  for (int j = 0; j < n; ++j) s0 += x[j];
  const double mean = s0 / n;
  double ss = 0.0;
  for (int j = 0; j < n; ++j) {
    double d = x[j] - mean;
    ss += d * d;
  }
  const double sc = ss > 0.0 ? sqrt((n - 1.0) / ss) : 0.0;
  auto xs = [&](int j) -> float { return static_cast<float>((x[j] - mean) * sc); };
  auto stored = [&](int j) -> float {
    float f = xs(j);
    if (!split) return f;
    uint16_t hi = f2bf(f);
    uint16_t lo = f2bf(f - bf2f(hi));
    return bf2f(hi) + bf2f(lo);
  };
  double S = 0.0;
  for (int j = 0; j < n; ++j) S += stored(j);
  const double mu = S / n;
  double Qc = 0.0, Q = 0.0;
  for (int j = 0; j < n; ++j) {
    double st = stored(j);
    Qc += (st - mu) * (st - mu);
    Q += st * st;
  }
  if (p.kb16) {
    for (int s = 0; s < p.ksteps; ++s) {
      uint32_t whi[8], wlo[8];
#pragma unroll
      for (int e2 = 0; e2 < 8; ++e2) {
        uint32_t phi = 0, plo = 0;
#pragma unroll
        for (int hlf = 0; hlf < 2; ++hlf) {
          const int j = 16 * s + 2 * e2 + hlf;
          uint16_t vh = 0, vl = 0;
          if (j < n) {
            const float f = xs(j);
            vh = f2bf(f);
            vl = f2bf(f - bf2f(vh));
          }
          phi |= static_cast<uint32_t>(vh) << (16 * hlf);
          plo |= static_cast<uint32_t>(vl) << (16 * hlf);
        }
        whi[e2] = phi;
        wlo[e2] = plo;
      }
      u32x4* d = reinterpret_cast<u32x4*>(p.kb16 + (static_cast<size_t>(s) * p.vpad + k) * 32);
      d[0] = u32x4{whi[0], whi[1], whi[2], whi[3]};
      d[1] = u32x4{whi[4], whi[5], whi[6], whi[7]};
      d[2] = u32x4{wlo[0], wlo[1], wlo[2], wlo[3]};
      d[3] = u32x4{wlo[4], wlo[5], wlo[6], wlo[7]};
    }
  }
  if (p.kb32) {
    for (int s = 0; s < p.ksteps; ++s) {
      float f[8], f2[8];
#pragma unroll
      for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int subj = 8 * s + 2 * q + hh;
          float val = subj < n ? xs(subj) : 0.0f;
          f[hh * 4 + q] = val;
          f2[hh * 4 + q] = val * val;
        }
      f32x4* d = reinterpret_cast<f32x4*>(p.kb32 + (static_cast<size_t>(s) * p.vpad + k) * 8);
      d[0] = f32x4{f[0], f[1], f[2], f[3]};
      d[1] = f32x4{f[4], f[5], f[6], f[7]};
      if (p.kb32sq) {
        f32x4* d2 = reinterpret_cast<f32x4*>(p.kb32sq + (static_cast<size_t>(s) * p.vpad + k) * 8);
        d2[0] = f32x4{f2[0], f2[1], f2[2], f2[3]};
        d2[1] = f32x4{f2[4], f2[5], f2[6], f2[7]};
      }
    }
  }
  if (p.rows) {
    float* r = p.rows + k * p.ldn;
    for (int j = 0; j < p.ldn; ++j) r[j] = j < n ? xs(j) : 0.0f;
  }
  if (p.cst) {
    const double rinv = Qc > 0.0 ? 1.0 / sqrt(Qc) : 0.0;
    p.cst[k] = make_float2(static_cast<float>(rinv), static_cast<float>(-0.5 * S * rinv));
  }
  if (p.cstg) p.cstg[k] = make_float2(static_cast<float>(S), static_cast<float>(Q));
}

}  // namespace

size_t prep_bytes(int64_t v, int n, int flags) {
  Carver c(nullptr);
  prep_carve(c, v, n, n / 2, flags);
  return c.off;
}

PrepX prep_carve(Carver& c, int64_t v, int n, int n1, int flags) {
  PrepX p;
  p.v = v;
  p.vpad = round_up(v, 32);
  p.n = n;
  p.n1 = n1;
  if (flags & kPrepSplit) {
    p.ksteps = static_cast<int>(ceil_div(n, 16));
    p.kb16 = c.take<uint16_t>(static_cast<size_t>(p.ksteps) * p.vpad * 32);
  } else if (flags & kPrepF32) {
    p.ksteps = static_cast<int>(ceil_div(n, 8));
    p.kb32 = c.take<float>(static_cast<size_t>(p.ksteps) * p.vpad * 8);
    if (flags & kPrepUnbal) p.kb32sq = c.take<float>(static_cast<size_t>(p.ksteps) * p.vpad * 8);
  }
  if (flags & kPrepRows) {
    p.ldn = static_cast<int>(round_up(n, 4));
    p.rows = c.take<float>(static_cast<size_t>(p.vpad) * p.ldn);
  }
  p.cst = c.take<float2>(p.vpad);
  if (flags & kPrepUnbal) p.cstg = c.take<float2>(p.vpad);
  return p;
}

rpt_status prep_launch(const PrepX& p, const float* X, int64_t ldx, int tail, int flags, hipStream_t s) {
  const int64_t blocks = ceil_div(p.vpad, kBlock);
  hipLaunchKernelGGL(prep_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, X, p.v, p.n, ldx, p,
                     tail, flags);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace rpt
