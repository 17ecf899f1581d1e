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
// Split path: every relabelling has exactly n1 group-1 subjects, so the
// constants fold into the data, x''_kj = x_kj rinv_k + c_k / n1, and the
// contraction of x'' is u itself (no per-voxel epilogue constants).
//
// Layouts written (vpad = v rounded up to 32; padding voxels are zero and get
// epilogue constants that can never win a maximum; in the folded split
// layout a padding voxel's entries are -1e30 / n1, so its u is -1e30):
//   kb16  [ks][vpad / 32][2][64][8] bf16: per K step and 32-voxel tile, the
//         hi block then the lo block, each in MFMA fragment order: lane
//         L = 32 h + c holds x''[voxel 32 t + c][subject 16 s + 8 h + 0..7]
//         (0 past n), so a wave's fragment is one contiguous 1 KB
//   kbm   [vpad / 32][64][8] bf16, when R = n mod 16 is 1..8: the last K
//         step as one mixed block, position kappa = hi of subject
//         16 (ks - 1) + kappa for kappa < R, lo of subject 16 (ks - 1) +
//         kappa - R for R <= kappa < 2 R, 0 beyond; same lane order
//   kb32  [ks][vpad][2][4] f32 subject 8s+2q+h at [s][k][h][q]
//   rows  [vpad][ldn] f32      standardised rows, for the sampled statistics
//   cst   [vpad] (rinv, -S/2 * rinv)       cstg [vpad] (S, Q)
#include "rpt_internal.h"

namespace rpt {

namespace {

constexpr int kPrepNMax = 512;  // subjects

// sum over the TPR consecutive lanes of a row group
template <int TPR>
__device__ __forceinline__ double row_sum(double x) {
#pragma unroll
  for (int off = 1; off < TPR; off <<= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// One workgroup prepares TILE voxel rows (64 for n <= 128, 16 up to 512, so
// that the rows fit in LDS): a coalesced load of the rows into LDS, FP64 row
// statistics with kBlock / TILE threads per row, then coalesced writes of
// every output layout.
template <int TILE, int NMAX>
__global__ __launch_bounds__(kBlock) void prep_kernel(const float* __restrict__ X, int64_t v, int n, int64_t ldx,
                                                     PrepX p, int tail, int flags) {
  constexpr int TPR = kBlock / TILE;
  __shared__ float xs[TILE][NMAX + 1];
  __shared__ double fold_c[TILE], fold_d[TILE];  // x'' = x * fold_c + fold_d
  const int tid = threadIdx.x;
  const int64_t v0 = static_cast<int64_t>(blockIdx.x) * TILE;
  const bool split = (flags & kPrepSplit) != 0;

  for (int idx = tid; idx < TILE * n; idx += kBlock) {
    const int r = idx / n, j = idx - r * n;
    const int64_t vox = v0 + r;
    xs[r][j] = vox < v ? X[vox * ldx + j] : 0.0f;
  }
  __syncthreads();

  // statistics: thread group of TPR per row (lanes TPR r .. TPR r + TPR - 1)
  const int r = tid / TPR, q = tid % TPR;
  const int64_t vox = v0 + r;
  double s0 = 0.0;
  for (int j = q; j < n; j += TPR) s0 += xs[r][j];
  s0 = row_sum<TPR>(s0);
  const double mean = s0 / n;
  double ss = 0.0;
  for (int j = q; j < n; j += TPR) {
    const double d = xs[r][j] - mean;
    ss += d * d;
  }
  ss = row_sum<TPR>(ss);
  const double sc = (ss > 0.0 && vox < v) ? sqrt((n - 1.0) / ss) : 0.0;
  // standardise in place (each thread its own entries)
  double S = 0.0;
  for (int j = q; j < n; j += TPR) {
    const float f = static_cast<float>((xs[r][j] - mean) * sc);
    xs[r][j] = f;
    float st = f;
    if (split) {
      const uint16_t hi = f2bf(f);
      st = bf2f(hi) + bf2f(f2bf(f - bf2f(hi)));
    }
    S += st;
  }
  S = row_sum<TPR>(S);
  const double mu = S / n;
  double Qc = 0.0, Q = 0.0;
  for (int j = q; j < n; j += TPR) {
    const float f = xs[r][j];
    float st = f;
    if (split) {
      const uint16_t hi = f2bf(f);
      st = bf2f(hi) + bf2f(f2bf(f - bf2f(hi)));
    }
    Qc += (st - mu) * (st - mu);
    Q += static_cast<double>(st) * st;
  }
  Qc = row_sum<TPR>(Qc);
  Q = row_sum<TPR>(Q);
  if (q == 0 && vox < p.vpad) {
    if (vox < v) {
      // t: scale to unit centred sum of squares; mean difference: undo the
      // standardisation's scale, so u is the centred group-1 sum of X itself
      const double rinv = (flags & kPrepMeanDiff) ? (sc > 0.0 ? 1.0 / sc : 0.0) : (Qc > 0.0 ? 1.0 / sqrt(Qc) : 0.0);
      if (p.cst) p.cst[vox] = make_float2(static_cast<float>(rinv), static_cast<float>(-0.5 * S * rinv));
      if (p.cstg) p.cstg[vox] = make_float2(static_cast<float>(S), static_cast<float>(Q));
      fold_c[r] = rinv;
      fold_d[r] = -0.5 * S * rinv / p.n1;
    } else {
      // padding voxels never win a maximum
      if (p.cst) p.cst[vox] = make_float2(0.0f, tail == RPT_TAIL_ABS ? 0.0f : -INFINITY);
      if (p.cstg) p.cstg[vox] = make_float2(0.0f, 0.0f);
      fold_c[r] = 0.0;
      fold_d[r] = tail == RPT_TAIL_ABS ? 0.0 : -1e30 / p.n1;
    }
  }
  __syncthreads();

  const int nv = static_cast<int>((p.vpad - v0) < TILE ? (p.vpad - v0) : TILE);
  if (p.kb16) {
    // per K step: TILE voxels x (hi 16 | lo 16) bf16 = 4 TILE chunks of 16 bytes
    for (int idx = tid; idx < p.ksteps * 4 * TILE; idx += kBlock) {
      const int s = idx / (4 * TILE), rr = (idx >> 2) % TILE, c = idx & 3;
      if (rr < nv) {
        uint32_t w[4];
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) {
          uint32_t pr = 0;
#pragma unroll
          for (int hl = 0; hl < 2; ++hl) {
            const int j = 16 * s + 8 * (c & 1) + 2 * e2 + hl;
            uint16_t val = 0;
            if (j < n) {
              const float f = static_cast<float>(static_cast<double>(xs[rr][j]) * fold_c[rr] + fold_d[rr]);
              const uint16_t hi = f2bf(f);
              val = (c < 2) ? hi : f2bf(f - bf2f(hi));
            }
            pr |= static_cast<uint32_t>(val) << (16 * hl);
          }
          w[e2] = pr;
        }
        const int64_t vx = v0 + rr;  // tile vx / 32, column vx % 32; c = 2 hl + h
        u32x4* d = reinterpret_cast<u32x4*>(p.kb16 + (static_cast<size_t>(s) * p.vpad + (vx & ~int64_t(31))) * 32 +
                                            (c >> 1) * 512 + ((c & 1) * 32 + (vx & 31)) * 8);
        *d = u32x4{w[0], w[1], w[2], w[3]};
      }
    }
  }
  if (p.kbm) {
    // the mixed K block: position kappa < R holds hi of subject 16 F + kappa,
    // R <= kappa < 2 R lo of subject 16 F + kappa - R (F full steps), then 0;
    // lane L = 32 h + c holds positions 8 h .. 8 h + 7 of voxel 32 t + c
    const int R = p.mixr, F = n / 16;
    for (int idx = tid; idx < 2 * TILE; idx += kBlock) {
      const int rr = idx >> 1, h = idx & 1;
      if (rr < nv) {
        uint32_t w[4];
#pragma unroll
        for (int e2 = 0; e2 < 4; ++e2) {
          uint32_t pr = 0;
#pragma unroll
          for (int hl = 0; hl < 2; ++hl) {
            const int kap = 8 * h + 2 * e2 + hl;
            uint16_t val = 0;
            if (kap < 2 * R) {
              const int j = 16 * F + (kap < R ? kap : kap - R);
              const float f = static_cast<float>(static_cast<double>(xs[rr][j]) * fold_c[rr] + fold_d[rr]);
              const uint16_t hi = f2bf(f);
              val = kap < R ? hi : f2bf(f - bf2f(hi));
            }
            pr |= static_cast<uint32_t>(val) << (16 * hl);
          }
          w[e2] = pr;
        }
        const int64_t vx = v0 + rr;
        u32x4* d = reinterpret_cast<u32x4*>(p.kbm + (vx & ~int64_t(31)) * 16 + (h * 32 + (vx & 31)) * 8);
        *d = u32x4{w[0], w[1], w[2], w[3]};
      }
    }
  }
  if (p.kb32) {
    // per K block: TILE voxels x 8 floats = 2 TILE chunks of 16 bytes
    for (int s = 0; s < p.ksteps; ++s) {
      for (int ch = tid; ch < 2 * TILE; ch += kBlock) {
        const int rr = ch >> 1, hh = ch & 1;
        if (rr >= nv) continue;
        float f[4], f2[4];
#pragma unroll
        for (int qq = 0; qq < 4; ++qq) {
          const int j = 8 * s + 2 * qq + hh;
          f[qq] = j < n ? xs[rr][j] : 0.0f;
          f2[qq] = f[qq] * f[qq];
        }
        const size_t off = (static_cast<size_t>(s) * p.vpad + v0 + rr) * 8 + 4 * hh;
        *reinterpret_cast<f32x4*>(p.kb32 + off) = f32x4{f[0], f[1], f[2], f[3]};
        if (p.kb32sq) *reinterpret_cast<f32x4*>(p.kb32sq + off) = f32x4{f2[0], f2[1], f2[2], f2[3]};
      }
    }
  }
  if (p.rows) {
    const int ld = p.ldn;
    for (int idx = tid; idx < nv * ld; idx += kBlock) {
      const int rr = idx / ld, j = idx - rr * ld;
      p.rows[(v0 + rr) * ld + j] = j < n ? xs[rr][j] : 0.0f;
    }
  }
}

}  // namespace

size_t prep_bytes(int64_t v, int n, int flags) {
  Carver c(nullptr);
  prep_carve(c, v, n, n / 2, flags);
  return c.off;
}

PrepX prep_carve(Carver& c, int64_t v, int n, int n1, int flags) {
  PrepX p;
  p.stat = (flags & kPrepMeanDiff) ? RPT_STAT_MEANDIFF : RPT_STAT_T;
  p.v = v;
  p.vpad = round_up(v, 32);
  p.n = n;
  p.n1 = n1;
  if (flags & kPrepSplit) {
    p.ksteps = static_cast<int>(ceil_div(n, 16));
    p.kb16 = c.take<uint16_t>(static_cast<size_t>(p.ksteps) * p.vpad * 32);
    if (p.ksteps <= 8 && n % 16 >= 1 && n % 16 <= 8) {
      p.mixr = n % 16;
      p.kbm = c.take<uint16_t>(static_cast<size_t>(p.vpad) * 16);
    }
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
  if (p.n > kPrepNMax) return RPT_ERR_UNSUPPORTED;
  RPT_STAGE("prep", s);
  if (p.n <= 128) {
    hipLaunchKernelGGL((prep_kernel<64, 128>), dim3(static_cast<unsigned>(ceil_div(p.vpad, 64))), dim3(kBlock), 0, s,
                       X, p.v, p.n, ldx, p, tail, flags);
  } else {
    hipLaunchKernelGGL((prep_kernel<16, kPrepNMax>), dim3(static_cast<unsigned>(ceil_div(p.vpad, 16))),
                       dim3(kBlock), 0, s, X, p.v, p.n, ldx, p, tail, flags);
  }
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace rpt
