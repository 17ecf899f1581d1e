// Training-phase kernels of RapidPT (Alg. 2, Sec. 4.1):
//
// * Re-orthonormalisation (Cholesky-QR): G = U^T U from per-workgroup partial
//   Gram matrices (split-BF16 matrix cores, FP32 within a workgroup, summed in
//   FP64), G = L L^T in FP64, R^{-1} = L^{-T}, then U <- U R^{-1} on the matrix
//   cores (3-pass split product).  Applied twice it gives the Q factor with a
//   positive-diagonal R ("Rand. Orth." of Alg. 2 and the retraction after
//   each tracking step).
// * Tracking update: U[omega_i, :] += gamma e_i w_i^T / |w_i|^2 summed over a
//   mini-batch (atomic FP32 adds: two columns of a batch may sample the same
//   voxel).  For one column this is GROUSE's greedy geodesic step up to the
//   choice of basis of the new subspace.
// * sigma: sample standard deviation of the sampled-entry residuals (FP64).
// * mu: mean of the per-column gaps (mean-gap rule) or the literal maximum
//   residual of Alg. 2.
#include "lds_linalg.h"
#include "rpt_internal.h"

namespace rpt {

namespace {

constexpr int kR = 128;          // rank bound
constexpr int kStage = 64;       // rows per LDS stage
constexpr int kLd = 72;          // bf16 per staged column (64 + pad)

// ---------------------------------------------------------------- Gram partials
template <int RT>
__global__ __launch_bounds__(kBlock) void gram_partial_kernel(const float* __restrict__ U, int64_t v, int r,
                                                             int64_t rows_per_blk, float* __restrict__ part) {
  __shared__ __align__(16) uint16_t uth[kR * kLd];
  __shared__ __align__(16) uint16_t utl[kR * kLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, col = lane & 31;
  const int64_t r0 = blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < v ? r0 + rows_per_blk : v;
  f32x16 acc[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) acc[t] = f32x16{};
  const int ac = tid & (kR - 1), par = tid >> 7;
  for (int64_t c0 = r0; c0 < r1; c0 += kStage) {
    float x[kStage / 2];
#pragma unroll
    for (int m = 0; m < kStage / 2; ++m) {
      const int64_t row = c0 + par + 2 * m;
      x[m] = (row < r1 && ac < r) ? U[row * r + ac] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kStage / 2; ++m) {
      const int kk = par + 2 * m;
      const uint16_t hi = f2bf(x[m]);
      uth[ac * kLd + kk] = hi;
      utl[ac * kLd + kk] = f2bf(x[m] - bf2f(hi));
    }
    __syncthreads();
    if (wave < RT) {
#pragma unroll
      for (int s = 0; s < kStage / 16; ++s) {
        const int ko = 16 * s + 8 * h;
        const u32x4 ah = *reinterpret_cast<const u32x4*>(uth + (wave * 32 + col) * kLd + ko);
        const u32x4 al = *reinterpret_cast<const u32x4*>(utl + (wave * 32 + col) * kLd + ko);
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          const u32x4 bh = *reinterpret_cast<const u32x4*>(uth + (t * 32 + col) * kLd + ko);
          const u32x4 bl = *reinterpret_cast<const u32x4*>(utl + (t * 32 + col) * kLd + ko);
          acc[t] = mfma_bf16(ah, bh, acc[t]);
          acc[t] = mfma_bf16(ah, bl, acc[t]);
          acc[t] = mfma_bf16(al, bh, acc[t]);
        }
      }
    }
  }
  if (wave < RT) {
    float* P = part + static_cast<int64_t>(blockIdx.x) * r * r;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = wave * 32 + mfma_row(e, h), cc = t * 32 + col;
        if (row < r && cc < r) P[row * r + cc] = acc[t][e];
      }
  }
}

// G = sum of the partials, in FP64: a workgroup owns 64 entries, its four
// waves sum interleaved quarters of the partials, LDS combines them.
__global__ __launch_bounds__(kBlock) void gram_reduce_kernel(const float* __restrict__ part, int nblk, int r,
                                                            double* __restrict__ G) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int idx = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (idx < r * r)
    for (int b = wave; b < nblk; b += 4) s += part[static_cast<int64_t>(b) * r * r + idx];
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && idx < r * r) G[idx] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// Factor G = L L^T (FP64, LDS) and write R^{-1} = L^{-T} transposed
// (RinvT[c][j] = Rinv[j][c] = Linv[c][j]) split into BF16 hi/lo.  A failed
// factorisation writes the identity (U is left unchanged) and info = j + 1.
__global__ __launch_bounds__(kBlock) void chol_rinv_kernel(const double* __restrict__ Gfull, int r,
                                                          uint16_t* __restrict__ rinvT_hi,
                                                          uint16_t* __restrict__ rinvT_lo, int32_t* info) {
  extern __shared__ __align__(16) unsigned char sm[];
  const int ntri = r * (r + 1) / 2;
  double* G = reinterpret_cast<double*>(sm);
  double* diag = G + ntri;
  double* dinv = diag + kR;
  float* Li = reinterpret_cast<float*>(dinv + kR);  // [r][kR]
  double* P = reinterpret_cast<double*>(Li + r * kR);  // [kCb][kPanelLd] Cholesky scratch
  const int tid = threadIdx.x;
  for (int idx = tid; idx < ntri; idx += kBlock) {
    // invert ptri: row i with i(i+1)/2 <= idx
    int i = static_cast<int>((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= idx) ++i;
    while (i * (i + 1) / 2 > idx) --i;
    const int c = idx - i * (i + 1) / 2;
    G[idx] = Gfull[i * r + c];
  }
  __syncthreads();
  const int failed = lds_cholesky_blocked<2>(G, dinv, P, r, r);
  if (!failed) lds_tri_inverse(G, dinv, r, Li, kR);
  __syncthreads();
  for (int idx = tid; idx < kR * kR; idx += kBlock) {
    const int c = idx / kR, j = idx - c * kR;
    float x = 0.0f;
    if (c < r && j < r) x = failed ? (c == j ? 1.0f : 0.0f) : Li[c * kR + j];
    const uint16_t hi = f2bf(x);
    rinvT_hi[idx] = hi;
    rinvT_lo[idx] = f2bf(x - bf2f(hi));
  }
  if (tid == 0 && info) *info = failed;
}

size_t chol_smem(int r) {
  return (static_cast<size_t>(r) * (r + 1) / 2 + 2 * kR + kCb * kPanelLd) * sizeof(double) + r * kR * sizeof(float);
}

// U <- U R^{-1}, in place; one wave per 32-row tile.
template <int KS>
__global__ __launch_bounds__(kBlock) void apply_rinv_kernel(float* __restrict__ U, int64_t v, int r,
                                                           const uint16_t* __restrict__ rth,
                                                           const uint16_t* __restrict__ rtl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
  const int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + wave;
  const int64_t v0 = tile * 32;
  if (v0 >= v) return;
  // A fragments: lane supplies U[v0 + col][16s + 8h + 0..7] (hi, lo)
  u32x4 Ah[KS], Al[KS];
  const int64_t vox = v0 + col;
  const bool vec = (r & 3) == 0;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int cb = 16 * s + 8 * h;
    float x[8];
    if (vec && vox < v && cb + 8 <= r) {
      const f32x4 p0 = *reinterpret_cast<const f32x4*>(U + vox * r + cb);
      const f32x4 p1 = *reinterpret_cast<const f32x4*>(U + vox * r + cb + 4);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        x[e] = p0[e];
        x[4 + e] = p1[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (vox < v && cb + e < r) ? U[vox * r + cb + e] : 0.0f;
    }
    unsigned wh[4], wl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t ph = 0, pl = 0;
#pragma unroll
      for (int hl = 0; hl < 2; ++hl) {
        const float xv = x[2 * q + hl];
        const uint16_t hi = f2bf(xv);
        ph |= static_cast<uint32_t>(hi) << (16 * hl);
        pl |= static_cast<uint32_t>(f2bf(xv - bf2f(hi))) << (16 * hl);
      }
      wh[q] = ph;
      wl[q] = pl;
    }
    Ah[s] = u32x4{wh[0], wh[1], wh[2], wh[3]};
    Al[s] = u32x4{wl[0], wl[1], wl[2], wl[3]};
  }
  const int CT = (r + 31) / 32;
  for (int ct = 0; ct < CT; ++ct) {
    f32x16 acc = f32x16{};
    const int c = ct * 32 + col;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int ko = 16 * s + 8 * h;
      const u32x4 bh = *reinterpret_cast<const u32x4*>(rth + c * kR + ko);
      const u32x4 bl = *reinterpret_cast<const u32x4*>(rtl + c * kR + ko);
      acc = mfma_bf16(Ah[s], bh, acc);
      acc = mfma_bf16(Ah[s], bl, acc);
      acc = mfma_bf16(Al[s], bh, acc);
    }
    // every lane's reads of this tile happened before the first MFMA above
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t row = v0 + mfma_row(e, h);
      if (row < v && c < r) U[row * r + c] = acc[e];
    }
  }
}

// ---------------------------------------------------------------- tracking update
__global__ __launch_bounds__(kBlock) void track_update_kernel(float* __restrict__ U, int64_t v, int r,
                                                             const int32_t* __restrict__ omega, int k,
                                                             const float* __restrict__ resid,
                                                             const float* __restrict__ W,
                                                             const float* __restrict__ wnorm2,
                                                             const int32_t* __restrict__ info, float gamma) {
  // one workgroup per batch column; thread t covers coefficient t % r of rows
  const int64_t i = blockIdx.x;
  if (info[i] != 0) return;
  const float n2 = wnorm2[i];
  if (!(n2 > 0.0f)) return;
  const float sc = gamma / n2;
  const int tid = threadIdx.x;
  const int per = kBlock / r > 0 ? kBlock / r : 1;  // rows handled per sweep
  const int c = tid % r, lr = tid / r;
  if (lr >= per) return;
  const float wc = W[i * r + c] * sc;
  for (int q = lr; q < k; q += per) {
    const int64_t row = omega[i * k + q];
    if (row < 0 || row >= v) continue;
    atomicAdd(U + row * r + c, resid[i * k + q] * wc);
  }
}

// ---------------------------------------------------------------- sigma, mu
// sums[0] += sum e, sums[1] += sum e^2 over n values (one pass, FP64)
__global__ __launch_bounds__(kBlock) void moments_kernel(const float* __restrict__ e, int64_t n, double* sums) {
  double s = 0.0, s2 = 0.0;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; t < n;
       t += static_cast<int64_t>(gridDim.x) * kBlock) {
    const double x = e[t];
    s += x;
    s2 += x * x;
  }
  s = wave_sum_d(s);
  s2 = wave_sum_d(s2);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(sums, s);
    atomicAdd(sums + 1, s2);
  }
}

__global__ void zero_doubles_kernel(double* p, int n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0.0;
}

__global__ void sigma_finish_kernel(const double* sums, int64_t n, float* sigma_mu) {
  const double mean = sums[0] / n;
  const double var = (sums[1] - n * mean * mean) / (n - 1);
  sigma_mu[0] = static_cast<float>(var > 0.0 ? sqrt(var) : 0.0);
}

// mu = mean of gaps (FP64), or max of per-column literal residual maxima, or 0
__global__ __launch_bounds__(kBlock) void mu_finish_kernel(const float* __restrict__ vals, int n, int rule,
                                                          float* sigma_mu) {
  __shared__ double red[kBlock];
  double acc = rule == RPT_MU_LITERAL ? -INFINITY : 0.0;
  for (int t = threadIdx.x; t < n; t += kBlock) acc = rule == RPT_MU_LITERAL ? fmax(acc, (double)vals[t]) : acc + vals[t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      red[threadIdx.x] = rule == RPT_MU_LITERAL ? fmax(red[threadIdx.x], red[threadIdx.x + w])
                                                : red[threadIdx.x] + red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (rule == RPT_MU_MEAN_GAP) sigma_mu[1] = static_cast<float>(red[0] / n);
    else if (rule == RPT_MU_LITERAL) sigma_mu[1] = static_cast<float>(red[0]);
    else sigma_mu[1] = 0.0f;
  }
}

// literal rule: per column i the maximum over voxels of T_ex[i, k] - (U w_i)_k
__global__ __launch_bounds__(kBlock) void literal_resid_max_kernel(const float* __restrict__ T, const float* __restrict__ U,
                                                                  const float* __restrict__ W, int64_t v, int r,
                                                                  float* __restrict__ out) {
  __shared__ float w[kR];
  __shared__ float red[4];
  const int64_t i = blockIdx.x;
  for (int c = threadIdx.x; c < r; c += kBlock) w[c] = W[i * r + c];
  __syncthreads();
  float best = -INFINITY;
  for (int64_t k = threadIdx.x; k < v; k += kBlock) {
    const float* u = U + k * r;
    float s = 0.0f;
    for (int c = 0; c < r; ++c) s = fmaf(u[c], w[c], s);
    best = fmaxf(best, T[i * v + k] - s);
  }
  best = wave_max(best);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x == 0) out[i] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

int gram_blocks(int64_t v) {
  int64_t nb = ceil_div(v, 256);
  if (nb > 256) nb = 256;
  if (nb < 1) nb = 1;
  return static_cast<int>(nb);
}

}  // namespace

size_t reorth_bytes(int64_t v, int r) {
  Carver c(nullptr);
  c.take<float>(static_cast<size_t>(gram_blocks(v)) * r * r);
  c.take<double>(static_cast<size_t>(r) * r);
  c.take<uint16_t>(static_cast<size_t>(kR) * kR);
  c.take<uint16_t>(static_cast<size_t>(kR) * kR);
  return c.off;
}

rpt_status reorth_launch(float* U, int64_t v, int r, int32_t* info, void* ws, hipStream_t s) {
  if (r < 1 || r > kR) return RPT_ERR_UNSUPPORTED;
  Carver c(ws);
  const int nb = gram_blocks(v);
  float* part = c.take<float>(static_cast<size_t>(nb) * r * r);
  double* gfull = c.take<double>(static_cast<size_t>(r) * r);
  uint16_t* rth = c.take<uint16_t>(static_cast<size_t>(kR) * kR);
  uint16_t* rtl = c.take<uint16_t>(static_cast<size_t>(kR) * kR);
  const int RT = (r + 31) / 32;
  const int64_t rpb = round_up(ceil_div(v, nb), kStage);
  RPT_STAGE("reorth", s);
  switch (RT) {
    case 1: hipLaunchKernelGGL(gram_partial_kernel<1>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part); break;
    case 2: hipLaunchKernelGGL(gram_partial_kernel<2>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part); break;
    case 3: hipLaunchKernelGGL(gram_partial_kernel<3>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part); break;
    default: hipLaunchKernelGGL(gram_partial_kernel<4>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part); break;
  }
  RPT_CHECK_LAUNCH();
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(static_cast<unsigned>(ceil_div(static_cast<int64_t>(r) * r, 64))),
                     dim3(kBlock), 0, s, part, nb, r, gfull);
  RPT_CHECK_LAUNCH();
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_rinv_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(chol_smem(kR)));
    attr_set = true;
  }
  hipLaunchKernelGGL(chol_rinv_kernel, dim3(1), dim3(kBlock), chol_smem(r), s, gfull, r, rth, rtl, info);
  RPT_CHECK_LAUNCH();
  const unsigned blocks = static_cast<unsigned>(ceil_div(ceil_div(v, 32), 4));
  const int KS = static_cast<int>(ceil_div(r, 16));
  switch (KS) {
    case 1: hipLaunchKernelGGL(apply_rinv_kernel<1>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl); break;
    case 2: hipLaunchKernelGGL(apply_rinv_kernel<2>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl); break;
    case 3: hipLaunchKernelGGL(apply_rinv_kernel<3>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl); break;
    case 4: hipLaunchKernelGGL(apply_rinv_kernel<4>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl); break;
    case 5: hipLaunchKernelGGL(apply_rinv_kernel<5>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl); break;
    case 6: hipLaunchKernelGGL(apply_rinv_kernel<6>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl); break;
    case 7: hipLaunchKernelGGL(apply_rinv_kernel<7>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl); break;
    default: hipLaunchKernelGGL(apply_rinv_kernel<8>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl); break;
  }
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status track_update_launch(float* U, int64_t v, int r, const int32_t* omega, int k, const float* resid,
                               const float* W, const float* wnorm2, const int32_t* info, int64_t B, float gamma,
                               hipStream_t s) {
  if (B == 0) return RPT_OK;
  RPT_STAGE("track_update", s);
  hipLaunchKernelGGL(track_update_kernel, dim3(static_cast<unsigned>(B)), dim3(kBlock), 0, s, U, v, r, omega, k, resid,
                     W, wnorm2, info, gamma);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status sigma_launch(const float* resid, int64_t n, double* sums, float* sigma_mu, hipStream_t s) {
  RPT_STAGE("sigma", s);
  hipLaunchKernelGGL(zero_doubles_kernel, dim3(1), dim3(64), 0, s, sums, 2);
  RPT_CHECK_LAUNCH();
  int64_t blocks = ceil_div(n, kBlock);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(moments_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, resid, n, sums);
  RPT_CHECK_LAUNCH();
  hipLaunchKernelGGL(sigma_finish_kernel, dim3(1), dim3(1), 0, s, sums, n, sigma_mu);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status mu_launch(const float* vals, int n, int rule, float* sigma_mu, hipStream_t s) {
  hipLaunchKernelGGL(mu_finish_kernel, dim3(1), dim3(kBlock), 0, s, vals, n, rule, sigma_mu);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status literal_resid_launch(const float* T, const float* U, const float* W, int64_t v, int r, int64_t ell,
                                float* out, hipStream_t s) {
  hipLaunchKernelGGL(literal_resid_max_kernel, dim3(static_cast<unsigned>(ell)), dim3(kBlock), 0, s, T, U, W, v, r,
                     out);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace rpt
