// Training-phase kernels of RapidPT (Alg. 2, Sec. 4.1):
//
// * Re-orthonormalisation (Cholesky-QR): G = U^T U from per-workgroup partial
//   Gram matrices (split-BF16 matrix cores, FP32 within a workgroup, summed in
//   FP64), G = L L^T in FP64, R^{-1} = L^{-T}, then U <- U R^{-1} on the matrix
//   cores (3-pass split product).  Applied twice it gives the Q factor with a
//   positive-diagonal R ("Rand. Orth." of Alg. 2 and the retraction after
//   each tracking step).
// * Tracking update: U[omega_i, :] += gamma e_i w_i^T / |w_i|^2 summed over a
//   mini-batch, e_i = y_i - U[omega_i, :] w_i with the basis before the update
//   (two columns of a batch may sample the same voxel: each voxel's entries
//   are linked into a list by Complete and applied together).  For one column
//   this is GROUSE's greedy geodesic step up to the choice of basis of the new
//   subspace.
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
// U^T U over a contiguous range of rows per workgroup, 64 rows at a time:
// the chunk (64 r contiguous floats) is read with coalesced 16-byte loads
// (the next chunk's loads are issued before this chunk's products), split
// into BF16 hi/lo and stored transposed in LDS; the lower-triangular 16 x 16
// tiles are spread over the four waves and accumulated on 16x16x32 MFMA as
// hi.hi + hi.lo + lo.hi.  Each wave writes its own tiles of the partial:
// tile t = (bi, bj), bj <= bi, element 64 e + lane (row 16 bi +
// 4 (lane / 16) + e, column 16 bj + lane % 16).
constexpr int kGramChunk = 64;
constexpr int kGramLd = kGramChunk + 8;  // bf16 per staged column (16-byte aligned fragments)
template <int RB>
__global__ __launch_bounds__(kBlock, 2) void gram_partial_kernel(const float* __restrict__ U, int64_t v, int r,
                                                                int64_t rows_per_blk, float* __restrict__ part,
                                                                const int32_t* stop, int pass) {
  constexpr int NTILE = RB * (RB + 1) / 2;
  constexpr int TPW = (NTILE + 3) / 4;                    // tiles per wave
  constexpr int NV = RB;  // column groups of 4 per thread per chunk (4 RB groups over 4 waves)
  __shared__ __align__(16) uint16_t uth[16 * RB * kGramLd];
  __shared__ __align__(16) uint16_t utl[16 * RB * kGramLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, c16 = lane & 15, kq = lane >> 4;
  if (stop && *stop < pass) return;
  const int64_t r0 = blockIdx.x * rows_per_blk;
  const int64_t r1 = r0 + rows_per_blk < v ? r0 + rows_per_blk : v;
  const bool vec = (r & 3) == 0 && (reinterpret_cast<uintptr_t>(U) & 15) == 0;
  f32x4 acc[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // lane = row of the chunk; wave w takes column groups 4 (w + 4 u) .. + 3, so
  // the transpose stores of a wave are 64 consecutive rows of one column
  f32x4 buf[NV];
  auto load = [&](int64_t c0) {
    const int64_t row = c0 + lane;
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int cb = 4 * (wave + 4 * u);
      if (vec) {
        buf[u] = (row < r1 && cb < r) ? *reinterpret_cast<const f32x4*>(U + row * r + cb) : f32x4{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) buf[u][e] = (row < r1 && cb + e < r) ? U[row * r + cb + e] : 0.0f;
      }
    }
  };
  if (r0 < r1) load(r0);
  for (int64_t c0 = r0; c0 < r1; c0 += kGramChunk) {
    __syncthreads();  // previous chunk's MFMA reads of the stage are done
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int cb = 4 * (wave + 4 * u);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int col = cb + e;
        if (col < 16 * RB) {
          const float xv = buf[u][e];
          const uint16_t hv = f2bf(xv);
          uth[col * kGramLd + lane] = hv;
          utl[col * kGramLd + lane] = f2bf(xv - bf2f(hv));
        }
      }
    }
    if (c0 + kGramChunk < r1) load(c0 + kGramChunk);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kGramChunk / 32; ++ks) {
      const int ko = 32 * ks + 8 * kq;
#pragma unroll
      for (int tt = 0; tt < TPW; ++tt) {
        const int t = wave + 4 * tt;
        if (t < NTILE) {
          int bi = 0;
#pragma unroll
          for (int q = 1; q < RB; ++q) bi += (q * (q + 1) / 2 <= t) ? 1 : 0;
          const int bj = t - bi * (bi + 1) / 2;
          const u32x4 ah = *reinterpret_cast<const u32x4*>(uth + (16 * bi + c16) * kGramLd + ko);
          const u32x4 al = *reinterpret_cast<const u32x4*>(utl + (16 * bi + c16) * kGramLd + ko);
          const u32x4 bh = *reinterpret_cast<const u32x4*>(uth + (16 * bj + c16) * kGramLd + ko);
          const u32x4 bl = *reinterpret_cast<const u32x4*>(utl + (16 * bj + c16) * kGramLd + ko);
          acc[tt] = mfma16_bf16(ah, bh, acc[tt]);
          acc[tt] = mfma16_bf16(ah, bl, acc[tt]);
          acc[tt] = mfma16_bf16(al, bh, acc[tt]);
        }
      }
    }
  }
  float* P = part + static_cast<int64_t>(blockIdx.x) * NTILE * 256;
#pragma unroll
  for (int tt = 0; tt < TPW; ++tt) {
    const int t = wave + 4 * tt;
    if (t < NTILE)
#pragma unroll
      for (int e = 0; e < 4; ++e) P[t * 256 + 64 * e + lane] = acc[tt][e];
  }
}

// G (lower triangle, FP64) = sum of the partials: a workgroup owns 64
// entries; its 16 waves sum interleaved sixteenths of the partials (eight
// loads in flight per lane), LDS combines them.
constexpr int kRedWaves = 16;
__global__ __launch_bounds__(64 * kRedWaves) void gram_reduce_kernel(const float* __restrict__ part, int nblk,
                                                                    int ntile, int r, double* __restrict__ G,
                                                                    const int32_t* stop, int pass) {
  __shared__ double red[kRedWaves][64];
  if (stop && *stop < pass) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int idx = blockIdx.x * 64 + lane;
  const int n = ntile * 256;
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (idx < n) {
    int b = wave;
    for (; b + 7 * kRedWaves < nblk; b += 8 * kRedWaves) {
#pragma unroll
      for (int u = 0; u < 8; ++u) s[u] += part[static_cast<int64_t>(b + u * kRedWaves) * n + idx];
    }
    for (; b < nblk; b += kRedWaves) s[0] += part[static_cast<int64_t>(b) * n + idx];
  }
  red[wave][lane] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  __syncthreads();
  if (wave == 0 && idx < n) {
    double tot = 0.0;
#pragma unroll
    for (int w = 0; w < kRedWaves; ++w) tot += red[w][lane];
    // decode (tile, element) -> (row, column)
    const int t = idx >> 8, el = idx & 255, e = el >> 6, l = el & 63;
    int bi = 0;
    while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
    const int bj = t - bi * (bi + 1) / 2;
    const int row = 16 * bi + 4 * (l >> 4) + e, col = 16 * bj + (l & 15);
    if (row < r && col <= row) G[row * r + col] = tot;
  }
}

// Factor G = L L^T (FP64, LDS) and write R^{-1} = L^{-T} transposed
// (RinvT[c][j] = Rinv[j][c] = Linv[c][j]) split into BF16 hi/lo.  A failed
// factorisation writes the identity (U is left unchanged) and info = j + 1.
// One workgroup of 16 waves: the kernel runs alone, so every phase gets all
// of a CU's waves.
constexpr int kCholThreads = 1024;
__global__ __launch_bounds__(kCholThreads) void chol_rinv_kernel(const double* __restrict__ Gfull, int r,
                                                                uint16_t* __restrict__ rinvT_hi,
                                                                uint16_t* __restrict__ rinvT_lo, int32_t* info,
                                                                const int32_t* stop, int pass) {
  extern __shared__ __align__(16) unsigned char sm[];
  if (stop && *stop < pass) return;
  const int ntri = r * (r + 1) / 2;
  double* G = reinterpret_cast<double*>(sm);
  double* diag = G + ntri;
  double* dinv = diag + kR;
  float* Li = reinterpret_cast<float*>(dinv + kR);  // [rp][kR]
  double* P = reinterpret_cast<double*>(Li + ((r + kCb - 1) / kCb) * kCb * kR);  // [kCb][kPanelLd] scratch
  const int tid = threadIdx.x;
  // packed lower triangle from the full matrix: thread (i, c) for row i
  for (int i = tid / 64; i < r; i += kCholThreads / 64)
    for (int c = tid & 63; c <= i; c += 64) G[ptri(i, c)] = Gfull[i * r + c];
  __syncthreads();
  const int failed = lds_cholesky_blocked<2>(G, dinv, P, r, r);
  if (!failed) lds_tri_inverse_blocked(G, dinv, r, Li, kR, P);
  __syncthreads();
  // eight consecutive entries per thread, written as 16-byte BF16 vectors
  for (int idx = tid * 8; idx < kR * kR; idx += kCholThreads * 8) {
    const int c = idx / kR, j0 = idx - c * kR;
    u32x4 hv, lv;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint16_t h2[2], l2[2];
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int j = j0 + 2 * q + e;
        float x = 0.0f;
        if (c < r && j < r) x = failed ? (c == j ? 1.0f : 0.0f) : Li[c * kR + j];
        h2[e] = f2bf(x);
        l2[e] = f2bf(x - bf2f(h2[e]));
      }
      hv[q] = pack_bf2(h2[0], h2[1]);
      lv[q] = pack_bf2(l2[0], l2[1]);
    }
    *reinterpret_cast<u32x4*>(rinvT_hi + idx) = hv;
    *reinterpret_cast<u32x4*>(rinvT_lo + idx) = lv;
  }
  if (tid == 0 && info) *info = failed;
}

size_t chol_smem(int r) {
  const size_t rp = static_cast<size_t>((r + kCb - 1) / kCb) * kCb;
  return (static_cast<size_t>(r) * (r + 1) / 2 + 2 * kR + kCb * kPanelLd) * sizeof(double) + rp * kR * sizeof(float);
}

// U <- U R^{-1}, in place.  R^{-T} (BF16 hi/lo) is staged in LDS once per
// workgroup (rows padded against bank conflicts); each wave then takes
// 32-row tiles of U in turn: A fragments straight from its rows, the
// product on the matrix cores as a 3-pass split, written back over the
// same rows (all reads of a tile happen before its first write).
constexpr int kRl = kR + 8;  // LDS row length of the staged R^{-T}
template <int KS>
__global__ __launch_bounds__(kBlock, 2) void apply_rinv_kernel(float* __restrict__ U, int64_t v, int r,
                                                              const uint16_t* __restrict__ rth,
                                                              const uint16_t* __restrict__ rtl,
                                                              const int32_t* stop, int pass) {
  __shared__ __align__(16) uint16_t sh[kR * kRl];
  __shared__ __align__(16) uint16_t sl[kR * kRl];
  if (stop && *stop < pass) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, col = lane & 31;
  for (int t = tid; t < kR * (kR / 8); t += kBlock) {
    const int row = t / (kR / 8), c8 = (t - row * (kR / 8)) * 8;
    *reinterpret_cast<u32x4*>(sh + row * kRl + c8) = *reinterpret_cast<const u32x4*>(rth + row * kR + c8);
    *reinterpret_cast<u32x4*>(sl + row * kRl + c8) = *reinterpret_cast<const u32x4*>(rtl + row * kR + c8);
  }
  __syncthreads();
  const bool vec = (r & 3) == 0 && (reinterpret_cast<uintptr_t>(U) & 15) == 0;
  const int CT = (r + 31) / 32;
  const int64_t ntile = (v + 31) / 32;
  for (int64_t tile = static_cast<int64_t>(blockIdx.x) * 4 + wave; tile < ntile;
       tile += static_cast<int64_t>(gridDim.x) * 4) {
    const int64_t v0 = tile * 32;
    // A fragments: lane supplies U[v0 + col][16s + 8h + 0..7] (hi, lo)
    u32x4 Ah[KS], Al[KS];
    const int64_t vox = v0 + col;
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
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint16_t h0 = f2bf(x[2 * q]), h1 = f2bf(x[2 * q + 1]);
        Ah[s][q] = pack_bf2(h0, h1);
        Al[s][q] = pack_bf2(f2bf(x[2 * q] - bf2f(h0)), f2bf(x[2 * q + 1] - bf2f(h1)));
      }
    }
    for (int ct = 0; ct < CT; ++ct) {
      f32x16 acc = f32x16{};
      const int c = ct * 32 + col;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int ko = 16 * s + 8 * h;
        const u32x4 bh = *reinterpret_cast<const u32x4*>(sh + c * kRl + ko);
        const u32x4 bl = *reinterpret_cast<const u32x4*>(sl + c * kRl + ko);
        acc = mfma_bf16(Ah[s], bh, acc);
        acc = mfma_bf16(Ah[s], bl, acc);
        acc = mfma_bf16(Al[s], bh, acc);
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t row = v0 + mfma_row(e, h);
        if (row < v && c < r) U[row * r + c] = acc[e];
      }
    }
  }
}

// ---------------------------------------------------------------- tracking update
// A quarter wave per voxel: read the voxel's basis row, walk its list of
// sampled entries (linked by the Complete kernel), form each entry's residual
// e = T[i][voxel] - row . w_i (a 16-lane reduction), sum gamma e / |w_i|^2 *
// w_i over the list, write the row plus the sum, and reset the list head.
// Lane l of the quarter covers columns l + 16 j, so row accesses are 64-byte
// segments; four voxels per wave keep four dependent list walks in flight.
constexpr int kTrackLanes = 16;
__global__ __launch_bounds__(kBlock) void track_apply_kernel(float* __restrict__ U, int64_t v, int r, int k,
                                                            const float* __restrict__ T, int64_t ldT,
                                                            const float* __restrict__ W,
                                                            const float* __restrict__ wnorm2,
                                                            const int32_t* __restrict__ info, float gamma,
                                                            int32_t* __restrict__ lhead,
                                                            const int32_t* __restrict__ lnext) {
  constexpr int NJ = (128 + kTrackLanes - 1) / kTrackLanes;
  const int64_t vox = static_cast<int64_t>(blockIdx.x) * (kBlock / kTrackLanes) + (threadIdx.x / kTrackLanes);
  const int l = threadIdx.x % kTrackLanes;
  if (vox >= v) return;
  int e = lhead[vox];
  if (e < 0) return;
  // the voxel's basis row before the update: every entry's residual uses it
  float* u = U + vox * r;
  float u0[NJ], acc[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int c = l + kTrackLanes * j;
    u0[j] = c < r ? u[c] : 0.0f;
    acc[j] = 0.0f;
  }
  while (e >= 0) {
    const int i = e / k;
    const float n2 = wnorm2[i];
    const float y = T[static_cast<int64_t>(i) * ldT + vox];
    const float* wi = W + static_cast<int64_t>(i) * r;
    float wv[NJ], dot = 0.0f;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int c = l + kTrackLanes * j;
      wv[j] = c < r ? wi[c] : 0.0f;
      dot = fmaf(u0[j], wv[j], dot);
    }
#pragma unroll
    for (int off = kTrackLanes / 2; off > 0; off >>= 1) dot += __shfl_xor(dot, off, kTrackLanes);
    // residual e = y - U_vox . w_i of this sampled entry
    const float coef = (info[i] == 0 && n2 > 0.0f) ? gamma * (y - dot) / n2 : 0.0f;
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[j] = fmaf(coef, wv[j], acc[j]);
    e = lnext[e];
  }
#pragma unroll
  for (int j = 0; j < NJ; ++j) {
    const int c = l + kTrackLanes * j;
    if (c < r) u[c] = u0[j] + acc[j];
  }
  if (l == 0) lhead[vox] = -1;  // every lane of this quarter wave read the head above
}

__global__ __launch_bounds__(kBlock) void fill_i32_kernel(int32_t* p, int64_t n, int32_t value) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; t < n;
       t += static_cast<int64_t>(gridDim.x) * kBlock)
    p[t] = value;
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
  // one atomic pair per workgroup
  __shared__ double red[2][kBlock / 64];
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = s;
    red[1][threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(sums, (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]));
    atomicAdd(sums + 1, (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
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
  if (nb > 768) nb = 768;  // three workgroups per CU (150 VGPRs: three waves per SIMD)
  if (nb < 1) nb = 1;
  return static_cast<int>(nb);
}

}  // namespace

size_t reorth_bytes(int64_t v, int r) {
  Carver c(nullptr);
  c.take<float>(static_cast<size_t>(gram_blocks(v)) * 36 * 256);
  c.take<double>(static_cast<size_t>(r) * r);
  c.take<uint16_t>(static_cast<size_t>(kR) * kR);
  c.take<uint16_t>(static_cast<size_t>(kR) * kR);
  return c.off;
}

rpt_status reorth_launch(float* U, int64_t v, int r, int32_t* info, void* ws, hipStream_t s,
                         const std::function<rpt_status()>* before_chol, const int32_t* stop, int pass) {
  if (r < 1 || r > kR) return RPT_ERR_UNSUPPORTED;
  Carver c(ws);
  const int nb = gram_blocks(v);
  float* part = c.take<float>(static_cast<size_t>(nb) * 36 * 256);
  double* gfull = c.take<double>(static_cast<size_t>(r) * r);
  uint16_t* rth = c.take<uint16_t>(static_cast<size_t>(kR) * kR);
  uint16_t* rtl = c.take<uint16_t>(static_cast<size_t>(kR) * kR);
  const int RB = (r + 15) / 16;
  const int ntile = RB * (RB + 1) / 2;
  const int64_t rpb = round_up(ceil_div(v, nb), kGramChunk);
  {
  RPT_STAGE("reorth_gram", s);
  switch (RB) {
    case 1: hipLaunchKernelGGL(gram_partial_kernel<1>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part, stop, pass); break;
    case 2: hipLaunchKernelGGL(gram_partial_kernel<2>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part, stop, pass); break;
    case 3: hipLaunchKernelGGL(gram_partial_kernel<3>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part, stop, pass); break;
    case 4: hipLaunchKernelGGL(gram_partial_kernel<4>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part, stop, pass); break;
    case 5: hipLaunchKernelGGL(gram_partial_kernel<5>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part, stop, pass); break;
    case 6: hipLaunchKernelGGL(gram_partial_kernel<6>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part, stop, pass); break;
    case 7: hipLaunchKernelGGL(gram_partial_kernel<7>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part, stop, pass); break;
    default: hipLaunchKernelGGL(gram_partial_kernel<8>, dim3(nb), dim3(kBlock), 0, s, U, v, r, rpb, part, stop, pass); break;
  }
  RPT_CHECK_LAUNCH();
  }
  {
    RPT_STAGE("reorth_reduce", s);
    hipLaunchKernelGGL(gram_reduce_kernel,
                       dim3(static_cast<unsigned>(ceil_div(static_cast<int64_t>(ntile) * 256, 64))),
                       dim3(64 * kRedWaves), 0, s, part, nb, ntile, r, gfull, stop, pass);
    RPT_CHECK_LAUNCH();
  }
  if (before_chol && *before_chol) RPT_TRY((*before_chol)());
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&chol_rinv_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(chol_smem(kR)));
    attr_set = true;
  }
  {
    RPT_STAGE("reorth_chol", s);
    hipLaunchKernelGGL(chol_rinv_kernel, dim3(1), dim3(kCholThreads), chol_smem(r), s, gfull, r, rth, rtl, info, stop,
                       pass);
    RPT_CHECK_LAUNCH();
  }
  int64_t ab = ceil_div(ceil_div(v, 32), 4);
  if (ab > 512) ab = 512;  // two workgroups per CU; each wave then loops over tiles
  const unsigned blocks = static_cast<unsigned>(ab);
  const int KS = static_cast<int>(ceil_div(r, 16));
  RPT_STAGE("reorth_apply", s);
  switch (KS) {
    case 1: hipLaunchKernelGGL(apply_rinv_kernel<1>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl, stop, pass); break;
    case 2: hipLaunchKernelGGL(apply_rinv_kernel<2>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl, stop, pass); break;
    case 3: hipLaunchKernelGGL(apply_rinv_kernel<3>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl, stop, pass); break;
    case 4: hipLaunchKernelGGL(apply_rinv_kernel<4>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl, stop, pass); break;
    case 5: hipLaunchKernelGGL(apply_rinv_kernel<5>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl, stop, pass); break;
    case 6: hipLaunchKernelGGL(apply_rinv_kernel<6>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl, stop, pass); break;
    case 7: hipLaunchKernelGGL(apply_rinv_kernel<7>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl, stop, pass); break;
    default: hipLaunchKernelGGL(apply_rinv_kernel<8>, dim3(blocks), dim3(kBlock), 0, s, U, v, r, rth, rtl, stop, pass); break;
  }
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

// ---------------------------------------------------------------- masked-loss step
// W^T of a batch (nb x r -> r x nb, the masked loss's layout) and the CSR
// offsets b k of its dense sampled sets
__global__ __launch_bounds__(kBlock) void grad_prep_kernel(const float* __restrict__ W, int nb, int r,
                                                          float* __restrict__ WT, int64_t* __restrict__ ptr, int k) {
  const int64_t n = static_cast<int64_t>(nb) * r;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; t < n;
       t += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t b = t / r, c = t - b * r;
    WT[c * nb + b] = W[t];
  }
  for (int64_t b = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; b <= nb;
       b += static_cast<int64_t>(gridDim.x) * kBlock)
    ptr[b] = b * k;
}

// U += a G over n entries (16-byte accesses over the first 4 n4)
__global__ __launch_bounds__(kBlock) void axpy_kernel(float* __restrict__ U, const float* __restrict__ G, int64_t n,
                                                     int64_t n4, float a) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; t < n4;
       t += static_cast<int64_t>(gridDim.x) * kBlock) {
    f32x4 u = reinterpret_cast<f32x4*>(U)[t];
    const f32x4 g = reinterpret_cast<const f32x4*>(G)[t];
#pragma unroll
    for (int e = 0; e < 4; ++e) u[e] = fmaf(a, g[e], u[e]);
    reinterpret_cast<f32x4*>(U)[t] = u;
  }
  for (int64_t t = 4 * n4 + blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; t < n;
       t += static_cast<int64_t>(gridDim.x) * kBlock)
    U[t] = fmaf(a, G[t], U[t]);
}

// *out += sum e^2 over n values, one workgroup in a fixed order (FP64)
__global__ __launch_bounds__(kBlock) void sumsq_add_kernel(const float* __restrict__ e, int64_t n, double* out) {
  __shared__ double red[kBlock / kWave];
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < n; t += kBlock) {
    const double x = e[t];
    s = fma(x, x, s);
  }
  s = wave_sum_d(s);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) t += red[w];
    *out += t;
  }
}

rpt_status grad_prep_launch(const float* W, int nb, int r, float* WT, int64_t* ptr, int k, hipStream_t s) {
  int64_t blocks = ceil_div(static_cast<int64_t>(nb) * r + 1, kBlock);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(grad_prep_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, W, nb, r, WT, ptr,
                     k);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status axpy_launch(float* U, const float* G, int64_t n, float a, hipStream_t s) {
  if (n <= 0) return RPT_OK;
  RPT_STAGE("grad_step", s);
  int64_t blocks = ceil_div(n / 4 + 1, kBlock);
  if (blocks > 4096) blocks = 4096;
  const bool al = ((reinterpret_cast<uintptr_t>(U) | reinterpret_cast<uintptr_t>(G)) & 15) == 0;
  hipLaunchKernelGGL(axpy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, U, G, n, al ? n / 4 : 0,
                     a);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status sumsq_add_launch(const float* e, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_add_kernel, dim3(1), dim3(kBlock), 0, s, e, n, out);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status track_apply_launch(float* U, int64_t v, int r, int k, const float* T, int64_t ldT, const float* W,
                              const float* wnorm2, const int32_t* info, float gamma, int32_t* lhead,
                              const int32_t* lnext, hipStream_t s) {
  if (r < 1 || r > kR) return RPT_ERR_UNSUPPORTED;
  RPT_STAGE("track_update", s);
  const unsigned blocks = static_cast<unsigned>(ceil_div(v, kBlock / kTrackLanes));
  hipLaunchKernelGGL(track_apply_kernel, dim3(blocks), dim3(kBlock), 0, s, U, v, r, k, T, ldT, W, wnorm2, info,
                     gamma, lhead, lnext);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t s) {
  if (n <= 0) return RPT_OK;
  int64_t blocks = ceil_div(n, kBlock);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, p, n, value);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status sigma_launch(const float* resid, int64_t n, double* sums, float* sigma_mu, hipStream_t s) {
  RPT_STAGE("sigma", s);
  hipLaunchKernelGGL(zero_doubles_kernel, dim3(1), dim3(64), 0, s, sums, 2);
  RPT_CHECK_LAUNCH();
  int64_t blocks = ceil_div(n, kBlock * 4);
  if (blocks > 256) blocks = 256;
  if (blocks < 1) blocks = 1;
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
