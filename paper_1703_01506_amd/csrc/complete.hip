// K3 + K4 -- Complete (Alg. 2): per column i, the masked least-squares fit
//     w_i = argmin_w | U[omega_i, :] w - y_i |_2
// from the normal equations G w = b, G = U_O^T U_O, b = U_O^T y.
//
// One workgroup per column.  The sampled basis rows are gathered 32 at a time
// (coalesced: a row is r contiguous floats) into LDS, transposed and split
// into BF16 hi/lo halves; G accumulates on the matrix cores as
// hi.hi + hi.lo + lo.hi (the split product keeps about 16 significant bits per
// term, FP32 accumulation).  b accumulates from the FP32 values in FP64.
// G is then moved to LDS in FP64 (packed lower triangle) and factored by a
// right-looking Cholesky in FP64; two triangular solves in one wave give w.
// A non-positive pivot at step j sets info[i] = j + 1 and w_i = 0.
// Optionally the residual y - U_O w is written (FP32 dot products).
#include "lds_linalg.h"
#include "rpt_internal.h"

namespace rpt {

namespace {

constexpr int kRMax = 128;           // basis rank handled in LDS
constexpr int kChunk = 64;           // sampled rows per LDS stage
constexpr int kStageLd = 72;         // bf16 per staged column (64 + pad: conflict-free 16-byte reads)
constexpr int kIdxBlk = 1024;        // sampled indices / values staged in LDS at a time

struct CompleteArgs {
  const float* U;
  int64_t v;
  int r;
  const int32_t* omega;
  int k;
  const float* y;       // [L][k]  (or nullptr when Trows is used)
  const float* Trows;   // alternative source: y[i][q] = Trows[trow(i) * ldT + omega[i][q]]
  int64_t ldT;
  const int32_t* trow;  // row of Trows for column i (nullptr: row i)
  int64_t L;
  float* W;             // [L][r]
  float* resid;         // [L][k] or nullptr
  int32_t* info;        // [L]
  float* wnorm2;        // [L] |w|^2 (or nullptr)
};

__device__ __forceinline__ float y_at(const CompleteArgs& a, int64_t i, int q) {
  if (a.y) return a.y[i * a.k + q];
  const int64_t row = a.trow ? a.trow[i] : i;
  const int64_t vox = a.omega[i * a.k + q];
  return (vox >= 0 && vox < a.ldT) ? a.Trows[row * a.ldT + vox] : 0.0f;
}

template <int RT>
__global__ __launch_bounds__(kBlock) void complete_kernel(CompleteArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  // stage: UT_hi[kRMax][kStageLd] bf16, UT_lo[...], ybuf[kIdxBlk] f32, ibuf[kIdxBlk] i32
  uint16_t* uth = reinterpret_cast<uint16_t*>(smem);
  uint16_t* utl = uth + kRMax * kStageLd;
  float* ybuf = reinterpret_cast<float*>(utl + kRMax * kStageLd);
  int* ibuf = reinterpret_cast<int*>(ybuf + kIdxBlk);
  // factor phase (aliases the stage): G64 packed lower [r(r+1)/2], diag[kRMax], rhs[kRMax], bpart[2][kRMax]
  double* G64 = reinterpret_cast<double*>(smem);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5, col = lane & 31;
  const int r = a.r, k = a.k;
  const int64_t i = blockIdx.x;
  const int32_t* om = a.omega + i * k;

  f32x16 acc[RT];
#pragma unroll
  for (int t = 0; t < RT; ++t) acc[t] = f32x16{};
  // thread t gathers column ac = t & 127 of the rows of parity t >> 7; b
  // accumulates from the FP32 values in FP64
  const int ac = tid & (kRMax - 1), par = tid >> 7;
  double bacc = 0.0;

  // indices and sampled values are staged in LDS a block at a time; inside a
  // block the basis rows of chunk c+1 are loaded while the matrix cores work
  // on chunk c
  float x[kChunk / 2];
  for (int b0 = 0; b0 < k; b0 += kIdxBlk) {
    const int nb = k - b0 < kIdxBlk ? k - b0 : kIdxBlk;
    __syncthreads();
    for (int t = tid; t < kIdxBlk; t += kBlock) {
      const bool in = t < nb;
      const int64_t row = in ? om[b0 + t] : -1;
      ibuf[t] = (row >= 0 && row < a.v) ? static_cast<int>(row) : -1;  // out-of-range: zero row
      ybuf[t] = in ? y_at(a, i, b0 + t) : 0.0f;
    }
    __syncthreads();
    auto gather = [&](int c0) {
#pragma unroll
      for (int m = 0; m < kChunk / 2; ++m) {
        const int row = ibuf[c0 + par + 2 * m];
        x[m] = (row >= 0 && ac < r) ? a.U[static_cast<int64_t>(row) * r + ac] : 0.0f;
      }
    };
    gather(0);
    for (int c0 = 0; c0 < nb; c0 += kChunk) {
      __syncthreads();  // the previous chunk's MFMA reads of the stage are done
#pragma unroll
      for (int m = 0; m < kChunk / 2; ++m) {
        const int kk = par + 2 * m;
        const uint16_t hi = f2bf(x[m]);
        uth[ac * kStageLd + kk] = hi;
        utl[ac * kStageLd + kk] = f2bf(x[m] - bf2f(hi));
        bacc += static_cast<double>(x[m]) * ybuf[c0 + kk];
      }
      if (c0 + kChunk < nb) gather(c0 + kChunk);
      __syncthreads();
      if (wave < RT) {
#pragma unroll
        for (int s = 0; s < kChunk / 16; ++s) {
          const int ko = 16 * s + 8 * h;
          const u32x4 ah = *reinterpret_cast<const u32x4*>(uth + (wave * 32 + col) * kStageLd + ko);
          const u32x4 al = *reinterpret_cast<const u32x4*>(utl + (wave * 32 + col) * kStageLd + ko);
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const u32x4 bh = *reinterpret_cast<const u32x4*>(uth + (t * 32 + col) * kStageLd + ko);
            const u32x4 bl = *reinterpret_cast<const u32x4*>(utl + (t * 32 + col) * kStageLd + ko);
            acc[t] = mfma_bf16(ah, bh, acc[t]);
            acc[t] = mfma_bf16(ah, bl, acc[t]);
            acc[t] = mfma_bf16(al, bh, acc[t]);
          }
        }
      }
    }
  }
  __syncthreads();
  // G (lower triangle) to LDS in FP64; b reduced over the two row parities
  const int ntri = r * (r + 1) / 2;
  double* diag = G64 + ntri;
  double* dinv = diag + kRMax;
  double* rhs = dinv + kRMax;
  double* bpart = rhs + kRMax;  // [2][kRMax]
  if (wave < RT) {
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = wave * 32 + mfma_row(e, h), cc = t * 32 + col;
        if (row < r && cc <= row) G64[ptri(row, cc)] = static_cast<double>(acc[t][e]);
      }
  }
  bpart[par * kRMax + ac] = bacc;
  __syncthreads();
  if (tid < r) rhs[tid] = bpart[tid] + bpart[kRMax + tid];

  const int failed = lds_cholesky(G64, diag, dinv, r);
  float* Wi = a.W + i * r;
  if (failed) {
    for (int c = tid; c < r; c += kBlock) Wi[c] = 0.0f;
    if (tid == 0) {
      a.info[i] = failed;
      if (a.wnorm2) a.wnorm2[i] = 0.0f;
    }
    if (a.resid)
      for (int q = tid; q < k; q += kBlock) a.resid[i * k + q] = y_at(a, i, q);
    return;
  }
  if (wave == 0) {
    double z0, z1;
    wave_chol_solve(G64, dinv, rhs, r, z0, z1);
    double nrm = 0.0;
    if (lane < r) {
      Wi[lane] = static_cast<float>(z0);
      rhs[lane] = z0;
      nrm += z0 * z0;
    }
    if (lane + 64 < r) {
      Wi[lane + 64] = static_cast<float>(z1);
      rhs[lane + 64] = z1;
      nrm += z1 * z1;
    }
    nrm = wave_sum_d(nrm);
    if (lane == 0) {
      a.info[i] = 0;
      if (a.wnorm2) a.wnorm2[i] = static_cast<float>(nrm);
    }
  }
  if (a.resid) {
    __syncthreads();
    for (int q = tid; q < k; q += kBlock) {
      const int64_t row = om[q];
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      if (row >= 0 && row < a.v) {
        const float* u = a.U + row * r;
        int c = 0;
        for (; c + 4 <= r; c += 4) {
          s0 += static_cast<double>(u[c]) * rhs[c];
          s1 += static_cast<double>(u[c + 1]) * rhs[c + 1];
          s2 += static_cast<double>(u[c + 2]) * rhs[c + 2];
          s3 += static_cast<double>(u[c + 3]) * rhs[c + 3];
        }
        for (; c < r; ++c) s0 += static_cast<double>(u[c]) * rhs[c];
      }
      a.resid[i * k + q] = static_cast<float>(y_at(a, i, q) - ((s0 + s1) + (s2 + s3)));
    }
  }
}

size_t smem_bytes(int r) {
  const size_t stage = 2 * kRMax * kStageLd * sizeof(uint16_t) + kIdxBlk * (sizeof(float) + sizeof(int));
  const size_t factor = (static_cast<size_t>(r) * (r + 1) / 2 + 5 * kRMax) * sizeof(double);
  return stage > factor ? stage : factor;
}

}  // namespace

rpt_status complete_run(const float* U, int64_t v, int r, const int32_t* omega, int k, const float* y,
                        const float* Trows, int64_t ldT, const int32_t* trow, int64_t L, float* W, float* resid,
                        int32_t* info, float* wnorm2, hipStream_t s) {
  if (L == 0) return RPT_OK;
  if (r < 1 || r > kRMax) return RPT_ERR_UNSUPPORTED;
  CompleteArgs a{U, v, r, omega, k, y, Trows, ldT, trow, L, W, resid, info, wnorm2};
  const int RT = (r + 31) / 32;
  void* fn = nullptr;
  switch (RT) {
    case 1: fn = reinterpret_cast<void*>(&complete_kernel<1>); break;
    case 2: fn = reinterpret_cast<void*>(&complete_kernel<2>); break;
    case 3: fn = reinterpret_cast<void*>(&complete_kernel<3>); break;
    default: fn = reinterpret_cast<void*>(&complete_kernel<4>); break;
  }
  const size_t sm = smem_bytes(r);
  static bool attr_set[4] = {false, false, false, false};
  if (!attr_set[RT - 1]) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem_bytes(kRMax)));
    attr_set[RT - 1] = true;
  }
  void* args[] = {&a};
  RPT_STAGE("complete", s);
  hipError_t e = hipLaunchKernel(fn, dim3(static_cast<unsigned>(L)), dim3(kBlock), args, sm, s);
  if (e != hipSuccess) {
    set_hip_error(e);
    return RPT_ERR_HIP;
  }
  return RPT_OK;
}

}  // namespace rpt
