// Masked completion loss of Eq. 1 and its gradient, over CSR sampled sets:
//     f  = 1/2 sum_b sum_{k in O_b} e_bk^2,   e_bk = t_bk - U[k, :] W[:, b]
//     dW[:, b] = - sum_{k in O_b} U[k, :]^T e_bk
//     dU[k, :] = - sum_{b : k in O_b} e_bk W[:, b]^T
// One workgroup per batch column; the column of W is staged in LDS.  The loss
// is reduced in FP64.  dU is zero-filled and then scattered with FP32 atomic
// adds (different columns may sample the same voxel).
#include "rpt_internal.h"

namespace rpt {

namespace {

constexpr int kRLoss = 1024;  // largest rank handled (W column in LDS)

__global__ __launch_bounds__(kBlock) void loss_fwd_kernel(const float* __restrict__ U, int64_t v, int r,
                                                         const float* __restrict__ W, int B,
                                                         const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const float* __restrict__ t, double* loss,
                                                         float* __restrict__ resid) {
  __shared__ float w[kRLoss];
  __shared__ double red[kBlock / 64];
  const int b = blockIdx.x;
  for (int c = threadIdx.x; c < r; c += kBlock) w[c] = W[static_cast<int64_t>(c) * B + b];
  __syncthreads();
  double acc = 0.0;
  for (int64_t q = ptr[b] + threadIdx.x; q < ptr[b + 1]; q += kBlock) {
    const int64_t row = idx[q];
    float s = 0.0f;
    if (row >= 0 && row < v) {  // out-of-range index: U row taken as zero
      const float* u = U + row * r;
      for (int c = 0; c < r; ++c) s = fmaf(u[c], w[c], s);
    }
    const float e = t[q] - s;
    if (resid) resid[q] = e;
    acc += static_cast<double>(e) * e;
  }
  acc = wave_sum_d(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, 0.5 * (red[0] + red[1] + red[2] + red[3]));
}

__global__ void zero_loss_kernel(double* loss) { *loss = 0.0; }

__global__ __launch_bounds__(kBlock) void fill_zero_kernel(float* __restrict__ p, int64_t n) {
  for (int64_t t = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; t < n;
       t += static_cast<int64_t>(gridDim.x) * kBlock)
    p[t] = 0.0f;
}

__global__ __launch_bounds__(kBlock) void loss_bwd_kernel(const float* __restrict__ U, int64_t v, int r,
                                                         const float* __restrict__ W, int B,
                                                         const int64_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ idx,
                                                         const float* __restrict__ e, float* __restrict__ dU,
                                                         float* __restrict__ dW, const double* grad_scale) {
  const int b = blockIdx.x;
  const int64_t q0 = ptr[b], q1 = ptr[b + 1];
  const float gs = grad_scale ? static_cast<float>(*grad_scale) : 1.0f;
  for (int c = threadIdx.x; c < r; c += kBlock) {
    const float wc = W[static_cast<int64_t>(c) * B + b] * gs;
    float g = 0.0f;
    for (int64_t q = q0; q < q1; ++q) {
      const int64_t vox = idx[q];
      if (vox < 0 || vox >= v) continue;
      const int64_t row = vox * r;
      const float eq = e[q];
      g = fmaf(U[row + c], eq, g);
      atomicAdd(dU + row + c, -eq * wc);
    }
    dW[static_cast<int64_t>(c) * B + b] = -g * gs;
  }
}

}  // namespace

rpt_status loss_fwd_launch(const float* U, int64_t v, int r, const float* W, int B, const int64_t* ptr, const int32_t* idx,
                           const float* t, double* loss, float* resid, hipStream_t s) {
  if (r > kRLoss) return RPT_ERR_UNSUPPORTED;
  hipLaunchKernelGGL(zero_loss_kernel, dim3(1), dim3(1), 0, s, loss);
  RPT_CHECK_LAUNCH();
  if (B == 0) return RPT_OK;
  RPT_STAGE("masked_loss_fwd", s);
  hipLaunchKernelGGL(loss_fwd_kernel, dim3(B), dim3(kBlock), 0, s, U, v, r, W, B, ptr, idx, t, loss, resid);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status loss_bwd_launch(const float* U, int64_t v, int r, const float* W, int B, const int64_t* ptr,
                           const int32_t* idx, const float* e, float* dU, float* dW, const double* grad_scale,
                           hipStream_t s) {
  if (r > kRLoss) return RPT_ERR_UNSUPPORTED;
  const int64_t n = v * r;
  int64_t blocks = ceil_div(n, kBlock);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, s, dU, n);
  RPT_CHECK_LAUNCH();
  if (B == 0) return RPT_OK;
  RPT_STAGE("masked_loss_bwd", s);
  hipLaunchKernelGGL(loss_bwd_kernel, dim3(B), dim3(kBlock), 0, s, U, v, r, W, B, ptr, idx, e, dU, dW, grad_scale);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace rpt
