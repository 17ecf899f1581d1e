// Small dense FP64 linear algebra on one workgroup (kBlock threads) with the
// matrix in LDS: Cholesky of a packed lower triangle, triangular solves, and
// the inverse of the Cholesky factor.  Used by Complete (one r x r normal
// matrix per column) and by the Cholesky-QR re-orthonormalisation.
#pragma once

#include "rpt_internal.h"

namespace rpt {

__device__ __forceinline__ int ptri(int i, int c) { return (i * (i + 1)) / 2 + c; }

__device__ __forceinline__ double readlane_d(double x, int l) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xFFFFFFFFull), l));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), l));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// sum_{k in [kb, ke)} a[k] b[k] with four independent FP64 accumulators so the
// LDS loads pipeline
__device__ __forceinline__ double dot4(const double* a, const double* b, int kb, int ke) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = kb;
  for (; k + 4 <= ke; k += 4) {
    s0 = fma(a[k], b[k], s0);
    s1 = fma(a[k + 1], b[k + 1], s1);
    s2 = fma(a[k + 2], b[k + 2], s2);
    s3 = fma(a[k + 3], b[k + 3], s3);
  }
  for (; k < ke; ++k) s0 = fma(a[k], b[k], s0);
  return (s0 + s1) + (s2 + s3);
}

// In-place Cholesky G = L L^T of the packed lower triangle G[ptri(i, c)],
// c <= i < r, in the left-looking (dot-product) order: for column j every row
// i >= j forms G[i][j] - sum_{k<j} L[i][k] L[j][k] from rows that are final,
// so the inner loop only reads LDS (row i is contiguous, row j is a broadcast)
// and pipelines.  Two threads share a row (each takes one contiguous half of
// k), combined with one shuffle.  On success G holds L (diagonal included),
// diag[j] = L_jj and dinv[j] = 1 / L_jj; returns 0.  A pivot that is not
// positive returns j + 1 (same value in every thread).
__device__ inline int lds_cholesky(double* G, double* diag, double* dinv, int r) {
  __shared__ int fail;
  const int tid = threadIdx.x;
  const int row = tid >> 1, half = tid & 1;
  if (tid == 0) fail = 0;
  for (int j = 0; j < r; ++j) {
    __syncthreads();
    double s = 0.0;
    const bool active = row >= j && row < r;
    if (active) {
      const int mid = j >> 1;
      s = dot4(G + ptri(row, 0), G + ptri(j, 0), half ? mid : 0, half ? j : mid);
    }
    s += __shfl_xor(s, 1, 64);
    if (active && half == 0) {
      const double g = G[ptri(row, j)] - s;
      if (row == j) {
        if (g > 0.0) {
          const double d = sqrt(g);
          diag[j] = d;
          dinv[j] = 1.0 / d;
          G[ptri(j, j)] = d;
        } else {
          fail = j + 1;
        }
      } else {
        G[ptri(row, j)] = g;  // scaled below once the pivot is known
      }
    }
    __syncthreads();
    if (fail) return fail;
    if (active && half == 0 && row > j) G[ptri(row, j)] *= dinv[j];
  }
  __syncthreads();
  return 0;
}

// Solve L L^T w = b in one wave (wave 0 calls it): lane owns rows lane and
// lane + 64 (r <= 128); the pivot broadcast is a scalar readlane.
__device__ inline void wave_chol_solve(const double* G, const double* dinv, const double* rhs, int r, double& z0,
                                       double& z1) {
  const int lane = threadIdx.x & 63;
  z0 = lane < r ? rhs[lane] : 0.0;
  z1 = lane + 64 < r ? rhs[lane + 64] : 0.0;
  for (int j = 0; j < r; ++j) {  // L z = b
    const double zj = readlane_d(j < 64 ? z0 : z1, j & 63) * dinv[j];
    if (lane == (j & 63)) {
      if (j < 64) z0 = zj; else z1 = zj;
    }
    if (lane > j && lane < r) z0 -= G[ptri(lane, j)] * zj;
    if (lane + 64 > j && lane + 64 < r) z1 -= G[ptri(lane + 64, j)] * zj;
  }
  for (int j = r - 1; j >= 0; --j) {  // L^T w = z
    const double wj = readlane_d(j < 64 ? z0 : z1, j & 63) * dinv[j];
    if (lane == (j & 63)) {
      if (j < 64) z0 = wj; else z1 = wj;
    }
    if (lane < j) z0 -= G[ptri(j, lane)] * wj;
    if (lane + 64 < j) z1 -= G[ptri(j, lane + 64)] * wj;
  }
}

// Linv = L^{-1} (lower), row by row: Linv[i][c] = (delta_ic - sum_{j<i}
// L[i][j] Linv[j][c]) / L_ii.  Thread c owns column c (c < r <= kBlock); all
// threads walk j in lockstep (Linv[j][c] = 0 for j < c) so L[i][j] is a
// broadcast read.  Linv is FP32 in LDS with leading dimension ld; sums FP64.
__device__ inline void lds_tri_inverse(const double* G, const double* dinv, int r, float* Li, int ld) {
  const int c = threadIdx.x;
  for (int i = 0; i < r; ++i) {
    if (c < r) {
      const double* gi = G + ptri(i, 0);
      double s0 = (i == c) ? 1.0 : 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int j = 0;
      for (; j + 4 <= i; j += 4) {
        s0 -= gi[j] * static_cast<double>(Li[j * ld + c]);
        s1 -= gi[j + 1] * static_cast<double>(Li[(j + 1) * ld + c]);
        s2 -= gi[j + 2] * static_cast<double>(Li[(j + 2) * ld + c]);
        s3 -= gi[j + 3] * static_cast<double>(Li[(j + 3) * ld + c]);
      }
      for (; j < i; ++j) s0 -= gi[j] * static_cast<double>(Li[j * ld + c]);
      Li[i * ld + c] = (c <= i) ? static_cast<float>(((s0 + s1) + (s2 + s3)) * dinv[i]) : 0.0f;
    }
    __syncthreads();
  }
}

}  // namespace rpt
