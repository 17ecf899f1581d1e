// Small dense FP64 linear algebra on one workgroup (kBlock threads) with the
// matrix in LDS: Cholesky of a packed lower triangle, triangular solves, and
// the inverse of the Cholesky factor.  Used by Complete (one r x r normal
// matrix per column) and by the Cholesky-QR re-orthonormalisation.
#pragma once

#include "rpt_internal.h"

namespace rpt {

__device__ __forceinline__ int ptri(int i, int c) { return (i * (i + 1)) / 2 + c; }

// In-place right-looking Cholesky G = L L^T of the packed lower triangle
// G[ptri(i, c)], c <= i < r.  On success the strictly lower part holds L and
// diag[j] = L_jj (G's diagonal is left unscaled); returns 0.  A pivot that is
// not positive returns j + 1 (every thread returns the same value).
// Thread t updates row t/2, columns of parity t%2, so no integer division is
// needed and each column step costs two barriers.
__device__ inline int lds_cholesky(double* G, double* diag, int r) {
  const int tid = threadIdx.x;
  const int row = tid >> 1, half = tid & 1;
  for (int j = 0; j < r; ++j) {
    __syncthreads();
    const double piv = G[ptri(j, j)];
    if (!(piv > 0.0)) return j + 1;
    const double dinv = 1.0 / sqrt(piv);
    for (int ii = j + 1 + tid; ii < r; ii += kBlock) G[ptri(ii, j)] *= dinv;
    if (tid == 0) diag[j] = sqrt(piv);
    __syncthreads();
    if (row > j && row < r) {
      const double lij = G[ptri(row, j)];
      double* grow = G + ptri(row, 0);
      for (int cc = j + 1 + half; cc <= row; cc += 2) grow[cc] -= lij * G[ptri(cc, j)];
    }
  }
  __syncthreads();
  return 0;
}

// Solve L L^T w = b in one wave (wave 0 calls it): lane owns rows lane and
// lane + 64 (r <= 128).  b in rhs[], result returned in z0/z1 registers.
__device__ inline void wave_chol_solve(const double* G, const double* diag, const double* rhs, int r, double& z0,
                                       double& z1) {
  const int lane = threadIdx.x & 63;
  z0 = lane < r ? rhs[lane] : 0.0;
  z1 = lane + 64 < r ? rhs[lane + 64] : 0.0;
  for (int j = 0; j < r; ++j) {  // L z = b
    const double own = (j < 64) ? z0 : z1;
    const double zj = __shfl(own, j & 63, 64) / diag[j];
    if (lane == (j & 63)) {
      if (j < 64) z0 = zj; else z1 = zj;
    }
    if (lane > j && lane < r) z0 -= G[ptri(lane, j)] * zj;
    if (lane + 64 > j && lane + 64 < r) z1 -= G[ptri(lane + 64, j)] * zj;
  }
  for (int j = r - 1; j >= 0; --j) {  // L^T w = z
    const double own = (j < 64) ? z0 : z1;
    const double wj = __shfl(own, j & 63, 64) / diag[j];
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
__device__ inline void lds_tri_inverse(const double* G, const double* diag, int r, float* Li, int ld) {
  const int c = threadIdx.x;
  for (int i = 0; i < r; ++i) {
    if (c < r) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int j = 0; j < i; ++j) s -= G[ptri(i, j)] * static_cast<double>(Li[j * ld + c]);
      Li[i * ld + c] = (c <= i) ? static_cast<float>(s / diag[i]) : 0.0f;
    }
    __syncthreads();
  }
}

}  // namespace rpt
