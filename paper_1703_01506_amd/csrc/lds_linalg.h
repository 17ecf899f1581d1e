// Small dense FP64 linear algebra on one workgroup (kBlock threads) with the
// matrix in LDS: Cholesky of a packed lower triangle, triangular solves, and
// the inverse of the Cholesky factor.  Used by Complete (one r x r normal
// matrix per column) and by the Cholesky-QR re-orthonormalisation.
#pragma once

#include "rpt_internal.h"

namespace rpt {

__device__ __forceinline__ int ptri(int i, int c) { return (i * (i + 1)) / 2 + c; }

// 1 / sqrt(x) for x > 0: the hardware estimate (relative error about 2^-23)
// and one Newton step (about 2^-45); the factorisations below need no
// correct rounding
__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

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
__device__ __forceinline__ int lds_cholesky(double* G, double* diag, double* dinv, int r) {
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
__device__ __forceinline__ void wave_chol_solve(const double* G, const double* dinv, const double* rhs, int r, double& z0,
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
__device__ __forceinline__ void lds_tri_inverse(const double* G, const double* dinv, int r, float* Li, int ld) {
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

// ---------------------------------------------------------------------------
// Blocked variants (block width kCb).  One wave factors each panel of kCb
// columns with the panel in registers (a lane owns up to three rows; pivots
// and the kCb x kCb diagonal block are broadcast by readlane), then every
// thread applies the panel to the trailing matrix in 4 x 4 register tiles.
// Two barriers per block of kCb columns.

constexpr int kCb = 16;
constexpr int kPanelLd = 132;  // > 129 rows below a diagonal block, multiple of 4

// One panel step on wave 0: rows [c0, nrows) x columns [c0, c0 + M) of G;
// lane l owns rows c0 + l + 64 s, s < NS (nrows - c0 <= 64 NS).  Rows past
// nrows and entries above the diagonal are loaded from clamped addresses
// and carried along unmasked: they are never read by a kept entry and never
// stored.  G must be followed by at least kCb doubles of readable LDS.
template <int M, int NS>
__device__ __forceinline__ int chol_panel(double* G, double* dinv, double* P, int c0, int m, int nrows, int lane_in,
                                          int pld) {
  // the lane index passes through an opaque register move so that the
  // lane-dependent predicates below are formed inside the caller's block loop
  // instead of being hoisted out of it (where they would stay live and spill)
  int lane;
  asm volatile("v_mov_b32 %0, %1" : "=v"(lane) : "v"(lane_in));
  const int mm = M ? M : m;
  double d[3][kCb];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int row = min(c0 + 64 * s + lane, nrows - 1);
    const double* gr = G + ptri(row, c0);  // entries c0.. of a row are contiguous
#pragma unroll
    for (int j = 0; j < kCb; ++j) d[s][j] = gr[j];
  }
  const bool two = NS > 1 && nrows - c0 > 64;  // second row slot in use
  const bool three = NS > 2 && nrows - c0 > 128;
  int bad = 0;
#pragma unroll
  for (int j = 0; j < kCb; ++j) {
    if (j < mm) {
      double piv = readlane_d(d[0][j], j);
      if (!(piv > 0.0)) {
        if (!bad) bad = c0 + j + 1;
        piv = 1.0;
      }
      const double inv = rsqrt_d(piv);
      d[0][j] = (lane == j) ? piv * inv : d[0][j] * inv;
      if (two) d[1][j] *= inv;
      if (three) d[2][j] *= inv;
      if (lane == 0) dinv[c0 + j] = inv;
      // column j of the diagonal block is broadcast by readlane; entries
      // above the diagonal are updated too (never read, never stored)
#pragma unroll
      for (int q = j + 1; q < kCb; ++q) {
        if (q < mm) {
          const double lq = readlane_d(d[0][j], q);  // L[c0 + q][c0 + j]
          d[0][q] = fma(-d[0][j], lq, d[0][q]);
          if (two) d[1][q] = fma(-d[1][j], lq, d[1][q]);
          if (three) d[2][q] = fma(-d[2][j], lq, d[2][q]);
        }
      }
      // finish this pivot's updates before the next pivot starts: deferring
      // them keeps every broadcast value live and exhausts the registers
#pragma unroll
      for (int q = j + 1; q < kCb; ++q)
#pragma unroll
        for (int s = 0; s < NS; ++s) asm volatile("" : "+v"(d[s][q]));
    }
  }
  const int b0 = c0 + m;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int row = c0 + 64 * s + lane;
    if (row < nrows) {
      double* gr = G + ptri(row, c0);
      double* pr = P + (row >= b0 ? row - b0 : 0);
#pragma unroll
      for (int j = 0; j < kCb; ++j) {
        if (j < mm && (s > 0 || j <= lane)) gr[j] = d[s][j];
        if (j < mm && row >= b0) pr[j * pld] = d[s][j];
      }
    }
  }
  return bad;
}

// Trailing update G[i][j] -= sum_q P[q][i - b0] P[q][j - b0], b0 <= j <= i,
// j < r, i < nrows, in 4 x 4 tiles.
template <int M>
__device__ __forceinline__ void chol_trailing(double* G, const double* P, int b0, int m, int r, int nrows, int pld) {
  const int nr = nrows - b0, nc = r - b0;
  if (nc <= 0) return;
  const int TR = (nr + 3) >> 2, TC = (nc + 3) >> 2;
  for (int t = threadIdx.x; t < TR * TC; t += blockDim.x) {
    const int ti = t / TC, tj = t - ti * TC;
    if (tj > ti) continue;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int w = 0; w < 4; ++w) acc[u][w] = 0.0;
    // partial unroll: full unrolling hoists all 8 x kCb loads and spills
#pragma unroll 4
    for (int q = 0; q < (M ? M : m); ++q) {
      {
        const double* pq = P + q * pld;
        double xi[4], xj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xi[u] = pq[4 * ti + u];
          xj[u] = pq[4 * tj + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int w = 0; w < 4; ++w) acc[u][w] = fma(xi[u], xj[w], acc[u][w]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = b0 + 4 * ti + u;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const int col = b0 + 4 * tj + w;
        if (row < nrows && col < r && col <= row) G[ptri(row, col)] -= acc[u][w];
      }
    }
  }
}

// The same trailing update for a full panel (M = kCb) on the FP64 matrix
// cores: 16 x 16 tiles of the lower part (and the rows past r), one wave per
// tile, K = kCb in four 16x16x4 products.  Lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and receives D[l / 16 + 4 e][l % 16] in element e.
// Tile loads read up to 15 entries past the last row of P (into readable LDS;
// they feed only discarded tile rows and columns).
typedef double dbl4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void chol_trailing_mfma(double* G, const double* P, int b0, int r, int nrows, int pld) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int ng = nrows - b0, nc = r - b0;
  if (nc <= 0) return;
  const int TC = (nc + 15) >> 4, TR = (ng + 15) >> 4;
  const int ntri = TC * (TC + 1) / 2;
  const int total = ntri + (TR > TC ? TR - TC : 0) * TC;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < total; t += nw) {
    int ti, tj;
    if (t < ntri) {
      ti = 0;
      while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
      tj = t - ti * (ti + 1) / 2;
    } else {
      const int u = t - ntri;
      ti = TC + u / TC;
      tj = u - (u / TC) * TC;
    }
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < kCb / 4; ++s4) {
      const double* pk = P + (4 * s4 + lk) * pld;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pk[16 * ti + li], pk[16 * tj + li], acc, 0, 0, 0);
    }
    const int col = 16 * tj + li;
    double g[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * ti + lk + 4 * e;
      g[e] = (row < ng && col < nc && col <= row) ? G[ptri(b0 + row, b0 + col)] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * ti + lk + 4 * e;
      if (row < ng && col < nc && col <= row) G[ptri(b0 + row, b0 + col)] = g[e] - acc[e];
    }
  }
}

// Cholesky of the leading r x r block of the packed lower trapezoid G (rows
// [0, nrows), r <= nrows <= 64 NS; entry (i, c) at ptri(i, c),
// c <= min(i, r - 1)).  On success the leading block holds L (diagonal
// included), dinv[j] = 1 / L_jj, and every row i >= r holds x_i with
// L x_i = a_i (for an appended row b^T: z = L^{-1} b).  P is LDS scratch of
// kCb rows of pld doubles, pld >= nrows - kCb (the rows below the first
// diagonal block); the trailing tiles read up to 15 entries past the last row
// of P, which must be readable LDS and feed only discarded tile rows.  Returns 0,
// or j + 1 for the first pivot j that is not positive (same value in every
// thread; later blocks are not factored).
template <int NS>
__device__ __forceinline__ int lds_cholesky_blocked(double* G, double* dinv, double* P, int r, int nrows,
                                                    int pld = kPanelLd) {
  __shared__ int fail;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) fail = 0;
  // full blocks, then the ragged last block (separate loops keep the two
  // unrolled variants out of each other's register live ranges)
  int c0 = 0;
#pragma clang loop unroll(disable)
  for (; c0 + kCb <= r; c0 += kCb) {
    __syncthreads();  // trailing update of the previous block is complete
    if (wave == 0) {
      // c0 made opaque: strength reduction would otherwise carry one address
      // per unrolled panel entry across the loop
      const int cb = __builtin_amdgcn_readfirstlane(c0);
      const int bad = chol_panel<kCb, NS>(G, dinv, P, cb, kCb, nrows, lane, pld);
      if (lane == 0 && bad) fail = bad;
    }
    __syncthreads();
    if (fail) return fail;
    chol_trailing_mfma(G, P, c0 + kCb, r, nrows, pld);
  }
  if (c0 < r) {
    const int m = r - c0;
    __syncthreads();
    if (wave == 0) {
      const int bad = chol_panel<0, NS>(G, dinv, P, c0, m, nrows, lane, pld);
      if (lane == 0 && bad) fail = bad;
    }
    __syncthreads();
    if (fail) return fail;
    chol_trailing<0>(G, P, c0 + m, m, r, nrows, pld);
  }
  __syncthreads();
  return 0;
}

// Solve L^T w = z in place (w holds z on entry) with L from
// lds_cholesky_blocked: blocks from the last, each solved by one wave
// (readlane broadcast of the finished entry), then its contribution removed
// from all earlier entries by every thread.
__device__ __forceinline__ void lds_chol_backsolve(const double* G, const double* dinv, double* w, int r) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  for (int c0 = ((r - 1) / kCb) * kCb; c0 >= 0; c0 -= kCb) {
    const int m = min(kCb, r - c0);
    __syncthreads();
    if (wave == 0) {
      // the block's column entries of this lane's row and the pivots, loaded
      // before the dependent chain starts
      double lc[kCb], di[kCb];
#pragma unroll
      for (int c = 0; c < kCb; ++c) {
        const bool ok = c < m && lane < c;
        lc[c] = ok ? G[ptri(c0 + c, c0 + lane)] : 0.0;
        di[c] = c < m ? dinv[c0 + c] : 0.0;
      }
      double val = lane < m ? w[c0 + lane] : 0.0;
#pragma unroll
      for (int c = kCb - 1; c >= 0; --c) {
        if (c < m) {
          const double wc = readlane_d(val, c) * di[c];
          val = (lane == c) ? wc : (lane < c ? fma(-lc[c], wc, val) : val);
        }
      }
      if (lane < m) w[c0 + lane] = val;
    }
    __syncthreads();
    for (int j = tid; j < c0; j += nt) {
      // unrolled with two accumulators: the loads do not wait on the sums
      double s0 = w[j], s1 = 0.0;
#pragma unroll
      for (int c = 0; c < kCb; ++c) {
        if (c < m) {
          const double g = G[ptri(c0 + c, 0) + j];
          if (c & 1) s1 = fma(-g, w[c0 + c], s1);
          else s0 = fma(-g, w[c0 + c], s0);
        }
      }
      w[j] = s0 + s1;
    }
  }
  __syncthreads();
}

// X = L^{-1} (lower) for the L left by lds_cholesky_blocked, by blocks of
// kCb rows: every diagonal block is inverted at once (one thread per column
// of a block, forward substitution in FP64 registers), then block row p is
//   S = L[p, 0:p] X[0:p, 0:p],   X[p, 0:p] = -X_pp S,
// two parallel products per block row.  X is FP32 in LDS with leading
// dimension ld (columns up to kCb * ceil(r / kCb) written, zeros above the
// diagonal); S uses the kCb * kPanelLd doubles at P.  FP64 sums throughout.
__device__ __forceinline__ void lds_tri_inverse_blocked(const double* G, const double* dinv, int r, float* X,
                                                        int ld, double* P) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int nb = (r + kCb - 1) / kCb;
  const int rp = nb * kCb;
  for (int t = tid; t < rp * ld; t += nt) X[t] = 0.0f;
  __syncthreads();
  // diagonal blocks: thread (p, c) solves L_pp x = e_c
  if (tid < nb * kCb) {
    const int p = tid / kCb, c = tid - p * kCb, c0 = p * kCb;
    const int m = min(kCb, r - c0);
    if (c < m) {
      double x[kCb];
#pragma unroll
      for (int i = 0; i < kCb; ++i) {
        if (i < m) {
          double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
          for (int j = 0; j < i; ++j) s = fma(-G[ptri(c0 + i, c0 + j)], x[j], s);
          x[i] = (i >= c) ? s * dinv[c0 + i] : 0.0;
          X[(c0 + i) * ld + c0 + c] = static_cast<float>(x[i]);
        }
      }
    }
  }
  for (int p = 1; p < nb; ++p) {
    const int c0 = p * kCb, m = min(kCb, r - c0);
    __syncthreads();  // block rows < p of X are final
    // S[a][col] = sum_{j = col}^{c0 - 1} L[c0 + a][j] X[j][col],  a < m, col < c0
    for (int t = tid; t < m * c0; t += nt) {
      const int a = t / c0, col = t - a * c0;
      const double* lr = G + ptri(c0 + a, 0);
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int j = col;
      // four independent sums keep several LDS loads in flight
#pragma unroll 2
      for (; j + 3 < c0; j += 4) {
        s0 = fma(lr[j], static_cast<double>(X[j * ld + col]), s0);
        s1 = fma(lr[j + 1], static_cast<double>(X[(j + 1) * ld + col]), s1);
        s2 = fma(lr[j + 2], static_cast<double>(X[(j + 2) * ld + col]), s2);
        s3 = fma(lr[j + 3], static_cast<double>(X[(j + 3) * ld + col]), s3);
      }
      for (; j < c0; ++j) s0 = fma(lr[j], static_cast<double>(X[j * ld + col]), s0);
      P[a * kPanelLd + col] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    // X[c0 + a][col] = -sum_{b <= a} X_pp[a][b] S[b][col]
    for (int t = tid; t < m * c0; t += nt) {
      const int a = t / c0, col = t - a * c0;
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int b = 0; b < kCb; ++b) {
        if (b <= a) {
          const double t2 = static_cast<double>(X[(c0 + a) * ld + c0 + b]) * P[b * kPanelLd + col];
          if (b & 1) s1 += t2;
          else s0 += t2;
        }
      }
      X[(c0 + a) * ld + col] = static_cast<float>(-(s0 + s1));
    }
  }
  __syncthreads();
}

}  // namespace rpt
