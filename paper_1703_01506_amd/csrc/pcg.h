// Conjugate gradients on an r x r SPD matrix held by one workgroup of four
// waves (r <= 128), shared by the tracking pass and the recovery solve.  The
// matrix is stored whole in LDS (16 RB rows of g_hld(RB) floats, rows 16-byte
// aligned) and held in FP64 registers during the solve: lane (rq, cb) of
// wave w keeps rows 32 w + 8 rq .. + 7 and columns 8 cb .. + 7, so H p is
// eight FMAs per row and a reduce-scatter over the 16 lanes of a DPP row.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "rpt_internal.h"

namespace rpt {
namespace {

constexpr int kGT = 256;           // threads of a tracking workgroup: one wave per SIMD
constexpr int kGWaves = kGT / 64;  // 4
constexpr int kGR = 128;           // rank bound
constexpr int kCgMaxIt = 300;      // conjugate-gradient iteration cap
constexpr double kCgTol = 1e-6;    // stop when (r, M r) <= kCgTol^2 (b, M b) (H is exact to about 1e-6)

// column blocks of 16 covering columns 0..r; H holds all 16 RB rows and
// columns of the symmetric matrix (row length 16 RB + 4 words)
__host__ __device__ constexpr int g_rb(int r) { return (r + 1 + 15) / 16; }
__host__ __device__ constexpr int g_hld(int rb) { return 16 * rb + 4; }  // rows 16-byte aligned
// DPP lane moves within rows of 16 lanes: quad_perm [1, 0, 3, 2] (0xB1),
// quad_perm [2, 3, 0, 1] (0x4E), row_half_mirror (0x141), row_mirror
// (0x140); row_bcast:15 (0x142) and row_bcast:31 (0x143) into the upper
// rows for whole-wave sums
// With every row enabled each lane reads a lane of its own row, so the
// destination's old value is never kept and needs no zeroing first; with a
// row mask the disabled rows keep 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_mov_i(int x) {
  if constexpr (ROWMASK == 0xF)
    return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
  else
    return __builtin_amdgcn_update_dpp(0, x, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_mov_d(double s) {
  const long long b = __double_as_longlong(s);
  const int lo = dpp_mov_i<CTRL, ROWMASK>(static_cast<int>(b & 0xFFFFFFFFll));
  const int hi = dpp_mov_i<CTRL, ROWMASK>(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov_f(float s) {
  return __int_as_float(dpp_mov_i<CTRL, 0xF>(__float_as_int(s)));
}
// sum over the 64 lanes of one wave; the total ends in lane 63 and is read
// back as a scalar, so every lane gets it
__device__ __forceinline__ double wave_sum_dpp(double s) {
  s += dpp_mov_d<0xB1, 0xF>(s);
  s += dpp_mov_d<0x4E, 0xF>(s);   // quad sums
  s += dpp_mov_d<0x141, 0xF>(s);  // sums of eight
  s += dpp_mov_d<0x140, 0xF>(s);  // row sums
  s += dpp_mov_d<0x142, 0xA>(s);  // rows 1 and 3 add rows 0 and 2
  s += dpp_mov_d<0x143, 0xC>(s);  // rows 2 and 3 add row 1: lane 63 holds the total
  const long long b = __double_as_longlong(s);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xFFFFFFFFll), 63));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), 63));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
// the same sum, left in lane 63 only (no broadcast back to the wave)
__device__ __forceinline__ double wave_sum_l63(double s) {
  s += dpp_mov_d<0xB1, 0xF>(s);
  s += dpp_mov_d<0x4E, 0xF>(s);
  s += dpp_mov_d<0x141, 0xF>(s);
  s += dpp_mov_d<0x140, 0xF>(s);
  s += dpp_mov_d<0x142, 0xA>(s);
  s += dpp_mov_d<0x143, 0xC>(s);
  return s;
}
// sum over the 16 lanes of a DPP row into every one of them
__device__ __forceinline__ float row16_sum_f(float x) {
  x += dpp_mov_f<0xB1>(x);
  x += dpp_mov_f<0x4E>(x);
  x += dpp_mov_f<0x141>(x);
  x += dpp_mov_f<0x140>(x);
  return x;
}
// Eight values per lane, summed over the 16 lanes of a DPP row; lane c of
// the row ends with the sum of value row8_sel(c) (two lanes per value, c
// and c ^ 1).  Each exchange sends the half the partner keeps: row_mirror
// pairs c with 15 - c (lanes from 8 on keep values 4..7), row_half_mirror
// pairs c with 7 - c in each half (c % 8 >= 4 keeps the upper two), the
// quad exchange c ^ 2 halves them again (c % 4 >= 2 keeps the upper one),
// c ^ 1 completes the sum.
__device__ __forceinline__ int row8_sel(int c) { return ((c >> 3) << 2) | (((c >> 2) & 1) << 1) | ((c >> 1) & 1); }
__device__ __forceinline__ double row16_reduce_scatter8(const double (&v)[8], int c) {
  const bool h8 = c >= 8, h4 = (c & 4) != 0, h2 = (c & 2) != 0;
  double k4[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const double keep = h8 ? v[4 + m] : v[m], send = h8 ? v[m] : v[4 + m];
    k4[m] = keep + dpp_mov_d<0x140, 0xF>(send);
  }
  double k2[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const double keep = h4 ? k4[2 + m] : k4[m], send = h4 ? k4[m] : k4[2 + m];
    k2[m] = keep + dpp_mov_d<0x141, 0xF>(send);
  }
  double k1 = h2 ? k2[1] : k2[0];
  const double s1 = h2 ? k2[0] : k2[1];
  k1 += dpp_mov_d<0x4E, 0xF>(s1);
  k1 += dpp_mov_d<0xB1, 0xF>(k1);
  return k1;
}

// The same reduce-scatter without lane-dependent selects, for operands
// stored in a lane-dependent order: v[m] holds value (c >> 1) ^ kRowX[m].
// Then every exchange keeps the low half and sends the high half: the
// mirror partner 15 - c holds value (c >> 1) ^ 7 ^ kRowX[m] in v[m], which is
// what this lane holds in v[4 + m] (kRowX[4 + m] = 7 ^ kRowX[m]); the
// half-mirror partner c ^ 7 likewise (kRowX[2 + m] = 3 ^ kRowX[m]), and the
// partner c ^ 2 holds in v[0] this lane's v[1].  Lane c ends with the sum of
// value c >> 1 (= row8_sel(c)).
__device__ constexpr int kRowX[8] = {0, 1, 3, 2, 7, 6, 4, 5};
__device__ __forceinline__ double row16_reduce_scatter8_px(const double (&v)[8]) {
  double k4[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) k4[m] = v[m] + dpp_mov_d<0x140, 0xF>(v[4 + m]);
  double k2[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) k2[m] = k4[m] + dpp_mov_d<0x141, 0xF>(k4[2 + m]);
  double k1 = k2[0] + dpp_mov_d<0x4E, 0xF>(k2[1]);
  k1 += dpp_mov_d<0xB1, 0xF>(k1);
  return k1;
}

// H z = b (b: row r of H) by Jacobi-preconditioned conjugate gradients in
// FP64, in the pipelined form (Ghysels & Vanroose 2014) whose only exchange
// per iteration is one barrier: the inner products (r, u) and (w, u) (u =
// M r, M the inverse diagonal) and the vector m = M w that the next product
// H m needs are written together.  The iteration stops when (r, M r) has
// fallen by kCgTol^2.  H is held in registers in the matrix layout (lane (rq, cb) of
// wave w: rows rbase .. rbase + 7, in the lane-dependent order of
// row16_reduce_scatter8_px, columns 8 cb .. 8 cb + 7; after the
// reduce-scatter the lane holds row myrow, owned by the even lane of its
// pair, and both lanes of the pair keep identical copies of every vector
// entry, so inner products add half of every lane's term).  The right-hand side is row r of H, or with WARM the vector bvec
// (FP64, in LDS) and the iteration starts from the z in sv.zv.  On return sv.zv and
// sv.zf hold z (zero from r on); the result is 0, 1 (a non-positive diagonal
// or curvature) or 2 (iteration cap).  Ends with a barrier.
// SV: the LDS vectors of the caller (zv, zf, mv[2], cgr, red, badf fields).
template <int HLD, bool WARM, class SV>
__device__ __forceinline__ int pcg_solve(const float* H, int r, SV& sv, int lane, int wave, int rbase, int cb,
                                         int myrow, bool owner, bool rowok, const double* bvec) {
  constexpr int hld = HLD;
  // H is stored whole with 16-byte aligned rows: two 16-byte loads per row
  // (row and column offsets clamped into the stored block, the entries
  // outside the r x r matrix then zeroed)
  double h[8][8];
  const int c0 = min(8 * cb, (hld & ~7) - 8);
#pragma unroll
  for (int ii = 0; ii < 8; ++ii) {
    const int rr = rbase + ((cb >> 1) ^ kRowX[ii]);
    const float* hrow = H + min(rr, r - 1) * hld + c0;
    const f32x4 a0 = *reinterpret_cast<const f32x4*>(hrow);
    const f32x4 a1 = *reinterpret_cast<const f32x4*>(hrow + 4);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int cc = 8 * cb + j;
      h[ii][j] = (rr < r && cc < r) ? static_cast<double>(j < 4 ? a0[j] : a1[j - 4]) : 0.0;
    }
  }
  const int rowc = rowok ? myrow : 0;
  const double bq = rowok ? (WARM ? bvec[rowc] : static_cast<double>(H[r * hld + rowc])) : 0.0;
  const double dg = rowok ? static_cast<double>(H[rowc * hld + rowc]) : 1.0;
  const double di = dg > 0.0 ? 1.0 / dg : 0.0;  // 1 where !rowok: every vector entry there is 0
  // H y at this lane's row for y given at every column through LDS
  auto hprod_r = [&](const double (&yc)[8]) -> double {
    double ap[8];
#pragma unroll
    for (int ii = 0; ii < 8; ++ii) {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < 8; ++j) a = fma(h[ii][j], yc[j], a);
      ap[ii] = a;
    }
    return row16_reduce_scatter8_px(ap);
  };
  auto hprod = [&](const double* y) -> double {
    double yc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) yc[j] = y[8 * cb + j];
    return hprod_r(yc);
  };
  // x_0 = 0 (or the previous solution in sv.zv), r_0 = b - H x_0,
  // u_0 = M r_0, w_0 = H u_0
  double xr = 0.0, rr_ = bq;
  if (WARM) {
    const double hx = hprod(sv.zv);
    xr = rowok ? sv.zv[myrow] : 0.0;
    rr_ = rowok ? bq - hx : 0.0;
  }
  double ur = di * rr_;
  const double pb = wave_sum_dpp(0.5 * (bq * di * bq));  // (r_0, M r_0)
  const bool anybad = __ballot(rowok && !(dg > 0.0)) != 0ull;
  if (lane == 0) {
    sv.red[3][wave] = pb;
    sv.badf[wave] = anybad ? 1 : 0;
  }
  if (owner) sv.mv[1][myrow] = ur;  // rows >= r hold 0
  __syncthreads();
  double bn2 = 0.0;
  int cg_fail = 0;
#pragma unroll
  for (int w = 0; w < kGWaves; ++w) {
    bn2 += sv.red[3][w];
    cg_fail |= sv.badf[w];
  }
  if (bn2 > 0.0 && !cg_fail) {
    const double stop2 = kCgTol * kCgTol * bn2;
    double wr = hprod(sv.mv[1]);
    double zr = 0.0, qr = 0.0, sr = 0.0, pr = 0.0;
    double rcp_gamma_old = 1.0, rcp_alpha_old = 1.0;
    int it = 0;
#pragma unroll 1
    for (; it < kCgMaxIt; ++it) {
      const int sl = it & 1;  // double-buffered exchange slots
      const double mr = di * wr;
      const double g0 = wave_sum_l63(0.5 * (rr_ * ur));
      const double g1 = wave_sum_l63(0.5 * (wr * ur));
      if (lane == 63) {
        sv.cgr[sl][wave][0] = g0;
        sv.cgr[sl][wave][1] = g1;
      }
      if (owner) sv.mv[sl][myrow] = mr;
      __syncthreads();  // the inner products and m = M w are in
      // the next product's operand is read with the sums, before the test
      double yc[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) yc[j] = sv.mv[sl][8 * cb + j];
      double gam = 0.0, del = 0.0;
#pragma unroll
      for (int w = 0; w < kGWaves; ++w) {
        gam += sv.cgr[sl][w][0];
        del += sv.cgr[sl][w][1];
      }
      if (gam <= stop2) break;
      const double nr = hprod_r(yc);
      // the step lengths with a hardware reciprocal and two Newton steps
      // (quadratic: relative error below 2^-52 from the rcp's 2^-22)
      auto rcp = [](double d) {
        double x = __builtin_amdgcn_rcp(d);
        x = fma(x, fma(-d, x, 1.0), x);
        return fma(x, fma(-d, x, 1.0), x);
      };
      double beta = 0.0, alpha;
      if (it == 0) {
        alpha = gam * rcp(del);
      } else {
        beta = gam * rcp_gamma_old;
        alpha = gam * rcp(del - beta * gam * rcp_alpha_old);
      }
      if (!(del > 0.0) || !(alpha > 0.0)) {
        cg_fail = 1;
        break;
      }
      zr = fma(beta, zr, nr);
      qr = fma(beta, qr, mr);
      sr = fma(beta, sr, wr);
      pr = fma(beta, pr, ur);
      xr = fma(alpha, pr, xr);
      rr_ = fma(-alpha, sr, rr_);
      ur = fma(-alpha, qr, ur);
      wr = fma(-alpha, zr, wr);
      rcp_gamma_old = rcp(gam);
      rcp_alpha_old = rcp(alpha);
    }
    if (it == kCgMaxIt) cg_fail = 2;
  }
  // every read of zv and mv[1] happened before the loop's first barrier
  if (owner) {
    sv.zv[myrow] = rowok ? xr : 0.0;
    sv.zf[myrow] = rowok ? static_cast<float>(xr) : 0.0f;
  }
  __syncthreads();
  return cg_fail;
}

}  // namespace
}  // namespace rpt
