// Sequential subspace tracking of RapidPT's training phase (Sec. 4.1; Alg. 2,
// Subspace-Tracking): GROUSE's geodesic step (Balzano, Nowak & Recht 2010)
// with the greedy angle (Zhang & Balzano 2016) applied to the training
// columns one at a time.  For column x observed at the sampled voxels O:
//     w = argmin |x_O - U_O w|,  p = U w,  e = x_O - U_O w (zero off O),
//     theta = gamma arctan(|e| / |p|),
//     U <- U + ((cos theta - 1) p / |p| + sin theta e / |e|) w^T / |w|.
// For orthonormal U, |p| = |w| and the step is
//     U <- U (I + (c - 1) wh wh^T) + s (e / |e|) wh^T,   wh = w / |w|,
// (c, s = cos, sin theta): a right factor of rank one plus a term that lives
// on the sampled rows only.  The basis is therefore kept as U = B N^{-1}
// (B v x r, N r x r; each pass starts from B = U, N = I).  With
//     N' = (I + (1/c - 1) wh wh^T) N,   u = N^T wh,
// the step is N <- N' and B[O] += (s / |e|) e (u / c)^T, so a step reads and
// writes the k sampled rows of B and the r x r matrix N, not all v x r
// entries of U.  The fit needs only B: U_O w = B_O (N^{-1} w), so
// z = argmin |x_O - B_O z| and w = N z.  A step depends on the basis only
// through its subspace (a rotation U Q of the basis gives w' = Q^T w and the
// same p, e and theta), and span(U) = span(B); so at the end of a pass B is
// orthonormalised (Cholesky-QR) and becomes the next pass's U with N = I.
//
// One workgroup of 8 waves runs a whole pass (the steps form a dependent
// chain).  Per step:
//  1. Gram of [B_O | x_O]: the sampled rows, SR at a time, are gathered with
//     16-byte loads (the next group in flight while the current one is
//     multiplied), split into BF16 hi/lo and staged transposed in LDS; the
//     lower 16 x 16 tiles of the (r+1) x (r+1) Gram matrix are spread over
//     the waves and accumulated on 16x16x32 matrix-core products as
//     hi.hi + hi.lo + lo.hi.  Column r is x_O, so row r holds b = B_O^T x_O.
//  2. H z = b by Jacobi-preconditioned conjugate gradients in FP64 (H in LDS
//     in FP32): a dependent chain of short matrix-vector products, much
//     shorter than an r-step Cholesky on one workgroup.
//  3. e = x_O - B_O z (16 lanes per sampled row, four rows per lane group
//     in flight), |e|^2 in FP64.
//  4. w = N z, the angle, u = N^T wh and the rank-one update of N (FP32 in
//     LDS), then B[O] += (s / |e|) e (u / c)^T.
// The Eq. 1 objective of the pass, the sum over its visits of |e|^2 before U
// moves, decides when tracking has converged.
#include "rpt_internal.h"

namespace rpt {

namespace {

constexpr int kGT = 512;           // threads of the tracking workgroup
constexpr int kGWaves = kGT / 64;  // 8
constexpr int kCB = kGT / 128;     // column blocks of the matrix-vector products
constexpr int kCW = 128 / kCB;     // their width
constexpr int kGR = 128;           // rank bound
constexpr int kCgMaxIt = 300;      // conjugate-gradient iteration cap
constexpr double kCgTol = 1e-8;    // stop when |b - H z| <= kCgTol |b|
constexpr int kRowLanes = 16;      // lanes per sampled row in the row phases
constexpr int kRowU = 4;           // rows per lane group in flight
constexpr size_t kLdsMax = 160 * 1024;

struct GrouseArgs {
  float* B;              // v x r, the pass's basis factor (in place)
  int64_t v;
  int r;
  const float* T;        // training columns, row i = t map of column i
  int64_t ldT;
  const int32_t* omega;  // this pass's sampled sets, ell x k
  int k;
  int ell;
  float gamma;
  float* ybuf;           // [k]: sampled values, then residuals
  double* objr;          // [2]: objectives of the previous and current pass
  double* obj_out;       // [passes] or null
  int pass;
  int32_t* stop;         // first pass at which tracking converged (INT_MAX: none)
  int32_t* used;         // passes run
  double tol;
  int32_t* info;         // [ell]
  int lidx;              // sampled indices held in LDS
};

// FP64 vectors of the solve and the move, then FP32 ones
struct GrouseVec {
  double x[kGR], p2[2][kGR], zv[kGR], wh[kGR];
  double part[kCB][kGR];
  double red[4][kGWaves];
  double red2[2][2][kGWaves];
  int badf[kGWaves];
  float zf[kGR], qf[kGR], u[kGR];
  float sink;
  int flag;
};

// dynamic LDS: [GrouseVec][N: r x (r + 1) FP32][union: staging | H][idx: k int]
struct GrouseLds {
  size_t n_off, u_off, idx_off, total;
};
__host__ __device__ inline int g_ncol(int r) { return 16 * ((r + 1 + 15) / 16); }
// H row length: at least r + 1 and 1 mod 32 words, so that the eight rows
// and four column blocks a half-wave reads in the solve fall in distinct banks
__host__ __device__ inline int g_hld(int r) { return ((r + 31) / 32) * 32 + 1; }
__host__ __device__ inline GrouseLds grouse_lds(int r, int k, int sr, bool lidx) {
  GrouseLds l;
  size_t off = (sizeof(GrouseVec) + 15) & ~size_t(15);
  l.n_off = off;
  off += static_cast<size_t>(r) * (r + 1) * sizeof(float);
  off = (off + 15) & ~size_t(15);
  l.u_off = off;
  const size_t stage = static_cast<size_t>(2) * g_ncol(r) * (sr + 8) * sizeof(uint16_t);
  const size_t h = static_cast<size_t>(r + 1) * g_hld(r) * sizeof(float);
  off += stage > h ? stage : h;
  off = (off + 15) & ~size_t(15);
  l.idx_off = off;
  if (lidx) off += static_cast<size_t>(k) * sizeof(int);
  l.total = off;
  return l;
}

// sum over the whole workgroup into every thread (red: kGWaves doubles, free
// on entry and not written again before the next barrier)
__device__ __forceinline__ double block_sum_d(double x, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  x = wave_sum_d(x);
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < kGWaves; ++i) t += red[i];
  return t;
}

// sum over threads 0..127 (the first two waves) into red[0..1]; callers
// synchronise before reading it
__device__ __forceinline__ void two_wave_sum(double x, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave < 2) {
    x = wave_sum_d(x);
    if (lane == 0) red[wave] = x;
  }
}

// sum over the 64 lanes of one wave with DPP moves (quad permutations, row
// mirrors, row broadcasts); the total ends in lane 63 and is read back as a
// scalar, so every lane gets it
__device__ __forceinline__ double dpp_add(double s, int ctrl_id) {
  const long long b = __double_as_longlong(s);
  int lo = static_cast<int>(b & 0xFFFFFFFFll), hi = static_cast<int>(b >> 32);
  switch (ctrl_id) {
    case 0:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false);
      break;
    case 1:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false);
      break;
    case 2:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false);
      break;
    case 3:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false);
      break;
    case 4:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x142, 0xA, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x142, 0xA, 0xF, false);
      break;
    default:
      lo = __builtin_amdgcn_update_dpp(0, lo, 0x143, 0xC, 0xF, false);
      hi = __builtin_amdgcn_update_dpp(0, hi, 0x143, 0xC, 0xF, false);
      break;
  }
  const long long m = (static_cast<long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo);
  return s + __longlong_as_double(m);
}
__device__ __forceinline__ double wave_sum_dpp(double s) {
  s = dpp_add(s, 0);  // quad_perm [1, 0, 3, 2]
  s = dpp_add(s, 1);  // quad_perm [2, 3, 0, 1]: quad sums
  s = dpp_add(s, 2);  // row_half_mirror: sums of eight
  s = dpp_add(s, 3);  // row_mirror: row sums
  s = dpp_add(s, 4);  // row_bcast:15 into rows 1 and 3
  s = dpp_add(s, 5);  // row_bcast:31 into rows 2 and 3: lane 63 holds the total
  const long long b = __double_as_longlong(s);
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b & 0xFFFFFFFFll), 63));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(b >> 32), 63));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

template <int RB, int SR>
__global__ __launch_bounds__(kGT) void grouse_pass_kernel(GrouseArgs a) {
  constexpr int NCOL = 16 * RB;
  constexpr int NG = NCOL / 4;                    // column groups of four
  constexpr int NU = (NG + kGWaves - 1) / kGWaves;
  constexpr int NT = RB * (RB + 1) / 2;           // lower 16 x 16 tiles
  constexpr int TPW = (NT + kGWaves - 1) / kGWaves;
  constexpr int RPL = SR / 64;                    // staged rows per lane
  constexpr int SLD = SR + 8;                     // BF16 per staged column
  extern __shared__ __align__(16) unsigned char lds[];
  if (*a.stop < a.pass) return;  // converged in an earlier pass
  const int r = a.r, k = a.k;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, c16 = lane & 15, kq = lane >> 4;
  const GrouseLds L = grouse_lds(r, k, SR, a.lidx != 0);
  GrouseVec& sv = *reinterpret_cast<GrouseVec*>(lds);
  float* N = reinterpret_cast<float*>(lds + L.n_off);
  uint16_t* sh = reinterpret_cast<uint16_t*>(lds + L.u_off);
  uint16_t* sl = sh + NCOL * SLD;
  float* H = reinterpret_cast<float*>(lds + L.u_off);
  int* sidx = reinterpret_cast<int*>(lds + L.idx_off);
  const int nld = r + 1, hld = g_hld(r);
  const bool vec = (r & 3) == 0 && (reinterpret_cast<uintptr_t>(a.B) & 15) == 0;
  // the pass starts from U = B, N = I
  for (int t = tid; t < r * nld; t += kGT) {
    const int i = t / nld, c = t - i * nld;
    N[t] = i == c ? 1.0f : 0.0f;
  }
  int tbi[TPW], tbj[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) {
    int t = wave + kGWaves * j, bi = 0;
    if (t < NT) {
      while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
      tbi[j] = bi;
      tbj[j] = t - bi * (bi + 1) / 2;
    } else {
      tbi[j] = tbj[j] = -1;
    }
  }
  double obj = 0.0;
  // row phases: lane group g = tid / 16 takes rows g, g + 32, ...; lane
  // covers columns 4 l + 64 h .. + 3 (h = 0, 1), l = lane % 16
  const int rg = tid / kRowLanes, rl = tid % kRowLanes;
  constexpr int NRG = kGT / kRowLanes;  // 32 row groups
  __syncthreads();

  for (int i = 0; i < a.ell; ++i) {
    const int32_t* om = a.omega + static_cast<int64_t>(i) * k;
    const float* Ti = a.T + static_cast<int64_t>(i) * a.ldT;
    // sampled voxels (out of range: -1, a zero row and a zero value) and values
    for (int q = tid; q < k; q += kGT) {
      const int64_t vox = om[q];
      const bool ok = vox >= 0 && vox < a.v;
      if (a.lidx) sidx[q] = ok ? static_cast<int>(vox) : -1;
      a.ybuf[q] = ok ? Ti[vox] : 0.0f;
    }
    if (tid == 0) sv.flag = 0;
    __threadfence_block();
    __syncthreads();
    auto voxel = [&](int q) -> int64_t {
      if (a.lidx) return sidx[q];
      const int64_t vx = om[q];
      return (vx >= 0 && vx < a.v) ? vx : -1;
    };
    // Warm the caches with this column's sampled rows before the Gram groups
    // gather them: one load per 128-byte line a row can touch, ten in flight
    // per lane, addresses clamped so that every load is issued.  The Gram
    // groups then wait for cache hits instead of one memory round trip each.
    {
      const int lines = (4 * r + 127) / 128 + 1;
      const int total = k * lines;
      for (int base = 0; base < total; base += 10 * kGT) {
        float pv[10];
#pragma unroll
        for (int u = 0; u < 10; ++u) {
          const int t = min(base + u * kGT + tid, total - 1);
          const int q = t / lines, l = t - q * lines;
          const int64_t vx = voxel(q);
          pv[u] = a.B[(vx >= 0 ? vx : 0) * r + min(32 * l, r - 1)];
        }
        float sum = 0.0f;
#pragma unroll
        for (int u = 0; u < 10; ++u) sum += pv[u];
        if (sum == -1.0e-37f) sv.sink = sum;  // keeps the loads (practically never taken)
      }
    }
    // ---------------------------------------------------------- 1. Gram
    f32x4 acc[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    float xv[RPL][NU][4];
    auto gather = [&](int s0) {
#pragma unroll
      for (int h = 0; h < RPL; ++h) {
        const int row = s0 + (RPL == 2 ? 2 * lane + h : lane);
        const int64_t vox = row < k ? voxel(row) : -1;
        const bool ok = vox >= 0;
        const float* br = a.B + (ok ? vox : 0) * r;
        const float yv = ok ? a.ybuf[row] : 0.0f;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          const int g = wave + kGWaves * u;
          const int c0 = 4 * g;
          if (vec) {
            // r is a multiple of 4: a group lies wholly below r or at and
            // above it; the load address is clamped, so every load is issued
            const f32x4 q = *reinterpret_cast<const f32x4*>(br + min(c0, r - 4));
#pragma unroll
            for (int e = 0; e < 4; ++e)
              xv[h][u][e] = (g < NG && ok) ? (c0 < r ? q[e] : (c0 + e == r ? yv : 0.0f)) : 0.0f;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int c = c0 + e;
              float x = 0.0f;
              if (g < NG && ok) x = c < r ? br[c] : (c == r ? yv : 0.0f);
              xv[h][u][e] = x;
            }
          }
        }
      }
    };
    const int ngrp = (k + SR - 1) / SR;
    gather(0);
    for (int s = 0; s < ngrp; ++s) {
      // stage the registers (the previous group's products are done); with
      // two rows per lane they are rows 2 lane and 2 lane + 1, stored as one
      // 32-bit word per column and half
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        const int g = wave + kGWaves * u;
        if (g < NG) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int c = 4 * g + e;
            if (RPL == 2) {
              const uint16_t h0 = f2bf(xv[0][u][e]), h1 = f2bf(xv[RPL - 1][u][e]);
              const uint16_t l0 = f2bf(xv[0][u][e] - bf2f(h0)), l1 = f2bf(xv[RPL - 1][u][e] - bf2f(h1));
              *reinterpret_cast<uint32_t*>(sh + c * SLD + 2 * lane) = pack_bf2(h0, h1);
              *reinterpret_cast<uint32_t*>(sl + c * SLD + 2 * lane) = pack_bf2(l0, l1);
            } else {
              const uint16_t hb = f2bf(xv[0][u][e]);
              sh[c * SLD + lane] = hb;
              sl[c * SLD + lane] = f2bf(xv[0][u][e] - bf2f(hb));
            }
          }
        }
      }
      __syncthreads();
      if (s + 1 < ngrp) gather((s + 1) * SR);
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        if (tbi[j] < 0) continue;
        const int ra = (16 * tbi[j] + c16) * SLD + 8 * kq;
        const int rb = (16 * tbj[j] + c16) * SLD + 8 * kq;
#pragma unroll
        for (int kk = 0; kk < SR; kk += 32) {
          const u32x4 ah = *reinterpret_cast<const u32x4*>(sh + ra + kk);
          const u32x4 al = *reinterpret_cast<const u32x4*>(sl + ra + kk);
          const u32x4 bh = *reinterpret_cast<const u32x4*>(sh + rb + kk);
          const u32x4 bl = *reinterpret_cast<const u32x4*>(sl + rb + kk);
          acc[j] = mfma16_bf16(ah, bh, acc[j]);
          acc[j] = mfma16_bf16(ah, bl, acc[j]);
          acc[j] = mfma16_bf16(al, bh, acc[j]);
        }
      }
      __syncthreads();
    }
    // tiles into H (aliases the staging buffer, whose reads are all done):
    // the lower triangle and its mirror, rows and columns 0..r
#pragma unroll
    for (int j = 0; j < TPW; ++j) {
      if (tbi[j] < 0) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = 16 * tbi[j] + 4 * kq + e, col = 16 * tbj[j] + c16;
        if (row >= col && row <= r) {
          H[row * hld + col] = acc[j][e];
          H[col * hld + row] = acc[j][e];
        }
      }
    }
    __syncthreads();

    // ---------------------------------------------------------- 2. H z = b
    // Wave w owns rows 16 w .. 16 w + 15: lane 4 j + q forms the part of row
    // 16 w + j over the columns 32 m + 8 q .. + 7 (m = 0..3), a quad
    // reduction completes it.
    // Every wave forms the search direction p_t = z_t + beta p_{t-1} itself
    // from z_t and p_{t-1} in LDS while the owners store p_t into the other
    // of two buffers, so an iteration needs two barriers (after the p.Hp
    // partial sums and after the residual partial sums).
    int cg_fail = 0;
    {
      const int jr = lane >> 2, qc = lane & 3;
      const int row = 16 * wave + jr;
      const bool ownr = row < r;
      const int rowc = ownr ? row : 0;
      const double b = ownr ? static_cast<double>(H[r * hld + row]) : 0.0;
      const double dg = ownr ? static_cast<double>(H[row * hld + row]) : 1.0;
      const double di = dg > 0.0 ? 1.0 / dg : 0.0;
      const bool lead = qc == 0;
      double xr = 0.0, sr = b, zr = di * b, pr = 0.0;
      const double pb = wave_sum_dpp(lead ? b * b : 0.0);
      const double pz = wave_sum_dpp(lead ? sr * zr : 0.0);
      const bool anybad = __ballot(ownr && !(dg > 0.0)) != 0ull;
      if (lane == 0) {
        sv.red[2][wave] = pb;
        sv.red[3][wave] = pz;
        sv.badf[wave] = anybad ? 1 : 0;
      }
      if (lead) {
        sv.zv[row] = zr;        // rows >= r hold 0
        sv.p2[1][row] = 0.0;    // p_{-1}
      }
      __syncthreads();
      double bn2 = 0.0, rz = 0.0;
#pragma unroll
      for (int w = 0; w < kGWaves; ++w) {
        bn2 += sv.red[2][w];
        rz += sv.red[3][w];
        cg_fail |= sv.badf[w];
      }
      if (bn2 > 0.0 && !cg_fail) {
        const double stop2 = kCgTol * kCgTol * bn2;
        const float* hrow = H + rowc * hld;
        double beta = 0.0;
        int it = 0;
        for (; it < kCgMaxIt; ++it) {
          const int slot = it & 1;
          const double* pold = sv.p2[slot ^ 1];
          pr = fma(beta, pr, zr);
          if (lead) sv.p2[slot][row] = ownr ? pr : 0.0;
          double a0 = 0.0, a1 = 0.0;
#pragma unroll 1
          for (int m = 0; m < 4; ++m) {
            double pc[8];
            float hv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const int c = 32 * m + 8 * qc + e;
              pc[e] = fma(beta, pold[c], sv.zv[c]);  // zero from column r on
              hv[e] = hrow[min(c, r)];                 // clamped into the row: finite
            }
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
              a0 = fma(static_cast<double>(hv[e]), pc[e], a0);
              a1 = fma(static_cast<double>(hv[e + 1]), pc[e + 1], a1);
            }
          }
          double apr = a0 + a1;
          apr += __shfl_xor(apr, 1, 64);
          apr += __shfl_xor(apr, 2, 64);
          if (!ownr) apr = 0.0;
          const double pap_w = wave_sum_dpp(lead ? pr * apr : 0.0);
          if (lane == 0) sv.red2[slot][0][wave] = pap_w;
          __syncthreads();  // every read of z and p_{t-1} is done, p.Hp partials are in
          double pap = 0.0;
#pragma unroll
          for (int w = 0; w < kGWaves; ++w) pap += sv.red2[slot][0][w];
          if (!(pap > 0.0)) {
            cg_fail = 1;
            break;
          }
          const double alpha = rz / pap;
          xr = fma(alpha, pr, xr);
          sr = fma(-alpha, apr, sr);
          zr = di * sr;
          if (lead) sv.zv[row] = ownr ? zr : 0.0;
          const double rz_w = wave_sum_dpp(lead ? sr * zr : 0.0);
          const double rr_w = wave_sum_dpp(lead ? sr * sr : 0.0);
          if (lane == 0) {
            sv.red2[slot][1][wave] = rz_w;
            sv.red[slot][wave] = rr_w;
          }
          __syncthreads();  // z_{t+1} and the residual partials are in
          double rz1 = 0.0, rr1 = 0.0;
#pragma unroll
          for (int w = 0; w < kGWaves; ++w) {
            rz1 += sv.red2[slot][1][w];
            rr1 += sv.red[slot][w];
          }
          if (rr1 <= stop2) break;
          beta = rz1 / rz;
          rz = rz1;
        }
        if (it == kCgMaxIt) cg_fail = 2;
      }
      if (lead) {
        sv.x[row] = ownr ? xr : 0.0;
        sv.zf[row] = ownr ? static_cast<float>(xr) : 0.0f;
      }
      __syncthreads();
    }
    const bool own = tid < r;

    // ---------------------------------------------------------- 3. residual
    float zl[8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int c = 4 * rl + 64 * h + e;
        zl[4 * h + e] = c < r ? sv.zf[c] : 0.0f;
      }
    double ee = 0.0;
    for (int q0 = rg; q0 < k; q0 += NRG * kRowU) {
      float d[kRowU];
      bool okr[kRowU];
      if (vec) {
        // every row's loads issued before the first product (rows out of
        // range read row 0 and are dropped)
        f32x4 b4[kRowU][2];
#pragma unroll
        for (int u = 0; u < kRowU; ++u) {
          const int q = q0 + NRG * u;
          const int64_t vx = q < k ? voxel(q) : -1;
          okr[u] = vx >= 0;
          const float* br = a.B + (okr[u] ? vx : 0) * r;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int c0 = 4 * rl + 64 * h;
            b4[u][h] = *reinterpret_cast<const f32x4*>(br + min(c0, r - 4));  // clamped: always issued
          }
        }
#pragma unroll
        for (int u = 0; u < kRowU; ++u) {
          float t = 0.0f;
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) t = fmaf(b4[u][h][e], zl[4 * h + e], t);
          d[u] = okr[u] ? t : 0.0f;
        }
      } else {
#pragma unroll
        for (int u = 0; u < kRowU; ++u) {
          const int q = q0 + NRG * u;
          const int64_t vx = q < k ? voxel(q) : -1;
          okr[u] = vx >= 0;
          d[u] = 0.0f;
          if (okr[u]) {
            const float* br = a.B + vx * r;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int c0 = 4 * rl + 64 * h;
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (c0 + e < r) d[u] = fmaf(br[c0 + e], zl[4 * h + e], d[u]);
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kRowU; ++u) {
#pragma unroll
        for (int off = kRowLanes / 2; off >= 1; off >>= 1) d[u] += __shfl_xor(d[u], off, 64);
        const int q = q0 + NRG * u;
        if (rl == 0 && q < k) {
          const float e = a.ybuf[q] - d[u];
          a.ybuf[q] = e;
          ee += static_cast<double>(e) * e;
        }
      }
    }
    __threadfence_block();
    ee = block_sum_d(ee, sv.red[3]);
    obj += ee;

    // ---------------------------------------------------------- 4. move
    // w = N z (thread (row, block of kCW columns))
    {
      const int row = tid & (kGR - 1), cb = tid >> 7;
      double s = 0.0;
      if (row < r) {
        // column indices clamped to r - 1 (x is zero from r on): no
        // conditional loads
        const float* nr = N + row * nld;
#pragma unroll 8
        for (int c = 0; c < kCW; ++c) {
          const int cc = kCW * cb + c;
          s = fma(static_cast<double>(nr[min(cc, r - 1)]), sv.x[cc], s);
        }
      }
      sv.part[cb][row] = s;
    }
    __syncthreads();
    if (tid < kGR) {
      double wv = 0.0;
#pragma unroll
      for (int b = 0; b < kCB; ++b) wv += sv.part[b][tid];
      if (!own) wv = 0.0;
      sv.wh[tid] = wv;
      two_wave_sum(wv * wv, sv.red[0]);
    }
    __syncthreads();
    const double nw = sqrt(sv.red[0][0] + sv.red[0][1]);
    const double ne = sqrt(ee);
    double cth = 1.0, sth = 0.0;
    if (nw > 0.0 && ne > 0.0 && !cg_fail) {
      const double th = static_cast<double>(a.gamma) * atan(ne / nw);
      cth = cos(th);
      sth = sin(th);
    }
    if (sth != 0.0 && fabs(cth) > 1e-12) {
      // u = N^T wh: thread (column, block of kCW rows)
      {
        const int col = tid & (kGR - 1), blk = tid >> 7;
        const double inw = 1.0 / nw;
        double su = 0.0;
        if (col < r) {
#pragma unroll 8
          for (int i2 = 0; i2 < kCW; ++i2) {
            const int rr = kCW * blk + i2;
            su = fma(sv.wh[rr] * inw, static_cast<double>(N[min(rr, r - 1) * nld + col]), su);
          }
        }
        sv.part[blk][col] = su;
      }
      __syncthreads();
      if (tid < kGR) {
        double tu = 0.0;
#pragma unroll
        for (int b = 0; b < kCB; ++b) tu += sv.part[b][tid];
        sv.u[tid] = own ? static_cast<float>(tu) : 0.0f;
        sv.qf[tid] = own ? static_cast<float>(tu / cth) : 0.0f;
        sv.zf[tid] = own ? static_cast<float>(sv.wh[tid] / nw) : 0.0f;  // wh
      }
      __syncthreads();
      // N += (1/c - 1) wh u^T
      const float fi = static_cast<float>(1.0 / cth - 1.0);
      for (int t = tid; t < r * nld; t += kGT) {
        const int i2 = t / nld, c = t - i2 * nld;
        if (c < r) N[t] = fmaf(fi * sv.zf[i2], sv.u[c], N[t]);
      }
      // B[O] += (s / |e|) e q^T
      const float g = static_cast<float>(sth / ne);
      float ql[8];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = 4 * rl + 64 * h + e;
          ql[4 * h + e] = c < r ? sv.qf[c] : 0.0f;
        }
      for (int q0 = rg; q0 < k; q0 += NRG * kRowU) {
        f32x4 b4[kRowU][2];
        int64_t vx[kRowU];
        float ge[kRowU];
#pragma unroll
        for (int u = 0; u < kRowU; ++u) {
          const int q = q0 + NRG * u;
          vx[u] = q < k ? voxel(q) : -1;
          ge[u] = vx[u] >= 0 ? g * a.ybuf[q] : 0.0f;
          if (vec) {
            const float* br = a.B + (vx[u] >= 0 ? vx[u] : 0) * r;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int c0 = 4 * rl + 64 * h;
              b4[u][h] = *reinterpret_cast<const f32x4*>(br + min(c0, r - 4));  // clamped: always issued
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kRowU; ++u) {
          if (vx[u] < 0) continue;
          float* br = a.B + vx[u] * r;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int c0 = 4 * rl + 64 * h;
            if (vec) {
              if (c0 + 4 <= r) {
                f32x4 t4 = b4[u][h];
#pragma unroll
                for (int e = 0; e < 4; ++e) t4[e] = fmaf(ge[u], ql[4 * h + e], t4[e]);
                *reinterpret_cast<f32x4*>(br + c0) = t4;
              }
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (c0 + e < r) br[c0 + e] = fmaf(ge[u], ql[4 * h + e], br[c0 + e]);
            }
          }
        }
      }
    }
    if (tid == 0) a.info[i] = cg_fail ? -cg_fail : 0;
    __threadfence_block();
    __syncthreads();
  }

  if (tid == 0) {
    const int slot = a.pass & 1;
    a.objr[slot] = obj;
    if (a.obj_out) a.obj_out[a.pass] = obj;
    *a.used = a.pass + 1;
    if (a.pass >= 1 && a.tol > 0.0) {
      const double prev = a.objr[slot ^ 1];
      if (prev - obj <= a.tol * prev) *a.stop = a.pass;
    }
  }
}

__global__ void grouse_init_kernel(int32_t* stop, int32_t* used, double* objr, double* obj_out, int passes) {
  if (threadIdx.x == 0) {
    *stop = 0x7FFFFFFF;
    *used = 0;
    objr[0] = 0.0;
    objr[1] = 0.0;
  }
  if (obj_out)
    for (int p = threadIdx.x; p < passes; p += blockDim.x) obj_out[p] = 0.0;
}

template <int RB, int SR>
rpt_status launch_pass(const GrouseArgs& a, size_t smem, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&grouse_pass_kernel<RB, SR>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsMax));
    attr = true;
  }
  hipLaunchKernelGGL((grouse_pass_kernel<RB, SR>), dim3(1), dim3(kGT), smem, s, a);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace

size_t grouse_bytes(int r, int k) {
  Carver c(nullptr);
  c.take<float>(static_cast<size_t>(k));
  c.take<double>(2);
  c.take<int32_t>(3);
  (void)r;
  return c.off;
}

GrouseState grouse_carve(void* ws, int r, int k) {
  Carver c(ws);
  GrouseState g;
  g.ybuf = c.take<float>(static_cast<size_t>(k));
  g.objr = c.take<double>(2);
  int32_t* flags = c.take<int32_t>(3);
  g.stop = flags;
  g.used_ws = flags ? flags + 1 : nullptr;
  g.rinfo = flags ? flags + 2 : nullptr;
  (void)r;
  return g;
}

rpt_status grouse_init_launch(const GrouseState& g, int32_t* used, double* obj_out, int passes, hipStream_t s) {
  hipLaunchKernelGGL(grouse_init_kernel, dim3(1), dim3(256), 0, s, g.stop, used ? used : g.used_ws, g.objr, obj_out,
                     passes);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status grouse_pass_launch(const GrouseState& g, float* B, int64_t v, int r, const float* T, int64_t ldT,
                              const int32_t* omega, int k, int ell, float gamma, int pass, double tol,
                              double* obj_out, int32_t* used, int32_t* info, hipStream_t s) {
  if (r < 1 || r > kGR) return RPT_ERR_UNSUPPORTED;
  GrouseArgs a;
  a.B = B;
  a.v = v;
  a.r = r;
  a.T = T;
  a.ldT = ldT;
  a.omega = omega;
  a.k = k;
  a.ell = ell;
  a.gamma = gamma;
  a.ybuf = g.ybuf;
  a.objr = g.objr;
  a.obj_out = obj_out;
  a.pass = pass;
  a.stop = g.stop;
  a.used = used ? used : g.used_ws;
  a.tol = tol;
  a.info = info;
  // 128 staged rows when they fit in LDS with the rest, else 64; the sampled
  // indices in LDS when they fit too
  const int RB = (r + 1 + 15) / 16;
  const bool big = RB <= 8 && grouse_lds(r, k, 128, false).total <= kLdsMax;
  const int sr = big ? 128 : 64;
  a.lidx = grouse_lds(r, k, sr, true).total <= kLdsMax ? 1 : 0;
  const size_t smem = grouse_lds(r, k, sr, a.lidx != 0).total;
  if (smem > kLdsMax) return RPT_ERR_UNSUPPORTED;
  RPT_STAGE("track_grouse", s);
#define RPT_GROUSE_CASE(rb) \
  case rb:                  \
    return big ? launch_pass<rb, 128>(a, smem, s) : launch_pass<rb, 64>(a, smem, s);
  switch (RB) {
    RPT_GROUSE_CASE(1)
    RPT_GROUSE_CASE(2)
    RPT_GROUSE_CASE(3)
    RPT_GROUSE_CASE(4)
    RPT_GROUSE_CASE(5)
    RPT_GROUSE_CASE(6)
    RPT_GROUSE_CASE(7)
    RPT_GROUSE_CASE(8)
    default:
      return launch_pass<9, 64>(a, smem, s);
  }
#undef RPT_GROUSE_CASE
}

}  // namespace rpt
