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
// A pass is one launch of nwg workgroups of four waves (one wave per SIMD,
// so each holds up to 512 registers).  The k sampled rows of a step are cut
// into slices of 32; workgroup g owns slices g, g + nwg, ... (one each up to
// 64 slices).  Per step:
//  1. Every workgroup gathers its rows once into LDS as [B_q | x_q | 0 ..]
//     and accumulates its partial Gram tiles of [B_O | x_O] on 16x16x4 FP32
//     matrix-core products (lane (c, q) holds row q of a group of four at
//     column c of each 16-column block; wave w takes the tiles t = w mod 4).
//  2. Grid barrier; each workgroup sums a share of the tiles over all
//     partials; grid barrier.  Row r of the summed H is b = B_O^T x_O.
//  3. Every workgroup solves H z = b itself by Jacobi-preconditioned
//     conjugate gradients in FP64, H in registers (lane (q, c) of wave w:
//     rows 32 w + 8 q .. + 7, columns 8 c .. 8 c + 7; H p is eight FMAs per
//     row and a reduce-scatter over the 16 lanes of a DPP row).  The solve
//     and the r x r updates below are identical in every workgroup, so z, w,
//     the angle and N agree bit for bit without being exchanged.
//  4. The residuals e = x_O - B_O z of its rows (from LDS); |e|^2 follows
//     from H itself (x_O^T x_O - b^T z) unless the fit leaves less than a
//     tenth of |x_O|^2, when the rows' partial sums are exchanged (grid
//     barrier; every workgroup adds them in one order).
//  5. w = N z, the angle, u = N^T wh and the rank-one update of N (each
//     lane keeps its 8 x 8 block of N, the layout of H, in registers); then
//     each workgroup writes B[q] + (s / |e|) e_q (u / c)^T for its rows;
//     grid barrier, so that the next step gathers the moved rows.
// N stretches by 1/c along wh at every step; when the steps are large it
// loses its conditioning within a pass, so the pass then refreshes
// B <- B N^{-1} (= U) over all rows and restarts from N = I (N^{-1} is kept
// by the same rank-one updates).
// A single workgroup would gather the 875 rows of a step at about 20 GB/s;
// spread over 28 workgroups the gathers overlap and the step is bounded by
// the solve and the three barriers.  The Eq. 1 objective of the pass, the
// sum over its visits of |e|^2 before U moves, decides when tracking has
// converged.
#include <type_traits>

#include "pcg.h"
#include "rpt_internal.h"

namespace rpt {

namespace {

constexpr size_t kLdsMax = 160 * 1024;

struct GrouseArgs {
  float* B;              // v x r, the pass's basis factor (in place)
  int64_t v;
  int r;
  const float* T;        // training columns, row i = t map of column i
  int64_t ldT;
  const int32_t* omega;  // this pass's sampled sets, ell x k
  const float* xo;       // their sampled values T[i][omega[i][q]], ell x k
  int k;
  int ell;
  float gamma;
  double* objr;          // [2]: objectives of the previous and current pass
  double* obj_out;       // [passes] or null
  int pass;
  int32_t* stop;         // first pass at which tracking converged (INT_MAX: none)
  int32_t* used;         // passes run
  double tol;
  int32_t* info;         // [ell]
};

// FP64 vectors of the solve and the move, then FP32 ones
struct GrouseVec {
  double zv[kGR];  // CG direction source z_t, then the solution z
  double wv[kGR];  // w = N z
  double uu[kGR];  // u = N^T wh
  double mw[kGR];   // N^{-1} wh
  double mv[2][kGR];  // M w of the conjugate-gradient iterations
  double gv[kGR];     // right-hand side of the l1 fit's solves
  double cgr[2][kGWaves][2];
  double red[4][kGWaves];
  double nf2[2];  // |N|_F^2, |N^{-1}|_F^2
  int badf[kGWaves];
  float zf[kGR], qf[kGR];
};

// the lower 16 x 16 tiles (bi >= bj) of an RB-block Gram matrix, numbered
// bi (bi + 1) / 2 + bj; tile group G of TG takes the tiles t = G mod TG.
// One 16x16x4 FP32 matrix-core product per tile and group of four rows:
// lane (c, q) holds row q of the group at column c of each block (x[b]).
__host__ __device__ constexpr int gram_ntw(int rb, int tg) { return (rb * (rb + 1) / 2 + tg - 1) / tg; }
template <int RB, int TG, int G>
__device__ __forceinline__ void gram_products(f32x4 (&acc)[gram_ntw(RB, TG)], const float (&x)[RB]) {
#pragma unroll
  for (int bi = 0; bi < RB; ++bi)
#pragma unroll
    for (int bj = 0; bj <= bi; ++bj) {
      const int t = bi * (bi + 1) / 2 + bj;
      if (t % TG == G) acc[t / TG] = __builtin_amdgcn_mfma_f32_16x16x4f32(x[bi], x[bj], acc[t / TG], 0, 0, 0);
    }
}

constexpr int kCoopSlice = 32;        // sampled rows per slice
constexpr int kCoopMaxWg = 64;        // workgroups of one pass
constexpr long kSpinMax = 1L << 22;   // polls of a grid barrier before it gives up
constexpr double kRefresh = 1.05;     // refresh B = U N when |N|_F |N^{-1}|_F > kRefresh r

struct CoopArgs {
  GrouseArgs g;
  float* part;      // [nwg][NT][256]: partial Gram tiles
  float* hred;      // [NT][256]: the summed tiles
  double* epart;    // [2 nwg]: partial |e|^2 (l1: |Gamma|^2 and the misfit)
  uint32_t* ctr;    // [2]: barrier counters of even and odd passes
  int32_t* abort;   // raised when a barrier wait expires
  int nwg;          // workgroups
  int spw;          // slices of 32 sampled rows per workgroup (at most)
  // robust (l1) tracking
  float* gpart;     // [nwg][kGR]: partial right-hand sides of the l1 fit's solves
  float rho;        // ADMM penalty
  int admm_iters;   // ADMM iterations per column
};

// dynamic LDS: [GrouseVec][H: 16 RB x hld FP32, later the partial sums of
// u][rows: 32 spw x rs FP32][voxel, e, and the l1 fit's s, lam, t: 32 spw
// each][flag]
__host__ __device__ constexpr int coop_rs(int rb) { return 16 * rb + 2; }
__host__ __device__ inline size_t coop_lds(int r, int spw) {
  const int rb = g_rb(r);
  size_t off = (sizeof(GrouseVec) + 15) & ~size_t(15);
  const size_t h = static_cast<size_t>(16 * rb) * g_hld(rb) * sizeof(float);
  const size_t up = static_cast<size_t>(4 * kGWaves) * kGR * sizeof(double);
  off += h > up ? h : up;
  off = (off + 15) & ~size_t(15);
  off += static_cast<size_t>(kCoopSlice) * spw * coop_rs(rb) * sizeof(float);
  off += static_cast<size_t>(5 * kCoopSlice * spw + 4) * sizeof(int);
  return off;
}

// Every workgroup arrives before any leaves.  Stores made before it are
// seen by loads after it in every workgroup: the release fence writes this
// XCD's L2 back, the acquire fence invalidates this CU's L1 and the L2.  The
// wait is bounded; when it expires the abort flag is raised, and every
// workgroup that sees it (or expires itself) returns false and leaves the
// pass.
__device__ __forceinline__ bool coop_barrier(uint32_t* ctr, uint32_t target, int32_t* abort, int* flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    long spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinMax) {
        __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag = ok;
  }
  __syncthreads();
  return *flag != 0;
}

template <int RB, int MODE>
__global__ __launch_bounds__(kGT) void grouse_coop_kernel(CoopArgs ca) {
  extern __shared__ __align__(16) unsigned char lds[];
  const GrouseArgs& a = ca.g;
  if (*a.stop < a.pass) return;  // converged in an earlier pass
  constexpr int hld = g_hld(RB), rs = coop_rs(RB);
  constexpr int NT = RB * (RB + 1) / 2, TG = kGWaves, NTW = gram_ntw(RB, kGWaves);
  const int r = a.r, k = a.k, nwg = ca.nwg, wg = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  GrouseVec& sv = *reinterpret_cast<GrouseVec*>(lds);
  size_t off = (sizeof(GrouseVec) + 15) & ~size_t(15);
  float* H = reinterpret_cast<float*>(lds + off);
  double* upart = reinterpret_cast<double*>(lds + off);
  {
    const size_t h = static_cast<size_t>(16 * RB) * hld * sizeof(float);
    const size_t up = static_cast<size_t>(4 * kGWaves) * kGR * sizeof(double);
    off += h > up ? h : up;
    off = (off + 15) & ~size_t(15);
  }
  // this workgroup's slices: wg, wg + nwg, ... (nsl of them)
  const int nslices = (k + kCoopSlice - 1) / kCoopSlice;
  const int nsl = (nslices - wg + nwg - 1) / nwg;
  float* rows = reinterpret_cast<float*>(lds + off);
  int* svox = reinterpret_cast<int*>(rows + kCoopSlice * ca.spw * rs);
  float* se = reinterpret_cast<float*>(svox + kCoopSlice * ca.spw);
  float* ss = se + kCoopSlice * ca.spw;   // the l1 fit's s, lam and x - s - lam / rho
  float* sl = ss + kCoopSlice * ca.spw;
  float* st = sl + kCoopSlice * ca.spw;
  int* flag = reinterpret_cast<int*>(st + kCoopSlice * ca.spw);
  uint32_t* ctr = ca.ctr + (a.pass & 1);
  if (wg == 0 && tid == 0) ca.ctr[(a.pass + 1) & 1] = 0;  // the next pass's counter, idle during this one
  uint32_t target = 0;
  const bool vec = (r & 3) == 0 && (reinterpret_cast<uintptr_t>(a.B) & 15) == 0;
  // this lane's 8 x 8 block of N (rows 32 w + 8 rq + i, columns 8 cb + j), in
  // registers; the pass starts from N = I
  // (and of N^{-1}, nin)
  float nreg[8][8], nin[8][8];
  // |N|_F^2 and |N^{-1}|_F^2 (sv.nf2 in LDS), followed through the rank-one
  // updates: with |wh| = 1, N' = (I + a wh wh^T) N has
  // |N'|^2 = |N|^2 + (2 a + a^2) |N^T wh|^2 and N^{-1}' = N^{-1} (I + (c - 1)
  // wh wh^T) has |N^{-1}'|^2 = |N^{-1}|^2 + (c^2 - 1) |N^{-1} wh|^2
  auto identity = [&]() {
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int rr = 32 * wave + 8 * (lane >> 4) + i, cc = 8 * (lane & 15) + j;
        nreg[i][j] = nin[i][j] = (rr == cc && rr < r) ? 1.0f : 0.0f;
      }
    if (tid == 0) sv.nf2[0] = sv.nf2[1] = static_cast<double>(r);
  };
  identity();
  double obj = 0.0;
  bool alive = true;

#pragma unroll 1
  for (int i = 0; i < a.ell && alive; ++i) {
    // Lane coordinates, formed afresh in every step: the empty asm hides the
    // lane id from loop-invariant code motion, which would otherwise keep
    // dozens of addresses and masks derived from it in registers for the
    // whole pass.
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int c16 = ln & 15, kq = ln >> 4;
    const int rq = ln >> 4, cb = ln & 15;
    const int rbase = 32 * wave + 8 * rq;
    const int myrow = rbase + row8_sel(cb);
    const bool owner = (cb & 1) == 0, rowok = myrow < r;
    const int rg = 4 * wave + (ln >> 4), rl = ln & 15;  // 16 row groups of 16 lanes
    // ---------------------------------------------------------- 0. refresh
    // Each step stretches N by 1/c along wh; where the steps are large (a
    // large share of the voxels sampled) N loses its conditioning within a
    // pass, and so do B = U N and the Gram matrices built from it.  When
    // |N|_F |N^{-1}|_F / r (1 for N = I) exceeds kRefresh, B <- B N^{-1} = U
    // over all v rows (each workgroup a share) and N <- I: the subspace and
    // the step are unchanged.
    if (i > 0) {
      if (sqrt(sv.nf2[0] * sv.nf2[1]) > kRefresh * r) {
        float* Md = H;  // N^{-1}, r x r
#pragma unroll
        for (int ii = 0; ii < 8; ++ii)
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (rbase + ii < r && 8 * cb + j < r) Md[(rbase + ii) * r + 8 * cb + j] = nin[ii][j];
        __syncthreads();
        const int64_t lo = a.v * wg / nwg, hi = a.v * (wg + 1) / nwg;
#pragma unroll 1
        for (int64_t b0 = lo; b0 < hi; b0 += kCoopSlice) {
          const int nr = static_cast<int>(min(static_cast<int64_t>(kCoopSlice), hi - b0));
#pragma unroll
          for (int u = 0; u < kCoopSlice / 16; ++u) {
            const int row = rg + 16 * u;
            if (row < nr)
              for (int c = rl; c < r; c += 16) rows[row * rs + c] = a.B[(b0 + row) * r + c];
          }
          __syncthreads();
          // thread (row, chunk): columns 16 chunk .. + 15 of one row
          const int row = tid >> 3, c0 = 16 * (tid & 7);
          if (row < nr && c0 < r) {
            float o[16];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) o[jj] = 0.0f;
#pragma unroll 1
            for (int ii = 0; ii < r; ++ii) {
              const float bv = rows[row * rs + ii];
#pragma unroll
              for (int jj = 0; jj < 16; ++jj) o[jj] = fmaf(bv, Md[ii * r + min(c0 + jj, r - 1)], o[jj]);
            }
#pragma unroll
            for (int jj = 0; jj < 16; ++jj)
              if (c0 + jj < r) a.B[(b0 + row) * r + c0 + jj] = o[jj];
          }
          __syncthreads();
        }
        identity();
        target += nwg;
        if (!(alive = coop_barrier(ctr, target, ca.abort, flag))) break;
      }
    }
    // ---------------------------------------------------------- 1. gather
    // local row lq = 32 m + j is sampled row q = 32 (wg + nwg m) + j
    // (the index and the value of a sampled row are read together: the
    // values were gathered into set order before the pass)
    const int32_t* om = a.omega + static_cast<int64_t>(i) * k;
    const float* xi = a.xo + static_cast<int64_t>(i) * k;
    for (int lq = tid; lq < kCoopSlice * nsl; lq += kGT) {
      const int q = kCoopSlice * (wg + nwg * (lq / kCoopSlice)) + lq % kCoopSlice;
      const int64_t vox = q < k ? om[q] : -1;
      const float xv = q < k ? xi[q] : 0.0f;
      const int vx = (vox >= 0 && vox < a.v) ? static_cast<int>(vox) : -1;
      svox[lq] = vx;
      se[lq] = vx >= 0 ? xv : 0.0f;  // x_q, later the residual
    }
    __syncthreads();
    // rows into LDS as [B_q | x_q | 0 ...] up to column 16 RB (rows out of
    // range: zeros); lane rl of a row group covers columns 4 rl + 64 h .. + 3
    constexpr int NCH = (16 * RB + 63) / 64;
#pragma unroll 1
    for (int m = 0; m < nsl; ++m) {
#pragma unroll
      for (int u = 0; u < kCoopSlice / 16; ++u) {
        const int lq = kCoopSlice * m + rg + 16 * u;
        const int vx = svox[lq];
        const float xq = se[lq];
        const float* br = a.B + static_cast<int64_t>(vx >= 0 ? vx : 0) * r;
        float* lr = rows + lq * rs;
        f32x4 b4[NCH];
#pragma unroll
        for (int hh = 0; hh < NCH; ++hh) {
          const int c0 = 4 * rl + 64 * hh;
          if (vec) {
            b4[hh] = *reinterpret_cast<const f32x4*>(br + min(c0, r - 4));  // clamped: always issued
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) b4[hh][e] = br[min(c0 + e, r - 1)];
          }
        }
#pragma unroll
        for (int hh = 0; hh < NCH; ++hh) {
          const int c0 = 4 * rl + 64 * hh;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int c = c0 + e;
            if (c < 16 * RB) lr[c] = (vx >= 0 && c < r) ? b4[hh][e] : (c == r ? xq : 0.0f);
          }
        }
      }
    }
    __syncthreads();
    // ---------------------------------------------------------- 2. partial Gram
    {
      f32x4 acc[NTW];
#pragma unroll
      for (int j = 0; j < NTW; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
      auto slices = [&](auto G) {
        constexpr int g = decltype(G)::value;
#pragma unroll 1
        for (int m = 0; m < nsl; ++m) {
#pragma unroll
          for (int st = 0; st < kCoopSlice / 4; ++st) {
            float x[RB];
#pragma unroll
            for (int b = 0; b < RB; ++b) x[b] = rows[(kCoopSlice * m + 4 * st + kq) * rs + 16 * b + c16];
            gram_products<RB, TG, g>(acc, x);
          }
        }
        float* pw = ca.part + static_cast<size_t>(wg) * NT * 256;
#pragma unroll
        for (int t = g; t < NT; t += TG) *reinterpret_cast<f32x4*>(pw + t * 256 + 4 * lane) = acc[t / TG];
      };
      // wave w takes the tiles t = w mod 4
      if (wave == 0)
        slices(std::integral_constant<int, 0>());
      else if (wave == 1)
        slices(std::integral_constant<int, 1>());
      else if (wave == 2)
        slices(std::integral_constant<int, 2>());
      else
        slices(std::integral_constant<int, 3>());
    }
    target += nwg;
    if (!(alive = coop_barrier(ctr, target, ca.abort, flag))) break;
    // ---------------------------------------------------------- 3. sum a share of the tiles
    // This workgroup's share: 16-byte quads q0 .. q1 of the NT * 256 entries.
    // Every (partial, quad) load goes out at once and lands in LDS (the H
    // region is free); each entry is then added in workgroup order.
    {
      constexpr int E4 = NT * 64;
      const int q0 = E4 * wg / nwg, q1 = E4 * (wg + 1) / nwg, nq = q1 - q0;
      f32x4* stage = reinterpret_cast<f32x4*>(H);
      const int nl = nq * nwg;
      constexpr int LPT = (E4 + kCoopMaxWg + kGT - 1) / kGT;  // loads per thread, at most
      const float inq = 1.0f / static_cast<float>(nq);
#pragma unroll
      for (int m = 0; m < LPT; ++m) {
        const int L = tid + kGT * m;
        if (L < nl) {
          // L / nq (exact: L < 2^12 and the quotient is rounded down from
          // within 2^-10 of an integer)
          const int p = static_cast<int>((static_cast<float>(L) + 0.5f) * inq), qq = L - p * nq;
          stage[L] = *reinterpret_cast<const f32x4*>(ca.part + (static_cast<size_t>(p) * E4 + q0 + qq) * 4);
        }
      }
      __syncthreads();
      const float* st = reinterpret_cast<const float*>(stage);
      for (int x = tid; x < 4 * nq; x += kGT) {
        const int qq = x >> 2, j = x & 3;
        float t = 0.0f;
        for (int p = 0; p < nwg; ++p) t += st[4 * (p * nq + qq) + j];
        ca.hred[4 * (q0 + qq) + j] = t;
      }
    }
    target += nwg;
    if (!(alive = coop_barrier(ctr, target, ca.abort, flag))) break;
    // the summed tiles into H (lower tiles; element e of tile t is row
    // 16 bi + 4 (l / 16) + e % 4, column 16 bj + l % 16, l = (e % 256) / 4)
    {
      constexpr int NE = (NT * 64 + kGT - 1) / kGT, NB4 = NE < 4 ? NE : 4;
#pragma unroll
      for (int m0 = 0; m0 < NE; m0 += NB4) {
        f32x4 v4[NB4];
#pragma unroll
        for (int m = 0; m < NB4; ++m) {
          const int e4 = min(tid + kGT * (m0 + m), NT * 64 - 1);
          v4[m] = *reinterpret_cast<const f32x4*>(ca.hred + 4 * e4);
        }
#pragma unroll
        for (int m = 0; m < NB4; ++m) {
          const int e4 = tid + kGT * (m0 + m);
          if (e4 < NT * 64) {
            const int t = e4 >> 6, l = e4 & 63;
            const int bi = static_cast<int>((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
            const int bj = t - bi * (bi + 1) / 2;
#pragma unroll
            for (int e = 0; e < 4; ++e) H[(16 * bi + 4 * (l >> 4) + e) * hld + 16 * bj + (l & 15)] = v4[m][e];
            // and the mirrored entries, so that H is stored whole
            if (bi != bj) *reinterpret_cast<f32x4*>(H + (16 * bj + (l & 15)) * hld + 16 * bi + 4 * (l >> 4)) = v4[m];
          }
        }
      }
    }
    __syncthreads();
    // ---------------------------------------------------------- 4. H z = b (every workgroup)
    int cg_fail = 0;
    double ee = 0.0;  // |e|^2, or |Gamma|^2 for the l1 fit
    if (MODE == 0) {
      // ---------------------------------------------------------- 4. H z = b (every workgroup)
      cg_fail = pcg_solve<hld, false>(H, r, sv, lane, wave, rbase, cb, myrow, owner, rowok, nullptr);
      // |e|^2 = x_O^T x_O - b^T z for the least-squares z, from H alone (row
      // r of H is [b^T, x_O^T x_O]): the same in every workgroup, so no
      // exchange is needed while the fit leaves at least a tenth of
      // |x_O|^2 (then the cancellation costs at most one digit of H's
      // FP32 sums); a closer fit sums the residuals across workgroups
      double xx, eef;
      {
        double t = 0.0;
        for (int j = lane; j < r; j += 64) t = fma(static_cast<double>(H[r * hld + j]), sv.zv[j], t);
        xx = static_cast<double>(H[r * hld + r]);
        eef = xx - wave_sum_dpp(t);
      }
      const bool exch = !(xx > 0.0 && eef >= 0.1 * xx);
      // ---------------------------------------------------------- 5. residuals of this slice
      {
        float zl[8];
  #pragma unroll
        for (int hh = 0; hh < 2; ++hh)
  #pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int c = 4 * rl + 64 * hh + e;
            zl[4 * hh + e] = c < r ? sv.zf[c] : 0.0f;
          }
        double ee = 0.0;
  #pragma unroll 1
        for (int lq = rg; lq < kCoopSlice * nsl; lq += 16) {
          const int q = lq;
          const float* lr = rows + q * rs;
          float t = 0.0f;
  #pragma unroll
          for (int hh = 0; hh < 2; ++hh)
  #pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int c = 4 * rl + 64 * hh + e;
              t = fmaf(lr[min(c, 16 * RB - 1)], zl[4 * hh + e], t);  // zl is zero from r on
            }
          const float d = row16_sum_f(t);
          if (rl == 0) {
            const float e = svox[q] >= 0 ? lr[r] - d : 0.0f;
            se[q] = e;
            ee += static_cast<double>(e) * e;
          }
        }
        if (exch) {
          ee = wave_sum_dpp(ee);
          if (lane == 0) sv.red[3][wave] = ee;
        }
        __syncthreads();  // the residuals se[] are in
        if (exch && tid == 0) {
          double t = 0.0;
  #pragma unroll
          for (int w = 0; w < kGWaves; ++w) t += sv.red[3][w];
          ca.epart[wg] = t;
        }
      }
      if (exch) {
        target += nwg;
        if (!(alive = coop_barrier(ctr, target, ca.abort, flag))) break;
        for (int p = 0; p < nwg; ++p) ee += ca.epart[p];
      } else {
        ee = eef;
      }
      obj += ee;
    } else {
      // ---------------------------------------------------------- 4'. the l1 fit (ADMM)
      // On this workgroup's rows x_q (column r of the row cache), s_q and
      // lam_q; every iteration solves H z = B_O^T (x - s - lam / rho) (the
      // right-hand side summed over the workgroups, the solve warm-started),
      // then s <- shrink(x - B_O z - lam / rho, 1 / rho), lam <- lam +
      // rho (B_O z + s - x).  A final solve gives the z whose gradient Gamma
      // = lam + rho (B_O z + s - x) is orthogonal to the basis.
      const float rho = ca.rho, irho = 1.0f / ca.rho;
      const int K = ca.admm_iters, nrow = kCoopSlice * nsl;
      for (int q = tid; q < nrow; q += kGT) {
        ss[q] = 0.0f;
        sl[q] = 0.0f;
      }
      if (tid < kGR) sv.zv[tid] = 0.0;
      __syncthreads();
      double gg = 0.0, mis = 0.0;
#pragma unroll 1
      for (int it = 0; it <= K; ++it) {
        for (int q = tid; q < nrow; q += kGT) st[q] = svox[q] >= 0 ? rows[q * rs + r] - ss[q] - sl[q] * irho : 0.0f;
        __syncthreads();
        if (tid < kGR) {
          float g = 0.0f;
          if (tid < r)
            for (int q = 0; q < nrow; ++q) g = fmaf(rows[q * rs + tid], st[q], g);
          ca.gpart[wg * kGR + tid] = g;
        }
        target += nwg;
        if (!(alive = coop_barrier(ctr, target, ca.abort, flag))) break;
        if (tid < kGR) {
          double g = 0.0;
          for (int p = 0; p < nwg; ++p) g += ca.gpart[p * kGR + tid];
          sv.gv[tid] = tid < r ? g : 0.0;
        }
        __syncthreads();
        cg_fail |= pcg_solve<hld, true>(H, r, sv, lane, wave, rbase, cb, myrow, owner, rowok, sv.gv);
        float zl[8];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int c = 4 * rl + 64 * hh + e;
            zl[4 * hh + e] = c < r ? sv.zf[c] : 0.0f;
          }
#pragma unroll 1
        for (int q = rg; q < nrow; q += 16) {
          const float* lr = rows + q * rs;
          float t = 0.0f;
#pragma unroll
          for (int hh = 0; hh < 2; ++hh)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int c = 4 * rl + 64 * hh + e;
              t = fmaf(lr[min(c, 16 * RB - 1)], zl[4 * hh + e], t);  // zl is zero from r on
            }
          const float f = row16_sum_f(t);
          if (rl == 0) {
            const bool ok = svox[q] >= 0;
            const float xq = lr[r];
            if (it < K) {
              if (ok) {
                const float d = xq - f - sl[q] * irho;
                const float sq = copysignf(fmaxf(fabsf(d) - irho, 0.0f), d);
                ss[q] = sq;
                sl[q] = fmaf(rho, f + sq - xq, sl[q]);
              }
            } else {
              const float g = ok ? fmaf(rho, f + ss[q] - xq, sl[q]) : 0.0f;
              se[q] = -g;  // the step moves along -Gamma
              gg += static_cast<double>(g) * g;
              mis += ok ? fabs(static_cast<double>(xq) - f) : 0.0;
            }
          }
        }
        __syncthreads();
      }
      if (!alive) break;
      gg = wave_sum_dpp(gg);
      mis = wave_sum_dpp(mis);
      if (lane == 0) {
        sv.red[2][wave] = gg;
        sv.red[3][wave] = mis;
      }
      __syncthreads();
      if (tid == 0) {
        double a2 = 0.0, a3 = 0.0;
#pragma unroll
        for (int w = 0; w < kGWaves; ++w) {
          a2 += sv.red[2][w];
          a3 += sv.red[3][w];
        }
        ca.epart[2 * wg] = a2;
        ca.epart[2 * wg + 1] = a3;
      }
      target += nwg;
      if (!(alive = coop_barrier(ctr, target, ca.abort, flag))) break;
      double misfit = 0.0;
      for (int p = 0; p < nwg; ++p) {
        ee += ca.epart[2 * p];
        misfit += ca.epart[2 * p + 1];
      }
      obj += misfit;
    }
    // ---------------------------------------------------------- 6. w = N z, the angle
    {
      double zc[8], wp[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) zc[j] = sv.zv[8 * cb + j];
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) t = fma(static_cast<double>(nreg[ii][j]), zc[j], t);
        wp[ii] = t;
      }
      const double wrow = row16_reduce_scatter8(wp, cb);
      if (owner) sv.wv[myrow] = wrow;
      const double ww = wave_sum_dpp(owner ? wrow * wrow : 0.0);
      if (lane == 0) sv.red[0][wave] = ww;
    }
    __syncthreads();
    double nw2 = 0.0;
#pragma unroll
    for (int w = 0; w < kGWaves; ++w) nw2 += sv.red[0][w];
    const double nw = sqrt(nw2);
    const double ne = sqrt(ee);
    double cth = 1.0, sth = 0.0;
    if (nw > 0.0 && ne > 0.0 && !cg_fail) {
      if (MODE == 1) {
        // the geodesic step along -Gamma w^T: angle eta |Gamma| |w|
        const double th = fmin(static_cast<double>(a.gamma) * ne * nw, 0.5 * M_PI);
        cth = cos(th);
        sth = sin(th);
      } else if (a.gamma == 1.0f) {
        const double hyp = sqrt(nw2 + ee);
        cth = nw / hyp;
        sth = ne / hyp;
      } else {
        const double th = static_cast<double>(a.gamma) * atan(ne / nw);
        cth = cos(th);
        sth = sin(th);
      }
    }
    if (sth != 0.0 && fabs(cth) > 1e-12) {
      // ---------------------------------------------------------- 7. u = N^T wh, N, this slice's rows
      const double inw = 1.0 / nw;
      double whv[8];
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) whv[ii] = sv.wv[rbase + ii] * inw;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        double t = 0.0;
#pragma unroll
        for (int ii = 0; ii < 8; ++ii) t = fma(static_cast<double>(nreg[ii][j]), whv[ii], t);
        upart[(4 * wave + rq) * kGR + 8 * cb + j] = t;
      }
      {
        // N^{-1} wh at this lane's rows, reduce-scattered onto the row owners
        double whc[8], mp[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) whc[j] = sv.wv[8 * cb + j] * inw;
#pragma unroll
        for (int ii = 0; ii < 8; ++ii) {
          double t = 0.0;
#pragma unroll
          for (int j = 0; j < 8; ++j) t = fma(static_cast<double>(nin[ii][j]), whc[j], t);
          mp[ii] = t;
        }
        const double mrow = row16_reduce_scatter8(mp, cb);
        if (owner) sv.mw[myrow] = mrow;
      }
      __syncthreads();
      if (tid < kGR) {
        double t = 0.0;
#pragma unroll
        for (int p = 0; p < 4 * kGWaves; ++p) t += upart[p * kGR + tid];
        const bool own = tid < r;
        sv.uu[tid] = own ? t : 0.0;
        sv.qf[tid] = own ? static_cast<float>(t / cth) : 0.0f;
      }
      __syncthreads();
      {
        double u2 = 0.0, m2 = 0.0;
        for (int j = lane; j < r; j += 64) {
          u2 = fma(sv.uu[j], sv.uu[j], u2);
          m2 = fma(sv.mw[j], sv.mw[j], m2);
        }
        u2 = wave_sum_dpp(u2);
        m2 = wave_sum_dpp(m2);
        const double a1 = 1.0 / cth - 1.0;
        if (tid == 0) {
          sv.nf2[0] += (2.0 * a1 + a1 * a1) * u2;
          sv.nf2[1] += (cth * cth - 1.0) * m2;
        }
      }
      const float fi = static_cast<float>(1.0 / cth - 1.0);
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) {
        const float fw = fi * static_cast<float>(whv[ii]);
#pragma unroll
        for (int j = 0; j < 8; ++j) nreg[ii][j] = fmaf(fw, static_cast<float>(sv.uu[8 * cb + j]), nreg[ii][j]);
      }
      // N^{-1} <- N^{-1} (I + (c - 1) wh wh^T)
      const double cm1 = cth - 1.0;
#pragma unroll
      for (int ii = 0; ii < 8; ++ii) {
        const float fm = static_cast<float>(cm1 * sv.mw[rbase + ii]);
#pragma unroll
        for (int j = 0; j < 8; ++j) nin[ii][j] = fmaf(fm, static_cast<float>(sv.wv[8 * cb + j] * inw), nin[ii][j]);
      }
      const float gs = static_cast<float>(sth / ne);
      float ql[8];
#pragma unroll
      for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int c = 4 * rl + 64 * hh + e;
          ql[4 * hh + e] = c < r ? sv.qf[c] : 0.0f;
        }
#pragma unroll 2
      for (int q = rg; q < kCoopSlice * nsl; q += 16) {
        const int vx = svox[q];
        if (vx < 0) continue;
        const float ge = gs * se[q];
        const float* lr = rows + q * rs;
        float* br = a.B + static_cast<int64_t>(vx) * r;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int c0 = 4 * rl + 64 * hh;
          if (vec) {
            if (c0 + 4 <= r) {
              f32x4 t4;
#pragma unroll
              for (int e = 0; e < 4; ++e) t4[e] = fmaf(ge, ql[4 * hh + e], lr[c0 + e]);
              *reinterpret_cast<f32x4*>(br + c0) = t4;
            }
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (c0 + e < r) br[c0 + e] = fmaf(ge, ql[4 * hh + e], lr[c0 + e]);
          }
        }
      }
    }
    if (wg == 0 && tid == 0) a.info[i] = cg_fail ? -cg_fail : 0;
    target += nwg;
    if (!(alive = coop_barrier(ctr, target, ca.abort, flag))) break;
  }

  if (wg == 0 && tid == 0) {
    const int slot = a.pass & 1;
    if (!alive) {
      *a.stop = a.pass;  // a barrier wait expired: no further passes
      a.info[0] = -3;
    }
    a.objr[slot] = obj;
    if (a.obj_out) a.obj_out[a.pass] = obj;
    *a.used = a.pass + 1;
    if (alive && a.pass >= 1 && a.tol > 0.0) {
      const double prev = a.objr[slot ^ 1];
      if (prev - obj <= a.tol * prev) *a.stop = a.pass;
    }
  }
}

// the sampled values of a pass in set order, xo[i][q] = T[i][omega[i][q]]
// (0 for an index out of range); skipped once tracking has converged
__global__ __launch_bounds__(kBlock) void grouse_xo_kernel(const float* __restrict__ T, int64_t ldT,
                                                           const int32_t* __restrict__ omega, int64_t n,
                                                           int k, int64_t v, float* __restrict__ xo,
                                                           const int32_t* stop, int pass) {
  if (*stop < pass) return;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(kBlock) + threadIdx.x; t < n;
       t += static_cast<int64_t>(gridDim.x) * kBlock) {
    const int64_t i = t / k, vox = omega[t];
    xo[t] = (vox >= 0 && vox < v) ? T[i * ldT + vox] : 0.0f;
  }
}

__global__ void grouse_init_kernel(int32_t* stop, int32_t* used, double* objr, double* obj_out, int passes,
                                   uint32_t* ctr, int32_t* abort) {
  if (threadIdx.x == 0) {
    *stop = 0x7FFFFFFF;
    *used = 0;
    objr[0] = 0.0;
    objr[1] = 0.0;
    ctr[0] = 0u;
    ctr[1] = 0u;
    *abort = 0;
  }
  if (obj_out)
    for (int p = threadIdx.x; p < passes; p += blockDim.x) obj_out[p] = 0.0;
}

template <int RB, int MODE>
rpt_status launch_coop_m(const CoopArgs& ca, size_t smem, hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&grouse_coop_kernel<RB, MODE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsMax));
    attr = true;
  }
  hipLaunchKernelGGL((grouse_coop_kernel<RB, MODE>), dim3(ca.nwg), dim3(kGT), smem, s, ca);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}
template <int RB>
rpt_status launch_coop(const CoopArgs& ca, int mode, size_t smem, hipStream_t s) {
  return mode == 1 ? launch_coop_m<RB, 1>(ca, smem, s) : launch_coop_m<RB, 0>(ca, smem, s);
}

}  // namespace

size_t grouse_bytes(int r, int k, int ell) {
  Carver c(nullptr);
  c.take<float>(static_cast<size_t>(ell) * k);
  const size_t nt = static_cast<size_t>(g_rb(r)) * (g_rb(r) + 1) / 2;
  c.take<float>(static_cast<size_t>(kCoopMaxWg) * nt * 256);
  c.take<float>(nt * 256);
  c.take<double>(2 * kCoopMaxWg);
  c.take<float>(static_cast<size_t>(kCoopMaxWg) * kGR);
  c.take<double>(2);
  c.take<int32_t>(3);
  c.take<uint32_t>(2);
  c.take<int32_t>(1);
  return c.off;
}

GrouseState grouse_carve(void* ws, int r, int k, int ell) {
  Carver c(ws);
  GrouseState g;
  g.xo = c.take<float>(static_cast<size_t>(ell) * k);
  const size_t nt = static_cast<size_t>(g_rb(r)) * (g_rb(r) + 1) / 2;
  g.part = c.take<float>(static_cast<size_t>(kCoopMaxWg) * nt * 256);
  g.hred = c.take<float>(nt * 256);
  g.epart = c.take<double>(2 * kCoopMaxWg);
  g.gpart = c.take<float>(static_cast<size_t>(kCoopMaxWg) * kGR);
  g.objr = c.take<double>(2);
  int32_t* flags = c.take<int32_t>(3);
  g.stop = flags;
  g.used_ws = flags ? flags + 1 : nullptr;
  g.rinfo = flags ? flags + 2 : nullptr;
  g.ctr = c.take<uint32_t>(2);
  g.abort = c.take<int32_t>(1);
  return g;
}

rpt_status grouse_init_launch(const GrouseState& g, int32_t* used, double* obj_out, int passes, hipStream_t s) {
  hipLaunchKernelGGL(grouse_init_kernel, dim3(1), dim3(256), 0, s, g.stop, used ? used : g.used_ws, g.objr, obj_out,
                     passes, g.ctr, g.abort);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status grouse_pass_launch(const GrouseState& g, float* B, int64_t v, int r, const float* T, int64_t ldT,
                              const int32_t* omega, int k, int ell, float gamma, int pass, double tol,
                              double* obj_out, int32_t* used, int32_t* info, const TrackOpts& opt, hipStream_t s) {
  if (r < 1 || r > kGR || k < 1) return RPT_ERR_UNSUPPORTED;
  const int mode = opt.mode == RPT_TRACK_L1 ? 1 : 0;
  CoopArgs ca;
  ca.gpart = g.gpart;
  ca.rho = opt.rho;
  ca.admm_iters = opt.admm_iters;
  GrouseArgs& a = ca.g;
  a.B = B;
  a.v = v;
  a.r = r;
  a.T = T;
  a.ldT = ldT;
  a.omega = omega;
  a.xo = g.xo;
  a.k = k;
  a.ell = ell;
  a.gamma = gamma;
  a.objr = g.objr;
  a.obj_out = obj_out;
  a.pass = pass;
  a.stop = g.stop;
  a.used = used ? used : g.used_ws;
  a.tol = tol;
  a.info = info;
  ca.part = g.part;
  ca.hred = g.hred;
  ca.epart = g.epart;
  ca.ctr = g.ctr;
  ca.abort = g.abort;
  // one slice of 32 sampled rows per workgroup up to 64 slices, then more
  // slices per workgroup while their rows fit in LDS
  const int nslices = (k + kCoopSlice - 1) / kCoopSlice;
  ca.nwg = nslices < kCoopMaxWg ? nslices : kCoopMaxWg;
  ca.spw = (nslices + ca.nwg - 1) / ca.nwg;
  const size_t smem = coop_lds(r, ca.spw);
  if (smem > kLdsMax) return RPT_ERR_UNSUPPORTED;
  {
    const int64_t n = static_cast<int64_t>(ell) * k;
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(grouse_xo_kernel, dim3(static_cast<unsigned>(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s, T,
                       ldT, omega, n, k, v, g.xo, g.stop, pass);
    RPT_CHECK_LAUNCH();
  }
  RPT_STAGE("track_grouse", s);
  switch (g_rb(r)) {
    case 1: return launch_coop<1>(ca, mode, smem, s);
    case 2: return launch_coop<2>(ca, mode, smem, s);
    case 3: return launch_coop<3>(ca, mode, smem, s);
    case 4: return launch_coop<4>(ca, mode, smem, s);
    case 5: return launch_coop<5>(ca, mode, smem, s);
    case 6: return launch_coop<6>(ca, mode, smem, s);
    case 7: return launch_coop<7>(ca, mode, smem, s);
    case 8: return launch_coop<8>(ca, mode, smem, s);
    default: return launch_coop<9>(ca, mode, smem, s);
  }
}

}  // namespace rpt
