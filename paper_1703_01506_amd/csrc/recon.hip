// K7 -- reconstruction + residual noise + column maximum (Alg. 2, recovery):
//     m_i = max_k ( (U w_i)_k + sigma z(seed, stream, col0 + i, k) ) + mu
// without forming U W.
//
// Filter: a 1-pass BF16 matrix-core contraction of W (relabelling x r, operand
// A, held in registers) with U (r x voxel, operand B, K-blocked BF16 layout)
// keeps, per accumulator register, the running maximum of the approximate
// reconstruction over the voxels a lane visits.  A "stream" is the set of
// voxels {32 t + c : t in chunk} seen by lane column c of one voxel chunk; the
// kernel writes one maximum per (relabelling, chunk, c).
//
// Refine (exact pruning): with M the largest approximate value of column i,
// delta_i a proven bound on |approx - exact| (BF16 rounding of both operands
// plus FP32 accumulation, times max_k |U_k| |w_i|), and |z| < Z (the uniform
// map never returns less than 2^-25, so |z| <= sqrt(50 ln 2) < 5.8872), a voxel
// can attain the noisy maximum only if its exact value is within
// 2 Z sigma of the exact maximum, i.e. only if its stream maximum is at least
// M - 2 Z sigma - 2 delta_i.  Those streams are recomputed in FP32 (r FMAs per
// voxel) with their Philox4x32-10 / Box-Muller draw; every other voxel is
// provably irrelevant to the maximum.
#include "rpt_internal.h"
#include "philox.h"

namespace rpt {

namespace {

constexpr int kRMaxRefine = 128;  // basis rank held in LDS by the refine

// max(a, b) in one v_max_f32: the library's fmaxf first quiets a possible
// NaN in an operand it cannot prove canonical (one more instruction per
// element in the running maxima below, whose inputs are never NaN)
__device__ __forceinline__ float vmax(float a, float b) {
  float r;
  asm("v_max_f32 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
}

// ---------------------------------------------------------------- U preparation
// ukb [ks][vpad][2][16] bf16: hi(U[k][16s+e]) then lo(...), zero past r and v;
// umax >= max_k |U_k|_2
__global__ void recon_init_kernel(unsigned* umax_bits) { *umax_bits = 0u; }

// 64 voxels per workgroup: the rows (64 r contiguous floats) are read with
// coalesced loads into LDS, then thread (voxel, quarter) converts one
// 16-byte chunk (hi 0-7, hi 8-15, lo 0-7 or lo 8-15) of every K step.  The
// largest row norm goes out with one atomic per workgroup.
constexpr int kPrepUVox = 64;
__global__ __launch_bounds__(kBlock) void recon_prep_u_kernel(const float* __restrict__ U, int64_t v, int r,
                                                             int64_t vpad, int ks, uint16_t* __restrict__ ukb,
                                                             unsigned* umax_bits) {
  __shared__ float rows[kPrepUVox][kRMaxRefine + 1];
  __shared__ float red[kBlock / 64];
  const int tid = threadIdx.x;
  const int64_t v0 = static_cast<int64_t>(blockIdx.x) * kPrepUVox;
  const int nv = static_cast<int>(v - v0 < kPrepUVox ? (v - v0 > 0 ? v - v0 : 0) : kPrepUVox);
  for (int idx = tid; idx < kPrepUVox * r; idx += kBlock) {
    const int rr = idx / r, c = idx - rr * r;
    rows[rr][c] = rr < nv ? U[(v0 + rr) * r + c] : 0.0f;
  }
  __syncthreads();
  const int rr = tid >> 2, q = tid & 3;  // voxel within the tile, chunk of 8 values
  const int64_t vox = v0 + rr;
  float nrm = 0.0f;
  if (vox < vpad) {
    for (int s = 0; s < ks; ++s) {
      uint32_t w[4];
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        uint32_t pr = 0;
#pragma unroll
        for (int hl = 0; hl < 2; ++hl) {
          const int c = 16 * s + 8 * (q & 1) + 2 * e2 + hl;
          const float x = c < r ? rows[rr][c] : 0.0f;
          if (q < 2) nrm = fmaf(x, x, nrm);
          const uint16_t hi = f2bf(x);
          const uint16_t val = (q < 2) ? hi : f2bf(x - bf2f(hi));
          pr |= static_cast<uint32_t>(val) << (16 * hl);
        }
        w[e2] = pr;
      }
      *reinterpret_cast<u32x4*>(ukb + (static_cast<size_t>(s) * vpad + vox) * 32 + 8 * q) =
          u32x4{w[0], w[1], w[2], w[3]};
    }
  }
  // row norm: the two hi quarters of a voxel hold its two halves
  nrm += __shfl_xor(nrm, 1, 64);
  nrm = wave_max(nrm);
  if ((tid & 63) == 0) red[tid >> 6] = nrm;
  __syncthreads();
  if (tid == 0)
    atomicMax(umax_bits, __float_as_uint(sqrtf(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]))) * 1.000001f));
}

// Path choice made on the device (sigma is a device value): exact pruning pays
// off only when the candidate band 2 Z sigma is narrow; otherwise every voxel
// needs its noise draw and the fused kernel draws them alongside the
// contraction.  Both paths compute the same maximum.
constexpr float kPruneBand = 0.5f;
__global__ void recon_decide_kernel(const float* sigma_mu, int* path) {
  *path = (2.0f * kZBound * sigma_mu[0] <= kPruneBand) ? 1 : 0;
}

// ---------------------------------------------------------------- filter
struct FilterArgs {
  const uint16_t* ukb;
  const float* W;
  int r, ks;
  int64_t v, vpad, vt, L;
  int tpc, pg, nc;
  float* smax;  // [L][nc * 32]
  const int* path;
};

template <int KS, int PT>
__global__ __launch_bounds__(kBlock) void recon_filter_kernel(FilterArgs a) {
  if (*a.path != 1) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
  const int b = blockIdx.x, xcd = b & 7, j = b >> 3;
  const int pg = j % a.pg;
  const int chunk = xcd + 8 * (j / a.pg);
  const int64_t pbase = static_cast<int64_t>(pg) * (4 * PT * 32) + static_cast<int64_t>(wave) * (PT * 32);

  // A fragments: lane supplies W[perm = col][16s + 8h + 0..7] in BF16
  u32x4 A[PT][KS];
#pragma unroll
  for (int p = 0; p < PT; ++p) {
    const int64_t perm = pbase + p * 32 + col;
    const bool valid = perm < a.L;
    const float* wr = a.W + (valid ? perm : 0) * a.r;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      unsigned w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c0 = 16 * s + 8 * h + 2 * q;
        const float x0 = (valid && c0 < a.r) ? wr[c0] : 0.0f;
        const float x1 = (valid && c0 + 1 < a.r) ? wr[c0 + 1] : 0.0f;
        w[q] = static_cast<unsigned>(f2bf(x0)) | (static_cast<unsigned>(f2bf(x1)) << 16);
      }
      A[p][s] = u32x4{w[0], w[1], w[2], w[3]};
    }
  }
  float rm[PT][16];
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) rm[p][e] = -INFINITY;

  const int64_t t0 = static_cast<int64_t>(chunk) * a.tpc;
  const int64_t t1 = t0 + a.tpc < a.vt ? t0 + a.tpc : a.vt;
  const size_t kstride = static_cast<size_t>(a.vpad) * 32;
  u32x4 Bc[KS], Bn[KS];
  auto load = [&](u32x4* B, int64_t t) {
    const uint16_t* bp = a.ukb + static_cast<size_t>(t * 32 + col) * 32 + h * 8;
#pragma unroll
    for (int s = 0; s < KS; ++s) B[s] = *reinterpret_cast<const u32x4*>(bp + s * kstride);
  };
  auto body = [&](const u32x4* B, int64_t t) {
    f32x16 acc[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) acc[p] = f32x16{};
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int p = 0; p < PT; ++p) acc[p] = mfma_bf16(A[p][s], B[s], acc[p]);
    if (t + 1 < a.vt) {
#pragma unroll
      for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int e = 0; e < 16; ++e) rm[p][e] = fmaxf(rm[p][e], acc[p][e]);
    } else {
      // last tile: padding voxels (past v) must not enter the maxima
      const bool ok = t * 32 + col < a.v;
#pragma unroll
      for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int e = 0; e < 16; ++e) rm[p][e] = ok ? fmaxf(rm[p][e], acc[p][e]) : rm[p][e];
    }
  };
  if (t0 < t1) load(Bc, t0);
  for (int64_t t = t0; t < t1; t += 2) {
    if (t + 1 < t1) load(Bn, t + 1);
    body(Bc, t);
    if (t + 1 >= t1) break;
    if (t + 2 < t1) load(Bc, t + 2);
    body(Bn, t + 1);
  }
  const int64_t ns = static_cast<int64_t>(a.nc) * 32;
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t perm = pbase + p * 32 + mfma_row(e, h);
      if (perm < a.L) a.smax[perm * ns + static_cast<int64_t>(chunk) * 32 + col] = rm[p][e];
    }
}

// ---------------------------------------------------------------- refine
struct RefineArgs {
  const int* path;
  const float* U;
  const float* W;
  int64_t v, vt, L;
  int r, tpc, nc;      // streams of the exact-pruning pass (path 1)
  int tpc_f, nc_f;     // streams of the fused pass (path 0)
  const float* smax;
  const unsigned* umax_bits;
  const float* sigma_mu;
  float eps;          // relative error bound of the filter
  uint64_t seed;
  unsigned stream;
  int64_t col0;
  float* out;         // [L] max + mu
  const float* tmax;  // optional: exact training maxima (mean-gap rule)
  float* gap;         // optional: [L] tmax - max(U w + s)
  unsigned study;     // study id of the noise counter
};

__global__ __launch_bounds__(kBlock) void recon_refine_kernel(RefineArgs a) {
  const int path = *a.path;
  __shared__ float wsh[4][kRMaxRefine];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 4 + wave;
  if (i >= a.L) return;
  const float sigma = a.sigma_mu[0];
  const float mu = a.sigma_mu[1];
  float* w = wsh[wave];
  float wn = 0.0f;
  for (int c = lane; c < a.r; c += 64) {
    const float x = a.W[i * a.r + c];
    w[c] = x;
    wn = fmaf(x, x, wn);
  }
  wn = sqrtf(wave_sum(wn));
  const float A = __uint_as_float(*a.umax_bits) * wn;  // >= |U_k w| for every voxel
  const bool vec = (a.r & 3) == 0 && (reinterpret_cast<uintptr_t>(a.U) & 15) == 0;
  const int nc = path == 0 ? a.nc_f : a.nc, tpc = path == 0 ? a.tpc_f : a.tpc;
  const int64_t ns = static_cast<int64_t>(nc) * 32;
  const float* sm = a.smax + i * ns;
  float M = -INFINITY;
  for (int64_t s = lane; s < ns; s += 64) M = fmaxf(M, sm[s]);
  M = wave_max(M);
  // path 1: stream maxima of U w alone, so the noise can move any value by
  // kZBound sigma; path 0: maxima of U w + sigma z (the same z as below), and
  // both this pass and the bound pass round the noisy value once in FP32
  // (values below A (1 + eps) + kZBound sigma)
  const float tau = path == 0 ? M - 2.0f * (a.eps * A + 2.4e-7f * (A + kZBound * sigma))
                              : M - 2.0f * kZBound * sigma - 2.0f * a.eps * A;
  float best = -INFINITY;
  for (int64_t s0 = 0; s0 < ns; s0 += 64) {
    const bool cand = (s0 + lane < ns) && sm[s0 + lane] >= tau;
    uint64_t mask = __ballot(cand);
    while (mask) {
      const int bit = __ffsll(static_cast<unsigned long long>(mask)) - 1;
      mask &= mask - 1;
      const int64_t stream_id = s0 + bit;
      const int64_t chunk = stream_id >> 5;
      const int colc = static_cast<int>(stream_id & 31);
      const int64_t t0 = chunk * tpc;
      const int64_t t1 = t0 + tpc < a.vt ? t0 + tpc : a.vt;
      // 64 voxels of the stream at a time, one per lane: the lane draws its
      // voxel's noise and dots the voxel's basis row with w (w broadcast from
      // LDS; the row's 16-byte loads are independent, so several stay in
      // flight per lane, and a stream of 81 voxels takes two rounds)
      for (int64_t tb = t0; tb < t1; tb += 64) {
        const int64_t tl = tb + lane, vox = tl * 32 + colc;
        if (tl < t1 && vox < a.v) {
          const float z = noise_z(a.seed, a.stream, static_cast<unsigned>(a.col0 + i), vox, a.study);
          const float* u = a.U + vox * a.r;
          float acc = 0.0f;
          if (vec) {
#pragma unroll 5
            for (int c = 0; c < a.r; c += 4) {
              const f32x4 x = *reinterpret_cast<const f32x4*>(u + c);
              acc = fmaf(x[0], w[c], acc);
              acc = fmaf(x[1], w[c + 1], acc);
              acc = fmaf(x[2], w[c + 2], acc);
              acc = fmaf(x[3], w[c + 3], acc);
            }
          } else {
            for (int c = 0; c < a.r; ++c) acc = fmaf(u[c], w[c], acc);
          }
          best = fmaxf(best, fmaf(sigma, z, acc));
        }
      }
    }
  }
  best = wave_max(best);
  if (lane == 0) {
    if (a.out) a.out[i] = best + mu;
    if (a.gap) a.gap[i] = a.tmax[i] - best;
  }
}

// ---------------------------------------------------------------- fused path
// One pass over every voxel: the reconstruction on the matrix cores in BF16
// (W and U rounded to BF16, FP32 accumulation), the exact noise of every
// element, and the running maximum of every stream (the voxels of one voxel
// column of the tiles of one chunk).  The BF16 products are within
// delta = eps |U_k| |w| of the FP32 value, so only the streams whose maximum
// comes within 2 delta (plus roundings) of the column's best stream can hold
// the maximum; recon_refine_kernel recomputes those in FP32 with the same
// noise.  Accumulator registers 4m..4m+3 of a lane hold four consecutive
// columns 4q..4q+3 at one voxel: exactly the four normals of one Philox call
// at counter (voxel, q, stream, 0).
struct FusedArgs {
  const uint16_t* ukb;
  const float* W;
  int r;
  int64_t v, vpad, vt, L;
  int tpc, pg, nc;
  int64_t col0;
  uint64_t seed;
  unsigned stream;
  const float* sigma_mu;
  const int* path;
  float* smax;  // [L][nc * 32] stream maxima of the bound values
  unsigned study;  // study id of the noise counter
};

__device__ __forceinline__ void box_muller4(const unsigned c[4], float z[4]) {
  const float r1 = bm_radius(c[0]), r2 = bm_radius(c[2]);
  const float t1 = bm_turns(c[1]), t2 = bm_turns(c[3]);
  z[0] = r1 * __builtin_amdgcn_cosf(t1);
  z[1] = r1 * __builtin_amdgcn_sinf(t1);
  z[2] = r2 * __builtin_amdgcn_cosf(t2);
  z[3] = r2 * __builtin_amdgcn_sinf(t2);
}

// One work item of the fused pass: permutation group j % pg and voxel chunk
// xcd + 8 (j / pg), so that every chunk of a study stays on one XCD (its U
// tiles are fetched into that XCD's L2 once for all permutation groups).
template <int KS, int PT, bool ALIGNED>
__device__ __forceinline__ void fused_item(const FusedArgs& a, int xcd, int j) {
  __shared__ __align__(16) uint16_t us[2][KS][64 * 8];
  typedef __attribute__((address_space(3))) void lds_void;
  typedef const __attribute__((address_space(1))) void gbl_void;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
  const int pg = j % a.pg;
  const int chunk = xcd + 8 * (j / a.pg);
  const int64_t pbase = static_cast<int64_t>(pg) * (4 * PT * 32) + static_cast<int64_t>(wave) * (PT * 32);
  const float sigma = a.sigma_mu[0];
  const unsigned k0 = static_cast<unsigned>(a.seed), k1 = static_cast<unsigned>(a.seed >> 32);

  u32x4 Ah[PT][KS];
#pragma unroll
  for (int p = 0; p < PT; ++p) {
    const int64_t perm = pbase + p * 32 + col;
    const bool valid = perm < a.L;
    const float* wr = a.W + (valid ? perm : 0) * a.r;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      unsigned wh[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t ph = 0;
#pragma unroll
        for (int hl = 0; hl < 2; ++hl) {
          const int c = 16 * s + 8 * h + 2 * q + hl;
          const float x = (valid && c < a.r) ? wr[c] : 0.0f;
          ph |= static_cast<uint32_t>(f2bf(x)) << (16 * hl);
        }
        wh[q] = ph;
      }
      Ah[p][s] = u32x4{wh[0], wh[1], wh[2], wh[3]};
    }
  }
  float rm[PT][16];
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) rm[p][e] = -INFINITY;

  const int64_t t0 = static_cast<int64_t>(chunk) * a.tpc;
  const int64_t t1 = t0 + a.tpc < a.vt ? t0 + a.tpc : a.vt;
  const size_t kstride = static_cast<size_t>(a.vpad) * 32;
  // The U tile of the current 32 voxels is shared by the four waves: it is
  // copied once per workgroup into LDS (double-buffered, global_load_lds),
  // already permuted so that lane l's 16-byte fragment sits at 16 l, and each
  // wave reads its fragments right before the products.
  auto issue = [&](int b, int64_t t) {
#pragma unroll
    for (int j = 0; j < KS; j += 4) {
      const int s = j + wave;
      if (s < KS) {
        const uint16_t* g = a.ukb + s * kstride + static_cast<size_t>(t * 32 + col) * 32 + h * 8;
        __builtin_amdgcn_global_load_lds((gbl_void*)g, (lds_void*)&us[b][s][0], 16, 0, 0);
      }
    }
  };
  auto body = [&](int b, int64_t t) {
    f32x16 acc[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) acc[p] = f32x16{};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const u32x4 bh = *reinterpret_cast<const u32x4*>(&us[b][s][lane * 8]);
#pragma unroll
      for (int p = 0; p < PT; ++p) acc[p] = mfma_bf16(Ah[p][s], bh, acc[p]);
    }
    const int64_t vox = t * 32 + col;
    const bool ok = vox < a.v;
    if (ALIGNED) {
#pragma unroll
      for (int p = 0; p < PT; ++p) {
        // the four calls of this column block, advanced together
        unsigned c[4][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int64_t g = a.col0 + pbase + p * 32 + 8 * m + 4 * h;  // column of register 4m
          c[m][0] = static_cast<unsigned>(vox);
          c[m][1] = static_cast<unsigned>(g >> 2);
          c[m][2] = a.stream;
          c[m][3] = a.study;
        }
        philox4x32_10_n<4>(c, k0, k1);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          float z[4];
          box_muller4(c[m], z);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const float val = fmaf(sigma, z[jj], acc[p][4 * m + jj]);
            rm[p][4 * m + jj] = vmax(rm[p][4 * m + jj], ok ? val : -INFINITY);
          }
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int64_t g = a.col0 + pbase + p * 32 + 8 * m + 4 * h;  // column of register 4m
          float z[4];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            z[jj] = noise_z(a.seed, a.stream, static_cast<unsigned>(g + jj), vox, a.study);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const float val = fmaf(sigma, z[jj], acc[p][4 * m + jj]);
            rm[p][4 * m + jj] = vmax(rm[p][4 * m + jj], ok ? val : -INFINITY);
          }
        }
    }
  };
  if (t0 < t1) issue(0, t0);
  for (int64_t t = t0; t < t1; ++t) {
    const int b = static_cast<int>((t - t0) & 1);
    // this wave's copies of tile t have landed; after the barrier every
    // wave's have, and every wave is done reading tile t - 1's buffer
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (t + 1 < t1) issue(b ^ 1, t + 1);
    body(b, t);
  }
  // the maximum of every stream (chunk, voxel column col): lane col holds it
  // for the 16 permutations of its accumulator rows
  const int64_t ns = static_cast<int64_t>(a.nc) * 32;
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int64_t perm = pbase + p * 32 + mfma_row(e, h);
      if (perm < a.L) a.smax[perm * ns + static_cast<int64_t>(chunk) * 32 + col] = rm[p][e];
    }
}

template <int KS, int PT, bool ALIGNED>
__global__ __launch_bounds__(kBlock, ALIGNED ? 3 : 2) void recon_fused_kernel(FusedArgs a) {
  if (*a.path != 0) return;
  fused_item<KS, PT, ALIGNED>(a, static_cast<int>(blockIdx.x & 7), static_cast<int>(blockIdx.x >> 3));
}

// ---------------------------------------------------------------- several studies
// The fused pass of up to kPersistMax studies in one persistent launch.  The
// work items of all studies form eight queues, one per XCD (item (study, j)
// of queue x is block 8 j + x of that study's own grid); workgroup b serves
// queue b % 8 through an atomic counter until the queue is empty, so every
// workgroup exits once all items are taken, and results equal the per-study
// launches exactly.  Studies share the launch's KS (smaller ranks are padded
// with zero U columns, whose products add exact zeros).
constexpr int kPersistMax = 16;
struct PersistTable {
  FusedArgs st[kPersistMax];
  int64_t items[kPersistMax];  // items per queue of each study (pg nc / 8)
  int ns;
  int64_t total;               // items per queue of all studies
  int* counters;               // [8], zero at launch
};

template <int KS, int PT, bool ALIGNED>
__global__ __launch_bounds__(kBlock, ALIGNED ? 3 : 2) void recon_fused_persistent_kernel(PersistTable t) {
  __shared__ int64_t item_s;
  const int x = static_cast<int>(blockIdx.x & 7);
  for (;;) {
    __syncthreads();  // the previous item's LDS reads are done; item_s is free
    if (threadIdx.x == 0) item_s = atomicAdd(t.counters + x, 1);
    __syncthreads();
    const int64_t it = item_s;
    if (it >= t.total) break;
    int q = 0;
    int64_t base = 0;
    while (q + 1 < t.ns && it >= base + t.items[q]) {
      base += t.items[q];
      ++q;
    }
    if (*t.st[q].path != 0) continue;  // this study takes the exact-pruning path
    fused_item<KS, PT, ALIGNED>(t.st[q], x, static_cast<int>(it - base));
  }
}

template <int PT, bool AL>
void* pick_fused(int ks) {
  switch (ks) {
    case 1: return reinterpret_cast<void*>(&recon_fused_kernel<1, PT, AL>);
    case 2: return reinterpret_cast<void*>(&recon_fused_kernel<2, PT, AL>);
    case 3: return reinterpret_cast<void*>(&recon_fused_kernel<3, PT, AL>);
    case 4: return reinterpret_cast<void*>(&recon_fused_kernel<4, PT, AL>);
    case 5: return reinterpret_cast<void*>(&recon_fused_kernel<5, PT, AL>);
    case 6: return reinterpret_cast<void*>(&recon_fused_kernel<6, PT, AL>);
    case 7: return reinterpret_cast<void*>(&recon_fused_kernel<7, PT, AL>);
    case 8: return reinterpret_cast<void*>(&recon_fused_kernel<8, PT, AL>);
    default: return nullptr;
  }
}

template <int PT>
void* pick_filter(int ks) {
  switch (ks) {
    case 1: return reinterpret_cast<void*>(&recon_filter_kernel<1, PT>);
    case 2: return reinterpret_cast<void*>(&recon_filter_kernel<2, PT>);
    case 3: return reinterpret_cast<void*>(&recon_filter_kernel<3, PT>);
    case 4: return reinterpret_cast<void*>(&recon_filter_kernel<4, PT>);
    case 5: return reinterpret_cast<void*>(&recon_filter_kernel<5, PT>);
    case 6: return reinterpret_cast<void*>(&recon_filter_kernel<6, PT>);
    case 7: return reinterpret_cast<void*>(&recon_filter_kernel<7, PT>);
    case 8: return reinterpret_cast<void*>(&recon_filter_kernel<8, PT>);
    default: return nullptr;
  }
}

struct ReconPlan {
  int ks, pt, pg, nc, tpc, nc_heur, nc_cap;
  int64_t vpad, vt;
};

constexpr int kFilterPT = 4, kFusedPT = 1;

// tuned: a measured chunk count of the fused kernel may replace the rule of
// thumb (force_nc > 0: the autotuner's trial)
ReconPlan recon_plan(int64_t v, int64_t L, int r, int pt, int force_nc = 0) {
  ReconPlan pl;
  pl.ks = static_cast<int>(ceil_div(r, 16));
  pl.pt = pt;
  pl.vpad = round_up(v, 32);
  pl.vt = pl.vpad / 32;
  const int64_t group = 4 * pl.pt * 32;
  pl.pg = static_cast<int>(ceil_div(L > 0 ? L : 1, group));
  int64_t nc = round_up(ceil_div(1280, pl.pg), 8);
  const int64_t ncmax = round_up(pl.vt, 8);
  if (nc > ncmax) nc = ncmax;
  if (nc < 8) nc = 8;
  pl.nc_heur = static_cast<int>(nc);
  pl.nc_cap = pt == kFusedPT ? static_cast<int>(chunk_cap(nc, ncmax)) : static_cast<int>(nc);
  if (pt == kFusedPT) {
    const int64_t pick = force_nc > 0 ? force_nc : tuned_chunks(kTuneRecon, v, L, r, 0);
    if (pick >= 8 && pick <= pl.nc_cap && pick % 8 == 0) nc = pick;
  }
  pl.nc = static_cast<int>(nc);
  pl.tpc = static_cast<int>(ceil_div(pl.vt, nc));
  return pl;
}

struct ReconBufs {
  uint16_t* ukb;
  float* smax;  // stream maxima of either pass
  unsigned* umax;
  int* path;
};

// ks: U slices of 16 columns in ukb (0: the rank's own ceil(r / 16))
ReconBufs recon_carve(Carver& c, int64_t v, int64_t L, int r, int ks) {
  const ReconPlan pf = recon_plan(v, L, r, kFilterPT);
  const ReconPlan pu = recon_plan(v, L, r, kFusedPT);
  ReconBufs b;
  b.ukb = c.take<uint16_t>(static_cast<size_t>(ks > pf.ks ? ks : pf.ks) * pf.vpad * 32);
  b.smax = c.take<float>(static_cast<size_t>(L > 0 ? L : 1) * (pf.nc > pu.nc_cap ? pf.nc : pu.nc_cap) * 32);
  b.umax = c.take<unsigned>(64);
  b.path = c.take<int>(64);
  return b;
}

// path decision and the BF16 hi/lo copy of U (ks slices)
rpt_status recon_prepare(const float* U, int64_t v, int r, int64_t L, const float* sigma_mu, int ks,
                         const ReconBufs& b, hipStream_t s) {
  const ReconPlan pl = recon_plan(v, L, r, kFilterPT);
  hipLaunchKernelGGL(recon_init_kernel, dim3(1), dim3(1), 0, s, b.umax);
  RPT_CHECK_LAUNCH();
  hipLaunchKernelGGL(recon_decide_kernel, dim3(1), dim3(1), 0, s, sigma_mu, b.path);
  RPT_CHECK_LAUNCH();
  hipLaunchKernelGGL(recon_prep_u_kernel, dim3(static_cast<unsigned>(ceil_div(pl.vpad, kPrepUVox))), dim3(kBlock), 0,
                     s, U, v, r, pl.vpad, ks, b.ukb, b.umax);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

FusedArgs fused_args(const ReconBufs& b, const float* W, int r, int64_t v, int64_t L, int64_t col0, uint64_t seed,
                     int stream_id, const float* sigma_mu, unsigned study, const ReconPlan& pu) {
  return FusedArgs{b.ukb, W,  r,           v,        pu.vpad, pu.vt,  L,       pu.tpc, pu.pg,
                   pu.nc, col0, seed, static_cast<unsigned>(stream_id), sigma_mu, b.path, b.smax, study};
}

// the exact-pruning pass (path 1 only), then the FP32 recomputation of the
// candidate streams of whichever pass ran
rpt_status recon_finish(const float* U, int64_t v, int r, const float* W, int64_t L, int64_t col0, uint64_t seed,
                        int stream_id, const float* sigma_mu, float* out_max, const float* Tmax_for_gap,
                        float* gap_out, int ks, const ReconBufs& b, const ReconPlan& pu, hipStream_t s,
                        unsigned study) {
  const ReconPlan pl = recon_plan(v, L, r, kFilterPT);
  // BF16 keeps 8 significant bits, so round-to-nearest moves each operand by
  // at most 2^-8 of itself and a product of two rounded operands by at most
  // (2 * 2^-8 + 2^-16) of the exact product; summed over the K terms that is
  // at most (2^-7 + 2^-16) |U_k| |w| (Cauchy-Schwarz).  FP32 accumulation in
  // the bound pass and in the exact pass adds K terms of 2^-24 each.
  const int kpad = 16 * ks;
  const float eps =
      static_cast<float>((ldexp(1.0, -7) + ldexp(1.0, -16) + 2.02 * (kpad + r) * ldexp(1.0, -24)) * 1.01);

  // exact-pruning path (runs when the device decided path 1)
  FilterArgs fa{b.ukb, W, r, ks, v, pl.vpad, pl.vt, L, pl.tpc, pl.pg, pl.nc, b.smax, b.path};
  void* fn = pick_filter<kFilterPT>(ks);
  if (!fn) return RPT_ERR_UNSUPPORTED;
  void* args[] = {&fa};
  hipError_t e;
  {
    RPT_STAGE("recon_filter", s);
    e = hipLaunchKernel(fn, dim3(static_cast<unsigned>(pl.pg) * pl.nc), dim3(kBlock), args, 0, s);
  }
  if (e != hipSuccess) {
    set_hip_error(e);
    return RPT_ERR_HIP;
  }
  RefineArgs ra;
  ra.path = b.path;
  ra.U = U;
  ra.W = W;
  ra.v = v;
  ra.vt = pl.vt;
  ra.L = L;
  ra.r = r;
  ra.tpc = pl.tpc;
  ra.nc = pl.nc;
  ra.tpc_f = pu.tpc;
  ra.nc_f = pu.nc;
  ra.smax = b.smax;
  ra.umax_bits = b.umax;
  ra.sigma_mu = sigma_mu;
  ra.eps = eps;
  ra.seed = seed;
  ra.stream = static_cast<unsigned>(stream_id);
  ra.col0 = col0;
  ra.out = out_max;
  ra.tmax = Tmax_for_gap;
  ra.gap = gap_out;
  ra.study = study;
  RPT_STAGE("recon_refine", s);
  hipLaunchKernelGGL(recon_refine_kernel, dim3(static_cast<unsigned>(ceil_div(L, 4))), dim3(kBlock), 0, s, ra);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

template <int PT, bool AL>
void* pick_persistent(int ks) {
  switch (ks) {
    case 1: return reinterpret_cast<void*>(&recon_fused_persistent_kernel<1, PT, AL>);
    case 2: return reinterpret_cast<void*>(&recon_fused_persistent_kernel<2, PT, AL>);
    case 3: return reinterpret_cast<void*>(&recon_fused_persistent_kernel<3, PT, AL>);
    case 4: return reinterpret_cast<void*>(&recon_fused_persistent_kernel<4, PT, AL>);
    case 5: return reinterpret_cast<void*>(&recon_fused_persistent_kernel<5, PT, AL>);
    case 6: return reinterpret_cast<void*>(&recon_fused_persistent_kernel<6, PT, AL>);
    case 7: return reinterpret_cast<void*>(&recon_fused_persistent_kernel<7, PT, AL>);
    case 8: return reinterpret_cast<void*>(&recon_fused_persistent_kernel<8, PT, AL>);
    default: return nullptr;
  }
}

}  // namespace

int recon_chunk_candidates(int64_t v, int64_t L, int r, int* out) {
  const ReconPlan pu = recon_plan(v, L, r, kFusedPT);
  return chunk_candidates(pu.nc_heur, round_up(pu.vt, 8), out);
}

size_t recon_bytes(int64_t v, int64_t L, int r, int ks) {
  Carver c(nullptr);
  (void)recon_carve(c, v, L, r, ks);
  return c.off;
}

rpt_status recon_launch(const float* U, int64_t v, int r, const float* W, int64_t L, int64_t col0, uint64_t seed,
                        int stream_id, const float* sigma_mu, float* out_max, const float* Tmax_for_gap,
                        float* gap_out, void* ws, hipStream_t s, unsigned study, int force_nc) {
  if (L == 0) return RPT_OK;
  if (r < 1 || r > kRMaxRefine) return RPT_ERR_UNSUPPORTED;
  Carver c(ws);
  const ReconBufs b = recon_carve(c, v, L, r, 0);
  const ReconPlan pu = recon_plan(v, L, r, kFusedPT, force_nc);
  RPT_STAGE("recon_total", s);
  RPT_TRY(recon_prepare(U, v, r, L, sigma_mu, pu.ks, b, s));
  FusedArgs ua = fused_args(b, W, r, v, L, col0, seed, stream_id, sigma_mu, study, pu);
  void* ufn = (col0 % 4 == 0) ? pick_fused<kFusedPT, true>(pu.ks) : pick_fused<kFusedPT, false>(pu.ks);
  if (!ufn) return RPT_ERR_UNSUPPORTED;
  void* uargs[] = {&ua};
  hipError_t e;
  {
    RPT_STAGE("recon_fused", s);
    e = hipLaunchKernel(ufn, dim3(static_cast<unsigned>(pu.pg) * pu.nc), dim3(kBlock), uargs, 0, s);
  }
  if (e != hipSuccess) {
    set_hip_error(e);
    return RPT_ERR_HIP;
  }
  return recon_finish(U, v, r, W, L, col0, seed, stream_id, sigma_mu, out_max, Tmax_for_gap, gap_out, pu.ks, b, pu,
                      s, study);
}

int recon_batch_ks(const ReconStudy* st, int ns) {
  int ks = 1;
  for (int q = 0; q < ns; ++q) {
    const int k = static_cast<int>(ceil_div(st[q].r, 16));
    if (k > ks) ks = k;
  }
  return ks;
}

size_t recon_batch_counters(int ns) { return 8 * static_cast<size_t>(ceil_div(ns > 0 ? ns : 1, kPersistMax)); }

rpt_status recon_prepare_study(const ReconStudy& st, int ks, hipStream_t s) {
  if (st.L == 0) return RPT_OK;
  if (st.r < 1 || st.r > kRMaxRefine || ks < 1 || ks > 8) return RPT_ERR_UNSUPPORTED;
  Carver c(st.ws);
  const ReconBufs b = recon_carve(c, st.v, st.L, st.r, ks);
  return recon_prepare(st.U, st.v, st.r, st.L, st.sigma_mu, ks, b, s);
}

rpt_status recon_batched(const ReconStudy* st, int ns, int ks, int* counters, hipStream_t s) {
  if (ks < 1 || ks > 8) return RPT_ERR_UNSUPPORTED;
  bool aligned = true;
  for (int q = 0; q < ns; ++q) aligned = aligned && (st[q].L == 0 || st[q].col0 % 4 == 0);
  void* fn = aligned ? pick_persistent<kFusedPT, true>(ks) : pick_persistent<kFusedPT, false>(ks);
  if (!fn) return RPT_ERR_UNSUPPORTED;
  // a resident grid: three (aligned) or two workgroups per compute unit
  int cus = 256;
  {
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      int n = 0;
      if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0) cus = n;
    }
  }
  const unsigned grid = static_cast<unsigned>(round_up(static_cast<int64_t>(cus) * (aligned ? 3 : 2), 8));
  RPT_TRY(fill_i32(counters, static_cast<int64_t>(recon_batch_counters(ns)), 0, s));
  for (int g0 = 0, gi = 0; g0 < ns; g0 += kPersistMax, ++gi) {
    PersistTable t{};
    t.ns = 0;
    t.total = 0;
    t.counters = counters + 8 * gi;
    for (int q = g0; q < ns && q < g0 + kPersistMax; ++q) {
      if (st[q].L == 0) continue;
      Carver c(st[q].ws);
      const ReconBufs b = recon_carve(c, st[q].v, st[q].L, st[q].r, ks);
      const ReconPlan pu = recon_plan(st[q].v, st[q].L, st[q].r, kFusedPT);
      t.st[t.ns] = fused_args(b, st[q].W, st[q].r, st[q].v, st[q].L, st[q].col0, st[q].seed, RPT_STREAM_RECOVERY,
                              st[q].sigma_mu, st[q].study, pu);
      t.items[t.ns] = static_cast<int64_t>(pu.pg) * pu.nc / 8;  // nc is a multiple of 8
      t.total += t.items[t.ns];
      ++t.ns;
    }
    if (t.ns == 0) continue;
    void* args[] = {&t};
    hipError_t e;
    {
      RPT_STAGE("recon_fused_batched", s);
      e = hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, 0, s);
    }
    if (e != hipSuccess) {
      set_hip_error(e);
      return RPT_ERR_HIP;
    }
  }
  for (int q = 0; q < ns; ++q) {
    if (st[q].L == 0) continue;
    Carver c(st[q].ws);
    const ReconBufs b = recon_carve(c, st[q].v, st[q].L, st[q].r, ks);
    const ReconPlan pu = recon_plan(st[q].v, st[q].L, st[q].r, kFusedPT);
    RPT_TRY(recon_finish(st[q].U, st[q].v, st[q].r, st[q].W, st[q].L, st[q].col0, st[q].seed, RPT_STREAM_RECOVERY,
                         st[q].sigma_mu, st[q].out_max, nullptr, nullptr, ks, b, pu, s, st[q].study));
  }
  return RPT_OK;
}

}  // namespace rpt
