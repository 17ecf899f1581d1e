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

namespace rpt {

namespace {

constexpr int kRMaxRefine = 128;  // basis rank held in LDS by the refine

// ---------------------------------------------------------------- Philox4x32-10
__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const unsigned lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const unsigned lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ float noise_z(uint64_t seed, unsigned stream, unsigned col, int64_t vox, unsigned study) {
  unsigned c[4] = {static_cast<unsigned>(vox >> 2), col, stream, study};
  philox4x32_10(c, static_cast<unsigned>(seed), static_cast<unsigned>(seed >> 32));
  const int lane4 = static_cast<int>(vox & 3);
  const unsigned xa = lane4 < 2 ? c[0] : c[2];
  const unsigned xb = lane4 < 2 ? c[1] : c[3];
  const float ua = (static_cast<float>(xa >> 8) + 0.5f) * 5.9604644775390625e-08f;  // 2^-24
  const float ub = (static_cast<float>(xb >> 8) + 0.5f) * 5.9604644775390625e-08f;
  const float rad = sqrtf(-2.0f * logf(ua));
  float sn, cs;
  sincospif(2.0f * ub, &sn, &cs);
  return rad * ((lane4 & 1) ? sn : cs);
}

// ---------------------------------------------------------------- U preparation
// ukb [ks][vpad][16] bf16 of U (zero past r and past v); umax >= max_k |U_k|_2
__global__ void recon_init_kernel(unsigned* umax_bits) { *umax_bits = 0u; }

__global__ __launch_bounds__(kBlock) void recon_prep_u_kernel(const float* __restrict__ U, int64_t v, int r,
                                                             int64_t vpad, int ks, uint16_t* __restrict__ ukb,
                                                             unsigned* umax_bits) {
  // thread per voxel; for a fixed K block consecutive threads write
  // consecutive 32-byte segments
  const int64_t vox = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  float nrm = 0.0f;
  if (vox < vpad) {
    const float* u = U + vox * r;
    for (int s = 0; s < ks; ++s) {
      uint32_t w[8];
#pragma unroll
      for (int e2 = 0; e2 < 8; ++e2) {
        uint32_t pr = 0;
#pragma unroll
        for (int hl = 0; hl < 2; ++hl) {
          const int c = 16 * s + 2 * e2 + hl;
          const float x = (vox < v && c < r) ? u[c] : 0.0f;
          nrm = fmaf(x, x, nrm);
          pr |= static_cast<uint32_t>(f2bf(x)) << (16 * hl);
        }
        w[e2] = pr;
      }
      u32x4* d = reinterpret_cast<u32x4*>(ukb + (static_cast<size_t>(s) * vpad + vox) * 16);
      d[0] = u32x4{w[0], w[1], w[2], w[3]};
      d[1] = u32x4{w[4], w[5], w[6], w[7]};
    }
  }
  nrm = wave_max(nrm);
  if ((threadIdx.x & 63) == 0) atomicMax(umax_bits, __float_as_uint(sqrtf(nrm) * 1.000001f));
}

// ---------------------------------------------------------------- filter
struct FilterArgs {
  const uint16_t* ukb;
  const float* W;
  int r, ks;
  int64_t v, vpad, vt, L;
  int tpc, pg, nc;
  float* smax;  // [L][nc * 32]
};

template <int KS, int PT>
__global__ __launch_bounds__(kBlock) void recon_filter_kernel(FilterArgs a) {
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
  const size_t kstride = static_cast<size_t>(a.vpad) * 16;
  u32x4 Bc[KS], Bn[KS];
  auto load = [&](u32x4* B, int64_t t) {
    const uint16_t* bp = a.ukb + static_cast<size_t>(t * 32 + col) * 16 + h * 8;
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
  const float* U;
  const float* W;
  int64_t v, vt, L;
  int r, tpc, nc;
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
};

__global__ __launch_bounds__(kBlock) void recon_refine_kernel(RefineArgs a) {
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
  const float umax = __uint_as_float(*a.umax_bits);
  const float delta = a.eps * umax * wn;
  const int64_t ns = static_cast<int64_t>(a.nc) * 32;
  const float* sm = a.smax + i * ns;
  float M = -INFINITY;
  for (int64_t s = lane; s < ns; s += 64) M = fmaxf(M, sm[s]);
  M = wave_max(M);
  const float tau = M - 2.0f * kZBound * sigma - 2.0f * delta;
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
      const int64_t t0 = chunk * a.tpc;
      const int64_t t1 = t0 + a.tpc < a.vt ? t0 + a.tpc : a.vt;
      for (int64_t t = t0 + lane; t < t1; t += 64) {
        const int64_t vox = t * 32 + colc;
        if (vox >= a.v) continue;
        const float* u = a.U + vox * a.r;
        float s = 0.0f;
        for (int c = 0; c < a.r; ++c) s = fmaf(u[c], w[c], s);
        const float z = noise_z(a.seed, a.stream, static_cast<unsigned>(a.col0 + i), vox, 0u);
        best = fmaxf(best, fmaf(sigma, z, s));
      }
    }
  }
  best = wave_max(best);
  if (lane == 0) {
    if (a.out) a.out[i] = best + mu;
    if (a.gap) a.gap[i] = a.tmax[i] - best;
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
  int ks, pt, pg, nc, tpc;
  int64_t vpad, vt;
};

ReconPlan recon_plan(int64_t v, int64_t L, int r) {
  ReconPlan pl;
  pl.ks = static_cast<int>(ceil_div(r, 16));
  pl.pt = 4;
  pl.vpad = round_up(v, 32);
  pl.vt = pl.vpad / 32;
  const int64_t group = 4 * pl.pt * 32;
  pl.pg = static_cast<int>(ceil_div(L > 0 ? L : 1, group));
  int64_t nc = round_up(ceil_div(1280, pl.pg), 8);
  const int64_t ncmax = round_up(pl.vt, 8);
  if (nc > ncmax) nc = ncmax;
  if (nc < 8) nc = 8;
  pl.nc = static_cast<int>(nc);
  pl.tpc = static_cast<int>(ceil_div(pl.vt, nc));
  return pl;
}

void recon_carve(Carver& c, int64_t v, int64_t L, int r, uint16_t** ukb, float** smax, unsigned** umax) {
  const ReconPlan pl = recon_plan(v, L, r);
  *ukb = c.take<uint16_t>(static_cast<size_t>(pl.ks) * pl.vpad * 16);
  *smax = c.take<float>(static_cast<size_t>(L > 0 ? L : 1) * pl.nc * 32);
  *umax = c.take<unsigned>(64);
}

}  // namespace

size_t recon_bytes(int64_t v, int64_t L, int r) {
  Carver c(nullptr);
  uint16_t* a;
  float* b;
  unsigned* d;
  recon_carve(c, v, L, r, &a, &b, &d);
  return c.off;
}

rpt_status recon_launch(const float* U, int64_t v, int r, const float* W, int64_t L, int64_t col0, uint64_t seed,
                        int stream_id, const float* sigma_mu, float* out_max, const float* Tmax_for_gap,
                        float* gap_out, void* ws, hipStream_t s) {
  if (L == 0) return RPT_OK;
  if (r < 1 || r > kRMaxRefine) return RPT_ERR_UNSUPPORTED;
  Carver c(ws);
  uint16_t* ukb;
  float* smax;
  unsigned* umax;
  recon_carve(c, v, L, r, &ukb, &smax, &umax);
  const ReconPlan pl = recon_plan(v, L, r);

  hipLaunchKernelGGL(recon_init_kernel, dim3(1), dim3(1), 0, s, umax);
  RPT_CHECK_LAUNCH();
  hipLaunchKernelGGL(recon_prep_u_kernel, dim3(static_cast<unsigned>(ceil_div(pl.vpad, kBlock))), dim3(kBlock), 0, s,
                     U, v, r, pl.vpad, pl.ks, ukb, umax);
  RPT_CHECK_LAUNCH();

  FilterArgs fa{ukb, W, r, pl.ks, v, pl.vpad, pl.vt, L, pl.tpc, pl.pg, pl.nc, smax};
  void* fn = pick_filter<4>(pl.ks);
  if (!fn) return RPT_ERR_UNSUPPORTED;
  void* args[] = {&fa};
  hipError_t e = hipLaunchKernel(fn, dim3(static_cast<unsigned>(pl.pg) * pl.nc), dim3(kBlock), args, 0, s);
  if (e != hipSuccess) {
    set_hip_error(e);
    return RPT_ERR_HIP;
  }
  RefineArgs ra;
  ra.U = U;
  ra.W = W;
  ra.v = v;
  ra.vt = pl.vt;
  ra.L = L;
  ra.r = r;
  ra.tpc = pl.tpc;
  ra.nc = pl.nc;
  ra.smax = smax;
  ra.umax_bits = umax;
  ra.sigma_mu = sigma_mu;
  const int kpad = 16 * pl.ks;
  // BF16 rounding of both operands (2^-9 each), their product term, and FP32
  // accumulation in the filter and in the refine (K terms each, 2^-24)
  ra.eps = static_cast<float>((ldexp(1.0, -8) + ldexp(1.0, -18) + 2.02 * (kpad + r) * ldexp(1.0, -24)) * 1.01);
  ra.seed = seed;
  ra.stream = static_cast<unsigned>(stream_id);
  ra.col0 = col0;
  ra.out = out_max;
  ra.tmax = Tmax_for_gap;
  ra.gap = gap_out;
  hipLaunchKernelGGL(recon_refine_kernel, dim3(static_cast<unsigned>(ceil_div(L, 4))), dim3(kBlock), 0, s, ra);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace rpt
