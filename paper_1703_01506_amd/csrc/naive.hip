// K1 -- NaivePT (Alg. 1): group sums as a 0/1-indicator x X contraction on the
// matrix cores, fused with the t epilogue and the column maximum.
//
// Output element (relabelling i, voxel k) of the contraction is
//     a_ik = sum_j I[i, j] x_kj,     I[i, j] = 1 if subject j is in group 1.
// Rows of the MFMA tile are relabellings (operand A = indicator, held in
// registers for the whole workgroup lifetime), columns are voxels (operand B =
// the prepared data, streamed from the K-blocked layout so that one wave's
// fragment load is a single contiguous 1 KB block).  With the 32x32 MFMA
// output layout each lane owns one voxel column, so the per-voxel epilogue
// constants are per-lane scalars and the running maximum over voxels is kept
// per accumulator register; one cross-lane reduction per workgroup finishes
// it.
//
// Balanced designs (n1 = n/2), split-BF16: the per-voxel constants are folded
// into the prepared data (see prep.hip), so the contraction yields u itself;
// partial maxima of u, t = t(max u) in the finalize kernel.  For the
// max-only launch the operands are swapped: voxels are the MFMA rows and
// relabellings the columns, so the 16 accumulator registers of a lane all
// belong to one relabelling and reduce to one running maximum per tile
// (four registers instead of 64), which fits two waves per SIMD.
// FP32 path: epilogue u = a * rinv + c.
// Unbalanced designs: a second contraction with the squared data gives the
// group-1 sums of squares and the epilogue evaluates Eq. 2 per element.
//
// Split-BF16: x = hi + lo with hi = bf16(x), lo = bf16(x - hi).  Each K step
// of 16 subjects issues two MFMAs with the same (exact) indicator fragment,
// one on the hi fragment and one on the lo fragment, accumulating both halves
// in FP32; sharing the indicator fragment halves its register footprint.
//
// Grid: workgroups = perm groups (4 waves x PT tiles x 32 relabellings) x
// voxel chunks.  Block ids are remapped so that every perm group of one voxel
// chunk lands on the same XCD (dispatch is round-robin over the 8 XCDs), so a
// chunk's data is fetched into one L2 only.
#include "rpt_internal.h"

namespace rpt {

namespace {

struct NaiveArgs {
  const uint16_t* kb16;
  const uint16_t* kbm;
  const float* kb32;
  const float* kb32sq;
  const float2* cst;
  const float2* cstg;
  const uint8_t* labels;
  int64_t vpad, v, vt, L;
  int n, n1, tpc, pg, abs_tail, store, mixr;
  float fs, tm;
  float* partial;
  float* T_out;
};

// label byte j of a relabelling row as a flag: 0 past n or for a row beyond
// L.  The load itself is unconditional (clamped index, and a row beyond L
// reads row 0), so that a lane's many label loads are issued back to back
// instead of each waiting behind a branch of its own.
__device__ __forceinline__ bool in_group1(const uint8_t* lab, int j, int n, bool valid) {
  const uint8_t b = lab[j < n ? j : n - 1];
  return valid && j < n && b != 0;
}

__device__ __forceinline__ void block_coords(const NaiveArgs& a, int pt, int& chunk, int64_t& pbase) {
  const int b = blockIdx.x, xcd = b & 7, j = b >> 3;
  const int pg = j % a.pg;
  chunk = xcd + 8 * (j / a.pg);
  const int wave = threadIdx.x >> 6;
  pbase = static_cast<int64_t>(pg) * (4 * pt * 32) + static_cast<int64_t>(wave) * (pt * 32);
}


// ----------------------------------------------------------------------------
// split-BF16, balanced.  K step s covers subjects 16s..16s+15; the same
// indicator fragment multiplies the hi fragment and the lo fragment.
template <int KS, int PT, bool ABS, bool STORE>
__global__ __launch_bounds__(kBlock) void naive_split_kernel(NaiveArgs a) {
  const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
  int chunk;
  int64_t pbase;
  block_coords(a, PT, chunk, pbase);

  // indicator fragments: lane supplies I[relabelling pbase + 32p + col][subject
  // 16s + 8h + 0..7] (the A operand layout of the T-storing orientation and
  // the B operand layout of the max-only one are the same)
  u32x4 I[PT][KS];
#pragma unroll
  for (int p = 0; p < PT; ++p) {
    const int64_t perm = pbase + p * 32 + col;
    const bool valid = perm < a.L;
    const uint8_t* lab = a.labels + (valid ? perm : 0) * a.n;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      unsigned w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j0 = 16 * s + 8 * h + 2 * q;
        const unsigned b0 = in_group1(lab, j0, a.n, valid) ? 0x3F80u : 0u;
        const unsigned b1 = in_group1(lab, j0 + 1, a.n, valid) ? 0x3F80u : 0u;
        w[q] = b0 | (b1 << 16);
      }
      I[p][s] = u32x4{w[0], w[1], w[2], w[3]};
    }
  }

  const int64_t t0 = static_cast<int64_t>(chunk) * a.tpc;
  const int64_t t1 = t0 + a.tpc < a.vt ? t0 + a.tpc : a.vt;
  const size_t kstride = static_cast<size_t>(a.vpad) * 32;  // uint16 per K step
  // data fragments of voxel tile t: lane supplies x''[voxel 32t + col][subject
  // 16s + 8h + 0..7]; the prepared layout stores them in lane order
  auto load = [&](u32x4* X, int64_t t) {
    const uint16_t* bp = a.kb16 + static_cast<size_t>(t) * 32 * 32 + lane * 8;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      X[2 * s] = *reinterpret_cast<const u32x4*>(bp + s * kstride);
      X[2 * s + 1] = *reinterpret_cast<const u32x4*>(bp + s * kstride + 512);
    }
  };
  const float init = ABS ? 0.0f : -INFINITY;

  // T-storing orientation: rows = relabellings, columns = voxels, so the
  // stores of one accumulator register are 32 consecutive voxels
  float rm[PT][16];
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) rm[p][e] = init;
  u32x4 Bc[2 * KS], Bn[2 * KS];
  auto body = [&](const u32x4* B, int64_t t) {
    f32x16 acc[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) acc[p] = f32x16{};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int p = 0; p < PT; ++p) acc[p] = mfma_bf16(I[p][s], B[2 * s], acc[p]);
#pragma unroll
      for (int p = 0; p < PT; ++p) acc[p] = mfma_bf16(I[p][s], B[2 * s + 1], acc[p]);
    }
    const int64_t vox = t * 32 + col;
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float u = acc[p][e];
        rm[p][e] = fmaxf(rm[p][e], ABS ? fabsf(u) : u);
        const int64_t perm = pbase + p * 32 + mfma_row(e, h);
        if (perm < a.L && vox < a.v) a.T_out[perm * a.v + vox] = t_from_u_f(u, a.fs, a.tm);
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
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      float x = rm[p][e];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
      rm[p][e] = x;
    }
  if (col == 0) {
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t perm = pbase + p * 32 + mfma_row(e, h);
        if (perm < a.L) a.partial[static_cast<int64_t>(chunk) * a.L + perm] = rm[p][e];
      }
  }
}

// ----------------------------------------------------------------------------
// split-BF16, balanced, maxima only.  Voxels are the MFMA rows and
// relabellings the columns (a lane's 16 accumulator registers belong to one
// relabelling).  Each voxel tile (KS steps x hi/lo x 1 KB) is copied once per
// workgroup straight into LDS (global_load_lds, double-buffered, one barrier
// per tile) and every wave reads its fragments from there: the four waves
// share one copy instead of fetching it four times through the vector memory
// path.
// MIX (R = n mod 16 in 1..8): the last, partial K step packs the hi and the
// lo half of its R subjects into one 16-wide block (hi at positions 0..R-1,
// lo at R..2R-1), paired with an indicator fragment that repeats the R
// indicators, so that step takes one MFMA instead of two.
template <int KS, int PT, bool ABS, bool MIX>
__global__ __launch_bounds__(kBlock, 2) void naive_max_kernel(NaiveArgs a) {
  // the label rows of the workgroup (n <= 16 KS bytes each), then the two
  // data tile buffers, share one LDS allocation
  constexpr int kLabBytes = 4 * PT * 32 * 16 * KS, kTileBytes = 2 * KS * 2 * 64 * 8 * 2;
  __shared__ __align__(16) uint8_t smem[kLabBytes > kTileBytes ? kLabBytes : kTileBytes];
  uint16_t (&xs)[2][KS][2][64 * 8] = *reinterpret_cast<uint16_t (*)[2][KS][2][64 * 8]>(smem);
  typedef __attribute__((address_space(3))) void lds_void;
  typedef const __attribute__((address_space(1))) void gbl_void;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
  int chunk;
  int64_t pbase;
  block_coords(a, PT, chunk, pbase);

  // indicator fragments (B operand): lane supplies I[relabelling pbase + 32p + col][subject 16s + 8h + 0..7].
  // The workgroup's label rows (4 PT 32 relabellings, one contiguous range of
  // 128 PT n bytes) are first copied into LDS with 16-byte loads, in the
  // space the data tiles take afterwards; each lane then reads its flags in
  // pairs (n is even on this path, so a pair is one aligned 2-byte read).
  // Reading them straight from global memory, one byte and one wait at a
  // time, cost about a seventh of the launch.
  u32x4 I[PT][KS];
  {
    const int64_t nbytes = a.L * a.n;
    const int64_t g0 = (pbase - static_cast<int64_t>(wave) * (PT * 32)) * a.n;  // 16-byte multiple
    const int span = 4 * PT * 32 * a.n;                                          // <= sizeof smem
    const bool al16 = (reinterpret_cast<uintptr_t>(a.labels) & 15) == 0;
    for (int off = 16 * threadIdx.x; off < span; off += 16 * kBlock) {
      const int64_t g = g0 + off;
      u32x4 v = u32x4{0u, 0u, 0u, 0u};
      if (al16 && g + 16 <= nbytes) {
        v = *reinterpret_cast<const u32x4*>(a.labels + g);
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e)
          if (g + e < nbytes) v[e >> 2] |= static_cast<unsigned>(a.labels[g + e]) << (8 * (e & 3));
      }
      *reinterpret_cast<u32x4*>(smem + off) = v;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      const bool valid = pbase + p * 32 + col < a.L;
      const uint8_t* row = smem + ((wave * PT + p) * 32 + col) * a.n;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        unsigned w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // block position kappa holds subject 16 s + kappa; under MIX the
          // last step's position kappa holds subject 16 s + kappa (hi,
          // kappa < R) or 16 s + kappa - R (lo, R <= kappa < 2 R); R is even,
          // so a pair of positions is a pair of consecutive subjects
          const int k0 = 8 * h + 2 * q;
          int j0 = 16 * s + k0;
          if (MIX && s == KS - 1) j0 = k0 < a.mixr ? 16 * s + k0 : (k0 < 2 * a.mixr ? 16 * s + k0 - a.mixr : a.n);
          const unsigned pr = (valid && j0 < a.n) ? *reinterpret_cast<const uint16_t*>(row + j0) : 0u;
          w[q] = ((pr & 0xFFu) ? 0x3F80u : 0u) | ((pr >> 8) ? 0x3F800000u : 0u);
        }
        I[p][s] = u32x4{w[0], w[1], w[2], w[3]};
      }
    }
    __syncthreads();  // every wave has its fragments before the tile copies reuse the space
  }

  const int64_t t0 = static_cast<int64_t>(chunk) * a.tpc;
  const int64_t t1 = t0 + a.tpc < a.vt ? t0 + a.tpc : a.vt;
  const size_t kstride = static_cast<size_t>(a.vpad) * 32;  // uint16 per K step
  // 1 KB blocks per tile: hi and lo of every K step, or under MIX hi and lo
  // of the KS - 1 full steps and the mixed block (into xs[b][KS - 1][0])
  constexpr int NB = MIX ? 2 * KS - 1 : 2 * KS;
  // copy of tile t into buffer b: wave w moves the 1 KB blocks j = w, w + 4, ...
  auto issue = [&](int b, int64_t t) {
#pragma unroll
    for (int j = 0; j < NB; j += 4) {
      const int jj = j + wave;
      if (jj < NB) {
        const int s = jj >> 1, hl = jj & 1;
        const uint16_t* g = (MIX && jj == NB - 1)
                                ? a.kbm + static_cast<size_t>(t) * 32 * 16 + lane * 8
                                : a.kb16 + s * kstride + static_cast<size_t>(t) * 32 * 32 + hl * 512 + lane * 8;
        __builtin_amdgcn_global_load_lds((gbl_void*)g, (lds_void*)&xs[b][s][hl][0], 16, 0, 0);
      }
    }
  };

  const float init = ABS ? 0.0f : -INFINITY;
  float rm[PT];
#pragma unroll
  for (int p = 0; p < PT; ++p) rm[p] = init;
  if (t0 < t1) issue(0, t0);
  for (int64_t t = t0; t < t1; ++t) {
    const int b = static_cast<int>((t - t0) & 1);
    // this wave's copies of tile t have landed; after the barrier every
    // wave's have, and every wave is done reading tile t - 1's buffer
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (t + 1 < t1) issue(b ^ 1, t + 1);
    f32x16 acc[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) acc[p] = f32x16{};
    // block j (hi / lo of step j / 2, or the mixed block) multiplies the
    // indicator of step j / 2; block j + 1 is read from LDS while block j's
    // MFMAs run
    u32x4 cur = *reinterpret_cast<const u32x4*>(&xs[b][0][0][lane * 8]);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      u32x4 nxt;
      if (j + 1 < NB) nxt = *reinterpret_cast<const u32x4*>(&xs[b][(j + 1) >> 1][(j + 1) & 1][lane * 8]);
#pragma unroll
      for (int p = 0; p < PT; ++p) acc[p] = mfma_bf16(cur, I[p][j >> 1], acc[p]);
      if (j + 1 < NB) cur = nxt;
    }
    // schedule: reads of blocks 0 and 1, then block j's MFMAs followed by
    // the read of block j + 2
    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      __builtin_amdgcn_sched_group_barrier(0x008, PT, 0);
      if (j + 2 < NB) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      float m = ABS ? fabsf(acc[p][0]) : acc[p][0];
#pragma unroll
      for (int e = 1; e < 16; ++e) m = fmaxf(m, ABS ? fabsf(acc[p][e]) : acc[p][e]);
      rm[p] = fmaxf(rm[p], m);
    }
  }
#pragma unroll
  for (int p = 0; p < PT; ++p) rm[p] = fmaxf(rm[p], __shfl_xor(rm[p], 32, 64));
  if (h == 0) {
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      const int64_t perm = pbase + p * 32 + col;
      if (perm < a.L) a.partial[static_cast<int64_t>(chunk) * a.L + perm] = rm[p];
    }
  }
}

// ----------------------------------------------------------------------------
// split-BF16, balanced, more than 128 subjects (up to 512: 32 K steps).  The
// K steps are taken kWideKC at a time for two consecutive 32-voxel tiles:
// the chunk (hi and lo, 2 KB per step and tile) is copied once per workgroup
// into LDS with global_load_lds, double-buffered over the (tile pair, chunk)
// sequence.  The indicator of a wave's relabellings is kept in LDS as bits,
// eight subjects per byte, and expanded to a BF16 fragment when it is used,
// once for both tiles (expanding it per tile took more VALU issue than the
// MFMAs it fed): two indicator bits x become the 32-bit pair
// ((x | x << 15) & 0x10001) * 0x3F80.  Relabellings
// are the MFMA rows (A operand), voxels the columns; the same kernel keeps
// running maxima and, in STORE mode, writes t for every element.
constexpr int kWideNT = 2;      // voxel tiles per unit
constexpr int kWideKC = 4;      // K steps per staged chunk
constexpr int kWideNMax = 512;  // subjects

__device__ __forceinline__ u32x4 indicator_frag(unsigned byte) {
  u32x4 f;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const unsigned x = (byte >> (2 * q)) & 3u;
    f[q] = ((x | (x << 15)) & 0x10001u) * 0x3F80u;
  }
  return f;
}

template <int PT, bool ABS, bool STORE>
__global__ __launch_bounds__(kBlock, 2) void naive_wide_kernel(NaiveArgs a) {
  // a unit is one K chunk of kWideNT voxel tiles, so that each indicator
  // fragment expanded from its bits serves the MFMAs of all of them
  __shared__ __align__(16) uint16_t xs[2][kWideNT][kWideKC][2][64 * 8];
  __shared__ uint8_t lb[4][PT][32][kWideNMax / 8];
  typedef __attribute__((address_space(3))) void lds_void;
  typedef const __attribute__((address_space(1))) void gbl_void;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, col = lane & 31;
  int chunk;
  int64_t pbase;
  block_coords(a, PT, chunk, pbase);
  const int ks = (a.n + 15) / 16;
  const int nkc = (ks + kWideKC - 1) / kWideKC;

  // indicator bits of this wave's relabellings: byte g holds subjects 8g..8g+7
  for (int idx = lane; idx < PT * 32 * 2 * ks; idx += 64) {
    const int p = idx / (64 * ks), rem = idx - p * 64 * ks, c = rem / (2 * ks), g = rem - c * 2 * ks;
    const int64_t perm = pbase + p * 32 + c;
    unsigned bits = 0;
    const bool valid = perm < a.L;
    const uint8_t* lab = a.labels + (valid ? perm : 0) * a.n;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (in_group1(lab, 8 * g + i, a.n, valid)) bits |= 1u << i;
    lb[wave][p][c][g] = static_cast<uint8_t>(bits);
  }

  const int64_t t0 = static_cast<int64_t>(chunk) * a.tpc;
  const int64_t t1 = t0 + a.tpc < a.vt ? t0 + a.tpc : a.vt;
  const size_t kstride = static_cast<size_t>(a.vpad) * 32;  // uint16 per K step
  // copy of K chunk c of the tiles tp .. tp + kWideNT - 1 (those below t1)
  // into buffer b: wave w moves the 1 KB blocks j = w, w + 4, ... (block j:
  // tile j / (2 kWideKC), K step kWideKC c + (j / 2) mod kWideKC, hi or lo)
  auto issue = [&](int b, int64_t tp, int c) {
    const int s0 = c * kWideKC, nks = ks - s0 < kWideKC ? ks - s0 : kWideKC;
    const int ntl = t1 - tp < kWideNT ? static_cast<int>(t1 - tp) : kWideNT;
#pragma unroll
    for (int j = 0; j < 2 * kWideNT * kWideKC; j += 4) {
      const int jj = j + wave, tt = jj / (2 * kWideKC), s = (jj >> 1) % kWideKC, hl = jj & 1;
      if (tt < ntl && s < nks) {
        const uint16_t* g =
            a.kb16 + (s0 + s) * kstride + static_cast<size_t>(tp + tt) * 32 * 32 + hl * 512 + lane * 8;
        __builtin_amdgcn_global_load_lds((gbl_void*)g, (lds_void*)&xs[b][tt][s][hl][0], 16, 0, 0);
      }
    }
  };

  const float init = ABS ? 0.0f : -INFINITY;
  float rm[PT][16];
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) rm[p][e] = init;
  f32x16 acc[kWideNT][PT];
#pragma unroll
  for (int tt = 0; tt < kWideNT; ++tt)
#pragma unroll
    for (int p = 0; p < PT; ++p) acc[tt][p] = f32x16{};
  // running maxima (and t in STORE mode) of tile t from its accumulators
  auto finish = [&](f32x16 (&ac)[PT], int64_t t) {
    const int64_t vox = t * 32 + col;
#pragma unroll
    for (int p = 0; p < PT; ++p) {
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const float u = ac[p][e];
        rm[p][e] = fmaxf(rm[p][e], ABS ? fabsf(u) : u);
        if (STORE) {
          const int64_t perm = pbase + p * 32 + mfma_row(e, h);
          if (perm < a.L && vox < a.v) a.T_out[perm * a.v + vox] = t_from_u_f(u, a.fs, a.tm);
        }
      }
      ac[p] = f32x16{};
    }
  };
  const int64_t nunit = (t1 - t0 + kWideNT - 1) / kWideNT * nkc;
  if (nunit > 0) issue(0, t0, 0);
  for (int64_t i = 0; i < nunit; ++i) {
    const int64_t tp = t0 + kWideNT * (i / nkc);
    const int c = static_cast<int>(i % nkc);
    const int b = static_cast<int>(i & 1);
    const int ntl = t1 - tp < kWideNT ? static_cast<int>(t1 - tp) : kWideNT;
    // this wave's copies have landed; after the barrier every wave's have
    // (and the indicator bytes are written), and every wave is done with
    // the other buffer
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (i + 1 < nunit) issue(b ^ 1, t0 + kWideNT * ((i + 1) / nkc), static_cast<int>((i + 1) % nkc));
    const int s0 = c * kWideKC, nks = ks - s0 < kWideKC ? ks - s0 : kWideKC;
#pragma unroll
    for (int s = 0; s < kWideKC; ++s) {
      if (s < nks) {
        u32x4 ind[PT];
#pragma unroll
        for (int p = 0; p < PT; ++p) ind[p] = indicator_frag(lb[wave][p][col][2 * (s0 + s) + h]);
#pragma unroll
        for (int tt = 0; tt < kWideNT; ++tt) {
          if (tt < ntl) {
            const u32x4 xh = *reinterpret_cast<const u32x4*>(&xs[b][tt][s][0][lane * 8]);
            const u32x4 xl = *reinterpret_cast<const u32x4*>(&xs[b][tt][s][1][lane * 8]);
#pragma unroll
            for (int p = 0; p < PT; ++p) {
              acc[tt][p] = mfma_bf16(ind[p], xh, acc[tt][p]);
              acc[tt][p] = mfma_bf16(ind[p], xl, acc[tt][p]);
            }
          }
        }
      }
    }
    if (c == nkc - 1) {
#pragma unroll
      for (int tt = 0; tt < kWideNT; ++tt)
        if (tt < ntl) finish(acc[tt], tp + tt);
    }
  }
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      float x = rm[p][e];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
      rm[p][e] = x;
    }
  if (col == 0) {
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t perm = pbase + p * 32 + mfma_row(e, h);
        if (perm < a.L) a.partial[static_cast<int64_t>(chunk) * a.L + perm] = rm[p][e];
      }
  }
}

// ----------------------------------------------------------------------------
// FP32 (balanced, or unbalanced with a second contraction of the squares)
template <int KSB, int PT, bool UNBAL>
__global__ __launch_bounds__(kBlock) void naive_f32_kernel(NaiveArgs a) {
  const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
  int chunk;
  int64_t pbase;
  block_coords(a, PT, chunk, pbase);

  // lane supplies A[row = col][subject 8s + 2q + h], q = 0..3
  f32x4 A[PT][KSB];
#pragma unroll
  for (int p = 0; p < PT; ++p) {
    const int64_t perm = pbase + p * 32 + col;
    const bool valid = perm < a.L;
    const uint8_t* lab = a.labels + (valid ? perm : 0) * a.n;
#pragma unroll
    for (int s = 0; s < KSB; ++s) {
      float f[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = 8 * s + 2 * q + h;
        f[q] = in_group1(lab, j, a.n, valid) ? 1.0f : 0.0f;
      }
      A[p][s] = f32x4{f[0], f[1], f[2], f[3]};
    }
  }

  const float init = a.abs_tail ? 0.0f : -INFINITY;
  float rm[PT][16];
#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) rm[p][e] = init;

  const int64_t t0 = static_cast<int64_t>(chunk) * a.tpc;
  const int64_t t1 = t0 + a.tpc < a.vt ? t0 + a.tpc : a.vt;
  const size_t kstride = static_cast<size_t>(a.vpad) * 8;
  const int n1 = a.n1, n2 = a.n - a.n1;
  const float rn1 = 1.0f / n1, rn2 = 1.0f / n2, rd1 = 1.0f / (n1 - 1), rd2 = 1.0f / (n2 - 1);

  for (int64_t t = t0; t < t1; ++t) {
    const int64_t vox = t * 32 + col;
    const float* bp = a.kb32 + static_cast<size_t>(vox) * 8 + h * 4;
    f32x16 acc[PT], acc2[PT];
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      acc[p] = f32x16{};
      if (UNBAL) acc2[p] = f32x16{};
    }
#pragma unroll
    for (int s = 0; s < KSB; ++s) {
      const f32x4 B = *reinterpret_cast<const f32x4*>(bp + s * kstride);
      f32x4 B2;
      if (UNBAL) B2 = *reinterpret_cast<const f32x4*>(a.kb32sq + static_cast<size_t>(vox) * 8 + h * 4 + s * kstride);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int p = 0; p < PT; ++p) {
          acc[p] = mfma_f32(A[p][s][q], B[q], acc[p]);
          if (UNBAL) acc2[p] = mfma_f32(A[p][s][q], B2[q], acc2[p]);
        }
    }
    if (!UNBAL) {
      const float2 c2 = a.cst[vox];
#pragma unroll
      for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float u = fmaf(acc[p][e], c2.x, c2.y);
          rm[p][e] = fmaxf(rm[p][e], a.abs_tail ? fabsf(u) : u);
          if (a.store) {
            const int64_t perm = pbase + p * 32 + mfma_row(e, h);
            if (perm < a.L && vox < a.v) a.T_out[perm * a.v + vox] = t_from_u_f(u, a.fs, a.tm);
          }
        }
    } else {
      const float2 sq = a.cstg[vox];
      const bool vvalid = vox < a.v;
#pragma unroll
      for (int p = 0; p < PT; ++p)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const float S1 = acc[p][e], Q1 = acc2[p][e];
          const float S2 = sq.x - S1, Q2 = sq.y - Q1;
          const float m1 = S1 * rn1, m2 = S2 * rn2;
          const float v1 = fmaxf((Q1 - S1 * m1) * rd1, 0.0f), v2 = fmaxf((Q2 - S2 * m2) * rd2, 0.0f);
          const float den2 = v1 * rn1 + v2 * rn2;
          const float t = den2 > 0.0f ? (m1 - m2) * rsqrtf(den2) : 0.0f;
          if (vvalid) rm[p][e] = fmaxf(rm[p][e], a.abs_tail ? fabsf(t) : t);
          if (a.store) {
            const int64_t perm = pbase + p * 32 + mfma_row(e, h);
            if (perm < a.L && vvalid) a.T_out[perm * a.v + vox] = t;
          }
        }
    }
  }

#pragma unroll
  for (int p = 0; p < PT; ++p)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      float x = rm[p][e];
#pragma unroll
      for (int off = 1; off < 32; off <<= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
      rm[p][e] = x;
    }
  if (col == 0) {
#pragma unroll
    for (int p = 0; p < PT; ++p)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t perm = pbase + p * 32 + mfma_row(e, h);
        if (perm < a.L) a.partial[static_cast<int64_t>(chunk) * a.L + perm] = rm[p][e];
      }
  }
}

// One wave per relabelling: the lanes take the chunks' partial maxima in
// turn (a few hundred chunks for short launches), then a wave maximum
// mode: 0 the partials are the statistic already (unbalanced FP32 path),
// 1 t of Eq. 2 from u, 2 the mean difference 2 u / m
__global__ __launch_bounds__(kBlock) void naive_finalize_kernel(const float* __restrict__ partial, int nc, int64_t L,
                                                                int m, int mode, float* __restrict__ max_out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6);
  if (i >= L) return;
  float u = -INFINITY;
  for (int c = lane; c < nc; c += 64) u = fmaxf(u, partial[static_cast<int64_t>(c) * L + i]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) u = fmaxf(u, __shfl_xor(u, off, 64));
  if (lane == 0)
    max_out[i] = mode == 1   ? static_cast<float>(t_from_u(static_cast<double>(u), m))
                 : mode == 2 ? static_cast<float>(2.0 * static_cast<double>(u) / m)
                             : u;
}

// T-storing launches use naive_split_kernel (PT = 1), max-only launches
// naive_max_kernel (PT = 4)
template <int PT, int KS>
void* split_ptr(int abs_tail, int store, int mix) {
  if (store) return abs_tail ? reinterpret_cast<void*>(&naive_split_kernel<KS, 1, true, true>)
                             : reinterpret_cast<void*>(&naive_split_kernel<KS, 1, false, true>);
  if (mix) return abs_tail ? reinterpret_cast<void*>(&naive_max_kernel<KS, 4, true, true>)
                           : reinterpret_cast<void*>(&naive_max_kernel<KS, 4, false, true>);
  return abs_tail ? reinterpret_cast<void*>(&naive_max_kernel<KS, 4, true, false>)
                  : reinterpret_cast<void*>(&naive_max_kernel<KS, 4, false, false>);
}
template <int PT, int KSB, bool U>
void* f32_ptr() { return reinterpret_cast<void*>(&naive_f32_kernel<KSB, PT, U>); }

template <int PT>
void* pick_split(int ks, int at, int st, int mx) {
  switch (ks) {
    case 1: return split_ptr<PT, 1>(at, st, mx); case 2: return split_ptr<PT, 2>(at, st, mx);
    case 3: return split_ptr<PT, 3>(at, st, mx); case 4: return split_ptr<PT, 4>(at, st, mx);
    case 5: return split_ptr<PT, 5>(at, st, mx); case 6: return split_ptr<PT, 6>(at, st, mx);
    case 7: return split_ptr<PT, 7>(at, st, mx); case 8: return split_ptr<PT, 8>(at, st, mx);
    default: return nullptr;
  }
}
template <int PT, bool U>
void* pick_f32(int ks) {
  switch (ks) {
    case 1: return f32_ptr<PT, 1, U>();   case 2: return f32_ptr<PT, 2, U>();
    case 3: return f32_ptr<PT, 3, U>();   case 4: return f32_ptr<PT, 4, U>();
    case 5: return f32_ptr<PT, 5, U>();   case 6: return f32_ptr<PT, 6, U>();
    case 7: return f32_ptr<PT, 7, U>();   case 8: return f32_ptr<PT, 8, U>();
    case 9: return f32_ptr<PT, 9, U>();   case 10: return f32_ptr<PT, 10, U>();
    case 11: return f32_ptr<PT, 11, U>(); case 12: return f32_ptr<PT, 12, U>();
    case 13: return f32_ptr<PT, 13, U>(); case 14: return f32_ptr<PT, 14, U>();
    case 15: return f32_ptr<PT, 15, U>(); case 16: return f32_ptr<PT, 16, U>();
    default: return nullptr;
  }
}

}  // namespace

NaivePlan naive_plan(int64_t v, int64_t L, int n, int prec, bool store, int force_nc) {
  NaivePlan pl;
  // split max-only path: 4 relabelling tiles per wave (data shared through
  // LDS, two waves per SIMD); the split T-writing path 1 (its data tiles
  // stay in registers, so one tile keeps two waves per SIMD); the wide-subject
  // path 2; the FP32 path 1 (its indicator, accumulators and per-row running
  // maxima of two tiles took 288 registers, one wave per SIMD, and every
  // data load then waited out its latency: 7.2 -> 5.0 ms balanced, 12.9 ->
  // 10.5 ms unbalanced at n = 100, v = 250k, L = 10k).
  pl.pt = (prec == RPT_SPLIT_BF16 && n <= 128) ? (store ? 1 : 4) : (prec == RPT_SPLIT_BF16 ? 2 : 1);
  pl.vt = round_up(v, 32) / 32;
  const int64_t group = 4 * pl.pt * 32;
  pl.pg = static_cast<int>(ceil_div(L > 0 ? L : 1, group));
  // rule of thumb: about 1,280 workgroups; a measured choice replaces it
  int64_t nc = round_up(ceil_div(1280, pl.pg), 8);
  const int64_t ncmax = round_up(pl.vt, 8);
  if (nc > ncmax) nc = ncmax;
  if (nc < 8) nc = 8;
  pl.nc_heur = static_cast<int>(nc);
  pl.nc_cap = static_cast<int>(chunk_cap(nc, ncmax));
  int64_t pick = force_nc > 0 ? force_nc : tuned_chunks(kTuneNaive, v, L, n, 2 * prec + (store ? 1 : 0));
  if (pick >= 8 && pick <= pl.nc_cap && pick % 8 == 0) nc = pick;
  pl.nc = static_cast<int>(nc);
  pl.tpc = static_cast<int>(ceil_div(pl.vt, nc));
  return pl;
}

size_t naive_bytes(int64_t v, int n, int64_t L, int prec) {
  // the larger of the two plans (max-only / T-writing), at their largest
  // candidate chunk count
  int64_t nc = 0;
  for (int st = 0; st < 2; ++st) {
    NaivePlan pl = naive_plan(v, L, n, prec, st != 0);
    if (pl.nc_cap > nc) nc = pl.nc_cap;
  }
  return round_up(nc * (L > 0 ? L : 1) * 4, 256);
}

rpt_status naive_launch(const PrepX& p, const NaivePlan& pl, const uint8_t* labels, int64_t L, int tail, int prec,
                        float* partial, float* T_out, float* max_out, hipStream_t s) {
  if (L == 0) return RPT_OK;
  NaiveArgs a;
  a.kb16 = p.kb16;
  a.kbm = nullptr;
  a.mixr = 0;
  a.kb32 = p.kb32;
  a.kb32sq = p.kb32sq;
  a.cst = p.cst;
  a.cstg = p.cstg;
  a.labels = labels;
  a.vpad = p.vpad;
  a.v = p.v;
  a.vt = pl.vt;
  a.L = L;
  a.n = p.n;
  a.n1 = p.n1;
  a.tpc = pl.tpc;
  a.pg = pl.pg;
  a.abs_tail = tail == RPT_TAIL_ABS;
  a.store = T_out != nullptr;
  const int m = p.n / 2;
  stat_consts(p, &a.fs, &a.tm);
  a.partial = partial;
  a.T_out = T_out;
  const bool unbal = 2 * p.n1 != p.n;
  void* fn = nullptr;
  if (prec == RPT_SPLIT_BF16 && p.ksteps > 8) {
    if (unbal || p.n > kWideNMax) return RPT_ERR_UNSUPPORTED;
    fn = a.store ? (a.abs_tail ? reinterpret_cast<void*>(&naive_wide_kernel<2, true, true>)
                               : reinterpret_cast<void*>(&naive_wide_kernel<2, false, true>))
                 : (a.abs_tail ? reinterpret_cast<void*>(&naive_wide_kernel<2, true, false>)
                               : reinterpret_cast<void*>(&naive_wide_kernel<2, false, false>));
  } else if (prec == RPT_SPLIT_BF16) {
    // split designs are balanced, so n is even (the max-only kernel reads
    // label flags in pairs)
    if (p.n & 1) return RPT_ERR_UNSUPPORTED;
    a.kbm = p.kbm;
    a.mixr = p.mixr;
    fn = pick_split<0>(p.ksteps, a.abs_tail, a.store, p.kbm != nullptr && !a.store);
  } else {
    fn = unbal ? pick_f32<1, true>(p.ksteps) : pick_f32<1, false>(p.ksteps);
  }
  if (!fn) return RPT_ERR_UNSUPPORTED;
  const unsigned blocks = static_cast<unsigned>(pl.pg) * static_cast<unsigned>(pl.nc);
  void* args[] = {&a};
  hipError_t e;
  {
    RPT_STAGE(a.store ? "naive_contract_store" : "naive_contract", s);
    e = hipLaunchKernel(fn, dim3(blocks), dim3(kBlock), args, 0, s);
  }
  if (e != hipSuccess) {
    set_hip_error(e);
    return RPT_ERR_HIP;
  }
  if (max_out) {
    RPT_STAGE("naive_finalize", s);
    hipLaunchKernelGGL(naive_finalize_kernel, dim3(static_cast<unsigned>(ceil_div(L, kBlock / 64))), dim3(kBlock), 0,
                       s, partial, pl.nc, L, m, unbal ? 0 : (p.stat == RPT_STAT_MEANDIFF ? 2 : 1), max_out);
    RPT_CHECK_LAUNCH();
  }
  return RPT_OK;
}

}  // namespace rpt
