// Inputs of Alg. 1 and Alg. 2 drawn from a seed: the relabellings (Alg. 1
// draws Permute[1, n] and gives the first n1 subjects group 1; Sec. 2.1), the
// sampled sets Omega of Alg. 2 (ceil(eta v) distinct voxels, uniform without
// replacement; Sec. 4.1, 4.2) and the Gaussian matrix that Rand. Orth.
// orthonormalises.  The paper names no generator; here every draw is a word of
// Philox4x32-10 with counter (j >> 2, row, stream, set) and key = seed, step
// j taking word j & 3, so any row can be regenerated alone:
//  * an index on [0, m) from word x is the high half of the product x m;
//  * a partial Fisher-Yates shuffle (Durstenfeld's in-place form) of k steps
//    over 0 .. m-1 -- step j draws t on [j, m) and swaps entries j and t --
//    leaves a uniform k-subset in entries 0 .. k-1;
//  * relabelling `row` (stream 0, set 0): k = n1 steps over the n subjects;
//  * sampled set `row` of set `set_id` (stream 1): k steps over the v voxels,
//    then sorted; only the displaced entries of the virtual array are kept,
//    in a hash table in LDS, so a set of k voxels needs O(k) memory;
//  * start basis (stream 3): entry (q, c) is the Box-Muller draw of column c
//    at voxel q, the layout of the residual noise.
#include "rpt_internal.h"
#include "philox.h"

namespace rpt {

namespace {

constexpr int kGenMaxN = 512;        // subjects
constexpr int kGenLabelWaves = 4;    // relabellings per workgroup (one per wave)
constexpr int kGenSetThreads = 256;  // threads per sampled set
constexpr int kGenSetEmpty = -1;

constexpr uint32_t kStreamLabels = 0, kStreamOmega = 1, kStreamStart = 3;

__host__ __device__ inline int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// index on [0, m): high half of x m
__device__ __forceinline__ uint32_t index_below(uint32_t x, uint32_t m) { return __umulhi(x, m); }

// one wave per relabelling; the sequential swaps run on lane 0 of each wave
__global__ __launch_bounds__(64 * kGenLabelWaves) void gen_labels_kernel(uint64_t seed, uint32_t row0, int64_t L,
                                                                         int n, int n1, uint8_t* __restrict__ out) {
  __shared__ uint16_t a[kGenLabelWaves][kGenMaxN];
  __shared__ uint16_t tt[kGenLabelWaves][kGenMaxN];
  __shared__ uint8_t grp[kGenLabelWaves][kGenMaxN];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t row = static_cast<int64_t>(blockIdx.x) * kGenLabelWaves + w;
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  for (int j = lane; j < n; j += 64) {
    a[w][j] = static_cast<uint16_t>(j);
    grp[w][j] = 0;
  }
  for (int q = lane; 4 * q < n1; q += 64) {
    unsigned c[4] = {static_cast<unsigned>(q), row0 + static_cast<uint32_t>(row), kStreamLabels, 0u};
    philox4x32_10(c, k0, k1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * q + e;
      if (j < n1) tt[w][j] = static_cast<uint16_t>(j + index_below(c[e], static_cast<uint32_t>(n - j)));
    }
  }
  __syncthreads();
  if (lane == 0) {
    for (int j = 0; j < n1; ++j) {
      const int t = tt[w][j];
      const uint16_t x = a[w][t];
      a[w][t] = a[w][j];
      a[w][j] = x;
    }
  }
  __syncthreads();
  for (int j = lane; j < n1; j += 64) grp[w][a[w][j]] = 1;
  __syncthreads();
  if (row < L)
    for (int j = lane; j < n; j += 64) out[row * n + j] = grp[w][j];
}

// one workgroup per sampled set.  LDS: the draws, then the set, padded to P
// (a power of two) for the sort; the hash table of displaced entries (keys,
// values), S = a power of two >= 2 k slots
__global__ __launch_bounds__(kGenSetThreads) void gen_sets_kernel(uint64_t seed, uint32_t set_id, uint32_t row0,
                                                                  int64_t v, int k, int P, int S,
                                                                  int32_t* __restrict__ out) {
  extern __shared__ int32_t gsm[];
  int32_t* tt = gsm;
  int32_t* hk = tt + P;
  int32_t* hv = hk + S;
  const int tid = threadIdx.x;
  const uint32_t row = row0 + blockIdx.x;
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  for (int i = tid; i < S; i += kGenSetThreads) hk[i] = kGenSetEmpty;
  for (int i = k + tid; i < P; i += kGenSetThreads) tt[i] = INT32_MAX;
  for (int q = tid; 4 * q < k; q += kGenSetThreads) {
    unsigned c[4] = {static_cast<unsigned>(q), row, kStreamOmega, set_id};
    philox4x32_10(c, k0, k1);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = 4 * q + e;
      if (j < k) tt[j] = j + static_cast<int32_t>(index_below(c[e], static_cast<uint32_t>(v - j)));
    }
  }
  __syncthreads();
  if (tid == 0) {
    const unsigned shift = 32u - static_cast<unsigned>(__builtin_ctz(static_cast<unsigned>(S)));
    const unsigned mask = static_cast<unsigned>(S) - 1u;
    // slot of key: the key's own slot or the empty one that ends its probe
    auto slot = [&](int32_t key) -> unsigned {
      unsigned h = (static_cast<unsigned>(key) * 2654435761u) >> shift;
      while (hk[h] != kGenSetEmpty && hk[h] != key) h = (h + 1u) & mask;
      return h;
    };
    for (int j = 0; j < k; ++j) {
      const int32_t t = tt[j];
      const unsigned st = slot(t);
      const int32_t at_t = hk[st] == t ? hv[st] : t;
      const unsigned sj = slot(j);
      const int32_t at_j = hk[sj] == j ? hv[sj] : j;
      tt[j] = at_t;
      // entry j is never read again; entry t now holds the old entry j
      hk[st] = t;
      hv[st] = at_j;
    }
  }
  __syncthreads();
  // bitonic sort of tt[0 .. P), ascending (padding INT32_MAX sorts last)
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = tid; i < P; i += kGenSetThreads) {
        const int pr = i ^ stride;
        if (pr > i) {
          const int32_t x = tt[i], y = tt[pr];
          const bool up = (i & size) == 0;
          if ((x > y) == up) {
            tt[i] = y;
            tt[pr] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  int32_t* o = out + static_cast<int64_t>(blockIdx.x) * k;
  for (int j = tid; j < k; j += kGenSetThreads) o[j] = tt[j];
}

// thread per (voxel, group of four columns): one Philox call gives the four
// normals of columns 4g .. 4g+3 at voxel q (words 0, 1: cos, sin; 2, 3: cos,
// sin), the layout of the residual noise
__global__ __launch_bounds__(kBlock) void gen_start_kernel(uint64_t seed, int64_t v, int r, float* __restrict__ U) {
  const int groups = (r + 3) / 4;
  const int64_t id = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (id >= v * groups) return;
  const int64_t q = id / groups;
  const int g = static_cast<int>(id - q * groups);
  unsigned c[4] = {static_cast<unsigned>(q), static_cast<unsigned>(g), kStreamStart, 0u};
  philox4x32_10(c, static_cast<unsigned>(seed), static_cast<unsigned>(seed >> 32));
  float z[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const float rad = bm_radius(c[2 * h]), t = bm_turns(c[2 * h + 1]);
    z[2 * h] = rad * __builtin_amdgcn_cosf(t);
    z[2 * h + 1] = rad * __builtin_amdgcn_sinf(t);
  }
  float* row = U + q * r;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (4 * g + e < r) row[4 * g + e] = z[e];
}

size_t gen_sets_lds(int k) {
  return sizeof(int32_t) * (static_cast<size_t>(pow2_at_least(k)) + 2 * static_cast<size_t>(pow2_at_least(2 * k)));
}

}  // namespace

rpt_status gen_labels_check(int64_t row0, int64_t L, int32_t n, int32_t n1) {
  if (n < 2 || n > kGenMaxN || n1 < 1 || n1 >= n || row0 < 0 || L < 0 || L > INT32_MAX ||
      row0 + L > (int64_t{1} << 32))
    return RPT_ERR_INVALID_ARG;
  return RPT_OK;
}

rpt_status gen_sets_check(int32_t set_id, int64_t row0, int64_t rows, int64_t v, int32_t k) {
  if (set_id < 0 || row0 < 0 || rows < 0 || rows > INT32_MAX || row0 + rows > (int64_t{1} << 32) || v < 1 ||
      v > INT32_MAX || k < 1 || k > v)
    return RPT_ERR_INVALID_ARG;
  if (k > kGenMaxSet) return RPT_ERR_UNSUPPORTED;
  return RPT_OK;
}

rpt_status gen_labels_launch(uint64_t seed, int64_t row0, int64_t L, int32_t n, int32_t n1, uint8_t* labels,
                             hipStream_t s) {
  if (L == 0) return RPT_OK;
  const int64_t blocks = (L + kGenLabelWaves - 1) / kGenLabelWaves;
  gen_labels_kernel<<<dim3(static_cast<unsigned>(blocks)), dim3(64 * kGenLabelWaves), 0, s>>>(
      seed, static_cast<uint32_t>(row0), L, n, n1, labels);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status gen_sets_launch(uint64_t seed, int32_t set_id, int64_t row0, int64_t rows, int64_t v, int32_t k,
                           int32_t* omega, hipStream_t s) {
  if (rows == 0) return RPT_OK;
  const int P = pow2_at_least(k), S = pow2_at_least(2 * k);
  const size_t smem = gen_sets_lds(k);
  if (smem > 64 * 1024) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(gen_sets_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(smem)) != hipSuccess) {
      set_hip_error(hipGetLastError());
      return RPT_ERR_HIP;
    }
  }
  gen_sets_kernel<<<dim3(static_cast<unsigned>(rows)), dim3(kGenSetThreads), smem, s>>>(
      seed, static_cast<uint32_t>(set_id), static_cast<uint32_t>(row0), v, k, P, S, omega);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

rpt_status gen_start_launch(uint64_t seed, int64_t v, int32_t r, float* U, hipStream_t s) {
  const int64_t n = v * ((r + 3) / 4);
  if (n == 0) return RPT_OK;
  gen_start_kernel<<<dim3(static_cast<unsigned>((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(seed, v, r, U);
  RPT_CHECK_LAUNCH();
  return RPT_OK;
}

}  // namespace rpt

extern "C" {

int64_t rpt_sample_count(int64_t v, int32_t eta_ppm) {
  if (v < 0 || eta_ppm < 0 || eta_ppm > 1000000 || v > (INT64_MAX - 999999) / 1000000) return -1;
  return (static_cast<int64_t>(eta_ppm) * v + 999999) / 1000000;
}

rpt_status rpt_gen_relabellings(uint64_t seed, int64_t row0, int64_t L, int32_t n, int32_t n1, uint8_t* labels,
                                void* stream) {
  RPT_TRY(rpt::gen_labels_check(row0, L, n, n1));
  if (L > 0 && !labels) return RPT_ERR_INVALID_ARG;
  return rpt::gen_labels_launch(seed, row0, L, n, n1, labels, static_cast<hipStream_t>(stream));
}

rpt_status rpt_gen_sampled_sets(uint64_t seed, int32_t set_id, int64_t row0, int64_t rows, int64_t v, int32_t k,
                                int32_t* omega, void* stream) {
  RPT_TRY(rpt::gen_sets_check(set_id, row0, rows, v, k));
  if (rows > 0 && !omega) return RPT_ERR_INVALID_ARG;
  return rpt::gen_sets_launch(seed, set_id, row0, rows, v, k, omega, static_cast<hipStream_t>(stream));
}

rpt_status rpt_gen_start_basis(uint64_t seed, int64_t v, int32_t r, float* U, void* stream) {
  if (v < 0 || r < 1 || r > 4096 || (v > 0 && !U) || v > INT32_MAX) return RPT_ERR_INVALID_ARG;
  return rpt::gen_start_launch(seed, v, r, U, static_cast<hipStream_t>(stream));
}

}  // extern "C"
