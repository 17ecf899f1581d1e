// K3 + K4 -- Complete (Alg. 2): per column i, the masked least-squares fit
//     w_i = argmin_w | U[omega_i, :] w - y_i |_2
// from the normal equations G w = b, G = U_O^T U_O, b = U_O^T y.
//
// One workgroup (4 waves) per column.  The sampled rows are split between the
// waves in groups of 32; every lane loads its MFMA fragments straight from
// the basis (for a fixed sampled row, 16 lanes read 16 consecutive floats),
// splits them into BF16 hi/lo halves and accumulates the lower-triangular
// 16 x 16 tiles of G on the matrix cores as hi.hi + hi.lo + lo.hi (about 16
// significant bits per term, FP32 accumulation); b accumulates in FP64 from
// the FP32 values.  The per-wave partial tiles are summed into a packed FP64
// lower triangle in LDS with b^T appended as row r, so that the blocked
// Cholesky of that trapezoid leaves z = L^{-1} b in row r; one blocked back
// substitution gives w.  A non-positive pivot j sets info[i] = j + 1 and
// w_i = 0.  (Recovery, with many columns and no residuals, solves by
// conjugate gradients instead: see the split form below.)  Optionally the residual y - U_O w is written, and optionally each
// sampled entry (i, q) of a solved column is pushed onto the list of its voxel
// (lhead / lnext), so that a later pass can apply all entries of one voxel
// together without floating-point atomics.
#include "lds_linalg.h"
#include "pcg.h"
#include "rpt_internal.h"

namespace rpt {

namespace {

constexpr int kRMax = 128;  // basis rank handled in LDS
constexpr int kNW = 4;      // waves per workgroup
constexpr int kNT = 64 * kNW;
constexpr int kIdx = 1024;  // sampled indices / values staged in LDS at a time

struct CompleteArgs {
  const float* U;
  int64_t v;
  int r;
  const int32_t* omega;
  int k;
  const float* y;       // [L][k]  (or nullptr when Trows is used)
  const float* Trows;   // alternative source: y[i][q] = Trows[trow(i) * ldT + omega[i][q]]
  int64_t ldT;
  const int32_t* trow;  // row of Trows for column i (nullptr: row i)
  int64_t L;
  float* W;             // [L][r]
  float* resid;         // [L][k] or nullptr
  int32_t* info;        // [L]
  float* wnorm2;        // [L] |w|^2 (or nullptr)
  int32_t* lhead;       // [v] per-voxel list heads (-1 = empty) or nullptr
  int32_t* lnext;       // [L][k] list links of the sampled entries
  const int64_t* optr;  // CSR offsets of uneven sampled sets (nullptr: k per column)
};

// sampled value q of column i, whose entries start at base (i k, or the CSR offset)
__device__ __forceinline__ float y_at(const CompleteArgs& a, int64_t i, int64_t base, int q) {
  if (a.y) return a.y[base + q];
  const int64_t row = a.trow ? a.trow[i] : i;
  const int64_t vox = a.omega[base + q];
  return (vox >= 0 && vox < a.ldT) ? a.Trows[row * a.ldT + vox] : 0.0f;
}

// LDS layout (doubles first): G packed (r + 1)(r + 2)/2 rounded to even,
// P [kCb][kPanelLd], dinv [kRMax], w [kRMax], then ibuf [kIdx] int, ybuf [kIdx] float
__host__ __device__ inline int gsize(int r) { return (((r + 1) * (r + 2) / 2) + 1) & ~1; }
size_t smem_bytes(int r) {
  return (static_cast<size_t>(gsize(r)) + kCb * kPanelLd + 2 * kRMax) * sizeof(double) +
         kIdx * (sizeof(int) + sizeof(float));
}

// The Gram step of column i: the packed FP64 trapezoid G with b^T as row r,
// complete in LDS when it returns.
template <int RB>
__device__ __forceinline__ void gram_phase(const CompleteArgs& a, int64_t i, int64_t base, int k, double* G,
                                           int* ibuf, float* ybuf) {
  constexpr int NTILE = RB * (RB + 1) / 2;
  const int r = a.r;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, c16 = lane & 15, kq = lane >> 4;
  const int32_t* om = a.omega + base;
  const int nrows = r + 1, ntri = nrows * (nrows + 1) / 2;
  for (int t = tid; t < ntri; t += kNT) G[t] = 0.0;

  f32x4 acc[NTILE];
#pragma unroll
  for (int t = 0; t < NTILE; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  double bacc[RB];
#pragma unroll
  for (int b = 0; b < RB; ++b) bacc[b] = 0.0;

  float x[RB][8];
  for (int b0 = 0; b0 < k; b0 += kIdx) {
    const int nb = k - b0 < kIdx ? k - b0 : kIdx;
    const int ngr = (nb + 31) >> 5;
    __syncthreads();  // previous index block fully consumed (and G cleared)
    for (int t = tid; t < ngr * 32; t += kNT) {
      const bool in = t < nb;
      const int64_t row = in ? om[b0 + t] : -1;
      ibuf[t] = (row >= 0 && row < a.v) ? static_cast<int>(row) : -1;  // out of range: zero row
      ybuf[t] = in ? y_at(a, i, base, b0 + t) : 0.0f;
    }
    __syncthreads();
    auto load = [&](int g) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int row = ibuf[32 * g + 8 * kq + j];
        const float* u = a.U + static_cast<int64_t>(row) * r;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
          const int c = 16 * b + c16;
          x[b][j] = (row >= 0 && c < r) ? u[c] : 0.0f;
        }
      }
    };
    // no register prefetch of the next group: x and the hi/lo fragments are
    // never live together (the other waves of the SIMD cover the latency)
    for (int g = wave; g < ngr; g += kNW) {
      load(g);
      u32x4 hi[RB], lo[RB];
      float yv[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) yv[j] = ybuf[32 * g + 8 * kq + j];
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          const uint16_t h0 = f2bf(x[b][j]), h1 = f2bf(x[b][j + 1]);
          hi[b][j >> 1] = pack_bf2(h0, h1);
          lo[b][j >> 1] = pack_bf2(f2bf(x[b][j] - bf2f(h0)), f2bf(x[b][j + 1] - bf2f(h1)));
          s = fma(static_cast<double>(x[b][j]), static_cast<double>(yv[j]), s);
          s = fma(static_cast<double>(x[b][j + 1]), static_cast<double>(yv[j + 1]), s);
        }
        bacc[b] += s;
      }
      int t = 0;
#pragma unroll
      for (int bi = 0; bi < RB; ++bi)
#pragma unroll
        for (int bj = 0; bj <= bi; ++bj) {
          acc[t] = mfma16_bf16(hi[bi], hi[bj], acc[t]);
          acc[t] = mfma16_bf16(hi[bi], lo[bj], acc[t]);
          acc[t] = mfma16_bf16(lo[bi], hi[bj], acc[t]);
          ++t;
        }
    }
  }
  // partial tiles and b of every wave summed into the packed FP64 trapezoid
  {
    int t = 0;
#pragma unroll
    for (int bi = 0; bi < RB; ++bi)
#pragma unroll
      for (int bj = 0; bj <= bi; ++bj) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = 16 * bi + 4 * kq + e, col = 16 * bj + c16;
          if (row < r && col <= row) atomicAdd(&G[ptri(row, col)], static_cast<double>(acc[t][e]));
        }
        ++t;
      }
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      double s = bacc[b];
      s += __shfl_xor(s, 16, 64);
      s += __shfl_xor(s, 32, 64);
      const int c = 16 * b + c16;
      if (kq == 0 && c < r) atomicAdd(&G[ptri(r, c)], s);
    }
  }
  __syncthreads();
}

// Cholesky, back substitution and the outputs of column i from the
// trapezoid G in LDS (P: kCb rows of pld doubles).
template <int RB>
__device__ __forceinline__ void solve_phase(const CompleteArgs& a, int64_t i, int64_t base, int k, double* G,
                                            double* P, int pld, double* dinv, double* wv) {
  const int r = a.r;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int32_t* om = a.omega + base;
  const int nrows = r + 1;
  const int failed = lds_cholesky_blocked<(RB >= 8 ? 3 : 2)>(G, dinv, P, r, nrows, pld);
  float* Wi = a.W + i * r;
  if (failed) {
    for (int c = tid; c < r; c += kNT) Wi[c] = 0.0f;
    if (tid == 0) {
      a.info[i] = failed;
      if (a.wnorm2) a.wnorm2[i] = 0.0f;
    }
    if (a.resid)
      for (int q = tid; q < k; q += kNT) a.resid[base + q] = y_at(a, i, base, q);
    return;
  }
  for (int c = tid; c < r; c += kNT) wv[c] = G[ptri(r, c)];
  lds_chol_backsolve(G, dinv, wv, r);
  for (int c = tid; c < r; c += kNT) Wi[c] = static_cast<float>(wv[c]);
  if (wave == 0) {
    double nrm = 0.0;
    for (int c = lane; c < r; c += 64) nrm = fma(wv[c], wv[c], nrm);
    nrm = wave_sum_d(nrm);
    if (lane == 0) {
      a.info[i] = 0;
      if (a.wnorm2) a.wnorm2[i] = static_cast<float>(nrm);
    }
  }
  if (a.resid) {
    // one sampled row per thread: every load of the row is independent, so a
    // thread's whole row is in flight at once
    __syncthreads();
    const bool vec = (r & 3) == 0 && (reinterpret_cast<uintptr_t>(a.U) & 15) == 0;
    for (int q = tid; q < k; q += kNT) {
      const int64_t row = om[q];
      const float yq = y_at(a, i, base, q);
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      if (row >= 0 && row < a.v) {
        const float* u = a.U + row * r;
        if (vec) {
          for (int c = 0; c < r; c += 4) {
            const f32x4 x4 = *reinterpret_cast<const f32x4*>(u + c);
            s0 = fma(static_cast<double>(x4[0]), wv[c], s0);
            s1 = fma(static_cast<double>(x4[1]), wv[c + 1], s1);
            s2 = fma(static_cast<double>(x4[2]), wv[c + 2], s2);
            s3 = fma(static_cast<double>(x4[3]), wv[c + 3], s3);
          }
        } else {
          for (int c = 0; c < r; ++c) s0 = fma(static_cast<double>(u[c]), wv[c], s0);
        }
      }
      a.resid[base + q] = static_cast<float>(yq - ((s0 + s1) + (s2 + s3)));
      if (a.lhead && row >= 0 && row < a.v) {
        const int32_t e = static_cast<int32_t>(base + q);
        a.lnext[e] = atomicExch(a.lhead + row, e);
      }
    }
  } else if (a.lhead) {
    // lists only: the tracking update forms the residual itself
    for (int q = tid; q < k; q += kNT) {
      const int64_t row = om[q];
      if (row >= 0 && row < a.v) {
        const int32_t e = static_cast<int32_t>(base + q);
        a.lnext[e] = atomicExch(a.lhead + row, e);
      }
    }
  }
}

template <int RB>
__global__ __launch_bounds__(kNT, (RB >= 8 ? 1 : 2)) void complete_kernel(CompleteArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* G = reinterpret_cast<double*>(smem);
  double* P = G + gsize(a.r);
  double* dinv = P + kCb * kPanelLd;
  double* wv = dinv + kRMax;
  int* ibuf = reinterpret_cast<int*>(wv + kRMax);
  float* ybuf = reinterpret_cast<float*>(ibuf + kIdx);
  const int64_t i = blockIdx.x;
  const int64_t base = a.optr ? a.optr[i] : i * a.k;
  const int k = a.optr ? static_cast<int>(a.optr[i + 1] - base) : a.k;
  gram_phase<RB>(a, i, base, k, G, ibuf, ybuf);
  solve_phase<RB>(a, i, base, k, G, P, kPanelLd, dinv, wv);
}

// ---------------------------------------------------------------- split form
// For many columns without residuals (recovery) the two steps run as two
// kernels: the Gram kernel writes G (FP32, rounded once from its exact FP64
// sum of the wave partials) and b (FP64) of every column to global memory,
// and the solve kernel (below) fits each column by conjugate gradients.
__host__ __device__ inline int ntri_r(int r) { return r * (r + 1) / 2; }
__host__ __device__ inline size_t gb_stride(int r) {  // bytes per column: G floats, then b doubles
  return ((static_cast<size_t>(ntri_r(r)) * sizeof(float) + 7) & ~static_cast<size_t>(7)) +
         static_cast<size_t>(r) * sizeof(double);
}
inline size_t gram_smem(int r) {
  return static_cast<size_t>(gsize(r)) * sizeof(double) + kIdx * (sizeof(int) + sizeof(float));
}

template <int RB>
__global__ __launch_bounds__(kNT, 2) void complete_gram_kernel(CompleteArgs a, char* gb) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* G = reinterpret_cast<double*>(smem);
  int* ibuf = reinterpret_cast<int*>(G + gsize(a.r));
  float* ybuf = reinterpret_cast<float*>(ibuf + kIdx);
  const int64_t i = blockIdx.x;
  const int64_t base = a.optr ? a.optr[i] : i * a.k;
  const int k = a.optr ? static_cast<int>(a.optr[i + 1] - base) : a.k;
  gram_phase<RB>(a, i, base, k, G, ibuf, ybuf);
  const int r = a.r, nt = ntri_r(r);
  float* go = reinterpret_cast<float*>(gb + i * gb_stride(r));
  double* bo = reinterpret_cast<double*>(gb + i * gb_stride(r) + gb_stride(r) - static_cast<size_t>(r) * sizeof(double));
  for (int t = threadIdx.x; t < nt; t += kNT) go[t] = static_cast<float>(G[t]);  // rows < r are entries [0, nt)
  for (int c = threadIdx.x; c < r; c += kNT) bo[c] = G[nt + c];                  // row r
}

// The recovery solve by conjugate gradients: G (packed lower FP32) is
// stored whole in LDS and b (FP64) is the right-hand side of the
// Jacobi-preconditioned conjugate gradients that the tracking pass also uses
// (pcg.h); a well-conditioned r x r system takes 10 to 20 iterations, a
// fraction of a Cholesky factorisation's dependent chain.  A set with fewer
// than r voxels fails as the factorisation would (info = its size + 1);
// non-positive curvature gives -1 and no convergence -2, with w = 0.
struct CgVec {
  double zv[kGR];
  double mv[2][kGR];
  double gv[kGR];  // b
  double cgr[2][kGWaves][2];
  double red[4][kGWaves];
  int badf[kGWaves];
  float zf[kGR];
};
__host__ __device__ inline size_t cg_smem(int rb) {
  return ((sizeof(CgVec) + 15) & ~static_cast<size_t>(15)) + sizeof(float) * 16 * rb * g_hld(rb);
}

template <int RB>
__global__ __launch_bounds__(kNT, 2) void complete_cg_kernel(CompleteArgs a, const char* gb) {
  extern __shared__ __align__(16) unsigned char smem[];
  static_assert(kNT == kGT, "the solver's layout takes four waves");
  constexpr int hld = g_hld(RB);
  CgVec& sv = *reinterpret_cast<CgVec*>(smem);
  float* H = reinterpret_cast<float*>(smem + ((sizeof(CgVec) + 15) & ~static_cast<size_t>(15)));
  const int r = a.r;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i = blockIdx.x;
  const int k = a.optr ? static_cast<int>(a.optr[i + 1] - a.optr[i]) : a.k;
  float* Wi = a.W + i * r;
  if (k < r) {
    for (int c = tid; c < r; c += kNT) Wi[c] = 0.0f;
    if (tid == 0) a.info[i] = k + 1;
    return;
  }
  const float* gi = reinterpret_cast<const float*>(gb + i * gb_stride(r));
  const double* bi = reinterpret_cast<const double*>(gb + i * gb_stride(r) + gb_stride(r) -
                                                     static_cast<size_t>(r) * sizeof(double));
  // row `row` of the packed triangle is contiguous: one wave per row
  for (int row = wave; row < r; row += kNW) {
    const float* gr = gi + (row * (row + 1)) / 2;
    for (int col = lane; col <= row; col += 64) {
      const float g = gr[col];
      H[row * hld + col] = g;
      H[col * hld + row] = g;
    }
  }
  for (int c = tid; c < kGR; c += kNT) {
    sv.gv[c] = c < r ? bi[c] : 0.0;
    sv.zv[c] = 0.0;
  }
  __syncthreads();
  const int rq = lane >> 4, cb = lane & 15, rbase = 32 * wave + 8 * rq, myrow = rbase + (cb >> 1);
  const int fail = pcg_solve<hld, true>(H, r, sv, lane, wave, rbase, cb, myrow, (cb & 1) == 0, myrow < r, sv.gv);
  for (int c = tid; c < r; c += kNT) Wi[c] = fail ? 0.0f : sv.zf[c];
  if (tid == 0) {
    a.info[i] = fail ? -fail : 0;
    if (a.wnorm2) {
      double t = 0.0;
      for (int c = 0; c < r; ++c) t = fma(sv.zv[c], sv.zv[c], t);
      a.wnorm2[i] = fail ? 0.0f : static_cast<float>(t);
    }
  }
}

}  // namespace

size_t complete_split_bytes(int64_t L, int r) { return static_cast<size_t>(L > 0 ? L : 1) * gb_stride(r); }

rpt_status complete_run(const float* U, int64_t v, int r, const int32_t* omega, int k, const float* y,
                        const float* Trows, int64_t ldT, const int32_t* trow, int64_t L, float* W, float* resid,
                        int32_t* info, float* wnorm2, hipStream_t s, int32_t* lhead, int32_t* lnext,
                        const int64_t* optr, void* split_ws) {
  if (L == 0) return RPT_OK;
  if (r < 1 || r > kRMax) return RPT_ERR_UNSUPPORTED;
  if (lhead && (!lnext || optr || L * static_cast<int64_t>(k) > INT32_MAX)) return RPT_ERR_INVALID_ARG;
  CompleteArgs a{U, v, r, omega, k, y, Trows, ldT, trow, L, W, resid, info, wnorm2, lhead, lnext, optr};
  const int RB = (r + 15) / 16;
#define RPT_FNS(K) \
  { reinterpret_cast<void*>(&K<1>), reinterpret_cast<void*>(&K<2>), reinterpret_cast<void*>(&K<3>), \
    reinterpret_cast<void*>(&K<4>), reinterpret_cast<void*>(&K<5>), reinterpret_cast<void*>(&K<6>), \
    reinterpret_cast<void*>(&K<7>), reinterpret_cast<void*>(&K<8>) }
  static void* const fused[8] = RPT_FNS(complete_kernel);
  static void* const gram[8] = RPT_FNS(complete_gram_kernel);
  static void* const solve[8] = RPT_FNS(complete_cg_kernel);
#undef RPT_FNS
  static bool attr_set[8] = {};
  if (!attr_set[RB - 1]) {
    (void)hipFuncSetAttribute(fused[RB - 1], hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(smem_bytes(kRMax)));
    (void)hipFuncSetAttribute(gram[RB - 1], hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(gram_smem(kRMax)));
    (void)hipFuncSetAttribute(solve[RB - 1], hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(cg_smem(RB)));
    attr_set[RB - 1] = true;
  }
  hipError_t e = hipSuccess;
  if (split_ws && !resid) {
    char* gb = static_cast<char*>(split_ws);
    const char* cgb = gb;
    void* ga[] = {&a, &gb};
    void* sa[] = {&a, &cgb};
    {
      RPT_STAGE("complete_gram", s);
      e = hipLaunchKernel(gram[RB - 1], dim3(static_cast<unsigned>(L)), dim3(kNT), ga, gram_smem(r), s);
    }
    if (e == hipSuccess) {
      RPT_STAGE("complete_solve", s);
      e = hipLaunchKernel(solve[RB - 1], dim3(static_cast<unsigned>(L)), dim3(kNT), sa, cg_smem(RB), s);
    }
  } else {
    RPT_STAGE("complete", s);
    void* args[] = {&a};
    e = hipLaunchKernel(fused[RB - 1], dim3(static_cast<unsigned>(L)), dim3(kNT), args, smem_bytes(r), s);
  }
  if (e != hipSuccess) {
    set_hip_error(e);
    return RPT_ERR_HIP;
  }
  return RPT_OK;
}

}  // namespace rpt
