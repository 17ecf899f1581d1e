// Internal declarations of librpt (HIP, gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <mutex>

#include "rpt.h"

namespace rpt {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;

constexpr int kWave = 64;
constexpr int kBlock = 256;          // 4 waves per workgroup
constexpr float kZBound = 5.8872f;   // > sqrt(50 ln 2): largest |z| of the noise map

// ---------------------------------------------------------------------------
// error reporting
void set_hip_error(hipError_t e);

#define RPT_CHECK_LAUNCH()                              \
  do {                                                  \
    hipError_t e_ = hipGetLastError();                  \
    if (e_ != hipSuccess) {                             \
      ::rpt::set_hip_error(e_);                         \
      return RPT_ERR_HIP;                               \
    }                                                   \
  } while (0)

#define RPT_TRY(expr)                      \
  do {                                     \
    rpt_status s_ = (expr);                \
    if (s_ != RPT_OK) return s_;           \
  } while (0)

// ---------------------------------------------------------------------------
// per-stage timing (timing.hip): records HIP events around a kernel stage on
// the stage's stream when timing is enabled through the C ABI.
class StageScope {
 public:
  StageScope(const char* name, hipStream_t s);
  ~StageScope();
  StageScope(const StageScope&) = delete;
  StageScope& operator=(const StageScope&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  hipEvent_t start_;
};
#define RPT_CAT2(a, b) a##b
#define RPT_CAT(a, b) RPT_CAT2(a, b)
#define RPT_STAGE(name, stream) ::rpt::StageScope RPT_CAT(rpt_stage_, __LINE__)(name, stream)

// ---------------------------------------------------------------------------
// workspace carving: every piece 256-byte aligned.  With base == nullptr the
// carver only measures.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ---------------------------------------------------------------------------
// device helpers
__device__ __forceinline__ uint16_t f2bf(float x) {
  // round to nearest even; inputs are finite
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ f32x16 mfma_bf16(const u32x4& a, const u32x4& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                  c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16_bf16(const u32x4& a, const u32x4& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                  c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_f32(float a, float b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row of the 32x32 MFMA output held by accumulator register e of a lane in
// half h (= lane / 32); the column is lane % 32.
__device__ __forceinline__ int mfma_row(int e, int h) { return 8 * (e >> 2) + 4 * h + (e & 3); }
// 16x16x32: lane l holds K = 8 (l / 16) .. + 7 of row (A) / column (B) l % 16;
// accumulator register e holds row 4 (l / 16) + e, column l % 16.
__device__ __forceinline__ uint32_t pack_bf2(uint16_t lo, uint16_t hi) {
  return static_cast<uint32_t>(lo) | (static_cast<uint32_t>(hi) << 16);
}

__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
  return x;
}
__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// ordered-int encoding so that unsigned atomicMax orders floats
__device__ __forceinline__ unsigned float_to_ordered(float f) {
  unsigned u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ordered_to_float(unsigned u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u);
}

// ---------------------------------------------------------------------------
// Balanced-design t from the scaled group contrast u (see prep.hip):
// t = 2u sqrt((m-1)/m) / sqrt(1 - 2u^2/m), m = n/2.  Monotone in u.
__host__ __device__ inline double t_from_u(double u, int m) {
  double d = 1.0 - 2.0 * u * u / m;
  double num = 2.0 * u * sqrt((m - 1.0) / m);
  if (d <= 0.0) return u == 0.0 ? 0.0 : (u > 0 ? INFINITY : -INFINITY);
  return num / sqrt(d);
}
__device__ __forceinline__ float t_from_u_f(float u, float fs, float tm) {
  // fs = 2 sqrt((m-1)/m), tm = 2/m
  float d = fmaxf(fmaf(-tm * u, u, 1.0f), 0.0f);
  return u == 0.0f ? 0.0f : u * fs * rsqrtf(d);
}

// ---------------------------------------------------------------------------
// Prepared data of one X (see prep.hip for the layouts).
struct PrepX {
  int64_t v = 0, vpad = 0;   // vpad = v rounded up to 32 voxels
  int n = 0, n1 = 0;
  int ksteps = 0;            // split: 16-wide K blocks; f32: 8-subject blocks
  uint16_t* kb16 = nullptr;  // split: [ksteps][vpad][2][16] bf16 (hi block, lo block)
  uint16_t* kbm = nullptr;   // split, R = n mod 16 in 1..8: per 32-voxel tile the mixed
                             // K block [hi of the last R subjects | their lo | 0]
  int mixr = 0;              // R when kbm is written, else 0
  float* kb32 = nullptr;     // f32:   [ksteps][vpad][2][4]   (subject 8s+2q+h)
  float* kb32sq = nullptr;   // f32 unbalanced: same layout, squared values
  float* rows = nullptr;     // [vpad][ldn] standardised rows (sampled t)
  int ldn = 0;
  float2* cst = nullptr;     // [vpad] balanced epilogue (rinv, -h*rinv)
  float2* cstg = nullptr;    // [vpad] unbalanced epilogue (S, Q)
  int stat = RPT_STAT_T;     // statistic the constants were made for
};
// (fs, tm) of t_from_u_f for the prepared statistic: Eq. 2's t, or the mean
// difference 2 u / m (fs = 2 / m, tm = 0)
inline void stat_consts(const PrepX& p, float* fs, float* tm) {
  const int m = p.n / 2;
  if (p.stat == RPT_STAT_MEANDIFF) {
    *fs = static_cast<float>(2.0 / m);
    *tm = 0.0f;
  } else {
    *fs = static_cast<float>(2.0 * sqrt((m - 1.0) / m));
    *tm = static_cast<float>(2.0 / m);
  }
}

// kPrepMeanDiff: the statistic is the linear mean difference m1 - m2 instead
// of Eq. 2's t (balanced designs): the rows are centred but not scaled in the
// contraction's constants, so u is the centred group-1 sum and the statistic
// is 2 u / m, again one increasing function of u shared by all voxels
enum PrepFlags { kPrepSplit = 1, kPrepF32 = 2, kPrepRows = 4, kPrepUnbal = 8, kPrepMeanDiff = 16 };
inline int stat_flags(int stat) { return stat == RPT_STAT_MEANDIFF ? kPrepMeanDiff : 0; }

size_t prep_bytes(int64_t v, int n, int flags);
PrepX prep_carve(Carver& c, int64_t v, int n, int n1, int flags);
rpt_status prep_launch(const PrepX& p, const float* X, int64_t ldx, int tail, int flags, hipStream_t s);

// NaivePT contraction; writes per-(chunk, perm) maxima or T rows.
struct NaivePlan {
  int pt = 4;       // perm tiles (32 perms) per wave
  int pg = 0;       // perm groups
  int nc = 0;       // voxel chunks (multiple of 8)
  int tpc = 0;      // voxel tiles per chunk
  int64_t vt = 0;   // voxel tiles
  int nc_heur = 0;  // the rule-of-thumb chunk count
  int nc_cap = 0;   // the largest candidate (workspace bound)
};
// force_nc > 0 replaces the chunk count (the autotuner's trials)
NaivePlan naive_plan(int64_t v, int64_t L, int n, int prec, bool store, int force_nc = 0);

// Voxel-chunk counts chosen by measurement (tune.hip): the candidates around
// the planner's rule of thumb (ascending, at most 6), the largest of them, and
// the table of measured choices keyed by kernel and shape (0: none).
enum { kTuneNaive = 0, kTuneRecon = 1 };
constexpr int kMaxChunkCandidates = 6;
int chunk_candidates(int64_t nc_heur, int64_t ncmax, int* out);
int64_t chunk_cap(int64_t nc_heur, int64_t ncmax);
int tuned_chunks(int kernel, int64_t v, int64_t L, int dim, int variant);
void set_tuned_chunks(int kernel, int64_t v, int64_t L, int dim, int variant, int nc);
size_t naive_bytes(int64_t v, int n, int64_t L, int prec);
rpt_status naive_launch(const PrepX& p, const NaivePlan& plan, const uint8_t* labels, int64_t L, int tail,
                        int prec, float* partial, float* T_out, float* max_out, hipStream_t s);

// Sampled t statistics (K2).
rpt_status sampled_launch(const PrepX& p, const uint8_t* labels, int64_t L, const int32_t* omega, int k,
                          const float* Tsrc, float* y, hipStream_t s,
                          const int64_t* optr = nullptr);

// The per-device second stream (streams.hip) and its events; `to` waits for
// everything enqueued on `from` so far.  side_stream returns null when the
// stream cannot be created (or is first asked for during graph capture).
struct SideStream {
  bool ok = false;
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, mid = nullptr, join = nullptr, step = nullptr;
  std::mutex mu;
};
SideStream* side_stream(hipStream_t s);
rpt_status stream_wait(SideStream* sd, hipEvent_t ev, hipStream_t from, hipStream_t to);

// Complete (Gram + FP64 Cholesky + solve).  The sampled values come either from
// y ([L][k]) or, when y is null, from rows of T: y[i][q] = Trows[i * ldT + omega[i][q]].
// With split_ws (complete_split_bytes(L, r) bytes) and no residual, the Gram
// step and the solve run as two kernels with the Gram matrices in split_ws.
size_t complete_split_bytes(int64_t L, int r);
rpt_status complete_run(const float* U, int64_t v, int r, const int32_t* omega, int k, const float* y,
                        const float* Trows, int64_t ldT, const int32_t* trow, int64_t L, float* W, float* resid,
                        int32_t* info, float* wnorm2, hipStream_t s, int32_t* lhead = nullptr,
                        int32_t* lnext = nullptr, const int64_t* optr = nullptr, void* split_ws = nullptr);

// Reconstruction filter + exact refine with noise (K7).
// ks: U slices of 16 columns held for the reconstruction (0: ceil(r / 16))
size_t recon_bytes(int64_t v, int64_t L, int r, int ks = 0);
rpt_status recon_launch(const float* U, int64_t v, int r, const float* W, int64_t L, int64_t col0,
                        uint64_t seed, int stream_id, const float* sigma_mu, float* out_max,
                        const float* Tmax_for_gap, float* gap_out, void* ws, hipStream_t s, unsigned study = 0,
                        int force_nc = 0);
// the fused reconstruction's chunk-count candidates for one shape (tune.hip)
int recon_chunk_candidates(int64_t v, int64_t L, int r, int* out);
// Reconstruction of several studies with one persistent fused launch (per
// group of up to 16 studies): recon_prepare_study for each study once its W is
// written (ws: recon_bytes(v, L, r, ks) bytes of its own), then recon_batched.
struct ReconStudy {
  const float* U;
  int64_t v;
  int r;
  const float* W;
  int64_t L;
  int64_t col0;
  uint64_t seed;
  const float* sigma_mu;
  float* out_max;
  void* ws;
  unsigned study;
};
int recon_batch_ks(const ReconStudy* st, int ns);
size_t recon_batch_counters(int ns);  // int32 counters recon_batched needs
rpt_status recon_prepare_study(const ReconStudy& st, int ks, hipStream_t s);
rpt_status recon_batched(const ReconStudy* st, int ns, int ks, int* counters, hipStream_t s);

// Orthonormalisation (one Cholesky-QR pass).  before_chol, when given, is
// called once the Gram reduction is enqueued and before the single-workgroup
// Cholesky (a point where the rest of the chip is about to idle).  With stop
// given, every kernel of the pass does nothing once *stop < pass (a
// converged tracking loop, decided on the device).
size_t reorth_bytes(int64_t v, int r);
rpt_status reorth_launch(float* U, int64_t v, int r, int32_t* info, void* ws, hipStream_t s,
                         const std::function<rpt_status()>* before_chol = nullptr, const int32_t* stop = nullptr,
                         int pass = 0);

// Training helpers (train.hip).
// U[x] += gamma sum_e resid[e] W[i(e)] / |w_i(e)|^2 over the entries linked
// at voxel x by complete_run (i(e) = e / k); every list head is reset to -1.
rpt_status track_apply_launch(float* U, int64_t v, int r, int k, const float* T, int64_t ldT, const float* W,
                              const float* wnorm2, const int32_t* info, float gamma, int32_t* lhead,
                              const int32_t* lnext, hipStream_t s);
rpt_status fill_i32(int32_t* p, int64_t n, int32_t value, hipStream_t s);
// The masked-loss-driven step: W^T (r x nb) and CSR offsets b k of a batch;
// U += a G; *out += sum e^2 (one workgroup, fixed order)
rpt_status grad_prep_launch(const float* W, int nb, int r, float* WT, int64_t* ptr, int k, hipStream_t s);
rpt_status axpy_launch(float* U, const float* G, int64_t n, float a, hipStream_t s);
rpt_status sumsq_add_launch(const float* e, int64_t n, double* out, hipStream_t s);
rpt_status sigma_launch(const float* resid, int64_t n, double* sums, float* sigma_mu, hipStream_t s);
rpt_status mu_launch(const float* vals, int n, int rule, float* sigma_mu, hipStream_t s);
rpt_status literal_resid_launch(const float* T, const float* U, const float* W, int64_t v, int r, int64_t ell,
                                float* out, hipStream_t s);

// Column-by-column subspace tracking (grouse.hip): the basis factor B of
// U = B N^{-1} is updated in place; the workspace holds the cooperative
// pass's partial Gram tiles, their sums, the partial residual norms and
// right-hand sides, the grid-barrier counters, the objectives of the last
// two passes and the convergence flags.
struct GrouseState {
  float* part = nullptr;     // partial Gram tiles of the cooperative pass
  float* hred = nullptr;     // their sums
  double* epart = nullptr;   // partial |e|^2
  float* gpart = nullptr;    // partial right-hand sides of the l1 fit
  uint32_t* ctr = nullptr;   // grid-barrier counters [2]
  int32_t* abort = nullptr;  // raised when a grid-barrier wait expires
  double* objr = nullptr;
  int32_t* stop = nullptr;
  int32_t* used_ws = nullptr;
  int32_t* rinfo = nullptr;  // status of the end-of-pass orthonormalisation
  float* xo = nullptr;       // [ell][k] the pass's sampled values in set order
};
size_t grouse_bytes(int r, int k, int ell);
GrouseState grouse_carve(void* ws, int r, int k, int ell);
// stop <- none, passes used <- 0 (used: caller's device int, or the workspace's),
// obj_out[0 .. passes) <- 0 when given
rpt_status grouse_init_launch(const GrouseState& g, int32_t* used, double* obj_out, int passes, hipStream_t s);
// The tracker: GROUSE (mode RPT_TRACK_GROUSE) or the robust l1 fit with
// the ADMM penalty rho and admm_iters iterations per column (RPT_TRACK_L1).
struct TrackOpts {
  int mode = RPT_TRACK_GROUSE;
  float rho = 1.0f;
  int admm_iters = 30;
};
// One pass of tracking steps over the ell training columns (rows of T,
// leading dimension ldT) with this pass's sampled sets (ell x k); B ends as
// a basis factor of the tracked subspace (the caller orthonormalises it).
// Skipped on the device once an earlier pass met the stopping rule.
rpt_status grouse_pass_launch(const GrouseState& g, float* B, int64_t v, int r, const float* T, int64_t ldT,
                              const int32_t* omega, int k, int ell, float gamma, int pass, double tol,
                              double* obj_out, int32_t* used, int32_t* info, const TrackOpts& opt, hipStream_t s);

// Masked loss (masked_loss.hip).
rpt_status loss_fwd_launch(const float* U, int64_t v, int r, const float* W, int B, const int64_t* ptr, const int32_t* idx,
                           const float* t, double* loss, float* resid, hipStream_t s);
rpt_status loss_bwd_launch(const float* U, int64_t v, int r, const float* W, int B, const int64_t* ptr,
                           const int32_t* idx, const float* e, float* dU, float* dW, const double* grad_scale, hipStream_t s);

// Inputs drawn from a seed (gen.hip): relabellings (stream 0), sampled sets
// (stream 1, at most kGenMaxSet voxels each) and the Gaussian start basis
// (stream 3).  The checks are synchronous; the launches assume them passed.
constexpr int kGenMaxSet = 4096;
rpt_status gen_labels_check(int64_t row0, int64_t L, int32_t n, int32_t n1);
rpt_status gen_sets_check(int32_t set_id, int64_t row0, int64_t rows, int64_t v, int32_t k);
rpt_status gen_labels_launch(uint64_t seed, int64_t row0, int64_t L, int32_t n, int32_t n1, uint8_t* labels,
                             hipStream_t s);
rpt_status gen_sets_launch(uint64_t seed, int32_t set_id, int64_t row0, int64_t rows, int64_t v, int32_t k,
                           int32_t* omega, hipStream_t s);
rpt_status gen_start_launch(uint64_t seed, int64_t v, int32_t r, float* U, hipStream_t s);

}  // namespace rpt
