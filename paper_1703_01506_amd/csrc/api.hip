// C ABI of librpt: argument validation, workspace carving and launch order.
// Every entry point enqueues on the caller's stream and never synchronises.
#include <algorithm>
#include <mutex>
#include <vector>

#include "rpt_internal.h"

namespace rpt {

static thread_local int g_last_hip_error = 0;
void set_hip_error(hipError_t e) { g_last_hip_error = static_cast<int>(e); }

namespace {

bool ws_ok(const void* ws, size_t have, size_t need) {
  if (need == 0) return true;
  return ws != nullptr && (reinterpret_cast<uintptr_t>(ws) & 255u) == 0 && have >= need;
}

bool design_ok(int64_t v, int32_t n, int64_t ldx, int32_t n1) {
  return v >= 1 && n >= 4 && n <= 512 && ldx >= n && n1 >= 2 && n1 <= n - 2;
}

bool stat_ok(int stat, int32_t n, int32_t n1) {
  return stat == RPT_STAT_T || (stat == RPT_STAT_MEANDIFF && 2 * n1 == n);
}

int naive_flags(int prec, bool unbal) {
  if (prec == RPT_SPLIT_BF16) return kPrepSplit;
  return kPrepF32 | (unbal ? kPrepUnbal : 0);
}

}  // namespace
}  // namespace rpt

using namespace rpt;

extern "C" {

const char* rpt_status_string(int status) {
  switch (status) {
    case RPT_OK: return "ok";
    case RPT_ERR_INVALID_ARG: return "invalid argument";
    case RPT_ERR_UNDERDETERMINED: return "sampled set smaller than the rank";
    case RPT_ERR_NOT_SPD: return "sampled Gram matrix not positive definite";
    case RPT_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case RPT_ERR_HIP: return "HIP launch failed";
    case RPT_ERR_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

int rpt_last_hip_error(void) { return g_last_hip_error; }

int rpt_version(void) { return 100; }

size_t rpt_naive_workspace(int64_t v, int32_t n, int64_t L, int prec) {
  if (v < 1 || n < 4 || L < 0) return 0;
  Carver c(nullptr);
  prep_carve(c, v, n, n / 2, naive_flags(prec, false) | (prec == RPT_FP32 ? kPrepUnbal : 0));
  return c.off + naive_bytes(v, n, L, prec);
}

rpt_status rpt_naive_maxnull(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* labels,
                             int64_t L, int tail, int prec, int stat, float* max_out, float* T_out, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!design_ok(v, n, ldx, n1) || L < 0) return RPT_ERR_INVALID_ARG;
  if (stat != RPT_STAT_T && stat != RPT_STAT_MEANDIFF) return RPT_ERR_INVALID_ARG;
  if (!stat_ok(stat, n, n1)) return RPT_ERR_UNSUPPORTED;
  if (tail != RPT_TAIL_SIGNED && tail != RPT_TAIL_ABS) return RPT_ERR_INVALID_ARG;
  if (prec != RPT_FP32 && prec != RPT_SPLIT_BF16) return RPT_ERR_INVALID_ARG;
  if (L > 0 && (!X || !labels || (!max_out && !T_out))) return RPT_ERR_INVALID_ARG;
  const bool unbal = 2 * n1 != n;
  if (unbal && prec != RPT_FP32) return RPT_ERR_UNSUPPORTED;
  if (prec == RPT_FP32 && n > 128) return RPT_ERR_UNSUPPORTED;  // FP32 path: fragments for up to 128 subjects
  if (!ws_ok(ws, ws_bytes, rpt_naive_workspace(v, n, L, prec))) return RPT_ERR_WORKSPACE;
  if (L == 0) return RPT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int flags = naive_flags(prec, unbal) | stat_flags(stat);
  Carver c(ws);
  PrepX p = prep_carve(c, v, n, n1, flags);
  const NaivePlan pl = naive_plan(v, L, n, prec, T_out != nullptr);
  float* partial = c.take<float>(static_cast<size_t>(pl.nc) * L);
  RPT_TRY(prep_launch(p, X, ldx, tail, flags, s));
  return naive_launch(p, pl, labels, L, tail, prec, partial, T_out, max_out, s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// sampled t statistics
size_t rpt_sampled_tstat_workspace(int64_t v, int32_t n) {
  if (v < 1 || n < 4) return 0;
  return prep_bytes(v, n, kPrepRows | kPrepUnbal);
}

rpt_status rpt_sampled_tstat(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* labels,
                             int64_t L, const int32_t* omega, int32_t k, int stat, float* y, void* ws,
                             size_t ws_bytes, void* stream) {
  if (!design_ok(v, n, ldx, n1) || L < 0 || k < 0) return RPT_ERR_INVALID_ARG;
  if (stat != RPT_STAT_T && stat != RPT_STAT_MEANDIFF) return RPT_ERR_INVALID_ARG;
  if (!stat_ok(stat, n, n1)) return RPT_ERR_UNSUPPORTED;
  if (L > 0 && k > 0 && (!X || !labels || !omega || !y)) return RPT_ERR_INVALID_ARG;
  if (!ws_ok(ws, ws_bytes, rpt_sampled_tstat_workspace(v, n))) return RPT_ERR_WORKSPACE;
  if (L == 0 || k == 0) return RPT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int flags = kPrepRows | (2 * n1 != n ? kPrepUnbal : 0) | stat_flags(stat);
  Carver c(ws);
  PrepX p = prep_carve(c, v, n, n1, flags | kPrepUnbal);
  if (!(flags & kPrepUnbal)) p.cstg = nullptr;
  RPT_TRY(prep_launch(p, X, ldx, RPT_TAIL_SIGNED, flags, s));
  return sampled_launch(p, labels, L, omega, k, nullptr, y, s);
}

// ---------------------------------------------------------------------------
// Complete
size_t rpt_complete_workspace(int64_t L, int32_t r) {
  (void)L;
  (void)r;
  return 0;
}

rpt_status rpt_complete(const float* U, int64_t v, int32_t r, const int32_t* omega, int32_t k, const float* y,
                        int64_t L, float* W, float* resid, int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  if (v < 1 || r < 1 || r > 128 || L < 0 || k < 1 || r > v) return RPT_ERR_INVALID_ARG;
  if (k < r) return RPT_ERR_UNDERDETERMINED;
  if (L > 0 && (!U || !omega || !y || !W || !info)) return RPT_ERR_INVALID_ARG;
  return complete_run(U, v, r, omega, k, y, nullptr, 0, nullptr, L, W, resid, info, nullptr,
                      static_cast<hipStream_t>(stream));
}

// ---------------------------------------------------------------------------
// re-orthonormalisation: two Cholesky-QR passes
size_t rpt_reorth_workspace(int64_t v, int32_t r) {
  if (v < 1 || r < 1) return 0;
  return reorth_bytes(v, r);
}

rpt_status rpt_reorth(float* U, int64_t v, int32_t r, int32_t* info, void* ws, size_t ws_bytes, void* stream) {
  if (!U || v < 1 || r < 1 || r > 128 || v < r) return RPT_ERR_INVALID_ARG;
  if (!ws_ok(ws, ws_bytes, rpt_reorth_workspace(v, r))) return RPT_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RPT_TRY(reorth_launch(U, v, r, info, ws, s));
  return reorth_launch(U, v, r, info, ws, s);
}

// ---------------------------------------------------------------------------
// training
namespace rpt {
namespace {
struct TrainWs {
  PrepX p;
  float* partial;
  float* T;
  float* W;
  float* resid;
  float* wnorm2;
  int32_t* info;
  double* sums;
  float* gap;
  void* reorth_ws;
  void* recon_ws;
  int32_t* lhead;  // [v] per-voxel lists of a batch's sampled entries
  int32_t* lnext;  // [ell][k]
  GrouseState g;   // sequential tracking (batch 1)
  float* WT;       // [r][ell] a batch's W in the masked loss's layout
  float* dW;       // [r][ell]
  int64_t* optr;   // [ell + 1] CSR offsets of a batch's sets
  float* dU;       // [v][r] the masked loss's gradient
};
TrainWs train_carve(void* ws, int64_t v, int n, int n1, int ell, int r, int k, int prec, size_t* total,
                    int stat = RPT_STAT_T) {
  Carver c(ws);
  TrainWs t;
  t.p = prep_carve(c, v, n, n1, naive_flags(prec, false) | stat_flags(stat));
  const NaivePlan pl = naive_plan(v, ell, n, prec, true);
  t.partial = c.take<float>(static_cast<size_t>(pl.nc_cap) * ell);
  t.T = c.take<float>(static_cast<size_t>(ell) * v);
  t.W = c.take<float>(static_cast<size_t>(ell) * r);
  t.resid = c.take<float>(static_cast<size_t>(ell) * k);
  t.wnorm2 = c.take<float>(ell);
  t.info = c.take<int32_t>(ell);
  t.sums = c.take<double>(4);
  t.gap = c.take<float>(ell);
  t.reorth_ws = c.take<char>(reorth_bytes(v, r));
  t.recon_ws = c.take<char>(recon_bytes(v, ell, r));
  t.lhead = c.take<int32_t>(v);
  t.lnext = c.take<int32_t>(static_cast<size_t>(ell) * k);
  t.g = grouse_carve(c.take<char>(grouse_bytes(r, k, ell)), r, k, ell);
  t.WT = c.take<float>(static_cast<size_t>(ell) * r);
  t.dW = c.take<float>(static_cast<size_t>(ell) * r);
  t.optr = c.take<int64_t>(static_cast<size_t>(ell) + 1);
  t.dU = c.take<float>(static_cast<size_t>(v) * r);
  if (total) *total = c.off;
  return t;
}
}  // namespace
}  // namespace rpt

extern "C" {

size_t rpt_train_workspace(int64_t v, int32_t n, int32_t ell, int32_t r, int32_t k, int prec) {
  if (v < 1 || n < 4 || ell < 1 || r < 1 || k < 1) return 0;
  size_t total = 0;
  train_carve(nullptr, v, n, n / 2, ell, r, k, prec, &total);
  return total;
}

}  // extern "C"

namespace rpt {
namespace {
TrackOpts track_opts(const rpt_tracker* t) {
  TrackOpts o;
  if (t) {
    o.mode = t->kind;
    o.rho = t->rho;
    o.admm_iters = t->admm_iters;
  }
  return o;
}
rpt_status train_check(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* train_labels,
                       int32_t ell, const float* U0, int32_t r, const int32_t* omega_train, int32_t k, int32_t passes,
                       int32_t batch, float gamma, double tol, const int32_t* omega_sm, int mu_rule, int prec,
                       int stat, const TrackOpts& opt, const float* U_out, const float* sigma_mu,
                       const float* train_max, const int32_t* info) {
  if (stat != RPT_STAT_T && stat != RPT_STAT_MEANDIFF) return RPT_ERR_INVALID_ARG;
  if (opt.mode != RPT_TRACK_GROUSE && opt.mode != RPT_TRACK_L1 && opt.mode != RPT_TRACK_GRADIENT)
    return RPT_ERR_INVALID_ARG;
  if (opt.mode == RPT_TRACK_GRADIENT && tol > 0.0) return RPT_ERR_UNSUPPORTED;  // fixed pass count
  if (opt.mode == RPT_TRACK_L1 && (!(opt.rho > 0.0f) || opt.admm_iters < 1 || opt.admm_iters > 1000))
    return RPT_ERR_INVALID_ARG;
  if (opt.mode == RPT_TRACK_L1 && batch != 1) return RPT_ERR_UNSUPPORTED;  // the l1 fit moves U column by column
  if (!design_ok(v, n, ldx, n1) || 2 * n1 != n) return design_ok(v, n, ldx, n1) ? RPT_ERR_UNSUPPORTED
                                                                               : RPT_ERR_INVALID_ARG;
  if (ell < 1 || r < 1 || r > 128 || r > v || k < 1 || k > v || passes < 0 || batch < 1 || batch > ell ||
      !(gamma > 0.0f) || static_cast<int64_t>(ell) * k > INT32_MAX || !(tol >= 0.0))
    return RPT_ERR_INVALID_ARG;
  if (batch == 1 && opt.mode == RPT_TRACK_GROUSE && !(gamma < 1.5f))
    return RPT_ERR_INVALID_ARG;  // geodesic angle below 3 pi / 4
  if (batch > 1 && tol > 0.0) return RPT_ERR_UNSUPPORTED;        // the stopping rule tracks one column at a time
  if (k < r) return RPT_ERR_UNDERDETERMINED;
  if (mu_rule != RPT_MU_MEAN_GAP && mu_rule != RPT_MU_LITERAL && mu_rule != RPT_MU_ZERO) return RPT_ERR_INVALID_ARG;
  if (prec != RPT_FP32 && prec != RPT_SPLIT_BF16) return RPT_ERR_INVALID_ARG;
  if (!X || !train_labels || !U0 || (passes > 0 && !omega_train) || !omega_sm || !U_out || !sigma_mu ||
      !train_max || !info)
    return RPT_ERR_INVALID_ARG;
  return RPT_OK;
}

// the training steps on stream s, arguments already checked
rpt_status train_tex(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* train_labels,
                     int32_t ell, int32_t r, int32_t k, int prec, int stat, float* train_max, float* T_ex_out,
                     void* ws, hipStream_t s);
rpt_status train_start_basis(int64_t v, int32_t n, int32_t n1, int32_t ell, const float* U0, int32_t r, int32_t k,
                             int prec, float* U_out, void* ws, hipStream_t s);
rpt_status train_track(int64_t v, int32_t n, int32_t n1, int32_t ell, int32_t r, const int32_t* omega_train,
                       int32_t k, int32_t passes, int32_t batch, float gamma, double tol, const int32_t* omega_sm,
                       uint64_t seed, int mu_rule, int prec, const TrackOpts& opt, float* U_out, float* sigma_mu,
                       float* train_max, float* T_ex_out, int32_t* info, double* objective, int32_t* passes_used,
                       void* ws, hipStream_t s, const std::function<rpt_status(int, int)>& at_step = nullptr);

rpt_status sigma_mu_run(const TrainWs& t, const float* U, int64_t v, int32_t r, const int32_t* omega, int32_t k,
                        const float* T, int32_t ell, const float* col_max, uint64_t seed, int mu_rule,
                        float* sigma_mu, int32_t* info, hipStream_t s);

rpt_status train_run(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* train_labels,
                     int32_t ell, const float* U0, int32_t r, const int32_t* omega_train, int32_t k, int32_t passes,
                     int32_t batch, float gamma, double tol, const int32_t* omega_sm, uint64_t seed, int mu_rule,
                     int prec, int stat, const TrackOpts& opt, float* U_out, float* sigma_mu, float* train_max,
                     float* T_ex_out, int32_t* info, double* objective, int32_t* passes_used, void* ws,
                     hipStream_t s) {
  RPT_TRY(train_tex(X, v, n, ldx, n1, train_labels, ell, r, k, prec, stat, train_max, T_ex_out, ws, s));
  RPT_TRY(train_start_basis(v, n, n1, ell, U0, r, k, prec, U_out, ws, s));
  return train_track(v, n, n1, ell, r, omega_train, k, passes, batch, gamma, tol, omega_sm, seed, mu_rule, prec,
                     opt, U_out, sigma_mu, train_max, T_ex_out, info, objective, passes_used, ws, s);
}

// 1. training columns T_ex and their exact maxima
rpt_status train_tex(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* train_labels,
                     int32_t ell, int32_t r, int32_t k, int prec, int stat, float* train_max, float* T_ex_out,
                     void* ws, hipStream_t s) {
  TrainWs t = train_carve(ws, v, n, n1, ell, r, k, prec, nullptr, stat);
  float* T = T_ex_out ? T_ex_out : t.T;
  const int flags = naive_flags(prec, false) | stat_flags(stat);
  RPT_TRY(prep_launch(t.p, X, ldx, RPT_TAIL_SIGNED, flags, s));
  const NaivePlan pl = naive_plan(v, ell, n, prec, true);
  return naive_launch(t.p, pl, train_labels, ell, RPT_TAIL_SIGNED, prec, t.partial, T, train_max, s);
}

// 2. U <- Rand. Orth. (independent of T_ex)
rpt_status train_start_basis(int64_t v, int32_t n, int32_t n1, int32_t ell, const float* U0, int32_t r, int32_t k,
                             int prec, float* U_out, void* ws, hipStream_t s) {
  TrainWs t = train_carve(ws, v, n, n1, ell, r, k, prec, nullptr);
  if (U0 != U_out &&
      hipMemcpyAsync(U_out, U0, sizeof(float) * static_cast<size_t>(v) * r, hipMemcpyDeviceToDevice, s) !=
          hipSuccess) {
    set_hip_error(hipGetLastError());
    return RPT_ERR_HIP;
  }
  RPT_TRY(reorth_launch(U_out, v, r, t.info, t.reorth_ws, s));
  return reorth_launch(U_out, v, r, t.info, t.reorth_ws, s);
}

// 3.-5. tracking passes, sigma and mu (T_ex and the start basis in place)
// at_step(j, steps), when given, runs before the Cholesky of tracking step j
// of `steps`.
rpt_status train_track(int64_t v, int32_t n, int32_t n1, int32_t ell, int32_t r, const int32_t* omega_train,
                       int32_t k, int32_t passes, int32_t batch, float gamma, double tol, const int32_t* omega_sm,
                       uint64_t seed, int mu_rule, int prec, const TrackOpts& opt, float* U_out, float* sigma_mu,
                       float* train_max, float* T_ex_out, int32_t* info, double* objective, int32_t* passes_used,
                       void* ws, hipStream_t s, const std::function<rpt_status(int, int)>& at_step) {
  TrainWs t = train_carve(ws, v, n, n1, ell, r, k, prec, nullptr);
  float* T = T_ex_out ? T_ex_out : t.T;
  RPT_TRY(grouse_init_launch(t.g, passes_used, objective, passes, s));
  const bool grad = opt.mode == RPT_TRACK_GRADIENT;
  if (batch == 1 && !grad) {
    // 3. GROUSE column by column (the paper's mode), one cooperative launch
    // per pass; the rest of the chip is free for whatever at_step starts
    for (int pp = 0; pp < passes; ++pp) {
      // whatever at_step starts goes out with the first pass, which leaves
      // all but a few dozen compute units free while it runs: the stopping
      // rule may end tracking after any pass, and work released with the
      // later passes would then hold up the launches that follow
      if (at_step && pp == 0) RPT_TRY(at_step(0, 1));
      RPT_TRY(grouse_pass_launch(t.g, U_out, v, r, T, v, omega_train + static_cast<int64_t>(pp) * ell * k, k, ell,
                                 gamma, pp, tol, objective, passes_used, t.info, opt, s));
      // span(B) is the tracked subspace: its orthonormal basis starts the next pass
      RPT_TRY(reorth_launch(U_out, v, r, t.g.rinfo, t.reorth_ws, s, nullptr, t.g.stop, pp));
    }
  }
  // 3'. the mini-batch variant: Complete links every sampled entry into the
  // list of its voxel; the update then adds each voxel's entries in one pass.
  // 3''. the masked loss drives U: Complete with residuals, the loss's
  // backward gives dU = -P_O(E) W^T, U <- U - gamma dU (the gradient is
  // tangent at the least-squares fit, U^T dU = 0), QR retraction.
  const bool minib = batch > 1 || grad;
  RPT_TRY(fill_i32(t.lhead, v, -1, s));
  if (minib && passes_used) RPT_TRY(fill_i32(passes_used, 1, passes, s));
  const int steps = minib ? passes * ((ell + batch - 1) / batch) : 0;
  int step = 0;
  for (int pp = 0; pp < (minib ? passes : 0); ++pp) {
    for (int b0 = 0; b0 < ell; b0 += batch) {
      const int nb = b0 + batch <= ell ? batch : ell - b0;
      const int32_t* om = omega_train + (static_cast<int64_t>(pp) * ell + b0) * k;
      const float* Tb = T + static_cast<int64_t>(b0) * v;
      if (grad) {
        RPT_TRY(complete_run(U_out, v, r, om, k, nullptr, Tb, v, nullptr, nb, t.W, t.resid, t.info, t.wnorm2, s));
        if (objective) RPT_TRY(sumsq_add_launch(t.resid, static_cast<int64_t>(nb) * k, objective + pp, s));
        RPT_TRY(grad_prep_launch(t.W, nb, r, t.WT, t.optr, k, s));
        RPT_TRY(loss_bwd_launch(U_out, v, r, t.WT, nb, t.optr, om, t.resid, t.dU, t.dW, nullptr, s));
        RPT_TRY(axpy_launch(U_out, t.dU, v * r, -gamma, s));
      } else {
        RPT_TRY(complete_run(U_out, v, r, om, k, nullptr, Tb, v, nullptr, nb, t.W, nullptr, t.info, t.wnorm2, s,
                             t.lhead, t.lnext));
        RPT_TRY(track_apply_launch(U_out, v, r, k, Tb, v, t.W, t.wnorm2, t.info, gamma, t.lhead, t.lnext, s));
      }
      const std::function<rpt_status()> hook = [&, j = step]() { return at_step(j, steps); };
      RPT_TRY(reorth_launch(U_out, v, r, t.info + ell - 1, t.reorth_ws, s, at_step ? &hook : nullptr));
      ++step;
    }
  }
  return sigma_mu_run(t, U_out, v, r, omega_sm, k, T, ell, train_max, seed, mu_rule, sigma_mu, info, s);
}

// 4. sigma from fresh sampled sets of the columns T (ell x v, exact maxima
// col_max) with the basis U; 5. mu
rpt_status sigma_mu_run(const TrainWs& t, const float* U, int64_t v, int32_t r, const int32_t* omega, int32_t k,
                        const float* T, int32_t ell, const float* col_max, uint64_t seed, int mu_rule,
                        float* sigma_mu, int32_t* info, hipStream_t s) {
  RPT_TRY(complete_run(U, v, r, omega, k, nullptr, T, v, nullptr, ell, t.W, t.resid, info, t.wnorm2, s));
  RPT_TRY(sigma_launch(t.resid, static_cast<int64_t>(ell) * k, t.sums, sigma_mu, s));
  if (mu_rule == RPT_MU_MEAN_GAP) {
    RPT_TRY(recon_launch(U, v, r, t.W, ell, 0, seed, RPT_STREAM_TRAINING, sigma_mu, nullptr, col_max, t.gap,
                         t.recon_ws, s));
    RPT_TRY(mu_launch(t.gap, ell, mu_rule, sigma_mu, s));
  } else if (mu_rule == RPT_MU_LITERAL) {
    RPT_TRY(literal_resid_launch(T, U, t.W, v, r, ell, t.gap, s));
    RPT_TRY(mu_launch(t.gap, ell, mu_rule, sigma_mu, s));
  } else {
    RPT_TRY(mu_launch(t.gap, 0, mu_rule, sigma_mu, s));
  }
  return RPT_OK;
}
}  // namespace
}  // namespace rpt

extern "C" {

rpt_status rpt_train_subspace(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                              const uint8_t* train_labels, int32_t ell, const float* U0, int32_t r,
                              const int32_t* omega_train, int32_t k, int32_t passes, int32_t batch, float gamma,
                              double tol, const int32_t* omega_sm, uint64_t seed, int mu_rule, int prec,
                              int stat, const rpt_tracker* tracker, float* U_out, float* sigma_mu,
                              float* train_max, float* T_ex_out, int32_t* info, double* objective,
                              int32_t* passes_used, void* ws, size_t ws_bytes, void* stream) {
  const TrackOpts opt = track_opts(tracker);
  RPT_TRY(train_check(X, v, n, ldx, n1, train_labels, ell, U0, r, omega_train, k, passes, batch, gamma, tol,
                      omega_sm, mu_rule, prec, stat, opt, U_out, sigma_mu, train_max, info));
  if (!ws_ok(ws, ws_bytes, rpt_train_workspace(v, n, ell, r, k, prec))) return RPT_ERR_WORKSPACE;
  return train_run(X, v, n, ldx, n1, train_labels, ell, U0, r, omega_train, k, passes, batch, gamma, tol, omega_sm,
                   seed, mu_rule, prec, stat, opt, U_out, sigma_mu, train_max, T_ex_out, info, objective,
                   passes_used, ws, static_cast<hipStream_t>(stream));
}

size_t rpt_sigma_mu_workspace(int64_t v, int32_t n, int32_t h, int32_t r, int32_t k, int prec) {
  return rpt_train_workspace(v, n, h, r, k, prec);
}

rpt_status rpt_sigma_mu(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* labels,
                        int32_t h, const float* U, int32_t r, const int32_t* omega, int32_t k, uint64_t seed,
                        int mu_rule, int prec, int stat, float* sigma_mu, float* col_max, int32_t* info, void* ws,
                        size_t ws_bytes, void* stream) {
  if (stat != RPT_STAT_T && stat != RPT_STAT_MEANDIFF) return RPT_ERR_INVALID_ARG;
  if (!design_ok(v, n, ldx, n1) || 2 * n1 != n) return design_ok(v, n, ldx, n1) ? RPT_ERR_UNSUPPORTED
                                                                               : RPT_ERR_INVALID_ARG;
  if (h < 1 || r < 1 || r > 128 || r > v || k < 1 || k > v || static_cast<int64_t>(h) * k > INT32_MAX)
    return RPT_ERR_INVALID_ARG;
  if (k < r) return RPT_ERR_UNDERDETERMINED;
  if (mu_rule != RPT_MU_MEAN_GAP && mu_rule != RPT_MU_LITERAL && mu_rule != RPT_MU_ZERO) return RPT_ERR_INVALID_ARG;
  if (prec != RPT_FP32 && prec != RPT_SPLIT_BF16) return RPT_ERR_INVALID_ARG;
  if (!X || !labels || !U || !omega || !sigma_mu || !col_max || !info) return RPT_ERR_INVALID_ARG;
  if (!ws_ok(ws, ws_bytes, rpt_sigma_mu_workspace(v, n, h, r, k, prec))) return RPT_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the held-out columns as T_ex of the training call (stored t maps and
  // their exact maxima), then the same sigma and mu rules
  RPT_TRY(train_tex(X, v, n, ldx, n1, labels, h, r, k, prec, stat, col_max, nullptr, ws, s));
  const TrainWs t = train_carve(ws, v, n, n1, h, r, k, prec, nullptr, stat);
  return sigma_mu_run(t, U, v, r, omega, k, t.T, h, col_max, seed, mu_rule, sigma_mu, info, s);
}

// ---------------------------------------------------------------------------
// recovery

}  // extern "C"

namespace rpt {
namespace {
rpt_status recover_check(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* labels,
                         int64_t L_rec, int64_t col0, const float* U, int32_t r, const float* sigma_mu,
                         const int32_t* omega, int32_t k, const float* max_out, const int32_t* info,
                         int stat = RPT_STAT_T) {
  if (!design_ok(v, n, ldx, n1)) return RPT_ERR_INVALID_ARG;
  if (stat != RPT_STAT_T && stat != RPT_STAT_MEANDIFF) return RPT_ERR_INVALID_ARG;
  if (2 * n1 != n) return RPT_ERR_UNSUPPORTED;
  if (L_rec < 0 || col0 < 0 || r < 1 || r > 128 || r > v || k < 1 || k > v) return RPT_ERR_INVALID_ARG;
  if (k < r) return RPT_ERR_UNDERDETERMINED;
  if (L_rec > 0 && (!X || !labels || !U || !sigma_mu || !omega || !max_out || !info)) return RPT_ERR_INVALID_ARG;
  return RPT_OK;
}

struct RecoverWs {
  PrepX p;
  float* y;
  float* W;
  void* rws;
  void* gb;  // Gram matrices of the split Complete
};
RecoverWs recover_carve(void* ws, int64_t v, int32_t n, int32_t n1, int64_t L_rec, int32_t r, int32_t k,
                        size_t* total = nullptr, int stat = RPT_STAT_T) {
  Carver c(ws);
  RecoverWs w;
  w.p = prep_carve(c, v, n, n1, kPrepRows | stat_flags(stat));
  w.y = c.take<float>(static_cast<size_t>(L_rec > 0 ? L_rec : 1) * k);
  w.W = c.take<float>(static_cast<size_t>(L_rec > 0 ? L_rec : 1) * r);
  w.rws = c.take<char>(recon_bytes(v, L_rec, r));
  w.gb = c.take<char>(complete_split_bytes(L_rec, r));
  if (total) *total = c.off;
  return w;
}

// the steps that do not need the basis: sampled t of every recovered column
rpt_status recover_front(const RecoverWs& w, const float* X, int64_t ldx, const uint8_t* labels, int64_t L_rec,
                         const int32_t* omega, int32_t k, hipStream_t s, const int64_t* optr = nullptr) {
  RPT_TRY(prep_launch(w.p, X, ldx, RPT_TAIL_SIGNED, kPrepRows | stat_flags(w.p.stat), s));
  return sampled_launch(w.p, labels, L_rec, omega, optr ? 0 : k, nullptr, w.y, s, optr);
}

// sampled t of recovered columns [c0, c1) (prep done)
rpt_status recover_sampled(const RecoverWs& w, const uint8_t* labels, int32_t n, int64_t c0, int64_t c1,
                           const int32_t* omega, int32_t k, hipStream_t s) {
  if (c1 <= c0) return RPT_OK;
  return sampled_launch(w.p, labels + c0 * n, c1 - c0, omega + c0 * k, k, nullptr, w.y + c0 * k, s);
}

// Complete, then U w + noise and the column maxima
rpt_status recover_back(const RecoverWs& w, int64_t v, int64_t L_rec, int64_t col0, const float* U, int32_t r,
                        const float* sigma_mu, const int32_t* omega, int32_t k, uint64_t seed, float* max_out,
                        float* W_out, int32_t* info, hipStream_t s, const int64_t* optr = nullptr) {
  float* W = W_out ? W_out : w.W;
  RPT_TRY(complete_run(U, v, r, omega, optr ? 0 : k, w.y, nullptr, 0, nullptr, L_rec, W, nullptr, info, nullptr, s,
                       nullptr, nullptr, optr, w.gb));
  return recon_launch(U, v, r, W, L_rec, col0, seed, RPT_STREAM_RECOVERY, sigma_mu, max_out, nullptr, nullptr,
                      w.rws, s);
}

}  // namespace
}  // namespace rpt

extern "C" {

size_t rpt_recover_workspace(int64_t v, int32_t n, int64_t L_rec, int32_t r, int32_t k) {
  if (v < 1 || n < 4 || L_rec < 0 || r < 1 || k < 1) return 0;
  size_t total = 0;
  recover_carve(nullptr, v, n, n / 2, L_rec, r, k, &total);
  return total;
}

rpt_status rpt_recover_maxnull(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* labels,
                               int64_t L_rec, int64_t col0, const float* U, int32_t r, const float* sigma_mu,
                               const int32_t* omega, int32_t k, const int64_t* omega_ptr, uint64_t seed, int stat,
                               float* max_out, float* W_out, int32_t* info, void* ws, size_t ws_bytes,
                               void* stream) {
  RPT_TRY(recover_check(X, v, n, ldx, n1, labels, L_rec, col0, U, r, sigma_mu, omega, k, max_out, info, stat));
  if (!ws_ok(ws, ws_bytes, rpt_recover_workspace(v, n, L_rec, r, k))) return RPT_ERR_WORKSPACE;
  if (L_rec == 0) return RPT_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const RecoverWs w = recover_carve(ws, v, n, n1, L_rec, r, k, nullptr, stat);
  RPT_TRY(recover_front(w, X, ldx, labels, L_rec, omega, k, s, omega_ptr));
  return recover_back(w, v, L_rec, col0, U, r, sigma_mu, omega, k, seed, max_out, W_out, info, s, omega_ptr);
}

// ---------------------------------------------------------------------------
// Alg. 2 end to end
size_t rpt_rapidpt_workspace(int64_t v, int32_t n, int32_t ell, int64_t L_rec, int32_t r, int32_t k, int prec) {
  const size_t a = rpt_train_workspace(v, n, ell, r, k, prec);
  const size_t b = rpt_recover_workspace(v, n, L_rec, r, k);
  return (a == 0 || b == 0) ? 0 : a + b;
}

}  // extern "C"

namespace rpt {
namespace {
// Inputs of the end-to-end call drawn from the seed, after its workspace:
// relabellings of columns 0..L-1 (training then recovered), the tracking
// passes' sets, the sigma/mu sets and the recovery sets
struct GenWs {
  uint8_t* labels;
  int32_t* om_train;
  int32_t* om_sm;
  int32_t* om_rec;
  size_t bytes;
};
GenWs gen_carve(void* base, int32_t n, int32_t ell, int64_t L_rec, int32_t k, int32_t passes) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  GenWs g{};
  char* p = static_cast<char*>(base);
  size_t off = 0;
  g.labels = reinterpret_cast<uint8_t*>(p + off);
  off += al(static_cast<size_t>(ell + L_rec) * n);
  g.om_train = reinterpret_cast<int32_t*>(p + off);
  off += al(sizeof(int32_t) * static_cast<size_t>(passes) * ell * k);
  g.om_sm = reinterpret_cast<int32_t*>(p + off);
  off += al(sizeof(int32_t) * static_cast<size_t>(ell) * k);
  g.om_rec = reinterpret_cast<int32_t*>(p + off);
  off += al(sizeof(int32_t) * static_cast<size_t>(L_rec) * k);
  g.bytes = off;
  return g;
}
}  // namespace
}  // namespace rpt

extern "C" {

size_t rpt_rapidpt_gen_workspace(int32_t n, int32_t ell, int64_t L_rec, int32_t k, int32_t passes) {
  if (n < 1 || ell < 0 || L_rec < 0 || k < 0 || passes < 0) return 0;
  return rpt::gen_carve(nullptr, n, ell, L_rec, k, passes).bytes;
}

rpt_status rpt_rapidpt_maxnull(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                               const uint8_t* train_labels, int32_t ell, const uint8_t* rec_labels, int64_t L_rec,
                               const float* U0, int32_t r, const int32_t* omega_train, int32_t k, int32_t passes,
                               int32_t batch, float gamma, double tol, const int32_t* omega_sm,
                               const int32_t* omega_rec, uint64_t seed, int mu_rule, int prec, int stat,
                               const rpt_tracker* tracker, float* h_out, float* U_out, float* sigma_mu,
                               int32_t* train_info, int32_t* rec_info, double* objective, int32_t* passes_used,
                               void* ws, size_t ws_bytes, void* stream) {
  const TrackOpts opt = track_opts(tracker);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // inputs left NULL are drawn from the seed into the workspace's tail (the
  // start basis straight into U_out)
  const size_t base = rpt_rapidpt_workspace(v, n, ell, L_rec, r, k, prec);
  // (a NULL pointer for an empty input is no request to draw it)
  const bool gen_lab = (!train_labels && ell > 0) || (!rec_labels && L_rec > 0);
  const bool gen_om = (!omega_train && passes > 0 && ell > 0) || (!omega_sm && ell > 0) || (!omega_rec && L_rec > 0);
  const bool gen_u0 = !U0;
  GenWs g{};
  if (gen_lab || gen_om) {
    if (n < 1 || ell < 0 || L_rec < 0 || k < 1 || passes < 0 || base == 0) return RPT_ERR_INVALID_ARG;
    if (gen_lab) RPT_TRY(gen_labels_check(0, ell + L_rec, n, n1));
    if (gen_om) RPT_TRY(gen_sets_check(passes + 1, 0, ell + L_rec, v, k));
    g = gen_carve(static_cast<char*>(ws) + base, n, ell, L_rec, k, passes);
    if (!train_labels) train_labels = g.labels;
    if (!rec_labels) rec_labels = g.labels + static_cast<size_t>(ell) * n;
    if (!omega_train) omega_train = g.om_train;
    if (!omega_sm) omega_sm = g.om_sm;
    if (!omega_rec) omega_rec = g.om_rec;
  }
  if (gen_u0) U0 = U_out;
  RPT_TRY(train_check(X, v, n, ldx, n1, train_labels, ell, U0, r, omega_train, k, passes, batch, gamma, tol,
                      omega_sm, mu_rule, prec, stat, opt, U_out, sigma_mu, h_out, train_info));
  RPT_TRY(recover_check(X, v, n, ldx, n1, rec_labels, L_rec, ell, U_out, r, sigma_mu, omega_rec, k, h_out,
                        rec_info, stat));
  const size_t tw = rpt_train_workspace(v, n, ell, r, k, prec);
  if (!ws_ok(ws, ws_bytes, base + g.bytes)) return RPT_ERR_WORKSPACE;
  // relabelling c and sampled sets of column c of h^L: row c; set 0 for the
  // sigma/mu and recovery sets, 1 + p for tracking pass p
  if (gen_lab) RPT_TRY(gen_labels_launch(seed, 0, ell + L_rec, n, n1, g.labels, s));
  if (gen_om && omega_train == g.om_train)
    for (int32_t p = 0; p < passes; ++p)
      RPT_TRY(gen_sets_launch(seed, 1 + p, 0, ell, v, k, g.om_train + static_cast<size_t>(p) * ell * k, s));
  if (gen_om && omega_sm == g.om_sm) RPT_TRY(gen_sets_launch(seed, 0, 0, ell, v, k, g.om_sm, s));
  if (gen_om && omega_rec == g.om_rec) RPT_TRY(gen_sets_launch(seed, 0, ell, L_rec, v, k, g.om_rec, s));
  if (gen_u0) RPT_TRY(gen_start_launch(seed, v, r, U_out, s));
  const RecoverWs w = recover_carve(static_cast<char*>(ws) + tw, v, n, n1, L_rec, r, k, nullptr, stat);
  // Two chains share the device: the caller's stream computes T_ex (matrix
  // cores, the whole chip) and then the tracking passes (latency-bound, a
  // few dozen workgroups); the second stream
  // orthonormalises the start basis meanwhile and then computes the sampled t
  // of the recovered columns, which need no basis, in one chunk per tracking
  // step, each started as that step's Cholesky is reached.
  SideStream* sd = side_stream(s);
  if (!sd) {
    RPT_TRY(train_run(X, v, n, ldx, n1, train_labels, ell, U0, r, omega_train, k, passes, batch, gamma, tol,
                      omega_sm, seed, mu_rule, prec, stat, opt, U_out, sigma_mu, h_out, nullptr, train_info,
                      objective, passes_used, ws, s));
    if (L_rec == 0) return RPT_OK;
    RPT_TRY(recover_front(w, X, ldx, rec_labels, L_rec, omega_rec, k, s));
    return recover_back(w, v, L_rec, ell, U_out, r, sigma_mu, omega_rec, k, seed, h_out + ell, nullptr, rec_info, s);
  }
  rpt_status st = stream_wait(sd, sd->fork, s, sd->st);
  if (st != RPT_OK) return st;
  // from here on every path joins the second stream back before returning
  rpt_status st_main = train_tex(X, v, n, ldx, n1, train_labels, ell, r, k, prec, stat, h_out, nullptr, ws, s);
  rpt_status st_side = train_start_basis(v, n, n1, ell, U0, r, k, prec, U_out, ws, sd->st);
  st = stream_wait(sd, sd->mid, sd->st, s);  // the basis is ready for the tracking passes
  if (st_side == RPT_OK && st == RPT_OK && L_rec > 0)
    st_side = prep_launch(w.p, X, ldx, RPT_TAIL_SIGNED, kPrepRows | stat_flags(stat), sd->st);
  // the sampled t of the recovered columns, released in chunks as the
  // tracking steps start (column by column tracking: all with the first pass)
  int64_t done = 0;
  const std::function<rpt_status(int, int)> at_step = [&](int j, int steps) -> rpt_status {
    if (st_side != RPT_OK || L_rec == 0) return RPT_OK;
    RPT_TRY(stream_wait(sd, sd->step, s, sd->st));
    const int64_t c1 = L_rec * (j + 1) / steps;
    st_side = recover_sampled(w, rec_labels, n, done, c1, omega_rec, k, sd->st);
    done = c1;
    return RPT_OK;
  };
  if (st_main == RPT_OK && st_side == RPT_OK && st == RPT_OK)
    st_main = train_track(v, n, n1, ell, r, omega_train, k, passes, batch, gamma, tol, omega_sm, seed, mu_rule,
                          prec, opt, U_out, sigma_mu, h_out, nullptr, train_info, objective, passes_used, ws, s,
                          at_step);
  if (st_side == RPT_OK && done < L_rec)  // no tracking steps: all columns now
    st_side = recover_sampled(w, rec_labels, n, done, L_rec, omega_rec, k, sd->st);
  const rpt_status st_join = stream_wait(sd, sd->join, sd->st, s);
  RPT_TRY(st);
  RPT_TRY(st_side);
  RPT_TRY(st_main);
  RPT_TRY(st_join);
  if (L_rec == 0) return RPT_OK;
  return recover_back(w, v, L_rec, ell, U_out, r, sigma_mu, omega_rec, k, seed, h_out + ell, nullptr, rec_info, s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// several studies, uneven sampled sets
namespace rpt {
namespace {
// Batched workspace: [counters][transient: the largest study's prep, sampled
// values and Complete buffers, used by the studies in turn][per study: W and
// the reconstruction buffers, kept until the shared reconstruction launch].
size_t study_transient_bytes(const rpt_study& st) {
  Carver c(nullptr);
  prep_carve(c, st.v, st.n, st.n1, kPrepRows);
  c.take<float>(static_cast<size_t>(st.nnz > 0 ? st.nnz : 1));
  c.take<char>(complete_split_bytes(st.L_rec, st.r));
  return c.off;
}
int batch_ks(const rpt_study* studies, int32_t n) {
  int ks = 1;
  for (int32_t q = 0; q < n; ++q) {
    const int k = (studies[q].r + 15) / 16;
    if (studies[q].L_rec > 0 && k > ks) ks = k;
  }
  return ks;
}
struct BatchLayout {
  int* counters;
  void* transient;
  std::vector<float*> W;
  std::vector<void*> rws;
  size_t total;
};
BatchLayout batch_layout(void* ws, const rpt_study* studies, int32_t n, int ks) {
  BatchLayout b;
  Carver c(ws);
  b.counters = c.take<int>(recon_batch_counters(n));
  size_t tr = 256;
  for (int32_t q = 0; q < n; ++q) tr = std::max(tr, study_transient_bytes(studies[q]));
  b.transient = c.take<char>(tr);
  for (int32_t q = 0; q < n; ++q) {
    const rpt_study& st = studies[q];
    b.W.push_back(c.take<float>(static_cast<size_t>(st.L_rec > 0 ? st.L_rec : 1) * st.r));
    b.rws.push_back(c.take<char>(st.L_rec > 0 ? recon_bytes(st.v, st.L_rec, st.r, ks) : 256));
  }
  b.total = c.off;
  return b;
}
rpt_status study_check(const rpt_study& st) {
  if (!design_ok(st.v, st.n, st.ldx, st.n1)) return RPT_ERR_INVALID_ARG;
  if (2 * st.n1 != st.n) return RPT_ERR_UNSUPPORTED;
  if (st.L_rec < 0 || st.col0 < 0 || st.r < 1 || st.r > 128 || st.r > st.v || st.nnz < 0 ||
      st.nnz > INT32_MAX)
    return RPT_ERR_INVALID_ARG;
  if (st.L_rec > 0 && (!st.X || !st.labels || !st.U || !st.sigma_mu || !st.omega_ptr || !st.max_out || !st.info ||
                       (st.nnz > 0 && !st.omega_idx)))
    return RPT_ERR_INVALID_ARG;
  return RPT_OK;
}
}  // namespace
}  // namespace rpt

extern "C" {

size_t rpt_recover_batched_workspace(const rpt_study* studies, int32_t n_studies) {
  if (!studies || n_studies < 0) return 0;
  for (int32_t q = 0; q < n_studies; ++q)
    if (study_check(studies[q]) != RPT_OK) return 0;
  return batch_layout(nullptr, studies, n_studies, batch_ks(studies, n_studies)).total;
}

rpt_status rpt_recover_maxnull_batched(const rpt_study* studies, int32_t n_studies, void* ws, size_t ws_bytes,
                                       void* stream) {
  if (n_studies < 0 || (n_studies > 0 && !studies)) return RPT_ERR_INVALID_ARG;
  for (int32_t q = 0; q < n_studies; ++q) RPT_TRY(study_check(studies[q]));
  const int ks = batch_ks(studies, n_studies);
  const size_t need = batch_layout(nullptr, studies, n_studies, ks).total;
  if (!ws_ok(ws, ws_bytes, need)) return RPT_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const BatchLayout lay = batch_layout(ws, studies, n_studies, ks);
  std::vector<ReconStudy> rec;
  // per study: sampled t and Complete in the shared region, then the study's
  // own copy of U for the reconstruction
  for (int32_t q = 0; q < n_studies; ++q) {
    const rpt_study& st = studies[q];
    if (st.L_rec == 0) continue;
    Carver c(lay.transient);
    PrepX p = prep_carve(c, st.v, st.n, st.n1, kPrepRows);
    float* y = c.take<float>(static_cast<size_t>(st.nnz > 0 ? st.nnz : 1));
    void* gb = c.take<char>(complete_split_bytes(st.L_rec, st.r));
    float* W = lay.W[q];
    RPT_TRY(prep_launch(p, st.X, st.ldx, RPT_TAIL_SIGNED, kPrepRows, s));
    RPT_TRY(sampled_launch(p, st.labels, st.L_rec, st.omega_idx, 0, nullptr, y, s, st.omega_ptr));
    RPT_TRY(complete_run(st.U, st.v, st.r, st.omega_idx, 0, y, nullptr, 0, nullptr, st.L_rec, W, nullptr, st.info,
                         nullptr, s, nullptr, nullptr, st.omega_ptr, gb));
    const ReconStudy rs{st.U, st.v, st.r, W, st.L_rec, st.col0, st.seed, st.sigma_mu, st.max_out, lay.rws[q],
                        st.study};
    RPT_TRY(recon_prepare_study(rs, ks, s));
    rec.push_back(rs);
  }
  // U w + noise + max of all studies: persistent launches over their work items
  if (!rec.empty()) RPT_TRY(recon_batched(rec.data(), static_cast<int>(rec.size()), ks, lay.counters, s));
  return RPT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuning of the voxel-chunk counts (synchronises the stream; not for graph
// capture; the measured choice is kept for the shape in the plan table)
namespace rpt {
namespace {
// times `reps` calls of fn (after one untimed call); -1 on a HIP error
template <class F>
float time_calls(F fn, int reps, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float ms = -1.0f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) goto done;
  if (fn() != RPT_OK) goto done;
  if (hipEventRecord(e0, s) != hipSuccess) goto done;
  for (int q = 0; q < reps; ++q)
    if (fn() != RPT_OK) goto done;
  if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) goto done;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ms = -1.0f;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return ms;
}

struct ReconTuneWs {
  void* rws;
  float *U, *W, *sm, *out;
};
ReconTuneWs recon_tune_carve(void* ws, int64_t v, int32_t r, int64_t L, size_t* total) {
  Carver c(ws);
  ReconTuneWs t;
  t.rws = c.take<char>(recon_bytes(v, L, r));
  t.U = c.take<float>(static_cast<size_t>(v) * r);
  t.W = c.take<float>(static_cast<size_t>(L > 0 ? L : 1) * r);
  t.sm = c.take<float>(2);
  t.out = c.take<float>(static_cast<size_t>(L > 0 ? L : 1));
  if (total) *total = c.off;
  return t;
}
}  // namespace
}  // namespace rpt

extern "C" {

rpt_status rpt_autotune_naive(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1, const uint8_t* labels,
                              int64_t L, int prec, float* T_out, int32_t reps, void* ws, size_t ws_bytes,
                              void* stream, int32_t* chosen) {
  if (!design_ok(v, n, ldx, n1) || L < 1 || reps < 1 || !X || !labels || !chosen) return RPT_ERR_INVALID_ARG;
  if (prec != RPT_FP32 && prec != RPT_SPLIT_BF16) return RPT_ERR_INVALID_ARG;
  const bool unbal = 2 * n1 != n;
  if ((unbal && prec != RPT_FP32) || (prec == RPT_FP32 && n > 128)) return RPT_ERR_UNSUPPORTED;
  if (!ws_ok(ws, ws_bytes, rpt_naive_workspace(v, n, L, prec))) return RPT_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int flags = naive_flags(prec, unbal);
  Carver c(ws);
  PrepX p = prep_carve(c, v, n, n1, flags);
  const bool store = T_out != nullptr;
  float* partial = c.take<float>(static_cast<size_t>(naive_plan(v, L, n, prec, store).nc_cap) * L);
  RPT_TRY(prep_launch(p, X, ldx, RPT_TAIL_SIGNED, flags, s));
  const NaivePlan base = naive_plan(v, L, n, prec, store);
  int cand[kMaxChunkCandidates];
  const int m = chunk_candidates(base.nc_heur, round_up(base.vt, 8), cand);
  int best = base.nc_heur;
  float best_ms = 0.0f;
  for (int q = 0; q < m; ++q) {
    const NaivePlan pl = naive_plan(v, L, n, prec, store, cand[q]);
    const float ms = time_calls(
        [&]() { return naive_launch(p, pl, labels, L, RPT_TAIL_SIGNED, prec, partial, T_out, nullptr, s); }, reps,
        s);
    if (ms < 0.0f) return RPT_ERR_HIP;
    if (q == 0 || ms < best_ms) {
      best_ms = ms;
      best = cand[q];
    }
  }
  set_tuned_chunks(kTuneNaive, v, L, n, 2 * prec + (store ? 1 : 0), best);
  *chosen = best;
  return RPT_OK;
}

size_t rpt_autotune_recover_workspace(int64_t v, int32_t r, int64_t L_rec) {
  if (v < 1 || r < 1 || L_rec < 1) return 0;
  size_t total = 0;
  recon_tune_carve(nullptr, v, r, L_rec, &total);
  return total;
}

rpt_status rpt_autotune_recover(int64_t v, int32_t r, int64_t L_rec, int32_t reps, void* ws, size_t ws_bytes,
                                void* stream, int32_t* chosen) {
  if (v < 1 || r < 1 || r > 128 || L_rec < 1 || reps < 1 || !chosen) return RPT_ERR_INVALID_ARG;
  if (!ws_ok(ws, ws_bytes, rpt_autotune_recover_workspace(v, r, L_rec))) return RPT_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ReconTuneWs t = recon_tune_carve(ws, v, r, L_rec, nullptr);
  // a zero basis and zero coefficients with sigma = 1: every voxel draws its
  // normal, the fused path's full work (its time does not depend on values)
  const float sm_host[2] = {1.0f, 0.0f};
  if (hipMemsetAsync(t.U, 0, sizeof(float) * static_cast<size_t>(v) * r, s) != hipSuccess ||
      hipMemsetAsync(t.W, 0, sizeof(float) * static_cast<size_t>(L_rec) * r, s) != hipSuccess ||
      hipMemcpyAsync(t.sm, sm_host, sizeof(sm_host), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_hip_error(hipGetLastError());
    return RPT_ERR_HIP;
  }
  int cand[kMaxChunkCandidates];
  const int m = recon_chunk_candidates(v, L_rec, r, cand);
  int best = cand[0];
  float best_ms = 0.0f;
  for (int q = 0; q < m; ++q) {
    const float ms = time_calls(
        [&]() {
          return recon_launch(t.U, v, r, t.W, L_rec, 0, 1, RPT_STREAM_RECOVERY, t.sm, t.out, nullptr, nullptr, t.rws,
                              s, 0, cand[q]);
        },
        reps, s);
    if (ms < 0.0f) return RPT_ERR_HIP;
    if (q == 0 || ms < best_ms) {
      best_ms = ms;
      best = cand[q];
    }
  }
  set_tuned_chunks(kTuneRecon, v, L_rec, r, 0, best);
  *chosen = best;
  return RPT_OK;
}

// ---------------------------------------------------------------------------
// masked loss
rpt_status rpt_masked_loss_fwd(const float* U, int64_t v, int32_t r, const float* W, int32_t B,
                               const int64_t* omega_ptr, const int32_t* omega_idx, const float* t_vals, int64_t nnz,
                               double* loss, float* resid, void* stream) {
  if (v < 1 || r < 1 || B < 0 || nnz < 0 || !loss) return RPT_ERR_INVALID_ARG;
  if (B > 0 && (!U || !W || !omega_ptr || (nnz > 0 && (!omega_idx || !t_vals)))) return RPT_ERR_INVALID_ARG;
  return loss_fwd_launch(U, v, r, W, B, omega_ptr, omega_idx, t_vals, loss, resid, static_cast<hipStream_t>(stream));
}

rpt_status rpt_masked_loss_bwd(const float* U, int64_t v, int32_t r, const float* W, int32_t B,
                               const int64_t* omega_ptr, const int32_t* omega_idx, const float* resid, int64_t nnz,
                               float* dU, float* dW, const double* grad_scale, void* stream) {
  if (v < 1 || r < 1 || B < 0 || nnz < 0 || !dU || (B > 0 && !dW)) return RPT_ERR_INVALID_ARG;
  if (B > 0 && (!U || !W || !omega_ptr || (nnz > 0 && (!omega_idx || !resid)))) return RPT_ERR_INVALID_ARG;
  return loss_bwd_launch(U, v, r, W, B, omega_ptr, omega_idx, resid, dU, dW, grad_scale,
                         static_cast<hipStream_t>(stream));
}

}  // extern "C"
