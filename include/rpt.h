/*
 * rpt.h -- C ABI of librpt: RapidPT permutation testing on MI355X (gfx950).
 *
 * The library computes the voxel-wise maximum null distribution of a
 * two-sample permutation test, either exactly (NaivePT, Alg. 1 of
 * Gutierrez-Barragan et al., "Accelerating Permutation Testing in Voxel-wise
 * Analysis through Subspace Tracking") or by RapidPT (Alg. 2): a low-rank
 * basis U of the permutation testing matrix T is learnt from l fully computed
 * columns by subspace tracking on sub-sampled entries, and every further
 * column is completed from ceil(eta v) sampled t statistics, a residual
 * noise draw and a maximum -- without ever forming T.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array argument is DEVICE memory owned by the caller.  The library
 *   never allocates, frees, or reads device memory on the host; scratch space
 *   comes from the caller's workspace `ws` of at least the size returned by
 *   the matching *_workspace() query (256-byte aligned).
 * - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *   and is asynchronous: outputs are valid after the stream is synchronised.
 *   No entry point synchronises, so every call can be captured in a HIP graph.
 * - Arguments are validated synchronously; violations return an error code
 *   and enqueue nothing.  Numeric failures that can only be seen on the device
 *   (a sampled Gram matrix that is not positive definite) are reported
 *   LAPACK-style in a caller-provided `info` array.
 * - Data layout: X is v x n row-major (row k = voxel k, column j = subject j)
 *   with leading dimension ldx >= n, FP32.  Columns 0..n1-1 of X are the
 *   observed group 1 (X = [X^1 X^2], Alg. 1).  Relabellings are L x n uint8
 *   rows with exactly n1 entries equal to 1 (= group 1) and the rest 0.
 *   T is logically L x v (row i = the t map of relabelling i).
 * - The t statistic is Eq. 2 with sigma_g read as the unbiased group variance
 *   (Welch form; equal to the pooled Student t when n1 = n2), positive when
 *   group 1 has the larger mean.  Voxels with zero spread give t = 0.
 * - Thread safety: calls are independent except through their arguments; two
 *   calls may run concurrently on different streams with distinct workspaces.
 */
#ifndef RPT_H
#define RPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RPT_OK = 0,
  RPT_ERR_INVALID_ARG = -1,     /* a size, pointer or enum is out of range  */
  RPT_ERR_UNDERDETERMINED = -2, /* sampled set smaller than the rank r      */
  RPT_ERR_NOT_SPD = -3,         /* (device info code) Gram not positive def. */
  RPT_ERR_WORKSPACE = -4,       /* ws NULL, misaligned or too small         */
  RPT_ERR_HIP = -5,             /* a HIP launch failed; see rpt_last_hip_error */
  RPT_ERR_UNSUPPORTED = -6      /* valid request the library does not handle */
} rpt_status;

/* Arithmetic of the dense contractions (indicator GEMM of NaivePT and the
 * training columns). */
typedef enum {
  RPT_FP32 = 0,       /* FP32 MFMA on FP32 data                               */
  RPT_SPLIT_BF16 = 1  /* data split x = hi + lo into two BF16 halves, both    */
                      /* multiplied by the exact 0/1 indicator, FP32 accumulate */
} rpt_precision;

typedef enum {
  RPT_TAIL_SIGNED = 0, /* m_i = max_k t_ik            (Alg. 1)               */
  RPT_TAIL_ABS = 1     /* m_i = max_k |t_ik|          (two-sided testing)     */
} rpt_tail;

/* The `stat` input of Alg. 2 (REQUIRE line): which two-sample statistic forms
 * T.  RPT_STAT_T is Eq. 2 (see the conventions above); RPT_STAT_MEANDIFF is
 * the linear difference of the group means, m1 - m2, whose permutation
 * testing matrix T = X C has rank at most n - 1 (Sec. 3.2), so that RapidPT
 * with an exact basis reproduces NaivePT (balanced designs only). */
typedef enum {
  RPT_STAT_T = 0,
  RPT_STAT_MEANDIFF = 1
} rpt_stat;

/* The subspace tracker of the training phase (Sec. 4.1, which cites GROUSE
 * and GRASTA).  NULL in the training calls means GROUSE. */
typedef enum {
  RPT_TRACK_GROUSE = 0, /* l2 fit, geodesic step (the default)                  */
  RPT_TRACK_L1 = 1,     /* robust l1 fit by ADMM, geodesic step along the     */
                        /* augmented Lagrangian's gradient (GRASTA)           */
  RPT_TRACK_GRADIENT = 2 /* the masked loss of Eq. 1 drives U: per batch the  */
                        /* least-squares fit, the loss's backward dU, the     */
                        /* step U - gamma dU and a QR retraction              */
} rpt_track_kind;
typedef struct {
  int32_t kind;       /* rpt_track_kind                                        */
  float rho;          /* RPT_TRACK_L1: ADMM penalty, > 0                       */
  int32_t admm_iters; /* RPT_TRACK_L1: ADMM iterations per column, 1..1000     */
} rpt_tracker;

typedef enum {
  RPT_MU_MEAN_GAP = 0, /* mu = mean_i [max T_ex[:,i] - max(U w_i + s_i)]       */
  RPT_MU_LITERAL = 1,  /* mu = sup_i max(T_ex[:,i] - U W_ex[:,i])  (Alg. 2)    */
  RPT_MU_ZERO = 2
} rpt_mu_rule;

/* Noise streams of the counter-based generator (Philox4x32-10 + Box-Muller):
 * z(seed, stream, i, k) for column i and voxel k uses key (seed mod 2^32,
 * seed >> 32) and counter (k, i >> 2, stream, study); words 0,1 give columns
 * 4q, 4q+1 (cos, sin), words 2,3 give 4q+2, 4q+3.  Each word x maps to
 * u = ((x >> 8) + 0.5) 2^-24 (so |z| < 5.8872). */
#define RPT_STREAM_RECOVERY 2
#define RPT_STREAM_TRAINING 4

const char* rpt_status_string(int status);
/* The last HIP error code seen by a call that returned RPT_ERR_HIP (per thread). */
int rpt_last_hip_error(void);
/* Library version, major*10000 + minor*100 + patch. */
int rpt_version(void);

/* Per-stage timing, for profiling (off by default).  While enabled, each
 * kernel stage of every call records a pair of HIP events on the caller's
 * stream ("prep", "naive_contract", "sampled_t", "complete", "recon_fused",
 * "recon_filter", "recon_refine", "reorth", "track_update", "sigma", ...).
 * rpt_timing_query waits for the recorded events of one stage and returns the
 * summed elapsed time in ms and the number of records (0 = found, -1 = no
 * records, -2 = HIP error).  rpt_timing_stages writes the recorded stage
 * names, comma separated, into buf and returns the full length.  Enabling
 * timing is not meant for calls under HIP graph capture. */
void rpt_timing_enable(int on);
void rpt_timing_reset(void);
int rpt_timing_query(const char* stage, double* total_ms, int64_t* count);
int rpt_timing_stages(char* buf, size_t len);

/* -------------------------------------------------------------------------
 * Autotuning of tile choices.
 *
 * The NaivePT contraction and the fused reconstruction (recovery) split the
 * voxels of every group of relabellings into chunks, one workgroup each.  The
 * planners start from a rule of thumb (about 1,280 workgroups); these calls
 * time the candidate chunk counts around it (half, same, 2, 4, 8 and 16 times,
 * multiples of 8) on the given shape and keep the fastest in the library's
 * plan table, which every later call of that exact shape (v, L, n or r,
 * precision) uses.  Workspace sizes already cover every candidate, so tuned
 * and untuned calls take the same workspaces, and results do not depend on
 * the choice (the column maxima are exact maxima of the same values).
 *
 * rpt_autotune_naive: prepares X, then times `reps` contractions of `labels`
 *   (L x n) per candidate: max-only when T_out is NULL, else the launch that
 *   also writes T (L x v FP32 DEVICE scratch owned by the caller, as
 *   rpt_naive_maxnull's T_out; its contents are overwritten), each form
 *   tuned for itself.  Other arguments and the workspace as
 *   rpt_naive_maxnull.  *chosen (HOST int32) receives the kept count.
 * rpt_autotune_recover: times `reps` reconstruction calls per candidate for
 *   L_rec columns of rank r over v voxels on synthetic data in its own
 *   workspace (rpt_autotune_recover_workspace bytes); sigma = 1, so every
 *   voxel draws its noise, the fused path's full work.
 * Both synchronise `stream`, create and destroy HIP events, and must not be
 * called during graph capture.
 * rpt_autotune_save / rpt_autotune_load: the plan table as text, one line
 *   "kernel v L dim variant chunks" per entry; return the number of entries
 *   written / read, or -1 if the file cannot be opened.  A file named by the
 *   environment variable RPT_TUNE_CACHE is read on first use of the table.
 * rpt_autotune_clear empties the table; rpt_autotune_count reports its size.
 * ------------------------------------------------------------------------- */
rpt_status rpt_autotune_naive(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                              const uint8_t* labels, int64_t L, int prec, float* T_out, int32_t reps,
                              void* ws, size_t ws_bytes, void* stream, int32_t* chosen);
size_t rpt_autotune_recover_workspace(int64_t v, int32_t r, int64_t L_rec);
rpt_status rpt_autotune_recover(int64_t v, int32_t r, int64_t L_rec, int32_t reps,
                                void* ws, size_t ws_bytes, void* stream, int32_t* chosen);
int rpt_autotune_save(const char* path);
int rpt_autotune_load(const char* path);
void rpt_autotune_clear(void);
int rpt_autotune_count(void);

/* -------------------------------------------------------------------------
 * NaivePT -- Alg. 1 (Sec. 2.1).
 *
 * For each of the L relabellings, computes the t statistic at all v voxels and
 * writes its maximum to max_out[i] (signed or absolute, `tail`).  Group sums
 * are formed as a GEMM of the per-voxel standardised data with the 0/1
 * relabelling indicator on the matrix cores (`prec`).
 *
 *   X        v x n FP32, leading dimension ldx >= n            (in)
 *   labels   L x n uint8 relabellings, exactly n1 ones per row (in)
 *   max_out  L FP32                                            (out)
 *   T_out    NULL, or L x v FP32: the full permutation testing matrix,
 *            row i = t map of relabelling i (for tests and training)   (out)
 *   stat     RPT_STAT_T (Eq. 2) or RPT_STAT_MEANDIFF (balanced designs only)
 * Requirements: v >= 1, 4 <= n <= 512, 2 <= n1 <= n-2, L >= 0.
 * n1 != n - n1 (unbalanced designs) needs prec == RPT_FP32 and stat ==
 * RPT_STAT_T; RPT_FP32 takes n <= 128 (RPT_ERR_UNSUPPORTED above).  The
 * subject limit n <= 512 applies to every entry point that takes X.
 * ------------------------------------------------------------------------- */
size_t rpt_naive_workspace(int64_t v, int32_t n, int64_t L, int prec);
rpt_status rpt_naive_maxnull(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                             const uint8_t* labels, int64_t L, int tail, int prec, int stat,
                             float* max_out, float* T_out,
                             void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Sampled t statistics -- the test() step of RapidPT recovery (Alg. 2).
 *
 * y[i*k + q] = statistic `stat` (as rpt_naive_maxnull) of voxel
 * omega[i*k + q] under relabelling i.
 *   omega  L x k int32 voxel indices in [0, v), k >= 1      (in)
 *   y      L x k FP32                                       (out)
 * ------------------------------------------------------------------------- */
size_t rpt_sampled_tstat_workspace(int64_t v, int32_t n);
rpt_status rpt_sampled_tstat(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                             const uint8_t* labels, int64_t L,
                             const int32_t* omega, int32_t k, int stat, float* y,
                             void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Complete -- the masked least-squares fit of Alg. 2 (Sec. 4.2).
 *
 * For each column i: w_i = argmin_w || U[omega_i, :] w - y_i ||_2, solved from
 * the normal equations (Gram matrix of the sampled basis rows, FP64 Cholesky).
 *   U      v x r FP32 row-major (row k = voxel k)              (in)
 *   omega  L x k int32, k >= r                                 (in)
 *   y      L x k FP32 sampled values                           (in)
 *   W      L x r FP32, row i = w_i                              (out)
 *   resid  NULL or L x k FP32: y - U[omega] w                   (out)
 *   info   L int32: 0 = ok, j > 0 = leading minor j not positive (out)
 * Requirements: 1 <= r <= 128, r <= k.
 * ------------------------------------------------------------------------- */
size_t rpt_complete_workspace(int64_t L, int32_t r);
rpt_status rpt_complete(const float* U, int64_t v, int32_t r,
                        const int32_t* omega, int32_t k, const float* y, int64_t L,
                        float* W, float* resid, int32_t* info,
                        void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Subspace training -- the TRAINING half of Alg. 2 (Sec. 4.1).
 *
 * 1. T_ex: the t maps of the l training relabellings (the same contraction as
 *    NaivePT); train_max[i] = max_k T_ex[i, k] (exact maxima).
 * 2. U <- orthonormalised U0 (Q factor with positive diagonal R).
 * 3. Subspace tracking, up to `passes` passes over the l columns; the visit of
 *    column i in pass p samples omega_train[(p*l + i)*k ..+k).
 *    batch == 1 (the paper's mode, Sec. 4.1: each column modifies the
 *      estimate of U in turn): GROUSE's geodesic step on the column, with
 *      w = Complete(U, omega, t), p = U w, e the sampled residual and
 *      theta = gamma * arctan(|e| / |p|) (gamma = 1: the greedy step):
 *      U <- U + ((cos theta - 1) p/|p| + sin theta e/|e|) w^T/|w|.  Needs
 *      0 < gamma < 1.5.
 *      Stopping rule ("until convergence"): the objective of a pass is Eq. 1
 *      on the entries it samples, sum_i |e_i|^2 taken before U moves; with
 *      tol > 0 tracking stops after the first pass p >= 1 (counted from 0)
 *      whose objective fell by at most tol (relative) from pass p - 1.
 *    batch > 1 (a variant, not the paper's): mini-batches of `batch` columns
 *      fitted on the same U move it by gamma * sum_i e_i w_i^T / |w_i|^2,
 *      then re-orthonormalisation; all `passes` passes run (tol must be 0).
 *    tracker->kind == RPT_TRACK_L1 (batch 1; GRASTA, He, Balzano & Szlam
 *      2012, cited beside GROUSE in Sec. 3.1 and 4.1): each column's fit is
 *      min |t_O - U_O w|_1, by tracker->admm_iters ADMM iterations on
 *      min |s|_1 s.t. U_O w + s = t_O with penalty tracker->rho, then one
 *      more w step; Gamma = lam + rho (U_O w + s - t_O) on the sampled
 *      voxels is orthogonal to U and U moves along the geodesic of -Gamma w^T
 *      by the angle min(gamma |Gamma| |w|, pi/2):
 *      U <- U + ((cos th - 1) U w/|w| - sin th Gamma/|Gamma|) w^T/|w|.
 *      The pass objective is sum_i |t_O - U_O w_i|_1.
 *    tracker->kind == RPT_TRACK_GRADIENT (any batch; the masked loss
 *      f(U, W) = 1/2 sum_i |P_O_i (t_i - U w_i)|^2 of Eq. 1 drives U, through
 *      the same backward as rpt_masked_loss_bwd): per mini-batch every
 *      column is fitted (w_i = Complete), dU = -sum_i P_O_i(e_i) w_i^T (its
 *      Riemannian projection (I - U U^T) dU equals dU at the least-squares
 *      fit), U <- qr(U - gamma dU).  gamma is the step length (scale it
 *      with the data: the step grows with |e| |w|); all `passes` passes run
 *      (tol must be 0); the pass objective is sum_i |e_i|^2.  Summation
 *      into dU uses atomics, so two runs may differ in FP32 rounding.
 * 4. sigma = sample std (N-1) of the Complete residuals of every training
 *    column on a fresh sampled set omega_sm (l x k); mu by `mu_rule`, with the
 *    mean-gap rule drawing the noise on stream RPT_STREAM_TRAINING.
 *
 *   U0           v x r FP32 Gaussian (or any full-rank) start       (in)
 *   omega_train  (passes*l) x k int32                               (in)
 *   omega_sm     l x k int32                                        (in)
 *   U_out        v x r FP32 orthonormal basis                       (out)
 *   sigma_mu     2 FP32 on the device: {sigma, mu}                  (out)
 *   train_max    l FP32                                             (out)
 *   T_ex_out     NULL or l x v FP32                                 (out)
 *   info         l int32: 0, or (batch 1) -1 / -2 when a column's fit
 *                failed (Gram not positive definite / no convergence) and
 *                U did not move; then the status of the sigma fits  (out)
 *   objective    NULL or passes FP64: each pass's objective (batch 1 and
 *                the gradient tracker; 0 for passes not run, and for the
 *                batch > 1 variant)                                 (out)
 *   passes_used  NULL or 1 int32: passes run                         (out)
 *   stat         the statistic of T_ex (as rpt_naive_maxnull)
 *   tracker      NULL (GROUSE) or host pointer to an rpt_tracker     (in)
 * Requirements: as NaivePT and Complete; balanced designs (n1 = n - n1);
 * 1 <= batch <= l; gamma > 0; tol >= 0; the l1 tracker needs batch 1.
 * ------------------------------------------------------------------------- */
size_t rpt_train_workspace(int64_t v, int32_t n, int32_t ell, int32_t r, int32_t k, int prec);
rpt_status rpt_train_subspace(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                              const uint8_t* train_labels, int32_t ell,
                              const float* U0, int32_t r,
                              const int32_t* omega_train, int32_t k, int32_t passes,
                              int32_t batch, float gamma, double tol,
                              const int32_t* omega_sm, uint64_t seed, int mu_rule, int prec, int stat,
                              const rpt_tracker* tracker,
                              float* U_out, float* sigma_mu, float* train_max, float* T_ex_out,
                              int32_t* info, double* objective, int32_t* passes_used,
                              void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * sigma and mu of Alg. 2 from held-out columns.  Sec. 4.1 estimates the
 * residual spread and the shift of the max null from training columns; the
 * basis was fitted to those columns, so their residuals understate the
 * residuals of unseen ones.  This call computes h further columns in full
 * (the relabellings `labels`, as T_ex of rpt_train_subspace: stored t maps
 * and their exact maxima col_max) and applies the same rules as step 4 of
 * rpt_train_subspace to them with the given basis: sigma = sample std of the
 * Complete residuals on the sampled sets omega (h x k), mu by mu_rule (the
 * mean-gap rule draws its noise on stream RPT_STREAM_TRAINING, columns
 * 0..h-1).  The result replaces the training call's sigma_mu for recovery.
 *
 *   labels    h x n uint8, exactly n1 ones per row                  (in)
 *   U         v x r FP32 trained basis                              (in)
 *   omega     h x k int32                                           (in)
 *   sigma_mu  2 FP32 on the device {sigma, mu}                      (out)
 *   col_max   h FP32: max_k of each held-out column                 (out)
 *   info      h int32 (as rpt_complete)                             (out)
 * Requirements: as rpt_train_subspace (balanced designs; r <= k).
 * ------------------------------------------------------------------------- */
size_t rpt_sigma_mu_workspace(int64_t v, int32_t n, int32_t h, int32_t r, int32_t k, int prec);
rpt_status rpt_sigma_mu(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                        const uint8_t* labels, int32_t h, const float* U, int32_t r,
                        const int32_t* omega, int32_t k, uint64_t seed, int mu_rule, int prec, int stat,
                        float* sigma_mu, float* col_max, int32_t* info,
                        void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Recovery -- the RECOVERY half of Alg. 2 (Sec. 4.2).
 *
 * For each recovered column j (global column index col0 + j): t at the sampled
 * voxels omega_j, w_j = Complete(U, omega_j, t), s ~ N^v(0, sigma^2) from the
 * counter-based generator on stream RPT_STREAM_RECOVERY, and
 *     max_out[j] = max_k ( (U w_j)_k + s_k ) + mu.
 * U W is never written out: a BF16 matrix-core pass bounds every voxel's
 * reconstructed value, and only voxels that can still attain the maximum are
 * recomputed in FP32 with their noise draw.  For small sigma the pass bounds
 * U w alone and the proven noise bound |z| < 5.8872 selects the candidates;
 * otherwise the pass adds every voxel's exact noise draw and only the voxel
 * streams whose bound maximum lies within twice the pass's error bound of the
 * column's best are recomputed.
 *
 *   U         v x r FP32 (orthonormal basis from training)          (in)
 *   sigma_mu  2 FP32 on the device {sigma, mu}                      (in)
 *   omega     L_rec x k int32 when omega_ptr is NULL; otherwise the
 *             CSR indices of uneven sampled sets: row j holds
 *             omega_ptr[j+1] - omega_ptr[j] distinct voxels, every row
 *             at most k long (k sizes the workspace); a row shorter
 *             than r gives a failed fit in info               (in)
 *   omega_ptr NULL or int64 [L_rec + 1] CSR offsets, omega_ptr[0] = 0 (in)
 *   stat      the statistic sampled (as rpt_naive_maxnull)          (in)
 *   max_out   L_rec FP32                                            (out)
 *   W_out     NULL or L_rec x r FP32 (the fitted coefficients)      (out)
 *   info      L_rec int32: 0, or the size + 1 of a sampled set with
 *             fewer than r voxels, or -1 / -2 when the fit's conjugate
 *             gradients met a non-positive curvature (a singular Gram
 *             matrix) / did not converge; a failed fit has w = 0      (out)
 * Requirements: balanced designs; 1 <= r <= 128; r <= k.
 * ------------------------------------------------------------------------- */
size_t rpt_recover_workspace(int64_t v, int32_t n, int64_t L_rec, int32_t r, int32_t k);
rpt_status rpt_recover_maxnull(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                               const uint8_t* labels, int64_t L_rec, int64_t col0,
                               const float* U, int32_t r, const float* sigma_mu,
                               const int32_t* omega, int32_t k, const int64_t* omega_ptr,
                               uint64_t seed, int stat,
                               float* max_out, float* W_out, int32_t* info,
                               void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Alg. 2 end to end: the TRAINING half (as rpt_train_subspace) followed by
 * the RECOVERY half (as rpt_recover_maxnull with col0 = l, the basis, sigma
 * and mu just trained).  h^L is returned as its L = l + L_rec samples:
 * h_out[0..l) the exact training maxima, h_out[l..l+L_rec) the recovered
 * maxima + mu.
 *
 * Steps that do not depend on each other run on a second stream of the same
 * device (created by the first call on that device, default priority, kept
 * until the process ends): the orthonormalisation of U0 while T_ex is
 * computed on `stream`, then the sampled t statistics of the recovered
 * columns (they need no basis) while the tracking passes run on `stream`.
 * The call joins that stream back into `stream` before it returns, so every
 * output is ordered on `stream` like any other call.  A first call made
 * while `stream` is being captured into a graph, or a device where the
 * second stream cannot be created, runs every step on `stream` instead.
 *
 *   train_labels  l x n uint8;  rec_labels  L_rec x n uint8             (in)
 *   U0, omega_train, omega_sm, passes, batch, gamma, tol, mu_rule, prec,
 *   stat, tracker: as rpt_train_subspace;  omega_rec  L_rec x k int32    (in)
 *   h_out         l + L_rec FP32                                        (out)
 *   U_out         v x r FP32 trained basis                              (out)
 *   sigma_mu      2 FP32 on the device {sigma, mu}                      (out)
 *   train_info    l int32 (as rpt_train_subspace);  rec_info  L_rec int32
 *                 (as rpt_recover_maxnull)                          (out)
 *   objective, passes_used: as rpt_train_subspace                       (out)
 *   ws            rpt_rapidpt_workspace(v, n, l, L_rec, r, k, prec) bytes,
 *                 plus rpt_rapidpt_gen_workspace(n, l, L_rec, k, passes)
 *                 when any of the labels or sampled sets is NULL
 * Inputs drawn from the seed: train_labels, rec_labels, U0, omega_train,
 * omega_sm and omega_rec may each be NULL.  The call then draws them as
 * rpt_gen_relabellings, rpt_gen_sampled_sets and rpt_gen_start_basis do with
 * the same seed: relabelling c and the sets of column c of h^L use row c
 * (training columns 0..l-1, then the recovered ones); the sigma/mu and
 * recovery sets are set 0 and tracking pass p uses set 1 + p; the labels and
 * sets go to the workspace after its first rpt_rapidpt_workspace bytes, the
 * Gaussian start basis straight into U_out.  Drawn sets need k <= 4096
 * (RPT_ERR_UNSUPPORTED above).
 * Errors: those of rpt_train_subspace and rpt_recover_maxnull, all checked
 * before the first launch.
 * ------------------------------------------------------------------------- */
size_t rpt_rapidpt_workspace(int64_t v, int32_t n, int32_t ell, int64_t L_rec, int32_t r, int32_t k, int prec);
size_t rpt_rapidpt_gen_workspace(int32_t n, int32_t ell, int64_t L_rec, int32_t k, int32_t passes);
rpt_status rpt_rapidpt_maxnull(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                               const uint8_t* train_labels, int32_t ell,
                               const uint8_t* rec_labels, int64_t L_rec,
                               const float* U0, int32_t r,
                               const int32_t* omega_train, int32_t k, int32_t passes,
                               int32_t batch, float gamma, double tol, const int32_t* omega_sm,
                               const int32_t* omega_rec, uint64_t seed, int mu_rule, int prec, int stat,
                               const rpt_tracker* tracker,
                               float* h_out, float* U_out, float* sigma_mu,
                               int32_t* train_info, int32_t* rec_info,
                               double* objective, int32_t* passes_used,
                               void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Inputs drawn from a seed (Alg. 1 draws Permute[1, n] per relabelling and
 * gives the first n1 subjects group 1, Sec. 2.1; Alg. 2 samples each Omega
 * uniformly without replacement, Sec. 4.1 and 4.2, and starts from Rand.
 * Orth.).  Every draw is a word of Philox4x32-10 (Salmon et al., SC'11) with
 * key = (seed mod 2^32, seed >> 32) and counter (j >> 2, row, stream, set),
 * step j taking word j & 3; an index on [0, m) is the high half of the
 * 64-bit product of the word and m.  A partial Fisher-Yates shuffle of k
 * steps over 0..m-1 (step j draws t on [j, m) and swaps entries j and t)
 * chooses the subset.  Rows are independent: any range can be drawn alone.
 *
 * rpt_sample_count: |Omega| = ceil(eta v) for eta = eta_ppm / 10^6, in
 *   integer arithmetic; -1 when v < 0 or eta_ppm is outside [0, 10^6].
 * rpt_gen_relabellings: rows row0..row0+L-1 (stream 0, set 0), each n uint8
 *   entries with 1 for the n1 shuffled-in subjects (group 1), to `labels`
 *   (L x n, device).  2 <= n <= 512, 1 <= n1 < n, row0 + L <= 2^32.
 * rpt_gen_sampled_sets: rows row0..row0+rows-1 of set `set_id` (stream 1),
 *   each k distinct voxel indices in [0, v) in ascending order, to `omega`
 *   (rows x k int32, device).  1 <= k <= v; k above 4096 returns
 *   RPT_ERR_UNSUPPORTED (the shuffle keeps its displaced entries in LDS).
 * rpt_gen_start_basis: the v x r FP32 Gaussian matrix (row-major, device)
 *   whose entry (q, c) is the residual-noise draw of column c at voxel q on
 *   stream 3 (Box-Muller of words 0, 1 or 2, 3 of the call (q, c >> 2, 3,
 *   0)); Rand. Orth. of rpt_train_subspace orthonormalises it.
 * All three validate synchronously, launch on `stream` and never allocate.
 * ------------------------------------------------------------------------- */
int64_t rpt_sample_count(int64_t v, int32_t eta_ppm);
rpt_status rpt_gen_relabellings(uint64_t seed, int64_t row0, int64_t L, int32_t n, int32_t n1, uint8_t* labels,
                                void* stream);
rpt_status rpt_gen_sampled_sets(uint64_t seed, int32_t set_id, int64_t row0, int64_t rows, int64_t v, int32_t k,
                                int32_t* omega, void* stream);
rpt_status rpt_gen_start_basis(uint64_t seed, int64_t v, int32_t r, float* U, void* stream);

/* -------------------------------------------------------------------------
 * Recovery phase of Alg. 2 for several studies in one call, with uneven
 * sampled sets (Alg. 2 RECOVERY; the per-study sampled-set sizes follow from
 * eta and each study's v).  Per study the same steps as rpt_recover_maxnull:
 * sampled t, Complete, U w + noise, Max + mu.  The noise counter of study s
 * carries its `study` field in the fourth word, so the studies draw
 * independent noise from one seed.
 *
 *   studies   HOST array of n_studies descriptors (read during the call
 *             only); every pointer inside is DEVICE memory owned by the caller:
 *     X, v, n, ldx, n1, labels, L_rec, col0, U, r, sigma_mu, seed: as in
 *             rpt_recover_maxnull
 *     omega_ptr  int64 [L_rec + 1], omega_ptr[0] = 0: CSR offsets of the
 *             sampled sets; row i holds omega_ptr[i + 1] - omega_ptr[i]
 *             distinct voxel indices (at least r of them for a solvable fit)
 *     omega_idx  int32 [nnz] voxel indices; nnz = omega_ptr[L_rec] must be
 *             passed as the host value `nnz`
 *     max_out  [L_rec] FP32 recovered maxima + mu;  info  [L_rec] int32 as
 *             rpt_recover_maxnull (a row with fewer than r entries fails)
 * Launches are only stream-ordered kernels on `stream` (no host
 * synchronisation, allocation or host reads of device memory), so the call
 * can be captured into a HIP graph.  The sampled-t and Complete steps of the
 * studies share one workspace region in turn; each study keeps its W and its
 * reconstruction buffers, and the fused U w + noise + max of up to 16 studies
 * runs as one persistent launch (results identical to rpt_recover_maxnull per
 * study).  rpt_recover_batched_workspace gives the bytes (0 for an invalid
 * descriptor).
 * Errors: as rpt_recover_maxnull, checked for every study before any launch.
 * ------------------------------------------------------------------------- */
typedef struct rpt_study {
  const float* X;
  int64_t v;
  int32_t n;
  int32_t n1;
  int64_t ldx;
  const uint8_t* labels;
  int64_t L_rec;
  int64_t col0;
  const float* U;
  int32_t r;
  uint32_t study;
  const float* sigma_mu;
  const int64_t* omega_ptr;
  const int32_t* omega_idx;
  int64_t nnz;
  uint64_t seed;
  float* max_out;
  int32_t* info;
} rpt_study;
size_t rpt_recover_batched_workspace(const rpt_study* studies, int32_t n_studies);
rpt_status rpt_recover_maxnull_batched(const rpt_study* studies, int32_t n_studies,
                                       void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * Inference on the observed labelling (Sec. 2; Sec. 5.5; Eq. 4).
 *
 * rpt_observed_tstat: t of Eq. 2 (reading: unbiased group variances) for
 *   every voxel under the observed labelling, group 1 = subjects 0..n1-1 of
 *   X (v x n FP32, row stride ldx), into t_out [v] FP32.  Workspace from
 *   rpt_observed_tstat_workspace (256-byte aligned).  4 <= n <= 512,
 *   2 <= n1 <= n - 2.
 * rpt_fwer_threshold: *thr_out (device FP32) = the ascending order statistic
 *   m_(L - floor(alpha L)) (1-based) of maxima [L]: the level-alpha
 *   family-wise threshold.  0 <= alpha < 1.
 * rpt_corrected_pvalues: p_out [v] = #{i : maxima_i >= t_k} / L for every
 *   entry of t [v] (the fraction of the max null at least as extreme).
 * rpt_rejection_counts: counts_out (device int64 [3]) = v1, v2, vc: voxels
 *   with corrected p <= alpha under maxima1 [L1], under maxima2 [L2], and
 *   under both; Eq. 4's resampling risk is ((v1-vc)/v1 + (v2-vc)/v2) / 2.
 * All pointers are device memory owned by the caller; the comparisons are
 * exact in FP32 and the p <= alpha decision is taken in FP64 as (c / L) <=
 * alpha.  Invalid sizes or null pointers give RPT_ERR_INVALID_ARG.
 * ------------------------------------------------------------------------- */
size_t rpt_observed_tstat_workspace(int64_t v, int32_t n);
rpt_status rpt_observed_tstat(const float* X, int64_t v, int32_t n, int64_t ldx, int32_t n1,
                              float* t_out, void* ws, size_t ws_bytes, void* stream);
rpt_status rpt_fwer_threshold(const float* maxima, int64_t L, double alpha, float* thr_out,
                              void* stream);
rpt_status rpt_corrected_pvalues(const float* maxima, int64_t L, const float* t, int64_t v,
                                 float* p_out, void* stream);
rpt_status rpt_rejection_counts(const float* maxima1, int64_t L1, const float* maxima2, int64_t L2,
                                const float* t, int64_t v, double alpha, int64_t* counts_out,
                                void* stream);

/* -------------------------------------------------------------------------
 * Orthonormalisation used by training: U <- U R^{-1}, with R^T R = U^T U
 * (Cholesky-QR, Gram and Cholesky in FP64, applied twice).  In place.
 *   U  v x r FP32 (in/out).  Requirements: 1 <= r <= 128, v >= r.
 * ------------------------------------------------------------------------- */
size_t rpt_reorth_workspace(int64_t v, int32_t r);
rpt_status rpt_reorth(float* U, int64_t v, int32_t r, int32_t* info,
                      void* ws, size_t ws_bytes, void* stream);

/* -------------------------------------------------------------------------
 * rpt_reorth without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  The arguments of rpt_reorth without the workspace,
 * and its kernels and results; the scratch space is a fixed device array
 * inside the library (every kernel writes what it later reads, so nothing
 * in it needs clearing between calls),
 * rpt_reorth_noalloc_capacity() bytes (28.5 MB: every v with r <= 128 fits),
 * held on each GPU the library runs on until the process ends.  The call
 * allocates nothing.  Every call on one GPU shares that GPU's array, so two
 * calls that overlap in time on one GPU (different streams without ordering
 * between them) race and corrupt each other's results.  The first call on a
 * GPU looks up the array's device address (hipGetSymbolAddress); later calls
 * do not touch the runtime beyond their launches.  A size beyond the array
 * gives RPT_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------- */
size_t rpt_reorth_noalloc_capacity(void);
rpt_status rpt_reorth_noalloc(float* U, int64_t v, int32_t r, int32_t* info, void* stream);

/* -------------------------------------------------------------------------
 * Masked completion loss of Eq. 1 and its gradient.
 *
 *   f = 1/2 sum_b sum_{k in Omega_b} (t_bk - U[k,:] W[:,b])^2
 * Sampled sets are CSR: omega_ptr[B+1] (int64, omega_ptr[0] = 0), omega_idx
 * [nnz] voxel indices (distinct within a row), t_vals[nnz].
 *   U       v x r FP32 row-major        W   r x B FP32 row-major
 *   loss    1 FP64 on the device (out)   resid  nnz FP32 = t - U W (out)
 *   dU      v x r FP32, fully overwritten (zero outside sampled rows) (out)
 *   dW      r x B FP32 (out)
 *   grad_scale  device FP64 scalar multiplying both gradients (the upstream
 *           gradient of an autograd chain), or NULL for 1.
 * The backward takes the residuals the forward wrote.  Errors: null required
 * pointers or negative sizes give RPT_ERR_INVALID_ARG; r > 1024 gives
 * RPT_ERR_UNSUPPORTED.  Out-of-range voxel indices are treated as zero rows.
 * ------------------------------------------------------------------------- */
rpt_status rpt_masked_loss_fwd(const float* U, int64_t v, int32_t r, const float* W, int32_t B,
                               const int64_t* omega_ptr, const int32_t* omega_idx,
                               const float* t_vals, int64_t nnz,
                               double* loss, float* resid, void* stream);
rpt_status rpt_masked_loss_bwd(const float* U, int64_t v, int32_t r, const float* W, int32_t B,
                               const int64_t* omega_ptr, const int32_t* omega_idx,
                               const float* resid, int64_t nnz,
                               float* dU, float* dW, const double* grad_scale, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RPT_H */
