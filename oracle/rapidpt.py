"""Oracle: RapidPT training and recovery (Sec. 4, Alg. 2).  TEST INFRASTRUCTURE.

Steps, in the paper's order and notation (T is stored L x v here: row i is
column i of the paper's v x L matrix):

TRAINING (Sec. 4.1)
  U <- Rand. Orth.          : Q factor (positive diag R) of a v x r Gaussian.
  T_ex[:, i] <- test(...)   : l fully computed columns (``tstat.tmatrix``).
  Subspace-Tracking(r)      : passes over the l columns, one column at a time;
                              each visit samples ceil(eta v) voxels, fits the
                              column on them by least squares (Complete) and
                              moves U; passes repeat until the subspace stops
                              moving (or a pass cap is reached).
  sigma, mu                 : residual spread and max-null shift.
RECOVERY (Sec. 4.2)
  for each remaining column: sample Omega_i, t on the sampled voxels,
  w = Complete(U, t_Omega), s ~ N^v(0, sigma^2), m_i = Max(U w + s) + mu.

Readings where the paper is silent:

* Subspace tracking is GROUSE (Balzano, Nowak & Recht 2010, the l2 tracker
  the paper cites), applied to the training columns one by one as Sec. 4.1
  describes, with the greedy step angle theta = arctan(|r| / |p|) (Zhang &
  Balzano 2016) scaled by gamma (1 = greedy): U <- U + ((cos theta - 1) p/|p|
  + sin theta r/|r|) w^T/|w|, p = U w the fitted column, r the residual on the
  sampled entries (zero elsewhere).  ``grouse_step``.
* "Until convergence": the tracking minimises Eq. 1 one visit at a time; the
  objective of a pass is the sum over its visits of the squared residual of
  the column's fit on its sampled entries, taken before U moves.  Tracking
  stops after the first pass (from the second on) whose objective fell by at
  most a relative tolerance from the pass before, or after the given number
  of passes (tol = 0 runs them all).
  ``subspace_change`` and ``calibration`` measure how far the basis moved and
  how far it is from T_ex's leading singular subspace; they are reports, not
  part of the rule.
* A non-paper variant (``batch`` > 1) moves U by the summed first-order
  updates r_b w_b^T / |w_b|^2 of a mini-batch of columns, all fitted on the
  same U, then re-orthonormalises by QR (Jacobi-style; B = 1 spans the same
  subspace as one greedy GROUSE step).  ``track_step``.
* A fresh sampled set is drawn for every (pass, column) visit.
* sigma: sample standard deviation (divisor N-1) of the least-squares residuals
  y - U_Omega w over all sampled entries of a final pass over the l columns
  with fresh sets and the final U (Alg. 2's Std over Omega).
* mu ("mean_gap", default): the mean over training columns of
  max(T_ex[:, i]) - max(U w_i + s_i), with s_i drawn like recovery noise on
  the training stream; it measures the downward shift of the recovered
  maximum that Sec. 4.1 describes.  ``mu_rule="literal"`` is Alg. 2's
  sup_i Max(T_ex[:, i] - U W_ex[:, i]); ``"zero"`` disables the shift.
* Complete is the ordinary least-squares fit on the sampled rows.
* The statistic is an input of Alg. 2: the t statistic of Eq. 2 (``"t"``) or
  the linear mean difference (``"meandiff"``), whose permutation matrix has
  rank at most n - 1 (Sec. 3.2).
* The first l maxima are the exact training maxima (Alg. 2), the rest are
  recovered; the recovered maximum is signed.

Pins (tests/test_oracle_rapidpt.py): least squares vs. the normal equations
and an explicit residual-orthogonality check; the geodesic step written out
from GROUSE's definition, orthonormality after every step and for any gamma;
the greedy-step identity (refitting the same column on the same set gives a
zero residual); sequential tracking and the mini-batch variant each recover
an exactly rank-r subspace from sampled (not full) observations, principal
angles going to zero, and a sign error in either update fails that; the
subspace change against principal angles; the stopping rule's pass count;
sigma and both mu rules on hand-computed cases (including the sign of the
mean gap); the linear mean-difference statistic, whose permutation matrix is
exactly low rank, where recovery with sigma = mu = 0 reproduces the NaivePT
maxima.  The convergence rate of tracking on t-statistics has no printed
value in the paper: parity unpinned there (GPU and oracle are compared on
identical inputs instead).
"""
from __future__ import annotations

import numpy as np

from . import philox
from .tstat import STATS


def orthonormalize(A: np.ndarray) -> np.ndarray:
    """Q factor of A = QR with R's diagonal made positive (unique for full
    column rank).  Used for 'Rand. Orth.' and after each tracking step."""
    Q, R = np.linalg.qr(np.asarray(A, dtype=np.float64))
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def complete(U: np.ndarray, idx: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Complete (Alg. 2): w = argmin_w |U[idx] w - y|_2 (ordinary least squares)."""
    A = np.asarray(U, dtype=np.float64)[np.asarray(idx)]
    if A.shape[0] < A.shape[1]:
        raise np.linalg.LinAlgError("fewer sampled entries than the rank")
    w, *_ = np.linalg.lstsq(A, np.asarray(y, dtype=np.float64), rcond=None)
    return w


def grouse_step(U: np.ndarray, x: np.ndarray, idx, gamma: float = 1.0, loss: list | None = None) -> np.ndarray:
    """One GROUSE step on column x (length v) observed at the voxels idx.

    w = Complete(U, idx, x[idx]); p = U w; r = x - p on idx, 0 elsewhere;
    theta = gamma * arctan(|r| / |p|);
    U <- U + ((cos theta - 1) p / |p| + sin theta r / |r|) (w / |w|)^T.
    No move when w = 0 or r = 0.  U must be orthonormal (the step keeps it so).
    `loss`, when given, receives |r|^2 (the fit's squared sampled residual
    before the move).
    """
    idx = np.asarray(idx)
    y = np.asarray(x, dtype=np.float64)[idx]
    w = complete(U, idx, y)
    p = U @ w
    r = np.zeros(U.shape[0])
    r[idx] = y - p[idx]
    nw, nr, npn = np.linalg.norm(w), np.linalg.norm(r), np.linalg.norm(p)
    if loss is not None:
        loss.append(nr * nr)
    if nw == 0.0 or nr == 0.0 or npn == 0.0:
        return U
    theta = gamma * np.arctan(nr / npn)
    step = (np.cos(theta) - 1.0) * p / npn + np.sin(theta) * r / nr
    return U + np.outer(step, w / nw)


def track_step(U: np.ndarray, T_rows: np.ndarray, sets, gamma: float = 1.0,
               loss: list | None = None) -> np.ndarray:
    """One mini-batch update of the non-paper Jacobi variant.

    T_rows[b] is the full column of T for batch member b, sets[b] its sampled
    voxel indices.  Returns the re-orthonormalised basis; `loss`, when given,
    receives each member's squared sampled residual.
    """
    D = np.zeros_like(U)
    for b in range(len(sets)):
        idx = np.asarray(sets[b])
        y = T_rows[b][idx]
        w = complete(U, idx, y)
        e = y - U[idx] @ w
        if loss is not None:
            loss.append(float(e @ e))
        nw2 = float(w @ w)
        if nw2 > 0.0:
            D[idx] += np.outer(e, w) * (gamma / nw2)
    return orthonormalize(U + D)


def subspace_change(U_old: np.ndarray, U_new: np.ndarray) -> float:
    """|P_new - P_old|_F / sqrt(2 r) for orthonormal bases (P = U U^T): 0 for
    the same subspace, 1 for orthogonal ones.  Uses |P_a - P_b|_F^2 =
    2 (r - |U_a^T U_b|_F^2)."""
    r = U_old.shape[1]
    C = U_old.T @ U_new
    return float(np.sqrt(max(0.0, r - float(np.sum(C * C))) / r))


def train_subspace(T_ex: np.ndarray, U0: np.ndarray, omega_train: np.ndarray,
                   passes: int, batch: int = 1, gamma: float = 1.0, tol: float = 0.0,
                   history: list | None = None) -> np.ndarray:
    """Subspace tracking over the training columns (Sec. 4.1).

    T_ex: l x v; U0: v x r (orthonormalised first); omega_train:
    (passes*l) x k, row p*l + i is the sampled set of column i in pass p.
    batch = 1 is GROUSE column by column (the paper's mode); batch > 1 the
    mini-batch variant.

    Until convergence: the objective of a pass is Eq. 1 on the entries the
    pass samples, sum_i |r_i|^2 with r_i the residual of column i's fit just
    before U moves.  Tracking stops after the first pass p >= 2 whose
    objective fell by at most tol (relative) from the pass before, else after
    `passes` passes (tol = 0: always `passes`).  `history`, when given,
    receives each pass's objective.
    """
    ell = T_ex.shape[0]
    batch = int(batch)
    U = orthonormalize(U0)
    prev = None
    for p in range(passes):
        loss: list = []
        if batch == 1:
            for i in range(ell):
                U = grouse_step(U, T_ex[i], omega_train[p * ell + i], gamma, loss)
        else:
            for b0 in range(0, ell, batch):
                b1 = min(ell, b0 + batch)
                U = track_step(U, T_ex[b0:b1], [omega_train[p * ell + i] for i in range(b0, b1)], gamma, loss)
        obj = float(np.sum(loss))
        if history is not None:
            history.append(obj)
        if tol > 0.0 and prev is not None and prev - obj <= tol * prev:
            break
        prev = obj
    return U


def gradient_step(U: np.ndarray, T_rows: np.ndarray, sets, alpha: float,
                  loss: list | None = None) -> np.ndarray:
    """One step in which the masked loss of Eq. 1 drives U.

    Every batch member b is fitted on the current U (w_b = Complete on its
    sampled set), giving f(U, W) = 1/2 sum_b |P_Omega_b (t_b - U w_b)|^2; the
    Euclidean gradient G = df/dU comes from ``masked_loss.grad``, the
    Riemannian gradient on the Grassmannian is (I - U U^T) G, and U moves
    along it with step size alpha and is retracted by QR:
        U <- qr(U - alpha (I - U U^T) G).
    (With each w_b the exact least-squares fit, U^T G = -sum_b U_O^T e_b w_b^T
    = 0, so the projection changes nothing but rounding.)  `loss`, when given,
    receives each member's |e_b|^2 before U moves."""
    from . import masked_loss as ML
    B = len(sets)
    ptr = np.zeros(B + 1, dtype=np.int64)
    idx, t, W = [], [], np.zeros((U.shape[1], B))
    for b in range(B):
        o = np.asarray(sets[b])
        y = np.asarray(T_rows[b], dtype=np.float64)[o]
        W[:, b] = complete(U, o, y)
        if loss is not None:
            e = y - U[o] @ W[:, b]
            loss.append(float(e @ e))
        ptr[b + 1] = ptr[b] + len(o)
        idx.append(o)
        t.append(y)
    idx = np.concatenate(idx) if B else np.zeros(0, dtype=np.int64)
    t = np.concatenate(t) if B else np.zeros(0)
    G, _ = ML.grad(U, W, ptr, idx, t)
    G = G - U @ (U.T @ G)
    return orthonormalize(U - alpha * G)


def train_subspace_gradient(T_ex: np.ndarray, U0: np.ndarray, omega_train: np.ndarray, passes: int,
                            batch: int, alpha: float, history: list | None = None) -> np.ndarray:
    """Subspace training driven by the masked loss (``gradient_step``) over
    mini-batches of `batch` consecutive training columns, `passes` passes
    (row p l + i of omega_train is column i's set in pass p); `history`
    receives each pass's objective sum_i |e_i|^2."""
    ell = T_ex.shape[0]
    U = orthonormalize(U0)
    for p in range(passes):
        loss: list = []
        for b0 in range(0, ell, batch):
            b1 = min(ell, b0 + batch)
            U = gradient_step(U, T_ex[b0:b1], [omega_train[p * ell + i] for i in range(b0, b1)], alpha, loss)
        if history is not None:
            history.append(float(np.sum(loss)))
    return U


def principal_angle_cosines(U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Cosines of the principal angles between span(U) and span(V)
    (orthonormal columns): the singular values of U^T V, descending."""
    return np.linalg.svd(U.T @ V, compute_uv=False)


def calibration(T_ex: np.ndarray, U: np.ndarray, T_held: np.ndarray | None = None) -> dict:
    """How far a tracked basis is from the best rank-r basis of T_ex: the
    principal angles between U and the r leading left singular vectors of
    T_ex (the brute-force alternative Sec. 4.1 describes), and the residual
    spread of T_ex and of held-out columns after projection onto U."""
    r = U.shape[1]
    Us = np.linalg.svd(T_ex.T, full_matrices=False)[0][:, :r]
    cs = np.clip(principal_angle_cosines(U, Us), 0.0, 1.0)
    out = {"max_angle_deg": float(np.degrees(np.arccos(cs.min()))),
           "mean_cos2": float(np.mean(cs ** 2)),
           "train_resid_std": float(np.std(T_ex - (T_ex @ U) @ U.T))}
    if T_held is not None:
        out["held_resid_std"] = float(np.std(T_held - (T_held @ U) @ U.T))
    return out


def sigma_mu(T_ex: np.ndarray, U: np.ndarray, omega_sm: np.ndarray, seed: int,
             mu_rule: str = "mean_gap"):
    """sigma and mu of Alg. 2 (see the module header for the reading).

    Returns (sigma, mu, train_max) with train_max[i] = max_k T_ex[i, k].
    """
    ell, v = T_ex.shape
    W = []
    res = []
    for i in range(ell):
        idx = omega_sm[i]
        y = T_ex[i, idx]
        w = complete(U, idx, y)
        W.append(w)
        res.append(y - U[idx] @ w)
    sigma = float(np.std(np.concatenate(res), ddof=1))
    train_max = T_ex.max(axis=1)
    ks = np.arange(v)
    if mu_rule == "mean_gap":
        gaps = []
        for i in range(ell):
            a = U @ W[i]
            s = sigma * philox.normals(seed, philox.STREAM_TRAINING, i, ks)
            gaps.append(train_max[i] - np.max(a + s))
        mu = float(np.mean(gaps))
    elif mu_rule == "literal":
        mu = float(max(np.max(T_ex[i] - U @ W[i]) for i in range(ell)))
    elif mu_rule == "zero":
        mu = 0.0
    else:
        raise ValueError(mu_rule)
    return sigma, mu, train_max


def recover_column(X, g1, U, sigma, mu, idx, seed, col, stat="t", study=0):
    """One recovered maximum: the statistic on the sampled voxels, Complete,
    U w + s, Max + mu.  ``study`` is the study field of the noise counter."""
    y = STATS[stat](np.asarray(X, dtype=np.float64)[idx], g1)
    w = complete(U, idx, y)
    a = U @ w
    s = sigma * philox.normals(seed, philox.STREAM_RECOVERY, col, np.arange(U.shape[0]), study)
    return float(np.max(a + s) + mu), w


def recover(X, labels, U, sigma, mu, omegas, seed, col0: int = 0, stat: str = "t", study: int = 0) -> np.ndarray:
    """Recovery phase of Alg. 2 for relabellings labels (L_rec x n) with sampled
    sets omegas (one index array per column, sizes may differ); column j has
    global index col0 + j."""
    return np.array([recover_column(X, labels[j] == 1, U, sigma, mu, omegas[j], seed, col0 + j, stat, study)[0]
                     for j in range(labels.shape[0])])


def rapidpt_maxnull(X, train_labels, rec_labels, U0, omega_train, omega_sm, omega_rec,
                    passes, seed, batch=1, gamma=1.0, mu_rule="mean_gap", stat="t", tol=0.0,
                    history=None):
    """Alg. 2 end to end.  Returns (h, U, sigma, mu): h holds the l exact
    training maxima followed by the L - l recovered ones."""
    X = np.asarray(X, dtype=np.float64)
    T_ex = np.stack([STATS[stat](X, train_labels[i] == 1) for i in range(train_labels.shape[0])])
    U = train_subspace(T_ex, U0, omega_train, passes, batch, gamma, tol, history)
    sigma, mu, tmax = sigma_mu(T_ex, U, omega_sm, seed, mu_rule)
    rec = recover(X, rec_labels, U, sigma, mu, omega_rec, seed, col0=T_ex.shape[0], stat=stat)
    return np.concatenate([tmax, rec]), U, sigma, mu


# ---------------------------------------------------------------------------
# Robust tracking (l1 loss).  Sec. 3.1 and Sec. 4.1 cite GRASTA (He, Balzano
# & Szlam 2012) beside GROUSE as the Grassmannian tracker behind the
# training phase.  Readings where the paper is silent: the column fit is
# min |x_O - U_O w|_1, solved by ADMM on  min |s|_1  s.t.  U_O w + s = x_O
# with a fixed penalty rho and a fixed number of iterations; U moves along
# the geodesic of the augmented Lagrangian's gradient with the constant-step
# angle theta = eta |Gamma| |w| (at most pi / 2).

def l1_fit(A: np.ndarray, y: np.ndarray, rho: float, iters: int):
    """ADMM for min_w |y - A w|_1 written as min |s|_1 s.t. A w + s = y.

    Augmented Lagrangian L = |s|_1 + lam^T (A w + s - y) + rho/2 |A w + s - y|^2;
    each iteration: w <- argmin_w L (least squares), s <- shrink(y - A w -
    lam / rho, 1 / rho), lam <- lam + rho (A w + s - y).  A final w step
    follows, so that Gamma = lam + rho (A w + s - y), the gradient of L with
    respect to the fitted column, satisfies A^T Gamma = 0.
    Returns (w, s, lam, Gamma)."""
    A = np.asarray(A, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    G = A.T @ A
    s = np.zeros_like(y)
    lam = np.zeros_like(y)
    solve = lambda t: np.linalg.solve(G, A.T @ t)
    for _ in range(int(iters)):
        w = solve(y - s - lam / rho)
        f = A @ w
        d = y - f - lam / rho
        s = np.sign(d) * np.maximum(np.abs(d) - 1.0 / rho, 0.0)
        lam = lam + rho * (f + s - y)
    w = solve(y - s - lam / rho)
    gam = lam + rho * (A @ w + s - y)
    return w, s, lam, gam


def grasta_step(U: np.ndarray, x: np.ndarray, idx, eta: float, rho: float, iters: int,
                loss: list | None = None) -> np.ndarray:
    """One robust step on column x observed at idx (U orthonormal, v x r).

    (w, s, lam, Gamma_O) = l1_fit(U[idx], x[idx]); Gamma is Gamma_O on idx
    and 0 elsewhere, so U^T Gamma = 0 and -Gamma w^T is the descent direction
    on the Grassmannian; sigma = |Gamma| |w|, theta = min(eta sigma, pi/2):
    U <- U + ((cos theta - 1) U w / |w| - sin theta Gamma / |Gamma|) w^T / |w|.
    No move when w = 0 or Gamma = 0.  `loss`, when given, receives the l1
    misfit |x_O - U_O w|_1 before the move."""
    idx = np.asarray(idx)
    y = np.asarray(x, dtype=np.float64)[idx]
    w, s, lam, g = l1_fit(U[idx], y, rho, iters)
    if loss is not None:
        loss.append(float(np.sum(np.abs(y - U[idx] @ w))))
    nw, ng = np.linalg.norm(w), np.linalg.norm(g)
    if nw == 0.0 or ng == 0.0:
        return U
    theta = min(eta * ng * nw, 0.5 * np.pi)
    gam = np.zeros(U.shape[0])
    gam[idx] = g
    step = (np.cos(theta) - 1.0) * (U @ w) / nw - np.sin(theta) * gam / ng
    return U + np.outer(step, w / nw)


def train_subspace_l1(T_ex: np.ndarray, U0: np.ndarray, omega_train: np.ndarray, passes: int,
                      eta: float, rho: float = 1.0, iters: int = 30, tol: float = 0.0,
                      history: list | None = None) -> np.ndarray:
    """Robust subspace tracking over the training columns, one column at a
    time (``grasta_step``), with the stopping rule of ``train_subspace`` on
    the pass objective sum_i |x_O - U_O w_i|_1."""
    ell = T_ex.shape[0]
    U = orthonormalize(U0)
    prev = None
    for p in range(passes):
        loss: list = []
        for i in range(ell):
            U = grasta_step(U, T_ex[i], omega_train[p * ell + i], eta, rho, iters, loss)
        obj = float(np.sum(loss))
        if history is not None:
            history.append(obj)
        if tol > 0.0 and prev is not None and prev - obj <= tol * prev:
            break
        prev = obj
    return U
