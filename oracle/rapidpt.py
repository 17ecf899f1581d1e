"""Oracle: RapidPT training and recovery (Sec. 4, Alg. 2).  TEST INFRASTRUCTURE.

Steps, in the paper's order and notation (T is stored L x v here: row i is
column i of the paper's v x L matrix):

TRAINING (Sec. 4.1)
  U <- Rand. Orth.          : Q factor (positive diag R) of a v x r Gaussian.
  T_ex[:, i] <- test(...)   : l fully computed columns (``tstat.tmatrix``).
  Subspace-Tracking(r)      : several passes over the l columns; each visit
                              samples ceil(eta v) voxels, fits the column on
                              them by least squares (Complete) and moves U.
  sigma, mu                 : residual spread and max-null shift.
RECOVERY (Sec. 4.2)
  for each remaining column: sample Omega_i, t on the sampled voxels,
  w = Complete(U, t_Omega), s ~ N^v(0, sigma^2), m_i = Max(U w + s) + mu.

Readings where the paper is silent:

* Subspace tracking is GROUSE (Balzano, Nowak & Recht 2010, the l2 tracker the
  paper cites) with the greedy step angle theta = arctan(|r| / |p|) (Zhang &
  Balzano 2016).  For one column that step maps span(U) to the span of U
  restricted to w-perp plus the imputed column p + r, which is exactly
  span(U + r w^T / |w|^2).  We apply this first-order form to a mini-batch of
  B columns at once (all w from the same U, updates summed), scaled by a
  damping factor gamma, then re-orthonormalise by QR.  B = 1 reproduces
  sequential GROUSE's subspace sequence.
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
* The first l maxima are the exact training maxima (Alg. 2), the rest are
  recovered; the recovered maximum is signed.

Pins (tests/test_oracle_rapidpt.py): least squares vs. the normal equations
and an explicit residual-orthogonality check; orthonormality after every
update; the single-column greedy-step identity (refitting the same column on
the same set gives a zero residual); exact recovery of an exactly rank-r
subspace from full observations; the linear mean-difference statistic, whose
permutation matrix is exactly low rank, where recovery with sigma = mu = 0
reproduces the NaivePT maxima.  The convergence rate of tracking on
t-statistics has no printed value in the paper: parity unpinned there (GPU
and oracle are compared on identical inputs instead).
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


def track_step(U: np.ndarray, T_rows: np.ndarray, sets, gamma: float = 1.0) -> np.ndarray:
    """One mini-batch tracking update.

    T_rows[b] is the full column of T for batch member b, sets[b] its sampled
    voxel indices.  Returns the re-orthonormalised basis.
    """
    D = np.zeros_like(U)
    for b in range(len(sets)):
        idx = np.asarray(sets[b])
        y = T_rows[b][idx]
        w = complete(U, idx, y)
        e = y - U[idx] @ w
        nw2 = float(w @ w)
        if nw2 > 0.0:
            D[idx] += np.outer(e, w) * (gamma / nw2)
    return orthonormalize(U + D)


def train_subspace(T_ex: np.ndarray, U0: np.ndarray, omega_train: np.ndarray,
                   passes: int, batch: int | None = None, gamma: float = 1.0) -> np.ndarray:
    """Subspace tracking over the training columns.

    T_ex: l x v; U0: v x r (orthonormalised first); omega_train:
    (passes*l) x k, row p*l + i is the sampled set of column i in pass p.
    """
    ell = T_ex.shape[0]
    batch = ell if batch is None else int(batch)
    U = orthonormalize(U0)
    for p in range(passes):
        for b0 in range(0, ell, batch):
            b1 = min(ell, b0 + batch)
            U = track_step(U, T_ex[b0:b1], [omega_train[p * ell + i] for i in range(b0, b1)], gamma)
    return U


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
                    passes, seed, batch=None, gamma=1.0, mu_rule="mean_gap"):
    """Alg. 2 end to end.  Returns (h, U, sigma, mu): h holds the l exact
    training maxima followed by the L - l recovered ones."""
    from .tstat import tmatrix
    T_ex = tmatrix(X, train_labels)
    U = train_subspace(T_ex, U0, omega_train, passes, batch, gamma)
    sigma, mu, tmax = sigma_mu(T_ex, U, omega_sm, seed, mu_rule)
    rec = recover(X, rec_labels, U, sigma, mu, omega_rec, seed, col0=T_ex.shape[0])
    return np.concatenate([tmax, rec]), U, sigma, mu
