"""Oracle: masked completion loss and its gradient.  TEST INFRASTRUCTURE.

Eq. 1 fits T on the sampled entries Omega with T_hat = U W.  For a batch of B
columns with sampled sets given in CSR form (ptr[B+1], idx[nnz]) and sampled
values t[nnz]:

    f(U, W) = 1/2 sum_b sum_{k in Omega_b} (t_bk - U[k, :] W[:, b])^2
    df/dW[:, b] = - sum_{k in Omega_b} U[k, :]^T e_bk
    df/dU[k, :] = - sum_{b : k in Omega_b} e_bk W[:, b]^T

with e_bk = t_bk - U[k, :] W[:, b].  Everything in FP64.

Pins (tests/test_oracle_masked_loss.py): the loss is quadratic in every single
coordinate, so central differences with h = 1e-3 carry no truncation error;
the analytic gradient must match them to rounding.  Also checked against a
dense formulation with an explicit 0/1 mask.
"""
from __future__ import annotations

import numpy as np


def residuals(U, W, ptr, idx, t):
    U = np.asarray(U, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    e = np.empty(len(idx), dtype=np.float64)
    for b in range(len(ptr) - 1):
        s = slice(ptr[b], ptr[b + 1])
        e[s] = np.asarray(t[s], dtype=np.float64) - U[idx[s]] @ W[:, b]
    return e


def loss(U, W, ptr, idx, t) -> float:
    e = residuals(U, W, ptr, idx, t)
    return 0.5 * float(e @ e)


def grad(U, W, ptr, idx, t):
    """(dU, dW) of ``loss``."""
    U = np.asarray(U, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    e = residuals(U, W, ptr, idx, t)
    dU = np.zeros_like(U)
    dW = np.zeros_like(W)
    for b in range(len(ptr) - 1):
        s = slice(ptr[b], ptr[b + 1])
        rows = idx[s]
        dW[:, b] = -U[rows].T @ e[s]
        np.add.at(dU, rows, -np.outer(e[s], W[:, b]))
    return dU, dW


def grad_rows(U, W, ptr, idx, t, rows):
    """dU restricted to the given voxel rows, and the full dW, of ``loss``
    (same sums as ``grad``, without forming the v x r gradient)."""
    U = np.asarray(U, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    e = residuals(U, W, ptr, idx, t)
    pos = {int(k): a for a, k in enumerate(rows)}
    dUr = np.zeros((len(rows), U.shape[1]))
    dW = np.zeros_like(W)
    for b in range(len(ptr) - 1):
        s = slice(ptr[b], ptr[b + 1])
        dW[:, b] = -U[idx[s]].T @ e[s]
        for q in range(ptr[b], ptr[b + 1]):
            a = pos.get(int(idx[q]))
            if a is not None:
                dUr[a] -= e[q] * W[:, b]
    return dUr, dW
