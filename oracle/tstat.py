"""Oracle: voxel-wise two-sample t statistic and NaivePT.  TEST INFRASTRUCTURE.

Pins (tests/test_oracle_tstat.py): hand-computed values, the pooled-variance
identity for equal group sizes, label-complement antisymmetry, the identity
labelling, per-voxel affine invariance, brute force over all labellings at tiny
n, and scipy.stats.ttest_ind(equal_var=False).

Readings of the paper used here:

* Eq. 2 divides each group's spread by its size inside the square root; the
  text calls sigma_g standard deviations but the formula needs variances.  We
  read sigma_g as the unbiased (divisor n_g - 1) sample variance, i.e. the
  Welch form.  For n1 = n2 this equals the pooled-variance Student t.
* The statistic is signed, positive when group 1 (columns marked 1) has the
  larger mean; Alg. 1 takes a signed maximum.  ``tail="abs"`` gives the
  maximum of |t| instead.
* When both groups have zero spread the denominator is zero and t := 0.
"""
from __future__ import annotations

import numpy as np


def tstat(X: np.ndarray, g1: np.ndarray) -> np.ndarray:
    """Eq. 2 for every row of X (v x n) under the group-1 mask g1 (n bools).

    Two-pass: group means first, then centred sums of squares.
    """
    X = np.asarray(X, dtype=np.float64)
    g1 = np.asarray(g1).astype(bool)
    x1 = X[:, g1]
    x2 = X[:, ~g1]
    n1 = x1.shape[1]
    n2 = x2.shape[1]
    if n1 < 2 or n2 < 2:
        raise ValueError("each group needs at least two subjects")
    m1 = x1.mean(axis=1)
    m2 = x2.mean(axis=1)
    s1 = ((x1 - m1[:, None]) ** 2).sum(axis=1) / (n1 - 1)
    s2 = ((x2 - m2[:, None]) ** 2).sum(axis=1) / (n2 - 1)
    # groups with no spread at all: force an exact zero (rounding in the mean
    # could otherwise leave a tiny positive variance)
    s1 = np.where(np.ptp(x1, axis=1) == 0, 0.0, s1)
    s2 = np.where(np.ptp(x2, axis=1) == 0, 0.0, s2)
    den = np.sqrt(s1 / n1 + s2 / n2)
    num = m1 - m2
    out = np.zeros_like(num)
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out


def tmatrix(X: np.ndarray, labels: np.ndarray) -> np.ndarray:
    """The permutation testing matrix, stored L x v: row i is the t map of
    relabelling i (labels is L x n, 1 = group 1).  Alg. 1, T[:, i]."""
    labels = np.asarray(labels)
    return np.stack([tstat(X, labels[i] == 1) for i in range(labels.shape[0])])


def column_max(t: np.ndarray, tail: str = "signed") -> float:
    """Max over voxels of one column of T (Alg. 1, m_i = Max(T[:, i]))."""
    if tail == "signed":
        return float(np.max(t))
    if tail == "abs":
        return float(np.max(np.abs(t)))
    raise ValueError(tail)


def naive_maxnull(X: np.ndarray, labels: np.ndarray, tail: str = "signed") -> np.ndarray:
    """NaivePT (Alg. 1): for every relabelling compute the full t map and keep
    its maximum.  Returns the L maxima m_1..m_L (the samples of h^L)."""
    labels = np.asarray(labels)
    X = np.asarray(X, dtype=np.float64)
    return np.array([column_max(tstat(X, labels[i] == 1), tail) for i in range(labels.shape[0])])


def meandiff(X: np.ndarray, g1: np.ndarray) -> np.ndarray:
    """The linear statistic mean(group 1) - mean(group 2) per voxel.

    Alg. 2 takes the statistic as an input ("stat"); with this linear choice
    every column of T lies in the span of the centred data, so T has rank at
    most n - 1 (Sec. 3.2) -- the exact special case used to pin recovery.
    """
    X = np.asarray(X, dtype=np.float64)
    g1 = np.asarray(g1).astype(bool)
    return X[:, g1].mean(axis=1) - X[:, ~g1].mean(axis=1)


STATS = {"t": tstat, "meandiff": meandiff}
