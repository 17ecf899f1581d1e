"""Pins for the oracle's t statistic (Eq. 2) and NaivePT (Alg. 1)."""
import itertools
import statistics

import numpy as np
import pytest
from scipy import stats

from conftest import golden_path
from oracle import tstat as OT


def _read_hand():
    rows = []
    for line in open(golden_path("tstat_hand.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b, t = [p.strip() for p in line.split("|")]
        rows.append(([float(x) for x in a.split(",")], [float(x) for x in b.split(",")], float(t)))
    return rows


@pytest.mark.parametrize("g1,g2,expect", _read_hand())
def test_hand_values(g1, g2, expect):
    X = np.array([g1 + g2])
    mask = np.array([True] * len(g1) + [False] * len(g2))
    assert OT.tstat(X, mask)[0] == pytest.approx(expect, rel=1e-14, abs=1e-15)


def test_welch_matches_scipy():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(50, 13)) * rng.uniform(0.1, 10, size=(50, 1)) + rng.normal(size=(50, 1)) * 5
    mask = np.zeros(13, bool)
    mask[[0, 3, 4, 7, 11]] = True
    ref = stats.ttest_ind(X[:, mask], X[:, ~mask], axis=1, equal_var=False).statistic
    np.testing.assert_allclose(OT.tstat(X, mask), ref, rtol=1e-12, atol=1e-13)


def test_equal_sizes_equal_pooled_student():
    rng = np.random.default_rng(1)
    X = rng.normal(size=(40, 16))
    mask = np.zeros(16, bool)
    mask[rng.permutation(16)[:8]] = True
    pooled = stats.ttest_ind(X[:, mask], X[:, ~mask], axis=1, equal_var=True).statistic
    np.testing.assert_allclose(OT.tstat(X, mask), pooled, rtol=1e-12, atol=1e-13)


def test_explicit_loop_statistics_module():
    """Per-voxel recomputation with the standard library's mean/variance."""
    rng = np.random.default_rng(2)
    X = rng.normal(size=(7, 9))
    mask = np.array([1, 0, 1, 1, 0, 0, 1, 0, 0], bool)
    got = OT.tstat(X, mask)
    for k in range(7):
        a = [float(x) for x in X[k, mask]]
        b = [float(x) for x in X[k, ~mask]]
        den = (statistics.variance(a) / len(a) + statistics.variance(b) / len(b)) ** 0.5
        assert got[k] == pytest.approx((statistics.mean(a) - statistics.mean(b)) / den, rel=1e-13)


def test_complement_identity_affine_within_group():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(30, 12))
    mask = np.zeros(12, bool)
    mask[[1, 2, 5, 8, 9, 10]] = True
    t = OT.tstat(X, mask)
    np.testing.assert_allclose(OT.tstat(X, ~mask), -t, rtol=1e-13, atol=1e-14)
    # per-voxel affine map with positive / negative scale
    a = rng.uniform(0.5, 3, size=(30, 1)) * np.where(np.arange(30) % 2, 1, -1)[:, None]
    b = rng.normal(size=(30, 1)) * 100
    np.testing.assert_allclose(OT.tstat(a * X + b, mask), np.sign(a[:, 0]) * t, rtol=1e-9, atol=1e-10)
    # shuffling subjects inside each group changes nothing
    g1 = np.flatnonzero(mask)
    g2 = np.flatnonzero(~mask)
    perm = np.concatenate([rng.permutation(g1), rng.permutation(g2)])
    Xp = X.copy()
    Xp[:, np.concatenate([g1, g2])] = X[:, perm]
    np.testing.assert_allclose(OT.tstat(Xp, mask), t, rtol=1e-12, atol=1e-13)
    # identity labelling (first n1 columns = group 1) gives the observed map
    X2 = X[:, np.concatenate([g1, g2])]
    ident = np.zeros(12, bool)
    ident[:len(g1)] = True
    np.testing.assert_allclose(OT.tstat(X2, ident), t, rtol=1e-13, atol=1e-14)


def test_zero_spread_gives_zero():
    X = np.array([[3.0] * 6, [1.0, 1.0, 1.0, 2.0, 2.0, 2.0]])
    mask = np.array([1, 1, 1, 0, 0, 0], bool)
    t = OT.tstat(X, mask)
    assert t[0] == 0.0 and t[1] == 0.0


@pytest.mark.parametrize("n", [8, 12])
def test_bruteforce_all_labellings(n):
    """All C(n, n/2) labellings, t by explicit scalar loops; the max null is
    closed under complementation (multiset of max t == multiset of -min t)."""
    rng = np.random.default_rng(n)
    v = 6
    X = rng.normal(size=(v, n))
    combos = list(itertools.combinations(range(n), n // 2))
    labels = np.zeros((len(combos), n), np.uint8)
    for i, c in enumerate(combos):
        labels[i, list(c)] = 1
    m = OT.naive_maxnull(X, labels)
    mins = []
    for i, c in enumerate(combos):
        best = -np.inf
        worst = np.inf
        for k in range(v):
            a = [X[k, j] for j in c]
            b = [X[k, j] for j in range(n) if j not in c]
            ma = sum(a) / len(a)
            mb = sum(b) / len(b)
            va = sum((x - ma) ** 2 for x in a) / (len(a) - 1)
            vb = sum((x - mb) ** 2 for x in b) / (len(b) - 1)
            t = (ma - mb) / (va / len(a) + vb / len(b)) ** 0.5
            best = max(best, t)
            worst = min(worst, t)
        assert m[i] == pytest.approx(best, rel=1e-12)
        mins.append(worst)
    np.testing.assert_allclose(np.sort(m), np.sort(-np.array(mins)), rtol=1e-12)


def test_naive_abs_tail_and_tmatrix():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(100, 10))
    labels = np.zeros((20, 10), np.uint8)
    for i in range(20):
        labels[i, rng.permutation(10)[:5]] = 1
    T = OT.tmatrix(X, labels)
    np.testing.assert_allclose(OT.naive_maxnull(X, labels), T.max(axis=1))
    np.testing.assert_allclose(OT.naive_maxnull(X, labels, "abs"), np.abs(T).max(axis=1))
