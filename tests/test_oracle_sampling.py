"""Pins of oracle/sampling.py: inputs drawn from a seed (relabellings, sampled
sets, the start basis), checked against hand-worked shuffles, exact
uniformity over every word sequence of tiny cases, chi-square tests of the
Philox-driven draws and the definitions of their pieces."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import philox, sampling as S


def test_sample_count_hand_values():
    # ceil(eta v) with eta in ppm, exactly
    assert S.sample_count(250_000, 3500) == 875
    assert S.sample_count(1_000_000, 1) == 1
    assert S.sample_count(999_999, 1) == 1          # 0.999999 rounds up
    assert S.sample_count(1_000_001, 1) == 2        # 1.000001 rounds up
    assert S.sample_count(20_000, 10_000) == 200
    assert S.sample_count(5_000, 1_000_000) == 5_000
    assert S.sample_count(7, 0) == 0


def test_uniform_index_is_the_high_half_of_the_product():
    assert S.uniform_index(0, 10) == 0
    assert S.uniform_index(0xFFFFFFFF, 10) == 9
    assert S.uniform_index(0x80000000, 10) == 5     # 2^31 * 10 / 2^32
    assert S.uniform_index(0x40000000, 3) == 0      # 0.75 -> 0
    assert S.uniform_index(0x55555556, 3) == 1      # just above 1/3
    # every cell of [0, m) gets floor or ceil of 2^32 / m words
    m = 7
    edges = [math.ceil(c * 2 ** 32 / m) for c in range(m + 1)]
    for c in range(m):
        assert S.uniform_index(edges[c], m) == c and S.uniform_index(edges[c + 1] - 1, m) == c


def test_partial_shuffle_hand_case():
    # m = 4, k = 2: word 0xC0000000 (0.75) picks t = 0 + 3 -> swap a[0], a[3]:
    # [3, 1, 2, 0]; word 0 picks t = 1 + 0 -> a[1] stays: first two = [3, 1]
    assert S.partial_shuffle([0xC0000000, 0], 4, 2) == [3, 1]
    # second step reaching the displaced entry: t = 1 + floor(0.99 * 3) = 3 -> a[3] = 0
    assert S.partial_shuffle([0xC0000000, 0xFD70A3D7], 4, 2) == [3, 0]
    # t equal to j keeps the entry
    assert S.partial_shuffle([0, 0, 0], 5, 3) == [0, 1, 2]
    # a full shuffle is a permutation
    w = S.step_words(9, 1, 0, 0, 10)
    assert sorted(S.partial_shuffle(w, 10, 10)) == list(range(10))


def test_partial_shuffle_exactly_uniform_over_word_grids():
    """With each step's word taken on a grid that gives every index on
    [0, m - j) exactly once (x = ceil(c 2^32 / (m - j))), the k-step shuffle
    produces every ordered k-tuple of distinct values exactly once: the
    definition of a uniform draw without replacement."""
    for m, k in ((4, 2), (5, 3), (6, 2)):
        grids = [[math.ceil(c * 2 ** 32 / (m - j)) for c in range(m - j)] for j in range(k)]
        seen = {}
        for words in itertools.product(*grids):
            out = tuple(S.partial_shuffle(list(words), m, k))
            assert out == tuple(S.partial_shuffle_dense(list(words), m, k))
            seen[out] = seen.get(out, 0) + 1
        assert len(seen) == math.perm(m, k) and set(seen.values()) == {1}


def test_dictionary_shuffle_equals_dense_array():
    for seed, m, k in ((1, 50, 50), (2, 1000, 37), (3, 300, 299), (4, 17, 5)):
        w = S.step_words(seed, 1, 5, 2, k)
        assert S.partial_shuffle(w, m, k) == S.partial_shuffle_dense(w, m, k)


def test_step_words_follow_the_counter_layout():
    key = (0x12345678, 0x9)
    seed = (0x9 << 32) | 0x12345678
    w = S.step_words(seed, 1, 7, 3, 10)
    calls = philox.philox4x32_10((np.arange(3), 7, 1, 3), key)
    assert np.array_equal(w, calls.T.reshape(-1)[:10])


def test_relabellings_have_n1_ones_and_uniform_subsets():
    n, n1, L = 5, 2, 20_000
    lab = S.relabellings(11, 0, L, n, n1)
    assert lab.shape == (L, n) and lab.dtype == np.uint8
    assert np.all(lab.sum(1) == n1)
    codes = lab @ (1 << np.arange(n))
    counts = np.bincount(codes, minlength=1 << n)
    counts = counts[[c for c in range(1 << n) if bin(c).count("1") == n1]]
    assert len(counts) == 10
    assert stats.chisquare(counts).pvalue > 1e-3
    # rows are regenerated independently of the others
    assert np.array_equal(S.relabellings(11, 123, 2, n, n1), lab[123:125])


def test_sampled_sets_distinct_sorted_uniform():
    v, k, rows = 12, 3, 30_000
    om = S.sampled_sets(5, 0, 0, rows, v, k)
    assert om.shape == (rows, k) and om.dtype == np.int32
    assert np.all(np.diff(om, axis=1) > 0) and om.min() >= 0 and om.max() < v
    # each voxel equally likely (k / v) and each pair equally likely
    cnt = np.bincount(om.reshape(-1), minlength=v)
    assert stats.chisquare(cnt).pvalue > 1e-3
    pairs = np.bincount(om[:, 0] * v + om[:, 1], minlength=v * v).reshape(v, v)
    first_two = pairs[np.triu_indices(v, 1)]
    # P(first two sorted entries = (a, b)) = (v - 1 - b) / C(v, 3) for a < b
    a, b = np.triu_indices(v, 1)
    expect = (v - 1 - b) / math.comb(v, 3) * rows
    keep = expect > 0
    assert stats.chisquare(first_two[keep], expect[keep] * first_two[keep].sum() / expect[keep].sum()).pvalue > 1e-3
    # sets and streams are independent of each other
    assert not np.array_equal(S.sampled_sets(5, 1, 0, 5, v, k), om[:5])
    assert np.array_equal(S.sampled_sets(5, 0, 700, 3, v, k), om[700:703])


def test_sampled_set_at_benchmark_shape():
    om = S.sampled_set(2017, 0, 9999, 250_000, 875)
    assert om.shape == (875,) and len(np.unique(om)) == 875
    assert np.all(np.diff(om) > 0) and om[0] >= 0 and om[-1] < 250_000
    full = S.sampled_set(3, 1, 0, 300, 300)
    assert np.array_equal(full, np.arange(300))


def test_gaussian_start_definition_and_moments():
    G = S.gaussian_start(77, 2000, 9)
    assert G.shape == (2000, 9)
    # entry (q, c) is the noise draw of column c at voxel q on stream 3
    for q, c in ((0, 0), (5, 3), (1999, 8), (17, 4)):
        assert G[q, c] == philox.normals(77, 3, c, np.array([q]))[0]
    z = G.reshape(-1)
    assert abs(z.mean()) < 0.05 and abs(z.std() - 1.0) < 0.03
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # the columns are not copies of one another
    assert np.max(np.abs(np.corrcoef(G.T) - np.eye(9))) < 0.1
