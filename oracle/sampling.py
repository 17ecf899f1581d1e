"""Oracle: inputs of Alg. 1 and Alg. 2 drawn from a seed.  TEST INFRASTRUCTURE.

Alg. 1 and Alg. 2 draw L relabellings of the n subjects (Permute[1, n], the
first n1 of the permuted order form group 1; Sec. 2.1) and, for every column
that RapidPT samples, a set Omega of |Omega| = ceil(eta v) distinct voxels
drawn uniformly without replacement (Sec. 4.1, 4.2); "Rand. Orth." starts
the tracking from an orthonormalised Gaussian matrix.  The paper names no
generator.  Read here as counter-based draws, so that any subset of rows can
be regenerated without the others:

* Words: Philox4x32-10 (``philox.philox4x32_10``) with key = (seed mod 2^32,
  seed >> 32) and counter (j >> 2, row, stream, set); step j of a row takes
  word j & 3.  Streams: 0 relabellings, 1 sampled sets, 3 the start basis
  (2 and 4 are the recovery and training noise of ``philox``).
* An index uniform on [0, m) from a 32-bit word x is floor(x m / 2^32) (the
  high half of the 64-bit product; bias at most m / 2^32 per value, below
  6e-5 at m = 250,000).
* Partial Fisher-Yates (Fisher & Yates 1938, in Durstenfeld's in-place form):
  for j = 0 .. k-1 draw t uniform on [j, m) and swap a[j] with a[t]; a[0..k)
  is then a uniform k-subset of 0..m-1 in uniform order.  ``partial_shuffle``.
* Relabelling i (row i, set 0): k = n1 steps over the n subjects; the chosen
  subjects form group 1.  ``relabelling``.
* Sampled set (row i, set s): k steps over the v voxels, the chosen voxels in
  ascending order.  Only displaced entries of the virtual array 0..v-1 are
  stored (a dictionary), which gives the same result as the dense array.
  ``sampled_set``.  In Alg. 2 end to end, column c of h^L (training columns
  0..l-1, then the recovered ones) has row c; the sets of the sigma/mu pass and
  of recovery are set 0 and tracking pass p uses set 1 + p.
* |Omega| = ceil(eta v) with eta in parts per million, in integer arithmetic:
  (eta_ppm v + 10^6 - 1) div 10^6.  ``sample_count``.
* Start basis: entry (q, c) of the v x r Gaussian matrix is the noise draw
  z(seed, stream 3, column c, voxel q) of ``philox.normals``.
  ``gaussian_start``.

Pins (tests/test_oracle_sampling.py): a hand-worked shuffle from given words;
exact uniformity of the partial shuffle over every word sequence of a tiny
case (with words restricted to a grid that makes each draw exactly uniform);
a chi-square test of relabelling subsets and of sampled sets drawn through
Philox; the dictionary form against the dense array; sizes, ranges,
distinctness and order; the sample count on hand cases; the start basis
against ``philox.normals`` moments and its definition at hand indices.
"""
from __future__ import annotations

import numpy as np

from . import philox

STREAM_LABELS = 0
STREAM_OMEGA = 1
STREAM_START = 3


def sample_count(v: int, eta_ppm: int) -> int:
    """ceil(eta v) for eta = eta_ppm / 10^6, exactly."""
    return (int(eta_ppm) * int(v) + 999_999) // 1_000_000


def uniform_index(x: int, m: int) -> int:
    """floor(x m / 2^32) for a 32-bit word x: an index on [0, m)."""
    return (int(x) * int(m)) >> 32


def step_words(seed: int, stream: int, row: int, set_id: int, steps: int) -> np.ndarray:
    """The 32-bit words of steps 0..steps-1 of one row: word j & 3 of the call
    with counter (j >> 2, row, stream, set_id)."""
    if steps <= 0:
        return np.zeros(0, dtype=np.uint32)
    key = (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    q = np.arange((steps + 3) // 4, dtype=np.uint64)
    w = philox.philox4x32_10((q, np.uint64(row), np.uint64(stream), np.uint64(set_id)), key)  # (4, calls)
    return w.T.reshape(-1)[:steps]


def partial_shuffle(words, m: int, k: int) -> list[int]:
    """First k entries of the partial Fisher-Yates shuffle of 0..m-1 driven by
    the given words (one per step), as a list in draw order."""
    displaced: dict[int, int] = {}
    out = []
    for j in range(k):
        t = j + uniform_index(words[j], m - j)
        at_t = displaced.get(t, t)
        at_j = displaced.get(j, j)
        out.append(at_t)
        displaced[t] = at_j  # position j is never read again
    return out


def partial_shuffle_dense(words, m: int, k: int) -> list[int]:
    """The same shuffle on an explicit array (for small m)."""
    a = list(range(m))
    for j in range(k):
        t = j + uniform_index(words[j], m - j)
        a[j], a[t] = a[t], a[j]
    return a[:k]


def relabelling(seed: int, i: int, n: int, n1: int) -> np.ndarray:
    """Relabelling i: n 0/1 entries, 1 for the n1 subjects of group 1."""
    words = step_words(seed, STREAM_LABELS, i, 0, n1)
    g = np.zeros(n, dtype=np.uint8)
    g[partial_shuffle(words, n, n1)] = 1
    return g


def relabellings(seed: int, row0: int, L: int, n: int, n1: int) -> np.ndarray:
    """Rows row0 .. row0 + L - 1 as an L x n uint8 matrix."""
    return np.stack([relabelling(seed, row0 + i, n, n1) for i in range(L)]) if L else \
        np.zeros((0, n), dtype=np.uint8)


def sampled_set(seed: int, set_id: int, i: int, v: int, k: int) -> np.ndarray:
    """Sampled set of row i in set set_id: k distinct voxels, ascending."""
    words = step_words(seed, STREAM_OMEGA, i, set_id, k)
    return np.sort(np.asarray(partial_shuffle(words, v, k), dtype=np.int64)).astype(np.int32)


def sampled_sets(seed: int, set_id: int, row0: int, rows: int, v: int, k: int) -> np.ndarray:
    """Rows row0 .. row0 + rows - 1 of set set_id as a rows x k int32 matrix."""
    return np.stack([sampled_set(seed, set_id, row0 + i, v, k) for i in range(rows)]) if rows else \
        np.zeros((0, k), dtype=np.int32)


def gaussian_start(seed: int, v: int, r: int) -> np.ndarray:
    """The v x r Gaussian matrix that Rand. Orth. orthonormalises (FP64)."""
    q = np.arange(v, dtype=np.int64)
    return np.stack([philox.normals(seed, STREAM_START, c, q) for c in range(r)], axis=1)
