"""Seeded synthetic inputs for the RapidPT permutation-testing path.

This module produces the *inputs* of the method and nothing else: data
volumes, group relabellings, sub-sampling index sets and raw Gaussian
matrices.  It contains none of the method's arithmetic (no t statistic, no
least squares, no subspace update, no maximum).  Both the HIP library's
tests/benchmarks and the CPU oracle draw their inputs from here, so the two
sides see identical relabellings and identical sampled voxel sets.

Random draws use numpy's PCG64 generator seeded from a list of integers
(seed, purpose-tag, index), so every array is reproducible on any machine.

Workload shapes follow the paper's experimental set-up: balanced two-group
designs (Table 1: n = 50, 100, 200, 400), per-column sub-sampling rate
eta (Table 3, e.g. 0.35%), training columns l and permutation counts L
(Tables 2 and 4), and the simulated data of Sec. 5.1 (i.i.d. N(0,1) voxels,
a planted group difference on a fraction of voxels).  Smoothed Gaussian
fields stand in for the VBM grey-matter maps of Sec. 5.3, which are not
available.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "ball_voxels",
    "smoothed_volumes",
    "iid_volumes",
    "relabellings",
    "omega_sets",
    "omega_count",
    "gaussian_matrix",
    "study_tuples",
]

# purpose tags keep the streams of different input kinds independent
_TAG_DATA, _TAG_SIGNAL, _TAG_LABELS, _TAG_OMEGA, _TAG_GAUSS, _TAG_STUDY = 11, 12, 13, 14, 15, 16


def _rng(seed: int, tag: int, idx: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed), int(tag), int(idx)]))


# ----------------------------------------------------------------------------
# volumes
# ----------------------------------------------------------------------------
def ball_voxels(v: int):
    """Grid side g and the flat indices (C order, g^3 grid) of the v voxels
    nearest the grid centre.

    The ball radius is R = (3v / 4 pi)^(1/3); the grid side is ceil(2R) + 1 so
    the ball always fits.  Voxels are ranked by squared distance to the centre
    ((g-1)/2 on each axis) with a stable tie-break on the linear index, and
    the first v are kept.
    """
    v = int(v)
    if v <= 0:
        raise ValueError("v must be positive")
    R = (3.0 * v / (4.0 * math.pi)) ** (1.0 / 3.0)
    g = int(math.ceil(2.0 * R)) + 1
    c = (g - 1) / 2.0
    ax = (np.arange(g, dtype=np.float64) - c) ** 2
    d2 = (ax[:, None, None] + ax[None, :, None] + ax[None, None, :]).ravel()
    order = np.argsort(d2, kind="stable")
    return g, np.sort(order[:v])


def _gauss_kernel(fwhm: float):
    sig = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    rad = int(math.floor(4.0 * sig))
    x = np.arange(-rad, rad + 1, dtype=np.float64)
    k = np.exp(-0.5 * (x / sig) ** 2)
    return k / k.sum(), rad


def smoothed_volumes(n: int, v: int, fwhm: float = 3.0, seed: int = 1703,
                     dtype=np.float32) -> np.ndarray:
    """X (v x n): each subject is an independent N(0,1) field on the padded
    grid, smoothed separably with a Gaussian of the given FWHM (in voxels,
    truncated at 4 sigma), cropped to g^3 and restricted to the ball of
    `ball_voxels(v)`.  Rows are voxels, columns are subjects."""
    from scipy.ndimage import convolve1d

    g, idx = ball_voxels(v)
    k, rad = _gauss_kernel(fwhm)
    gp = g + 2 * rad
    X = np.empty((v, n), dtype=dtype)
    for j in range(n):
        f = _rng(seed, _TAG_DATA, j).standard_normal((gp, gp, gp))
        for ax in range(3):
            f = convolve1d(f, k, axis=ax, mode="constant")
        f = f[rad:rad + g, rad:rad + g, rad:rad + g]
        X[:, j] = f.ravel()[idx].astype(dtype)
    return X


def iid_volumes(n: int, v: int, n1: int, signal_frac: float = 0.0,
                shift: float = 0.0, seed: int = 1703, dtype=np.float64,
                signal_group: int = 1):
    """Simulated data of the kind of Sec. 5.1 and 5.2 (Simulation Data I and
    II): X (v x n) with i.i.d. N(0,1) entries; the columns of one group (group
    1 = the first n1 columns, group 2 = the rest) get +shift, i.e. N(shift, 1),
    on a seeded subset of round(signal_frac * v) voxels.
    Returns (X, signal_voxel_indices)."""
    if signal_group not in (1, 2):
        raise ValueError("signal_group is 1 or 2")
    X = _rng(seed, _TAG_DATA).standard_normal((v, n))
    ns = int(round(signal_frac * v))
    sig = np.sort(_rng(seed, _TAG_SIGNAL).choice(v, size=ns, replace=False)) if ns else np.zeros(0, np.int64)
    if ns:
        cols = np.arange(n1) if signal_group == 1 else np.arange(n1, n)
        X[np.ix_(sig, cols)] += shift
    return X.astype(dtype), sig


# ----------------------------------------------------------------------------
# relabellings and sub-sampling sets
# ----------------------------------------------------------------------------
def relabellings(L: int, n: int, n1: int, seed: int = 1506) -> np.ndarray:
    """L x n uint8 group-membership rows: row i marks the first n1 entries of
    an independent uniformly random permutation of 1..n as group 1 (the
    relabelling step of Alg. 1 and Alg. 2).  Draws are independent, so
    repeats are possible; the identity labelling is not forced in."""
    if not (1 <= n1 <= n - 1):
        raise ValueError("need 1 <= n1 <= n-1")
    out = np.zeros((L, n), dtype=np.uint8)
    block = 4096
    for b0 in range(0, L, block):
        b1 = min(L, b0 + block)
        keys = _rng(seed, _TAG_LABELS, b0 // block).random((b1 - b0, n))
        sel = np.argsort(keys, axis=1, kind="stable")[:, :n1]
        np.put_along_axis(out[b0:b1], sel, 1, axis=1)
    return out


def omega_count(v: int, eta_ppm: int) -> int:
    """ceil(eta * v) with eta given in parts per million, in integer arithmetic."""
    return int((int(v) * int(eta_ppm) + 999_999) // 1_000_000)


def omega_sets(rows: int, v: int, k: int, seed: int = 2017, tag_idx: int = 0) -> np.ndarray:
    """rows x k int32: each row holds k distinct voxel indices drawn uniformly
    without replacement from 0..v-1, sorted ascending (one sampled set per
    column of T, Alg. 2)."""
    if k > v:
        raise ValueError("k > v")
    rng = _rng(seed, _TAG_OMEGA, tag_idx)
    out = np.empty((rows, k), dtype=np.int32)
    for i in range(rows):
        out[i] = np.sort(rng.choice(v, size=k, replace=False))
    return out


def gaussian_matrix(rows: int, cols: int, seed: int = 3, dtype=np.float64) -> np.ndarray:
    """rows x cols matrix of i.i.d. N(0,1) draws (the random matrix that the
    'Rand. Orth.' initialisation of Alg. 2 orthonormalises)."""
    return _rng(seed, _TAG_GAUSS).standard_normal((rows, cols)).astype(dtype)


def study_tuples(count: int = 16, seed: int = 3, eta_ppm: int = 3500,
                 ns=(30, 50, 100, 150, 200, 300, 400),
                 vs=(50_000, 150_000, 250_000, 500_000),
                 Ls=(5_000, 10_000, 50_000)):
    """`count` (n, v, L) study shapes drawn uniformly from the given sets,
    rejecting shapes whose sampled set is smaller than the rank r = n."""
    rng = _rng(seed, _TAG_STUDY)
    out = []
    while len(out) < count:
        n = int(rng.choice(ns)); v = int(rng.choice(vs)); L = int(rng.choice(Ls))
        if omega_count(v, eta_ppm) < n:
            continue
        out.append((n, v, L))
    return out
