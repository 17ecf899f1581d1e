"""Pins for the oracle's counter-based noise generator."""
import numpy as np
import pytest
from scipy import stats

from conftest import golden_path
from oracle import philox as PH


def _kat():
    out = []
    for line in open(golden_path("philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out.append((tuple(w[0:4]), tuple(w[4:6]), tuple(w[6:10])))
    return out


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_published_known_answers(ctr, key, expect):
    got = PH.philox4x32_10(ctr, key)
    assert tuple(int(x) for x in got) == expect


def test_vectorised_matches_scalar():
    ks = np.arange(0, 4000, 7)
    z = PH.normals(123456789012345, PH.STREAM_RECOVERY, 17, ks)
    for j, k in enumerate(ks[:40]):
        assert z[j] == PH.normals(123456789012345, PH.STREAM_RECOVERY, 17, np.array([k]))[0]


def test_layout_four_columns_per_call():
    """One Philox call at counter (k, i >> 2, stream, study) feeds columns
    4q..4q+3 at voxel k, as cos/sin pairs of words (0,1) and (2,3)."""
    seed, k, q = 99, 12345, 7
    w = PH.philox4x32_10((k, q, PH.STREAM_RECOVERY, 0), (seed, 0))
    u = PH.uniform_from_word(w)
    r1, r2 = np.sqrt(-2 * np.log(u[0])), np.sqrt(-2 * np.log(u[2]))
    expect = [r1 * np.cos(2 * np.pi * u[1]), r1 * np.sin(2 * np.pi * u[1]),
              r2 * np.cos(2 * np.pi * u[3]), r2 * np.sin(2 * np.pi * u[3])]
    got = [PH.normals(seed, PH.STREAM_RECOVERY, 4 * q + j, np.array([k]))[0] for j in range(4)]
    np.testing.assert_allclose(got, expect, rtol=1e-15)


def test_uniform_map_range():
    u = PH.uniform_from_word(np.array([0, 255, 256, 0xFFFFFFFF], dtype=np.uint64))
    assert u[0] == 0.5 * 2.0 ** -24 and u[1] == u[0]
    assert u[2] == 1.5 * 2.0 ** -24
    assert u[3] == 1.0 - 0.5 * 2.0 ** -24
    assert PH.Z_BOUND == pytest.approx(np.sqrt(50 * np.log(2.0)))


def test_normals_distribution():
    z = PH.normals(2017, PH.STREAM_RECOVERY, 3, np.arange(200_000))
    assert abs(z.mean()) < 0.01
    assert abs(z.std() - 1.0) < 0.01
    assert np.abs(z).max() <= PH.Z_BOUND
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # different columns / streams are different draws
    z2 = PH.normals(2017, PH.STREAM_RECOVERY, 4, np.arange(1000))
    z3 = PH.normals(2017, PH.STREAM_TRAINING, 3, np.arange(1000))
    assert not np.allclose(z[:1000], z2) and not np.allclose(z[:1000], z3)
    assert abs(np.corrcoef(z[:1000], z2)[0, 1]) < 0.1
