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
