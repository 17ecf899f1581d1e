"""Pins for the accuracy measures (Sec. 5.5)."""
import numpy as np
import pytest

from conftest import golden_path
from oracle import metrics as M


def _risk_rows():
    rows = []
    for line in open(golden_path("resampling_risk.txt")):
        if line.startswith("#") or not line.strip():
            continue
        a, b, r = [p.strip() for p in line.split("|")]
        rows.append((int(a), int(b), float(r)))
    return rows


@pytest.mark.parametrize("v1,v2,printed", _risk_rows())
def test_resampling_risk_reproduces_printed_values(v1, v2, printed):
    vc = min(v1, v2)  # nested rejection sets
    assert round(100 * M.resampling_risk(v1, v2, vc), 2) == printed


def test_risk_disjoint_and_equal():
    assert M.resampling_risk(10, 10, 10) == 0.0
    assert M.resampling_risk(10, 5, 0) == 1.0


def test_kl_self_zero_and_positive():
    rng = np.random.default_rng(0)
    a = rng.normal(size=5000)
    assert M.kl_divergence(a, a) == 0.0
    assert M.kl_divergence(a, a + 0.5) > 0.05


def test_kl_hand_value_fixes_direction_binning_and_pseudocount():
    """3 equal-width bins over the common range [0, 3] (edges 0, 1, 2, 3; the
    last bin closed).  ref = (0, 0.5, 1, 3): counts (2, 1, 1); test = (2.1,
    2.9, 3, 3): counts (0, 0, 4).  With 0.5 added per bin the normalised masses
    are p = (2.5, 1.5, 1.5)/5.5 and q = (0.5, 0.5, 4.5)/5.5, and
    D_KL(p || q) = sum p log(p / q)."""
    ref = [0.0, 0.5, 1.0, 3.0]
    test = [2.1, 2.9, 3.0, 3.0]
    hand = (2.5 / 5.5) * np.log(2.5 / 0.5) + (1.5 / 5.5) * np.log(1.5 / 0.5) + (1.5 / 5.5) * np.log(1.5 / 4.5)
    assert M.kl_divergence(ref, test, bins=3) == pytest.approx(hand, rel=1e-14)
    assert hand == pytest.approx(0.73156, abs=1e-5)
    back = (0.5 / 5.5) * np.log(0.5 / 2.5) + (0.5 / 5.5) * np.log(0.5 / 1.5) + (4.5 / 5.5) * np.log(4.5 / 1.5)
    assert M.kl_divergence(test, ref, bins=3) == pytest.approx(back, rel=1e-14)
    assert abs(back - hand) > 0.05   # the direction matters


def test_threshold_order_statistic():
    m = np.arange(1, 101, dtype=float)[::-1]  # 100 .. 1
    # alpha = 0.05, L = 100: m_(100 - 5) = 95
    assert M.threshold(m, 0.05) == 95.0
    assert M.threshold(m, 0.0) == 100.0
    p = M.corrected_pvalue(m, np.array([95.0, 95.5, 100.0, 0.0]))
    np.testing.assert_allclose(p, [0.06, 0.05, 0.01, 1.0])
    rej = M.rejected(m, np.array([95.0, 95.5, 101.0]), 0.05)
    assert list(rej) == [False, True, True]


def test_bench_kl_matches_the_oracle_definition():
    """The benchmark's own KL of two max nulls (it may not call the oracle)
    follows the same binning as the oracle's."""
    import importlib.util
    import os
    from conftest import ROOT
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    rng = np.random.default_rng(3)
    a = rng.gumbel(size=5000) * 0.3 + 4.0
    b = a + rng.normal(size=5000) * 0.05
    assert abs(bench.kl_max_nulls(a, b) - M.kl_divergence(a, b)) <= 1e-12
    assert bench.kl_max_nulls(a, a) == 0.0
