"""Oracle: accuracy measures of Sec. 5.5.  TEST INFRASTRUCTURE.

* KL divergence between a reference max null and an approximation.  The paper
  does not fix the binning; we read it as D_KL(P_ref || Q_test) over B equal
  width bins spanning the common range of both samples, with 0.5 added to
  every bin count before normalising (B = 50 unless stated).
* FWER threshold at level alpha: the ascending order statistic
  m_(L - floor(alpha L)) (1-based) of the L maxima.
* Corrected p-value of a statistic t: the fraction of maxima >= t
  (Sec. 2: the fraction of the max null at least as extreme).
* Resampling risk, Eq. 4: ((v1 - vc)/v1 + (v2 - vc)/v2) / 2, with v1, v2 the
  voxel counts rejected under each max null and vc their intersection.

Pins (tests/test_oracle_metrics.py): Eq. 4 reproduces the paper's printed
risks (8.45% at n = 200 and 1.85% at n = 400, Sec. 7.1.3) from its printed
rejection counts; KL(P || P) = 0; order statistics on hand lists.
"""
from __future__ import annotations

import math

import numpy as np


def kl_divergence(ref, test, bins: int = 50, pseudocount: float = 0.5) -> float:
    ref = np.asarray(ref, dtype=np.float64)
    test = np.asarray(test, dtype=np.float64)
    lo = min(ref.min(), test.min())
    hi = max(ref.max(), test.max())
    if hi <= lo:
        return 0.0
    edges = np.linspace(lo, hi, bins + 1)
    p = np.histogram(ref, edges)[0] + pseudocount
    q = np.histogram(test, edges)[0] + pseudocount
    p = p / p.sum()
    q = q / q.sum()
    return float(np.sum(p * np.log(p / q)))


def threshold(maxima, alpha: float = 0.05) -> float:
    m = np.sort(np.asarray(maxima, dtype=np.float64))
    L = m.size
    return float(m[L - int(math.floor(alpha * L)) - 1])


def corrected_pvalue(maxima, t) -> np.ndarray:
    m = np.sort(np.asarray(maxima, dtype=np.float64))
    t = np.asarray(t, dtype=np.float64)
    return (m.size - np.searchsorted(m, t, side="left")) / m.size


def rejected(maxima, tmap, alpha: float = 0.05) -> np.ndarray:
    """Voxels whose corrected p-value is <= alpha."""
    return corrected_pvalue(maxima, tmap) <= alpha


def resampling_risk(v1: int, v2: int, vc: int) -> float:
    parts = []
    for vi in (v1, v2):
        parts.append(0.0 if vi == 0 else (vi - vc) / vi)
    return 0.5 * (parts[0] + parts[1])
