"""Helpers for the GPU parity tests: device selection and tolerances."""
import sys

import numpy as np
import pytest

TOL_T_FP32_REL = 1e-5      # |dt| <= 1e-5 * max(|t|, 1)
TOL_T_SPLIT_ABS = 1e-4     # |dt| <= 1e-4


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1703_01506_amd  # noqa: F401  (loads librpt.so, fails loudly if absent)
    return torch


def announce(msg: str):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def amplification(t, m):
    """Sensitivity of the balanced t to its group contrast relative to t = 0:
    t = c u / sqrt(1 - 2u^2/m) gives dt/du proportional to
    (1 + t^2 / (2(m-1)))^(3/2).  Equal to 1 at t = 0 and below 1.5 for
    |t| <= 5 at m = 50; large only for tiny groups with extreme t."""
    return (1.0 + np.asarray(t, dtype=np.float64) ** 2 / (2.0 * (m - 1))) ** 1.5


def assert_t_close(got, ref, prec: str, what: str = "t", m: int | None = None):
    """t within the stated bars: FP32 |dt| <= 1e-5 max(|t|, 1), split-BF16
    |dt| <= 1e-4; with m given (balanced group size) both bars are scaled by
    the statistic's own amplification of input rounding (see amplification)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin), f"{what}: non-finite pattern differs"
    d = np.abs(got[fin] - ref[fin])
    if prec == "fp32":
        bound = TOL_T_FP32_REL * np.maximum(np.abs(ref[fin]), 1.0)
    else:
        bound = np.full_like(d, TOL_T_SPLIT_ABS)
    if m is not None:
        bound = bound * amplification(ref[fin], m)
    worst = int(np.argmax(d - bound)) if d.size else 0
    assert (d <= bound).all(), (f"{what}: {int((d > bound).sum())} of {d.size} outside tolerance; "
                                f"worst |d|={d[worst]:.3g} at ref={ref[fin][worst]:.6g}")
