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


def assert_t_close(got, ref, prec: str, what: str = "t"):
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
    worst = int(np.argmax(d - bound)) if d.size else 0
    assert (d <= bound).all(), (f"{what}: {int((d > bound).sum())} of {d.size} outside tolerance; "
                                f"worst |d|={d[worst]:.3g} at ref={ref[fin][worst]:.6g}")
