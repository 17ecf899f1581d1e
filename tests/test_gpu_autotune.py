"""GPU: the autotuner picks one of its candidate chunk counts, and a tuned
call returns exactly what the untuned call returned (column maxima are exact
maxima of the same values, whatever the chunking)."""
import numpy as np
import pytest

import rpt_synth as S
from gpu_util import announce, torch_cuda
from oracle import rapidpt as OR

pytestmark = pytest.mark.gpu


def _d(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_autotune_naive_keeps_results():
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce("autotune naive")
    rpt.autotune_clear()
    n, v, L = 100, 50_003, 2_000
    X = S.smoothed_volumes(n, v, seed=5)
    labels = S.relabellings(L, n, n // 2, seed=6)
    Xd, Ld = _d(torch, X), _d(torch, labels)
    before = rpt.naive_maxnull(Xd, Ld).cpu().numpy()
    chosen = rpt.autotune_naive(Xd, Ld, reps=2)
    assert chosen >= 8 and chosen % 8 == 0 and rpt.autotune_count() == 1
    after = rpt.naive_maxnull(Xd, Ld).cpu().numpy()
    np.testing.assert_array_equal(after, before)
    rpt.autotune_clear()


def test_autotune_recover_keeps_results():
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce("autotune recover")
    rpt.autotune_clear()
    n, v, L, r, k = 40, 30_011, 600, 24, 120
    rng = np.random.default_rng(3)
    X = rng.normal(size=(v, n)).astype(np.float32)
    labels = S.relabellings(L, n, n // 2, seed=4)
    U = OR.orthonormalize(rng.normal(size=(v, r))).astype(np.float32)
    om = S.omega_sets(L, v, k, seed=5)
    sm = np.array([0.9, 0.1], dtype=np.float32)
    args = (_d(torch, X), _d(torch, labels), _d(torch, U), _d(torch, sm), _d(torch, om), 2017)
    before, _ = rpt.recover_maxnull(*args, col0=300)
    before = before.cpu().numpy()
    chosen = rpt.autotune_recover(v, r, L, reps=1)
    assert chosen >= 8 and chosen % 8 == 0 and rpt.autotune_count() == 1
    after, _ = rpt.recover_maxnull(*args, col0=300)
    np.testing.assert_array_equal(after.cpu().numpy(), before)
    rpt.autotune_clear()


def test_autotune_naive_t_writing_keeps_results():
    """The T-writing launch is tuned on its own (separate table entry); T and
    the maxima stay bit for bit the same."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce("autotune naive, T-writing")
    rpt.autotune_clear()
    n, v, L = 100, 30_011, 300
    X = S.smoothed_volumes(n, v, seed=7)
    labels = S.relabellings(L, n, n // 2, seed=8)
    Xd, Ld = _d(torch, X), _d(torch, labels)
    m0, T0 = rpt.naive_maxnull(Xd, Ld, return_T=True)
    m0, T0 = m0.cpu().numpy(), T0.cpu().numpy()
    scratch = torch.empty((L, v), dtype=torch.float32, device="cuda")
    chosen = rpt.autotune_naive(Xd, Ld, reps=2, T=scratch)
    assert chosen >= 8 and chosen % 8 == 0 and rpt.autotune_count() == 1
    m1, T1 = rpt.naive_maxnull(Xd, Ld, return_T=True)
    np.testing.assert_array_equal(m1.cpu().numpy(), m0)
    np.testing.assert_array_equal(T1.cpu().numpy(), T0)
    rpt.autotune_clear()
