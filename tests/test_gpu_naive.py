"""GPU parity: NaivePT (Alg. 1) through the C ABI against the FP64 oracle."""
import numpy as np
import pytest

import rpt_synth as S
from gpu_util import announce, assert_t_close, torch_cuda
from oracle import tstat as OT

pytestmark = pytest.mark.gpu


def _run(torch, X, labels, n1, tail, prec, return_T=False):
    import paper_1703_01506_amd as rpt
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    Ld = torch.from_numpy(labels).cuda()
    out = rpt.naive_maxnull(Xd, Ld, n1=n1, tail=tail, prec=prec, return_T=return_T)
    torch.cuda.synchronize()
    if return_T:
        return out[0].cpu().numpy(), out[1].cpu().numpy()
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_naive_simulated_small(prec):
    """n = 20 (10/10), v = 10,000 i.i.d. N(0,1) with +0.5 on a seeded 2% of
    voxels in group 1, L = 1,000 relabellings."""
    torch = torch_cuda()
    announce(f"naive small prec={prec}")
    X, _ = S.iid_volumes(20, 10_000, 10, signal_frac=0.02, shift=0.5, seed=1703)
    labels = S.relabellings(1000, 20, 10, seed=1506)
    X32 = X.astype(np.float32)
    got = _run(torch, X32, labels, 10, "signed", prec)
    ref = OT.naive_maxnull(X32.astype(np.float64), labels)
    assert_t_close(got, ref, prec, "max")
    # deterministic (no atomics on this path)
    got2 = _run(torch, X32, labels, 10, "signed", prec)
    assert np.array_equal(got, got2)


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
@pytest.mark.parametrize("tail", ["signed", "abs"])
def test_naive_ragged_full_T(prec, tail):
    """Ragged sizes (v, L not multiples of the 32-wide tiles, n not a multiple
    of the K block), full T compared element by element."""
    torch = torch_cuda()
    announce(f"naive ragged prec={prec} tail={tail}")
    rng = np.random.default_rng(11)
    n, v, L = 36, 1007, 517
    X = (rng.normal(size=(v, n)) * rng.uniform(0.5, 2.0, size=(v, 1)) + rng.normal(size=(v, 1)) * 3).astype(np.float32)
    labels = S.relabellings(L, n, n // 2, seed=5)
    mx, T = _run(torch, X, labels, n // 2, tail, prec, return_T=True)
    Tref = OT.tmatrix(X.astype(np.float64), labels)
    assert_t_close(T, Tref, prec, "T")
    ref = np.abs(Tref).max(axis=1) if tail == "abs" else Tref.max(axis=1)
    assert_t_close(mx, ref, prec, "max")


def test_naive_unbalanced_fp32():
    torch = torch_cuda()
    announce("naive unbalanced fp32")
    rng = np.random.default_rng(12)
    n, n1, v, L = 30, 12, 2005, 100
    X = rng.normal(size=(v, n)).astype(np.float32)
    labels = S.relabellings(L, n, n1, seed=6)
    for tail in ("signed", "abs"):
        mx, T = _run(torch, X, labels, n1, tail, "fp32", return_T=True)
        Tref = OT.tmatrix(X.astype(np.float64), labels)
        assert_t_close(T, Tref, "fp32", "T")
        ref = np.abs(Tref).max(axis=1) if tail == "abs" else Tref.max(axis=1)
        assert_t_close(mx, ref, "fp32", "max")


@pytest.mark.parametrize("prec", ["fp32", "split_bf16"])
def test_naive_constant_voxels_and_large_offsets(prec):
    """Zero-spread voxels give t = 0; raw values with a large mean and tiny
    spread (grey-matter-like) keep full accuracy after the FP64 standardisation."""
    torch = torch_cuda()
    announce(f"naive degenerate prec={prec}")
    rng = np.random.default_rng(13)
    n, v, L = 24, 300, 64
    X = (1000.0 + 0.01 * rng.normal(size=(v, n))).astype(np.float32)
    X[[0, 17, 299]] = 3.25
    labels = S.relabellings(L, n, n // 2, seed=7)
    mx, T = _run(torch, X, labels, n // 2, "signed", prec, return_T=True)
    Tref = OT.tmatrix(X.astype(np.float64), labels)
    assert (T[:, [0, 17, 299]] == 0).all()
    assert_t_close(T, Tref, prec, "T")
    assert_t_close(mx, Tref.max(axis=1), prec, "max")


def test_naive_tiny_edge_cases():
    torch = torch_cuda()
    announce("naive tiny")
    rng = np.random.default_rng(14)
    for (n, v, L) in [(4, 1, 1), (4, 33, 3), (128, 40, 40)]:
        X = rng.normal(size=(v, n)).astype(np.float32)
        labels = S.relabellings(L, n, n // 2, seed=8)
        ref = OT.naive_maxnull(X.astype(np.float64), labels)
        for prec in ("fp32", "split_bf16"):
            assert_t_close(_run(torch, X, labels, n // 2, "signed", prec), ref, prec, f"max n={n} v={v}", m=n // 2)


@pytest.mark.parametrize("n", [18, 24, 30, 32, 100, 120, 122])
@pytest.mark.parametrize("tail", ["signed", "abs"])
def test_naive_split_max_tail_step(n, tail):
    """Max-only split-BF16 launch for every kind of last K step (balanced, so n
    is even): R = n mod 16 of 2..8 packs hi and lo of the last R subjects into
    one mixed block (n = 18, 24, 100, 120), R of 10..14 keeps two blocks
    (n = 30, 122), R = 0 has no partial step (n = 32); ragged voxel and
    relabelling tiles, maxima against the oracle's full T."""
    torch = torch_cuda()
    announce(f"naive split max n={n} tail={tail}")
    rng = np.random.default_rng(100 + n)
    v, L = 1531, 389
    X = (rng.normal(size=(v, n)) * rng.uniform(0.5, 2.0, size=(v, 1)) + rng.normal(size=(v, 1)) * 3).astype(np.float32)
    labels = S.relabellings(L, n, n // 2, seed=n + 7)
    Tref = OT.tmatrix(X.astype(np.float64), labels)
    ref = np.abs(Tref).max(axis=1) if tail == "abs" else Tref.max(axis=1)
    got = _run(torch, X, labels, n // 2, tail, "split_bf16")
    assert_t_close(got, ref, "split", f"max n={n}", m=n // 2)


@pytest.mark.parametrize("n", [36, 100])
def test_naive_labels_unaligned_view(n):
    """Labels passed as a row-offset view (its first byte n bytes into the
    allocation, not 16-byte aligned) take the bytewise staging path of the
    max-only kernel; the maxima must equal, bit for bit, those of an aligned
    copy, and both must match the oracle."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce(f"naive unaligned labels n={n}")
    rng = np.random.default_rng(300 + n)
    v, L = 1100, 700
    X = (rng.normal(size=(v, n)) * rng.uniform(0.5, 2.0, size=(v, 1))).astype(np.float32)
    labels = S.relabellings(L + 1, n, n // 2, seed=n + 3)
    Xd = torch.from_numpy(X).cuda()
    Lfull = torch.from_numpy(labels).cuda()
    view = Lfull[1:]
    assert view.data_ptr() % 16 != 0
    got_view = rpt.naive_maxnull(Xd, view).cpu().numpy()
    got_copy = rpt.naive_maxnull(Xd, view.clone()).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(got_view, got_copy)
    ref = OT.naive_maxnull(X.astype(np.float64), labels[1:])
    assert_t_close(got_view, ref, "split", f"max n={n}", m=n // 2)


@pytest.mark.parametrize("prec", ["split_bf16", "fp32"])
def test_naive_full_size_sampled(prec):
    """n = 100 (50/50), v = 250,000 smoothed (FWHM 3) volume, L = 10,000 in the
    benchmark's launch configuration; 12 relabellings spread over the range are
    recomputed by the oracle one by one."""
    torch = torch_cuda()
    announce(f"naive full-size prec={prec}")
    X = S.smoothed_volumes(100, 250_000, seed=1703)
    labels = S.relabellings(10_000, 100, 50, seed=1506)
    got = _run(torch, X, labels, 50, "signed", prec)
    idx = np.linspace(0, 9_999, 12).astype(int)
    X64 = X.astype(np.float64)
    ref = np.array([OT.tstat(X64, labels[i] == 1).max() for i in idx])
    assert_t_close(got[idx], ref, prec, "max")
    assert np.isfinite(got).all()


@pytest.mark.parametrize("n", [136, 200, 400, 512])
@pytest.mark.parametrize("tail", ["signed", "abs"])
def test_naive_wide_subjects(n, tail):
    """More than 128 subjects (the multi-study range 150-400 and the limit
    512): K steps staged in chunks of 8 with a ragged last chunk (n = 136 has
    9 steps), ragged voxel and relabelling tiles; full T element by element
    and the maxima, split BF16.  The FP32 path refuses these sizes."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce(f"naive wide n={n} tail={tail}")
    rng = np.random.default_rng(n)
    v, L = 2011, 261
    X = (rng.normal(size=(v, n)) * rng.uniform(0.5, 2.0, size=(v, 1)) + rng.normal(size=(v, 1)) * 3).astype(np.float32)
    labels = S.relabellings(L, n, n // 2, seed=n + 1)
    mx, T = _run(torch, X, labels, n // 2, tail, "split_bf16", return_T=True)
    Tref = OT.tmatrix(X.astype(np.float64), labels)
    assert_t_close(T, Tref, "split", "T")
    ref = np.abs(Tref).max(axis=1) if tail == "abs" else Tref.max(axis=1)
    assert_t_close(mx, ref, "split", "max")
    mx2 = _run(torch, X, labels, n // 2, tail, "split_bf16")  # max-only launch
    assert_t_close(mx2, ref, "split", "max (max-only)")
    with pytest.raises(RuntimeError):
        _run(torch, X, labels, n // 2, tail, "fp32")


def test_naive_wide_full_size_sampled():
    """n = 400 (200/200) on the 250,000-voxel smoothed volume, L = 2,000:
    10 relabellings recomputed by the oracle one by one."""
    torch = torch_cuda()
    announce("naive wide full-size n=400")
    X = S.smoothed_volumes(400, 250_000, seed=1703)
    labels = S.relabellings(2_000, 400, 200, seed=1506)
    got = _run(torch, X, labels, 200, "signed", "split_bf16")
    idx = np.linspace(0, 1_999, 10).astype(int)
    X64 = X.astype(np.float64)
    ref = np.array([OT.tstat(X64, labels[i] == 1).max() for i in idx])
    assert_t_close(got[idx], ref, "split", "max")
    assert np.isfinite(got).all()
