"""GPU parity for the linear mean-difference statistic (the `stat` input of
Alg. 2) and for uneven (CSR) sampled sets in single-study recovery.

With stat = mean difference, T = X C has rank at most n - 1 (Sec. 3.2): with
U an orthonormal basis of the centred data, sigma = mu = 0 and at least n - 1
sampled voxels per column, RapidPT's recovery reproduces NaivePT's maxima up
to rounding.  That exact case is checked at the benchmark's shape (n = 100,
v = 250,000)."""
import numpy as np
import pytest

import rpt_synth as S
from gpu_util import announce, torch_cuda
from oracle import rapidpt as OR
from oracle import tstat as OT

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("prec", ["split_bf16", "fp32"])
def test_naive_meandiff_matches_oracle(prec):
    """NaivePT with the mean difference: every t map entry and every maximum
    against the FP64 oracle (split BF16 within 1e-4 of the data scale, FP32
    within 1e-5)."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce(f"naive meandiff {prec}")
    rng = np.random.default_rng(3)
    n, v, L = 24, 3001, 70
    X = (rng.normal(size=(v, n)) * 1.7 + 40.0).astype(np.float32)   # mean far above the spread
    labels = S.relabellings(L, n, n // 2, seed=4)
    m, T = rpt.naive_maxnull(_dev(torch, X), _dev(torch, labels), prec=prec, stat="meandiff", return_T=True)
    X64 = X.astype(np.float64)
    Tref = np.stack([OT.meandiff(X64, labels[i] == 1) for i in range(L)])
    tol = (1e-4 if prec == "split_bf16" else 1e-5) * max(1.0, float(np.abs(Tref).max()))
    np.testing.assert_allclose(T.cpu().numpy(), Tref, atol=tol, rtol=0)
    np.testing.assert_allclose(m.cpu().numpy(), Tref.max(axis=1), atol=tol, rtol=0)


def test_sampled_meandiff_and_unbalanced_rejected():
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    from paper_1703_01506_amd._lib import RPTError
    announce("sampled meandiff")
    rng = np.random.default_rng(5)
    n, v, L, k = 40, 5003, 33, 211
    X = rng.normal(size=(v, n)).astype(np.float32)
    labels = S.relabellings(L, n, n // 2, seed=6)
    om = S.omega_sets(L, v, k, seed=7)
    y = rpt.sampled_tstat(_dev(torch, X), _dev(torch, labels), _dev(torch, om), stat="meandiff").cpu().numpy()
    X64 = X.astype(np.float64)
    ref = np.stack([OT.meandiff(X64[om[i]], labels[i] == 1) for i in range(L)])
    np.testing.assert_allclose(y, ref, atol=1e-5, rtol=0)
    unb = S.relabellings(4, n, 15, seed=8)
    with pytest.raises(RPTError):
        rpt.naive_maxnull(_dev(torch, X), _dev(torch, unb), n1=15, prec="fp32", stat="meandiff")


def test_recover_exact_meandiff_full_size():
    """The exact special case at n = 100, v = 250,000, L = 2,000 recovered
    columns, 875 sampled voxels each: U = orthonormal basis of the centred
    data (r = n - 1 = 99), sigma = mu = 0.  Recovered maxima equal NaivePT's
    mean-difference maxima to rounding, within 2e-4 of the largest maximum
    (the least-squares fit reproduces each sampled column, whose values lie
    in span(U) exactly; the fit's split-BF16 Gram matrix keeps about 16 bits
    per term)."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce("recover exact meandiff v=250k")
    n, v, Lr, r = 100, 250_000, 2_000, 99
    k = S.omega_count(v, 3500)
    X = S.smoothed_volumes(n, v, seed=1703)
    labels = S.relabellings(Lr, n, n // 2, seed=1506)
    om = S.omega_sets(Lr, v, k, seed=43)
    Xd = _dev(torch, X)
    Xc = Xd.double() - Xd.double().mean(dim=1, keepdim=True)
    Q, _ = torch.linalg.qr(Xc[:, :r])         # the n - 1 first centred columns span all n
    U = Q.float().contiguous()
    sm = torch.zeros(2, dtype=torch.float32, device=Xd.device)
    got, info = rpt.recover_maxnull(Xd, _dev(torch, labels), U, sm, _dev(torch, om), seed=2017, stat="meandiff")
    ref = rpt.naive_maxnull(Xd, _dev(torch, labels), stat="meandiff")
    assert (info.cpu().numpy() == 0).all()
    got, ref = got.cpu().numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64)
    # the FP64 oracle's maxima of a few columns, recomputed one by one
    X64 = X.astype(np.float64)
    scale = float(np.abs(ref).max())
    for i in (0, 977, Lr - 1):
        assert abs(ref[i] - OT.meandiff(X64, labels[i] == 1).max()) <= 1e-4 * scale
    print(f"max |recovered - naive| {np.abs(got - ref).max():.3e} (scale {scale:.3f})", flush=True)
    np.testing.assert_allclose(got, ref, atol=2e-4 * scale, rtol=0)


def test_recover_csr_matches_dense_and_oracle():
    """rpt_recover_maxnull with CSR sampled sets: equal-length rows give the
    dense call's maxima bit for bit; uneven rows (30..260 voxels, r = 12)
    match the oracle's recovery column by column."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce("recover csr")
    rng = np.random.default_rng(9)
    n, v, L, r, seed = 20, 4001, 57, 12, 2017
    X, _ = S.iid_volumes(n, v, n // 2, signal_frac=0.02, shift=0.5, seed=21)
    X = X.astype(np.float32)
    labels = S.relabellings(L, n, n // 2, seed=22)
    U = np.linalg.qr(S.gaussian_matrix(v, r, seed=23))[0].astype(np.float32)
    sm = np.array([0.3, 0.05], dtype=np.float32)
    k = 150
    om = S.omega_sets(L, v, k, seed=24)
    dense, di = rpt.recover_maxnull(_dev(torch, X), _dev(torch, labels), _dev(torch, U), _dev(torch, sm),
                                    _dev(torch, om), seed)
    ptr = np.arange(L + 1, dtype=np.int64) * k
    csr, ci = rpt.recover_maxnull(_dev(torch, X), _dev(torch, labels), _dev(torch, U), _dev(torch, sm),
                                  _dev(torch, om.reshape(-1)), seed, omega_ptr=_dev(torch, ptr))
    assert torch.equal(dense, csr) and torch.equal(di, ci)
    sizes = rng.integers(30, 261, size=L)
    sets = [np.sort(rng.choice(v, s_, replace=False)).astype(np.int32) for s_ in sizes]
    ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    got, info = rpt.recover_maxnull(_dev(torch, X), _dev(torch, labels), _dev(torch, U), _dev(torch, sm),
                                    _dev(torch, np.concatenate(sets)), seed, omega_ptr=_dev(torch, ptr))
    assert (info.cpu().numpy() == 0).all()
    ref = OR.recover(X.astype(np.float64), labels, U.astype(np.float64), float(sm[0]), float(sm[1]), sets, seed)
    np.testing.assert_allclose(got.cpu().numpy(), ref, atol=5e-4, rtol=0)
