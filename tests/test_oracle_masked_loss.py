"""Pins for the masked completion loss gradient (Eq. 1)."""
import numpy as np

from oracle import masked_loss as ML


def _problem(seed=0, v=40, r=5, B=6):
    rng = np.random.default_rng(seed)
    U = rng.normal(size=(v, r))
    W = rng.normal(size=(r, B))
    sizes = rng.integers(3, 12, size=B)
    ptr = np.concatenate([[0], np.cumsum(sizes)])
    idx = np.concatenate([np.sort(rng.choice(v, s, replace=False)) for s in sizes]).astype(np.int64)
    t = rng.normal(size=ptr[-1])
    return U, W, ptr, idx, t


def test_gradient_vs_central_differences():
    U, W, ptr, idx, t = _problem()
    dU, dW = ML.grad(U, W, ptr, idx, t)
    h = 1e-3
    for (A, dA) in ((U, dU), (W, dW)):
        num = np.zeros_like(A)
        for pos in np.ndindex(A.shape):
            old = A[pos]
            A[pos] = old + h
            fp = ML.loss(U, W, ptr, idx, t)
            A[pos] = old - h
            fm = ML.loss(U, W, ptr, idx, t)
            A[pos] = old
            num[pos] = (fp - fm) / (2 * h)
        # quadratic in each coordinate: central differences are exact up to rounding
        np.testing.assert_allclose(dA, num, rtol=1e-8, atol=1e-9)


def test_dense_mask_formulation():
    U, W, ptr, idx, t = _problem(1)
    v, B = U.shape[0], W.shape[1]
    Tfull = np.zeros((v, B))
    mask = np.zeros((v, B))
    for b in range(B):
        Tfull[idx[ptr[b]:ptr[b + 1]], b] = t[ptr[b]:ptr[b + 1]]
        mask[idx[ptr[b]:ptr[b + 1]], b] = 1
    E = mask * (Tfull - U @ W)
    assert np.isclose(ML.loss(U, W, ptr, idx, t), 0.5 * np.sum(E ** 2))
    dU, dW = ML.grad(U, W, ptr, idx, t)
    np.testing.assert_allclose(dU, -E @ W.T, atol=1e-12)
    np.testing.assert_allclose(dW, -U.T @ E, atol=1e-12)


def test_grad_rows_matches_full_gradient():
    """The row-restricted gradient is the same sums as the full one."""
    U, W, ptr, idx, t = _problem(2, v=60, r=4, B=9)
    dU, dW = ML.grad(U, W, ptr, idx, t)
    rows = np.array([0, 3, int(idx[5]), int(idx[-1]), 59])
    dUr, dW2 = ML.grad_rows(U, W, ptr, idx, t, rows)
    np.testing.assert_allclose(dUr, dU[rows], atol=1e-12)
    np.testing.assert_allclose(dW2, dW, atol=1e-12)
