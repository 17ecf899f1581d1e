"""Pins of the masked-loss-driven training in oracle/rapidpt.py
(``gradient_step``, ``train_subspace_gradient``): the gradient against
central differences of Eq. 1's loss, its tangency at the least-squares fit,
the first-order form of the retracted step, descent, and recovery of an
exactly low-rank subspace from sampled entries."""
import numpy as np

from oracle import masked_loss as ML
from oracle import rapidpt as R


def _problem(seed=0, v=80, r=3, ell=40, k=20, passes=60):
    rng = np.random.default_rng(seed)
    A = np.linalg.qr(rng.normal(size=(v, r)))[0]
    T = (A @ rng.normal(size=(r, ell)) * 3.0).T
    U0 = rng.normal(size=(v, r))
    om = np.stack([np.sort(rng.choice(v, k, replace=False)) for _ in range(passes * ell)])
    return A, T, U0, om


def _batch(U, T_rows, sets):
    B = len(sets)
    ptr = np.zeros(B + 1, dtype=np.int64)
    W = np.zeros((U.shape[1], B))
    idx, t = [], []
    for b, o in enumerate(sets):
        y = T_rows[b][o]
        W[:, b] = R.complete(U, o, y)
        ptr[b + 1] = ptr[b] + len(o)
        idx.append(o)
        t.append(y)
    return W, ptr, np.concatenate(idx), np.concatenate(t)


def test_gradient_matches_central_differences_and_is_tangent():
    A, T, U0, om = _problem(1)
    U = R.orthonormalize(U0)
    sets = [om[i] for i in range(6)]
    W, ptr, idx, t = _batch(U, T[:6], sets)
    G, _ = ML.grad(U, W, ptr, idx, t)
    h = 1e-3
    for (q, c) in ((int(om[0][0]), 0), (int(om[3][5]), 2), (int(om[5][-1]), 1)):
        Up, Um = U.copy(), U.copy()
        Up[q, c] += h
        Um[q, c] -= h
        fd = (ML.loss(Up, W, ptr, idx, t) - ML.loss(Um, W, ptr, idx, t)) / (2 * h)
        assert abs(fd - G[q, c]) <= 1e-8 * max(1.0, abs(fd))
    # the least-squares residual of every member is orthogonal to U_O
    assert np.abs(U.T @ G).max() <= 1e-10 * max(1.0, np.abs(G).max())


def test_gradient_step_first_order_form():
    """For a small step the retracted move is -alpha times the Riemannian
    gradient: the sign, the scale and the projection of the step."""
    A, T, U0, om = _problem(2)
    U = R.orthonormalize(U0)
    sets = [om[i] for i in range(5)]
    W, ptr, idx, t = _batch(U, T[:5], sets)
    G, _ = ML.grad(U, W, ptr, idx, t)
    G = G - U @ (U.T @ G)
    alpha = 1e-7
    U1 = R.gradient_step(U, T[:5], sets, alpha)
    # compare subspaces through the projector: P1 - P = -alpha (G U^T + U G^T) + O(alpha^2)
    dP = (U1 @ U1.T - U @ U.T) / alpha
    ref = -(G @ U.T + U @ G.T)
    assert np.linalg.norm(dP - ref) <= 1e-4 * np.linalg.norm(ref)


def test_gradient_step_descends():
    A, T, U0, om = _problem(3)
    U = R.orthonormalize(U0)
    sets = [om[i] for i in range(8)]
    before, after = [], []
    U1 = R.gradient_step(U, T[:8], sets, 0.01, before)
    R.gradient_step(U1, T[:8], sets, 0.0, after)
    assert sum(after) < sum(before)


def test_gradient_training_recovers_low_rank_subspace():
    """Exactly rank-3 columns observed on 20 of 80 voxels each: 60 passes of
    batches of 8 at step 0.02 recover the subspace and fit the samples."""
    A, T, U0, om = _problem(0)
    hist = []
    U = R.train_subspace_gradient(T, U0, om, 60, 8, 0.02, hist)
    assert R.principal_angle_cosines(U, A).min() > 1.0 - 1e-9
    assert hist[-1] < 1e-12 * hist[0]
    assert np.allclose(U.T @ U, np.eye(3), atol=1e-12)
