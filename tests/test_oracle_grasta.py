"""Pins of the oracle's robust (l1) tracker, the GRASTA reading of Sec. 3.1
and Sec. 4.1: the ADMM column fit against an exact linear program, the
geodesic step's direction, orthonormality and fixed points, and recovery of
a low-rank subspace through sparse gross outliers where the l2 tracker
fails."""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import rapidpt as OR


def _lp_l1(A, y):
    """min_w |y - A w|_1 as a linear program in (w, t): min sum t, -t <= y - A w <= t."""
    k, r = A.shape
    c = np.concatenate([np.zeros(r), np.ones(k)])
    Aub = np.block([[A, -np.eye(k)], [-A, -np.eye(k)]])
    bub = np.concatenate([y, -y])
    res = linprog(c, A_ub=Aub, b_ub=bub, bounds=[(None, None)] * r + [(0, None)] * k, method="highs")
    assert res.success
    return res.x[:r], res.fun


def test_l1_fit_matches_linear_program():
    """The ADMM fixed point is the l1 regression: coefficients and objective
    equal the linear program's; the final w step leaves A^T Gamma = 0."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 3))
    y = A @ rng.standard_normal(3) + 0.05 * rng.standard_normal(40)
    y[[3, 11, 20, 33, 37]] += 8.0
    w_lp, f_lp = _lp_l1(A, y)
    w, s, lam, g = OR.l1_fit(A, y, 1.0, 3000)
    np.testing.assert_allclose(w, w_lp, atol=1e-9)
    assert abs(np.sum(np.abs(y - A @ w)) - f_lp) <= 1e-9 * f_lp
    assert np.abs(A.T @ g).max() < 1e-12
    # the outliers are the entries the fit leaves to s
    assert set(np.flatnonzero(np.abs(s) > 1.0)) == {3, 11, 20, 33, 37}


def test_l1_fit_exact_column_has_no_outliers():
    """A column in the span is fitted exactly after one iteration: s = 0,
    lam = 0 and Gamma = 0."""
    rng = np.random.default_rng(6)
    A = rng.standard_normal((30, 4))
    w0 = rng.standard_normal(4)
    w, s, lam, g = OR.l1_fit(A, A @ w0, 1.0, 5)
    np.testing.assert_allclose(w, w0, atol=1e-12)
    assert np.abs(s).max() == 0.0 and np.abs(lam).max() < 1e-12 and np.abs(g).max() < 1e-12


@pytest.mark.parametrize("eta", [1e-3, 0.05, 3.0])
def test_grasta_step_keeps_orthonormality(eta):
    """The geodesic step keeps U orthonormal for any step (Gamma is
    orthogonal to span U), up to the pi/2 cap."""
    rng = np.random.default_rng(7)
    U = OR.orthonormalize(rng.standard_normal((60, 4)))
    x = rng.standard_normal(60)
    idx = np.sort(rng.choice(60, 25, replace=False))
    U1 = OR.grasta_step(U, x, idx, eta, 1.0, 40)
    np.testing.assert_allclose(U1.T @ U1, np.eye(4), atol=1e-12)
    assert np.abs(U1 - U).max() > 1e-6


def test_grasta_step_direction_is_the_negative_gradient():
    """For a small step the change of U is -eta Gamma w^T (the descent
    direction of the augmented Lagrangian on the Grassmannian): pins the
    sign and the scale of the angle eta |Gamma| |w|."""
    rng = np.random.default_rng(8)
    U = OR.orthonormalize(rng.standard_normal((50, 3)))
    x = rng.standard_normal(50)
    idx = np.sort(rng.choice(50, 20, replace=False))
    w, s, lam, g = OR.l1_fit(U[idx], x[idx], 1.0, 40)
    gam = np.zeros(50)
    gam[idx] = g
    eta = 1e-9  # theta about 5e-8: the second-order term is below 1e-7 of the first
    D = (OR.grasta_step(U, x, idx, eta, 1.0, 40) - U) / eta
    np.testing.assert_allclose(D, -np.outer(gam, w), atol=1e-5 * np.abs(np.outer(gam, w)).max())


def test_grasta_step_fixes_a_column_in_the_span():
    """A column inside span U gives Gamma = 0 (to rounding): U does not move."""
    rng = np.random.default_rng(9)
    U = OR.orthonormalize(rng.standard_normal((40, 3)))
    x = U @ rng.standard_normal(3)
    idx = np.sort(rng.choice(40, 15, replace=False))
    np.testing.assert_allclose(OR.grasta_step(U, x, idx, 0.1, 1.0, 10), U, atol=1e-14)


def test_grasta_recovers_subspace_through_outliers():
    """Rank-3 columns with 10% of the entries hit by +-20 outliers, 40% of
    the voxels sampled per visit: robust tracking recovers the subspace
    (largest principal angle below 3 degrees after 40 passes) where the l2
    tracker, on the same visits, ends almost orthogonal to it."""
    rng = np.random.default_rng(5)
    v, r, ell, P = 400, 3, 60, 40
    Us = OR.orthonormalize(rng.standard_normal((v, r)))
    X = (Us @ (10.0 * rng.standard_normal((r, ell)))).T.copy()
    mask = rng.random(X.shape) < 0.1
    X[mask] += rng.choice([-1, 1], mask.sum()) * 20.0
    om = np.array([np.sort(rng.choice(v, 160, replace=False)) for _ in range(P * ell)])
    U0 = rng.standard_normal((v, r))
    U1 = OR.train_subspace_l1(X, U0, om, P, eta=1e-4, rho=1.0, iters=30)
    sin_l1 = np.sqrt(max(0.0, 1.0 - OR.principal_angle_cosines(U1, Us).min() ** 2))
    U2 = OR.train_subspace(X, U0, om, P)
    sin_l2 = np.sqrt(max(0.0, 1.0 - OR.principal_angle_cosines(U2, Us).min() ** 2))
    assert sin_l1 < 0.05
    assert sin_l2 > 0.5
