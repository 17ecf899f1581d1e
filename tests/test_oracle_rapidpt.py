"""Pins for the oracle's RapidPT steps (Alg. 2)."""
import numpy as np
import pytest
import scipy.linalg as sla

import rpt_synth as S
from oracle import philox as PH
from oracle import rapidpt as R
from oracle import tstat as OT


def _orth(rng, v, r):
    return R.orthonormalize(rng.normal(size=(v, r)))


def test_orthonormalize_is_positive_qr():
    rng = np.random.default_rng(0)
    A = rng.normal(size=(50, 7))
    Q = R.orthonormalize(A)
    np.testing.assert_allclose(Q.T @ Q, np.eye(7), atol=1e-13)
    Rm = Q.T @ A
    np.testing.assert_allclose(np.tril(Rm, -1), 0, atol=1e-12)
    assert (np.diag(Rm) > 0).all()
    # same as Cholesky-QR: R = chol(A^T A)^T
    C = np.linalg.cholesky(A.T @ A)
    np.testing.assert_allclose(Rm, C.T, rtol=1e-10, atol=1e-12)


def test_complete_is_least_squares():
    rng = np.random.default_rng(1)
    U = _orth(rng, 300, 6)
    idx = np.sort(rng.choice(300, 40, replace=False))
    y = rng.normal(size=40)
    w = R.complete(U, idx, y)
    A = U[idx]
    # normal equations via Cholesky
    w_ne = sla.cho_solve(sla.cho_factor(A.T @ A), A.T @ y)
    np.testing.assert_allclose(w, w_ne, rtol=1e-10, atol=1e-12)
    # residual orthogonal to the sampled basis rows
    np.testing.assert_allclose(A.T @ (y - A @ w), 0, atol=1e-12)
    with pytest.raises(np.linalg.LinAlgError):
        R.complete(U, idx[:5], y[:5])


def test_greedy_step_interpolates_column_and_stays_orthonormal():
    rng = np.random.default_rng(2)
    v, r = 200, 5
    U = _orth(rng, v, r)
    x = rng.normal(size=v)
    idx = np.sort(rng.choice(v, 30, replace=False))
    U2 = R.track_step(U, x[None, :], [idx])
    np.testing.assert_allclose(U2.T @ U2, np.eye(r), atol=1e-12)
    w2 = R.complete(U2, idx, x[idx])
    np.testing.assert_allclose(U2[idx] @ w2, x[idx], atol=1e-10)


def test_first_order_step_spans_grouse_geodesic():
    """B = 1, gamma = 1 gives the same subspace as GROUSE's geodesic update
    with the greedy angle (Balzano et al. 2010; Zhang & Balzano 2016)."""
    rng = np.random.default_rng(3)
    v, r = 120, 4
    U = _orth(rng, v, r)
    x = rng.normal(size=v)
    idx = np.sort(rng.choice(v, 25, replace=False))
    w = R.complete(U, idx, x[idx])
    p = U @ w
    res = np.zeros(v)
    res[idx] = x[idx] - U[idx] @ w
    theta = np.arctan(np.linalg.norm(res) / np.linalg.norm(p))
    Ug = U + np.outer((np.cos(theta) - 1) * p / np.linalg.norm(p)
                      + np.sin(theta) * res / np.linalg.norm(res), w / np.linalg.norm(w))
    np.testing.assert_allclose(Ug.T @ Ug, np.eye(r), atol=1e-12)
    U1 = R.track_step(U, x[None, :], [idx])
    np.testing.assert_allclose(U1 @ U1.T, Ug @ Ug.T, atol=1e-12)


def test_tracking_full_observation_recovers_exact_low_rank():
    rng = np.random.default_rng(4)
    v, r, ell = 150, 4, 12
    A = _orth(rng, v, r)
    T = (A @ rng.normal(size=(r, ell))).T          # ell x v, rank r
    om = np.tile(np.arange(v), (16 * ell, 1))
    # sequential tracking (B = 1, i.e. GROUSE's greedy step column by column)
    U = R.train_subspace(T, rng.normal(size=(v, r)), om, passes=16, batch=1)
    sv = np.linalg.svd(A.T @ U, compute_uv=False)  # cosines of principal angles
    assert sv.min() > 1 - 1e-12


def test_linear_statistic_recovery_is_exact():
    """stat = mean difference: T = X C has rank <= n-1, so with U spanning the
    centred data and sigma = mu = 0 the recovered maxima equal NaivePT's."""
    n, n1, v = 10, 5, 400
    X, _ = S.iid_volumes(n, v, n1, seed=7)
    labels = S.relabellings(12, n, n1, seed=8)
    Xc = X - X.mean(axis=1, keepdims=True)
    U = R.orthonormalize(Xc[:, :n - 1])
    om = S.omega_sets(12, v, 40, seed=9)
    rec = R.recover(X, labels, U, 0.0, 0.0, om, seed=1, stat="meandiff")
    naive = np.array([OT.meandiff(X, labels[i] == 1).max() for i in range(12)])
    np.testing.assert_allclose(rec, naive, rtol=1e-10, atol=1e-12)


def test_recovery_noise_and_shift_enter_as_written():
    rng = np.random.default_rng(5)
    n, n1, v = 8, 4, 60
    X = rng.normal(size=(v, n))
    U = _orth(rng, v, 3)
    lab = S.relabellings(3, n, n1, seed=2)
    om = S.omega_sets(3, v, 20, seed=3)
    sigma, mu, seed = 0.25, 0.7, 99
    got = R.recover(X, lab, U, sigma, mu, om, seed, col0=10)
    for j in range(3):
        y = OT.tstat(X[om[j]], lab[j] == 1)
        w = np.linalg.lstsq(U[om[j]], y, rcond=None)[0]
        z = PH.normals(seed, PH.STREAM_RECOVERY, 10 + j, np.arange(v))
        assert got[j] == pytest.approx(np.max(U @ w + sigma * z) + mu, rel=1e-12)


def test_sigma_mu_rules():
    rng = np.random.default_rng(6)
    v, r, ell = 300, 3, 5
    U = _orth(rng, v, r)
    T = (U @ rng.normal(size=(r, ell))).T + 0.01 * rng.normal(size=(ell, v))
    om = S.omega_sets(ell, v, 60, seed=4)
    sig, mu, tmax = R.sigma_mu(T, U, om, seed=5)
    res = np.concatenate([T[i, om[i]] - U[om[i]] @ np.linalg.lstsq(U[om[i]], T[i, om[i]], rcond=None)[0]
                          for i in range(ell)])
    assert sig == pytest.approx(np.std(res, ddof=1), rel=1e-12)
    assert 0.005 < sig < 0.015
    np.testing.assert_allclose(tmax, T.max(axis=1))
    assert R.sigma_mu(T, U, om, seed=5, mu_rule="zero")[1] == 0.0
    lit = R.sigma_mu(T, U, om, seed=5, mu_rule="literal")[1]
    assert 0.0 < lit < 0.1
