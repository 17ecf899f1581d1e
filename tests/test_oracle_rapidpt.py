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
    assert 0.005 < sig < 0.015
    np.testing.assert_allclose(tmax, T.max(axis=1))
    assert R.sigma_mu(T, U, om, seed=5, mu_rule="zero")[1] == 0.0
    lit = R.sigma_mu(T, U, om, seed=5, mu_rule="literal")[1]
    assert 0.0 < lit < 0.1


def test_sigma_mu_hand_case():
    """One training column T_ex = (1, 2, 3, 6), basis U = (1, 1, 1, 1)/2,
    sampled set {0, 1, 2}: the fit is w = (1 + 2 + 3)/2 / (3/4) = 4, the
    sampled residuals (-1, 0, 1) have sample std 1 (sigma), U w = (2, 2, 2, 2).
    Literal mu (Alg. 2) = max(T_ex - U w) = 6 - 2 = 4.  Mean-gap mu =
    max T_ex - max(U w + sigma z) = 6 - (2 + max z), z the four training-stream
    normals of column 0 (generator pinned by its known-answer vectors)."""
    T = np.array([[1.0, 2.0, 3.0, 6.0]])
    U = np.full((4, 1), 0.5)
    om = np.array([[0, 1, 2]])
    seed = 77
    z = PH.normals(seed, PH.STREAM_TRAINING, 0, np.arange(4))
    sig, mu, tmax = R.sigma_mu(T, U, om, seed)
    assert sig == pytest.approx(1.0, rel=1e-14)
    assert tmax[0] == 6.0
    assert mu == pytest.approx(4.0 - z.max(), rel=1e-13)
    assert R.sigma_mu(T, U, om, seed, mu_rule="literal")[1] == pytest.approx(4.0, rel=1e-14)
    assert R.sigma_mu(T, U, om, seed, mu_rule="zero")[1] == 0.0


def test_mean_gap_mu_is_zero_for_an_exact_fit():
    """A basis that spans every training column leaves no residual: sigma = 0
    and the recovered maxima equal the exact ones, so the shift is zero."""
    rng = np.random.default_rng(11)
    v, r, ell = 200, 3, 6
    U = _orth(rng, v, r)
    T = (U @ rng.normal(size=(r, ell))).T
    om = S.omega_sets(ell, v, 20, seed=12)
    sig, mu, _ = R.sigma_mu(T, U, om, seed=3)
    assert sig < 1e-13
    assert abs(mu) < 1e-12


def test_grouse_step_rotates_by_theta_and_keeps_orthonormality():
    """The geodesic step turns span(U) by exactly theta = gamma arctan(|r|/|p|)
    in one direction (one principal angle theta, the others zero), keeps U
    orthonormal for any gamma, and gamma = 1 (greedy) makes the refitted
    column exact on its sampled set."""
    rng = np.random.default_rng(12)
    v, r = 240, 6
    U = _orth(rng, v, r)
    x = rng.normal(size=v)
    idx = np.sort(rng.choice(v, 40, replace=False))
    w = np.linalg.lstsq(U[idx], x[idx], rcond=None)[0]
    nres = np.linalg.norm(x[idx] - U[idx] @ w)
    for gamma in (0.3, 1.0, 1.7):
        U2 = R.grouse_step(U, x, idx, gamma)
        np.testing.assert_allclose(U2.T @ U2, np.eye(r), atol=1e-12)
        cs = R.principal_angle_cosines(U, U2)
        theta = gamma * np.arctan(nres / np.linalg.norm(w))
        assert np.arccos(min(1.0, cs.min())) == pytest.approx(theta, rel=1e-8)
        np.testing.assert_allclose(cs[:-1], 1.0, atol=1e-12)
    U2 = R.grouse_step(U, x, idx, 1.0)
    w2 = np.linalg.lstsq(U2[idx], x[idx], rcond=None)[0]
    np.testing.assert_allclose(U2[idx] @ w2, x[idx], atol=1e-10)


def _sampled_low_rank(seed, v=300, r=4, ell=20, k=30, passes=60):
    rng = np.random.default_rng(seed)
    A = R.orthonormalize(rng.normal(size=(v, r)))
    T = (A @ rng.normal(size=(r, ell))).T
    om = np.stack([np.sort(rng.choice(v, k, replace=False)) for _ in range(passes * ell)])
    return A, T, om, rng.normal(size=(v, r))


@pytest.mark.parametrize("batch", [1, 5])
def test_tracking_recovers_exact_low_rank_from_sampled_entries(batch):
    """Only 10% of each column is seen per visit: sequential GROUSE (batch 1,
    the paper's mode) and the mini-batch variant both converge to the true
    rank-r subspace (principal angles -> 0)."""
    A, T, om, U0 = _sampled_low_rank(4)
    U = R.train_subspace(T, U0, om, passes=60, batch=batch)
    cs = R.principal_angle_cosines(A, U)
    assert cs.min() > 1 - 1e-6
    # a wrong sign in the update would not converge: the start is far away
    assert R.principal_angle_cosines(A, R.orthonormalize(U0)).min() < 0.5


def test_subspace_change_hand_case_and_stopping_rule():
    """span(e1, e2) against span(cos a e1 + sin a e3, e2): one principal angle
    a, so |P - P'|_F / sqrt(2 r) = sin(a) / sqrt(2).  The stopping rule ends
    tracking after the first pass whose objective (the summed squared sampled
    residuals of its visits) fell by at most tol relative to the pass before."""
    a = 0.3
    U = np.zeros((5, 2)); U[0, 0] = 1; U[1, 1] = 1
    V = np.zeros((5, 2)); V[0, 0] = np.cos(a); V[2, 0] = np.sin(a); V[1, 1] = 1
    assert R.subspace_change(U, V) == pytest.approx(np.sin(a) / np.sqrt(2), rel=1e-14)
    assert R.subspace_change(U, U) == 0.0
    A, T, om, U0 = _sampled_low_rank(5, passes=8)
    hist = []
    R.train_subspace(T, U0, om, passes=8, tol=0.0, history=hist)
    assert len(hist) == 8
    # the objective is what the steps report: pass 1 by hand
    U = R.orthonormalize(U0)
    first = 0.0
    for i in range(T.shape[0]):
        w = np.linalg.lstsq(U[om[i]], T[i, om[i]], rcond=None)[0]
        first += float(np.sum((T[i, om[i]] - U[om[i]] @ w) ** 2))
        U = R.grouse_step(U, T[i], om[i])
    assert hist[0] == pytest.approx(first, rel=1e-10)
    drops = [(hist[p - 1] - hist[p]) / hist[p - 1] for p in range(1, 8)]
    tol = 0.5 * (min(drops) + max(drops))
    stop = next(p for p in range(1, 8) if drops[p - 1] <= tol) + 1
    h2 = []
    U2 = R.train_subspace(T, U0, om, passes=8, tol=tol, history=h2)
    assert 1 < stop < 8 and len(h2) == stop and h2 == hist[:stop]
    np.testing.assert_array_equal(U2, R.train_subspace(T, U0, om, passes=stop))
