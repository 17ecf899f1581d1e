"""RapidPT (Alg. 2) end to end on the simulated datasets of Sec. 5.1 and 5.2
(Simulation Data I: n = 30, v = 20,000, 1% of voxels N(1, 1) in one group;
Simulation Data II: n up to 150 here, a quarter of the voxels shifted by 5),
GPU against the FP64 oracle on the same seeded inputs.  These shapes add the
smallest (r = 10) and the largest (r = 128) basis ranks the library takes,
sampling rates of 3.2% and 4% and a 150-subject design."""
import numpy as np
import pytest

import rpt_synth as S
from gpu_util import announce, torch_cuda
from oracle import metrics as OM
from oracle import rapidpt as OR


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_simulated_data_generators():
    """Simulation Data II puts the signal in group 2 (columns n1..n-1): the
    shifted voxels carry +shift there and nothing in group 1."""
    n, v, n1 = 30, 2_000, 15
    X1, s1 = S.iid_volumes(n, v, n1, 0.05, 7.0, seed=9, signal_group=1)
    X2, s2 = S.iid_volumes(n, v, n1, 0.05, 7.0, seed=9, signal_group=2)
    X0, _ = S.iid_volumes(n, v, n1, 0.0, 0.0, seed=9)
    assert np.array_equal(s1, s2) and s1.size == 100
    np.testing.assert_allclose((X1 - X0)[np.ix_(s1, np.arange(n1))], 7.0, rtol=0, atol=1e-12)
    np.testing.assert_allclose((X2 - X0)[np.ix_(s2, np.arange(n1, n))], 7.0, rtol=0, atol=1e-12)
    assert not (X2 - X0)[:, :n1].any() and not (X1 - X0)[:, n1:].any()
    with pytest.raises(ValueError):
        S.iid_volumes(n, v, n1, 0.05, 1.0, signal_group=3)


@pytest.mark.gpu
@pytest.mark.parametrize("case", [
    # (n, ell, r, eta_ppm, frac, shift, L): Sim I at l = n/3 and l = 2n; Sim II at n = 150
    (30, 10, 10, 40_000, 0.01, 1.0, 600),
    (30, 60, 30, 40_000, 0.01, 1.0, 600),
    (150, 150, 128, 32_000, 0.25, 5.0, 400),
])
def test_rapidpt_simulated_data_matches_oracle(case):
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    n, ell, r, eta_ppm, frac, shift, L = case
    v, passes, seed = 20_000, 4, 2017
    announce(f"rapidpt simulated n={n} l={ell} r={r} eta_ppm={eta_ppm} L={L}")
    k = S.omega_count(v, eta_ppm)
    X, _ = S.iid_volumes(n, v, n // 2, frac, shift, seed=1703, signal_group=2)
    X = X.astype(np.float32)
    labels = S.relabellings(L, n, n // 2, seed=1506)
    U0 = S.gaussian_matrix(v, r, seed=3).astype(np.float32)
    omt = S.omega_sets(passes * ell, v, k, seed=41)
    oms = S.omega_sets(ell, v, k, seed=42)
    omr = S.omega_sets(L - ell, v, k, seed=43)
    h, tr, info = rpt.rapidpt_maxnull(_dev(torch, X), _dev(torch, labels[:ell]), _dev(torch, labels[ell:]),
                                      _dev(torch, U0), _dev(torch, omt), _dev(torch, oms), _dev(torch, omr),
                                      passes=passes, seed=seed, prec="split_bf16")
    h = h.cpu().numpy()
    assert (info.cpu().numpy() == 0).all()
    href, Uo, so, muo = OR.rapidpt_maxnull(X.astype(np.float64), labels[:ell], labels[ell:], U0.astype(np.float64),
                                           omt, oms, omr, passes, seed)
    sigma, mu = [float(x) for x in tr["sigma_mu"].cpu().numpy()]
    assert abs(sigma - so) <= 1e-3 * so
    assert abs(mu - muo) <= 2e-3
    assert OM.kl_divergence(href, h) < 1e-3
    t_ref, t_gpu = OM.threshold(href, 0.05), OM.threshold(h, 0.05)
    assert abs(t_gpu - t_ref) <= 0.01 * abs(t_ref)
    np.testing.assert_allclose(h, href, atol=5e-3, rtol=0)
