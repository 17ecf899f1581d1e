"""GPU parity for the inputs drawn from a seed (relabellings, sampled sets,
the start basis) against oracle/sampling.py, and for the end-to-end call
with those inputs left NULL: it must equal the same call given the drawn
inputs explicitly."""
import numpy as np
import pytest

import rpt_synth as S
from gpu_util import announce, torch_cuda
from oracle import sampling as OS

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,row0,L,n,n1", [
    (2017, 0, 700, 100, 50),       # the benchmark's design
    (5, 3, 50, 512, 256),          # largest n
    (9, 0, 33, 7, 3),              # odd n, unbalanced
    (11, (1 << 32) - 20, 20, 40, 1),  # last rows of the counter range, one subject shuffled in
    (13, 10, 9, 2, 1),
])
def test_relabellings_match_oracle(seed, row0, L, n, n1):
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce(f"gen relabellings seed={seed} row0={row0} L={L} n={n} n1={n1}")
    got = rpt.gen_relabellings(seed, row0, L, n, n1).cpu().numpy()
    ref = OS.relabellings(seed, row0, L, n, n1)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("seed,set_id,row0,rows,v,k", [
    (2017, 0, 300, 64, 250_000, 875),   # recovery sets at the benchmark shape
    (2017, 3, 0, 40, 250_000, 875),     # a tracking pass's sets
    (7, 0, 0, 6, 300, 300),             # every voxel
    (8, 1, 5, 4, 5_000, 4_096),         # largest set, many displaced entries
    (9, 2, 0, 5, (1 << 31) - 1, 5),     # largest v
    (10, 0, 2, 17, 1_000, 1),
])
def test_sampled_sets_match_oracle(seed, set_id, row0, rows, v, k):
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce(f"gen sets seed={seed} set={set_id} row0={row0} rows={rows} v={v} k={k}")
    got = rpt.gen_sampled_sets(seed, set_id, row0, rows, v, k).cpu().numpy()
    ref = OS.sampled_sets(seed, set_id, row0, rows, v, k)
    assert np.array_equal(got, ref)


def test_start_basis_matches_oracle():
    """The Gaussian start basis: FP32 Box-Muller on the hardware log, sin and
    cos units against the FP64 oracle (|z| < 5.9, so 5e-5 absolute covers a
    few FP32 ulps of the radius and of the turn)."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce("gen start basis v=3001 r=37")
    got = rpt.gen_start_basis(31, 3001, 37).cpu().numpy().astype(np.float64)
    ref = OS.gaussian_start(31, 3001, 37)
    np.testing.assert_allclose(got, ref, atol=5e-5, rtol=0)


def test_sample_count():
    torch_cuda()
    import paper_1703_01506_amd as rpt
    for v, eta in ((250_000, 3500), (999_999, 1), (1_000_001, 1), (20_000, 10_000), (5_000, 1_000_000)):
        assert rpt.sample_count(v, eta) == OS.sample_count(v, eta)


@pytest.mark.parametrize("tracker", ["grouse", "l1"])
def test_rapidpt_seeded_equals_explicit_inputs(tracker):
    """rpt_rapidpt_maxnull with every input drawn from the seed (NULL
    pointers) against the same call given the drawn inputs, which are the
    oracle's draws: training maxima bit for bit, recovered maxima within
    1e-5."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    n, v, ell, L, r, eta_ppm, passes, seed = 20, 5000, 30, 100, 8, 8000, 3, 77
    announce(f"rapidpt seeded tracker={tracker}")
    k = rpt.sample_count(v, eta_ppm)
    assert k == 40
    X = torch.from_numpy(S.smoothed_volumes(n, v, seed=5)).cuda()
    kw = dict(tol=1e-3 if tracker == "grouse" else 0.0, tracker=tracker, gamma=1.0)
    h1, t1, i1 = rpt.rapidpt_maxnull_seeded(X, ell, L, r, eta_ppm, passes, seed, **kw)
    labels = rpt.gen_relabellings(seed, 0, L, n, n // 2)
    om_train = torch.cat([rpt.gen_sampled_sets(seed, 1 + p, 0, ell, v, k) for p in range(passes)])
    om_sm = rpt.gen_sampled_sets(seed, 0, 0, ell, v, k)
    om_rec = rpt.gen_sampled_sets(seed, 0, ell, L - ell, v, k)
    U0 = rpt.gen_start_basis(seed, v, r)
    # the drawn inputs are the oracle's
    assert np.array_equal(labels.cpu().numpy(), OS.relabellings(seed, 0, L, n, n // 2))
    assert np.array_equal(om_rec[:5].cpu().numpy(), OS.sampled_sets(seed, 0, ell, 5, v, k))
    assert np.array_equal(om_train[ell:ell + 3].cpu().numpy(), OS.sampled_sets(seed, 2, 0, 3, v, k))
    h2, t2, i2 = rpt.rapidpt_maxnull(X, labels[:ell], labels[ell:], U0, om_train, om_sm, om_rec, passes, seed, **kw)
    torch.cuda.synchronize()
    assert int(t1["passes_used"].item()) == int(t2["passes_used"].item())
    assert torch.equal(h1[:ell], h2[:ell])
    torch.testing.assert_close(h1[ell:], h2[ell:], atol=1e-5, rtol=0)
    torch.testing.assert_close(t1["sigma_mu"], t2["sigma_mu"], atol=1e-6, rtol=0)
    assert torch.equal(i1, i2) and torch.equal(t1["info"], t2["info"])
