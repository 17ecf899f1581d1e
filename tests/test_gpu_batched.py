"""GPU: recovery of several studies in one call with uneven sampled sets
(CSR), against the FP64 oracle, and captured into a HIP graph."""
import numpy as np
import pytest

import rpt_synth as S
from gpu_util import announce, torch_cuda
from oracle import rapidpt as OR

pytestmark = pytest.mark.gpu

# (n, v, r, L, sigma, mu, col0, study id)
# the last study has more subjects than one 128-wide piece of a row
STUDIES = [(20, 3001, 8, 40, 0.3, 0.05, 0, 3), (36, 5003, 17, 33, 0.0, -0.1, 300, 7),
           (100, 20000, 40, 25, 0.05, 0.2, 301, 11), (200, 7001, 30, 21, 0.1, 0.0, 600, 13)]


def _study(torch, q, n, v, r, L, sigma, mu, col0, sid, seed=2017):
    rng = np.random.default_rng(100 + q)
    X = (rng.normal(size=(v, n)) * rng.uniform(0.5, 2, size=(v, 1)) + rng.normal(size=(v, 1))).astype(np.float32)
    labels = S.relabellings(L, n, n // 2, seed=200 + q)
    U = OR.orthonormalize(rng.normal(size=(v, r)))
    sizes = rng.integers(2 * r + 10, 5 * r + 20, size=L)  # uneven, well-conditioned fits
    om = [np.sort(rng.choice(v, s_, replace=False)).astype(np.int32) for s_ in sizes]
    ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    st = {"X": d(X), "labels": d(labels), "U": d(U.astype(np.float32)),
          "sigma_mu": d(np.array([sigma, mu], dtype=np.float32)), "omega_ptr": d(ptr),
          "omega_idx": d(np.concatenate(om)), "seed": seed, "col0": col0, "study": sid}
    ref = dict(X=X, labels=labels, U=U.astype(np.float32).astype(np.float64), om=om, sigma=float(np.float32(sigma)),
               mu=float(np.float32(mu)), seed=seed, col0=col0, study=sid)
    return st, ref


def _oracle(ref):
    return OR.recover(ref["X"].astype(np.float64), ref["labels"], ref["U"], ref["sigma"], ref["mu"], ref["om"],
                      ref["seed"], col0=ref["col0"], study=ref["study"])


def test_batched_recovery_matches_oracle():
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce("batched recovery")
    pairs = [_study(torch, q, *cfg) for q, cfg in enumerate(STUDIES)]
    outs = rpt.recover_maxnull_batched([p[0] for p in pairs])
    torch.cuda.synchronize()
    for (st, ref), (got, info) in zip(pairs, outs):
        assert (info.cpu().numpy() == 0).all()
        ref_m = _oracle(ref)
        got_m = got.cpu().numpy()
        assert np.all(np.abs(got_m - ref_m) <= 2e-4 * np.maximum(1.0, np.abs(ref_m))), np.abs(got_m - ref_m).max()
    # the study id is part of the noise counter: another id, another draw
    st, ref = pairs[0]
    st2 = dict(st, study=ref["study"] + 1)
    alt = rpt.recover_maxnull_batched([st2])[0][0].cpu().numpy()
    assert not np.allclose(alt, outs[0][0].cpu().numpy())


def test_batched_recovery_graph_replays():
    """Capture the batched call, replay it three times with eager work and
    synchronisation in between; every replay equals the eager result."""
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    announce("batched recovery graph")
    pairs = [_study(torch, q, *cfg) for q, cfg in enumerate(STUDIES)]
    arr, outs, ws = rpt.recover_studies_prepare([p[0] for p in pairs])
    dev = ws.device
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        rpt.recover_studies_launch(arr, len(pairs), ws, dev)  # eager reference on the side stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    eager = [o[0].cpu().numpy().copy() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rpt.recover_studies_launch(arr, len(pairs), ws, dev)
    for rep in range(3):
        for o, _ in outs:
            o.fill_(float("nan"))
        junk = torch.randn(1 << 20, device=dev).sum()  # unrelated eager work
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert bool(torch.isfinite(junk))
        for (o, info), e in zip(outs, eager):
            np.testing.assert_allclose(o.cpu().numpy(), e, atol=1e-5, rtol=0)
            assert (info.cpu().numpy() == 0).all()
