"""The allocation-free orthonormalisation entry point against rpt_reorth.

rpt_reorth_noalloc runs rpt_reorth's kernels on a fixed device array inside
the library instead of a caller workspace; on the same input it must give the
same basis bit for bit (the kernels are deterministic: fixed reduction order,
one workgroup for the factorisation).  Two calls in a row, the second on a
smaller input, so that the second reuses the array the first filled."""
import ctypes as C

import numpy as np
import pytest

import rpt_synth as S
from gpu_util import announce, torch_cuda

pytestmark = pytest.mark.gpu


def _with_workspace(rpt, lib, torch, U):
    v, r = U.shape
    out = U.clone()
    info = torch.zeros(1, dtype=torch.int32, device=U.device)
    ws = torch.empty(lib.rpt_reorth_workspace(v, r), dtype=torch.uint8, device=U.device)
    rc = lib.rpt_reorth(out.data_ptr(), v, r, info.data_ptr(), ws.data_ptr(), ws.numel(),
                        torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    return out, info


def _without_workspace(lib, torch, U):
    v, r = U.shape
    out = U.clone()
    info = torch.full((1,), 7, dtype=torch.int32, device=U.device)
    rc = lib.rpt_reorth_noalloc(out.data_ptr(), v, r, info.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    return out, info


def test_reorth_noalloc_matches_reorth_twice():
    torch = torch_cuda()
    import paper_1703_01506_amd as rpt
    from paper_1703_01506_amd import _lib
    lib = _lib.load()
    assert lib.rpt_reorth_noalloc_capacity() >= lib.rpt_reorth_workspace(10_000_000, 128)
    for (v, r, seed) in [(250_000, 100, 5), (3_001, 17, 6)]:
        announce(f"reorth noalloc v={v} r={r}")
        U = torch.from_numpy(S.gaussian_matrix(v, r, seed=seed).astype(np.float32)).cuda()
        ref, iref = _with_workspace(rpt, lib, torch, U)
        got, igot = _without_workspace(lib, torch, U)
        torch.cuda.synchronize()
        assert int(iref.item()) == 0 and int(igot.item()) == 0
        assert torch.equal(got, ref)
        G = (got.double().T @ got.double()).cpu().numpy()
        np.testing.assert_allclose(G, np.eye(r), atol=5e-5)


def test_reorth_noalloc_rejects_bad_arguments():
    torch = torch_cuda()
    from paper_1703_01506_amd import _lib
    lib = _lib.load()
    d = C.c_void_p(256)
    assert lib.rpt_reorth_noalloc(None, 10, 2, None, None) == -1
    assert lib.rpt_reorth_noalloc(d, 10, 129, None, None) == -1
    assert lib.rpt_reorth_noalloc(d, 3, 4, None, None) == -1
