"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/rpt.h declares, and rejects invalid arguments synchronously (before any
device work, so these run without a GPU)."""
import ctypes as C
import os
import re
import sys

import pytest

from conftest import ROOT

LIB = os.path.join(ROOT, "paper_1703_01506_amd", "librpt.so")
HEADER = os.path.join(ROOT, "include", "rpt.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rpt_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librpt.so is not built (python paper_1703_01506_amd/build.py)")
    from paper_1703_01506_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    from paper_1703_01506_amd._lib import SIGNATURES
    assert sorted(SIGNATURES) == names


def test_status_strings(lib):
    assert lib.rpt_status_string(0) == b"ok"
    assert b"workspace" in lib.rpt_status_string(-4)
    assert lib.rpt_version() >= 100


def test_naive_argument_validation(lib):
    dummy = C.c_void_p(256)  # never dereferenced: validation fails first
    ws_need = lib.rpt_naive_workspace(1000, 20, 50, 1)
    assert ws_need > 0
    # n1 out of range
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 1, dummy, 50, 0, 1, 0, dummy, None, dummy, ws_need, None) == -1
    # ldx < n
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 10, 10, dummy, 50, 0, 1, 0, dummy, None, dummy, ws_need, None) == -1
    # bad tail / precision
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 10, dummy, 50, 7, 1, 0, dummy, None, dummy, ws_need, None) == -1
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 10, dummy, 50, 0, 9, 0, dummy, None, dummy, ws_need, None) == -1
    # unbalanced split-BF16 is not provided
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 8, dummy, 50, 0, 1, 0, dummy, None, dummy, ws_need, None) == -6
    # more than 512 subjects; the FP32 path above 128
    ws_wide = lib.rpt_naive_workspace(1000, 513, 50, 1)
    assert lib.rpt_naive_maxnull(dummy, 1000, 513, 513, 256, dummy, 50, 0, 1, 0, dummy, None, dummy, ws_wide,
                                 None) == -1
    ws_f32 = lib.rpt_naive_workspace(1000, 200, 50, 0)
    assert lib.rpt_naive_maxnull(dummy, 1000, 200, 200, 100, dummy, 50, 0, 0, 0, dummy, None, dummy, ws_f32,
                                 None) == -6
    # workspace too small / misaligned
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 10, dummy, 50, 0, 1, 0, dummy, None, dummy, ws_need - 1,
                                 None) == -4
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 10, dummy, 50, 0, 1, 0, dummy, None, C.c_void_p(257), ws_need,
                                 None) == -4
    # L == 0 is a valid no-op
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 10, dummy, 0, 0, 1, 0, dummy, None, dummy, ws_need, None) == 0
    # the statistic: 0 = Eq. 2's t, 1 = mean difference (balanced designs only)
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 10, dummy, 50, 0, 1, 2, dummy, None, dummy, ws_need, None) == -1
    assert lib.rpt_naive_maxnull(dummy, 1000, 20, 20, 8, dummy, 50, 0, 0, 1, dummy, None, dummy, ws_need, None) == -6


def test_batched_recovery_validation(lib):
    from paper_1703_01506_amd._lib import RptStudy
    dummy = 256
    arr = (RptStudy * 2)()
    for d in arr:
        d.X, d.v, d.n, d.n1, d.ldx = dummy, 5000, 20, 10, 20
        d.labels, d.L_rec, d.col0, d.U, d.r, d.study = dummy, 30, 0, dummy, 8, 0
        d.sigma_mu, d.omega_ptr, d.omega_idx, d.nnz, d.seed = dummy, dummy, dummy, 3000, 1
        d.max_out, d.info = dummy, dummy
    need = lib.rpt_recover_batched_workspace(arr, 2)
    assert need > 0
    ws = C.c_void_p(512)
    # workspace too small, and a bad study caught before any launch
    assert lib.rpt_recover_maxnull_batched(arr, 2, ws, need - 1, None) == -4
    arr[1].n1 = 9
    assert lib.rpt_recover_batched_workspace(arr, 2) == 0
    assert lib.rpt_recover_maxnull_batched(arr, 2, ws, need, None) == -6
    arr[1].n1 = 10
    arr[1].r = 129
    assert lib.rpt_recover_maxnull_batched(arr, 2, ws, need, None) == -1
    # no studies is a valid no-op
    assert lib.rpt_recover_maxnull_batched(arr, 0, ws, need, None) == 0


def test_rapidpt_end_to_end_validation(lib):
    """rpt_rapidpt_maxnull checks the training and the recovery arguments and
    the combined workspace before any launch."""
    d = C.c_void_p(256)
    v, n, ell, L_rec, r, k, prec = 5000, 20, 30, 70, 8, 40, 1
    need = lib.rpt_rapidpt_workspace(v, n, ell, L_rec, r, k, prec)
    assert need >= lib.rpt_train_workspace(v, n, ell, r, k, prec) + lib.rpt_recover_workspace(v, n, L_rec, r, k)
    ws = C.c_void_p(512)

    def call(n1=10, r_=r, k_=k, ws_bytes=need, batch=ell, passes=2, gamma=1.0, tol=0.0, stat=0, tracker=None):
        tr = C.byref(tracker) if tracker is not None else None
        return lib.rpt_rapidpt_maxnull(d, v, n, n, n1, d, ell, d, L_rec, d, r_, d, k_, passes, batch, gamma, tol, d,
                                       d, 7, 0, prec, stat, tr, d, d, d, d, d, d, d, ws, ws_bytes, None)

    assert call(ws_bytes=need - 1) == -4      # workspace
    assert call(n1=9) == -6                    # unbalanced designs are not provided
    assert call(r_=129) == -1                  # rank above 128
    assert call(k_=7) == -2                    # fewer sampled voxels than the rank
    assert call(batch=ell + 1) == -1           # mini-batch larger than l
    assert call(batch=1, gamma=1.5) == -1      # geodesic angle must stay below 3 pi / 4
    assert call(tol=-1.0) == -1                # negative stopping tolerance
    assert call(batch=2, tol=1e-3) == -6       # the stopping rule belongs to column-by-column tracking
    assert call(stat=2) == -1                  # no such statistic
    from paper_1703_01506_amd._lib import RptTracker as T
    assert call(tracker=T(3, 1.0, 30)) == -1               # no such tracker
    assert call(batch=5, tol=1e-3, tracker=T(2, 1.0, 30)) == -6   # the gradient tracker runs every pass
    assert call(batch=1, tol=1e-3, tracker=T(2, 1.0, 30)) == -6
    assert call(batch=5, gamma=0.0, tracker=T(2, 1.0, 30)) == -1  # step length must be positive
    assert call(batch=1, tracker=T(1, 0.0, 30)) == -1      # ADMM penalty must be positive
    assert call(batch=1, tracker=T(1, 1.0, 0)) == -1       # at least one ADMM iteration
    assert call(batch=2, tracker=T(1, 1.0, 30)) == -6      # the l1 fit moves U one column at a time
    assert call(batch=1, gamma=2.0, tracker=T(1, 1.0, 30), ws_bytes=need - 1) == -4  # gamma is its step size


def test_sigma_mu_heldout_validation(lib):
    """rpt_sigma_mu checks its arguments and workspace before any launch."""
    d = C.c_void_p(256)
    v, n, h, r, k, prec = 5000, 20, 25, 8, 40, 1
    need = lib.rpt_sigma_mu_workspace(v, n, h, r, k, prec)
    assert need == lib.rpt_train_workspace(v, n, h, r, k, prec)
    ws = C.c_void_p(512)

    def call(n1=10, h_=h, r_=r, k_=k, mu_rule=0, stat=0, ws_bytes=need):
        return lib.rpt_sigma_mu(d, v, n, n, n1, d, h_, d, r_, d, k_, 7, mu_rule, prec, stat, d, d, d, ws, ws_bytes,
                                None)

    assert call(ws_bytes=need - 1) == -4
    assert call(n1=9) == -6
    assert call(h_=0) == -1
    assert call(r_=129) == -1
    assert call(k_=7) == -2
    assert call(mu_rule=3) == -1
    assert call(stat=2) == -1


def test_seeded_inputs_validation(lib):
    """The generators and the end-to-end call's NULL inputs check their
    arguments before any launch."""
    from oracle import sampling as OS
    for v, eta in ((250_000, 3500), (999_999, 1), (1_000_001, 1), (0, 5), (7, 1_000_000)):
        assert lib.rpt_sample_count(v, eta) == OS.sample_count(v, eta)
    assert lib.rpt_sample_count(-1, 5) == -1 and lib.rpt_sample_count(10, 1_000_001) == -1
    d = C.c_void_p(256)
    gl = lib.rpt_gen_relabellings
    assert gl(1, 0, 10, 20, 20, d, None) == -1        # n1 = n
    assert gl(1, 0, 10, 513, 100, d, None) == -1      # more than 512 subjects
    assert gl(1, (1 << 32) - 5, 6, 20, 10, d, None) == -1  # rows past the counter range
    assert gl(1, 0, 10, 20, 10, None, None) == -1     # no output
    assert gl(1, 0, 0, 20, 10, None, None) == 0       # no rows: a no-op
    gs = lib.rpt_gen_sampled_sets
    assert gs(1, 0, 0, 5, 100, 101, d, None) == -1    # k > v
    assert gs(1, 0, 0, 5, 100, 0, d, None) == -1      # empty set
    assert gs(1, -1, 0, 5, 100, 10, d, None) == -1    # negative set id
    assert gs(1, 0, 0, 5, 100_000, 4097, d, None) == -6  # above the LDS-resident shuffle
    assert gs(1, 0, 0, 0, 100, 10, None, None) == 0
    assert lib.rpt_gen_start_basis(1, 100, 0, d, None) == -1
    assert lib.rpt_gen_start_basis(1, 100, 4, None, None) == -1
    # the end-to-end call with NULL inputs needs the generated inputs' workspace
    v, n, ell, L_rec, r, k, prec, passes = 5000, 20, 30, 70, 8, 40, 1, 2
    base = lib.rpt_rapidpt_workspace(v, n, ell, L_rec, r, k, prec)
    extra = lib.rpt_rapidpt_gen_workspace(n, ell, L_rec, k, passes)
    assert extra >= (ell + L_rec) * n + 4 * k * (passes * ell + ell + L_rec)
    ws = C.c_void_p(512)

    def call(ws_bytes, k_=k, v_=v, labels=None, omegas=None):
        return lib.rpt_rapidpt_maxnull(d, v_, n, n, n // 2, labels, ell, labels, L_rec, None, r, omegas, k_, passes,
                                       1, 1.0, 0.0, omegas, omegas, 7, 0, prec, 0, None, d, d, d, d, d, d, d, ws,
                                       ws_bytes, None)

    assert call(base + extra - 1) == -4
    assert call(base - 1, labels=d, omegas=d) == -4   # explicit labels and sets: the base workspace
    big = 5000
    assert call(1 << 40, k_=big, v_=250_000) == -6    # drawn sets above 4096 voxels
    assert lib.rpt_rapidpt_gen_workspace(0, ell, L_rec, k, passes) == 0


def test_autotune_table_roundtrip(lib, tmp_path):
    """The plan table is plain text and survives a save / load round trip
    (no GPU: entries are written by hand)."""
    lib.rpt_autotune_clear()
    assert lib.rpt_autotune_count() == 0
    src = tmp_path / "plans.txt"
    src.write_text("0 250000 10000 100 2 128\n1 250000 9700 100 0 64\n0 5 5 5 5 12\n")  # last: not a multiple of 8
    assert lib.rpt_autotune_load(str(src).encode()) == 2
    assert lib.rpt_autotune_count() == 2
    out = tmp_path / "saved.txt"
    assert lib.rpt_autotune_save(str(out).encode()) == 2
    assert sorted(out.read_text().split("\n")[:2]) == ["0 250000 10000 100 2 128", "1 250000 9700 100 0 64"]
    assert lib.rpt_autotune_load(str(tmp_path / "missing.txt").encode()) == -1
    # workspaces cover every candidate: unchanged by a tuned entry for the shape
    before = lib.rpt_naive_workspace(250000, 100, 10000, 1)
    lib.rpt_autotune_clear()
    assert lib.rpt_naive_workspace(250000, 100, 10000, 1) == before
    dummy = C.c_void_p(256)
    chosen = C.c_int32(0)
    assert lib.rpt_autotune_naive(dummy, 1000, 20, 20, 10, dummy, 0, 1, None, 3, dummy, 1 << 30, None,
                                  C.byref(chosen)) == -1   # L = 0
    assert lib.rpt_autotune_recover(1000, 129, 50, 2, dummy, 1 << 30, None, C.byref(chosen)) == -1


def test_autotune_table_from_environment(tmp_path):
    """A table named by RPT_TUNE_CACHE is read on the table's first use (in a
    fresh process, so that this process's table is not involved)."""
    import subprocess
    src = tmp_path / "plans.txt"
    src.write_text("0 250000 10000 100 2 128\n1 250000 9700 100 0 64\n")
    code = ("import sys; sys.path.insert(0, %r); from paper_1703_01506_amd import _lib; "
            "l = _lib.load(); print(l.rpt_autotune_count())" % ROOT)
    env = dict(os.environ, RPT_TUNE_CACHE=str(src))
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "2"
    env["RPT_TUNE_CACHE"] = str(tmp_path / "missing.txt")  # unreadable file: empty table, no error
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "0"


def test_bench_refuses_more_than_one_gpu():
    """The benchmark is one-GPU only: --gpus above 1 exits with status 2 and a
    message, before touching any device."""
    import subprocess
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU only" in out.stderr
    for mode in ("--studies", "--masked-loss"):
        out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), mode, "--gpus", "2"],
                             capture_output=True, text=True, timeout=120)
        assert out.returncode == 2 and "one GPU only" in out.stderr, mode
