"""Torch-facing wrappers of librpt's C ABI.

Argument marshalling only: tensors must already live on the GPU; every step of
the computation runs in librpt's HIP kernels on torch's current stream.  Scratch
workspaces are allocated through torch's caching allocator and passed in.
Functions raise RPTError (a RuntimeError) with the library's status string.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib

PREC = {"fp32": 0, "split_bf16": 1}
TAIL = {"signed": 0, "abs": 1}
MU_RULE = {"mean_gap": 0, "literal": 1, "zero": 2}
STAT = {"t": 0, "meandiff": 1}
TRACKER = {"grouse": 0, "l1": 1, "gradient": 2}


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _dev(t: torch.Tensor, dtype, name: str, ndim: int | None = None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return t


def _data(X: torch.Tensor):
    _dev(X, torch.float32, "X", 2)
    if X.stride(1) != 1:
        raise ValueError("X must have unit stride along subjects")
    return X.shape[0], X.shape[1], X.stride(0)


def naive_maxnull(X: torch.Tensor, labels: torch.Tensor, n1: int | None = None, tail: str = "signed",
                  prec: str = "split_bf16", return_T: bool = False, stat: str = "t"):
    """NaivePT (Alg. 1).  X (v, n) float32, labels (L, n) uint8 with n1 ones per
    row; stat "t" (Eq. 2) or "meandiff".  Returns max (L,) float32, and T (L, v)
    if return_T."""
    lib = _lib.load()
    v, n, ldx = _data(X)
    labels = _dev(labels, torch.uint8, "labels", 2).contiguous()
    L = labels.shape[0]
    if labels.shape[1] != n:
        raise ValueError("labels must have n columns")
    n1 = n // 2 if n1 is None else int(n1)
    dev = X.device
    out = torch.empty(L, dtype=torch.float32, device=dev)
    T = torch.empty((L, v), dtype=torch.float32, device=dev) if return_T else None
    nb = lib.rpt_naive_workspace(v, n, L, PREC[prec])
    ws = _workspace(nb, dev)
    rc = lib.rpt_naive_maxnull(_ptr(X), v, n, ldx, n1, _ptr(labels), L, TAIL[tail], PREC[prec], STAT[stat],
                               _ptr(out), _ptr(T), _ptr(ws), ws.numel(), _stream(dev))
    _lib.check(rc, "rpt_naive_maxnull")
    return (out, T) if return_T else out


def sampled_tstat(X: torch.Tensor, labels: torch.Tensor, omega: torch.Tensor, n1: int | None = None,
                  stat: str = "t"):
    """Statistics at sampled voxels: y[i, q] = stat(voxel omega[i, q], labels[i])."""
    lib = _lib.load()
    v, n, ldx = _data(X)
    labels = _dev(labels, torch.uint8, "labels", 2).contiguous()
    omega = _dev(omega, torch.int32, "omega", 2).contiguous()
    L, k = omega.shape
    if labels.shape[0] != L:
        raise ValueError("labels and omega must have the same number of rows")
    n1 = n // 2 if n1 is None else int(n1)
    y = torch.empty((L, k), dtype=torch.float32, device=X.device)
    ws = _workspace(lib.rpt_sampled_tstat_workspace(v, n), X.device)
    rc = lib.rpt_sampled_tstat(_ptr(X), v, n, ldx, n1, _ptr(labels), L, _ptr(omega), k, STAT[stat], _ptr(y),
                               _ptr(ws), ws.numel(), _stream(X.device))
    _lib.check(rc, "rpt_sampled_tstat")
    return y


def complete(U: torch.Tensor, omega: torch.Tensor, y: torch.Tensor, return_resid: bool = False):
    """Masked least squares per row: W[i] = argmin |U[omega[i]] w - y[i]|.
    Returns (W (L, r), info (L,) int32[, resid (L, k)])."""
    lib = _lib.load()
    U = _dev(U, torch.float32, "U", 2).contiguous()
    omega = _dev(omega, torch.int32, "omega", 2).contiguous()
    y = _dev(y, torch.float32, "y", 2).contiguous()
    v, r = U.shape
    L, k = omega.shape
    dev = U.device
    W = torch.empty((L, r), dtype=torch.float32, device=dev)
    info = torch.empty(L, dtype=torch.int32, device=dev)
    resid = torch.empty((L, k), dtype=torch.float32, device=dev) if return_resid else None
    ws = _workspace(lib.rpt_complete_workspace(L, r), dev)
    rc = lib.rpt_complete(_ptr(U), v, r, _ptr(omega), k, _ptr(y), L, _ptr(W), _ptr(resid), _ptr(info),
                          _ptr(ws), ws.numel(), _stream(dev))
    _lib.check(rc, "rpt_complete")
    return (W, info, resid) if return_resid else (W, info)


def reorth(U: torch.Tensor):
    """In-place orthonormalisation U <- U R^{-1} (Cholesky-QR2, FP64).  Returns info (1,)."""
    lib = _lib.load()
    U = _dev(U, torch.float32, "U", 2)
    if not U.is_contiguous():
        raise ValueError("U must be contiguous")
    v, r = U.shape
    info = torch.empty(1, dtype=torch.int32, device=U.device)
    ws = _workspace(lib.rpt_reorth_workspace(v, r), U.device)
    rc = lib.rpt_reorth(_ptr(U), v, r, _ptr(info), _ptr(ws), ws.numel(), _stream(U.device))
    _lib.check(rc, "rpt_reorth")
    return info


def _tracker(tracker: str, rho: float, admm_iters: int):
    """rpt_tracker for the tracker name: "grouse" (l2) or "l1" (GRASTA)."""
    if tracker not in TRACKER:
        raise ValueError(f"unknown tracker {tracker!r}")
    return C.byref(_lib.RptTracker(TRACKER[tracker], float(rho), int(admm_iters)))


def train_subspace(X, train_labels, U0, omega_train, omega_sm, passes: int, seed: int,
                   batch: int = 1, gamma: float = 1.0, mu_rule: str = "mean_gap",
                   prec: str = "split_bf16", n1: int | None = None, return_T: bool = False, tol: float = 0.0,
                   stat: str = "t", tracker: str = "grouse", rho: float = 1.0, admm_iters: int = 30):
    """Training half of Alg. 2.  batch = 1 tracks one column at a time
    (GROUSE, the paper's mode); tol > 0 stops once a pass's objective no longer
    falls by more than tol (relative).  tracker = "l1" fits each column in the
    l1 norm (ADMM with penalty rho, admm_iters iterations) and moves U along
    the robust gradient with the angle gamma |Gamma| |w| (GRASTA).  Returns a
    dict with U (v, r), sigma_mu (2,), train_max (l,), info (l,), objective
    (passes,) FP64, passes_used (1,) and optionally T_ex (l, v)."""
    lib = _lib.load()
    v, n, ldx = _data(X)
    train_labels = _dev(train_labels, torch.uint8, "train_labels", 2).contiguous()
    U0 = _dev(U0, torch.float32, "U0", 2).contiguous()
    omega_train = _dev(omega_train, torch.int32, "omega_train", 2).contiguous()
    omega_sm = _dev(omega_sm, torch.int32, "omega_sm", 2).contiguous()
    ell = train_labels.shape[0]
    r = U0.shape[1]
    k = omega_sm.shape[1]
    if omega_train.shape != (passes * ell, k) or omega_sm.shape[0] != ell or U0.shape[0] != v:
        raise ValueError("inconsistent shapes")
    batch = int(batch)
    n1 = n // 2 if n1 is None else int(n1)
    dev = X.device
    U = torch.empty((v, r), dtype=torch.float32, device=dev)
    sm = torch.empty(2, dtype=torch.float32, device=dev)
    tmax = torch.empty(ell, dtype=torch.float32, device=dev)
    info = torch.empty(ell, dtype=torch.int32, device=dev)
    obj = torch.empty(max(passes, 1), dtype=torch.float64, device=dev)
    used = torch.empty(1, dtype=torch.int32, device=dev)
    T = torch.empty((ell, v), dtype=torch.float32, device=dev) if return_T else None
    ws = _workspace(lib.rpt_train_workspace(v, n, ell, r, k, PREC[prec]), dev)
    rc = lib.rpt_train_subspace(_ptr(X), v, n, ldx, n1, _ptr(train_labels), ell, _ptr(U0), r,
                                _ptr(omega_train), k, passes, batch, float(gamma), float(tol), _ptr(omega_sm),
                                int(seed), MU_RULE[mu_rule], PREC[prec], STAT[stat],
                                _tracker(tracker, rho, admm_iters), _ptr(U), _ptr(sm), _ptr(tmax),
                                _ptr(T), _ptr(info), _ptr(obj), _ptr(used), _ptr(ws), ws.numel(), _stream(dev))
    _lib.check(rc, "rpt_train_subspace")
    out = {"U": U, "sigma_mu": sm, "train_max": tmax, "info": info, "objective": obj[:passes],
           "passes_used": used}
    if return_T:
        out["T_ex"] = T
    return out


def sigma_mu_heldout(X, labels, U, omega, seed: int, mu_rule: str = "mean_gap", prec: str = "split_bf16",
                     stat: str = "t"):
    """sigma and mu for the basis U from h held-out relabellings (labels h x n,
    fully computed) and their sampled sets omega (h x k).  Returns
    (sigma_mu (2,), col_max (h,), info (h,))."""
    lib = _lib.load()
    v, n, ldx = _data(X)
    labels = _dev(labels, torch.uint8, "labels", 2).contiguous()
    U = _dev(U, torch.float32, "U", 2).contiguous()
    omega = _dev(omega, torch.int32, "omega", 2).contiguous()
    h, r, k = labels.shape[0], U.shape[1], omega.shape[1]
    if omega.shape[0] != h or U.shape[0] != v:
        raise ValueError("inconsistent shapes")
    dev = X.device
    sm = torch.empty(2, dtype=torch.float32, device=dev)
    cmax = torch.empty(h, dtype=torch.float32, device=dev)
    info = torch.empty(h, dtype=torch.int32, device=dev)
    ws = _workspace(lib.rpt_sigma_mu_workspace(v, n, h, r, k, PREC[prec]), dev)
    rc = lib.rpt_sigma_mu(_ptr(X), v, n, ldx, n // 2, _ptr(labels), h, _ptr(U), r, _ptr(omega), k, int(seed),
                          MU_RULE[mu_rule], PREC[prec], STAT[stat], _ptr(sm), _ptr(cmax), _ptr(info), _ptr(ws),
                          ws.numel(), _stream(dev))
    _lib.check(rc, "rpt_sigma_mu")
    return sm, cmax, info


def recover_maxnull(X, labels, U, sigma_mu, omega, seed: int, col0: int = 0, n1: int | None = None,
                    return_W: bool = False, stat: str = "t", omega_ptr=None):
    """Recovery half of Alg. 2.  omega is (L, k) int32, or with omega_ptr (L + 1
    int64 CSR offsets) the flat int32 indices of uneven sampled sets.  Returns
    (max (L,), info (L,)[, W (L, r)])."""
    lib = _lib.load()
    v, n, ldx = _data(X)
    labels = _dev(labels, torch.uint8, "labels", 2).contiguous()
    U = _dev(U, torch.float32, "U", 2).contiguous()
    sigma_mu = _dev(sigma_mu, torch.float32, "sigma_mu", 1).contiguous()
    if omega_ptr is None:
        omega = _dev(omega, torch.int32, "omega", 2).contiguous()
        L, k = omega.shape
    else:
        omega = _dev(omega, torch.int32, "omega", 1).contiguous()
        omega_ptr = _dev(omega_ptr, torch.int64, "omega_ptr", 1).contiguous()
        L = omega_ptr.shape[0] - 1
        if L != labels.shape[0]:
            raise ValueError("omega_ptr must have one entry per relabelling plus one")
        # the longest row sizes the workspace (a host read of the offsets,
        # marshalling only)
        offs = omega_ptr.cpu()
        k = int((offs[1:] - offs[:-1]).max().item()) if L > 0 else 1
    r = U.shape[1]
    n1 = n // 2 if n1 is None else int(n1)
    dev = X.device
    out = torch.empty(L, dtype=torch.float32, device=dev)
    info = torch.empty(L, dtype=torch.int32, device=dev)
    W = torch.empty((L, r), dtype=torch.float32, device=dev) if return_W else None
    ws = _workspace(lib.rpt_recover_workspace(v, n, L, r, max(k, 1)), dev)
    rc = lib.rpt_recover_maxnull(_ptr(X), v, n, ldx, n1, _ptr(labels), L, int(col0), _ptr(U), r,
                                 _ptr(sigma_mu), _ptr(omega), max(k, 1), _ptr(omega_ptr), int(seed), STAT[stat],
                                 _ptr(out), _ptr(W), _ptr(info), _ptr(ws), ws.numel(), _stream(dev))
    _lib.check(rc, "rpt_recover_maxnull")
    return (out, info, W) if return_W else (out, info)


def recover_studies_prepare(studies):
    """Marshal a list of study dicts (keys: X, labels, U, sigma_mu, omega_ptr
    (int64 CSR offsets), omega_idx (int32), seed, col0, study, optional n1)
    into the descriptor array of rpt_recover_maxnull_batched.  Returns
    (descriptors, outputs [(max (L,), info (L,))], workspace)."""
    import ctypes as C
    lib = _lib.load()
    arr = (_lib.RptStudy * max(len(studies), 1))()
    outs = []
    dev = None
    for q, st in enumerate(studies):
        X = st["X"]
        v, n, ldx = _data(X)
        dev = X.device
        labels = _dev(st["labels"], torch.uint8, "labels", 2).contiguous()
        U = _dev(st["U"], torch.float32, "U", 2).contiguous()
        sm = _dev(st["sigma_mu"], torch.float32, "sigma_mu", 1).contiguous()
        optr = _dev(st["omega_ptr"], torch.int64, "omega_ptr", 1).contiguous()
        oidx = _dev(st["omega_idx"], torch.int32, "omega_idx", 1).contiguous()
        L = labels.shape[0]
        out = torch.empty(L, dtype=torch.float32, device=dev)
        info = torch.empty(L, dtype=torch.int32, device=dev)
        outs.append((out, info))
        d = arr[q]
        d.X, d.v, d.n, d.n1, d.ldx = _ptr(X), v, n, int(st.get("n1", n // 2)), ldx
        d.labels, d.L_rec, d.col0 = _ptr(labels), L, int(st.get("col0", 0))
        d.U, d.r, d.study, d.sigma_mu = _ptr(U), U.shape[1], int(st.get("study", q)), _ptr(sm)
        d.omega_ptr, d.omega_idx, d.nnz = _ptr(optr), _ptr(oidx), oidx.numel()
        d.seed, d.max_out, d.info = int(st["seed"]), _ptr(out), _ptr(info)
        st["_keep"] = (labels, U, sm, optr, oidx)  # keep the marshalled tensors alive
    need = lib.rpt_recover_batched_workspace(arr, len(studies))
    if need == 0:
        raise ValueError("invalid study descriptor")
    ws = _workspace(need, dev)
    return arr, outs, ws


def recover_studies_launch(arr, n_studies: int, ws, device):
    """Enqueue rpt_recover_maxnull_batched (no allocation: capturable)."""
    lib = _lib.load()
    rc = lib.rpt_recover_maxnull_batched(arr, n_studies, _ptr(ws), ws.numel(), _stream(device))
    _lib.check(rc, "rpt_recover_maxnull_batched")


def recover_maxnull_batched(studies):
    """Recovery half of Alg. 2 for several studies with uneven sampled sets
    (CSR).  Returns [(max (L,), info (L,))] per study."""
    arr, outs, ws = recover_studies_prepare(studies)
    recover_studies_launch(arr, len(studies), ws, ws.device)
    return outs


def observed_tstat(X, n1: int | None = None):
    """t of every voxel under the observed labelling (group 1 = the first n1
    subjects).  Returns t (v,) FP32."""
    lib = _lib.load()
    v, n, ldx = _data(X)
    n1 = n // 2 if n1 is None else int(n1)
    t = torch.empty(v, dtype=torch.float32, device=X.device)
    ws = _workspace(lib.rpt_observed_tstat_workspace(v, n), X.device)
    rc = lib.rpt_observed_tstat(_ptr(X), v, n, ldx, n1, _ptr(t), _ptr(ws), ws.numel(), _stream(X.device))
    _lib.check(rc, "rpt_observed_tstat")
    return t


def fwer_threshold(maxima, alpha: float = 0.05):
    """Level-alpha family-wise threshold (a (1,) FP32 device tensor)."""
    lib = _lib.load()
    maxima = _dev(maxima, torch.float32, "maxima", 1).contiguous()
    out = torch.empty(1, dtype=torch.float32, device=maxima.device)
    rc = lib.rpt_fwer_threshold(_ptr(maxima), maxima.numel(), float(alpha), _ptr(out), _stream(maxima.device))
    _lib.check(rc, "rpt_fwer_threshold")
    return out


def corrected_pvalues(maxima, t):
    """Corrected p-value of every entry of t against the max null."""
    lib = _lib.load()
    maxima = _dev(maxima, torch.float32, "maxima", 1).contiguous()
    t = _dev(t, torch.float32, "t", 1).contiguous()
    p = torch.empty_like(t)
    rc = lib.rpt_corrected_pvalues(_ptr(maxima), maxima.numel(), _ptr(t), t.numel(), _ptr(p), _stream(t.device))
    _lib.check(rc, "rpt_corrected_pvalues")
    return p


def rejection_counts(maxima1, maxima2, t, alpha: float = 0.05):
    """(v1, v2, vc) rejections at alpha under two max nulls (int64 device (3,))."""
    lib = _lib.load()
    m1 = _dev(maxima1, torch.float32, "maxima1", 1).contiguous()
    m2 = _dev(maxima2, torch.float32, "maxima2", 1).contiguous()
    t = _dev(t, torch.float32, "t", 1).contiguous()
    out = torch.empty(3, dtype=torch.int64, device=t.device)
    rc = lib.rpt_rejection_counts(_ptr(m1), m1.numel(), _ptr(m2), m2.numel(), _ptr(t), t.numel(), float(alpha),
                                  _ptr(out), _stream(t.device))
    _lib.check(rc, "rpt_rejection_counts")
    return out


def rapidpt_maxnull(X, train_labels, rec_labels, U0, omega_train, omega_sm, omega_rec, passes: int, seed: int,
                    batch: int = 1, gamma: float = 1.0, mu_rule: str = "mean_gap",
                    prec: str = "split_bf16", tol: float = 0.0, stat: str = "t", tracker: str = "grouse",
                    rho: float = 1.0, admm_iters: int = 30):
    """Alg. 2 end to end in one library call: the l exact training maxima
    followed by the recovered ones.  Returns (h (L,), train dict, recovery
    info); the train dict holds U, sigma_mu, train_max (a view of h), info,
    objective and passes_used (as train_subspace, whose tracker arguments
    these are)."""
    v = X.shape[0]
    train_labels = _dev(train_labels, torch.uint8, "train_labels", 2).contiguous()
    rec_labels = _dev(rec_labels, torch.uint8, "rec_labels", 2).contiguous()
    U0 = _dev(U0, torch.float32, "U0", 2).contiguous()
    omega_train = _dev(omega_train, torch.int32, "omega_train", 2).contiguous()
    omega_sm = _dev(omega_sm, torch.int32, "omega_sm", 2).contiguous()
    omega_rec = _dev(omega_rec, torch.int32, "omega_rec", 2).contiguous()
    ell, L_rec = train_labels.shape[0], rec_labels.shape[0]
    r, k = U0.shape[1], omega_sm.shape[1]
    if (omega_train.shape != (passes * ell, k) or omega_sm.shape[0] != ell or omega_rec.shape != (L_rec, k)
            or U0.shape[0] != v):
        raise ValueError("inconsistent shapes")
    return _rapidpt_call(X, (train_labels, rec_labels, U0, omega_train, omega_sm, omega_rec), ell, L_rec, r, k,
                         passes, seed, batch, gamma, mu_rule, prec, tol, stat, tracker, rho, admm_iters)


def rapidpt_maxnull_seeded(X, ell: int, L: int, r: int, eta_ppm: int, passes: int, seed: int, **kw):
    """Alg. 2 end to end with every relabelling, sampled set and the start
    basis drawn from the seed inside the library (NULL inputs of
    rpt_rapidpt_maxnull).  L counts all columns (l training + L - l
    recovered); |Omega| = sample_count(v, eta_ppm).  Keyword arguments as
    rapidpt_maxnull.  Returns what rapidpt_maxnull returns."""
    k = sample_count(X.shape[0], eta_ppm)
    opts = dict(batch=1, gamma=1.0, mu_rule="mean_gap", prec="split_bf16", tol=0.0, stat="t", tracker="grouse",
                rho=1.0, admm_iters=30)
    opts.update(kw)
    return _rapidpt_call(X, (None,) * 6, int(ell), int(L) - int(ell), int(r), k, passes, seed, **opts)


def _rapidpt_call(X, inputs, ell, L_rec, r, k, passes, seed, batch, gamma, mu_rule, prec, tol, stat, tracker,
                  rho, admm_iters):
    lib = _lib.load()
    v, n, ldx = _data(X)
    train_labels, rec_labels, U0, omega_train, omega_sm, omega_rec = inputs
    batch = int(batch)
    dev = X.device
    h = torch.empty(ell + L_rec, dtype=torch.float32, device=dev)
    U = torch.empty((v, r), dtype=torch.float32, device=dev)
    sm = torch.empty(2, dtype=torch.float32, device=dev)
    tinfo = torch.empty(ell, dtype=torch.int32, device=dev)
    rinfo = torch.empty(L_rec, dtype=torch.int32, device=dev)
    obj = torch.empty(max(passes, 1), dtype=torch.float64, device=dev)
    used = torch.empty(1, dtype=torch.int32, device=dev)
    nbytes = lib.rpt_rapidpt_workspace(v, n, ell, L_rec, r, k, PREC[prec])
    if any(t is None for t in (train_labels, rec_labels, omega_train, omega_sm, omega_rec)):
        nbytes += lib.rpt_rapidpt_gen_workspace(n, ell, L_rec, k, passes)
    ws = _workspace(nbytes, dev)
    rc = lib.rpt_rapidpt_maxnull(_ptr(X), v, n, ldx, n // 2, _ptr(train_labels), ell, _ptr(rec_labels), L_rec,
                                 _ptr(U0), r, _ptr(omega_train), k, passes, batch, float(gamma), float(tol),
                                 _ptr(omega_sm), _ptr(omega_rec), int(seed), MU_RULE[mu_rule], PREC[prec],
                                 STAT[stat], _tracker(tracker, rho, admm_iters), _ptr(h),
                                 _ptr(U), _ptr(sm), _ptr(tinfo), _ptr(rinfo), _ptr(obj), _ptr(used), _ptr(ws),
                                 ws.numel(), _stream(dev))
    _lib.check(rc, "rpt_rapidpt_maxnull")
    return h, {"U": U, "sigma_mu": sm, "train_max": h[:ell], "info": tinfo, "objective": obj[:passes],
               "passes_used": used}, rinfo


def sample_count(v: int, eta_ppm: int) -> int:
    """|Omega| = ceil(eta v) for eta = eta_ppm / 10^6 (integer arithmetic)."""
    k = _lib.load().rpt_sample_count(int(v), int(eta_ppm))
    if k < 0:
        raise ValueError("v must be >= 0 and eta_ppm in [0, 10^6]")
    return int(k)


def gen_relabellings(seed: int, row0: int, L: int, n: int, n1: int, device=None):
    """Relabellings row0 .. row0 + L - 1 drawn from the seed: (L, n) uint8 on
    the device, n1 ones per row."""
    device = torch.device(device or "cuda")
    out = torch.empty((L, n), dtype=torch.uint8, device=device)
    rc = _lib.load().rpt_gen_relabellings(int(seed), int(row0), int(L), int(n), int(n1), _ptr(out), _stream(device))
    _lib.check(rc, "rpt_gen_relabellings")
    return out


def gen_sampled_sets(seed: int, set_id: int, row0: int, rows: int, v: int, k: int, device=None):
    """Sampled sets row0 .. row0 + rows - 1 of set set_id drawn from the seed:
    (rows, k) int32 on the device, ascending distinct voxel indices."""
    device = torch.device(device or "cuda")
    out = torch.empty((rows, k), dtype=torch.int32, device=device)
    rc = _lib.load().rpt_gen_sampled_sets(int(seed), int(set_id), int(row0), int(rows), int(v), int(k), _ptr(out),
                                          _stream(device))
    _lib.check(rc, "rpt_gen_sampled_sets")
    return out


def gen_start_basis(seed: int, v: int, r: int, device=None):
    """The (v, r) FP32 Gaussian matrix that Rand. Orth. orthonormalises."""
    device = torch.device(device or "cuda")
    out = torch.empty((v, r), dtype=torch.float32, device=device)
    rc = _lib.load().rpt_gen_start_basis(int(seed), int(v), int(r), _ptr(out), _stream(device))
    _lib.check(rc, "rpt_gen_start_basis")
    return out


def masked_loss_fwd(U, W, omega_ptr, omega_idx, t_vals):
    """f = 1/2 sum (t - U W)^2 over the CSR sampled entries.  Returns
    (loss (1,) float64 on the device, resid (nnz,) float32)."""
    lib = _lib.load()
    v, r = U.shape
    B = W.shape[1]
    nnz = omega_idx.numel()
    loss = torch.empty(1, dtype=torch.float64, device=U.device)
    resid = torch.empty(nnz, dtype=torch.float32, device=U.device)
    rc = lib.rpt_masked_loss_fwd(_ptr(U), v, r, _ptr(W), B, _ptr(omega_ptr), _ptr(omega_idx), _ptr(t_vals), nnz,
                                 _ptr(loss), _ptr(resid), _stream(U.device))
    _lib.check(rc, "rpt_masked_loss_fwd")
    return loss, resid


def masked_loss_bwd(U, W, omega_ptr, omega_idx, resid, grad_scale=None):
    """Gradient of the masked loss: (dU (v, r), dW (r, B)), both multiplied
    by ``grad_scale`` (a float64 device scalar) when given."""
    lib = _lib.load()
    v, r = U.shape
    B = W.shape[1]
    nnz = omega_idx.numel()
    dU = torch.empty_like(U)
    dW = torch.empty_like(W)
    gs = None if grad_scale is None else _dev(grad_scale.reshape(1), torch.float64, "grad_scale", 1)
    rc = lib.rpt_masked_loss_bwd(_ptr(U), v, r, _ptr(W), B, _ptr(omega_ptr), _ptr(omega_idx), _ptr(resid), nnz,
                                 _ptr(dU), _ptr(dW), _ptr(gs), _stream(U.device))
    _lib.check(rc, "rpt_masked_loss_bwd")
    return dU, dW


def autotune_naive(X, labels, n1: int | None = None, prec: str = "split_bf16", reps: int = 3, T=None) -> int:
    """Times the NaivePT contraction's candidate voxel-chunk counts on this
    shape and keeps the fastest in the library's plan table (synchronises).
    With T (an (L, v) float32 GPU scratch tensor) the T-writing launch is
    tuned instead of the max-only one."""
    lib = _lib.load()
    v, n, ldx = _data(X)
    labels = _dev(labels, torch.uint8, "labels", 2).contiguous()
    L = labels.shape[0]
    n1 = n // 2 if n1 is None else int(n1)
    ws = _workspace(lib.rpt_naive_workspace(v, n, L, PREC[prec]), X.device)
    chosen = C.c_int32(0)
    if T is not None:
        T = _dev(T, torch.float32, "T", 2)
        if tuple(T.shape) != (L, v) or not T.is_contiguous():
            raise ValueError("T must be a contiguous (L, v) tensor")
    rc = lib.rpt_autotune_naive(_ptr(X), v, n, ldx, n1, _ptr(labels), L, PREC[prec], _ptr(T), int(reps), _ptr(ws),
                                ws.numel(), _stream(X.device), C.byref(chosen))
    _lib.check(rc, "rpt_autotune_naive")
    return chosen.value


def autotune_recover(v: int, r: int, L_rec: int, reps: int = 2, device=None) -> int:
    """Times the fused reconstruction's candidate voxel-chunk counts for
    (v, r, L_rec) and keeps the fastest in the plan table (synchronises)."""
    lib = _lib.load()
    device = torch.device("cuda") if device is None else device
    ws = _workspace(lib.rpt_autotune_recover_workspace(v, r, L_rec), device)
    chosen = C.c_int32(0)
    rc = lib.rpt_autotune_recover(v, r, L_rec, int(reps), _ptr(ws), ws.numel(), _stream(device), C.byref(chosen))
    _lib.check(rc, "rpt_autotune_recover")
    return chosen.value


def autotune_save(path: str) -> int:
    """Writes the plan table as text; returns the number of entries."""
    n = _lib.load().rpt_autotune_save(str(path).encode())
    if n < 0:
        raise OSError(f"cannot write {path}")
    return n


def autotune_load(path: str) -> int:
    """Reads a plan table written by autotune_save; returns the number of entries."""
    n = _lib.load().rpt_autotune_load(str(path).encode())
    if n < 0:
        raise OSError(f"cannot read {path}")
    return n


def autotune_clear() -> None:
    _lib.load().rpt_autotune_clear()


def autotune_count() -> int:
    return _lib.load().rpt_autotune_count()
