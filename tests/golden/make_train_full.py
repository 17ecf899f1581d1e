"""Writes train_full_n100_v250k.txt: the FP64 oracle's Alg. 2 end to end on
the benchmark's full-size smoothed workload, n = 100 (50/50), v = 250,000,
L = 10,000, l = 300, r = 100, eta = 0.35% (875 voxels per column).  Training
follows Sec. 4.1 as read: GROUSE one column at a time, passes repeated until
the stopping rule holds (tol 1e-3 on the pass objective) or 10 passes.  The
inputs are the seeded ones of the benchmark step.

Stored: the passes used and their objectives, sigma, mu, the 300 training
maxima, the oracle basis U at 48 sampled voxels (the GPU test compares the
projectors U_S U_S^T on them) and the whole max null h (10,000 values: the 300
exact maxima followed by the 9,700 recovered ones).

Run from the repository root:  python tests/golden/make_train_full.py
(about 10 minutes on eight cores; calls nothing but the oracle and the input
generators).
"""
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import rpt_synth as S  # noqa: E402
from oracle import rapidpt as OR  # noqa: E402
from oracle import tstat as OT  # noqa: E402

N, V, L, ELL, R, ETA_PPM, SEED, PASSES, TOL = 100, 250_000, 10_000, 300, 100, 3500, 2017, 10, 1e-3
N_SAMPLE = 48
OUT = os.path.join(ROOT, "tests", "golden", "train_full_n100_v250k.txt")

_G = {}


def sample_voxels():
    """The voxels whose basis rows are stored (seeded, sorted)."""
    return np.sort(np.random.default_rng(4242).choice(V, N_SAMPLE, replace=False))


def inputs():
    """The benchmark's seeded inputs (same generators and seeds as bench.py)."""
    k = S.omega_count(V, ETA_PPM)
    X = S.smoothed_volumes(N, V, seed=1703).astype(np.float32).astype(np.float64)
    labels = S.relabellings(L, N, N // 2, seed=1506)
    U0 = S.gaussian_matrix(V, R, seed=3).astype(np.float32).astype(np.float64)
    omt = S.omega_sets(PASSES * ELL, V, k, seed=41)
    oms = S.omega_sets(ELL, V, k, seed=42)
    omr = S.omega_sets(L - ELL, V, k, seed=43)
    return X, labels, U0, omt, oms, omr


def _init(X, labels, U, sigma, mu, omr):
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)  # one BLAS thread per worker process
    _G.update(X=X, labels=labels, U=U, sigma=sigma, mu=mu, omr=omr)


def _recover_range(j0_j1):
    j0, j1 = j0_j1
    return OR.recover(_G["X"], _G["labels"][ELL + j0:ELL + j1], _G["U"], _G["sigma"], _G["mu"],
                      _G["omr"][j0:j1], SEED, col0=ELL + j0)


def main():
    t0 = time.time()
    X, labels, U0, omt, oms, omr = inputs()
    T = OT.tmatrix(X, labels[:ELL])
    print(f"T_ex {time.time() - t0:.0f} s", flush=True)
    hist = []
    U = OR.train_subspace(T, U0, omt, PASSES, batch=1, tol=TOL, history=hist)
    print(f"tracking {time.time() - t0:.0f} s, {len(hist)} passes", flush=True)
    sigma, mu, tmax = OR.sigma_mu(T, U, oms, SEED)
    chunks = [(j, min(L - ELL, j + 250)) for j in range(0, L - ELL, 250)]
    parts = {}
    with mp.get_context("fork").Pool(min(8, os.cpu_count() or 1), initializer=_init,
                                     initargs=(X, labels, U, sigma, mu, omr)) as pool:
        for j, part in zip([c[0] for c in chunks], pool.imap(_recover_range, chunks)):
            parts[j] = part
            print(f"recovered columns {j}..{j + len(part)} at {time.time() - t0:.0f} s", flush=True)
    rec = np.concatenate([parts[c[0]] for c in chunks])
    print(f"recovery {time.time() - t0:.0f} s", flush=True)
    h = np.concatenate([tmax, rec])
    sv = sample_voxels()
    with open(OUT, "w") as f:
        f.write("# Alg. 2 end to end by the FP64 oracle, written by make_train_full.py.\n")
        f.write(f"# n={N} (50/50) v={V} L={L} l={ELL} r={R} k={S.omega_count(V, ETA_PPM)} batch=1 "
                f"passes<={PASSES} tol={TOL} seed={SEED}\n")
        f.write(f"passes_used {len(hist)}\n")
        f.write("objective " + " ".join(f"{x:.17e}" for x in hist) + "\n")
        f.write(f"sigma {sigma:.17e}\n")
        f.write(f"mu {mu:.17e}\n")
        f.write("train_max " + " ".join(f"{x:.17e}" for x in tmax) + "\n")
        f.write("h " + " ".join(f"{x:.9e}" for x in h) + "\n")
        f.write("voxels " + " ".join(str(int(i)) for i in sv) + "\n")
        for i in sv:
            f.write("U " + " ".join(f"{x:.10e}" for x in U[i]) + "\n")
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)


def load():
    """Reads the stored values back: dict with passes_used, objective, sigma,
    mu, train_max, h, voxels, U_rows."""
    out = {"U_rows": []}
    with open(OUT) as f:
        for line in f:
            if line.startswith("#"):
                continue
            key, *vals = line.split()
            if key == "U":
                out["U_rows"].append([float(x) for x in vals])
            elif key == "voxels":
                out["voxels"] = np.array([int(x) for x in vals], dtype=np.int64)
            elif key in ("train_max", "h", "objective"):
                out[key] = np.array([float(x) for x in vals])
            elif key == "passes_used":
                out[key] = int(vals[0])
            else:
                out[key] = float(vals[0])
    out["U_rows"] = np.array(out["U_rows"])
    return out


if __name__ == "__main__":
    main()
