"""Writes train_full_n100_v250k.txt: the FP64 oracle's training half of Alg. 2
(Sec. 4.1: exact t maps of the l training relabellings, tracking passes over
their sampled entries, then sigma and mu from one more sampled pass) on the
full-size smoothed workload, n = 100 (50/50), v = 250,000, l = 300, r = 100,
eta = 0.35% (875 voxels per column), 10 passes with one mini-batch of l per
pass.  The inputs are the seeded ones of the benchmark step.

Stored: sigma, mu, the 300 training maxima, and the oracle basis U at 48
sampled voxels (the GPU test compares the projectors U_S U_S^T on them).

Run from the repository root:  python tests/golden/make_train_full.py
(about 5 minutes on one core; calls nothing but the oracle and the input
generators).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import rpt_synth as S  # noqa: E402
from oracle import rapidpt as OR  # noqa: E402
from oracle import tstat as OT  # noqa: E402

N, V, L, ELL, R, ETA_PPM, SEED, PASSES = 100, 250_000, 10_000, 300, 100, 3500, 2017, 10
N_SAMPLE = 48
OUT = os.path.join(ROOT, "tests", "golden", "train_full_n100_v250k.txt")


def sample_voxels():
    """The voxels whose basis rows are stored (seeded, sorted)."""
    return np.sort(np.random.default_rng(4242).choice(V, N_SAMPLE, replace=False))


def main():
    t0 = time.time()
    k = S.omega_count(V, ETA_PPM)
    X = S.smoothed_volumes(N, V, seed=1703).astype(np.float32).astype(np.float64)
    tl = S.relabellings(L, N, N // 2, seed=1506)[:ELL]
    U0 = S.gaussian_matrix(V, R, seed=3).astype(np.float32).astype(np.float64)
    omt = S.omega_sets(PASSES * ELL, V, k, seed=41)
    oms = S.omega_sets(ELL, V, k, seed=42)
    T = OT.tmatrix(X, tl)
    print(f"T_ex {time.time() - t0:.0f} s", flush=True)
    U = OR.train_subspace(T, U0, omt, PASSES, batch=ELL)
    print(f"tracking {time.time() - t0:.0f} s", flush=True)
    sigma, mu, _ = OR.sigma_mu(T, U, oms, SEED)
    sv = sample_voxels()
    with open(OUT, "w") as f:
        f.write("# Training half of Alg. 2 (Sec. 4.1) by the FP64 oracle, written by make_train_full.py.\n")
        f.write(f"# n={N} (50/50) v={V} l={ELL} r={R} k={k} passes={PASSES} batch={ELL} seed={SEED}\n")
        f.write(f"sigma {sigma:.17e}\n")
        f.write(f"mu {mu:.17e}\n")
        f.write("train_max " + " ".join(f"{x:.17e}" for x in T.max(axis=1)) + "\n")
        f.write("voxels " + " ".join(str(int(i)) for i in sv) + "\n")
        for i in sv:
            f.write("U " + " ".join(f"{x:.10e}" for x in U[i]) + "\n")
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)


def load():
    """Reads the stored values back: dict with sigma, mu, train_max, voxels, U_rows."""
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
            elif key == "train_max":
                out["train_max"] = np.array([float(x) for x in vals])
            else:
                out[key] = float(vals[0])
    out["U_rows"] = np.array(out["U_rows"])
    return out


if __name__ == "__main__":
    main()
