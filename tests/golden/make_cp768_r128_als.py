"""Writes cp768_r128_als.json: the FP64 oracle's CP-ALS on the 768^3 rank-128
slice-scaled workload (20 sweeps from the seeded initial factors), summarised
as the final fit, lambda and the model at 512 sampled entries.

Calls only the oracle (and the seeded input generators).  Run from the
repository root:  python tests/golden/make_cp768_r128_als.py
(about 4 minutes on 8 cores)."""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2411_04785_amd import synth  # noqa: E402

SWEEPS = 20
SAMPLE_SEED = 768128


def sample_indices(dims, n_slices=8, per_slice=64, seed=SAMPLE_SEED):
    """(i, j, k) of the sampled model entries: n_slices slices, per_slice
    (j, k) pairs each (shared by the writer and the tests)."""
    g = np.random.default_rng(seed)
    I, J, K = dims
    si = np.sort(g.choice(I, n_slices, replace=False))
    jk = g.integers(0, [J, K], size=(n_slices, per_slice, 2))
    return si, jk


def main():
    w = synth.WORKLOADS["cp768_r128_sliced"]
    t0 = time.time()
    X = synth.tensor(w)
    init = synth.init_factors(w)
    print(f"tensor in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    facs, lam, _ = oracle.cp_als(X, init, SWEEPS, fit_every_sweep=False)
    print(f"{SWEEPS} sweeps in {time.time() - t0:.1f} s", flush=True)
    fit = oracle.fit(X, facs, lam)
    si, jk = sample_indices(w.dims)
    model = []
    for s, i in enumerate(si):
        sl = oracle.reconstruct_slices(facs, lam, int(i), int(i) + 1)[0]
        model.append([float(sl[j, k]) for j, k in jk[s]])
    out = {
        "workload": w.name, "dims": list(w.dims), "R": w.R, "sweeps": SWEEPS,
        "what": "FP64 oracle CP-ALS (LU normal-equation solves, modes 1->2->3, lambda = column 2-norms) "
                "from synth.init_factors; fit = 1 - ||X - Xhat||_F / ||X||_F on the FP32 tensor",
        "fit": fit, "lambda": [float(v) for v in lam],
        "sample_seed": SAMPLE_SEED, "sample_slices": [int(i) for i in si],
        "sample_jk": jk.tolist(), "model_at_samples": model,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cp768_r128_als.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"fit {fit:.9f} -> {path}", flush=True)


if __name__ == "__main__":
    main()
