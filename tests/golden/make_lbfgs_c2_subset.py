"""Write lbfgs_c2_subset.json: the float64 oracle's L-BFGS on the 100^3 workload.

The problem is the 100^3 / ell_max 8 / 100x100 x 8-segment workload (twisted
fibre phantom, radius 45, mu = 1e-3) restricted to every tenth of its 240
projections (24 projections, 6 rotations per tilt), with 1% Gaussian noise of
the subset's largest clean value.  Starting from c = 0 the oracle runs 50
iterations of L-BFGS (m = 10, exact line search of the quadratic loss; paper
section 3.5, "Optimization").  Stored: the loss and relative residual after
every iteration, the final relative residual recomputed from an explicit
forward projection, the norm of the result and its values at 4096 seeded
flat indices.

Only the oracle and the shared input generators are used.  Run from the
repository root:  python tests/golden/make_lbfgs_c2_subset.py  (minutes).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import tt_inputs  # noqa: E402
from oracle import phantom  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lbfgs_c2_subset.json")
SUBSET_STEP = 10
ITERS = 50
N_SAMPLES = 4096
SAMPLE_SEED = 77


def problem():
    """(geometry, workload, float32-representable data) of the subset problem."""
    w = tt_inputs.WORKLOADS["c2"]
    inner, outer = tt_inputs.angles(w)
    sel = np.arange(0, w.n_proj, SUBSET_STEP)
    og = oracle.Geometry(w.n, w.ell_max, inner[sel], outer[sel], w.nj, w.nk, w.n_seg,
                         tt_inputs.lab_frame(), n_sub=w.n_sub, step=w.step)
    c_true = phantom.phantom_coeffs(w)
    data, _ = phantom.noisy_data(og, w, c_true)
    return og, w, data.astype(np.float32).astype(np.float64)


def sample_indices(n_total):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n_total, N_SAMPLES, replace=False))


def main():
    og, w, data = problem()
    t0 = time.time()
    c, it, hist, final_rel = oracle.lbfgs(og, np.zeros(og.vol_shape), data, None, w.mu, m=10, max_iter=ITERS)
    idx = sample_indices(c.size)
    rec = {
        "citation": "paper section 3.5 (Optimization): L-BFGS on the squared loss with L2 regularisation; "
                    "written by tests/golden/make_lbfgs_c2_subset.py from the float64 oracle",
        "workload": "c2 (100^3, ell_max 8, 100x100 x 8 segments, mu 1e-3), projections 0, 10, ..., 230",
        "subset_step": SUBSET_STEP, "iterations": int(it), "m": 10,
        "loss": hist[:, 0].tolist(), "rel_residual": hist[:, 1].tolist(),
        "final_rel_residual_explicit": float(final_rel),
        "c_norm": float(np.linalg.norm(c)),
        "sample_seed": SAMPLE_SEED, "sample_values": c.reshape(-1)[idx].tolist(),
        "oracle_seconds": time.time() - t0, "oracle_threads": oracle.max_threads(),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f)
    print("wrote", OUT, "iterations", it, "final rel residual", final_rel, f"{time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
