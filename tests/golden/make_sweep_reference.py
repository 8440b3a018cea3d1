"""Write the oracle's reference results for the basis-format sweep workload
(3D convection-diffusion on a 100^3 grid, n = 10^6, GMRES(100), tol 1e-10):
iterations, restarts, re-orthogonalisation count, final explicit relative
residual and the solution sampled at 4096 fixed rows, one JSON file per
basis format.  Calls only the oracle (and the seeded input generator).

    python tests/golden/make_sweep_reference.py frsz2_32 [float64 ...]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SAMPLE = np.unique(np.linspace(0, 10 ** 6 - 1, 4096).astype(np.int64))


def main(formats):
    s = synth.sweep_3d(N=100, seed=1)
    digest = hashlib.sha256(s.A.sha256().encode() + s.b.tobytes()).hexdigest()
    for fmt in formats:
        t = time.time()
        r = oracle.gmres(s.A, s.b, 100, 1e-10, fmt, hist_cap=100000)
        out = {
            "workload": "cd3d N=100 beta=(10,5,2) seed=1, GMRES(100), tol 1e-10",
            "format": fmt,
            "inputs_sha256": digest,
            "iterations": r.iterations,
            "restarts": r.restarts,
            "reorths": r.reorths,
            "breakdowns": r.breakdowns,
            "converged": r.converged,
            "rel_residual": r.rel_residual,
            "err_vs_xstar": float(np.linalg.norm(r.x - s.x_star) / np.linalg.norm(s.x_star)),
            "oracle_seconds": time.time() - t,
            "sample_rows": SAMPLE.tolist(),
            "x_sample": [float(v) for v in r.x[SAMPLE]],
            "history_every_10": [float(v) for v in r.history[::10]],
        }
        with open(os.path.join(HERE, f"sweep_oracle_{fmt}.json"), "w") as f:
            json.dump(out, f)
        print(fmt, r.iterations, r.restarts, r.rel_residual, f"{time.time() - t:.0f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(oracle.FORMATS))
