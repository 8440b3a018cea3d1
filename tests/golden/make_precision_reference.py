"""Write the oracle's reference for the precision workload: the random banded
system of n = 2^22 rows (27 distinct columns per row within +-1000 of the
diagonal, off-diagonals U(-1,1), diagonal 1.2 x the absolute row sum, seed 3;
x* ~ U(-1,1) from the same stream, b = A x*), solved to 1e-12 by

* FP64 iterative refinement around one cycle of GMRES(100) with a frsz2_16
  basis and inner tolerance 1e-4 (the precision form), and
* plain GMRES(100) with a float64 basis,

each with its outer steps / restarts, Arnoldi steps, final explicit relative
residual, error against x* and the solution at 4096 fixed rows.  Calls only
the oracle and the seeded input generator; takes a few minutes.

    python tests/golden/make_precision_reference.py
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
OUT = os.path.join(HERE, "precision_oracle.json")
N = 1 << 22
SAMPLE = np.unique(np.linspace(0, N - 1, 4096).astype(np.int64))


def main():
    t0 = time.time()
    s = synth.banded_random(n=N, per_row=27, half_band=1000, seed=3)
    digest = hashlib.sha256(s.A.sha256().encode() + s.b.tobytes()).hexdigest()
    print(f"inputs {time.time() - t0:.0f}s", flush=True)
    xs = s.x_star
    out = {"workload": "banded random n=2^22, 27 nnz/row within +-1000, seed 3; tol 1e-12",
           "inputs_sha256": digest, "sample_rows": SAMPLE.tolist()}

    t = time.time()
    ir = oracle.ir_solve(s.A, s.b, 100, 1e-4, 1e-12, "frsz2_16")
    out["ir_frsz2_16"] = {
        "m": 100, "inner_tol": 1e-4, "outer": ir.outer, "iterations": ir.iterations,
        "converged": ir.converged, "rel_residual": ir.rel_residual,
        "err_vs_xstar": float(np.linalg.norm(ir.x - xs) / np.linalg.norm(xs)),
        "oracle_seconds": time.time() - t, "x_sample": [float(v) for v in ir.x[SAMPLE]]}
    print("ir", ir.outer, ir.iterations, ir.rel_residual, f"{time.time() - t:.0f}s", flush=True)

    t = time.time()
    r = oracle.gmres(s.A, s.b, 100, 1e-12, "float64")
    out["gmres_float64"] = {
        "m": 100, "restarts": r.restarts, "iterations": r.iterations, "reorths": r.reorths,
        "converged": r.converged, "rel_residual": r.rel_residual,
        "err_vs_xstar": float(np.linalg.norm(r.x - xs) / np.linalg.norm(xs)),
        "oracle_seconds": time.time() - t, "x_sample": [float(v) for v in r.x[SAMPLE]]}
    print("f64", r.restarts, r.iterations, r.rel_residual, f"{time.time() - t:.0f}s", flush=True)
    out["ir_vs_float64_rel_diff"] = float(np.linalg.norm(ir.x - r.x) / np.linalg.norm(r.x))
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
