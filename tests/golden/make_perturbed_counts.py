"""Write the oracle's iteration counts under last-bit perturbations of the
right-hand side, for the parity cases whose basis keeps at most 16 bits per
value (float16, frsz2 with l <= 16).

Such bases amplify differences in the last bit of the FP64 reductions: two
correct implementations that sum in different orders follow trajectories that
part after a few hundred steps, and so does the oracle itself when b moves by
one unit in its last place.  For each case this script records the oracle's
count on the unperturbed system and on K perturbed copies
b_k = b * (1 + 2^-52 s_k), s_k drawn entry-wise from {-1, 0, +1} by
numpy.random.default_rng(0) in sequence.  The GPU tests accept a count outside
2% of the unperturbed oracle's only if it lies within 2% of the range these
counts span.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_perturbed_counts.py
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
OUT = os.path.join(HERE, "perturbed_counts.json")


def digest(A, b, x0=None) -> str:
    h = hashlib.sha256(A.sha256().encode() + np.ascontiguousarray(b).tobytes())
    if x0 is not None:
        h.update(np.ascontiguousarray(x0).tobytes())
    return h.hexdigest()


def counts(solve, b, K):
    rng = np.random.default_rng(0)
    ref = solve(b).iterations
    pert = [solve(b * (1 + 2.0 ** -52 * rng.choice([-1.0, 0.0, 1.0], b.size))).iterations for _ in range(K)]
    return ref, pert


def main():
    cases = {}
    t0 = time.time()

    # the plain configuration: 2D convection-diffusion 64x64, GMRES(50), 1e-10
    s = synth.plain_2d(N=64, seed=0)
    for fmt in ["float16", "frsz2_16", "frsz2_8", "frsz2_12", "frsz2b64_16"]:
        ref, pert = counts(lambda bb: oracle.gmres(s.A, bb, 50, 1e-10, fmt, max_iters=4000), s.b, 6)
        cases[f"plain64_m50/{fmt}"] = {"oracle": ref, "perturbed": pert, "inputs_sha256": digest(s.A, s.b)}
        print(fmt, ref, sorted(pert), f"{time.time() - t0:.0f}s", flush=True)

    # Jacobi-preconditioned, column-scaled 48x48 operator, GMRES(60), 1e-10
    sc = synth.column_scaled(synth.plain_2d(N=48, seed=0), decades=3.0)
    d = oracle.jacobi(sc.A)
    for fmt in ["float16", "frsz2_16"]:
        ref, pert = counts(lambda bb: oracle.gmres(sc.A, bb, 60, 1e-10, fmt, dinv=d), sc.b, 8)
        cases[f"precond48_m60/{fmt}"] = {"oracle": ref, "perturbed": pert, "inputs_sha256": digest(sc.A, sc.b)}
        print("precond", fmt, ref, sorted(pert), f"{time.time() - t0:.0f}s", flush=True)

    # probing, then GMRES(40) from the 15-step probe's iterate (plain system)
    for fmt in ["float16", "frsz2_16"]:
        pr = oracle.auto_probe(s.A, s.b, np.zeros(s.A.n), fmt, 15, 1e-10)
        ref, pert = counts(lambda bb: oracle.gmres(s.A, bb, 40, 1e-10, fmt, x0=pr.x), s.b, 6)
        cases[f"auto_plain64_p15_m40/{fmt}"] = {"oracle": ref, "perturbed": pert,
                                               "inputs_sha256": digest(s.A, s.b)}
        print("auto", fmt, ref, sorted(pert), f"{time.time() - t0:.0f}s", flush=True)

    # probing with one candidate on the ragged 17^3 system, then GMRES(25)
    A = synth.convection_diffusion(17, 3, (10.0, 5.0, 2.0))
    rng = np.random.default_rng(11)
    b = synth.rhs_from_solution(A, rng.uniform(-1, 1, A.n))
    x0 = rng.standard_normal(A.n) * 0.1
    for fmt in ["float16", "frsz2_16"]:
        pr = oracle.auto_probe(A, b, x0, fmt, 9, 1e-9)
        ref, pert = counts(lambda bb: oracle.gmres(A, bb, 25, 1e-9, fmt, x0=pr.x), b, 6)
        cases[f"auto_cd3d17_p9_m25/{fmt}"] = {"oracle": ref, "perturbed": pert,
                                             "inputs_sha256": digest(A, b, x0)}
        print("auto17", fmt, ref, sorted(pert), f"{time.time() - t0:.0f}s", flush=True)

    # served requests (the first 24 of the seeded stream with n <= 40^3) that
    # the serving test checks against the oracle: those with n <= 10^4 and a
    # basis of at most 16 bits per value
    for r in synth.serving_requests(count=24, seed=4, n_max=40 ** 3):
        if r.n > 10000 or r.fmt not in ("float16", "frsz2_16"):
            continue
        sy = r.system()
        ref, pert = counts(lambda bb: oracle.gmres(sy.A, bb, r.m, r.tol, r.fmt), sy.b, 6)
        cases[f"served24_r{r.rid}/{r.fmt}"] = {"oracle": ref, "perturbed": pert,
                                              "inputs_sha256": digest(sy.A, sy.b)}
        print("served", r.rid, r.fmt, ref, sorted(pert), f"{time.time() - t0:.0f}s", flush=True)

    out = {
        "recipe": "b_k = b * (1 + 2^-52 s_k), s_k in {-1,0,1}^n from numpy default_rng(0) drawn in sequence; "
                  "'oracle' is the unperturbed count, 'perturbed' the K perturbed counts",
        "cases": cases,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
