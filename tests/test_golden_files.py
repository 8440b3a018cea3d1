"""The stored oracle results under tests/golden are the oracle's (CPU only):
the perturbed iteration counts are reproduced for every stored case (the
unperturbed count and the first perturbed copy of b), and the inputs they were
computed from still hash to the stored digests."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests._golden import GOLDEN, inputs_digest, perturbed_cases


def _case_inputs(case):
    """(A, b, x0, solve(b) -> oracle result) for a stored case name."""
    if case.startswith("plain64_m50/"):
        fmt = case.split("/")[1]
        s = synth.plain_2d(N=64, seed=0)
        return s.A, s.b, None, lambda bb: oracle.gmres(s.A, bb, 50, 1e-10, fmt, max_iters=4000)
    if case.startswith("precond48_m60/"):
        fmt = case.split("/")[1]
        s = synth.column_scaled(synth.plain_2d(N=48, seed=0), decades=3.0)
        d = oracle.jacobi(s.A)
        return s.A, s.b, None, lambda bb: oracle.gmres(s.A, bb, 60, 1e-10, fmt, dinv=d)
    if case.startswith("auto_plain64_p15_m40/"):
        fmt = case.split("/")[1]
        s = synth.plain_2d(N=64, seed=0)
        pr = oracle.auto_probe(s.A, s.b, np.zeros(s.A.n), fmt, 15, 1e-10)
        return s.A, s.b, None, lambda bb: oracle.gmres(s.A, bb, 40, 1e-10, fmt, x0=pr.x)
    if case.startswith("auto_cd3d17_p9_m25/"):
        fmt = case.split("/")[1]
        A = synth.convection_diffusion(17, 3, (10.0, 5.0, 2.0))
        rng = np.random.default_rng(11)
        b = synth.rhs_from_solution(A, rng.uniform(-1, 1, A.n))
        x0 = rng.standard_normal(A.n) * 0.1
        pr = oracle.auto_probe(A, b, x0, fmt, 9, 1e-9)
        return A, b, x0, lambda bb: oracle.gmres(A, bb, 25, 1e-9, fmt, x0=pr.x)
    if case.startswith("served24_r"):
        rid = int(case.split("/")[0][len("served24_r"):])
        r = synth.serving_requests(count=24, seed=4, n_max=40 ** 3)[rid]
        s = r.system()
        return s.A, s.b, None, lambda bb: oracle.gmres(s.A, bb, r.m, r.tol, r.fmt)
    raise KeyError(case)


@pytest.mark.parametrize("case", sorted(perturbed_cases()))
def test_perturbed_counts_are_the_oracles(case):
    entry = perturbed_cases()[case]
    A, b, x0, solve = _case_inputs(case)
    assert inputs_digest(A, b, x0) == entry["inputs_sha256"]
    assert solve(b).iterations == entry["oracle"]
    rng = np.random.default_rng(0)
    b1 = b * (1 + 2.0 ** -52 * rng.choice([-1.0, 0.0, 1.0], b.size))
    assert solve(b1).iterations == entry["perturbed"][0]


def test_sweep_golden_inputs_match_the_generator():
    import hashlib
    s = synth.sweep_3d(N=100, seed=1)
    digest = hashlib.sha256(s.A.sha256().encode() + s.b.tobytes()).hexdigest()
    for fmt in ["float64", "float32", "float16", "frsz2_16", "frsz2_21", "frsz2_32"]:
        with open(os.path.join(GOLDEN, f"sweep_oracle_{fmt}.json")) as f:
            assert json.load(f)["inputs_sha256"] == digest, fmt


def test_microbench_golden_is_the_oracles_first_column():
    """The first column of the stored microbenchmark reference: its inputs,
    its frsz2_32 encoding hash and its projection are the oracle's."""
    import hashlib
    with open(os.path.join(GOLDEN, "microbench_oracle.json")) as f:
        ref = json.load(f)
    n = ref["n"]
    w = synth.basis_probe_vector(n, ref["seed"])
    assert hashlib.sha256(w.tobytes()).hexdigest() == ref["w_sha256"]
    col = next(synth.basis_columns(n, 1, ref["seed"]))
    assert hashlib.sha256(col.tobytes()).hexdigest() == ref["column_sha256"][0]
    exps, words, _ = oracle.frsz2_encode(col, 32)
    assert hashlib.sha256(words.tobytes() + exps.tobytes()).hexdigest() == ref["encoded_sha256"]["32"][0]
    assert oracle.dot(oracle.frsz2_decode(exps, words, n, 32), w) == ref["h"]["32"][0]
