"""Pins of the oracle's format-selection-by-probing (the autotuning of the
paper's conclusions, Section VIII) and of the library's host-side pick rule
against it (CPU only).

The rule: a probe's rate is ln(rel0 / rel) / seconds; the first candidate
with the highest rate wins.  Pinned by hand-computed cases; the probe itself
(GMRES(p) from x0, p steps) is pinned against the Krylov minimum computed by
brute force."""
import math

import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb
import synth


def test_rate_closed_forms():
    assert oracle.auto_rate(1.0, math.exp(-3.0), 1.5) == pytest.approx(2.0, rel=1e-15)
    assert oracle.auto_rate(1e-2, 1e-5, 2.0) == pytest.approx(math.log(1e3) / 2.0, rel=1e-15)
    assert oracle.auto_rate(1.0, 1.0, 1.0) == -math.inf         # no progress
    assert oracle.auto_rate(1.0, 2.0, 1.0) == -math.inf         # divergence
    assert oracle.auto_rate(1.0, math.nan, 1.0) == -math.inf
    assert oracle.auto_rate(1.0, math.inf, 1.0) == -math.inf
    assert oracle.auto_rate(1.0, 0.0, 1.0) == math.inf          # exact solution


def test_pick_hand_cases():
    e = math.exp
    # rates 2, 1.5, 3 -> the third
    assert oracle.auto_pick(1.0, [e(-2), e(-3), e(-3)], [1.0, 2.0, 1.0]) == 2
    # equal rates -> the first
    assert oracle.auto_pick(1.0, [0.5, 0.25], [1.0, 2.0]) == 0
    # a fast probe that did not converge loses to a slower one that did progress
    assert oracle.auto_pick(1.0, [1.0, 0.9], [0.001, 10.0]) == 1
    # nothing progressed: the first candidate
    assert oracle.auto_pick(1.0, [1.0, math.nan, 3.0], [1.0, 1.0, 1.0]) == 0
    # an exact solution wins whatever its time
    assert oracle.auto_pick(1.0, [1e-300, 0.0], [1e-9, 1e9]) == 1


def test_library_pick_rule_matches_oracle():
    """cb_auto_pick is pure host code: compared with the oracle's rule on
    seeded random cases, ties and non-finite residuals included."""
    rng = np.random.default_rng(5)
    for trial in range(400):
        k = int(rng.integers(1, 9))
        rel0 = float(10.0 ** rng.uniform(-3, 0))
        rel = rel0 * 10.0 ** rng.uniform(-4, 0.5, k)
        sec = 10.0 ** rng.uniform(-4, 0, k)
        if trial % 5 == 0:
            rel[rng.integers(0, k)] = math.nan
        if trial % 7 == 0:
            rel[:] = rel[0]
            sec[:] = sec[0]
        if trial % 11 == 0:
            rel[rng.integers(0, k)] = 0.0
        assert cb.cb_auto_pick(rel0, rel, sec) == oracle.auto_pick(rel0, list(rel), list(sec)), trial
    assert cb.lib().cb_auto_pick(1.0, None, None, 1) == -1
    assert cb.cb_auto_pick(1.0, [], []) == -1


def test_probe_is_the_krylov_minimum():
    """A float64 probe of p steps (no breakdown) lands on argmin ||b - A x||
    over x0 + K_p(A, r0); brute force with a dense least-squares solve."""
    s = synth.plain_2d(N=12, seed=3)
    A = s.A.scipy().toarray()
    rng = np.random.default_rng(1)
    x0 = rng.standard_normal(s.A.n)
    r0 = s.b - A @ x0
    for p in (1, 4, 9):
        K = np.empty((s.A.n, p))
        v = r0 / np.linalg.norm(r0)
        for i in range(p):  # Krylov vectors, orthonormalised for conditioning
            K[:, i] = v
            v = A @ v
            v -= K[:, :i + 1] @ (K[:, :i + 1].T @ v)
            v -= K[:, :i + 1] @ (K[:, :i + 1].T @ v)
            v /= np.linalg.norm(v)
        c, *_ = np.linalg.lstsq(A @ K, r0, rcond=None)
        best = np.linalg.norm(r0 - A @ K @ c) / np.linalg.norm(s.b)
        pr = oracle.auto_probe(s.A, s.b, x0, "float64", p, 1e-14)
        assert pr.iterations == p and pr.restarts == 1
        assert pr.rel_residual == pytest.approx(best, rel=1e-9)


def test_probe_replay_is_two_solves_in_sequence():
    """Probing then continuing equals a GMRES(p) run capped at p steps
    followed by GMRES(m) from its iterate: the probe's iterate is kept."""
    s = synth.plain_2d(N=16, seed=4)
    pr = oracle.auto_probe(s.A, s.b, np.zeros(s.A.n), "frsz2_21", 7, 1e-10)
    rest = oracle.gmres(s.A, s.b, 20, 1e-10, "frsz2_21", x0=pr.x)
    assert pr.iterations == 7 and rest.converged
    assert np.linalg.norm(s.b - s.A.scipy() @ rest.x) / np.linalg.norm(s.b) <= 1e-10 * (1 + 1e-9)
    # a probe that meets tol stops there
    loose = oracle.auto_probe(s.A, s.b, np.zeros(s.A.n), "float64", 200, 1e-3)
    assert loose.converged and loose.iterations < 200
