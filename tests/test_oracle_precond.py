"""Pins of the oracle's right-preconditioned GMRES (Fig. 1 steps 3 and 17 with
M = diag(A), Jacobi) and of its Jacobi set-up (CPU only)."""
import numpy as np
import pytest

import oracle
import synth


def pow2_diag_system(N=24, seed=8):
    """The plain 2D operator with its diagonal replaced by powers of two, so
    that M^-1 and A M^-1 are exact in floating point."""
    s = synth.plain_2d(N=N, seed=seed)
    A = s.A
    rng = np.random.default_rng(seed)
    k = rng.integers(3, 7, A.n)
    val = A.val.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    diag = A.col == rows
    val[diag] = np.ldexp(1.0, k[rows[diag]])
    A2 = synth.CSR(A.n, A.row_ptr, A.col, val)
    return A2, synth.rhs_from_solution(A2, s.x_star), k


def test_jacobi_definition():
    A, _, k = pow2_diag_system()
    d = oracle.jacobi(A)
    assert np.array_equal(d, np.ldexp(1.0, -k))
    # missing, zero, non-finite and negative diagonals
    row_ptr = np.array([0, 2, 3, 5, 6], np.int32)
    col = np.array([0, 1, 0, 1, 2, 3], np.int32)
    val = np.array([-3.0, 1.0, 2.0, 5.0, 0.0, np.inf])
    d = oracle.jacobi(synth.CSR(4, row_ptr, col, val))
    assert d[0] == 1.0 / -3.0 and d[1] == 1.0 and d[2] == 1.0 and d[3] == 1.0


@pytest.mark.parametrize("fmt", ["float64", "frsz2_21", "float16"])
def test_right_preconditioning_is_gmres_on_a_minv(fmt):
    """With M^-1 exact, preconditioned GMRES on A equals plain GMRES on
    A M^-1 step for step (bit-identical residual history), and x = M^-1 u."""
    A, b, _ = pow2_diag_system()
    d = oracle.jacobi(A)
    Ahat = synth.CSR(A.n, A.row_ptr, A.col, A.val * d[A.col])
    pc = oracle.gmres(A, b, 20, 1e-9, fmt, dinv=d, hist_cap=3000, max_iters=600)
    pl = oracle.gmres(Ahat, b, 20, 1e-9, fmt, hist_cap=3000, max_iters=600)
    assert pc.iterations == pl.iterations and pc.restarts == pl.restarts
    assert np.array_equal(pc.history, pl.history)
    assert np.array_equal(pc.x, d * pl.x)
    assert pc.rel_residual == pl.rel_residual


def test_identity_preconditioner_is_the_plain_solve():
    s = synth.plain_2d(N=20, seed=2)
    a = oracle.gmres(s.A, s.b, 15, 1e-10, "frsz2_32", dinv=np.ones(s.A.n), hist_cap=999)
    b = oracle.gmres(s.A, s.b, 15, 1e-10, "frsz2_32", hist_cap=999)
    assert a.iterations == b.iterations and np.array_equal(a.x, b.x) and np.array_equal(a.history, b.history)


def test_first_cycle_is_the_preconditioned_krylov_minimum():
    """After p steps from x0, x minimises ||b - A x|| over
    x0 + M^-1 K_p(A M^-1, r0); brute force with a dense least-squares solve."""
    s = synth.column_scaled(synth.plain_2d(N=12, seed=5), decades=2.0)
    A = s.A.scipy().toarray()
    d = oracle.jacobi(s.A)
    AM = A * d[None, :]
    x0 = np.random.default_rng(3).standard_normal(s.A.n)
    r0 = s.b - A @ x0
    for p in (1, 5, 10):
        K = np.empty((s.A.n, p))
        v = r0 / np.linalg.norm(r0)
        for i in range(p):
            K[:, i] = v
            v = AM @ v
            v -= K[:, :i + 1] @ (K[:, :i + 1].T @ v)
            v -= K[:, :i + 1] @ (K[:, :i + 1].T @ v)
            v /= np.linalg.norm(v)
        c, *_ = np.linalg.lstsq(AM @ K, r0, rcond=None)
        best = np.linalg.norm(r0 - AM @ K @ c) / np.linalg.norm(s.b)
        r = oracle.gmres(s.A, s.b, p, 1e-15, "float64", x0=x0, max_iters=p, dinv=d)
        assert r.iterations == p
        assert r.rel_residual == pytest.approx(best, rel=1e-8)


def test_jacobi_undoes_column_scaling():
    """On a column-scaled operator A S, Jacobi gives A S (diag(A) S)^-1 =
    A diag(A)^-1: the preconditioned solve takes the unscaled system's steps
    (up to rounding), while the plain solve needs many more."""
    base = synth.plain_2d(N=24, seed=1)
    s = synth.column_scaled(base, decades=3.0)
    d = oracle.jacobi(s.A)
    pc = oracle.gmres(s.A, s.b, 30, 1e-10, "float64", dinv=d)
    ref = oracle.gmres(base.A, base.b, 30, 1e-10, "float64")
    plain = oracle.gmres(s.A, s.b, 30, 1e-10, "float64", max_iters=3 * ref.iterations)
    assert pc.converged and abs(pc.iterations - ref.iterations) <= max(2, ref.iterations // 50)
    assert not plain.converged or plain.iterations > 2 * ref.iterations
    rrn = np.linalg.norm(s.b - s.A.scipy() @ pc.x) / np.linalg.norm(s.b)
    assert rrn <= 1e-10 * (1 + 1e-9)
