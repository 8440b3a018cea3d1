"""Pins for the oracle's FP64 kernels and GMRES (CPU only).

The oracle is checked against exact rational arithmetic (dot products, SpMV),
LAPACK (numpy.linalg.solve / lstsq) on small systems, closed-form cases
(A = I, diagonal matrices with k distinct eigenvalues), the Arnoldi relation
and orthonormality of the basis, the minimal-residual property of GMRES over
the explicit Krylov space, the invariance of the whole iteration under
power-of-two scaling, and the stopping rule of Eq. 4.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

FORMATS = ["float64", "float32", "float16", "frsz2_16", "frsz2_21", "frsz2_32"]


def csr_from_dense(M):
    S = sp.csr_matrix(M)
    S.sort_indices()
    return synth.CSR(M.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                     S.data.astype(np.float64))


# ---------------------------------------------------------------- FP64 kernels
def test_dot_and_spmv_against_exact_rationals():
    rng = np.random.default_rng(0)
    a = rng.standard_normal(300) * 10.0 ** rng.uniform(-8, 8, 300)
    b = rng.standard_normal(300) * 10.0 ** rng.uniform(-8, 8, 300)
    exact = sum(Fraction(x) * Fraction(y) for x, y in zip(a, b))
    got = oracle.dot(a, b)
    absum = float(sum(abs(Fraction(x) * Fraction(y)) for x, y in zip(a, b)))
    u = 2.0 ** -53
    # compensated sum of correctly rounded products
    assert abs(Fraction(got) - exact) <= Fraction(2 * u * abs(float(exact)) + 2 * u * absum)
    assert oracle.nrm2(np.array([3.0, 4.0])) == 5.0
    A = synth.convection_diffusion(6, 2, (20.0, 0.0))
    x = rng.standard_normal(A.n)
    y = oracle.spmv(A, x)
    for i in range(A.n):
        terms = [Fraction(A.val[k]) * Fraction(x[A.col[k]]) for k in range(A.row_ptr[i], A.row_ptr[i + 1])]
        ex = sum(terms)
        s = float(sum(abs(t) for t in terms))
        assert abs(Fraction(y[i]) - ex) <= Fraction(4 * u * s)


def test_cgs_project_and_subtract():
    rng = np.random.default_rng(1)
    V = rng.standard_normal((500, 7))
    w = rng.standard_normal(500)
    h = oracle.cgs_project(V, w)
    np.testing.assert_allclose(h, V.T @ w, rtol=1e-13, atol=1e-13)
    w2 = oracle.cgs_subtract(V, h, w)
    np.testing.assert_allclose(w2, w - V @ h, rtol=1e-12, atol=1e-12)


def test_dense_solve_matches_lapack():
    rng = np.random.default_rng(2)
    M = rng.standard_normal((30, 30)) + 30 * np.eye(30)
    b = rng.standard_normal(30)
    np.testing.assert_allclose(oracle.dense_solve(M, b), np.linalg.solve(M, b), rtol=1e-12)


# ---------------------------------------------------------------- synthetic generators
def test_generators_shape_and_structure():
    for N in (4, 9, 64):
        A = synth.convection_diffusion(N, 2, (20.0, 0.0))
        assert A.nnz == 5 * N * N - 4 * N
    for N in (3, 10):
        A = synth.convection_diffusion(N, 3, (10.0, 5.0, 2.0))
        assert A.nnz == 7 * N ** 3 - 6 * N ** 2
        D = A.scipy().toarray()
        h = 1.0 / (N + 1)
        assert D[0, 0] == 6.0 and np.isclose(D[0, 1], -1 + 10 * h / 2) and np.isclose(D[1, 0], -1 - 10 * h / 2)
        assert np.isclose(D[0, N], -1 + 5 * h / 2) and np.isclose(D[0, N * N], -1 + 2 * h / 2)
    s = synth.banded_random(n=5000, half_band=100, seed=3)
    A = s.A
    assert A.nnz == 27 * 5000
    rows = np.repeat(np.arange(A.n), 27)
    assert np.all(np.abs(A.col.astype(np.int64) - rows) <= 100)
    D = A.scipy()
    diag = D.diagonal()
    off = np.asarray(abs(D).sum(axis=1)).ravel() - np.abs(diag)
    np.testing.assert_allclose(diag, 1.2 * off, rtol=1e-12)
    for i in range(0, A.n, 97):  # distinct sorted columns per row
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    assert synth.banded_random(n=5000, half_band=100, seed=3).A.sha256() == A.sha256()


# ---------------------------------------------------------------- GMRES
def test_tiny_full_gmres_matches_lapack():
    rng = np.random.default_rng(4)
    n = 40
    M = rng.standard_normal((n, n)) + 8 * np.eye(n)
    A = csr_from_dense(M)
    b = rng.standard_normal(n)
    r = oracle.gmres(A, b, m=n + 5, tol=1e-13, fmt="float64")
    xs = np.linalg.solve(M, b)
    kappa = np.linalg.cond(M)
    assert r.converged and r.restarts == 1
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) <= kappa * 1e-12


def test_identity_converges_in_one_step():
    n = 100
    A = csr_from_dense(np.eye(n))
    b = np.random.default_rng(5).standard_normal(n)
    c = oracle.gmres_cycle(A, b, oracle.nrm2(b), m=10, fmt="float64")
    assert c.steps == 1 and c.breakdown
    assert abs(c.Hraw[0, 0] - 1.0) < 1e-15 and c.Hraw[1, 0] < 1e-15
    r = oracle.gmres(A, b, m=10, tol=1e-12)
    assert r.converged and r.iterations == 1
    np.testing.assert_allclose(r.x, b, rtol=1e-14)


@pytest.mark.parametrize("k", [1, 3, 5, 8])
def test_diagonal_with_k_distinct_values(k):
    n = 400
    vals = np.linspace(1.0, 3.0, k)
    d = vals[np.arange(n) % k]
    A = csr_from_dense(np.diag(d))
    b = np.random.default_rng(k).uniform(-1, 1, n)
    r = oracle.gmres(A, b, m=20, tol=1e-11, fmt="float64")
    assert r.converged and r.iterations <= k
    np.testing.assert_allclose(r.x, b / d, rtol=1e-9)


def _small_system(N=12):
    A = synth.convection_diffusion(N, 2, (20.0, 0.0))
    b = synth.rhs_from_solution(A, np.random.default_rng(6).uniform(-1, 1, A.n))
    return A, b


def test_arnoldi_relation_and_orthonormality():
    A, b = _small_system()
    m = 25
    c = oracle.gmres_cycle(A, b, oracle.nrm2(b), m=m, fmt="float64")
    assert c.steps == m
    V = c.Vdec[:, :m + 1]
    H = c.Hraw
    Ad = A.scipy()
    # with a float64 basis the stored vectors are the FP64 v_j themselves
    AV = Ad @ V[:, :m]
    res = AV - V @ H
    scale = np.linalg.norm(Ad.toarray(), 2) + np.abs(H).sum()
    assert np.linalg.norm(res) <= 100 * 2.0 ** -52 * scale
    assert np.linalg.norm(V.T @ V - np.eye(m + 1)) <= 1e-12
    # the rotated H is upper triangular
    assert np.all(np.tril(c.R[:m, :m], -1) == 0)


PIN_IV_FORMATS = FORMATS + ["frsz2_12", "frsz2b64_16", "frsz2b64_32"]


@pytest.mark.parametrize("fmt", PIN_IV_FORMATS)
def test_arnoldi_relation_with_compressed_basis(fmt):
    """The Arnoldi relation of a compressed-basis cycle, with the FP64 v_j on
    the left and the decoded basis on the right:
        A v_j = sum_{i<=j} h_ij D(Q(v_i)) + h_{j+1,j} v_{j+1}
    to within c eps (||A|| + sum |h|).  It holds only if the SpMV of Fig. 1
    step 3 reads the FP64 v_j (step 3 is not a highlighted decode site), the
    Gram-Schmidt passes of steps 5 and 8 read the decoded columns, and the new
    vector is w / h_{j+1,j} in FP64 before it is encoded (steps 13-14).  Each
    stored column is Q(v_j) bit for bit and decodes to the column the cycle
    used.  The last part checks that the relation separates the readings: had
    the SpMV read D(Q(v_j)), or the projections the FP64 v_i, the residual
    would exceed the bound by orders of magnitude for every lossy format."""
    A, b = _small_system()
    m = 25
    c = oracle.gmres_cycle(A, b, oracle.nrm2(b), m=m, fmt=fmt)
    assert c.status == 0 and c.steps == m and not c.breakdown
    n = A.n
    Ad = A.scipy()
    normA = np.linalg.norm(Ad.toarray(), 2)
    eps = 2.0 ** -52
    f = oracle._fmt(fmt)
    cbytes = oracle.col_bytes(f, n)
    ew = oracle.exp_words(f, n)
    worst, gap_spmv, gap_proj = 0.0, np.inf, np.inf
    for j in range(m):
        v = c.Vfp[:, j]
        # stored column j is Q(v_j), and the cycle's decoded column is D(Q(v_j))
        vals, ex, bad = oracle.basis_encode(f, v)
        assert not bad
        assert np.array_equal(c.enc[j, :cbytes], vals)
        if ew:
            assert np.array_equal(c.exps[j, :ew], ex)
        assert np.array_equal(c.Vdec[:, j].view(np.uint64),
                              oracle.basis_decode(f, vals, ex, n).view(np.uint64))
        h = c.Hraw[:j + 2, j]
        rhs = c.Vdec[:, :j + 1] @ h[:j + 1] + h[j + 1] * c.Vfp[:, j + 1]
        res = np.linalg.norm(Ad @ v - rhs)
        bound = 10 * eps * (normA + np.abs(h).sum())
        worst = max(worst, res / bound)
        if f != 0:
            # the other readings: SpMV on the decoded vector, or projections
            # against the FP64 vectors
            alt_spmv = np.linalg.norm(Ad @ c.Vdec[:, j] - rhs)
            alt_proj = np.linalg.norm(Ad @ v - c.Vfp[:, :j + 1] @ h[:j + 1] - h[j + 1] * c.Vfp[:, j + 1])
            gap_spmv = min(gap_spmv, alt_spmv / bound)
            gap_proj = min(gap_proj, alt_proj / bound)
    assert worst <= 1.0, worst
    if f != 0:
        # the most accurate lossy formats, float32 and frsz2_32, miss the
        # bound by a factor of about 1e5 under either wrong reading
        assert gap_spmv > 1e3 and gap_proj > 1e3, (gap_spmv, gap_proj)


def test_implicit_residual_is_the_krylov_minimum():
    A, b = _small_system(10)
    beta = oracle.nrm2(b)
    m = 12
    c = oracle.gmres_cycle(A, b, beta, m=m, fmt="float64")
    Ad = A.scipy().toarray()
    # minimum of ||b - A K y|| over an orthonormal basis of the explicit Krylov
    # space span{b, Ab, ..., A^(j-1) b}, computed by LAPACK
    K = np.empty((A.n, m))
    q = b / np.linalg.norm(b)
    for j in range(m):
        K[:, j] = q
        q = Ad @ q
        q /= np.linalg.norm(q)
    for j in range(1, m + 1):
        Q, _ = np.linalg.qr(K[:, :j])
        y, *_ = np.linalg.lstsq(Ad @ Q, b, rcond=None)
        rmin = np.linalg.norm(b - Ad @ Q @ y)
        assert abs(c.gabs_hist[j - 1] - rmin) <= 1e-8 * beta
    assert np.all(np.diff(c.gabs_hist) <= 1e-15 * beta)  # never increases


@pytest.mark.parametrize("fmt", FORMATS)
def test_power_of_two_scaling_invariance(fmt):
    A, b = _small_system(10)
    r0 = oracle.gmres(A, b, m=15, tol=1e-10, fmt=fmt)
    t = 37
    As = synth.CSR(A.n, A.row_ptr, A.col, np.ldexp(A.val, t))
    r1 = oracle.gmres(As, np.ldexp(b, t), m=15, tol=1e-10, fmt=fmt)
    assert r0.iterations == r1.iterations
    assert np.array_equal(r0.x.view(np.uint64), r1.x.view(np.uint64))
    c0 = oracle.gmres_cycle(A, b, oracle.nrm2(b), m=15, fmt=fmt)
    c1 = oracle.gmres_cycle(As, np.ldexp(b, t), oracle.nrm2(np.ldexp(b, t)), m=15, fmt=fmt)
    np.testing.assert_array_equal(c0.enc, c1.enc)
    np.testing.assert_array_equal(c0.exps, c1.exps)


@pytest.mark.parametrize("fmt", FORMATS)
def test_plain_config_converges_to_tolerance(fmt):
    s = synth.plain_2d(N=32)
    r = oracle.gmres(s.A, s.b, m=50, tol=1e-10, fmt=fmt)
    assert r.converged and r.status == 0
    assert 0 < r.rel_residual <= 1e-10
    xr = oracle.spmv(s.A, r.x)
    assert np.linalg.norm(s.b - xr) / np.linalg.norm(s.b) <= 1.01e-10


def test_special_cases():
    A, b = _small_system(8)
    r = oracle.gmres(A, np.zeros(A.n), m=10, tol=1e-10)
    assert r.converged and r.iterations == 0 and np.all(r.x == 0)
    r = oracle.gmres(A, b, m=5, tol=1e-14, max_iters=12)
    assert not r.converged and r.status == 3 and r.iterations == 12
    # x0 already the solution to tolerance: zero iterations
    x0 = np.linalg.solve(A.scipy().toarray(), b)
    r = oracle.gmres(A, b, m=10, tol=1e-8, x0=x0)
    assert r.converged and r.iterations == 0
    # cycle cap
    r = oracle.gmres(A, b, m=5, tol=1e-14, max_cycles=2)
    assert r.restarts == 2 and r.iterations == 10 and r.rel_residual == -1.0
    # literal reading of step 12 ends cycles at least as early
    s = synth.plain_2d(N=16)
    lit = oracle.gmres(s.A, s.b, m=30, tol=1e-10, literal_breakdown=True)
    dflt = oracle.gmres(s.A, s.b, m=30, tol=1e-10)
    assert dflt.breakdowns == 0 and lit.breakdowns >= dflt.breakdowns
    assert lit.restarts >= dflt.restarts


def test_history_records_implicit_residuals():
    s = synth.plain_2d(N=16)
    r = oracle.gmres(s.A, s.b, m=20, tol=1e-10, hist_cap=10000)
    assert r.history.size == r.iterations
    assert r.history[-1] <= 1e-10 or r.restarts > 1
    assert abs(r.history[-1] - r.implicit_rel_residual) == 0


def test_iterative_refinement_precision_form():
    s = synth.banded_random(n=4096, half_band=200, seed=3)
    ir = oracle.ir_solve(s.A, s.b, m=100, inner_tol=1e-4, tol=1e-12, fmt="frsz2_16")
    assert ir.converged and ir.rel_residual <= 1e-12 and ir.outer >= 2
    ref = oracle.gmres(s.A, s.b, m=100, tol=1e-12, fmt="float64")
    assert ref.converged
    err = np.linalg.norm(ir.x - ref.x) / np.linalg.norm(ref.x)
    assert err <= 1e-10
    xs = np.linalg.norm(ir.x - s.x_star) / np.linalg.norm(s.x_star)
    assert xs <= 1e-10
