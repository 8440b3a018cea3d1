"""Trajectory parity of cbgmres_solve against the oracle's GMRES: every basis
format reaches its stated relative residual (checked again on the host), the
iteration count is within 2% of the oracle's, the error against the
FP64-basis oracle is reported, and the edge cases of the method behave as the
oracle does (b = 0, A = I, x0 exact, caps, non-finite input, tiny and ragged
n, GMRES(1)).  Solves are deterministic run to run."""
import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb
import synth
from tests._golden import count_agrees, inputs_digest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
FORMATS = list(oracle.FORMATS)
# unit of the stored representation: the relative truncation/rounding step
UNIT = {"float64": 2.0 ** -53, "float32": 2.0 ** -24, "float16": 2.0 ** -11,
        "frsz2_16": 2.0 ** -14, "frsz2_21": 2.0 ** -19, "frsz2_32": 2.0 ** -30}


def gpu_solve(A, b, m, tol, fmt, x0=None, **kw):
    Ad = cb.DeviceCSR.from_host(A.row_ptr, A.col, A.val)
    bd = torch.from_numpy(np.ascontiguousarray(b)).cuda()
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda") if x0 is None else \
        torch.from_numpy(np.array(x0, dtype=np.float64)).cuda()
    res, hist = cb.cbgmres_solve(Ad, bd, xd, m, tol, fmt, **kw)
    torch.cuda.synchronize()
    return res, xd.cpu().numpy(), hist


def within_2pct(a, b):
    return abs(a - b) <= max(1, int(np.ceil(0.02 * b)))


def host_rrn(A, b, x):
    return np.linalg.norm(b - A.scipy() @ x) / np.linalg.norm(b)


@pytest.mark.parametrize("fmt", FORMATS)
def test_plain_config_all_formats(fmt):
    """2D convection-diffusion 64x64, GMRES(50), tol 1e-10 (the plain
    configuration), every basis format."""
    s = synth.plain_2d(N=64, seed=0)
    res, x, hist = gpu_solve(s.A, s.b, 50, 1e-10, fmt, history_cap=5000)
    ref = oracle.gmres(s.A, s.b, 50, 1e-10, fmt, hist_cap=5000)
    ref64 = oracle.gmres(s.A, s.b, 50, 1e-10, "float64")
    print(f"{fmt}: gpu iters={res['iterations']} restarts={res['restarts']} reorths={res['reorths']} "
          f"| oracle iters={ref.iterations}; err vs fp64 oracle="
          f"{np.linalg.norm(x - ref64.x) / np.linalg.norm(ref64.x):.2e}")
    assert res["status"] == 0 and res["converged"]
    assert host_rrn(s.A, s.b, x) <= 1e-10 * (1 + 1e-6)
    assert 0 < res["rel_residual"] <= 1e-10
    # an 11- or 15-bit basis may instead land in the oracle's own spread under
    # last-bit perturbations of b (stored by golden/make_perturbed_counts.py)
    assert count_agrees(res["iterations"], ref.iterations, "plain64_m50", fmt, inputs_digest(s.A, s.b)), \
        (res["iterations"], ref.iterations)
    assert np.linalg.norm(x - ref64.x) / np.linalg.norm(ref64.x) < 1e-6
    # the implicit residual history follows the oracle's over the first cycle,
    # to within what the storage format's rounding lets trajectories drift
    k = min(40, hist.size, ref.history.size)
    np.testing.assert_allclose(hist[:k], ref.history[:k], rtol=max(1e-6, 64 * UNIT[fmt]))


def dominant_random(n, avg, seed):
    """About `avg` entries per row at random columns, U(-1, 1), plus a diagonal
    of twice the absolute row sum: a well-conditioned system whose steps run
    the windowed store + SpMV at 8 (avg 12) or 32 (avg 45) lanes per row."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    lens = rng.poisson(avg, n)
    rows = np.repeat(np.arange(n), lens)
    cols = rng.integers(0, n, rows.size)
    M = sp.csr_matrix((rng.uniform(-1.0, 1.0, rows.size), (rows, cols)), shape=(n, n))
    M.sum_duplicates()
    M = (M + sp.diags(2.0 * np.asarray(abs(M).sum(axis=1)).ravel() + 1.0)).tocsr()
    M.sort_indices()
    return synth.CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data)


@pytest.mark.parametrize("fmt", ["frsz2_32", "frsz2_16"])
@pytest.mark.parametrize("n,avg", [(2500, 12.0), (2600, 45.0), (9000, 45.0)])
def test_windowed_spmv_widths_solve(fmt, n, avg):
    """Solves whose SpMV takes 8 and 32 lanes per row, with the window of x
    staged (n <= 3072) or gathered (n = 9000): iterations within 2% of the
    oracle's and the residual met."""
    A = dominant_random(n, avg, seed=n)
    x_star = np.random.default_rng(n + 1).uniform(-1.0, 1.0, n)
    b = A.scipy() @ x_star
    res, x, _ = gpu_solve(A, b, 30, 1e-10, fmt)
    ref = oracle.gmres(A, b, 30, 1e-10, fmt)
    print(f"{fmt} n={n} avg={avg}: gpu iters={res['iterations']} | oracle iters={ref.iterations}")
    assert res["status"] == 0 and res["converged"]
    assert host_rrn(A, b, x) <= 1e-10 * (1 + 1e-6)
    assert within_2pct(res["iterations"], ref.iterations), (res["iterations"], ref.iterations)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-8


def test_solve_deterministic():
    s = synth.plain_2d(N=48, seed=7)
    r1, x1, _ = gpu_solve(s.A, s.b, 30, 1e-9, "frsz2_21")
    r2, x2, _ = gpu_solve(s.A, s.b, 30, 1e-9, "frsz2_21")
    assert r1["iterations"] == r2["iterations"]
    assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64))


def test_edge_cases():
    A = synth.convection_diffusion(10, 2, (20.0, 0.0))
    b = synth.rhs_from_solution(A, np.random.default_rng(1).uniform(-1, 1, A.n))
    # b = 0
    res, x, _ = gpu_solve(A, np.zeros(A.n), 10, 1e-10, "frsz2_32", x0=np.ones(A.n))
    assert res["converged"] and res["iterations"] == 0 and np.all(x == 0)
    # x0 already accurate
    xs = np.linalg.solve(A.scipy().toarray(), b)
    res, x, _ = gpu_solve(A, b, 10, 1e-8, "frsz2_32", x0=xs)
    assert res["converged"] and res["iterations"] == 0
    # A = I: one step, lucky breakdown
    I = synth.CSR(100, np.arange(101, dtype=np.int32), np.arange(100, dtype=np.int32), np.ones(100))
    bb = np.random.default_rng(2).standard_normal(100)
    res, x, _ = gpu_solve(I, bb, 10, 1e-12, "float64")
    assert res["iterations"] == 1 and res["converged"]
    np.testing.assert_allclose(x, bb, rtol=1e-14)
    # iteration cap
    res, x, _ = gpu_solve(A, b, 5, 1e-14, "float64", max_iters=12)
    ref = oracle.gmres(A, b, 5, 1e-14, "float64", max_iters=12)
    assert res["status"] == cb.CB_ERR_NOT_CONVERGED and res["iterations"] == 12 == ref.iterations
    # cycle cap: no explicit residual afterwards
    res, x, _ = gpu_solve(A, b, 5, 1e-14, "float64", max_cycles=2)
    assert res["restarts"] == 2 and res["iterations"] == 10 and res["rel_residual"] == -1.0
    # non-finite right-hand side
    bn = b.copy()
    bn[3] = np.nan
    res, x, _ = gpu_solve(A, bn, 5, 1e-10, "frsz2_16")
    assert res["status"] == cb.CB_ERR_NONFINITE


@pytest.mark.parametrize("fmt", ["float64", "frsz2_21"])
@pytest.mark.parametrize("N,m", [(3, 4), (5, 1), (23, 7), (47, 120)])
def test_small_ragged_and_restart_lengths(fmt, N, m):
    A = synth.convection_diffusion(N, 2, (20.0, 0.0))
    b = synth.rhs_from_solution(A, np.random.default_rng(N).uniform(-1, 1, A.n))
    tol = 1e-9
    res, x, _ = gpu_solve(A, b, m, tol, fmt, max_iters=3000)
    ref = oracle.gmres(A, b, m, tol, fmt, max_iters=3000)
    assert res["converged"] == ref.converged
    if ref.converged:
        assert host_rrn(A, b, x) <= tol * (1 + 1e-6)
        assert within_2pct(res["iterations"], ref.iterations), (res["iterations"], ref.iterations)


def test_literal_breakdown_option():
    s = synth.plain_2d(N=16)
    res, x, _ = gpu_solve(s.A, s.b, 30, 1e-10, "float64", literal_breakdown=True)
    ref = oracle.gmres(s.A, s.b, 30, 1e-10, literal_breakdown=True)
    assert res["converged"] and within_2pct(res["iterations"], ref.iterations)
    assert res["breakdowns"] == ref.breakdowns


def test_iterative_refinement_precision_form():
    s = synth.banded_random(n=20000, half_band=1000, seed=3)
    Ad = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    bd = torch.from_numpy(s.b).cuda()
    xd = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
    res = cb.cbgmres_ir_solve(Ad, bd, xd, 100, 1e-4, 1e-12, "frsz2_16")
    x = xd.cpu().numpy()
    ref = oracle.ir_solve(s.A, s.b, 100, 1e-4, 1e-12, "frsz2_16")
    ref64 = oracle.gmres(s.A, s.b, 100, 1e-12, "float64")
    assert res["converged"] and host_rrn(s.A, s.b, x) <= 1e-12 * (1 + 1e-6)
    assert res["restarts"] == ref.outer
    assert within_2pct(res["iterations"], ref.iterations)
    assert np.linalg.norm(x - ref64.x) / np.linalg.norm(ref64.x) < 1e-10


@pytest.mark.parametrize("fmt,inner_tol", [("frsz2_21", 1e-6), ("float16", 1e-3), ("frsz2b64_32", 1e-8)])
def test_iterative_refinement_other_inner_formats(fmt, inner_tol):
    """The refinement with other inner bases and inner tolerances: the same
    outer steps as the oracle, inner steps within 2%, FP64 accuracy."""
    s = synth.banded_random(n=12000, half_band=500, seed=5)
    Ad = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    bd = torch.from_numpy(s.b).cuda()
    xd = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
    res = cb.cbgmres_ir_solve(Ad, bd, xd, 60, inner_tol, 1e-12, fmt)
    x = xd.cpu().numpy()
    ref = oracle.ir_solve(s.A, s.b, 60, inner_tol, 1e-12, fmt)
    print(fmt, res["restarts"], res["iterations"], "| oracle", ref.outer, ref.iterations)
    assert res["converged"] and ref.converged
    assert host_rrn(s.A, s.b, x) <= 1e-12 * (1 + 1e-6)
    assert res["restarts"] == ref.outer
    assert within_2pct(res["iterations"], ref.iterations)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < 1e-10


def test_tall_system_short_restart():
    """n = 5e6 with GMRES(1): the norm of b uses one partial per 2048-row group
    (2442 of them), more than the projection partials of a restart length of
    1 need; the workspace holds both."""
    n = 5_000_000
    A = synth.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, 2.0))
    b = np.random.default_rng(9).standard_normal(n)
    assert cb.cbgmres_workspace_bytes(n, 1, "float64") >= 8 * ((n + 2047) // 2048)
    res, x, _ = gpu_solve(A, b, 1, 1e-12, "float64")
    assert res["converged"] and res["iterations"] == 1
    np.testing.assert_allclose(x, b / 2, rtol=1e-13)


@pytest.mark.parametrize("fmt", ["frsz2_21", "float32", "float64"])
@pytest.mark.parametrize("fuse", [1, 2])
def test_fused_and_separate_first_update(fmt, fuse):
    """The first Gram-Schmidt update run separately (fuse_updates=1) or fused
    with the speculative second projection (2) solves the plain configuration
    with the oracle's iteration count; the steps that do not need the second
    pass drop the speculative projection."""
    s = synth.plain_2d(N=64, seed=0)
    res, x, _ = gpu_solve(s.A, s.b, 50, 1e-10, fmt, fuse_updates=fuse)
    ref = oracle.gmres(s.A, s.b, 50, 1e-10, fmt)
    assert res["converged"] and host_rrn(s.A, s.b, x) <= 1e-10 * (1 + 1e-6)
    assert within_2pct(res["iterations"], ref.iterations), (res["iterations"], ref.iterations)
    assert abs(res["reorths"] - ref.reorths) <= max(2, int(0.02 * ref.reorths))


@pytest.mark.parametrize("l", [8, 12, 18, 24, 28])
def test_generic_width_solves(l):
    """FRSZ2 with other widths (the generic codec) on the plain configuration:
    tolerance met on the host, iterations within 2% of the oracle's (for
    l < 16, or within the oracle's own spread under last-bit perturbations of
    b, which coarse bases amplify), the first cycle's history alongside."""
    fmt = f"frsz2_{l}"
    s = synth.plain_2d(N=64, seed=0)
    res, x, hist = gpu_solve(s.A, s.b, 50, 1e-10, fmt, history_cap=5000, max_iters=4000)
    ref = oracle.gmres(s.A, s.b, 50, 1e-10, fmt, hist_cap=5000, max_iters=4000)
    print(f"{fmt}: gpu {res['iterations']} oracle {ref.iterations}")
    assert res["status"] == 0 and res["converged"]
    assert host_rrn(s.A, s.b, x) <= 1e-10 * (1 + 1e-6)
    assert count_agrees(res["iterations"], ref.iterations, "plain64_m50" if l < 16 else None, fmt,
                        inputs_digest(s.A, s.b)), (res["iterations"], ref.iterations)
    k = min(40, hist.size, ref.history.size)
    np.testing.assert_allclose(hist[:k], ref.history[:k], rtol=max(1e-6, 64 * 2.0 ** -(l - 2)))


@pytest.mark.parametrize("l", [16, 21])
def test_generic_codec_solve_is_the_specialised_solve(l):
    """At l = 16 and 21 the generic codec has the specialised tiles' lane map
    and summation order, so the whole solve is bit-identical."""
    s = synth.plain_2d(N=40, seed=6)
    r1, x1, h1 = gpu_solve(s.A, s.b, 30, 1e-10, f"frsz2_{l}", history_cap=2000)
    r2, x2, h2 = gpu_solve(s.A, s.b, 30, 1e-10, f"frsz2g_{l}", history_cap=2000)
    assert r1["iterations"] == r2["iterations"] and r1["reorths"] == r2["reorths"]
    assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64)) and np.array_equal(h1, h2)


@pytest.mark.parametrize("fmt", ["frsz2b64_16", "frsz2b64_32", "frsz2b64_21"])
def test_block64_solves(fmt):
    """Blocks of 64 values on the plain configuration: tolerance met on the
    host, iterations within 2% of the oracle's with the same block size (or,
    for the 16-bit code, within the oracle's spread under last-bit
    perturbations of b), the first cycle's history alongside."""
    s = synth.plain_2d(N=64, seed=0)
    res, x, hist = gpu_solve(s.A, s.b, 50, 1e-10, fmt, history_cap=5000)
    ref = oracle.gmres(s.A, s.b, 50, 1e-10, fmt, hist_cap=5000)
    print(f"{fmt}: gpu {res['iterations']} oracle {ref.iterations}")
    assert res["status"] == 0 and res["converged"]
    assert host_rrn(s.A, s.b, x) <= 1e-10 * (1 + 1e-6)
    assert count_agrees(res["iterations"], ref.iterations, "plain64_m50", fmt, inputs_digest(s.A, s.b)), \
        (res["iterations"], ref.iterations)
    l = int(fmt.split("_")[1])
    k = min(40, hist.size, ref.history.size)
    np.testing.assert_allclose(hist[:k], ref.history[:k], rtol=max(1e-6, 64 * 2.0 ** -(l - 2)))
