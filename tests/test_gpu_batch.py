"""The one-workgroup batched solver (cbgmres_solve_batch) against the oracle:
every format reaches its relative residual with iteration counts within 2% of
the oracle's, the basis columns of the first cycle follow the oracle's cycle
step by step and are valid FRSZ2 / cast streams, a system's result is
bit-identical alone and inside a mixed batch, and the method's edge cases and
argument errors behave as in cbgmres_solve."""
import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb
import synth
from tests._golden import count_agrees, inputs_digest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
FORMATS = list(oracle.FORMATS)
UNIT = {"float64": 2.0 ** -53, "float32": 2.0 ** -24, "float16": 2.0 ** -11,
        "frsz2_16": 2.0 ** -14, "frsz2_21": 2.0 ** -19, "frsz2_32": 2.0 ** -30}


def within_2pct(a, b):
    return abs(a - b) <= max(1, int(np.ceil(0.02 * b)))


def host_rrn(A, b, x):
    return np.linalg.norm(b - A.scipy() @ x) / np.linalg.norm(b)


def device_system(A, b, x0=None):
    Ad = cb.DeviceCSR.from_host(A.row_ptr, A.col, A.val)
    bd = torch.from_numpy(np.ascontiguousarray(b, np.float64)).cuda()
    xd = torch.zeros(A.n, dtype=torch.float64, device="cuda") if x0 is None else \
        torch.from_numpy(np.array(x0, np.float64)).cuda()
    return Ad, bd, xd


def batch(systems, **kw):
    """systems: list of (A, b, m, tol, fmt[, x0]); returns (results, xs, workspaces)."""
    dev, wss = [], []
    for s in systems:
        A, b, m, tol, fmt = s[:5]
        x0 = s[5] if len(s) > 5 else None
        Ad, bd, xd = device_system(A, b, x0)
        dev.append((Ad, bd, xd, m, tol, fmt))
        wss.append(torch.empty(cb.cbgmres_batch_workspace_bytes(A.n, m, fmt), dtype=torch.uint8,
                               device="cuda"))
    res = cb.cbgmres_solve_batch(dev, workspaces=wss, **kw)
    torch.cuda.synchronize()
    return res, [d[2].cpu().numpy() for d in dev], wss


def random_dd(n, seed, per_row=5):
    """Random nonsymmetric, strictly diagonally dominant CSR with ragged n."""
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(n):
        cols = set(rng.integers(0, n, per_row).tolist()) - {i}
        cols = sorted(cols | {i})
        v = rng.uniform(-1, 1, len(cols))
        d = cols.index(i)
        v[d] = 1.5 * (np.abs(v).sum() - abs(v[d])) + 1.0
        rows.append((cols, v))
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(c) for c, _ in rows])
    col = np.concatenate([np.array(c, np.int32) for c, _ in rows])
    val = np.concatenate([v for _, v in rows])
    return synth.CSR(n, rp, col, val)


def test_limits():
    assert cb.cbgmres_batch_max_n() >= 16384
    assert cb.cbgmres_batch_max_restart() >= 100
    assert cb.cbgmres_batch_workspace_bytes(4096, 50, "frsz2_32") > 51 * 4096 * 4
    assert cb.cbgmres_batch_workspace_bytes(cb.cbgmres_batch_max_n() + 1, 50, "float64") == -1
    assert cb.cbgmres_batch_workspace_bytes(100, cb.cbgmres_batch_max_restart() + 1, "float64") == -1


def test_plain_config_all_formats_one_batch():
    """2D convection-diffusion 64x64, GMRES(50), tol 1e-10, all six formats in
    one launch."""
    s = synth.plain_2d(N=64, seed=0)
    res, xs, _ = batch([(s.A, s.b, 50, 1e-10, f) for f in FORMATS])
    ref64 = oracle.gmres(s.A, s.b, 50, 1e-10, "float64")
    for fmt, r, x in zip(FORMATS, res, xs):
        ref = oracle.gmres(s.A, s.b, 50, 1e-10, fmt)
        err = np.linalg.norm(x - ref64.x) / np.linalg.norm(ref64.x)
        print(f"{fmt}: batch iters={r['iterations']} cycles={r['restarts']} reorths={r['reorths']} | "
              f"oracle iters={ref.iterations}; err vs fp64 oracle={err:.2e}")
        assert r["status"] == 0 and r["converged"]
        assert host_rrn(s.A, s.b, x) <= 1e-10 * (1 + 1e-6)
        # see the multi-workgroup solver's test: an 11- or 15-bit basis may
        # land in the oracle's stored spread under last-bit perturbations of b
        assert count_agrees(r["iterations"], ref.iterations, "plain64_m50", fmt, inputs_digest(s.A, s.b)), \
            (fmt, r["iterations"], ref.iterations)
        assert err < 1e-6


def _columns(ws, fmt, n, m, ncols):
    """The basis columns a batch item left in its workspace."""
    stride = cb.cb_basis_column_bytes(fmt, n)
    data = oracle.col_bytes(oracle.FORMATS[fmt], n)
    ew = cb.cb_basis_exponent_words(fmt, n)
    raw = ws.cpu().numpy()
    eoff = ((m + 1) * stride + 255) // 256 * 256
    cols = []
    for c in range(ncols):
        vals = raw[c * stride: c * stride + data]
        exps = raw[eoff + 4 * c * ew: eoff + 4 * (c + 1) * ew].view(np.uint32) if ew else \
            np.zeros(1, np.uint32)
        cols.append((vals, exps))
    return cols


@pytest.mark.parametrize("fmt", FORMATS)
def test_first_cycle_columns_follow_oracle(fmt):
    """Stop after 12 steps of the first cycle; the 12 stored columns decode to
    the oracle cycle's D(Q(v_i)) up to a few storage units (the two
    trajectories differ only in FP64 rounding order), and every stored column
    is a valid stream: encoding its decoded values gives the same bytes."""
    A = synth.convection_diffusion(37, 2, (20.0, 0.0))  # n = 1369: ragged tail
    b = synth.rhs_from_solution(A, np.random.default_rng(5).uniform(-1, 1, A.n))
    m, k = 40, 12
    res, xs, wss = batch([(A, b, m, 1e-14, fmt)], max_iters=k)
    assert res[0]["status"] == cb.CB_ERR_NOT_CONVERGED and res[0]["iterations"] == k
    cyc = oracle.gmres_cycle(A, b, float(np.linalg.norm(b)), m, fmt, max_steps=k)
    assert cyc.steps == k
    for c, (vals, exps) in enumerate(_columns(wss[0], fmt, A.n, m, k)):
        dec = oracle.basis_decode(fmt, vals, exps, A.n)
        ref = cyc.Vdec[:, c]
        scale = np.abs(ref).max()
        assert np.abs(dec - ref).max() <= (8 * UNIT[fmt] + 1e-11) * scale, (fmt, c)
        v2, e2, _ = oracle.basis_encode(fmt, dec)
        assert np.array_equal(v2, vals), (fmt, c)
        if oracle.FORMATS[fmt] >= 3:
            assert np.array_equal(e2, exps), (fmt, c)


def test_alone_equals_mixed():
    """Each system of a mixed batch (sizes, formats, restarts, tolerances)
    gives bit-identically the x and statistics it gives alone."""
    specs = [(16, 2, "frsz2_32", 30, 1e-8), (45, 2, "frsz2_16", 64, 1e-10), (33, 2, "float32", 100, 1e-12),
             (64, 2, "frsz2_21", 50, 1e-9), (10, 3, "float16", 40, 1e-8), (17, 3, "frsz2_32", 77, 1e-11),
             (25, 3, "float64", 104, 1e-10), (100, 2, "frsz2_16", 35, 1e-9), (7, 3, "frsz2_21", 1, 1e-6)]
    systems = []
    for i, (N, d, fmt, m, tol) in enumerate(specs):
        A = synth.convection_diffusion(N, d, (20.0, 0.0) if d == 2 else (10.0, 5.0, 2.0))
        b = synth.rhs_from_solution(A, np.random.default_rng(100 + i).uniform(-1, 1, A.n))
        systems.append((A, b, m, tol, fmt))
    res_mix, xs_mix, _ = batch(systems, max_iters=5000)
    for s, r, x in zip(systems, res_mix, xs_mix):
        r1, x1, _ = batch([s], max_iters=5000)
        assert np.array_equal(x.view(np.uint64), x1[0].view(np.uint64))
        for k in ("iterations", "restarts", "reorths", "status", "rel_residual"):
            assert r[k] == r1[0][k], k
        assert r["converged"] and host_rrn(s[0], s[1], x) <= s[3] * (1 + 1e-6)


def test_many_systems_per_workgroup():
    """More systems than workgroups: each workgroup solves several in turn."""
    systems = []
    for i in range(300):
        N = 8 + i % 13
        A = synth.convection_diffusion(N, 2, (20.0, 0.0))
        b = synth.rhs_from_solution(A, np.random.default_rng(i).uniform(-1, 1, A.n))
        systems.append((A, b, 20, 1e-9, FORMATS[i % 6]))
    res, xs, _ = batch(systems)
    for s, r, x in zip(systems, res, xs):
        assert r["converged"] and host_rrn(s[0], s[1], x) <= 1e-9 * (1 + 1e-6)
    for i in (0, 77, 299):
        r1, x1, _ = batch([systems[i]])
        assert np.array_equal(xs[i].view(np.uint64), x1[0].view(np.uint64))


@pytest.mark.parametrize("fmt", ["float64", "frsz2_21"])
@pytest.mark.parametrize("n,m", [(1, 3), (33, 4), (100, 1), (1000, 25), (5000, 104)])
def test_ragged_sizes_and_restarts(fmt, n, m):
    A = random_dd(n, seed=n)
    b = np.random.default_rng(n + 1).standard_normal(n)
    tol = 1e-10
    res, xs, _ = batch([(A, b, m, tol, fmt)], max_iters=3000)
    ref = oracle.gmres(A, b, m, tol, fmt, max_iters=3000)
    assert res[0]["converged"] == ref.converged
    assert ref.converged
    assert host_rrn(A, b, xs[0]) <= tol * (1 + 1e-6)
    assert within_2pct(res[0]["iterations"], ref.iterations), (res[0]["iterations"], ref.iterations)


def test_edge_cases():
    A = synth.convection_diffusion(10, 2, (20.0, 0.0))
    b = synth.rhs_from_solution(A, np.random.default_rng(1).uniform(-1, 1, A.n))
    xs_exact = np.linalg.solve(A.scipy().toarray(), b)
    I = synth.CSR(100, np.arange(101, dtype=np.int32), np.arange(100, dtype=np.int32), np.ones(100))
    bb = np.random.default_rng(2).standard_normal(100)
    bn = b.copy()
    bn[3] = np.nan
    res, xs, _ = batch([(A, np.zeros(A.n), 10, 1e-10, "frsz2_32", np.ones(A.n)),   # b = 0
                        (A, b, 10, 1e-8, "frsz2_32", xs_exact),                   # x0 exact
                        (I, bb, 10, 1e-12, "float64"),                            # A = I
                        (A, bn, 5, 1e-10, "frsz2_16")])                           # NaN in b
    assert res[0]["converged"] and res[0]["iterations"] == 0 and np.all(xs[0] == 0)
    assert res[1]["converged"] and res[1]["iterations"] == 0
    assert res[2]["iterations"] == 1 and res[2]["converged"]
    np.testing.assert_allclose(xs[2], bb, rtol=1e-14)
    assert res[3]["status"] == cb.CB_ERR_NONFINITE
    # iteration cap, as the oracle counts it
    res, xs, _ = batch([(A, b, 5, 1e-14, "float64")], max_iters=12)
    ref = oracle.gmres(A, b, 5, 1e-14, "float64", max_iters=12)
    assert res[0]["status"] == cb.CB_ERR_NOT_CONVERGED and res[0]["iterations"] == 12 == ref.iterations


def test_literal_breakdown_option():
    s = synth.plain_2d(N=16)
    res, xs, _ = batch([(s.A, s.b, 30, 1e-10, "float64")], literal_breakdown=True)
    ref = oracle.gmres(s.A, s.b, 30, 1e-10, literal_breakdown=True)
    assert res[0]["converged"] and within_2pct(res[0]["iterations"], ref.iterations)
    assert res[0]["breakdowns"] == ref.breakdowns


def test_argument_errors():
    A = synth.convection_diffusion(8, 2, (20.0, 0.0))
    Ad, bd, xd = device_system(A, np.ones(A.n))
    with pytest.raises(cb.CbError) as e:
        cb.cbgmres_solve_batch([(Ad, bd, xd, cb.cbgmres_batch_max_restart() + 1, 1e-8, "float64")],
                               workspaces=[torch.empty(1 << 20, dtype=torch.uint8, device="cuda")])
    assert e.value.status == cb.CB_ERR_INVALID_ARG
    with pytest.raises(cb.CbError) as e:
        cb.cbgmres_solve_batch([(Ad, bd, xd, 10, 1e-8, "float64")],
                               workspaces=[torch.empty(64, dtype=torch.uint8, device="cuda")])
    assert e.value.status == cb.CB_ERR_WORKSPACE
    with pytest.raises(cb.CbError) as e:
        cb.cbgmres_solve_batch([(Ad, bd, xd, 10, -1.0, "float64")])
    assert e.value.status == cb.CB_ERR_INVALID_ARG
    big = synth.convection_diffusion(300, 2, (20.0, 0.0))  # n = 90000 > the batch limit
    Ab, bb, xb = device_system(big, np.ones(big.n))
    with pytest.raises(cb.CbError) as e:
        cb.cbgmres_solve_batch([(Ab, bb, xb, 10, 1e-8, "float64")],
                               workspaces=[torch.empty(1 << 20, dtype=torch.uint8, device="cuda")])
    assert e.value.status == cb.CB_ERR_INVALID_ARG
    assert cb.cbgmres_solve_batch([]) == []
