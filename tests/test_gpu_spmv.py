"""GPU parity of the CSR SpMV and residual kernels against the oracle, for
row lengths that select every scheme (the staged short-row scheme with its
long-block fallback, and the lanes-per-row widths: empty rows, stencils,
27-entry banded rows, long rows), plus the fused squared norm.  Rows of more
than 8 entries on average run with and without the column-window plan (x
staged in LDS per 512-row block when the block's window fits, else gathered):
y must be bit-identical either way (each row's sum is formed the same way)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2409_15468_amd as cb
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def random_rows(n, avg, seed):
    rng = np.random.default_rng(seed)
    lens = rng.poisson(avg, n)
    lens[rng.random(n) < 0.05] = 0
    rows = np.repeat(np.arange(n), lens)
    cols = rng.integers(0, n, rows.size)
    M = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(n, n))
    M.sum_duplicates()
    M.sort_indices()
    return synth.CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data)


def skewed(n, seed):
    """Mostly 2-entry rows with a few 600-entry rows: short on average (the
    staged scheme) but with 64-row blocks longer than its 512-entry stage,
    which take the one-lane-per-row path."""
    rng = np.random.default_rng(seed)
    lens = np.full(n, 2)
    lens[rng.choice(n, 8, replace=False)] = 600
    rows = np.repeat(np.arange(n), lens)
    cols = rng.integers(0, n, rows.size)
    M = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(n, n))
    M.sum_duplicates()
    M.sort_indices()
    return synth.CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data)


MATRICES = {
    "cd2d": lambda: synth.convection_diffusion(40, 2, (20.0, 0.0)),
    "cd3d": lambda: synth.convection_diffusion(17, 3, (10.0, 5.0, 2.0)),
    "banded": lambda: synth.banded_random(n=3001, half_band=300, seed=3).A,
    "sparse1": lambda: random_rows(2000, 1.0, 1),
    "long64": lambda: random_rows(700, 140.0, 2),
    "mid20": lambda: random_rows(1500, 20.0, 3),
    "skewed": lambda: skewed(3001, 4),
    "banded50k": lambda: synth.banded_random(n=50000, half_band=1000, seed=7).A,
    "wide20": lambda: random_rows(20000, 20.0, 6),  # windows wider than the LDS stage: gathers
    "mid12": lambda: random_rows(2500, 12.0, 8),  # 8 lanes per row
    "mid45": lambda: random_rows(2600, 45.0, 9),  # 32 lanes per row
    "wide45": lambda: random_rows(9000, 45.0, 10),  # 32 lanes per row, gathers
}


@pytest.mark.parametrize("plan", [True, False])
@pytest.mark.parametrize("name", list(MATRICES))
def test_spmv_and_residual(name, plan):
    A = MATRICES[name]()
    rng = np.random.default_rng(5)
    x = rng.standard_normal(A.n)
    b = rng.standard_normal(A.n)
    Ad = cb.DeviceCSR.from_host(A.row_ptr, A.col, A.val)
    xd, bd = torch.from_numpy(x).cuda(), torch.from_numpy(b).cuda()
    n2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    y = cb.cb_spmv(Ad, xd, norm2=n2, plan=plan).cpu().numpy()
    y_other = cb.cb_spmv(Ad, xd, plan=not plan).cpu().numpy()
    np.testing.assert_array_equal(y.view(np.uint64), y_other.view(np.uint64))
    y_or = oracle.spmv(A, x)
    scale = abs(A.scipy()) @ np.abs(x)
    assert np.all(np.abs(y - y_or) <= 1e-14 * scale + 1e-300)
    assert abs(n2.item() - oracle.dot(y_or, y_or)) <= 1e-13 * oracle.dot(y_or, y_or)
    r = cb.cb_residual(Ad, bd, xd, norm2=n2, plan=plan).cpu().numpy()
    r_or = b - y_or
    assert np.all(np.abs(r - r_or) <= 1e-14 * (scale + np.abs(b)))
    assert abs(n2.item() - oracle.dot(r_or, r_or)) <= 1e-13 * oracle.dot(r_or, r_or)
