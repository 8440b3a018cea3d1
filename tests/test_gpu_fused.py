"""GPU parity of the first Gram-Schmidt update fused with the second
projection (cb_cgs_subtract_project, Fig. 1 steps 5b, 6 and 8) against the
oracle, fed the same stored basis, h and w (lockstep at the kernel level):

* w' = w - D(V) h within 1e-14 of the oracle relative to |w| + sum_i |h_i v_ik|
  per row;
* u = D(V)^T w' within 1e-12 of the oracle's projection of the oracle's w',
  relative to sum_k |v_ik w'_k| (the Hessenberg tolerance), plus the
  difference the tolerated w' error can make (sum_k |v_ik| |dw'_k|);
* ||w'||^2 within 1e-13.

Cases cover every kernel format (float64 and the generic widths use the
narrow projection path), single and many column groups, ragged tails, row
counts below and above one 2048-row group per workgroup, and launches whose
grid is rounded down to whole rounds of resident workgroups."""
import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FORMATS = ["frsz2_32", "frsz2_21", "frsz2_16", "float32", "float16", "frsz2b64_16", "frsz2b64_32",
           "float64", "frsz2_12", "frsz2g_32"]


def stored_basis(fmt, n, j, seed):
    rng = np.random.default_rng(seed)
    V = cb.Basis.empty(fmt, n, j)
    dec = np.zeros((n, j), order="F")
    for c in range(j):
        x = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 0, n) / np.sqrt(n)
        cb.cb_basis_store(V, c, torch.from_numpy(x).cuda())
        vals, exps, _ = oracle.basis_encode(fmt, x)
        dec[:, c] = oracle.basis_decode(fmt, vals, exps, n)
    torch.cuda.synchronize()
    return V, dec


def check(fmt, n, j, seed):
    print(f"fused {fmt} n={n} j={j}", flush=True)
    V, dec = stored_basis(fmt, n, j, seed)
    rng = np.random.default_rng(seed + 1)
    w = rng.standard_normal(n)
    h = dec.T @ w * (1 + 1e-3 * rng.standard_normal(j))  # close to the projection, as in a step
    wd = torch.from_numpy(w).cuda()
    out = cb.cb_cgs_subtract_project(V, j, torch.from_numpy(h).cuda(), wd).cpu().numpy()
    w2 = wd.cpu().numpy()
    w2_or = oracle.cgs_subtract(dec, h, w)
    row_scale = np.abs(w) + np.abs(dec) @ np.abs(h)
    dw = np.abs(w2 - w2_or)
    assert np.all(dw <= 1e-14 * row_scale), np.max(dw / row_scale)
    u_or = oracle.cgs_project(dec, w2_or)
    scale = np.abs(dec).T @ np.abs(w2_or)
    slack = np.abs(dec).T @ (1e-14 * row_scale)
    err = np.abs(out[:j] - u_or)
    assert np.all(err <= 1e-12 * scale + slack), np.max(err / (1e-12 * scale + slack))
    nr = oracle.dot(w2_or, w2_or)
    assert abs(out[j] - nr) <= 1e-13 * nr + 2 * np.sqrt(nr) * np.linalg.norm(1e-14 * row_scale)
    del V


@pytest.mark.parametrize("fmt", FORMATS)
@pytest.mark.parametrize("n,j", [(777, 3), (2048 * 5 + 13, 17), (2048 * 33, 9), (2048 * 40 + 77, 1),
                                 (2048 * 50 + 5, 60), (2048 * 36 + 31, 101), (2048 * 33 + 7, 105)])
def test_fused_update_projection(fmt, n, j):
    check(fmt, n, j, seed=n + j)


@pytest.mark.parametrize("fmt", ["frsz2_16", "float16", "frsz2b64_16", "frsz2_32"])
def test_fused_update_projection_whole_rounds(fmt):
    """Above 2^21 rows there are more row groups than workgroups (at most
    1024), and the grid is rounded down to whole rounds of the workgroups the
    GPU holds at once: 768 for the 16-bit formats (three per CU), so each
    workgroup loops over one or two row groups and the last one is ragged;
    frsz2_32 (two per CU) keeps 1024."""
    check(fmt, 2048 * 1100 + 37, 5, seed=11)


def test_fused_matches_separate_update_and_projection():
    """The fused call equals cb_cgs_subtract followed by cb_cgs_project on
    the updated w, up to their summation orders (1e-13 relative)."""
    n, j = 2048 * 40 + 3, 50
    V, dec = stored_basis("frsz2_32", n, j, 5)
    rng = np.random.default_rng(6)
    w = torch.from_numpy(rng.standard_normal(n)).cuda()
    h = torch.from_numpy(rng.standard_normal(j) * 1e-2).cuda()
    w_a = w.clone()
    out = cb.cb_cgs_subtract_project(V, j, h, w_a)
    w_b = w.clone()
    norm2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    cb.cb_cgs_subtract(V, j, h, w_b, norm2=norm2)
    u = cb.cb_cgs_project(V, j, w_b)
    torch.cuda.synchronize()
    np.testing.assert_allclose(w_a.cpu().numpy(), w_b.cpu().numpy(), rtol=0, atol=1e-13)
    np.testing.assert_allclose(out[:j].cpu().numpy(), u.cpu().numpy(), rtol=1e-11, atol=1e-13)
    assert abs(out[j].item() - norm2.item()) <= 1e-12 * norm2.item()
