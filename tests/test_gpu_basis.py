"""GPU parity of the fused basis kernels against the oracle, fed the same
inputs (lockstep at the kernel level):

* cb_basis_store: v = w / d by IEEE division and the stored column are
  bit-exact against numpy division and the oracle's encoder, all six formats
  and generic-codec FRSZ2 widths;
* cb_cgs_project: h = D(V)^T w within 1e-12 of the oracle, relative to
  sum_k |v_ik w_k| (the Hessenberg tolerance);
* cb_cgs_subtract / cb_basis_combine: w -/+= D(V) h within 1e-14 relative to
  |w| + sum_i |h_i v_ik| per row; the fused norm within 1e-13.
"""
import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb
from tests._inputs import mixed_vector

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def u32(t):
    return t.cpu().numpy().view(np.uint32)

FORMATS = list(oracle.FORMATS)
# generic-codec widths (frsz2g_32: the generic codec at l = 32)
GENERIC = ["frsz2_3", "frsz2_7", "frsz2_12", "frsz2_27", "frsz2g_32"]
# blocks of 64 values: the specialised l = 16, 32 and the generic codec
B64 = ["frsz2b64_16", "frsz2b64_32", "frsz2b64_21", "frsz2b64_5"]


def build_basis(fmt, n, j, seed):
    """j columns stored on the GPU from random unit-scale vectors; returns the
    GPU basis, the oracle's encoded bytes and decoded columns."""
    rng = np.random.default_rng(seed)
    V = cb.Basis.empty(fmt, n, j)
    enc, dec = [], np.zeros((n, j), order="F")
    for c in range(j):
        x = rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 0, n) / np.sqrt(n)
        cb.cb_basis_store(V, c, torch.from_numpy(x).cuda())
        vals, exps, _ = oracle.basis_encode(fmt, x)
        enc.append((vals, exps))
        dec[:, c] = oracle.basis_decode(fmt, vals, exps, n)
    torch.cuda.synchronize()
    return V, enc, dec


@pytest.mark.parametrize("fmt", FORMATS + GENERIC + B64)
@pytest.mark.parametrize("n", [777, 4101, 2048 * 5 + 13])
def test_store_bit_exact_with_division(fmt, n):
    w = mixed_vector(n, seed=n, spread=4)
    d = 3.0517578125e-3 * np.pi
    V = cb.Basis.empty(fmt, n, 3)
    wd = torch.from_numpy(w).cuda()
    dd = torch.tensor([d], dtype=torch.float64, device="cuda")
    vout = torch.empty(n, dtype=torch.float64, device="cuda")
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    cb.cb_basis_store(V, 2, wd, divisor=dd, v_out=vout, nonfinite_flag=flag)
    torch.cuda.synchronize()
    v = w / d
    assert np.array_equal(vout.cpu().numpy().view(np.uint64), v.view(np.uint64))
    vals, exps, bad = oracle.basis_encode(fmt, v)
    assert bad == bool(flag.item())  # float16 overflows on the largest entries
    np.testing.assert_array_equal(V.column(2).cpu().numpy(), vals)
    if V.exps is not None:
        np.testing.assert_array_equal(u32(V.column_exps(2)), exps)
    back = cb.cb_basis_load(V, 2).cpu().numpy()
    ref = oracle.basis_decode(fmt, vals, exps, n)
    assert np.array_equal(back.view(np.uint64), ref.view(np.uint64))


def test_store_float16_overflow_flag():
    V = cb.Basis.empty("float16", 64, 1)
    w = np.ones(64)
    w[5] = 7e4
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    cb.cb_basis_store(V, 0, torch.from_numpy(w).cuda(), nonfinite_flag=flag)
    assert int(flag.item()) == 1


@pytest.mark.parametrize("fmt", FORMATS + GENERIC + B64)
@pytest.mark.parametrize("n,j", [(777, 1), (4101, 5), (2048 * 5 + 13, 17), (3000, 70)])
def test_project_subtract_combine(fmt, n, j):
    V, enc, dec = build_basis(fmt, n, j, seed=n + j)
    for c in range(j):  # stored columns are bit-exact against the oracle
        np.testing.assert_array_equal(V.column(c).cpu().numpy(), enc[c][0])
    w = np.random.default_rng(j).standard_normal(n)
    wd = torch.from_numpy(w).cuda()
    h = cb.cb_cgs_project(V, j, wd).cpu().numpy()
    h_or = oracle.cgs_project(dec, w)
    scale = np.abs(dec).T @ np.abs(w)
    assert np.all(np.abs(h - h_or) <= 1e-12 * scale + 1e-300), np.max(np.abs(h - h_or) / scale)

    # update with the oracle's h fed to both sides
    hd = torch.from_numpy(h_or).cuda()
    norm2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    w2 = wd.clone()
    cb.cb_cgs_subtract(V, j, hd, w2, norm2=norm2)
    w2_or = oracle.cgs_subtract(dec, h_or, w)
    row_scale = np.abs(w) + np.abs(dec) @ np.abs(h_or)
    assert np.all(np.abs(w2.cpu().numpy() - w2_or) <= 1e-14 * row_scale)
    nr = oracle.dot(w2_or, w2_or)
    assert abs(norm2.item() - nr) <= 1e-13 * nr

    x = torch.from_numpy(w).cuda()
    cb.cb_basis_combine(V, j, hd, x)
    x_or = w + dec @ h_or
    assert np.all(np.abs(x.cpu().numpy() - x_or) <= 1e-14 * row_scale)


def test_project_is_deterministic():
    V, _, _ = build_basis("frsz2_21", 50000, 12, seed=1)
    w = torch.from_numpy(np.random.default_rng(2).standard_normal(50000)).cuda()
    h1 = cb.cb_cgs_project(V, 12, w).cpu().numpy()
    h2 = cb.cb_cgs_project(V, 12, w).cpu().numpy()
    assert np.array_equal(h1.view(np.uint64), h2.view(np.uint64))
