"""The precision form at its full size (n = 2^22 banded system, 27 nonzeros per
row) against the oracle: FP64 iterative refinement around GMRES(100) on a
frsz2_16 basis, and the plain float64-basis GMRES(100), both to 1e-12.  The
oracle's outer steps, Arnoldi steps and the solution at 4096 rows are stored
in tests/golden/precision_oracle.json (written by make_precision_reference.py,
which calls only the oracle).  Each GPU solve reaches 1e-12 (checked on the
host), takes the oracle's outer steps and Arnoldi steps within 2%, and its
solution agrees with the oracle's at the stored rows; the error of the
refinement against the oracle's float64-basis solution is reported."""
import hashlib
import json
import os

import numpy as np
import pytest

import paper_2409_15468_amd as cb
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def within_2pct(a, b):
    return abs(a - b) <= max(1, int(np.ceil(0.02 * b)))


def test_iterative_refinement_full_size():
    with open(os.path.join(GOLDEN, "precision_oracle.json")) as f:
        ref = json.load(f)
    s = synth.banded_random(seed=3)
    assert s.A.n == 1 << 22 and s.A.nnz == 27 * s.A.n
    assert hashlib.sha256(s.A.sha256().encode() + s.b.tobytes()).hexdigest() == ref["inputs_sha256"]
    rows = np.array(ref["sample_rows"])
    A = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    b = torch.from_numpy(s.b).cuda()
    x = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
    ws = torch.empty(cb.cbgmres_ir_workspace_bytes(s.A.n, 100, "frsz2_16"), dtype=torch.uint8, device="cuda")
    res = cb.cbgmres_ir_solve(A, b, x, 100, 1e-4, 1e-12, "frsz2_16", workspace=ws)
    xi = x.cpu().numpy()
    x.zero_()
    r64, _ = cb.cbgmres_solve(A, b, x, 100, 1e-12, "float64")
    x64 = x.cpu().numpy()
    M = s.A.scipy()
    nb = np.linalg.norm(s.b)
    ir, f64 = ref["ir_frsz2_16"], ref["gmres_float64"]
    xs_ir, xs_64 = np.array(ir["x_sample"]), np.array(f64["x_sample"])
    err_ir = np.linalg.norm(xi[rows] - xs_ir) / np.linalg.norm(xs_ir)
    err_64 = np.linalg.norm(x64[rows] - xs_64) / np.linalg.norm(xs_64)
    err_ir_vs_or64 = np.linalg.norm(xi[rows] - xs_64) / np.linalg.norm(xs_64)
    print(f"IR frsz2_16: gpu {res['restarts']} outer / {res['iterations']} steps, oracle {ir['outer']} / "
          f"{ir['iterations']}; sampled error vs oracle IR {err_ir:.2e}, vs oracle float64 {err_ir_vs_or64:.2e}")
    print(f"float64 basis: gpu {r64['iterations']} steps, oracle {f64['iterations']}; "
          f"sampled error vs oracle {err_64:.2e}")
    assert res["converged"] and np.linalg.norm(s.b - M @ xi) / nb <= 1e-12 * (1 + 1e-6)
    assert r64["converged"] and np.linalg.norm(s.b - M @ x64) / nb <= 1e-12 * (1 + 1e-6)
    assert res["restarts"] == ir["outer"]
    assert within_2pct(res["iterations"], ir["iterations"]), (res["iterations"], ir["iterations"])
    assert within_2pct(r64["iterations"], f64["iterations"]), (r64["iterations"], f64["iterations"])
    # A is strictly diagonally dominant (diagonal 1.2 x the off-diagonal row
    # sum), so the error follows the 1e-12 residual closely
    assert err_ir < 1e-10 and err_64 < 1e-10 and err_ir_vs_or64 < 1e-10
    assert np.linalg.norm(xi - s.x_star) / np.linalg.norm(s.x_star) < 1e-10
