"""A solve's result does not depend on other work on the GPU: the same
system solved alone and while other solves run on a second stream (from a
second host thread) gives bit-identical iterates and iteration counts.  The
solver's control words are read with device-scope loads, so a kernel never
acts on a stale value that another stream's work left in a cache; this test
guards that.  Covers the plain, Jacobi-preconditioned and generic-width
paths."""
import threading

import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def make(system):
    A = cb.DeviceCSR.from_host(system.A.row_ptr, system.A.col, system.A.val)
    return A, torch.from_numpy(system.b).cuda()


def solve(A, b, n, fmt, m, tol, stream, diag_inv=None):
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(stream):
        res, _ = cb.cbgmres_solve(A, b, x, m, tol, fmt, stream=stream, diag_inv=diag_inv)
        stream.synchronize()
    return res, x.cpu().numpy()


@pytest.mark.parametrize("fmt,precond", [("frsz2_21", False), ("frsz2_32", True), ("frsz2_24", False)])
def test_solve_is_identical_alone_and_beside_other_work(fmt, precond):
    s = synth.column_scaled(synth.sweep_3d(N=40, seed=2), decades=2.0) if precond else synth.sweep_3d(N=40, seed=2)
    A, b = make(s)
    d = cb.cb_jacobi_setup(A) if precond else None
    main = torch.cuda.Stream()
    base_res, base_x = solve(A, b, s.A.n, fmt, 40, 1e-10, main, d)
    assert base_res["converged"]
    other = synth.plain_2d(N=150, seed=3)
    A2, b2 = make(other)
    side = torch.cuda.Stream()
    errors = []

    def background():
        try:
            x2 = torch.zeros(other.A.n, dtype=torch.float64, device="cuda")
            for fmt2 in ("float32", "frsz2_16", "float64"):
                x2.zero_()
                cb.cbgmres_solve(A2, b2, x2, 40, 1e-10, fmt2, stream=side)
            side.synchronize()
        except Exception as e:  # reported by the main thread
            errors.append(e)

    for _ in range(2):
        t = threading.Thread(target=background)
        t.start()
        res, x = solve(A, b, s.A.n, fmt, 40, 1e-10, main, d)
        t.join()
        assert not errors, errors
        assert res["iterations"] == base_res["iterations"] and res["reorths"] == base_res["reorths"]
        assert np.array_equal(x.view(np.uint64), base_x.view(np.uint64))
    # and the result is a correct one: the oracle's step count within 2%
    ref = oracle.gmres(s.A, s.b, 40, 1e-10, fmt, dinv=oracle.jacobi(s.A) if precond else None)
    assert abs(base_res["iterations"] - ref.iterations) <= max(1, int(np.ceil(0.02 * ref.iterations)))
