"""Serving (cb_server_*): HBM-budget admission, continuous batching and result
independence from the mix.

* Each request's solution is bit-identical whether it ran alone on the
  server or among others (same kernels, same reduction order per request),
  and meets its own tolerance.
* The served requests with n <= 10^4 (15 of the 24, every basis format of the
  stream) agree with the oracle's GMRES on the same system: iteration counts
  within 2% (for the 15-bit frsz2_16 basis, or within the oracle's own
  spread under last-bit perturbations of b, stored by
  golden/make_perturbed_counts.py), and the solution within the accuracy
  the tolerance implies.
* A budget that fits one request at a time forces queueing; every request
  still completes, admitted in arrival order within its kind (small requests
  batched, large ones one per lane).
* A request larger than the whole budget is rejected with CB_ERR_OVER_BUDGET.
"""
import time

import numpy as np
import pytest

import oracle
import paper_2409_15468_amd as cb
import synth
from tests._golden import count_agrees, inputs_digest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def requests(k):
    reqs = synth.serving_requests(count=k, seed=4, n_max=40 ** 3)
    return [(r, r.system()) for r in reqs]


def run_all(server, items, stagger=0.0):
    tickets = []
    for r, s in items:
        tickets.append(server.submit(s.A.row_ptr, s.A.col, s.A.val, s.b, r.m, r.tol, r.fmt))
        if stagger:
            time.sleep(stagger)
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < 120:
        for (r, s), t in zip(items, tickets):
            if r.rid in out:
                continue
            got = server.poll(t, s.A.n)
            if got is not None:
                out[r.rid] = got
        time.sleep(0.002)
    assert len(out) == len(tickets), "server did not finish in time"
    return out


def test_alone_equals_mixed_and_meets_tolerance():
    items = requests(24)
    srv = cb.Server(8 << 30, 0, lanes=6)
    mixed = run_all(srv, items, stagger=0.001)
    charged, queued, running = srv.stats()
    assert charged == 0 and queued == 0 and running == 0
    srv.close()
    for r, s in items:
        x, res, times = mixed[r.rid]
        assert res["status"] == 0 and res["converged"], (r, res)
        rel = np.linalg.norm(s.b - s.A.scipy() @ x) / np.linalg.norm(s.b)
        assert rel <= r.tol * (1 + 1e-6)
        assert times[0] <= times[1] <= times[2]
    # a seeded subset against the CPU oracle
    checked = 0
    for r, s in items:
        if s.A.n > 10000:
            continue
        x, res, _ = mixed[r.rid]
        ref = oracle.gmres(s.A, s.b, r.m, r.tol, r.fmt)
        print(f"request {r.rid} n={s.A.n} {r.fmt} m={r.m} tol={r.tol:.1e}: served {res['iterations']} steps, "
              f"oracle {ref.iterations}")
        assert ref.converged
        assert count_agrees(res["iterations"], ref.iterations, f"served24_r{r.rid}", r.fmt,
                            inputs_digest(s.A, s.b)), (r.rid, res["iterations"], ref.iterations)
        # both meet tol on a system with cond(A) <= ~1e3: the solutions agree
        # to what the residuals allow
        assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) <= 1e4 * r.tol
        checked += 1
    assert checked == 15
    # the same requests one at a time
    alone_srv = cb.Server(8 << 30, 0, lanes=1)
    for r, s in items[:8]:
        got = run_all(alone_srv, [(r, s)])[r.rid]
        assert np.array_equal(got[0].view(np.uint64), mixed[r.rid][0].view(np.uint64)), r
        assert got[1]["iterations"] == mixed[r.rid][1]["iterations"]
    alone_srv.close()


def test_budget_forces_queueing_and_rejects_oversize():
    items = requests(6)
    need = max(cb.Server.request_bytes(s.A.n, s.A.nnz, r.m, r.fmt) for r, s in items)
    srv = cb.Server(need, 0, lanes=4)
    out = run_all(srv, items)
    spans = [(out[r.rid][2][1], out[r.rid][2][2], cb.Server.request_bytes(s.A.n, s.A.nnz, r.m, r.fmt))
             for r, s in items]
    for t0, _, _ in spans:  # at every admission the running set fits the budget
        assert sum(b for s0, e0, b in spans if s0 <= t0 < e0) <= need
    # admission in arrival order within each kind (batched small / large)
    for small in (True, False):
        starts = [out[r.rid][2][1] for r, s in items if (s.A.n <= 16384 and r.m <= 104) == small]
        assert starts == sorted(starts)
    big = synth.sweep_3d(N=60, seed=1)
    assert cb.Server.request_bytes(big.A.n, big.A.nnz, 100, "float64") > need
    with pytest.raises(cb.CbError) as ei:
        srv.submit(big.A.row_ptr, big.A.col, big.A.val, big.b, 100, 1e-8, "float64")
    assert ei.value.status == cb.CB_ERR_OVER_BUDGET
    srv.close()


def test_generic_and_block64_formats_are_served_by_the_solve_lanes():
    """Small requests in the generic-width and block-64 FRSZ2 formats (which
    the one-workgroup batched solver does not run) are admitted and solved by
    the solve lanes, with the same result as a direct cbgmres_solve."""
    s = synth.plain_2d(N=40, seed=9)
    fmts = ["frsz2_12", "frsz2b64_32", "frsz2b64_21", "frsz2_32"]
    srv = cb.Server(4 << 30, 0, lanes=2)

    class R:
        def __init__(self, rid, fmt):
            self.rid, self.m, self.tol, self.fmt = rid, 30, 1e-10, fmt
    items = [(R(i, f), s) for i, f in enumerate(fmts)]
    out = run_all(srv, items)
    srv.close()
    A = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    b = torch.from_numpy(s.b).cuda()
    for r, _ in items:
        x, res, _ = out[r.rid]
        assert res["status"] == 0 and res["converged"], (r.fmt, res)
        xd = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
        ref, _ = cb.cbgmres_solve(A, b, xd, 30, 1e-10, r.fmt)
        torch.cuda.synchronize()
        if r.fmt == "frsz2_32":  # batched: another kernel, its own reduction order
            assert abs(res["iterations"] - ref["iterations"]) <= max(1, int(np.ceil(0.02 * ref["iterations"])))
        else:  # the solve lanes run cbgmres_solve itself: bit for bit
            assert res["iterations"] == ref["iterations"], r.fmt
            assert np.array_equal(x.view(np.uint64), xd.cpu().numpy().view(np.uint64)), r.fmt


def test_small_requests_join_the_running_launch():
    """The device-resident loop: small requests submitted one after another
    while earlier ones are being solved are taken by the launch that is
    already running (continuous admission, counted by cb_server_ring_stats),
    and each result is bit for bit the one-workgroup solver's result for the
    same system solved by itself (cbgmres_solve_batch with one item)."""
    items = [(r, s) for r, s in requests(64) if s.A.n <= 16384 and r.m <= 104][:20]
    assert len(items) == 20
    srv = cb.Server(8 << 30, 0, lanes=2)
    out = run_all(srv, items, stagger=0.003)
    published, joined, launches = srv.ring_stats()
    srv.close()
    print(f"ring: {published} published, {joined} served by the launch already running, {launches} launches")
    assert published == len(items)
    assert joined >= len(items) // 2 and launches >= 1
    for r, s in items:
        x, res, _ = out[r.rid]
        A = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
        b = torch.from_numpy(s.b).cuda()
        xd = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
        ref = cb.cbgmres_solve_batch([(A, b, xd, r.m, r.tol, r.fmt)])[0]
        torch.cuda.synchronize()
        assert res["status"] == 0 and res["converged"], (r.rid, res)
        assert res["iterations"] == ref["iterations"], (r.rid, res["iterations"], ref["iterations"])
        assert np.array_equal(x.view(np.uint64), xd.cpu().numpy().view(np.uint64)), r.rid
