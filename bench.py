"""Benchmark: compressed-basis GMRES time-to-solution and the fused
decompress + Gram-Schmidt bandwidth on one MI355X.

Step: one full solve of the 3D convection-diffusion system on a 100^3 grid
(n = 10^6, 6.94e6 nonzeros, convection (10,5,2), x* ~ U(-1,1) seed 1,
b = A x*), GMRES(100), relative residual 1e-10, x0 = 0, basis stored as
frsz2_32.  The same solve with a float64 basis is timed beside it.

Roofline: the fused decompress + CGS projection kernel (h = V^T w over 101
frsz2_32 columns of 2^24 rows, the tall-skinny test basis, seed 2), timed with
HIP events on the stream it runs on; algorithmic bytes per launch =
101 * 2^24 * 4.125 (codes + block exponents) + 8 * 2^24 (w).

`traffic` is the HBM bytes per launch of that kernel from the committed
FETCH_SIZE / WRITE_SIZE counter summary under profiles/ (scaled by the same
counters' reading for a 1 GiB copy), reported only while the kernel sources
hash to the value recorded there; otherwise null.

CPU baseline: the FP64 oracle's whole frsz2_32 solve of the same system,
single thread, timed in a background thread beside the GPU legs; the host's
CPU model and logical core count are reported with it.

Other workloads (--workload): `serving` runs the seeded request stream through
the continuous-batching server (p50/p99 latency, solves/s); `precision` runs
FP64 iterative refinement around a frsz2_16-basis GMRES(100) against the
float64-basis solve on the 2^22-row banded system; `intensity` the
arithmetic-intensity sweep; `adaptive` the solve with its basis format picked
by probing candidates before the first restart, against every fixed format;
`precond` Jacobi right preconditioning on the column-scaled sweep operator.

Prints one JSON line.
"""
import argparse
import itertools
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "CB-GMRES time-to-1e-10 residual, frsz2 vs fp64 basis; decompress+CGS HBM GB/s"
HBM_PEAK_GBS = 8000.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_project_frsz2_32_microbench_2p24x101.md")
# The sources k_project is compiled from: the stored counter traffic is used
# only while these hash to the value recorded beside it.
TRAFFIC_KERNEL_SOURCES = ("basis.hip", "cb_internal.hpp", "codec.hpp", "epilogue.hpp", "reduce.hpp", "tiles.hpp")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2409_15468_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per k_project<frsz2_32> launch from the committed FETCH_SIZE /
    WRITE_SIZE counter summary, or None if the kernel sources changed since
    the counters were taken."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "kernel_source_sha256"):
            k, v = line.split(":", 1)
            vals[k] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash() or "traffic_bytes_per_launch" not in vals:
        return None
    return float(vals["traffic_bytes_per_launch"])


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def solve_algorithmic_bytes(cb, n, nnz, fmt, res):
    """Compulsory HBM bytes of one solve, from its own counts: every basis
    pass (the solver's basis_bytes, which counts the columns' code bytes, scaled
    to include the block exponents), the CSR once per SpMV (each Arnoldi step
    and each cycle's residual), and the FP64 vectors each launch must read or
    write (per step: the SpMV's x and y, the projection's w, the update's w in
    and out; with the second Gram-Schmidt pass its projection's w and update's
    w in and out; per cycle: the residual's x, b and r and the x update's x
    in and out)."""
    codes = cb.cb_basis_column_bytes(fmt, n)
    withexp = codes + 4 * cb.cb_basis_exponent_words(fmt, n)
    it, cyc, ro = res["iterations"], res["restarts"], res["reorths"]
    csr = 12 * nnz + 4 * (n + 1)
    basis = res["basis_bytes"] * withexp / codes
    vectors = it * 40 * n + ro * 24 * n + (cyc + 1) * 40 * n
    return basis + (it + cyc + 1) * csr + vectors


def timed_solves(cb, torch, A, b, x, fmt, m, tol, steps, warmup, ws):
    res = None
    for _ in range(warmup):
        x.zero_()
        res, _ = cb.cbgmres_solve(A, b, x, m, tol, fmt, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        res, _ = cb.cbgmres_solve(A, b, x, m, tol, fmt, workspace=ws)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, res


def event_time(torch, fn, reps):
    """Duration of fn() from HIP events recorded around each of `reps`
    launches on the current stream (the stream the library launches on), after
    one untimed launch: (mean, minimum, median) in seconds."""
    s = torch.cuda.current_stream()
    fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record(s)
        fn()
        e1.record(s)
    ev[-1][1].synchronize()
    t = sorted(e0.elapsed_time(e1) / 1e3 for e0, e1 in ev)
    return sum(t) / len(t), t[0], t[len(t) // 2]


def microbench(cb, torch, n, ncols, reps, formats):
    import synth
    out = {}
    log(f"microbench: generating {ncols} columns of {n} rows")
    t = time.time()
    cols = [torch.from_numpy(c).cuda() for c in synth.basis_columns(n, ncols, seed=2)]
    w = torch.from_numpy(synth.basis_probe_vector(n, seed=2)).cuda()
    log(f"microbench: inputs ready in {time.time() - t:.1f}s")
    for fmt in formats:
        V = cb.Basis.empty(fmt, n, ncols)
        for c in range(ncols):
            cb.cb_basis_store(V, c, cols[c])
        torch.cuda.synchronize()
        bv = (cb.cb_basis_column_bytes(fmt, n) + 4 * cb.cb_basis_exponent_words(fmt, n)) / n
        h = torch.empty(ncols, dtype=torch.float64, device="cuda")
        work = torch.empty(cb.cb_reduce_workspace_bytes(n, ncols + 1) // 8 + 1, dtype=torch.float64,
                           device="cuda")
        t_dot, n_dot, m_dot = event_time(torch, lambda: cb.cb_cgs_project(V, ncols, w, h, work), reps)
        wt = w.clone()
        hs = torch.full((ncols,), 1e-3, dtype=torch.float64, device="cuda")
        n2 = torch.empty(1, dtype=torch.float64, device="cuda")
        t_upd, n_upd, m_upd = event_time(torch, lambda: cb.cb_cgs_subtract(V, ncols, hs, wt, n2, work), reps)
        # the first update fused with the second projection (one launch; the
        # updated w feeds the next launch, which keeps the work the same)
        wf = w.clone()
        fo = torch.empty(ncols + 1, dtype=torch.float64, device="cuda")
        hz = torch.full((ncols,), 1e-9, dtype=torch.float64, device="cuda")
        t_fus, n_fus, m_fus = event_time(torch, lambda: cb.cb_cgs_subtract_project(V, ncols, hz, wf, fo, work), reps)
        del wf
        # A different column each launch, written to one of four output
        # vectors in turn (compress: stored from its own input vector, so V
        # stays as it is).  Otherwise one column's codes or one input vector
        # would stay in the 256 MB Infinity Cache from one launch to the next,
        # and so would one output, whose writes the cache would then absorb
        # without writing them back: the figures would not be HBM's.
        xo = [torch.empty(n, dtype=torch.float64, device="cuda") for _ in range(4)]
        rot = itertools.count()

        def dec():
            k = next(rot)
            cb.cb_basis_load(V, k % ncols, xo[k % 4])

        t_dec, n_dec, m_dec = event_time(torch, dec, reps * 4)
        del xo
        rot = itertools.count()

        def enc():
            c = next(rot) % ncols
            cb.cb_basis_store(V, c, cols[c])

        t_enc, n_enc, m_enc = event_time(torch, enc, reps * 4)
        dot_bytes = ncols * n * bv + 8 * n
        upd_bytes = ncols * n * bv + 16 * n  # also the fused update + projection's
        codec_bytes = (8 + bv) * n
        out[fmt] = {
            "bytes_per_value": bv,
            # *_s: the mean over the timed launches (GB/s from it), *_min_s and
            # *_median_s beside it
            "dot_s": t_dot, "dot_GBs": dot_bytes / t_dot / 1e9, "dot_min_s": n_dot, "dot_median_s": m_dot,
            "update_s": t_upd, "update_GBs": upd_bytes / t_upd / 1e9, "update_min_s": n_upd,
            "update_median_s": m_upd,
            "fused_s": t_fus, "fused_GBs": upd_bytes / t_fus / 1e9, "fused_min_s": n_fus, "fused_median_s": m_fus,
            "decompress_s": t_dec, "decompress_GBs": codec_bytes / t_dec / 1e9, "decompress_min_s": n_dec,
            "decompress_median_s": m_dec,
            "compress_s": t_enc, "compress_GBs": codec_bytes / t_enc / 1e9, "compress_min_s": n_enc,
            "compress_median_s": m_enc,
        }
        log(f"microbench {fmt}: dot {out[fmt]['dot_GBs']:.0f} GB/s, update {out[fmt]['update_GBs']:.0f} GB/s, "
            f"fused update+projection {out[fmt]['fused_GBs']:.0f} GB/s, "
            f"decompress {out[fmt]['decompress_GBs']:.0f} GB/s, compress {out[fmt]['compress_GBs']:.0f} GB/s")
        del V, work
        torch.cuda.empty_cache()
    return out


def host_cpu():
    """The host's CPU model (from /proc/cpuinfo) and its logical core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


class CpuBaseline:
    """The oracle's whole frsz2_32 solve of the benchmark system, timed on one
    host core in a thread of its own (the oracle is a C library called
    through ctypes, which releases the interpreter lock, so the thread runs
    beside the GPU legs without holding them up)."""

    def __init__(self, s, m, tol):
        import threading
        import oracle
        self.out = None

        def run():
            t = time.perf_counter()
            r = oracle.gmres(s.A, s.b, m, tol, "frsz2_32")
            self.out = (time.perf_counter() - t, r.iterations, r.restarts, bool(r.converged))
        self.thread = threading.Thread(target=run, daemon=True)
        self.thread.start()

    def result(self, gpu_iters):
        self.thread.join()
        dt, iters, cycles, conv = self.out
        model, cores = host_cpu()
        return {
            "value": dt, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": f"the whole frsz2_32 solve of the same system by the oracle ({iters} Arnoldi steps in "
                      f"{cycles} cycles, converged={conv}; GPU: {gpu_iters} steps), single thread, run "
                      f"beside the GPU legs",
            "host_cpu": model, "host_logical_cores": cores,
        }


def serving_bench(cb, torch, count, rate, budget_gb, lanes, seed=4, standalone=False):
    """Continuous-batching server on the seeded request stream (the first
    `count` requests of the 512-request stream): requests are submitted at
    their Poisson arrival times, results polled as they finish.  Latency =
    finish - submit on the server's clock.  With `standalone`, every request is
    then solved again on its own (one at a time through the same server) and
    the sum of those times is reported beside the makespan: how much the mix
    overlapped on the GPU."""
    import synth
    reqs = synth.serving_requests(512, rate, seed)[:count]
    log(f"serving: building {count} systems")
    t = time.time()
    mats = {}
    systems = []
    for r in reqs:
        if r.rid % 64 == 0:
            log(f"serving: building request {r.rid}/{count}")
        key = (r.dim, r.N)
        if key not in mats:
            mats[key] = synth.convection_diffusion(r.N, r.dim, (20.0, 0.0) if r.dim == 2 else (10.0, 5.0, 2.0))
        A = mats[key]
        xs = np.random.default_rng(r.seed).uniform(-1.0, 1.0, A.n)
        systems.append((A, synth.rhs_from_solution(A, xs)))
    log(f"serving: inputs ready in {time.time() - t:.1f}s ({len(mats)} distinct matrices)")
    server = cb.Server(int(budget_gb * (1 << 30)), 0, lanes)
    pending = {}
    done = {}
    t0 = time.perf_counter()
    nxt = 0
    last_log = 0.0
    while nxt < count or pending:
        now = time.perf_counter() - t0
        if now - last_log > 5.0:
            log(f"serving: t={now:.1f}s submitted {nxt}, finished {len(done)}")
            last_log = now
        while nxt < count and reqs[nxt].arrival_s <= now:
            A, b = systems[nxt]
            tk = server.submit(A.row_ptr, A.col, A.val, b, reqs[nxt].m, reqs[nxt].tol, reqs[nxt].fmt)
            pending[tk] = nxt
            nxt += 1
        for tk in list(pending):
            out = server.poll(tk, systems[pending[tk]][0].n)
            if out is not None:
                done[pending.pop(tk)] = out
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    alone = None
    if standalone:
        log("serving: each request alone")
        alone = []
        differ = 0
        for i in range(count):
            A, b = systems[i]
            tk = server.submit(A.row_ptr, A.col, A.val, b, reqs[i].m, reqs[i].tol, reqs[i].fmt)
            while (out := server.poll(tk, A.n)) is None:
                time.sleep(0.0002)
            alone.append(out[2][2] - out[2][1])
            differ += int(not np.array_equal(out[0], done[i][0]))
    server.close()
    lat = np.array([done[i][2][2] - done[i][2][0] for i in range(count)])
    queue = np.array([done[i][2][1] - done[i][2][0] for i in range(count)])
    first = min(done[i][2][0] for i in range(count))
    last = max(done[i][2][2] for i in range(count))
    ok = 0
    worst = 0.0
    for i in range(count):
        A, b = systems[i]
        x, res, _ = done[i]
        rrn = float(np.linalg.norm(b - A.scipy() @ x) / np.linalg.norm(b))
        worst = max(worst, rrn / reqs[i].tol)
        ok += int(res["status"] == 0 and res["converged"] and rrn <= reqs[i].tol * (1 + 1e-6))
    small = np.array([reqs[i].n <= 16384 for i in range(count)])
    out = {"requests": count, "rate_per_s": rate, "budget_gb": budget_gb, "lanes": lanes,
           "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
           "mean_latency_s": float(lat.mean()), "p50_queue_s": float(np.percentile(queue, 50)),
           "solves_per_s": count / (last - first), "makespan_s": last - first, "wall_s": wall,
           "small_requests": int(small.sum()),
           "p50_latency_small_s": float(np.percentile(lat[small], 50)) if small.any() else None,
           "p50_latency_large_s": float(np.percentile(lat[~small], 50)) if (~small).any() else None,
           "converged_within_tol": ok, "worst_rrn_over_tol": worst}
    if alone is not None:
        out["standalone_sum_s"] = float(sum(alone))
        out["standalone_over_makespan"] = float(sum(alone) / (last - first))
        out["alone_differs_from_mix"] = differ  # requests whose x alone is not bit-identical to the mix's
    log(f"serving: p50 {out['p50_latency_s'] * 1e3:.1f} ms, p99 {out['p99_latency_s'] * 1e3:.1f} ms, "
        f"{out['solves_per_s']:.1f} solves/s, {ok}/{count} within tol")
    return out


def precision_bench(cb, torch, steps, warmup):
    """FP64 iterative refinement around GMRES(100) on a frsz2_16 basis (inner
    tolerance 1e-4 relative, one cycle per outer step) against plain
    GMRES(100) on a float64 basis, both to 1e-12, on the banded random system
    (n = 2^22, 27 nonzeros per row, |i - j| <= 1000, seed 3)."""
    import synth
    log("precision: building the banded system")
    t = time.time()
    s = synth.banded_random(seed=3)
    log(f"precision: inputs ready in {time.time() - t:.1f}s (n={s.A.n}, nnz={s.A.nnz})")
    A = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    b = torch.from_numpy(s.b).cuda()
    x = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
    # one caller-owned workspace for every solve: nothing is allocated in the
    # timed region
    ws = torch.empty(max(cb.cbgmres_ir_workspace_bytes(s.A.n, 100, "frsz2_16"),
                         cb.cbgmres_workspace_bytes(s.A.n, 100, "float64")), dtype=torch.uint8, device="cuda")
    out = {}

    def run(fn):
        for _ in range(warmup):
            x.zero_()
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, r

    # the inner relative tolerance of the refinement: 1e-4 is the reading the
    # oracle pins; looser and tighter inner solves are timed beside it
    inner = {}
    for itol in (1e-2, 1e-6, 1e-8):
        t_i, r_i = run(lambda: cb.cbgmres_ir_solve(A, b, x, 100, itol, 1e-12, "frsz2_16", workspace=ws))
        inner[f"{itol:g}"] = {"seconds": t_i, "iterations": r_i["iterations"], "outer": r_i["restarts"],
                              "converged": bool(r_i["converged"])}
        log(f"precision ir inner_tol {itol:g}: {t_i * 1e3:.1f} ms, {r_i['iterations']} iterations, "
            f"{r_i['restarts']} outer")
    out["ir_inner_tol_sweep"] = inner
    t_ir, r_ir = run(lambda: cb.cbgmres_ir_solve(A, b, x, 100, 1e-4, 1e-12, "frsz2_16", workspace=ws))
    x_ir = x.cpu().numpy()
    t_64, r_64 = run(lambda: cb.cbgmres_solve(A, b, x, 100, 1e-12, "float64", workspace=ws)[0])
    x_64 = x.cpu().numpy()
    for name, tt, r, xx in (("ir_frsz2_16", t_ir, r_ir, x_ir), ("float64", t_64, r_64, x_64)):
        rrn = float(np.linalg.norm(s.b - s.A.scipy() @ xx) / np.linalg.norm(s.b))
        out[name] = {"seconds": tt, "iterations": r["iterations"], "outer_or_cycles": r["restarts"],
                     "converged": bool(r["converged"]), "rel_residual": rrn,
                     "err_vs_xstar": float(np.linalg.norm(xx - s.x_star) / np.linalg.norm(s.x_star))}
        if name == "float64":
            by = solve_algorithmic_bytes(cb, s.A.n, s.A.nnz, "float64", r)
            out[name]["algorithmic_bytes"] = by
            out[name]["roofline_frac"] = by / tt / 1e9 / HBM_PEAK_GBS
        log(f"precision {name}: {tt * 1e3:.1f} ms, {r['iterations']} iterations, rrn {rrn:.2e}")
    out["err_ir_vs_float64_solve"] = float(np.linalg.norm(x_ir - x_64) / np.linalg.norm(x_64))
    out["speedup_ir_vs_float64"] = t_64 / t_ir
    return out, s


def adaptive_bench(cb, torch, grid, steps, warmup, probe_steps):
    """Basis format picked by probing before the first restart against every
    fixed format, on the sweep system (GMRES(100), tol 1e-10, x0 = 0).  The
    probing solve's time includes its probes."""
    import synth
    s = synth.sweep_3d(N=grid, seed=1)
    A = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    b = torch.from_numpy(s.b).cuda()
    x = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
    m, tol = 100, 1e-10
    cands = ["frsz2_32", "float32", "float16", "frsz2_16"]
    out = {"candidates": cands, "probe_steps": probe_steps, "fixed": {}}

    def run(fn):
        r = None
        for _ in range(warmup):
            x.zero_()
            r = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, r

    for fmt in ("float64",) + tuple(cands):
        tt, r = run(lambda: cb.cbgmres_solve(A, b, x, m, tol, fmt)[0])
        out["fixed"][fmt] = {"seconds": tt, "iterations": r["iterations"], "converged": bool(r["converged"])}
        log(f"adaptive: fixed {fmt}: {tt * 1e3:.1f} ms, {r['iterations']} iterations")
    ws = torch.empty(cb.cbgmres_auto_workspace_bytes(s.A.n, m, probe_steps, cands), dtype=torch.uint8,
                     device="cuda")
    picks = []

    def auto():
        r, _ = cb.cbgmres_solve_auto(A, b, x, m, tol, cands, probe_steps, workspace=ws)
        picks.append(cands[r["chosen"]])
        return r
    tt, r = run(auto)
    rrn = float(np.linalg.norm(s.b - s.A.scipy() @ x.cpu().numpy()) / np.linalg.norm(s.b))
    best = min(out["fixed"].values(), key=lambda v: v["seconds"])["seconds"]
    out["auto"] = {"seconds": tt, "picks": picks, "probe_seconds": r["probe_seconds"],
                   "probe_rel_residual": r["probe_rel_residual"], "probe_rate": r["probe_rate"],
                   "continuation_iterations": r["solve"]["iterations"],
                   "total_steps": sum(r["probe_steps"]) + r["solve"]["iterations"],
                   "converged": bool(r["solve"]["converged"]), "rel_residual": rrn,
                   "vs_best_fixed": tt / best}
    log(f"adaptive: auto {tt * 1e3:.1f} ms (best fixed {best * 1e3:.1f} ms), picks {picks}, "
        f"probe rates {[round(v, 1) for v in r['probe_rate']]}")
    return out, s


def precond_bench(cb, torch, grid, steps, warmup):
    """Jacobi right preconditioning on the sweep operator with its columns
    scaled by 10^U(-3,3) (seed 6): the preconditioned solve per basis format,
    the unpreconditioned one capped at 2000 steps, and the unscaled system's
    plain solve for reference."""
    import synth
    base = synth.sweep_3d(N=grid, seed=1)
    s = synth.column_scaled(base, decades=3.0)
    A = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    b = torch.from_numpy(s.b).cuda()
    x = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
    m, tol = 100, 1e-10
    out = {}

    def run(fn):
        r = None
        for _ in range(warmup):
            x.zero_()
            r = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, r

    t_setup, d = run(lambda: cb.cb_jacobi_setup(A))
    out["jacobi_setup_s"] = t_setup
    for fmt in ("frsz2_32", "float64", "frsz2_16", "float32"):
        tt, r = run(lambda: cb.cbgmres_solve(A, b, x, m, tol, fmt, diag_inv=d)[0])
        rrn = float(np.linalg.norm(s.b - s.A.scipy() @ x.cpu().numpy()) / np.linalg.norm(s.b))
        out[f"jacobi_{fmt}"] = {"seconds": tt, "iterations": r["iterations"], "converged": bool(r["converged"]),
                                "rel_residual": rrn}
        log(f"precond: jacobi {fmt}: {tt * 1e3:.1f} ms, {r['iterations']} iterations, rrn {rrn:.2e}")
    tt, r = run(lambda: cb.cbgmres_solve(A, b, x, m, tol, "frsz2_32", max_iters=2000)[0])
    out["none_frsz2_32_capped_2000"] = {"seconds": tt, "iterations": r["iterations"],
                                        "converged": bool(r["converged"]), "rel_residual": r["rel_residual"]}
    log(f"precond: none frsz2_32: {tt * 1e3:.1f} ms, {r['iterations']} iterations, rel {r['rel_residual']:.2e}")
    Ab = cb.DeviceCSR.from_host(base.A.row_ptr, base.A.col, base.A.val)
    bb = torch.from_numpy(base.b).cuda()
    tt, r = run(lambda: cb.cbgmres_solve(Ab, bb, x, m, tol, "frsz2_32")[0])
    out["unscaled_plain_frsz2_32"] = {"seconds": tt, "iterations": r["iterations"]}
    log(f"precond: unscaled plain frsz2_32: {tt * 1e3:.1f} ms, {r['iterations']} iterations")
    return out, s


SWEEP_OPS = (0, 1, 2, 3, 4, 5, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64, 80, 96, 112, 128, 160,
             192, 256)


def intensity_sweep(cb, torch, n, formats, reps):
    """The arithmetic-intensity sweep (the synthetic benchmark of Section
    IV-C, 27 settings): one column of n values, N(0,1) scaled per 32-value
    block by 10^u, u ~ U(-8, 0) (seed 2), read through each format's decoder
    with `ops` FP64 multiply-adds per value."""
    rng = np.random.default_rng(2)
    x = rng.standard_normal(n) / np.sqrt(n) * np.repeat(10.0 ** rng.uniform(-8, 0, (n + 31) // 32), 32)[:n]
    xd = torch.from_numpy(x).cuda()
    del x
    out = {}
    s = torch.cuda.current_stream()
    for fmt in formats:
        V = cb.Basis.empty(fmt, n, 1)
        cb.cb_basis_store(V, 0, xd)
        part = torch.empty(cb.cb_intensity_groups(n), dtype=torch.float64, device="cuda")
        bv = (cb.cb_basis_column_bytes(fmt, n) + 4 * cb.cb_basis_exponent_words(fmt, n)) / n
        rows = []
        for ops in SWEEP_OPS:
            cb.cb_intensity_run(V, 0, ops, 0.999, 1e-3, part)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(reps):
                cb.cb_intensity_run(V, 0, ops, 0.999, 1e-3, part)
            e1.record(s)
            e1.synchronize()
            t = e0.elapsed_time(e1) / 1e3 / reps
            rows.append({"ops": ops, "flop_per_byte": 2 * ops / bv, "seconds": t, "GBs": n * bv / t / 1e9,
                         "GFLOPs": 2 * ops * n / t / 1e9})
        out[fmt] = {"bytes_per_value": bv, "points": rows}
        log(f"sweep {fmt}: ops=0 {rows[0]['GBs']:.0f} GB/s; ops=16 {rows[11]['GBs']:.0f} GB/s "
            f"{rows[11]['GFLOPs']:.0f} GFLOP/s; ops=256 {rows[-1]['GFLOPs']:.0f} GFLOP/s")
        del V, part
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=100)
    ap.add_argument("--micro-rows", type=int, default=1 << 24)
    ap.add_argument("--micro-reps", type=int, default=10)
    ap.add_argument("--micro-formats", default="frsz2_32,frsz2_21,frsz2_16,float32,float64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--all-formats", action="store_true",
                    help="also time the sweep solve with the float32, float16, frsz2_16 and frsz2_21 bases")
    ap.add_argument("--extra-formats", default="",
                    help="further basis formats to time in the sweep solve, e.g. frsz2b64_32,frsz2_24")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="microbench only (counter runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also copy 1 GiB once: the reference kernel for FETCH/WRITE_SIZE")
    ap.add_argument("--probe-steps", type=int, default=20, help="probe length of the adaptive workload")
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "serving", "precision", "intensity", "adaptive", "precond"],
                    help="sweep: the n=1e6 solve + kernel microbench (default); serving: the "
                         "request stream through the continuous-batching server; precision: FP64 "
                         "iterative refinement around a frsz2_16-basis GMRES at n=2^22; intensity: the "
                         "arithmetic-intensity sweep over 2^28 values per format; adaptive: the basis "
                         "format picked by probing against every fixed format; precond: Jacobi right "
                         "preconditioning on the column-scaled sweep operator")
    ap.add_argument("--serve-count", type=int, default=512)
    ap.add_argument("--serve-leg", type=int, default=128,
                    help="requests of the seeded serving stream run after the sweep legs of the default "
                         "workload (0: none)")
    ap.add_argument("--serve-standalone", action="store_true",
                    help="serving workload: also solve every request alone and report the sum of those "
                         "times against the makespan")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-lanes", type=int, default=8)
    ap.add_argument("--serve-hw-queues", type=int, default=0,
                    help="hardware queues per process for the serving run (GPU_MAX_HW_QUEUES, <= 32; "
                         "0: the runtime default); streams beyond the queue count share queues")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the benchmark runs on one GPU; multi-GPU runs are not supported (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving" and args.serve_hw_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(min(32, args.serve_hw_queues))
    import torch

    import paper_2409_15468_amd as cb
    import synth

    torch.cuda.set_device(0)
    if args.workload == "serving":
        sv = serving_bench(cb, torch, args.serve_count, args.serve_rate, args.serve_budget_gb, args.serve_lanes,
                           standalone=args.serve_standalone)
        rec = {"metric": "serving p50/p99 latency and solves/s", "value": sv["solves_per_s"],
               "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": sv["wall_s"] * 1e3,
               "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic",
               "config": {"workload": f"{args.serve_count} seeded convection-diffusion solve requests, Poisson "
                                      f"arrivals {args.serve_rate}/s, n 32^2..128^3, formats f32/frsz2_16/21/32, "
                                      f"tol 1e-12..1e-8, m 30..100, HBM budget {args.serve_budget_gb} GB"},
               "serving": dict(sv, hw_queues=os.environ.get("GPU_MAX_HW_QUEUES", "default"))}
        print(json.dumps(rec), flush=True)
        return
    if args.workload == "intensity":
        fm = [f for f in args.micro_formats.split(",") if f] + ["float16"]
        sw = intensity_sweep(cb, torch, 1 << 28, fm, args.micro_reps)
        z = sw.get("frsz2_32", {}).get("points", [{}])[0]
        rec = {"metric": "decompression read bandwidth vs arithmetic intensity (2^28 values)",
               "value": z.get("GBs"), "unit": "GB/s", "n_gpus": 1, "steps": args.micro_reps, "warmup": 1,
               "ms_per_step": z.get("seconds", 0) * 1e3, "higher_is_better": True, "scaling": "strong",
               "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": "2^28 values, N(0,1)/sqrt(n) x 10^U(-8,0) per 32-value block, seed 2; "
                                      f"{len(SWEEP_OPS)} settings of 0..256 FP64 multiply-adds per value"},
               "intensity": sw}
        print(json.dumps(rec), flush=True)
        return
    if args.workload == "precision":
        pv, ps = precision_bench(cb, torch, args.steps, args.warmup)
        rec = {"metric": "time-to-1e-12 residual, FP64 IR around frsz2_16-basis GMRES(100) vs fp64-basis "
                         "GMRES(100)", "value": pv["ir_frsz2_16"]["seconds"], "unit": "s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": pv["ir_frsz2_16"]["seconds"] * 1e3,
               "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic",
               "config": {"workload": f"banded random n={ps.A.n}, nnz={ps.A.nnz} (27 per row, |i-j|<=1000, "
                                      "diagonal 1.2 x row sum, seed 3), tol 1e-12"},
               "precision": pv}
        print(json.dumps(rec), flush=True)
        return
    if args.workload == "adaptive":
        av, s = adaptive_bench(cb, torch, args.grid, args.steps, args.warmup, args.probe_steps)
        rec = {"metric": "time-to-1e-10 residual, basis format picked by probing vs fixed formats",
               "value": av["auto"]["seconds"], "unit": "s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": av["auto"]["seconds"] * 1e3, "higher_is_better": False,
               "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"cd3d N={args.grid} (n={s.A.n}, nnz={s.A.nnz}), GMRES(100), tol 1e-10, "
                                      f"x0=0; candidates {','.join(av['candidates'])}, "
                                      f"{args.probe_steps}-step probes"},
               "adaptive": av}
        print(json.dumps(rec), flush=True)
        return
    if args.workload == "precond":
        pv, s = precond_bench(cb, torch, args.grid, args.steps, args.warmup)
        rec = {"metric": "time-to-1e-10 residual, Jacobi right-preconditioned GMRES(100), frsz2_32 basis",
               "value": pv["jacobi_frsz2_32"]["seconds"], "unit": "s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": pv["jacobi_frsz2_32"]["seconds"] * 1e3,
               "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
               "data": "synthetic",
               "config": {"workload": f"cd3d N={args.grid} (n={s.A.n}, nnz={s.A.nnz}) with columns scaled by "
                                      "10^U(-3,3) (seed 6), GMRES(100), tol 1e-10, x0=0"},
               "precond": pv}
        print(json.dumps(rec), flush=True)
        return
    m, tol = 100, 1e-10
    log(f"bench: building cd3d N={args.grid}")
    s = synth.sweep_3d(N=args.grid, seed=1)
    A = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    b = torch.from_numpy(s.b).cuda()
    x = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
    ws = torch.empty(cb.cbgmres_workspace_bytes(s.A.n, m, "float64") // 8 + 1, dtype=torch.float64,
                     device="cuda")
    cpu = None
    if not args.no_cpu and not args.no_solve:
        log("bench: oracle CPU baseline started (whole frsz2_32 solve, one host core, in the background)")
        cpu = CpuBaseline(s, m, tol)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copied 1 GiB (counter calibration)")
        del src, dst
    rec = {"metric": METRIC, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"cd3d N={args.grid} (n={s.A.n}, nnz={s.A.nnz}), GMRES({m}), tol {tol}, "
                                  "basis frsz2_32, x0=0",
                      "n": s.A.n, "nnz": s.A.nnz, "m": m, "tol": tol, "basis": "frsz2_32"}}
    r_z = None
    if not args.no_solve:
        log("bench: frsz2_32 solves")
        t_z, r_z = timed_solves(cb, torch, A, b, x, "frsz2_32", m, tol, args.steps, args.warmup, ws)
        xr = x.cpu().numpy()
        rel = float(np.linalg.norm(s.b - s.A.scipy() @ xr) / np.linalg.norm(s.b))
        err = float(np.linalg.norm(xr - s.x_star) / np.linalg.norm(s.x_star))
        log(f"bench: frsz2_32 {t_z * 1e3:.1f} ms, {r_z['iterations']} iters, {r_z['restarts']} cycles, "
            f"rel {rel:.2e}")
        log("bench: float64 solves")
        t_d, r_d = timed_solves(cb, torch, A, b, x, "float64", m, tol, args.steps, args.warmup, ws)
        x64 = x.cpu().numpy()
        log(f"bench: float64 {t_d * 1e3:.1f} ms, {r_d['iterations']} iters")
        rec.update({"value": t_z, "ms_per_step": t_z * 1e3})
        by_z = solve_algorithmic_bytes(cb, s.A.n, s.A.nnz, "frsz2_32", r_z)
        by_d = solve_algorithmic_bytes(cb, s.A.n, s.A.nnz, "float64", r_d)
        rec["solve_roofline"] = {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "frsz2_32": {"bytes": by_z, "achieved": by_z / t_z / 1e9, "frac": by_z / t_z / 1e9 / HBM_PEAK_GBS},
            "float64": {"bytes": by_d, "achieved": by_d / t_d / 1e9, "frac": by_d / t_d / 1e9 / HBM_PEAK_GBS},
            "note": "algorithmic bytes of the whole solve (basis passes, CSR per SpMV, FP64 vectors) over its "
                    "time; passes the Infinity Cache serves count as HBM bytes"}
        log(f"bench: solve-level fraction of the HBM roofline: frsz2_32 {rec['solve_roofline']['frsz2_32']['frac']:.2f}, "
            f"float64 {rec['solve_roofline']['float64']['frac']:.2f}")
        rec["solve"] = {
            "frsz2_32": {"seconds": t_z, "iterations": r_z["iterations"], "cycles": r_z["restarts"],
                         "reorths": r_z["reorths"], "rel_residual": rel, "err_vs_xstar": err,
                         "err_vs_fp64_basis": float(np.linalg.norm(xr - x64) / np.linalg.norm(x64))},
            "float64": {"seconds": t_d, "iterations": r_d["iterations"], "cycles": r_d["restarts"],
                        "reorths": r_d["reorths"], "rel_residual": r_d["rel_residual"]},
            "speedup_frsz2_32_vs_float64": t_d / t_z,
        }
        extra = (["float32", "float16", "frsz2_16", "frsz2_21"] if args.all_formats else []) + \
            [f for f in args.extra_formats.split(",") if f]
        if extra:
            for fmt in extra:
                log(f"bench: {fmt} solves")
                t_f, r_f = timed_solves(cb, torch, A, b, x, fmt, m, tol, args.steps, args.warmup, ws)
                xf = x.cpu().numpy()
                rec["solve"][fmt] = {
                    "seconds": t_f, "iterations": r_f["iterations"], "cycles": r_f["restarts"],
                    "reorths": r_f["reorths"], "converged": bool(r_f["converged"]),
                    "rel_residual": float(np.linalg.norm(s.b - s.A.scipy() @ xf) / np.linalg.norm(s.b)),
                    "err_vs_xstar": float(np.linalg.norm(xf - s.x_star) / np.linalg.norm(s.x_star)),
                    "err_vs_fp64_basis": float(np.linalg.norm(xf - x64) / np.linalg.norm(x64)),
                    "speedup_vs_float64": t_d / t_f}
                log(f"bench: {fmt} {t_f * 1e3:.1f} ms, {r_f['iterations']} iters")
    del ws
    torch.cuda.empty_cache()

    if not args.no_micro:
        mb = microbench(cb, torch, args.micro_rows, 101, args.micro_reps,
                        [f for f in args.micro_formats.split(",") if f])
        z = mb.get("frsz2_32")
        if z:
            traffic = measured_traffic() if args.micro_rows == 1 << 24 else None
            rec["roofline"] = {"bound": "hbm", "achieved": z["dot_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": z["dot_GBs"] / HBM_PEAK_GBS, "traffic": traffic,
                               "kernel": "k_project<frsz2_32> (fused decompress + CGS projection)",
                               "per_launch_bytes": 101 * args.micro_rows * z["bytes_per_value"] + 8 * args.micro_rows,
                               "avg_launch_s": z["dot_s"]}
        rec["microbench"] = {"rows": args.micro_rows, "columns": 101, "formats": mb}
    if args.serve_leg > 0 and not args.no_solve:
        sv = serving_bench(cb, torch, args.serve_leg, args.serve_rate, args.serve_budget_gb, args.serve_lanes)
        rec["serving"] = dict(sv, workload=f"the first {args.serve_leg} of the 512 seeded requests (Poisson "
                                           f"{args.serve_rate}/s, n 32^2..128^3, formats f32/frsz2_16/21/32, "
                                           f"tol 1e-12..1e-8, m 30..100), HBM budget {args.serve_budget_gb} GB")
    if cpu is not None and r_z is not None:
        log("bench: waiting for the oracle CPU baseline")
        rec["cpu_baseline"] = cpu.result(r_z["iterations"])
        log(f"bench: oracle solve {rec['cpu_baseline']['value']:.1f} s on one core of {rec['cpu_baseline']['host_cpu']}")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
