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

CPU baseline: the FP64 oracle, single thread, on the first 40 Arnoldi steps of
the same solve, scaled to the whole solve by basis-column work.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "CB-GMRES time-to-1e-10 residual, frsz2 vs fp64 basis; decompress+CGS HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


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
    """Average duration of fn() over reps launches, HIP events on the current
    stream (the stream the library launches on)."""
    s = torch.cuda.current_stream()
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


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
        work = torch.empty(cb.cb_reduce_workspace_bytes(n, ncols) // 8 + 1, dtype=torch.float64,
                           device="cuda")
        t_dot = event_time(torch, lambda: cb.cb_cgs_project(V, ncols, w, h, work), reps)
        wt = w.clone()
        hs = torch.full((ncols,), 1e-3, dtype=torch.float64, device="cuda")
        n2 = torch.empty(1, dtype=torch.float64, device="cuda")
        t_upd = event_time(torch, lambda: cb.cb_cgs_subtract(V, ncols, hs, wt, n2, work), reps)
        xo = torch.empty(n, dtype=torch.float64, device="cuda")
        t_dec = event_time(torch, lambda: cb.cb_basis_load(V, 7, xo), reps * 4)
        t_enc = event_time(torch, lambda: cb.cb_basis_store(V, 7, cols[7]), reps * 4)
        dot_bytes = ncols * n * bv + 8 * n
        upd_bytes = ncols * n * bv + 16 * n
        codec_bytes = (8 + bv) * n
        out[fmt] = {
            "bytes_per_value": bv,
            "dot_s": t_dot, "dot_GBs": dot_bytes / t_dot / 1e9,
            "update_s": t_upd, "update_GBs": upd_bytes / t_upd / 1e9,
            "decompress_GBs": codec_bytes / t_dec / 1e9,
            "compress_GBs": codec_bytes / t_enc / 1e9,
        }
        log(f"microbench {fmt}: dot {out[fmt]['dot_GBs']:.0f} GB/s, update {out[fmt]['update_GBs']:.0f} GB/s, "
            f"decompress {out[fmt]['decompress_GBs']:.0f} GB/s, compress {out[fmt]['compress_GBs']:.0f} GB/s")
        del V, work
        torch.cuda.empty_cache()
    return out


def cpu_baseline(s, gpu_iters, gpu_cycles, m, sample_steps=40):
    """The oracle on the first `sample_steps` Arnoldi steps of the same solve,
    scaled to the whole solve by the Gram-Schmidt work, which dominates the
    oracle's time: step j of a cycle costs in proportion to its j + 1 basis
    columns."""
    import oracle
    t = time.perf_counter()
    r = oracle.gmres(s.A, s.b, m, 1e-10, "frsz2_32", max_iters=sample_steps)
    dt = time.perf_counter() - t
    steps = [m] * (gpu_cycles - 1) + [gpu_iters - m * (gpu_cycles - 1)]
    work = sum(sum(j + 1 for j in range(k)) for k in steps)
    sample_work = sum(j + 1 for j in range(r.iterations))
    return {
        "value": dt * work / sample_work,
        "unit": "s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the first {r.iterations} Arnoldi steps of the same frsz2_32 solve took {dt:.2f}s on one "
                  f"host core; scaled by basis-column work ({work} vs {sample_work} column passes) to the "
                  f"GPU solve's {gpu_iters} steps in {gpu_cycles} cycles",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=100)
    ap.add_argument("--micro-rows", type=int, default=1 << 24)
    ap.add_argument("--micro-reps", type=int, default=5)
    ap.add_argument("--micro-formats", default="frsz2_32,frsz2_21,frsz2_16,float32,float64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--no-solve", action="store_true", help="microbench only (counter runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also copy 1 GiB once: the reference kernel for FETCH/WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2409_15468_amd as cb
    import synth

    torch.cuda.set_device(0)
    m, tol = 100, 1e-10
    log(f"bench: building cd3d N={args.grid}")
    s = synth.sweep_3d(N=args.grid, seed=1)
    A = cb.DeviceCSR.from_host(s.A.row_ptr, s.A.col, s.A.val)
    b = torch.from_numpy(s.b).cuda()
    x = torch.zeros(s.A.n, dtype=torch.float64, device="cuda")
    ws = torch.empty(cb.cbgmres_workspace_bytes(s.A.n, m, "float64") // 8 + 1, dtype=torch.float64,
                     device="cuda")

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
        rec["solve"] = {
            "frsz2_32": {"seconds": t_z, "iterations": r_z["iterations"], "cycles": r_z["restarts"],
                         "reorths": r_z["reorths"], "rel_residual": rel, "err_vs_xstar": err,
                         "err_vs_fp64_basis": float(np.linalg.norm(xr - x64) / np.linalg.norm(x64))},
            "float64": {"seconds": t_d, "iterations": r_d["iterations"], "cycles": r_d["restarts"],
                        "reorths": r_d["reorths"], "rel_residual": r_d["rel_residual"]},
            "speedup_frsz2_32_vs_float64": t_d / t_z,
        }
    del ws
    torch.cuda.empty_cache()

    if not args.no_micro:
        mb = microbench(cb, torch, args.micro_rows, 101, args.micro_reps,
                        [f for f in args.micro_formats.split(",") if f])
        z = mb.get("frsz2_32")
        if z:
            rec["roofline"] = {"bound": "hbm", "achieved": z["dot_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": z["dot_GBs"] / HBM_PEAK_GBS, "traffic": None,
                               "kernel": "k_project<frsz2_32> (fused decompress + CGS projection)",
                               "per_launch_bytes": 101 * args.micro_rows * z["bytes_per_value"] + 8 * args.micro_rows,
                               "avg_launch_s": z["dot_s"]}
        rec["microbench"] = {"rows": args.micro_rows, "columns": 101, "formats": mb}
    if not args.no_cpu and r_z is not None:
        log("bench: oracle CPU baseline (bounded sample)")
        rec["cpu_baseline"] = cpu_baseline(s, r_z["iterations"], r_z["restarts"], m)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
