#!/usr/bin/env python3
"""Time-to-tolerance of the mixed-precision LOBPCG hot path on one MI355X.

Workload: 3D 7-point variable-coefficient diffusion on a 64^3 grid (n = 262,144,
cell coefficients exp(N(0,1)), nested dissection), k = 16, m = 32, tol = 1e-10.
One step = numeric factorization of the permuted matrix (FP32 factor) plus
lobpcg_solve to tolerance, with the matrix and start block already on the GPU.
The same step with an FP64 factor (and FP64 Algorithm 2 step 1) is timed on the
same GPU for the mixed-vs-FP64 comparison.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-tol (s) + iters, mixed vs FP64 on same GPU; SpMM/trisolve HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import synth
    if name == "diffusion3d_64":
        return synth.cfg2(N=64)
    if name.startswith("diffusion3d_"):
        return synth.cfg2(N=int(name.split("_")[1]))
    if name == "laplace2d_32":
        return synth.cfg1()
    raise SystemExit(f"unknown workload {name}")


def time_steps(torch, solver, X0, steps, warmup, label):
    infos = []
    for w in range(warmup):
        solver.factor()
        solver.solve(X0)
        log(f"{label} warmup {w + 1}/{warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        solver.factor()
        lam, X, info = solver.solve(X0)
        infos.append(info)
        log(f"{label} step {s + 1}/{steps}: iters={info['iters']} t_factor={info['t_factor']:.4f}s "
            f"t_solve={info['t_solve']:.4f}s")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    return dt, infos, lam, X


def event_time(torch, fn, reps):
    """Average GPU time (ms) of fn() between events recorded on the current stream."""
    fn()
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def batched_run(torch, pk, steps, count):
    """Batched Schrodinger workload: `count` 2D operators (side U{48..128}), k=8, m=16, FP32 factors, one
    context; a step = numeric factorization of the union + lobpcg_solve_batched to tol for all of them."""
    import numpy as np
    import synth
    probs = synth.cfg4(count)
    log(f"batched: setup {count} problems, n total {sum(p.n for p in probs)}")
    t0 = time.perf_counter()
    bs = pk.BatchedSolver([p.A for p in probs], 8, 16, 1e-10, factor_precision="fp32",
                          grids=[p.grid for p in probs])
    t_setup = time.perf_counter() - t0
    X0s = [torch.from_numpy(np.ascontiguousarray(p.X0)).cuda() for p in probs]
    from paper_2302_12528_amd import native as nv
    bs.solve(X0s)   # warmup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        nv.check(bs.lib.lobpcg_factor(bs.ctx))
        evals, evecs, infos, st = bs.solve(X0s)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    # parity: host FP64 residuals of every problem against the estimate the test used
    worst = 0.0
    for b, p in enumerate(probs):
        lam = evals[b].cpu().numpy()
        X = evecs[b].cpu().numpy()
        r = np.linalg.norm(p.A @ X - X * lam, axis=0) / ((infos[b]["norm_a"] + np.abs(lam)) * np.linalg.norm(X, axis=0))
        worst = max(worst, float(r.max()))
    iters = [i["iters"] for i in infos]
    bs.close()
    return {"workload": f"schrodinger2d_batch{count}: {count} 2D -Laplacian+V operators, side U{{48..128}}, "
                        f"k=8, m=16, tol=1e-10, FP32 factors; step = factorization + batched solve",
            "time_to_tol_s": round(dt, 5), "problems_per_s": round(count / dt, 2), "t_setup_s": round(t_setup, 3),
            "iters_min": int(min(iters)), "iters_max": int(max(iters)), "iters_mean": float(np.mean(iters)),
            "max_stop_residual": worst, "n_total": int(sum(p.n for p in probs))}


def cpu_baseline():
    """The oracle on a bounded sample: the same generator at 32^3, factor + solve to tol."""
    import synth
    from oracle import dense, lobpcg, precond
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    p = synth.cfg2(N=32)
    na = dense.norm2(p.A)
    t0 = time.perf_counter()
    P = precond.Preconditioner(p.A, "fp64")
    r = lobpcg.lobpcg(p.A, p.X0, p.k, p.tol, precond=P, norm_a=na, stop="paper")
    dt = time.perf_counter() - t0
    return {"value": round(dt, 3), "unit": "s", "cores": threads, "kind": "oracle",
            "sample": f"same recipe at 32^3 (n=32768, k=16, m=32, tol=1e-10): oracle FP64 LOBPCG with SuperLU "
                      f"FP64 factor (single-threaded) + numpy BLAS, factor + solve, {r.iters} iterations; "
                      f"not scaled to 64^3"}


def traffic_from_profile():
    """HBM bytes per preconditioner application from the committed counter summary (FETCH_SIZE and
    WRITE_SIZE passes, each scaled by a copy of known size), or None once the solve sources differ
    from the ones the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "precond_traffic_diffusion3d_64.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ": " in line and line.split(": ", 1)[0] in ("traffic_bytes_per_application", "solve_sources_sha256",
                                                           "solve_sources"):
                k, v = line.rstrip("\n").split(": ", 1)
                fields[k] = v
    if len(fields) != 3:
        return None
    h = hashlib.sha256()
    for src in fields["solve_sources"].split():
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    return float(fields["traffic_bytes_per_application"]) if h.hexdigest() == fields["solve_sources_sha256"] else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffusion3d_64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--batched", type=int, default=256, help="problems in the batched run (0 = skip)")
    ap.add_argument("--pinvit-maxit", type=int, default=400, help="iteration cap of the PINVIT run (0 = skip)")
    ap.add_argument("--autotune", action="store_true", help="time the solve-plan split and reduction chunk at setup")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first copy a 256 MiB buffer once (reference dispatch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2302_12528_amd as pk

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.calibration_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    log(f"generating {args.workload}")
    p = workload(args.workload)
    X0 = torch.from_numpy(np.ascontiguousarray(p.X0)).cuda()
    log(f"setup mixed (fp32 factor), n={p.n}")
    t0 = time.perf_counter()
    mixed = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision="fp32", grid=p.grid, autotune=args.autotune)
    t_setup = time.perf_counter() - t0
    dt, infos, lam, X = time_steps(torch, mixed, X0, args.steps, args.warmup, "mixed")
    info = infos[-1]
    lam_np, X_np = lam.cpu().numpy(), X.cpu().numpy()

    # parity at full size: residuals recomputed on the host in FP64 against ||A||_2 from Lanczos
    from oracle import dense as odense
    na = odense.norm2(p.A)
    res = np.linalg.norm(p.A @ X_np - X_np * lam_np, axis=0) / (na * np.linalg.norm(X_np, axis=0))
    parity = {"max_residual": float(res.max()), "tol": p.tol, "norm2_lanczos": na,
              "orthonormality": float(np.max(np.abs(X_np.T @ X_np - np.eye(p.k))))}
    gold = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        ref = np.array(g["evals"])
        parity["max_eig_rel_err_vs_oracle"] = float(np.max(np.abs(lam_np - ref) / ref))

    # Dominant step: the preconditioner (lines 9-10: forward and backward supernodal sweeps), timed
    # live by the library with HIP events on its stream around every application inside the timed
    # solves.  Algorithmic bytes per application: the lower factor read once per sweep, lower(R)
    # read, the intermediate y written and read, and W (FP64) written.
    nnzL = info["nnz_factor"]
    n_pc = sum(i["n_precond"] for i in infos)
    ms_pc = 1e3 * sum(i["t_precond_gpu"] for i in infos) / max(1, n_pc)
    bytes_pc = 2 * nnzL * 4 + 3 * p.n * p.m * 4 + p.n * p.m * 8
    gbs_pc = bytes_pc / (ms_pc * 1e-3) / 1e9
    # SpMM A W (line 13), c = m, timed the same way: A's CSR arrays read once, W read, A W written.
    nnz = p.A.nnz
    n_sp = sum(i["n_spmm"] for i in infos)
    ms_spmm = 1e3 * sum(i["t_spmm_gpu"] for i in infos) / max(1, n_sp)
    bytes_spmm = 12 * nnz + 4 * (p.n + 1) + 2 * 8 * p.n * p.m
    gbs_spmm = bytes_spmm / (ms_spmm * 1e-3) / 1e9
    # the same two steps in isolation (back-to-back launches), for reference
    rng = np.random.default_rng(7)
    R = torch.from_numpy(rng.standard_normal((p.n, p.m))).cuda()
    ms_pc_iso = event_time(torch, lambda: mixed.apply_precond(R), args.reps)
    # Algorithm 1 (mixed-precision block PINVIT) on the same context and start block, one run to tol
    # (solve only: it reuses this context's FP32 factor)
    pinvit = None
    if args.pinvit_maxit > 0:
        log("pinvit")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam_pv, _, info_pv = mixed.pinvit(X0, maxit=args.pinvit_maxit, allow_not_converged=True)
        torch.cuda.synchronize()
        pinvit = {"t_solve_s": round(time.perf_counter() - t0, 5), "iters": info_pv["iters"],
                  "converged": info_pv["status"] == 0, "lobpcg_iters": info["iters"],
                  "max_eig_rel_diff_vs_lobpcg": float(np.max(np.abs(lam_pv.cpu().numpy() - lam_np) / lam_np))}
    mixed.close()

    fp64 = None
    if not args.no_fp64:
        log("setup fp64 factor")
        s64 = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision="fp64", grid=p.grid, qr_lower=False,
                        autotune=args.autotune)
        dt64, infos64, lam64, _ = time_steps(torch, s64, X0, max(1, min(args.steps, 2)), 1, "fp64")
        n64 = sum(i["n_precond"] for i in infos64)
        ms_pc64 = 1e3 * sum(i["t_precond_gpu"] for i in infos64) / max(1, n64)
        bytes_pc64 = 2 * nnzL * 8 + 3 * p.n * p.m * 8 + p.n * p.m * 8
        s64.close()
        fp64 = {"time_to_tol_s": round(dt64, 5), "iters": infos64[-1]["iters"],
                "t_factor_s": round(infos64[-1]["t_factor"], 5), "t_solve_s": round(infos64[-1]["t_solve"], 5),
                "precond_ms": round(ms_pc64, 4), "precond_GBs": round(bytes_pc64 / (ms_pc64 * 1e-3) / 1e9, 1),
                "max_eig_rel_diff_vs_mixed": float(np.max(np.abs(lam64.cpu().numpy() - lam_np) / lam_np))}

    out = {
        "metric": METRIC, "value": round(dt, 5), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: 3D 7-point variable-coefficient diffusion, n={p.n}, nnz={nnz}, "
                               f"k={p.k}, m={p.m}, tol={p.tol}, nested dissection, FP32 factor; step = numeric "
                               f"factorization + solve to tol",
                   "n": p.n, "k": p.k, "m": p.m, "tol": p.tol},
        "iters": info["iters"], "t_factor_s": round(info["t_factor"], 5), "t_solve_s": round(info["t_solve"], 5),
        "t_setup_s": round(t_setup, 3), "t_symbolic_s": round(info["t_symbolic"], 4),
        "nnz_factor": nnzL, "factor_flops": info["factor_flops"], "norm_a_estimate": info["norm_a"],
        "fp64": fp64,
        "speedup_vs_fp64": round(fp64["time_to_tol_s"] / dt, 3) if fp64 else None,
        "roofline": {"bound": "hbm", "achieved": round(gbs_pc, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs_pc / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(),
                     "kernel": "preconditioner application (forward + backward supernodal sweeps, FP32 factor), "
                               "HIP events around each application in the timed solves",
                     "ms": round(ms_pc, 4), "applications": n_pc, "algorithmic_bytes": bytes_pc,
                     "ms_isolated": round(ms_pc_iso, 4)},
        "spmm": {"ms": round(ms_spmm, 4), "GBs": round(gbs_spmm, 1), "frac": round(gbs_spmm / HBM_PEAK_GBS, 4),
                 "launches": n_sp, "algorithmic_bytes": bytes_spmm},
        "parity": parity,
        "pinvit": pinvit,
    }
    if args.batched > 0:
        out["batched"] = batched_run(torch, pk, 1, args.batched)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a 32^3 sample)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
