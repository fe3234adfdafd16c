#!/usr/bin/env python3
"""Time-to-tolerance of the mixed-precision LOBPCG hot path on one MI355X.

Workload: 3D 7-point variable-coefficient diffusion on a 64^3 grid (n = 262,144,
cell coefficients exp(N(0,1)), nested dissection), k = 16, m = 32, tol = 1e-10.
One step = numeric factorization of the permuted matrix (FP32 factor) plus
lobpcg_solve to tolerance with Algorithm 3 as a whole (MPLOBPCG-schol: the
single-precision first stage of line 1 to 5e-6, then the working-precision loop
with the FP32-factor preconditioner and Algorithm 2), with the matrix and start
block already on the GPU.  The same step with an FP64 factor (DLOBPCG-dchol:
FP64 Algorithm 2 step 1, no first stage) is timed on the same GPU for the
mixed-vs-FP64 comparison, and without the first stage (DLOBPCG-schol).  Side records: the dense SPD
workload (n = 8192), the batched Schrodinger workload, the backward of the 3D
Schrodinger workload, Algorithm 1 and the CPU oracle.  Prints one JSON line.
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


def batched_run(torch, pk, steps, count, graph=False):
    """Batched Schrodinger workload: `count` 2D operators (side U{48..128}), k=8, m=16, FP32 factors, one
    context; a step = numeric factorization of the union + lobpcg_solve_batched to tol for all of them."""
    import numpy as np
    import synth
    probs = synth.cfg4(count)
    log(f"batched: setup {count} problems, n total {sum(p.n for p in probs)}")
    t0 = time.perf_counter()
    bs = pk.BatchedSolver([p.A for p in probs], 8, 16, 1e-10, factor_precision="fp32",
                          grids=[p.grid for p in probs], graph=graph)
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
            "graph": graph,
            "time_to_tol_s": round(dt, 5), "problems_per_s": round(count / dt, 2), "t_setup_s": round(t_setup, 3),
            "iters_min": int(min(iters)), "iters_max": int(max(iters)), "iters_mean": float(np.mean(iters)),
            "max_stop_residual": worst, "n_total": int(sum(p.n for p in probs))}


def cpu_baseline():
    """The oracle on a bounded sample: the same generator at 32^3, factor + solve to tol, with the host's
    BLAS threads and again with one thread; next to it the oracle's full-size 64^3 time recorded when
    tests/golden/diffusion3d_64.json was written (on the 8-core build container, not this host)."""
    import synth
    from oracle import dense, lobpcg, precond
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    p = synth.cfg2(N=32)
    na = dense.norm2(p.A)

    def run():
        t0 = time.perf_counter()
        P = precond.Preconditioner(p.A, "fp64")
        r = lobpcg.lobpcg(p.A, p.X0, p.k, p.tol, precond=P, norm_a=na, stop="paper")
        return time.perf_counter() - t0, r.iters
    dt, iters = run()
    out = {"value": round(dt, 3), "unit": "s", "cores": threads, "kind": "oracle",
           "sample": f"same recipe at 32^3 (n=32768, k=16, m=32, tol=1e-10): oracle FP64 LOBPCG with SuperLU "
                     f"FP64 factor (single-threaded) + numpy BLAS, factor + solve, {iters} iterations; "
                     f"not scaled to 64^3"}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            dt1, _ = run()
        out["single_thread_s"] = round(dt1, 3)
    gold = os.path.join(ROOT, "tests", "golden", "diffusion3d_64.json")
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)
        out["full_size_64cubed"] = {"factor_s": round(g["t_factor"], 1), "solve_s": round(g["t_solve"], 1),
                                    "iters": g["iters"], "cores": 8,
                                    "where": "build container (8 cores), when the golden file was written"}
    return out


def dense_run(torch, pk, steps):
    """Dense SPD workload at full size (n = 8192, geometric spectrum in [1, 1e6], k = 32, m = 64, tol 1e-10 with
    the eigenvalue guard ||r_j||^2 <= 1e-12 |theta_j| (theta_m - theta_j)): time to tol with the FP32 dense factor
    (matrix cores) and with the FP64 one, the dense A W (FP64 matrix cores) and the two dense triangular solves."""
    import numpy as np
    import synth
    log("dense: generating dense_spd_8192")
    p = synth.cfg3()
    X0 = torch.from_numpy(np.ascontiguousarray(p.X0)).cuda()
    n, m = p.n, p.m
    out = {"workload": "dense_spd_8192: A = Q diag(geomspace(1, 1e6)) Q^T, n=8192, k=32, m=64, tol=1e-10, "
                       "eig_tol=1e-12; step = numeric factorization + solve to tol"}
    for prec, tol1 in (("fp32", 0.0), ("fp64", 0.0), ("fp32", 5e-6)):
        label = "mixed" if prec == "fp32" and tol1 == 0 else ("fp64" if prec == "fp64" else "mp_schol")
        log(f"dense: setup {label}")
        s = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision=prec, qr_lower=(prec == "fp32"), eig_tol=1e-12,
                      stage1_tol=tol1)
        dt, infos, lam, X = time_steps(torch, s, X0, steps if label == "mixed" else 1, 1, f"dense {label}")
        info = infos[-1]
        rec = {"time_to_tol_s": round(dt, 5), "iters": info["iters"], "t_factor_s": round(info["t_factor"], 5),
               "t_solve_s": round(info["t_solve"], 5)}
        if tol1 > 0:
            rec["stage1_iters"] = info["stage1_iters"]
            rec["t_stage1_s"] = round(info["t_stage1"], 5)
        lam = lam.cpu().numpy()
        spec = p.extra["spectrum"][: p.k]
        rec["max_eig_rel_err_vs_prescribed"] = float(np.max(np.abs(lam - spec) / spec))
        if label == "mixed":
            Xr = torch.randn(n, m, dtype=torch.float64, device="cuda")
            ms_mm = event_time(torch, lambda: s.apply_a(Xr), 20)
            ms_tr = event_time(torch, lambda: s.apply_precond(Xr), 20)
            flops = 2.0 * n * n * m
            out["dense_aw"] = {"ms": round(ms_mm, 4), "TFLOPs": round(flops / (ms_mm * 1e-3) / 1e12, 2),
                               "peak_TFLOPs": 78.6, "frac": round(flops / (ms_mm * 1e-3) / 1e12 / 78.6, 4),
                               "note": "A W, c = 64, FP64 matrix cores; 2 n^2 c flop"}
            out["dense_trisolve"] = {"ms": round(ms_tr, 4), "TFLOPs": round(flops / (ms_tr * 1e-3) / 1e12, 2),
                                     "peak_TFLOPs": 157.3, "frac": round(flops / (ms_tr * 1e-3) / 1e12 / 157.3, 4),
                                     "note": "two FP32 triangular solves with 64 right-hand sides (with the cast "
                                             "in and out); 2 n^2 c flop"}
        s.close()
        out[label] = rec
    out["speedup_vs_fp64"] = round(out["fp64"]["time_to_tol_s"] / out["mixed"]["time_to_tol_s"], 3)
    return out


def backward_run(torch, pk, fd_amps=2):
    """Differentiation workload at full size (3D -Laplacian + V on 48^3, V = 32 Gaussian bumps, loss = sum of the
    8 smallest eigenvalues + <x_1, g>^2): forward solve to tol 1e-12 with the FP32 factor, the adjoint, and
    central differences (h = 1e-6) of the loss on the first few amplitudes."""
    import numpy as np
    import synth
    from paper_2302_12528_amd.autograd import eigh_potential
    log("backward: generating schrodinger3d_48")
    p = synth.cfg5()
    L0, phi, a0, g = p.extra["L0"], p.extra["phi"], p.extra["amps"], p.extra["g"]
    s = pk.Solver(L0, p.k, p.m, 1e-12, factor_precision="fp32", grid=p.grid)
    phit = torch.from_numpy(phi).cuda()
    gt = torch.from_numpy(g).cuda()
    X0 = torch.from_numpy(np.ascontiguousarray(p.X0)).cuda()

    def loss_of(amp):
        lam, X = eigh_potential(phit @ amp, s, X0)
        return lam.sum() + (X[:, 0] @ gt) ** 2

    amp = torch.from_numpy(a0.copy()).cuda().requires_grad_(True)
    loss_of(amp.detach())   # warm-up (factorization plan, buffers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    L = loss_of(amp)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    (ga,) = torch.autograd.grad(L, amp)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pcg = s.backward_iters()
    ga = ga.cpu().numpy()
    fd = []
    h = 1e-6
    for q in range(fd_amps):
        e = torch.zeros_like(amp)
        e[q] = h
        with torch.no_grad():
            d = (loss_of(amp.detach() + e) - loss_of(amp.detach() - e)).item() / (2 * h)
        fd.append({"amp": q, "fd": d, "adjoint": float(ga[q]), "rel_diff": abs(d - ga[q]) / max(1.0, abs(ga[q]))})
    s.close()
    return {"workload": "schrodinger3d_48: -Laplacian + V on 48^3 (n=110592), 32 bumps, k=8, m=16, tol=1e-12, FP32 "
                        "factor; loss = sum of 8 eigenvalues + <x_1, g>^2",
            "t_forward_s": round(t1 - t0, 5), "t_backward_s": round(t2 - t1, 5), "adjoint_pcg_iters": pcg,
            "loss": float(L.item()), "fd_check": fd}


def hermitian_run(torch, pk):
    """Complex Hermitian workload: the reconstructed 5 x 5000 Laplacian with random node phases
    (D L D^H, D = diag(exp(i phi)); the paper's complex 2D-Laplace of section 5.5 stands behind it), k = 30,
    m = 32, tol = 1e-12 under eq. (stop) with the exact ||A||_2, through the real symmetric embedding:
    time to tol with the FP32 factor (and the first stage) and with the FP64 factor, same GPU."""
    import numpy as np
    import synth
    A = synth.gauge_laplace2d(5, 5000)
    eigs = synth.laplace2d_rect_eigs(5, 5000)
    na = float(eigs[-1])
    X0 = torch.from_numpy(synth.complex_block(25000, 32, 23)).cuda()
    out = {"workload": "gauge_laplace2d_5x5000: complex Hermitian D L D^H, n=25000, k=30, m=32, tol=1e-12; step "
                       "= numeric factorization + solve to tol"}
    for label, prec, tol1 in (("mixed", "fp32", 5e-6), ("fp64", "fp64", 0.0)):
        log(f"hermitian: {label}")
        s = pk.Solver(A, 30, 32, 1e-12, factor_precision=prec, grid=(5, 5000, 1), stop="paper", norm_a=na,
                      stage1_tol=tol1, qr_lower=(prec == "fp32"))
        for _ in range(1):
            s.factor()
            s.solve(X0, maxit=5000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.factor()
        lam, X, info = s.solve(X0, maxit=5000)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        lam = lam.cpu().numpy()
        out[label] = {"time_to_tol_s": round(dt, 5), "iters": info["iters"], "stage1_iters": info["stage1_iters"],
                      "max_eig_rel_err_vs_closed_form": float(np.max(np.abs(lam - eigs[:30]) / eigs[:30]))}
    out["speedup_vs_fp64"] = round(out["fp64"]["time_to_tol_s"] / out["mixed"]["time_to_tol_s"], 3)
    return out


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
    ap.add_argument("--stage1-tol", type=float, default=5e-6,
                    help="first-stage tolerance of the timed solve (Algorithm 3 line 1; 0 = no first stage)")
    ap.add_argument("--no-schol", action="store_true", help="skip the record without the first stage")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense n = 8192 record")
    ap.add_argument("--no-backward", action="store_true", help="skip the 48^3 backward record")
    ap.add_argument("--no-hermitian", action="store_true", help="skip the complex Hermitian record")
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
    log(f"setup mixed (fp32 factor, first stage to {args.stage1_tol}), n={p.n}")
    t0 = time.perf_counter()
    mixed = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision="fp32", grid=p.grid, autotune=args.autotune,
                      stage1_tol=args.stage1_tol)
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
    # Algorithmic bytes per application: the exact factor L (no explicit zeros) read once per sweep in FP32,
    # and 4 FP32 passes over the n x m right-hand side block: 2 * 4 * nnz(L) + 16 n m.  The supernodal
    # factor also stores the explicit zeros of its dense fronts and the solve writes W in FP64; the byte
    # count with those is reported beside it (stored_bytes).
    nnzL = info["nnz_factor"]
    nnzL_exact = pk.exact_fill(p.A, grid=p.grid)
    n_pc = sum(i["n_precond"] for i in infos)
    ms_pc = 1e3 * sum(i["t_precond_gpu"] for i in infos) / max(1, n_pc)
    bytes_pc = 2 * nnzL_exact * 4 + 16 * p.n * p.m
    bytes_pc_stored = 2 * nnzL * 4 + 3 * p.n * p.m * 4 + p.n * p.m * 8
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

    # DLOBPCG-schol: the same FP32 factor and Algorithm 2, without the first stage of line 1
    schol = None
    if not args.no_schol:
        log("setup schol (fp32 factor, no first stage)")
        sch = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision="fp32", grid=p.grid)
        dts, infos_s, lam_s, _ = time_steps(torch, sch, X0, max(1, min(args.steps, 3)), 1, "schol")
        sch.close()
        i_s = infos_s[-1]
        schol = {"time_to_tol_s": round(dts, 5), "iters": i_s["iters"], "t_factor_s": round(i_s["t_factor"], 5),
                 "t_solve_s": round(i_s["t_solve"], 5),
                 "max_eig_rel_diff_vs_mixed": float(np.max(np.abs(lam_s.cpu().numpy() - lam_np) / lam_np))}

    fp64 = None
    if not args.no_fp64:
        log("setup fp64 factor")
        s64 = pk.Solver(p.A, p.k, p.m, p.tol, factor_precision="fp64", grid=p.grid, qr_lower=False,
                        autotune=args.autotune)
        dt64, infos64, lam64, _ = time_steps(torch, s64, X0, max(1, min(args.steps, 2)), 1, "fp64")
        n64 = sum(i["n_precond"] for i in infos64)
        ms_pc64 = 1e3 * sum(i["t_precond_gpu"] for i in infos64) / max(1, n64)
        bytes_pc64 = 2 * nnzL_exact * 8 + 4 * 8 * p.n * p.m
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
                               f"k={p.k}, m={p.m}, tol={p.tol}, nested dissection, FP32 factor; Algorithm 3 with "
                               f"the single-precision first stage to {args.stage1_tol} (MPLOBPCG-schol); step = "
                               f"numeric factorization + solve to tol",
                   "n": p.n, "k": p.k, "m": p.m, "tol": p.tol, "stage1_tol": args.stage1_tol},
        "iters": info["iters"], "stage1_iters": info["stage1_iters"], "t_stage1_s": round(info["t_stage1"], 5),
        "t_factor_s": round(info["t_factor"], 5), "t_solve_s": round(info["t_solve"], 5),
        "t_setup_s": round(t_setup, 3), "t_symbolic_s": round(info["t_symbolic"], 4),
        "nnz_factor": nnzL, "factor_flops": info["factor_flops"], "norm_a_estimate": info["norm_a"],
        "fp64": fp64,
        "speedup_vs_fp64": round(fp64["time_to_tol_s"] / dt, 3) if fp64 else None,
        "roofline": {"bound": "hbm", "achieved": round(gbs_pc, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs_pc / HBM_PEAK_GBS, 4), "traffic": traffic_from_profile(),
                     "kernel": "preconditioner application (forward + backward supernodal sweeps, FP32 factor), "
                               "HIP events around each application in the working-precision iterations of the "
                               "timed solves",
                     "ms": round(ms_pc, 4), "applications": n_pc, "algorithmic_bytes": bytes_pc,
                     "nnz_factor_exact": nnzL_exact, "stored_bytes": bytes_pc_stored,
                     "frac_on_stored_bytes": round(bytes_pc_stored / (ms_pc * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "target_frac": 0.6, "ms_isolated": round(ms_pc_iso, 4)},
        "spmm": {"ms": round(ms_spmm, 4), "GBs": round(gbs_spmm, 1), "frac": round(gbs_spmm / HBM_PEAK_GBS, 4),
                 "launches": n_sp, "algorithmic_bytes": bytes_spmm},
        "parity": parity,
        "schol_no_stage1": schol,
        "pinvit": pinvit,
    }
    if args.batched > 0:
        out["batched"] = batched_run(torch, pk, 1, args.batched)
        out["batched_graph"] = batched_run(torch, pk, 1, args.batched, graph=True)
    if not args.no_dense:
        out["dense"] = dense_run(torch, pk, 2)
    if not args.no_backward:
        out["backward"] = backward_run(torch, pk)
    if not args.no_hermitian:
        out["hermitian"] = hermitian_run(torch, pk)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a 32^3 sample)")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
