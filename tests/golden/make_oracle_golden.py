"""Write oracle eigenvalues for full-size workloads (calls only oracle/ and synth/).

Usage: python tests/golden/make_oracle_golden.py diffusion3d_64
Writes tests/golden/<name>.json with the oracle's k smallest eigenvalues,
its ||A||_2 (Lanczos), iteration count and timings; for dense_spd_<n> the
dense brute-force eigenvalues of the stored matrix; for laplace2d_5x5000 the
iteration counts of the three LOBPCG variants of section 5.1.  The oracle is the plain
FP64 LOBPCG of Algorithm 3 with an exact FP64 preconditioner, run to a
tolerance tighter than the GPU gate.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dense, lobpcg, precond  # noqa: E402


def run_dense(name):
    """Dense brute force (the plain definition of the result): the k smallest eigenvalues of the stored
    dense matrix by LAPACK's symmetric eigensolver, next to the prescribed spectrum it was built from."""
    p = synth.cfg3(n=int(name.split("_")[-1]))
    t0 = time.time()
    lam, _ = dense.smallest_eigenpairs(p.A, p.m + 1)
    t1 = time.time()
    spec = p.extra["spectrum"]
    out = {"workload": name, "n": p.n, "k": p.k, "m": p.m, "evals": lam[:p.k].tolist(),
           "eval_m_plus_1": float(lam[p.m]), "norm2": float(spec[-1]),
           "max_rel_dev_from_prescribed": float(np.max(np.abs(lam[:p.k] - spec[:p.k]) / spec[:p.k])),
           "t_eigh": t1 - t0,
           "note": "oracle dense brute force (numpy eigh of the stored symmetric matrix)"}
    path = os.path.join(os.path.dirname(__file__), f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "evals"}))


def run_paper2d(name):
    """The reconstructed 2D-Laplace test (5 x 5000 grid, k = 30, m = 45, tol = 1e-12, eq. (stop) with the
    exact ||A||_2 from the closed form): iteration counts of the three variants of section 5.1 from the
    seeded start block - DLOBPCG-dchol (FP64 factor), DLOBPCG-schol (FP32 factor) and MPLOBPCG-schol
    (FP32 factor plus the single-precision first stage to 5e-6)."""
    p = synth.paper2d()
    na = float(p.extra["eigs"][-1])
    out = {"workload": name, "n": p.n, "k": p.k, "m": p.m, "tol": p.tol, "stage1_tol": 5e-6, "norm2": na,
           "stop": "paper"}
    P64 = precond.Preconditioner(p.A, "fp64")
    P32 = precond.Preconditioner(p.A, "fp32")
    t0 = time.time()
    r = lobpcg.lobpcg(p.A, p.X0, p.k, p.tol, precond=P64, norm_a=na, maxit=5000, stop="paper")
    out["dchol_iters"] = r.iters
    r = lobpcg.lobpcg(p.A, p.X0, p.k, p.tol, precond=P32, norm_a=na, maxit=5000, stop="paper")
    out["schol_iters"] = r.iters
    r = lobpcg.mixed_lobpcg(p.A, p.X0, p.k, p.tol, 5e-6, precond=P32, norm_a=na, maxit=5000, stop="paper")
    out["mp_schol_stage1_iters"] = r.stage1_iters
    out["mp_schol_iters"] = r.iters
    out["converged"] = bool(r.converged and r.stage1_converged)
    out["max_rel_err_vs_closed_form"] = float(np.max(np.abs(r.evals - p.extra["eigs"][:p.k]) / p.extra["eigs"][:p.k]))
    out["t_total"] = time.time() - t0
    out["note"] = ("oracle LOBPCG (Algorithm 3) counts: dchol/schol = lines 2-17 with an FP64/FP32 factor; "
                   "mp_schol = line 1 in float32 to 5e-6, then lines 2-17 with the FP32 factor")
    path = os.path.join(os.path.dirname(__file__), f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def run(name):
    if name.startswith("dense_spd_"):
        return run_dense(name)
    if name == "laplace2d_5x5000":
        return run_paper2d(name)
    if name == "diffusion3d_64":
        p = synth.cfg2(N=64)
    elif name == "diffusion3d_48":
        p = synth.cfg2(N=48)
    elif name == "schrodinger3d_48":
        p = synth.cfg5(N=48)
    else:
        raise SystemExit(f"unknown workload {name}")
    t0 = time.time()
    na = dense.norm2(p.A)
    t1 = time.time()
    P = precond.Preconditioner(p.A, "fp64")
    t2 = time.time()
    r = lobpcg.lobpcg(p.A, p.X0, p.k, 1e-11, precond=P, norm_a=na, maxit=300)
    t3 = time.time()
    res = lobpcg.residual_norms(p.A, r.evecs, r.evals, na)
    out = {"workload": name, "n": p.n, "k": p.k, "m": p.m, "oracle_tol": 1e-11, "converged": bool(r.converged),
           "iters": r.iters, "evals": r.evals.tolist(), "norm2": na, "max_residual": float(res.max()),
           "t_norm": t1 - t0, "t_factor": t2 - t1, "t_solve": t3 - t2,
           "note": "oracle FP64 LOBPCG (Algorithm 3 loop, exact FP64 preconditioner, Householder QR)"}
    path = os.path.join(os.path.dirname(__file__), f"{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "evals"}))


if __name__ == "__main__":
    run(sys.argv[1])
