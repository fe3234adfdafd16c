"""Python front end of liblobpcg: argument marshalling over the C-ABI only.

Every numerical step runs in the library's HIP kernels; torch provides device
memory (tensors) and the current stream.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np

from . import native as nv

_PREC = {"fp32": nv.LOBPCG_FP32, "fp64": nv.LOBPCG_FP64}
_STOP = {"paper": nv.LOBPCG_STOP_PAPER, "norma": nv.LOBPCG_STOP_NORMA}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("liblobpcg needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _stream():
    return ct.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _ptr(t) -> ct.c_void_p:
    return ct.c_void_p(t.data_ptr()) if t is not None else ct.c_void_p(None)


def _dev_f64(x, shape=None):
    torch = _torch()
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    x = x.to(device="cuda", dtype=torch.float64).contiguous()
    if shape is not None and tuple(x.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(x.shape)}")
    return x


@nv.ALLOC_FN
def _torch_alloc(nbytes, user):
    try:
        torch = _torch()
        return torch.cuda.caching_allocator_alloc(max(int(nbytes), 1), torch.cuda.current_device(),
                                                  torch.cuda.current_stream())
    except Exception:   # the library reports LOBPCG_ERR_ALLOC
        return None


@nv.FREE_FN
def _torch_free(ptr, user):
    import torch
    torch.cuda.caching_allocator_delete(ptr)


# lobpcg_allocator over torch's caching allocator: every device byte of a context is a torch block
TORCH_ALLOCATOR = nv.Allocator(_torch_alloc, _torch_free, None)


def _allocator(kind: str):
    if kind == "torch":
        return ct.pointer(TORCH_ALLOCATOR)
    if kind == "hip":
        return None
    raise ValueError(f"allocator must be 'torch' or 'hip', not {kind!r}")


def make_matrix(A, grid=(0, 0, 0)):
    """Build the lobpcg_matrix struct for a scipy CSR matrix or a dense numpy array.

    Returns (struct, keepalive) -- keep the second item alive while the struct is used.
    """
    M = nv.Matrix()
    M.grid[0], M.grid[1], M.grid[2] = [int(g) for g in grid]
    if isinstance(A, np.ndarray):
        cplx = np.iscomplexobj(A)
        Ad = np.ascontiguousarray(A, dtype=np.complex128 if cplx else np.float64)
        M.format = 3 if cplx else 1
        M.n = Ad.shape[0]
        M.ld = Ad.shape[1]
        M.dense = Ad.ctypes.data
        return M, (Ad,)
    import scipy.sparse as sp
    Ac = sp.csr_matrix(A)
    Ac.sort_indices()
    cplx = np.iscomplexobj(Ac.data)
    rp = np.ascontiguousarray(Ac.indptr, dtype=np.int32)
    ci = np.ascontiguousarray(Ac.indices, dtype=np.int32)
    va = np.ascontiguousarray(Ac.data, dtype=np.complex128 if cplx else np.float64)
    M.format = 2 if cplx else 0
    M.n = Ac.shape[0]
    M.nnz = va.size
    M.rowptr = rp.ctypes.data
    M.colind = ci.ctypes.data
    M.val = va.ctypes.data
    return M, (rp, ci, va)


def symbolic(A, grid=(0, 0, 0), leaf_size=0):
    """Host-only ordering and supernode statistics (no GPU)."""
    lib = nv.load()
    M, keep = make_matrix(A, grid)
    perm = np.zeros(M.n, dtype=np.int32)
    stats = np.zeros(8, dtype=np.float64)
    nv.check(lib.lobpcg_symbolic(ct.byref(M), leaf_size, perm.ctypes.data, stats.ctypes.data))
    del keep
    keys = ["supernodes", "levels", "nnz_factor", "flops", "max_front_rows", "max_supernode_cols",
            "update_entries", "panel_entries"]
    return perm, dict(zip(keys, stats.tolist()))


def exact_fill(A, grid=(0, 0, 0), leaf_size=0):
    """Entries of the exact Cholesky factor for the ordering setup builds (host only, no GPU)."""
    lib = nv.load()
    M, keep = make_matrix(A, grid)
    out = np.zeros(1, dtype=np.float64)
    nv.check(lib.lobpcg_exact_fill(ct.byref(M), leaf_size, out.ctypes.data))
    del keep
    return float(out[0])


class Solver:
    """k smallest eigenpairs of an SPD matrix with the mixed-precision LOBPCG of Algorithm 3."""

    def __init__(self, A, k: int, m: int, tol: float = 1e-10, factor_precision: str = "fp32",
                 grid=(0, 0, 0), leaf_size: int = 0, stop: str = "paper", qr_lower: bool = True,
                 norm_a: float = 0.0, eig_tol: float = 0.0, graph: bool = False, autotune: bool = False,
                 subtree_levels: int = 0, schur_wide_tiles: int = 0, stage1_tol: float = 0.0,
                 force_fp64_redo: bool = False, allocator: str = "torch"):
        self.lib = nv.load()
        _torch()
        M, keep = make_matrix(A, grid)
        opt = nv.Options()
        opt.allocator = _allocator(allocator)
        opt.leaf_size = leaf_size
        opt.subtree_levels = subtree_levels
        opt.schur_wide_tiles = schur_wide_tiles
        opt.stage1_tol = stage1_tol
        opt.stop_rule = _STOP[stop]
        opt.qr_lower = 1 if qr_lower else 0
        opt.norm_a = norm_a
        opt.eig_tol = eig_tol
        opt.flags = ((nv.LOBPCG_FLAG_GRAPH if graph else 0) | (nv.LOBPCG_FLAG_AUTOTUNE if autotune else 0) |
                     (nv.LOBPCG_FLAG_FORCE_FP64_REDO if force_fp64_redo else 0))
        ctx = ct.c_void_p()
        self.ctx = None
        self.hermitian = M.format in (2, 3)
        setup = self.lib.lobpcg_setup_hermitian if self.hermitian else self.lib.lobpcg_setup
        st = setup(ct.byref(M), k, m, tol, _PREC[factor_precision], _stream(), ct.byref(opt), ct.byref(ctx))
        del keep
        nv.check(st)
        self.ctx = ctx
        self.n, self.k, self.m = int(M.n), k, m
        self.factor_precision = factor_precision

    def close(self):
        if self.ctx is not None:
            self.lib.lobpcg_destroy(self.ctx)
            self.ctx = None

    def tuning(self) -> dict:
        out = np.zeros(3, dtype=np.int32)
        nv.check(self.lib.lobpcg_get_tuning(self.ctx, out.ctypes.data))
        return {"split_target": int(out[0]), "chunk_rows": int(out[1]),
                "source": ("default", "measured", "cache")[int(out[2])]}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, X0=None, maxit: int = 1000, allow_not_converged: bool = False):
        """(evals, evecs, info); evecs is complex128 (n x k) for a Hermitian matrix."""
        torch = _torch()
        if self.hermitian:
            x0 = None
            if X0 is not None:
                x0 = (torch.from_numpy(np.ascontiguousarray(X0, dtype=np.complex128)) if isinstance(X0, np.ndarray)
                      else X0).to(device="cuda", dtype=torch.complex128).contiguous()
                if tuple(x0.shape) != (self.n, self.m):
                    raise ValueError(f"expected shape {(self.n, self.m)}, got {tuple(x0.shape)}")
            evecs = torch.empty((self.n, self.k), dtype=torch.complex128, device="cuda")
            solve = self.lib.lobpcg_solve_hermitian
        else:
            x0 = _dev_f64(X0, (self.n, self.m)) if X0 is not None else None
            evecs = torch.empty((self.n, self.k), dtype=torch.float64, device="cuda")
            solve = self.lib.lobpcg_solve
        evals = torch.empty(self.k, dtype=torch.float64, device="cuda")
        info = nv.Info()
        res = np.zeros(self.k, dtype=np.float64)
        info.resid = res.ctypes.data
        allow = (nv.LOBPCG_OK, nv.LOBPCG_NOT_CONVERGED) if allow_not_converged else (nv.LOBPCG_OK,)
        st = solve(self.ctx, _ptr(x0), maxit, _ptr(evals), _ptr(evecs), ct.byref(info))
        nv.check(st, allow)
        out = {f: getattr(info, f) for f, _ in nv.Info._fields_ if f != "resid"}
        out["resid"] = res.copy()
        out["status"] = st
        return evals, evecs, out

    def pinvit(self, X0=None, maxit: int = 1000, allow_not_converged: bool = False, history: bool = False):
        """Algorithm 1 (mixed-precision block PINVIT) with this context's factor; returns evals, evecs, info
        (info["theta_hist"]: the k smallest Ritz values of each iteration when history is set)."""
        torch = _torch()
        x0 = _dev_f64(X0, (self.n, self.m)) if X0 is not None else None
        evals = torch.empty(self.k, dtype=torch.float64, device="cuda")
        evecs = torch.empty((self.n, self.k), dtype=torch.float64, device="cuda")
        info = nv.Info()
        res = np.zeros(self.k, dtype=np.float64)
        info.resid = res.ctypes.data
        hist = np.full((maxit, self.k), np.nan) if history else None
        allow = (nv.LOBPCG_OK, nv.LOBPCG_NOT_CONVERGED) if allow_not_converged else (nv.LOBPCG_OK,)
        st = self.lib.lobpcg_pinvit(self.ctx, _ptr(x0), maxit, _ptr(evals), _ptr(evecs), ct.byref(info),
                                    hist.ctypes.data if hist is not None else None)
        nv.check(st, allow)
        out = {f: getattr(info, f) for f, _ in nv.Info._fields_ if f != "resid"}
        out["resid"] = res.copy()
        out["status"] = st
        if hist is not None:
            out["theta_hist"] = hist[: out["iters"]].copy()
        return evals, evecs, out

    def factor(self):
        nv.check(self.lib.lobpcg_factor(self.ctx))

    def update_values(self, vals=None, shift=None):
        v = _dev_f64(vals) if vals is not None else None
        s = _dev_f64(shift, (self.n,)) if shift is not None else None
        nv.check(self.lib.lobpcg_update_values(self.ctx, _ptr(v), 1, _ptr(s)))

    def backward(self, d_evals=None, d_evecs=None):
        torch = _torch()
        de = _dev_f64(d_evals, (self.k,)) if d_evals is not None else None
        dx = _dev_f64(d_evecs, (self.n, self.k)) if d_evecs is not None else None
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        nv.check(self.lib.lobpcg_backward(self.ctx, _ptr(de), _ptr(dx), _ptr(out)))
        return out

    def backward_iters(self) -> int:
        """Projected PCG iterations of the latest backward()."""
        return int(self.lib.lobpcg_backward_iters(self.ctx))

    def permutation(self) -> np.ndarray:
        perm = np.zeros(self.n, dtype=np.int32)
        nv.check(self.lib.lobpcg_get_permutation(self.ctx, perm.ctypes.data))
        return perm

    def apply_a(self, X):
        """Y = A_perm X for a device block X (n x c) in the permuted ordering."""
        torch = _torch()
        X = _dev_f64(X)
        c = X.shape[1]
        Y = torch.empty_like(X)
        nv.check(self.lib.lobpcg_apply_a(self.ctx, _ptr(X), c, _ptr(Y), c, c))
        return Y

    def apply_precond(self, R):
        """W = working(f_T(lower(R))) for R (n x m, permuted ordering)."""
        torch = _torch()
        R = _dev_f64(R, (self.n, self.m))
        W = torch.empty_like(R)
        nv.check(self.lib.lobpcg_apply_precond(self.ctx, _ptr(R), _ptr(W)))
        return W


class BatchedSolver:
    """k smallest eigenpairs of each of several SPD matrices (one context, one factorization of their
    block-diagonal union, per-problem convergence)."""

    def __init__(self, mats, k: int, m: int, tol: float = 1e-10, factor_precision: str = "fp32",
                 grids=None, leaf_size: int = 0, stop: str = "paper", qr_lower: bool = True,
                 eig_tol: float = 0.0, graph: bool = False, autotune: bool = False, stage1_tol: float = 0.0,
                 allocator: str = "torch"):
        self.lib = nv.load()
        _torch()
        count = len(mats)
        if count < 1:
            raise ValueError("need at least one matrix")
        grids = grids if grids is not None else [(0, 0, 0)] * count
        arr = (nv.Matrix * count)()
        keep = []
        for b, A in enumerate(mats):
            M, kp = make_matrix(A, grids[b])
            arr[b] = M
            keep.append(kp)
        opt = nv.Options()
        opt.leaf_size = leaf_size
        opt.stop_rule = _STOP[stop]
        opt.qr_lower = 1 if qr_lower else 0
        opt.eig_tol = eig_tol
        opt.stage1_tol = stage1_tol
        opt.allocator = _allocator(allocator)
        opt.flags = (nv.LOBPCG_FLAG_GRAPH if graph else 0) | (nv.LOBPCG_FLAG_AUTOTUNE if autotune else 0)
        ctx = ct.c_void_p()
        self.ctx = None
        st = self.lib.lobpcg_setup_batched(arr, count, k, m, tol, _PREC[factor_precision], _stream(),
                                           ct.byref(opt), ct.byref(ctx))
        del keep
        nv.check(st)
        self.ctx = ctx
        self.sizes = [int(arr[b].n) for b in range(count)]
        self.count, self.k, self.m = count, k, m

    def close(self):
        if self.ctx is not None:
            self.lib.lobpcg_destroy(self.ctx)
            self.ctx = None

    def tuning(self) -> dict:
        out = np.zeros(3, dtype=np.int32)
        nv.check(self.lib.lobpcg_get_tuning(self.ctx, out.ctypes.data))
        return {"split_target": int(out[0]), "chunk_rows": int(out[1]),
                "source": ("default", "measured", "cache")[int(out[2])]}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, X0s=None, maxit: int = 1000, allow_not_converged: bool = False):
        """Returns (list of evals, list of evecs, list of info dicts, overall status)."""
        torch = _torch()
        B = self.count
        x0 = [(_dev_f64(X0s[b], (self.sizes[b], self.m)) if X0s is not None and X0s[b] is not None else None)
              for b in range(B)]
        evals = [torch.empty(self.k, dtype=torch.float64, device="cuda") for _ in range(B)]
        evecs = [torch.empty((self.sizes[b], self.k), dtype=torch.float64, device="cuda") for b in range(B)]
        P = ct.c_void_p * B
        px0 = P(*[(t.data_ptr() if t is not None else None) for t in x0])
        pev = P(*[t.data_ptr() for t in evals])
        pec = P(*[t.data_ptr() for t in evecs])
        infos = (nv.Info * B)()
        res = [np.zeros(self.k, dtype=np.float64) for _ in range(B)]
        for b in range(B):
            infos[b].resid = res[b].ctypes.data
        allow = (nv.LOBPCG_OK, nv.LOBPCG_NOT_CONVERGED) if allow_not_converged else (nv.LOBPCG_OK,)
        st = self.lib.lobpcg_solve_batched(self.ctx, px0, maxit, pev, pec, infos)
        nv.check(st, allow)
        outs = []
        for b in range(B):
            o = {f: getattr(infos[b], f) for f, _ in nv.Info._fields_ if f != "resid"}
            o["resid"] = res[b].copy()
            outs.append(o)
        return evals, evecs, outs, st


def mixed_qr(W, lower: bool = True, ld: int = 0):
    """Algorithm 2 on a device block W (n x c); returns (Q, R).  ld > c runs it on W held in the first
    c columns of an n x ld buffer (the other columns are left untouched)."""
    torch = _torch()
    lib = nv.load()
    W = _dev_f64(W)
    n, c = W.shape
    ld = max(ld, c)
    buf = torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda")
    buf[:, :c] = W
    R = torch.empty((c, c), dtype=torch.float64, device="cuda")
    nv.check(lib.lobpcg_mixed_qr(_ptr(buf), n, c, ld, 1 if lower else 0, _ptr(R), _stream()))
    if ld > c and not bool(torch.all(buf[:, c:] == 7.0)):
        raise RuntimeError("lobpcg_mixed_qr wrote outside the block's columns")
    return buf[:, :c].contiguous(), R


def gram(X, Y):
    torch = _torch()
    lib = nv.load()
    X = _dev_f64(X)
    Y = _dev_f64(Y)
    G = torch.empty((X.shape[1], Y.shape[1]), dtype=torch.float64, device="cuda")
    nv.check(lib.lobpcg_gram(_ptr(X), X.shape[1], _ptr(Y), Y.shape[1], X.shape[0], X.shape[1], Y.shape[1], _ptr(G),
                             _stream()))
    return G


def syev_small(H, nev=None):
    torch = _torch()
    lib = nv.load()
    H = _dev_f64(H)
    c = H.shape[0]
    nev = c if nev is None else int(nev)
    w = torch.empty(nev, dtype=torch.float64, device="cuda")
    V = torch.empty((c, c), dtype=torch.float64, device="cuda")
    nv.check(lib.lobpcg_syev_small(_ptr(H), c, nev, _ptr(w), _ptr(V), _stream()))
    return w, V[:, :nev]
