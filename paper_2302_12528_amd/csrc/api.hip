// C-ABI of liblobpcg (include/lobpcg.h): context, setup, factorization and the
// Algorithm 3 working-precision loop driven from the host, with every
// numerical step in the HIP kernels of k_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lobpcg.h"
#include "common.hpp"
#include "symbolic.hpp"

using namespace lobpcg;

namespace {

thread_local std::string g_last_error;

lobpcg_status fail(lobpcg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(LOBPCG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define ST_TRY(expr)                    \
  do {                                  \
    lobpcg_status s_ = (expr);          \
    if (s_ != LOBPCG_OK) return s_;     \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int pad_m(int m) { return m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : 64; }

}  // namespace

struct lobpcg_ctx_s {
  hipStream_t st = nullptr;
  int64_t n = 0, nnz = 0;
  int k = 0, m = 0, mp = 0;
  double tol = 0;
  lobpcg_precision prec = LOBPCG_FP32;
  lobpcg_options opt{};
  bool dense = false;
  Symbolic S;
  FactorPlan FP;
  SolvePlan SP;
  FactorDev FD{};
  SolveDev SD{};
  std::vector<void*> allocs;
  // matrix
  int32_t *d_prow = nullptr, *d_pcol = nullptr, *d_vmap = nullptr, *d_perm = nullptr, *d_iperm = nullptr;
  double *d_aval_orig = nullptr, *d_aval = nullptr, *d_dense = nullptr;
  int64_t ld_dense = 0;
  // factor (T = float or double)
  void *panel = nullptr, *upd = nullptr, *dinv = nullptr, *lcopy = nullptr;
  int* d_flag = nullptr;   // [0] factor breakdown, [1] alg2 breakdown, [2] syev sweeps
  // iteration
  double* Sb[2] = {nullptr, nullptr};
  double* ASb[2] = {nullptr, nullptr};
  void *rhs = nullptr, *ybuf = nullptr, *xbuf = nullptr, *uvec = nullptr, *fpart = nullptr, *bpart = nullptr;
  double *gpart = nullptr, *H = nullptr, *Cev = nullptr, *evals = nullptr, *Gupd = nullptr, *Gc = nullptr;
  double *norms = nullptr, *rpart = nullptr, *syev_work = nullptr;
  void *tsqr_ws = nullptr, *Rl = nullptr;
  double *Gv = nullptr, *Tm = nullptr;
  double norm_a = 0;
  int cur = 0;
  bool solved = false;
  double t_symbolic = 0, t_factor = 0;
  int fallbacks = 0;
  // backward (adjoint) buffers, allocated on first use
  double* bw_g = nullptr;
  double* bw_blk[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double* bw_small = nullptr;
  double* bw_part = nullptr;
  int bw_iters = 0;

  template <typename X>
  lobpcg_status alloc(X*& p, int64_t count) {
    p = nullptr;
    if (count <= 0) count = 1;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)count * sizeof(X));
    if (e != hipSuccess) return fail(LOBPCG_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
    allocs.push_back(q);
    p = static_cast<X*>(q);
    return LOBPCG_OK;
  }
  lobpcg_status alloc_bytes(void*& p, int64_t bytes) {
    char* c = nullptr;
    lobpcg_status s = alloc(c, bytes);
    p = c;
    return s;
  }
  ~lobpcg_ctx_s() {
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

template <typename V>
lobpcg_status upload(lobpcg_ctx c, V*& dst, const std::vector<V>& src) {
  ST_TRY(c->alloc(dst, (int64_t)src.size()));
  if (!src.empty()) HIP_TRY(hipMemcpy(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
  return LOBPCG_OK;
}

lobpcg_status validate_matrix(const lobpcg_matrix* A) {
  if (!A) return fail(LOBPCG_ERR_INVALID_ARG, "A is NULL");
  if (A->n < 1 || A->n > (int64_t)INT32_MAX - 1) return fail(LOBPCG_ERR_INVALID_ARG, "n out of range");
  const int64_t n = A->n;
  if (A->format == 1) {
    if (!A->dense) return fail(LOBPCG_ERR_INVALID_ARG, "dense pointer is NULL");
    if (A->ld < n) return fail(LOBPCG_ERR_INVALID_ARG, "ld < n");
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j <= i; ++j) {
        const double a = A->dense[i * A->ld + j], b = A->dense[j * A->ld + i];
        if (!std::isfinite(a)) return fail(LOBPCG_ERR_INVALID_ARG, "non-finite matrix entry");
        if (std::fabs(a - b) > 1e-12 * std::max(std::fabs(a), std::fabs(b)))
          return fail(LOBPCG_ERR_INVALID_ARG, "matrix is not symmetric");
      }
    for (int64_t i = 0; i < n; ++i)
      if (!(A->dense[i * A->ld + i] > 0)) return fail(LOBPCG_ERR_INVALID_ARG, "non-positive diagonal");
    return LOBPCG_OK;
  }
  if (A->format != 0) return fail(LOBPCG_ERR_INVALID_ARG, "format must be 0 (CSR) or 1 (dense)");
  if (!A->rowptr || !A->colind || !A->val) return fail(LOBPCG_ERR_INVALID_ARG, "CSR pointer is NULL");
  if (A->rowptr[0] != 0 || A->rowptr[n] != A->nnz || A->nnz < n)
    return fail(LOBPCG_ERR_INVALID_ARG, "rowptr inconsistent with nnz");
  for (int64_t i = 0; i < n; ++i) {
    const int32_t e0 = A->rowptr[i], e1 = A->rowptr[i + 1];
    if (e1 < e0) return fail(LOBPCG_ERR_INVALID_ARG, "rowptr not monotone");
    bool diag = false;
    for (int32_t e = e0; e < e1; ++e) {
      const int32_t j = A->colind[e];
      if (j < 0 || j >= n) return fail(LOBPCG_ERR_INVALID_ARG, "column index out of range");
      if (e > e0 && A->colind[e - 1] >= j) return fail(LOBPCG_ERR_INVALID_ARG, "columns not sorted/unique");
      if (!std::isfinite(A->val[e])) return fail(LOBPCG_ERR_INVALID_ARG, "non-finite matrix entry");
      if (j == i) {
        diag = true;
        if (!(A->val[e] > 0)) return fail(LOBPCG_ERR_INVALID_ARG, "non-positive diagonal");
      }
      // symmetric pattern and values
      const int32_t* b = A->colind + A->rowptr[j];
      const int32_t* en = A->colind + A->rowptr[j + 1];
      const int32_t* it = std::lower_bound(b, en, (int32_t)i);
      if (it == en || *it != i) return fail(LOBPCG_ERR_INVALID_ARG, "pattern is not symmetric");
      const double a = A->val[e], t = A->val[it - A->colind];
      if (std::fabs(a - t) > 1e-12 * std::max(std::fabs(a), std::fabs(t)))
        return fail(LOBPCG_ERR_INVALID_ARG, "matrix is not symmetric");
    }
    if (!diag) return fail(LOBPCG_ERR_INVALID_ARG, "missing diagonal entry");
  }
  return LOBPCG_OK;
}

lobpcg_status check_launch(const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LOBPCG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
  return LOBPCG_OK;
}

// Y = A X in the permuted basis
void apply_a(lobpcg_ctx c, const double* X, int64_t ldx, double* Y, int64_t ldy, int cols) {
  if (c->dense)
    launch_dense_mm(c->d_dense, c->ld_dense, c->n, X, ldx, Y, ldy, cols, c->st);
  else
    launch_spmm_csr(c->d_prow, c->d_pcol, c->d_aval, c->n, X, ldx, Y, ldy, cols, c->st);
}

template <typename T>
lobpcg_status factor_t(lobpcg_ctx c) {
  T* panel = static_cast<T*>(c->panel);
  T* upd = static_cast<T*>(c->upd);
  T* dinv = static_cast<T*>(c->dinv);
  T* lcopy = static_cast<T*>(c->lcopy);
  for (const FactorPlan::Step& s : c->FP.steps) {
    const int64_t a0 = c->FP.asm_level_off[s.level], a1 = c->FP.asm_level_off[s.level + 1];
    launch_factor_step<T>(c->FD, s.kind, s.level, s.off, s.count, a0, a1 - a0, panel, upd, dinv, lcopy, c->d_flag,
                          c->st);
  }
  return check_launch("factorization");
}

lobpcg_status factor(lobpcg_ctx c) {
  const double t0 = now_s();
  HIP_TRY(hipMemsetAsync(c->d_flag, 0, 4 * sizeof(int), c->st));
  ST_TRY(c->prec == LOBPCG_FP32 ? factor_t<float>(c) : factor_t<double>(c));
  int flag[4];
  HIP_TRY(hipMemcpyAsync(flag, c->d_flag, sizeof(flag), hipMemcpyDeviceToHost, c->st));
  HIP_TRY(hipStreamSynchronize(c->st));
  c->t_factor = now_s() - t0;
  if (flag[0] != 0)
    return fail(LOBPCG_ERR_FACTOR_BREAKDOWN,
                "non-positive pivot in the " + std::string(c->prec == LOBPCG_FP32 ? "FP32" : "FP64") +
                    " Cholesky factor at permuted column " + std::to_string(flag[0] - 1));
  return LOBPCG_OK;
}

// W = working(f_T(lower(rhs))): rhs already holds lower(R) (T, n x mp); W (n x mw, ldw)
template <typename T>
void precond_t(lobpcg_ctx c, double* W, int64_t ldw, int mw) {
  launch_precond<T>(c->FD, c->SD, c->S.nlevels, c->mp, static_cast<const T*>(c->panel), static_cast<T*>(c->rhs),
                    static_cast<T*>(c->ybuf), static_cast<T*>(c->xbuf), static_cast<T*>(c->uvec),
                    static_cast<T*>(c->fpart), static_cast<T*>(c->bpart), W, ldw, mw, c->st);
}

void precond(lobpcg_ctx c, double* W, int64_t ldw, int mw = -1) {
  if (mw < 0) mw = c->m;
  if (c->prec == LOBPCG_FP32)
    precond_t<float>(c, W, ldw, mw);
  else
    precond_t<double>(c, W, ldw, mw);
}

// rhs = lower(R) for R (n x cols, ld), zero padded to the solve width
void load_rhs(lobpcg_ctx c, const double* R, int64_t ld, int cols) {
  if (c->prec == LOBPCG_FP32)
    launch_cast_to<float>(R, ld, static_cast<float*>(c->rhs), c->n, cols, c->mp, c->st);
  else
    launch_cast_to<double>(R, ld, static_cast<double*>(c->rhs), c->n, cols, c->mp, c->st);
}

// Algorithm 2 on W (n x cc, ld) in place; flag set on a step-3 breakdown.
template <typename T>
void mixed_qr_t(hipStream_t st, double* W, int64_t ld, int64_t n, int cc, void* ws, void* Rl_, double* Lt,
                double* Gv, double* gpart, int* flag, double* Rout) {
  T* Rl = static_cast<T*>(Rl_);
  launch_tsqr<T>(W, ld, n, cc, static_cast<T*>(ws), Rl, st);      // step 1: lower(W) = Q_l R_l
  launch_trsm_rows<T>(W, ld, n, cc, Rl, st);                       // step 2: V = W working(R_l)^{-1}
  launch_gram(W, ld, W, ld, n, cc, cc, Gv, gpart, st);             // step 3: V^T V = L L^T
  launch_chol_upper<T>(Gv, Rl, cc, Lt, Rout, flag, st);
  launch_trsm_rows<double>(W, ld, n, cc, Lt, st);                  // step 4: Q = V L^{-T}
}

lobpcg_status ortho(lobpcg_ctx c, double* W, int64_t ld, int cc) {
  int flag = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const bool lower = (attempt == 0) && c->opt.qr_lower;
    HIP_TRY(hipMemsetAsync(c->d_flag + 1, 0, sizeof(int), c->st));
    if (lower)
      mixed_qr_t<float>(c->st, W, ld, c->n, cc, c->tsqr_ws, c->Rl, c->Tm, c->Gv, c->gpart, c->d_flag + 1, nullptr);
    else
      mixed_qr_t<double>(c->st, W, ld, c->n, cc, c->tsqr_ws, c->Rl, c->Tm, c->Gv, c->gpart, c->d_flag + 1,
                         nullptr);
    ST_TRY(check_launch("mixed QR"));
    HIP_TRY(hipMemcpyAsync(&flag, c->d_flag + 1, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(hipStreamSynchronize(c->st));
    if (flag == 0) return LOBPCG_OK;
    if (!lower) break;
    c->fallbacks++;
  }
  return fail(LOBPCG_ERR_ORTHO_BREAKDOWN, "Algorithm 2 Cholesky of V^T V failed (W rank deficient)");
}

}  // namespace

extern "C" {

const char* lobpcg_status_string(lobpcg_status s) {
  switch (s) {
    case LOBPCG_OK: return "ok";
    case LOBPCG_NOT_CONVERGED: return "not converged";
    case LOBPCG_ERR_INVALID_ARG: return "invalid argument";
    case LOBPCG_ERR_FACTOR_BREAKDOWN: return "factor breakdown";
    case LOBPCG_ERR_ORTHO_BREAKDOWN: return "orthogonalization breakdown";
    case LOBPCG_ERR_NONFINITE: return "non-finite values";
    case LOBPCG_ERR_ALLOC: return "allocation failure";
    case LOBPCG_ERR_HIP: return "HIP runtime error";
    case LOBPCG_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* lobpcg_last_error(void) { return g_last_error.c_str(); }

lobpcg_status lobpcg_setup(const lobpcg_matrix* A, int32_t k, int32_t m, double tol,
                           lobpcg_precision factor_precision, void* hip_stream, const lobpcg_options* opts,
                           lobpcg_ctx* out) {
  if (!out) return fail(LOBPCG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ST_TRY(validate_matrix(A));
  const int64_t n = A->n;
  if (k < 1 || m < k) return fail(LOBPCG_ERR_INVALID_ARG, "need 1 <= k <= m");
  if (m > 64) return fail(LOBPCG_ERR_INVALID_ARG, "block size m must be <= 64");
  if (A->format == 1 && A->n > 16384) return fail(LOBPCG_ERR_INVALID_ARG, "dense matrices are limited to n <= 16384");
  if (3 * (int64_t)m > n) return fail(LOBPCG_ERR_INVALID_ARG, "need 3m <= n");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(LOBPCG_ERR_INVALID_ARG, "tol must be positive and finite");
  if (factor_precision != LOBPCG_FP32 && factor_precision != LOBPCG_FP64)
    return fail(LOBPCG_ERR_INVALID_ARG, "factor_precision must be LOBPCG_FP32 or LOBPCG_FP64");
  lobpcg_options opt{};
  opt.leaf_size = 64;
  opt.stop_rule = LOBPCG_STOP_PAPER;
  opt.qr_lower = 1;
  if (opts) {
    opt = *opts;
    if (opt.leaf_size <= 0) opt.leaf_size = 64;
    if (opt.stop_rule != LOBPCG_STOP_PAPER && opt.stop_rule != LOBPCG_STOP_NORMA)
      return fail(LOBPCG_ERR_INVALID_ARG, "stop_rule");
    if (opt.norm_a < 0 || !std::isfinite(opt.norm_a)) return fail(LOBPCG_ERR_INVALID_ARG, "norm_a");
    if (opt.eig_tol < 0 || !std::isfinite(opt.eig_tol)) return fail(LOBPCG_ERR_INVALID_ARG, "eig_tol");
  }
  auto c = new lobpcg_ctx_s();
  lobpcg_ctx_s& C = *c;
  C.st = static_cast<hipStream_t>(hip_stream);
  C.n = n;
  C.k = k;
  C.m = m;
  C.mp = pad_m(m);
  C.tol = tol;
  C.prec = factor_precision;
  C.opt = opt;
  C.dense = (A->format == 1);
  // ---- host symbolic analysis (pattern only) ----
  const double t0 = now_s();
  std::string err = analyze(n, C.dense ? nullptr : A->rowptr, C.dense ? nullptr : A->colind, A->grid, C.dense,
                            opt.leaf_size, C.S);
  if (!err.empty()) {
    delete c;
    return fail(LOBPCG_ERR_INVALID_ARG, "symbolic analysis: " + err);
  }
  build_factor_plan(C.S, C.FP);
  build_solve_plan(C.S, 64, 256, C.SP);
  std::vector<int32_t> prow, pcol, vmap, apos;
  if (!C.dense) {
    permute_pattern(C.S, A->rowptr, A->colind, prow, pcol, vmap);
    assembly_positions(C.S, prow, pcol, apos);
    C.nnz = A->nnz;
  }
  err = verify(C.S, C.FP, C.SP, prow, apos);
  if (!err.empty()) {
    delete c;
    return fail(LOBPCG_ERR_INVALID_ARG, "symbolic structures failed verification: " + err);
  }
  C.t_symbolic = now_s() - t0;
  auto cleanup = [&](lobpcg_status s) {
    delete c;
    return s;
  };
#define SETUP_TRY(expr)                 \
  do {                                  \
    lobpcg_status s_ = (expr);          \
    if (s_ != LOBPCG_OK) return cleanup(s_); \
  } while (0)
  // ---- device structures ----
  const Symbolic& S = C.S;
  FactorDev& D = C.FD;
  D.max_nr = S.max_nr;
  SETUP_TRY(upload(c, D.begin, S.begin));
  SETUP_TRY(upload(c, D.nc, S.nc));
  SETUP_TRY(upload(c, D.nr, S.nr));
  SETUP_TRY(upload(c, D.rows, S.rows));
  SETUP_TRY(upload(c, D.row_off, S.row_off));
  SETUP_TRY(upload(c, D.relpos, S.relpos));
  SETUP_TRY(upload(c, D.child_ptr, S.child_ptr));
  SETUP_TRY(upload(c, D.child_list, S.child_list));
  SETUP_TRY(upload(c, D.inv_off, S.inv_off));
  SETUP_TRY(upload(c, D.invmap, S.invmap));
  SETUP_TRY(upload(c, D.panel_off, S.panel_off));
  SETUP_TRY(upload(c, D.upd_off, S.upd_off));
  SETUP_TRY(upload(c, D.uvec_off, S.uvec_off));
  SETUP_TRY(upload(c, D.dinv_off, S.dinv_off));
  SETUP_TRY(upload(c, D.lcopy_off, S.lcopy_off));
  SETUP_TRY(upload(c, D.asm_items, C.FP.asm_items));
  SETUP_TRY(upload(c, D.tasks, C.FP.tasks));
  SETUP_TRY(upload(c, D.ownrow_items, C.FP.ownrow_items));
  {
    int32_t *fi = nullptr, *ff = nullptr, *bi = nullptr, *bf = nullptr;
    SETUP_TRY(upload(c, fi, C.SP.fwd_items));
    SETUP_TRY(upload(c, ff, C.SP.fwd_fin));
    SETUP_TRY(upload(c, bi, C.SP.bwd_items));
    SETUP_TRY(upload(c, bf, C.SP.bwd_fin));
    C.SD.fwd_items = fi;
    C.SD.fwd_fin = ff;
    C.SD.bwd_items = bi;
    C.SD.bwd_fin = bf;
    C.SD.fwd_level_off = C.SP.fwd_level_off.data();
    C.SD.fwd_fin_level_off = C.SP.fwd_fin_level_off.data();
    C.SD.bwd_level_off = C.SP.bwd_level_off.data();
    C.SD.bwd_fin_level_off = C.SP.bwd_fin_level_off.data();
    C.SD.ownrow_level_off = C.FP.ownrow_level_off.data();
  }
  SETUP_TRY(upload(c, C.d_perm, S.perm));
  SETUP_TRY(upload(c, C.d_iperm, S.iperm));
  if (C.dense) {
    C.ld_dense = n;
    SETUP_TRY(C.alloc(C.d_dense, n * n));
    if (hipMemcpy2D(C.d_dense, n * sizeof(double), A->dense, A->ld * sizeof(double), n * sizeof(double), n,
                    hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(LOBPCG_ERR_HIP, "copy of dense A failed"));
    D.dense = C.d_dense;
    D.ld_dense = n;
    D.is_dense = 1;
  } else {
    SETUP_TRY(upload(c, C.d_prow, prow));
    SETUP_TRY(upload(c, C.d_pcol, pcol));
    SETUP_TRY(upload(c, C.d_vmap, vmap));
    SETUP_TRY(upload(c, D.apos, apos));
    SETUP_TRY(C.alloc(C.d_aval_orig, C.nnz));
    SETUP_TRY(C.alloc(C.d_aval, C.nnz));
    if (hipMemcpy(C.d_aval_orig, A->val, C.nnz * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(LOBPCG_ERR_HIP, "copy of A values failed"));
    launch_gather_values(C.d_aval_orig, C.d_vmap, C.d_aval, C.nnz, C.st);   // Pi^T A Pi, once
    D.prow = C.d_prow;
    D.pcol = C.d_pcol;
    D.aval = C.d_aval;
    D.is_dense = 0;
  }
  // ---- factor storage ----
  const size_t tsz = (C.prec == LOBPCG_FP32) ? 4 : 8;
  SETUP_TRY(C.alloc_bytes(C.panel, S.panel_total * tsz));
  SETUP_TRY(C.alloc_bytes(C.upd, S.upd_total * tsz));
  SETUP_TRY(C.alloc_bytes(C.dinv, S.dinv_total * tsz));
  SETUP_TRY(C.alloc_bytes(C.lcopy, S.lcopy_max * tsz));
  SETUP_TRY(C.alloc(C.d_flag, 4));
  // ---- iteration buffers ----
  const int m3 = 3 * m;
  for (int b = 0; b < 2; ++b) {
    SETUP_TRY(C.alloc(C.Sb[b], n * m3));
    SETUP_TRY(C.alloc(C.ASb[b], n * m3));
  }
  SETUP_TRY(C.alloc_bytes(C.rhs, n * C.mp * tsz));
  SETUP_TRY(C.alloc_bytes(C.ybuf, n * C.mp * tsz));
  SETUP_TRY(C.alloc_bytes(C.xbuf, n * C.mp * tsz));
  SETUP_TRY(C.alloc_bytes(C.uvec, std::max<int64_t>(1, S.uvec_total) * C.mp * tsz));
  SETUP_TRY(C.alloc_bytes(C.fpart, std::max<int64_t>(1, C.SP.fwd_slots) * 64 * C.mp * tsz));
  SETUP_TRY(C.alloc_bytes(C.bpart, std::max<int64_t>(1, C.SP.bwd_slots) * 64 * C.mp * tsz));
  if (hipMemset(C.rhs, 0, n * C.mp * tsz) != hipSuccess) return cleanup(fail(LOBPCG_ERR_HIP, "memset"));
  int64_t gp = std::max(gram_scratch(n, m3, m3), gram_scratch(n, m, m));
  gp = std::max(gp, gram_scratch(n, 2 * m, m));
  SETUP_TRY(C.alloc(C.gpart, gp));
  SETUP_TRY(C.alloc(C.H, m3 * m3));
  SETUP_TRY(C.alloc(C.Cev, m3 * m3));
  SETUP_TRY(C.alloc(C.evals, m3));
  SETUP_TRY(C.alloc(C.Gupd, m3 * 2 * m));
  SETUP_TRY(C.alloc(C.Gc, 2 * m * m));
  SETUP_TRY(C.alloc(C.norms, 2 * m));
  SETUP_TRY(C.alloc(C.rpart, std::max(resid_scratch(n, m), resid_scratch(n, m3))));
  SETUP_TRY(C.alloc(C.syev_work, syev_scratch(m3)));
  SETUP_TRY(C.alloc_bytes(C.tsqr_ws, tsqr_scratch_elems(n, m) * 8));
  SETUP_TRY(C.alloc_bytes(C.Rl, (int64_t)m * m * 8));
  SETUP_TRY(C.alloc(C.Gv, (int64_t)m * m));
  SETUP_TRY(C.alloc(C.Tm, (int64_t)m * m));
  if (check_launch("setup") != LOBPCG_OK) return cleanup(LOBPCG_ERR_HIP);
  // ---- numeric factorization ----
  {
    lobpcg_status s = factor(c);
    if (s != LOBPCG_OK) return cleanup(s);
  }
  // ---- ||A||_2 estimate (section 5.1): ||A Omega||_F / ||Omega||_F, Omega Gaussian n x m ----
  if (opt.norm_a > 0) {
    C.norm_a = opt.norm_a;
  } else {
    launch_gaussian_fill(C.Sb[1], n, m, m3, 0x5eed5eedull, C.st);
    apply_a(c, C.Sb[1], m3, C.ASb[1], m3, m);
    launch_colnorms(C.Sb[1], m3, n, m, C.norms, C.rpart, C.st);
    launch_colnorms(C.ASb[1], m3, n, m, C.norms + m, C.rpart, C.st);
    std::vector<double> h(2 * m);
    if (hipMemcpy(h.data(), C.norms, 2 * m * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return cleanup(fail(LOBPCG_ERR_HIP, "norm estimate readback"));
    double so = 0, sa = 0;
    for (int j = 0; j < m; ++j) { so += h[j]; sa += h[m + j]; }
    C.norm_a = std::sqrt(sa / so);
  }
  *out = c;
  return LOBPCG_OK;
#undef SETUP_TRY
}

lobpcg_status lobpcg_factor(lobpcg_ctx c) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  c->solved = false;
  return factor(c);
}

lobpcg_status lobpcg_update_values(lobpcg_ctx c, const double* vals, int32_t vals_on_device, const double* shift) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  if (c->dense) return fail(LOBPCG_ERR_INVALID_ARG, "update_values supports CSR matrices only");
  if (vals) {
    HIP_TRY(hipMemcpyAsync(c->d_aval_orig, vals, c->nnz * sizeof(double),
                           vals_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st));
  }
  launch_gather_values(c->d_aval_orig, c->d_vmap, c->d_aval, c->nnz, c->st);
  if (shift) launch_add_diag_shift(c->d_prow, c->d_pcol, c->d_aval, c->d_perm, shift, c->n, c->st);
  ST_TRY(check_launch("update_values"));
  c->solved = false;
  return factor(c);
}

lobpcg_status lobpcg_solve(lobpcg_ctx c, const double* X0, int32_t maxit, double* evals, double* evecs,
                           lobpcg_info* info) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  if (maxit < 1) return fail(LOBPCG_ERR_INVALID_ARG, "maxit must be >= 1");
  if (!evals || !evecs) return fail(LOBPCG_ERR_INVALID_ARG, "output pointer is NULL");
  const double t0 = now_s();
  lobpcg_ctx_s& C = *c;
  hipStream_t st = C.st;
  const int64_t n = C.n;
  const int m = C.m, k = C.k, m3 = 3 * m;
  C.solved = false;
  C.fallbacks = 0;
  int cur = 0;
  double* X = C.Sb[cur];
  // line 2 (reading: orthonormalise X0 and one Rayleigh-Ritz step so Theta is diagonal)
  if (X0)
    launch_gather_rows(X0, m, C.d_perm, X, m3, n, m, st);
  else
    launch_gaussian_fill(X, n, m, m3, 0x1234abcdull, st);
  ST_TRY(check_launch("start block"));
  ST_TRY(ortho(c, X, m3, m));
  apply_a(c, X, m3, C.ASb[cur], m3, m);
  launch_gram(X, m3, C.ASb[cur], m3, n, m, m, C.H, C.gpart, st);
  launch_syev(C.H, m, m, C.evals, C.Cev, C.syev_work, C.d_flag + 2, st);
  launch_hl_build(C.Cev, m, m, C.Gupd, nullptr, st);
  launch_block_update(C.Sb[cur], m3, C.Gupd, m, C.Sb[1 - cur], m3, n, m, m, 1.0, 0.0, st);
  launch_block_update(C.ASb[cur], m3, C.Gupd, m, C.ASb[1 - cur], m3, n, m, m, 1.0, 0.0, st);
  cur = 1 - cur;
  ST_TRY(check_launch("initial Rayleigh-Ritz"));
  bool haveP = false;
  int iters = 0, nconv = 0;
  std::vector<double> hn(2 * m), th(m3), res(m);
  lobpcg_status status = LOBPCG_NOT_CONVERGED;
  for (int it = 1; it <= maxit; ++it) {
    double* Sx = C.Sb[cur];
    double* ASx = C.ASb[cur];
    // line 4: R = AX - X Theta, lower(R) into the solve buffer, column norms
    if (C.prec == LOBPCG_FP32)
      launch_residual<float>(ASx, m3, Sx, m3, C.evals, n, m, static_cast<float*>(C.rhs), C.mp, C.norms, C.rpart, st);
    else
      launch_residual<double>(ASx, m3, Sx, m3, C.evals, n, m, static_cast<double*>(C.rhs), C.mp, C.norms, C.rpart, st);
    ST_TRY(check_launch("residual"));
    HIP_TRY(hipMemcpyAsync(hn.data(), C.norms, 2 * m * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(th.data(), C.evals, m * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    iters = it;
    // line 5: n_c = leading run of columns passing the test
    nconv = 0;
    bool finite = true;
    for (int j = 0; j < m; ++j) {
      const double rn = std::sqrt(hn[j]), xn = std::sqrt(hn[m + j]);
      if (!std::isfinite(rn) || !std::isfinite(xn) || !std::isfinite(th[j])) finite = false;
      const double denom = (C.opt.stop_rule == LOBPCG_STOP_PAPER) ? (C.norm_a + std::fabs(th[j])) * xn : C.norm_a * xn;
      res[j] = rn / denom;
    }
    if (!finite) {
      status = fail(LOBPCG_ERR_NONFINITE, "non-finite residual or Ritz value");
      break;
    }
    for (int j = 0; j < m; ++j) {
      bool ok = res[j] <= C.tol;
      if (ok && C.opt.eig_tol > 0) {
        const double rn2 = hn[j], gap = std::max(th[m - 1] - th[j], 0.0);
        ok = rn2 <= C.opt.eig_tol * std::fabs(th[j]) * gap;
      }
      if (!ok) break;
      nconv++;
    }
    if (nconv >= k) {   // lines 6-8
      status = LOBPCG_OK;
      break;
    }
    if (it == maxit) break;
    // lines 9-10: W = working(f_T(lower(R)))
    const int wslot = haveP ? 2 * m : m;
    double* W = Sx + wslot;
    precond(c, W, m3);
    ST_TRY(check_launch("preconditioner"));
    // line 11: orthogonalize W against [X, P] twice
    for (int pass = 0; pass < 2; ++pass) {
      launch_gram(Sx, m3, W, m3, n, wslot, m, C.Gc, C.gpart, st);
      launch_block_update(Sx, m3, C.Gc, m, W, m3, n, wslot, m, -1.0, 1.0, st);
    }
    ST_TRY(check_launch("block Gram-Schmidt"));
    // line 12: W = Q of Algorithm 2
    ST_TRY(ortho(c, W, m3, m));
    // line 13: A_p = S^T A S, with A W the only new product
    apply_a(c, W, m3, ASx + wslot, m3, m);
    const int cc = wslot + m;
    launch_gram(Sx, m3, ASx, m3, n, cc, cc, C.H, C.gpart, st);
    // line 14: A_p C = C D
    launch_syev(C.H, cc, cc, C.evals, C.Cev, C.syev_work, C.d_flag + 2, st);
    // lines 15-16: HL basis and the new X, P (and A X, A P by the same combination)
    launch_hl_build(C.Cev, cc, m, C.Gupd, nullptr, st);
    launch_block_update(Sx, m3, C.Gupd, 2 * m, C.Sb[1 - cur], m3, n, cc, 2 * m, 1.0, 0.0, st);
    launch_block_update(ASx, m3, C.Gupd, 2 * m, C.ASb[1 - cur], m3, n, cc, 2 * m, 1.0, 0.0, st);
    ST_TRY(check_launch("Rayleigh-Ritz"));
    cur = 1 - cur;
    haveP = true;
  }
  C.cur = cur;
  if (status == LOBPCG_OK || status == LOBPCG_NOT_CONVERGED) {
    launch_gather_rows(C.Sb[cur], m3, C.d_iperm, evecs, k, n, k, st);
    HIP_TRY(hipMemcpyAsync(evals, C.evals, k * sizeof(double), hipMemcpyDeviceToDevice, st));
    ST_TRY(check_launch("output"));
    HIP_TRY(hipStreamSynchronize(st));
    C.solved = true;
  }
  if (info) {
    info->iters = iters;
    info->n_conv = nconv;
    info->fallbacks = C.fallbacks;
    info->nlevels = C.S.nlevels;
    info->norm_a = C.norm_a;
    info->t_symbolic = C.t_symbolic;
    info->t_factor = C.t_factor;
    info->t_solve = now_s() - t0;
    info->nnz_factor = C.S.nnz_lower;
    info->factor_flops = C.S.flops;
    if (info->resid)
      for (int j = 0; j < k; ++j) info->resid[j] = res[j];
  }
  return status;
}

// Gradient with respect to a diagonal potential (first-order perturbation theory):
//   g = sum_i dtheta_i x_i o x_i - sum_i y_i o x_i,   y_i = (A - theta_i I)^+ (I - x_i x_i^T) dX_i.
// With X = [x_1..x_k] the computed eigenvectors, y_i splits into its part in span(X),
// sum_{l != i} x_l (x_l^T dX_i) / (theta_l - theta_i), and its part z_i in X^perp, where
// A - theta_i I is positive definite (theta_i <= theta_k < lambda_{k+1}); z_i is found by
// projected preconditioned CG in FP64 with the factor of A as preconditioner (FP64 residuals,
// factor in its own precision), all k right-hand sides at once.
lobpcg_status lobpcg_backward(lobpcg_ctx c, const double* d_evals, const double* d_evecs, double* d_diag) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  if (!d_diag) return fail(LOBPCG_ERR_INVALID_ARG, "d_diag is NULL");
  if (!c->solved) return fail(LOBPCG_ERR_STATE, "backward needs a successful lobpcg_solve first");
  lobpcg_ctx_s& C = *c;
  hipStream_t st = C.st;
  const int64_t n = C.n;
  const int k = C.k, m3 = 3 * C.m;
  const double* X = C.Sb[C.cur];   // x_i = X(:, i), ld 3m, permuted ordering
  const double* theta = C.evals;
  if (!C.bw_g) {
    ST_TRY(C.alloc(C.bw_g, n));
    for (double*& b : C.bw_blk) ST_TRY(C.alloc(b, n * k));
    ST_TRY(C.alloc(C.bw_small, 2 * (int64_t)k * k + 8 * k));
    ST_TRY(C.alloc(C.bw_part, std::max(coldots_scratch(n, k), gram_scratch(n, k, k))));
  }
  double *B = C.bw_blk[0], *Z = C.bw_blk[1], *R = C.bw_blk[2], *P = C.bw_blk[3], *Q = C.bw_blk[4],
         *Zp = C.bw_blk[5];
  double* coef = C.bw_small;                 // k x k: X^T dX
  double* Km = C.bw_small + k * k;           // k x k: span(X) coefficients of y
  double* dots = C.bw_small + 2 * k * k;     // rz | pq | rr | alpha | beta | bb
  double *rz = dots, *pq = dots + k, *rr = dots + 2 * k, *alpha = dots + 3 * k, *beta = dots + 4 * k,
         *bb = dots + 5 * k;
  int iters = 0;
  bool conv = true;
  if (d_evecs) {
    // B = dX in the permuted ordering; coef = X^T B; B <- (I - X X^T) B
    launch_gather_rows(d_evecs, k, C.d_perm, B, k, n, k, st);
    launch_gram(X, m3, B, k, n, k, k, coef, C.bw_part, st);
    std::vector<double> hc(k * k), th(k), hk(k * k, 0.0);
    HIP_TRY(hipMemcpyAsync(hc.data(), coef, hc.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(th.data(), theta, k * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int l = 0; l < k; ++l)
      for (int i = 0; i < k; ++i) {
        const double gap = th[l] - th[i];
        if (l != i && std::fabs(gap) > 1e-13 * std::max(std::fabs(th[l]), std::fabs(th[i])))
          hk[l * k + i] = hc[l * k + i] / gap;
      }
    HIP_TRY(hipMemcpyAsync(Km, hk.data(), hk.size() * sizeof(double), hipMemcpyHostToDevice, st));
    launch_block_update(X, m3, coef, k, B, k, n, k, k, -1.0, 1.0, st);
    // projected PCG on (A - theta_i I) z_i = b_i in X^perp
    auto project = [&](double* V) {   // V <- (I - X X^T) V
      launch_gram(X, m3, V, k, n, k, k, coef, C.bw_part, st);
      launch_block_update(X, m3, coef, k, V, k, n, k, k, -1.0, 1.0, st);
    };
    auto apply_prec = [&](const double* Rin, double* Out) {   // Out = P_X T Rin
      load_rhs(c, Rin, k, k);
      precond(c, Out, k, k);
      project(Out);
    };
    HIP_TRY(hipMemsetAsync(Z, 0, n * k * sizeof(double), st));
    launch_copy_block(B, k, R, k, n, k, st);
    launch_coldots(B, k, B, k, n, k, bb, C.bw_part, st);
    apply_prec(R, Zp);
    launch_copy_block(Zp, k, P, k, n, k, st);
    launch_coldots(R, k, Zp, k, n, k, rz, C.bw_part, st);
    std::vector<double> hbb(k), hrz(k), hpq(k), hrr(k), ha(k), hb(k);
    HIP_TRY(hipMemcpyAsync(hbb.data(), bb, k * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(hrz.data(), rz, k * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double tol = 1e-12;
    std::vector<char> done(k, 0);
    for (int i = 0; i < k; ++i) done[i] = (hbb[i] == 0.0);
    conv = false;
    for (iters = 0; iters < 500; ++iters) {
      bool all = true;
      for (int i = 0; i < k; ++i) all = all && done[i];
      if (all) { conv = true; break; }
      apply_a(c, P, k, Q, k, k);                              // Q = (A - theta I) P, projected
      launch_shift_cols(Q, k, P, k, theta, Q, k, n, k, st);
      project(Q);
      launch_coldots(P, k, Q, k, n, k, pq, C.bw_part, st);
      HIP_TRY(hipMemcpyAsync(hpq.data(), pq, k * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      for (int i = 0; i < k; ++i) ha[i] = (done[i] || hpq[i] == 0.0) ? 0.0 : hrz[i] / hpq[i];
      HIP_TRY(hipMemcpyAsync(alpha, ha.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
      launch_axpy_cols(alpha, 1.0, P, k, Z, k, n, k, st);
      launch_axpy_cols(alpha, -1.0, Q, k, R, k, n, k, st);
      launch_coldots(R, k, R, k, n, k, rr, C.bw_part, st);
      apply_prec(R, Zp);
      launch_coldots(R, k, Zp, k, n, k, pq, C.bw_part, st);   // new r^T z
      HIP_TRY(hipMemcpyAsync(hrr.data(), rr, k * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(hpq.data(), pq, k * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      for (int i = 0; i < k; ++i) {
        if (!std::isfinite(hrr[i])) return fail(LOBPCG_ERR_NONFINITE, "adjoint solve diverged");
        if (hrr[i] <= tol * tol * hbb[i]) done[i] = 1;
        hb[i] = (done[i] || hrz[i] == 0.0) ? 0.0 : hpq[i] / hrz[i];
        hrz[i] = hpq[i];
      }
      HIP_TRY(hipMemcpyAsync(beta, hb.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
      launch_xpby_cols(beta, Zp, k, P, k, n, k, st);
    }
    // y = z + X K
    launch_block_update(X, m3, Km, k, Z, k, n, k, k, 1.0, 1.0, st);
  }
  launch_diag_grad(X, m3, d_evals, d_evecs ? Z : nullptr, k, n, k, C.bw_g, st);
  launch_gather_rows(C.bw_g, 1, C.d_iperm, d_diag, 1, n, 1, st);
  ST_TRY(check_launch("backward"));
  HIP_TRY(hipStreamSynchronize(st));
  C.bw_iters = iters;
  if (!conv) return fail(LOBPCG_NOT_CONVERGED, "adjoint PCG did not reach its tolerance in 500 iterations");
  return LOBPCG_OK;
}

lobpcg_status lobpcg_destroy(lobpcg_ctx c) {
  if (!c) return LOBPCG_OK;
  if (c->st) (void)hipStreamSynchronize(c->st);
  delete c;
  return LOBPCG_OK;
}

lobpcg_status lobpcg_symbolic(const lobpcg_matrix* A, int32_t leaf_size, int32_t* perm_host, double* stats) {
  ST_TRY(validate_matrix(A));
  Symbolic S;
  const bool dense = (A->format == 1);
  std::string err = analyze(A->n, dense ? nullptr : A->rowptr, dense ? nullptr : A->colind, A->grid, dense,
                            leaf_size > 0 ? leaf_size : 64, S);
  if (!err.empty()) return fail(LOBPCG_ERR_INVALID_ARG, "symbolic analysis: " + err);
  {
    FactorPlan F;
    SolvePlan P;
    build_factor_plan(S, F);
    build_solve_plan(S, 64, 256, P);
    std::vector<int32_t> prow, pcol, vmap, apos;
    if (!dense) {
      permute_pattern(S, A->rowptr, A->colind, prow, pcol, vmap);
      assembly_positions(S, prow, pcol, apos);
    }
    err = verify(S, F, P, prow, apos);
    if (!err.empty()) return fail(LOBPCG_ERR_INVALID_ARG, "symbolic verification: " + err);
  }
  if (perm_host) std::memcpy(perm_host, S.perm.data(), A->n * sizeof(int32_t));
  if (stats) {
    stats[0] = S.nsuper;
    stats[1] = S.nlevels;
    stats[2] = S.nnz_lower;
    stats[3] = S.flops;
    stats[4] = S.max_nr;
    stats[5] = S.max_nc;
    stats[6] = (double)S.upd_total;
    stats[7] = (double)S.panel_total;
  }
  return LOBPCG_OK;
}

lobpcg_status lobpcg_get_permutation(lobpcg_ctx c, int32_t* perm_host) {
  if (!c || !perm_host) return fail(LOBPCG_ERR_INVALID_ARG, "NULL argument");
  std::memcpy(perm_host, c->S.perm.data(), c->n * sizeof(int32_t));
  return LOBPCG_OK;
}

lobpcg_status lobpcg_apply_a(lobpcg_ctx c, const double* X, int64_t ldx, double* Y, int64_t ldy, int32_t cols) {
  if (!c || !X || !Y) return fail(LOBPCG_ERR_INVALID_ARG, "NULL argument");
  if (cols < 1 || cols > 256 || ldx < cols || ldy < cols) return fail(LOBPCG_ERR_INVALID_ARG, "bad block shape");
  apply_a(c, X, ldx, Y, ldy, cols);
  ST_TRY(check_launch("apply_a"));
  HIP_TRY(hipStreamSynchronize(c->st));
  return LOBPCG_OK;
}

lobpcg_status lobpcg_apply_precond(lobpcg_ctx c, const double* R, double* W) {
  if (!c || !R || !W) return fail(LOBPCG_ERR_INVALID_ARG, "NULL argument");
  load_rhs(c, R, c->m, c->m);
  precond(c, W, c->m);
  ST_TRY(check_launch("apply_precond"));
  HIP_TRY(hipStreamSynchronize(c->st));
  return LOBPCG_OK;
}

lobpcg_status lobpcg_mixed_qr(double* W, int64_t n, int32_t cc, int64_t ldw, int32_t lower_step1, double* R,
                              void* hip_stream) {
  if (!W || n < 1 || cc < 1 || cc > 64 || ldw < cc || n < cc)
    return fail(LOBPCG_ERR_INVALID_ARG, "bad arguments to lobpcg_mixed_qr");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  std::vector<void*> mem;
  auto get = [&](int64_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)std::max<int64_t>(bytes, 8)) != hipSuccess) return nullptr;
    mem.push_back(p);
    return p;
  };
  void* ws = get(tsqr_scratch_elems(n, cc) * 8);
  void* Rl = get((int64_t)cc * cc * 8);
  double* Gv = (double*)get((int64_t)cc * cc * 8);
  double* Tm = (double*)get((int64_t)cc * cc * 8);
  double* gp = (double*)get(gram_scratch(n, cc, cc) * 8);
  int* flag = (int*)get(16);
  lobpcg_status s = LOBPCG_OK;
  if (!ws || !Rl || !Gv || !Tm || !gp || !flag) {
    s = fail(LOBPCG_ERR_ALLOC, "hipMalloc failed");
  } else {
    (void)hipMemsetAsync(flag, 0, 16, st);
    if (lower_step1)
      mixed_qr_t<float>(st, W, ldw, n, cc, ws, Rl, Tm, Gv, gp, flag, R);
    else
      mixed_qr_t<double>(st, W, ldw, n, cc, ws, Rl, Tm, Gv, gp, flag, R);
    int h = 0;
    s = check_launch("mixed_qr");
    if (s == LOBPCG_OK && hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
      s = fail(LOBPCG_ERR_HIP, "flag readback");
    if (s == LOBPCG_OK && hipStreamSynchronize(st) != hipSuccess) s = fail(LOBPCG_ERR_HIP, "sync");
    if (s == LOBPCG_OK && h) s = fail(LOBPCG_ERR_ORTHO_BREAKDOWN, "Cholesky of V^T V failed");
  }
  (void)hipStreamSynchronize(st);
  for (void* p : mem) (void)hipFree(p);
  return s;
}

lobpcg_status lobpcg_gram(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n, int32_t c1,
                          int32_t c2, double* G, void* hip_stream) {
  if (!X || !Y || !G || n < 1 || c1 < 1 || c2 < 1 || c1 > 256 || c2 > 256 || ldx < c1 || ldy < c2)
    return fail(LOBPCG_ERR_INVALID_ARG, "bad arguments to lobpcg_gram");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  void* part = nullptr;
  HIP_TRY(hipMalloc(&part, (size_t)gram_scratch(n, c1, c2) * 8));
  launch_gram(X, ldx, Y, ldy, n, c1, c2, G, static_cast<double*>(part), st);
  lobpcg_status s = check_launch("gram");
  (void)hipStreamSynchronize(st);
  (void)hipFree(part);
  return s;
}

lobpcg_status lobpcg_syev_small(const double* H, int32_t cc, double* evals, double* evecs, void* hip_stream) {
  if (!H || !evals || !evecs || cc < 1 || cc > 192) return fail(LOBPCG_ERR_INVALID_ARG, "bad arguments to syev");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  void* work = nullptr;
  HIP_TRY(hipMalloc(&work, (size_t)syev_scratch(cc) * 8 + 64));
  int* info = reinterpret_cast<int*>(static_cast<char*>(work) + syev_scratch(cc) * 8);
  launch_syev(H, cc, cc, evals, evecs, static_cast<double*>(work), info, st);
  lobpcg_status s = check_launch("syev");
  (void)hipStreamSynchronize(st);
  (void)hipFree(work);
  return s;
}

}  // extern "C"
