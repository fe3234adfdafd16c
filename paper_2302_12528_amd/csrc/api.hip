// C-ABI of liblobpcg (include/lobpcg.h): context, setup, factorization and the
// Algorithm 3 working-precision loop driven from the host, with every
// numerical step in the HIP kernels of k_*.hip.
//
// A context holds B >= 1 independent problems stored as one block-diagonal
// matrix (one problem is B = 1): ordering, factorization, products with A and
// the triangular solves run on the union; the dense block operations are
// segmented per instance; converged instances are frozen by an active mask.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
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

#define HIP_TRY(expr)                                                                                       \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) return fail(LOBPCG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define ST_TRY(expr)                \
  do {                              \
    lobpcg_status s_ = (expr);      \
    if (s_ != LOBPCG_OK) return s_; \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int pad_m(int m) { return m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : 64; }

// lobpcg_options.subtree_levels (0 automatic, -1 none, L > 0) as build_solve_plan's argument (-1 automatic)
int plan_sub_levels(const lobpcg_options& o) { return o.subtree_levels == 0 ? -1 : o.subtree_levels < 0 ? 0 : o.subtree_levels; }

constexpr int64_t kMaxBufferBytes = ((int64_t)1 << 31) - 64;   // buffer-resource extent limit of the solve kernels

// Host side of an instance segmentation.
struct SegHost {
  std::vector<int64_t> inst_off;
  std::vector<int32_t> tile_inst, tile_rows, chunk_inst, chunk_rows, inst_chunk_off;
  std::vector<int64_t> tile_r0, chunk_r0;
};

// Default rows per reduction chunk: about 512 chunks over the union (two per compute unit), within [256, 4096].
int64_t default_chunk_rows(int64_t N) { return std::max<int64_t>(256, std::min<int64_t>(4096, N / 512)); }

void build_segments(const std::vector<int64_t>& inst_off, int64_t rpc, SegHost& H) {
  H = SegHost();
  H.inst_off = inst_off;
  const int B = (int)inst_off.size() - 1;
  H.inst_chunk_off.push_back(0);
  for (int b = 0; b < B; ++b) {
    const int64_t r0 = inst_off[b], nb = inst_off[b + 1] - r0;
    for (int64_t r = 0; r < nb; r += 64) {
      H.tile_inst.push_back(b);
      H.tile_r0.push_back(r0 + r);
      H.tile_rows.push_back((int32_t)std::min<int64_t>(64, nb - r));
    }
    const int64_t cnt = std::max<int64_t>(1, (nb + rpc - 1) / rpc);
    for (int64_t q = 0; q < cnt; ++q) {
      const int64_t a = r0 + nb * q / cnt, e = r0 + nb * (q + 1) / cnt;
      H.chunk_inst.push_back(b);
      H.chunk_r0.push_back(a);
      H.chunk_rows.push_back((int32_t)(e - a));
    }
    H.inst_chunk_off.push_back((int32_t)H.chunk_inst.size());
  }
}

// Householder TSQR reduction tree for instances with row ranges inst_off and row blocks of rb.
struct TsqrHost {
  int rb = 0, rbu = 0;
  std::vector<int64_t> level_off;
  std::vector<int32_t> items;
  int64_t half = 1;
  int combine = 0;
};

// rb rows per item at level 0, rbu (a multiple of c) at the levels above
void build_tsqr(const std::vector<int64_t>& inst_off, int c, int rb, int rbu, TsqrHost& T) {
  T = TsqrHost();
  T.rb = rb;
  T.rbu = rbu;
  const int B = (int)inst_off.size() - 1;
  std::vector<int64_t> rows(B), in0(B), cnt(B), newbase(B);
  for (int b = 0; b < B; ++b) {
    rows[b] = inst_off[b + 1] - inst_off[b];
    in0[b] = inst_off[b];
  }
  T.level_off.push_back(0);
  int64_t maxout = 1;
  for (;;) {
    bool last = true;
    for (int b = 0; b < B; ++b) {
      cnt[b] = (rows[b] + rb - 1) / rb;
      if (cnt[b] > 1) last = false;
    }
    int64_t base = 0;
    for (int b = 0; b < B; ++b) {
      for (int64_t q = 0; q < cnt[b]; ++q) {
        T.items.push_back(b);
        T.items.push_back((int32_t)(in0[b] + q * rb));
        T.items.push_back((int32_t)std::min<int64_t>(rb, rows[b] - q * rb));
        T.items.push_back((int32_t)(last ? b : base + q));
      }
      newbase[b] = base;
      base += cnt[b];
    }
    T.level_off.push_back((int64_t)T.items.size() / 4);
    maxout = std::max(maxout, base);
    if (last) break;
    for (int b = 0; b < B; ++b) {
      in0[b] = newbase[b] * c;
      rows[b] = cnt[b] * c;
    }
    rb = rbu;
  }
  T.half = maxout * c * c;
}

// FP32 plans for c <= 64: leaves of kTsqrCombineRows rows, Gram chunks of kTsqrCombineSlots leaf factors,
// one combining item per instance (see TsqrPlanDev); other plans: the Householder tree above.
void build_tsqr_plan(const std::vector<int64_t>& inst_off, int c, int elem_bytes, TsqrHost& T) {
  if (elem_bytes != 4 || c > 64) {
    build_tsqr(inst_off, c, tsqr_rows_per_block(c, elem_bytes), tsqr_upper_rows_per_block(c, elem_bytes), T);
    return;
  }
  T = TsqrHost();
  T.rb = kTsqrCombineRows;
  T.rbu = 0;
  T.combine = 1;
  const int B = (int)inst_off.size() - 1;
  std::vector<int64_t> cnt(B), sbase(B), nchk(B), pbase(B);
  int64_t nslots = 0, nparts = 0;
  T.level_off.push_back(0);
  for (int b = 0; b < B; ++b) {
    const int64_t rows = inst_off[b + 1] - inst_off[b];
    cnt[b] = (rows + kTsqrCombineRows - 1) / kTsqrCombineRows;
    sbase[b] = nslots;
    for (int64_t q = 0; q < cnt[b]; ++q) {
      T.items.push_back(b);
      T.items.push_back((int32_t)(inst_off[b] + q * kTsqrCombineRows));
      T.items.push_back((int32_t)std::min<int64_t>(kTsqrCombineRows, rows - q * kTsqrCombineRows));
      T.items.push_back((int32_t)(nslots + q));
    }
    nslots += cnt[b];
  }
  T.level_off.push_back((int64_t)T.items.size() / 4);
  for (int b = 0; b < B; ++b) {
    nchk[b] = (cnt[b] + kTsqrCombineSlots - 1) / kTsqrCombineSlots;
    pbase[b] = nparts;
    for (int64_t q = 0; q < nchk[b]; ++q) {
      T.items.push_back(b);
      T.items.push_back((int32_t)(sbase[b] + q * kTsqrCombineSlots));
      T.items.push_back((int32_t)std::min<int64_t>(kTsqrCombineSlots, cnt[b] - q * kTsqrCombineSlots));
      T.items.push_back((int32_t)(nparts + q));
    }
    nparts += nchk[b];
  }
  T.level_off.push_back((int64_t)T.items.size() / 4);
  for (int b = 0; b < B; ++b) {
    T.items.push_back(b);
    T.items.push_back((int32_t)pbase[b]);
    T.items.push_back((int32_t)nchk[b]);
    T.items.push_back(b);
  }
  T.level_off.push_back((int64_t)T.items.size() / 4);
  // first half: the leaf factors (FP32); second half: the FP64 partials and then the B per-instance
  // sums (two FP32 elements each)
  T.half = std::max<int64_t>(nslots * c * c, 2 * (nparts + B) * c * c);
  T.half += T.half & 1;   // the FP64 partials start 8-byte aligned
}

}  // namespace

struct lobpcg_ctx_s {
  hipStream_t st = nullptr;
  int B = 1;
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
  SegHost SH;
  SegDev SG{};
  TsqrHost TQ32, TQ64;
  TsqrPlanDev TP32{}, TP64{};
  std::vector<void*> allocs;
  // matrix
  int32_t *d_prow = nullptr, *d_pcol = nullptr, *d_vmap = nullptr, *d_perm = nullptr, *d_iperm = nullptr;
  double *d_aval_orig = nullptr, *d_aval = nullptr, *d_dense = nullptr;
  int64_t ld_dense = 0;
  double* d_mmpart = nullptr;   // dense A: partial products of the split reduction ranges of A X
  int64_t mmpart_elems = 0;
  // factor (T = float or double)
  void *panel = nullptr, *upd = nullptr, *dinv = nullptr, *lcopy = nullptr;
  int* d_flag = nullptr;      // factor breakdown
  int* d_qflag = nullptr;     // 2B: Algorithm 2 step-3 breakdown per instance, FP32 try | FP64 retry
  int* d_info = nullptr;      // B: eigensolver diagnostics
  int32_t* d_active = nullptr;
  int32_t* d_active2 = nullptr;
  std::vector<int32_t> active;
  // iteration
  double* Sb[2] = {nullptr, nullptr};
  double* ASb[2] = {nullptr, nullptr};
  // lower-precision first stage (Algorithm 3 line 1), allocated on its first use: FP32 copies of
  // S and AS (same layout), of A's values (CSR) or of dense A
  float* Sf[2] = {nullptr, nullptr};
  float* ASf[2] = {nullptr, nullptr};
  float* d_aval32 = nullptr;
  float* d_dense32 = nullptr;
  void *rhs = nullptr, *ybuf = nullptr, *xbuf = nullptr, *uvec = nullptr, *fpart = nullptr, *bpart = nullptr;
  double *gpart = nullptr, *H = nullptr, *Cev = nullptr, *evals = nullptr, *Gupd = nullptr, *Gc = nullptr;
  double *norms = nullptr, *syev_work = nullptr;
  void *tsqr_ws = nullptr, *Rl = nullptr;
  double *Gv = nullptr, *Lt = nullptr;
  std::vector<double> norm_a;
  int cur = 0;
  bool solved = false;
  // complex Hermitian problem held as its real symmetric embedding (lobpcg_setup_hermitian): the
  // complex size, number of pairs and block size; 0 for real problems
  int64_t herm_n = 0;
  int herm_k = 0, herm_m = 0;
  double* herm_scratch = nullptr;
  double t_symbolic = 0, t_factor = 0;
  int fallbacks = 0;
  // backward (adjoint) buffers, allocated on first use
  double* bw_g = nullptr;
  double* bw_blk[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  double* bw_small = nullptr;
  double* bw_part = nullptr;
  int bw_iters = 0;
  // events around the preconditioner and A W of one iteration (timed solves)
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // factorization: side stream for the inverse phase of each level, and its ordering events
  hipStream_t fst = nullptr;
  std::vector<hipEvent_t> fev;
  // graph mode: private stream, ordering event, one executable graph per buffer parity
  hipStream_t gst = nullptr;
  hipEvent_t ev_order = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // tuning: split target of the triangular-solve plan, rows per reduction chunk, how they were chosen
  int split_target = default_split_target(4);   // tile items per level the solve plan aims at
  int64_t chunk_rows = 0;
  int tuned = 0;   // 0 defaults, 1 measured at setup, 2 read from the cache file
  int64_t gpart_bytes = 0, fpart_bytes = 0, bpart_bytes = 0;
  void* h_rb = nullptr;       // pinned host copy of the norms | evals | flags block
  int64_t rb_bytes = 0;

  // device memory: the caller's allocator (lobpcg_options.allocator) when given, else hipMalloc
  lobpcg_allocator ua{};
  template <typename X>
  lobpcg_status alloc(X*& p, int64_t count) {
    p = nullptr;
    if (count <= 0) count = 1;
    void* q = nullptr;
    const size_t bytes = (size_t)count * sizeof(X);
    if (ua.alloc) {
      q = ua.alloc(bytes, ua.user);
      if (!q) return fail(LOBPCG_ERR_ALLOC, "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes");
      if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
        ua.free(q, ua.user);
        return fail(LOBPCG_ERR_ALLOC, "the caller's allocator returned memory that is not 256-byte aligned");
      }
    } else {
      hipError_t e = hipMalloc(&q, bytes);
      if (e != hipSuccess) return fail(LOBPCG_ERR_ALLOC, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
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
    // the memory may go straight back to the caller's allocator: every queued kernel finishes first
    if (st) (void)hipStreamSynchronize(st);
    if (fst) (void)hipStreamSynchronize(fst);
    if (gst) (void)hipStreamSynchronize(gst);
    if (h_rb) (void)hipHostFree(h_rb);
    for (hipGraphExec_t g : gexec)
      if (g) (void)hipGraphExecDestroy(g);
    if (ev_order) (void)hipEventDestroy(ev_order);
    if (gst) (void)hipStreamDestroy(gst);
    for (hipEvent_t e : fev)
      if (e) (void)hipEventDestroy(e);
    if (fst) (void)hipStreamDestroy(fst);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (void* p : allocs) {
      if (ua.free)
        ua.free(p, ua.user);
      else
        (void)hipFree(p);
    }
  }
};

namespace {

template <typename V>
lobpcg_status upload(lobpcg_ctx c, V*& dst, const std::vector<V>& src) {
  ST_TRY(c->alloc(dst, (int64_t)src.size()));
  if (!src.empty()) HIP_TRY(hipMemcpy(dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
  return LOBPCG_OK;
}

template <typename V>
lobpcg_status upload_const(lobpcg_ctx c, const V*& dst, const std::vector<V>& src) {
  V* p = nullptr;
  ST_TRY(upload(c, p, src));
  dst = p;
  return LOBPCG_OK;
}

lobpcg_status upload_segments(lobpcg_ctx c) {
  SegHost& H = c->SH;
  SegDev& D = c->SG;
  D.B = (int)H.inst_off.size() - 1;
  ST_TRY(upload_const(c, D.tile_inst, H.tile_inst));
  ST_TRY(upload_const(c, D.tile_r0, H.tile_r0));
  ST_TRY(upload_const(c, D.tile_rows, H.tile_rows));
  ST_TRY(upload_const(c, D.chunk_inst, H.chunk_inst));
  ST_TRY(upload_const(c, D.chunk_r0, H.chunk_r0));
  ST_TRY(upload_const(c, D.chunk_rows, H.chunk_rows));
  ST_TRY(upload_const(c, D.inst_chunk_off, H.inst_chunk_off));
  D.ntiles = (int64_t)H.tile_inst.size();
  D.nchunks = (int64_t)H.chunk_inst.size();
  D.active = c->d_active;
  return LOBPCG_OK;
}

lobpcg_status upload_tsqr(lobpcg_ctx c, TsqrHost& H, TsqrPlanDev& D) {
  D.rb = H.rb;
  D.rbu = H.rbu;
  D.nlevels = (int)H.level_off.size() - 1;
  D.level_off = H.level_off.data();
  D.half = H.half;
  D.combine = H.combine;
  ST_TRY(upload_const(c, D.items, H.items));
  return LOBPCG_OK;
}

lobpcg_status install_solve_plan(lobpcg_ctx c) {
  lobpcg_ctx_s& C = *c;
  ST_TRY(upload_const(c, C.SD.fwd_items, C.SP.fwd_items));
  ST_TRY(upload_const(c, C.SD.fwd_fin, C.SP.fwd_fin));
  ST_TRY(upload_const(c, C.SD.bwd_items, C.SP.bwd_items));
  ST_TRY(upload_const(c, C.SD.bwd_fin, C.SP.bwd_fin));
  C.SD.fwd_level_off = C.SP.fwd_level_off.data();
  C.SD.fwd_fin_level_off = C.SP.fwd_fin_level_off.data();
  C.SD.bwd_level_off = C.SP.bwd_level_off.data();
  C.SD.bwd_fin_level_off = C.SP.bwd_fin_level_off.data();
  ST_TRY(upload_const(c, C.SD.gather_dst, C.SP.gather_dst));
  ST_TRY(upload_const(c, C.SD.gather_ptr, C.SP.gather_ptr));
  ST_TRY(upload_const(c, C.SD.gather_src, C.SP.gather_src));
  C.SD.gather_level_off = C.SP.gather_level_off.data();
  C.SD.fwd_wide = C.SP.fwd_wide.data();
  C.SD.bwd_wide = C.SP.bwd_wide.data();
  ST_TRY(upload_const(c, C.SD.bwd_src, C.SP.bwd_src));
  C.SD.n = C.n;
  C.SD.sub_levels = C.SP.sub_levels;
  C.SD.nsub = C.SP.nsub;
  if (C.SP.nsub > 0) {
    ST_TRY(upload_const(c, C.SD.sub_gather_dst, C.SP.sub_gather_dst));
    ST_TRY(upload_const(c, C.SD.sub_gather_ptr, C.SP.sub_gather_ptr));
    ST_TRY(upload_const(c, C.SD.sub_gather_src, C.SP.sub_gather_src));
    ST_TRY(upload_const(c, C.SD.sub_gather_off, C.SP.sub_gather_off));
    ST_TRY(upload_const(c, C.SD.sub_fwd_items, C.SP.sub_fwd_items));
    ST_TRY(upload_const(c, C.SD.sub_fwd_off, C.SP.sub_fwd_off));
    ST_TRY(upload_const(c, C.SD.sub_bwd_items, C.SP.sub_bwd_items));
    ST_TRY(upload_const(c, C.SD.sub_bwd_off, C.SP.sub_bwd_off));
  }
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

// Y = A X in the permuted basis (the whole union)
void apply_a(lobpcg_ctx c, const double* X, int64_t ldx, double* Y, int64_t ldy, int cols) {
  if (c->dense)
    launch_dense_mm(c->d_dense, c->ld_dense, c->n, X, ldx, Y, ldy, cols, c->d_mmpart, c->mmpart_elems, c->st);
  else
    launch_spmm_csr(c->d_prow, c->d_pcol, c->d_aval, c->n, X, ldx, Y, ldy, cols, c->st);
}

template <typename T>
lobpcg_status factor_t(lobpcg_ctx c) {
  T* panel = static_cast<T*>(c->panel);
  T* upd = static_cast<T*>(c->upd);
  T* dinv = static_cast<T*>(c->dinv);
  T* lcopy = static_cast<T*>(c->lcopy);
  const std::vector<FactorPlan::Step>& steps = c->FP.steps;
  size_t groups = 0;   // runs of steps of one level
  for (size_t q = 0; q < steps.size(); ++q)
    if (q == 0 || steps[q].level != steps[q - 1].level) ++groups;
  if (!c->fst) HIP_TRY(hipStreamCreateWithFlags(&c->fst, hipStreamNonBlocking));
  while (c->fev.size() < 2 * groups + 2) {
    hipEvent_t ev = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    c->fev.push_back(ev);
  }
  hipStream_t ms = c->st, ss = c->fst;
  auto launch = [&](const FactorPlan::Step& s, hipStream_t st) {
    const int64_t a0 = c->FP.asm_level_off[s.level], a1 = c->FP.asm_level_off[s.level + 1];
    launch_factor_step<T>(c->FD, s.kind, c->FP.level_max_nr[s.level], s.off, s.count, a0, a1 - a0, panel, upd, dinv,
                          lcopy, c->d_flag, st);
  };
  auto is_inv = [](int k) { return k == kInvPrep || k == kInvT1 || k == kInvX21 || k == kInvP21; };
  // Per level, the main stream runs the assembly, the panel steps and then the Schur complement;
  // the inverse phase (P_s = [inv(L11); L21 inv(L11)]) runs on the side stream once the panel steps
  // are done, concurrently with the Schur complement and the levels above: it reads the panel and
  // the diagonal-tile inverses, writes inv(L11) over the panel's own rows (which the Schur
  // complement does not read) and the level scratch lcopy (reused level after level, so the side
  // stream keeps the levels in order), and only L21 inv(L11) overwrites rows that the Schur
  // complement reads, so that step waits for it.
  // Panel steps with one step of lookahead (FP32 factors): the update of the columns beyond p + 1
  // by panel p shares one launch with the factorization of panel p + 1, which applies panel p to
  // column p + 1 itself and reads and writes that column only.  (An FP64 workgroup of that launch
  // would hold the LDS of the factorization kernel, one workgroup per CU, so FP64 factors keep one
  // update launch per panel step.)
  int e = 0;
  HIP_TRY(hipEventRecord(c->fev[e], ms));
  HIP_TRY(hipStreamWaitEvent(ss, c->fev[e++], 0));
  size_t i = 0;
  while (i < steps.size()) {
    const int l = steps[i].level;
    size_t j = i;
    while (j < steps.size() && steps[j].level == l) ++j;
    for (size_t q = i; q < j; ++q) {
      const int kind = steps[q].kind;
      if (is_inv(kind) || kind == kSchur || kind == kSchur2) continue;
      if constexpr (sizeof(T) == 4) {
        if (kind == kUpdate && q + 1 < j && steps[q + 1].kind == kPotrf) {
          launch_potrf_update(c->FD, steps[q + 1].off, steps[q + 1].count, steps[q].off, steps[q].count, panel, upd,
                              dinv, c->d_flag, ms);
          ++q;
          continue;
        }
      }
      launch(steps[q], ms);
    }
    hipEvent_t panels_done = c->fev[e++];
    HIP_TRY(hipEventRecord(panels_done, ms));
    for (size_t q = i; q < j; ++q)
      if (steps[q].kind == kSchur || steps[q].kind == kSchur2) launch(steps[q], ms);
    hipEvent_t schur_done = c->fev[e++];
    HIP_TRY(hipEventRecord(schur_done, ms));
    HIP_TRY(hipStreamWaitEvent(ss, panels_done, 0));
    for (size_t q = i; q < j; ++q)
      if (is_inv(steps[q].kind) && steps[q].kind != kInvP21) launch(steps[q], ss);
    HIP_TRY(hipStreamWaitEvent(ss, schur_done, 0));
    for (size_t q = i; q < j; ++q)
      if (steps[q].kind == kInvP21) launch(steps[q], ss);
    i = j;
  }
  HIP_TRY(hipEventRecord(c->fev[e], ss));
  HIP_TRY(hipStreamWaitEvent(ms, c->fev[e], 0));
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

// Algorithm 2 on each active instance's block W (rows of the instance, cc columns, ld) in place.
template <typename T>
void mixed_qr_seg(hipStream_t st, const SegDev& S, const TsqrPlanDev& P, double* W, int64_t ld, int cc, void* ws,
                  void* Rl_, double* Lt, double* Gv, double* gpart, int* flag, double* Rout) {
  T* Rl = static_cast<T*>(Rl_);
  launch_stsqr<T>(S, P, W, ld, cc, static_cast<T*>(ws), Rl, st);          // step 1: lower(W) = Q_l R_l
  launch_strsm_rows<T>(S, W, ld, cc, Rl, (int64_t)cc * cc, st);           // step 2: V = W working(R_l)^{-1}
  launch_sgram(S, W, ld, W, ld, cc, cc, Gv, (int64_t)cc * cc, gpart, st); // step 3: V^T V = L L^T
  launch_chol_upper<T>(Gv, Rl, cc, Lt, Rout, flag, S.active, S.B, st);
  launch_strsm_rows<double>(S, W, ld, cc, Lt, (int64_t)cc * cc, st);      // step 4: Q = V L^{-T}
}

// Orthonormalise each active instance's W with Algorithm 2, without a host round trip: with
// step 1 in FP32, an instance whose step-3 Cholesky breaks down (flag qflag[b]) is redone with
// step 1 in FP64 by kernels that take qflag as their active mask (its W then holds V, a basis of
// the same span); a breakdown of that retry sets qflag2[b].  The host reads both flags at its
// next synchronisation.
lobpcg_status ortho(lobpcg_ctx c, double* W, int64_t ld, int cc) {
  lobpcg_ctx_s& C = *c;
  launch_fill_int(C.d_qflag, 0, 2 * C.B, C.st);
  int* qflag2 = C.d_qflag + C.B;
  // (LOBPCG_FLAG_FORCE_FP64_REDO: the FP32 attempt counts as broken down, so step 1 runs in FP64 on W itself)
  if (C.opt.qr_lower && !(C.opt.flags & LOBPCG_FLAG_FORCE_FP64_REDO)) {
    mixed_qr_seg<float>(C.st, C.SG, C.TP32, W, ld, cc, C.tsqr_ws, C.Rl, C.Lt, C.Gv, C.gpart, C.d_qflag, nullptr);
    SegDev R = C.SG;
    R.active = C.d_qflag;
    mixed_qr_seg<double>(C.st, R, C.TP64, W, ld, cc, C.tsqr_ws, C.Rl, C.Lt, C.Gv, C.gpart, qflag2, nullptr);
  } else {
    mixed_qr_seg<double>(C.st, C.SG, C.TP64, W, ld, cc, C.tsqr_ws, C.Rl, C.Lt, C.Gv, C.gpart, qflag2, nullptr);
  }
  return check_launch("mixed QR");
}

lobpcg_status set_active(lobpcg_ctx c) {
  HIP_TRY(hipMemcpyAsync(c->d_active, c->active.data(), c->B * sizeof(int32_t), hipMemcpyHostToDevice, c->st));
  return LOBPCG_OK;
}

lobpcg_status autotune(lobpcg_ctx c);

lobpcg_status setup_core(const lobpcg_matrix* mats, int32_t count, int32_t k, int32_t m, double tol,
                         lobpcg_precision factor_precision, void* hip_stream, const lobpcg_options* opts,
                         lobpcg_ctx* out) {
  if (!out) return fail(LOBPCG_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!mats || count < 1) return fail(LOBPCG_ERR_INVALID_ARG, "need at least one matrix");
  for (int b = 0; b < count; ++b) ST_TRY(validate_matrix(&mats[b]));
  if (k < 1 || m < k) return fail(LOBPCG_ERR_INVALID_ARG, "need 1 <= k <= m");
  if (m > 64) return fail(LOBPCG_ERR_INVALID_ARG, "block size m must be <= 64");
  for (int b = 0; b < count; ++b) {
    if (3 * (int64_t)m > mats[b].n) return fail(LOBPCG_ERR_INVALID_ARG, "need 3m <= n");
    if (mats[b].format == 1 && count > 1) return fail(LOBPCG_ERR_INVALID_ARG, "dense matrices are not batched");
    if (mats[b].format == 1 && mats[b].n > 16384)
      return fail(LOBPCG_ERR_INVALID_ARG, "dense matrices are limited to n <= 16384");
  }
  if (!(tol > 0) || !std::isfinite(tol)) return fail(LOBPCG_ERR_INVALID_ARG, "tol must be positive and finite");
  if (factor_precision != LOBPCG_FP32 && factor_precision != LOBPCG_FP64)
    return fail(LOBPCG_ERR_INVALID_ARG, "factor_precision must be LOBPCG_FP32 or LOBPCG_FP64");
  lobpcg_options opt{};
  opt.leaf_size = 0;
  opt.stop_rule = LOBPCG_STOP_PAPER;
  opt.qr_lower = 1;
  if (opts) {
    opt = *opts;
    if (opt.leaf_size < 0) opt.leaf_size = 0;
    if (opt.stop_rule != LOBPCG_STOP_PAPER && opt.stop_rule != LOBPCG_STOP_NORMA)
      return fail(LOBPCG_ERR_INVALID_ARG, "stop_rule");
    if (opt.norm_a < 0 || !std::isfinite(opt.norm_a)) return fail(LOBPCG_ERR_INVALID_ARG, "norm_a");
    if (opt.eig_tol < 0 || !std::isfinite(opt.eig_tol)) return fail(LOBPCG_ERR_INVALID_ARG, "eig_tol");
    if (opt.flags & ~(LOBPCG_FLAG_GRAPH | LOBPCG_FLAG_AUTOTUNE | LOBPCG_FLAG_FORCE_FP64_REDO))
      return fail(LOBPCG_ERR_INVALID_ARG, "unknown flags");
    if (opt.subtree_levels < -1) return fail(LOBPCG_ERR_INVALID_ARG, "subtree_levels must be >= -1");
    if (opt.schur_wide_tiles < 0) return fail(LOBPCG_ERR_INVALID_ARG, "schur_wide_tiles must be >= 0");
    if (opt.stage1_tol < 0 || !std::isfinite(opt.stage1_tol))
      return fail(LOBPCG_ERR_INVALID_ARG, "stage1_tol must be >= 0 and finite");
  }
  if (opt.schur_wide_tiles == 0) opt.schur_wide_tiles = kSchurWideTiles;
  if (opt.allocator && (!opt.allocator->alloc || !opt.allocator->free))
    return fail(LOBPCG_ERR_INVALID_ARG, "allocator needs both alloc and free");
  auto c = new lobpcg_ctx_s();
  lobpcg_ctx_s& C = *c;
  if (opt.allocator) C.ua = *opt.allocator;
  opt.allocator = nullptr;   // the context keeps its own copy
  C.st = static_cast<hipStream_t>(hip_stream);
  C.B = count;
  C.k = k;
  C.m = m;
  C.mp = pad_m(m);
  C.tol = tol;
  C.prec = factor_precision;
  C.opt = opt;
  C.dense = (mats[0].format == 1);
  // ---- union of the instances (block-diagonal), host pattern ----
  std::vector<int64_t> inst_off(count + 1, 0);
  for (int b = 0; b < count; ++b) inst_off[b + 1] = inst_off[b] + mats[b].n;
  const int64_t n = inst_off[count];
  C.n = n;
  std::vector<int32_t> urow, ucol;
  std::vector<double> uval;
  const int32_t* rowptr = nullptr;
  const int32_t* colind = nullptr;
  const double* vals = nullptr;
  std::vector<Component> comps(count);
  for (int b = 0; b < count; ++b) {
    comps[b].off = inst_off[b];
    comps[b].n = mats[b].n;
    for (int d = 0; d < 3; ++d) comps[b].grid[d] = mats[b].grid[d];
  }
  if (!C.dense) {
    if (count == 1) {
      rowptr = mats[0].rowptr;
      colind = mats[0].colind;
      vals = mats[0].val;
      C.nnz = mats[0].nnz;
    } else {
      int64_t nnz = 0;
      for (int b = 0; b < count; ++b) nnz += mats[b].nnz;
      if (nnz > INT32_MAX) {
        delete c;
        return fail(LOBPCG_ERR_INVALID_ARG, "batch has more than 2^31 nonzeros");
      }
      urow.reserve(n + 1);
      ucol.reserve(nnz);
      uval.reserve(nnz);
      urow.push_back(0);
      for (int b = 0; b < count; ++b) {
        const lobpcg_matrix& A = mats[b];
        for (int64_t i = 0; i < A.n; ++i) {
          for (int32_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) {
            ucol.push_back((int32_t)(A.colind[e] + inst_off[b]));
            uval.push_back(A.val[e]);
          }
          urow.push_back((int32_t)ucol.size());
        }
      }
      rowptr = urow.data();
      colind = ucol.data();
      vals = uval.data();
      C.nnz = nnz;
    }
  }
  // ---- host symbolic analysis (pattern only) ----
  const double t0 = now_s();
  std::string err = analyze_multi(n, rowptr, colind, comps, C.dense, opt.leaf_size, C.S);
  if (!err.empty()) {
    delete c;
    return fail(LOBPCG_ERR_INVALID_ARG, "symbolic analysis: " + err);
  }
  build_factor_plan(C.S, C.FP, opt.schur_wide_tiles);
  C.split_target = default_split_target(factor_precision == LOBPCG_FP32 ? 4 : 8);
  build_solve_plan(C.S, 64, C.split_target, C.SP, plan_sub_levels(opt));
  std::vector<int32_t> prow, pcol, vmap, apos;
  if (!C.dense) {
    permute_pattern(C.S, rowptr, colind, prow, pcol, vmap);
    assembly_positions(C.S, prow, pcol, apos);
  }
  err = verify(C.S, C.FP, C.SP, prow, apos);
  if (!err.empty()) {
    delete c;
    return fail(LOBPCG_ERR_INVALID_ARG, "symbolic structures failed verification: " + err);
  }
  for (int b = 0; b < count; ++b)
    for (int64_t i = inst_off[b]; i < inst_off[b + 1]; ++i)
      if (C.S.perm[i] < inst_off[b] || C.S.perm[i] >= inst_off[b + 1]) {
        delete c;
        return fail(LOBPCG_ERR_INVALID_ARG, "ordering mixed two instances");
      }
  C.chunk_rows = default_chunk_rows(n);
  build_segments(inst_off, C.chunk_rows, C.SH);
  build_tsqr_plan(inst_off, m, 4, C.TQ32);
  build_tsqr_plan(inst_off, m, 8, C.TQ64);
  C.t_symbolic = now_s() - t0;
  auto cleanup = [&](lobpcg_status s) {
    delete c;
    return s;
  };
#define SETUP_TRY(expr)                      \
  do {                                       \
    lobpcg_status s_ = (expr);               \
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
  SETUP_TRY(install_solve_plan(c));
  SETUP_TRY(upload(c, C.d_perm, S.perm));
  SETUP_TRY(upload(c, C.d_iperm, S.iperm));
  C.active.assign(count, 1);
  SETUP_TRY(upload(c, C.d_active, C.active));
  SETUP_TRY(upload(c, C.d_active2, C.active));
  SETUP_TRY(upload_segments(c));
  SETUP_TRY(upload_tsqr(c, C.TQ32, C.TP32));
  SETUP_TRY(upload_tsqr(c, C.TQ64, C.TP64));
  if (C.dense) {
    const lobpcg_matrix* A = &mats[0];
    C.ld_dense = n;
    SETUP_TRY(C.alloc(C.d_dense, n * n));
    if (hipMemcpy2D(C.d_dense, n * sizeof(double), A->dense, A->ld * sizeof(double), n * sizeof(double), n,
                    hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(LOBPCG_ERR_HIP, "copy of dense A failed"));
    D.dense = C.d_dense;
    D.ld_dense = n;
    D.is_dense = 1;
    C.mmpart_elems = dense_mm_scratch(n);
    SETUP_TRY(C.alloc(C.d_mmpart, C.mmpart_elems));
  } else {
    SETUP_TRY(upload(c, C.d_prow, prow));
    SETUP_TRY(upload(c, C.d_pcol, pcol));
    SETUP_TRY(upload(c, C.d_vmap, vmap));
    SETUP_TRY(upload(c, D.apos, apos));
    SETUP_TRY(C.alloc(C.d_aval_orig, C.nnz));
    SETUP_TRY(C.alloc(C.d_aval, C.nnz));
    if (hipMemcpy(C.d_aval_orig, vals, C.nnz * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
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
  // the padding rows of every panel column stay zero (the factorization writes rows < nr only)
  if (hipMemset(C.panel, 0, S.panel_total * tsz) != hipSuccess) return cleanup(fail(LOBPCG_ERR_HIP, "memset"));
  SETUP_TRY(C.alloc_bytes(C.upd, S.upd_total * tsz));
  SETUP_TRY(C.alloc_bytes(C.dinv, S.dinv_total * tsz));
  SETUP_TRY(C.alloc_bytes(C.lcopy, S.lcopy_max * tsz));
  SETUP_TRY(C.alloc(C.d_flag, 4));
  // one device block read back to pinned host memory once per iteration: norms | evals | flags
  {
    const int64_t nd = (int64_t)count * 2 * m + (int64_t)count * 3 * m;
    C.rb_bytes = nd * 8 + 2 * (int64_t)count * 4;
    void* blk = nullptr;
    SETUP_TRY(C.alloc_bytes(blk, C.rb_bytes));
    C.norms = static_cast<double*>(blk);
    C.evals = C.norms + (int64_t)count * 2 * m;
    C.d_qflag = reinterpret_cast<int*>(C.evals + (int64_t)count * 3 * m);
    if (hipHostMalloc(&C.h_rb, C.rb_bytes, hipHostMallocDefault) != hipSuccess)
      return cleanup(fail(LOBPCG_ERR_ALLOC, "hipHostMalloc failed"));
  }
  SETUP_TRY(C.alloc(C.d_info, count));
  // ---- iteration buffers ----
  const int m3 = 3 * m;
  for (int b = 0; b < 2; ++b) {
    SETUP_TRY(C.alloc(C.Sb[b], n * m3));
    SETUP_TRY(C.alloc(C.ASb[b], n * m3));
  }
  SETUP_TRY(C.alloc_bytes(C.rhs, n * C.mp * tsz));
  // the solve kernels address y, x = y + n mp and each supernode panel with 32-bit byte offsets
  {
    int64_t max_panel = 0;
    for (int s = 0; s < S.nsuper; ++s) max_panel = std::max(max_panel, panel_ld(S.nr[s]) * S.nc[s]);
    if (2 * n * C.mp * tsz >= kMaxBufferBytes || max_panel * tsz >= kMaxBufferBytes)
      return cleanup(fail(LOBPCG_ERR_INVALID_ARG, "problem too large for the solve kernels' 32-bit buffer offsets"));
  }
  SETUP_TRY(C.alloc_bytes(C.ybuf, 2 * n * C.mp * tsz));
  C.xbuf = static_cast<char*>(C.ybuf) + n * C.mp * tsz;
  SETUP_TRY(C.alloc_bytes(C.uvec, std::max<int64_t>(1, S.uvec_total) * C.mp * tsz));
  C.fpart_bytes = std::max<int64_t>(1, C.SP.fwd_slots) * 64 * C.mp * tsz;
  C.bpart_bytes = std::max<int64_t>(1, C.SP.bwd_slots) * 64 * C.mp * tsz;
  SETUP_TRY(C.alloc_bytes(C.fpart, C.fpart_bytes));
  SETUP_TRY(C.alloc_bytes(C.bpart, C.bpart_bytes));
  if (hipMemset(C.rhs, 0, n * C.mp * tsz) != hipSuccess) return cleanup(fail(LOBPCG_ERR_HIP, "memset"));
  const int64_t nch = C.SG.nchunks;
  C.gpart_bytes = nch * std::max<int64_t>((int64_t)m3 * m3, 2 * m) * 8;
  SETUP_TRY(C.alloc(C.gpart, C.gpart_bytes / 8));
  SETUP_TRY(C.alloc(C.H, (int64_t)count * m3 * m3));
  SETUP_TRY(C.alloc(C.Cev, (int64_t)count * m3 * m3));
  SETUP_TRY(C.alloc(C.Gupd, (int64_t)count * m3 * 2 * m));
  SETUP_TRY(C.alloc(C.Gc, (int64_t)count * 2 * m * m));
  SETUP_TRY(C.alloc(C.syev_work, (int64_t)count * syev_scratch(m3)));
  SETUP_TRY(C.alloc_bytes(C.tsqr_ws, 2 * std::max(C.TQ32.half * 4, C.TQ64.half * 8)));
  SETUP_TRY(C.alloc_bytes(C.Rl, (int64_t)count * m * m * 8));
  SETUP_TRY(C.alloc(C.Gv, (int64_t)count * m * m));
  SETUP_TRY(C.alloc(C.Lt, (int64_t)count * m * m));
  for (hipEvent_t& e : C.ev)
    if (hipEventCreate(&e) != hipSuccess) return cleanup(fail(LOBPCG_ERR_HIP, "hipEventCreate failed"));
  if (opt.flags & LOBPCG_FLAG_GRAPH) {
    if (hipStreamCreateWithFlags(&C.gst, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&C.ev_order, hipEventDisableTiming) != hipSuccess)
      return cleanup(fail(LOBPCG_ERR_HIP, "graph stream setup failed"));
  }
  if (check_launch("setup") != LOBPCG_OK) return cleanup(LOBPCG_ERR_HIP);
  // ---- numeric factorization ----
  {
    lobpcg_status s = factor(c);
    if (s != LOBPCG_OK) return cleanup(s);
    if (opt.flags & LOBPCG_FLAG_AUTOTUNE) {
      s = autotune(c);
      if (s != LOBPCG_OK) return cleanup(s);
    }
  }
  // ---- ||A_b||_2 estimates (section 5.1): ||A Omega||_F / ||Omega||_F, Omega Gaussian n x m ----
  C.norm_a.assign(count, opt.norm_a);
  if (!(opt.norm_a > 0)) {
    launch_gaussian_fill(C.Sb[1], n, m, m3, 0x5eed5eedull, C.st);
    apply_a(c, C.Sb[1], m3, C.ASb[1], m3, m);
    launch_scolnorms(C.SG, C.Sb[1], m3, m, C.norms, 2 * m, C.gpart, C.st);
    launch_scolnorms(C.SG, C.ASb[1], m3, m, C.norms + m, 2 * m, C.gpart, C.st);
    std::vector<double> h((int64_t)count * 2 * m);
    if (hipMemcpy(h.data(), C.norms, h.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      return cleanup(fail(LOBPCG_ERR_HIP, "norm estimate readback"));
    for (int b = 0; b < count; ++b) {
      double so = 0, sa = 0;
      for (int j = 0; j < m; ++j) {
        so += h[(int64_t)b * 2 * m + j];
        sa += h[(int64_t)b * 2 * m + m + j];
      }
      C.norm_a[b] = std::sqrt(sa / so);
    }
  }
  *out = c;
  return LOBPCG_OK;
#undef SETUP_TRY
}

// ---- setup-time autotuning (LOBPCG_FLAG_AUTOTUNE) ----
uint64_t fnv_mix(uint64_t h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xff;
    h *= 1099511628211ull;
  }
  return h;
}

// Key of a tuning result: the device architecture and everything that shapes the launches.
uint64_t tune_key(const lobpcg_ctx_s& C) {
  uint64_t h = 1469598103934665603ull;
  int dev = 0;
  hipDeviceProp_t p{};
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
    for (const char* q = p.gcnArchName; *q; ++q) h = fnv_mix(h, (uint64_t)(unsigned char)*q);
  for (int64_t v : {C.n, C.nnz, (int64_t)C.B, (int64_t)C.m, (int64_t)C.prec, (int64_t)C.S.nsuper,
                    (int64_t)C.S.nlevels, C.S.panel_total, C.S.upd_total})
    h = fnv_mix(h, (uint64_t)v);
  return h;
}

// The cache is a text file named by the environment variable LOBPCG_TUNE_CACHE (unset = no cache),
// one line per key: "<key, 16 hex digits> <split target> <rows per chunk>".
bool tune_cache_lookup(uint64_t key, int& target, int64_t& rpc) {
  const char* path = getenv("LOBPCG_TUNE_CACHE");
  if (!path || !*path) return false;
  FILE* f = fopen(path, "r");
  if (!f) return false;
  unsigned long long k = 0;
  int kc = 0;
  long long r = 0;
  bool found = false;
  while (fscanf(f, "%llx %d %lld", &k, &kc, &r) == 3)
    if (k == key && kc >= 16 && kc % 16 == 0 && r >= 64) {   // the last entry for a key wins
      target = kc;
      rpc = r;
      found = true;
    }
  fclose(f);
  return found;
}

void tune_cache_store(uint64_t key, int target, int64_t rpc) {
  const char* path = getenv("LOBPCG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%016llx %d %lld\n", (unsigned long long)key, target, (long long)rpc);
  fclose(f);
}

// Mean GPU time (ms) of fn() over reps launches on the context's stream, after one warm-up call.
template <typename F>
float time_launches(lobpcg_ctx c, F fn, int reps) {
  fn();
  if (hipEventRecord(c->ev[0], c->st) != hipSuccess) return 1e30f;
  for (int r = 0; r < reps; ++r) fn();
  if (hipEventRecord(c->ev[1], c->st) != hipSuccess || hipEventSynchronize(c->ev[1]) != hipSuccess) return 1e30f;
  float ms = 0;
  if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) != hipSuccess) return 1e30f;
  return ms / reps;
}

lobpcg_status ensure_bytes(lobpcg_ctx c, void*& buf, int64_t& have, int64_t need) {
  if (need <= have) return LOBPCG_OK;
  ST_TRY(c->alloc_bytes(buf, need));
  have = need;
  return LOBPCG_OK;
}

lobpcg_status apply_chunk_rows(lobpcg_ctx c, int64_t rpc) {
  c->chunk_rows = rpc;
  const std::vector<int64_t> off = c->SH.inst_off;   // build_segments resets SH
  build_segments(off, rpc, c->SH);
  ST_TRY(upload_segments(c));
  const int m3 = 3 * c->m;
  void* g = c->gpart;
  ST_TRY(ensure_bytes(c, g, c->gpart_bytes, c->SG.nchunks * std::max<int64_t>((int64_t)m3 * m3, 2 * c->m) * 8));
  c->gpart = static_cast<double*>(g);
  return LOBPCG_OK;
}

lobpcg_status apply_split_target(lobpcg_ctx c, int target) {
  c->split_target = target;
  build_solve_plan(c->S, 64, target, c->SP, plan_sub_levels(c->opt));
  const std::string err = verify_solve_plan(c->S, c->SP);
  if (!err.empty()) return fail(LOBPCG_ERR_INVALID_ARG, "solve plan failed verification: " + err);
  ST_TRY(install_solve_plan(c));
  const int64_t tsz = (c->prec == LOBPCG_FP32) ? 4 : 8;
  ST_TRY(ensure_bytes(c, c->fpart, c->fpart_bytes, std::max<int64_t>(1, c->SP.fwd_slots) * 64 * c->mp * tsz));
  ST_TRY(ensure_bytes(c, c->bpart, c->bpart_bytes, std::max<int64_t>(1, c->SP.bwd_slots) * 64 * c->mp * tsz));
  return LOBPCG_OK;
}

// Pick the split target of the triangular-solve plan by timing the preconditioner, and the rows per
// reduction chunk by timing the Rayleigh-Ritz Gram matrix and the residual, on the context's buffers.
lobpcg_status autotune(lobpcg_ctx c) {
  lobpcg_ctx_s& C = *c;
  const uint64_t key = tune_key(C);
  int kc = 0;
  int64_t rpc = 0;
  if (tune_cache_lookup(key, kc, rpc)) {
    ST_TRY(apply_split_target(c, kc));
    ST_TRY(apply_chunk_rows(c, rpc));
    C.tuned = 2;
    return LOBPCG_OK;
  }
  const int m = C.m, m3 = 3 * m;
  launch_gaussian_fill(C.Sb[1], C.n, m3, m3, 0x7a11eull, C.st);
  launch_gaussian_fill(C.ASb[1], C.n, m3, m3, 0x7a11full, C.st);
  float best = 1e30f;
  int best_st = C.split_target;
  for (int cand : {256, 1024, 2048, 4096}) {
    ST_TRY(apply_split_target(c, cand));
    const float t = time_launches(c, [&] { precond(c, C.Sb[1], m3); }, 3);
    ST_TRY(check_launch("autotune preconditioner"));
    if (t < best) {
      best = t;
      best_st = cand;
    }
  }
  ST_TRY(apply_split_target(c, best_st));
  best = 1e30f;
  int64_t best_rpc = C.chunk_rows;
  for (int64_t cand : {512, 1024, 2048, 4096, 8192}) {
    ST_TRY(apply_chunk_rows(c, cand));
    const float t = time_launches(
        c,
        [&] {
          launch_sgram(C.SG, C.Sb[1], m3, C.ASb[1], m3, m3, m3, C.H, (int64_t)m3 * m3, C.gpart, C.st);
          launch_scolnorms(C.SG, C.Sb[1], m3, m, C.norms, 2 * m, C.gpart, C.st);
        },
        3);
    ST_TRY(check_launch("autotune reductions"));
    if (t < best) {
      best = t;
      best_rpc = cand;
    }
  }
  ST_TRY(apply_chunk_rows(c, best_rpc));
  C.tuned = 1;
  tune_cache_store(key, best_st, best_rpc);
  return LOBPCG_OK;
}

// Algorithm 3 lines 9-16 of one steady-state or first iteration on the context's current stream:
// S = [X | P | W] in Sb[cur] (W at column wslot), AS likewise; the new X, P, AX, AP go to Sb[1 - cur].
// With `timed`, events ev[0..3] bracket the preconditioner and the product A W.
lobpcg_status iteration_tail(lobpcg_ctx c, int cur, bool haveP, const SegDev& S, bool retry, bool timed);

lobpcg_status iteration_body(lobpcg_ctx c, int cur, bool haveP, bool timed) {
  lobpcg_ctx_s& C = *c;
  const int m = C.m, m3 = 3 * m;
  // lines 9-10: W = working(f_T(lower(R)))   (on the union; frozen instances are ignored below)
  double* W = C.Sb[cur] + (haveP ? 2 * m : m);
  if (timed) HIP_TRY(hipEventRecord(C.ev[0], C.st));
  precond(c, W, m3);
  if (timed) HIP_TRY(hipEventRecord(C.ev[1], C.st));
  ST_TRY(check_launch("preconditioner"));
  return iteration_tail(c, cur, haveP, C.SG, false, timed);
}

// Lines 11-16 for the instances S.active selects.  retry = false: Algorithm 2 with the context's step 1
// (FP32 step 1: a breakdown of step 3 sets qflag[b]; FP64 step 1: qflag[B + b]).  retry = true: the
// redo of an iteration whose FP32 attempt broke down, with step 1 in FP64 (qflag[B + b] on breakdown).
lobpcg_status iteration_tail(lobpcg_ctx c, int cur, bool haveP, const SegDev& S, bool retry, bool timed) {
  lobpcg_ctx_s& C = *c;
  hipStream_t st = C.st;
  const int B = C.B, m = C.m, m3 = 3 * m;
  double* Sx = C.Sb[cur];
  double* ASx = C.ASb[cur];
  const int wslot = haveP ? 2 * m : m;
  double* W = Sx + wslot;
  // line 11: orthogonalize W against [X, P] twice (for one instance the first pass's update also forms
  // the second pass's Gram matrix from the updated rows)
  launch_sgram(S, Sx, m3, W, m3, wslot, m, C.Gc, (int64_t)2 * m * m, C.gpart, st);
  if (!(B == 1 && launch_supdate_gram(S, Sx, m3, C.Gc, m, W, m3, wslot, m, C.gpart, C.gpart_bytes / 8, C.Gc, st))) {
    launch_supdate(S, Sx, m3, C.Gc, m, (int64_t)2 * m * m, W, m3, wslot, m, -1.0, 1.0, st);
    launch_sgram(S, Sx, m3, W, m3, wslot, m, C.Gc, (int64_t)2 * m * m, C.gpart, st);
  }
  launch_supdate(S, Sx, m3, C.Gc, m, (int64_t)2 * m * m, W, m3, wslot, m, -1.0, 1.0, st);
  ST_TRY(check_launch("block Gram-Schmidt"));
  // line 12: W = Q of Algorithm 2
  int* qflag2 = C.d_qflag + B;
  if (retry) {
    launch_fill_int(qflag2, 0, B, st);
    mixed_qr_seg<double>(st, S, C.TP64, W, m3, m, C.tsqr_ws, C.Rl, C.Lt, C.Gv, C.gpart, qflag2, nullptr);
  } else {
    launch_fill_int(C.d_qflag, 0, 2 * B, st);
    if (C.opt.qr_lower)
      mixed_qr_seg<float>(st, S, C.TP32, W, m3, m, C.tsqr_ws, C.Rl, C.Lt, C.Gv, C.gpart, C.d_qflag, nullptr);
    else
      mixed_qr_seg<double>(st, S, C.TP64, W, m3, m, C.tsqr_ws, C.Rl, C.Lt, C.Gv, C.gpart, qflag2, nullptr);
  }
  ST_TRY(check_launch("mixed QR"));
  // line 13: A_p = S^T A S, with A W the only new product
  if (timed) HIP_TRY(hipEventRecord(C.ev[2], st));
  apply_a(c, W, m3, ASx + wslot, m3, m);
  if (timed) HIP_TRY(hipEventRecord(C.ev[3], st));
  const int cc = wslot + m;
  launch_sgram(S, Sx, m3, ASx, m3, cc, cc, C.H, (int64_t)m3 * m3, C.gpart, st);
  // line 14: A_p C = C D
  launch_syev(C.H, cc, (int64_t)m3 * m3, cc, m, C.evals, m3, C.Cev, (int64_t)m3 * m3, C.syev_work, C.d_info,
              S.active, B, st);
  // lines 15-16: HL basis and the new X, P (and A X, A P by the same combination)
  launch_hl_build(C.Cev, (int64_t)m3 * m3, cc, m, C.Gupd, (int64_t)m3 * 2 * m, S.active, B, st);
  launch_supdate_pair(S, Sx, ASx, m3, C.Gupd, 2 * m, (int64_t)m3 * 2 * m, C.Sb[1 - cur], C.ASb[1 - cur], m3, cc,
                     2 * m, st);
  return check_launch("Rayleigh-Ritz");
}

// Redo of the iteration that read S = Sb[prev] for the instances whose FP32 Algorithm 2 broke down
// (qflag[b] set): W is restored from the solve's result x, which still holds that iteration's
// f_T(lower(R)) exactly as it was widened into W, and lines 11-16 run again with step 1 in FP64 for those
// instances only; their new X, P, A X, A P replace the failed ones in Sb[1 - prev].
lobpcg_status retry_iteration(lobpcg_ctx c, int prev, bool haveP, bool all_active) {
  lobpcg_ctx_s& C = *c;
  const int m = C.m, m3 = 3 * m;
  double* W = C.Sb[prev] + (haveP ? 2 * m : m);
  if (C.prec == LOBPCG_FP32)
    launch_convert_block<float, double>(static_cast<const float*>(C.xbuf), C.mp, W, m3, C.n, m, C.st);
  else
    launch_convert_block<double, double>(static_cast<const double*>(C.xbuf), C.mp, W, m3, C.n, m, C.st);
  SegDev R = C.SG;
  R.active = all_active ? C.d_active : C.d_qflag;
  return iteration_tail(c, prev, haveP, R, true, false);
}

// Capture iteration_body(cur, haveP = true) as an executable graph on the context's stream.
lobpcg_status capture_iteration(lobpcg_ctx c, int cur) {
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  const lobpcg_status s = iteration_body(c, cur, true, false);
  const hipError_t e = hipStreamEndCapture(c->st, &g);
  if (s != LOBPCG_OK) {
    if (e == hipSuccess && g) (void)hipGraphDestroy(g);
    return s;
  }
  if (e != hipSuccess) return fail(LOBPCG_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  const hipError_t ei = hipGraphInstantiate(&c->gexec[cur], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    c->gexec[cur] = nullptr;
    return fail(LOBPCG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  return LOBPCG_OK;
}

// Runs the solve on the context's private stream (graph mode), ordered after the caller's stream.
struct StreamSwap {
  lobpcg_ctx c;
  hipStream_t saved;
  ~StreamSwap() { c->st = saved; }
};

// ---- Algorithm 3 line 1: the lower-precision LOBPCG that computes the start block ----
// Every n-sized step (products with A, Gram matrices, block updates, residual, the preconditioner,
// the QR of W) runs on FP32 blocks in FP32 arithmetic; the small matrices they produce (Gram
// matrices, the Rayleigh-Ritz matrix, the Cholesky factor of Algorithm 2 step 3) are widened to FP64
// and handled by the working-precision small kernels, whose cost does not depend on n.

// Y = A X in FP32 (A's values rounded to FP32 by prepare_stage1)
void apply_a32(lobpcg_ctx c, const float* X, int64_t ldx, float* Y, int64_t ldy, int cols) {
  if (c->dense)
    launch_dense_mm<float>(c->d_dense32, c->ld_dense, c->n, X, ldx, Y, ldy, cols, reinterpret_cast<float*>(c->d_mmpart),
                           2 * c->mmpart_elems, c->st);
  else
    launch_spmm_csr<float>(c->d_prow, c->d_pcol, c->d_aval32, c->n, X, ldx, Y, ldy, cols, c->st);
}

// FP32 buffers of the first stage and single(A), refreshed from the current values on every solve
lobpcg_status prepare_stage1(lobpcg_ctx c) {
  lobpcg_ctx_s& C = *c;
  const int64_t n = C.n, m3 = 3 * C.m;
  for (int b = 0; b < 2; ++b) {
    if (!C.Sf[b]) ST_TRY(C.alloc(C.Sf[b], n * m3));
    if (!C.ASf[b]) ST_TRY(C.alloc(C.ASf[b], n * m3));
  }
  if (C.dense) {
    if (!C.d_dense32) ST_TRY(C.alloc(C.d_dense32, n * C.ld_dense));
    launch_convert_block<double, float>(C.d_dense, C.ld_dense, C.d_dense32, C.ld_dense, n, (int)n, C.st);
  } else {
    if (!C.d_aval32) ST_TRY(C.alloc(C.d_aval32, C.nnz));
    launch_convert_block<double, float>(C.d_aval, 1, C.d_aval32, 1, C.nnz, 1, C.st);
  }
  return check_launch("first-stage buffers");
}

// Algorithm 2 with every n-sized step in FP32 on an FP32 block W (the first stage's QR): FP32
// Householder R_l, V = W R_l^{-1}, the Gram matrix V^T V by FP32 products (chunk sums in FP64),
// its Cholesky factor in FP64, Q = V L^{-T}.  A breakdown of the Cholesky sets qflag[b]; there is
// no retry (the host ends the first stage for that instance).
lobpcg_status ortho32(lobpcg_ctx c, float* W, int64_t ld, int cc) {
  lobpcg_ctx_s& C = *c;
  float* Rl = static_cast<float*>(C.Rl);
  launch_fill_int(C.d_qflag, 0, 2 * C.B, C.st);
  launch_stsqr<float>(C.SG, C.TP32, W, ld, cc, static_cast<float*>(C.tsqr_ws), Rl, C.st);
  launch_strsm_rows<float>(C.SG, W, ld, cc, Rl, (int64_t)cc * cc, C.st);
  launch_sgram<float>(C.SG, W, ld, W, ld, cc, cc, C.Gv, (int64_t)cc * cc, C.gpart, C.st);
  launch_chol_upper<float>(C.Gv, Rl, cc, C.Lt, nullptr, C.d_qflag, C.SG.active, C.B, C.st);
  launch_strsm_rows<double>(C.SG, W, ld, cc, C.Lt, (int64_t)cc * cc, C.st);
  return check_launch("first-stage QR");
}

// Rayleigh-Ritz of S = Sx (cc columns) with AS = ASx into the next buffers: X, P (cc > m) and A X,
// A P by the Hetmaniuk-Lehoucq basis, as the working-precision loop does.
void rayleigh_ritz32(lobpcg_ctx c, float* Sx, float* ASx, float* Sn, float* ASn, int cc) {
  lobpcg_ctx_s& C = *c;
  const int m = C.m, m3 = 3 * m;
  const int nout = (cc > m) ? 2 * m : m;
  launch_sgram<float>(C.SG, Sx, m3, ASx, m3, cc, cc, C.H, (int64_t)m3 * m3, C.gpart, C.st);
  launch_syev(C.H, cc, (int64_t)m3 * m3, cc, m, C.evals, m3, C.Cev, (int64_t)m3 * m3, C.syev_work, C.d_info,
              C.d_active, C.B, C.st);
  launch_hl_build(C.Cev, (int64_t)m3 * m3, cc, m, C.Gupd, (int64_t)m3 * 2 * m, C.d_active, C.B, C.st);
  launch_supdate<float>(C.SG, Sx, m3, C.Gupd, nout, (int64_t)m3 * 2 * m, Sn, m3, cc, nout, 1.0, 0.0, C.st);
  launch_supdate<float>(C.SG, ASx, m3, C.Gupd, nout, (int64_t)m3 * 2 * m, ASn, m3, cc, nout, 1.0, 0.0, C.st);
}

// One first-stage iteration (lines 9-16 in FP32) from S = Sf[cur] into Sf[1 - cur].
template <typename T>
lobpcg_status iteration_body32(lobpcg_ctx c, int cur, bool haveP) {
  lobpcg_ctx_s& C = *c;
  const int m = C.m, m3 = 3 * m;
  float* Sx = C.Sf[cur];
  float* ASx = C.ASf[cur];
  const int wslot = haveP ? 2 * m : m;
  float* W = Sx + wslot;
  // lines 9-10: the solve result x (the factor's precision) becomes W
  precond_t<T>(c, nullptr, 0, 0);
  launch_convert_block<T, float>(static_cast<const T*>(C.xbuf), C.mp, W, m3, C.n, m, C.st);
  for (int pass = 0; pass < 2; ++pass) {   // line 11
    launch_sgram<float>(C.SG, Sx, m3, W, m3, wslot, m, C.Gc, (int64_t)2 * m * m, C.gpart, C.st);
    launch_supdate<float>(C.SG, Sx, m3, C.Gc, m, (int64_t)2 * m * m, W, m3, wslot, m, -1.0, 1.0, C.st);
  }
  ST_TRY(ortho32(c, W, m3, m));   // line 12
  apply_a32(c, W, m3, ASx + wslot, m3, m);   // line 13
  rayleigh_ritz32(c, Sx, ASx, C.Sf[1 - cur], C.ASf[1 - cur], wslot + m);   // lines 14-16
  return check_launch("first-stage iteration");
}

// Runs the first stage for every instance from the FP64 start block in columns 0 .. m - 1 of Sb[0]
// (permuted rows) to the test of eq. (stop) with tolerance tol1, and leaves its X there, widened to
// FP64.  An instance whose FP32 QR breaks down or whose residuals stop being finite ends the stage
// with the X of the iteration before (the start block if that was the first one).  Per instance:
// iters1 = outer iterations, exit1 = 1 converged, 2 iteration cap, 3 ended early.
template <typename T>
lobpcg_status stage1_t(lobpcg_ctx c, double tol1, int32_t maxit, std::vector<int>& iters1, std::vector<int>& exit1) {
  lobpcg_ctx_s& C = *c;
  const int B = C.B, m = C.m, k = C.k, m3 = 3 * m;
  const std::vector<int64_t>& off = C.SH.inst_off;
  hipStream_t st = C.st;
  ST_TRY(prepare_stage1(c));
  iters1.assign(B, 0);
  exit1.assign(B, 0);
  std::vector<int> src(B, -1);   // where each instance's result X lives: -1 = the start block in Sb[0]
  C.active.assign(B, 1);
  ST_TRY(set_active(c));
  launch_convert_block<double, float>(C.Sb[0], m3, C.Sf[0], m3, C.n, m, st);   // single(X0)
  ST_TRY(ortho32(c, C.Sf[0], m3, m));
  apply_a32(c, C.Sf[0], m3, C.ASf[0], m3, m);
  rayleigh_ritz32(c, C.Sf[0], C.ASf[0], C.Sf[1], C.ASf[1], m);
  ST_TRY(check_launch("first-stage start"));
  int cur = 1;
  bool haveP = false;
  for (int it = 1; it <= maxit; ++it) {
    launch_sresidual<T, float>(C.SG, C.ASf[cur], m3, C.Sf[cur], m3, C.evals, m3, m, static_cast<T*>(C.rhs), C.mp,
                               C.norms, C.gpart, st);
    ST_TRY(check_launch("first-stage residual"));
    int active_before = 0;
    for (int b = 0; b < B; ++b) active_before += C.active[b];
    HIP_TRY(hipMemcpyAsync(C.h_rb, C.norms, C.rb_bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double* hn = static_cast<const double*>(C.h_rb);
    const double* th = hn + (int64_t)B * 2 * m;
    const int32_t* qf = reinterpret_cast<const int32_t*>(th + (int64_t)B * m3);
    int nactive = 0;
    for (int b = 0; b < B; ++b) {
      if (!C.active[b]) continue;
      iters1[b] = it;
      const double* hb = hn + (int64_t)b * 2 * m;
      const double* tb = th + (int64_t)b * m3;
      bool finite = true;
      for (int j = 0; j < m; ++j)
        if (!std::isfinite(hb[j]) || !std::isfinite(hb[m + j]) || !std::isfinite(tb[j])) finite = false;
      if (qf[b] || !finite) {   // the QR that produced this X broke down: keep the previous X
        src[b] = (it == 1) ? -1 : 1 - cur;
        exit1[b] = 3;
        C.active[b] = 0;
        continue;
      }
      int nc = 0;
      for (int j = 0; j < m; ++j) {
        const double rn = std::sqrt(hb[j]), xn = std::sqrt(hb[m + j]);
        const double denom = (C.opt.stop_rule == LOBPCG_STOP_PAPER) ? (C.norm_a[b] + std::fabs(tb[j])) * xn
                                                                     : C.norm_a[b] * xn;
        if (!(rn <= tol1 * denom)) break;
        nc++;
      }
      if (nc >= k || it == maxit) {
        src[b] = cur;
        exit1[b] = (nc >= k) ? 1 : 2;
        C.active[b] = 0;
      } else {
        ++nactive;
      }
    }
    if (nactive == 0) break;
    if (nactive != active_before) ST_TRY(set_active(c));
    ST_TRY(iteration_body32<T>(c, cur, haveP));
    cur = 1 - cur;
    haveP = true;
  }
  // working(X) into the start block of the working-precision loop
  for (int b = 0; b < B; ++b) {
    if (src[b] < 0) continue;
    const int64_t r0 = off[b], nb = off[b + 1] - off[b];
    launch_convert_block<float, double>(C.Sf[src[b]] + r0 * m3, m3, C.Sb[0] + r0 * m3, m3, nb, m, st);
  }
  return check_launch("first-stage result");
}

// Algorithm 3 lines 2-17 for every instance of the context.
lobpcg_status solve_core(lobpcg_ctx c, const double* const* X0, int32_t maxit, double* const* evals_out,
                         double* const* evecs_out, lobpcg_info* infos) {
  lobpcg_ctx_s& C = *c;
  const bool graph = (C.gst != nullptr);
  StreamSwap swap{c, C.st};
  if (graph) {
    HIP_TRY(hipEventRecord(C.ev_order, C.st));
    HIP_TRY(hipStreamWaitEvent(C.gst, C.ev_order, 0));
    C.st = C.gst;
  }
  hipStream_t st = C.st;
  const int B = C.B;
  const int m = C.m, k = C.k, m3 = 3 * m;
  const std::vector<int64_t>& off = C.SH.inst_off;
  C.solved = false;
  C.fallbacks = 0;
  const double t_start = now_s();
  std::vector<double> t_end(B, 0.0);
  std::vector<int> iters(B, 0), nconv(B, 0);
  std::vector<lobpcg_status> status(B, LOBPCG_NOT_CONVERGED);
  std::vector<std::vector<double>> resid(B, std::vector<double>(k, 0.0));
  C.active.assign(B, 1);
  ST_TRY(set_active(c));
  int cur = 0;
  double* X = C.Sb[cur];
  // line 2 (reading: orthonormalise X0 and one Rayleigh-Ritz step so Theta is diagonal)
  for (int b = 0; b < B; ++b) {
    const int64_t nb = off[b + 1] - off[b];
    if (X0 && X0[b])
      launch_gather_rows(X0[b], m, C.d_perm + off[b], off[b], X + off[b] * m3, m3, nb, m, st);
    else
      launch_gaussian_fill(X + off[b] * m3, nb, m, m3, 0x1234abcdull + (uint64_t)b, st);
  }
  ST_TRY(check_launch("start block"));
  // line 1 (optional): a lower-precision LOBPCG refines the start block
  std::vector<int> iters1(B, 0), exit1(B, 0);
  double t_stage1 = 0;
  if (C.opt.stage1_tol > 0) {
    const double t1 = now_s();
    ST_TRY(C.prec == LOBPCG_FP32 ? stage1_t<float>(c, C.opt.stage1_tol, maxit, iters1, exit1)
                                 : stage1_t<double>(c, C.opt.stage1_tol, maxit, iters1, exit1));
    HIP_TRY(hipStreamSynchronize(st));
    t_stage1 = now_s() - t1;
    C.active.assign(B, 1);
    ST_TRY(set_active(c));
  }
  ST_TRY(ortho(c, X, m3, m));
  apply_a(c, X, m3, C.ASb[cur], m3, m);
  launch_sgram(C.SG, X, m3, C.ASb[cur], m3, m, m, C.H, (int64_t)m3 * m3, C.gpart, st);
  launch_syev(C.H, m, (int64_t)m3 * m3, m, m, C.evals, m3, C.Cev, (int64_t)m3 * m3, C.syev_work, C.d_info, C.d_active, B,
              st);
  launch_hl_build(C.Cev, (int64_t)m3 * m3, m, m, C.Gupd, (int64_t)m3 * 2 * m, C.d_active, B, st);
  launch_supdate(C.SG, C.Sb[cur], m3, C.Gupd, m, (int64_t)m3 * 2 * m, C.Sb[1 - cur], m3, m, m, 1.0, 0.0, st);
  launch_supdate(C.SG, C.ASb[cur], m3, C.Gupd, m, (int64_t)m3 * 2 * m, C.ASb[1 - cur], m3, m, m, 1.0, 0.0, st);
  cur = 1 - cur;
  ST_TRY(check_launch("initial Rayleigh-Ritz"));
  bool haveP = false, prev_haveP = false;
  const bool timed = (B == 1) && !graph;
  bool pending = false;
  double t_pc = 0, t_sp = 0;
  int n_pc = 0, n_sp = 0;
  auto harvest = [&]() {   // events of the previous iteration, complete after a stream sync
    if (!pending) return;
    float a = 0, b = 0;
    if (hipEventElapsedTime(&a, C.ev[0], C.ev[1]) == hipSuccess) {
      t_pc += 1e-3 * a;
      ++n_pc;
    }
    if (hipEventElapsedTime(&b, C.ev[2], C.ev[3]) == hipSuccess) {
      t_sp += 1e-3 * b;
      ++n_sp;
    }
    pending = false;
  };
  auto emit = [&](int b) -> lobpcg_status {   // write instance b's current Ritz pairs
    const int64_t nb = off[b + 1] - off[b];
    launch_gather_rows(C.Sb[cur], m3, C.d_iperm + off[b], 0, evecs_out[b], k, nb, k, st);
    HIP_TRY(hipMemcpyAsync(evals_out[b], C.evals + (int64_t)b * m3, k * sizeof(double), hipMemcpyDeviceToDevice,
                           st));
    return LOBPCG_OK;
  };
  for (int it = 1; it <= maxit; ++it) {
    double* Sx = C.Sb[cur];
    double* ASx = C.ASb[cur];
    // line 4: R = AX - X Theta, lower(R) into the solve buffer, column norms
    if (C.prec == LOBPCG_FP32)
      launch_sresidual<float>(C.SG, ASx, m3, Sx, m3, C.evals, m3, m, static_cast<float*>(C.rhs), C.mp, C.norms,
                              C.gpart, st);
    else
      launch_sresidual<double>(C.SG, ASx, m3, Sx, m3, C.evals, m3, m, static_cast<double*>(C.rhs), C.mp, C.norms,
                               C.gpart, st);
    ST_TRY(check_launch("residual"));
    int active_before = 0;
    for (int b = 0; b < B; ++b) active_before += C.active[b];
    HIP_TRY(hipMemcpyAsync(C.h_rb, C.norms, C.rb_bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double* hn = static_cast<const double*>(C.h_rb);
    const double* th = hn + (int64_t)B * 2 * m;
    const int32_t* qf = reinterpret_cast<const int32_t*>(th + (int64_t)B * m3);
    harvest();
    // the previous iteration's Algorithm 2: an FP32 attempt that broke down is redone with step 1 in
    // FP64 (that iteration's lines 11-16 for those instances), then the residual is formed again
    if (it == 1) {   // the start block's Algorithm 2 retried on the device already
      for (int b = 0; b < B; ++b) C.fallbacks += (C.active[b] && qf[b]) ? 1 : 0;
    } else {
      const bool force = (C.opt.flags & LOBPCG_FLAG_FORCE_FP64_REDO) && C.opt.qr_lower;
      bool redo = false;
      for (int b = 0; b < B; ++b) redo = redo || (C.active[b] && (qf[b] || force));
      if (redo) {
        for (int b = 0; b < B; ++b) C.fallbacks += (C.active[b] && (qf[b] || force)) ? 1 : 0;
        ST_TRY(retry_iteration(c, 1 - cur, prev_haveP, force));
        if (C.prec == LOBPCG_FP32)
          launch_sresidual<float>(C.SG, ASx, m3, Sx, m3, C.evals, m3, m, static_cast<float*>(C.rhs), C.mp, C.norms,
                                  C.gpart, st);
        else
          launch_sresidual<double>(C.SG, ASx, m3, Sx, m3, C.evals, m3, m, static_cast<double*>(C.rhs), C.mp,
                                   C.norms, C.gpart, st);
        ST_TRY(check_launch("residual after the FP64 retry"));
        HIP_TRY(hipMemcpyAsync(C.h_rb, C.norms, C.rb_bytes, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
      }
    }
    // Algorithm 2 that broke down with step 1 in FP64 (the retry, or the FP64-only configuration)
    for (int b = 0; b < B; ++b) {
      if (!C.active[b]) continue;
      if (qf[B + b]) {
        status[b] = LOBPCG_ERR_ORTHO_BREAKDOWN;
        C.active[b] = 0;
        iters[b] = it - 1;
      }
    }
    // line 5: n_c = leading run of columns passing the test, per instance
    int nactive = 0;
    for (int b = 0; b < B; ++b) {
      if (!C.active[b]) continue;
      iters[b] = it;
      const double* hb = hn + (int64_t)b * 2 * m;
      const double* tb = th + (int64_t)b * m3;
      bool finite = true;
      std::vector<double> res(m);
      for (int j = 0; j < m; ++j) {
        const double rn = std::sqrt(hb[j]), xn = std::sqrt(hb[m + j]);
        if (!std::isfinite(rn) || !std::isfinite(xn) || !std::isfinite(tb[j])) finite = false;
        const double denom = (C.opt.stop_rule == LOBPCG_STOP_PAPER) ? (C.norm_a[b] + std::fabs(tb[j])) * xn
                                                                     : C.norm_a[b] * xn;
        res[j] = rn / denom;
      }
      for (int j = 0; j < k; ++j) resid[b][j] = res[j];
      if (!finite) {
        status[b] = LOBPCG_ERR_NONFINITE;
        C.active[b] = 0;
        continue;
      }
      int nc = 0;
      for (int j = 0; j < m; ++j) {
        bool ok = res[j] <= C.tol;
        if (ok && C.opt.eig_tol > 0) {
          const double gap = std::max(tb[m - 1] - tb[j], 0.0);
          ok = hb[j] <= C.opt.eig_tol * std::fabs(tb[j]) * gap;
        }
        if (!ok) break;
        nc++;
      }
      nconv[b] = nc;
      if (nc >= k) {   // lines 6-8
        status[b] = LOBPCG_OK;
        C.active[b] = 0;
        ST_TRY(emit(b));
        t_end[b] = now_s();
      } else if (it == maxit) {
        C.active[b] = 0;
        ST_TRY(emit(b));
        t_end[b] = now_s();
      } else {
        ++nactive;
      }
    }
    if (nactive == 0) break;
    if (nactive != active_before) ST_TRY(set_active(c));   // the device mask is stale only after a change
    if (graph && haveP) {
      if (!C.gexec[cur]) ST_TRY(capture_iteration(c, cur));
      HIP_TRY(hipGraphLaunch(C.gexec[cur], st));
    } else {
      ST_TRY(iteration_body(c, cur, haveP, timed));
      pending = timed;
    }
    cur = 1 - cur;
    prev_haveP = haveP;
    haveP = true;
    // frozen instances keep their (already emitted) results; their rows of the new buffers are not used
  }
  C.cur = cur;
  ST_TRY(check_launch("output"));
  HIP_TRY(hipStreamSynchronize(st));
  harvest();
  const double t_done = now_s();
  lobpcg_status overall = LOBPCG_OK;
  for (int b = 0; b < B; ++b) {
    if (status[b] != LOBPCG_OK && overall == LOBPCG_OK) overall = status[b];
    if (infos) {
      lobpcg_info& I = infos[b];
      I.iters = iters[b];
      I.n_conv = nconv[b];
      I.fallbacks = C.fallbacks;
      I.nlevels = C.S.nlevels;
      I.norm_a = C.norm_a[b];
      I.t_symbolic = C.t_symbolic;
      I.t_factor = C.t_factor;
      I.t_solve = (t_end[b] > 0 ? t_end[b] : t_done) - t_start;
      I.nnz_factor = C.S.nnz_lower;
      I.factor_flops = C.S.flops;
      if (I.resid)
        for (int j = 0; j < k; ++j) I.resid[j] = resid[b][j];
      I.t_precond_gpu = t_pc;
      I.t_spmm_gpu = t_sp;
      I.n_precond = n_pc;
      I.n_spmm = n_sp;
      I.stage1_iters = iters1[b];
      I.stage1_exit = exit1[b];
      I.t_stage1 = t_stage1;
    }
  }
  // the context keeps the final Ritz pairs of a single instance for lobpcg_backward
  C.solved = (B == 1) && (status[0] == LOBPCG_OK || status[0] == LOBPCG_NOT_CONVERGED);
  if (overall != LOBPCG_OK && overall != LOBPCG_NOT_CONVERGED && g_last_error.empty())
    g_last_error = lobpcg_status_string(overall);
  if (overall == LOBPCG_ERR_NONFINITE) return fail(overall, "non-finite residual or Ritz value");
  if (overall == LOBPCG_ERR_ORTHO_BREAKDOWN)
    return fail(overall, "Algorithm 2 Cholesky of V^T V failed (W rank deficient) after the FP64 retry");
  return overall;
}

// Algorithm 1 (mixed-precision block PINVIT) for a single-problem context; see lobpcg_pinvit.
// X~, then X and A X, live in columns 0 .. m - 1 of Sb[cur] / ASb[cur]; the diagonalised X and A X
// go to Sb[1 - cur] / ASb[1 - cur], whose columns m .. 2m - 1 take W.
lobpcg_status pinvit_core(lobpcg_ctx c, const double* X0, int32_t maxit, double* evals_out, double* evecs_out,
                          lobpcg_info* info, double* theta_hist) {
  lobpcg_ctx_s& C = *c;
  hipStream_t st = C.st;
  const int m = C.m, k = C.k, m3 = 3 * m;
  const int64_t n = C.n;
  C.solved = false;
  C.fallbacks = 0;
  const double t_start = now_s();
  C.active.assign(1, 1);
  ST_TRY(set_active(c));
  int cur = 0;
  // line 1: X~ = X0
  if (X0)
    launch_gather_rows(X0, m, C.d_perm, 0, C.Sb[cur], m3, n, m, st);
  else
    launch_gaussian_fill(C.Sb[cur], n, m, m3, 0x1234abcdull, st);
  ST_TRY(check_launch("start block"));
  lobpcg_status status = LOBPCG_NOT_CONVERGED;
  int iters = 0, nconv = 0;
  std::vector<double> resid(k, 0.0);
  auto emit = [&](const double* Xr) -> lobpcg_status {
    launch_gather_rows(Xr, m3, C.d_iperm, 0, evecs_out, k, n, k, st);
    HIP_TRY(hipMemcpyAsync(evals_out, C.evals, k * sizeof(double), hipMemcpyDeviceToDevice, st));
    return LOBPCG_OK;
  };
  for (int it = 1; it <= maxit; ++it) {
    double* X = C.Sb[cur];
    double* AX = C.ASb[cur];
    double* Xr = C.Sb[1 - cur];
    double* AXr = C.ASb[1 - cur];
    // line 3: X = Q of X~ (Algorithm 2)
    ST_TRY(ortho(c, X, m3, m));
    // line 4: Theta = X^T A X, diagonalised (Theta = C D C^T; X <- X C, A X <- A X C)
    apply_a(c, X, m3, AX, m3, m);
    launch_sgram(C.SG, X, m3, AX, m3, m, m, C.H, (int64_t)m3 * m3, C.gpart, st);
    launch_syev(C.H, m, (int64_t)m3 * m3, m, m, C.evals, m3, C.Cev, (int64_t)m3 * m3, C.syev_work, C.d_info,
                C.d_active, 1, st);
    launch_supdate(C.SG, X, m3, C.Cev, m, (int64_t)m3 * m3, Xr, m3, m, m, 1.0, 0.0, st);
    launch_supdate(C.SG, AX, m3, C.Cev, m, (int64_t)m3 * m3, AXr, m3, m, m, 1.0, 0.0, st);
    // line 5: R = A X - X Theta, lower(R) into the solve buffer, column norms
    if (C.prec == LOBPCG_FP32)
      launch_sresidual<float>(C.SG, AXr, m3, Xr, m3, C.evals, m3, m, static_cast<float*>(C.rhs), C.mp, C.norms,
                              C.gpart, st);
    else
      launch_sresidual<double>(C.SG, AXr, m3, Xr, m3, C.evals, m3, m, static_cast<double*>(C.rhs), C.mp, C.norms,
                               C.gpart, st);
    ST_TRY(check_launch("PINVIT Rayleigh quotient and residual"));
    HIP_TRY(hipMemcpyAsync(C.h_rb, C.norms, C.rb_bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double* hn = static_cast<const double*>(C.h_rb);
    const double* th = hn + 2 * m;
    const int32_t* qf = reinterpret_cast<const int32_t*>(th + m3);
    iters = it;
    C.fallbacks += qf[0];
    if (qf[1]) {
      status = LOBPCG_ERR_ORTHO_BREAKDOWN;
      break;
    }
    if (theta_hist)
      for (int j = 0; j < k; ++j) theta_hist[(int64_t)(it - 1) * k + j] = th[j];
    // lines 6-8: the test of Algorithm 3 (eq. (stop)) on the leading columns
    bool finite = true;
    std::vector<double> res(m);
    for (int j = 0; j < m; ++j) {
      const double rn = std::sqrt(hn[j]), xn = std::sqrt(hn[m + j]);
      if (!std::isfinite(rn) || !std::isfinite(xn) || !std::isfinite(th[j])) finite = false;
      const double denom = (C.opt.stop_rule == LOBPCG_STOP_PAPER) ? (C.norm_a[0] + std::fabs(th[j])) * xn
                                                                   : C.norm_a[0] * xn;
      res[j] = rn / denom;
    }
    for (int j = 0; j < k; ++j) resid[j] = res[j];
    if (!finite) {
      status = LOBPCG_ERR_NONFINITE;
      break;
    }
    int nc = 0;
    for (int j = 0; j < m; ++j) {
      bool ok = res[j] <= C.tol;
      if (ok && C.opt.eig_tol > 0) {
        const double gap = std::max(th[m - 1] - th[j], 0.0);
        ok = hn[j] <= C.opt.eig_tol * std::fabs(th[j]) * gap;
      }
      if (!ok) break;
      nc++;
    }
    nconv = nc;
    if (nc >= k) {
      status = LOBPCG_OK;
      ST_TRY(emit(Xr));
      break;
    }
    if (it == maxit) {
      ST_TRY(emit(Xr));
      break;
    }
    // lines 9-10: W = working(f_T(lower(R))) into columns m .. 2m - 1 of Xr
    precond(c, Xr + m, m3);
    ST_TRY(check_launch("PINVIT preconditioner"));
    // line 11: X~ = X - W
    launch_sub_block(Xr + m, m3, Xr, m3, n, m, st);
    cur = 1 - cur;
  }
  ST_TRY(check_launch("PINVIT output"));
  HIP_TRY(hipStreamSynchronize(st));
  if (info) {
    info->iters = iters;
    info->n_conv = nconv;
    info->fallbacks = C.fallbacks;
    info->nlevels = C.S.nlevels;
    info->norm_a = C.norm_a[0];
    info->t_symbolic = C.t_symbolic;
    info->t_factor = C.t_factor;
    info->t_solve = now_s() - t_start;
    info->nnz_factor = C.S.nnz_lower;
    info->factor_flops = C.S.flops;
    if (info->resid)
      for (int j = 0; j < k; ++j) info->resid[j] = resid[j];
    info->t_precond_gpu = 0;
    info->t_spmm_gpu = 0;
    info->n_precond = 0;
    info->n_spmm = 0;
  }
  if (status == LOBPCG_ERR_NONFINITE) return fail(status, "non-finite residual or Ritz value");
  if (status == LOBPCG_ERR_ORTHO_BREAKDOWN)
    return fail(status, "Algorithm 2 Cholesky of V^T V failed (X~ rank deficient) after the FP64 retry");
  return status;
}

// One-instance segmentation on the fly for the standalone entry points.
struct TempSeg {
  std::vector<void*> mem;
  SegDev S{};
  SegHost H;
  template <typename V>
  bool put(const V*& dst, const std::vector<V>& src) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(8, src.size() * sizeof(V))) != hipSuccess) return false;
    mem.push_back(p);
    if (!src.empty() && hipMemcpy(p, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice) != hipSuccess)
      return false;
    dst = static_cast<const V*>(p);
    return true;
  }
  bool init(int64_t n) {
    build_segments(std::vector<int64_t>{0, n}, default_chunk_rows(n), H);
    std::vector<int32_t> one{1};
    S.B = 1;
    S.ntiles = (int64_t)H.tile_inst.size();
    S.nchunks = (int64_t)H.chunk_inst.size();
    return put(S.active, one) && put(S.tile_inst, H.tile_inst) && put(S.tile_r0, H.tile_r0) &&
           put(S.tile_rows, H.tile_rows) && put(S.chunk_inst, H.chunk_inst) && put(S.chunk_r0, H.chunk_r0) &&
           put(S.chunk_rows, H.chunk_rows) && put(S.inst_chunk_off, H.inst_chunk_off);
  }
  void* get(int64_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, (size_t)std::max<int64_t>(bytes, 8)) != hipSuccess) return nullptr;
    mem.push_back(p);
    return p;
  }
  ~TempSeg() {
    for (void* p : mem) (void)hipFree(p);
  }
};

}  // namespace

// ---- scratch of lobpcg_mixed_qr_noalloc ----
// One fixed array per GPU (each device holds its own copy at its own address), held until the process
// ends.  Host code never uses the name itself: its device address comes from hipGetSymbolAddress, once
// per device, and is kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[LOBPCG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

lobpcg_status scratch_for_current_device(unsigned char*& out) {
  out = nullptr;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LOBPCG_ERR_INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(LOBPCG_ERR_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return LOBPCG_OK;
}

// Layout of a fixed buffer: 256-byte aligned pieces in order, as byte offsets.
struct Carve {
  int64_t used = 0;
  int64_t take(int64_t bytes) {
    const int64_t off = used;
    used += (std::max<int64_t>(bytes, 1) + 255) & ~(int64_t)255;
    return off;
  }
};

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
  if (!A) {
    if (out) *out = nullptr;
    return fail(LOBPCG_ERR_INVALID_ARG, "A is NULL");
  }
  return setup_core(A, 1, k, m, tol, factor_precision, hip_stream, opts, out);
}

lobpcg_status lobpcg_setup_batched(const lobpcg_matrix* A, int32_t count, int32_t k, int32_t m, double tol,
                                   lobpcg_precision factor_precision, void* hip_stream, const lobpcg_options* opts,
                                   lobpcg_ctx* out) {
  return setup_core(A, count, k, m, tol, factor_precision, hip_stream, opts, out);
}

// ---- complex Hermitian matrices (section 1: A Hermitian positive definite) ----
// A = B + iC (B symmetric, C antisymmetric) is held as the real symmetric positive definite
// M = [[B, -C], [C, B]] of order 2n.  A x = lambda x with x = u + iv gives M [u; v] = lambda [u; v] and
// M [-v; u] = lambda [-v; u], so every eigenvalue of A is a double eigenvalue of M, the k smallest
// eigenpairs of A are the 2k smallest of M, and x = u + iv is read from any unit vector [u; v] of the
// pair.  The working-precision loop, the lower-precision factor of M (the real form of the complex
// Cholesky factor of A) and Algorithm 2 run unchanged on M.
namespace {

lobpcg_status validate_hermitian(const lobpcg_matrix* A) {
  if (!A) return fail(LOBPCG_ERR_INVALID_ARG, "A is NULL");
  if (A->n < 1 || A->n > (int64_t)INT32_MAX / 2 - 1) return fail(LOBPCG_ERR_INVALID_ARG, "n out of range");
  const int64_t n = A->n;
  auto herm_pair = [](double ar, double ai, double br, double bi) {   // (a, b) = (A_ij, A_ji): b = conj(a)
    const double s = std::max(std::max(std::fabs(ar), std::fabs(ai)), std::max(std::fabs(br), std::fabs(bi)));
    return std::fabs(ar - br) <= 1e-12 * s && std::fabs(ai + bi) <= 1e-12 * s;
  };
  if (A->format == 3) {
    if (!A->dense) return fail(LOBPCG_ERR_INVALID_ARG, "dense pointer is NULL");
    if (A->ld < n) return fail(LOBPCG_ERR_INVALID_ARG, "ld < n");
    if (n > 8192) return fail(LOBPCG_ERR_INVALID_ARG, "dense Hermitian matrices are limited to n <= 8192");
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j <= i; ++j) {
        const double* a = A->dense + 2 * (i * A->ld + j);
        const double* b = A->dense + 2 * (j * A->ld + i);
        if (!std::isfinite(a[0]) || !std::isfinite(a[1])) return fail(LOBPCG_ERR_INVALID_ARG, "non-finite matrix entry");
        if (!herm_pair(a[0], a[1], b[0], b[1])) return fail(LOBPCG_ERR_INVALID_ARG, "matrix is not Hermitian");
      }
    for (int64_t i = 0; i < n; ++i)
      if (!(A->dense[2 * (i * A->ld + i)] > 0)) return fail(LOBPCG_ERR_INVALID_ARG, "non-positive diagonal");
    return LOBPCG_OK;
  }
  if (A->format != 2) return fail(LOBPCG_ERR_INVALID_ARG, "Hermitian format must be 2 (CSR) or 3 (dense)");
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
      const double ar = A->val[2 * e], ai = A->val[2 * e + 1];
      if (!std::isfinite(ar) || !std::isfinite(ai)) return fail(LOBPCG_ERR_INVALID_ARG, "non-finite matrix entry");
      if (j == i) {
        diag = true;
        if (!(ar > 0)) return fail(LOBPCG_ERR_INVALID_ARG, "non-positive diagonal");
      }
      const int32_t* b = A->colind + A->rowptr[j];
      const int32_t* en = A->colind + A->rowptr[j + 1];
      const int32_t* it = std::lower_bound(b, en, (int32_t)i);
      if (it == en || *it != i) return fail(LOBPCG_ERR_INVALID_ARG, "pattern is not symmetric");
      const int64_t t = it - A->colind;
      if (!herm_pair(ar, ai, A->val[2 * t], A->val[2 * t + 1]))
        return fail(LOBPCG_ERR_INVALID_ARG, "matrix is not Hermitian");
    }
    if (!diag) return fail(LOBPCG_ERR_INVALID_ARG, "missing diagonal entry");
  }
  return LOBPCG_OK;
}

}  // namespace

lobpcg_status lobpcg_setup_hermitian(const lobpcg_matrix* A, int32_t k, int32_t m, double tol,
                                     lobpcg_precision factor_precision, void* hip_stream, const lobpcg_options* opts,
                                     lobpcg_ctx* out) {
  if (out) *out = nullptr;
  if (!out) return fail(LOBPCG_ERR_INVALID_ARG, "out is NULL");
  ST_TRY(validate_hermitian(A));
  if (k < 1 || m < k) return fail(LOBPCG_ERR_INVALID_ARG, "need 1 <= k <= m");
  if (m > 32) return fail(LOBPCG_ERR_INVALID_ARG, "Hermitian block size m must be <= 32");
  const int64_t n = A->n, n2 = 2 * n;
  lobpcg_matrix M{};
  M.n = n2;
  std::vector<int32_t> rp, ci;
  std::vector<double> va;
  if (A->format == 3) {
    M.format = 1;
    M.ld = n2;
    va.assign((size_t)n2 * n2, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) {
        const double br = A->dense[2 * (i * A->ld + j)], bi = A->dense[2 * (i * A->ld + j) + 1];
        va[i * n2 + j] = br;
        va[i * n2 + n + j] = -bi;
        va[(n + i) * n2 + j] = bi;
        va[(n + i) * n2 + n + j] = br;
      }
    M.dense = va.data();
  } else {
    // rows i < n: B_i then -C_i (columns n + j); rows n + i: C_i then B_i.  Entries of C that are zero
    // (the diagonal, real couplings) are left out; C's pattern is symmetric, so M's is too.
    rp.reserve(n2 + 1);
    rp.push_back(0);
    for (int half = 0; half < 2; ++half)
      for (int64_t i = 0; i < n; ++i) {
        for (int pass = 0; pass < 2; ++pass) {
          const bool b_block = (pass == half);   // which n x n block supplies columns pass * n + j
          for (int32_t e = A->rowptr[i]; e < A->rowptr[i + 1]; ++e) {
            const double re = A->val[2 * e], im = A->val[2 * e + 1];
            if (b_block) {
              ci.push_back((int32_t)(pass * n + A->colind[e]));
              va.push_back(re);
            } else if (im != 0.0) {
              ci.push_back((int32_t)(pass * n + A->colind[e]));
              va.push_back(half == 0 ? -im : im);
            }
          }
        }
        rp.push_back((int32_t)ci.size());
      }
    M.format = 0;
    M.nnz = (int64_t)ci.size();
    M.rowptr = rp.data();
    M.colind = ci.data();
    M.val = va.data();
    // a 2D grid hint (g0, g1, 1) becomes (2, g0, g1): the two copies are the outer dimension
    if (A->grid[0] > 0 && A->grid[1] > 0 && A->grid[2] <= 1 &&
        (int64_t)A->grid[0] * A->grid[1] == n) {
      M.grid[0] = 2;
      M.grid[1] = A->grid[0];
      M.grid[2] = A->grid[1];
    }
  }
  lobpcg_ctx c = nullptr;
  ST_TRY(setup_core(&M, 1, 2 * k, 2 * m, tol, factor_precision, hip_stream, opts, &c));
  c->herm_n = n;
  c->herm_k = k;
  c->herm_m = m;
  *out = c;
  return LOBPCG_OK;
}

lobpcg_status lobpcg_solve_hermitian(lobpcg_ctx c, const double* X0, int32_t maxit, double* evals, double* evecs,
                                     lobpcg_info* info) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  if (!c->herm_n) return fail(LOBPCG_ERR_INVALID_ARG, "not a Hermitian context (lobpcg_setup_hermitian)");
  if (maxit < 1) return fail(LOBPCG_ERR_INVALID_ARG, "maxit must be >= 1");
  if (!evals || !evecs) return fail(LOBPCG_ERR_INVALID_ARG, "output pointer is NULL");
  g_last_error.clear();
  lobpcg_ctx_s& C = *c;
  const int64_t n = C.herm_n;
  const int k = C.herm_k, m = C.herm_m;
  // scratch: the real start block (2n x 2m), the 2k real Ritz values and vectors (2n x 2k)
  // scratch: the real start block (2n x 2m), the 2k real Ritz values and vectors (2n x 2k), and a seeded
  // complex start block (n x m) when the caller gives none
  if (!C.herm_scratch) ST_TRY(C.alloc(C.herm_scratch, 2 * n * 2 * m + 2 * k + 2 * n * 2 * k + n * 2 * m));
  double* X0r = C.herm_scratch;
  double* evr = X0r + 2 * n * 2 * m;
  double* Zr = evr + 2 * k;
  double* Xg = Zr + 2 * n * 2 * k;
  if (X0) {
    launch_herm_expand(X0, n, m, X0r, C.st);
  } else {
    launch_gaussian_fill(Xg, n, 2 * m, 2 * m, 0x6e7a11ull, C.st);   // re, im of a seeded complex block
    launch_herm_expand(Xg, n, m, X0r, C.st);
  }
  ST_TRY(check_launch("Hermitian start block"));
  lobpcg_info ri{};
  std::vector<double> res(2 * k);
  ri.resid = info && info->resid ? res.data() : nullptr;
  const double* x0[1] = {X0r};
  double* ev[1] = {evr};
  double* ec[1] = {Zr};
  const lobpcg_status s = solve_core(c, x0, maxit, ev, ec, &ri);
  if (s == LOBPCG_OK || s == LOBPCG_NOT_CONVERGED) {
    launch_herm_extract(Zr, evr, n, k, evecs, evals, C.st);
    // The real pair vectors are orthonormal; the complex vectors read from them are so only up to how far
    // each pair's span is from closed under multiplication by i (about residual / gap).  A Cholesky QR in
    // complex arithmetic (Gram matrix G = X^H X from the real Gram matrix of X over the first n rows of
    // Zr, the rest zero) makes them orthonormal: X <- X L^{-H}, G = L L^H.
    launch_convert_block<double, double>(evecs, 2 * k, Zr, 2 * k, n, 2 * k, C.st);
    HIP_TRY(hipMemsetAsync(Zr + n * 2 * k, 0, (size_t)n * 2 * k * sizeof(double), C.st));
    C.active.assign(1, 1);
    ST_TRY(set_active(c));
    launch_sgram(C.SG, Zr, 2 * k, Zr, 2 * k, 2 * k, 2 * k, C.H, 0, C.gpart, C.st);
    launch_herm_orthonormalize(evecs, n, k, C.H, C.Cev, C.st);
    ST_TRY(check_launch("Hermitian extraction"));
    HIP_TRY(hipStreamSynchronize(C.st));
  }
  C.solved = false;   // the context's pairs are those of M
  if (info) {
    double* r = info->resid;
    *info = ri;
    info->resid = r;
    info->n_conv = ri.n_conv / 2;
    if (r)
      for (int j = 0; j < k; ++j) r[j] = res[2 * j];
  }
  return s;
}

lobpcg_status lobpcg_factor(lobpcg_ctx c) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  c->solved = false;
  return factor(c);
}

lobpcg_status lobpcg_update_values(lobpcg_ctx c, const double* vals, int32_t vals_on_device, const double* shift) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  if (c->dense || c->herm_n) return fail(LOBPCG_ERR_INVALID_ARG, "update_values supports real CSR matrices only");
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
  if (c->herm_n) return fail(LOBPCG_ERR_INVALID_ARG, "Hermitian context: use lobpcg_solve_hermitian");
  if (c->B != 1) return fail(LOBPCG_ERR_INVALID_ARG, "batched context: use lobpcg_solve_batched");
  if (maxit < 1) return fail(LOBPCG_ERR_INVALID_ARG, "maxit must be >= 1");
  if (!evals || !evecs) return fail(LOBPCG_ERR_INVALID_ARG, "output pointer is NULL");
  g_last_error.clear();
  const double* x0[1] = {X0};
  double* ev[1] = {evals};
  double* ec[1] = {evecs};
  return solve_core(c, x0, maxit, ev, ec, info);
}

lobpcg_status lobpcg_pinvit(lobpcg_ctx c, const double* X0, int32_t maxit, double* evals, double* evecs,
                            lobpcg_info* info, double* theta_hist) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  if (c->B != 1 || c->herm_n) return fail(LOBPCG_ERR_INVALID_ARG, "PINVIT supports real single-problem contexts");
  if (maxit < 1) return fail(LOBPCG_ERR_INVALID_ARG, "maxit must be >= 1");
  if (!evals || !evecs) return fail(LOBPCG_ERR_INVALID_ARG, "output pointer is NULL");
  g_last_error.clear();
  return pinvit_core(c, X0, maxit, evals, evecs, info, theta_hist);
}

lobpcg_status lobpcg_solve_batched(lobpcg_ctx c, const double* const* X0, int32_t maxit, double* const* evals,
                                   double* const* evecs, lobpcg_info* infos) {
  if (!c) return fail(LOBPCG_ERR_INVALID_ARG, "ctx is NULL");
  if (maxit < 1) return fail(LOBPCG_ERR_INVALID_ARG, "maxit must be >= 1");
  if (!evals || !evecs) return fail(LOBPCG_ERR_INVALID_ARG, "output pointer array is NULL");
  for (int b = 0; b < c->B; ++b)
    if (!evals[b] || !evecs[b]) return fail(LOBPCG_ERR_INVALID_ARG, "output pointer is NULL");
  g_last_error.clear();
  return solve_core(c, X0, maxit, evals, evecs, infos);
}

int32_t lobpcg_batch_count(lobpcg_ctx c) { return c ? c->B : 0; }

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
  if (c->B != 1 || c->herm_n) return fail(LOBPCG_ERR_INVALID_ARG, "backward supports real single-instance contexts");
  if (!c->solved) return fail(LOBPCG_ERR_STATE, "backward needs a successful lobpcg_solve first");
  lobpcg_ctx_s& C = *c;
  hipStream_t st = C.st;
  const int64_t n = C.n;
  const int k = C.k, m3 = 3 * C.m;
  const double* X = C.Sb[C.cur];   // x_i = X(:, i), ld 3m, permuted ordering
  const double* theta = C.evals;
  const SegDev& SG = C.SG;         // one instance, active
  if (!C.bw_g) {
    ST_TRY(C.alloc(C.bw_g, n));
    for (double*& b : C.bw_blk) ST_TRY(C.alloc(b, n * k));
    ST_TRY(C.alloc(C.bw_small, 2 * (int64_t)k * k + 8 * k));
    ST_TRY(C.alloc(C.bw_part, std::max(coldots_scratch(n, k), SG.nchunks * (int64_t)k * k)));
  }
  C.active.assign(1, 1);
  ST_TRY(set_active(c));
  double *Bm = C.bw_blk[0], *Z = C.bw_blk[1], *R = C.bw_blk[2], *P = C.bw_blk[3], *Q = C.bw_blk[4],
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
    launch_gather_rows(d_evecs, k, C.d_perm, 0, Bm, k, n, k, st);
    launch_sgram(SG, X, m3, Bm, k, k, k, coef, 0, C.bw_part, st);
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
    launch_supdate(SG, X, m3, coef, k, 0, Bm, k, k, k, -1.0, 1.0, st);
    auto project = [&](double* V) {   // V <- (I - X X^T) V
      launch_sgram(SG, X, m3, V, k, k, k, coef, 0, C.bw_part, st);
      launch_supdate(SG, X, m3, coef, k, 0, V, k, k, k, -1.0, 1.0, st);
    };
    auto apply_prec = [&](const double* Rin, double* Out) {   // Out = P_X T Rin
      load_rhs(c, Rin, k, k);
      precond(c, Out, k, k);
      project(Out);
    };
    HIP_TRY(hipMemsetAsync(Z, 0, n * k * sizeof(double), st));
    launch_copy_block(Bm, k, R, k, n, k, st);
    launch_coldots(Bm, k, Bm, k, n, k, bb, C.bw_part, st);
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
      if (all) {
        conv = true;
        break;
      }
      apply_a(c, P, k, Q, k, k);   // Q = (A - theta I) P, projected
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
    launch_supdate(SG, X, m3, Km, k, 0, Z, k, k, k, 1.0, 1.0, st);
  }
  launch_diag_grad(X, m3, d_evals, d_evecs ? Z : nullptr, k, n, k, C.bw_g, st);
  launch_gather_rows(C.bw_g, 1, C.d_iperm, 0, d_diag, 1, n, 1, st);
  ST_TRY(check_launch("backward"));
  HIP_TRY(hipStreamSynchronize(st));
  C.bw_iters = iters;
  if (!conv) return fail(LOBPCG_NOT_CONVERGED, "adjoint PCG did not reach its tolerance in 500 iterations");
  return LOBPCG_OK;
}

int32_t lobpcg_backward_iters(lobpcg_ctx c) { return c ? c->bw_iters : 0; }

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
                            leaf_size, S);
  if (!err.empty()) return fail(LOBPCG_ERR_INVALID_ARG, "symbolic analysis: " + err);
  {
    FactorPlan F;
    SolvePlan P;
    build_factor_plan(S, F);
    build_solve_plan(S, 64, default_split_target(4), P);
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

lobpcg_status lobpcg_exact_fill(const lobpcg_matrix* A, int32_t leaf_size, double* nnz_exact) {
  if (!nnz_exact) return fail(LOBPCG_ERR_INVALID_ARG, "NULL argument");
  ST_TRY(validate_matrix(A));
  if (A->format == 1) {
    *nnz_exact = (double)A->n * (A->n + 1) / 2;
    return LOBPCG_OK;
  }
  Symbolic S;
  std::string err = analyze(A->n, A->rowptr, A->colind, A->grid, false, leaf_size, S);
  if (!err.empty()) return fail(LOBPCG_ERR_INVALID_ARG, "symbolic analysis: " + err);
  std::vector<int32_t> prow, pcol, vmap;
  permute_pattern(S, A->rowptr, A->colind, prow, pcol, vmap);
  *nnz_exact = (double)exact_fill(A->n, prow, pcol);
  return LOBPCG_OK;
}

lobpcg_status lobpcg_get_tuning(lobpcg_ctx c, int32_t* out3) {
  if (!c || !out3) return fail(LOBPCG_ERR_INVALID_ARG, "NULL argument");
  out3[0] = c->split_target;
  out3[1] = (int32_t)c->chunk_rows;
  out3[2] = c->tuned;
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
  if (!W || n < 1 || cc < 1 || cc > 64 || ldw < cc || ldw >= (1 << 22) || n < cc)
    return fail(LOBPCG_ERR_INVALID_ARG, "bad arguments to lobpcg_mixed_qr");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  TempSeg T;
  if (!T.init(n)) return fail(LOBPCG_ERR_ALLOC, "hipMalloc failed");
  TsqrHost th;
  build_tsqr_plan(std::vector<int64_t>{0, n}, cc, lower_step1 ? 4 : 8, th);
  TsqrPlanDev tp{};
  tp.rb = th.rb;
  tp.rbu = th.rbu;
  tp.nlevels = (int)th.level_off.size() - 1;
  tp.level_off = th.level_off.data();
  tp.half = th.half;
  tp.combine = th.combine;
  void* ws = T.get(2 * th.half * 8);
  void* Rl = T.get((int64_t)cc * cc * 8);
  double* Gv = (double*)T.get((int64_t)cc * cc * 8);
  double* Lt = (double*)T.get((int64_t)cc * cc * 8);
  double* gp = (double*)T.get(T.S.nchunks * (int64_t)cc * cc * 8);
  int* flag = (int*)T.get(16);
  if (!ws || !Rl || !Gv || !Lt || !gp || !flag || !T.put(tp.items, th.items))
    return fail(LOBPCG_ERR_ALLOC, "hipMalloc failed");
  lobpcg_status s = LOBPCG_OK;
  (void)hipMemsetAsync(flag, 0, 16, st);
  if (lower_step1)
    mixed_qr_seg<float>(st, T.S, tp, W, ldw, cc, ws, Rl, Lt, Gv, gp, flag, R);
  else
    mixed_qr_seg<double>(st, T.S, tp, W, ldw, cc, ws, Rl, Lt, Gv, gp, flag, R);
  int h = 0;
  s = check_launch("mixed_qr");
  if (s == LOBPCG_OK && hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    s = fail(LOBPCG_ERR_HIP, "flag readback");
  if (s == LOBPCG_OK && hipStreamSynchronize(st) != hipSuccess) s = fail(LOBPCG_ERR_HIP, "sync");
  if (s == LOBPCG_OK && h) s = fail(LOBPCG_ERR_ORTHO_BREAKDOWN, "Cholesky of V^T V failed");
  (void)hipStreamSynchronize(st);
  return s;
}

lobpcg_status lobpcg_mixed_qr_noalloc(double* W, int64_t n, int32_t cc, int64_t ldw, int32_t lower_step1,
                                      double* R, void* hip_stream) {
  if (!W || n < 1 || cc < 1 || cc > 64 || ldw < cc || ldw >= (1 << 22) || n < cc)
    return fail(LOBPCG_ERR_INVALID_ARG, "bad arguments to lobpcg_mixed_qr_noalloc");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // host plans: the one-instance segmentation and the TSQR tree, as lobpcg_mixed_qr builds them
  SegHost H;
  build_segments(std::vector<int64_t>{0, n}, default_chunk_rows(n), H);
  const int eb = lower_step1 ? 4 : 8;
  TsqrHost th;
  build_tsqr_plan(std::vector<int64_t>{0, n}, cc, eb, th);
  const int64_t nt = (int64_t)H.tile_inst.size(), nch = (int64_t)H.chunk_inst.size();
  const int64_t c2 = (int64_t)cc * cc;
  // layout of the scratch array (sizes first, so that too large a problem is rejected before any work)
  Carve K;
  const int64_t o_active = K.take(4), o_tile_inst = K.take(4 * nt), o_tile_r0 = K.take(8 * nt),
                o_tile_rows = K.take(4 * nt), o_chunk_inst = K.take(4 * nch), o_chunk_r0 = K.take(8 * nch),
                o_chunk_rows = K.take(4 * nch), o_chunk_off = K.take(8),
                o_items = K.take(4 * (int64_t)th.items.size()), o_flag = K.take(16), o_Rl = K.take(8 * c2),
                o_Gv = K.take(8 * c2), o_Lt = K.take(8 * c2), o_gp = K.take(8 * nch * c2),
                o_ws = K.take(2 * th.half * eb);
  if (K.used > (int64_t)LOBPCG_NOALLOC_SCRATCH_BYTES)
    return fail(LOBPCG_ERR_INVALID_ARG, "lobpcg_mixed_qr_noalloc: n = " + std::to_string(n) + ", c = " +
                                            std::to_string(cc) + " needs " + std::to_string(K.used) +
                                            " bytes of scratch, more than the fixed " +
                                            std::to_string((long long)LOBPCG_NOALLOC_SCRATCH_BYTES));
  unsigned char* base = nullptr;
  ST_TRY(scratch_for_current_device(base));
  auto i32 = [&](int64_t off) { return reinterpret_cast<int32_t*>(base + off); };
  auto i64 = [&](int64_t off) { return reinterpret_cast<int64_t*>(base + off); };
  auto f64 = [&](int64_t off) { return reinterpret_cast<double*>(base + off); };
  SegDev S{};
  S.B = 1;
  S.active = i32(o_active);
  S.tile_inst = i32(o_tile_inst);
  S.tile_r0 = i64(o_tile_r0);
  S.tile_rows = i32(o_tile_rows);
  S.ntiles = nt;
  S.chunk_inst = i32(o_chunk_inst);
  S.chunk_r0 = i64(o_chunk_r0);
  S.chunk_rows = i32(o_chunk_rows);
  S.nchunks = nch;
  S.inst_chunk_off = i32(o_chunk_off);
  TsqrPlanDev tp{};
  tp.rb = th.rb;
  tp.rbu = th.rbu;
  tp.nlevels = (int)th.level_off.size() - 1;
  tp.level_off = th.level_off.data();
  tp.half = th.half;
  tp.combine = th.combine;
  tp.items = i32(o_items);
  // the plans into the array (ordinary copies on the stream; the host vectors outlive them because the
  // call synchronises the stream before it returns), the breakdown flag cleared by a kernel
  const int32_t one = 1;
  auto put = [&](const void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(const_cast<void*>(dst), src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  HIP_TRY(put(S.active, &one, sizeof(one)));
  HIP_TRY(put(S.tile_inst, H.tile_inst.data(), nt * sizeof(int32_t)));
  HIP_TRY(put(S.tile_r0, H.tile_r0.data(), nt * sizeof(int64_t)));
  HIP_TRY(put(S.tile_rows, H.tile_rows.data(), nt * sizeof(int32_t)));
  HIP_TRY(put(S.chunk_inst, H.chunk_inst.data(), nch * sizeof(int32_t)));
  HIP_TRY(put(S.chunk_r0, H.chunk_r0.data(), nch * sizeof(int64_t)));
  HIP_TRY(put(S.chunk_rows, H.chunk_rows.data(), nch * sizeof(int32_t)));
  HIP_TRY(put(S.inst_chunk_off, H.inst_chunk_off.data(), 2 * sizeof(int32_t)));
  HIP_TRY(put(tp.items, th.items.data(), th.items.size() * sizeof(int32_t)));
  int* dflag = i32(o_flag);
  launch_fill_int(dflag, 0, 4, st);
  if (lower_step1)
    mixed_qr_seg<float>(st, S, tp, W, ldw, cc, base + o_ws, base + o_Rl, f64(o_Lt), f64(o_Gv), f64(o_gp), dflag, R);
  else
    mixed_qr_seg<double>(st, S, tp, W, ldw, cc, base + o_ws, base + o_Rl, f64(o_Lt), f64(o_Gv), f64(o_gp), dflag,
                         R);
  lobpcg_status s = check_launch("mixed_qr_noalloc");
  int h = 0;
  if (s == LOBPCG_OK && hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess)
    s = fail(LOBPCG_ERR_HIP, "flag readback");
  if (hipStreamSynchronize(st) != hipSuccess && s == LOBPCG_OK) s = fail(LOBPCG_ERR_HIP, "sync");
  if (s == LOBPCG_OK && h) s = fail(LOBPCG_ERR_ORTHO_BREAKDOWN, "Cholesky of V^T V failed");
  return s;
}

lobpcg_status lobpcg_gram(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n, int32_t c1,
                          int32_t c2, double* G, void* hip_stream) {
  // ldx, ldy <= 32768: a reduction chunk (at most 4096 rows) then spans less than 2 GiB, the range of
  // the Gram kernel's 32-bit buffer offsets
  if (!X || !Y || !G || n < 1 || c1 < 1 || c2 < 1 || c1 > 256 || c2 > 256 || ldx < c1 || ldy < c2 ||
      ldx > 32768 || ldy > 32768)
    return fail(LOBPCG_ERR_INVALID_ARG, "bad arguments to lobpcg_gram");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  TempSeg T;
  if (!T.init(n)) return fail(LOBPCG_ERR_ALLOC, "hipMalloc failed");
  double* part = (double*)T.get(T.S.nchunks * (int64_t)c1 * c2 * 8);
  if (!part) return fail(LOBPCG_ERR_ALLOC, "hipMalloc failed");
  launch_sgram(T.S, X, ldx, Y, ldy, c1, c2, G, 0, part, st);
  lobpcg_status s = check_launch("gram");
  (void)hipStreamSynchronize(st);
  return s;
}

lobpcg_status lobpcg_syev_small(const double* H, int32_t cc, int32_t nev, double* evals, double* evecs,
                                void* hip_stream) {
  if (!H || !evals || !evecs || cc < 1 || cc > 192 || nev < 1 || nev > cc)
    return fail(LOBPCG_ERR_INVALID_ARG, "bad arguments to syev");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  void* work = nullptr;
  HIP_TRY(hipMalloc(&work, (size_t)syev_scratch(cc) * 8 + 64));
  int* info = reinterpret_cast<int*>(static_cast<char*>(work) + syev_scratch(cc) * 8);
  launch_syev(H, cc, 0, cc, nev, evals, 0, evecs, 0, static_cast<double*>(work), info, nullptr, 1, st);
  lobpcg_status s = check_launch("syev");
  (void)hipStreamSynchronize(st);
  (void)hipFree(work);
  return s;
}

}  // extern "C"
