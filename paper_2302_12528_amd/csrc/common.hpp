// Shared declarations of the HIP kernels' host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

namespace lobpcg {

// v if c, else +0, by a bit mask rather than a select: a select between a loaded value and a constant
// may be compiled into a branch around the load, and a load inside a per-lane branch is waited for
// there, one round trip per load.
__device__ inline float keep_if(bool c, float v) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) & (c ? 0xffffffffu : 0u));
}
__device__ inline double keep_if(bool c, double v) {
  return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) & (c ? ~(uint64_t)0 : (uint64_t)0));
}

// Cholesky factor of a c x c symmetric positive definite matrix held by one wave, lane i holding row i
// in a[0 .. CP) (c <= CP <= 64, entries past c zero).  Step j publishes column j of the current matrix in
// the wave's LDS column buffer cb (64 doubles) and every lane reads the pivot and the column entries it
// needs from there (uniform addresses; one wave's LDS accesses complete in order, so no barrier), with
// l_i l_k = (l_i / l_jj) a_kj.  On return a[j] = L[i][j] for j <= i (entries above the diagonal are not
// meaningful); a non-positive or non-finite pivot is replaced by 1 and reported through bad.
template <int CP>
__device__ inline void wave_cholesky(double (&a)[CP], int c, double* cb, bool& bad) {
  const int i = threadIdx.x % 64;
#pragma unroll
  for (int j = 0; j < CP; ++j) {
    if (j < c) {   // uniform
      cb[i] = a[j];
      __builtin_amdgcn_wave_barrier();
      double d = cb[j];
      if (!(d > 0.0) || !isfinite(d)) {
        bad = true;
        d = 1.0;
      }
      const double ljj = sqrt(d), rinv = 1.0 / ljj;
      const double l = (i == j) ? ljj : a[j] * rinv;
      a[j] = l;
      const double t = l * rinv;
#pragma unroll
      for (int k = j + 1; k < CP; ++k) a[k] -= t * cb[k];
      __builtin_amdgcn_wave_barrier();   // this step's reads of cb before the next step's writes
    }
  }
}

// f(std::integral_constant<int, A>), ..., f(std::integral_constant<int, B - 1>), so that f may index
// register arrays with its argument.
template <int A, int B, typename F>
__device__ __attribute__((always_inline)) void static_for(F&& f) {
  if constexpr (A < B) {
    f(std::integral_constant<int, A>{});
    static_for<A + 1, B>(f);
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2): block b runs on XCD
// b % 8.  xcd_block(b, G) renumbers the G blocks so that each XCD receives a contiguous range of
// logical block indices, and work items that share operands (the tiles of one supernode) share an
// L2.  A bijection on [0, G).
constexpr int kXcds = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t G) {
  const int64_t q = G / kXcds, r = G % kXcds;
  const int64_t x = b % kXcds, j = b / kXcds;
  return x * q + (x < r ? x : r) + j;
}

// ---- instance segmentation of tall blocks (k_seg.hip) ----
// Rows [inst_off[b], inst_off[b+1]) of a tall block belong to instance b.  Row tiles (<= 64 rows)
// and reduction chunks never straddle instances.  All pointers are device pointers.
struct SegDev {
  int B;
  const int32_t* active;                                                  // B, 0 = skip
  const int32_t* tile_inst; const int64_t* tile_r0; const int32_t* tile_rows; int64_t ntiles;
  const int32_t* chunk_inst; const int64_t* chunk_r0; const int32_t* chunk_rows; int64_t nchunks;
  const int32_t* inst_chunk_off;                                          // B + 1
};
// Householder TSQR reduction tree: level l has items [level_off[l], level_off[l+1]) of 4 ints
// {instance, first row, rows, output slot}; level 0 reads the block (rb rows per item), later levels
// the stacked R's of the previous level (rbu rows per item; ping-pong halves of `half` elements);
// the last level writes slot b of R.
struct TsqrPlanDev {
  int rb; int rbu; int nlevels;
  const int64_t* level_off;   // host, nlevels + 1
  const int32_t* items;       // device
  int64_t half;               // elements per scratch half
  // combine = 1 (FP32 plans with c <= 64): three levels - the FP32 Householder leaves of kTsqrCombineRows
  // rows (slots in the first scratch half), chunk items {instance, first slot, slots, partial} whose FP64
  // Gram partials go to the second scratch half, and per-instance items {instance, first partial,
  // partials, slot} that sum them (the sums follow the partials) and write their Cholesky factor as R
  int combine;
};
constexpr int kTsqrCombineRows = 256;    // leaf rows of combining plans
constexpr int kTsqrCombineSlots = 4;     // leaf factors per Gram chunk

// Block element types TI / TX / TW: double (working precision) or float (the lower-precision first
// stage of Algorithm 3 line 1); small matrices (G, M, theta, norms) are FP64 either way.
template <typename TI>
void launch_sgram(const SegDev& S, const TI* X, int64_t ldx, const TI* Y, int64_t ldy, int c1, int c2,
                  double* G, int64_t gstride, double* part, hipStream_t st);
template <typename TX>
void launch_supdate(const SegDev& S, const TX* X, int64_t ldx, const double* M, int64_t ldm, int64_t mstride,
                    TX* Y, int64_t ldy, int cin, int cout, double alpha, double beta, hipStream_t st);
// Y <- X M and Y2 <- X2 M (FP64, alpha 1, beta 0) in one launch when the shapes allow, else two.
void launch_supdate_pair(const SegDev& S, const double* X, const double* X2, int64_t ldx, const double* M, int64_t ldm,
                         int64_t mstride, double* Y, double* Y2, int64_t ldy, int cin, int cout, hipStream_t st);
// Y <- Y - X M (FP64, one instance, cin = K <= 64 and K % 4 == 0, cout = 32, 16-byte aligned rows) fused
// with G = X(:, 0:K)^T Y of the updated Y (part: scratch of part_elems doubles for the workgroups'
// partials).  Returns false, launching nothing, when the shapes do not qualify.
bool launch_supdate_gram(const SegDev& S, const double* X, int64_t ldx, const double* M, int64_t ldm, double* Y,
                         int64_t ldy, int K, int cols, double* part, int64_t part_elems, double* G, hipStream_t st);
template <typename T, typename TI>
void launch_sresidual(const SegDev& S, const TI* AX, int64_t ldax, const TI* X, int64_t ldx,
                      const double* theta, int64_t tstride, int m, T* R, int64_t ldr, double* norms, double* part,
                      hipStream_t st);
template <typename TI>
void launch_scolnorms(const SegDev& S, const TI* X, int64_t ldx, int c, double* norms, int64_t nstride,
                      double* part, hipStream_t st);
template <typename TU, typename TW>
void launch_strsm_rows(const SegDev& S, TW* W, int64_t ld, int c, const TU* U, int64_t ustride, hipStream_t st);
template <typename T, typename Tin>
void launch_stsqr(const SegDev& S, const TsqrPlanDev& P, const Tin* W, int64_t ldw, int c, T* scratch, T* R,
                  hipStream_t st);
int tsqr_rows_per_block(int c, int elem_bytes);
int tsqr_upper_rows_per_block(int c, int elem_bytes);

// ---- products with A and data movement (k_block.hip) ----
// Y = A X for permuted CSR A; X, Y n x c row-major (ld), any c >= 1; T = double, or float for the
// lower-precision first stage.
template <typename T>
void launch_spmm_csr(const int32_t* rowptr, const int32_t* colind, const T* val, int64_t n,
                     const T* X, int64_t ldx, T* Y, int64_t ldy, int c, hipStream_t st);
// Y = A X for dense row-major A (n x n, lda) on the FP64 matrix cores; part (part_elems doubles) holds
// the partial products of split reduction ranges (dense_mm_scratch(n) covers every c <= 64 fully).
// (T = float: the same on the FP32 matrix cores.)
int64_t dense_mm_scratch(int64_t n);
template <typename T>
void launch_dense_mm(const T* A, int64_t lda, int64_t n, const T* X, int64_t ldx, T* Y,
                     int64_t ldy, int c, T* part, int64_t part_elems, hipStream_t st);
// Complex blocks (interleaved re, im; row-major) and the real symmetric embedding of a Hermitian
// problem: Y (2n x 2m) = [[Re X, -Im X], [Im X, Re X]] for X (n x m); X (n x k) and lam (k) from the 2k
// Ritz pairs of the embedding (Z 2n x 2k, theta 2k): x_j = Z[0:n, 2j] + i Z[n:2n, 2j], lam_j = theta_2j.
void launch_herm_expand(const double* X, int64_t n, int m, double* Y, hipStream_t st);
void launch_herm_extract(const double* Z, const double* theta, int64_t n, int k, double* X, double* lam,
                         hipStream_t st);
// X (n x k complex, k <= 32) <- X L^{-H} with G = X^H X = L L^H formed from R, the real Gram matrix of X
// read as real n x 2k; L: k x k complex scratch.
void launch_herm_orthonormalize(double* X, int64_t n, int k, const double* R, double* L, hipStream_t st);
// dst[i*ldd + j] = (Tout) src[i*lds + j], i < n, j < c (IEEE round to nearest when narrowing)
template <typename Tin, typename Tout>
void launch_convert_block(const Tin* src, int64_t lds, Tout* dst, int64_t ldd, int64_t n, int c, hipStream_t st);
// dst[i*ldd + j] = src[(idx[i] - base)*lds + j], i < nrows, j < c (idx NULL = identity)
void launch_gather_rows(const double* src, int64_t lds, const int32_t* idx, int64_t base, double* dst, int64_t ldd,
                        int64_t nrows, int c, hipStream_t st);
void launch_gather_values(const double* src, const int32_t* map, double* dst, int64_t nnz, hipStream_t st);
void launch_add_diag_shift(const int32_t* rowptr, const int32_t* colind, double* val, const int32_t* perm,
                           const double* shift, int64_t n, hipStream_t st);
// Deterministic N(0,1) fill (counter-based splitmix64 + Box-Muller).
void launch_gaussian_fill(double* X, int64_t n, int c, int64_t ld, uint64_t seed, hipStream_t st);
void launch_copy_block(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int c, hipStream_t st);
// dst[i*ldd + j] -= src[i*lds + j], i < n, j < c
void launch_sub_block(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int c, hipStream_t st);
void launch_fill_int(int32_t* p, int32_t v, int64_t count, hipStream_t st);

// ---- small dense kernels (k_small.hip), one workgroup per instance ----
// Symmetric eigensolver: the nev smallest eigenpairs of H (c x c, ldh): evals ascending, columns 0..nev-1
// of C (c x c, row stride c) the eigenvectors.  work: syev_scratch(c) doubles per instance.
int64_t syev_scratch(int c);
void launch_syev(const double* H, int64_t ldh, int64_t hstride, int c, int nev, double* evals, int64_t estride,
                 double* C, int64_t cstride, double* work, int* info, const int32_t* active, int B, hipStream_t st);
// Hetmaniuk-Lehoucq: G (c x 2m, ld 2m) = [C1, Pc] with C1 = C(:, 0:m) and Pc an orthonormal basis of
// (I - C1 C1^T) E1 (the span of C(:, m:c) C(0:m, m:c)^T); if c == m, G = C1 (ld m).
void launch_hl_build(const double* C, int64_t cstride, int c, int m, double* G, int64_t gstride,
                     const int32_t* active, int B, hipStream_t st);
// Algorithm 2 step 3 per instance: G = V^T V = L L^T; Lt = L^T; Rout = L^T working(Rl) if non-NULL;
// flag[b] set on a non-positive pivot.  Matrices at stride c*c.
template <typename T>
void launch_chol_upper(const double* G, const T* Rl, int c, double* Lt, double* Rout, int* flag,
                       const int32_t* active, int B, hipStream_t st);

// ---- factorization (k_factor.hip) ----
struct FactorDev {
  int32_t* begin; int32_t* nc; int32_t* nr; int32_t* rows; int64_t* row_off; int32_t* relpos;
  int32_t* child_ptr; int32_t* child_list; int64_t* inv_off; int32_t* invmap;
  int64_t* panel_off; int64_t* upd_off; int64_t* uvec_off; int64_t* dinv_off; int64_t* lcopy_off;
  int32_t* prow; int32_t* pcol; int32_t* apos; double* aval;   // permuted A (CSR)
  const double* dense; int64_t ld_dense; int is_dense; int max_nr;
  int32_t* asm_items; int32_t* tasks;
};
// level_max_nr: the largest front of the step's level (sizes the assembly's LDS column buffer)
template <typename T>
void launch_factor_step(const FactorDev& D, int kind, int level_max_nr, int64_t task_off, int count,
                        int64_t asm_off, int64_t asm_count, T* panel, T* upd, T* dinv, T* lcopy, int* flag,
                        hipStream_t st);
// the panel step p + 1 (npotrf tasks from potrf_off) and the update of panel p's columns beyond p + 1
// (nupd tasks from upd_off) in one launch (FP32 factors)
void launch_potrf_update(const FactorDev& D, int64_t potrf_off, int npotrf, int64_t upd_off, int nupd, float* panel,
                         float* upd, float* dinv, int* flag, hipStream_t st);

// ---- supernodal triangular solves (k_trisolve.hip) ----
struct SolveDev {
  const int32_t* fwd_items; const int32_t* fwd_fin; const int32_t* bwd_items; const int32_t* bwd_fin;  // device
  const int32_t* gather_dst; const int32_t* gather_ptr; const int32_t* gather_src;                     // device
  const int64_t* fwd_level_off; const int64_t* fwd_fin_level_off;                                       // host
  const int64_t* bwd_level_off; const int64_t* bwd_fin_level_off; const int64_t* gather_level_off;      // host
  const char* fwd_wide; const char* bwd_wide;                                                           // host
  // backward operand rows: for item aux a and panel row k, bwd_src[a + k] indexes [y; x] (2n rows)
  const int32_t* bwd_src;                                                                                // device
  int64_t n;
  // bottom levels 0 .. sub_levels - 1 as nsub subtrees (lists and offsets as in SolvePlan; device)
  int sub_levels; int64_t nsub;
  const int32_t* sub_gather_dst; const int32_t* sub_gather_ptr; const int32_t* sub_gather_src;
  const int64_t* sub_gather_off;
  const int32_t* sub_fwd_items; const int64_t* sub_fwd_off; const int32_t* sub_bwd_items; const int64_t* sub_bwd_off;
};
// Both sweeps: rhs (T, n x M, permuted, overwritten by the forward assembly) -> y -> x, and W (FP64, n x mw,
// ld ldw) = working(x).  x must equal y + n M (one allocation of 2 n M elements, fewer than 2^31 bytes).
// fpart / bpart: partial tiles (slots x 64 x M).
template <typename T>
void launch_precond(const FactorDev& D, const SolveDev& Sd, int nlevels, int M, const T* panel, T* rhs, T* y, T* x,
                    T* uvec, T* fpart, T* bpart, double* W, int64_t ldw, int mw, hipStream_t st);
// rhs (T, n x M padded with zeros) = lower(R) given R FP64 (n x m, ld)
template <typename T>
void launch_cast_to(const double* src, int64_t lds, T* dst, int64_t n, int m, int M, hipStream_t st);

// ---- adjoint solve helpers (k_adjoint.hip) ----
int64_t coldots_scratch(int64_t n, int c);
void launch_coldots(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n, int c, double* out,
                    double* part, hipStream_t st);
void launch_axpy_cols(const double* alpha, double sign, const double* X, int64_t ldx, double* Y, int64_t ldy,
                      int64_t n, int c, hipStream_t st);
void launch_xpby_cols(const double* beta, const double* Z, int64_t ldz, double* P, int64_t ldp, int64_t n, int c,
                      hipStream_t st);
void launch_shift_cols(const double* AP, int64_t lda, const double* P, int64_t ldp, const double* theta, double* Q,
                       int64_t ldq, int64_t n, int c, hipStream_t st);
void launch_diag_grad(const double* X, int64_t ldx, const double* dtheta, const double* Y, int64_t ldy, int64_t n,
                      int k, double* g, hipStream_t st);

}  // namespace lobpcg
