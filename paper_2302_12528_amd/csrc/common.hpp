// Shared declarations of the HIP kernels' host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lobpcg {

// ---- block kernels (k_block.hip) ----
// Y = A X for permuted CSR A; X, Y n x c row-major (ld), any c >= 1.
void launch_spmm_csr(const int32_t* rowptr, const int32_t* colind, const double* val, int64_t n,
                     const double* X, int64_t ldx, double* Y, int64_t ldy, int c, hipStream_t st);
// Y = A X for dense row-major A (n x n, lda).
void launch_dense_mm(const double* A, int64_t lda, int64_t n, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, int c, hipStream_t st);
// Gram: G (c1 x c2, row-major, ld c2) = X^T Y; part is scratch of gram_scratch(n, c1, c2) doubles.
int64_t gram_scratch(int64_t n, int c1, int c2);
void launch_gram(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n, int c1, int c2,
                 double* G, double* part, hipStream_t st);
// Y = alpha X M + beta Y; X n x cin, M cin x cout (row-major, ldm), Y n x cout.
// Y may alias X only if cout <= 64 and ldy == ldx.
void launch_block_update(const double* X, int64_t ldx, const double* M, int64_t ldm, double* Y, int64_t ldy,
                         int64_t n, int cin, int cout, double alpha, double beta, hipStream_t st);
// R = AX - X diag(theta) cast to T (ld = m); norms[0..m) = ||R_j||^2, norms[m..2m) = ||X_j||^2.
int64_t resid_scratch(int64_t n, int m);
template <typename T>
void launch_residual(const double* AX, int64_t ldax, const double* X, int64_t ldx, const double* theta,
                     int64_t n, int m, T* R, int64_t ldr, double* norms, double* part, hipStream_t st);
// Column sums of squares of an n x c block: norms[j] = ||X_j||^2 (deterministic).
void launch_colnorms(const double* X, int64_t ldx, int64_t n, int c, double* norms, double* part, hipStream_t st);
// dst[i*ldd + j] = src[idx[i]*lds + j], i < n_rows, j < c (idx NULL = identity); optional scale.
void launch_gather_rows(const double* src, int64_t lds, const int32_t* idx, double* dst, int64_t ldd,
                        int64_t nrows, int c, hipStream_t st);
// vals[e] = src[map[e]] (+ shift[perm_row(e)] on the diagonal if shift != NULL).
void launch_gather_values(const double* src, const int32_t* map, double* dst, int64_t nnz, hipStream_t st);
void launch_add_diag_shift(const int32_t* rowptr, const int32_t* colind, double* val, const int32_t* perm,
                           const double* shift, int64_t n, hipStream_t st);
// Deterministic N(0,1) fill (counter-based splitmix64 + Box-Muller).
void launch_gaussian_fill(double* X, int64_t n, int c, int64_t ld, uint64_t seed, hipStream_t st);
// Convert / copy blocks.
void launch_copy_block(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int c, hipStream_t st);
void launch_cast_f64_f32(const double* src, int64_t lds, float* dst, int64_t ldd, int64_t n, int c, hipStream_t st);
void launch_cast_f32_f64(const float* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int c, hipStream_t st);
// sum of partial vectors part[nb][len] in fixed order into out[len]
void launch_reduce_parts(const double* part, int nb, int len, double* out, hipStream_t st);

// ---- small dense kernels (k_small.hip), one workgroup each ----
// Symmetric eigensolver (cyclic Jacobi): H c x c (ld) -> evals (c, ascending), C (c x c, ld c,
// column j = eigenvector j).  work: syev_scratch(c) doubles of global scratch.
int64_t syev_scratch(int c);
void launch_syev(const double* H, int64_t ldh, int c, double* evals, double* C, double* work, int* info,
                 hipStream_t st);
// Hetmaniuk-Lehoucq: from C (c x c) of the Rayleigh-Ritz, G (c x 2m, ld 2m) = [C(:,1:m), C(:,m+1:c) V],
// V = Householder Q of C(1:m, m+1:c)^T.  If c == m, G = C(:, 1:m) (ld m).
void launch_hl_build(const double* C, int c, int m, double* G, double* work, hipStream_t st);
// Algorithm 2 steps 2 and 4: W <- W U^{-1} row by row (U c x c upper, row-major, type TU), in place.
template <typename TU>
void launch_trsm_rows(double* W, int64_t ld, int64_t n, int c, const TU* U, hipStream_t st);
// Algorithm 2 step 3: G = V^T V = L L^T; Lt = L^T (c x c row-major); Rout = L^T working(Rl) if non-NULL.
template <typename T>
void launch_chol_upper(const double* G, const T* Rl, int c, double* Lt, double* Rout, int* flag, hipStream_t st);

// ---- TSQR (k_tsqr.hip): R factor only of an n x c block, Householder in precision T ----
int64_t tsqr_scratch_elems(int64_t n, int c);   // elements of T
template <typename T>
void launch_tsqr(const double* W, int64_t ldw, int64_t n, int c, T* scratch, T* R, hipStream_t st);

// ---- factorization (k_factor.hip) ----
struct FactorDev {
  int32_t* begin; int32_t* nc; int32_t* nr; int32_t* rows; int64_t* row_off; int32_t* relpos;
  int32_t* child_ptr; int32_t* child_list; int64_t* inv_off; int32_t* invmap;
  int64_t* panel_off; int64_t* upd_off; int64_t* uvec_off; int64_t* dinv_off; int64_t* lcopy_off;
  int32_t* prow; int32_t* pcol; int32_t* apos; double* aval;   // permuted A (CSR)
  const double* dense; int64_t ld_dense; int is_dense; int max_nr;
  int32_t* asm_items; int32_t* tasks; int32_t* ownrow_items;
};
template <typename T>
void launch_factor_step(const FactorDev& D, int kind, int level, int64_t task_off, int count,
                        int64_t asm_off, int64_t asm_count, T* panel, T* upd, T* dinv, T* lcopy, int* flag,
                        hipStream_t st);

// ---- supernodal triangular solves (k_trisolve.hip) ----
struct SolveDev {
  const int32_t* fwd_items; const int32_t* fwd_fin; const int32_t* bwd_items; const int32_t* bwd_fin;  // device
  const int64_t* fwd_level_off; const int64_t* fwd_fin_level_off;                                       // host
  const int64_t* bwd_level_off; const int64_t* bwd_fin_level_off; const int64_t* ownrow_level_off;      // host
};
// Both sweeps: rhs (T, n x M, permuted, overwritten by the forward assembly) -> y -> x, and W (FP64, n x mw,
// ld ldw) = working(x).  fpart / bpart: partial tiles (slots x 64 x M).
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
