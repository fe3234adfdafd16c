// Column-wise kernels of the adjoint (backward) solve: per-column dot products
// (deterministic two-stage reduction), column-scaled updates, the shifted
// product (A - theta_j I) p_j, and the diagonal-potential gradient
//   g_r = sum_i dtheta_i X(r,i)^2 - sum_i Y(r,i) X(r,i).
// Blocks are n x c row-major FP64 (c <= 64).
#include "common.hpp"

namespace lobpcg {

namespace {

constexpr int kT = 256;

inline int nblocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (int)b;
}

__global__ void __launch_bounds__(kT) coldots_kernel(const double* __restrict__ X, int64_t ldx,
                                                     const double* __restrict__ Y, int64_t ldy, int64_t n, int c,
                                                     int64_t rows_per_block, double* __restrict__ part) {
  __shared__ double red[4][64];
  const int t = threadIdx.x, j = t % 64, g = t / 64;
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t rend = min(n, rbeg + rows_per_block);
  double s = 0.0;
  if (j < c)
    for (int64_t r = rbeg + g; r < rend; r += 4) s = fma(X[r * ldx + j], Y[r * ldy + j], s);
  red[g][j] = s;
  __syncthreads();
  if (t < c) part[(int64_t)blockIdx.x * c + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

__global__ void __launch_bounds__(64) coldots_reduce_kernel(const double* __restrict__ part, int nb, int c,
                                                            double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= c) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * c + j];
  out[j] = s;
}

// Y(:, j) += sign * alpha_j X(:, j)
__global__ void axpy_cols_kernel(const double* __restrict__ alpha, double sign, const double* __restrict__ X,
                                 int64_t ldx, double* __restrict__ Y, int64_t ldy, int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t r = e / c;
  const int j = (int)(e % c);
  Y[r * ldy + j] = fma(sign * alpha[j], X[r * ldx + j], Y[r * ldy + j]);
}

// P(:, j) = Z(:, j) + beta_j P(:, j)
__global__ void xpby_cols_kernel(const double* __restrict__ beta, const double* __restrict__ Z, int64_t ldz,
                                 double* __restrict__ P, int64_t ldp, int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t r = e / c;
  const int j = (int)(e % c);
  P[r * ldp + j] = fma(beta[j], P[r * ldp + j], Z[r * ldz + j]);
}

// Q(:, j) = AP(:, j) - theta_j P(:, j)
__global__ void shift_cols_kernel(const double* __restrict__ AP, int64_t lda, const double* __restrict__ P,
                                  int64_t ldp, const double* __restrict__ theta, double* __restrict__ Q, int64_t ldq,
                                  int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t r = e / c;
  const int j = (int)(e % c);
  Q[r * ldq + j] = AP[r * lda + j] - theta[j] * P[r * ldp + j];
}

__global__ void diag_grad_kernel(const double* __restrict__ X, int64_t ldx, const double* __restrict__ dtheta,
                                 const double* __restrict__ Y, int64_t ldy, int64_t n, int k,
                                 double* __restrict__ g) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double s = 0.0;
  for (int i = 0; i < k; ++i) {
    const double x = X[r * ldx + i];
    if (dtheta) s = fma(dtheta[i] * x, x, s);
    if (Y) s = fma(-Y[r * ldy + i], x, s);
  }
  g[r] = s;
}

inline unsigned grid_of(int64_t total) { return (unsigned)((total + kT - 1) / kT); }

}  // namespace

int64_t coldots_scratch(int64_t n, int c) { return (int64_t)nblocks(n) * c; }

void launch_coldots(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n, int c, double* out,
                    double* part, hipStream_t st) {
  const int nb = nblocks(n);
  const int64_t rpb = (n + nb - 1) / nb;
  coldots_kernel<<<nb, kT, 0, st>>>(X, ldx, Y, ldy, n, c, rpb, part);
  coldots_reduce_kernel<<<1, 64, 0, st>>>(part, nb, c, out);
}

void launch_axpy_cols(const double* alpha, double sign, const double* X, int64_t ldx, double* Y, int64_t ldy,
                      int64_t n, int c, hipStream_t st) {
  if (n * c > 0) axpy_cols_kernel<<<grid_of(n * c), kT, 0, st>>>(alpha, sign, X, ldx, Y, ldy, n, c);
}

void launch_xpby_cols(const double* beta, const double* Z, int64_t ldz, double* P, int64_t ldp, int64_t n, int c,
                      hipStream_t st) {
  if (n * c > 0) xpby_cols_kernel<<<grid_of(n * c), kT, 0, st>>>(beta, Z, ldz, P, ldp, n, c);
}

void launch_shift_cols(const double* AP, int64_t lda, const double* P, int64_t ldp, const double* theta, double* Q,
                       int64_t ldq, int64_t n, int c, hipStream_t st) {
  if (n * c > 0) shift_cols_kernel<<<grid_of(n * c), kT, 0, st>>>(AP, lda, P, ldp, theta, Q, ldq, n, c);
}

void launch_diag_grad(const double* X, int64_t ldx, const double* dtheta, const double* Y, int64_t ldy, int64_t n,
                      int k, double* g, hipStream_t st) {
  if (n > 0) diag_grad_kernel<<<grid_of(n), kT, 0, st>>>(X, ldx, dtheta, Y, ldy, n, k, g);
}

}  // namespace lobpcg
