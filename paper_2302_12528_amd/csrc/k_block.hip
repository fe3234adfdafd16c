// FP64 products with A (Algorithm 3 line 13: CSR SpMM, or a dense product
// for dense A) and the data-movement kernels around them (row gathers for
// the permutation, value gathers, start-block generation).  Blocks are
// row-major so that one row of an n x c block is contiguous.
#include "common.hpp"

namespace lobpcg {

namespace {

constexpr int kThreads = 256;

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ----------------------------------------------------------------------------
// SpMM: a group of G lanes handles one row; lane j handles column blockIdx.y*G + j.
// ----------------------------------------------------------------------------
template <int G>
__global__ void __launch_bounds__(kThreads) spmm_csr_kernel(const int32_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ colind,
                                                            const double* __restrict__ val, int64_t n,
                                                            const double* __restrict__ X, int64_t ldx,
                                                            double* __restrict__ Y, int64_t ldy, int c) {
  const int lane = threadIdx.x % G;
  const int64_t row = (int64_t)blockIdx.x * (kThreads / G) + threadIdx.x / G;
  const int col = blockIdx.y * G + lane;
  if (row >= n || col >= c) return;
  const int32_t e0 = rowptr[row], e1 = rowptr[row + 1];
  double acc = 0.0;
  for (int32_t e = e0; e < e1; ++e) acc = fma(val[e], X[(int64_t)colind[e] * ldx + col], acc);
  Y[row * ldy + col] = acc;
}

// Two columns per lane with 16-byte loads and stores (c, ldx, ldy even, X and Y 16-byte aligned):
// a group of G lanes covers 2G columns of one row; the entries of a row are fetched four at a
// time so that four row gathers of X are in flight per lane.  Each output is the same fma chain
// in entry order as the one-column kernel.
template <int G>
__global__ void __launch_bounds__(kThreads) spmm_csr2_kernel(const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ colind,
                                                             const double* __restrict__ val, int64_t n,
                                                             const double* __restrict__ X, int64_t ldx,
                                                             double* __restrict__ Y, int64_t ldy, int c) {
  const int lane = threadIdx.x % G;
  const int64_t row = (int64_t)blockIdx.x * (kThreads / G) + threadIdx.x / G;
  const int col = (blockIdx.y * G + lane) * 2;
  if (row >= n || col >= c) return;
  const int32_t e0 = rowptr[row], e1 = rowptr[row + 1];
  double ax = 0.0, ay = 0.0;
  int32_t e = e0;
  for (; e + 4 <= e1; e += 4) {
    int32_t j[4];
    double v[4];
    double2 x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      j[q] = colind[e + q];
      v[q] = val[e + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = *reinterpret_cast<const double2*>(X + (int64_t)j[q] * ldx + col);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ax = fma(v[q], x[q].x, ax);
      ay = fma(v[q], x[q].y, ay);
    }
  }
  for (; e < e1; ++e) {
    const double v = val[e];
    const double2 x = *reinterpret_cast<const double2*>(X + (int64_t)colind[e] * ldx + col);
    ax = fma(v, x.x, ax);
    ay = fma(v, x.y, ay);
  }
  *reinterpret_cast<double2*>(Y + row * ldy + col) = make_double2(ax, ay);
}

// ----------------------------------------------------------------------------
// 64 x 64 output tile of C = alpha * A B + beta * C with A (rows x K) and B (K x cols)
// both row-major.  256 threads, 4 x 4 outputs each, K staged through LDS 16 at a time.
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) gemm_nn_kernel(const double* A, int64_t lda,
                                                           const double* __restrict__ B, int64_t ldb,
                                                           double* C, int64_t ldc, int64_t rows, int K,
                                                           int cols, double alpha, double beta) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][64];
  const int t = threadIdx.x;
  const int tx = t % 16, ty = t / 16;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const int c0 = blockIdx.y * 64;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  const int lr = t / 4, lk = (t % 4) * 4;      // A loader: row lr, k lk..lk+3
  const int bk = t / 16, bc = (t % 16) * 4;    // B loader: k bk, cols bc..bc+3
  for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + lr;
      const int k = k0 + lk + q;
      As[lk + q][lr] = (r < rows && k < K) ? A[r * lda + k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + bk;
      const int cc = c0 + bc + q;
      Bs[bk][bc + q] = (k < K && cc < cols) ? B[(int64_t)k * ldb + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t r = r0 + ty + 16 * i;
    if (r >= rows) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cc = c0 + tx + 16 * j;
      if (cc >= cols) continue;
      double v = alpha * acc[i][j];
      if (beta != 0.0) v = fma(beta, C[r * ldc + cc], v);
      C[r * ldc + cc] = v;
    }
  }
}

__global__ void gather_rows_kernel(const double* __restrict__ src, int64_t lds, const int32_t* __restrict__ idx,
                                   int64_t base, double* __restrict__ dst, int64_t ldd, int64_t nrows, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  const int64_t si = idx ? (int64_t)idx[i] - base : i;
  dst[i * ldd + j] = src[si * lds + j];
}

__global__ void fill_int_kernel(int32_t* p, int32_t v, int64_t count) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) p[e] = v;
}

__global__ void gather_values_kernel(const double* __restrict__ src, const int32_t* __restrict__ map,
                                     double* __restrict__ dst, int64_t nnz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) dst[e] = src[map[e]];
}

__global__ void add_diag_shift_kernel(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                      double* __restrict__ val, const int32_t* __restrict__ perm,
                                      const double* __restrict__ shift, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
    if (colind[e] == i) val[e] += shift[perm[i]];
}

__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void gaussian_fill_kernel(double* X, int64_t n, int c, int64_t ld, uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  const uint64_t a = splitmix64(seed ^ (2ull * (uint64_t)e));
  const uint64_t b = splitmix64(seed ^ (2ull * (uint64_t)e + 1ull));
  const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740992.0);   // (0, 1]
  const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
  X[i * ld + j] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

__global__ void copy_block_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                                  int64_t ldd, int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  dst[i * ldd + j] = src[i * lds + j];
}

__global__ void sub_block_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                                 int64_t ldd, int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  dst[i * ldd + j] -= src[i * lds + j];
}

inline dim3 grid1(int64_t total) { return dim3((unsigned)((total + kThreads - 1) / kThreads)); }

}  // namespace

void launch_spmm_csr(const int32_t* rowptr, const int32_t* colind, const double* val, int64_t n, const double* X,
                     int64_t ldx, double* Y, int64_t ldy, int c, hipStream_t st) {
  if (n <= 0 || c <= 0) return;
  const bool pairs = (c % 2 == 0) && (ldx % 2 == 0) && (ldy % 2 == 0) && ((uintptr_t)X % 16 == 0) &&
                     ((uintptr_t)Y % 16 == 0);
  if (pairs) {
    const int half = c / 2;
    if (half <= 4) {
      spmm_csr2_kernel<4><<<dim3(ceil_div(n, kThreads / 4), 1), kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx,
                                                                                 Y, ldy, c);
    } else if (half <= 8) {
      spmm_csr2_kernel<8><<<dim3(ceil_div(n, kThreads / 8), 1), kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx,
                                                                                 Y, ldy, c);
    } else if (half <= 16) {
      spmm_csr2_kernel<16><<<dim3(ceil_div(n, kThreads / 16), 1), kThreads, 0, st>>>(rowptr, colind, val, n, X,
                                                                                   ldx, Y, ldy, c);
    } else {
      spmm_csr2_kernel<32><<<dim3(ceil_div(n, kThreads / 32), ceil_div(half, 32)), kThreads, 0, st>>>(
          rowptr, colind, val, n, X, ldx, Y, ldy, c);
    }
    return;
  }
  if (c <= 8) {
    dim3 g(ceil_div(n, kThreads / 8), 1);
    spmm_csr_kernel<8><<<g, kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx, Y, ldy, c);
  } else if (c <= 16) {
    dim3 g(ceil_div(n, kThreads / 16), 1);
    spmm_csr_kernel<16><<<g, kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx, Y, ldy, c);
  } else if (c <= 32) {
    dim3 g(ceil_div(n, kThreads / 32), 1);
    spmm_csr_kernel<32><<<g, kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx, Y, ldy, c);
  } else {
    dim3 g(ceil_div(n, kThreads / 64), ceil_div(c, 64));
    spmm_csr_kernel<64><<<g, kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx, Y, ldy, c);
  }
}

void launch_dense_mm(const double* A, int64_t lda, int64_t n, const double* X, int64_t ldx, double* Y,
                     int64_t ldy, int c, hipStream_t st) {
  if (n <= 0 || c <= 0) return;
  dim3 g(ceil_div(n, 64), ceil_div(c, 64));
  gemm_nn_kernel<<<g, kThreads, 0, st>>>(A, lda, X, ldx, Y, ldy, n, (int)n, c, 1.0, 0.0);
}

void launch_gather_rows(const double* src, int64_t lds, const int32_t* idx, int64_t base, double* dst, int64_t ldd,
                        int64_t nrows, int c, hipStream_t st) {
  if (nrows * c <= 0) return;
  gather_rows_kernel<<<grid1(nrows * c), kThreads, 0, st>>>(src, lds, idx, base, dst, ldd, nrows, c);
}

void launch_fill_int(int32_t* p, int32_t v, int64_t count, hipStream_t st) {
  if (count > 0) fill_int_kernel<<<grid1(count), kThreads, 0, st>>>(p, v, count);
}

void launch_gather_values(const double* src, const int32_t* map, double* dst, int64_t nnz, hipStream_t st) {
  if (nnz <= 0) return;
  gather_values_kernel<<<grid1(nnz), kThreads, 0, st>>>(src, map, dst, nnz);
}

void launch_add_diag_shift(const int32_t* rowptr, const int32_t* colind, double* val, const int32_t* perm,
                           const double* shift, int64_t n, hipStream_t st) {
  add_diag_shift_kernel<<<grid1(n), kThreads, 0, st>>>(rowptr, colind, val, perm, shift, n);
}

void launch_gaussian_fill(double* X, int64_t n, int c, int64_t ld, uint64_t seed, hipStream_t st) {
  if (n * c <= 0) return;
  gaussian_fill_kernel<<<grid1(n * c), kThreads, 0, st>>>(X, n, c, ld, seed);
}

void launch_copy_block(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int c, hipStream_t st) {
  if (n * c <= 0) return;
  copy_block_kernel<<<grid1(n * c), kThreads, 0, st>>>(src, lds, dst, ldd, n, c);
}

void launch_sub_block(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int c, hipStream_t st) {
  if (n * c <= 0) return;
  sub_block_kernel<<<grid1(n * c), kThreads, 0, st>>>(src, lds, dst, ldd, n, c);
}

}  // namespace lobpcg
