// FP64 block kernels of the LOBPCG iteration: SpMM A*X (Algorithm 3 line 13),
// Gram products S^T Y (lines 11 and 13), block updates S*C (lines 11, 16),
// the residual R = A X - X Theta with its column norms (line 4, eq. (stop)).
// Blocks are row-major so that one row of an n x c block is contiguous.
// Reductions are two-stage with a fixed summation order (no atomics), so
// repeated runs give bitwise identical results.
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

// ----------------------------------------------------------------------------
// Gram partials: block (chunk, tile) computes a (16 RT) x (16 CT) tile of X^T Y over its
// row chunk; 256 threads in a 16 x 16 grid, each owning RT x CT outputs.  Rows are
// staged through LDS 16 at a time.  One tile covers c1, c2 <= 96.
// ----------------------------------------------------------------------------
template <int RT, int CT>
__global__ void __launch_bounds__(kThreads) gram_partial_kernel(const double* __restrict__ X, int64_t ldx,
                                                                const double* __restrict__ Y, int64_t ldy,
                                                                int64_t n, int c1, int c2, int64_t rows_per_chunk,
                                                                int tiles_j, double* __restrict__ part) {
  constexpr int T1 = 16 * RT, T2 = 16 * CT, KR = 16;
  __shared__ double Xs[KR][T1 + 1];
  __shared__ double Ys[KR][T2 + 1];
  const int t = threadIdx.x;
  const int tx = t % 16, ty = t / 16;
  const int chunk = blockIdx.x;
  const int ti = blockIdx.y / tiles_j, tj = blockIdx.y % tiles_j;
  const int i0 = ti * T1, j0 = tj * T2;
  const int64_t rbeg = (int64_t)chunk * rows_per_chunk;
  const int64_t rend = min(n, rbeg + rows_per_chunk);
  double acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = 0.0;
  for (int64_t r0 = rbeg; r0 < rend; r0 += KR) {
    for (int e = t; e < KR * T1; e += kThreads) {
      const int k = e / T1, c = e % T1;
      const int64_t r = r0 + k;
      Xs[k][c] = (r < rend && i0 + c < c1) ? X[r * ldx + i0 + c] : 0.0;
    }
    for (int e = t; e < KR * T2; e += kThreads) {
      const int k = e / T2, c = e % T2;
      const int64_t r = r0 + k;
      Ys[k][c] = (r < rend && j0 + c < c2) ? Y[r * ldy + j0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < KR; ++k) {
      double a[RT], b[CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i] = Xs[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < CT; ++j) b[j] = Ys[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* P = part + (int64_t)chunk * c1 * c2;
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    const int gi = i0 + ty + 16 * i;
    if (gi >= c1) continue;
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int gj = j0 + tx + 16 * j;
      if (gj < c2) P[gi * c2 + gj] = acc[i][j];
    }
  }
}

// out[e] = sum_b part[b][e] in a fixed order: four interleaved partial sums per output
// (b = g, g + 4, ...), combined in order g = 0..3.
__global__ void __launch_bounds__(256) reduce_parts_kernel(const double* __restrict__ part, int nb, int len,
                                                           double* __restrict__ out) {
  __shared__ double red[4][64];
  const int g = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int e = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (e < len) {
#pragma unroll 4
    for (int b = g; b < nb; b += 4) s += part[(int64_t)b * len + e];
  }
  red[g][lane] = s;
  __syncthreads();
  if (g == 0 && e < len) out[e] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

inline int gram_rt(int c) { return c <= 16 ? 1 : c <= 32 ? 2 : c <= 48 ? 3 : c <= 64 ? 4 : 6; }

int gram_chunks(int64_t n, int c1, int c2) {
  const int tiles = ceil_div(c1, 16 * gram_rt(c1)) * ceil_div(c2, 16 * gram_rt(c2));
  int chunks = ceil_div(n, 512);
  const int target = (384 + tiles - 1) / tiles;
  if (chunks > target) chunks = target;
  if (chunks < 1) chunks = 1;
  return chunks;
}

// ----------------------------------------------------------------------------
// Residual R = AX - X diag(theta) (cast to T) with per-block column sums of squares.
// ----------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kThreads) residual_kernel(const double* __restrict__ AX, int64_t ldax,
                                                            const double* __restrict__ X, int64_t ldx,
                                                            const double* __restrict__ theta, int64_t n, int m,
                                                            int64_t rows_per_block, T* __restrict__ R,
                                                            int64_t ldr, double* __restrict__ part) {
  __shared__ double red[2][4][64];
  const int t = threadIdx.x;
  const int j = t % 64, g = t / 64;
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t rend = min(n, rbeg + rows_per_block);
  double rs = 0.0, xs = 0.0;
  if (j < m) {
    const double th = theta[j];
    for (int64_t r = rbeg + g; r < rend; r += 4) {
      const double x = X[r * ldx + j];
      const double v = AX[r * ldax + j] - x * th;
      R[r * ldr + j] = (T)v;
      rs = fma(v, v, rs);
      xs = fma(x, x, xs);
    }
  }
  red[0][g][j] = rs;
  red[1][g][j] = xs;
  __syncthreads();
  if (t < 64 && t < m) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < 4; ++q) { a += red[0][q][t]; b += red[1][q][t]; }
    part[(int64_t)blockIdx.x * 2 * m + t] = a;
    part[(int64_t)blockIdx.x * 2 * m + m + t] = b;
  }
}

__global__ void __launch_bounds__(kThreads) colnorm_kernel(const double* __restrict__ X, int64_t ldx, int64_t n,
                                                           int c, int64_t rows_per_block, double* __restrict__ part) {
  __shared__ double red[4][64];
  const int t = threadIdx.x;
  const int j = t % 64, g = t / 64;
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_block;
  const int64_t rend = min(n, rbeg + rows_per_block);
  double xs = 0.0;
  if (j < c)
    for (int64_t r = rbeg + g; r < rend; r += 4) {
      const double x = X[r * ldx + j];
      xs = fma(x, x, xs);
    }
  red[g][j] = xs;
  __syncthreads();
  if (t < c) {
    double a = 0.0;
    for (int q = 0; q < 4; ++q) a += red[q][t];
    part[(int64_t)blockIdx.x * c + t] = a;
  }
}

int resid_blocks(int64_t n) {
  int nb = ceil_div(n, 256);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return nb;
}

__global__ void gather_rows_kernel(const double* __restrict__ src, int64_t lds, const int32_t* __restrict__ idx,
                                   double* __restrict__ dst, int64_t ldd, int64_t nrows, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  const int64_t si = idx ? (int64_t)idx[i] : i;
  dst[i * ldd + j] = src[si * lds + j];
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

__global__ void cast_f64_f32_kernel(const double* __restrict__ src, int64_t lds, float* __restrict__ dst,
                                    int64_t ldd, int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  dst[i * ldd + j] = (float)src[i * lds + j];
}

__global__ void cast_f32_f64_kernel(const float* __restrict__ src, int64_t lds, double* __restrict__ dst,
                                    int64_t ldd, int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  dst[i * ldd + j] = (double)src[i * lds + j];
}

inline dim3 grid1(int64_t total) { return dim3((unsigned)((total + kThreads - 1) / kThreads)); }

}  // namespace

void launch_spmm_csr(const int32_t* rowptr, const int32_t* colind, const double* val, int64_t n, const double* X,
                     int64_t ldx, double* Y, int64_t ldy, int c, hipStream_t st) {
  if (n <= 0 || c <= 0) return;
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

int64_t gram_scratch(int64_t n, int c1, int c2) { return (int64_t)gram_chunks(n, c1, c2) * c1 * c2; }

template <int RT, int CT>
void gram_launch(dim3 g, const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n, int c1, int c2,
                 int64_t rpc, int tj, double* part, hipStream_t st) {
  gram_partial_kernel<RT, CT><<<g, kThreads, 0, st>>>(X, ldx, Y, ldy, n, c1, c2, rpc, tj, part);
}

template <int RT>
void gram_dispatch_ct(int ct, dim3 g, const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n, int c1,
                      int c2, int64_t rpc, int tj, double* part, hipStream_t st) {
  switch (ct) {
    case 1: gram_launch<RT, 1>(g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
    case 2: gram_launch<RT, 2>(g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
    case 3: gram_launch<RT, 3>(g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
    case 4: gram_launch<RT, 4>(g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
    default: gram_launch<RT, 6>(g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
  }
}

void launch_gram(const double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t n, int c1, int c2, double* G,
                 double* part, hipStream_t st) {
  if (c1 <= 0 || c2 <= 0) return;
  const int chunks = gram_chunks(n, c1, c2);
  const int64_t rpc = n > 0 ? (n + chunks - 1) / chunks : 1;
  const int rt = gram_rt(c1), ct = gram_rt(c2);
  const int tj = ceil_div(c2, 16 * ct);
  dim3 g(chunks, ceil_div(c1, 16 * rt) * tj);
  switch (rt) {
    case 1: gram_dispatch_ct<1>(ct, g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
    case 2: gram_dispatch_ct<2>(ct, g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
    case 3: gram_dispatch_ct<3>(ct, g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
    case 4: gram_dispatch_ct<4>(ct, g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
    default: gram_dispatch_ct<6>(ct, g, X, ldx, Y, ldy, n, c1, c2, rpc, tj, part, st); break;
  }
  const int len = c1 * c2;
  reduce_parts_kernel<<<ceil_div(len, 64), 256, 0, st>>>(part, chunks, len, G);
}

void launch_block_update(const double* X, int64_t ldx, const double* M, int64_t ldm, double* Y, int64_t ldy,
                         int64_t n, int cin, int cout, double alpha, double beta, hipStream_t st) {
  if (n <= 0 || cout <= 0) return;
  dim3 g(ceil_div(n, 64), ceil_div(cout, 64));
  gemm_nn_kernel<<<g, kThreads, 0, st>>>(X, ldx, M, ldm, Y, ldy, n, cin, cout, alpha, beta);
}

int64_t resid_scratch(int64_t n, int m) { return (int64_t)resid_blocks(n) * 2 * m; }

template <typename T>
void launch_residual(const double* AX, int64_t ldax, const double* X, int64_t ldx, const double* theta, int64_t n,
                     int m, T* R, int64_t ldr, double* norms, double* part, hipStream_t st) {
  const int nb = resid_blocks(n);
  const int64_t rpb = (n + nb - 1) / nb;
  residual_kernel<T><<<nb, kThreads, 0, st>>>(AX, ldax, X, ldx, theta, n, m, rpb, R, ldr, part);
  reduce_parts_kernel<<<ceil_div(2 * m, 64), 256, 0, st>>>(part, nb, 2 * m, norms);
}
template void launch_residual<float>(const double*, int64_t, const double*, int64_t, const double*, int64_t, int,
                                     float*, int64_t, double*, double*, hipStream_t);
template void launch_residual<double>(const double*, int64_t, const double*, int64_t, const double*, int64_t, int,
                                      double*, int64_t, double*, double*, hipStream_t);

void launch_colnorms(const double* X, int64_t ldx, int64_t n, int c, double* norms, double* part, hipStream_t st) {
  const int nb = resid_blocks(n);
  const int64_t rpb = (n + nb - 1) / nb;
  colnorm_kernel<<<nb, kThreads, 0, st>>>(X, ldx, n, c, rpb, part);
  reduce_parts_kernel<<<ceil_div(c, 64), 256, 0, st>>>(part, nb, c, norms);
}

void launch_gather_rows(const double* src, int64_t lds, const int32_t* idx, double* dst, int64_t ldd, int64_t nrows,
                        int c, hipStream_t st) {
  if (nrows * c <= 0) return;
  gather_rows_kernel<<<grid1(nrows * c), kThreads, 0, st>>>(src, lds, idx, dst, ldd, nrows, c);
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

void launch_cast_f64_f32(const double* src, int64_t lds, float* dst, int64_t ldd, int64_t n, int c, hipStream_t st) {
  if (n * c <= 0) return;
  cast_f64_f32_kernel<<<grid1(n * c), kThreads, 0, st>>>(src, lds, dst, ldd, n, c);
}

void launch_cast_f32_f64(const float* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int c, hipStream_t st) {
  if (n * c <= 0) return;
  cast_f32_f64_kernel<<<grid1(n * c), kThreads, 0, st>>>(src, lds, dst, ldd, n, c);
}

void launch_reduce_parts(const double* part, int nb, int len, double* out, hipStream_t st) {
  reduce_parts_kernel<<<ceil_div(len, 64), 256, 0, st>>>(part, nb, len, out);
}

}  // namespace lobpcg
