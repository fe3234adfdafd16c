// FP64 products with A (Algorithm 3 line 13: CSR SpMM, or a dense product
// for dense A) and the data-movement kernels around them (row gathers for
// the permutation, value gathers, start-block generation).  Blocks are
// row-major so that one row of an n x c block is contiguous.
#include <algorithm>

#include "common.hpp"
#include "mfma.hpp"

namespace lobpcg {

namespace {

constexpr int kThreads = 256;
constexpr int kMmMaxSplits = 8;   // reduction ranges of the dense product

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ----------------------------------------------------------------------------
// SpMM: a group of G lanes handles one row; lane j handles column blockIdx.y*G + j.
// ----------------------------------------------------------------------------
template <int G, typename T>
__global__ void __launch_bounds__(kThreads) spmm_csr_kernel(const int32_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ colind,
                                                            const T* __restrict__ val, int64_t n,
                                                            const T* __restrict__ X, int64_t ldx,
                                                            T* __restrict__ Y, int64_t ldy, int c) {
  const int lane = threadIdx.x % G;
  const int64_t row = (int64_t)blockIdx.x * (kThreads / G) + threadIdx.x / G;
  const int col = blockIdx.y * G + lane;
  if (row >= n || col >= c) return;
  const int32_t e0 = rowptr[row], e1 = rowptr[row + 1];
  T acc = 0;
  for (int32_t e = e0; e < e1; ++e) acc = fma(val[e], X[(int64_t)colind[e] * ldx + col], acc);
  Y[row * ldy + col] = acc;
}

// Two columns per lane with 16-byte loads and stores (c, ldx, ldy even, X and Y 16-byte aligned):
// a group of G lanes covers 2G columns of one row; the entries of a row are fetched four at a
// time so that four row gathers of X are in flight per lane.  Each output is the same fma chain
// in entry order as the one-column kernel.  (FP32, for the lower-precision first stage: 8-byte
// accesses, the same structure.)
template <int G, typename T>
__global__ void __launch_bounds__(kThreads) spmm_csr2_kernel(const int32_t* __restrict__ rowptr,
                                                             const int32_t* __restrict__ colind,
                                                             const T* __restrict__ val, int64_t n,
                                                             const T* __restrict__ X, int64_t ldx,
                                                             T* __restrict__ Y, int64_t ldy, int c) {
  typedef T V2 __attribute__((ext_vector_type(2)));
  const int lane = threadIdx.x % G;
  const int64_t row = (int64_t)blockIdx.x * (kThreads / G) + threadIdx.x / G;
  const int col = (blockIdx.y * G + lane) * 2;
  if (row >= n || col >= c) return;
  const int32_t e0 = rowptr[row], e1 = rowptr[row + 1];
  T ax = 0, ay = 0;
  int32_t e = e0;
  for (; e + 4 <= e1; e += 4) {
    int32_t j[4];
    T v[4];
    V2 x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      j[q] = colind[e + q];
      v[q] = val[e + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = *reinterpret_cast<const V2*>(X + (int64_t)j[q] * ldx + col);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ax = fma(v[q], x[q].x, ax);
      ay = fma(v[q], x[q].y, ay);
    }
  }
  for (; e < e1; ++e) {
    const T v = val[e];
    const V2 x = *reinterpret_cast<const V2*>(X + (int64_t)colind[e] * ldx + col);
    ax = fma(v, x.x, ax);
    ay = fma(v, x.y, ay);
  }
  *reinterpret_cast<V2*>(Y + row * ldy + col) = V2{ax, ay};
}

// ----------------------------------------------------------------------------
// Dense Y = A X on the FP64 matrix cores (dense A, Algorithm 3 line 13).  A workgroup of 8 waves
// computes a 128 x 64 output tile over one range of the reduction index (gridDim.z ranges of kspan):
// wave w owns rows 16 w .. 16 w + 15 as four 16 x 16 blocks accumulated by v_mfma_f64_16x16x4f64.
// Chunks of 32 reduction indices of the A rows ([row][k], row-major as A) and of the X rows
// ([k][col]) pass through LDS; the next chunk is loaded into registers (16-byte loads) while the
// current one is multiplied.  With one range the tile is written to Y, otherwise to part[z] and
// dense_mm_reduce_kernel adds the ranges in a fixed order.
// LDS strides: A rows of 34 doubles (lanes i, g of an operand read fall on banks 4 i + 2 g, all
// distinct over a half wave), X rows of 80 doubles (the two k rows of a half wave 128 bytes apart).
// ----------------------------------------------------------------------------
constexpr int kMmRows = 128, kMmK = 32, kMmLdA = kMmK + 2, kMmLdX = 64 + 16, kMmThreads = 512;

template <bool VEC, typename T>
__global__ void __launch_bounds__(kMmThreads) dense_mm_kernel(const T* __restrict__ A, int64_t lda, int64_t n,
                                                              const T* __restrict__ X, int64_t ldx,
                                                              T* __restrict__ Y, int64_t ldy, int c,
                                                              int64_t kspan, T* __restrict__ part) {
  typedef Mfma<T> MF;
  typedef typename MF::v4 V4;
  typedef T V2 __attribute__((ext_vector_type(2)));
  __shared__ __align__(16) T As[kMmRows][kMmLdA];
  __shared__ __align__(16) T Xs[kMmK][kMmLdX];
  const int t = threadIdx.x, lane = t % 64, w = t / 64, i = lane % 16, g = lane / 16;
  const int64_t r0 = (int64_t)blockIdx.x * kMmRows;
  const int c0 = blockIdx.y * 64;
  const int64_t kb = (int64_t)blockIdx.z * kspan;
  const int64_t ke = min(n, kb + kspan);
  // loaders: A pair e = t + 512 q (q < 4) is row e / 16, reduction pair e % 16; X pair e = t + 512 q
  // (q < 2) is reduction row e / 32, column pair e % 32
  V2 ra[4], rx[2];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + kMmThreads * q;
      const int64_t r = r0 + e / 16, k = k0 + 2 * (e % 16);
      V2 v = V2{0, 0};
      if (r < n) {
        const T* src = A + r * lda + k;
        if (VEC && k + 1 < ke) {
          v = *reinterpret_cast<const V2*>(src);
        } else {
          if (k < ke) v.x = src[0];
          if (k + 1 < ke) v.y = src[1];
        }
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + kMmThreads * q;
      const int64_t k = k0 + e / 32;
      const int col = c0 + 2 * (e % 32);
      V2 v = V2{0, 0};
      if (k < ke) {
        const T* src = X + k * ldx + col;
        if (VEC && col + 1 < c) {
          v = *reinterpret_cast<const V2*>(src);
        } else {
          if (col < c) v.x = src[0];
          if (col + 1 < c) v.y = src[1];
        }
      }
      rx[q] = v;
    }
  };
  V4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = V4{0, 0, 0, 0};
  if (kb < ke) load(kb);
  for (int64_t k0 = kb; k0 < ke; k0 += kMmK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + kMmThreads * q;
      *reinterpret_cast<V2*>(&As[e / 16][2 * (e % 16)]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int e = t + kMmThreads * q;
      *reinterpret_cast<V2*>(&Xs[e / 32][2 * (e % 32)]) = rx[q];
    }
    __syncthreads();
    if (k0 + kMmK < ke) load(k0 + kMmK);
#pragma unroll
    for (int kk = 0; kk < kMmK; kk += 4) {
      const T a = As[16 * w + i][kk + g];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = MF::op(a, Xs[kk + g][16 * cb + i], acc[cb]);
    }
  }
  const int cpad = gridDim.y * 64;
  T* P = part ? part + (int64_t)blockIdx.z * n * cpad : nullptr;
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t r = r0 + 16 * w + MF::drow(lane, q);
      const int col = c0 + 16 * cb + i;
      if (r >= n || col >= c) continue;
      if (P)
        P[r * cpad + col] = acc[cb][q];
      else
        Y[r * ldy + col] = acc[cb][q];
    }
}

// Y(r, col) = sum over z = 0 .. nz - 1, in order, of part[z](r, col)
template <typename T>
__global__ void __launch_bounds__(kThreads) dense_mm_reduce_kernel(const T* __restrict__ part, int nz,
                                                                   int64_t n, int c, int cpad,
                                                                   T* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n * c) return;
  const int64_t r = e / c;
  const int col = (int)(e % c);
  T s = 0;
  for (int z = 0; z < nz; ++z) s += part[((int64_t)z * n + r) * cpad + col];
  Y[r * ldy + col] = s;
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

template <typename Tin, typename Tout>
__global__ void convert_block_kernel(const Tin* __restrict__ src, int64_t lds, Tout* __restrict__ dst, int64_t ldd,
                                     int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  dst[i * ldd + j] = (Tout)src[i * lds + j];
}

__global__ void sub_block_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                                 int64_t ldd, int64_t n, int c) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * c) return;
  const int64_t i = e / c;
  const int j = (int)(e % c);
  dst[i * ldd + j] -= src[i * lds + j];
}

// Complex n x m block X (element (i, j) = X[2 (i m + j)] + i X[2 (i m + j) + 1]) -> the real 2n x 2m block
// [[Re X, -Im X], [Im X, Re X]] of the real symmetric embedding (its columns span the embedded complex
// span, closed under multiplication by i).
__global__ void herm_expand_kernel(const double* __restrict__ X, int64_t n, int m, double* __restrict__ Y) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m;
  const int j = (int)(e % m);
  const double re = X[2 * e], im = X[2 * e + 1];
  const int64_t ld = 2 * m;
  Y[i * ld + j] = re;
  Y[i * ld + m + j] = -im;
  Y[(n + i) * ld + j] = im;
  Y[(n + i) * ld + m + j] = re;
}

// The k complex eigenpairs from the 2k real Ritz pairs of the embedding (Z 2n x 2k, row-major): pair j
// is columns 2j, 2j + 1 (one double eigenvalue); x_j = Z[0:n, 2j] + i Z[n:2n, 2j], lambda_j = theta_2j.
__global__ void herm_extract_kernel(const double* __restrict__ Z, const double* __restrict__ theta, int64_t n, int k,
                                    double* __restrict__ X, double* __restrict__ lam) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < k) lam[e] = theta[2 * e];
  if (e >= n * k) return;
  const int64_t i = e / k;
  const int j = (int)(e % k);
  X[2 * e] = Z[i * 2 * k + 2 * j];
  X[2 * e + 1] = Z[(n + i) * 2 * k + 2 * j];
}

// Complex Gram matrix of the extracted eigenvectors from the real Gram R (2k x 2k) of the same block read
// as real n x 2k (columns Re x_1, Im x_1, Re x_2, ...): G_ij = x_i^H x_j = (R_{2i,2j} + R_{2i+1,2j+1}) +
// i (R_{2i,2j+1} - R_{2i+1,2j}); then its Cholesky factor G = L L^H (complex, L lower), by one thread
// (k <= 32, once per solve).  A non-positive pivot leaves L = I (the vectors are then returned as read).
__global__ void herm_chol_kernel(const double* __restrict__ R, int k, double* __restrict__ L) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k2 = 2 * k;
  auto re = [&](int i, int j) { return R[(2 * i) * k2 + 2 * j] + R[(2 * i + 1) * k2 + 2 * j + 1]; };
  auto im = [&](int i, int j) { return R[(2 * i) * k2 + 2 * j + 1] - R[(2 * i + 1) * k2 + 2 * j]; };
  bool ok = true;
  for (int j = 0; j < k && ok; ++j) {
    double dj = re(j, j);
    for (int q = 0; q < j; ++q) dj -= L[2 * (j * k + q)] * L[2 * (j * k + q)] + L[2 * (j * k + q) + 1] * L[2 * (j * k + q) + 1];
    if (!(dj > 0.0)) {
      ok = false;
      break;
    }
    const double ljj = sqrt(dj);
    L[2 * (j * k + j)] = ljj;
    L[2 * (j * k + j) + 1] = 0.0;
    for (int i = j + 1; i < k; ++i) {   // L_ij = (G_ij - sum_q L_iq conj(L_jq)) / L_jj, G_ij = conj(G_ji)
      double sr = re(j, i), si = -im(j, i);
      for (int q = 0; q < j; ++q) {
        const double ar = L[2 * (i * k + q)], ai = L[2 * (i * k + q) + 1];
        const double br = L[2 * (j * k + q)], bi = -L[2 * (j * k + q) + 1];
        sr -= ar * br - ai * bi;
        si -= ar * bi + ai * br;
      }
      L[2 * (i * k + j)] = sr / ljj;
      L[2 * (i * k + j) + 1] = si / ljj;
    }
    for (int i = 0; i < j; ++i) {
      L[2 * (i * k + j)] = 0.0;
      L[2 * (i * k + j) + 1] = 0.0;
    }
  }
  if (!ok)
    for (int e = 0; e < k * k; ++e) {
      L[2 * e] = (e / k == e % k) ? 1.0 : 0.0;
      L[2 * e + 1] = 0.0;
    }
}

// X <- X L^{-H} row by row (X n x k complex, one thread per row): y L^H = x, with (L^H)_{qj} = conj(L_{jq}).
__global__ void herm_rowsolve_kernel(double* __restrict__ X, int64_t n, int k, const double* __restrict__ L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double yr[32], yi[32];
  double* x = X + 2 * i * k;
  for (int j = 0; j < k; ++j) {
    double sr = x[2 * j], si = x[2 * j + 1];
    for (int q = 0; q < j; ++q) {   // subtract y_q conj(L_jq)
      const double lr = L[2 * (j * k + q)], li = -L[2 * (j * k + q) + 1];
      sr -= yr[q] * lr - yi[q] * li;
      si -= yr[q] * li + yi[q] * lr;
    }
    const double d = L[2 * (j * k + j)];
    yr[j] = sr / d;
    yi[j] = si / d;
  }
  for (int j = 0; j < k; ++j) {
    x[2 * j] = yr[j];
    x[2 * j + 1] = yi[j];
  }
}

inline dim3 grid1(int64_t total) { return dim3((unsigned)((total + kThreads - 1) / kThreads)); }

}  // namespace

template <typename T>
void launch_spmm_csr(const int32_t* rowptr, const int32_t* colind, const T* val, int64_t n, const T* X,
                     int64_t ldx, T* Y, int64_t ldy, int c, hipStream_t st) {
  if (n <= 0 || c <= 0) return;
  const bool pairs = (c % 2 == 0) && (ldx % 2 == 0) && (ldy % 2 == 0) && ((uintptr_t)X % 16 == 0) &&
                     ((uintptr_t)Y % 16 == 0);
  if (pairs) {
    const int half = c / 2;
    if (half <= 4) {
      spmm_csr2_kernel<4, T><<<dim3(ceil_div(n, kThreads / 4), 1), kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx,
                                                                                 Y, ldy, c);
    } else if (half <= 8) {
      spmm_csr2_kernel<8, T><<<dim3(ceil_div(n, kThreads / 8), 1), kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx,
                                                                                 Y, ldy, c);
    } else if (half <= 16) {
      spmm_csr2_kernel<16, T><<<dim3(ceil_div(n, kThreads / 16), 1), kThreads, 0, st>>>(rowptr, colind, val, n, X,
                                                                                   ldx, Y, ldy, c);
    } else {
      spmm_csr2_kernel<32, T><<<dim3(ceil_div(n, kThreads / 32), ceil_div(half, 32)), kThreads, 0, st>>>(
          rowptr, colind, val, n, X, ldx, Y, ldy, c);
    }
    return;
  }
  if (c <= 8) {
    dim3 g(ceil_div(n, kThreads / 8), 1);
    spmm_csr_kernel<8, T><<<g, kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx, Y, ldy, c);
  } else if (c <= 16) {
    dim3 g(ceil_div(n, kThreads / 16), 1);
    spmm_csr_kernel<16, T><<<g, kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx, Y, ldy, c);
  } else if (c <= 32) {
    dim3 g(ceil_div(n, kThreads / 32), 1);
    spmm_csr_kernel<32, T><<<g, kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx, Y, ldy, c);
  } else {
    dim3 g(ceil_div(n, kThreads / 64), ceil_div(c, 64));
    spmm_csr_kernel<64, T><<<g, kThreads, 0, st>>>(rowptr, colind, val, n, X, ldx, Y, ldy, c);
  }
}

template void launch_spmm_csr<double>(const int32_t*, const int32_t*, const double*, int64_t, const double*, int64_t,
                                       double*, int64_t, int, hipStream_t);
template void launch_spmm_csr<float>(const int32_t*, const int32_t*, const float*, int64_t, const float*, int64_t,
                                      float*, int64_t, int, hipStream_t);

int64_t dense_mm_scratch(int64_t n) { return (int64_t)kMmMaxSplits * n * 64; }

template <typename T>
void launch_dense_mm(const T* A, int64_t lda, int64_t n, const T* X, int64_t ldx, T* Y,
                     int64_t ldy, int c, T* part, int64_t part_elems, hipStream_t st) {
  if (n <= 0 || c <= 0) return;
  const int rt = ceil_div(n, kMmRows), ct = ceil_div(c, 64);
  // split the reduction range until about 512 workgroups are in flight (two per compute unit), as far
  // as the partial products fit in part
  int64_t nz = 1;
  while (nz < kMmMaxSplits && (int64_t)rt * ct * nz < 512 && 2 * nz * n * ct * 64 <= part_elems &&
         n >= 2 * nz * kMmK)
    nz *= 2;
  const int64_t kspan = (int64_t)ceil_div(ceil_div(n, nz), kMmK) * kMmK;
  nz = ceil_div(n, kspan);
  const bool vec = ((lda | ldx) % 2 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)X % 16 == 0);
  T* P = (nz > 1) ? part : nullptr;
  dim3 g(rt, ct, (unsigned)nz);
  if (vec)
    dense_mm_kernel<true, T><<<g, kMmThreads, 0, st>>>(A, lda, n, X, ldx, Y, ldy, c, kspan, P);
  else
    dense_mm_kernel<false, T><<<g, kMmThreads, 0, st>>>(A, lda, n, X, ldx, Y, ldy, c, kspan, P);
  if (P) dense_mm_reduce_kernel<T><<<grid1(n * c), kThreads, 0, st>>>(P, (int)nz, n, c, ct * 64, Y, ldy);
}
template void launch_dense_mm<double>(const double*, int64_t, int64_t, const double*, int64_t, double*, int64_t, int,
                                      double*, int64_t, hipStream_t);
template void launch_dense_mm<float>(const float*, int64_t, int64_t, const float*, int64_t, float*, int64_t, int,
                                     float*, int64_t, hipStream_t);

void launch_herm_expand(const double* X, int64_t n, int m, double* Y, hipStream_t st) {
  if (n <= 0 || m <= 0) return;
  herm_expand_kernel<<<grid1(n * m), kThreads, 0, st>>>(X, n, m, Y);
}

void launch_herm_extract(const double* Z, const double* theta, int64_t n, int k, double* X, double* lam,
                         hipStream_t st) {
  if (n <= 0 || k <= 0) return;
  herm_extract_kernel<<<grid1(std::max<int64_t>(n * k, k)), kThreads, 0, st>>>(Z, theta, n, k, X, lam);
}

void launch_herm_orthonormalize(double* X, int64_t n, int k, const double* R, double* L, hipStream_t st) {
  if (n <= 0 || k <= 0 || k > 32) return;
  herm_chol_kernel<<<1, 64, 0, st>>>(R, k, L);
  herm_rowsolve_kernel<<<grid1(n), kThreads, 0, st>>>(X, n, k, L);
}

template <typename Tin, typename Tout>
void launch_convert_block(const Tin* src, int64_t lds, Tout* dst, int64_t ldd, int64_t n, int c, hipStream_t st) {
  if (n <= 0 || c <= 0) return;
  convert_block_kernel<Tin, Tout><<<grid1(n * c), kThreads, 0, st>>>(src, lds, dst, ldd, n, c);
}
template void launch_convert_block<double, float>(const double*, int64_t, float*, int64_t, int64_t, int, hipStream_t);
template void launch_convert_block<float, double>(const float*, int64_t, double*, int64_t, int64_t, int, hipStream_t);
template void launch_convert_block<float, float>(const float*, int64_t, float*, int64_t, int64_t, int, hipStream_t);
template void launch_convert_block<double, double>(const double*, int64_t, double*, int64_t, int64_t, int,
                                                   hipStream_t);

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
