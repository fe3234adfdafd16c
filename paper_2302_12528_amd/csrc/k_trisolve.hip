// Preconditioner application W_l = L^{-T} L^{-1} lower(R) in the factor's
// precision T (Algorithm 3 lines 9-10; section 5.1's two triangular solves),
// over the supernodal elimination tree, one launch per level and direction.
//
// After factorization each supernode's panel holds P_s = [inv(L11); L21 inv(L11)]
// (nr x nc, column-major), so with b_s the right-hand side at its own rows
//   forward:  [y_s; d] = P_s b_s,  y_s = inv(L11) b_s, and d = L21 y_s is
//             subtracted from the rows below (passed up the tree in a
//             per-supernode update vector, pulled by the parent; no atomics);
//   backward: x_s = P_s^T [y_s; -x_below] = inv(L11)^T (y_s - L21^T x_below).
// Right-hand sides are n x M row-major blocks (M = padded block size) in the
// permuted ordering; tiles of 64 rows of P_s are streamed through LDS with the
// matching rows of the right-hand side.
#include "common.hpp"

namespace lobpcg {

namespace {

constexpr int RT_ROWS = 64;
constexpr int KC = 32;

template <int M> struct Shape;
template <> struct Shape<8>  { static constexpr int RT = 2, CT = 1; };
template <> struct Shape<16> { static constexpr int RT = 2, CT = 2; };
template <> struct Shape<32> { static constexpr int RT = 4, CT = 2; };
template <> struct Shape<64> { static constexpr int RT = 4, CT = 4; };

template <typename T>
__global__ void __launch_bounds__(256) fwd_assemble_kernel(FactorDev D, int64_t item_off, int64_t count, T* rhs,
                                                           const T* __restrict__ uvec, int M) {
  const int lane = threadIdx.x % 64;
  const int64_t item = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (item >= count || lane >= M) return;
  const int s = D.ownrow_items[2 * (item_off + item)];
  const int r = D.ownrow_items[2 * (item_off + item) + 1];
  T v = rhs[(int64_t)(D.begin[s] + r) * M + lane];
  for (int q = D.child_ptr[s]; q < D.child_ptr[s + 1]; ++q) {
    const int c = D.child_list[q];
    const int jr = D.invmap[D.inv_off[c] + r];
    if (jr >= 0) v += uvec[(D.uvec_off[c] + jr) * M + lane];
  }
  rhs[(int64_t)(D.begin[s] + r) * M + lane] = v;
}

template <typename T, int M>
__global__ void __launch_bounds__(256) fwd_gemm_kernel(FactorDev D, int64_t item_off, const T* __restrict__ panel,
                                                       const T* __restrict__ rhs, T* __restrict__ y,
                                                       T* __restrict__ uvec) {
  constexpr int RT = Shape<M>::RT, CT = Shape<M>::CT;
  constexpr int NCG = M / CT, NRG = RT_ROWS / RT;
  static_assert(NCG * NRG == 256, "thread layout");
  __shared__ T Ps[KC][RT_ROWS + 1];
  __shared__ T Bs[KC][M];
  const int tid = threadIdx.x;
  const int s = D.fwd_items[2 * (item_off + blockIdx.x)];
  const int tile = D.fwd_items[2 * (item_off + blockIdx.x) + 1];
  const int begin = D.begin[s], nc = D.nc[s], nr = D.nr[s];
  const int64_t poff = D.panel_off[s];
  const int r0 = tile * RT_ROWS;
  const int h = min(RT_ROWS, nr - r0);
  const int kmax = (r0 < nc) ? min(nc, r0 + RT_ROWS) : nc;
  const int cg = tid % NCG, rg = tid / NCG;
  T acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = 0;
  for (int k0 = 0; k0 < kmax; k0 += KC) {
    for (int e = tid; e < KC * RT_ROWS; e += 256) {
      const int r = e % RT_ROWS, kk = e / RT_ROWS;
      Ps[kk][r] = (r < h && k0 + kk < kmax) ? panel[poff + (int64_t)(k0 + kk) * nr + r0 + r] : (T)0;
    }
    for (int e = tid; e < KC * M; e += 256) {
      const int kk = e / M, j = e % M;
      Bs[kk][j] = (k0 + kk < kmax) ? rhs[(int64_t)(begin + k0 + kk) * M + j] : (T)0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < KC; ++k) {
      T a[RT], b[CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i] = Ps[k][rg + NRG * i];
#pragma unroll
      for (int j = 0; j < CT; ++j) b[j] = Bs[k][cg * CT + j];
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  const int c0 = D.child_ptr[s], c1 = D.child_ptr[s + 1];
  const int64_t uoff = D.uvec_off[s];
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    const int row = r0 + rg + NRG * i;
    if (row >= r0 + h) continue;
    if (row < nc) {
#pragma unroll
      for (int j = 0; j < CT; ++j) y[(int64_t)(begin + row) * M + cg * CT + j] = acc[i][j];
    } else {
      T pass[CT];
#pragma unroll
      for (int j = 0; j < CT; ++j) pass[j] = 0;
      for (int q = c0; q < c1; ++q) {
        const int c = D.child_list[q];
        const int jr = D.invmap[D.inv_off[c] + row];
        if (jr >= 0)
#pragma unroll
          for (int j = 0; j < CT; ++j) pass[j] += uvec[(D.uvec_off[c] + jr) * M + cg * CT + j];
      }
#pragma unroll
      for (int j = 0; j < CT; ++j) uvec[(uoff + row - nc) * M + cg * CT + j] = pass[j] - acc[i][j];
    }
  }
}

template <typename T, int M>
__global__ void __launch_bounds__(256) bwd_gemm_kernel(FactorDev D, int64_t item_off, const T* __restrict__ panel,
                                                       const T* __restrict__ y, T* __restrict__ x, double* W,
                                                       int64_t ldw, int mw) {
  constexpr int RT = Shape<M>::RT, CT = Shape<M>::CT;
  constexpr int NCG = M / CT, NRG = RT_ROWS / RT;
  __shared__ T Ps[KC][RT_ROWS + 1];
  __shared__ T Zs[KC][M];
  const int tid = threadIdx.x;
  const int s = D.bwd_items[2 * (item_off + blockIdx.x)];
  const int tile = D.bwd_items[2 * (item_off + blockIdx.x) + 1];
  const int begin = D.begin[s], nc = D.nc[s], nr = D.nr[s];
  const int64_t poff = D.panel_off[s];
  const int64_t roff = D.row_off[s];
  const int j0 = tile * RT_ROWS;
  const int h = min(RT_ROWS, nc - j0);
  const int cg = tid % NCG, rg = tid / NCG;
  T acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = 0;
  for (int k0 = j0; k0 < nr; k0 += KC) {
    for (int e = tid; e < KC * RT_ROWS; e += 256) {
      const int kk = e % KC, jj = e / KC;
      Ps[kk][jj] = (jj < h && k0 + kk < nr) ? panel[poff + (int64_t)(j0 + jj) * nr + k0 + kk] : (T)0;
    }
    for (int e = tid; e < KC * M; e += 256) {
      const int kk = e / M, j = e % M;
      const int r = k0 + kk;
      T v = 0;
      if (r < nc)
        v = y[(int64_t)(begin + r) * M + j];
      else if (r < nr)
        v = -x[(int64_t)D.rows[roff + r] * M + j];
      Zs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < KC; ++k) {
      T a[RT], b[CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i] = Ps[k][rg + NRG * i];
#pragma unroll
      for (int j = 0; j < CT; ++j) b[j] = Zs[k][cg * CT + j];
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RT; ++i) {
    const int jj = rg + NRG * i;
    if (jj >= h) continue;
    const int64_t row = begin + j0 + jj;
#pragma unroll
    for (int j = 0; j < CT; ++j) {
      const int col = cg * CT + j;
      x[row * M + col] = acc[i][j];
      if (W && col < mw) W[row * ldw + col] = (double)acc[i][j];
    }
  }
}

template <typename T>
__global__ void cast_to_kernel(const double* __restrict__ src, int64_t lds, T* __restrict__ dst, int64_t n, int m,
                               int M) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * M) return;
  const int64_t i = e / M;
  const int j = (int)(e % M);
  dst[e] = (j < m) ? (T)src[i * lds + j] : (T)0;
}

}  // namespace

template <typename T>
void launch_fwd_assemble(const FactorDev& D, int64_t item_off, int64_t count, T* rhs, const T* uvec, int M,
                         hipStream_t st) {
  if (count <= 0) return;
  fwd_assemble_kernel<T><<<(unsigned)((count + 3) / 4), 256, 0, st>>>(D, item_off, count, rhs, uvec, M);
}

template <typename T>
void launch_fwd_gemm(const FactorDev& D, int64_t item_off, int64_t count, const T* panel, const T* rhs, T* y,
                     T* uvec, int M, hipStream_t st) {
  if (count <= 0) return;
  switch (M) {
    case 8: fwd_gemm_kernel<T, 8><<<(unsigned)count, 256, 0, st>>>(D, item_off, panel, rhs, y, uvec); break;
    case 16: fwd_gemm_kernel<T, 16><<<(unsigned)count, 256, 0, st>>>(D, item_off, panel, rhs, y, uvec); break;
    case 32: fwd_gemm_kernel<T, 32><<<(unsigned)count, 256, 0, st>>>(D, item_off, panel, rhs, y, uvec); break;
    default: fwd_gemm_kernel<T, 64><<<(unsigned)count, 256, 0, st>>>(D, item_off, panel, rhs, y, uvec); break;
  }
}

template <typename T>
void launch_bwd_gemm(const FactorDev& D, int64_t item_off, int64_t count, const T* panel, const T* y, T* x,
                     double* W, int64_t ldw, int m, hipStream_t st) {
  if (count <= 0) return;
  int M = m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : 64;
  switch (M) {
    case 8: bwd_gemm_kernel<T, 8><<<(unsigned)count, 256, 0, st>>>(D, item_off, panel, y, x, W, ldw, m); break;
    case 16: bwd_gemm_kernel<T, 16><<<(unsigned)count, 256, 0, st>>>(D, item_off, panel, y, x, W, ldw, m); break;
    case 32: bwd_gemm_kernel<T, 32><<<(unsigned)count, 256, 0, st>>>(D, item_off, panel, y, x, W, ldw, m); break;
    default: bwd_gemm_kernel<T, 64><<<(unsigned)count, 256, 0, st>>>(D, item_off, panel, y, x, W, ldw, m); break;
  }
}

template <typename T>
void launch_cast_to(const double* src, int64_t lds, T* dst, int64_t n, int m, hipStream_t st) {
  const int M = m <= 8 ? 8 : m <= 16 ? 16 : m <= 32 ? 32 : 64;
  const int64_t total = n * M;
  if (total <= 0) return;
  cast_to_kernel<T><<<(unsigned)((total + 255) / 256), 256, 0, st>>>(src, lds, dst, n, m, M);
}

#define INST(T)                                                                                                  \
  template void launch_fwd_assemble<T>(const FactorDev&, int64_t, int64_t, T*, const T*, int, hipStream_t);     \
  template void launch_fwd_gemm<T>(const FactorDev&, int64_t, int64_t, const T*, const T*, T*, T*, int,         \
                                   hipStream_t);                                                                \
  template void launch_bwd_gemm<T>(const FactorDev&, int64_t, int64_t, const T*, const T*, T*, double*, int64_t, \
                                   int, hipStream_t);                                                           \
  template void launch_cast_to<T>(const double*, int64_t, T*, int64_t, int, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace lobpcg
