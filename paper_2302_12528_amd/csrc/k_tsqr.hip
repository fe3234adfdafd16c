// Householder QR of a tall n x c block giving R only (Algorithm 2 step 1:
// the QR of lower(W) in the lower precision; the FP64 instantiation is the
// working-precision comparison).  Tall-skinny reduction tree: each workgroup
// factors a row block in LDS and emits its c x c R; the stacked R factors are
// factored again until one block remains.  All arithmetic is in T.
#include "common.hpp"

namespace lobpcg {

namespace {

constexpr int kQrThreads = 64;           // one wave per row block: barriers are a single wave's
constexpr int kQrLdsBytes = 32 * 1024;

template <typename T>
__device__ inline T wave_sum_t(T v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T, typename Tin>
__global__ void __launch_bounds__(kQrThreads) tsqr_block_kernel(const Tin* __restrict__ in, int64_t ldin,
                                                                int64_t nrows, int c, int rb, T* __restrict__ out) {
  extern __shared__ unsigned char smem_raw[];
  T* z = reinterpret_cast<T*>(smem_raw);          // rb x c, row-major, row stride ldz (odd)
  const int ldz = c + 1;
  __shared__ T wv[64];
  __shared__ T red[kQrThreads / 64];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid % 64, wid = tid / 64, nw = nt / 64;
  const int64_t r0 = (int64_t)blockIdx.x * rb;
  for (int e = tid; e < rb * c; e += nt) {
    const int i = e / c, j = e % c;
    const int64_t r = r0 + i;
    z[i * ldz + j] = (r < nrows) ? (T)in[r * ldin + j] : (T)0;
  }
  __syncthreads();
  const int kmax = (c < rb) ? c : rb;
  for (int j = 0; j < kmax; ++j) {
    T s = 0;
    for (int i = j + 1 + tid; i < rb; i += nt) s += z[i * ldz + j] * z[i * ldz + j];
    s = wave_sum_t(s);
    if (lane == 0) red[wid] = s;
    __syncthreads();
    s = 0;
    for (int q = 0; q < nw; ++q) s += red[q];
    const T alpha = z[j * ldz + j];
    T tj = 0, beta = alpha, scale = 0;
    if (s > (T)0) {
      const T xn = sqrt(alpha * alpha + s);
      beta = (alpha >= (T)0) ? -xn : xn;
      tj = (beta - alpha) / beta;
      scale = (T)1 / (alpha - beta);
    }
    __syncthreads();
    if (s > (T)0)
      for (int i = j + 1 + tid; i < rb; i += nt) z[i * ldz + j] *= scale;
    if (tid == 0) z[j * ldz + j] = beta;
    __syncthreads();
    for (int k = j + 1 + wid; k < c; k += nw) {
      T w = 0;
      for (int i = j + lane; i < rb; i += 64) w += (i == j ? (T)1 : z[i * ldz + j]) * z[i * ldz + k];
      w = wave_sum_t(w);
      if (lane == 0) wv[k] = w;
    }
    __syncthreads();
    const int wc = c - j - 1;
    if (wc > 0)
      for (int e = tid; e < (rb - j) * wc; e += nt) {
        const int i = j + e / wc, k = j + 1 + e % wc;
        const T vi = (i == j) ? (T)1 : z[i * ldz + j];
        z[i * ldz + k] -= tj * vi * wv[k];
      }
    __syncthreads();
  }
  T* R = out + (int64_t)blockIdx.x * c * c;
  for (int e = tid; e < c * c; e += nt) {
    const int i = e / c, j = e % c;
    R[e] = (j >= i && i < rb) ? z[i * ldz + j] : (T)0;
  }
}

template <typename T>
int rows_per_block(int c) {
  int rb = kQrLdsBytes / (int)((c + 1) * sizeof(T));
  if (rb > 1024) rb = 1024;
  if (rb < 2 * c) rb = 2 * c;
  return rb;
}

}  // namespace

int64_t tsqr_scratch_elems(int64_t n, int c) {
  // level-0 output of the smallest row block (FP64), two ping-pong halves
  const int rb = rows_per_block<double>(c);
  const int64_t nb = (n + rb - 1) / rb;
  return 2 * (nb * c * (int64_t)c + (int64_t)c * c);
}

template <typename T>
void launch_tsqr(const double* W, int64_t ldw, int64_t n, int c, T* scratch, T* R, hipStream_t st) {
  const int rb = rows_per_block<T>(c);
  const size_t lds = (size_t)rb * (c + 1) * sizeof(T);
  int64_t nb = (n + rb - 1) / rb;
  const int64_t half = tsqr_scratch_elems(n, c) / 2;
  T* bufs[2] = {scratch, scratch + half};
  T* dst = (nb == 1) ? R : bufs[0];
  tsqr_block_kernel<T, double><<<(unsigned)nb, kQrThreads, lds, st>>>(W, ldw, n, c, rb, dst);
  int cur = 0;
  while (nb > 1) {
    const int64_t rows = nb * c;
    const int64_t nb2 = (rows + rb - 1) / rb;
    T* out = (nb2 == 1) ? R : bufs[1 - cur];
    tsqr_block_kernel<T, T><<<(unsigned)nb2, kQrThreads, lds, st>>>(bufs[cur], c, rows, c, rb, out);
    cur = 1 - cur;
    nb = nb2;
  }
}
template void launch_tsqr<float>(const double*, int64_t, int64_t, int, float*, float*, hipStream_t);
template void launch_tsqr<double>(const double*, int64_t, int64_t, int, double*, double*, hipStream_t);

}  // namespace lobpcg
