// Small dense FP64 kernels, one workgroup each:
//  * symmetric eigensolver for the c x c Rayleigh-Ritz matrix (Algorithm 3
//    line 14), by parallel cyclic Jacobi (round-robin pairing, so the N/2
//    rotations of a round are disjoint and applied together as J^T A J);
//  * the Hetmaniuk-Lehoucq step (lines 15-16): V = orthonormal factor of
//    C(1:m, m+1:c)^T and G = [C(:,1:m), C(:,m+1:c) V];
//  * Algorithm 2's steps 2-4: row-wise triangular solves with the lower-precision
//    R factor and with L^T, and the Cholesky factorization of V^T V.
#include <cmath>

#include "common.hpp"

namespace lobpcg {

namespace {

constexpr int kEigThreads = 1024;
constexpr int kLdsMax = 96;   // matrices up to 96 x 96 stay in LDS

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum over all threads of the block; red must hold blockDim/64 doubles.
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int nw = blockDim.x / 64;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int q = 0; q < nw; ++q) s += red[q];
  __syncthreads();
  return s;
}

// Round-robin (circle method) pairing of N (even) indices for round r.
__device__ inline void rr_pair(int r, int i, int N, int& p, int& q) {
  if (i == 0) {
    p = r;
    q = N - 1;
  } else {
    const int M = N - 1;
    p = (r + i) % M;
    q = (r - i + M) % M;
  }
  if (p > q) { int t = p; p = q; q = t; }
}

__device__ void jacobi_core(double* a, double* v, int c, int N, double* cs, double* sn, int* pp, int* qq,
                            double* red, int* info) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int half = N / 2;
  double fro2 = 0.0;
  for (int e = tid; e < N * N; e += nt) fro2 += a[e] * a[e];
  fro2 = block_sum(fro2, red);
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int e = tid; e < N * N; e += nt) {
      const int i = e / N, j = e % N;
      if (i != j) off += a[e] * a[e];
    }
    off = block_sum(off, red);
    if (!(off > 1e-32 * fro2)) break;
    for (int r = 0; r < N - 1; ++r) {
      if (tid < half) {
        int p, q;
        rr_pair(r, tid, N, p, q);
        const double apq = a[p * N + q];
        double c = 1.0, s = 0.0;
        if (apq != 0.0) {
          const double th = (a[q * N + q] - a[p * N + p]) / (2.0 * apq);
          const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          c = 1.0 / sqrt(1.0 + t * t);
          s = t * c;
        }
        pp[tid] = p; qq[tid] = q; cs[tid] = c; sn[tid] = s;
      }
      __syncthreads();
      for (int e = tid; e < half * half; e += nt) {
        const int bi = e / half, bj = e % half;
        const int pi = pp[bi], qi = qq[bi], pj = pp[bj], qj = qq[bj];
        const double ci = cs[bi], si = sn[bi], cj = cs[bj], sj = sn[bj];
        const double b00 = a[pi * N + pj], b01 = a[pi * N + qj];
        const double b10 = a[qi * N + pj], b11 = a[qi * N + qj];
        // rows: J_i^T B
        const double t00 = ci * b00 - si * b10, t01 = ci * b01 - si * b11;
        const double t10 = si * b00 + ci * b10, t11 = si * b01 + ci * b11;
        // columns: (J_i^T B) J_j
        double n00 = cj * t00 - sj * t01, n01 = sj * t00 + cj * t01;
        double n10 = cj * t10 - sj * t11, n11 = sj * t10 + cj * t11;
        if (bi == bj) { n01 = 0.0; n10 = 0.0; }
        a[pi * N + pj] = n00; a[pi * N + qj] = n01;
        a[qi * N + pj] = n10; a[qi * N + qj] = n11;
      }
      for (int e = tid; e < N * half; e += nt) {
        const int row = e / half, bi = e % half;
        const int p = pp[bi], q = qq[bi];
        const double c = cs[bi], s = sn[bi];
        const double vp = v[row * N + p], vq = v[row * N + q];
        v[row * N + p] = c * vp - s * vq;
        v[row * N + q] = s * vp + c * vq;
      }
      __syncthreads();
    }
  }
  if (tid == 0 && info) info[0] = sweep;
}

template <bool kLds>
__global__ void __launch_bounds__(kEigThreads) syev_kernel(const double* __restrict__ H, int64_t ldh, int c,
                                                           double* __restrict__ evals, double* __restrict__ C,
                                                           double* __restrict__ work, int* info) {
  __shared__ double sA[kLds ? kLdsMax * kLdsMax : 1];
  __shared__ double sV[kLds ? kLdsMax * kLdsMax : 1];
  __shared__ double cs[kLdsMax + 2], sn[kLdsMax + 2];
  __shared__ int pp[kLdsMax + 2], qq[kLdsMax + 2];
  __shared__ double red[kEigThreads / 64];
  __shared__ double dsh[2 * kLdsMax + 2];
  const int N = c + (c & 1);
  double* a = kLds ? sA : work;
  double* v = kLds ? sV : work + (int64_t)N * N;
  double* cs_ = kLds ? cs : work + 2 * (int64_t)N * N;
  double* sn_ = kLds ? sn : cs_ + N;
  int* pp_ = kLds ? pp : (int*)(sn_ + N);
  int* qq_ = kLds ? qq : pp_ + N;
  double* d = kLds ? dsh : (double*)(qq_ + N + 2);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < N * N; e += nt) {
    const int i = e / N, j = e % N;
    double x = 0.0;
    if (i < c && j < c) x = 0.5 * (H[(int64_t)i * ldh + j] + H[(int64_t)j * ldh + i]);
    a[e] = x;
    v[e] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_core(a, v, c, N, cs_, sn_, pp_, qq_, red, info);
  __syncthreads();
  for (int i = tid; i < c; i += nt) d[i] = a[i * N + i];
  __syncthreads();
  // ascending order by rank (ties broken by index)
  for (int i = tid; i < c; i += nt) {
    const double di = d[i];
    int rank = 0;
    for (int j = 0; j < c; ++j) {
      const double dj = d[j];
      rank += (dj < di || (dj == di && j < i)) ? 1 : 0;
    }
    evals[rank] = di;
    for (int row = 0; row < c; ++row) C[(int64_t)row * c + rank] = v[row * N + i];
  }
}

// HL: Z = C(0:m, m:c)^T (r x m, r = c - m); Householder QR; Q explicit; G = [C(:,0:m), C(:,m:c) Q].
constexpr int kHlThreads = 512;
constexpr int kHlMaxR = 128;
constexpr int kHlMaxM = 64;

__global__ void __launch_bounds__(kHlThreads) hl_build_kernel(const double* __restrict__ C, int c, int m,
                                                              double* __restrict__ G) {
  __shared__ double z[kHlMaxR * (kHlMaxM + 1)];
  __shared__ double qm[kHlMaxR * (kHlMaxM + 1)];
  __shared__ double tau[kHlMaxM];
  __shared__ double wv[kHlMaxM];
  __shared__ double red[kHlThreads / 64];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid % 64, wid = tid / 64, nw = nt / 64;
  const int r = c - m;
  const int lz = m + 1;   // odd LDS row stride
  const int ldg = (r > 0) ? 2 * m : m;
  // copy C(:, 0:m)
  for (int e = tid; e < c * m; e += nt) {
    const int i = e / m, j = e % m;
    G[(int64_t)i * ldg + j] = C[(int64_t)i * c + j];
  }
  if (r <= 0) return;
  for (int e = tid; e < r * m; e += nt) {
    const int i = e / m, j = e % m;
    z[i * lz + j] = C[(int64_t)j * c + m + i];
    qm[i * lz + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kmax = (m < r) ? m : r;
  for (int j = 0; j < kmax; ++j) {
    double s = 0.0;
    for (int i = j + 1 + tid; i < r; i += nt) s += z[i * lz + j] * z[i * lz + j];
    s = block_sum(s, red);
    const double alpha = z[j * lz + j];
    const double xn = sqrt(alpha * alpha + s);
    double tj = 0.0, beta = alpha, scale = 0.0;
    if (s > 0.0) {
      beta = (alpha >= 0.0) ? -xn : xn;
      tj = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();
    if (s > 0.0)
      for (int i = j + 1 + tid; i < r; i += nt) z[i * lz + j] *= scale;
    if (tid == 0) { tau[j] = tj; z[j * lz + j] = beta; }
    __syncthreads();
    // apply H_j = I - tau v v^T (v_j = 1) to columns k > j
    for (int k = j + 1 + wid; k < m; k += nw) {
      double w = 0.0;
      for (int i = j + lane; i < r; i += 64) w += (i == j ? 1.0 : z[i * lz + j]) * z[i * lz + k];
      w = wave_sum(w);
      if (lane == 0) wv[k] = w;
    }
    __syncthreads();
    for (int e = tid; e < (r - j) * (m - j - 1); e += nt) {
      const int i = j + e / (m - j - 1), k = j + 1 + e % (m - j - 1);
      const double vi = (i == j) ? 1.0 : z[i * lz + j];
      z[i * lz + k] -= tj * vi * wv[k];
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{kmax-1} [I; 0]
  for (int j = kmax - 1; j >= 0; --j) {
    const double tj = tau[j];
    for (int k = wid; k < m; k += nw) {
      double w = 0.0;
      for (int i = j + lane; i < r; i += 64) w += (i == j ? 1.0 : z[i * lz + j]) * qm[i * lz + k];
      w = wave_sum(w);
      if (lane == 0) wv[k] = w;
    }
    __syncthreads();
    for (int e = tid; e < (r - j) * m; e += nt) {
      const int i = j + e / m, k = e % m;
      const double vi = (i == j) ? 1.0 : z[i * lz + j];
      qm[i * lz + k] -= tj * vi * wv[k];
    }
    __syncthreads();
  }
  // G(:, m:2m) = C(:, m:c) Q
  for (int e = tid; e < c * m; e += nt) {
    const int i = e / m, j = e % m;
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += C[(int64_t)i * c + m + k] * qm[k * lz + j];
    G[(int64_t)i * ldg + m + j] = acc;
  }
}

// Algorithm 2 steps 2 and 4: solve Y U = X row by row (U upper triangular, c x c,
// row-major), in place, by forward substitution over the columns.  One thread
// owns one row; 64 rows per workgroup sit in LDS column-major (Ws[j*64 + t]),
// so the lanes of a wave read consecutive words, and U is broadcast from LDS.
template <typename TU>
__global__ void __launch_bounds__(64) trsm_rows_kernel(double* W, int64_t ld, int64_t n, int c,
                                                       const TU* __restrict__ U) {
  extern __shared__ double smem[];
  double* Us = smem;            // c x c
  double* Ws = smem + c * c;    // c x 64
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  for (int e = t; e < c * c; e += 64) Us[e] = (double)U[e];
  for (int e = t; e < 64 * c; e += 64) {
    const int i = e / c, j = e % c;
    Ws[j * 64 + i] = (r0 + i < n) ? W[(r0 + i) * ld + j] : 0.0;
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    double s = Ws[j * 64 + t];
#pragma unroll 4
    for (int i = 0; i < j; ++i) s -= Ws[i * 64 + t] * Us[i * c + j];
    Ws[j * 64 + t] = s / Us[j * c + j];
  }
  __syncthreads();
  for (int e = t; e < 64 * c; e += 64) {
    const int i = e / c, j = e % c;
    if (r0 + i < n) W[(r0 + i) * ld + j] = Ws[j * 64 + i];
  }
}

// Algorithm 2 step 3: V^T V = L L^T (FP64).  Writes Lt = L^T (upper, row-major) for
// the step-4 solve, and Rout = L^T working(Rl) (the R factor) when requested.
// Flags a non-positive or non-finite pivot (W numerically rank deficient).
template <typename T>
__global__ void __launch_bounds__(256) chol_upper_kernel(const double* __restrict__ G, const T* __restrict__ Rl,
                                                         int c, double* __restrict__ Lt, double* __restrict__ Rout,
                                                         int* flag) {
  __shared__ double L[64 * 64];
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int e = tid; e < c * c; e += nt) {
    const int i = e / c, j = e % c;
    L[e] = 0.5 * (G[i * c + j] + G[j * c + i]);
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    if (tid == 0) {
      double d = L[j * c + j];
      if (!(d > 0.0) || !isfinite(d)) { flag[0] = 1; d = 1.0; }
      L[j * c + j] = sqrt(d);
    }
    __syncthreads();
    const double ljj = L[j * c + j];
    for (int i = j + 1 + tid; i < c; i += nt) L[i * c + j] /= ljj;
    __syncthreads();
    const int w = c - j - 1;
    for (int e = tid; e < w * w; e += nt) {
      const int i = j + 1 + e / w, k = j + 1 + e % w;
      if (k <= i) L[i * c + k] -= L[i * c + j] * L[k * c + j];
    }
    __syncthreads();
  }
  for (int e = tid; e < c * c; e += nt) {
    const int i = e / c, j = e % c;
    Lt[e] = (j >= i) ? L[j * c + i] : 0.0;
  }
  if (Rout) {
    for (int e = tid; e < c * c; e += nt) {
      const int i = e / c, j = e % c;
      double s = 0.0;
      for (int k = i; k < c; ++k) s += L[k * c + i] * (double)Rl[k * c + j];
      Rout[e] = s;
    }
  }
}

}  // namespace

int64_t syev_scratch(int c) {
  const int64_t N = c + (c & 1);
  return 2 * N * N + 6 * N + 16;
}

void launch_syev(const double* H, int64_t ldh, int c, double* evals, double* C, double* work, int* info,
                 hipStream_t st) {
  if (c <= kLdsMax)
    syev_kernel<true><<<1, kEigThreads, 0, st>>>(H, ldh, c, evals, C, work, info);
  else
    syev_kernel<false><<<1, kEigThreads, 0, st>>>(H, ldh, c, evals, C, work, info);
}

void launch_hl_build(const double* C, int c, int m, double* G, double* work, hipStream_t st) {
  (void)work;
  hl_build_kernel<<<1, kHlThreads, 0, st>>>(C, c, m, G);
}

template <typename TU>
void launch_trsm_rows(double* W, int64_t ld, int64_t n, int c, const TU* U, hipStream_t st) {
  if (n <= 0) return;
  const size_t lds = (size_t)(c * c + 64 * c) * sizeof(double);
  trsm_rows_kernel<TU><<<(unsigned)((n + 63) / 64), 64, lds, st>>>(W, ld, n, c, U);
}
template void launch_trsm_rows<float>(double*, int64_t, int64_t, int, const float*, hipStream_t);
template void launch_trsm_rows<double>(double*, int64_t, int64_t, int, const double*, hipStream_t);

template <typename T>
void launch_chol_upper(const double* G, const T* Rl, int c, double* Lt, double* Rout, int* flag, hipStream_t st) {
  chol_upper_kernel<T><<<1, 256, 0, st>>>(G, Rl, c, Lt, Rout, flag);
}
template void launch_chol_upper<float>(const double*, const float*, int, double*, double*, int*, hipStream_t);
template void launch_chol_upper<double>(const double*, const double*, int, double*, double*, int*, hipStream_t);

}  // namespace lobpcg
