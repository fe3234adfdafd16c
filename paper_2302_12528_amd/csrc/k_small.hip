// Small dense FP64 kernels, one workgroup each:
//  * symmetric eigensolver for the c x c Rayleigh-Ritz matrix (Algorithm 3
//    line 14): tridiagonalization, bisection, inverse iteration;
//  * the Hetmaniuk-Lehoucq step (lines 15-16): V = orthonormal factor of
//    C(1:m, m+1:c)^T and G = [C(:,1:m), C(:,m+1:c) V];
//  * Algorithm 2's step 3: the Cholesky factorization of V^T V.
#include <cmath>

#include "common.hpp"

namespace lobpcg {

namespace {


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

// Symmetric eigensolver for the c x c Rayleigh-Ritz matrix, one wave per matrix:
//  1. Householder reduction to tridiagonal form T = Q^T H Q (reflectors stored
//     below the subdiagonal, as in LAPACK's sytd2);
//  2. every eigenvalue of T by bisection on Sturm counts, one lane per
//     eigenvalue (the count is backward stable, so each eigenvalue is accurate
//     to a few ulps of ||T||);
//  3. eigenvectors of T by three sweeps of inverse iteration with a pivoted
//     tridiagonal LU, one lane per eigenvector; after each sweep the vectors of
//     every cluster (a chain of eigenvalues whose consecutive gaps are below
//     1e-3 ||T||_1) are re-orthonormalised by modified Gram-Schmidt in eigenvalue
//     order, so the next sweep purifies what the orthogonalisation mixed in;
//  4. back-transformation C = Q Z, one lane per column.
// Matrices up to 96 x 96 live in LDS, larger ones in the global scratch.  With a
// single wave the barriers below only order LDS traffic between lanes.
constexpr int kSyevThreads = 64;
constexpr int kSyevLds = 96;
constexpr int kSyevMax = 192;

__global__ void __launch_bounds__(kSyevThreads) syev_kernel(const double* __restrict__ H, int64_t ldh,
                                                            int64_t hstride, int c, double* __restrict__ evals,
                                                            int64_t estride, double* __restrict__ C, int64_t cstride,
                                                            double* __restrict__ work, int64_t wstride, int* info,
                                                            const int32_t* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  H += (int64_t)blockIdx.x * hstride;
  evals += (int64_t)blockIdx.x * estride;
  C += (int64_t)blockIdx.x * cstride;
  work += (int64_t)blockIdx.x * wstride;
  __shared__ double sa[kSyevLds * (kSyevLds + 1)];
  __shared__ double sz[kSyevLds * (kSyevLds + 1)];
  __shared__ double d[kSyevMax], e[kSyevMax], e2[kSyevMax], tau[kSyevMax], v[kSyevMax], p[kSyevMax];
  __shared__ double lam[kSyevMax];
  __shared__ int cstart[kSyevMax], cend[kSyevMax];
  const int lane = threadIdx.x;
  const int la = c + 1;
  const bool in_lds = (c <= kSyevLds);
  double* a = in_lds ? sa : work;
  double* Z = in_lds ? sz : work + (int64_t)c * la;
  double* lu = work + 2 * (int64_t)c * la;   // U0 | U1 | U2 | L | piv, each c x c, index [k * c + j]
  for (int q = lane; q < c * c; q += 64) {
    const int i = q / c, j = q % c;
    a[i * la + j] = 0.5 * (H[(int64_t)i * ldh + j] + H[(int64_t)j * ldh + i]);
  }
  __syncthreads();
  // ---- 1. tridiagonalization ----
  for (int k = 0; k + 2 < c; ++k) {
    const int nk = c - k - 1;
    double ss = 0.0;
    for (int i = k + 2 + lane; i < c; i += 64) ss += a[i * la + k] * a[i * la + k];
    ss = wave_sum(ss);
    const double alpha = a[(k + 1) * la + k];
    double t = 0.0, beta = alpha, scale = 0.0;
    if (ss > 0.0) {
      const double xn = sqrt(alpha * alpha + ss);
      beta = (alpha >= 0.0) ? -xn : xn;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    if (lane == 0) {
      tau[k] = t;
      e[k] = beta;
      d[k] = a[k * la + k];
    }
    if (t == 0.0) continue;   // uniform
    __syncthreads();
    for (int i = lane; i < nk; i += 64) {
      const double vi = (i == 0) ? 1.0 : a[(k + 1 + i) * la + k] * scale;
      v[i] = vi;
      if (i > 0) a[(k + 1 + i) * la + k] = vi;
    }
    if (lane == 0) a[(k + 1) * la + k] = beta;
    __syncthreads();
    // p = t A22 v, by columns of the symmetric A22 (lane i reads row j's entry i: contiguous)
    for (int i = lane; i < nk; i += 64) {
      double s = 0.0;
      for (int j = 0; j < nk; ++j) s += a[(k + 1 + j) * la + k + 1 + i] * v[j];
      p[i] = t * s;
    }
    double pv = 0.0;
    for (int i = lane; i < nk; i += 64) pv += p[i] * v[i];
    const double K = 0.5 * t * wave_sum(pv);
    for (int i = lane; i < nk; i += 64) p[i] -= K * v[i];
    __syncthreads();
    for (int q = lane; q < nk * nk; q += 64) {
      const int i = q / nk, j = q % nk;
      a[(k + 1 + i) * la + k + 1 + j] -= v[i] * p[j] + p[i] * v[j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (lane == 0) {
    for (int k = (c >= 2 ? c - 2 : 0); k < c; ++k) d[k] = a[k * la + k];
    if (c >= 2) e[c - 2] = a[(c - 1) * la + c - 2];
    if (c >= 2) tau[c - 2] = 0.0;
    tau[c - 1] = 0.0;
    e[c - 1] = 0.0;
  }
  __syncthreads();
  // ---- 2. eigenvalues by bisection ----
  double gl = 1e300, gu = -1e300, tnorm = 0.0, emax2 = 0.0;
  for (int i = 0; i < c; ++i) {
    const double ei = (i < c - 1) ? fabs(e[i]) : 0.0;
    const double em = (i > 0) ? fabs(e[i - 1]) : 0.0;
    gl = fmin(gl, d[i] - ei - em);
    gu = fmax(gu, d[i] + ei + em);
    tnorm = fmax(tnorm, fabs(d[i]) + ei + em);
    emax2 = fmax(emax2, ei * ei);
  }
  for (int i = lane; i < c; i += 64) e2[i] = (i < c - 1) ? e[i] * e[i] : 0.0;
  const double eps = 2.220446049250313e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  gl -= 2.0 * eps * tnorm * c + 2.0 * pivmin;
  gu += 2.0 * eps * tnorm * c + 2.0 * pivmin;
  __syncthreads();
  for (int j = lane; j < c; j += 64) {
    double lo = gl, hi = gu;
    for (int it = 0; it < 120; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (!(hi - lo > 2.0 * eps * fmax(fabs(lo), fabs(hi)) + pivmin) || mid == lo || mid == hi) break;
      int cnt = 0;
      double q = d[0] - mid;
      if (fabs(q) < pivmin) q = -pivmin;
      cnt += (q < 0.0);
      for (int i = 1; i < c; ++i) {
        q = (d[i] - mid) - e2[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
      }
      if (cnt >= j + 1) hi = mid; else lo = mid;
    }
    lam[j] = 0.5 * (lo + hi);
  }
  __syncthreads();
  // ---- 3. eigenvectors of T by inverse iteration ----
  const double ortol = 1e-3 * tnorm;
  int maxrank = 0;
  if (lane == 0) {
    cstart[0] = 0;
    for (int j = 1; j < c; ++j) cstart[j] = (lam[j] - lam[j - 1] < ortol) ? cstart[j - 1] : j;
    cend[c - 1] = c;
    for (int j = c - 2; j >= 0; --j) cend[j] = (cstart[j + 1] == cstart[j]) ? cend[j + 1] : j + 1;
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) maxrank = max(maxrank, j - cstart[j]);
  double* U0 = lu;
  double* U1 = lu + (int64_t)c * c;
  double* U2 = lu + 2 * (int64_t)c * c;
  double* Lm = lu + 3 * (int64_t)c * c;
  double* Pv = lu + 4 * (int64_t)c * c;
  const double tiny = eps * tnorm + pivmin;
  for (int j = lane; j < c; j += 64) {
    const double lj = lam[j];
    // pivoted LU of T - lj I (U with two superdiagonals)
    double cd = d[0] - lj, cs = (c > 1) ? e[0] : 0.0;
    for (int k = 0; k + 1 < c; ++k) {
      const double sub = e[k];
      const double nd = d[k + 1] - lj;
      const double ns = (k + 2 < c) ? e[k + 1] : 0.0;
      if (fabs(cd) >= fabs(sub)) {
        const double m = (cd != 0.0) ? sub / cd : 0.0;
        U0[k * c + j] = cd; U1[k * c + j] = cs; U2[k * c + j] = 0.0; Pv[k * c + j] = 0.0; Lm[k * c + j] = m;
        cd = nd - m * cs;
        cs = ns;
      } else {
        const double m = cd / sub;
        U0[k * c + j] = sub; U1[k * c + j] = nd; U2[k * c + j] = ns; Pv[k * c + j] = 1.0; Lm[k * c + j] = m;
        cd = cs - m * nd;
        cs = -m * ns;
      }
    }
    U0[(c - 1) * c + j] = cd;
    for (int k = 0; k < c; ++k)
      if (fabs(U0[k * c + j]) < tiny) U0[k * c + j] = (U0[k * c + j] < 0.0) ? -tiny : tiny;
    for (int i = 0; i < c; ++i) Z[i * la + j] = 1.0 + 0.25 * (double)((i * 7 + j * 13) % 11) / 11.0;
  }
  for (int itn = 0; itn < 3; ++itn) {
    // one inverse-iteration step per column (lane j owns column j), then normalise
    for (int j = lane; j < c; j += 64) {
      for (int k = 0; k + 1 < c; ++k) {
        if (Pv[k * c + j] != 0.0) {
          const double t0 = Z[k * la + j];
          Z[k * la + j] = Z[(k + 1) * la + j];
          Z[(k + 1) * la + j] = t0;
        }
        Z[(k + 1) * la + j] -= Lm[k * c + j] * Z[k * la + j];
      }
      double nrm = 0.0;
      for (int k = c - 1; k >= 0; --k) {
        double y = Z[k * la + j];
        if (k + 1 < c) y -= U1[k * c + j] * Z[(k + 1) * la + j];
        if (k + 2 < c) y -= U2[k * c + j] * Z[(k + 2) * la + j];
        y /= U0[k * c + j];
        Z[k * la + j] = y;
        nrm += y * y;
      }
      nrm = 1.0 / sqrt(nrm);
      for (int i = 0; i < c; ++i) Z[i * la + j] *= nrm;
    }
    __syncthreads();
    // modified Gram-Schmidt inside each cluster, in eigenvalue order
    for (int q = 0; q + 1 < c; ++q) {
      const int qe = cend[q];
      if (qe - q < 2) continue;   // uniform: no later member of q's cluster
      for (int r = q + 1 + lane; r < qe; r += 64) {
        double dot = 0.0;
        for (int i = 0; i < c; ++i) dot += Z[i * la + q] * Z[i * la + r];
        for (int i = 0; i < c; ++i) Z[i * la + r] -= dot * Z[i * la + q];
      }
      __syncthreads();
      double nn = 0.0;
      for (int i = lane; i < c; i += 64) nn += Z[i * la + q + 1] * Z[i * la + q + 1];
      nn = 1.0 / sqrt(wave_sum(nn));
      for (int i = lane; i < c; i += 64) Z[i * la + q + 1] *= nn;
      __syncthreads();
    }
  }
  // ---- 4. back-transformation C = Q Z (lane j owns column j) ----
  for (int k = c - 3; k >= 0; --k) {
    const double t = tau[k];
    if (t == 0.0) continue;
    const int nk = c - k - 1;
    for (int j = lane; j < c; j += 64) {
      double sw = Z[(k + 1) * la + j];
      for (int i = 1; i < nk; ++i) sw += a[(k + 1 + i) * la + k] * Z[(k + 1 + i) * la + j];
      sw *= t;
      Z[(k + 1) * la + j] -= sw;
      for (int i = 1; i < nk; ++i) Z[(k + 1 + i) * la + j] -= a[(k + 1 + i) * la + k] * sw;
    }
  }
  __syncthreads();
  for (int q = lane; q < c * c; q += 64) {
    const int i = q / c, j = q % c;
    C[(int64_t)i * c + j] = Z[i * la + j];
  }
  for (int j = lane; j < c; j += 64) evals[j] = lam[j];
  if (lane == 0 && info) info[blockIdx.x] = maxrank;
}

// HL: Z = C(0:m, m:c)^T (r x m, r = c - m); Householder QR; Q explicit; G = [C(:,0:m), C(:,m:c) Q].
// One wave per matrix; in the QR and in forming Q each lane owns columns of Z or Q, so the only
// cross-lane traffic is the reflector vector (one barrier before and one after it is formed).
constexpr int kHlThreads = 64;
constexpr int kHlMaxR = 128;
constexpr int kHlMaxM = 64;

__global__ void __launch_bounds__(kHlThreads) hl_build_kernel(const double* __restrict__ C, int64_t cstride, int c,
                                                              int m, double* __restrict__ G, int64_t gstride,
                                                              const int32_t* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  C += (int64_t)blockIdx.x * cstride;
  G += (int64_t)blockIdx.x * gstride;
  __shared__ double z[kHlMaxR * (kHlMaxM + 1)];
  __shared__ double qm[kHlMaxR * (kHlMaxM + 1)];
  __shared__ double tau[kHlMaxM];
  const int lane = threadIdx.x;
  const int r = c - m;
  const int lz = m + 1;   // odd LDS row stride
  const int ldg = (r > 0) ? 2 * m : m;
  // copy C(:, 0:m)
  for (int e = lane; e < c * m; e += 64) {
    const int i = e / m, j = e % m;
    G[(int64_t)i * ldg + j] = C[(int64_t)i * c + j];
  }
  if (r <= 0) return;
  for (int e = lane; e < r * m; e += 64) {
    const int i = e / m, j = e % m;
    z[i * lz + j] = C[(int64_t)j * c + m + i];
    qm[i * lz + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int kmax = (m < r) ? m : r;
  for (int j = 0; j < kmax; ++j) {
    double s = 0.0;
    for (int i = j + 1 + lane; i < r; i += 64) s += z[i * lz + j] * z[i * lz + j];
    s = wave_sum(s);
    const double alpha = z[j * lz + j];
    double tj = 0.0, beta = alpha, scale = 0.0;
    if (s > 0.0) {
      const double xn = sqrt(alpha * alpha + s);
      beta = (alpha >= 0.0) ? -xn : xn;
      tj = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();   // every lane has read column j before it is overwritten by v
    if (s > 0.0)
      for (int i = j + 1 + lane; i < r; i += 64) z[i * lz + j] *= scale;
    if (lane == 0) {
      tau[j] = tj;
      z[j * lz + j] = beta;
    }
    __syncthreads();
    // apply H_j = I - tau v v^T (v_j = 1) to columns k > j; lane owns column k
    if (tj != 0.0)
      for (int k = j + 1 + lane; k < m; k += 64) {
        double w = z[j * lz + k];
        for (int i = j + 1; i < r; ++i) w += z[i * lz + j] * z[i * lz + k];
        w *= tj;
        z[j * lz + k] -= w;
        for (int i = j + 1; i < r; ++i) z[i * lz + k] -= z[i * lz + j] * w;
      }
    __syncthreads();
  }
  // Q = H_0 ... H_{kmax-1} [I; 0], lane owns column k of Q
  for (int j = kmax - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    for (int k = lane; k < m; k += 64) {
      double w = qm[j * lz + k];
      for (int i = j + 1; i < r; ++i) w += z[i * lz + j] * qm[i * lz + k];
      w *= tj;
      qm[j * lz + k] -= w;
      for (int i = j + 1; i < r; ++i) qm[i * lz + k] -= z[i * lz + j] * w;
    }
  }
  __syncthreads();
  // G(:, m:2m) = C(:, m:c) Q
  for (int e = lane; e < c * m; e += 64) {
    const int i = e / m, j = e % m;
    double acc = 0.0;
    for (int k = 0; k < r; ++k) acc += C[(int64_t)i * c + m + k] * qm[k * lz + j];
    G[(int64_t)i * ldg + m + j] = acc;
  }
}

// Algorithm 2 step 3: V^T V = L L^T (FP64).  Writes Lt = L^T (upper, row-major) for
// the step-4 solve, and Rout = L^T working(Rl) (the R factor) when requested.
// Flags a non-positive or non-finite pivot (W numerically rank deficient).
template <typename T>
__global__ void __launch_bounds__(256) chol_upper_kernel(const double* __restrict__ G, const T* __restrict__ Rl,
                                                         int c, double* __restrict__ Lt, double* __restrict__ Rout,
                                                         int* flag, const int32_t* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  const int64_t off = (int64_t)blockIdx.x * c * c;
  G += off;
  Rl += off;
  Lt += off;
  if (Rout) Rout += off;
  flag += blockIdx.x;
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

int64_t syev_scratch(int c) { return 2 * (int64_t)c * (c + 1) + 5 * (int64_t)c * c + 16; }

void launch_syev(const double* H, int64_t ldh, int64_t hstride, int c, double* evals, int64_t estride, double* C,
                 int64_t cstride, double* work, int* info, const int32_t* active, int B, hipStream_t st) {
  syev_kernel<<<B, kSyevThreads, 0, st>>>(H, ldh, hstride, c, evals, estride, C, cstride, work, syev_scratch(c),
                                          info, active);
}

void launch_hl_build(const double* C, int64_t cstride, int c, int m, double* G, int64_t gstride,
                     const int32_t* active, int B, hipStream_t st) {
  hl_build_kernel<<<B, kHlThreads, 0, st>>>(C, cstride, c, m, G, gstride, active);
}

template <typename T>
void launch_chol_upper(const double* G, const T* Rl, int c, double* Lt, double* Rout, int* flag,
                       const int32_t* active, int B, hipStream_t st) {
  chol_upper_kernel<T><<<B, 256, 0, st>>>(G, Rl, c, Lt, Rout, flag, active);
}
template void launch_chol_upper<float>(const double*, const float*, int, double*, double*, int*, const int32_t*, int,
                                       hipStream_t);
template void launch_chol_upper<double>(const double*, const double*, int, double*, double*, int*, const int32_t*,
                                        int, hipStream_t);

}  // namespace lobpcg
