// Numeric supernodal (multifrontal) Cholesky factorization Pi^T A Pi = L L^T in
// precision T (FP32: the lower-precision factor of section 5.1, computed from
// lower(A); FP64: the working-precision comparison), followed by the partial
// inversion that the triangular solves use.
//
// Each supernode s owns a dense front: rows = its nc own columns followed by
// its nb below rows.  The first nc columns live in the panel (nr x nc,
// column-major), the trailing nb x nb Schur complement U_s in its own buffer.
// Levels of the supernodal elimination tree are processed bottom-up; inside a
// level every supernode is independent.  Per level:
//   assemble  front(:, t) = A(:, t) + sum over children of their U, pulled by
//             target row (no atomics, deterministic);
//   for each 64-column panel p: potrf of tile (p,p) and its inverse, trsm of
//             the tiles below it, symmetric update of the trailing tiles;
//   inverse   panel <- [I; L21] inv(L11) = [inv(L11); L21 inv(L11)], so that
//             each solve is one product per supernode (see k_trisolve.hip).
#include "common.hpp"
#include "symbolic.hpp"

namespace lobpcg {

namespace {

constexpr int TB = kTile;

struct Sn {
  int begin, nc, nr, nb, np;
  int64_t panel, upd;
};

__device__ inline Sn sn_of(const FactorDev& D, int s) {
  Sn S;
  S.begin = D.begin[s];
  S.nc = D.nc[s];
  S.nr = D.nr[s];
  S.nb = S.nr - S.nc;
  S.np = (S.nc + TB - 1) / TB;
  S.panel = D.panel_off[s];
  S.upd = D.upd_off[s];
  return S;
}

__device__ inline void tile_rows(const Sn& S, int I, int& r0, int& h) {
  if (I < S.np) {
    r0 = I * TB;
    h = min(TB, S.nc - r0);
  } else {
    r0 = S.nc + (I - S.np) * TB;
    h = min(TB, S.nr - r0);
  }
}

// Pointer to front element (r, c) (c < nc: panel; else U with r >= nc) and its leading dimension.
template <typename T>
__device__ inline T* front_ptr(T* panel, T* upd, const Sn& S, int r, int c, int64_t& ld) {
  if (c < S.nc) {
    ld = S.nr;
    return panel + S.panel + (int64_t)c * S.nr + r;
  }
  ld = S.nb;
  return upd + S.upd + (int64_t)(c - S.nc) * S.nb + (r - S.nc);
}

// ---------------------------------------------------------------------------
// Assembly, one wave per front column.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) assemble_kernel(FactorDev D, int64_t item_off, int64_t count, T* panel,
                                                       T* upd) {
  const int lane = threadIdx.x % 64;
  const int64_t item = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (item >= count) return;
  const int s = D.asm_items[2 * (item_off + item)];
  const int t = D.asm_items[2 * (item_off + item) + 1];
  const Sn S = sn_of(D, s);
  const int c0 = D.child_ptr[s], c1 = D.child_ptr[s + 1];
  const int rlo = (t < S.nc) ? 0 : t;
  int64_t ld;
  T* col = front_ptr(panel, upd, S, (t < S.nc) ? 0 : t, t, ld);
  const int64_t colbase = (t < S.nc) ? 0 : t;   // row index of col[0]
  if (D.is_dense) {
    for (int r = rlo + lane; r < S.nr; r += 64)
      col[r - colbase] = (r >= t) ? (T)D.dense[(int64_t)r * D.ld_dense + t] : (T)0;
    return;
  }
  const int j = S.begin + t;
  const int e0 = (t < S.nc) ? D.prow[j] : 0;
  const int e1 = (t < S.nc) ? D.prow[j + 1] : 0;
  for (int r = rlo + lane; r < S.nr; r += 64) {
    T v = 0;
    for (int e = e0; e < e1; ++e)
      if (D.apos[e] == r) v += (T)D.aval[e];
    for (int q = c0; q < c1; ++q) {
      const int c = D.child_list[q];
      const int64_t io = D.inv_off[c];
      const int jt = D.invmap[io + t];
      if (jt < 0) continue;
      const int jr = D.invmap[io + r];
      if (jr < jt) continue;
      const int nbc = D.nr[c] - D.nc[c];
      v += upd[D.upd_off[c] + (int64_t)jt * nbc + jr];
    }
    col[r - colbase] = v;
  }
}

// ---------------------------------------------------------------------------
// Tile kernels (one workgroup of 256 threads per task).
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void tile_fma(const T (*As)[TB + 1], const T (*Bs)[TB + 1], int K, T acc[4][4], int tx, int ty) {
  for (int k = 0; k < K; ++k) {
    T a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = As[k][ty + 16 * i];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = Bs[k][tx + 16 * j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
  }
}

// As[k][r] = M[r + k*ld] for r < h, k < K (column-major tile), zero elsewhere.
template <typename T>
__device__ inline void load_cm(T (*As)[TB + 1], const T* M, int64_t ld, int h, int K) {
  for (int e = threadIdx.x; e < TB * TB; e += 256) {
    const int r = e % TB, k = e / TB;
    As[k][r] = (r < h && k < K) ? M[r + (int64_t)k * ld] : (T)0;
  }
}

// Bs[k][c] = M[k + c*ld] (element (k, c) of a column-major matrix) for k < K, c < w.
template <typename T>
__device__ inline void load_cm_t(T (*Bs)[TB + 1], const T* M, int64_t ld, int K, int w) {
  for (int e = threadIdx.x; e < TB * TB; e += 256) {
    const int k = e % TB, c = e / TB;
    Bs[k][c] = (k < K && c < w) ? M[k + (int64_t)c * ld] : (T)0;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) potrf_kernel(FactorDev D, int64_t task_off, T* panel, T* upd, T* dinv,
                                                    int* flag) {
  __shared__ T a[TB][TB + 1];
  __shared__ T b[TB][TB + 1];
  const int* tk = D.tasks + 4 * (task_off + blockIdx.x);
  const int s = tk[0], p = tk[3];
  const Sn S = sn_of(D, s);
  const int r0 = p * TB, h = min(TB, S.nc - r0);
  int64_t ld;
  T* tile = front_ptr(panel, upd, S, r0, r0, ld);
  const int tid = threadIdx.x;
  for (int e = tid; e < TB * TB; e += 256) {
    const int i = e % TB, j = e / TB;
    a[i][j] = (i < h && j < h) ? tile[i + (int64_t)j * ld] : (T)0;
  }
  __syncthreads();
  for (int j = 0; j < h; ++j) {
    if (tid == 0) {
      T d = a[j][j];
      if (!(d > (T)0) || !isfinite((double)d)) {
        flag[0] = S.begin + r0 + j + 1;
        d = (T)1;
      }
      a[j][j] = sqrt(d);
    }
    __syncthreads();
    const T ljj = a[j][j];
    for (int i = j + 1 + tid; i < h; i += 256) a[i][j] /= ljj;
    __syncthreads();
    const int w = h - j - 1;
    for (int e = tid; e < w * w; e += 256) {
      const int i = j + 1 + e % w, k = j + 1 + e / w;
      if (k <= i) a[i][k] -= a[i][j] * a[k][j];
    }
    __syncthreads();
  }
  // inverse of the h x h lower factor, one column per thread
  if (tid < TB) {
    const int j = tid;
    for (int i = 0; i < TB; ++i) b[i][j] = (T)0;
    if (j < h) {
      b[j][j] = (T)1 / a[j][j];
      for (int i = j + 1; i < h; ++i) {
        T s2 = 0;
        for (int k = j; k < i; ++k) s2 += a[i][k] * b[k][j];
        b[i][j] = -s2 / a[i][i];
      }
    }
  }
  __syncthreads();
  T* di = dinv + D.dinv_off[s] + (int64_t)p * TB * TB;
  for (int e = tid; e < TB * TB; e += 256) {
    const int i = e % TB, j = e / TB;
    di[i + TB * j] = b[i][j];
    if (i < h && j < h) tile[i + (int64_t)j * ld] = (i >= j) ? a[i][j] : (T)0;
  }
}

// kind 0: trsm   C = C dinv_p^T            (task s, I, p, p)
// kind 1: update C(I,J) -= C(I,p) C(J,p)^T   (task s, I, J, p)
// kind 2: invscale C(I,q) = C(I,q) dinv_q, or dinv_q itself when I == q
// kind 3: invupdate C(I,r) -= C(I,q) Lcopy(q, r)
template <typename T, int KIND>
__global__ void __launch_bounds__(256) tile_kernel(FactorDev D, int64_t task_off, T* panel, T* upd, T* dinv,
                                                   T* lcopy) {
  __shared__ T As[TB][TB + 1];
  __shared__ T Bs[TB][TB + 1];
  const int* tk = D.tasks + 4 * (task_off + blockIdx.x);
  const int s = tk[0], I = tk[1], J = tk[2], p = tk[3];
  const Sn S = sn_of(D, s);
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  int rI, hI, rJ, hJ, rP, wP;
  tile_rows(S, I, rI, hI);
  tile_rows(S, J, rJ, hJ);
  tile_rows(S, p, rP, wP);
  int64_t ldc, lda;
  T* C = front_ptr(panel, upd, S, rI, rJ, ldc);            // tile (I, J): rows hI, cols hJ
  const T* di = dinv + D.dinv_off[s] + (int64_t)p * TB * TB;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0;
  int K = 0;
  if (KIND == 0) {              // C(I,p) dinv_p^T, K = wP
    K = wP;
    load_cm(As, C, ldc, hI, K);
    load_cm(Bs, di, TB, hJ, K);   // Bs[k][c] = dinv[c + 64k] = dinv(c, k)
  } else if (KIND == 1) {
    K = wP;
    const T* Ap = front_ptr(panel, upd, S, rI, rP, lda);
    int64_t ldb;
    const T* Bp = front_ptr(panel, upd, S, rJ, rP, ldb);
    load_cm(As, Ap, lda, hI, K);
    load_cm(Bs, Bp, ldb, hJ, K);
  } else if (KIND == 2) {
    if (I == p) {
      for (int e = tid; e < TB * TB; e += 256) {
        const int i = e % TB, j = e / TB;
        if (i < hI && j < hJ) C[i + (int64_t)j * ldc] = di[i + TB * j];
      }
      return;
    }
    K = wP;
    load_cm(As, C, ldc, hI, K);
    load_cm_t(Bs, di, TB, K, hJ);   // Bs[k][c] = dinv(k, c)
  } else {
    int64_t ldq;
    const T* Aq = front_ptr(panel, upd, S, rI, rP, ldq);   // X(I, q), q = p
    K = wP;
    load_cm(As, Aq, ldq, hI, K);
    const T* Lc = lcopy + D.lcopy_off[s] + (int64_t)rJ * S.nc + rP;   // element (rP + k, rJ + c)
    load_cm_t(Bs, Lc, S.nc, K, hJ);
  }
  __syncthreads();
  tile_fma<T>(As, Bs, K, acc, tx, ty);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ty + 16 * i;
    if (r >= hI) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = tx + 16 * j;
      if (c >= hJ) continue;
      T* dst = C + r + (int64_t)c * ldc;
      if (KIND == 0 || KIND == 2)
        *dst = acc[i][j];
      else
        *dst -= acc[i][j];
    }
  }
}

// Copy L11 column t (rows t..nc-1) to the level scratch and clear the panel's own part of column t.
template <typename T>
__global__ void __launch_bounds__(256) invprep_kernel(FactorDev D, int64_t task_off, int64_t count, T* panel,
                                                      T* lcopy) {
  const int lane = threadIdx.x % 64;
  const int64_t item = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (item >= count) return;
  const int* tk = D.tasks + 4 * (task_off + item);
  const int s = tk[0], t = tk[1];
  const Sn S = sn_of(D, s);
  T* col = panel + S.panel + (int64_t)t * S.nr;
  T* lc = lcopy + D.lcopy_off[s] + (int64_t)t * S.nc;
  for (int r = lane; r < S.nc; r += 64) {
    if (r >= t) lc[r] = col[r];
  }
  __threadfence_block();
  for (int r = lane; r < S.nc; r += 64) col[r] = (T)0;
}

}  // namespace

template <typename T>
void launch_factor_step(const FactorDev& D, int kind, int level, int64_t task_off, int count, int64_t asm_off,
                        int64_t asm_count, T* panel, T* upd, T* dinv, T* lcopy, int* flag, hipStream_t st) {
  (void)level;
  switch (kind) {
    case kAssemble:
      if (asm_count > 0)
        assemble_kernel<T><<<(unsigned)((asm_count + 3) / 4), 256, 0, st>>>(D, asm_off, asm_count, panel, upd);
      break;
    case kPotrf:
      potrf_kernel<T><<<count, 256, 0, st>>>(D, task_off, panel, upd, dinv, flag);
      break;
    case kTrsm:
      tile_kernel<T, 0><<<count, 256, 0, st>>>(D, task_off, panel, upd, dinv, lcopy);
      break;
    case kUpdate:
      tile_kernel<T, 1><<<count, 256, 0, st>>>(D, task_off, panel, upd, dinv, lcopy);
      break;
    case kInvPrep:
      invprep_kernel<T><<<(unsigned)((count + 3) / 4), 256, 0, st>>>(D, task_off, count, panel, lcopy);
      break;
    case kInvScale:
      tile_kernel<T, 2><<<count, 256, 0, st>>>(D, task_off, panel, upd, dinv, lcopy);
      break;
    case kInvUpdate:
      tile_kernel<T, 3><<<count, 256, 0, st>>>(D, task_off, panel, upd, dinv, lcopy);
      break;
    default:
      break;
  }
}
template void launch_factor_step<float>(const FactorDev&, int, int, int64_t, int, int64_t, int64_t, float*, float*,
                                        float*, float*, int*, hipStream_t);
template void launch_factor_step<double>(const FactorDev&, int, int, int64_t, int, int64_t, int64_t, double*,
                                         double*, double*, double*, int*, hipStream_t);

}  // namespace lobpcg
