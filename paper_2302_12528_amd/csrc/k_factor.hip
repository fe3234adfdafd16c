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
#include "mfma.hpp"
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
    ld = panel_ld(S.nr);
    return panel + S.panel + (int64_t)c * ld + r;
  }
  ld = S.nb;
  return upd + S.upd + (int64_t)(c - S.nc) * S.nb + (r - S.nc);
}

// ---------------------------------------------------------------------------
// Assembly, one wave per front column t of supernode s: the column is built in
// LDS (zero, the entries of A, then each child's Schur-complement column
// scattered through the child's relative row map; children are added one after
// another, so every target element has one writer at a time), then written out
// once.  Every child entry is read exactly once over the whole level.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) assemble_kernel(FactorDev D, int64_t item_off, int64_t count, T* panel,
                                                      T* upd) {
  extern __shared__ unsigned char asm_smem[];
  T* colbuf = reinterpret_cast<T*>(asm_smem);
  const int lane = threadIdx.x;
  const int64_t item = (int64_t)blockIdx.x;
  if (item >= count) return;
  const int s = D.asm_items[2 * (item_off + item)];
  const int t = D.asm_items[2 * (item_off + item) + 1];
  const Sn S = sn_of(D, s);
  const int rlo = (t < S.nc) ? 0 : t;
  int64_t ld;
  T* col = front_ptr(panel, upd, S, rlo, t, ld);   // col[r - rlo] is front element (r, t)
  if (D.is_dense) {
    for (int r = rlo + lane; r < S.nr; r += 64)
      col[r - rlo] = (r >= t) ? (T)D.dense[(int64_t)r * D.ld_dense + t] : (T)0;
    return;
  }
  for (int r = rlo + lane; r < S.nr; r += 64) colbuf[r] = (T)0;
  __syncthreads();
  if (t < S.nc) {
    const int j = S.begin + t;
    for (int e = D.prow[j] + lane; e < D.prow[j + 1]; e += 64) {
      const int pos = D.apos[e];
      if (pos >= 0) colbuf[pos] += (T)D.aval[e];
    }
  }
  __syncthreads();
  for (int q = D.child_ptr[s]; q < D.child_ptr[s + 1]; ++q) {
    const int c = D.child_list[q];
    const int jt = D.invmap[D.inv_off[c] + t];
    if (jt < 0) continue;
    const int nbc = D.nr[c] - D.nc[c];
    const T* uc = upd + D.upd_off[c] + (int64_t)jt * nbc;
    const int32_t* rel = D.relpos + D.row_off[c] + D.nc[c];
    for (int ic = jt + lane; ic < nbc; ic += 64) colbuf[rel[ic]] += uc[ic];
    __syncthreads();
  }
  for (int r = rlo + lane; r < S.nr; r += 64) col[r - rlo] = colbuf[r];
}

// ---------------------------------------------------------------------------
// Tile kernels (one workgroup of 256 threads per task).
// ---------------------------------------------------------------------------
// Uniform read of lane l's value (l must be wave-uniform).
__device__ inline float rdl(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ inline double rdl(double v, int l) {
  const long long x = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// acc (transposed) for this wave's 32 x 32 quadrant of the 64 x 64 tile C = As^T Bs, i.e.
// C[r][c] = sum_k As[k][r] Bs[k][c], with 16x16x4 MFMAs.  The MFMA computes D = C^T so that lane l's
// outputs (D rows Mfma<T>::drow(l, q) = C columns, D column l%16 = C row) are stored
// row-contiguously into the column-major panel.  K is zero padded to a multiple of 4 in LDS.
template <typename T>
__device__ inline void tile_mfma(const T (*As)[TB + 1], const T (*Bs)[TB + 1], int K,
                                 typename Mfma<T>::v4 acc[2][2]) {
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int qr = (w / 2) * 32, qc = (w % 2) * 32;
  const int kl = lane / 16, il = lane % 16;
  for (int ks = 0; ks < K; ks += 4) {
    T bf[2], af[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) bf[b] = Bs[ks + kl][qc + 16 * b + il];
#pragma unroll
    for (int a = 0; a < 2; ++a) af[a] = As[ks + kl][qr + 16 * a + il];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) acc[b][a] = Mfma<T>::op(bf[b], af[a], acc[b][a]);
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

// Cholesky of the h x h diagonal tile (p, p) and the inverse of its factor, by one wave.
// Lane i holds row i of the tile in registers (rows/columns >= h padded with the identity);
// column j is eliminated with uniform reads of the pivot and of column j; the inverse is
// formed column by column (lane j owns column j) from L staged in LDS.
template <typename T>
__global__ void __launch_bounds__(64) potrf_kernel(FactorDev D, int64_t task_off, T* panel, T* upd, T* dinv,
                                                   int* flag) {
  __shared__ T Ls[TB][TB + 1];
  const int* tk = D.tasks + 4 * (task_off + blockIdx.x);
  const int s = tk[0], p = tk[3];
  const Sn S = sn_of(D, s);
  const int r0 = p * TB, h = min(TB, S.nc - r0);
  int64_t ld;
  T* tile = front_ptr(panel, upd, S, r0, r0, ld);
  const int lane = threadIdx.x;
  T a[TB];
#pragma unroll
  for (int j = 0; j < TB; ++j) a[j] = (lane < h && j < h) ? tile[lane + (int64_t)j * ld] : (lane == j ? (T)1 : (T)0);
  int bad = 0;
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    T d = rdl(a[j], j);
    if (!(d > (T)0) || !isfinite((double)d)) {
      if (bad == 0) bad = j + 1;
      d = (T)1;
    }
    const T ljj = sqrt(d);
    const T rinv = (T)1 / ljj;
    const T l = (lane > j) ? a[j] * rinv : (lane == j ? ljj : (T)0);
    a[j] = l;
#pragma unroll
    for (int k = j + 1; k < TB; ++k) a[k] -= l * rdl(l, k);
  }
  if (bad != 0 && lane == 0 && bad <= h) flag[0] = S.begin + r0 + bad;
#pragma unroll
  for (int j = 0; j < TB; ++j) {
    const T v = (j <= lane) ? a[j] : (T)0;
    Ls[lane][j] = v;
    if (lane < h && j < h) tile[lane + (int64_t)j * ld] = v;
  }
  __syncthreads();
  // column `lane` of inv(L): forward substitution, L read from LDS (uniform addresses)
  T x[TB];
#pragma unroll
  for (int i = 0; i < TB; ++i) {
    T sacc = (i == lane) ? (T)1 : (T)0;
#pragma unroll
    for (int k = 0; k < i; ++k) sacc -= Ls[i][k] * x[k];
    x[i] = sacc / Ls[i][i];
  }
  T* di = dinv + D.dinv_off[s] + (int64_t)p * TB * TB;
#pragma unroll
  for (int i = 0; i < TB; ++i) di[i + TB * lane] = (i < h && lane < h) ? x[i] : (T)0;
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
  const int* tk = D.tasks + 4 * (task_off + xcd_block(blockIdx.x, gridDim.x));
  const int s = tk[0], I = tk[1], J = tk[2], p = tk[3];
  const Sn S = sn_of(D, s);
  const int tid = threadIdx.x;
  int rI, hI, rJ, hJ, rP, wP;
  tile_rows(S, I, rI, hI);
  tile_rows(S, J, rJ, hJ);
  tile_rows(S, p, rP, wP);
  int64_t ldc, lda;
  T* C = front_ptr(panel, upd, S, rI, rJ, ldc);            // tile (I, J): rows hI, cols hJ
  const T* di = dinv + D.dinv_off[s] + (int64_t)p * TB * TB;
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
  typename Mfma<T>::v4 acc[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[b][a][q] = 0;
  tile_mfma<T>(As, Bs, K, acc);
  const int lane = tid % 64, w = tid / 64;
  const int qr = (w / 2) * 32, qc = (w % 2) * 32;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int r = qr + 16 * a + lane % 16;
      if (r >= hI) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = qc + 16 * b + Mfma<T>::drow(lane, q);
        if (c >= hJ) continue;
        T* dst = C + r + (int64_t)c * ldc;
        if (KIND == 0 || KIND == 2)
          *dst = acc[b][a][q];
        else
          *dst -= acc[b][a][q];
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
  T* col = panel + S.panel + (int64_t)t * panel_ld(S.nr);
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
      if (asm_count > 0) {
        const size_t lds = D.is_dense ? 0 : (size_t)D.max_nr * sizeof(T);
        if (lds > 65536)
          (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&assemble_kernel<T>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        assemble_kernel<T><<<(unsigned)asm_count, 64, lds, st>>>(D, asm_off, asm_count, panel, upd);
      }
      break;
    case kPotrf:
      potrf_kernel<T><<<count, 64, 0, st>>>(D, task_off, panel, upd, dinv, flag);
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
