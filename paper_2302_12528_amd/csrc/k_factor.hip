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
#include "bufload.hpp"
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
// Assembly, one workgroup of NT threads per front column t of supernode s: the
// column is built in LDS (zero, the entries of A, then each child's
// Schur-complement column scattered through the child's relative row map;
// children are added one after another, so every target element has one writer
// at a time), then written out once.  Every child entry is read exactly once over
// the whole level.  Levels of tall fronts take NT = 256, the others NT = 64.
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ void __launch_bounds__(NT) assemble_kernel(FactorDev D, int64_t item_off, int64_t count, T* panel,
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
    for (int r = rlo + lane; r < S.nr; r += NT)
      col[r - rlo] = (r >= t) ? (T)D.dense[(int64_t)r * D.ld_dense + t] : (T)0;
    return;
  }
  for (int r = rlo + lane; r < S.nr; r += NT) colbuf[r] = (T)0;
  __syncthreads();
  if (t < S.nc) {
    const int j = S.begin + t;
    for (int e = D.prow[j] + lane; e < D.prow[j + 1]; e += NT) {
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
    // four entries per thread in flight before their scatter (the child's rows map to distinct rows)
    for (int ic0 = jt; ic0 < nbc; ic0 += 4 * NT) {
      int ri[4];
      T uv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int ic = ic0 + lane + NT * u;
        ri[u] = (ic < nbc) ? rel[ic] : -1;
        uv[u] = (ic < nbc) ? uc[ic] : (T)0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (ri[u] >= 0) colbuf[ri[u]] += uv[u];
    }
    __syncthreads();
  }
  for (int r = rlo + lane; r < S.nr; r += NT) col[r - rlo] = colbuf[r];
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


template <typename T>
struct Chunk4 {
  T v[4][4];   // 4 vectors of 4 consecutive rows: element e = tid + 256 q is rows 4 (e % 16) .. + 3 of column e / 16
};
// vec: M and ld * sizeof(T) are multiples of 16 bytes (rows below the own columns start at nc,
// which need not be a multiple of 4; such tiles take scalar loads)
template <typename T>
__device__ inline void chunk_load(Chunk4<T>& c, const T* M, int64_t ld, int h, int K, bool vec) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q, k = e / 16, r = 4 * (e % 16);
    if (k < K && r < h) {
      const T* src = M + r + (int64_t)k * ld;
      if (!vec) {
#pragma unroll
        for (int j = 0; j < 4; ++j) c.v[q][j] = (r + j < h) ? src[j] : (T)0;
      } else {
        if constexpr (sizeof(T) == 4) {
          const f32x4_t x = *reinterpret_cast<const f32x4_t*>(src);
          c.v[q][0] = x.x; c.v[q][1] = x.y; c.v[q][2] = x.z; c.v[q][3] = x.w;
        } else {
          const f64x2_t x0 = *reinterpret_cast<const f64x2_t*>(src), x1 = *reinterpret_cast<const f64x2_t*>(src + 2);
          c.v[q][0] = x0.x; c.v[q][1] = x0.y; c.v[q][2] = x1.x; c.v[q][3] = x1.y;
        }
#pragma unroll
        for (int j = 1; j < 4; ++j)
          if (r + j >= h) c.v[q][j] = (T)0;   // rows past the tile (padding or the next block)
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) c.v[q][j] = (T)0;
    }
  }
}
template <typename T>
__device__ inline void chunk_store(const Chunk4<T>& c, T (*As)[TB + 1]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q, k = e / 16, r = 4 * (e % 16);
#pragma unroll
    for (int j = 0; j < 4; ++j) As[k][r + j] = c.v[q][j];
  }
}

// The chunk transposed: Bs[r][k] = element (row r, column k) of the loaded block.
template <typename T>
__device__ inline void chunk_store_t(const Chunk4<T>& c, T (*Bs)[TB + 1]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = threadIdx.x + 256 * q, k = e / 16, r = 4 * (e % 16);
#pragma unroll
    for (int j = 0; j < 4; ++j) Bs[r + j][k] = c.v[q][j];
  }
}

// As[k][r] = M[r + k ld] for r < h, k < K, zero elsewhere, with 16-byte loads when M and ld allow.
template <typename T>
__device__ inline void load_cm_vec(T (*As)[TB + 1], const T* M, int64_t ld, int h, int K) {
  const bool vec = ((reinterpret_cast<uintptr_t>(M) | (uintptr_t)(ld * sizeof(T))) & 15) == 0;
  Chunk4<T> c;
  chunk_load(c, M, ld, h, K, vec);
  chunk_store(c, As);
}

// Task (s, I, p) of a panel step: first the update of tile (I, p) and of the diagonal tile (p, p) by
// panel p - 1 (the trailing update of the previous step leaves column p to this step), then the
// Cholesky factor L_pp of the diagonal tile and its inverse are formed in the workgroup (every task of
// the step repeats this small computation, so the step needs one launch); the task with I == p writes
// L_pp and inv(L_pp), every other task replaces its tile (I, p) by C inv(L_pp)^T.  Rows and columns of
// the tile at or beyond h are padded with the identity.
//   factorization: thread (row i, quarter w) holds row i, columns 16 w .. 16 w + 15 in registers,
//     so wave w holds 16 whole columns.  Quarter by quarter, the owning wave factors its 16 columns
//     alone (L[c][j] of another row c is a readlane) and publishes them through LDS; after one
//     barrier the waves to its right subtract the rank-16 product from their columns;
//   inverse X = inv(L) by 16 x 16 blocks: wave w inverts the diagonal block L_ww by forward
//     substitution (lane c < 16 holds column c), then forms its blocks below the diagonal in order,
//     X_iw = -X_ii (sum_{k = w}^{i - 1} L_ik X_kw), on the matrix cores (one barrier per block row).
template <typename T>
constexpr int potrf_lds_elems() { return 2 * TB * (TB + 1) + 2 * TB * ((sizeof(T) == 4) ? 20 : 18); }

// One task of the panel step (tk: {s, I, J, p}); lds: potrf_lds_elems<T>() elements of LDS, 16-byte
// aligned.
template <typename T>
__device__ __attribute__((always_inline)) void potrf_trsm_body(const FactorDev& D, const int* tk, T* panel,
                                                               T* upd, T* dinv, int* flag, T* lds) {
  T(*Ls)[TB + 1] = reinterpret_cast<T(*)[TB + 1]>(lds);                  // L, then the K-major tile C(I, p)
  T(*Xs)[TB + 1] = reinterpret_cast<T(*)[TB + 1]>(lds + TB * (TB + 1));  // Xs[k][c] = inv(L)[c][k]
  constexpr int LBS = (sizeof(T) == 4) ? 20 : 18;   // 16-byte aligned rows
  // the published quarter of L, double-buffered; after the factorization the first TB entries hold
  // the reciprocals of L's diagonal
  T(*Lb)[TB][LBS] = reinterpret_cast<T(*)[TB][LBS]>(lds + 2 * TB * (TB + 1));
  T* rd = lds + 2 * TB * (TB + 1);
  const int s = tk[0], I = tk[1], p = tk[3];
  const Sn S = sn_of(D, s);
  const int r0 = p * TB, h = min(TB, S.nc - r0);
  int64_t ld;
  T* tile = front_ptr(panel, upd, S, r0, r0, ld);
  const int tid = threadIdx.x, i = tid % 64, w = __builtin_amdgcn_readfirstlane(tid / 64);
  // tile (I, p) of the trsm, loaded early so that its latency hides behind the factorization
  int rI, hI;
  tile_rows(S, I, rI, hI);
  int64_t ldc;
  T* C = front_ptr(panel, upd, S, rI, r0, ldc);
  T cv[16];
  if (I != p) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q, r = e % TB, k = e / TB;
      cv[q] = (r < hI && k < h) ? C[r + (int64_t)k * ldc] : (T)0;
    }
  }
  T a[16];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int c = 16 * w + kk;
    a[kk] = (i < h && c < h) ? tile[i + (int64_t)c * ld] : (i == c ? (T)1 : (T)0);
  }
  if (p > 0) {
    // Column p still lacks panel p - 1's contribution (the step's own part of the trailing update):
    // C(I, p) -= L(I, p - 1) L(p, p - 1)^T and the diagonal tile's D -= L(p, p - 1) L(p, p - 1)^T (every
    // task forms the latter, as it forms the factorization), on the matrix cores with K-major operands
    // in Ls and Xs; the products go through LDS into the layouts of a[] and cv[].
    int rQ, wQ;
    tile_rows(S, p - 1, rQ, wQ);
    int64_t lda, ldb;
    const T* Ap = front_ptr(panel, upd, S, rI, rQ, lda);
    const T* Bp = front_ptr(panel, upd, S, r0, rQ, ldb);
    if (I != p) load_cm_vec(Ls, Ap, lda, hI, wQ);
    load_cm_vec(Xs, Bp, ldb, h, wQ);
    __syncthreads();
    // one product at a time, so that only one set of accumulators is live: tile I's into Ls (after
    // every wave has read its operand there), then the diagonal tile's into Xs
    const int lane = tid % 64, qr = (w / 2) * 32, qc = (w % 2) * 32;
    typename Mfma<T>::v4 acc[2][2];
    auto to_lds = [&](T (*M)[TB + 1]) {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int q = 0; q < 4; ++q) M[qr + 16 * a2 + lane % 16][qc + 16 * b + Mfma<T>::drow(lane, q)] = acc[b][a2][q];
    };
    auto zero = [&]() {
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[b][a2][q] = 0;
    };
    if (I != p) {
      zero();
      tile_mfma<T>(Ls, Xs, (wQ + 3) & ~3, acc);
      __syncthreads();
      to_lds(Ls);
    }
    zero();
    tile_mfma<T>(Xs, Xs, (wQ + 3) & ~3, acc);
    __syncthreads();
    to_lds(Xs);
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) a[kk] -= Xs[i][16 * w + kk];
    if (I != p) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q;
        cv[q] -= Ls[e % TB][e / TB];
      }
    }
    __syncthreads();
  }
  // X starts as zero: its blocks above the diagonal stay so
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    Xs[e / TB][e % TB] = (T)0;
  }
  int bad = 0;
  T rrow = (T)1;   // 1 / L[i][i] on lane i of the wave owning column i
  // the outer loop stays rolled: this kernel runs once per panel step, so its code is fetched cold
  // each time and must stay short
#pragma unroll 1
  for (int jb = 0; jb < 4; ++jb) {
    T (*lb)[LBS] = Lb[jb & 1];
    if (w == jb) {
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int j = 16 * jb + jj;
        // the column's entries in the rows of the quarter's diagonal block, read before the pivot is
        // known: l_i l_r = a_ij a_rj / d, so the update needs a_rj, not l_rj
        T sk[16];
#pragma unroll
        for (int kk = jj + 1; kk < 16; ++kk) sk[kk] = rdl(a[jj], 16 * jb + kk);
        T d = rdl(a[jj], j);
        const bool ok = (d > (T)0) && (d < (T)INFINITY);
        if (!ok) {
          d = (T)1;
          if (bad == 0) bad = j + 1;
        }
        T ljj, rinv;
        if constexpr (sizeof(T) == 4) {
          rinv = __builtin_amdgcn_rsqf(d);   // 1 ulp: L of the FP32 preconditioner
          ljj = d * rinv;
        } else {
          ljj = sqrt(d);
          rinv = (T)1 / ljj;
        }
        if (i == j) rrow = rinv;
        const T li = a[jj] * rinv;
        const T t = li * rinv;   // a_ij / d
        a[jj] = (i > j) ? li : (i == j ? ljj : (T)0);
#pragma unroll
        for (int kk = jj + 1; kk < 16; ++kk) a[kk] -= t * sk[kk];
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) lb[i][jj] = a[jj];
    }
    __syncthreads();
    if (w > jb) {
      T lrow[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) lrow[jj] = lb[i][jj];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj)
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) a[kk] -= lrow[jj] * lb[16 * w + kk][jj];
    }
  }
  if (I == p && bad != 0 && i == 0 && bad <= h) flag[0] = S.begin + r0 + bad;
  // L_pp goes to its staging slot (column-major, ld 64); the update step moves it into the panel
  T* lstage = dinv + D.dinv_off[s] + (int64_t)(S.np + p) * TB * TB;
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) {
    const int c = 16 * w + kk;
    if (I == p) lstage[i + TB * c] = (c <= i) ? a[kk] : (T)0;
    Ls[i][c] = a[kk];
  }
  if (i >= 16 * w && i < 16 * w + 16) rd[i] = rrow;   // Lb is no longer read
  __syncthreads();
  // X_ww = inv(L_ww): lane c < 16 of wave w solves L_ww x = e_c
  const int w16 = 16 * w;
  if (i < 16) {
    T x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      T sum = (r == i) ? (T)1 : (T)0;
#pragma unroll
      for (int k = 0; k < r; ++k) sum -= Ls[w16 + r][w16 + k] * x[k];
      x[r] = sum * rd[w16 + r];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) Xs[w16 + i][w16 + r] = x[r];
  }
  __syncthreads();
  // X_iw for i = w + 1 + t, one block row per round; k-index of step u for this lane: drow(lane, u),
  // so that register u of a product's accumulator is the left operand of the next product at step u
  {
    const int lane = tid % 64, l16 = lane % 16;
#pragma unroll 1
    for (int t = 0; t < 3; ++t) {
      const int ib = w + 1 + t;
      if (ib < 4) {
        typename Mfma<T>::v4 acc = {0, 0, 0, 0};
        for (int kb = w; kb < ib; ++kb)
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kx = 16 * kb + Mfma<T>::drow(lane, u);
            acc = Mfma<T>::op(Ls[16 * ib + l16][kx], Xs[w16 + l16][kx], acc);   // T = sum_k L_ik X_kw
          }
        typename Mfma<T>::v4 m = {0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < 4; ++u) {   // M^T = T^T X_ii^T
          const int kx = 16 * ib + Mfma<T>::drow(lane, u);
          m = Mfma<T>::op(acc[u], Xs[kx][16 * ib + l16], m);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Xs[w16 + Mfma<T>::drow(lane, q)][16 * ib + l16] = -m[q];
      }
      __syncthreads();
    }
  }
  if (I == p) {
    T* di = dinv + D.dinv_off[s] + (int64_t)p * TB * TB;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int c = 16 * w + kk;
      di[i + TB * c] = (i < h && c < h) ? Xs[c][i] : (T)0;
    }
    return;
  }
  auto& As = Ls;   // As[k][r] = C(r, k)
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, r = e % TB, k = e / TB;
    As[k][r] = cv[q];
  }
  __syncthreads();
  typename Mfma<T>::v4 acc[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[b][a2][q] = 0;
  tile_mfma<T>(As, Xs, (h + 3) & ~3, acc);
  const int lane = tid % 64;
  const int qr = (w / 2) * 32, qc = (w % 2) * 32;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2) {
      const int r = qr + 16 * a2 + lane % 16;
      if (r >= hI) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = qc + 16 * b + Mfma<T>::drow(lane, q);
        if (c < h) C[r + (int64_t)c * ldc] = acc[b][a2][q];
      }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) potrf_trsm_kernel(FactorDev D, int64_t task_off, T* panel, T* upd,
                                                         T* dinv, int* flag) {
  __shared__ __align__(16) T lds[potrf_lds_elems<T>()];
  potrf_trsm_body<T>(D, D.tasks + 4 * (task_off + xcd_block(blockIdx.x, gridDim.x)), panel, upd, dinv, flag, lds);
}

// Trailing update of a panel step, C(I,J) -= C(I,p) C(J,p)^T for p < J < np (task s, I, J, p); the
// task (s, p, p, p) instead stores L_pp from its staging slot into tile (p, p).  lds: 2 TB (TB + 1)
// elements.
template <typename T>
__device__ __attribute__((always_inline)) void update_body(const FactorDev& D, const int* tk, T* panel, T* upd,
                                                           T* dinv, T* lds) {
  T(*As)[TB + 1] = reinterpret_cast<T(*)[TB + 1]>(lds);
  T(*Bs)[TB + 1] = reinterpret_cast<T(*)[TB + 1]>(lds + TB * (TB + 1));
  const int s = tk[0], I = tk[1], J = tk[2], p = tk[3];
  const Sn S = sn_of(D, s);
  const int tid = threadIdx.x;
  int rI, hI, rJ, hJ, rP, wP;
  tile_rows(S, I, rI, hI);
  tile_rows(S, J, rJ, hJ);
  tile_rows(S, p, rP, wP);
  int64_t ldc, lda, ldb;
  T* C = front_ptr(panel, upd, S, rI, rJ, ldc);            // tile (I, J): rows hI, cols hJ
  if (I == p && J == p) {
    const T* ls = dinv + D.dinv_off[s] + (int64_t)(S.np + p) * TB * TB;
    for (int e = tid; e < TB * TB; e += 256) {
      const int r = e % TB, c = e / TB;
      if (r < hI && c < hJ) C[r + (int64_t)c * ldc] = ls[r + TB * c];
    }
    return;
  }
  const int K = wP;
  const T* Ap = front_ptr(panel, upd, S, rI, rP, lda);
  const T* Bp = front_ptr(panel, upd, S, rJ, rP, ldb);
  // this thread's 16 entries of C are requested first, so that their latency overlaps the panel loads
  const int lane = tid % 64, w = tid / 64;
  const int qr = (w / 2) * 32, qc = (w % 2) * 32;
  T cv[2][2][4];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = qr + 16 * a + lane % 16, c = qc + 16 * b + Mfma<T>::drow(lane, q);
        cv[b][a][q] = (r < hI && c < hJ) ? C[r + (int64_t)c * ldc] : (T)0;
      }
  load_cm_vec(As, Ap, lda, hI, K);
  load_cm_vec(Bs, Bp, ldb, hJ, K);
  __syncthreads();
  typename Mfma<T>::v4 acc[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[b][a][q] = 0;
  tile_mfma<T>(As, Bs, (K + 3) & ~3, acc);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int r = qr + 16 * a + lane % 16;
      if (r >= hI) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = qc + 16 * b + Mfma<T>::drow(lane, q);
        if (c < hJ) C[r + (int64_t)c * ldc] = cv[b][a][q] - acc[b][a][q];
      }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) update_kernel(FactorDev D, int64_t task_off, T* panel, T* upd, T* dinv) {
  __shared__ __align__(16) T lds[2 * TB * (TB + 1)];
  update_body<T>(D, D.tasks + 4 * (task_off + xcd_block(blockIdx.x, gridDim.x)), panel, upd, dinv, lds);
}

// The update of panel p's columns beyond p + 1 and the move of L_pp into the panel (blocks npotrf ..)
// together with the factorization of panel p + 1, which applies panel p to column p + 1 itself (blocks
// 0 .. npotrf - 1), in one launch: they read and write disjoint tiles (column p, which both read, is
// final), so the second may start before the first has finished without a second stream and its
// synchronization.
template <typename T>
__global__ void __launch_bounds__(256) potrf_update_kernel(FactorDev D, int64_t potrf_off, int npotrf,
                                                           int64_t upd_off, int nupd, T* panel, T* upd, T* dinv,
                                                           int* flag) {
  constexpr int NL = potrf_lds_elems<T>() > 2 * TB * (TB + 1) ? potrf_lds_elems<T>() : 2 * TB * (TB + 1);
  __shared__ __align__(16) T lds[NL];
  const int64_t b = blockIdx.x;
  if (b < npotrf)
    potrf_trsm_body<T>(D, D.tasks + 4 * (potrf_off + xcd_block(b, npotrf)), panel, upd, dinv, flag, lds);
  else
    update_body<T>(D, D.tasks + 4 * (upd_off + xcd_block(b - npotrf, nupd)), panel, upd, dinv, lds);
}

// Schur complement tile (I, J) of U_s (I >= J >= np): C -= L(I, :) L(J, :)^T over all nc panel
// columns, 64 at a time through LDS, accumulated in registers; C is read and written once.  The
// next 64-column chunk is loaded into registers (16-byte loads of 4 consecutive rows) while the
// current one is multiplied.
template <typename T>
__global__ void __launch_bounds__(256) schur_kernel(FactorDev D, int64_t task_off, T* panel, T* upd) {
  __shared__ T As[TB][TB + 1];
  __shared__ T Bs[TB][TB + 1];
  const int* tk = D.tasks + 4 * (task_off + xcd_block(blockIdx.x, gridDim.x));
  const int s = tk[0], I = tk[1], J = tk[2];
  const Sn S = sn_of(D, s);
  int rI, hI, rJ, hJ;
  tile_rows(S, I, rI, hI);
  tile_rows(S, J, rJ, hJ);
  int64_t ldc;
  T* C = front_ptr(panel, upd, S, rI, rJ, ldc);
  const int64_t ldp = panel_ld(S.nr);
  const T* Ap = panel + S.panel + rI;   // L(rI + r, k) = Ap[r + k ldp]
  const T* Bp = panel + S.panel + rJ;
  typename Mfma<T>::v4 acc[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[b][a][q] = 0;
  const bool va = ((reinterpret_cast<uintptr_t>(Ap) | (uintptr_t)(ldp * sizeof(T))) & 15) == 0;
  const bool vb = ((reinterpret_cast<uintptr_t>(Bp) | (uintptr_t)(ldp * sizeof(T))) & 15) == 0;
  Chunk4<T> na, nb;
  chunk_load(na, Ap, ldp, hI, min(TB, S.nc), va);
  chunk_load(nb, Bp, ldp, hJ, min(TB, S.nc), vb);
  for (int k0 = 0; k0 < S.nc; k0 += TB) {
    const int K = min(TB, S.nc - k0);
    __syncthreads();   // the previous chunk's products are done with As, Bs
    chunk_store(na, As);
    chunk_store(nb, Bs);
    __syncthreads();
    if (k0 + TB < S.nc) {
      const int K2 = min(TB, S.nc - k0 - TB);
      chunk_load(na, Ap + (int64_t)(k0 + TB) * ldp, ldp, hI, K2, va);
      chunk_load(nb, Bp + (int64_t)(k0 + TB) * ldp, ldp, hJ, K2, vb);
    }
    tile_mfma<T>(As, Bs, (K + 3) & ~3, acc);
  }
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
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
        if (c < hJ) C[r + (int64_t)c * ldc] -= acc[b][a][q];
      }
    }
}

// Schur complement on 128 x 128 blocks (task (s, I, J): tiles I, I + 1 by J, J + 1 of U_s, I >= J,
// both counted from np in pairs): wave w takes the 64 x 64 tile (I + w / 2, J + w % 2), skipping the
// one above the diagonal of a diagonal block and tiles past the front.  The operands are staged 16
// panel columns at a time for all 128 rows, in two LDS buffers (the next chunk is written into the
// other buffer after the current one's products, one barrier per chunk; 32-column chunks in two
// buffers hold twice the LDS, fewer workgroups per compute unit, and were slower), so each staged
// element feeds two tiles: half the operand traffic per product of schur_kernel, for the levels with
// large fronts.
constexpr int kSchurK = 16;
template <typename T>
__global__ void __launch_bounds__(256) schur2_kernel(FactorDev D, int64_t task_off, T* panel, T* upd) {
  constexpr int W2 = 2 * TB;   // 128 rows
  // row padding: the four 16-lane groups of an MFMA operand read fall in different banks
  constexpr int LP = (sizeof(T) == 4) ? W2 + 16 : W2 + 8;
  __shared__ T As[2][kSchurK][LP];
  __shared__ T Bs[2][kSchurK][LP];
  const int* tk = D.tasks + 4 * (task_off + xcd_block(blockIdx.x, gridDim.x));
  const int s = tk[0], I = tk[1], J = tk[2];
  const Sn S = sn_of(D, s);
  int rI, hI0, rJ, hJ0;
  tile_rows(S, I, rI, hI0);
  tile_rows(S, J, rJ, hJ0);
  const int hI = min(W2, S.nr - rI), hJ = min(W2, S.nr - rJ);   // rows of the two tile rows / columns
  int64_t ldc;
  T* C = front_ptr(panel, upd, S, rI, rJ, ldc);
  const int64_t ldp = panel_ld(S.nr);
  const T* Ap = panel + S.panel + rI;   // L(rI + r, k) = Ap[r + k ldp]
  const T* Bp = panel + S.panel + rJ;
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
  const int qr = (w / 2) * TB, qc = (w % 2) * TB;   // this wave's tile in the block
  const bool live = (qr < hI) && (qc < hJ) && !(I == J && qr < qc);   // wave-uniform
  typename Mfma<T>::v4 acc[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[b][a][q] = 0;
  const bool va = ((reinterpret_cast<uintptr_t>(Ap) | (uintptr_t)(ldp * sizeof(T))) & 15) == 0;
  const bool vb = ((reinterpret_cast<uintptr_t>(Bp) | (uintptr_t)(ldp * sizeof(T))) & 15) == 0;
  // loader: element e = tid + 256 q (q < NQ) is rows 4 (e % 32) .. + 3 of chunk column e / 32
  constexpr int NQ = kSchurK / 8;
  auto load = [&](T (&v)[NQ][4], const T* M, int h, int K, bool vec) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + 256 * q, k = e / 32, r = 4 * (e % 32);
      if (k < K && r < h) {
        const T* src = M + r + (int64_t)k * ldp;
        if (vec && r + 3 < h) {
          if constexpr (sizeof(T) == 4) {
            const f32x4_t x = *reinterpret_cast<const f32x4_t*>(src);
            v[q][0] = x.x; v[q][1] = x.y; v[q][2] = x.z; v[q][3] = x.w;
          } else {
            const f64x2_t x0 = *reinterpret_cast<const f64x2_t*>(src), x1 = *reinterpret_cast<const f64x2_t*>(src + 2);
            v[q][0] = x0.x; v[q][1] = x0.y; v[q][2] = x1.x; v[q][3] = x1.y;
          }
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) v[q][j] = (r + j < h) ? src[j] : (T)0;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[q][j] = (T)0;
      }
    }
  };
  auto store = [&](const T (&v)[NQ][4], T (*Ls)[LP]) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = tid + 256 * q, k = e / 32, r = 4 * (e % 32);
#pragma unroll
      for (int j = 0; j < 4; ++j) Ls[k][r + j] = v[q][j];
    }
  };
  T na[NQ][4], nb[NQ][4];
  load(na, Ap, hI, min(kSchurK, S.nc), va);
  load(nb, Bp, hJ, min(kSchurK, S.nc), vb);
  store(na, As[0]);
  store(nb, Bs[0]);
  __syncthreads();
  const int kl = lane / 16, il = lane % 16;
  int buf = 0;
  for (int k0 = 0; k0 < S.nc; k0 += kSchurK) {
    const int K = min(kSchurK, S.nc - k0);
    const bool more = k0 + kSchurK < S.nc;
    if (more) {
      const int K2 = min(kSchurK, S.nc - k0 - kSchurK);
      load(na, Ap + (int64_t)(k0 + kSchurK) * ldp, hI, K2, va);
      load(nb, Bp + (int64_t)(k0 + kSchurK) * ldp, hJ, K2, vb);
    }
    if (live) {
      const T (*Ac)[LP] = As[buf];
      const T (*Bc)[LP] = Bs[buf];
      for (int ks = 0; ks < K; ks += 4) {
        T af[4], bf[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) bf[b] = Bc[ks + kl][qc + 16 * b + il];
#pragma unroll
        for (int a = 0; a < 4; ++a) af[a] = Ac[ks + kl][qr + 16 * a + il];
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int a = 0; a < 4; ++a) acc[b][a] = Mfma<T>::op(bf[b], af[a], acc[b][a]);
      }
    }
    if (more) {
      store(na, As[buf ^ 1]);
      store(nb, Bs[buf ^ 1]);
    }
    __syncthreads();
    buf ^= 1;
  }
  if (!live) return;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = qr + 16 * a + lane % 16;
      if (r >= hI) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = qc + 16 * b + Mfma<T>::drow(lane, q);
        if (c < hJ) C[r + (int64_t)c * ldc] -= acc[b][a][q];
      }
    }
}

// Inverse phase, column t of supernode s: L11 column t (rows t..nc-1) and L21 column t go to the
// level scratch, and the panel's own part of column t becomes column t of the block-diagonal
// start of X = inv(L11): the inverse of the diagonal tile holding t, zero elsewhere.
template <typename T>
__global__ void __launch_bounds__(256) invprep_kernel(FactorDev D, int64_t task_off, int64_t count, T* panel,
                                                      T* dinv, T* lcopy) {
  const int lane = threadIdx.x % 64;
  const int64_t item = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (item >= count) return;
  const int* tk = D.tasks + 4 * (task_off + item);
  const int s = tk[0], t = tk[1];
  const Sn S = sn_of(D, s);
  T* col = panel + S.panel + (int64_t)t * panel_ld(S.nr);
  T* lc = lcopy + D.lcopy_off[s];
  T* l21 = lc + 2 * (int64_t)S.nc * S.nc;
  // eight rows per lane in flight: the loads of a group are issued before its stores (which could
  // otherwise not pass them, as the compiler cannot tell the buffers apart)
  constexpr int G = 8;
  for (int r0 = 0; r0 < S.nr; r0 += 64 * G) {
    T v[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int r = r0 + lane + 64 * u;
      v[u] = (r < S.nr) ? col[r] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int r = r0 + lane + 64 * u;
      if (r >= S.nr) break;
      if (r < S.nc) {
        if (r >= t) lc[(int64_t)t * S.nc + r] = v[u];
      } else {
        l21[(int64_t)t * S.nb + (r - S.nc)] = v[u];
      }
    }
  }
  __threadfence_block();
  const int qt = t / TB;
  const T* di = dinv + D.dinv_off[s] + (int64_t)qt * TB * TB + (int64_t)(t - qt * TB) * TB;   // column of inv(L_qq)
  for (int r0 = 0; r0 < S.nc; r0 += 64 * G) {
    T v[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int r = r0 + lane + 64 * u;
      v[u] = (r < S.nc && r / TB == qt) ? di[r - qt * TB] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int r = r0 + lane + 64 * u;
      if (r < S.nc) col[r] = v[u];
    }
  }
}

// One 64 x 64 output tile of the inverse phase, C = alpha sum_k A(:, k) B(k, :) over the task's
// nonzero reduction tiles, 64 columns of A (rows of B) at a time through LDS, the next chunk
// loaded while the current one is multiplied.  For a task (s, I, J, t):
//   kInvT1:  T1(I, J) = sum_{J <= k < m} L(I, k) X(k, J)   (L from the L11 copy, T1 to the scratch)
//   kInvX21: X(I, J) = -sum_{m <= k <= I} X(I, k) T1(k, J)
//   kInvP21: P(I, J) = sum_{J <= k < np} L21(I, k) X(k, J)   (L21 from its copy, I >= np)
// with m the first tile of the lower half of the 2^t-tile block holding I and J.  X lives in the
// panel's own rows (column-major, ld panel_ld(nr)).
template <typename T, int KIND>
__global__ void __launch_bounds__(256) inv_gemm_kernel(FactorDev D, int64_t task_off, T* panel, T* lcopy) {
  __shared__ T As[TB][TB + 1];
  __shared__ T Bs[TB][TB + 1];
  const int* tk = D.tasks + 4 * (task_off + xcd_block(blockIdx.x, gridDim.x));
  const int s = tk[0], I = tk[1], J = tk[2], t = tk[3];
  const Sn S = sn_of(D, s);
  const int nc = S.nc;
  const int64_t ldp = panel_ld(S.nr);
  T* X = panel + S.panel;
  T* Lc = lcopy + D.lcopy_off[s];
  T* Tc = Lc + (int64_t)nc * nc;
  T* L21c = Lc + 2 * (int64_t)nc * nc;
  int rI, hI;
  tile_rows(S, I, rI, hI);
  const int hJ = min(TB, nc - J * TB);
  const T *A, *B;
  int64_t lda, ldb, ldc;
  T* C;
  int k0, k1;   // reduction range (rows of B)
  T alpha = (T)1;
  if (KIND == kInvT1) {
    const int m = ((I >> t) << t) + (1 << (t - 1));
    k0 = J * TB; k1 = m * TB;
    A = Lc + rI; lda = nc;
    B = X + (int64_t)J * TB * ldp; ldb = ldp;
    C = Tc + rI + (int64_t)J * TB * nc; ldc = nc;
  } else if (KIND == kInvX21) {
    const int m = ((I >> t) << t) + (1 << (t - 1));
    k0 = m * TB; k1 = min(nc, (I + 1) * TB);
    A = X + rI; lda = ldp;
    B = Tc + (int64_t)J * TB * nc; ldb = nc;
    C = X + rI + (int64_t)J * TB * ldp; ldc = ldp;
    alpha = (T)-1;
  } else {
    k0 = J * TB; k1 = nc;
    A = L21c + (rI - nc); lda = S.nb;
    B = X + (int64_t)J * TB * ldp; ldb = ldp;
    C = X + rI + (int64_t)J * TB * ldp; ldc = ldp;
  }
  const bool va = ((reinterpret_cast<uintptr_t>(A) | (uintptr_t)(lda * sizeof(T))) & 15) == 0;
  const bool vb = ((reinterpret_cast<uintptr_t>(B) | (uintptr_t)(ldb * sizeof(T))) & 15) == 0;
  typename Mfma<T>::v4 acc[2][2];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[b][a][q] = 0;
  // A chunk: As[k][r] = A(r, k); B chunk loaded as (rows k, columns c) and stored transposed
  Chunk4<T> na, nb;
  chunk_load(na, A + (int64_t)k0 * lda, lda, hI, min(TB, k1 - k0), va);
  chunk_load(nb, B + k0, ldb, min(TB, k1 - k0), hJ, vb);
  for (int kc = k0; kc < k1; kc += TB) {
    const int K = min(TB, k1 - kc);
    __syncthreads();
    chunk_store(na, As);
    chunk_store_t(nb, Bs);
    __syncthreads();
    if (kc + TB < k1) {
      const int K2 = min(TB, k1 - kc - TB);
      chunk_load(na, A + (int64_t)(kc + TB) * lda, lda, hI, K2, va);
      chunk_load(nb, B + kc + TB, ldb, K2, hJ, vb);
    }
    tile_mfma<T>(As, Bs, (K + 3) & ~3, acc);
  }
  const int tid = threadIdx.x, lane = tid % 64, w = tid / 64;
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
        if (c < hJ) C[r + (int64_t)c * ldc] = alpha * acc[b][a][q];
      }
    }
}

}  // namespace

template <typename T>
void launch_factor_step(const FactorDev& D, int kind, int level_max_nr, int64_t task_off, int count, int64_t asm_off,
                        int64_t asm_count, T* panel, T* upd, T* dinv, T* lcopy, int* flag, hipStream_t st) {
  switch (kind) {
    case kAssemble:
      if (asm_count > 0) {
        const size_t lds = D.is_dense ? 0 : (size_t)level_max_nr * sizeof(T);
        if (level_max_nr >= 1024) {
          if (lds > 65536)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&assemble_kernel<T, 256>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
          assemble_kernel<T, 256><<<(unsigned)asm_count, 256, lds, st>>>(D, asm_off, asm_count, panel, upd);
        } else {
          if (lds > 65536)
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&assemble_kernel<T, 64>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
          assemble_kernel<T, 64><<<(unsigned)asm_count, 64, lds, st>>>(D, asm_off, asm_count, panel, upd);
        }
      }
      break;
    case kPotrf:
      potrf_trsm_kernel<T><<<count, 256, 0, st>>>(D, task_off, panel, upd, dinv, flag);
      break;

    case kUpdate:
      update_kernel<T><<<count, 256, 0, st>>>(D, task_off, panel, upd, dinv);
      break;
    case kSchur:
      schur_kernel<T><<<count, 256, 0, st>>>(D, task_off, panel, upd);
      break;
    case kSchur2:
      schur2_kernel<T><<<count, 256, 0, st>>>(D, task_off, panel, upd);
      break;
    case kInvPrep:
      invprep_kernel<T><<<(unsigned)((count + 3) / 4), 256, 0, st>>>(D, task_off, count, panel, dinv, lcopy);
      break;
    case kInvT1:
      inv_gemm_kernel<T, kInvT1><<<count, 256, 0, st>>>(D, task_off, panel, lcopy);
      break;
    case kInvX21:
      inv_gemm_kernel<T, kInvX21><<<count, 256, 0, st>>>(D, task_off, panel, lcopy);
      break;
    case kInvP21:
      inv_gemm_kernel<T, kInvP21><<<count, 256, 0, st>>>(D, task_off, panel, lcopy);
      break;

    default:
      break;
  }
}
void launch_potrf_update(const FactorDev& D, int64_t potrf_off, int npotrf, int64_t upd_off, int nupd, float* panel,
                         float* upd, float* dinv, int* flag, hipStream_t st) {
  potrf_update_kernel<float><<<npotrf + nupd, 256, 0, st>>>(D, potrf_off, npotrf, upd_off, nupd, panel, upd, dinv,
                                                            flag);
}

template void launch_factor_step<float>(const FactorDev&, int, int, int64_t, int, int64_t, int64_t, float*, float*,
                                        float*, float*, int*, hipStream_t);
template void launch_factor_step<double>(const FactorDev&, int, int, int64_t, int, int64_t, int64_t, double*,
                                         double*, double*, double*, int*, hipStream_t);

}  // namespace lobpcg
