// Preconditioner application W_l = L^{-T} L^{-1} lower(R) in the factor's
// precision T (Algorithm 3 lines 9-10; section 5.1's two triangular solves),
// over the supernodal elimination tree, level by level.
//
// After factorization each supernode's panel holds P_s = [inv(L11); L21 inv(L11)]
// (nr x nc, column-major), so with b_s the right-hand side at its own rows
//   forward:  [y_s; d] = P_s b_s,  y_s = inv(L11) b_s, and d = L21 y_s is
//             subtracted from the rows below (passed up the tree in a
//             per-supernode update vector, pulled by the parent; no atomics);
//   backward: x_s = P_s^T [y_s; -x_below] = inv(L11)^T (y_s - L21^T x_below).
// Per level, a gather pass first adds the children's update vectors to the own
// rows of the right-hand side and passes them through to the supernode's own
// update vector; then every output tile (64 rows x M right-hand sides) is one
// workgroup that streams its panel block into matrix-core products.  A tile whose
// reduction range is split over several items writes partial tiles that a
// finalize pass sums in a fixed order.
#include "common.hpp"
#include "mfma.hpp"
#include "symbolic.hpp"

namespace lobpcg {

namespace {

constexpr int TR = 64;   // output tile rows

// Forward gather, one destination row per 64 lanes (lane = right-hand side): the sum of the
// children's update-vector rows listed for it is added to an own row of the right-hand side or
// initialises a below row of the supernode's update vector.
template <typename T>
__global__ void __launch_bounds__(256) fwd_gather_kernel(const int32_t* __restrict__ dst,
                                                         const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ src, int64_t item_off,
                                                         int64_t count, T* rhs, T* uvec, int M) {
  const int lane = threadIdx.x % 64;
  const int64_t item = item_off + (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (item >= item_off + count || lane >= M) return;
  const int32_t d = dst[item];
  const int32_t p0 = ptr[item], p1 = ptr[item + 1];
  T v = 0;
  for (int32_t q = p0; q < p1; ++q) v += uvec[(int64_t)src[q] * M + lane];
  if (d >= 0)
    rhs[(int64_t)d * M + lane] += v;
  else
    uvec[(int64_t)(-d - 1) * M + lane] = v;
}

// ---------------------------------------------------------------------------
// Matrix-core forms of the two tile products, one wave per item.  16-byte vector loads of the
// panel feed 16x16x4 MFMAs directly (each panel element is used once per item, so it is not
// staged through LDS); the right-hand-side operand is reused from registers by the 4 row blocks.
// ---------------------------------------------------------------------------
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef float4 type; };
template <> struct Vec16<double> { typedef double2 type; };

template <typename T, int N>
__device__ inline void load16(const T* p, T (&v)[N]) {
  static_assert(N * sizeof(T) == 16, "16-byte vector");
  const typename Vec16<T>::type q = *reinterpret_cast<const typename Vec16<T>::type*>(p);
  if constexpr (N == 4) {
    v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
  } else {
    v[0] = q.x; v[1] = q.y;
  }
}

// Forward: out tile (64 rows x M) = P_s[r0:r0+64, k0:k1] * b_s[k0:k1, :].  Lane (i = l % 16, g = l / 16)
// reads VW consecutive panel rows of column k = kc + g; element w of its p-th vector is row
// 16 VW p + VW i + w, the A operand of row block q = VW p + w.  Output row rb of block q is tile
// row 16 VW p + VW rb + w.
// Waves per tile item; wave w takes every NW-th reduction step.  Items of levels whose reduction
// ranges are short run one wave each (four items per block, no combine); FP64 items always do:
// their accumulators already fill the register file.
template <typename T, bool WIDE> constexpr int solve_waves() { return (WIDE && sizeof(T) == 4) ? 4 : 1; }

struct SolveItem {
  int s, tile, k0, k1, slot, begin, nr, nc;
  int64_t poff;
  int aux;      // update-vector offset (forward) or row-list offset (backward)
  bool parent;  // s has children
};

// Item `item` of a level, or nullptr-equivalent (false) past the end; wave-uniform.
__device__ inline SolveItem read_item(const int32_t* items, int64_t item) {
  const int4* p = reinterpret_cast<const int4*>(items + (int64_t)kSolveItemInts * item);
  const int4 a = p[0], b = p[1], c = p[2];
  SolveItem it;
  it.s = a.x; it.tile = a.y; it.k0 = a.z; it.k1 = a.w;
  it.slot = b.x; it.begin = b.y; it.nr = b.z; it.nc = b.w;
  it.poff = (int64_t)(uint32_t)c.x | ((int64_t)c.y << 32);
  it.aux = c.z;
  it.parent = (c.w & 1) != 0;
  return it;
}

// Sum of the per-wave accumulators into wave 0 (fixed order w = 0, 1, ..., so deterministic).
template <int NW, typename V4, int NQ>
__device__ inline bool reduce_waves(V4 (&acc)[NQ], V4* red) {
  if (NW == 1) return true;
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  if (w > 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) red[((w - 1) * NQ + q) * 64 + lane] = acc[q];
  }
  __syncthreads();
  if (w > 0) return false;
#pragma unroll
  for (int v = 1; v < NW; ++v)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] += red[((v - 1) * NQ + q) * 64 + lane];
  return true;
}

template <typename T, int M, bool WIDE>
__global__ void __launch_bounds__(256) fwd_mfma_kernel(const int32_t* __restrict__ items, int64_t item_off,
                                                       int64_t count, const T* __restrict__ panel,
                                                       const T* __restrict__ rhs, T* __restrict__ y,
                                                       T* __restrict__ uvec, T* __restrict__ part) {
  typedef Mfma<T> MF;
  typedef typename MF::v4 V4;
  constexpr int VW = 16 / sizeof(T);
  constexpr int NP = 4 / VW;
  constexpr int NCB = (M + 15) / 16;
  constexpr int NW = solve_waves<T, WIDE>();
  __shared__ V4 red[(NW > 1 ? NW - 1 : 1) * 4 * NCB * 64];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int i = lane % 16, g = lane / 16;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t item = (NW > 1) ? blk : blk * 4 + wave;
  if (item >= count) return;   // whole waves (NW == 1) or never (NW > 1)
  const int ksub = (NW > 1) ? wave : 0;
  const SolveItem it = read_item(items, item_off + item);
  const int tile = it.tile, k0 = it.k0, k1 = it.k1, slot = it.slot;
  const int begin = it.begin, nr = it.nr, nc = it.nc;
  const bool parent = it.parent;
  const int64_t ldp = panel_ld(nr);
  const int r0 = tile * TR;
  const int h = min(TR, nr - r0);
  const T* pbase = panel + it.poff + r0 + VW * i;
  V4 acc[4][NCB];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[q][c] = V4{0, 0, 0, 0};
  // U reduction steps per batch: all their loads are issued before the first MFMA of the batch
  constexpr int U = (sizeof(T) == 4) ? 8 : 4;
  for (int kb = k0 + 4 * ksub; kb < k1; kb += 4 * NW * U) {
    T a[U][NP][VW];
    T b[U][NCB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kb + 4 * NW * u + g;
      const bool kok = k < k1;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (kok && 16 * VW * p + VW * i < h) {
          load16(pbase + 16 * VW * p + (int64_t)k * ldp, a[u][p]);
        } else {
#pragma unroll
          for (int w = 0; w < VW; ++w) a[u][p][w] = 0;
        }
      }
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        const int col = 16 * c + i;
        b[u][c] = (kok && col < M) ? rhs[(int64_t)(begin + k) * M + col] : (T)0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int w = 0; w < VW; ++w)
#pragma unroll
          for (int c = 0; c < NCB; ++c)
            acc[VW * p + w][c] = MF::op(a[u][p][w], b[u][c], acc[VW * p + w][c]);
  }
  if (!reduce_waves<NW>(reinterpret_cast<V4(&)[4 * NCB]>(acc), red)) return;
#pragma unroll
  for (int p = 0; p < NP; ++p)
#pragma unroll
    for (int w = 0; w < VW; ++w)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = 16 * VW * p + VW * MF::drow(lane, v) + w;
        if (rr >= h) continue;
        const int row = r0 + rr;
        if (slot >= 0) {
#pragma unroll
          for (int c = 0; c < NCB; ++c) {
            const int col = 16 * c + i;
            if (col < M) part[((int64_t)slot * TR + rr) * M + col] = acc[VW * p + w][c][v];
          }
        } else if (row < nc) {
#pragma unroll
          for (int c = 0; c < NCB; ++c) {
            const int col = 16 * c + i;
            if (col < M) y[(int64_t)(begin + row) * M + col] = acc[VW * p + w][c][v];
          }
        } else {
          // below row: -d = -L21 y_s, added to the children's contributions the gather pass put
          // there when s has children
          T* u = uvec + ((int64_t)it.aux + row - nc) * M;
#pragma unroll
          for (int c = 0; c < NCB; ++c) {
            const int col = 16 * c + i;
            if (col < M) u[col] = (parent ? u[col] : (T)0) - acc[VW * p + w][c][v];
          }
        }
      }
}

// Backward: out tile (64 own columns x M) = P_s[k0:k1, j0:j0+64]^T z[k0:k1, :], z = [y_s; -x_below].
// Lane (i, g) reads VW consecutive k (k = kc + VW g + t) of panel column j0 + 16 jb + i; MFMA t
// pairs them with z row kc + VW g + t, so the 4 VW values of k in a step are reduced in VW MFMAs.
template <typename T, int M, bool WIDE>
__global__ void __launch_bounds__(256) bwd_mfma_kernel(const int32_t* __restrict__ rows, const int32_t* __restrict__ items,
                                                       int64_t item_off, int64_t count, const T* __restrict__ panel,
                                                       const T* __restrict__ y, T* __restrict__ x, double* W,
                                                       int64_t ldw, int mw, T* __restrict__ part) {
  typedef Mfma<T> MF;
  typedef typename MF::v4 V4;
  constexpr int VW = 16 / sizeof(T);
  constexpr int NCB = (M + 15) / 16;
  constexpr int NW = solve_waves<T, WIDE>();
  __shared__ V4 red[(NW > 1 ? NW - 1 : 1) * 4 * NCB * 64];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int i = lane % 16, g = lane / 16;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t item = (NW > 1) ? blk : blk * 4 + wave;
  if (item >= count) return;
  const int ksub = (NW > 1) ? wave : 0;
  const SolveItem it = read_item(items, item_off + item);
  const int tile = it.tile, k0 = it.k0, k1 = it.k1, slot = it.slot;
  const int begin = it.begin, nc = it.nc, nr = it.nr;
  const int64_t ldp = panel_ld(nr);
  const int64_t roff = it.aux;
  const int j0 = tile * TR;
  const int h = min(TR, nc - j0);
  const T* pbase = panel + it.poff + (int64_t)(j0 + i) * ldp + VW * g;
  V4 acc[4][NCB];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[q][c] = V4{0, 0, 0, 0};
  // U reduction steps (of 4 VW rows) per batch: panel loads and the row indices of the gathered
  // operand first, then the operand rows, then the MFMAs
  constexpr int U = (sizeof(T) == 4) ? 4 : 2;
  for (int kb = k0 + 4 * VW * ksub; kb < k1; kb += 4 * VW * NW * U) {
    T a[U][4][VW];
    int src_row[U][VW];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kc = kb + 4 * VW * NW * u;
      const int kk = kc + VW * g;
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        if (kk < k1 && 16 * jb + i < h) {
          load16(pbase + (int64_t)(16 * jb) * ldp + kc, a[u][jb]);
        } else {
#pragma unroll
          for (int t = 0; t < VW; ++t) a[u][jb][t] = 0;
        }
      }
#pragma unroll
      for (int t = 0; t < VW; ++t) {
        const int k = kk + t;
        // own rows read y at begin + k; below rows read -x at the listed row; -1 = past the range
        src_row[u][t] = (k >= k1) ? -1 : (k < nc ? begin + k : rows[roff + k]);
      }
    }
    T b[U][VW][NCB];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = kb + 4 * VW * NW * u + VW * g;
#pragma unroll
      for (int t = 0; t < VW; ++t) {
        const int r = src_row[u][t];
        const bool own = (kk + t < nc);
        const T* src = own ? y : x;
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
          const int col = 16 * c + i;
          const T v = (r >= 0 && col < M) ? src[(int64_t)r * M + col] : (T)0;
          b[u][t][c] = own ? v : -v;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < VW; ++t)
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
          for (int c = 0; c < NCB; ++c) acc[jb][c] = MF::op(a[u][jb][t], b[u][t][c], acc[jb][c]);
  }
  if (!reduce_waves<NW>(reinterpret_cast<V4(&)[4 * NCB]>(acc), red)) return;
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int jj = 16 * jb + MF::drow(lane, v);
      if (jj >= h) continue;
      const int64_t row = begin + j0 + jj;
#pragma unroll
      for (int c = 0; c < NCB; ++c) {
        const int col = 16 * c + i;
        if (col >= M) continue;
        const T val = acc[jb][c][v];
        if (slot >= 0) {
          part[((int64_t)slot * TR + jj) * M + col] = val;
        } else {
          x[row * M + col] = val;
          if (W && col < mw) W[row * ldw + col] = (double)val;
        }
      }
    }
}


// Sum of a split tile's partial tiles in slot order, then the same epilogue as an unsplit item.
// One block per 256 / M rows of a split tile (grid.y = 64 M / 256), one thread per element.
template <typename T, int M>
__global__ void __launch_bounds__(256) fwd_fin_kernel(FactorDev D, const int32_t* __restrict__ fin, int64_t fin_off,
                                                      const T* __restrict__ part, T* __restrict__ y,
                                                      T* __restrict__ uvec) {
  const int* f = fin + 4 * (fin_off + blockIdx.x);
  const int s = f[0], tile = f[1], slot0 = f[2], nch = f[3];
  const int r0 = tile * TR;
  const int h = min(TR, D.nr[s] - r0);
  const int nc = D.nc[s], begin = D.begin[s];
  const bool parent = D.child_ptr[s + 1] > D.child_ptr[s];
  {
    const int e = blockIdx.y * 256 + threadIdx.x;
    const int rr = e / M, col = e % M;
    if (rr >= h) return;
    T acc = 0;
    for (int q = 0; q < nch; ++q) acc += part[((int64_t)(slot0 + q) * TR + rr) * M + col];
    const int row = r0 + rr;
    if (row < nc) {
      y[(int64_t)(begin + row) * M + col] = acc;
    } else {
      T* u = uvec + (D.uvec_off[s] + row - nc) * M + col;
      *u = (parent ? *u : (T)0) - acc;
    }
  }
}

template <typename T, int M>
__global__ void __launch_bounds__(256) bwd_fin_kernel(FactorDev D, const int32_t* __restrict__ fin, int64_t fin_off,
                                                      const T* __restrict__ part, T* __restrict__ x, double* W,
                                                      int64_t ldw, int mw) {
  const int* f = fin + 4 * (fin_off + blockIdx.x);
  const int s = f[0], tile = f[1], slot0 = f[2], nch = f[3];
  const int j0 = tile * TR;
  const int h = min(TR, D.nc[s] - j0);
  const int begin = D.begin[s];
  {
    const int e = blockIdx.y * 256 + threadIdx.x;
    const int jj = e / M, col = e % M;
    if (jj >= h) return;
    T acc = 0;
    for (int q = 0; q < nch; ++q) acc += part[((int64_t)(slot0 + q) * TR + jj) * M + col];
    const int64_t row = begin + j0 + jj;
    x[row * M + col] = acc;
    if (W && col < mw) W[row * ldw + col] = (double)acc;
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


template <typename T, int M>
void sweep_level(const FactorDev& D, const SolveDev& Sd, int level, const T* panel, T* rhs, T* y, T* x, T* uvec,
                 T* fpart, T* bpart, double* W, int64_t ldw, int mw, bool forward, hipStream_t st) {
  if (forward) {
    const int64_t a0 = Sd.gather_level_off[level], a1 = Sd.gather_level_off[level + 1];
    if (a1 > a0)
      fwd_gather_kernel<T><<<(unsigned)((a1 - a0 + 3) / 4), 256, 0, st>>>(Sd.gather_dst, Sd.gather_ptr, Sd.gather_src,
                                                                          a0, a1 - a0, rhs, uvec, M);
    const int64_t f0 = Sd.fwd_level_off[level], f1 = Sd.fwd_level_off[level + 1];
    const int64_t fn = f1 - f0;
    if (fn > 0 && Sd.fwd_wide[level])
      fwd_mfma_kernel<T, M, true><<<(unsigned)(solve_waves<T, true>() > 1 ? fn : (fn + 3) / 4), 256, 0, st>>>(
          Sd.fwd_items, f0, fn, panel, rhs, y, uvec, fpart);
    else if (fn > 0)
      fwd_mfma_kernel<T, M, false><<<(unsigned)((fn + 3) / 4), 256, 0, st>>>(Sd.fwd_items, f0, fn, panel, rhs, y,
                                                                              uvec, fpart);
    const int64_t g0 = Sd.fwd_fin_level_off[level], g1 = Sd.fwd_fin_level_off[level + 1];
    if (g1 > g0)
      fwd_fin_kernel<T, M><<<dim3((unsigned)(g1 - g0), TR * M / 256), 256, 0, st>>>(D, Sd.fwd_fin, g0, fpart, y, uvec);
  } else {
    const int64_t b0 = Sd.bwd_level_off[level], b1 = Sd.bwd_level_off[level + 1];
    const int64_t bn = b1 - b0;
    if (bn > 0 && Sd.bwd_wide[level])
      bwd_mfma_kernel<T, M, true><<<(unsigned)(solve_waves<T, true>() > 1 ? bn : (bn + 3) / 4), 256, 0, st>>>(
          D.rows, Sd.bwd_items, b0, bn, panel, y, x, W, ldw, mw, bpart);
    else if (bn > 0)
      bwd_mfma_kernel<T, M, false><<<(unsigned)((bn + 3) / 4), 256, 0, st>>>(D.rows, Sd.bwd_items, b0, bn, panel, y,
                                                                              x, W, ldw, mw, bpart);
    const int64_t g0 = Sd.bwd_fin_level_off[level], g1 = Sd.bwd_fin_level_off[level + 1];
    if (g1 > g0)
      bwd_fin_kernel<T, M><<<dim3((unsigned)(g1 - g0), TR * M / 256), 256, 0, st>>>(D, Sd.bwd_fin, g0, bpart, x, W,
                                                                                   ldw, mw);
  }
}

}  // namespace

template <typename T>
void launch_precond(const FactorDev& D, const SolveDev& Sd, int nlevels, int M, const T* panel, T* rhs, T* y, T* x,
                    T* uvec, T* fpart, T* bpart, double* W, int64_t ldw, int mw, hipStream_t st) {
  for (int pass = 0; pass < 2; ++pass) {
    const bool fwd = (pass == 0);
    for (int q = 0; q < nlevels; ++q) {
      const int l = fwd ? q : nlevels - 1 - q;
      switch (M) {
        case 8: sweep_level<T, 8>(D, Sd, l, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, fwd, st); break;
        case 16: sweep_level<T, 16>(D, Sd, l, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, fwd, st); break;
        case 32: sweep_level<T, 32>(D, Sd, l, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, fwd, st); break;
        default: sweep_level<T, 64>(D, Sd, l, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, fwd, st); break;
      }
    }
  }
}

template <typename T>
void launch_cast_to(const double* src, int64_t lds, T* dst, int64_t n, int m, int M, hipStream_t st) {
  const int64_t total = n * M;
  if (total <= 0) return;
  cast_to_kernel<T><<<(unsigned)((total + 255) / 256), 256, 0, st>>>(src, lds, dst, n, m, M);
}

#define INST(T)                                                                                                 \
  template void launch_precond<T>(const FactorDev&, const SolveDev&, int, int, const T*, T*, T*, T*, T*, T*, T*, \
                                  double*, int64_t, int, hipStream_t);                                          \
  template void launch_cast_to<T>(const double*, int64_t, T*, int64_t, int, int, hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace lobpcg
