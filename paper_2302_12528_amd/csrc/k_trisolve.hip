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
#include "bufload.hpp"
#include "common.hpp"
#include "mfma.hpp"
#include "symbolic.hpp"

namespace lobpcg {

namespace {

constexpr int TR = 64;   // output tile rows

template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef f32x4_t type; };
template <> struct Vec16<double> { typedef f64x2_t type; };

// Forward gather: each destination row takes the sum of the children's update-vector rows listed
// for it, added to an own row of the right-hand side or initialising a below row of the
// supernode's update vector.  A row of M values is read and written as 16-byte vectors by
// LPR = M sizeof(T) / 16 lanes, so a wave handles 64 / LPR rows.
template <typename T, int M>
__device__ inline void gather_row(const int32_t* __restrict__ dst, const int32_t* __restrict__ ptr,
                                  const int32_t* __restrict__ src, int64_t item, int cl, T* rhs, T* uvec) {
  typedef typename Vec16<T>::type V;
  const int32_t d = dst[item];
  const int32_t p0 = ptr[item], p1 = ptr[item + 1];
  V v = {};
  int32_t q = p0;
  for (; q + 1 < p1; q += 2) {   // two children's rows in flight at a time
    const V a = *reinterpret_cast<const V*>(uvec + (int64_t)src[q] * M + cl);
    const V b = *reinterpret_cast<const V*>(uvec + (int64_t)src[q + 1] * M + cl);
    v += a;
    v += b;
  }
  if (q < p1) v += *reinterpret_cast<const V*>(uvec + (int64_t)src[q] * M + cl);
  if (d >= 0) {
    V* o = reinterpret_cast<V*>(rhs + (int64_t)d * M + cl);
    *o += v;
  } else {
    *reinterpret_cast<V*>(uvec + (int64_t)(-d - 1) * M + cl) = v;
  }
}

template <typename T, int M>
__global__ void __launch_bounds__(256) fwd_gather_kernel(const int32_t* __restrict__ dst,
                                                         const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ src, int64_t item_off,
                                                         int64_t count, T* rhs, T* uvec) {
  constexpr int VW = 16 / sizeof(T);
  constexpr int LPR = M / VW;
  constexpr int RPW = 64 / LPR;
  const int lane = threadIdx.x % 64;
  const int64_t r = ((int64_t)blockIdx.x * 4 + threadIdx.x / 64) * RPW + lane / LPR;
  if (r >= count) return;
  gather_row<T, M>(dst, ptr, src, item_off + r, (lane % LPR) * VW, rhs, uvec);
}

// ---------------------------------------------------------------------------
// Matrix-core forms of the two tile products.  Panel blocks are streamed with 16-byte buffer loads
// straight into 16x16x4 MFMA operands (each panel element is used once per item, so it is not
// staged through LDS); the right-hand-side operand is reused from registers by the 4 row blocks.
// The reduction range is walked in stages of U steps; the loads of stage j + 1 are issued before
// the MFMAs of stage j, so every wave keeps a stage of panel data in flight while it computes.
// ---------------------------------------------------------------------------
// Waves per tile item; wave w takes every NW-th stage.  Items of levels whose reduction ranges are
// short run one wave each (four items per block, no combine); FP64 items always do: their
// accumulators already fill most of the register file.
template <typename T, bool WIDE> constexpr int solve_waves() { return (WIDE && sizeof(T) == 4) ? 4 : 1; }

struct SolveItem {
  int s, tile, k0, k1, slot, begin, nr, nc;
  int64_t poff;
  int aux;      // update-vector offset (forward) or source-row list offset (backward)
  bool parent;  // s has children
};

// Item `item` of a level (wave-uniform).
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

// Four waves that split one item's reduction range: each writes its accumulators to LDS, then wave w
// sums accumulator block w over the waves in the fixed order 0, 1, 2, 3 (deterministic) into
// out[0..NCB) and writes that block of the tile.
template <typename V4, int NCB>
__device__ inline void reduce_blocks(const V4 (&acc)[4][NCB], V4 (&out)[NCB], V4* red, int wave) {
  const int lane = threadIdx.x % 64;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < NCB; ++c) red[((wave * 4 + q) * NCB + c) * 64 + lane] = acc[q][c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NCB; ++c) {
    V4 sum = red[((0 * 4 + wave) * NCB + c) * 64 + lane];
#pragma unroll
    for (int v = 1; v < 4; ++v) sum += red[((v * 4 + wave) * NCB + c) * 64 + lane];
    out[c] = sum;
  }
}

template <typename T> __device__ constexpr T kZero4[4] = {0, 0, 0, 0};

// The 4 values a lane holds for one output row: columns c0 + drow(lane, v), v = 0..3 (in FP32 4
// consecutive columns, one 16-byte access).  load_cols reads the current values there (row must be a
// valid row; columns past M read column 0 instead).
template <typename T, int M>
__device__ inline void load_cols(const T* row, int c0, T (&o)[4]) {
  const int lane = threadIdx.x % 64;
  if constexpr (sizeof(T) == 4) {
    const int col = c0 + 4 * (lane / 16);
    const f32x4_t v = *reinterpret_cast<const f32x4_t*>(row + (col < M ? col : 0));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = c0 + Mfma<T>::drow(lane, q);
      o[q] = row[col < M ? col : 0];
    }
  }
}

// Store of those values; sub: dst = old - val (old from load_cols), else dst = val.
template <typename T, int M>
__device__ inline void store_cols(T* row, int c0, const typename Mfma<T>::v4& val, bool sub, const T (&old)[4]) {
  const int lane = threadIdx.x % 64;
  if constexpr (sizeof(T) == 4) {
    const int col = c0 + 4 * (lane / 16);
    if (col >= M) return;
    f32x4_t v = val;
    if (sub) v = f32x4_t{old[0], old[1], old[2], old[3]} - v;
    *reinterpret_cast<f32x4_t*>(row + col) = v;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = c0 + Mfma<T>::drow(lane, q);
      if (col >= M) continue;
      row[col] = sub ? old[q] - val[q] : val[q];
    }
  }
}

// The same values widened to FP64 into the working-precision block (columns < mw).
template <typename T>
__device__ inline void store_cols_f64(double* row, int c0, const typename Mfma<T>::v4& val, int mw) {
  const int lane = threadIdx.x % 64;
  if constexpr (sizeof(T) == 4) {
    const int col = c0 + 4 * (lane / 16);
    if (col + 3 < mw && (reinterpret_cast<uintptr_t>(row + col) & 15) == 0) {
      f64x2_t* d = reinterpret_cast<f64x2_t*>(row + col);
      d[0] = f64x2_t{(double)val[0], (double)val[1]};
      d[1] = f64x2_t{(double)val[2], (double)val[3]};
      return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (col + q < mw) row[col + q] = (double)val[q];
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = c0 + Mfma<T>::drow(lane, q);
      if (col < mw) row[col] = val[q];
    }
  }
}

// Forward: out tile (64 rows x M) = P_s[r0:r0+64, k0:k1] * b_s[k0:k1, :].  A reduction step covers
// 4 panel columns: lane (i = l % 16, g = l / 16) reads VW consecutive rows of column kc + g; element
// w of its p-th vector is row 16 VW p + VW i + w, the A operand of row block q = VW p + w, and the
// B operand is b_s row kc + g, columns 16 c + i.  Output row rb of block q is tile row
// 16 VW p + VW rb + w.
template <typename T, int M, int NP, int NCB, int U>
struct FwdStage {
  T a[U][NP][16 / sizeof(T)];
  T b[U][NCB];
};

// One forward tile item by NW waves (wave = this wave's index among them; red: LDS for NW > 1).
template <typename T, int M, int NW>
__device__ inline void fwd_tile(const SolveItem& it, int wave, typename Mfma<T>::v4* red, const T* __restrict__ panel,
                                const T* __restrict__ rhs, T* __restrict__ y, T* __restrict__ uvec,
                                T* __restrict__ part) {
  typedef Mfma<T> MF;
  typedef typename MF::v4 V4;
  constexpr int VW = 16 / sizeof(T);
  constexpr int NP = 4 / VW;
  constexpr int NCB = (M + 15) / 16;
  constexpr int U = (sizeof(T) == 4) ? 4 : 2;   // reduction steps per stage
  constexpr int SC = 4 * U;                       // panel columns per stage
  const int lane = threadIdx.x % 64;
  const int i = lane % 16, g = lane / 16;
  const int tile = it.tile, k0 = it.k0, k1 = it.k1, slot = it.slot;
  const int begin = it.begin, nr = it.nr, nc = it.nc;
  const bool parent = it.parent;
  const int64_t ldp = panel_ld(nr);
  const int r0 = tile * TR;
  const int h = min(TR, nr - r0);
  const i32x4_t prs = make_rsrc(panel + it.poff, ldp * nc * (int64_t)sizeof(T));
  const i32x4_t brs = make_rsrc(rhs + (int64_t)begin * M, (int64_t)nc * M * sizeof(T));
  int32_t va[NP], vb[NCB];
#pragma unroll
  for (int p = 0; p < NP; ++p)
    va[p] = (16 * VW * p + VW * i < h) ? (int32_t)((r0 + 16 * VW * p + VW * i + g * ldp) * (int64_t)sizeof(T)) : kOob;
#pragma unroll
  for (int c = 0; c < NCB; ++c) vb[c] = (16 * c + i < M) ? (int32_t)((g * M + 16 * c + i) * sizeof(T)) : kOob;
  V4 acc[4][NCB];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[q][c] = V4{0, 0, 0, 0};
  typedef FwdStage<T, M, NP, NCB, U> St;
  auto load = [&](St& S, int kc) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ku = kc + 4 * u;
      const bool kok = ku + g < k1;
      const int32_t sa = (int32_t)(ku * ldp * (int64_t)sizeof(T));
      const int32_t sb = (int32_t)((int64_t)ku * M * sizeof(T));
#pragma unroll
      for (int p = 0; p < NP; ++p) Buf<T>::load16(prs, kok ? va[p] : kOob, sa, S.a[u][p]);
#pragma unroll
      for (int c = 0; c < NCB; ++c) S.b[u][c] = Buf<T>::load1(brs, kok ? vb[c] : kOob, sb);
    }
  };
  // one accumulator's U products back to back (an MFMA whose C operand is the previous MFMA's
  // result issues without a stall), accumulators one after another
  auto compute = [&](const St& S) {
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
      for (int w = 0; w < VW; ++w)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
          for (int u = 0; u < U; ++u) acc[VW * p + w][c] = MF::op(S.b[u][c], S.a[u][p][w], acc[VW * p + w][c]);
  };
  constexpr int stride = SC * NW;
  St cur, nxt;
  int kc = k0 + SC * wave;
  if (kc < k1) load(cur, kc);
  for (; kc < k1; kc += stride) {
    load(nxt, kc + stride);   // zeros, without memory traffic, past the end of the range
    __builtin_amdgcn_sched_barrier(0);
    compute(cur);
    __builtin_amdgcn_sched_barrier(0);
    cur = nxt;
  }
  // The MFMA computed D = b^T P^T: register v of lane (i, g) in block (p, w, c) is output row
  // 16 VW p + VW i + w, column 16 c + drow(lane, v) (4 consecutive columns in FP32).  Rows below the
  // own columns of a supernode with children subtract from the gathered update vector: when the tile
  // has such rows (a uniform test), the current values of all of a lane's rows are requested first,
  // unconditionally (an address clamped into the tile) and masked per row afterwards, so that they are
  // in flight together; a load under a per-lane condition would be waited for inside its branch.
  constexpr int NRL = (NW > 1) ? 1 : VW * NP;   // rows per lane
  auto row_of = [&](int e) { return (NW > 1) ? 16 * VW * (wave / VW) + VW * i + wave % VW
                                             : 16 * VW * (e / VW) + VW * i + e % VW; };
  auto dest = [&](int rr, bool& sub) -> T* {
    const int row = r0 + rr;
    sub = false;
    if (slot >= 0) return part + ((int64_t)slot * TR + rr) * M;
    if (row < nc) return y + (int64_t)(begin + row) * M;
    sub = true;   // below row: -d = -L21 y_s, added to the gathered children's contributions
    return uvec + ((int64_t)it.aux + row - nc) * M;
  };
  const bool rmw = parent && slot < 0 && r0 + h > nc;   // uniform
  // rows in groups whose current values take at most 64 registers
  constexpr int RG = (sizeof(T) * NRL * NCB * 4 <= 256) ? NRL : 1;
  auto emit = [&](int e, const V4 (&blk)[NCB], const T (&old)[NCB][4]) {
    const int rr = row_of(e);
    if (rr >= h) return;
    bool sub;
    T* base = dest(rr, sub);
#pragma unroll
    for (int c = 0; c < NCB; ++c) store_cols<T, M>(base, 16 * c, blk[c], sub, old[c]);
  };
  V4 blk[NCB];
  if constexpr (NW > 1) reduce_blocks<V4, NCB>(acc, blk, red, wave);
#pragma unroll
  for (int e0 = 0; e0 < NRL; e0 += RG) {
    T old[RG][NCB][4];
    if (rmw) {
      bool keep[RG];
#pragma unroll
      for (int e = 0; e < RG; ++e) {
        const T* base = dest(min(row_of(e0 + e), h - 1), keep[e]);
#pragma unroll
        for (int c = 0; c < NCB; ++c) load_cols<T, M>(base, 16 * c, old[e][c]);
      }
#pragma unroll
      for (int e = 0; e < RG; ++e)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
          for (int q = 0; q < 4; ++q) old[e][c][q] = keep_if(keep[e], old[e][c][q]);
    } else {
#pragma unroll
      for (int e = 0; e < RG; ++e)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
          for (int q = 0; q < 4; ++q) old[e][c][q] = (T)0;
    }
#pragma unroll
    for (int e = 0; e < RG; ++e) {
      if constexpr (NW > 1) emit(e0 + e, blk, old[e]);
      else emit(e0 + e, acc[e0 + e], old[e]);
    }
  }
}

template <typename T, int M, bool WIDE>
__global__ void __launch_bounds__(256) fwd_mfma_kernel(const int32_t* __restrict__ items, int64_t item_off,
                                                       int64_t count, const T* __restrict__ panel,
                                                       const T* __restrict__ rhs, T* __restrict__ y,
                                                       T* __restrict__ uvec, T* __restrict__ part) {
  typedef typename Mfma<T>::v4 V4;
  constexpr int NCB = (M + 15) / 16;
  constexpr int NW = solve_waves<T, WIDE>();
  __shared__ V4 red[(NW > 1 ? NW : 0) * 4 * NCB * 64 + 1];
  // the wave index is uniform: item fields and buffer resources then live in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t item = (NW > 1) ? blk : blk * 4 + wave;
  if (item >= count) return;   // whole waves (NW == 1) or never (NW > 1)
  fwd_tile<T, M, NW>(read_item(items, item_off + item), NW > 1 ? wave : 0, red, panel, rhs, y, uvec, part);
}

// Backward: out tile (64 own columns x M) = P_s[k0:k1, j0:j0+64]^T z[k0:k1, :], z = [y_s; -x_below].
// A reduction step covers 4 VW panel rows: lane (i, g) reads VW consecutive rows (k = kc + VW g + t)
// of panel column j0 + 16 jb + i, and MFMA t pairs them with z row kc + VW g + t.  The rows of z are
// read through the supernode's source-row list (an index into yx = [y; x]: own rows point into y,
// below rows into x); the list entries of stage j + 2 are loaded while stage j computes, so each
// stage's z loads can be issued as soon as the previous stage's MFMAs start.
template <typename T, int NCB, int U>
struct BwdStage {
  T a[U][4][16 / sizeof(T)];
  T b[U][16 / sizeof(T)][NCB];
};
template <typename T, int U>
struct BwdIdx {
  int32_t r[U][16 / sizeof(T)];
};

// One backward tile item by NW waves.
template <typename T, int M, int NW>
__device__ inline void bwd_tile(const SolveItem& it, int wave, typename Mfma<T>::v4* red,
                                const int32_t* __restrict__ srcrows, const T* __restrict__ panel,
                                const T* __restrict__ yx, int64_t yx_rows, T* __restrict__ x, double* W, int64_t ldw,
                                int mw, T* __restrict__ part) {
  typedef Mfma<T> MF;
  typedef typename MF::v4 V4;
  constexpr int VW = 16 / sizeof(T);
  constexpr int NCB = (M + 15) / 16;
  constexpr int U = 1;             // reduction steps per stage
  constexpr int SR = 4 * VW * U;   // panel rows per stage
  const int lane = threadIdx.x % 64;
  const int i = lane % 16, g = lane / 16;
  const int tile = it.tile, k0 = it.k0, k1 = it.k1, slot = it.slot;
  const int begin = it.begin, nc = it.nc, nr = it.nr;
  const int64_t ldp = panel_ld(nr);
  const int j0 = tile * TR;
  const int h = min(TR, nc - j0);
  const i32x4_t prs = make_rsrc(panel + it.poff, ldp * nc * (int64_t)sizeof(T));
  const i32x4_t irs = make_rsrc(srcrows + it.aux, panel_ld(nr) * (int64_t)sizeof(int32_t));
  const i32x4_t zrs = make_rsrc(yx, yx_rows * M * (int64_t)sizeof(T));
  int32_t va[4];
#pragma unroll
  for (int jb = 0; jb < 4; ++jb)
    va[jb] = (16 * jb + i < h) ? (int32_t)(((j0 + 16 * jb + i) * ldp + VW * g) * (int64_t)sizeof(T)) : kOob;
  const int32_t vi = VW * g * (int32_t)sizeof(int32_t);
  V4 acc[4][NCB];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[q][c] = V4{0, 0, 0, 0};
  typedef BwdStage<T, NCB, U> St;
  typedef BwdIdx<T, U> Ix;
  auto load_idx = [&](Ix& I, int kc) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ku = kc + 4 * VW * u;
      Buf<T>::load_idx(irs, ku + VW * g < k1 ? vi : kOob, ku * (int32_t)sizeof(int32_t), I.r[u]);
    }
  };
  auto load = [&](St& S, const Ix& I, int kc) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ku = kc + 4 * VW * u;
      const bool kok = ku + VW * g < k1;
      const int32_t sa = ku * (int32_t)sizeof(T);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) Buf<T>::load16(prs, kok ? va[jb] : kOob, sa, S.a[u][jb]);
#pragma unroll
      for (int t = 0; t < VW; ++t) {
        const bool ok = ku + VW * g + t < k1;
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
          const int col = 16 * c + i;
          const int32_t off = (ok && col < M) ? (int32_t)(((int64_t)I.r[u][t] * M + col) * sizeof(T)) : kOob;
          S.b[u][t][c] = Buf<T>::load1(zrs, off, 0);
        }
      }
    }
  };
  auto compute = [&](St& S, int kc) {
    // own rows (k < nc) contribute +y, below rows -x
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < VW; ++t) {
        const bool own = kc + 4 * VW * u + VW * g + t < nc;
#pragma unroll
        for (int c = 0; c < NCB; ++c) S.b[u][t][c] = own ? S.b[u][t][c] : -S.b[u][t][c];
      }
    // one accumulator's products back to back, accumulators one after another
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int c = 0; c < NCB; ++c)
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int t = 0; t < VW; ++t) acc[jb][c] = MF::op(S.b[u][t][c], S.a[u][jb][t], acc[jb][c]);
  };
  constexpr int stride = SR * NW;
  St cur, nxt;
  Ix i1, i2;   // source rows of the next stage and of the one after
  int kc = k0 + SR * wave;
  if (kc < k1) {
    load_idx(i1, kc);
    load_idx(i2, kc + stride);
    load(cur, i1, kc);
    i1 = i2;
    load_idx(i2, kc + 2 * stride);
  }
  for (; kc < k1; kc += stride) {
    load(nxt, i1, kc + stride);
    i1 = i2;
    load_idx(i2, kc + 3 * stride);
    __builtin_amdgcn_sched_barrier(0);
    compute(cur, kc);
    __builtin_amdgcn_sched_barrier(0);
    cur = nxt;
  }
  // D = z^T P: register v of lane (i, g) in block (jb, c) is own column 16 jb + i of the tile,
  // right-hand side 16 c + drow(lane, v)
  auto emit = [&](int jb, const V4 (&blk)[NCB]) {
    const int jj = 16 * jb + i;
    if (jj >= h) return;
    const int64_t row = begin + j0 + jj;
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      if (slot >= 0) {
        store_cols<T, M>(part + ((int64_t)slot * TR + jj) * M, 16 * c, blk[c], false, kZero4<T>);
      } else {
        store_cols<T, M>(x + row * M, 16 * c, blk[c], false, kZero4<T>);
        if (W) store_cols_f64<T>(W + row * ldw, 16 * c, blk[c], mw);
      }
    }
  };
  if constexpr (NW > 1) {
    V4 blk[NCB];
    reduce_blocks<V4, NCB>(acc, blk, red, wave);
    emit(wave, blk);
  } else {
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) emit(jb, acc[jb]);
  }
}

template <typename T, int M, bool WIDE>
__global__ void __launch_bounds__(256) bwd_mfma_kernel(const int32_t* __restrict__ srcrows,
                                                       const int32_t* __restrict__ items, int64_t item_off,
                                                       int64_t count, const T* __restrict__ panel,
                                                       const T* __restrict__ yx, int64_t yx_rows,
                                                       T* __restrict__ x, double* W, int64_t ldw, int mw,
                                                       T* __restrict__ part) {
  typedef typename Mfma<T>::v4 V4;
  constexpr int NCB = (M + 15) / 16;
  constexpr int NW = solve_waves<T, WIDE>();
  __shared__ V4 red[(NW > 1 ? NW : 0) * 4 * NCB * 64 + 1];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t item = (NW > 1) ? blk : blk * 4 + wave;
  if (item >= count) return;
  bwd_tile<T, M, NW>(read_item(items, item_off + item), NW > 1 ? wave : 0, red, srcrows, panel, yx, yx_rows, x, W,
                     ldw, mw, part);
}

// ---------------------------------------------------------------------------
// Bottom subtrees: workgroup q runs subtree q level by level (forward: gather rows, then tile
// items, bottom-up; backward: tile items top-down), its waves sharing each level's work, with a
// workgroup barrier between levels instead of a launch.  Items are unsplit, one wave each.
// ---------------------------------------------------------------------------
constexpr int kSubWaves = 8;

template <typename T, int M>
__global__ void __launch_bounds__(64 * kSubWaves) fwd_subtree_kernel(
    const int32_t* __restrict__ gdst, const int32_t* __restrict__ gptr, const int32_t* __restrict__ gsrc,
    const int64_t* __restrict__ goff, const int32_t* __restrict__ items, const int64_t* __restrict__ ioff, int L,
    const T* __restrict__ panel, T* rhs, T* y, T* uvec) {
  constexpr int VW = 16 / sizeof(T);
  constexpr int LPR = M / VW;
  constexpr int RPW = 64 / LPR;
  const int q = blockIdx.x;
  const int lane = threadIdx.x % 64, wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  for (int l = 0; l < L; ++l) {
    const int64_t e = (int64_t)q * L + l;
    const int64_t g1 = goff[e + 1];
    for (int64_t base = goff[e] + (int64_t)wave * RPW; base < g1; base += kSubWaves * RPW) {
      const int64_t r = base + lane / LPR;
      if (r < g1) gather_row<T, M>(gdst, gptr, gsrc, r, (lane % LPR) * VW, rhs, uvec);
    }
    __syncthreads();
    const int64_t i1 = ioff[e + 1];
    for (int64_t it = ioff[e] + wave; it < i1; it += kSubWaves)
      fwd_tile<T, M, 1>(read_item(items, it), 0, nullptr, panel, rhs, y, uvec, y);   // unsplit: no partial tile
    __syncthreads();
  }
}

template <typename T, int M>
__global__ void __launch_bounds__(64 * kSubWaves) bwd_subtree_kernel(
    const int32_t* __restrict__ srcrows, const int32_t* __restrict__ items, const int64_t* __restrict__ ioff, int L,
    const T* __restrict__ panel, const T* __restrict__ yx, int64_t yx_rows, T* x, double* W, int64_t ldw, int mw) {
  const int q = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  for (int l = L - 1; l >= 0; --l) {
    const int64_t e = (int64_t)q * L + l;
    const int64_t i1 = ioff[e + 1];
    for (int64_t it = ioff[e] + wave; it < i1; it += kSubWaves)
      bwd_tile<T, M, 1>(read_item(items, it), 0, nullptr, srcrows, panel, yx, yx_rows, x, W, ldw, mw, x);   // unsplit
    __syncthreads();
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
    constexpr int rows_per_block = 4 * 64 / (M * (int)sizeof(T) / 16);
    if (a1 > a0)
      fwd_gather_kernel<T, M><<<(unsigned)((a1 - a0 + rows_per_block - 1) / rows_per_block), 256, 0, st>>>(
          Sd.gather_dst, Sd.gather_ptr, Sd.gather_src, a0, a1 - a0, rhs, uvec);
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
    // x follows y in one allocation: the backward operand z is read through one buffer resource
    const int64_t yx_rows = 2 * Sd.n;
    if (bn > 0 && Sd.bwd_wide[level])
      bwd_mfma_kernel<T, M, true><<<(unsigned)(solve_waves<T, true>() > 1 ? bn : (bn + 3) / 4), 256, 0, st>>>(
          Sd.bwd_src, Sd.bwd_items, b0, bn, panel, y, yx_rows, x, W, ldw, mw, bpart);
    else if (bn > 0)
      bwd_mfma_kernel<T, M, false><<<(unsigned)((bn + 3) / 4), 256, 0, st>>>(
          Sd.bwd_src, Sd.bwd_items, b0, bn, panel, y, yx_rows, x, W, ldw, mw, bpart);
    const int64_t g0 = Sd.bwd_fin_level_off[level], g1 = Sd.bwd_fin_level_off[level + 1];
    if (g1 > g0)
      bwd_fin_kernel<T, M><<<dim3((unsigned)(g1 - g0), TR * M / 256), 256, 0, st>>>(D, Sd.bwd_fin, g0, bpart, x, W,
                                                                                   ldw, mw);
  }
}

template <typename T, int M>
void precond_m(const FactorDev& D, const SolveDev& Sd, int nlevels, const T* panel, T* rhs, T* y, T* x, T* uvec,
               T* fpart, T* bpart, double* W, int64_t ldw, int mw, hipStream_t st) {
  const int L = (Sd.nsub > 0) ? Sd.sub_levels : 0;
  if (L > 0)
    fwd_subtree_kernel<T, M><<<(unsigned)Sd.nsub, 64 * kSubWaves, 0, st>>>(
        Sd.sub_gather_dst, Sd.sub_gather_ptr, Sd.sub_gather_src, Sd.sub_gather_off, Sd.sub_fwd_items, Sd.sub_fwd_off,
        L, panel, rhs, y, uvec);
  for (int l = L; l < nlevels; ++l)
    sweep_level<T, M>(D, Sd, l, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, true, st);
  for (int l = nlevels - 1; l >= L; --l)
    sweep_level<T, M>(D, Sd, l, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, false, st);
  if (L > 0)
    bwd_subtree_kernel<T, M><<<(unsigned)Sd.nsub, 64 * kSubWaves, 0, st>>>(
        Sd.bwd_src, Sd.sub_bwd_items, Sd.sub_bwd_off, L, panel, y, 2 * Sd.n, x, W, ldw, mw);
}

}  // namespace

template <typename T>
void launch_precond(const FactorDev& D, const SolveDev& Sd, int nlevels, int M, const T* panel, T* rhs, T* y, T* x,
                    T* uvec, T* fpart, T* bpart, double* W, int64_t ldw, int mw, hipStream_t st) {
  switch (M) {
    case 8: precond_m<T, 8>(D, Sd, nlevels, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, st); break;
    case 16: precond_m<T, 16>(D, Sd, nlevels, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, st); break;
    case 32: precond_m<T, 32>(D, Sd, nlevels, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, st); break;
    default: precond_m<T, 64>(D, Sd, nlevels, panel, rhs, y, x, uvec, fpart, bpart, W, ldw, mw, st); break;
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
