// Instance-segmented FP64 block kernels.  A batch of B independent problems is
// stored as one tall block whose rows [inst_off[b], inst_off[b+1]) belong to
// instance b (one instance is the case B = 1).  Row tiles and reduction
// chunks never straddle instances; per-instance small matrices sit at fixed
// strides; instances whose active flag is 0 are skipped.
//   gram      G_b = X_b^T Y_b          (deterministic two-stage reduction)
//   update    Y_b = alpha X_b M_b + beta Y_b
//   residual  R_b = AX_b - X_b diag(theta_b), lower(R) to the solve buffer, column norms
//   colnorms  ||X_b(:, j)||^2
//   trsm      Y_b U_b = X_b row by row (Algorithm 2 steps 2 and 4)
//   tsqr      R factor of each X_b (Algorithm 2 step 1), Householder in T
#include <algorithm>

#include "common.hpp"
#include "mfma.hpp"
#include "bufload.hpp"

namespace lobpcg {

namespace {

constexpr int kThreads = 256;

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Gram partials over one chunk of rows with FP64 matrix cores: the (32 RB) x (32 CB) output tile
// is split 2 x 2 over the four waves, each wave RB x CB blocks of 16 x 16 accumulated by
// v_mfma_f64_16x16x4f64 over 4 rows at a time.  Lane (i, g) = (l % 16, l / 16) reads row r + g,
// columns 16 b + i, of X and Y directly (16 consecutive doubles per row and lane group); the loads
// of the next rows are in flight while the current ones are multiplied.
// ---------------------------------------------------------------------------
template <int RB, int CB, typename TI>
__global__ void __launch_bounds__(kThreads) sgram_partial_kernel(SegDev S, const TI* __restrict__ X, int64_t ldx,
                                                                 const TI* __restrict__ Y, int64_t ldy, int c1,
                                                                 int c2, int tiles_j, double* __restrict__ part) {
  typedef Mfma<TI> MF;
  typedef typename MF::v4 V4;
  constexpr int T1 = 32 * RB, T2 = 32 * CB;
  const int q = blockIdx.x;
  const int b = S.chunk_inst[q];
  if (!S.active[b]) return;
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int i = lane % 16, g = lane / 16;
  const int ti = blockIdx.y / tiles_j, tj = blockIdx.y % tiles_j;
  const int ci0 = ti * T1 + (w / 2) * 16 * RB;   // first X column of this wave
  const int cj0 = tj * T2 + (w % 2) * 16 * CB;   // first Y column of this wave
  const int64_t rbeg = S.chunk_r0[q];
  V4 acc[RB][CB];
#pragma unroll
  for (int u = 0; u < RB; ++u)
#pragma unroll
    for (int v = 0; v < CB; ++v) acc[u][v] = V4{0, 0, 0, 0};
  // Buffer loads over the chunk: a row past the chunk reads zero by the resource's range, a column past
  // c1 (c2) by an out-of-range offset, so every load is issued unconditionally.  The row step is the
  // wave-uniform offset; the loads of the next rows are issued before the current ones are multiplied.
  // Groups of 32 rows where the registers allow (FP32, or few columns), else 16.
  constexpr int U = (RB + CB <= 2 || sizeof(TI) == 4) ? 8 : 4;
  constexpr int64_t SZ = sizeof(TI);
  const int nrows = S.chunk_rows[q];
  const i32x4_t xr = make_rsrc(X + rbeg * ldx, (int64_t)nrows * ldx * SZ);
  const i32x4_t yr = make_rsrc(Y + rbeg * ldy, (int64_t)nrows * ldy * SZ);
  int32_t xo[U][RB], yo[U][CB];
#pragma unroll
  for (int s = 0; s < U; ++s) {
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      const int col = ci0 + 16 * u + i;
      xo[s][u] = col < c1 ? (int32_t)(((4 * s + g) * ldx + col) * SZ) : kOob;
    }
#pragma unroll
    for (int v = 0; v < CB; ++v) {
      const int col = cj0 + 16 * v + i;
      yo[s][v] = col < c2 ? (int32_t)(((4 * s + g) * ldy + col) * SZ) : kOob;
    }
  }
  const int32_t xstep = (int32_t)(4 * U * ldx * SZ), ystep = (int32_t)(4 * U * ldy * SZ);
  auto load_group = [&](int32_t xs, int32_t ys, TI (&xd)[U][RB], TI (&yd)[U][CB]) {
#pragma unroll
    for (int s = 0; s < U; ++s) {
#pragma unroll
      for (int u = 0; u < RB; ++u) xd[s][u] = Buf<TI>::load1(xr, xo[s][u], xs);
#pragma unroll
      for (int v = 0; v < CB; ++v) yd[s][v] = Buf<TI>::load1(yr, yo[s][v], ys);
    }
  };
  auto mult_group = [&](const TI (&xd)[U][RB], const TI (&yd)[U][CB]) {
#pragma unroll
    for (int s = 0; s < U; ++s)
#pragma unroll
      for (int u = 0; u < RB; ++u)
#pragma unroll
        for (int v = 0; v < CB; ++v) acc[u][v] = MF::op(xd[s][u], yd[s][v], acc[u][v]);
  };
  // Two register groups in turn (no copies between them, so no load is waited for early); groups past
  // the chunk read zeros.
  TI xa[U][RB], yb[U][CB], xn[U][RB], yn[U][CB];
  load_group(0, 0, xa, yb);
  int32_t xs = 0, ys = 0;
  for (int r = 0; r < nrows; r += 8 * U) {
    load_group(xs + xstep, ys + ystep, xn, yn);
    mult_group(xa, yb);
    xs += 2 * xstep;
    ys += 2 * ystep;
    load_group(xs, ys, xa, yb);
    mult_group(xn, yn);
  }
  double* P = part + (int64_t)q * c1 * c2;
#pragma unroll
  for (int u = 0; u < RB; ++u)
#pragma unroll
    for (int v = 0; v < CB; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = ci0 + 16 * u + MF::drow(lane, e);
        const int gj = cj0 + 16 * v + i;
        if (gi < c1 && gj < c2) P[gi * c2 + gj] = (double)acc[u][v][e];
      }
}

// out_b[e] = sum over the chunks of instance b of part[chunk][e]: a block takes 16 elements, its 16
// thread groups every 16th chunk each with four independent partial sums (so that loads overlap),
// and the 64 partial sums of an element are combined in a fixed order (deterministic).
constexpr int kRedElems = 16, kRedGroups = 16;
__global__ void __launch_bounds__(256) sreduce_kernel(SegDev S, const double* __restrict__ part, int len,
                                                      double* __restrict__ out, int64_t ostride) {
  __shared__ double red[kRedGroups][kRedElems];
  const int b = blockIdx.y;
  if (!S.active[b]) return;
  const int g = threadIdx.x / kRedElems, l = threadIdx.x % kRedElems;
  const int e = blockIdx.x * kRedElems + l;
  const int q0 = S.inst_chunk_off[b], q1 = S.inst_chunk_off[b + 1];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < len) {
    int q = q0 + g;
    for (; q + 3 * kRedGroups < q1; q += 4 * kRedGroups) {
      s0 += part[(int64_t)q * len + e];
      s1 += part[(int64_t)(q + kRedGroups) * len + e];
      s2 += part[(int64_t)(q + 2 * kRedGroups) * len + e];
      s3 += part[(int64_t)(q + 3 * kRedGroups) * len + e];
    }
    for (; q < q1; q += kRedGroups) s0 += part[(int64_t)q * len + e];
  }
  red[g][l] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (g == 0 && e < len) {
    double t = 0.0;
#pragma unroll
    for (int h = 0; h < kRedGroups; ++h) t += red[h][l];
    out[(int64_t)b * ostride + e] = t;
  }
}

// ---------------------------------------------------------------------------
// Block update on one 64-row tile: Y = alpha X M_b + beta Y (64 x 64 output tile) in the blocks'
// precision TX (M is FP64 and rounded to TX).  X (64 rows x 32 reduction columns) and M (32 x 64) are
// staged through LDS, the next 32 columns loaded into registers (8 consecutive elements per thread,
// 16-byte loads when the rows allow) while the current ones are multiplied; wave w accumulates output
// rows 16 w .. 16 w + 15 over all four 16-column blocks with 16x16x4 MFMAs in TX.
// ---------------------------------------------------------------------------
constexpr int kUpdK = 32;
template <typename TX>
__global__ void __launch_bounds__(kThreads) supdate_kernel(SegDev S, const TX* X, int64_t ldx,
                                                           const double* __restrict__ M, int64_t ldm, int64_t mstride,
                                                           TX* Y, int64_t ldy, int K, int cols, double alpha,
                                                           double beta, bool vec) {
  typedef Mfma<TX> MF;
  typedef typename MF::v4 V4;
  __shared__ TX As[kUpdK][65];   // As[k][row]
  __shared__ TX Bs[kUpdK][65];   // Bs[k][col]
  const int q = blockIdx.x;
  const int b = S.tile_inst[q];
  if (!S.active[b]) return;
  const int64_t r0 = S.tile_r0[q];
  const int rows = S.tile_rows[q];
  const double* Mb = M + (int64_t)b * mstride;
  const int t = threadIdx.x;
  const int lane = t % 64, w = t / 64;
  const int i = lane % 16, g = lane / 16;
  const int c0 = blockIdx.y * 64;
  V4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = V4{0, 0, 0, 0};
  const int lr = t / 4, lk = (t % 4) * 8;   // X loader: row lr, reduction columns lk .. lk + 7
  const int bk = t / 8, bc = (t % 8) * 8;   // M loader: reduction row bk, columns bc .. bc + 7
  const TX* xrow = X + (r0 + lr) * ldx;
  const bool rok = lr < rows;
  TX xa[8], mb[8];
  auto load = [&](int k0) {
    const int kx = k0 + lk;
    if (vec && rok && kx + 8 <= K) {
      if constexpr (sizeof(TX) == 8) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const f64x2_t v = *reinterpret_cast<const f64x2_t*>(xrow + kx + 2 * u);
          xa[2 * u] = v.x;
          xa[2 * u + 1] = v.y;
        }
      } else {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const f32x4_t v = *reinterpret_cast<const f32x4_t*>(xrow + kx + 4 * u);
          xa[4 * u] = v.x; xa[4 * u + 1] = v.y; xa[4 * u + 2] = v.z; xa[4 * u + 3] = v.w;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < 8; ++u) xa[u] = (rok && kx + u < K) ? xrow[kx + u] : (TX)0;
    }
    const int kb = k0 + bk;
    // clamped addresses, so that the loads are unconditional (issued together) and masked afterwards
    const int kbc = min(kb, K - 1);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int cc = c0 + bc + u;
      const double v = Mb[(int64_t)kbc * ldm + min(cc, cols - 1)];
      mb[u] = (kb < K && cc < cols) ? (TX)v : (TX)0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < K; k0 += kUpdK) {
    __syncthreads();   // the previous chunk's products are done with As, Bs
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      As[lk + u][lr] = xa[u];
      Bs[bk][bc + u] = mb[u];
    }
    __syncthreads();
    if (k0 + kUpdK < K) load(k0 + kUpdK);
    const int kc = min(kUpdK, K - k0);   // columns past it are zero in both operands
    for (int kk = 0; kk < kc; kk += 4) {
      const TX av = As[kk + g][16 * w + i];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = MF::op(av, Bs[kk + g][16 * cb + i], acc[cb]);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * w + MF::drow(lane, e);
      const int cc = c0 + 16 * cb + i;
      if (r >= rows || cc >= cols) continue;
      TX v = (TX)alpha * acc[cb][e];
      if (beta != 0.0) v = fma((TX)beta, Y[(r0 + r) * ldy + cc], v);
      Y[(r0 + r) * ldy + cc] = v;
    }
}

// The same update with M staged once per workgroup, for K <= kUpdMaxK: the 16 NCB-column slice of M_b
// (rounded to TX) sits in LDS column-major, Ms[c][k], and each workgroup walks 64-row tiles with a grid
// stride, staging M again only when the instance changes.  Wave w takes tile rows 16 w .. 16 w + 15 with
// no barriers: for every 16 reduction columns lane (i, g) loads its row's columns 16 kb + 4 g .. + 3 (one
// 16-byte load in FP32) and uses them as the B operand of four MFMAs whose k-index is that column (the
// order of the reduction index is free as long as both operands follow it); the A operand is M^T, read
// as 4 consecutive k from Ms.  D = M^T X^T, so lane (i, g) ends with row i and 4 consecutive columns of
// each 16-column block (in FP64 the A operand takes the columns in the order ci = 4 (i % 4) + i / 4 to
// make them consecutive), written as 16-byte vectors.
//
// A pair launch (gridDim.z = 2) applies the same M to a second pair of blocks (X2, Y2) in its z = 1 half.
//
// GRAM = true (FP64, one instance, K <= kGramMaxK, K % 4 == 0, cols = 16 NCB, beta = 1): the workgroup
// also accumulates X(:, 0:K)^T Y_new over its tiles, for the next Gram-Schmidt pass, without reading X
// and Y again from memory: each wave puts its 16 new rows of Y in LDS (zeros past the tile) and runs
// 16 x 16 x 4 products with X's rows (re-read, cache-resident) as the A operand and the LDS rows as B;
// after the last tile the four waves' sums are added in LDS in wave order and the workgroup writes
// its K x cols partial to gpart[blockIdx.x] (deterministic for a fixed grid).
constexpr int kUpdMaxK = 96;
constexpr int kGramMaxK = 64;
template <typename TX, int NCB, bool GRAM = false>
__global__ void __launch_bounds__(kThreads) supdate_ms_kernel(SegDev S, const TX* X, int64_t ldx,
                                                              const double* __restrict__ M, int64_t ldm,
                                                              int64_t mstride, TX* Y, int64_t ldy, int K, int cols,
                                                              double alpha, double beta,
                                                              double* __restrict__ gpart = nullptr,
                                                              const TX* X2 = nullptr, TX* Y2 = nullptr) {
  typedef Mfma<TX> MF;
  typedef typename MF::v4 V4;
  constexpr int LK = kUpdMaxK + 4;   // 16-byte aligned rows; consecutive rows start 4 banks apart
  constexpr int NKB = kUpdMaxK / 16;
  constexpr int VW = 16 / sizeof(TX);
  constexpr int NAB = kGramMaxK / 16;
  if (blockIdx.z == 1) {   // the second product of a pair launch: same M, other blocks
    X = X2;
    Y = Y2;
  }
  constexpr int WP = 16 * NCB + 2;   // LDS pitch of the new rows (16-byte aligned rows)
  static_assert(!GRAM || sizeof(TX) == 8, "the fused Gram is FP64");
  static_assert(!GRAM || kGramMaxK * 16 * NCB <= 16 * NCB * LK, "the Gram partial must fit in Ms");
  __shared__ __align__(16) TX Ms[16 * NCB][LK];
  __shared__ __align__(16) TX Wl[GRAM ? 4 : 1][GRAM ? 16 : 1][GRAM ? WP : 1];
  V4 acc2[GRAM ? NAB : 1][GRAM ? NCB : 1];
  if constexpr (GRAM) {
#pragma unroll
    for (int ab = 0; ab < NAB; ++ab)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc2[ab][cb] = V4{0, 0, 0, 0};
  }
  const int t = threadIdx.x, lane = t % 64, w = t / 64;
  const int i = lane % 16, g = lane / 16;
  const int ci = (sizeof(TX) == 8) ? 4 * (i % 4) + i / 4 : i;
  const int c0 = blockIdx.y * 16 * NCB;
  const int nkb = (K + 15) / 16;
  const TX al = (TX)alpha, be = (TX)beta;
  int cur = -1;
  for (int64_t q = blockIdx.x; q < S.ntiles; q += gridDim.x) {
    // tile fields are uniform: in scalar registers, buffer resources need no per-lane loop
    const int b = __builtin_amdgcn_readfirstlane(S.tile_inst[q]);
    if (!S.active[b]) continue;   // uniform
    const int64_t r0t = S.tile_r0[q];
    const int64_t r0 = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)r0t) |
                       ((int64_t)__builtin_amdgcn_readfirstlane((int)(r0t >> 32)) << 32);
    const int rows = __builtin_amdgcn_readfirstlane(S.tile_rows[q]);
    const int r = 16 * w + i;
    const bool rok = r < rows;
    if (b != cur) {   // uniform
      __syncthreads();   // the previous instance's products are done with Ms
      const double* Mb = M + (int64_t)b * mstride;
      // unconditional buffer loads (out-of-range offsets read zeros), all issued before the LDS stores
      const i32x4_t mrs = make_rsrc(Mb, ((int64_t)(K - 1) * ldm + cols) * (int64_t)sizeof(double));
      constexpr int NE = 16 * NCB * kUpdMaxK / kThreads;
      double mt[NE];
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = t + kThreads * u, k = e / (16 * NCB), c = e % (16 * NCB);
        const bool ok = k < K && c0 + c < cols;
        mt[u] = Buf<double>::load1(mrs, ok ? (int32_t)(((int64_t)k * ldm + c0 + c) * (int64_t)sizeof(double)) : kOob, 0);
      }
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const int e = t + kThreads * u;
        Ms[e % (16 * NCB)][e / (16 * NCB)] = (TX)mt[u];
      }
      __syncthreads();
      cur = b;
    }
    // this tile's rows: unconditional buffer loads, zeros past the tile's rows and past K
    TX xv[NKB][4];
    const i32x4_t xrs = make_rsrc(X + r0 * ldx, (int64_t)rows * ldx * (int64_t)sizeof(TX));
    // per-lane part of the offset in the VGPR (row, the lane group's 4 columns), uniform part in the SGPR
    const int32_t xoff = (int32_t)(((int64_t)r * ldx + 4 * g) * (int64_t)sizeof(TX));
    if ((K & 3) == 0) {   // uniform: every group of four columns is whole or past K
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        const int32_t v = (rok && kb < nkb && 16 * kb + 4 * g < K) ? xoff : kOob;
#pragma unroll
        for (int h = 0; h < 4 / VW; ++h) {
          TX q[VW];
          Buf<TX>::load16(xrs, v, 16 * kb * (int32_t)sizeof(TX) + 16 * h, q);
#pragma unroll
          for (int u = 0; u < VW; ++u) xv[kb][VW * h + u] = q[u];
        }
      }
    } else {
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          xv[kb][u] = Buf<TX>::load1(xrs, (rok && 16 * kb + 4 * g + u < K) ? xoff + u * (int32_t)sizeof(TX) : kOob,
                                     16 * kb * (int32_t)sizeof(TX));
    }
    V4 acc[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) acc[cb] = V4{0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      if (kb >= nkb) break;   // uniform; Ms is zero past K
      TX mv[NCB][4];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const TX* src = &Ms[16 * cb + ci][16 * kb + 4 * g];
        if constexpr (sizeof(TX) == 4) {
          const f32x4_t v = *reinterpret_cast<const f32x4_t*>(src);
          mv[cb][0] = v.x; mv[cb][1] = v.y; mv[cb][2] = v.z; mv[cb][3] = v.w;
        } else {
          const f64x2_t v0 = *reinterpret_cast<const f64x2_t*>(src), v1 = *reinterpret_cast<const f64x2_t*>(src + 2);
          mv[cb][0] = v0.x; mv[cb][1] = v0.y; mv[cb][2] = v1.x; mv[cb][3] = v1.y;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[cb] = MF::op(mv[cb][u], xv[kb][u], acc[cb]);
    }
    if constexpr (GRAM) {
      TX* yr = Y + (r0 + r) * ldy;
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        const int c = 16 * cb + 4 * g;
        f64x2_t o0 = {0.0, 0.0}, o1 = {0.0, 0.0};
        if (rok) {
          f64x2_t* d = reinterpret_cast<f64x2_t*>(yr + c);
          const f64x2_t y0 = d[0], y1 = d[1];
          o0 = f64x2_t{fma(be, y0.x, al * acc[cb][0]), fma(be, y0.y, al * acc[cb][1])};
          o1 = f64x2_t{fma(be, y1.x, al * acc[cb][2]), fma(be, y1.y, al * acc[cb][3])};
          d[0] = o0;
          d[1] = o1;
        }
        *reinterpret_cast<f64x2_t*>(&Wl[w][i][c]) = o0;
        *reinterpret_cast<f64x2_t*>(&Wl[w][i][c + 2]) = o1;
      }
      __builtin_amdgcn_wave_barrier();   // the wave's LDS rows are read back by other lanes of the wave
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int rr = 16 * w + 4 * s4 + g;   // rows past the tile read zeros (resource range)
        double xa[NAB], wb[NCB];
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab)
          xa[ab] = Buf<double>::load1(xrs, (16 * ab + i < K) ? (int32_t)(((int64_t)rr * ldx + 16 * ab + i) * 8) : kOob, 0);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) wb[cb] = Wl[w][4 * s4 + g][16 * cb + i];
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb) acc2[ab][cb] = MF::op(xa[ab], wb[cb], acc2[ab][cb]);
      }
      __builtin_amdgcn_wave_barrier();
      continue;
    }
    if (!rok) continue;
    TX* yr = Y + (r0 + r) * ldy;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int c = c0 + 16 * cb + 4 * g;   // register v holds column c + v
      if (c >= cols) continue;
      TX v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = al * acc[cb][u];
      if (c + 3 < cols) {
        if constexpr (sizeof(TX) == 4) {
          f32x4_t* d = reinterpret_cast<f32x4_t*>(yr + c);
          f32x4_t o = {v[0], v[1], v[2], v[3]};
          if (beta != 0.0) {
            const f32x4_t y = *d;
            o = f32x4_t{fmaf(be, y.x, v[0]), fmaf(be, y.y, v[1]), fmaf(be, y.z, v[2]), fmaf(be, y.w, v[3])};
          }
          *d = o;
        } else {
          f64x2_t* d = reinterpret_cast<f64x2_t*>(yr + c);
          f64x2_t o0 = {v[0], v[1]}, o1 = {v[2], v[3]};
          if (beta != 0.0) {
            const f64x2_t y0 = d[0], y1 = d[1];
            o0 = f64x2_t{fma(be, y0.x, v[0]), fma(be, y0.y, v[1])};
            o1 = f64x2_t{fma(be, y1.x, v[2]), fma(be, y1.y, v[3])};
          }
          d[0] = o0;
          d[1] = o1;
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (c + u < cols) yr[c + u] = (beta != 0.0) ? fma(be, yr[c + u], v[u]) : v[u];
      }
    }
  }
  if constexpr (GRAM) {
    // sum of the four waves' partials in wave order (Ms is free: every product is done after the barrier)
    constexpr int NC = 16 * NCB;
    TX* red = &Ms[0][0];
    __syncthreads();
#pragma unroll 1
    for (int ww = 0; ww < 4; ++ww) {
      if (w == ww) {
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab)
#pragma unroll
          for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int idx = (16 * ab + MF::drow(lane, e)) * NC + 16 * cb + i;
              red[idx] = (ww == 0) ? acc2[ab][cb][e] : red[idx] + acc2[ab][cb][e];
            }
      }
      __syncthreads();
    }
    double* P = gpart + (int64_t)blockIdx.x * K * NC;
    for (int e = t; e < K * NC; e += kThreads) P[e] = red[e];
  }
}

// out[e] = sum over p < nparts of part[p][e] (len elements each), in a fixed order: as sreduce_kernel, a
// block takes 16 elements and its 16 thread groups every 16th partial with four independent sums.
__global__ void __launch_bounds__(256) preduce_kernel(const double* __restrict__ part, int nparts, int len,
                                                      double* __restrict__ out) {
  __shared__ double red[kRedGroups][kRedElems];
  const int g = threadIdx.x / kRedElems, l = threadIdx.x % kRedElems;
  const int e = blockIdx.x * kRedElems + l;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < len) {
    int q = g;
    for (; q + 3 * kRedGroups < nparts; q += 4 * kRedGroups) {
      s0 += part[(int64_t)q * len + e];
      s1 += part[(int64_t)(q + kRedGroups) * len + e];
      s2 += part[(int64_t)(q + 2 * kRedGroups) * len + e];
      s3 += part[(int64_t)(q + 3 * kRedGroups) * len + e];
    }
    for (; q < nparts; q += kRedGroups) s0 += part[(int64_t)q * len + e];
  }
  red[g][l] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (g == 0 && e < len) {
    double t = 0.0;
#pragma unroll
    for (int h = 0; h < kRedGroups; ++h) t += red[h][l];
    out[e] = t;
  }
}

// ---------------------------------------------------------------------------
// Residual over one chunk: R = AX - X diag(theta_b) (cast to T), partial column sums of squares.
// ---------------------------------------------------------------------------
template <typename T, typename TI>
__global__ void __launch_bounds__(kThreads) sresidual_kernel(SegDev S, const TI* __restrict__ AX, int64_t ldax,
                                                             const TI* __restrict__ X, int64_t ldx,
                                                             const double* __restrict__ theta, int64_t tstride,
                                                             int m, T* __restrict__ R, int64_t ldr,
                                                             double* __restrict__ part) {
  __shared__ double red[2][4][64];
  const int q = blockIdx.x;
  const int b = S.chunk_inst[q];
  if (!S.active[b]) return;
  const int t = threadIdx.x;
  const int j = t % 64, g = t / 64;
  const int64_t rbeg = S.chunk_r0[q];
  const int64_t rend = rbeg + S.chunk_rows[q];
  double rs = 0.0, xs = 0.0;
  if (j < m) {
    const TI th = (TI)theta[(int64_t)b * tstride + j];
    for (int64_t r = rbeg + g; r < rend; r += 4) {
      const TI x = X[r * ldx + j];
      const TI v = AX[r * ldax + j] - x * th;
      R[r * ldr + j] = (T)v;
      rs = fma((double)v, (double)v, rs);
      xs = fma((double)x, (double)x, xs);
    }
  }
  red[0][g][j] = rs;
  red[1][g][j] = xs;
  __syncthreads();
  if (t < m) {
    part[(int64_t)q * 2 * m + t] = ((red[0][0][t] + red[0][1][t]) + red[0][2][t]) + red[0][3][t];
    part[(int64_t)q * 2 * m + m + t] = ((red[1][0][t] + red[1][1][t]) + red[1][2][t]) + red[1][3][t];
  }
}

// The same residual with two columns per lane (16-byte loads of X and AX, 8-byte stores of R): a
// row is read by CPL = m / 2 consecutive lanes, a wave covers 64 / CPL rows per step and four steps
// are loaded together.  Per-lane partial sums go through LDS and are added in a fixed order.
template <typename T, int CPL, typename TI>
__global__ void __launch_bounds__(kThreads) sresidual2_kernel(SegDev S, const TI* __restrict__ AX, int64_t ldax,
                                                              const TI* __restrict__ X, int64_t ldx,
                                                              const double* __restrict__ theta, int64_t tstride,
                                                              T* __restrict__ R, int64_t ldr,
                                                              double* __restrict__ part) {
  constexpr int M = 2 * CPL, RPW = 64 / CPL, RPB = 4 * RPW, U = 4;
  __shared__ double red[4][RPW][M][2];
  const int q = blockIdx.x;
  const int b = S.chunk_inst[q];
  if (!S.active[b]) return;
  const int t = threadIdx.x, lane = t % 64, w = t / 64;
  const int jp = lane % CPL, rl = lane / CPL;
  const int64_t rbeg = S.chunk_r0[q];
  const int64_t rend = rbeg + S.chunk_rows[q];
  typedef TI V2 __attribute__((ext_vector_type(2)));
  const TI th0 = (TI)theta[(int64_t)b * tstride + 2 * jp], th1 = (TI)theta[(int64_t)b * tstride + 2 * jp + 1];
  double rs0 = 0.0, rs1 = 0.0, xs0 = 0.0, xs1 = 0.0;
  for (int64_t r0 = rbeg + w * RPW + rl; r0 < rend; r0 += (int64_t)U * RPB) {
    V2 xv[U], av[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + (int64_t)u * RPB;
      if (r < rend) {
        xv[u] = *reinterpret_cast<const V2*>(X + r * ldx + 2 * jp);
        av[u] = *reinterpret_cast<const V2*>(AX + r * ldax + 2 * jp);
      } else {
        xv[u] = V2{0, 0};
        av[u] = V2{0, 0};
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = r0 + (int64_t)u * RPB;
      const TI v0 = av[u].x - xv[u].x * th0, v1 = av[u].y - xv[u].y * th1;
      if (r < rend) {
        R[r * ldr + 2 * jp] = (T)v0;
        R[r * ldr + 2 * jp + 1] = (T)v1;
      }
      rs0 = fma((double)v0, (double)v0, rs0);
      rs1 = fma((double)v1, (double)v1, rs1);
      xs0 = fma((double)xv[u].x, (double)xv[u].x, xs0);
      xs1 = fma((double)xv[u].y, (double)xv[u].y, xs1);
    }
  }
  red[w][rl][2 * jp][0] = rs0;
  red[w][rl][2 * jp + 1][0] = rs1;
  red[w][rl][2 * jp][1] = xs0;
  red[w][rl][2 * jp + 1][1] = xs1;
  __syncthreads();
  if (t < 2 * M) {
    const int j = t % M, k = t / M;
    double sum = 0.0;
    for (int ww = 0; ww < 4; ++ww)
      for (int g = 0; g < RPW; ++g) sum += red[ww][g][j][k];
    part[(int64_t)q * 2 * M + k * M + j] = sum;
  }
}

template <typename TI>
__global__ void __launch_bounds__(kThreads) scolnorm_kernel(SegDev S, const TI* __restrict__ X, int64_t ldx,
                                                            int c, double* __restrict__ part) {
  __shared__ double red[4][64];
  const int q = blockIdx.x;
  const int b = S.chunk_inst[q];
  if (!S.active[b]) return;
  const int t = threadIdx.x;
  const int j = t % 64, g = t / 64;
  const int64_t rbeg = S.chunk_r0[q];
  const int64_t rend = rbeg + S.chunk_rows[q];
  double xs = 0.0;
  if (j < c)
    for (int64_t r = rbeg + g; r < rend; r += 4) {
      const double x = (double)X[r * ldx + j];
      xs = fma(x, x, xs);
    }
  red[g][j] = xs;
  __syncthreads();
  if (t < c) part[(int64_t)q * c + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// ---------------------------------------------------------------------------
// Row-wise triangular solve on one 64-row tile: W_b <- W_b U_b^{-1}.
// ---------------------------------------------------------------------------
template <typename TU, typename TW>
__global__ void __launch_bounds__(64) strsm_rows_kernel(SegDev S, TW* W, int64_t ld, int c,
                                                        const TU* __restrict__ U, int64_t ustride) {
  extern __shared__ double smem[];
  double* Us = smem;            // c x c
  double* Ws = smem + c * c;    // c x 64, column-major per thread row
  const int q = blockIdx.x;
  const int b = S.tile_inst[q];
  if (!S.active[b]) return;
  const int64_t r0 = S.tile_r0[q];
  const int rows = S.tile_rows[q];
  const TU* Ub = U + (int64_t)b * ustride;
  const int t = threadIdx.x;
  for (int e = t; e < c * c; e += 64) Us[e] = (double)Ub[e];
  // eight reads in flight per batch (clamped rows, masked afterwards), then their LDS stores
  for (int e0 = 0; e0 < 64 * c; e0 += 8 * 64) {
    double v[8];
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int e = min(e0 + h * 64 + t, 64 * c - 1), i = e / c, j = e % c;
      v[h] = keep_if(i < rows, (double)W[(r0 + min(i, rows - 1)) * ld + j]);
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int e = e0 + h * 64 + t;
      if (e < 64 * c) Ws[(e % c) * 64 + e / c] = v[h];
    }
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
    if (i < rows) W[(r0 + i) * ld + j] = (TW)Ws[j * 64 + i];
  }
}

// The same solve for c == CP columns with the row in registers (fully unrolled), one row per
// thread.  The tile moves between memory and LDS in consecutive 16-byte pieces (whole rows per
// instruction, so each cache line is requested once, where one row per lane would touch 64 lines
// per instruction) and each thread takes its row from LDS; LDS rows are padded by 16 bytes so that
// the row reads and the piece writes both spread over the banks.  While the rows are in registers
// the same LDS holds U_b in the blocks' precision with reciprocal diagonal entries, read by all lanes
// at once (broadcast) as the solve proceeds.  Arithmetic in FP64 for FP64 blocks, in the blocks'
// precision otherwise.
template <typename TU, int CP, typename TW>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) strsm_rows_reg_kernel(SegDev S, TW* W, int64_t ld,
                                                            const TU* __restrict__ U, int64_t ustride) {
  constexpr int VW = 16 / sizeof(TW);     // elements per 16-byte piece
  constexpr int PPR = CP / VW;            // pieces per row
  constexpr int PITCH = CP + VW;          // LDS row pitch (elements)
  constexpr int NP = PPR;                 // pieces per lane (64 rows x PPR pieces / 64 lanes)
  constexpr int NU = CP * CP / 64;        // elements of U_b per lane
  static_assert(CP * CP <= 64 * PITCH, "U_b must fit in the tile's LDS");
  __shared__ __align__(16) TW Ws[64 * PITCH];
  const int q = blockIdx.x;
  const int b = S.tile_inst[q];
  if (!S.active[b]) return;
  const int64_t r0 = S.tile_r0[q];
  const int rows = S.tile_rows[q];
  const TU* Ub = U + (int64_t)b * ustride;
  const int t = threadIdx.x;
  TW* tile = W + r0 * ld;
  // Buffer accesses over the tile's rows: rows past it read zeros and their stores are dropped, so
  // every access is issued unconditionally (64 ld elements stay below 2^31 bytes: ld < 2^22).
  const i32x4_t rs = make_rsrc(tile, (int64_t)rows * ld * (int64_t)sizeof(TW));
  // 16-byte pieces when the tile's rows allow (uniform), else element by element
  const bool vec = ((reinterpret_cast<uintptr_t>(tile) | (uintptr_t)(ld * sizeof(TW))) % 16) == 0;
  auto voff = [&](int r, int k) { return (int32_t)(((int64_t)r * ld + k) * (int64_t)sizeof(TW)); };
  // U_b's reads are issued with the tile's (for CP = 64 after the rows are in registers, which would
  // otherwise hold both at once)
  TU u[NU];
  if constexpr (CP < 64) {
#pragma unroll
    for (int s = 0; s < NU; ++s) u[s] = Ub[s * 64 + t];
  }
  if (vec) {
    TW v[NP][VW];
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int e = s * 64 + t;
      Buf<TW>::load16(rs, voff(e / PPR, (e % PPR) * VW), 0, v[s]);
    }
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int e = s * 64 + t;
#pragma unroll
      for (int h = 0; h < VW; ++h) Ws[(e / PPR) * PITCH + (e % PPR) * VW + h] = v[s][h];
    }
  } else {
    TW v[CP];
#pragma unroll
    for (int s = 0; s < CP; ++s) {
      const int e = s * 64 + t;
      v[s] = Buf<TW>::load1(rs, voff(e / CP, e % CP), 0);
    }
#pragma unroll
    for (int s = 0; s < CP; ++s) {
      const int e = s * 64 + t;
      Ws[(e / CP) * PITCH + e % CP] = v[s];
    }
  }
  __syncthreads();
  TW x[CP];
#pragma unroll
  for (int k = 0; k < CP; ++k) x[k] = Ws[t * PITCH + k];
  if constexpr (CP >= 64) {
#pragma unroll
    for (int s = 0; s < NU; ++s) u[s] = Ub[s * 64 + t];
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NU; ++s) {
    const int e = s * 64 + t;
    const TW w = (TW)u[s];
    Ws[e] = (e / CP == e % CP) ? (TW)1 / w : w;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < CP; ++j) {
    x[j] *= Ws[j * CP + j];
#pragma unroll
    for (int k = j + 1; k < CP; ++k) x[k] -= x[j] * Ws[j * CP + k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < CP; ++k) Ws[t * PITCH + k] = x[k];
  __syncthreads();
  if (vec) {
    TW v[NP][VW];
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int e = s * 64 + t;
#pragma unroll
      for (int h = 0; h < VW; ++h) v[s][h] = Ws[(e / PPR) * PITCH + (e % PPR) * VW + h];
    }
#pragma unroll
    for (int s = 0; s < NP; ++s) {
      const int e = s * 64 + t;
      Buf<TW>::store16(rs, voff(e / PPR, (e % PPR) * VW), 0, v[s]);
    }
  } else {
    TW v[CP];
#pragma unroll
    for (int s = 0; s < CP; ++s) {
      const int e = s * 64 + t;
      v[s] = Ws[(e / CP) * PITCH + e % CP];
    }
#pragma unroll
    for (int s = 0; s < CP; ++s) {
      const int e = s * 64 + t;
      Buf<TW>::store1(rs, voff(e / CP, e % CP), 0, v[s]);
    }
  }
}

// ---------------------------------------------------------------------------
// TSQR block: Householder QR (R only) of a block of at most NR rows starting at `in`.
// The block is held column-major in LDS (A[k][t], row t = thread t).  For column j one pass
// gives every sum the step needs, S_k = sum_{t > j} a_tj a_tk for k >= j (S_j is the squared
// norm below the diagonal), each column pair summed by NR / CP threads and a shuffle; with
// v = e_j + scale * a(j+1:, j), w_k = v^T a(:, k) = a_jk + scale S_k, and thread t then
// updates its own row.
// ---------------------------------------------------------------------------
constexpr int kTsqrRows = 256;
constexpr int kTsqrRowsWide = 1024;   // FP32 blocks of the upper levels (stacked R factors), c <= 32
constexpr int kTsqrCombineRpl = kTsqrCombineRows / 64;   // rows per lane of the leaves of combining plans

template <typename T, typename Tin, int CP, int NR = kTsqrRows>
__global__ void __launch_bounds__(NR) stsqr_kernel(SegDev S, const Tin* in, int64_t ldin,
                                                   const int32_t* __restrict__ items, int c, T* out) {
  constexpr int PARTS = NR / CP;        // threads per column sum
  constexpr int LP = NR + 8;            // padded LDS column (columns of a sum group in other banks)
  __shared__ T A[CP * LP];              // A[k * LP + t] = element (t, k)
  __shared__ T sk[CP];                  // S_k
  const int* it = items + 4 * blockIdx.x;   // {instance, first row, rows, output slot}
  const int b = it[0];
  if (!S.active[b]) return;
  const int64_t r0 = it[1];
  const int rows = it[2];
  const int slot = it[3];
  const int t = threadIdx.x;
  for (int k = 0; k < c; ++k) A[k * LP + t] = (t < rows) ? (T)in[(r0 + t) * ldin + k] : (T)0;
  __syncthreads();
  const int kmax = (c < rows) ? c : rows;
  const int sk_k = t / PARTS, sk_part = t % PARTS;
  for (int j = 0; j < kmax; ++j) {
    // S_k for k >= j over the rows below the diagonal (the PARTS threads of a column are
    // consecutive lanes of one wave)
    if (sk_k >= j && sk_k < c) {
      // part p sums rows p, p + PARTS, ...: the lanes of a column read consecutive words
      const T* cj = A + j * LP + sk_part;
      const T* ck = A + sk_k * LP + sk_part;
      T x[CP], y[CP];
#pragma unroll
      for (int q = 0; q < CP; ++q) {
        x[q] = cj[q * PARTS];
        y[q] = ck[q * PARTS];
      }
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int q = 0; q < CP; q += 2) {
        s0 += (sk_part + q * PARTS > j) ? x[q] * y[q] : (T)0;
        s1 += (sk_part + (q + 1) * PARTS > j) ? x[q + 1] * y[q + 1] : (T)0;
      }
      T sum = s0 + s1;
#pragma unroll
      for (int off = PARTS / 2; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
      if (sk_part == 0) sk[sk_k] = sum;
    }
    __syncthreads();
    const T sigma = sk[j];
    if (sigma > (T)0) {   // otherwise nothing below the diagonal: H_j = I (uniform)
      const T alpha = A[j * LP + j];
      const T xn = sqrt(alpha * alpha + sigma);
      const T beta = (alpha >= (T)0) ? -xn : xn;
      const T tau = (beta - alpha) / beta;
      const T scale = (T)1 / (alpha - beta);
      if (t > j) {
        const T tv = tau * scale * A[j * LP + t];
        // loads of 8 columns first, then the stores (the compiler cannot reorder them itself)
        for (int k0 = j + 1; k0 < c; k0 += 8) {
          T x[8], w[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int k = k0 + u < c ? k0 + u : c - 1;
            x[u] = A[k * LP + t];
            w[u] = A[k * LP + j] + scale * sk[k];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (k0 + u < c) A[(k0 + u) * LP + t] = x[u] - tv * w[u];
        }
      }
      __syncthreads();   // every thread has read row j before it is updated
      // row j itself (v_j = 1): thread k updates element (j, k)
      if (t > j && t < c) A[t * LP + j] -= tau * (A[t * LP + j] + scale * sk[t]);
      if (t == j) A[j * LP + j] = beta;
    }
    __syncthreads();
  }
  T* R = out + (int64_t)slot * c * c;
  if (t < c)
    for (int k = 0; k < c; ++k) R[(int64_t)t * c + k] = (k >= t && t < rows) ? A[k * LP + t] : (T)0;
}

// Exchange with lane ^ M (M = 1, 2, 4, 8, 16) inside 32-lane halves: DPP moves for 1, 2 (quad
// permutes) and 8 (rotation by 8 inside a 16-lane row), swizzles in bit-mask mode for 4 and 16.
template <int M>
__device__ inline float lane_xor(float v) {
  const int x = __builtin_bit_cast(int, v);
  int y;
  if constexpr (M == 1) y = __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);        // quad_perm [1,0,3,2]
  else if constexpr (M == 2) y = __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  else if constexpr (M == 4) y = __builtin_amdgcn_ds_swizzle(x, 0x101F);                // and 31, xor 4
  else if constexpr (M == 8) y = __builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false);  // row_ror 8
  else y = __builtin_amdgcn_ds_swizzle(x, 0x401F);                                       // and 31, xor 16
  return __builtin_bit_cast(float, y);
}

// Sum over the 64 lanes of a wave of each of the N values q[0..N) (N <= 32), returned in out[] as
// wave-uniform values.  With P = 2^LOG >= N (the values padded with zeros), recursive halving over lane
// bits 0 .. LOG - 1: at the exchange on bit b a lane keeps half of its vector and adds the partner lane's
// copy of that half (P - 1 exchanges in all), the lane bits LOG .. 4 are summed directly, and value k then
// sits in the lanes whose low LOG bits are k's bit-reversal, as two halves (bit 5) added on extraction.
template <int N>
__device__ inline void wave_allreduce(const float (&qin)[N], float (&out)[N]) {
  constexpr int LOG = (N <= 1) ? 0 : (N <= 2) ? 1 : (N <= 4) ? 2 : (N <= 8) ? 3 : (N <= 16) ? 4 : 5;
  constexpr int P = 1 << LOG;
  static_assert(N <= 32, "at most 32 values");
  const int lane = threadIdx.x % 64;
  float q[P];
#pragma unroll
  for (int k = 0; k < P; ++k) q[k] = (k < N) ? qin[k] : 0.f;
  static_for<0, LOG>([&](auto S) {
    constexpr int st = decltype(S)::value, m = 1 << st, half = P >> (st + 1);
    // lane-dependent choice between q[i] and q[i + half] by bit masks (a select between two array
    // elements would be folded into a lane-dependent array index)
    const uint32_t hm = (lane & m) ? 0xffffffffu : 0u;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const uint32_t lo_b = __builtin_bit_cast(uint32_t, q[i]), hi_b = __builtin_bit_cast(uint32_t, q[i + half]);
      const float keep = __builtin_bit_cast(float, (hi_b & hm) | (lo_b & ~hm));
      const float send = __builtin_bit_cast(float, (lo_b & hm) | (hi_b & ~hm));
      q[i] = keep + lane_xor<m>(send);
    }
  });
  static_for<LOG, 5>([&](auto S) { q[0] += lane_xor<(1 << decltype(S)::value)>(q[0]); });
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int r = 0;   // bit-reversal of k over LOG bits
#pragma unroll
    for (int b = 0; b < LOG; ++b) r |= ((k >> b) & 1) << (LOG - 1 - b);
    out[k] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, q[0]), r)) +
             __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, q[0]), r + 32));
  }
}

__device__ inline float lane_value(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

__device__ inline double lane_f64(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// TSQR block in FP32 by one wave, four blocks per workgroup, no barriers: lane l holds rows l, l + 64,
// ..., l + 64 (RPL - 1) of the block (at most 64 RPL rows) in registers.  The column loop is unrolled,
// so step j touches only columns j .. CP - 1.  For column j the wave all-reduce gives
// sigma = sum_{r > j} a_rj^2 and S_k = sum_{r > j} a_rj a_rk together; with v = e_j + scale a(j+1:, j),
// w_k = a_jk + scale S_k and every row is updated in place.  Row j is final after step j (later
// reflectors leave rows above their own untouched), so lane j ends up holding row j of R (its
// diagonal kept aside as beta_j).
template <typename Tin, int CP, int RPL = 4>
__global__ void __launch_bounds__(256) stsqr_wave_kernel(SegDev S, const Tin* in, int64_t ldin,
                                                         const int32_t* __restrict__ items, int64_t nitems, int c,
                                                         float* out) {
  const int lane = threadIdx.x % 64, wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int64_t item = (int64_t)blockIdx.x * 4 + wv;
  if (item >= nitems) return;   // whole wave
  const int* it = items + 4 * item;   // {instance, first row, rows, output slot}
  const int b = it[0];
  if (!S.active[b]) return;
  const int64_t r0 = it[1];
  const int rows = it[2];
  const int slot = it[3];
  float a[RPL][CP];
  // loads from clamped addresses, masked afterwards: unconditional, so that they are all in flight
  // together; FP64 rows two columns per load when the rows allow
  bool pairs = false;
  if constexpr (sizeof(Tin) == 8)
    pairs = (c % 2 == 0) && ((reinterpret_cast<uintptr_t>(in) | (uintptr_t)(ldin * 8)) % 16 == 0);   // uniform
  if (pairs) {
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = 64 * s + lane;
      const Tin* src = in + (r0 + min(r, rows - 1)) * ldin;
#pragma unroll
      for (int kp = 0; kp < CP / 2; ++kp) {
        const f64x2_t v = *reinterpret_cast<const f64x2_t*>(src + 2 * min(kp, c / 2 - 1));
        a[s][2 * kp] = keep_if(r < rows && 2 * kp < c, (float)v.x);
        a[s][2 * kp + 1] = keep_if(r < rows && 2 * kp + 1 < c, (float)v.y);
      }
    }
  } else {
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const int r = 64 * s + lane;
      const Tin* src = in + (r0 + min(r, rows - 1)) * ldin;
#pragma unroll
      for (int k = 0; k < CP; ++k) a[s][k] = keep_if(r < rows && k < c, (float)src[min(k, c - 1)]);
    }
  }
  const int kmax = (c < rows) ? c : rows;
  float rjj = 0.f;
  static_for<0, CP>([&](auto J) {
    constexpr int j = decltype(J)::value;
    constexpr int N = CP - j;   // columns j .. CP - 1
    if (j >= kmax) return;      // uniform
    float q[N];
#pragma unroll
    for (int k = 0; k < N; ++k) q[k] = 0.f;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const float x = (64 * s + lane > j) ? a[s][j] : 0.f;
#pragma unroll
      for (int k = 0; k < N; ++k) q[k] += x * a[s][j + k];
    }
    float qs[N];
    wave_allreduce<N>(q, qs);
    const float sigma = qs[0];
    const float alpha = lane_value(a[0][j], j);
    float beta = alpha;
    if (sigma > 0.f) {   // otherwise nothing below the diagonal: H_j = I (uniform)
      const float xn = sqrtf(alpha * alpha + sigma);
      beta = (alpha >= 0.f) ? -xn : xn;
      const float tau = (beta - alpha) / beta;
      const float scale = 1.f / (alpha - beta);
      float w[N];
#pragma unroll
      for (int k = 1; k < N; ++k) w[k] = lane_value(a[0][j + k], j) + scale * qs[k];
#pragma unroll
      for (int s = 0; s < RPL; ++s) {
        const int r = 64 * s + lane;
        const float coef = (r > j) ? tau * scale * a[s][j] : ((r == j) ? tau : 0.f);
#pragma unroll
        for (int k = 1; k < N; ++k) a[s][j + k] -= coef * w[k];
      }
    }
    if (lane == j) rjj = beta;
  });
  // lane l < c writes row l of R (zero below row kmax)
  if (lane < c) {
    float* Ro = out + (int64_t)slot * c * c + (int64_t)lane * c;
#pragma unroll
    for (int k = 0; k < CP; ++k)
      if (k < c) Ro[k] = (lane >= kmax || k < lane) ? 0.f : (k == lane ? rjj : a[0][k]);
  }
}

// Combining step of the TSQR tree for c <= 64 (FP32 plans): the R factor of the stacked leaf factors
// [R_1; ...; R_q] is the Cholesky factor of sum_s R_s^T R_s.  The leaves are FP32, so every product
// R_s(i, j) R_s(i, k) is exact in FP64 and the sums carry FP64 rounding only: the combined factor is
// perturbed by O(kappa^2 u64), below the leaves' own O(kappa u32) for kappa < u32 / u64.
// Partial sums: one workgroup per chunk item {instance, first slot, slots (<= kTsqrCombineSlots),
// partial index}; wave w owns the (16 CB) x (16 CB) block (w / 2, w % 2) of the Gram matrix (CB = 1 for
// c <= 32, 2 for c <= 64), accumulated by v_mfma_f64_16x16x4f64 over the rows of the chunk's leaf factors
// (slot s occupies c x c FP32 at in + s c^2), 64 rows at a time with their loads issued together.
template <int CB>
__global__ void __launch_bounds__(256) tsqr_gram_partial_kernel(const SegDev S, const float* __restrict__ in,
                                                                const int32_t* __restrict__ items, int c,
                                                                double* __restrict__ part) {
  typedef Mfma<double> MF;
  typedef MF::v4 V4;
  const int* it = items + 4 * blockIdx.x;
  const int b = it[0];
  if (!S.active[b]) return;
  const int64_t s0 = it[1];
  const int ns = it[2];
  const int q = it[3];
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  const int i = lane % 16, g = lane / 16;
  const int ci0 = 16 * CB * (w / 2), cj0 = 16 * CB * (w % 2);
  const int rows = ns * c;
  const float* base = in + s0 * c * c;
  V4 acc[CB][CB];
#pragma unroll
  for (int u = 0; u < CB; ++u)
#pragma unroll
    for (int v = 0; v < CB; ++v) acc[u][v] = V4{0, 0, 0, 0};
  for (int r0 = 0; r0 < rows; r0 += 64) {
    float xa[16][CB], yb[16][CB];
#pragma unroll
    for (int st = 0; st < 16; ++st) {
      const int r = r0 + 4 * st + g;
      const bool ok = r < rows;
      const float* src = base + (int64_t)min(r, rows - 1) * c;   // clamped: unconditional loads
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int cx = ci0 + 16 * u + i, cy = cj0 + 16 * u + i;
        xa[st][u] = keep_if(ok && cx < c, src[min(cx, c - 1)]);
        yb[st][u] = keep_if(ok && cy < c, src[min(cy, c - 1)]);
      }
    }
#pragma unroll
    for (int st = 0; st < 16; ++st)
#pragma unroll
      for (int u = 0; u < CB; ++u)
#pragma unroll
        for (int v = 0; v < CB; ++v) acc[u][v] = MF::op((double)xa[st][u], (double)yb[st][v], acc[u][v]);
  }
  double* P = part + (int64_t)q * c * c;
#pragma unroll
  for (int u = 0; u < CB; ++u)
#pragma unroll
    for (int v = 0; v < CB; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = ci0 + 16 * u + MF::drow(lane, e), gj = cj0 + 16 * v + i;
        if (gi < c && gj < c) P[gi * c + gj] = acc[u][v][e];
      }
}

// G_b = sum of instance b's partials {instance, first partial, partials, -} in a fixed order, written to
// part[gbase + b]: a block takes 16 elements, its 16 thread groups every 16th partial each (four
// independent sums), and the 16 group sums are added in order.
__global__ void __launch_bounds__(256) tsqr_gram_reduce_kernel(const SegDev S, double* __restrict__ part,
                                                               const int32_t* __restrict__ items, int len,
                                                               int64_t gbase) {
  __shared__ double red[kRedGroups][kRedElems];
  const int* it = items + 4 * blockIdx.y;
  const int b = it[0];
  if (!S.active[b]) return;
  const int q0 = it[1], q1 = it[1] + it[2];
  const int g = threadIdx.x / kRedElems, l = threadIdx.x % kRedElems;
  const int e = blockIdx.x * kRedElems + l;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < len) {
    int q = q0 + g;
    for (; q + 3 * kRedGroups < q1; q += 4 * kRedGroups) {
      s0 += part[(int64_t)q * len + e];
      s1 += part[(int64_t)(q + kRedGroups) * len + e];
      s2 += part[(int64_t)(q + 2 * kRedGroups) * len + e];
      s3 += part[(int64_t)(q + 3 * kRedGroups) * len + e];
    }
    for (; q < q1; q += kRedGroups) s0 += part[(int64_t)q * len + e];
  }
  red[g][l] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (g == 0 && e < len) {
    double t = 0.0;
#pragma unroll
    for (int h = 0; h < kRedGroups; ++h) t += red[h][l];
    part[(gbase + b) * len + e] = t;
  }
}

// Cholesky factor of G_b (at part[gbase + b]) by one wave (lane i holds row i), written as the upper
// triangular R (FP32, c x c at out + slot c^2) for item {instance, -, -, slot}.  A non-positive pivot
// (lower(W) numerically rank deficient) is replaced by 1, which keeps R nonsingular: W R^{-1} then spans
// span(W) and the Cholesky of Algorithm 2 step 3 reports the breakdown.
template <int CP>
__global__ void __launch_bounds__(64) tsqr_combine_chol_kernel(const SegDev S, const double* __restrict__ part,
                                                               const int32_t* __restrict__ items, int c,
                                                               int64_t gbase, float* __restrict__ out) {
  const int* it = items + 4 * blockIdx.x;
  const int b = it[0];
  if (!S.active[b]) return;
  const int slot = it[3];
  const int i = threadIdx.x;
  const int64_t cc = (int64_t)c * c;
  const double* G = part + (gbase + b) * cc;
  __shared__ double cb[64];
  double a[CP];
  const int ic = min(i, c - 1);   // clamped: unconditional loads
#pragma unroll
  for (int k = 0; k < CP; ++k) {
    const int kc = min(k, c - 1);
    a[k] = keep_if(i < c && k < c, 0.5 * (G[ic * c + kc] + G[kc * c + ic]));
  }
  bool bad = false;   // a non-positive pivot is replaced by 1
  wave_cholesky<CP>(a, c, cb, bad);
  // row i of L is column i of R (a compile-time loop: a[] stays in registers)
  float* R = out + (int64_t)slot * cc;
  if (i < c) {
#pragma unroll
    for (int k = 0; k < CP; ++k)
      if (k < c) R[k * c + i] = (k <= i) ? (float)a[k] : 0.f;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace {
inline int gram_rt(int c) { return c <= 32 ? 1 : c <= 64 ? 2 : 3; }

template <int RB, int CB, typename TI>
void sgram_launch(dim3 g, const SegDev& S, const TI* X, int64_t ldx, const TI* Y, int64_t ldy, int c1, int c2,
                  int tj, double* part, hipStream_t st) {
  sgram_partial_kernel<RB, CB, TI><<<g, kThreads, 0, st>>>(S, X, ldx, Y, ldy, c1, c2, tj, part);
}
template <int RB, typename TI>
void sgram_ct(int ct, dim3 g, const SegDev& S, const TI* X, int64_t ldx, const TI* Y, int64_t ldy, int c1,
              int c2, int tj, double* part, hipStream_t st) {
  switch (ct) {
    case 1: sgram_launch<RB, 1>(g, S, X, ldx, Y, ldy, c1, c2, tj, part, st); break;
    case 2: sgram_launch<RB, 2>(g, S, X, ldx, Y, ldy, c1, c2, tj, part, st); break;
    default: sgram_launch<RB, 3>(g, S, X, ldx, Y, ldy, c1, c2, tj, part, st); break;
  }
}
}  // namespace

template <typename TI>
void launch_sgram(const SegDev& S, const TI* X, int64_t ldx, const TI* Y, int64_t ldy, int c1, int c2,
                  double* G, int64_t gstride, double* part, hipStream_t st) {
  if (c1 <= 0 || c2 <= 0 || S.nchunks <= 0) return;
  const int rt = gram_rt(c1), ct = gram_rt(c2);
  const int tj = cdiv(c2, 32 * ct);
  dim3 g((unsigned)S.nchunks, cdiv(c1, 32 * rt) * tj);
  switch (rt) {
    case 1: sgram_ct<1>(ct, g, S, X, ldx, Y, ldy, c1, c2, tj, part, st); break;
    case 2: sgram_ct<2>(ct, g, S, X, ldx, Y, ldy, c1, c2, tj, part, st); break;
    default: sgram_ct<3>(ct, g, S, X, ldx, Y, ldy, c1, c2, tj, part, st); break;
  }
  const int len = c1 * c2;
  sreduce_kernel<<<dim3(cdiv(len, kRedElems), S.B), 256, 0, st>>>(S, part, len, G, gstride);
}
template void launch_sgram<double>(const SegDev&, const double*, int64_t, const double*, int64_t, int, int, double*,
                                   int64_t, double*, hipStream_t);
template void launch_sgram<float>(const SegDev&, const float*, int64_t, const float*, int64_t, int, int, double*,
                                  int64_t, double*, hipStream_t);

// Workgroups of `threads` threads of a kernel that the device holds at once (occupancy times compute
// units); 1024 if the runtime cannot tell.
static int64_t resident_blocks(const void* kernel, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || cus <= 0 || per_cu <= 0)
    return 1024;
  return (int64_t)cus * per_cu;
}

template <typename TX>
void launch_supdate(const SegDev& S, const TX* X, int64_t ldx, const double* M, int64_t ldm, int64_t mstride,
                    TX* Y, int64_t ldy, int cin, int cout, double alpha, double beta, hipStream_t st) {
  if (cout <= 0 || S.ntiles <= 0) return;
  const bool vec = ((reinterpret_cast<uintptr_t>(X) | (uintptr_t)(ldx * sizeof(TX))) & 15) == 0;
  const bool yvec = ((reinterpret_cast<uintptr_t>(Y) | (uintptr_t)(ldy * sizeof(TX))) & 15) == 0;
  if (vec && yvec && cin <= kUpdMaxK) {
    // as many workgroups per column block as are resident at once (no partial last round), each
    // walking several tiles, so that M is staged a few times per launch rather than once per tile
    if (cout <= 32) {
      static const int64_t cap = resident_blocks(reinterpret_cast<const void*>(&supdate_ms_kernel<TX, 2>), kThreads);
      const unsigned gx = (unsigned)std::min<int64_t>(S.ntiles, cap);
      supdate_ms_kernel<TX, 2><<<dim3(gx, cdiv(cout, 32)), kThreads, 0, st>>>(S, X, ldx, M, ldm, mstride, Y, ldy, cin,
                                                                             cout, alpha, beta);
    } else {
      static const int64_t cap = resident_blocks(reinterpret_cast<const void*>(&supdate_ms_kernel<TX, 4>), kThreads);
      const unsigned gx = (unsigned)std::min<int64_t>(S.ntiles, cap);
      supdate_ms_kernel<TX, 4><<<dim3(gx, cdiv(cout, 64)), kThreads, 0, st>>>(S, X, ldx, M, ldm, mstride, Y, ldy, cin,
                                                                             cout, alpha, beta);
    }
    return;
  }
  dim3 g((unsigned)S.ntiles, cdiv(cout, 64));
  supdate_kernel<TX><<<g, kThreads, 0, st>>>(S, X, ldx, M, ldm, mstride, Y, ldy, cin, cout, alpha, beta, vec);
}
template void launch_supdate<double>(const SegDev&, const double*, int64_t, const double*, int64_t, int64_t, double*,
                                     int64_t, int, int, double, double, hipStream_t);

void launch_supdate_pair(const SegDev& S, const double* X, const double* X2, int64_t ldx, const double* M, int64_t ldm,
                         int64_t mstride, double* Y, double* Y2, int64_t ldy, int cin, int cout, hipStream_t st) {
  const bool vec = ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(X2) | (uintptr_t)(ldx * 8)) & 15) == 0;
  const bool yvec = ((reinterpret_cast<uintptr_t>(Y) | reinterpret_cast<uintptr_t>(Y2) | (uintptr_t)(ldy * 8)) & 15) == 0;
  if (cout <= 32 || cout > 64 || cin > kUpdMaxK || !vec || !yvec || S.ntiles <= 0) {
    launch_supdate(S, X, ldx, M, ldm, mstride, Y, ldy, cin, cout, 1.0, 0.0, st);
    launch_supdate(S, X2, ldx, M, ldm, mstride, Y2, ldy, cin, cout, 1.0, 0.0, st);
    return;
  }
  // half of the resident workgroups for each product, so that both halves run at once
  static const int64_t cap = resident_blocks(reinterpret_cast<const void*>(&supdate_ms_kernel<double, 4>), kThreads);
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(S.ntiles, cap / 2));
  supdate_ms_kernel<double, 4><<<dim3(gx, 1, 2), kThreads, 0, st>>>(S, X, ldx, M, ldm, mstride, Y, ldy, cin, cout, 1.0,
                                                                    0.0, nullptr, X2, Y2);
}

bool launch_supdate_gram(const SegDev& S, const double* X, int64_t ldx, const double* M, int64_t ldm, double* Y,
                         int64_t ldy, int K, int cols, double* part, int64_t part_elems, double* G, hipStream_t st) {
  if (S.B != 1 || S.ntiles <= 0 || K < 4 || K > kGramMaxK || (K & 3) != 0 || cols != 32) return false;
  const bool vec = ((reinterpret_cast<uintptr_t>(X) | (uintptr_t)(ldx * 8)) & 15) == 0;
  const bool yvec = ((reinterpret_cast<uintptr_t>(Y) | (uintptr_t)(ldy * 8)) & 15) == 0;
  if (!vec || !yvec) return false;
  static const int64_t cap =
      resident_blocks(reinterpret_cast<const void*>(&supdate_ms_kernel<double, 2, true>), kThreads);
  const int64_t len = (int64_t)K * cols;
  const int64_t gx = std::min<int64_t>(std::min<int64_t>(S.ntiles, cap), part_elems / len);
  if (gx < 1) return false;
  supdate_ms_kernel<double, 2, true><<<dim3((unsigned)gx, 1), kThreads, 0, st>>>(S, X, ldx, M, ldm, 0, Y, ldy, K, cols,
                                                                               -1.0, 1.0, part);
  preduce_kernel<<<cdiv(len, kRedElems), 256, 0, st>>>(part, (int)gx, (int)len, G);
  return true;
}
template void launch_supdate<float>(const SegDev&, const float*, int64_t, const double*, int64_t, int64_t, float*,
                                    int64_t, int, int, double, double, hipStream_t);

template <typename T, typename TI>
void launch_sresidual(const SegDev& S, const TI* AX, int64_t ldax, const TI* X, int64_t ldx,
                      const double* theta, int64_t tstride, int m, T* R, int64_t ldr, double* norms, double* part,
                      hipStream_t st) {
  if (S.nchunks <= 0) return;
  const bool vec = (ldx % 2 == 0) && (ldax % 2 == 0) && (ldr % 2 == 0) &&
                   ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(AX)) % 16 == 0);
  const unsigned g = (unsigned)S.nchunks;
  if (vec && m == 32) sresidual2_kernel<T, 16, TI><<<g, kThreads, 0, st>>>(S, AX, ldax, X, ldx, theta, tstride, R, ldr, part);
  else if (vec && m == 16) sresidual2_kernel<T, 8, TI><<<g, kThreads, 0, st>>>(S, AX, ldax, X, ldx, theta, tstride, R, ldr, part);
  else if (vec && m == 8) sresidual2_kernel<T, 4, TI><<<g, kThreads, 0, st>>>(S, AX, ldax, X, ldx, theta, tstride, R, ldr, part);
  else sresidual_kernel<T, TI><<<g, kThreads, 0, st>>>(S, AX, ldax, X, ldx, theta, tstride, m, R, ldr, part);
  sreduce_kernel<<<dim3(cdiv(2 * m, kRedElems), S.B), 256, 0, st>>>(S, part, 2 * m, norms, 2 * m);
}
#define INST_RES(T, TI)                                                                                            \
  template void launch_sresidual<T, TI>(const SegDev&, const TI*, int64_t, const TI*, int64_t, const double*, int64_t, \
                                        int, T*, int64_t, double*, double*, hipStream_t);
INST_RES(float, double)
INST_RES(double, double)
INST_RES(float, float)
INST_RES(double, float)
#undef INST_RES

template <typename TI>
void launch_scolnorms(const SegDev& S, const TI* X, int64_t ldx, int c, double* norms, int64_t nstride,
                      double* part, hipStream_t st) {
  if (S.nchunks <= 0) return;
  scolnorm_kernel<TI><<<(unsigned)S.nchunks, kThreads, 0, st>>>(S, X, ldx, c, part);
  sreduce_kernel<<<dim3(cdiv(c, kRedElems), S.B), 256, 0, st>>>(S, part, c, norms, nstride);
}
template void launch_scolnorms<double>(const SegDev&, const double*, int64_t, int, double*, int64_t, double*,
                                       hipStream_t);
template void launch_scolnorms<float>(const SegDev&, const float*, int64_t, int, double*, int64_t, double*,
                                      hipStream_t);

template <typename TU, typename TW>
void launch_strsm_rows(const SegDev& S, TW* W, int64_t ld, int c, const TU* U, int64_t ustride, hipStream_t st) {
  if (S.ntiles <= 0) return;
  const size_t lds = (size_t)(c * c + 64 * c) * sizeof(double);
  const unsigned g = (unsigned)S.ntiles;
  if (c == 8) strsm_rows_reg_kernel<TU, 8, TW><<<g, 64, 0, st>>>(S, W, ld, U, ustride);
  else if (c == 16) strsm_rows_reg_kernel<TU, 16, TW><<<g, 64, 0, st>>>(S, W, ld, U, ustride);
  else if (c == 32) strsm_rows_reg_kernel<TU, 32, TW><<<g, 64, 0, st>>>(S, W, ld, U, ustride);
  else if (c == 64) strsm_rows_reg_kernel<TU, 64, TW><<<g, 64, 0, st>>>(S, W, ld, U, ustride);
  else strsm_rows_kernel<TU, TW><<<g, 64, lds, st>>>(S, W, ld, c, U, ustride);
}
template void launch_strsm_rows<float, double>(const SegDev&, double*, int64_t, int, const float*, int64_t, hipStream_t);
template void launch_strsm_rows<double, double>(const SegDev&, double*, int64_t, int, const double*, int64_t,
                                                hipStream_t);
template void launch_strsm_rows<float, float>(const SegDev&, float*, int64_t, int, const float*, int64_t, hipStream_t);
template void launch_strsm_rows<double, float>(const SegDev&, float*, int64_t, int, const double*, int64_t,
                                               hipStream_t);

template <typename T, typename Tin, int CP>
void stsqr_go(unsigned grid, const SegDev& S, const Tin* in, int64_t ld, const int32_t* items, int c, T* out,
              hipStream_t st) {
  stsqr_kernel<T, Tin, CP><<<grid, kTsqrRows, 0, st>>>(S, in, ld, items, c, out);
}

template <typename T, typename Tin>
void stsqr_launch(unsigned grid, const SegDev& S, const Tin* in, int64_t ld, const int32_t* items, int c, T* out,
                  hipStream_t st) {
  // FP32 blocks of up to 32 columns, many of them (a level that fills the chip): one wave per block.
  // A few blocks (the top of the tree) finish sooner with a whole workgroup on each.
  if constexpr (sizeof(T) == 4) {
    if (grid >= 256) {
      const unsigned g4 = (grid + 3) / 4;
      if (c <= 8) { stsqr_wave_kernel<Tin, 8><<<g4, 256, 0, st>>>(S, in, ld, items, grid, c, out); return; }
      if (c <= 16) { stsqr_wave_kernel<Tin, 16><<<g4, 256, 0, st>>>(S, in, ld, items, grid, c, out); return; }
      if (c <= 32) { stsqr_wave_kernel<Tin, 32><<<g4, 256, 0, st>>>(S, in, ld, items, grid, c, out); return; }
    }
  }
  if (c <= 8) stsqr_go<T, Tin, 8>(grid, S, in, ld, items, c, out, st);
  else if (c <= 16) stsqr_go<T, Tin, 16>(grid, S, in, ld, items, c, out, st);
  else if (c <= 32) stsqr_go<T, Tin, 32>(grid, S, in, ld, items, c, out, st);
  else stsqr_go<T, Tin, 64>(grid, S, in, ld, items, c, out, st);
}

template <typename T, typename Tin>
void launch_stsqr(const SegDev& S, const TsqrPlanDev& P, const Tin* W, int64_t ldw, int c, T* scratch, T* R,
                  hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (P.combine) {   // FP32 leaves of kTsqrRowsCombine rows, then the FP64 Gram and its Cholesky factor
      const int64_t i0 = P.level_off[0], i1 = P.level_off[1], i2 = P.level_off[2], i3 = P.level_off[3];
      const unsigned g4 = (unsigned)((i1 - i0 + 3) / 4);
      const int32_t* it0 = P.items + 4 * i0;
      if (c <= 8) stsqr_wave_kernel<Tin, 8, kTsqrCombineRpl><<<g4, 256, 0, st>>>(S, W, ldw, it0, i1 - i0, c, scratch);
      else if (c <= 16) stsqr_wave_kernel<Tin, 16, kTsqrCombineRpl><<<g4, 256, 0, st>>>(S, W, ldw, it0, i1 - i0, c, scratch);
      else if (c <= 32) stsqr_wave_kernel<Tin, 32, kTsqrCombineRpl><<<g4, 256, 0, st>>>(S, W, ldw, it0, i1 - i0, c, scratch);
      else stsqr_go<T, Tin, 64>((unsigned)(i1 - i0), S, W, ldw, it0, c, scratch, st);   // one workgroup per leaf
      double* part = reinterpret_cast<double*>(scratch + P.half);
      const int64_t gbase = i2 - i1;   // the per-instance Gram matrices follow the partials
      const int32_t* it2 = P.items + 4 * i2;
      if (c <= 32)
        tsqr_gram_partial_kernel<1><<<(unsigned)(i2 - i1), 256, 0, st>>>(S, scratch, P.items + 4 * i1, c, part);
      else
        tsqr_gram_partial_kernel<2><<<(unsigned)(i2 - i1), 256, 0, st>>>(S, scratch, P.items + 4 * i1, c, part);
      tsqr_gram_reduce_kernel<<<dim3(cdiv(c * c, kRedElems), (unsigned)(i3 - i2)), 256, 0, st>>>(S, part, it2, c * c,
                                                                                              gbase);
      if (c <= 8) tsqr_combine_chol_kernel<8><<<(unsigned)(i3 - i2), 64, 0, st>>>(S, part, it2, c, gbase, R);
      else if (c <= 16) tsqr_combine_chol_kernel<16><<<(unsigned)(i3 - i2), 64, 0, st>>>(S, part, it2, c, gbase, R);
      else if (c <= 32) tsqr_combine_chol_kernel<32><<<(unsigned)(i3 - i2), 64, 0, st>>>(S, part, it2, c, gbase, R);
      else tsqr_combine_chol_kernel<64><<<(unsigned)(i3 - i2), 64, 0, st>>>(S, part, it2, c, gbase, R);
      return;
    }
  }
  for (int l = 0; l < P.nlevels; ++l) {
    const int64_t i0 = P.level_off[l], i1 = P.level_off[l + 1];
    if (i1 <= i0) continue;
    T* out = (l == P.nlevels - 1) ? R : scratch + (l % 2) * P.half;
    const unsigned grid = (unsigned)(i1 - i0);
    if (l == 0) {
      stsqr_launch<T, Tin>(grid, S, W, ldw, P.items + 4 * i0, c, out, st);
      continue;
    }
    const T* in = scratch + ((l - 1) % 2) * P.half;
    if constexpr (sizeof(T) == 4) {
      if (P.rbu == kTsqrRowsWide) {   // plan guarantees c <= 32
        if (c <= 8) stsqr_kernel<T, T, 8, kTsqrRowsWide><<<grid, kTsqrRowsWide, 0, st>>>(S, in, c, P.items + 4 * i0, c, out);
        else if (c <= 16) stsqr_kernel<T, T, 16, kTsqrRowsWide><<<grid, kTsqrRowsWide, 0, st>>>(S, in, c, P.items + 4 * i0, c, out);
        else stsqr_kernel<T, T, 32, kTsqrRowsWide><<<grid, kTsqrRowsWide, 0, st>>>(S, in, c, P.items + 4 * i0, c, out);
        continue;
      }
    }
    stsqr_launch<T, T>(grid, S, in, c, P.items + 4 * i0, c, out, st);
  }
}
template void launch_stsqr<float, double>(const SegDev&, const TsqrPlanDev&, const double*, int64_t, int, float*,
                                          float*, hipStream_t);
template void launch_stsqr<double, double>(const SegDev&, const TsqrPlanDev&, const double*, int64_t, int, double*,
                                           double*, hipStream_t);
template void launch_stsqr<float, float>(const SegDev&, const TsqrPlanDev&, const float*, int64_t, int, float*, float*,
                                         hipStream_t);

int tsqr_rows_per_block(int c, int elem_bytes) {
  (void)c;
  (void)elem_bytes;
  return kTsqrRows;
}

int tsqr_upper_rows_per_block(int c, int elem_bytes) { return (elem_bytes == 4 && c <= 32) ? kTsqrRowsWide : kTsqrRows; }

}  // namespace lobpcg
