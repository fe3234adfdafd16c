// Small dense FP64 kernels, one workgroup each:
//  * symmetric eigensolver for the c x c Rayleigh-Ritz matrix (Algorithm 3
//    line 14): tridiagonalization, bisection, inverse iteration;
//  * the Hetmaniuk-Lehoucq step (lines 15-16): V = orthonormal factor of
//    C(1:m, m+1:c)^T and G = [C(:,1:m), C(:,m+1:c) V];
//  * Algorithm 2's step 3: the Cholesky factorization of V^T V.
#include <cmath>
#include <type_traits>

#include "bufload.hpp"
#include "common.hpp"
#include "mfma.hpp"

namespace lobpcg {

namespace {


__device__ inline double rdl64(double v, int l) {
  const uint64_t x = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// 64-bit DPP move (one 32-bit DPP move per half); CTRL = 0x120 + r rotates each 16-lane row by r.
template <int CTRL>
__device__ inline double dpp_f64(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  // every row and bank enabled and a rotation inside each row: every lane receives a value, so the
  // destination needs no initial value
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 16 lanes of a row (lanes 16 r .. 16 r + 15).  Rotations by 8, 4, 2, 1: at each
// stage the two lanes of a pair add the same two values, so every lane ends with the same bits.
__device__ inline double row16_sum(double x) {
  x += dpp_f64<0x128>(x);
  x += dpp_f64<0x124>(x);
  x += dpp_f64<0x122>(x);
  x += dpp_f64<0x121>(x);
  return x;
}

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

// Symmetric eigensolver for the c x c Rayleigh-Ritz matrix: the nev smallest eigenpairs, one
// workgroup of four waves per matrix.
//  1. Householder reduction to tridiagonal form T = Q^T H Q (reflectors stored below the
//     subdiagonal, as in LAPACK's sytd2);
//  2. the nev smallest eigenvalues of T by multisection on Sturm counts: every round, each
//     eigenvalue's bracket is cut at P interior points evaluated by P threads (the Sturm count is
//     backward stable, so each eigenvalue is accurate to a few ulps of ||T||);
//  3. their eigenvectors by two sweeps of inverse iteration with a pivoted tridiagonal LU, one
//     thread per vector; after each sweep the vectors of every cluster (a chain of eigenvalues
//     whose consecutive gaps are below 1e-3 ||T||_1) are re-orthonormalised by modified
//     Gram-Schmidt in eigenvalue order, so the next sweep purifies what that mixed in;
//  4. back-transformation C = Q Z of the nev vectors, several threads per column.
// Matrices up to 96 x 96 live in LDS, larger ones in the global scratch.
constexpr int kSyevThreads = 256;
constexpr int kSyevWaves = kSyevThreads / 64;
constexpr int kSyevLds = 96;
constexpr int kSyevMax = 192;
// from this many eigenvalues on, the register eigensolver bisects them in a launch of its own with
// one workgroup per eigenvalue (fewer rounds than splitting one workgroup's points among them), as
// long as that launch stays within kSyevSplitMaxBlocks workgroups; a larger batch already fills the
// chip with one workgroup per problem (c = 96, nev = 32: 353 -> 286 us for one problem; c = 48,
// nev = 16: 177 -> 248 us for 256 problems)
constexpr int kSyevSplitMinNev = 8;
constexpr int kSyevSplitMaxBlocks = 1024;

// 1/q from the hardware reciprocal refined by two Newton steps (about one ulp), a shorter
// dependency chain than the IEEE division sequence.
__device__ inline double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  r = fma(r, fma(-q, r, 1.0), r);
  return r;
}

// Number of eigenvalues of T below x, from T scaled by a power of two to norm about one (diagonal
// ds, squared off-diagonal e2s, shift xs).  The leading principal minors
// p_i = (ds_i - xs) p_{i-1} - e2s_{i-1} p_{i-2} (p_{-1} = 1) are the products of the LDL^T pivots
// q_i = p_i / p_{i-1}, so a sign change from p_{i-1} to p_i is a negative pivot.  Without a division a
// tiny pivot needs no guard; a zero one (p_i = 0, which would stall the recurrence where e_i = 0) is
// replaced by -pmin (p_i = -pmin p_{i-1}), as LAPACK replaces pivots below pivmin.  The only dependent
// operations per step are one FMA and the zero test (e2s_{i-1} p_{i-2} is ready a step earlier);
// p_{i-1} and p_i are rescaled by a power of two every four steps.  The arrays are padded
// to c + 8 entries with ds = 8 and e2s = 0 (|xs| < 4): steps past the end change no sign, so the
// four-step groups need no exit test and the next group's loads overlap the current one.
__device__ inline int sturm_count_scaled(const double* ds, const double* e2s, int c, double xs, double pmin) {
  double pm2 = 1.0, pm1 = ds[0] - xs;
  if (fabs(pm1) < pmin) pm1 = -pmin;
  int cnt = (pm1 < 0.0);
  double dd[4], ee[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    dd[u] = ds[1 + u];
    ee[u] = e2s[u];
  }
  for (int i0 = 1; i0 < c; i0 += 4) {
    double dn[4], en[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dn[u] = ds[i0 + 4 + u];
      en[u] = e2s[i0 + 3 + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double p = fma(dd[u] - xs, pm1, -ee[u] * pm2);
      if (p == 0.0) p = -pmin * pm1;
      cnt += ((p < 0.0) != (pm1 < 0.0));
      pm2 = pm1;
      pm1 = p;
    }
    const int k = __builtin_amdgcn_frexp_exp(pm1);
    pm1 = ldexp(pm1, -k);
    pm2 = ldexp(pm2, -k);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dd[u] = dn[u];
      ee[u] = en[u];
    }
  }
  return cnt;
}

// Modified Gram-Schmidt inside the clusters of eigenvectors (eigenvalue order) with Z (c x nev,
// c <= 16 NR, nev <= 16 NC) in registers: thread (slot s = tid / 16, lane q16 of its 16-lane row) holds
// rows q16 + 16 u of columns s + 16 h, so column sums are 16-lane DPP sums.  Column q is published by
// its owners (one barrier, buffers alternating per executed step); the later members of its cluster
// subtract their projections on it and the owners of q + 1 normalise it right away.  HQ is static
// (column block of q), so register indices are static.
template <int NR, int NC, int HQ>
__device__ __attribute__((always_inline)) void cluster_mgs_cols(double (&z)[NC][NR], int nev, const short* cend,
                                                                double* wb0, double* wb1, int& ns) {
  const int tid = threadIdx.x, q16 = tid & 15, slot = tid >> 4;
#pragma unroll 1
  for (int sq = 0; sq < 16; ++sq) {
    const int q = 16 * HQ + sq;
    if (q + 1 >= nev) break;   // uniform
    const int qe = cend[q];
    if (qe - q < 2) continue;   // uniform
    double* wb = (ns & 1) ? wb1 : wb0;
    ++ns;
    if (slot == sq) {
#pragma unroll
      for (int u = 0; u < NR; ++u) wb[q16 + 16 * u] = z[HQ][u];
    }
    __syncthreads();
    double wq[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) wq[u] = wb[q16 + 16 * u];
#pragma unroll
    for (int h = HQ; h < NC; ++h) {
      const int col = slot + 16 * h;
      if (col > q && col < qe) {   // uniform over the 16 lanes of a slot
        double dt = 0.0;
#pragma unroll
        for (int u = 0; u < NR; ++u) dt = fma(z[h][u], wq[u], dt);
        dt = row16_sum(dt);
#pragma unroll
        for (int u = 0; u < NR; ++u) z[h][u] = fma(-dt, wq[u], z[h][u]);
        if (col == q + 1) {
          double nn = 0.0;
#pragma unroll
          for (int u = 0; u < NR; ++u) nn = fma(z[h][u], z[h][u], nn);
          const double inv = 1.0 / sqrt(row16_sum(nn));
#pragma unroll
          for (int u = 0; u < NR; ++u) z[h][u] *= inv;
        }
      }
    }
  }
  if constexpr (HQ + 1 < NC) cluster_mgs_cols<NR, NC, HQ + 1>(z, nev, cend, wb0, wb1, ns);
}

// Inverse iteration for eigenvector j of the tridiagonal T (diagonal d, off-diagonal e) at its
// eigenvalue lj, one thread per vector.  The factors of P (T - lj I) = L U (partial pivoting, as LAPACK's
// dlagtf) are stored per step k at [k nev + j]: U0 the reciprocal of U's diagonal (an entry below tiny
// in magnitude taken as +-tiny), U1 its first superdiagonal, Lm the multiplier of L, Pv 1 where rows k
// and k + 1 were swapped (U's second superdiagonal is then e[k + 1], else 0).  Every pass runs in chunks
// of CH steps whose loads carry no condition, so that they are issued together before the chunk's
// arithmetic, and a step-by-step tail.
//
// One elimination step on the active row (cd, cs) and the next row (sub, nd, ns) of T - lj I, with the
// forward substitution of the right-hand side (zk, zn) carried along.  With FAST the multiplier uses the
// reciprocal pivot from rcp_nr (no division in the dependent chain) and bad is set where the pivot lies
// outside [2^-1000, 2^1000], where that reciprocal is not accurate; otherwise it is the quotient itself.
template <bool FAST>
__device__ __attribute__((always_inline)) void ii_step(double& cd, double& cs, double& zk, double sub, double nd,
                                                       double ns, double zn, double tiny, double rtiny, bool& bad,
                                                       double* u0, double* u1, double* lm, double* pv, double* zo) {
  const bool sw = !(fabs(cd) >= fabs(sub));
  const double piv = sw ? sub : cd, oth = sw ? cd : sub;
  const double big = (piv < 0.0) ? -rtiny : rtiny;
  double m, rp;
  if constexpr (FAST) {
    rp = rcp_nr(piv);
    bad |= !(fabs(piv) >= 0x1p-1000 && fabs(piv) <= 0x1p+1000);
    m = oth * rp;
  } else {
    rp = 1.0 / piv;
    m = (piv != 0.0) ? oth / piv : 0.0;   // |m| <= 1; piv == 0 only when sub == cd == 0
  }
  *u0 = (fabs(piv) >= tiny) ? rp : big;
  *u1 = sw ? nd : cs;
  *lm = m;
  *pv = sw ? 1.0 : 0.0;
  const double ncd = sw ? cs - m * nd : nd - m * cs;
  cs = sw ? -m * ns : ns;
  cd = ncd;
  const double lo = sw ? zn : zk, hi = sw ? zk : zn;
  *zo = lo;
  zk = hi - m * lo;
}

// Factorization fused with the first forward substitution P, L^-1 of the fixed start vector
// s_i = 1 + ((7 i + 13 j) mod 11) / 44 (not orthogonal to any eigenvector of interest); the result goes to
// Z.  A thread whose fast pass met a pivot outside rcp_nr's range redoes the pass with divisions.
template <int CH>
__device__ __attribute__((always_inline)) void ii_factor(const double* d, const double* e, int c, int nev, int j,
                                                         double lj, double tiny, double rtiny, double* U0, double* U1,
                                                         double* Lm, double* Pv, double* Z, int lz) {
  auto start = [j](int i) { return 1.0 + (double)((7 * i + 13 * j) % 11) * (0.25 / 11.0); };
  auto pass = [&](auto fast) -> bool {
    constexpr bool F = decltype(fast)::value;
    bool bad = false;
    double cd = d[0] - lj, cs = (c > 1) ? e[0] : 0.0, zk = start(0);
    int k0 = 0;
    if constexpr (F) {
      for (; k0 + CH + 1 < c; k0 += CH) {   // every step of the chunk has k + 2 < c
        double ek[CH], dn[CH], en[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          ek[u] = e[k0 + u];
          dn[u] = d[k0 + u + 1];
          en[u] = e[k0 + u + 1];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int k = k0 + u;
          ii_step<true>(cd, cs, zk, ek[u], dn[u] - lj, en[u], start(k + 1), tiny, rtiny, bad, &U0[k * nev + j],
                        &U1[k * nev + j], &Lm[k * nev + j], &Pv[k * nev + j], &Z[k * lz + j]);
        }
      }
    }
    for (; k0 + 1 < c; ++k0)
      ii_step<F>(cd, cs, zk, e[k0], d[k0 + 1] - lj, (k0 + 2 < c) ? e[k0 + 1] : 0.0, start(k0 + 1), tiny, rtiny, bad,
                 &U0[k0 * nev + j], &U1[k0 * nev + j], &Lm[k0 * nev + j], &Pv[k0 * nev + j], &Z[k0 * lz + j]);
    const double rl = F ? rcp_nr(cd) : 1.0 / cd;
    if (F) bad |= !(fabs(cd) >= 0x1p-1000 && fabs(cd) <= 0x1p+1000);
    U0[(c - 1) * nev + j] = (fabs(cd) >= tiny) ? rl : ((cd < 0.0) ? -rtiny : rtiny);
    Z[(c - 1) * lz + j] = zk;
    return bad;
  };
  if (pass(std::true_type{})) pass(std::false_type{});
}

// Forward substitution P, L^-1 applied to Z's column j in place.
template <int CH>
__device__ __attribute__((always_inline)) void ii_forward(int c, int nev, int j, const double* Lm, const double* Pv,
                                                          double* Z, int lz) {
  double zk = Z[j];
  int k0 = 0;
  for (; k0 + CH < c; k0 += CH) {   // every step of the chunk has k + 1 < c
    double pv[CH], lm[CH], zn[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      pv[u] = Pv[(k0 + u) * nev + j];
      lm[u] = Lm[(k0 + u) * nev + j];
      zn[u] = Z[(k0 + u + 1) * lz + j];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const bool sw = pv[u] != 0.0;
      const double lo = sw ? zn[u] : zk, hi = sw ? zk : zn[u];
      Z[(k0 + u) * lz + j] = lo;
      zk = hi - lm[u] * lo;
    }
  }
  for (; k0 + 1 < c; ++k0) {
    const bool sw = Pv[k0 * nev + j] != 0.0;
    const double zn = Z[(k0 + 1) * lz + j];
    const double lo = sw ? zn : zk, hi = sw ? zk : zn;
    Z[k0 * lz + j] = lo;
    zk = hi - Lm[k0 * nev + j] * lo;
  }
  Z[(c - 1) * lz + j] = zk;
}

// Back substitution U^-1 on Z's column j in place, then scaling of the column to unit 2-norm.
template <int CH>
__device__ __attribute__((always_inline)) void ii_backward(const double* e, int c, int nev, int j, const double* U0,
                                                           const double* U1, const double* Pv, double* Z, int lz) {
  // rows c - 1 and c - 2 first (no superdiagonal entries beyond the matrix)
  double z1 = Z[(c - 1) * lz + j] * U0[(c - 1) * nev + j], z2 = 0.0;   // Z[k + 1], Z[k + 2]
  Z[(c - 1) * lz + j] = z1;
  double nrm = z1 * z1;
  if (c >= 2) {
    const int k = c - 2;
    const double y = (Z[k * lz + j] - U1[k * nev + j] * z1) * U0[k * nev + j];
    Z[k * lz + j] = y;
    nrm = fma(y, y, nrm);
    z2 = z1;
    z1 = y;
  }
  int k0 = c - 3;
  for (; k0 - CH + 1 >= 0; k0 -= CH) {   // rows k0 .. k0 - CH + 1
    double u0[CH], u1[CH], u2[CH], zz[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const int k = k0 - u;
      u0[u] = U0[k * nev + j];
      u1[u] = U1[k * nev + j];
      u2[u] = Pv[k * nev + j] * e[k + 1];
      zz[u] = Z[k * lz + j];
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      const double y = ((zz[u] - u1[u] * z1) - u2[u] * z2) * u0[u];
      Z[(k0 - u) * lz + j] = y;
      nrm = fma(y, y, nrm);
      z2 = z1;
      z1 = y;
    }
  }
  for (; k0 >= 0; --k0) {
    const double y = ((Z[k0 * lz + j] - U1[k0 * nev + j] * z1) - Pv[k0 * nev + j] * e[k0 + 1] * z2) * U0[k0 * nev + j];
    Z[k0 * lz + j] = y;
    nrm = fma(y, y, nrm);
    z2 = z1;
    z1 = y;
  }
  const double sc = 1.0 / sqrt(nrm);
  int i0 = 0;
  for (; i0 + CH <= c; i0 += CH) {
    double zz[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) zz[u] = Z[(i0 + u) * lz + j];
#pragma unroll
    for (int u = 0; u < CH; ++u) Z[(i0 + u) * lz + j] = zz[u] * sc;
  }
  for (; i0 < c; ++i0) Z[i0 * lz + j] *= sc;
}

// Steps 2 and 3 for the tridiagonal T (diagonal d, off-diagonal e in LDS, e[c - 1] = 0): the nev
// smallest eigenvalues in lam and the eigenvectors of T in Z (c x nev, row stride lz).  s1, s3:
// c + 8 doubles of LDS each, s2: c; cnt: one int per thread; lu: 4 c nev doubles (LDS or global scratch).
// Returns the largest number of later members of a cluster (0 when every eigenvalue is isolated);
// Z and lam are complete and visible to the whole workgroup on return.
template <int NR, int NC, bool PRESET = false, int CH = 8>
__device__ __attribute__((always_inline)) int tridiag_eigs(const double* d, const double* e, int c, int nev, double* s1, double* s2,
                            double* s3, double* lam, int* cnt, short* cend, double* Z, int lz, double* lu) {
  const int tid = threadIdx.x, lane = tid % 64, wid = tid / 64;
  // ---- 2. the nev smallest eigenvalues by multisection ----
  double* e2 = s1;
  double* lo = s2;
  double* hi = lam;
  // Gershgorin bounds, ||T||_inf and max e^2: every wave reduces them over its lanes (min / max are
  // exact, so every wave gets the same values)
  double gl = 1e300, gu = -1e300, tnorm = 0.0, emax2 = 0.0;
  for (int i = lane; i < c; i += 64) {
    const double ei = (i < c - 1) ? fabs(e[i]) : 0.0;
    const double em = (i > 0) ? fabs(e[i - 1]) : 0.0;
    gl = fmin(gl, d[i] - ei - em);
    gu = fmax(gu, d[i] + ei + em);
    tnorm = fmax(tnorm, fabs(d[i]) + ei + em);
    emax2 = fmax(emax2, ei * ei);
  }
  for (int off = 32; off > 0; off >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, off, 64));
    gu = fmax(gu, __shfl_xor(gu, off, 64));
    tnorm = fmax(tnorm, __shfl_xor(tnorm, off, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, off, 64));
  }
  const double eps = 2.220446049250313e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  if constexpr (!PRESET) {   // otherwise lam holds the eigenvalues already
  gl -= 2.0 * eps * tnorm * c + 2.0 * pivmin;
  gu += 2.0 * eps * tnorm * c + 2.0 * pivmin;
  // T scaled by sc = 2^-ilogb(||T||) for the Sturm counts (s3: scaled diagonal; both padded to
  // c + 8 entries, ds = 8 and e2 = 0 past the end)
  const double sc = (tnorm > 0.0) ? ldexp(1.0, -ilogb(tnorm)) : 1.0;
  const double pmin = fmax(sc * pivmin, 0x1p-100);
  double* ds = s3;
  for (int i = tid; i < c + 8; i += kSyevThreads) {
    const double es = (i < c - 1) ? sc * e[i] : 0.0;
    e2[i] = es * es;
    ds[i] = (i < c) ? sc * d[i] : 8.0;
  }
  __syncthreads();
  // first round, shared by all brackets: kSyevThreads points spread over [gl, gu]; the bracket of
  // eigenvalue j is then found by bisection on the counts, keeping count(lo) <= j < count(hi)
  // (index -1 stands for gl and kSyevThreads for gu)
  auto point = [gl, gu](int t) { return gl + (gu - gl) * (double)(t + 1) / (double)(kSyevThreads + 1); };
  cnt[tid] = sturm_count_scaled(ds, e2, c, sc * point(tid), pmin);
  __syncthreads();
  for (int j = tid; j < nev; j += kSyevThreads) {
    int a = -1, b = kSyevThreads;
    while (b - a > 1) {
      const int mid = (a + b) / 2;
      if (cnt[mid] <= j) a = mid;
      else b = mid;
    }
    lo[j] = (a < 0) ? gl : point(a);
    hi[j] = (b >= kSyevThreads) ? gu : point(b);
  }
  __syncthreads();
  const int P = max(1, kSyevThreads / nev);   // interior points per bracket
  for (int round = 0; round < 200; ++round) {
    const int j = tid / P, q = tid % P;
    bool open = false;
    if (j < nev) {
      const double l = lo[j], h = hi[j];
      open = (h - l > 2.0 * eps * fmax(fabs(l), fabs(h)) + pivmin);
      const double x = l + (h - l) * (double)(q + 1) / (double)(P + 1);
      cnt[tid] = (open && x > l && x < h) ? sturm_count_scaled(ds, e2, c, sc * x, pmin) : -1;
    }
    if (!__syncthreads_or(open)) break;
    if (j < nev && q == 0) {
      const double l = lo[j], h = hi[j];
      if (h - l > 2.0 * eps * fmax(fabs(l), fabs(h)) + pivmin) {
        double nl = l, nh = h;
        for (int r = 0; r < P; ++r) {
          const int cr = cnt[tid + r];
          if (cr < 0) continue;
          const double x = l + (h - l) * (double)(r + 1) / (double)(P + 1);
          if (cr >= j + 1) {
            nh = x;
            break;
          }
          nl = x;
        }
        if (nl == l && nh == h) nh = nl;   // no interior point strictly inside: the bracket is at ulp level
        lo[j] = nl;
        hi[j] = nh;
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < nev; j += kSyevThreads) lam[j] = 0.5 * (lo[j] + hi[j]);
  __syncthreads();
  }
  // ---- 3. eigenvectors of T by inverse iteration ----
  const double ortol = 1e-3 * tnorm;
  if (tid == 0) {
    short ce = (short)nev;
    cend[nev - 1] = ce;
    for (int j = nev - 2; j >= 0; --j) {
      ce = (lam[j + 1] - lam[j] < ortol) ? ce : (short)(j + 1);
      cend[j] = ce;
    }
  }
  double* U0 = lu;
  double* U1 = lu + (int64_t)c * nev;
  double* Lm = lu + 2 * (int64_t)c * nev;
  double* Pv = lu + 3 * (int64_t)c * nev;
  const double tiny = eps * tnorm + pivmin;
  const double rtiny = 1.0 / tiny;
  int maxrank = 0;
  for (int itn = 0; itn < 2; ++itn) {
    for (int j = tid; j < nev; j += kSyevThreads) {
      if (itn == 0) ii_factor<CH>(d, e, c, nev, j, lam[j], tiny, rtiny, U0, U1, Lm, Pv, Z, lz);
      else ii_forward<CH>(c, nev, j, Lm, Pv, Z, lz);
      ii_backward<CH>(e, c, nev, j, U0, U1, Pv, Z, lz);
    }
    __syncthreads();
    if (itn == 0)
      for (int j = 0; j < nev; ++j) maxrank = max(maxrank, (int)cend[j] - j - 1);
    if constexpr (NC > 0) {
      if (maxrank > 0) {   // uniform
        const int q16 = tid & 15, slot = tid >> 4;
        double z[NC][NR];
#pragma unroll
        for (int h = 0; h < NC; ++h)
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int i = q16 + 16 * u, j = slot + 16 * h;
            z[h][u] = (i < c && j < nev) ? Z[i * lz + j] : 0.0;
          }
        int ns = 0;
        cluster_mgs_cols<NR, NC, 0>(z, nev, cend, s1, s3, ns);
#pragma unroll
        for (int h = 0; h < NC; ++h)
#pragma unroll
          for (int u = 0; u < NR; ++u) {
            const int i = q16 + 16 * u, j = slot + 16 * h;
            if (i < c && j < nev) Z[i * lz + j] = z[h][u];
          }
        __syncthreads();
      }
    } else {
      // modified Gram-Schmidt inside each cluster, in eigenvalue order: wave w takes the later
      // members r = q + 1 + w, q + 1 + w + kSyevWaves, ...; lanes split the rows
      for (int q = 0; q + 1 < nev; ++q) {
        const int qe = cend[q];
        if (qe - q < 2) continue;   // uniform
        for (int r = q + 1 + wid; r < qe; r += kSyevWaves) {
          // a lane holds at most 3 rows (c <= 192): load them, reduce, then store
          double zq[3], zr[3];
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            const int i = lane + 64 * u;
            zq[u] = (i < c) ? Z[i * lz + q] : 0.0;
            zr[u] = (i < c) ? Z[i * lz + r] : 0.0;
          }
          const double dot = wave_sum((zq[0] * zr[0] + zq[1] * zr[1]) + zq[2] * zr[2]);
#pragma unroll
          for (int u = 0; u < 3; ++u) {
            const int i = lane + 64 * u;
            if (i < c) Z[i * lz + r] = zr[u] - dot * zq[u];
          }
        }
        __syncthreads();
        if (wid == 0) {
          double z[3];
#pragma unroll
          for (int u = 0; u < 3; ++u) z[u] = (lane + 64 * u < c) ? Z[(lane + 64 * u) * lz + q + 1] : 0.0;
          const double nn = 1.0 / sqrt(wave_sum((z[0] * z[0] + z[1] * z[1]) + z[2] * z[2]));
#pragma unroll
          for (int u = 0; u < 3; ++u)
            if (lane + 64 * u < c) Z[(lane + 64 * u) * lz + q + 1] = z[u] * nn;
        }
        __syncthreads();
      }
    }
  }
  return maxrank;
}

// Global scratch of the split forms (doubles from the instance's start).  For c <= 96: the
// inverse-iteration factors (4 c^2, when they do not fit in LDS), Q (c x c, row stride c + 1), the
// diagonal and off-diagonal of T (e[c - 1] = 0) and the eigenvalues.
// For c > 96 (the reflector form) the scratch instead holds the reflector rows V
// (c x c, row stride c + 1) at 0, then a c x (c + 1) block only syev_kernel uses (its Z; its matrix takes
// the place of V), the inverse-iteration factors (4 c^2), and after them d, e, the eigenvalues and the
// reflector scalars tau (q unused).
struct SyevSplit {
  int64_t q, d, e, lam, tau;
};
__device__ __host__ inline SyevSplit syev_split_offsets(int c) {
  if (c > 96) {
    const int64_t d = 2 * (int64_t)c * (c + 1) + 4 * (int64_t)c * c;
    return {0, d, d + c, d + 2 * c, d + 3 * c};
  }
  const int64_t q = 4 * (int64_t)c * c, d = q + (int64_t)c * (c + 1);
  return {q, d, d + c, d + 2 * c, d + 3 * c};
}

// All four steps in one workgroup per problem, the matrix in LDS (c <= 96) or in the global scratch: the
// form for c > 96 when the three-launch form does not apply (large batches, nev > 64).
__global__ void __launch_bounds__(kSyevThreads) syev_kernel(const double* __restrict__ H, int64_t ldh,
                                                            int64_t hstride, int c, int nev,
                                                            double* __restrict__ evals, int64_t estride,
                                                            double* __restrict__ C, int64_t cstride,
                                                            double* __restrict__ work, int64_t wstride, int* info,
                                                            const int32_t* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  H += (int64_t)blockIdx.x * hstride;
  evals += (int64_t)blockIdx.x * estride;
  C += (int64_t)blockIdx.x * cstride;
  work += (int64_t)blockIdx.x * wstride;
  __shared__ double sa[kSyevLds * (kSyevLds + 1)];
  __shared__ double sz[kSyevLds * (kSyevLds + 1)];
  __shared__ double d[kSyevMax], e[kSyevMax], tau[kSyevMax];
  __shared__ double s1[kSyevMax + 8], s2[kSyevMax];   // v, p (step 1) | e^2, bracket lows (step 2)
  __shared__ double s3[kSyevMax + 8];
  __shared__ double lam[kSyevMax];                // bracket highs, then eigenvalues
  __shared__ int cnt[kSyevThreads];
  __shared__ short cend[kSyevMax];
  __shared__ double sc[8];
  const int tid = threadIdx.x, lane = tid % 64, wid = tid / 64;
  const int la = c + 1;
  const bool in_lds = (c <= kSyevLds);
  double* a = in_lds ? sa : work;
  double* Z = in_lds ? sz : work + (int64_t)c * la;   // c x nev, row stride la
  double* lu = work + 2 * (int64_t)c * la;            // U0 | U1 | L | piv, each c x nev, index [k * nev + j]
  for (int q = tid; q < c * c; q += kSyevThreads) {
    const int i = q / c, j = q % c;
    a[i * la + j] = 0.5 * (H[(int64_t)i * ldh + j] + H[(int64_t)j * ldh + i]);
  }
  __syncthreads();
  // ---- 1. tridiagonalization ----
  double* v = s1;
  double* p = s2;
  for (int k = 0; k + 2 < c; ++k) {
    const int nk = c - k - 1;
    if (wid == 0) {
      double ss = 0.0;
      for (int i = k + 2 + lane; i < c; i += 64) ss += a[i * la + k] * a[i * la + k];
      ss = wave_sum(ss);
      if (lane == 0) sc[k & 1] = ss;
    }
    __syncthreads();
    const double ss = sc[k & 1];
    const double alpha = a[(k + 1) * la + k];
    double t = 0.0, beta = alpha, scale = 0.0;
    if (ss > 0.0) {
      const double xn = sqrt(alpha * alpha + ss);
      beta = (alpha >= 0.0) ? -xn : xn;
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    if (tid == 0) {
      tau[k] = t;
      e[k] = beta;
      d[k] = a[k * la + k];
    }
    if (t == 0.0) continue;   // uniform; sc is double-buffered across this barrier-free skip
    for (int i = tid; i < nk; i += kSyevThreads) v[i] = (i == 0) ? 1.0 : a[(k + 1 + i) * la + k] * scale;
    __syncthreads();
    for (int i = tid + 1; i < nk; i += kSyevThreads) a[(k + 1 + i) * la + k] = v[i];
    if (tid == 0) a[(k + 1) * la + k] = beta;
    // p = t A22 v: two threads per row, each half of the columns of the symmetric A22 (read by
    // columns so that consecutive threads read consecutive addresses), four partial sums each
    for (int i = tid >> 1; i < nk; i += kSyevThreads / 2) {
      const int h = tid & 1;
      double s0 = 0.0, s1p = 0.0, s2p = 0.0, s3 = 0.0;
      int j = h;
      for (; j + 6 < nk; j += 8) {
        s0 += a[(k + 1 + j) * la + k + 1 + i] * v[j];
        s1p += a[(k + 3 + j) * la + k + 1 + i] * v[j + 2];
        s2p += a[(k + 5 + j) * la + k + 1 + i] * v[j + 4];
        s3 += a[(k + 7 + j) * la + k + 1 + i] * v[j + 6];
      }
      for (; j < nk; j += 2) s0 += a[(k + 1 + j) * la + k + 1 + i] * v[j];
      double sum = (s0 + s1p) + (s2p + s3);
      sum += __shfl_xor(sum, 1, 64);
      if (h == 0) p[i] = t * sum;
    }
    __syncthreads();
    if (wid == 0) {
      double pv = 0.0;
      for (int i = lane; i < nk; i += 64) pv += p[i] * v[i];
      pv = wave_sum(pv);
      if (lane == 0) sc[2 + (k & 1)] = pv;
    }
    __syncthreads();
    const double K = 0.5 * t * sc[2 + (k & 1)];
    // A22 -= v w^T + w v^T with w = p - K v: lane owns columns j, wave w the rows i = w mod
    // kSyevWaves, four rows per step so that their loads are in flight together
    for (int j = lane; j < nk; j += 64) {
      const double vj = v[j], wj = p[j] - K * vj;
      double* col = a + (k + 1) * la + k + 1 + j;
      constexpr int NV = kSyevWaves;
      int i = wid;
      for (; i + 3 * NV < nk; i += 4 * NV) {
        const double v0 = v[i], v1 = v[i + NV], v2 = v[i + 2 * NV], v3 = v[i + 3 * NV];
        const double w0 = p[i] - K * v0, w1 = p[i + NV] - K * v1, w2 = p[i + 2 * NV] - K * v2,
                     w3 = p[i + 3 * NV] - K * v3;
        const double a0 = col[i * la], a1 = col[(i + NV) * la], a2 = col[(i + 2 * NV) * la],
                     a3 = col[(i + 3 * NV) * la];
        col[i * la] = a0 - (v0 * wj + w0 * vj);
        col[(i + NV) * la] = a1 - (v1 * wj + w1 * vj);
        col[(i + 2 * NV) * la] = a2 - (v2 * wj + w2 * vj);
        col[(i + 3 * NV) * la] = a3 - (v3 * wj + w3 * vj);
      }
      for (; i < nk; i += NV) {
        const double vi = v[i], wi = p[i] - K * vi;
        col[i * la] -= vi * wj + wi * vj;
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) {
    for (int k = (c >= 2 ? c - 2 : 0); k < c; ++k) d[k] = a[k * la + k];
    if (c >= 2) e[c - 2] = a[(c - 1) * la + c - 2];
    if (c >= 2) tau[c - 2] = 0.0;
    tau[c - 1] = 0.0;
    e[c - 1] = 0.0;
  }
  __syncthreads();
  const int maxrank = tridiag_eigs<0, 0>(d, e, c, nev, s1, s2, s3, lam, cnt, cend, Z, in_lds ? la : nev, lu);
  const int lz = in_lds ? la : nev;   // row stride of Z
  // ---- 4. back-transformation C = Q Z: G threads per column (a power of two), each a row segment ----
  int G = 1;
  while (G * 2 * nev <= kSyevThreads && G < 64) G *= 2;
  {
    const int j = tid / G, g = tid % G;
    for (int k = c - 3; k >= 0; --k) {
      const double t = tau[k];
      if (t == 0.0) continue;
      const int nk = c - k - 1;
      // a thread's rows of this column: at most ceil(191 / G) <= 192 / G; held in registers in
      // chunks of 8 so that the loads are issued before the stores
      double sw = 0.0;
      if (j < nev)
        for (int i0 = g; i0 < nk; i0 += 8 * G) {
          double vv[8], zz[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * G;
            vv[u] = (i < nk) ? (i == 0 ? 1.0 : a[(k + 1 + i) * la + k]) : 0.0;
            zz[u] = (i < nk) ? Z[(k + 1 + i) * lz + j] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) sw += vv[u] * zz[u];
        }
      for (int off = G / 2; off > 0; off >>= 1) sw += __shfl_xor(sw, off, 64);
      sw *= t;
      if (j < nev)
        for (int i0 = g; i0 < nk; i0 += 8 * G) {
          double vv[8], zz[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * G;
            vv[u] = (i < nk) ? (i == 0 ? 1.0 : a[(k + 1 + i) * la + k]) : 0.0;
            zz[u] = (i < nk) ? Z[(k + 1 + i) * lz + j] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (i0 + u * G < nk) Z[(k + 1 + i0 + u * G) * lz + j] = zz[u] - vv[u] * sw;
        }
      __syncthreads();   // the next reflector reads rows another thread of the group wrote
    }
  }
  __syncthreads();
  for (int q = tid; q < c * nev; q += kSyevThreads) {
    const int i = q / nev, j = q % nev;
    C[(int64_t)i * c + j] = Z[i * lz + j];
  }
  for (int j = tid; j < nev; j += kSyevThreads) evals[j] = lam[j];
  if (tid == 0 && info) info[blockIdx.x] = maxrank;
}


// Reflectors k = 16 AK .. 16 AK + 15 of the register tridiagonalization (see syev_reg_kernel);
// AK is static so that the owner's row A[AK] and the finished blocks below AK are known at compile
// time.  vb, pb: 2 x 16 NB doubles of LDS, pvp: 2 x 16, tb: 2 (double-buffered by step parity).
template <int NB, int AK>
__device__ __attribute__((always_inline)) void tridiag_rows(double (&A)[NB][NB], double (&Q)[NB][NB], int c, int ti,
                                                            int tj, double* vb, double* pb, double* pvp, double* tb,
                                                            double* d, double* e) {
  constexpr int CM = 16 * NB;
#pragma unroll 1
  for (int r = 0; r < 16; ++r) {
    const int k = 16 * AK + r;
    if (k + 2 >= c) break;   // uniform
    const int buf = k & 1;
    if (ti == r) {
      double ss = 0.0, al = 0.0;
#pragma unroll
      for (int b = AK; b < NB; ++b) {
        const int j = tj + 16 * b;
        const double x = A[AK][b];
        ss += (j >= k + 2) ? x * x : 0.0;
        al += (j == k + 1) ? x : 0.0;
        if (j == k) d[k] = x;
      }
      ss = row16_sum(ss);
      al = row16_sum(al);
      double t = 0.0, beta = al, scale = 0.0;
      if (ss > 0.0) {
        const double xn = sqrt(al * al + ss);
        beta = (al >= 0.0) ? -xn : xn;
        t = (beta - al) / beta;
        scale = 1.0 / (al - beta);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = tj + 16 * b;
        vb[buf * CM + j] = (b >= AK && j > k + 1) ? A[AK][b] * scale : (j == k + 1 ? 1.0 : 0.0);
      }
      if (tj == 0) {
        tb[buf] = t;
        e[k] = beta;
      }
    }
    __syncthreads();
    const double t = tb[buf];
    if (t == 0.0) continue;   // uniform; every buffer is double-buffered by step parity
    // rows and columns below 16 AK are finished: their blocks are skipped (AK is static here)
    double vc[NB], vr[NB], pp[NB], qq[NB];
#pragma unroll
    for (int b = AK; b < NB; ++b) vc[b] = vb[buf * CM + tj + 16 * b];
#pragma unroll
    for (int a = AK; a < NB; ++a) vr[a] = vb[buf * CM + ti + 16 * a];
    double pv = 0.0;
#pragma unroll
    for (int a = AK; a < NB; ++a) {
      double sp = 0.0;
#pragma unroll
      for (int b = AK; b < NB; ++b) sp = fma(A[a][b], vc[b], sp);
      pp[a] = t * row16_sum(sp);
      pv = fma(pp[a], vr[a], pv);
    }
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      double sq_ = 0.0;
#pragma unroll
      for (int b = AK; b < NB; ++b) sq_ = fma(Q[a][b], vc[b], sq_);
      qq[a] = t * row16_sum(sq_);
    }
    if (tj == 0) {
#pragma unroll
      for (int a = AK; a < NB; ++a) pb[buf * CM + ti + 16 * a] = pp[a];
      pvp[buf * 16 + ti] = pv;
    }
    __syncthreads();
    double K = 0.0;
#pragma unroll
    for (int g = 0; g < 16; ++g) K += pvp[buf * 16 + g];
    K *= 0.5 * t;
    double wc[NB];
#pragma unroll
    for (int b = AK; b < NB; ++b) wc[b] = pb[buf * CM + tj + 16 * b] - K * vc[b];
#pragma unroll
    for (int a = AK; a < NB; ++a) {
      const double wr = pp[a] - K * vr[a];
#pragma unroll
      for (int b = AK; b < NB; ++b) A[a][b] -= vr[a] * wc[b] + wr * vc[b];
    }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = AK; b < NB; ++b) Q[a][b] -= qq[a] * vc[b];
  }
  if constexpr (AK + 1 < NB) tridiag_rows<NB, AK + 1>(A, Q, c, ti, tj, vb, pb, pvp, tb, d, e);
}

// The eigensolver above for c <= 16 NB with the matrix in registers.  Thread (ti, tj) of a 16 x 16
// grid (wave ti / 4, lanes 16 (ti % 4) .. 16 (ti % 4) + 15) holds H(ti + 16 a, tj + 16 b),
// a, b < NB, and the same entries of Q = H_0 H_1 ... H_{c-3}, the product of the reflectors.
// Reflector k (step 1): the 16 lanes of row k form v and t from that row and publish them; after
// a barrier every row forms its entries of p = t H v and Q v by a 16-lane sum and publishes p and
// its share of p^T v; after a second barrier every thread applies H -= v w^T + w v^T,
// w = p - (t / 2) (p^T v) v, and Q -= t (Q v) v^T to its own entries.  Steps 2 and 3 are those of
// the LDS form; step 4 is C = Q Z, one matrix-core product of Q and Z from LDS.
// Eigenvalue j = blockIdx.x of the tridiagonal T that syev_tridiag_kernel<NB> left in the scratch,
// by multisection on Sturm counts with kSyevThreads points per round (the Gershgorin interval,
// tolerance and scaled counts are those of tridiag_eigs, so the bracket invariant
// count(lo) <= j < count(hi) and the stopping rule are the same; only the number of points per
// round differs).  The new bracket is the last point before the first point whose count exceeds j
// and that point, found with wave ballots.
__global__ void __launch_bounds__(kSyevThreads) syev_bisect_kernel(double* __restrict__ work, int64_t wstride, int c,
                                                                   int nev, const int32_t* __restrict__ active) {
  if (active && !active[blockIdx.y]) return;
  work += (int64_t)blockIdx.y * wstride;
  const int j = blockIdx.x;
  if (j >= nev) return;
  const SyevSplit sp = syev_split_offsets(c);
  __shared__ double ds[kSyevMax + 8], e2[kSyevMax + 8];
  __shared__ int wfirst[kSyevWaves], wva[kSyevWaves], wvb[kSyevWaves];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const double* d = work + sp.d;
  const double* e = work + sp.e;
  double gl = 1e300, gu = -1e300, tnorm = 0.0, emax2 = 0.0;
  for (int i = lane; i < c; i += 64) {
    const double ei = (i < c - 1) ? fabs(e[i]) : 0.0;
    const double em = (i > 0) ? fabs(e[i - 1]) : 0.0;
    gl = fmin(gl, d[i] - ei - em);
    gu = fmax(gu, d[i] + ei + em);
    tnorm = fmax(tnorm, fabs(d[i]) + ei + em);
    emax2 = fmax(emax2, ei * ei);
  }
  for (int off = 32; off > 0; off >>= 1) {
    gl = fmin(gl, __shfl_xor(gl, off, 64));
    gu = fmax(gu, __shfl_xor(gu, off, 64));
    tnorm = fmax(tnorm, __shfl_xor(tnorm, off, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, off, 64));
  }
  const double eps = 2.220446049250313e-16;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  gl -= 2.0 * eps * tnorm * c + 2.0 * pivmin;
  gu += 2.0 * eps * tnorm * c + 2.0 * pivmin;
  const double sc = (tnorm > 0.0) ? ldexp(1.0, -ilogb(tnorm)) : 1.0;
  const double pmin = fmax(sc * pivmin, 0x1p-100);
  for (int i = tid; i < c + 8; i += kSyevThreads) {
    const double es = (i < c - 1) ? sc * e[i] : 0.0;
    e2[i] = es * es;
    ds[i] = (i < c) ? sc * d[i] : 8.0;
  }
  __syncthreads();
  double l = gl, h = gu;   // the same in every thread
  constexpr double inv = 1.0 / (double)(kSyevThreads + 1);
  for (int round = 0; round < 200; ++round) {
    if (!(h - l > 2.0 * eps * fmax(fabs(l), fabs(h)) + pivmin)) break;
    const double w = h - l;
    const double x = l + w * ((double)(tid + 1) * inv);
    // the points are nondecreasing in tid, so the valid ones (strictly inside) are a contiguous run
    const bool valid = (x > l && x < h);
    const bool above = valid && sturm_count_scaled(ds, e2, c, sc * x, pmin) >= j + 1;
    const uint64_t ma = __ballot(above), mv = __ballot(valid);
    if (lane == 0) {
      wfirst[wid] = ma ? 64 * wid + __builtin_ctzll(ma) : kSyevThreads;
      wva[wid] = mv ? 64 * wid + __builtin_ctzll(mv) : kSyevThreads;
      wvb[wid] = mv ? 64 * wid + 64 - __builtin_clzll(mv) : -1;
    }
    __syncthreads();
    int tc = kSyevThreads, va = kSyevThreads, vb = -1;
#pragma unroll
    for (int w2 = 0; w2 < kSyevWaves; ++w2) {
      tc = min(tc, wfirst[w2]);
      va = min(va, wva[w2]);
      vb = max(vb, wvb[w2]);
    }
    __syncthreads();
    auto point = [l, w](int t) { return l + w * ((double)(t + 1) * inv); };
    const int end = (tc < kSyevThreads) ? tc : vb;   // one past the last point kept as the low end
    const double nl = (end - 1 >= va) ? point(end - 1) : l;
    double nh = (tc < kSyevThreads) ? point(tc) : h;
    if (nl == l && nh == h) nh = nl;   // no interior point strictly inside: the bracket is at ulp level
    l = nl;
    h = nh;
  }
  if (tid == 0) work[sp.lam + j] = 0.5 * (l + h);
}

// Step 1 with the work of each reflector split between two groups of four waves on the same 16 x 16
// thread grid: the matrix group holds H (thread (ti, tj): entries (ti + 16 a, tj + 16 b)), forms v
// and t and applies H -= v w^T + w v^T as tridiag_rows does; the Q group holds the same entries of
// Q and applies Q -= t (Q v) v^T, rows a < NB / 2 while the matrix group forms p = t H v and the
// others while it applies the update.  The reflector of step k + 1 is formed ahead: after the second
// barrier of step k, the grid row owning row k + 1 updates that row first, forms and publishes v and t
// from it, and only then updates its other rows, so that the next step's first barrier does not wait
// for a whole update followed by the owner's norms and divisions.  M is H or Q by group; QG: this thread
// is in the Q group (wave-uniform).

// Owner phase: v and t of the reflector of row kk (in the static 16-row block AO) from that row's
// entries, published in buffer kk & 1, with d[kk] and e[kk].
template <int NB, int AO>
__device__ __attribute__((always_inline)) void tri_owner(const double (&M)[NB][NB], int kk, int tj, double* vb,
                                                         double* tb, double* d, double* e, double* tau, double* ga,
                                                         int la, int c) {
  constexpr int CM = 16 * NB;
  const int buf = kk & 1;
  double ss = 0.0, al = 0.0;
#pragma unroll
  for (int b = AO; b < NB; ++b) {
    const int j = tj + 16 * b;
    const double x = M[AO][b];
    ss += (j >= kk + 2) ? x * x : 0.0;
    al += (j == kk + 1) ? x : 0.0;
    if (j == kk) d[kk] = x;
  }
  ss = row16_sum(ss);
  al = row16_sum(al);
  double t = 0.0, beta = al, scale = 0.0;
  if (ss > 0.0) {
    const double xn = sqrt(al * al + ss);
    beta = (al >= 0.0) ? -xn : xn;
    t = (beta - al) / beta;
    scale = 1.0 / (al - beta);
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = tj + 16 * b;
    const double v = (b >= AO && j > kk + 1) ? M[AO][b] * scale : (j == kk + 1 ? 1.0 : 0.0);
    vb[buf * CM + j] = v;
    if (ga && j < c) ga[(int64_t)kk * la + j] = v;
  }
  if (tj == 0) {
    tb[buf] = t;
    e[kk] = beta;
    if (tau) tau[kk] = t;
  }
}

// Q rows a in [A0, A1): Q(a, :) -= t (Q(a, :) v) v^T, over the column blocks from B0 (v is zero before).
template <int NB, int A0, int A1, int B0>
__device__ __attribute__((always_inline)) void tri_qrows(double (&M)[NB][NB], const double (&vc)[NB], double t) {
#pragma unroll
  for (int a = A0; a < A1; ++a) {
    double sq_ = 0.0;
#pragma unroll
    for (int b = B0; b < NB; ++b) sq_ = fma(M[a][b], vc[b], sq_);
    const double qa = t * row16_sum(sq_);
#pragma unroll
    for (int b = B0; b < NB; ++b) M[a][b] -= qa * vc[b];
  }
}

template <int NB, int AK>
__device__ __attribute__((always_inline)) void tridiag_rows_split(double (&M)[NB][NB], bool QG, int c, int ti,
                                                                  int tj, double* vb, double* pb, double* pvp,
                                                                  double* tb, double* d, double* e, double* tau,
                                                                  double* ga, int la) {
  constexpr int CM = 16 * NB, QH = NB / 2;
#pragma unroll 1
  for (int r = 0; r < 16; ++r) {
    const int k = 16 * AK + r;
    if (k + 2 >= c) break;   // uniform
    const int buf = k & 1;
    // the owner of row k + 1 (when there is a reflector k + 1): grid row (k + 1) % 16, block AK or AK + 1
    const bool own = !QG && (k + 3 < c) && ti == ((r + 1) & 15);
    __syncthreads();
    const double t = tb[buf];
    double vc[NB];
#pragma unroll
    for (int b = AK; b < NB; ++b) vc[b] = vb[buf * CM + tj + 16 * b];
    if (t == 0.0) {   // uniform: the reflector is the identity, H and Q stay as they are
      if (own) {
        if (r < 15) tri_owner<NB, AK>(M, k + 1, tj, vb, tb, d, e, tau, ga, la, c);
        else if constexpr (AK + 1 < NB) tri_owner<NB, AK + 1>(M, k + 1, tj, vb, tb, d, e, tau, ga, la, c);
      }
      continue;   // every buffer is double-buffered by step parity
    }
    double pp[NB], vr[NB];
    if (QG) {
      tri_qrows<NB, 0, QH, AK>(M, vc, t);
    } else {
#pragma unroll
      for (int a = AK; a < NB; ++a) vr[a] = vb[buf * CM + ti + 16 * a];
      double pv = 0.0;
#pragma unroll
      for (int a = AK; a < NB; ++a) {
        double sp = 0.0;
#pragma unroll
        for (int b = AK; b < NB; ++b) sp = fma(M[a][b], vc[b], sp);
        pp[a] = t * row16_sum(sp);
        pv = fma(pp[a], vr[a], pv);
      }
      if (tj == 0) {
#pragma unroll
        for (int a = AK; a < NB; ++a) pb[buf * CM + ti + 16 * a] = pp[a];
        pvp[buf * 16 + ti] = pv;
      }
    }
    __syncthreads();
    if (QG) {
      tri_qrows<NB, QH, NB, AK>(M, vc, t);
    } else {
      double g[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) g[q] = pvp[buf * 16 + q];
#pragma unroll
      for (int h = 8; h > 0; h >>= 1)
#pragma unroll
        for (int q = 0; q < h; ++q) g[q] += g[q + h];
      const double K = 0.5 * t * g[0];
      double wc[NB];
#pragma unroll
      for (int b = AK; b < NB; ++b) wc[b] = pb[buf * CM + tj + 16 * b] - K * vc[b];
      // row a of this thread's block: H(a, :) -= v_a w^T + w_a v^T
      auto upd = [&](auto ac) {
        constexpr int a = decltype(ac)::value;
        const double wr = pp[a] - K * vr[a];
#pragma unroll
        for (int b = AK; b < NB; ++b) M[a][b] -= vr[a] * wc[b] + wr * vc[b];
      };
      // the owner's row k + 1 first, then its reflector, then the other rows
      const int ao = (r < 15) ? AK : AK + 1;
      if (own) {
        if (r < 15) {
          upd(std::integral_constant<int, AK>{});
          tri_owner<NB, AK>(M, k + 1, tj, vb, tb, d, e, tau, ga, la, c);
        } else if constexpr (AK + 1 < NB) {
          upd(std::integral_constant<int, AK + 1>{});
          tri_owner<NB, AK + 1>(M, k + 1, tj, vb, tb, d, e, tau, ga, la, c);
        }
      }
      static_for<AK, NB>([&](auto ac) {
        if (!(own && decltype(ac)::value == ao)) upd(ac);
      });
    }
  }
  if constexpr (AK + 1 < NB) tridiag_rows_split<NB, AK + 1>(M, QG, c, ti, tj, vb, pb, pvp, tb, d, e, tau, ga, la);
}

// Step 1 of the three-launch form: T (d, e with e[c - 1] = 0) and Q^T to the global scratch, with
// 2 kSyevThreads threads (the two groups of tridiag_rows_split).
template <int NB>
__global__ void __launch_bounds__(2 * kSyevThreads) syev_tridiag_kernel(const double* __restrict__ H, int64_t ldh,
                                                                        int64_t hstride, int c,
                                                                        double* __restrict__ work, int64_t wstride,
                                                                        const int32_t* __restrict__ active) {
  constexpr int CM = 16 * NB;
  if (active && !active[blockIdx.x]) return;
  H += (int64_t)blockIdx.x * hstride;
  work += (int64_t)blockIdx.x * wstride;
  __shared__ double vb[2][CM], pb[2][CM], pvp[2][16], tb[2];
  __shared__ double d[CM], e[CM];
  const SyevSplit sp = syev_split_offsets(c);
  const int tid = threadIdx.x;
  const bool QG = tid >= kSyevThreads;   // waves 4..7
  const int g = tid & (kSyevThreads - 1), lane = g & 63, wid = g >> 6;
  const int ti = wid * 4 + (lane >> 4), tj = lane & 15;
  double M[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = ti + 16 * a, j = tj + 16 * b;
      if (QG) {
        M[a][b] = (i == j) ? 1.0 : 0.0;
      } else {   // clamped addresses: unconditional loads, all in flight together
        const int ic = min(i, c - 1), jc = min(j, c - 1);
        M[a][b] = keep_if(i < c && j < c, 0.5 * (H[(int64_t)ic * ldh + jc] + H[(int64_t)jc * ldh + ic]));
      }
    }
  // reflector 0 is formed before the loop; every later one by the owner of its row at the end of the step
  // before it
  if (!QG && ti == 0 && c > 2) tri_owner<NB, 0>(M, 0, tj, &vb[0][0], tb, d, e, nullptr, nullptr, 0, c);
  tridiag_rows_split<NB, 0>(M, QG, c, ti, tj, &vb[0][0], &pb[0][0], &pvp[0][0], tb, d, e, nullptr, nullptr, 0);
  double* gq = work + sp.q;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = ti + 16 * a, j = tj + 16 * b;
      if (QG) {
        if (i < c && j < c) gq[j * (c + 1) + i] = M[a][b];   // transposed
      } else {
        if (i == j && i + 2 >= c && i < c) d[i] = M[a][b];
        if (c >= 2 && i == c - 1 && j == c - 2) e[c - 2] = M[a][b];
      }
    }
  __syncthreads();
  for (int i = tid; i < c; i += 2 * kSyevThreads) {
    work[sp.d + i] = d[i];
    work[sp.e + i] = (i < c - 1) ? e[i] : 0.0;
  }
}

// Sum over the 32 lanes of a half wave (lanes 32 h .. 32 h + 15 and 32 h + 16 .. 32 h + 31): both halves
// of the pair add the same two values, so every lane of the half ends with the same bits.
__device__ inline double row32_sum(double x) {
  x = row16_sum(x);
  return x + __shfl_xor(x, 16, 64);
}

// Step 1 for 96 < c <= 192 (three-launch form): the matrix in the registers of a 16 x 32 thread grid of
// 512 threads, thread (ti, tj) = (2 wave + lane / 32, lane % 32) holding H(ti + 16 a, tj + 32 b), a < 12,
// b < 6 (72 doubles).  Reflector k: the 32 lanes of grid row k % 16 form v and t from their entries of row
// k and publish them; after a barrier every grid row forms its entries of p = t H v by a 32-lane sum and
// publishes them with its share of p^T v; after a second barrier every thread applies H -= v w^T + w v^T
// with w = p - (t / 2)(p^T v) v.  Q is not formed: reflector k goes to row k of the scratch's V (row
// stride c + 1; zero before entry k + 1, which is 1), with tau, d and e after it, for syev_bt_kernel to
// apply to Z.  Rows of the 16-row blocks before AK and columns of the 32-column blocks before AK / 2 are
// finished and skipped.
constexpr int kT32Rows = 12, kT32Cols = 6, kSyevThreads32 = 512;

template <int AK>
__device__ __attribute__((always_inline)) void tridiag32_rows(double (&A)[kT32Rows][kT32Cols], int c, int ti, int tj,
                                                              double* vb, double* pb, double* pvp, double* tb,
                                                              double* d, double* e, double* tau, double* ga, int la) {
  constexpr int CM = 192, NA = kT32Rows, NBC = kT32Cols, BK = AK / 2;
#pragma unroll 1
  for (int r = 0; r < 16; ++r) {
    const int k = 16 * AK + r;
    if (k + 2 >= c) break;   // uniform
    const int buf = k & 1;
    if (ti == r) {
      double ss = 0.0, al = 0.0;
#pragma unroll
      for (int b = BK; b < NBC; ++b) {
        const int j = tj + 32 * b;
        const double x = A[AK][b];
        ss += (j >= k + 2) ? x * x : 0.0;
        al += (j == k + 1) ? x : 0.0;
        if (j == k) d[k] = x;
      }
      ss = row32_sum(ss);
      al = row32_sum(al);
      double t = 0.0, beta = al, scale = 0.0;
      if (ss > 0.0) {
        const double xn = sqrt(al * al + ss);
        beta = (al >= 0.0) ? -xn : xn;
        t = (beta - al) / beta;
        scale = 1.0 / (al - beta);
      }
#pragma unroll
      for (int b = 0; b < NBC; ++b) {
        const int j = tj + 32 * b;
        const double v = (b >= BK && j > k + 1) ? A[AK][b] * scale : (j == k + 1 ? 1.0 : 0.0);
        vb[buf * CM + j] = v;
        if (j < c) ga[(int64_t)k * la + j] = v;
      }
      if (tj == 0) {
        tb[buf] = t;
        tau[k] = t;
        e[k] = beta;
      }
    }
    __syncthreads();
    const double t = tb[buf];
    if (t == 0.0) continue;   // uniform; every buffer is double-buffered by step parity
    double vc[NBC];
#pragma unroll
    for (int b = BK; b < NBC; ++b) vc[b] = vb[buf * CM + tj + 32 * b];
    double pv = 0.0;
#pragma unroll
    for (int a = AK; a < NA; ++a) {
      double sp = 0.0;
#pragma unroll
      for (int b = BK; b < NBC; ++b) sp = fma(A[a][b], vc[b], sp);
      const double pa = t * row32_sum(sp);
      pv = fma(pa, vb[buf * CM + ti + 16 * a], pv);
      if (tj == 0) pb[buf * CM + ti + 16 * a] = pa;
    }
    if (tj == 0) pvp[buf * 16 + ti] = pv;
    __syncthreads();
    double K = 0.0;
#pragma unroll
    for (int g = 0; g < 16; ++g) K += pvp[buf * 16 + g];
    K *= 0.5 * t;
    double wc[NBC];
#pragma unroll
    for (int b = BK; b < NBC; ++b) wc[b] = pb[buf * CM + tj + 32 * b] - K * vc[b];
#pragma unroll
    for (int a = AK; a < NA; ++a) {
      const double vr = vb[buf * CM + ti + 16 * a];
      const double wr = pb[buf * CM + ti + 16 * a] - K * vr;
#pragma unroll
      for (int b = BK; b < NBC; ++b) A[a][b] -= vr * wc[b] + wr * vc[b];
    }
  }
  if constexpr (AK + 1 < NA) tridiag32_rows<AK + 1>(A, c, ti, tj, vb, pb, pvp, tb, d, e, tau, ga, la);
}

__global__ void __launch_bounds__(kSyevThreads32) syev_tridiag32_kernel(const double* __restrict__ H, int64_t ldh,
                                                                        int64_t hstride, int c,
                                                                        double* __restrict__ work, int64_t wstride,
                                                                        const int32_t* __restrict__ active) {
  constexpr int CM = 192;
  if (active && !active[blockIdx.x]) return;
  H += (int64_t)blockIdx.x * hstride;
  work += (int64_t)blockIdx.x * wstride;
  __shared__ double vb[2][CM], pb[2][CM], pvp[2][16], tb[2];
  __shared__ double d[CM], e[CM], tau[CM];
  const SyevSplit sp = syev_split_offsets(c);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int ti = 2 * wid + (lane >> 5), tj = lane & 31;
  const int la = c + 1;
  double A[kT32Rows][kT32Cols];
#pragma unroll
  for (int a = 0; a < kT32Rows; ++a)
#pragma unroll
    for (int b = 0; b < kT32Cols; ++b) {
      const int i = ti + 16 * a, j = tj + 32 * b;
      const int ic = min(i, c - 1), jc = min(j, c - 1);   // clamped: unconditional loads
      A[a][b] = keep_if(i < c && j < c, 0.5 * (H[(int64_t)ic * ldh + jc] + H[(int64_t)jc * ldh + ic]));
    }
  tridiag32_rows<0>(A, c, ti, tj, &vb[0][0], &pb[0][0], &pvp[0][0], tb, d, e, tau, work, la);
#pragma unroll
  for (int a = 0; a < kT32Rows; ++a)
#pragma unroll
    for (int b = 0; b < kT32Cols; ++b) {
      const int i = ti + 16 * a, j = tj + 32 * b;
      if (i == j && i + 2 >= c && i < c) d[i] = A[a][b];
      if (c >= 2 && i == c - 1 && j == c - 2) e[c - 2] = A[a][b];
    }
  __syncthreads();
  for (int i = tid; i < c; i += kSyevThreads32) {
    work[sp.d + i] = d[i];
    work[sp.e + i] = (i < c - 1) ? e[i] : 0.0;
    work[sp.tau + i] = (i + 2 < c) ? tau[i] : 0.0;
  }
}

// Step 3 of the reflector form (96 < c <= 192, nev <= 64; after syev_tridiag32_kernel and
// syev_bisect_kernel): inverse iteration with Z in LDS, the factors in LDS when
// they fit beside it and in the global scratch otherwise, and the cluster re-orthonormalisation in
// registers (NR rows x NC columns per thread, c <= 16 NR, nev <= 16 NC); Z goes to C(:, 0:nev) for
// syev_bt_kernel.
constexpr int kVecNev = 64, kVecPool = 18528;   // doubles: Z, and the factors when c (5 nev + 1) fits
template <int NR, int NC>
__global__ void __launch_bounds__(kSyevThreads) syev_vec_kernel(double* __restrict__ C, int64_t cstride, int c,
                                                                int nev, double* __restrict__ evals, int64_t estride,
                                                                double* __restrict__ work, int64_t wstride, int* info,
                                                                const int32_t* __restrict__ active) {
  constexpr int CM = 16 * NR;
  static_assert(CM * (kVecNev + 1) <= kVecPool, "Z fits in the pool");
  if (active && !active[blockIdx.x]) return;
  evals += (int64_t)blockIdx.x * estride;
  C += (int64_t)blockIdx.x * cstride;
  work += (int64_t)blockIdx.x * wstride;
  __shared__ double pool[kVecPool];
  __shared__ double d[CM], e[CM], lam[CM];
  __shared__ double s1[CM + 8], s2[CM], s3[CM + 8];
  __shared__ int cnt[kSyevThreads];
  __shared__ short cend[CM];
  const SyevSplit sp = syev_split_offsets(c);
  const int tid = threadIdx.x;
  for (int i = tid; i < c; i += kSyevThreads) {
    d[i] = work[sp.d + i];
    e[i] = work[sp.e + i];
    lam[i] = (i < nev) ? work[sp.lam + i] : 0.0;
  }
  __syncthreads();
  const int lz = nev + 1;
  double* Z = pool;
  const bool lu_lds = (int64_t)c * lz + 4 * (int64_t)c * nev <= kVecPool;   // uniform
  // two inlined copies, so that the factors are addressed as LDS or as global memory
  const int maxrank =
      lu_lds ? tridiag_eigs<NR, NC, true, 8>(d, e, c, nev, s1, s2, s3, lam, cnt, cend, Z, lz, pool + (int64_t)c * lz)
             : tridiag_eigs<NR, NC, true, 16>(d, e, c, nev, s1, s2, s3, lam, cnt, cend, Z, lz,
                                              work + 2 * (int64_t)c * (c + 1));
  for (int q = tid; q < c * nev; q += kSyevThreads) {
    const int i = q / nev, j = q - i * nev;
    C[(int64_t)i * c + j] = Z[i * lz + j];
  }
  for (int j = tid; j < nev; j += kSyevThreads) evals[j] = lam[j];
  if (tid == 0 && info) info[blockIdx.x] = maxrank;
}

// Step 4 of the reflector form: C(:, 0:nev) <- Q C(:, 0:nev) with Q = H_0 H_1 ... H_{c-3} from the reflector
// rows V, H_k = I - tau_k v_k v_k^T applied for k = c - 3 down to 0.  Columns are independent: workgroup
// (x, problem) takes 8 of them, 32 lanes per column, each lane RPL rows (i = lane32 + 32 u, c <= 32 RPL)
// in registers, so a reflector costs a 32-lane sum and no barrier.  Reflectors are staged through LDS 16
// at a time (double-buffered; one barrier per 16).
constexpr int kBtCols = 8, kBtStage = 16;
template <int RPL>
__global__ void __launch_bounds__(kSyevThreads) syev_bt_kernel(double* __restrict__ C, int64_t cstride, int c,
                                                               int nev, const double* __restrict__ work,
                                                               int64_t wstride, const int32_t* __restrict__ active) {
  constexpr int CM = 32 * RPL;
  if (active && !active[blockIdx.y]) return;
  C += (int64_t)blockIdx.y * cstride;
  work += (int64_t)blockIdx.y * wstride;
  __shared__ double vs[2][kBtStage][CM];
  __shared__ double ts[2][kBtStage];
  const SyevSplit sp = syev_split_offsets(c);
  const int tid = threadIdx.x, l32 = tid & 31;
  const int j = kBtCols * blockIdx.x + (tid >> 5);
  const bool jok = j < nev;
  const int la = c + 1;
  double z[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int i = l32 + 32 * u;
    z[u] = (jok && i < c) ? C[(int64_t)i * c + j] : 0.0;
  }
  const int kt = c - 3;   // first reflector applied; stage s holds k = kt - 16 s - r, r < 16
  const int nst = (kt + kBtStage) / kBtStage;
  auto load_stage = [&](int st, int buf) {
    for (int q = tid; q < kBtStage * CM; q += kSyevThreads) {
      const int r = q / CM, i = q - r * CM;
      const int k = kt - kBtStage * st - r;
      vs[buf][r][i] = (k >= 0 && i < c) ? work[(int64_t)k * la + i] : 0.0;
    }
    if (tid < kBtStage) {
      const int k = kt - kBtStage * st - tid;
      ts[buf][tid] = (k >= 0) ? work[sp.tau + k] : 0.0;
    }
  };
  if (kt >= 0) load_stage(0, 0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) load_stage(st + 1, buf ^ 1);   // the other buffer was released by the last barrier
#pragma unroll 4
    for (int r = 0; r < kBtStage; ++r) {
      const double t = ts[buf][r];
      if (t == 0.0) continue;   // uniform
      double v[RPL];
#pragma unroll
      for (int u = 0; u < RPL; ++u) v[u] = vs[buf][r][l32 + 32 * u];
      double sdot = 0.0;
#pragma unroll
      for (int u = 0; u < RPL; ++u) sdot = fma(v[u], z[u], sdot);
      sdot = t * row32_sum(sdot);
#pragma unroll
      for (int u = 0; u < RPL; ++u) z[u] = fma(-sdot, v[u], z[u]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int i = l32 + 32 * u;
    if (jok && i < c) C[(int64_t)i * c + j] = z[u];
  }
}

// MODE 0 does all four steps.  In the three-launch form syev_tridiag_kernel does step 1 and leaves
// T and Q^T in the global scratch (layout of syev_split_offsets), syev_bisect_kernel finds the
// eigenvalues with one workgroup each, and MODE 1 loads T, Q^T and the eigenvalues and does steps 3
// and 4.
template <int NB, int MODE>
__global__ void __launch_bounds__(kSyevThreads) syev_reg_kernel(const double* __restrict__ H, int64_t ldh,
                                                                int64_t hstride, int c, int nev,
                                                                double* __restrict__ evals, int64_t estride,
                                                                double* __restrict__ C, int64_t cstride,
                                                                double* __restrict__ work, int64_t wstride,
                                                                int* info, const int32_t* __restrict__ active) {
  static_assert(kSyevThreads == 256, "a 16 x 16 thread grid");
  constexpr int CM = 16 * NB;
  constexpr int LQ = CM + 1;
  if (active && !active[blockIdx.x]) return;
  H += (int64_t)blockIdx.x * hstride;
  evals += (int64_t)blockIdx.x * estride;
  C += (int64_t)blockIdx.x * cstride;
  work += (int64_t)blockIdx.x * wstride;
  // Z (c x nev, row stride nev + 1), then the inverse-iteration factors (4 c nev) and Q (c x c,
  // row stride c + 1) where they fit; what does not fit goes to the global scratch
  constexpr int POOL = (NB <= 3) ? 2 * CM * LQ + 4 * CM * CM : 2 * CM * LQ;
  __shared__ double pool[POOL];
  __shared__ double vb[2][CM], pb[2][CM], pvp[2][16], tb[2];
  __shared__ double d[CM], e[CM], s1[CM + 8], s2[CM], s3[CM + 8], lam[CM];
  __shared__ int cnt[kSyevThreads];
  __shared__ short cend[CM];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int ti = wid * 4 + (lane >> 4), tj = lane & 15;
  const SyevSplit sp = syev_split_offsets(c);
  double Q[NB][NB];
  if constexpr (MODE == 0) {
    double A[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = ti + 16 * a, j = tj + 16 * b;
        const int ic = min(i, c - 1), jc = min(j, c - 1);   // clamped: unconditional loads
        A[a][b] = keep_if(i < c && j < c, 0.5 * (H[(int64_t)ic * ldh + jc] + H[(int64_t)jc * ldh + ic]));
        Q[a][b] = (i == j) ? 1.0 : 0.0;
      }
    // ---- 1. tridiagonalization, accumulating Q ----
    tridiag_rows<NB, 0>(A, Q, c, ti, tj, &vb[0][0], &pb[0][0], &pvp[0][0], tb, d, e);
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = ti + 16 * a, j = tj + 16 * b;
        if (i == j && i + 2 >= c && i < c) d[i] = A[a][b];
        if (c >= 2 && i == c - 1 && j == c - 2) e[c - 2] = A[a][b];
      }
  } else {
    for (int i = tid; i < c; i += kSyevThreads) {
      d[i] = work[sp.d + i];
      e[i] = work[sp.e + i];
      lam[i] = (i < nev) ? work[sp.lam + i] : 0.0;
    }
  }
  const int lz = nev + 1;
  double* Z = pool;
  int64_t used = (int64_t)c * lz;
  double* sq;
  const bool lu_lds = (used + 4 * (int64_t)c * nev <= POOL);   // uniform
  double* const lu = pool + used;
  if (lu_lds) used += 4 * (int64_t)c * nev;
  const int lq = c + 1;
  if constexpr (MODE == 1) {
    sq = work + sp.q;   // Q^T, as step 1 left it
  } else {
    if (used + (int64_t)c * (c + 1) <= POOL) sq = pool + used;
    else sq = work + 4 * (int64_t)c * nev;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = ti + 16 * a, j = tj + 16 * b;
        if (i < c && j < c) sq[i * lq + j] = Q[a][b];
      }
    if (tid == 0) e[c - 1] = 0.0;
  }
  __syncthreads();
  // ---- 2, 3. eigenvalues and eigenvectors of T ----
  // two inlined copies, so that the factors are addressed as LDS or as global memory, not through
  // generic pointers
  const int maxrank = lu_lds ? tridiag_eigs<NB, NB, MODE == 1>(d, e, c, nev, s1, s2, s3, lam, cnt, cend, Z, lz, lu)
                             : tridiag_eigs<NB, NB, MODE == 1>(d, e, c, nev, s1, s2, s3, lam, cnt, cend, Z, lz, work);
  // ---- 4. C = Q Z (c x nev): 16 x 16 tiles, one wave per tile, 16x16x4 FP64 MFMAs ----
  typedef Mfma<double>::v4 v4;
  const int tn = (nev + 15) / 16, c4 = (c + 3) & ~3;
  for (int tile = wid; tile < NB * tn; tile += kSyevThreads / 64) {
    const int i0 = 16 * (tile / tn), j0 = 16 * (tile % tn);
    v4 acc = {0.0, 0.0, 0.0, 0.0};
    const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
    if constexpr (MODE == 1) {
      // Q^T from global memory: rows l of 16 consecutive entries, every load issued before the
      // products
      // products (clamped indices, masked afterwards: no read waits inside a branch)
      const int iac = min(ia, c - 1), jbc = min(jb, nev - 1);
      double qa[CM / 4], zv[CM / 4];
#pragma unroll
      for (int u = 0; u < CM / 4; ++u) {
        const int l = 4 * u + (lane >> 4), lc = min(l, c - 1);
        qa[u] = keep_if(l < c && ia < c, sq[lc * lq + iac]);
        zv[u] = keep_if(l < c && jb < nev, Z[lc * lz + jbc]);
      }
#pragma unroll
      for (int u = 0; u < CM / 4; ++u) acc = Mfma<double>::op(qa[u], zv[u], acc);
    } else {
      const int iac = min(ia, c - 1), jbc = min(jb, nev - 1);
      for (int l0 = 0; l0 < c4; l0 += 4) {
        const int l = l0 + (lane >> 4), lc = min(l, c - 1);
        const double qa = keep_if(l < c && ia < c, sq[iac * lq + lc]);
        const double zb = keep_if(l < c && jb < nev, Z[lc * lz + jbc]);
        acc = Mfma<double>::op(qa, zb, acc);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + Mfma<double>::drow(lane, q);
      if (i < c && jb < nev) C[(int64_t)i * c + jb] = acc[q];
    }
  }
  for (int j = tid; j < nev; j += kSyevThreads) evals[j] = lam[j];
  if (tid == 0 && info) info[blockIdx.x] = maxrank;
}

// Hetmaniuk-Lehoucq basis from the m leading eigenvectors C1 = C(:, 0:m) (c x m, row stride c):
// G = [C1, Pc] with Pc an orthonormal basis of (I - C1 C1^T) E1, E1 the first m unit vectors.
// Since C2 C2^T = I - C1 C1^T, this is the span of C(:, m:c) C(0:m, m:c)^T, so S Pc spans the same
// P as S C(:, m:c) V with V the orthonormal factor of C(0:m, m:c)^T, without the c - m other
// eigenvectors.  Pc is projected against C1 and orthonormalised by modified Gram-Schmidt, twice,
// so that Pc^T Pc - I and Pc^T C1 are at rounding level.  C1 is staged in LDS when it fits.
constexpr int kHlThreads = 256;
constexpr int kHlLds = 20224;   // doubles

__global__ void __launch_bounds__(kHlThreads) hl_build_kernel(const double* __restrict__ C, int64_t cstride, int c,
                                                              int m, double* __restrict__ G, int64_t gstride,
                                                              const int32_t* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  C += (int64_t)blockIdx.x * cstride;
  G += (int64_t)blockIdx.x * gstride;
  __shared__ double lds[kHlLds];
  const int tid = threadIdx.x, lane = tid % 64, wid = tid / 64;
  const int lw = m + 1;
  const int ldg = (c > m) ? 2 * m : m;
  double* w = lds;                  // c x m (row stride lw)
  double* tm = lds + c * lw;        // m x m
  const bool c1_lds = (2 * c * lw + m * lw <= kHlLds);
  double* c1 = c1_lds ? tm + m * lw : nullptr;
  const int ldc1 = c1_lds ? lw : c;
  const double* C1 = c1_lds ? c1 : C;
  for (int q = tid; q < c * m; q += kHlThreads) {
    const int i = q / m, j = q % m;
    const double x = C[(int64_t)i * c + j];
    G[(int64_t)i * ldg + j] = x;
    if (c1_lds) c1[i * lw + j] = x;
  }
  if (c <= m) return;
  __syncthreads();
  // W = E1 - C1 C1(0:m, :)^T
  for (int q = tid; q < c * m; q += kHlThreads) {
    const int i = q / m, j = q % m;
    double s0 = 0.0, s1 = 0.0;
    int l = 0;
    for (; l + 1 < m; l += 2) {
      s0 += C1[i * ldc1 + l] * C1[j * ldc1 + l];
      s1 += C1[i * ldc1 + l + 1] * C1[j * ldc1 + l + 1];
    }
    if (l < m) s0 += C1[i * ldc1 + l] * C1[j * ldc1 + l];
    w[i * lw + j] = ((i == j) ? 1.0 : 0.0) - (s0 + s1);
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    // W -= C1 (C1^T W)
    for (int q = tid; q < m * m; q += kHlThreads) {
      const int l = q / m, j = q % m;
      double s0 = 0.0, s1 = 0.0;
      int i = 0;
      for (; i + 1 < c; i += 2) {
        s0 += C1[i * ldc1 + l] * w[i * lw + j];
        s1 += C1[(i + 1) * ldc1 + l] * w[(i + 1) * lw + j];
      }
      if (i < c) s0 += C1[i * ldc1 + l] * w[i * lw + j];
      tm[l * lw + j] = s0 + s1;
    }
    __syncthreads();
    for (int q = tid; q < c * m; q += kHlThreads) {
      const int i = q / m, j = q % m;
      double s0 = 0.0, s1 = 0.0;
      int l = 0;
      for (; l + 1 < m; l += 2) {
        s0 += C1[i * ldc1 + l] * tm[l * lw + j];
        s1 += C1[i * ldc1 + l + 1] * tm[(l + 1) * lw + j];
      }
      if (l < m) s0 += C1[i * ldc1 + l] * tm[l * lw + j];
      w[i * lw + j] -= s0 + s1;
    }
    __syncthreads();
    // modified Gram-Schmidt on the columns of W
    for (int j = 0; j < m; ++j) {
      // a lane holds at most 3 rows (c <= 192): loads first, then stores
      if (wid == 0) {
        double z[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) z[u] = (lane + 64 * u < c) ? w[(lane + 64 * u) * lw + j] : 0.0;
        const double nn = wave_sum((z[0] * z[0] + z[1] * z[1]) + z[2] * z[2]);
        const double inv = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
#pragma unroll
        for (int u = 0; u < 3; ++u)
          if (lane + 64 * u < c) w[(lane + 64 * u) * lw + j] = z[u] * inv;
      }
      __syncthreads();
      double zj[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) zj[u] = (lane + 64 * u < c) ? w[(lane + 64 * u) * lw + j] : 0.0;
      for (int r = j + 1 + wid; r < m; r += 4) {
        double zr[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) zr[u] = (lane + 64 * u < c) ? w[(lane + 64 * u) * lw + r] : 0.0;
        const double dot = wave_sum((zj[0] * zr[0] + zj[1] * zr[1]) + zj[2] * zr[2]);
#pragma unroll
        for (int u = 0; u < 3; ++u)
          if (lane + 64 * u < c) w[(lane + 64 * u) * lw + r] = zr[u] - dot * zj[u];
      }
      __syncthreads();
    }
  }
  for (int q = tid; q < c * m; q += kHlThreads) {
    const int i = q / m, j = q % m;
    G[(int64_t)i * ldg + m + j] = w[i * lw + j];
  }
}

// One 16x16 output tile of D = A B on the matrix cores (FP64, 16x16x4 steps over k < K, K padded
// to a multiple of 4 with zeros); lda/ldb: element (r, k) of A at A[r * ars + k * aks], (k, n) of
// B at B[k * bks + n * bns], rows of A at or beyond ra and columns of B at or beyond nb read as
// zero.  Returns the lane's four entries (rows Mfma<double>::drow(lane, q), column lane % 16).
// Reads come from clamped indices and are masked afterwards (`keep_if`), four steps' reads issued together,
// so that no read waits inside a branch.
__device__ inline Mfma<double>::v4 tile_mm(const double* A, int ars, int aks, int ra, const double* B, int bks,
                                            int bns, int nb, int K) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, kk = lane >> 4;
  const bool aok = r < ra, bok = r < nb;
  const double* Ar = A + min(r, ra - 1) * ars;
  const double* Br = B + min(r, nb - 1) * bns;
  Mfma<double>::v4 acc = {0.0, 0.0, 0.0, 0.0};
  int k0 = 0;
  for (; k0 + 16 <= K; k0 += 16) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * u + kk;
      a[u] = keep_if(aok, Ar[k * aks]);
      b[u] = keep_if(bok, Br[k * bks]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = Mfma<double>::op(a[u], b[u], acc);
  }
  for (; k0 < K; k0 += 4) {
    const int k = k0 + kk, kc = min(k, K - 1);
    const double a = keep_if(aok && k < K, Ar[kc * aks]);
    const double b = keep_if(bok && k < K, Br[kc * bks]);
    acc = Mfma<double>::op(a, b, acc);
  }
  return acc;
}

// The Hetmaniuk-Lehoucq step above for m <= 16 NCOL and c <= 16 RC.  The three products (W =
// E1 - C1 C1(0:m, :)^T, T = C1^T W, W -= C1 T) run on the matrix cores from LDS; modified
// Gram-Schmidt keeps W in registers: thread (slot s, lane q of its 16-lane row) holds rows
// q + 16 u (u < RC) of columns s + 16 h (h < NCOL), so every column sum is a 16-lane DPP sum, and a
// column step needs one barrier (the owners of column j normalise it and publish it; every later
// column then subtracts its projection on it, with the next column's owners already done).
// C1G: C1 is read from the eigenvector matrix in global memory (L2-resident) instead of an LDS copy, so
// that W and T fit in LDS for c = 192, m = 64.
template <int NCOL, int RC, bool C1G = false>
__global__ void __launch_bounds__(kHlThreads) hl_reg_kernel(const double* __restrict__ C, int64_t cstride, int c,
                                                            int m, double* __restrict__ G, int64_t gstride,
                                                            const int32_t* __restrict__ active) {
  static_assert(kHlThreads == 256, "16 slots of 16 lanes");
  constexpr int MM = 16 * NCOL, CM = 16 * RC, LD = MM + 1;
  if (active && !active[blockIdx.x]) return;
  C += (int64_t)blockIdx.x * cstride;
  G += (int64_t)blockIdx.x * gstride;
  __shared__ double c1s[C1G ? 1 : CM * LD], w[CM * LD], tm[MM * LD], wb[2][CM];
  const double* c1 = C1G ? C : c1s;
  const int l1 = C1G ? c : LD;   // row stride of c1
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int ldg = (c > m) ? 2 * m : m;
  // C1 in: every thread's reads issued before its first store (clamped indices, stores guarded)
  constexpr int NE = (CM * MM + kHlThreads - 1) / kHlThreads;
  {
    double xv[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int q = min(tid + u * kHlThreads, c * m - 1);
      xv[u] = C[(int64_t)(q / m) * c + q % m];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int q = tid + u * kHlThreads;
      if (q < c * m) {
        const int i = q / m, j = q % m;
        G[(int64_t)i * ldg + j] = xv[u];
        if constexpr (!C1G) c1s[i * LD + j] = xv[u];
      }
    }
  }
  if (c <= m) return;
  __syncthreads();
  const int tr = (c + 15) / 16, tcm = (m + 15) / 16;
  // W = E1 - C1 C1(0:m, :)^T
  for (int tile = wid; tile < tr * tcm; tile += 4) {
    const int i0 = 16 * (tile / tcm), j0 = 16 * (tile % tcm);
    const Mfma<double>::v4 acc = tile_mm(c1 + i0 * l1, l1, 1, c - i0, c1 + j0 * l1, 1, l1, m - j0, m);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = i0 + Mfma<double>::drow(lane, q), j = j0 + (lane & 15);
      if (i < c && j < m) w[i * LD + j] = ((i == j) ? 1.0 : 0.0) - acc[q];
    }
  }
  __syncthreads();
  const int q16 = lane & 15, slot = tid >> 4;
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    // T = C1^T W, then W -= C1 T
    for (int tile = wid; tile < tcm * tcm; tile += 4) {
      const int l0 = 16 * (tile / tcm), j0 = 16 * (tile % tcm);
      const Mfma<double>::v4 acc = tile_mm(c1 + l0, 1, l1, m - l0, w + j0, LD, 1, m - j0, c);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int l = l0 + Mfma<double>::drow(lane, q), j = j0 + (lane & 15);
        if (l < m && j < m) tm[l * LD + j] = acc[q];
      }
    }
    __syncthreads();
    for (int tile = wid; tile < tr * tcm; tile += 4) {
      const int i0 = 16 * (tile / tcm), j0 = 16 * (tile % tcm);
      const Mfma<double>::v4 acc = tile_mm(c1 + i0 * l1, l1, 1, c - i0, tm + j0, LD, 1, m - j0, m);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + Mfma<double>::drow(lane, q), j = j0 + (lane & 15);
        if (i < c && j < m) w[i * LD + j] -= acc[q];
      }
    }
    __syncthreads();
    // modified Gram-Schmidt on the columns of W, in registers
    double W[NCOL][RC];
#pragma unroll
    for (int h = 0; h < NCOL; ++h)
#pragma unroll
      for (int u = 0; u < RC; ++u) {   // clamped reads, masked: all in flight together
        const int i = q16 + 16 * u, j = slot + 16 * h;
        W[h][u] = keep_if(i < c && j < m, w[min(i, c - 1) * LD + min(j, m - 1)]);
      }
#pragma unroll
    for (int hj = 0; hj < NCOL; ++hj) {
#pragma unroll 1
      for (int sj = 0; sj < 16; ++sj) {
        const int j = 16 * hj + sj;
        if (j >= m) break;   // uniform
        const int buf = j & 1;
        if (slot == sj) {
          double ss = 0.0;
#pragma unroll
          for (int u = 0; u < RC; ++u) ss = fma(W[hj][u], W[hj][u], ss);
          ss = row16_sum(ss);
          const double inv = (ss > 0.0) ? 1.0 / sqrt(ss) : 0.0;
#pragma unroll
          for (int u = 0; u < RC; ++u) {
            W[hj][u] *= inv;
            wb[buf][q16 + 16 * u] = W[hj][u];
          }
        }
        __syncthreads();
        double wj[RC];
#pragma unroll
        for (int u = 0; u < RC; ++u) wj[u] = wb[buf][q16 + 16 * u];
#pragma unroll
        for (int h = hj; h < NCOL; ++h) {
          const int col = slot + 16 * h;
          if (col > j && col < m) {   // uniform over the 16 lanes of a slot
            double dt = 0.0;
#pragma unroll
            for (int u = 0; u < RC; ++u) dt = fma(W[h][u], wj[u], dt);
            dt = row16_sum(dt);
#pragma unroll
            for (int u = 0; u < RC; ++u) W[h][u] = fma(-dt, wj[u], W[h][u]);
          }
        }
      }
    }
#pragma unroll
    for (int h = 0; h < NCOL; ++h)
#pragma unroll
      for (int u = 0; u < RC; ++u) {
        const int i = q16 + 16 * u, j = slot + 16 * h;
        if (i < c && j < m) w[i * LD + j] = W[h][u];
      }
    __syncthreads();
  }
  {
    double xv[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int q = min(tid + u * kHlThreads, c * m - 1);
      xv[u] = w[(q / m) * LD + q % m];
    }
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int q = tid + u * kHlThreads;
      if (q < c * m) G[(int64_t)(q / m) * ldg + m + q % m] = xv[u];
    }
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

// The same for 32 < c <= CP (registers for the row of G and the column of Rl leave no room for the
// staged form below): lane i holds row i of the symmetrised G, the diagonal and L[k][j] of another row
// k are readlanes, no barrier is needed.  Rout = L^T Rl with lane j forming column j.
template <typename T, int CP>
__global__ void __launch_bounds__(64) chol_upper_wave_rl_kernel(const double* __restrict__ G, const T* __restrict__ Rl,
                                                             int c, double* __restrict__ Lt, double* __restrict__ Rout,
                                                             int* flag, const int32_t* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  const int64_t off = (int64_t)blockIdx.x * c * c;
  G += off;
  Rl += off;
  Lt += off;
  if (Rout) Rout += off;
  flag += blockIdx.x;
  const int i = threadIdx.x;
  double a[CP];
  const int ic = min(i, c - 1);   // clamped addresses: the loads are unconditional and in flight together
#pragma unroll
  for (int k = 0; k < CP; ++k) {
    const int kc = min(k, c - 1);
    a[k] = keep_if(i < c && k < c, 0.5 * (G[ic * c + kc] + G[kc * c + ic]));
  }
  bool bad = false;
#pragma unroll
  for (int j = 0; j < CP; ++j) {
    if (j < c) {   // uniform
      double d = rdl64(a[j], j);
      if (!(d > 0.0) || !isfinite(d)) {
        bad = true;
        d = 1.0;
      }
      const double ljj = sqrt(d);
      a[j] = (i == j) ? ljj : a[j] / ljj;
#pragma unroll
      for (int k = j + 1; k < CP; ++k) a[k] -= a[j] * rdl64(a[j], k);
    }
  }
  if (bad && i == 0) flag[0] = 1;
  // column i of Lt = row i of L (zeros below the diagonal of Lt)
  if (i < c)
    for (int k = 0; k < c; ++k) Lt[k * c + i] = 0.0;
#pragma unroll
  for (int k = 0; k < CP; ++k)
    if (i < c && k <= i) Lt[k * c + i] = a[k];
  if (Rout) {
    double rl[CP];
#pragma unroll
    for (int k = 0; k < CP; ++k) {
      rl[k] = keep_if(i < c && k < c, (double)Rl[min(k, c - 1) * c + ic]);
    }
#pragma unroll
    for (int r = 0; r < CP; ++r) {
      double sum = 0.0;
#pragma unroll
      for (int k = r; k < CP; ++k) sum += rdl64(a[r], k) * rl[k];
      if (i < c && r < c) Rout[r * c + i] = sum;
    }
  }
}

// The same factorization by one wave for c <= CP <= 32: lane i holds row i of the symmetrised G and
// the pivot column goes through LDS each step (wave_cholesky), so no barrier is needed.  Rout = L^T Rl
// with lane j forming column j from the rows of L staged in LDS.
template <typename T, int CP>
__global__ void __launch_bounds__(64) chol_upper_wave_kernel(const double* __restrict__ G, const T* __restrict__ Rl,
                                                             int c, double* __restrict__ Lt, double* __restrict__ Rout,
                                                             int* flag, const int32_t* __restrict__ active) {
  if (active && !active[blockIdx.x]) return;
  const int64_t off = (int64_t)blockIdx.x * c * c;
  G += off;
  Rl += off;
  Lt += off;
  if (Rout) Rout += off;
  flag += blockIdx.x;
  __shared__ __align__(16) double cb[64];
  __shared__ __align__(16) double Ls[CP][CP + 2];
  const int i = threadIdx.x;
  double a[CP];
  const int ic = min(i, c - 1);   // clamped addresses: the loads are unconditional and in flight together
#pragma unroll
  for (int k = 0; k < CP; ++k) {
    const int kc = min(k, c - 1);
    a[k] = keep_if(i < c && k < c, 0.5 * (G[ic * c + kc] + G[kc * c + ic]));
  }
  // Rl's column i, requested before the factorization
  double rl[CP];
  if (Rout) {
#pragma unroll
    for (int k = 0; k < CP; ++k) rl[k] = keep_if(i < c && k < c, (double)Rl[min(k, c - 1) * c + ic]);
  }
  bool bad = false;
  wave_cholesky<CP>(a, c, cb, bad);
  if (bad && i == 0) flag[0] = 1;
  // column i of Lt = row i of L (zeros below the diagonal of Lt)
  if (i < c) {
#pragma unroll
    for (int k = 0; k < CP; ++k)
      if (k < c) Lt[k * c + i] = (k <= i) ? a[k] : 0.0;
  }
  if (Rout) {
    {
      // Rout[r][i] = sum_{k >= r} L[k][r] Rl[k][i]: row k of L from LDS (uniform reads, two columns each)
      if (i < CP) {
#pragma unroll
        for (int k = 0; k < CP; ++k) Ls[i][k] = (k <= i) ? a[k] : 0.0;
      }
      __builtin_amdgcn_wave_barrier();
      double sum[CP];
#pragma unroll
      for (int r = 0; r < CP; ++r) sum[r] = 0.0;
#pragma unroll
      for (int k = 0; k < CP; ++k) {
        if (k < c) {   // uniform
#pragma unroll
          for (int r = 0; r <= k; r += 2) {   // Ls[k][k + 1] is zero
            const f64x2_t l2 = *reinterpret_cast<const f64x2_t*>(&Ls[k][r]);
            sum[r] += l2.x * rl[k];
            if (r + 1 < CP) sum[r + 1] += l2.y * rl[k];
          }
        }
      }
      if (i < c) {
#pragma unroll
        for (int r = 0; r < CP; ++r)
          if (r < c) Rout[r * c + i] = sum[r];
      }
    }
  }
}

}  // namespace

int64_t syev_scratch(int c) { return 2 * (int64_t)c * (c + 1) + 4 * (int64_t)c * c + 4 * (int64_t)c + 16; }

namespace {
template <int NB>
void launch_syev_reg(const double* H, int64_t ldh, int64_t hstride, int c, int nev, double* evals, int64_t estride,
                     double* C, int64_t cstride, double* work, int64_t ws, int* info, const int32_t* active, int B,
                     hipStream_t st) {
  if (nev < kSyevSplitMinNev || (int64_t)B * nev > kSyevSplitMaxBlocks) {
    syev_reg_kernel<NB, 0><<<B, kSyevThreads, 0, st>>>(H, ldh, hstride, c, nev, evals, estride, C, cstride, work, ws,
                                                       info, active);
    return;
  }
  syev_tridiag_kernel<NB><<<B, 2 * kSyevThreads, 0, st>>>(H, ldh, hstride, c, work, ws, active);
  syev_bisect_kernel<<<dim3(nev, B), kSyevThreads, 0, st>>>(work, ws, c, nev, active);
  syev_reg_kernel<NB, 1><<<B, kSyevThreads, 0, st>>>(H, ldh, hstride, c, nev, evals, estride, C, cstride, work, ws,
                                                     info, active);
}
}  // namespace

void launch_syev(const double* H, int64_t ldh, int64_t hstride, int c, int nev, double* evals, int64_t estride,
                 double* C, int64_t cstride, double* work, int* info, const int32_t* active, int B, hipStream_t st) {
  const int64_t ws = syev_scratch(c);
  if (c <= 16)
    launch_syev_reg<1>(H, ldh, hstride, c, nev, evals, estride, C, cstride, work, ws, info, active, B, st);
  else if (c <= 32)
    launch_syev_reg<2>(H, ldh, hstride, c, nev, evals, estride, C, cstride, work, ws, info, active, B, st);
  else if (c <= 48)
    launch_syev_reg<3>(H, ldh, hstride, c, nev, evals, estride, C, cstride, work, ws, info, active, B, st);
  else if (c <= 96)
    launch_syev_reg<6>(H, ldh, hstride, c, nev, evals, estride, C, cstride, work, ws, info, active, B, st);
  else if (c <= 192 && nev >= kSyevSplitMinNev && nev <= kVecNev && (int64_t)B * nev <= kSyevSplitMaxBlocks) {
    // reflector form: tridiagonalization, bisection, inverse iteration, back-transformation
    syev_tridiag32_kernel<<<B, kSyevThreads32, 0, st>>>(H, ldh, hstride, c, work, ws, active);
    syev_bisect_kernel<<<dim3(nev, B), kSyevThreads, 0, st>>>(work, ws, c, nev, active);
    syev_vec_kernel<12, 4><<<B, kSyevThreads, 0, st>>>(C, cstride, c, nev, evals, estride, work, ws, info, active);
    syev_bt_kernel<6><<<dim3((nev + kBtCols - 1) / kBtCols, B), kSyevThreads, 0, st>>>(C, cstride, c, nev, work, ws,
                                                                                       active);
  } else
    syev_kernel<<<B, kSyevThreads, 0, st>>>(H, ldh, hstride, c, nev, evals, estride, C, cstride, work, ws, info, active);
}

void launch_hl_build(const double* C, int64_t cstride, int c, int m, double* G, int64_t gstride,
                     const int32_t* active, int B, hipStream_t st) {
  if (m <= 16 && c <= 48) hl_reg_kernel<1, 3><<<B, kHlThreads, 0, st>>>(C, cstride, c, m, G, gstride, active);
  else if (m <= 32 && c <= 96) hl_reg_kernel<2, 6><<<B, kHlThreads, 0, st>>>(C, cstride, c, m, G, gstride, active);
  else if (m <= 64 && c <= 192)
    hl_reg_kernel<4, 12, true><<<B, kHlThreads, 0, st>>>(C, cstride, c, m, G, gstride, active);
  else hl_build_kernel<<<B, kHlThreads, 0, st>>>(C, cstride, c, m, G, gstride, active);
}

template <typename T>
void launch_chol_upper(const double* G, const T* Rl, int c, double* Lt, double* Rout, int* flag,
                       const int32_t* active, int B, hipStream_t st) {
  if (c <= 32) chol_upper_wave_kernel<T, 32><<<B, 64, 0, st>>>(G, Rl, c, Lt, Rout, flag, active);
  else if (c <= 64) chol_upper_wave_rl_kernel<T, 64><<<B, 64, 0, st>>>(G, Rl, c, Lt, Rout, flag, active);
  else chol_upper_kernel<T><<<B, 256, 0, st>>>(G, Rl, c, Lt, Rout, flag, active);
}
template void launch_chol_upper<float>(const double*, const float*, int, double*, double*, int*, const int32_t*, int,
                                       hipStream_t);
template void launch_chol_upper<double>(const double*, const double*, int, double*, double*, int*, const int32_t*,
                                        int, hipStream_t);

}  // namespace lobpcg
