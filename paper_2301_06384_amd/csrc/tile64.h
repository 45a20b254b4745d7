// Device toolkit for small float64 matrices held as 64 x 64 tiles in LDS:
// register-blocked products, tile staging, FP64 MFMA 16 x 16 tiles and the
// blocked Cholesky factor with inverse used by the CholQR, orthogonality
// estimate and banded spline kernels.
#pragma once
#include "gk_internal.h"

namespace gk {

constexpr int WS = 64;
constexpr int LP = WS + 2;   // even pitch: rows start 16-byte aligned
constexpr int ST = 256;

typedef double dv4 __attribute__((ext_vector_type(4)));

// Output layout of lds_mm (the FP64 matrix-core tile layout): this thread's
// acc[a][b] is element (acc_row(a), acc_col(b)) of the 64 x 64 product.
__device__ __forceinline__ int acc_row(int a) {
  return 16 * (int)(threadIdx.x >> 6) + 4 * a + (int)((threadIdx.x & 63) >> 4);
}
__device__ __forceinline__ int acc_col(int b) { return 16 * b + (int)(threadIdx.x & 15); }

// NT steps of four contraction indices (rows 4t + k, masked at s) of the
// product below.
template <int NT>
__device__ __forceinline__ void mm_steps(const double (*A)[LP], const double (*B)[LP], int s, dv4 (&d)[4]) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
  double av[2], bv[2][4];
  // operands of step t are loaded while the MFMAs of step t - 1 run
  av[0] = A[lk][16 * w + li];
#pragma unroll
  for (int b = 0; b < 4; ++b) bv[0][b] = B[lk][16 * b + li];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int cur = t & 1, nxt = cur ^ 1;
    if (t + 1 < NT) {
      const int kn = 4 * (t + 1) + lk;
      av[nxt] = A[kn][16 * w + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[nxt][b] = B[kn][16 * b + li];
    }
    const bool in = 4 * t + lk < s;
    const double a = in ? av[cur] : 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      d[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, in ? bv[cur][b] : 0.0, d[b], 0, 0, 0);
  }
}

// Two independent products in one loop (eight accumulator chains per
// wavefront instead of four): acc1 = A1^T B1, acc2 = A2^T B2, layout as lds_mm.
template <int NT>
__device__ __forceinline__ void mm_steps2(const double (*A1)[LP], const double (*B1)[LP], const double (*A2)[LP],
                                          const double (*B2)[LP], int s, dv4 (&d1)[4], dv4 (&d2)[4]) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int kk = 4 * t + lk;
    const bool in = kk < s;
    const double a1 = A1[kk][16 * w + li], a2 = A2[kk][16 * w + li];
    double b1[4], b2[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      b1[b] = B1[kk][16 * b + li];
      b2[b] = B2[kk][16 * b + li];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      d1[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? a1 : 0.0, in ? b1[b] : 0.0, d1[b], 0, 0, 0);
      d2[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? a2 : 0.0, in ? b2[b] : 0.0, d2[b], 0, 0, 0);
    }
  }
}
__device__ __forceinline__ void lds_mm2(const double (*A1)[LP], const double (*B1)[LP], const double (*A2)[LP],
                                        const double (*B2)[LP], int s, double (&acc1)[4][4], double (&acc2)[4][4]) {
  dv4 d1[4], d2[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) d1[b] = d2[b] = dv4{0.0, 0.0, 0.0, 0.0};
  if (s > 48) mm_steps2<16>(A1, B1, A2, B2, s, d1, d2);
  else if (s > 32) mm_steps2<12>(A1, B1, A2, B2, s, d1, d2);
  else if (s > 16) mm_steps2<8>(A1, B1, A2, B2, s, d1, d2);
  else mm_steps2<4>(A1, B1, A2, B2, s, d1, d2);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc1[a][b] = d1[b][a];
      acc2[a][b] = d2[b][a];
    }
}

// lds_mm2 restricted to the output tiles on and above the block diagonal
// (wave w forms tiles (w, b), b >= w) and to the contraction tiles whose
// terms can be non-zero; the tiles below the diagonal are left zero.  Per
// product, KR_LEAD sums contraction tiles 0..w (A^T B with A and B upper
// triangular: U^T U) and KR_BAND tiles w..b (A^T and B upper triangular: the
// product is upper triangular).  The skipped terms are exact zeros, so the
// formed tiles equal those of lds_mm2 bit for bit.
enum { KR_LEAD = 0, KR_BAND = 1 };
template <int W, int K1, int K2>
__device__ __forceinline__ void mm_steps2_upper(const double (*A1)[LP], const double (*B1)[LP],
                                                const double (*A2)[LP], const double (*B2)[LP], int s, dv4 (&d1)[4],
                                                dv4 (&d2)[4]) {
  const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int kt = t >> 2;
    const int kk = 4 * t + lk;
    const bool in = kk < s;
    const double a1 = A1[kk][16 * W + li], a2 = A2[kk][16 * W + li];
#pragma unroll
    for (int b = W; b < 4; ++b) {
      const bool u1 = K1 == KR_LEAD ? kt <= W : (kt >= W && kt <= b);
      const bool u2 = K2 == KR_LEAD ? kt <= W : (kt >= W && kt <= b);
      if (u1) d1[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? a1 : 0.0, in ? B1[kk][16 * b + li] : 0.0, d1[b], 0, 0, 0);
      if (u2) d2[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? a2 : 0.0, in ? B2[kk][16 * b + li] : 0.0, d2[b], 0, 0, 0);
    }
  }
}
template <int K1, int K2>
__device__ __forceinline__ void lds_mm2_upper(const double (*A1)[LP], const double (*B1)[LP], const double (*A2)[LP],
                                              const double (*B2)[LP], int s, double (&acc1)[4][4],
                                              double (&acc2)[4][4]) {
  if (s <= 48) {   // few contraction steps: the full products
    lds_mm2(A1, B1, A2, B2, s, acc1, acc2);
    return;
  }
  dv4 d1[4], d2[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) d1[b] = d2[b] = dv4{0.0, 0.0, 0.0, 0.0};
  switch (__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))) {
    case 0: mm_steps2_upper<0, K1, K2>(A1, B1, A2, B2, s, d1, d2); break;
    case 1: mm_steps2_upper<1, K1, K2>(A1, B1, A2, B2, s, d1, d2); break;
    case 2: mm_steps2_upper<2, K1, K2>(A1, B1, A2, B2, s, d1, d2); break;
    default: mm_steps2_upper<3, K1, K2>(A1, B1, A2, B2, s, d1, d2); break;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc1[a][b] = d1[b][a];
      acc2[a][b] = d2[b][a];
    }
}

// acc = A^T B summed over the first s rows of two 64 x 64 LDS operands
// (256 threads).  Wave w computes output rows 16w .. 16w+15 as four 16 x 16
// tiles of v_mfma_f64_16x16x4f64: lane l = i + 16k holds A[4t+k][16w+i] and
// B[4t+k][16b+i]; accumulator register a holds row 4a + k, column i.  Rows at
// and beyond s are masked, so no zero padding of the operands is assumed.
template <bool TA, bool TB>
__device__ __forceinline__ void lds_mm(const double (*A)[LP], const double (*B)[LP], int s, double (&acc)[4][4]) {
  static_assert(TA && !TB, "products run as A^T B");
  dv4 d[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) d[b] = dv4{0.0, 0.0, 0.0, 0.0};
  if (s > 48) mm_steps<16>(A, B, s, d);
  else if (s > 32) mm_steps<12>(A, B, s, d);
  else if (s > 16) mm_steps<8>(A, B, s, d);
  else mm_steps<4>(A, B, s, d);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d[b][a];
}

// D[i][c] = src[i * lds + c] for i, c < s and 0 elsewhere in the 64 x 64
// tile (256 threads).  All loads are issued before the LDS stores.
__device__ __forceinline__ void fetch64(const double* __restrict__ src, int s, int lds, double (&v)[16]) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ty + 16 * a, c = tx + 16 * b;
      v[4 * a + b] = (src && i < s && c < s) ? src[i * lds + c] : 0.0;
    }
}
__device__ __forceinline__ void put64(double (*D)[LP], const double (&v)[16]) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) D[ty + 16 * a][tx + 16 * b] = v[4 * a + b];
}
// D[c][i] = v (the transpose of what put64 stores)
__device__ __forceinline__ void put64T(double (*D)[LP], const double (&v)[16]) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) D[tx + 16 * b][ty + 16 * a] = v[4 * a + b];
}
__device__ __forceinline__ void stage64(double (*D)[LP], const double* __restrict__ src, int s, int lds) {
  double v[16];
  fetch64(src, s, lds, v);
  put64(D, v);
}

// Lower Cholesky of the symmetric A (s x s, lower part used) together with
// Y = L^{-1}, blocked by 16 (256 threads):
//   for each diagonal block b:  A_bb = L_bb L_bb^T and Y_bb = L_bb^{-1}
//   (one wavefront, registers and lane shuffles);  then
//   L_ib = A_ib Y_bb^T,  Y_b = Y_bb Z_b,  A_ij -= L_ib L_jb^T,  Z_i -= L_ib Y_b
//   for the block rows i, j > b, where Z (= I initially) carries the
//   right-hand sides of L Y = I.
// Inside a diagonal block the pivots follow the rules of `mode`:
//   0: plain (non-positive pivot -> *bad = 3, pivot 1 used);
//   1 / 2: the CholQR deflation rules (see cholqr_factor_kernel).
// Deflated columns give zero columns of L and zero rows of Y.  A column whose
// pivot rule 1 clamps (numerically dependent on the earlier ones) is kept with
// its clamped diagonal but decoupled: its entries of L below the diagonal are
// zero, so no later column is eliminated against it; without that, chains of
// clamped pivots compound 1 / l factors in L^{-1} until it overflows.  The
// flags go to clf[column] when clf is not null.  Indices s..63 are padded with
// an identity block.  Z is clobbered.
// 1/sqrt(p) for p > 0: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double p) {
  double y = __builtin_amdgcn_rsq(p);
  y = y * fma(-0.5 * p * y, y, 1.5);
  y = y * fma(-0.5 * p * y, y, 1.5);
  return y;
}

// Pivot rule of column j (global index gj): returns l_jj and 1 / l_jj (0 for
// a deflated column).  gjj = original Gram diagonal (mode 1), dpj = first-pass
// diagonal (mode 2).
// cl (rule 1): the pivot was clamped; the column is then decoupled (its
// entries of L below the diagonal are zero), see blk_chol_inv_t.
template <int MODE>
__device__ __forceinline__ void chol_pivot(double piv, int gj, int s, double gjj, double dpj, double thr, int* bad,
                                           double& l, double& inv, bool& cl) {
  cl = false;
  // branch-free: the reciprocal square root is taken of a safe argument and
  // the rule selects the result
  if (MODE == 0) {
    const bool ok = piv > 0.0;
    const double y = rsqrt_nr(ok ? piv : 1.0);
    l = ok ? piv * y : 1.0;
    inv = ok ? y : 1.0;
    if (!ok && gj < s && bad) *bad = 3;
  } else if (MODE == 1) {
    const double eta = 1e-7;
    const bool keep = gjj > thr * thr;
    cl = keep && gj < s && !(piv >= eta * eta * gjj);
    const double pp = keep ? fmax(piv, eta * eta * gjj) : 1.0;
    const double y = rsqrt_nr(pp);
    l = keep ? pp * y : 0.0;
    inv = keep ? y : 0.0;
  } else {
    const bool pos = piv > 0.0;
    const double y = rsqrt_nr(pos ? piv : 1.0);
    const double ll = piv * y;
    const bool keep = pos && !(ll * dpj < thr);
    l = keep ? ll : 0.0;
    inv = keep ? y : 0.0;
  }
  if (gj >= s) { l = 1.0; inv = 1.0; }   // identity padding
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffu), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// One pivot step J of the 16 x 16 diagonal-block factorisation by wavefront
// 0.  Lane c < 16 holds column c of the block (both triangles) and lane
// 16 + c column c of its inverse, in the same registers v, so one stream of
// FMAs updates both: with f = v[J] / l_JJ (L[c][J] on a factor lane, row J of
// the inverse on an inverse lane), v[r] -= L[r][J] f for r > J.  Factor lanes
// store their entry of column J of L straight into the LDS tile (zeros above
// the diagonal) and every lane reads the column back (a wavefront executes
// its LDS accesses in order, so no barrier is involved).  Factor lanes c <= J
// update entries that are never read again, so they need no mask.
// piv: the pivot A[J][J] after the steps before J.  The next pivot needs only
// lane J+1's own entries (v[J+1] - f^2), so it is read out before the column
// exchange; the exchange gives that lane the same value.
template <int MODE, int J>
struct DiagStep {
  __device__ __forceinline__ static void run(double (&v)[16], int c, bool ylane, int o, int s, double gl, double dl,
                                             double thr, int* bad, double* dg, int* clf, double (*A)[LP],
                                             double piv) {
    const double gjj = MODE == 1 ? readlane_d(gl, J) : 0.0;
    const double dpj = MODE == 2 ? readlane_d(dl, J) : 0.0;
    double ljj, inv;
    bool cl;
    chol_pivot<MODE>(piv, o + J, s, gjj, dpj, thr, bad, ljj, inv, cl);
    if (threadIdx.x == 0) {
      if (dg) dg[o + J] = (o + J < s) ? ljj : 0.0;
      if (clf) clf[o + J] = cl ? 1 : 0;
    }
    // a clamped pivot decouples its column: L[c][J] = 0 below the diagonal
    const double f = (cl && !ylane) ? 0.0 : v[J] * inv;
    if (ylane) v[J] = f;
    double pnext = 0.0;
    if (J + 1 < 16) pnext = readlane_d(fma(-f, f, v[J + 1 < 16 ? J + 1 : J]), J + 1);
    if (threadIdx.x < 16) A[o + c][o + J] = c > J ? f : (c == J ? ljj : 0.0);
#pragma unroll
    for (int r = J + 1; r < 16; ++r) v[r] = fma(-A[o + r][o + J], f, v[r]);
    DiagStep<MODE, J + 1>::run(v, c, ylane, o, s, gl, dl, thr, bad, dg, clf, A, pnext);
  }
};
template <int MODE>
struct DiagStep<MODE, 16> {
  __device__ __forceinline__ static void run(double (&)[16], int, bool, int, int, double, double, double, int*,
                                             double*, int*, double (*)[LP], double) {}
};

// 16 x 16 tile product on FP64 matrix cores (v_mfma_f64_16x16x4f64, lane
// l = i + 16 k holds A[i][k] and B[k][i]; register r holds D[4 r + k][i]):
// acc += op(A) op(B) with op(A)[i][k] = TA ? A[ra + k][ca + i] : A[ra + i][ca + k]
// and op(B)[k][j] = TB ? B[rb + j][cb + k] : B[rb + k][cb + j].
template <bool TA, bool TB>
__device__ __forceinline__ dv4 mma_tile(const double (*A)[LP], int ra, int ca, const double (*B)[LP], int rb, int cb,
                                        dv4 acc) {
  const int l = threadIdx.x & 63, i = l & 15, k = l >> 4;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int kk = 4 * ks + k;
    const double av = TA ? A[ra + kk][ca + i] : A[ra + i][ca + kk];
    const double bv = TB ? B[rb + i][cb + kk] : B[rb + kk][cb + i];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  return acc;
}
__device__ __forceinline__ dv4 tile_load(const double (*A)[LP], int r0, int c0) {
  const int l = threadIdx.x & 63, i = l & 15, k = l >> 4;
  return dv4{A[r0 + k][c0 + i], A[r0 + 4 + k][c0 + i], A[r0 + 8 + k][c0 + i], A[r0 + 12 + k][c0 + i]};
}
__device__ __forceinline__ void tile_store(double (*A)[LP], int r0, int c0, dv4 v) {
  const int l = threadIdx.x & 63, i = l & 15, k = l >> 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) A[r0 + 4 * r + k][c0 + i] = v[r];
}

template <int MODE>
__device__ __forceinline__ void blk_chol_inv_t(double (*A)[LP], double (*Y)[LP], double (*Z)[LP], int s, const double* g0,
                               const double* dprev, double thr, double* dg, int* bad, int* clf) {
  const int tid = threadIdx.x;
  const int wv = tid >> 6;
  const int nbk = (s + 15) >> 4;
  const int S16 = nbk << 4;
  // pad A with an identity block, Z = I, Y = 0
  for (int r = tid >> 4; r < S16; r += 16)
    for (int c = tid & 15; c < S16; c += 16) {
      if (r >= s || c >= s) A[r][c] = (r == c) ? 1.0 : 0.0;
      Z[r][c] = (r == c) ? 1.0 : 0.0;
      Y[r][c] = 0.0;
    }
  __syncthreads();
  for (int b = 0; b < nbk; ++b) {
    const int o = 16 * b;
    const int T = nbk - 1 - b;                 // tile rows below the diagonal block
    // ---- diagonal block: wavefront 0; lane c < 16 holds column c of the
    //      block, lane 16 + c column c of its inverse (starting from I)
    if (tid < 64) {
      const int c = tid & 15;
      const bool ylane = (tid & 16) != 0;
      double v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = ylane ? ((r == c) ? 1.0 : 0.0) : A[o + r][o + c];
      // the pivot rule's per-column data, lane c holding column o + c
      const double gl = (MODE == 1 && o + c < s) ? g0[o + c] : 0.0;
      const double dl = (MODE == 2 && o + c < s) ? dprev[o + c] : 0.0;
      DiagStep<MODE, 0>::run(v, c, ylane, o, s, gl, dl, thr, bad, dg, clf, A, readlane_d(v[0], 0));   // L_bb into A
      if (tid >= 16 && tid < 32) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          Z[o + r][o + c] = (r >= c) ? v[r] : 0.0;   // Y_bb, kept in the diagonal block of Z
          Y[o + r][o + c] = (r >= c) ? v[r] : 0.0;
        }
      }
    }
    __syncthreads();
    // ---- panel: L_ib = A_ib Y_bb^T (i > b, written after a barrier: in place)
    //      and Y_b[:, c] = Y_bb Z_b[:, c] (c < b)
    {
      dv4 res = dv4{0.0, 0.0, 0.0, 0.0};
      const int task = wv;                     // at most 3 panel tiles + 3 inverse tiles
      const int ntask = T + b;
      dv4 res2 = dv4{0.0, 0.0, 0.0, 0.0};
      if (task < ntask) {
        if (task < T) res = mma_tile<false, true>(A, o + 16 * (1 + task), o, Z, o, o, res);
        else tile_store(Y, o, 16 * (task - T), mma_tile<false, false>(Z, o, o, Z, o, 16 * (task - T), res));
      }
      if (task + 4 < ntask) {
        const int t2 = task + 4;
        if (t2 < T) res2 = mma_tile<false, true>(A, o + 16 * (1 + t2), o, Z, o, o, res2);
        else tile_store(Y, o, 16 * (t2 - T), mma_tile<false, false>(Z, o, o, Z, o, 16 * (t2 - T), res2));
      }
      __syncthreads();
      // columns with a clamped pivot stay decoupled (lane i holds column o + i)
      if (clf && clf[o + (threadIdx.x & 15)]) res = res2 = dv4{0.0, 0.0, 0.0, 0.0};
      if (task < T) tile_store(A, o + 16 * (1 + task), o, res);
      if (task + 4 < T) tile_store(A, o + 16 * (1 + task + 4), o, res2);
    }
    __syncthreads();
    // ---- trailing: A_ij -= L_ib L_jb^T (b < j <= i), Z_i[:, c] -= L_ib Y_b[:, c] (c <= b)
    {
      const int na = T * (T + 1) / 2;
      const int nz = T * (b + 1);
      for (int task = wv; task < na + nz; task += 4) {
        if (task < na) {
          int ii = 0, rem = task;
          while (rem > ii) { rem -= ii + 1; ++ii; }
          const int ti = b + 1 + ii, tj = b + 1 + rem;     // tile (ti, tj), tj <= ti
          const dv4 p = mma_tile<false, true>(A, 16 * ti, o, A, 16 * tj, o, dv4{0.0, 0.0, 0.0, 0.0});
          tile_store(A, 16 * ti, 16 * tj, tile_load(A, 16 * ti, 16 * tj) - p);
        } else {
          const int q = task - na;
          const int ti = b + 1 + q / (b + 1), tc = q % (b + 1);
          const dv4 p = mma_tile<false, false>(A, 16 * ti, o, Y, o, 16 * tc, dv4{0.0, 0.0, 0.0, 0.0});
          tile_store(Z, 16 * ti, 16 * tc, tile_load(Z, 16 * ti, 16 * tc) - p);
        }
      }
    }
    __syncthreads();
  }
  // strict upper part of L is zero
  for (int r = tid >> 4; r < S16; r += 16)
    for (int c = tid & 15; c < S16; c += 16)
      if (c > r) A[r][c] = 0.0;
  __syncthreads();
}

__device__ __forceinline__ void blk_chol_inv(double (*A)[LP], double (*Y)[LP], double (*Z)[LP], int s, int mode, const double* g0,
                             const double* dprev, double thr, double* dg, int* bad, int* clf) {
  if (mode == 0) blk_chol_inv_t<0>(A, Y, Z, s, g0, dprev, thr, dg, bad, clf);
  else if (mode == 1) blk_chol_inv_t<1>(A, Y, Z, s, g0, dprev, thr, dg, bad, clf);
  else blk_chol_inv_t<2>(A, Y, Z, s, g0, dprev, thr, dg, bad, clf);
}

}  // namespace gk
