// Spline kernel columns U = (eps I + H_m)^{-k} F_1 (Sec. 2, the variational
// spline kernel as an inverse power of the shifted Laplacian, here of its
// block Lanczos matrix) for block widths s <= 64, by block cyclic reduction
// of the block tridiagonal SPD matrix A = eps I + H_m.
//
// A has diagonal blocks D_j = H_jj + eps I and the blocks A_{j+1,j} = H_{j+1,j}
// below them.  Level l (stride h = 2^l) eliminates the blocks o = h mod 2h of
// the current reduced system; with D_o = L L^T and Li = L^{-1}:
//   T_lo = Li A_{o,o-h},  T_hi = Li A_{o,o+h},  g_o = Li f_o,
//   D_{o-h} -= T_lo^T T_lo,  D_{o+h} -= T_hi^T T_hi,
//   A_{o+h,o-h} = -T_hi^T T_lo  (the coupling of the next level),
//   f_{o-h} -= T_lo^T g_o,  f_{o+h} -= T_hi^T g_o,
// and after the last level (one block left) x_0 = D_0^{-1} f_0; then level by
// level downwards x_o = Li^T (g_o - T_lo x_{o-h} - T_hi x_{o+h}).  This is
// Cholesky of A in the odd-even order, so it is as stable as the sequential
// block factorisation, but its dependency chain has ceil(log2 m) levels of
// independent s x s factorisations instead of m.  For k > 1 the factors
// (Li, T_lo, T_hi of every eliminated block and Li of block 0) are kept and
// only the right-hand side passes are repeated.
//
// One workgroup of 256 threads per block of a level; s x s operands are 64 x 64
// LDS tiles, products on the FP64 matrix cores (tile64.h).
#include "tile64.h"

namespace gk {

namespace {

// write the s x s part of a 64 x 64 accumulator tile: dst[r * s + c] = acc
__device__ __forceinline__ void store_acc(double* __restrict__ dst, int s, const double (&acc)[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = acc_row(a), c = acc_col(b);
      if (r < s && c < s) dst[r * s + c] = acc[a][b];
    }
}
// T = acc (zero outside s x s), for use as a product operand
__device__ __forceinline__ void put_acc(double (*T)[LP], int s, const double (&acc)[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = acc_row(a), c = acc_col(b);
      T[r][c] = (r < s && c < s) ? acc[a][b] : 0.0;
    }
}
__device__ __forceinline__ void stage64T(double (*D)[LP], const double* __restrict__ src, int s) {
  double v[16];
  fetch64(src, s, s, v);
  put64T(D, v);
}

// D_j = H_jj + eps I, E_j = A_{j+1,j} = H_{j+1,j}, F_j = (j == 0 ? I : 0)
__global__ void bcr_init_kernel(int m, int s, const double* __restrict__ Hd, const double* __restrict__ Bd,
                                double eps, double* __restrict__ D, double* __restrict__ E, double* __restrict__ F) {
  const int64_t ss = (int64_t)s * s;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * ss) return;
  const int64_t j = t / ss;
  const int r = (int)((t % ss) / s), c = (int)(t % s);
  D[t] = Hd[t] + (r == c ? eps : 0.0);
  E[t] = j + 1 < m ? Bd[t] : 0.0;
  F[t] = (j == 0 && r == c) ? 1.0 : 0.0;
}

// Level with stride h, block o = h + 2 h blockIdx.x: Li = chol(D_o)^{-1},
// T_lo = Li A_{o,o-h}, T_hi = Li A_{o,o+h} (= Li E_o^T).
__global__ void __launch_bounds__(ST)
bcr_odd_kernel(int m, int s, int h, const double* __restrict__ D, const double* __restrict__ E,
               double* __restrict__ Li, double* __restrict__ Tlo, double* __restrict__ Thi, int* __restrict__ bad) {
  __shared__ __align__(16) double A[WS][LP];
  __shared__ __align__(16) double Y[WS][LP];
  __shared__ __align__(16) double Z[WS][LP];
  const int o = h + 2 * h * blockIdx.x;
  const int64_t ss = (int64_t)s * s;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  stage64(A, D + o * ss, s, s);
  __syncthreads();
  blk_chol_inv(A, Y, Z, s, 0, nullptr, nullptr, 0.0, nullptr, bad, nullptr);
  double* LiG = Li + o * ss;
  for (int i = ty; i < s; i += 16)
    for (int c = tx; c < s; c += 16) LiG[i * s + c] = (c <= i) ? Y[i][c] : 0.0;
  // A <- Li^T (L is no longer needed), Z <- A_{o,o-h} = E_{o-h}, Y <- A_{o,o+h} = E_o^T
  for (int i = ty; i < WS; i += 16)
    for (int c = tx; c < WS; c += 16) A[c][i] = (i < s && c < s && c <= i) ? Y[i][c] : 0.0;
  __syncthreads();
  stage64(Z, E + (o - h) * ss, s, s);
  const bool hi = o + h < m;
  stage64T(Y, hi ? E + o * ss : nullptr, s);
  __syncthreads();
  double tlo[4][4], thi[4][4];
  lds_mm2(A, Z, A, Y, s, tlo, thi);
  store_acc(Tlo + o * ss, s, tlo);
  if (hi) store_acc(Thi + o * ss, s, thi);
}

// Level with stride h, block e = 2 h blockIdx.x, neighbours o1 = e - h and
// o2 = e + h (where they exist): g_o = Li_o f_o (stored for o2, whose lower
// neighbour e is), f_e -= T_lo(o2)^T g_o2 + T_hi(o1)^T g_o1 and, when
// factoring, D_e -= T_lo(o2)^T T_lo(o2) + T_hi(o1)^T T_hi(o1) and the coupling
// of the next level A_{e+2h,e} = -T_hi(o2)^T T_lo(o2).
__global__ void __launch_bounds__(ST)
bcr_even_kernel(int m, int s, int h, int factor, double* __restrict__ D, double* __restrict__ E,
                double* __restrict__ F, const double* __restrict__ Li, const double* __restrict__ Tlo,
                const double* __restrict__ Thi, double* __restrict__ G) {
  __shared__ __align__(16) double T0[WS][LP];
  __shared__ __align__(16) double T1[WS][LP];
  __shared__ __align__(16) double T2[WS][LP];
  __shared__ __align__(16) double T3[WS][LP];
  const int e = 2 * h * blockIdx.x;
  const int64_t ss = (int64_t)s * s;
  const bool lo = e >= h, hi = e + h < m;
  const int o1 = e - h, o2 = e + h;
  // g_o2 = Li_o2 f_o2 and g_o1 = Li_o1 f_o1 (products run as X^T B)
  stage64T(T0, hi ? Li + o2 * ss : nullptr, s);
  stage64(T1, hi ? F + o2 * ss : nullptr, s, s);
  stage64T(T2, lo ? Li + o1 * ss : nullptr, s);
  stage64(T3, lo ? F + o1 * ss : nullptr, s, s);
  __syncthreads();
  double g2[4][4], g1[4][4];
  lds_mm2(T0, T1, T2, T3, s, g2, g1);
  __syncthreads();
  put_acc(T1, s, g2);
  put_acc(T3, s, g1);
  if (hi) store_acc(G + o2 * ss, s, g2);
  stage64(T0, hi ? Tlo + o2 * ss : nullptr, s, s);
  stage64(T2, lo ? Thi + o1 * ss : nullptr, s, s);
  __syncthreads();
  double a1[4][4], a2[4][4];
  lds_mm2(T0, T1, T2, T3, s, a1, a2);
  double* Fe = F + e * ss;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = acc_row(a), c = acc_col(b);
      if (r < s && c < s) Fe[r * s + c] -= a1[a][b] + a2[a][b];
    }
  if (!factor) return;
  lds_mm2(T0, T0, T2, T2, s, a1, a2);
  double* De = D + e * ss;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = acc_row(a), c = acc_col(b);
      if (r < s && c < s) De[r * s + c] -= a1[a][b] + a2[a][b];
    }
  if (e + 2 * h < m) {
    __syncthreads();   // T1 (g_o2) has been read
    stage64(T1, Thi + o2 * ss, s, s);
    __syncthreads();
    lds_mm<true, false>(T1, T0, s, a1);
    double* Ee = E + e * ss;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int r = acc_row(a), c = acc_col(b);
        if (r < s && c < s) Ee[r * s + c] = -a1[a][b];
      }
  }
}

// Last level (block 0 alone): x_0 = D_0^{-1} f_0 = Li^T (Li f_0); when
// factoring, Li = chol(D_0)^{-1} is formed and kept.  x_0 goes to X and, for
// a further power, to F.
__global__ void __launch_bounds__(ST)
bcr_top_kernel(int s, int factor, const double* __restrict__ D, const double* __restrict__ F0,
               double* __restrict__ Li, double* __restrict__ X, double* __restrict__ Fn, int* __restrict__ bad) {
  __shared__ __align__(16) double A[WS][LP];
  __shared__ __align__(16) double Y[WS][LP];
  __shared__ __align__(16) double Z[WS][LP];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (factor) {
    stage64(A, D, s, s);
    __syncthreads();
    blk_chol_inv(A, Y, Z, s, 0, nullptr, nullptr, 0.0, nullptr, bad, nullptr);
    for (int i = ty; i < s; i += 16)
      for (int c = tx; c < s; c += 16) Li[i * s + c] = (c <= i) ? Y[i][c] : 0.0;
    for (int i = ty; i < WS; i += 16)
      for (int c = tx; c < WS; c += 16) {
        const double v = (i < s && c < s && c <= i) ? Y[i][c] : 0.0;
        Y[i][c] = v;
        A[c][i] = v;
      }
  } else {
    double v[16];
    fetch64(Li, s, s, v);
    put64(Y, v);
    put64T(A, v);
  }
  stage64(Z, F0, s, s);
  __syncthreads();
  double acc[4][4];
  lds_mm<true, false>(A, Z, s, acc);   // Li f_0
  __syncthreads();
  put_acc(Z, s, acc);
  __syncthreads();
  lds_mm<true, false>(Y, Z, s, acc);   // Li^T (Li f_0)
  store_acc(X, s, acc);
  if (Fn) store_acc(Fn, s, acc);
}

// Level with stride h, block o = h + 2 h blockIdx.x:
// x_o = Li^T (g_o - T_lo x_{o-h} - T_hi x_{o+h}).
__global__ void __launch_bounds__(ST)
bcr_back_kernel(int m, int s, int h, const double* __restrict__ Li, const double* __restrict__ Tlo,
                const double* __restrict__ Thi, const double* __restrict__ G, double* __restrict__ X,
                double* __restrict__ Fn) {
  __shared__ __align__(16) double T0[WS][LP];
  __shared__ __align__(16) double T1[WS][LP];
  __shared__ __align__(16) double T2[WS][LP];
  __shared__ __align__(16) double T3[WS][LP];
  const int o = h + 2 * h * blockIdx.x;
  const int64_t ss = (int64_t)s * s;
  const bool hi = o + h < m;
  stage64T(T0, Tlo + o * ss, s);
  stage64(T1, X + (o - h) * ss, s, s);
  stage64T(T2, hi ? Thi + o * ss : nullptr, s);
  stage64(T3, hi ? X + (o + h) * ss : nullptr, s, s);
  double gv[16];
  fetch64(G + o * ss, s, s, gv);
  __syncthreads();
  double a1[4][4], a2[4][4];
  lds_mm2(T0, T1, T2, T3, s, a1, a2);
  __syncthreads();
  put64(T3, gv);   // fetch64 layout: element (ty + 16 a, tx + 16 b)
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = acc_row(a), c = acc_col(b);
      a1[a][b] = T3[r][c] - a1[a][b] - a2[a][b];
    }
  __syncthreads();
  put_acc(T1, s, a1);
  stage64(T0, Li + o * ss, s, s);
  __syncthreads();
  lds_mm<true, false>(T0, T1, s, a2);   // Li^T t
  store_acc(X + o * ss, s, a2);
  if (Fn) store_acc(Fn + o * ss, s, a2);
}

}  // namespace

size_t bcr_work_elems(int m, int s) { return (size_t)7 * m * s * s; }

void launch_banded_spline_reg(int m, int s, const double* Hd, const double* Bd, double eps, int k, double* work,
                              double* U, int* bad, hipStream_t st) {
  GK_REQUIRE(m >= 1 && s >= 1 && s <= WS && k >= 1, GK_EINVAL, "block cyclic reduction needs 1 <= s <= 64");
  const size_t ss = (size_t)s * s;
  double* D = work;
  double* E = D + m * ss;
  double* F = E + m * ss;
  double* Li = F + m * ss;
  double* Tlo = Li + m * ss;
  double* Thi = Tlo + m * ss;
  double* G = Thi + m * ss;
  hipLaunchKernelGGL(bcr_init_kernel, dim3((unsigned)((m * ss + 255) / 256)), dim3(256), 0, st, m, s, Hd, Bd, eps,
                     D, E, F);
  GK_HIP(hipGetLastError());
  int top = 1;
  while (top < m) top *= 2;   // first stride with block 0 alone
  for (int pass = 0; pass < k; ++pass) {
    const int factor = pass == 0 ? 1 : 0;
    const int cls = factor ? KC_BANDED_FACTOR : KC_BANDED_SOLVE;
    double* Fn = pass + 1 < k ? F : nullptr;
    for (int h = 1; h < m; h *= 2) {
      const int nodd = (m - h + 2 * h - 1) / (2 * h), neven = (m + 2 * h - 1) / (2 * h);
      if (factor) {
        kt_begin(cls, st);
        hipLaunchKernelGGL(bcr_odd_kernel, dim3(nodd), dim3(ST), 0, st, m, s, h, D, E, Li, Tlo, Thi, bad);
        GK_HIP(hipGetLastError());
        kt_end(st, 8.0 * 5 * nodd * ss, nodd * (double)ss * s * (1.0 / 3.0 + 1.0 + 4.0));
      }
      kt_begin(cls, st);
      hipLaunchKernelGGL(bcr_even_kernel, dim3(neven), dim3(ST), 0, st, m, s, h, factor, D, E, F, Li, Tlo, Thi, G);
      GK_HIP(hipGetLastError());
      kt_end(st, 8.0 * (factor ? 10 : 7) * neven * ss, neven * (double)ss * s * (factor ? 14.0 : 8.0));
    }
    kt_begin(cls, st);
    hipLaunchKernelGGL(bcr_top_kernel, dim3(1), dim3(ST), 0, st, s, factor, D, F, Li, U, Fn, bad);
    GK_HIP(hipGetLastError());
    kt_end(st, 8.0 * 4 * ss, (double)ss * s * (factor ? 4.0 + 1.0 / 3.0 : 4.0));
    for (int h = top / 2; h >= 1; h /= 2) {
      const int nodd = (m - h + 2 * h - 1) / (2 * h);
      kt_begin(KC_BANDED_SOLVE, st);
      hipLaunchKernelGGL(bcr_back_kernel, dim3(nodd), dim3(ST), 0, st, m, s, h, Li, Tlo, Thi, G, U, Fn);
      GK_HIP(hipGetLastError());
      kt_end(st, 8.0 * 7 * nodd * ss, nodd * (double)ss * s * 6.0);
    }
  }
}

}  // namespace gk
