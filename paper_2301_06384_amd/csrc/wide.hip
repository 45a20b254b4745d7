// Small float64 kernels for block widths 65..512: the CholQR factors of the
// Lanczos blocks (Alg. 1, QR of X), the block orthogonality estimate of
// partial reorthogonalisation and the banded spline evaluation
// (eps I + H_m)^(-k) F_1, for matrices of up to 8 x 8 tiles of 64 x 64.
//
// One workgroup of 256 threads walks the tiles of a blocked algorithm: every
// tile product stages its two operand tiles from device memory (L2-resident
// at these sizes) into LDS and runs the 64-wide register-blocked product of
// tile64.h; the 64 x 64 diagonal Cholesky steps run the FP64-MFMA blocked
// factorisation of tile64.h on one tile.  Matrices are row-major with zero
// padding beyond s, so a partial last tile needs no special case.
//
// Global stores made by a workgroup are read back by other threads of the
// same workgroup after a barrier; the vector L1 is shared by the waves of a
// workgroup and written through, so the barrier orders them.
#include "gk_internal.h"
#include "tile64.h"

namespace gk {

constexpr int WQ_MAX = 8;            // tiles per side (s <= 512)
constexpr int WCOL = 64 * WQ_MAX;

bool wide_ok(int ld) { return ld > WS && ld <= WCOL; }

// v[4a+b] = src[i * lds + c] (i = ty + 16a, c = tx + 16b) for i < nr, c < nc
__device__ __forceinline__ void fetch_rc(const double* __restrict__ src, int nr, int nc, int lds, double (&v)[16]) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = ty + 16 * a, c = tx + 16 * b;
      v[4 * a + b] = (i < nr && c < nc) ? src[i * lds + c] : 0.0;
    }
}

__device__ __forceinline__ void zero44(double (&t)[4][4]) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) t[a][b] = 0.0;
}

// This thread's 16 elements of tile (I, J) of an s x s matrix with leading
// dimension ld, in the lds_mm output layout: load (0 outside) and store.
__device__ __forceinline__ void tile_get(const double* __restrict__ M, int ld, int s, int I, int J, double (&t)[4][4]) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = 64 * I + acc_row(a), c = 64 * J + acc_col(b);
      t[a][b] = (r < s && c < s) ? M[(int64_t)r * ld + c] : 0.0;
    }
}
__device__ __forceinline__ void tile_put(double* __restrict__ M, int ld, int s, int I, int J, const double (&t)[4][4]) {
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = 64 * I + acc_row(a), c = 64 * J + acc_col(b);
      if (r < s && c < s) M[(int64_t)r * ld + c] = t[a][b];
    }
}

// tot += sign * sum_{K0 <= K < K1} op(X)_{IK} op(Y)_{KJ} on tiles of s x s
// matrices (op = transpose when tX / tY).  Both operand tiles go through LDS
// in the X^T B form of lds_mm: SA[l][r] = op(X)[r][l], SB[l][c] = op(Y)[l][c].
__device__ __forceinline__ void wterm(double (&tot)[4][4], double sign, const double* __restrict__ X, int ldx, bool tX,
                                      const double* __restrict__ Y, int ldy, bool tY, int s, int I, int J, int K0,
                                      int K1, double (*SA)[LP], double (*SB)[LP]) {
  for (int K = K0; K < K1; ++K) {
    const int kext = min(64, s - 64 * K);
    double va[16], vb[16];
    __syncthreads();   // earlier stores visible, earlier readers of SA / SB done
    if (!tX) fetch_rc(X + (int64_t)(64 * I) * ldx + 64 * K, s - 64 * I, s - 64 * K, ldx, va);
    else fetch_rc(X + (int64_t)(64 * K) * ldx + 64 * I, s - 64 * K, s - 64 * I, ldx, va);
    if (!tY) fetch_rc(Y + (int64_t)(64 * K) * ldy + 64 * J, s - 64 * K, s - 64 * J, ldy, vb);
    else fetch_rc(Y + (int64_t)(64 * J) * ldy + 64 * K, s - 64 * J, s - 64 * K, ldy, vb);
    if (!tX) put64T(SA, va); else put64(SA, va);
    if (!tY) put64(SB, vb); else put64T(SB, vb);
    __syncthreads();
    double acc[4][4];
    lds_mm<true, false>(SA, SB, kext, acc);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) tot[a][b] = fma(sign, acc[a][b], tot[a][b]);
  }
}

// Right-looking blocked Cholesky with inverse of an s x s symmetric matrix
// (tiles of 64): for each tile column b
//   A_bb = L_bb L_bb^T, Y_bb = L_bb^{-1}   (tile64 blocked factor, pivot rule MODE)
//   L_ib = A_ib Y_bb^T,  A_ij -= L_ib L_jb^T   (b < j <= i)
// then the off-diagonal tiles of Y = L^{-1} by block forward substitution
//   Y_ib = -Y_ii sum_{b <= k < i} L_ik Y_kb.
// A (ld) holds the lower tiles of the matrix on entry (diagonal tiles in full)
// and L on exit; Y (ld) receives L^{-1}.  Upper tiles of both are zeroed.
// g0 / dp / dg: per-column data of the pivot rule (LDS, global column index).
template <int MODE>
__device__ __forceinline__ void wide_chol_inv(double* __restrict__ A, double* __restrict__ Y, int ld, int s, const double* g0,
                              const double* dp, double thr, double* dg, int* bad, int* clf, double (*T0)[LP],
                              double (*T1)[LP], double (*T2)[LP], double (*T3)[LP]) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int nQ = (s + 63) >> 6;
  for (int b = 0; b < nQ; ++b) {
    const int sb = min(64, s - 64 * b);
    double* Abb = A + (int64_t)(64 * b) * ld + 64 * b;
    double* Ybb = Y + (int64_t)(64 * b) * ld + 64 * b;
    {
      double v[16];
      __syncthreads();
      fetch_rc(Abb, sb, sb, ld, v);
      put64(T0, v);
    }
    __syncthreads();
    blk_chol_inv_t<MODE>(T0, T1, T2, sb, g0 ? g0 + 64 * b : nullptr, dp ? dp + 64 * b : nullptr, thr,
                         dg ? dg + 64 * b : nullptr, bad, clf ? clf + 64 * b : nullptr);
    // L_bb, Y_bb out; T3 = Y_bb^T for the panel products
    for (int i = ty; i < WS; i += 16)
      for (int c = tx; c < WS; c += 16) {
        if (i < sb && c < sb) {
          Abb[(int64_t)i * ld + c] = T0[i][c];
          Ybb[(int64_t)i * ld + c] = T1[i][c];
        }
        T3[c][i] = T1[i][c];
      }
    // panel: L_ib = A_ib Y_bb^T (i > b), in place
    for (int i = b + 1; i < nQ; ++i) {
      double v[16];
      __syncthreads();
      fetch_rc(A + (int64_t)(64 * i) * ld + 64 * b, s - 64 * i, sb, ld, v);
      put64T(T2, v);    // T2[l][r] = A_ib[r][l]
      __syncthreads();
      double acc[4][4];
      lds_mm<true, false>(T2, T3, sb, acc);
      if (clf) {
        // columns with a clamped pivot stay decoupled
#pragma unroll
        for (int bb = 0; bb < 4; ++bb)
          if (clf[64 * b + acc_col(bb)])
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a][bb] = 0.0;
      }
      tile_put(A, ld, s, i, b, acc);
    }
    // trailing update of the lower tiles
    for (int i = b + 1; i < nQ; ++i)
      for (int j = b + 1; j <= i; ++j) {
        double t[4][4];
        tile_get(A, ld, s, i, j, t);
        wterm(t, -1.0, A, ld, false, A, ld, true, s, i, j, b, b + 1, T0, T2);
        tile_put(A, ld, s, i, j, t);
      }
  }
  // off-diagonal tiles of the inverse
  for (int i = 1; i < nQ; ++i)
    for (int b = 0; b < i; ++b) {
      double t[4][4];
      zero44(t);
      wterm(t, 1.0, A, ld, false, Y, ld, false, s, i, b, b, i, T0, T2);
      tile_put(Y, ld, s, i, b, t);   // sum_k L_ik Y_kb (Y_ib is not among its inputs)
      double u[4][4];
      zero44(u);
      // every thread staged its tiles before the barrier inside wterm, so
      // Y_ib can be overwritten in place
      wterm(u, -1.0, Y, ld, false, Y, ld, false, s, i, b, i, i + 1, T0, T2);
      tile_put(Y, ld, s, i, b, u);
    }
  // upper tiles are zero
  __syncthreads();
  for (int i = 0; i < nQ; ++i)
    for (int j = i + 1; j < nQ; ++j) {
      double z[4][4];
      zero44(z);
      tile_put(A, ld, s, i, j, z);
      tile_put(Y, ld, s, i, j, z);
    }
  __syncthreads();
}

// dst (ld x ld) = the transpose of the lower triangle of src (ld x ld), zero
// padded, through 64 x 64 LDS tiles (coalesced reads and writes); dst2
// (non-null) receives its leading n2 x n2 block with leading dimension n2.
__device__ __forceinline__ void put_upper_transposed(double* __restrict__ dst, double* __restrict__ dst2, int n2,
                                                     const double* __restrict__ src, int ld, int s,
                                                     double (*T)[LP]) {
  const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
  const int nT = (ld + 63) >> 6;
  for (int I = 0; I < nT; ++I)
    for (int J = 0; J < nT; ++J) {
      if (I <= J) {
        __syncthreads();
        for (int r = ty; r < 64; r += ST / 64) {
          const int gr = 64 * J + r, gc = 64 * I + tx;
          T[r][tx] = (gr < s && gc < s && gc <= gr) ? src[(int64_t)gr * ld + gc] : 0.0;
        }
        __syncthreads();
      }
      for (int r = ty; r < 64; r += ST / 64) {
        const int gr = 64 * I + r, gc = 64 * J + tx;
        const double v = (I <= J) ? T[tx][r] : 0.0;
        if (gr < ld && gc < ld) dst[(int64_t)gr * ld + gc] = v;
        if (dst2 && gr < n2 && gc < n2) dst2[(int64_t)gr * n2 + gc] = v;
      }
    }
  __syncthreads();
}

// ---------------------------------------------------------------- CholQR
// Same factor as the 64-wide kernel (pass 1: clamped pivots, pass 2:
// combined-diagonal deflation, then Rc = R1inv R2inv and B = R2 R1), for
// 64 < ld <= 512.  Aw, Yw: ld x ld device scratch.
__device__ __forceinline__ void
cholqr_wide_body(const double* __restrict__ G, int ld, int s, int pass, const double* __restrict__ diag_prev,
                   double thr, double* __restrict__ Aw, double* __restrict__ Yw, double* __restrict__ R,
                   double* __restrict__ Rinv, double* __restrict__ diag_out, int* __restrict__ n_defl,
                   const double* __restrict__ R1, const double* __restrict__ R1inv, double* __restrict__ Rc,
                   double* __restrict__ Bout, double* __restrict__ BT, int* __restrict__ gate) {
  // second pass not needed (decided by the first pass and the projection):
  // counted in the slot five entries after the deflation count
  if (pass == 2 && gate && *gate == 0) {
    if (threadIdx.x == 0 && n_defl) n_defl[5] += 1;
    return;
  }
  __shared__ __align__(16) double T0[WS][LP];
  __shared__ __align__(16) double T1[WS][LP];
  __shared__ __align__(16) double T2[WS][LP];
  __shared__ __align__(16) double T3[WS][LP];
  __shared__ double g0[WCOL], dp[WCOL], dg[WCOL];
  __shared__ int clf[WCOL];
  const int tid = threadIdx.x;
  const int nQ = (s + 63) >> 6;
  for (int q = tid; q < ld * ld; q += ST) Aw[q] = G[q];
  for (int q = tid; q < s; q += ST) {
    g0[q] = G[(int64_t)q * ld + q];
    dp[q] = (pass == 2) ? diag_prev[q] : 0.0;
  }
  __syncthreads();
  if (pass == 1)
    wide_chol_inv<1>(Aw, Yw, ld, s, g0, dp, thr, dg, nullptr, clf, T0, T1, T2, T3);
  else
    wide_chol_inv<2>(Aw, Yw, ld, s, g0, dp, thr, dg, nullptr, clf, T0, T1, T2, T3);
  // Pass 1 with a gate: one pass leaves X R^-1 orthonormal to about
  // s u |D R^-1|_2^2 with D = diag(G)^(1/2) (Gram and Cholesky errors are
  // relative to the column norms), and |D R^-1|_2^2 <= |Z|_1 |Z|_inf for
  // Z = L^-1 D (R = L^T, L^-1 in Yw).  When that gives 1e-10 or better and
  // no pivot was clamped, the first factor is final: Rc = R^-1, B = R and
  // B^T are written with R and R^-1 below, and the gate tells the second
  // pass (and the Gram launch before it) to do nothing.  Column sums one
  // thread per column, row sums one wavefront per row.
  bool sk = false;
  if (pass == 1 && gate) {
    __shared__ double nred[3][ST / 64];
    __shared__ int skip_s;
    const int lane = tid & 63, wv = tid >> 6;
    double cmax = 0.0, rmax = 0.0, cl = 0.0;
    for (int c = tid; c < s; c += ST) {
      double a = 0.0;
      for (int i = c; i < s; ++i) a += fabs(Yw[(int64_t)i * ld + c]);
      cmax = fmax(cmax, a * sqrt(fmax(g0[c], 0.0)));
      cl = (clf[c] != 0 || dg[c] == 0.0) ? 1.0 : cl;
    }
    for (int i = wv; i < s; i += ST / 64) {
      double a = 0.0;
      for (int j = lane; j <= i; j += 64) a += fabs(Yw[(int64_t)i * ld + j]) * sqrt(fmax(g0[j], 0.0));
      for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
      rmax = fmax(rmax, a);
    }
    for (int o = 32; o > 0; o >>= 1) {
      cmax = fmax(cmax, __shfl_xor(cmax, o));
      cl = fmax(cl, __shfl_xor(cl, o));
    }
    if (lane == 0) {
      nred[0][wv] = cmax;
      nred[1][wv] = rmax;
      nred[2][wv] = cl;
    }
    __syncthreads();
    if (tid == 0) {
      double nm[3] = {0.0, 0.0, 0.0};
      for (int w = 0; w < ST / 64; ++w)
        for (int t = 0; t < 3; ++t) nm[t] = fmax(nm[t], nred[t][w]);
      const bool skip = nm[2] == 0.0 && nm[0] * nm[1] * (double)s * 0x1p-53 <= 1e-10;
      *gate = skip ? 0 : 1;
      skip_s = skip ? 1 : 0;
    }
    __syncthreads();
    sk = skip_s != 0;
  }
  // R = L^T, Rinv = Y^T (upper, zero padded) through 64 x 64 LDS transposes;
  // skipped when R is null
  if (R) {
    put_upper_transposed(R, sk ? Bout : nullptr, s, Aw, ld, s, T0);      // B = R (s x s)
    put_upper_transposed(Rinv, sk ? Rc : nullptr, ld, Yw, ld, s, T1);   // Rc = R^-1 (ld x ld)
    if (sk && BT)
      for (int q = tid; q < ld * ld; q += ST) {
        const int i = q / ld, c = q - i * ld;
        BT[q] = (i < s && c < s && i >= c) ? Aw[q] : 0.0;   // R^T = L
      }
  }
  for (int q = tid; q < ld; q += ST) diag_out[q] = (q < s) ? dg[q] : 0.0;
  if (pass != 2) return;
  if (tid == 0 && n_defl) {
    int cnt = 0;
    for (int j = 0; j < s; ++j) cnt += (dg[j] == 0.0);
    n_defl[0] += cnt;
  }
  // upper triangular products: tile (I, J) sums over I <= K <= J
  for (int I = 0; I < nQ; ++I)
    for (int J = 0; J < nQ; ++J) {
      double b[4][4], c[4][4];
      zero44(b);
      zero44(c);
      if (I <= J) {
        wterm(b, 1.0, Aw, ld, true, R1, ld, false, s, I, J, I, J + 1, T0, T1);       // B = L2^T R1
        wterm(c, 1.0, R1inv, ld, false, Yw, ld, true, s, I, J, I, J + 1, T0, T1);    // Rc = R1inv Y2^T
      }
      tile_put(Bout, s, s, I, J, b);
      tile_put(Rc, ld, s, I, J, c);
    }
  // Rc padding (rows / columns s..ld-1) is zero
  for (int q = tid; q < ld * ld; q += ST) {
    const int i = q / ld, c = q % ld;
    if (i >= s || c >= s) Rc[q] = 0.0;
  }
  if (BT) {
    // B^T zero padded to ld x ld, from this workgroup's B written above
    __syncthreads();
    for (int q = tid; q < ld * ld; q += ST) {
      const int i = q / ld, c = q % ld;
      BT[q] = (i < s && c < s) ? Bout[(int64_t)c * s + i] : 0.0;
    }
  }
}

__global__ void __launch_bounds__(ST)
cholqr_wide_kernel(const double* __restrict__ G, int ld, int s, int pass, const double* __restrict__ diag_prev,
                   double thr, double* __restrict__ Aw, double* __restrict__ Yw, double* __restrict__ R,
                   double* __restrict__ Rinv, double* __restrict__ diag_out, int* __restrict__ n_defl,
                   const double* __restrict__ R1, const double* __restrict__ R1inv, double* __restrict__ Rc,
                   double* __restrict__ Bout, double* __restrict__ BT) {
  cholqr_wide_body(G, ld, s, pass, diag_prev, thr, Aw, Yw, R, Rinv, diag_out, n_defl, R1, R1inv, Rc, Bout, BT,
                   nullptr);
}

struct CholqrWideBatch {
  CholqrArgs a[kCholqrBatch];
};
__global__ void __launch_bounds__(ST) cholqr_wide_batch_kernel(CholqrWideBatch b) {
  const CholqrArgs& a = b.a[blockIdx.x];
  cholqr_wide_body(a.G, a.ld, a.s, a.pass, a.diag_prev, a.thr, a.wk, a.wk + (size_t)a.ld * a.ld, a.R, a.Rinv,
                   a.diag_out, a.n_defl, a.R1, a.R1inv, a.Rc, a.Bout, a.BT, a.gate);
}

size_t cholqr_wide_scratch_elems(int ld) { return (size_t)2 * ld * ld; }

void launch_cholqr_wide(const double* G, int ld, int s, int pass, const double* diag_prev, double thr, double* wk,
                        double* R, double* Rinv, double* diag_out, int* n_defl, const double* R1, const double* R1inv,
                        double* Rc, double* Bout, double* BT, hipStream_t st) {
  kt_begin(KC_CHOLQR, st);
  hipLaunchKernelGGL(cholqr_wide_kernel, dim3(1), dim3(ST), 0, st, G, ld, s, pass, diag_prev, thr, wk,
                     wk + (size_t)ld * ld, R, Rinv, diag_out, n_defl, R1, R1inv, Rc, Bout, BT);
  GK_HIP(hipGetLastError());
  kt_end(st, 8.0 * 6 * ld * ld, (double)s * s * s * (pass == 2 ? 3.0 : 1.0));
}

void launch_cholqr_wide_batched(const CholqrArgs* a, int count, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += kCholqrBatch) {
    const int nb = std::min(kCholqrBatch, count - c0);
    CholqrWideBatch b{};
    double bytes = 0, flops = 0;
    for (int i = 0; i < nb; ++i) {
      b.a[i] = a[c0 + i];
      bytes += 8.0 * 6 * a[c0 + i].ld * a[c0 + i].ld;
      flops += (double)a[c0 + i].s * a[c0 + i].s * a[c0 + i].s * (a[c0 + i].pass == 2 ? 3.0 : 1.0);
    }
    kt_begin(KC_CHOLQR, st);
    hipLaunchKernelGGL(cholqr_wide_batch_kernel, dim3(nb), dim3(ST), 0, st, b);
    GK_HIP(hipGetLastError());
    kt_end(st, bytes, flops);
  }
}

// ------------------------------------------------- orthogonality estimate
// Block omega recurrence (the same estimate as the 64-wide kernel): first
// the right-hand side
//   W_{k,j+1} B_j + W_{k,j} H_j - H_k W_{k,j} + W_{k,j-1} B_{j-1}^T - B_{k-1} W_{k-1,j}
// plus the rounding model (+-nu in the direction of each entry), one
// workgroup per (j, tile); then W_{k+1,j} = Rc^T RHS and the tile maxima.
__global__ void __launch_bounds__(ST)
omega_rhs_wide_kernel(int k, int s, const double* __restrict__ Wk, const double* __restrict__ Wkm1,
                      const double* __restrict__ Hd, const double* __restrict__ Bd, double nu,
                      double* __restrict__ rhs) {
  __shared__ __align__(16) double SA[WS][LP];
  __shared__ __align__(16) double SB[WS][LP];
  const int j = blockIdx.x, I = blockIdx.y, J = blockIdx.z;
  const int nQ = (s + 63) >> 6;
  const int64_t ss = (int64_t)s * s;
  double t[4][4];
  zero44(t);
  wterm(t, 1.0, Wk + (j + 1) * ss, s, false, Bd + j * ss, s, false, s, I, J, 0, nQ, SA, SB);
  wterm(t, 1.0, Wk + j * ss, s, false, Hd + j * ss, s, false, s, I, J, 0, nQ, SA, SB);
  wterm(t, -1.0, Hd + (int64_t)k * ss, s, false, Wk + j * ss, s, false, s, I, J, 0, nQ, SA, SB);
  if (j >= 1) wterm(t, 1.0, Wk + (j - 1) * ss, s, false, Bd + (j - 1) * ss, s, true, s, I, J, 0, nQ, SA, SB);
  wterm(t, -1.0, Bd + (int64_t)(k - 1) * ss, s, false, Wkm1 + j * ss, s, false, s, I, J, 0, nQ, SA, SB);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) t[a][b] += copysign(nu, t[a][b]);
  tile_put(rhs + j * ss, s, s, I, J, t);
}

__global__ void __launch_bounds__(ST)
omega_apply_wide_kernel(int s, int ld, const double* __restrict__ Rc, const double* __restrict__ rhs,
                        double* __restrict__ Wk1, double* __restrict__ est_part) {
  __shared__ __align__(16) double SA[WS][LP];
  __shared__ __align__(16) double SB[WS][LP];
  __shared__ double red[ST];
  const int j = blockIdx.x, I = blockIdx.y, J = blockIdx.z;
  const int nQ = (s + 63) >> 6;
  const int64_t ss = (int64_t)s * s;
  const int tid = threadIdx.x;
  double t[4][4];
  zero44(t);
  wterm(t, 1.0, Rc, ld, true, rhs + j * ss, s, false, s, I, J, 0, nQ, SA, SB);
  tile_put(Wk1 + j * ss, s, s, I, J, t);
  double mx = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) mx = fmax(mx, fabs(t[a][b]));   // zero outside s
  red[tid] = mx;
  __syncthreads();
  for (int w = ST / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  if (tid == 0) est_part[((int64_t)j * nQ + I) * nQ + J] = red[0];
}

size_t omega_wide_scratch_elems(int m, int s) { return (size_t)m * s * s; }

void launch_omega_wide(int k, int s, int ld, const double* Wk, const double* Wkm1, double* Wk1, const double* Hd,
                       const double* Bd, const double* Rc, double nu, double* rhs, double* est_part, hipStream_t st) {
  const int nj = k - 1;
  const int nQ = (s + 63) >> 6;
  kt_begin(KC_OMEGA, st);
  hipLaunchKernelGGL(omega_rhs_wide_kernel, dim3(nj, nQ, nQ), dim3(ST), 0, st, k, s, Wk, Wkm1, Hd, Bd, nu, rhs);
  GK_HIP(hipGetLastError());
  hipLaunchKernelGGL(omega_apply_wide_kernel, dim3(nj, nQ, nQ), dim3(ST), 0, st, s, ld, Rc, rhs, Wk1, est_part);
  GK_HIP(hipGetLastError());
  kt_end(st, 8.0 * 12 * nj * (double)s * s, 12.0 * nj * (double)s * s * s);
}

// ------------------------------------------------------ banded spline
// (eps I + H_m)^(-k) F_1 by block Cholesky of the block tridiagonal
// eps I + H_m (same factorisation as the 64-wide kernels):
//   A_j = eps I + H_jj - Lsub_{j-1} Lsub_{j-1}^T = L_jj L_jj^T,
//   Linv_j = L_jj^{-1},  Lsub_j = B_j Linv_j^T,
// then k forward / backward block substitutions.  Work layout (s x s each):
// Linv_0..m-1, Lsub_0..m-1, one factor scratch.
__global__ void __launch_bounds__(ST)
banded_factor_wide_kernel(int m, int s, const double* __restrict__ Hd, const double* __restrict__ Bd, double eps,
                          double* __restrict__ Linv, double* __restrict__ Lsub, double* __restrict__ Aw,
                          int* __restrict__ bad) {
  __shared__ __align__(16) double T0[WS][LP];
  __shared__ __align__(16) double T1[WS][LP];
  __shared__ __align__(16) double T2[WS][LP];
  __shared__ __align__(16) double T3[WS][LP];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int nQ = (s + 63) >> 6;
  const int64_t ss = (int64_t)s * s;
  for (int j = 0; j < m; ++j) {
    // A = eps I + H_jj - Lsub_{j-1} Lsub_{j-1}^T on the lower tiles
    for (int I = 0; I < nQ; ++I)
      for (int J = 0; J <= I; ++J) {
        double t[4][4];
        tile_get(Hd + j * ss, s, s, I, J, t);
        if (I == J) {
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
              if (acc_row(a) == acc_col(b)) t[a][b] += eps;
        }
        if (j > 0) wterm(t, -1.0, Lsub + (j - 1) * ss, s, false, Lsub + (j - 1) * ss, s, true, s, I, J, 0, nQ, T0, T1);
        tile_put(Aw, s, s, I, J, t);
      }
    double* Li = Linv + j * ss;
    wide_chol_inv<0>(Aw, Li, s, s, nullptr, nullptr, 0.0, nullptr, bad, nullptr, T0, T1, T2, T3);
    if (j + 1 < m) {
      // Lsub_j = B_j Linv_j^T: tile (I, J) sums over K <= J (Linv_j lower)
      for (int I = 0; I < nQ; ++I)
        for (int J = 0; J < nQ; ++J) {
          double t[4][4];
          zero44(t);
          wterm(t, 1.0, Bd + j * ss, s, false, Li, s, true, s, I, J, 0, J + 1, T0, T1);
          tile_put(Lsub + j * ss, s, s, I, J, t);
        }
    }
  }
}

// One workgroup per column tile J of U (the columns are independent).
// forward:  Z_j = Linv_j (Y_j - Lsub_{j-1} Z_{j-1})
// backward: Y_j = Linv_j^T (Z_j - Lsub_j^T Y_{j+1})
// T: s x s scratch per column tile (this workgroup's columns only).
__global__ void __launch_bounds__(ST)
banded_solve_wide_kernel(int m, int s, int kpow, const double* __restrict__ Linv, const double* __restrict__ Lsub,
                         double* __restrict__ U, double* __restrict__ T) {
  __shared__ __align__(16) double SA[WS][LP];
  __shared__ __align__(16) double SB[WS][LP];
  const int J = blockIdx.x;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int nQ = (s + 63) >> 6;
  const int64_t ss = (int64_t)s * s;
  // U = F_1 on this column tile
  for (int j = 0; j < m; ++j)
    for (int I = 0; I < nQ; ++I) {
      double t[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int r = 64 * I + acc_row(a), c = 64 * J + acc_col(b);
          t[a][b] = (j == 0 && r == c) ? 1.0 : 0.0;
        }
      tile_put(U + j * ss, s, s, I, J, t);
    }
  for (int rep = 0; rep < kpow; ++rep) {
    for (int j = 0; j < m; ++j) {
      double* Uj = U + j * ss;
      for (int I = 0; I < nQ; ++I) {
        double t[4][4];
        __syncthreads();
        tile_get(Uj, s, s, I, J, t);
        if (j > 0) wterm(t, -1.0, Lsub + (j - 1) * ss, s, false, U + (j - 1) * ss, s, false, s, I, J, 0, nQ, SA, SB);
        tile_put(T, s, s, I, J, t);
      }
      for (int I = 0; I < nQ; ++I) {
        double t[4][4];
        zero44(t);
        wterm(t, 1.0, Linv + j * ss, s, false, T, s, false, s, I, J, 0, I + 1, SA, SB);
        tile_put(Uj, s, s, I, J, t);
      }
    }
    for (int j = m - 1; j >= 0; --j) {
      double* Uj = U + j * ss;
      for (int I = 0; I < nQ; ++I) {
        double t[4][4];
        __syncthreads();
        tile_get(Uj, s, s, I, J, t);
        if (j + 1 < m) wterm(t, -1.0, Lsub + j * ss, s, true, U + (j + 1) * ss, s, false, s, I, J, 0, nQ, SA, SB);
        tile_put(T, s, s, I, J, t);
      }
      for (int I = 0; I < nQ; ++I) {
        double t[4][4];
        zero44(t);
        wterm(t, 1.0, Linv + j * ss, s, true, T, s, false, s, I, J, I, nQ, SA, SB);
        tile_put(Uj, s, s, I, J, t);
      }
    }
  }
}

size_t banded_wide_work_elems(int m, int s) { return (size_t)(2 * m + 2) * s * s; }

void launch_banded_spline_wide(int m, int s, const double* Hd, const double* Bd, double eps, int k, double* work,
                               double* U, int* bad, hipStream_t st) {
  const size_t ss = (size_t)s * s;
  const int nQ = (s + 63) >> 6;
  double* Linv = work;
  double* Lsub = work + m * ss;
  double* Aw = work + 2 * m * ss;
  double* T = Aw + ss;   // one s x s scratch; each column tile workgroup uses its own columns
  kt_begin(KC_BANDED_FACTOR, st);
  hipLaunchKernelGGL(banded_factor_wide_kernel, dim3(1), dim3(ST), 0, st, m, s, Hd, Bd, eps, Linv, Lsub, Aw, bad);
  GK_HIP(hipGetLastError());
  kt_end(st, 8.0 * 4 * m * (double)ss, (double)m * ss * s * (2.0 + 1.0 / 3.0 + 1.0));
  kt_begin(KC_BANDED_SOLVE, st);
  hipLaunchKernelGGL(banded_solve_wide_kernel, dim3(nQ), dim3(ST), 0, st, m, s, k, Linv, Lsub, U, T);
  GK_HIP(hipGetLastError());
  kt_end(st, 8.0 * 4 * 2 * k * m * (double)ss, 4.0 * 2 * k * m * (double)ss * s);
}

// ------------------------------------------------ Chebyshev series step
// One term of the series of exp(-t lam) applied to F_1 through the block
// tridiagonal H_m (blocks H_jj, sub-diagonal B_j = H_{j+1,j}):
//   out_j = alpha (B_{j-1} Y_{j-1} + H_jj Y_j + B_j^T Y_{j+1}) + beta Y_j + gamma Yp_j,
//   acc_j += coef[kk] out_j,
// one workgroup per 64 x 64 output tile (j, I, J) on the tile path above.
__global__ void __launch_bounds__(ST)
btd_cheb_tile_kernel(int m, int s, const double* __restrict__ Hd, const double* __restrict__ Bd,
                     const double* __restrict__ Y, const double* __restrict__ Yp, double* __restrict__ out,
                     double alpha, double beta, double gamma, double* __restrict__ acc,
                     const double* __restrict__ coef, int kk) {
  __shared__ __align__(16) double SA[WS][LP];
  __shared__ __align__(16) double SB[WS][LP];
  const int j = blockIdx.x, I = blockIdx.y, J = blockIdx.z;
  const int nQ = (s + 63) >> 6;
  const int64_t ss = (int64_t)s * s;
  double t[4][4];
  zero44(t);
  wterm(t, 1.0, Hd + j * ss, s, false, Y + j * ss, s, false, s, I, J, 0, nQ, SA, SB);
  if (j > 0) wterm(t, 1.0, Bd + (j - 1) * ss, s, false, Y + (j - 1) * ss, s, false, s, I, J, 0, nQ, SA, SB);
  if (j + 1 < m) wterm(t, 1.0, Bd + j * ss, s, true, Y + (j + 1) * ss, s, false, s, I, J, 0, nQ, SA, SB);
  double yv[4][4], pv[4][4], av[4][4];
  tile_get(Y + j * ss, s, s, I, J, yv);
  if (Yp) tile_get(Yp + j * ss, s, s, I, J, pv);
  else zero44(pv);
  tile_get(acc + j * ss, s, s, I, J, av);
  const double ck = coef[kk];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double v = alpha * t[a][b] + beta * yv[a][b] + gamma * pv[a][b];
      t[a][b] = v;
      av[a][b] += ck * v;
    }
  tile_put(out + j * ss, s, s, I, J, t);
  tile_put(acc + j * ss, s, s, I, J, av);
}

void launch_btd_cheb_tile(int m, int s, const double* Hd, const double* Bd, const double* Y, const double* Yp,
                          double* out, double alpha, double beta, double gamma, double* acc, const double* coef,
                          int kk, hipStream_t st) {
  GK_REQUIRE(s <= WCOL, GK_EINVAL, "Chebyshev step: block width above 512");
  const int nQ = (s + 63) >> 6;
  hipLaunchKernelGGL(btd_cheb_tile_kernel, dim3(m, nQ, nQ), dim3(ST), 0, st, m, s, Hd, Bd, Y, Yp, out, alpha, beta,
                     gamma, acc, coef, kk);
  GK_HIP(hipGetLastError());
}

}  // namespace gk
