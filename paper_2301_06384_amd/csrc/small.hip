// Small dense float64 work: QR factors of the Lanczos blocks, the projected
// matrix H_m, its spectral decomposition and phi(H_m) F_1, the exact banded
// evaluation of spline kernels, and the s x s kernel system.
//
// Everything here is float64 (the small factors of the method).  Matrices
// live in device memory; one workgroup owns one matrix, so these kernels
// need no grid-wide synchronisation.
#include "gk_internal.h"
#include "tile64.h"
#include "decide.h"

namespace gk {

constexpr int SB = 1024;   // threads of the single-workgroup kernels

// ------------------------------------------------------------- CholQR
// Upper Cholesky G = R^T R of a Gram matrix with column deflation, followed
// by the pseudo-inverse Rinv on the kept columns (X Rinv has orthonormal kept
// columns and zero deflated columns; X ~ (X Rinv) R).
//
// pass 1: a column whose Gram diagonal is below thr^2 is deflated; otherwise
//   the pivot is clamped from below by eta^2 G_jj, so nearly dependent
//   columns survive into pass 2 scaled down instead of being dropped on a
//   noisy pivot.
// pass 2: a column is deflated when its pivot is not positive or when the
//   combined diagonal R2_jj * R1_jj (the true residual norm of the column
//   after the first pass) is below thr.  This matches the rank decision of a
//   Householder QR with threshold thr.
__global__ void __launch_bounds__(SB)
cholqr_factor_kernel(const double* __restrict__ G, int ld, int s, int pass,
                     const double* __restrict__ diag_prev, double thr, double* __restrict__ W,
                     double* __restrict__ R, double* __restrict__ Rinv, double* __restrict__ diag_out,
                     int* __restrict__ n_defl) {
  __shared__ double rjj_sh;
  __shared__ int ndef_sh, clamp_sh;
  const int tid = threadIdx.x;
  const double eta = 1e-7;
  for (int q = tid; q < ld * ld; q += SB) {
    W[q] = G[q];
    R[q] = 0.0;
    Rinv[q] = 0.0;
  }
  if (tid == 0) ndef_sh = 0;
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    if (tid == 0) {
      const double piv = W[j * ld + j];
      double r = 0.0;
      int cl = 0;
      if (pass == 1) {
        const double g0 = G[j * ld + j];
        if (g0 > thr * thr) {
          r = sqrt(fmax(piv, eta * eta * g0));
          cl = !(piv >= eta * eta * g0);   // clamped: decoupled below
        }
      } else {
        if (piv > 0.0) {
          r = sqrt(piv);
          if (r * diag_prev[j] < thr) r = 0.0;
        }
      }
      if (r == 0.0) ndef_sh++;
      rjj_sh = r;
      clamp_sh = cl;
      diag_out[j] = r;
      R[j * ld + j] = r;
    }
    __syncthreads();
    const double rjj = rjj_sh;
    // a clamped pivot keeps its (clamped) diagonal but no coupling to the
    // later columns: R[j][c] = 0 for c > j, no Schur update
    if (rjj != 0.0 && !clamp_sh) {
      for (int c = j + 1 + tid; c < s; c += SB) R[j * ld + c] = W[j * ld + c] / rjj;
      __syncthreads();
      const int w = s - j - 1;
      for (int q = tid; q < w * w; q += SB) {
        const int r = j + 1 + q / w, c = j + 1 + q % w;
        if (c >= r) W[r * ld + c] -= R[j * ld + r] * R[j * ld + c];
      }
    }
    __syncthreads();
  }
  for (int j = s + tid; j < ld; j += SB) diag_out[j] = 0.0;
  // Rinv: one thread per column, back substitution over kept rows
  for (int c = tid; c < s; c += SB) {
    if (R[c * ld + c] == 0.0) continue;
    Rinv[c * ld + c] = 1.0 / R[c * ld + c];
    for (int i = c - 1; i >= 0; --i) {
      const double rii = R[i * ld + i];
      if (rii == 0.0) continue;
      double acc = 0.0;
      for (int l = i + 1; l <= c; ++l) acc += R[i * ld + l] * Rinv[l * ld + c];
      Rinv[i * ld + c] = -acc / rii;
    }
  }
  if (tid == 0 && n_defl && pass == 2) *n_defl += ndef_sh;
}

void launch_cholqr_factor(const double* G, int ld, int s, int pass, const double* diag_prev, double thr,
                          double* W, double* R, double* Rinv, double* diag_out, int* n_defl,
                          hipStream_t st) {
  kt_begin(KC_CHOLQR, st);
  hipLaunchKernelGGL(cholqr_factor_kernel, dim3(1), dim3(SB), 0, st, G, ld, s, pass, diag_prev, thr, W, R,
                     Rinv, diag_out, n_defl);
  GK_HIP(hipGetLastError());
  kt_end(st, 8.0 * 4 * ld * ld, (double)s * s * s);
}

// ------------------------------------------------------------ small GEMM
// C = alpha * op(A) op(B) + beta * C, one thread per entry (small sizes).
__global__ void small_gemm_kernel(int M, int N, int K, const double* __restrict__ A, int lda, int ta,
                                  const double* __restrict__ B, int ldb, int tb, double* __restrict__ C,
                                  int ldc, double alpha, double beta) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * N) return;
  const int i = (int)(t / N), j = (int)(t % N);
  double acc = 0.0;
  for (int l = 0; l < K; ++l) {
    const double a = ta ? A[(int64_t)l * lda + i] : A[(int64_t)i * lda + l];
    const double b = tb ? B[(int64_t)j * ldb + l] : B[(int64_t)l * ldb + j];
    acc = fma(a, b, acc);
  }
  double* c = C + (int64_t)i * ldc + j;
  *c = alpha * acc + (beta != 0.0 ? beta * (*c) : 0.0);
}

void launch_small_gemm(int M, int N, int K, const double* A, int lda, bool ta, const double* B, int ldb,
                       bool tb, double* C, int ldc, double alpha, double beta, hipStream_t st) {
  const int64_t tot = (int64_t)M * N;
  hipLaunchKernelGGL(small_gemm_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, M, N, K, A,
                     lda, ta ? 1 : 0, B, ldb, tb ? 1 : 0, C, ldc, alpha, beta);
  GK_HIP(hipGetLastError());
}

// Hk = sym(C[0:s, 0:s]) (C has leading dimension ld; Hk is s x s)
__global__ void store_H_kernel(const double* __restrict__ C, int ld, int s, double* __restrict__ Hk) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= s * s) return;
  const int i = t / s, j = t % s;
  Hk[t] = 0.5 * (C[i * ld + j] + C[j * ld + i]);
}

void launch_store_H(const double* C, int ld, int s, double* Hk, hipStream_t st) {
  hipLaunchKernelGGL(store_H_kernel, dim3((s * s + 255) / 256), dim3(256), 0, st, C, ld, s, Hk);
  GK_HIP(hipGetLastError());
}

// Dense H_m from its blocks: H_kk on the diagonal, H_{k+1,k} = B_k below and
// its transpose above (Sec. 3.1: H_{k,k+1} = H_{k+1,k}^*).
__global__ void assemble_T_kernel(int m, int s, const double* __restrict__ Hd, const double* __restrict__ Bd,
                                  double* __restrict__ T, int ldt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ms = (int64_t)m * s;
  if (t >= ms * ms) return;
  const int r = (int)(t / ms), c = (int)(t % ms);
  const int br = r / s, bc = c / s, i = r % s, j = c % s;
  double v = 0.0;
  if (br == bc) v = Hd[((int64_t)br * s + i) * s + j];
  else if (br == bc + 1) v = Bd[((int64_t)bc * s + i) * s + j];
  else if (bc == br + 1) v = Bd[((int64_t)br * s + j) * s + i];
  T[(int64_t)r * ldt + c] = v;
}

void launch_assemble_T(int m, int s, const double* Hd, const double* Bd, double* T, int ldt,
                       hipStream_t st) {
  const int64_t tot = (int64_t)m * s * m * s;
  hipLaunchKernelGGL(assemble_T_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, m, s, Hd, Bd,
                     T, ldt);
  GK_HIP(hipGetLastError());
}

// ------------------------------------------------- symmetric eigensolver
// Cyclic two-sided Jacobi with round-robin pair ordering (n/2 disjoint
// rotations per round), one workgroup per matrix.  A is overwritten
// (diagonal -> eigenvalues), V receives the eigenvectors as columns:
// A_in = V diag(theta) V^T.  Sweeps stop when the off-diagonal mass is
// below (1e-17 ||A||_F)^2 or after 40 sweeps.
__global__ void __launch_bounds__(SB)
jacobi_eig_kernel(int n, double* __restrict__ Abase, int lda, double* __restrict__ Vbase, int ldv,
                  double* __restrict__ thbase, int64_t strideA, int64_t strideV, int64_t strideT,
                  int* __restrict__ order_base, double* __restrict__ cs_base) {
  double* A = Abase + blockIdx.x * strideA;
  double* V = Vbase + blockIdx.x * strideV;
  double* theta = thbase + blockIdx.x * strideT;
  const int np = (n + 1) & ~1;          // even number of players (one dummy if n odd)
  int* order = order_base + (int64_t)blockIdx.x * np;
  double* cs = cs_base + (int64_t)blockIdx.x * np;   // (c, s) per pair
  __shared__ double red[SB];
  __shared__ int go_sh;
  const int tid = threadIdx.x;
  for (int q = tid; q < n * n; q += SB) {
    const int i = q / n, j = q % n;
    V[(int64_t)i * ldv + j] = (i == j) ? 1.0 : 0.0;
  }
  for (int q = tid; q < np; q += SB) order[q] = q;
  __syncthreads();
  const int npairs = np / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test
    double off = 0.0, tot = 0.0;
    for (int q = tid; q < n * n; q += SB) {
      const int i = q / n, j = q % n;
      const double a = A[(int64_t)i * lda + j];
      tot += a * a;
      if (i != j) off += a * a;
    }
    red[tid] = off;
    __syncthreads();
    for (int w = SB / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double offs = red[0];
    __syncthreads();
    red[tid] = tot;
    __syncthreads();
    for (int w = SB / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double tots = red[0];
    __syncthreads();
    if (tid == 0) go_sh = (offs > 1e-34 * tots && offs > 1e-300) ? 1 : 0;
    __syncthreads();
    if (!go_sh) break;
    for (int round = 0; round < np - 1; ++round) {
      // rotation parameters
      for (int pi = tid; pi < npairs; pi += SB) {
        int p = order[pi], q = order[np - 1 - pi];
        double c = 1.0, sn = 0.0;
        if (p < n && q < n) {
          if (p > q) { const int t = p; p = q; q = t; }
          const double apq = A[(int64_t)p * lda + q];
          const double app = A[(int64_t)p * lda + p], aqq = A[(int64_t)q * lda + q];
          if (apq != 0.0 && fabs(apq) > 1e-300) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
          }
        }
        cs[2 * pi] = c;
        cs[2 * pi + 1] = sn;
      }
      __syncthreads();
      // columns of A and V:  col_p' = c col_p - s col_q ; col_q' = s col_p + c col_q
      for (int q2 = tid; q2 < npairs * n; q2 += SB) {
        const int pi = q2 / n, r = q2 % n;
        int p = order[pi], q = order[np - 1 - pi];
        if (p >= n || q >= n) continue;
        if (p > q) { const int t = p; p = q; q = t; }
        const double c = cs[2 * pi], sn = cs[2 * pi + 1];
        if (sn == 0.0) continue;
        double* ar = A + (int64_t)r * lda;
        const double ap = ar[p], aq = ar[q];
        ar[p] = c * ap - sn * aq;
        ar[q] = sn * ap + c * aq;
        double* vr = V + (int64_t)r * ldv;
        const double vp = vr[p], vq = vr[q];
        vr[p] = c * vp - sn * vq;
        vr[q] = sn * vp + c * vq;
      }
      __syncthreads();
      // rows of A
      for (int q2 = tid; q2 < npairs * n; q2 += SB) {
        const int pi = q2 / n, cc = q2 % n;
        int p = order[pi], q = order[np - 1 - pi];
        if (p >= n || q >= n) continue;
        if (p > q) { const int t = p; p = q; q = t; }
        const double c = cs[2 * pi], sn = cs[2 * pi + 1];
        if (sn == 0.0) continue;
        const double ap = A[(int64_t)p * lda + cc], aq = A[(int64_t)q * lda + cc];
        A[(int64_t)p * lda + cc] = c * ap - sn * aq;
        A[(int64_t)q * lda + cc] = sn * ap + c * aq;
      }
      __syncthreads();
      for (int pi = tid; pi < npairs; pi += SB) {
        int p = order[pi], q = order[np - 1 - pi];
        if (p < n && q < n && cs[2 * pi + 1] != 0.0) {
          A[(int64_t)p * lda + q] = 0.0;
          A[(int64_t)q * lda + p] = 0.0;
        }
      }
      __syncthreads();
      // rotate players 1..np-1 by one position
      if (tid == 0) {
        const int last = order[np - 1];
        for (int q = np - 1; q > 1; --q) order[q] = order[q - 1];
        order[1] = last;
      }
      __syncthreads();
    }
  }
  for (int q = tid; q < n; q += SB) theta[q] = A[(int64_t)q * lda + q];
}

void launch_sym_eig(int n, double* A, int lda, double* V, int ldv, double* theta, int batch,
                    int64_t strideA, int64_t strideV, int64_t strideTheta, int* order_ws, double* cs_ws,
                    hipStream_t st) {
  kt_begin(KC_EIG, st);
  hipLaunchKernelGGL(jacobi_eig_kernel, dim3(batch), dim3(SB), 0, st, n, A, lda, V, ldv, theta, strideA,
                     strideV, strideTheta, order_ws, cs_ws);
  GK_HIP(hipGetLastError());
  kt_end(st, 16.0 * batch * (double)n * n, 10.0 * batch * (double)n * n * n);
}

size_t eig_order_elems(int n, int batch) { return (size_t)(((n + 1) & ~1)) * batch; }

// ------------------------------------------------------------- phi
struct PhiDev {
  int kind;
  double t, eps, k;
  int plen;
};

__device__ __forceinline__ double phi_eval(const PhiDev& f, const double* poly, double lam, int* bad) {
  if (f.kind == GK_PHI_DIFFUSION) return exp(-f.t * lam);
  if (f.kind == GK_PHI_SPLINE) {
    const double z = f.eps + lam;
    if (!(z > 0.0)) {
      if (bad) *bad = 1;
      return 0.0;
    }
    return pow(z, -f.k);
  }
  double acc = 0.0;
  for (int j = f.plen - 1; j >= 0; --j) acc = acc * lam + poly[j];
  return acc;
}

static PhiDev to_dev(const gk_phi& p) {
  PhiDev f;
  f.kind = p.kind;
  f.t = p.t;
  f.eps = p.eps;
  f.k = p.k;
  f.plen = p.poly_len;
  return f;
}

// fv[l] = scale_l * phi(theta_l); kind of scale: 0 plain, 1 sqrt (needs phi >= 0)
__global__ void phi_values_kernel(int n, const double* __restrict__ theta, PhiDev f,
                                  const double* __restrict__ poly, double* __restrict__ fv, int use_sqrt,
                                  int* __restrict__ bad) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n) return;
  double v = phi_eval(f, poly, theta[l], bad);
  if (use_sqrt) {
    if (v < 0.0) {
      if (bad) *bad = 2;
      v = 0.0;
    }
    v = sqrt(v);
  }
  fv[l] = v;
}

// U[i, c] = outer * sum_l S[i, l] fv[l] S[row0 + c*rstride, l]
__global__ void phi_apply_kernel(int n, int s, const double* __restrict__ S, int lds,
                                 const double* __restrict__ fv, double* __restrict__ U, int ldu,
                                 double outer) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * s) return;
  const int i = (int)(t / s), c = (int)(t % s);
  const double* si = S + (int64_t)i * lds;
  const double* sc = S + (int64_t)c * lds;
  double acc = 0.0;
  for (int l = 0; l < n; ++l) acc = fma(si[l] * fv[l], sc[l], acc);
  U[(int64_t)i * ldu + c] = outer * acc;
}

void launch_phi_values(int n, const double* theta, const gk_phi& phi, const double* poly_dev, double* fv,
                       bool use_sqrt, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(phi_values_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, theta, to_dev(phi),
                     poly_dev, fv, use_sqrt ? 1 : 0, bad);
  GK_HIP(hipGetLastError());
}

void launch_phi_apply(int n, int s, const double* S, int lds, const double* fv, double* U, int ldu,
                      double outer, hipStream_t st) {
  const int64_t tot = (int64_t)n * s;
  hipLaunchKernelGGL(phi_apply_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, s, S, lds,
                     fv, U, ldu, outer);
  GK_HIP(hipGetLastError());
}

// K[i, j] = sum_l (g_l S[i,l]) (g_l S[j,l]),  g = sqrt(phi(theta))   (i, j < s)
__global__ void kww_gram_kernel(int n, int s, const double* __restrict__ S, int lds,
                                const double* __restrict__ g, double* __restrict__ K) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= s * s) return;
  const int i = t / s, j = t % s;
  const double* si = S + (int64_t)i * lds;
  const double* sj = S + (int64_t)j * lds;
  double acc = 0.0;
  for (int l = 0; l < n; ++l) acc = fma(g[l] * si[l], g[l] * sj[l], acc);
  K[t] = acc;
}

void launch_kww_gram(int n, int s, const double* S, int lds, const double* g, double* K, hipStream_t st) {
  hipLaunchKernelGGL(kww_gram_kernel, dim3((s * s + 255) / 256), dim3(256), 0, st, n, s, S, lds, g, K);
  GK_HIP(hipGetLastError());
}

// ------------------------------------- banded evaluation of spline kernels
// (eps I + H_m)^(-k) F_1 for integer k by block Cholesky of the block
// tridiagonal eps I + H_m (blocks D_j = eps I + H_jj, sub-diagonal B_j):
//   L_00 = chol(D_0); L_{j+1,j} = B_j L_jj^{-T};
//   L_{j+1,j+1} = chol(D_{j+1} - L_{j+1,j} L_{j+1,j}^T)
// then k forward / backward block substitutions.  eps I + H_m is SPD
// because spec(H_m) lies in [0, Lambda] (Theorem 3.1, Cauchy interlacing).
// All blocks are s x s row-major; U is (m s) x s row-major.
__device__ void wg_chol_lower(double* A, int s, int* bad) {
  // in place lower Cholesky A = L L^T (A row-major s x s, full storage)
  const int tid = threadIdx.x;
  for (int j = 0; j < s; ++j) {
    __syncthreads();
    if (tid == 0) {
      const double d = A[j * s + j];
      if (!(d > 0.0)) {
        *bad = 3;
        A[j * s + j] = 1.0;
      } else {
        A[j * s + j] = sqrt(d);
      }
    }
    __syncthreads();
    const double ljj = A[j * s + j];
    for (int r = j + 1 + tid; r < s; r += SB) A[r * s + j] /= ljj;
    __syncthreads();
    const int w = s - j - 1;
    for (int q = tid; q < w * w; q += SB) {
      const int r = j + 1 + q / w, c = j + 1 + q % w;
      if (c <= r) A[r * s + c] -= A[r * s + j] * A[c * s + j];
    }
  }
  __syncthreads();
  for (int q = tid; q < s * s; q += SB) {
    const int r = q / s, c = q % s;
    if (c > r) A[q] = 0.0;
  }
  __syncthreads();
}

// X <- L^{-1} X (trans=0) or L^{-T} X (trans=1); L lower s x s, X s x nr (ld ldx)
__device__ void wg_trsm_lower(const double* L, int s, double* X, int nr, int ldx, int trans) {
  const int tid = threadIdx.x;
  for (int c = tid; c < nr; c += SB) {
    if (!trans) {
      for (int i = 0; i < s; ++i) {
        double acc = X[i * ldx + c];
        for (int l = 0; l < i; ++l) acc -= L[i * s + l] * X[l * ldx + c];
        X[i * ldx + c] = acc / L[i * s + i];
      }
    } else {
      for (int i = s - 1; i >= 0; --i) {
        double acc = X[i * ldx + c];
        for (int l = i + 1; l < s; ++l) acc -= L[l * s + i] * X[l * ldx + c];
        X[i * ldx + c] = acc / L[i * s + i];
      }
    }
  }
  __syncthreads();
}

// C (s x nr) += alpha * op(A) (s x s) * B (s x nr)
__device__ void wg_gemm_acc(const double* A, int s, int ta, const double* B, int ldb, double* C, int ldc,
                            int nr, double alpha) {
  const int tid = threadIdx.x;
  for (int q = tid; q < s * nr; q += SB) {
    const int i = q / nr, c = q % nr;
    double acc = 0.0;
    for (int l = 0; l < s; ++l) acc += (ta ? A[l * s + i] : A[i * s + l]) * B[l * ldb + c];
    C[i * ldc + c] += alpha * acc;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(SB)
banded_spline_kernel(int m, int s, const double* __restrict__ Hd, const double* __restrict__ Bd, double eps,
                     int kpow, double* __restrict__ Ld, double* __restrict__ Lsub, double* __restrict__ U,
                     double* __restrict__ tmp, int* __restrict__ bad) {
  const int tid = threadIdx.x;
  const int ss = s * s;
  // factorisation
  for (int j = 0; j < m; ++j) {
    double* D = Ld + (int64_t)j * ss;
    for (int q = tid; q < ss; q += SB) D[q] = Hd[(int64_t)j * ss + q] + ((q / s == q % s) ? eps : 0.0);
    __syncthreads();
    if (j > 0) {
      // D -= Lsub_{j-1} Lsub_{j-1}^T
      const double* Ls = Lsub + (int64_t)(j - 1) * ss;
      for (int q = tid; q < ss; q += SB) {
        const int r = q / s, c = q % s;
        double acc = 0.0;
        for (int l = 0; l < s; ++l) acc += Ls[r * s + l] * Ls[c * s + l];
        D[q] -= acc;
      }
      __syncthreads();
    }
    wg_chol_lower(D, s, bad);
    if (j + 1 < m) {
      // Lsub_j = B_j L_jj^{-T}  <=>  Lsub_j^T = L_jj^{-1} B_j^T
      double* Ls = Lsub + (int64_t)j * ss;
      const double* B = Bd + (int64_t)j * ss;
      for (int q = tid; q < ss; q += SB) {
        const int r = q / s, c = q % s;
        tmp[q] = B[c * s + r];   // B^T
      }
      __syncthreads();
      wg_trsm_lower(D, s, tmp, s, s, 0);
      for (int q = tid; q < ss; q += SB) {
        const int r = q / s, c = q % s;
        Ls[q] = tmp[c * s + r];
      }
      __syncthreads();
    }
  }
  // right-hand side F_1
  const int64_t ms = (int64_t)m * s;
  for (int64_t q = tid; q < ms * s; q += SB) {
    const int64_t r = q / s;
    const int c = (int)(q % s);
    U[q] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int rep = 0; rep < kpow; ++rep) {
    // forward: Z_j = L_jj^{-1} (Y_j - Lsub_{j-1} Z_{j-1})
    for (int j = 0; j < m; ++j) {
      double* Yj = U + (int64_t)j * ss;
      if (j > 0) wg_gemm_acc(Lsub + (int64_t)(j - 1) * ss, s, 0, U + (int64_t)(j - 1) * ss, s, Yj, s, s, -1.0);
      wg_trsm_lower(Ld + (int64_t)j * ss, s, Yj, s, s, 0);
    }
    // backward: Y_j = L_jj^{-T} (Z_j - Lsub_j^T Y_{j+1})
    for (int j = m - 1; j >= 0; --j) {
      double* Yj = U + (int64_t)j * ss;
      if (j + 1 < m) wg_gemm_acc(Lsub + (int64_t)j * ss, s, 1, U + (int64_t)(j + 1) * ss, s, Yj, s, s, -1.0);
      wg_trsm_lower(Ld + (int64_t)j * ss, s, Yj, s, s, 1);
    }
  }
}

size_t banded_work_elems(int m, int s) { return (size_t)(2 * m + 1) * s * s; }

void launch_banded_spline(int m, int s, const double* Hd, const double* Bd, double eps, int k, double* work,
                          double* U, int* bad, hipStream_t st) {
  const size_t ss = (size_t)s * s;
  kt_begin(KC_BANDED_FACTOR, st);
  hipLaunchKernelGGL(banded_spline_kernel, dim3(1), dim3(SB), 0, st, m, s, Hd, Bd, eps, k, work,
                     work + m * ss, U, work + 2 * m * ss, bad);
  GK_HIP(hipGetLastError());
  kt_end(st, 8.0 * 6 * m * (double)ss, (double)m * ss * s * (3.0 + 4.0 * k));
}

// ------------------------------------------------------------ s x s solve
// (K + gamma I) c = y.  spd: Cholesky; otherwise LU with partial pivoting.
// W is scratch of s*s doubles.  bad = 4 when the system is not solvable: a
// non-finite entry, a Cholesky pivot <= 0, or (LU) a pivot at or below
// piv_rel * max|K + gamma I|: numerically singular at the accuracy K carries
// (the caller passes 2^-40 for K formed in float64, a condition number beyond
// about 1e12; 2^-20 for K gathered from a float32 basis, whose entries carry
// float32 rounding).  The collocation matrices of gbl, sbl and cheb can be
// singular or indefinite at small m (Sec. 8.3).
__global__ void __launch_bounds__(SB)
small_solve_kernel(int s, const double* __restrict__ K, double gamma, const double* __restrict__ y,
                   double* __restrict__ c, double* __restrict__ W, int* __restrict__ piv, int spd,
                   double piv_rel, int* __restrict__ bad) {
  const int tid = threadIdx.x;
  __shared__ int pr_sh;
  __shared__ int fail_sh;
  __shared__ double amax_sh[SB];
  double am = 0.0;
  bool fin = true;
  for (int q = tid; q < s * s; q += SB) {
    const double v = K[q] + ((q / s == q % s) ? gamma : 0.0);
    W[q] = v;
    fin = fin && isfinite(v);
    am = fmax(am, fabs(v));
  }
  for (int q = tid; q < s; q += SB) {
    c[q] = y[q];
    fin = fin && isfinite(y[q]);
  }
  amax_sh[tid] = fin ? am : INFINITY;
  __syncthreads();
  for (int w = SB / 2; w > 0; w >>= 1) {
    if (tid < w) amax_sh[tid] = fmax(amax_sh[tid], amax_sh[tid + w]);
    __syncthreads();
  }
  const double amax = amax_sh[0];
  const double piv_floor = piv_rel * amax;
  if (tid == 0) fail_sh = isfinite(amax) ? 0 : 1;
  __syncthreads();
  if (fail_sh) {
    if (tid == 0) *bad = 4;
    return;
  }
  if (spd) {
    // symmetrise (K is symmetric up to rounding) and factor
    for (int q = tid; q < s * s; q += SB) {
      const int r = q / s, cc = q % s;
      if (cc < r) {
        const double v = 0.5 * (W[r * s + cc] + W[cc * s + r]);
        W[r * s + cc] = v;
        W[cc * s + r] = v;
      }
    }
    int b = 0;
    wg_chol_lower(W, s, &b);
    if (tid == 0 && b) fail_sh = 1;
    __syncthreads();
    if (!fail_sh) {
      wg_trsm_lower(W, s, c, 1, 1, 0);
      wg_trsm_lower(W, s, c, 1, 1, 1);
    }
  } else {
    for (int j = 0; j < s; ++j) {
      if (tid == 0) {
        int p = j;
        double best = fabs(W[j * s + j]);
        for (int r = j + 1; r < s; ++r)
          if (fabs(W[r * s + j]) > best) {
            best = fabs(W[r * s + j]);
            p = r;
          }
        pr_sh = p;
        if (!(best > piv_floor)) fail_sh = 1;
        piv[j] = p;
      }
      __syncthreads();
      if (fail_sh) break;
      const int p = pr_sh;
      if (p != j) {
        for (int q = tid; q < s; q += SB) {
          const double t = W[j * s + q];
          W[j * s + q] = W[p * s + q];
          W[p * s + q] = t;
        }
        if (tid == 0) {
          const double t = c[j];
          c[j] = c[p];
          c[p] = t;
        }
      }
      __syncthreads();
      const double d = W[j * s + j];
      for (int r = j + 1 + tid; r < s; r += SB) W[r * s + j] /= d;
      __syncthreads();
      const int w = s - j - 1;
      for (int q = tid; q < w * w; q += SB) {
        const int r = j + 1 + q / w, cc = j + 1 + q % w;
        W[r * s + cc] -= W[r * s + j] * W[j * s + cc];
      }
      __syncthreads();
    }
    if (!fail_sh && tid == 0) {
      for (int i = 0; i < s; ++i) {
        double acc = c[i];
        for (int l = 0; l < i; ++l) acc -= W[i * s + l] * c[l];
        c[i] = acc;
      }
      for (int i = s - 1; i >= 0; --i) {
        double acc = c[i];
        for (int l = i + 1; l < s; ++l) acc -= W[i * s + l] * c[l];
        c[i] = acc / W[i * s + i];
      }
    }
  }
  __syncthreads();
  if (tid == 0 && fail_sh) *bad = 4;
}

void launch_small_solve(int s, const double* K, double gamma, const double* y, double* c, double* work,
                        int* piv, bool spd, double piv_rel, int* bad, hipStream_t st) {
  hipLaunchKernelGGL(small_solve_kernel, dim3(1), dim3(SB), 0, st, s, K, gamma, y, c, work, piv, spd ? 1 : 0,
                     piv_rel, bad);
  GK_HIP(hipGetLastError());
}

}  // namespace gk

namespace gk {

// ===================================================================
// Small-matrix kernels for block widths up to 64: one workgroup of 256
// threads, s x s operands staged in LDS (row pitch 66 doubles), products on
// the FP64 matrix cores (toolkit in tile64.h).
// ===================================================================

// CholQR factor of a Gram matrix (ld <= 64), 256 threads.
//   pass 1: R1 = chol(G) with clamped pivots, R1inv, diag_out = diag(R1)
//   pass 2: R2 with the combined-diagonal deflation rule, R2inv, and the
//           products Rc = R1inv R2inv and B = R2 R1 (s x s, H_{k+1,k}),
//           and (BT non-null) B^T = H_{k,k+1} zero padded to ld x ld.
__device__ __forceinline__ void
cholqr_blk_body(const double* __restrict__ G, int ld, int s, int pass, const double* __restrict__ diag_prev,
                double thr, double* __restrict__ R, double* __restrict__ Rinv, double* __restrict__ diag_out,
                int* __restrict__ n_defl, const double* __restrict__ R1, const double* __restrict__ R1inv,
                double* __restrict__ Rc, double* __restrict__ Bout, double* __restrict__ BT,
                int* __restrict__ gate) {
  // second pass not needed (decided by the first pass and the projection):
  // counted in the slot five entries after the deflation count
  if (pass == 2 && gate && *gate == 0) {
    if (threadIdx.x == 0 && n_defl) n_defl[5] += 1;
    return;
  }
  __shared__ __align__(16) double A[WS][LP];
  __shared__ __align__(16) double Y[WS][LP];
  __shared__ __align__(16) double S1[WS][LP];
  __shared__ __align__(16) double S2[WS][LP];
  __shared__ double g0[WS], dp[WS], dg[WS], dq[WS];
  __shared__ int clf[WS];
  __shared__ double red[2][ST];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  // the second pass's first-pass factors are loaded up front, their latency
  // hidden behind the factorisation
  double v1[16], v2[16];
  if (pass == 2) {
    fetch64(R1, s, ld, v1);
    fetch64(R1inv, s, ld, v2);
  }
  // deflation and series-path counters of the second pass: read now, written
  // back at the end, so their latency is off the critical path
  const bool rec = pass == 2 && n_defl && tid == 0;
  int nd0 = 0, nd4 = 0;
  if (rec) {
    nd0 = n_defl[0];
    nd4 = n_defl[4];   // counter slot four entries after the deflation count
  }
  stage64(A, G, s, ld);
  for (int q = tid; q < s; q += ST) {
    g0[q] = G[q * ld + q];
    dp[q] = (pass == 2) ? diag_prev[q] : 0.0;
    if (pass == 1 && gate) dq[q] = sqrt(fmax(g0[q], 0.0));
  }
  __syncthreads();
  // Second pass with G = I + E, |E| <= 1e-6 and no column near the deflation
  // threshold: the Cholesky factor of I + E and its inverse follow from the
  // expansion R = I + U + W, R^{-1} = I - U - W + U^2 with U = triu(E) - diag(E)/2
  // and W = -(triu(M) - diag(M)/2), M = U^T U; the neglected terms are O(|E|^3).
  bool fast = false;
  if (pass == 2) {
    double e = 0.0, dmin = INFINITY;
    for (int i = ty; i < s; i += 16)
      for (int c = tx; c < s; c += 16) e = fmax(e, fabs(A[i][c] - (i == c ? 1.0 : 0.0)));
    for (int q = tid; q < s; q += ST) dmin = fmin(dmin, dp[q]);
    // wavefront reductions, then the four wavefront results
    for (int o = 32; o > 0; o >>= 1) {
      e = fmax(e, __shfl_xor(e, o));
      dmin = fmin(dmin, __shfl_xor(dmin, o));
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = e;
      red[1][tid >> 6] = dmin;
    }
    __syncthreads();
    const double emax = fmax(fmax(red[0][0], red[0][1]), fmax(red[0][2], red[0][3]));
    const double dlo = fmin(fmin(red[1][0], red[1][1]), fmin(red[1][2], red[1][3]));
    fast = emax <= 1e-6 && dlo >= 2.0 * thr;
  }
  if (fast) {
    for (int i = ty; i < WS; i += 16)
      for (int c = tx; c < WS; c += 16) {
        double u = 0.0;
        if (i < s && c < s) {
          if (c > i) u = A[i][c];
          else if (c == i) u = 0.5 * (A[i][i] - 1.0);
        }
        S1[i][c] = u;
        S2[c][i] = u;
      }
    __syncthreads();
    double mm[4][4], u2[4][4];
    // U^T U and U U, upper block triangles (only c >= r is read below)
    lds_mm2_upper<KR_LEAD, KR_BAND>(S1, S1, S2, S1, s, mm, u2);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = acc_row(i), c = acc_col(j);
        if (r < s && c < s) {
          const double u = S1[r][c];
          const double w = (c > r) ? -mm[i][j] : (c == r ? -0.5 * mm[i][j] : 0.0);
          const double del = (r == c) ? 1.0 : 0.0;
          const double r2 = (c >= r) ? del + u + w : 0.0;
          const double r2i = (c >= r) ? del - u - w + u2[i][j] : 0.0;
          A[c][r] = r2;    // L = R^T
          // L^{-1} = R^{-T} when R^{-1} is returned; otherwise R^{-1} itself
          // (row-major), the operand of Rc = R1inv R2inv below
          if (R) Y[c][r] = r2i;
          else Y[r][c] = r2i;
          if (r == c) dg[r] = r2;
        }
      }
    __syncthreads();
  } else {
    blk_chol_inv(A, Y, S1, s, pass, g0, dp, thr, dg, nullptr, clf);
  }
  // Pass 1 with a gate: one pass leaves X R^-1 orthonormal to about
  // s u |D R^-1|_2^2 with D = diag(G)^(1/2) (Gram and Cholesky errors are
  // relative to the column norms), and |D R^-1|_2^2 <= |Z|_1 |Z|_inf for
  // Z = L^-1 D (R = L^T, L^-1 in Y).  When that gives 1e-10 or better and no
  // pivot was clamped, the first factor is final: Rc = R^-1, B = R and B^T
  // are written with R and R^-1 below, and the gate tells the second pass
  // (and the Gram launch before it) to do nothing.
  // Thread (q, h): row q and column q of Z over entries 16h .. 16h+15.
  __shared__ int skip_s;
  bool sk = false;
  if (pass == 1 && gate) {
    const int q = tid & 63, h = tid >> 6;
    double rs = 0.0, cs = 0.0;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * h + jj;
      const bool inr = q < s && j <= q, inc = q < s && j < s && j >= q;
      const double zr = Y[q][j], zc = Y[j][q];
      rs += inr ? fabs(zr) * dq[j] : 0.0;
      cs += inc ? fabs(zc) : 0.0;
    }
    red[0][tid] = rs;
    red[1][tid] = cs;
    __syncthreads();
    if (tid < 64) {
      double r = 0.0, c = 0.0;
      for (int hh = 0; hh < 4; ++hh) {
        r += red[0][64 * hh + q];
        c += red[1][64 * hh + q];
      }
      c *= (q < s) ? dq[q] : 0.0;
      double cl = (q < s && (clf[q] != 0 || dg[q] == 0.0)) ? 1.0 : 0.0;
      for (int o = 32; o > 0; o >>= 1) {
        r = fmax(r, __shfl_xor(r, o));
        c = fmax(c, __shfl_xor(c, o));
        cl = fmax(cl, __shfl_xor(cl, o));
      }
      if (tid == 0) {
        const bool skip = cl == 0.0 && r * c * (double)s * 0x1p-53 <= 1e-10;
        *gate = skip ? 0 : 1;
        skip_s = skip ? 1 : 0;
      }
    }
    __syncthreads();
    sk = skip_s != 0;
  }
  // R = L^T, Rinv = Y^T (upper), coalesced stores with zero padding; skipped
  // when the caller passes null (pass 2 returns its factors through Rc and B)
  if (R)
    for (int i = tid >> 6; i < ld; i += ST / 64) {
      const int c = tid & 63;   // ld <= 64: one row per wavefront pass
      if (c < ld) {
        const bool in = i < s && c < s && c >= i;
        const double r = in ? A[c][i] : 0.0, ri = in ? Y[c][i] : 0.0;
        R[i * ld + c] = r;
        Rinv[i * ld + c] = ri;
        if (sk) {
          Rc[i * ld + c] = ri;
          if (BT) BT[i * ld + c] = (i < s && c < s && i >= c) ? A[i][c] : 0.0;   // R^T
          if (i < s && c < s) Bout[i * s + c] = r;
        }
      }
    }
  for (int q = tid; q < ld; q += ST) diag_out[q] = (q < s) ? dg[q] : 0.0;
  if (pass == 1) return;
  if (pass == 2) {
    auto record = [&]() {
      if (rec) {
        int cnt = 0;
        for (int j = 0; j < s; ++j) cnt += (dg[j] == 0.0);
        n_defl[0] = nd0 + cnt;
        n_defl[4] = nd4 + (fast ? 1 : 0);
      }
    };
    put64(S1, v1);
    put64T(S2, v2);
    __syncthreads();
    double acc[4][4];
    if (fast && !R) {
      // B = R2 R1 = L^T S1 and Rc = R1inv R2inv = (R1inv^T)^T (R2inv in Y),
      // interleaved
      double rc[4][4];
      lds_mm2_upper<KR_BAND, KR_BAND>(A, S1, S2, Y, s, acc, rc);   // products of upper triangular factors
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = acc_row(i), c = acc_col(j);
          if (r < s && c < s) Bout[r * s + c] = acc[i][j];
          if (BT && r < ld && c < ld) BT[c * ld + r] = (r < s && c < s) ? acc[i][j] : 0.0;
          if (r < ld && c < ld) Rc[r * ld + c] = (r < s && c < s) ? rc[i][j] : 0.0;
        }
      record();
      return;
    }
    // B = R2 * R1 = L^T * S1
    lds_mm<true, false>(A, S1, s, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = acc_row(i), c = acc_col(j);
        if (r < s && c < s) Bout[r * s + c] = acc[i][j];
        if (BT && r < ld && c < ld) BT[c * ld + r] = (r < s && c < s) ? acc[i][j] : 0.0;
      }
    __syncthreads();
    // S1 <- R2inv = Y^T; Rc = R1inv * R2inv = (R1inv^T)^T R2inv
    for (int i = ty; i < WS; i += 16)
      for (int c = tx; c < WS; c += 16) S1[c][i] = (i < s && c < s) ? Y[i][c] : 0.0;
    __syncthreads();
    lds_mm<true, false>(S2, S1, s, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = acc_row(i), c = acc_col(j);
        if (r < ld && c < ld) Rc[r * ld + c] = (r < s && c < s) ? acc[i][j] : 0.0;
      }
    record();
  }
}

__global__ void __launch_bounds__(ST)
cholqr_blk_kernel(const double* __restrict__ G, int ld, int s, int pass, const double* __restrict__ diag_prev,
                  double thr, double* __restrict__ R, double* __restrict__ Rinv, double* __restrict__ diag_out,
                  int* __restrict__ n_defl, const double* __restrict__ R1, const double* __restrict__ R1inv,
                  double* __restrict__ Rc, double* __restrict__ Bout, double* __restrict__ BT) {
  cholqr_blk_body(G, ld, s, pass, diag_prev, thr, R, Rinv, diag_out, n_defl, R1, R1inv, Rc, Bout, BT, nullptr);
}

// A batch of independent factorisations, one workgroup each (the serving
// loop advances several requests in lockstep); count <= kCholqrBatch.
struct CholqrBatch {
  CholqrArgs a[kCholqrBatch];
};
__global__ void __launch_bounds__(ST) cholqr_blk_batch_kernel(CholqrBatch b) {
  const CholqrArgs& a = b.a[blockIdx.x];
  cholqr_blk_body(a.G, a.ld, a.s, a.pass, a.diag_prev, a.thr, a.R, a.Rinv, a.diag_out, a.n_defl, a.R1, a.R1inv,
                  a.Rc, a.Bout, a.BT, a.gate);
}

// 64 x 16 column slices of a product (the orthogonality estimate below).
constexpr int SLP = 17;   // LDS pitch of a 64 x 16 slice

// acc[a] = (A^T B)[acc_row(a)][lane & 15] for a 16-column slice B, summed
// over the first s rows (NT steps of four, two accumulator chains).
template <int NT>
__device__ __forceinline__ void mm_slice_steps(const double (*A)[LP], const double (*B)[SLP], int s, dv4& d0,
                                               dv4& d1) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int kk = 4 * t + lk;
    const bool in = kk < s;
    const double a0 = A[kk][16 * w + li], b0 = B[kk][li];
    if (t & 1) d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? a0 : 0.0, in ? b0 : 0.0, d1, 0, 0, 0);
    else d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(in ? a0 : 0.0, in ? b0 : 0.0, d0, 0, 0, 0);
  }
}
__device__ __forceinline__ void lds_mm_slice(const double (*A)[LP], const double (*B)[SLP], int s, double (&acc)[4]) {
  dv4 d0 = dv4{0.0, 0.0, 0.0, 0.0}, d1 = dv4{0.0, 0.0, 0.0, 0.0};
  if (s > 48) mm_slice_steps<16>(A, B, s, d0, d1);
  else if (s > 32) mm_slice_steps<12>(A, B, s, d0, d1);
  else if (s > 16) mm_slice_steps<8>(A, B, s, d0, d1);
  else mm_slice_steps<4>(A, B, s, d0, d1);
#pragma unroll
  for (int a = 0; a < 4; ++a) acc[a] = d0[a] + d1[a];
}

// ---------------------------------------------------------------------
// Orthogonality estimate for partial reorthogonalisation (block form of the
// omega recurrence).  With W_{k,j} = V_k^T V_j and the block Lanczos relation
// L V_j = V_{j+1} B_j + V_j H_j + V_{j-1} B_{j-1}^T + F_j (B_j = H_{j+1,j}),
// symmetry of L gives
//   B_k^T W_{k+1,j} = W_{k,j+1} B_j + W_{k,j} H_j - H_k W_{k,j}
//                     + W_{k,j-1} B_{j-1}^T - B_{k-1} W_{k-1,j} + (rounding),
// so W_{k+1,j} = B_k^{-T} (...).  B_k^{-1} is taken as Rc = R1^{-1} of the
// first CholQR pass (B_k = R2 R1 with R2 = I + O(u)), so that the decision
// comes before the block is normalised.  The rounding
// term is modelled pessimistically by +-nu added in the direction of each
// entry.  Every product is column-separable, so the output is split into
// 16-column slices: one workgroup per (j <= k-2, slice), each forming its
// slice of the right-hand side and of W_{k+1,j} from full 64 x 64 left
// operands and 64 x 16 right operands.  W_{k+1,k-1} and W_{k+1,k} are kept at
// a floor because the new block is orthogonalised against V_{k-1}, V_k.
__device__ __forceinline__ void fetch_slice(const double* __restrict__ src, int s, int c0, bool tr,
                                            double (&v)[4]) {
  const int c = c0 + (threadIdx.x & 15);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = (threadIdx.x + ST * e) >> 4;
    const bool in = src && r < s && c < s;
    v[e] = in ? src[tr ? c * s + r : r * s + c] : 0.0;
  }
}
__device__ __forceinline__ void put_slice(double (*D)[SLP], const double (&v)[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) D[(threadIdx.x + ST * e) >> 4][threadIdx.x & 15] = v[e];
}

__global__ void __launch_bounds__(ST)
omega_kernel(int k, int s, int ld, const double* __restrict__ Wk, const double* __restrict__ Wkm1,
             double* __restrict__ Wk1, const double* __restrict__ Hd, const double* __restrict__ Bd,
             const double* __restrict__ Rc, double nu, double* __restrict__ est_part) {
  __shared__ __align__(16) double SL[3][WS][LP];   // left operands
  __shared__ double SR[3][WS][SLP];                // right operand slices
  __shared__ double red[ST / 64];
  const int j = blockIdx.x, q = blockIdx.y, c0 = 16 * q;
  const int tid = threadIdx.x;
  const int64_t ss = (int64_t)s * s;
  double tot[4], acc[4];
  // Left operands are staged so that lds_mm_slice (A^T B) forms M B:
  // transposed for W and B_{k-1}, as they are for the symmetric H_k.
  double l0[16], l1[16], l2[16], r0[4], r1[4], r2[4];
  // W_{k,j+1} B_j + W_{k,j} H_j - H_k W_{k,j}
  fetch64(Wk + (j + 1) * ss, s, s, l0);
  fetch64(Wk + j * ss, s, s, l1);
  fetch64(Hd + (int64_t)k * ss, s, s, l2);
  fetch_slice(Bd + j * ss, s, c0, false, r0);
  fetch_slice(Hd + j * ss, s, c0, false, r1);
  fetch_slice(Wk + j * ss, s, c0, false, r2);
  put64T(SL[0], l0); put64T(SL[1], l1); put64(SL[2], l2);
  put_slice(SR[0], r0); put_slice(SR[1], r1); put_slice(SR[2], r2);
  __syncthreads();
  // W_{k,j-1} B_{j-1}^T - B_{k-1} W_{k-1,j}: loads in flight during the products
  fetch64(j >= 1 ? Wk + (j - 1) * ss : nullptr, s, s, l0);
  fetch64(Bd + (int64_t)(k - 1) * ss, s, s, l1);
  fetch_slice(j >= 1 ? Bd + (j - 1) * ss : nullptr, s, c0, true, r0);
  fetch_slice(Wkm1 + j * ss, s, c0, false, r1);
  lds_mm_slice(SL[0], SR[0], s, tot);
  lds_mm_slice(SL[1], SR[1], s, acc);
#pragma unroll
  for (int a = 0; a < 4; ++a) tot[a] += acc[a];
  lds_mm_slice(SL[2], SR[2], s, acc);
#pragma unroll
  for (int a = 0; a < 4; ++a) tot[a] -= acc[a];
  __syncthreads();
  put64T(SL[0], l0); put64T(SL[1], l1);
  put_slice(SR[0], r0); put_slice(SR[1], r1);
  __syncthreads();
  fetch64(Rc, s, ld, l2);
  if (j >= 1) {
    lds_mm_slice(SL[0], SR[0], s, acc);
#pragma unroll
    for (int a = 0; a < 4; ++a) tot[a] += acc[a];
  }
  lds_mm_slice(SL[1], SR[1], s, acc);
  // W_{k+1,j} = Rc^T (RHS + rounding model)
  const int w = tid >> 6, li = tid & 15, lk = (tid & 63) >> 4;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = 16 * w + 4 * a + lk, c = c0 + li;
    const double t = tot[a] - acc[a];
    SR[2][r][li] = (r < s && c < s) ? t + copysign(nu, t) : 0.0;
  }
  put64(SL[2], l2);
  __syncthreads();
  lds_mm_slice(SL[2], SR[2], s, acc);
  double mx = 0.0;
  double* out = Wk1 + j * ss;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int r = 16 * w + 4 * a + lk, c = c0 + li;
    if (r < s && c < s) {
      out[r * s + c] = acc[a];
      mx = fmax(mx, fabs(acc[a]));
    }
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((tid & 63) == 0) red[w] = mx;
  __syncthreads();
  if (tid == 0) est_part[j * gridDim.y + q] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// The reorthogonalisation decision of step k as a launch of its own (when no
// archive projection follows to take it): one workgroup per block of
// estimates to reset.
__global__ void __launch_bounds__(ST) omega_decide_kernel(OmegaDecide d) {
  __shared__ double red[ST / 64];
  omega_decide(d, blockIdx.x, gridDim.x, red);
}


}  // namespace gk


namespace gk {

bool small_wave_ok(int ld) { return ld <= WS; }

int omega_est_per_block(int s) {
  const int nq = (s + WS - 1) / WS;
  return s > WS ? nq * nq : (s + 15) / 16;
}

void launch_cholqr_reg(const double* G, int ld, int s, int pass, const double* diag_prev, double thr, double* R,
                       double* Rinv, double* diag_out, int* n_defl, const double* R1, const double* R1inv, double* Rc,
                       double* Bout, double* BT, hipStream_t st) {
  kt_begin(KC_CHOLQR, st);
  hipLaunchKernelGGL(cholqr_blk_kernel, dim3(1), dim3(ST), 0, st, G, ld, s, pass, diag_prev, thr, R, Rinv, diag_out,
                     n_defl, R1, R1inv, Rc, Bout, BT);
  GK_HIP(hipGetLastError());
  kt_end(st, 8.0 * 4 * ld * ld, (double)s * s * s);
}

void launch_cholqr_reg_batched(const CholqrArgs* a, int count, hipStream_t st) {
  for (int c0 = 0; c0 < count; c0 += kCholqrBatch) {
    const int nb = std::min(kCholqrBatch, count - c0);
    CholqrBatch b{};
    double bytes = 0, flops = 0;
    for (int i = 0; i < nb; ++i) {
      b.a[i] = a[c0 + i];
      bytes += 8.0 * 4 * a[c0 + i].ld * a[c0 + i].ld;
      flops += (double)a[c0 + i].s * a[c0 + i].s * a[c0 + i].s;
    }
    kt_begin(KC_CHOLQR, st);
    hipLaunchKernelGGL(cholqr_blk_batch_kernel, dim3(nb), dim3(ST), 0, st, b);
    GK_HIP(hipGetLastError());
    kt_end(st, bytes, flops);
  }
}

void launch_omega(int k, int s, int ld, const double* Wk, const double* Wkm1, double* Wk1, const double* Hd,
                  const double* Bd, const double* Rc, double nu, double tau, double floor_re, double floor_loc,
                  double* est_part, int* fr, int* forced, double* est_out, int* nre, double* rhs_wide,
                  hipStream_t st, OmegaDecide* defer, int* gate) {
  const int nj = k - 1;   // recurrence for j <= k-2
  if (nj > 0) {
    if (s > WS) {
      GK_REQUIRE(rhs_wide, GK_EINVAL, "wide orthogonality estimate needs its scratch");
      launch_omega_wide(k, s, ld, Wk, Wkm1, Wk1, Hd, Bd, Rc, nu, rhs_wide, est_part, st);
    } else {
      kt_begin(KC_OMEGA, st);
      hipLaunchKernelGGL(omega_kernel, dim3(nj, (s + 15) / 16), dim3(ST), 0, st, k, s, ld, Wk, Wkm1, Wk1, Hd, Bd,
                         Rc, nu, est_part);
      GK_HIP(hipGetLastError());
      kt_end(st, 8.0 * 10 * nj * (double)s * s, 12.0 * nj * (double)s * s * s);
    }
  }
  const int ne = nj > 0 ? nj * omega_est_per_block(s) : 0;
  const OmegaDecide d{k, s, nj > 0 ? nj : 0, ne, est_part, tau, floor_re, floor_loc, Wk1, fr, forced, est_out, nre,
                      gate};
  if (defer) {
    *defer = d;
    return;
  }
  // one workgroup per block of estimates to reset (at most 64)
  const int dgrid = nj < 1 ? 1 : (nj < 64 ? nj : 64);
  hipLaunchKernelGGL(omega_decide_kernel, dim3(dgrid), dim3(ST), 0, st, d);
  GK_HIP(hipGetLastError());
}

}  // namespace gk

namespace gk {

// ---------------------------------------------------------------------
// phi(H_m) F_1 for the diffusion kernel without a spectral decomposition:
// exp(-t lam) on [0, Lambda] (spec(H_m) lies there, Theorem 3.1) is expanded
// in Chebyshev polynomials of x = 1 - 2 lam / Lambda and the series is applied
// to F_1 with the three-term recurrence, each term one block tridiagonal
// product.  The degree is chosen past the point where the coefficients
// (2 e^{-z} I_k(z), z = t Lambda / 2) fall below 1e-17.
// out = alpha * (H Y) + beta * Y + gamma * Yp ;  acc += coef[kk] * out
// (H Y)_j = H_{j,j-1} Y_{j-1} + H_jj Y_j + H_{j,j+1} Y_{j+1}, H_{j,j-1} = B_{j-1},
// H_{j,j+1} = B_j^T.  Blocks up to 512 wide run on 64 x 64 tiles
// (launch_btd_cheb_tile); wider ones with one thread per entry (j, r, c) of
// the m s x s output here.
__global__ void btd_cheb_step_kernel(int m, int s, const double* __restrict__ Hd, const double* __restrict__ Bd,
                                     const double* __restrict__ Y, const double* __restrict__ Yp,
                                     double* __restrict__ out, double alpha, double beta, double gamma,
                                     double* __restrict__ acc, const double* __restrict__ coef, int kk) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ss = (int64_t)s * s;
  if (t >= (int64_t)m * ss) return;
  const int j = (int)(t / ss);
  const int r = (int)((t / s) % s), c = (int)(t % s);
  double hy = 0.0;
  const double* Hj = Hd + j * ss + (int64_t)r * s;
  const double* Yj = Y + j * ss + c;
  for (int l = 0; l < s; ++l) hy = fma(Hj[l], Yj[(int64_t)l * s], hy);
  if (j > 0) {
    const double* B = Bd + (j - 1) * ss + (int64_t)r * s;     // B_{j-1}[r][l]
    const double* Ym = Y + (j - 1) * ss + c;
    for (int l = 0; l < s; ++l) hy = fma(B[l], Ym[(int64_t)l * s], hy);
  }
  if (j + 1 < m) {
    const double* B = Bd + j * ss + r;                        // B_j^T[r][l] = B_j[l][r]
    const double* Yn = Y + (j + 1) * ss + c;
    for (int l = 0; l < s; ++l) hy = fma(B[(int64_t)l * s], Yn[(int64_t)l * s], hy);
  }
  double v = alpha * hy + beta * Y[t];
  if (Yp) v += gamma * Yp[t];
  out[t] = v;
  acc[t] += coef[kk] * v;
}

__global__ void f1_init_kernel(int64_t rows, int s, double* __restrict__ Y, double* __restrict__ acc,
                               const double* __restrict__ coef) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * s) return;
  const double v = ((t / s) == (t % s)) ? 1.0 : 0.0;
  Y[t] = v;
  acc[t] = coef[0] * v;
}

// The coefficients 2 e^{-z} I_k(z) fall below 1e-17 before k = sqrt(80 z) + 24
// for every z (they decay like exp(-k^2 / (2 z)) once k exceeds sqrt(z));
// sqrt(90 z) + 24 keeps a margin.
__global__ void cheb_fvals_kernel(int deg, double Lam, int kind, double eps, double kexp,
                                  const double* __restrict__ poly, int plen, double* __restrict__ f) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > deg) return;
  const double lam = 0.5 * Lam * (1.0 - cospi((double)j / deg));
  double v;
  if (kind == GK_PHI_SPLINE) {
    v = pow(eps + lam, -kexp);
  } else {
    v = 0.0;
    for (int q = plen - 1; q >= 0; --q) v = v * lam + poly[q];
  }
  f[j] = v;
}
// a_k = (2/deg) sum_j'' f_j cos(pi j k / deg), a_0 and a_deg halved; the
// angle j k / deg is reduced modulo 2 in integers before cospi
__global__ void cheb_dct_kernel(int deg, const double* __restrict__ f, double* __restrict__ a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > deg) return;
  const int64_t two = 2 * (int64_t)deg;
  double acc = 0.0;
  for (int j = 0; j <= deg; ++j) {
    const int64_t r = ((int64_t)j * k) % two;
    const double w = (j == 0 || j == deg) ? 0.5 : 1.0;
    acc += w * f[j] * cospi((double)r / deg);
  }
  acc *= 2.0 / deg;
  if (k == 0 || k == deg) acc *= 0.5;
  a[k] = acc;
}
void launch_cheb_coef_phi(int deg, double Lam, const gk_phi& phi, const double* poly_dev, double* fv, double* a,
                          hipStream_t st) {
  const unsigned nb = (unsigned)((deg + 1 + 255) / 256);
  hipLaunchKernelGGL(cheb_fvals_kernel, dim3(nb), dim3(256), 0, st, deg, Lam, (int)phi.kind, phi.eps, phi.k,
                     poly_dev, phi.poly_len, fv);
  GK_HIP(hipGetLastError());
  hipLaunchKernelGGL(cheb_dct_kernel, dim3(nb), dim3(256), 0, st, deg, (const double*)fv, a);
  GK_HIP(hipGetLastError());
}

int cheb_diffusion_degree(double t, double Lam) {
  const double z = 0.5 * t * Lam;
  const double k = sqrt(90.0 * z) + 24.0;
  return (int)fmin(4096.0, ceil(k));
}

void launch_cheb_series(int m, int s, const double* Hd, const double* Bd, double t, double Lam, int deg,
                           const double* coef, double* Y0, double* Y1, double* Y2, double* U, hipStream_t st) {
  const int64_t tot = (int64_t)m * s * s;
  const unsigned nb = (unsigned)((tot + 255) / 256);
  hipLaunchKernelGGL(f1_init_kernel, dim3(nb), dim3(256), 0, st, (int64_t)m * s, s, Y0, U, coef);
  GK_HIP(hipGetLastError());
  if (deg < 1) return;
  double* Y[3] = {Y0, Y1, Y2};
  // T_1: out = Y - (2/Lam) H Y
  const double cb = 8.0 * 6 * (double)m * s * s, cf = 2.0 * 3 * (double)m * s * s * s;
  auto step = [&](const double* Yc, const double* Yp, double* out, double a, double b, double g, int kk) {
    kt_begin(KC_CHEB, st);
    if (s <= 512) {
      launch_btd_cheb_tile(m, s, Hd, Bd, Yc, Yp, out, a, b, g, U, coef, kk, st);
    } else {
      hipLaunchKernelGGL(btd_cheb_step_kernel, dim3(nb), dim3(256), 0, st, m, s, Hd, Bd, Yc, Yp, out, a, b, g, U,
                         coef, kk);
      GK_HIP(hipGetLastError());
    }
    kt_end(st, cb, cf);
  };
  step(Y[0], nullptr, Y[1], -2.0 / Lam, 1.0, 0.0, 1);
  for (int k = 1; k < deg; ++k) step(Y[k % 3], Y[(k - 1) % 3], Y[(k + 1) % 3], -4.0 / Lam, 2.0, -1.0, k + 1);
}

}  // namespace gk
