// Krylov drivers: classical block Lanczos (Alg. 1), global block Lanczos
// (Alg. 2), sequential Lanczos (Sec. 3.3), Chebyshev and squared Chebyshev
// (Sec. 3.4), followed by phi of the projected matrix, assembly of the kernel
// columns and the kernel RLS machine (Sec. 2.3, Alg. 3).
//
// Every step is enqueued on one stream; all data-dependent decisions
// (deflation, breakdown) are taken on the device, so the host never waits
// inside the iteration.
//
// Precision paths
//   GK_FP64  : all blocks float64; each new block is orthogonalised against
//              its two predecessors and then twice against the whole basis.
//   GK_MIXED : the three-term recurrence (current and previous block, X) and
//              all small factors stay float64, the operator uses float32
//              weights and the basis is archived in float32 for the
//              reorthogonalisation against older blocks and the final
//              assembly.  Rounding the recurrence vectors themselves would
//              perturb the Krylov space at first order (the unconverged Ritz
//              values move), which the near-singular spline kernels amplify
//              beyond a 1e-5 budget; the archive copy only enters through
//              small projection coefficients and the final linear
//              combination.
#include <cmath>
#include <memory>

#include "gk_internal.h"

namespace gk {

// Gram partials of the panel passes and of the fused 64-wide product + Gram
static size_t pass_scratch_elems(int64_t n, int ld) {
  return std::max(panel_scratch_elems(n, ld), ld == 64 ? spmm_gram64_scratch_elems(n) : (size_t)0);
}

// ------------------------------------------------------------ glue kernels
// Upad[b*ld + r, c] = U[b*s + r, c] (r < s), zero for padding rows
__global__ void pad_rows_kernel(int nb, int s, int ld, const double* __restrict__ U, double* __restrict__ Up) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (int64_t)nb * ld * s;
  if (t >= tot) return;
  const int c = (int)(t % s);
  const int64_t row = t / s;
  const int b = (int)(row / ld), r = (int)(row % ld);
  Up[t] = (r < s) ? U[((int64_t)b * s + r) * s + c] : 0.0;
}

// out (ld x ld) = block k of U (m*s x s), zero padded: out[r, c] = U[k*s + r, c]
__global__ void pad_block_kernel(int k, int s, int ld, const double* __restrict__ U, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ld * ld) return;
  const int r = t / ld, c = t % ld;
  out[t] = (r < s && c < s) ? U[((int64_t)k * s + r) * s + c] : 0.0;
}

// out (ld x s) = [I_s; 0]
__global__ void ident_rows_kernel(int s, int ld, double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ld * s) return;
  out[t] = (t / s == t % s) ? 1.0 : 0.0;
}

// gbl: coef_j = sum_{c<s} cd[j*ld + c]; D[j*ld + c] = coef_j (c < ld);
// optionally store coef of the last block into alpha_out
__global__ void frob_coef_kernel(int nb, int s, int ld, const double* __restrict__ cd, double* __restrict__ D,
                                 double* __restrict__ alpha_out, const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  const int j = blockIdx.x;
  __shared__ double red[256];
  double v = 0.0;
  for (int c = threadIdx.x; c < s; c += 256) v += cd[j * ld + c];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double coef = red[0];
  for (int c = threadIdx.x; c < ld; c += 256) D[j * ld + c] = (c < s) ? coef : 0.0;
  if (threadIdx.x == 0 && alpha_out && j == nb - 1) *alpha_out = coef;
}

// gbl norm: beta = ||X||_F from column sums of squares; scale = 1/beta or 0
__global__ void frob_norm_kernel(int s, int ld, const double* __restrict__ cd, double thr,
                                 double* __restrict__ beta_out, double* __restrict__ scale,
                                 double* __restrict__ resid) {
  __shared__ double red[256];
  double v = 0.0;
  for (int c = threadIdx.x; c < s; c += 256) v += cd[c];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double b = sqrt(red[0]);
  const double keep = (b >= thr) ? b : 0.0;
  if (threadIdx.x == 0) {
    if (beta_out) *beta_out = keep;
    if (resid) *resid = b;
  }
  for (int c = threadIdx.x; c < ld; c += 256) scale[c] = (keep > 0.0 && c < s) ? 1.0 / keep : 0.0;
}

// sbl: per-column norms beta_c = sqrt(cd[c]); scale_c = 1/beta_c or 0
__global__ void col_norm_kernel(int s, int ld, const double* __restrict__ cd, double thr,
                                double* __restrict__ beta_out, double* __restrict__ scale,
                                double* __restrict__ resid) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ld) return;
  double b = (c < s) ? sqrt(cd[c]) : 0.0;
  const double keep = (b >= thr) ? b : 0.0;
  if (c < s && beta_out) beta_out[c] = keep;
  if (c < s && resid) resid[c] = b;
  scale[c] = (keep > 0.0) ? 1.0 / keep : 0.0;
}

// Orthogonality estimate of the scalar-coefficient Lanczos variants (gbl:
// one recurrence in the Frobenius inner product; sbl: one per column), the
// omega recurrence of partial reorthogonalisation (Simon 1984) on the
// tridiagonal coefficients of Alg. 2 / Sec. 3.3:
//   b_k w_{k+1,j} = b_j w_{k,j+1} + (a_j - a_k) w_{k,j} + b_{j-1} w_{k,j-1}
//                   - b_{k-1} w_{k-1,j} +- nu,
// with w_{k,j} = q_k . q_j, a_j = alpha, b_j = beta (coupling q_j, q_{j+1})
// and b_k the norm of X before it is normalised (from cd, its column sums
// of squares).  The two local neighbours sit at floor_loc (they are
// orthogonalised explicitly in float64).  Decision as for the block
// estimate: project X against the archive when max_j |w_{k+1,j}| > tau, and
// once more on the next step; after a projection the estimates restart at
// floor_re.  One workgroup; nw recurrences (1 for gbl, s for sbl).
__global__ void __launch_bounds__(1024)
omega_scalar_kernel(int k, int nw, int s, int global, const double* __restrict__ alpha,
                    const double* __restrict__ beta, const double* __restrict__ cd, double thr, double nu,
                    double tau, double floor_re, double floor_loc, const double* __restrict__ Okm1,
                    const double* __restrict__ Ok, double* __restrict__ Ok1, int* __restrict__ fr,
                    int* __restrict__ forced, double* __restrict__ est_out, int* __restrict__ nre) {
  __shared__ double bk[1024];
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  if (global) {
    double v = 0.0;
    for (int c = tid; c < s; c += 1024) v += cd[c];
    red[tid] = v;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) bk[0] = sqrt(red[0]);
  } else {
    for (int c = tid; c < nw; c += 1024) bk[c] = sqrt(cd[c]);
  }
  __syncthreads();
  const int64_t tot = (int64_t)(k - 1 > 0 ? k - 1 : 0) * nw;   // j = 0..k-2
  double mx = 0.0;
  for (int64_t q = tid; q < tot; q += 1024) {
    const int j = (int)(q / nw), c = (int)(q % nw);
    const double b = bk[c];
    double w = 0.0;
    if (b >= thr) {
      const int64_t jc = (int64_t)j * nw + c;
      w = beta[jc] * Ok[jc + nw] + (alpha[jc] - alpha[(int64_t)k * nw + c]) * Ok[jc];
      if (j > 0) w += beta[jc - nw] * Ok[jc - nw];
      w -= beta[(int64_t)(k - 1) * nw + c] * Okm1[jc];
      w = (w + copysign(nu, w)) / b;
    }
    Ok1[(int64_t)j * nw + c] = w;
    mx = fmax(mx, fabs(w));
  }
  red[tid] = mx;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double e = red[0];
  const int f = forced[k];
  const bool go = e > tau || f;
  if (tid == 0) {
    fr[k] = go ? 1 : 0;
    forced[k + 1] = (go && !f) ? 1 : 0;
    if (go) *nre += 1;
    *est_out = fmax(*est_out, go ? floor_re : e);
  }
  if (go)
    for (int64_t q = tid; q < tot; q += 1024) {
      const int c = (int)(q % nw);
      Ok1[q] = bk[c] >= thr ? floor_re : 0.0;
    }
  for (int q = tid; q < 2 * nw; q += 1024) {
    const int j = k - 1 + q / nw, c = q % nw;
    if (j >= 0) Ok1[(int64_t)j * nw + c] = bk[c] >= thr ? floor_loc : 0.0;
  }
}

// dense symmetric tridiagonal matrices from (alpha, beta): batch b uses
// alpha[k*astride + b], beta[k*astride + b]
__global__ void tridiag_dense_kernel(int m, int batch, int astride, const double* __restrict__ alpha,
                                     const double* __restrict__ beta, double* __restrict__ T) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)m * m;
  if (t >= per * batch) return;
  const int b = (int)(t / per);
  const int r = (int)((t % per) / m), c = (int)(t % m);
  double v = 0.0;
  if (r == c) v = alpha[(int64_t)r * astride + b];
  else if (r == c + 1) v = beta[(int64_t)c * astride + b];
  else if (c == r + 1) v = beta[(int64_t)r * astride + b];
  T[t] = v;
}

// sequential: D[k*ld + c] = outer * sum_l S_c[k, l] fv_c[l] S_c[0, l]
__global__ void seq_coef_kernel(int m, int s, int ld, const double* __restrict__ S,
                                const double* __restrict__ fv, double* __restrict__ D) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * ld) return;
  const int k = t / ld, c = t % ld;
  if (c >= s) {
    D[t] = 0.0;
    return;
  }
  const double* Sc = S + (int64_t)c * m * m;
  const double* fc = fv + (int64_t)c * m;
  double acc = 0.0;
  for (int l = 0; l < m; ++l) acc = fma(Sc[k * m + l] * fc[l], Sc[l], acc);
  D[t] = acc;
}

// gbl: D[k*ld + c] = u[k] (c < s)
__global__ void bcast_coef_kernel(int m, int s, int ld, const double* __restrict__ u, double* __restrict__ D) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * ld) return;
  const int k = t / ld, c = t % ld;
  D[t] = (c < s) ? u[k] : 0.0;
}

// z[k*ld + c] = D[k*ld + c] * coef[c]
__global__ void zdiag_kernel(int m, int s, int ld, const double* __restrict__ D, const double* __restrict__ coef,
                             double* __restrict__ z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m * ld) return;
  const int c = t % ld;
  z[t] = (c < s) ? D[t] * coef[c] : 0.0;
}

// Chebyshev-Lobatto coefficients of phi (or sqrt(phi)) of degree deg on
// [0, Lam]: a_k = (2/deg) sum_j'' f(lam_j) cos(pi j k / deg), lam_j =
// (Lam/2)(1 - cos(pi j / deg)); a_0 and a_deg halved (Sec. 3.4, standard
// Lobatto interpolant).
__global__ void cheb_coef_kernel(int deg, double Lam, int kind, double t, double eps, double kexp,
                                 const double* __restrict__ poly, int plen, int use_sqrt,
                                 double* __restrict__ a, int* __restrict__ bad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > deg) return;
  const double pi = 3.14159265358979323846;
  double acc = 0.0;
  for (int j = 0; j <= deg; ++j) {
    const double lam = 0.5 * Lam * (1.0 - cos(pi * j / deg));
    double f;
    if (kind == GK_PHI_DIFFUSION) {
      f = exp(-t * lam);
    } else if (kind == GK_PHI_SPLINE) {
      f = pow(eps + lam, -kexp);
    } else {
      f = 0.0;
      for (int q = plen - 1; q >= 0; --q) f = f * lam + poly[q];
    }
    if (use_sqrt) {
      if (f < 0.0) {
        *bad = 2;
        f = 0.0;
      }
      f = sqrt(f);
    }
    const double w = (j == 0 || j == deg) ? 0.5 : 1.0;
    acc += w * f * cos(pi * (double)j * (double)k / deg);
  }
  acc *= 2.0 / deg;
  if (k == 0 || k == deg) acc *= 0.5;
  a[k] = acc;
}

// out = sqrt(sum_{c<s} G[c, c])
__global__ void trace_sqrt_kernel(const double* __restrict__ G, int ld, int s, double* __restrict__ out) {
  __shared__ double red[256];
  double v = 0.0;
  for (int c = threadIdx.x; c < s; c += 256) v += G[(int64_t)c * ld + c];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

// acc = a0 * Y
__global__ void scale_copy_kernel(int64_t cnt, const double* __restrict__ a0, const double* __restrict__ Y,
                                  double* __restrict__ acc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) acc[i] = (*a0) * Y[i];
}

// column-major copy of a row-major s x s matrix
__global__ void transpose_kernel(int s, const double* __restrict__ A, double* __restrict__ B) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= s * s) return;
  const int r = t / s, c = t % s;
  B[(int64_t)c * s + r] = A[t];
}

__global__ void fill_kernel(double* __restrict__ p, int cnt, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = v;
}

// samples given in caller numbering -> device numbering
__global__ void map_samples_kernel(int s, const int64_t* __restrict__ in, const int64_t* __restrict__ iperm,
                                   int64_t* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < s) out[j] = iperm ? iperm[in[j]] : in[j];
}

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------ job state
struct Job {
  gk_graph* g = nullptr;
  int s = 0, ld = 0, m = 0, variant = 0, precision = 0;
  uint32_t flags = 0;
  gk_phi phi{};
  hipStream_t st = nullptr;
  Arena ar;
  PhaseTimer tm;
  int64_t* samp = nullptr;        // device numbering
  int* dflags = nullptr;          // [0] phi bad, [1] deflations, [2] solve bad, [3] reorth count,
                                  // [5] second CholQR passes by series expansion, [6] second
                                  // CholQR passes left out
  double* dscal = nullptr;        // [0] residual norm
  double* poly_dev = nullptr;
  bool mixed() const { return precision == GK_MIXED; }
  // Full reorthogonalisation every step: always for GK_FP64, on request for
  // GK_MIXED, and for GK_MIXED cbl blocks wider than 512 (the block
  // orthogonality estimate of partial reorthogonalisation is built for widths
  // up to 512).  GK_MIXED gbl / sbl use scalar estimates at any width.
  bool full_reorth() const {
    if (flags & GK_TWO_PASS) return false;   // no stored basis to project against
    return !mixed() || (flags & GK_FULL_REORTH) || (variant == GK_CBL && !(small_wave_ok(ld) || wide_ok(ld)));
  }
  double thr() const { return 1e-12 * g->lambda_max; }
  // result of the Krylov stage
  BlockList arch;                 // archived basis (nb blocks)
  double* Upad = nullptr;         // dense coefficients (nb*ld x s) or null
  double* D = nullptr;            // diagonal coefficients (nb*ld) or null
  double* K = nullptr;            // s x s sampled block
  bool spd = false;               // K symmetric positive definite by construction
  int phi_method = 0;
};

static void phi_check(const gk_phi& p) {
  if (p.kind == GK_PHI_DIFFUSION) {
    GK_REQUIRE(std::isfinite(p.t) && p.t >= 0.0, GK_EINVAL, "diffusion needs finite t >= 0");
  } else if (p.kind == GK_PHI_SPLINE) {
    GK_REQUIRE(std::isfinite(p.eps) && p.eps > 0.0, GK_EINVAL, "spline needs eps > 0");
    GK_REQUIRE(std::isfinite(p.k) && p.k > 0.0, GK_EINVAL, "spline needs k > 0");
  } else if (p.kind == GK_PHI_POLYNOMIAL) {
    GK_REQUIRE(p.poly && p.poly_len >= 1 && p.poly_len <= 4096, GK_EINVAL, "polynomial needs coefficients");
    for (int i = 0; i < p.poly_len; ++i) GK_REQUIRE(std::isfinite(p.poly[i]), GK_EINVAL, "non-finite coefficient");
  } else {
    throw Error{GK_EINVAL, "unknown phi kind"};
  }
}

// ------------------------------------------------------------- phi stage
// U (m*s x s) = phi(H_m) F_1 and K = F_1^T phi(H_m) F_1 from the blocks
// (Hd: H_kk, Bd: H_{k+1,k}) of the block tridiagonal projected matrix.
static void phi_stage_block(Job& J, const double* Hd, const double* Bd, double* U, double* K) {
  const int m = J.m, s = J.s;
  const int ms = m * s;
  const double kk = J.phi.k;
  const bool int_spline = J.phi.kind == GK_PHI_SPLINE && kk == std::floor(kk) && kk >= 1 && kk <= 16;
  if (int_spline && !(J.flags & GK_PHI_EIG)) {
    // exact banded evaluation (block tridiagonal Cholesky solves)
    if (small_wave_ok(s)) {
      double* work = J.ar.get<double>(bcr_work_elems(m, s));
      launch_banded_spline_reg(m, s, Hd, Bd, J.phi.eps, (int)kk, work, U, J.dflags + 0, J.st);
    } else if (wide_ok(s)) {
      double* work = J.ar.get<double>(banded_wide_work_elems(m, s));
      launch_banded_spline_wide(m, s, Hd, Bd, J.phi.eps, (int)kk, work, U, J.dflags + 0, J.st);
    } else {
      double* work = J.ar.get<double>(banded_work_elems(m, s));
      launch_banded_spline(m, s, Hd, Bd, J.phi.eps, (int)kk, work, U, J.dflags + 0, J.st);
    }
    launch_store_H(U, s, s, K, J.st);          // K = sym(U[0:s, :])
    J.phi_method = 1;
    return;
  }
  if (J.phi.kind == GK_PHI_DIFFUSION && !(J.flags & GK_PHI_EIG)) {
    // Chebyshev series of exp(-t lam) on [0, Lambda] applied to F_1
    const double Lam = J.g->lambda_max;
    const int deg = cheb_diffusion_degree(J.phi.t, Lam);
    double* coef = J.ar.get<double>(deg + 1);
    hipLaunchKernelGGL(cheb_coef_kernel, dim3(nblk(deg + 1)), dim3(256), 0, J.st, deg, Lam, (int)GK_PHI_DIFFUSION,
                       J.phi.t, 0.0, 0.0, (const double*)nullptr, 0, 0, coef, J.dflags + 0);
    GK_HIP(hipGetLastError());
    const size_t tot = (size_t)m * s * s;
    double* Y0 = J.ar.get<double>(tot);
    double* Y1 = J.ar.get<double>(tot);
    double* Y2 = J.ar.get<double>(tot);
    launch_cheb_series(m, s, Hd, Bd, J.phi.t, Lam, deg, coef, Y0, Y1, Y2, U, J.st);
    launch_store_H(U, s, s, K, J.st);          // K = sym(U[0:s, :])
    J.phi_method = 2;
    return;
  }
  if (ms > kEigMaxOrder && !(J.flags & GK_PHI_EIG)) {
    // Projected matrices beyond the one-workgroup spectral decomposition:
    // phi(H_m) F_1 by the Chebyshev series of phi on [0, Lambda] (spec(H_m)
    // lies there, Theorem 3.1).  A polynomial is its own finite series; for
    // a spline (eps + lam)^-k the coefficients decay like rho^-k with
    // rho = x0 + sqrt(x0^2 - 1), x0 = 1 + 2 eps / Lambda (its pole at
    // lam = -eps), so the degree starts at 40 / ln rho and doubles until
    // the tail is below 1e-16 of the largest coefficient.
    const double Lam = J.g->lambda_max;
    const bool poly = J.phi.kind == GK_PHI_POLYNOMIAL;
    int deg;
    if (poly) {
      deg = std::max(1, J.phi.poly_len - 1);
    } else {
      const double x0 = 1.0 + 2.0 * J.phi.eps / Lam;
      const double rho = x0 + std::sqrt(x0 * x0 - 1.0);
      deg = (int)std::min(32768.0, std::ceil(40.0 / std::log(rho)) + 16.0);
    }
    double* coef = nullptr;
    for (;;) {
      coef = J.ar.get<double>(deg + 1);
      double* fv = J.ar.get<double>(deg + 1);
      launch_cheb_coef_phi(deg, Lam, J.phi, J.poly_dev, fv, coef, J.st);
      if (poly) break;
      std::vector<double> h(deg + 1);
      GK_HIP(hipMemcpyAsync(h.data(), coef, sizeof(double) * (deg + 1), hipMemcpyDeviceToHost, J.st));
      GK_HIP(hipStreamSynchronize(J.st));
      double amax = 0.0;
      for (double v : h) amax = std::max(amax, std::fabs(v));
      GK_REQUIRE(std::isfinite(amax), GK_EINVAL, "non-finite Chebyshev coefficients of phi");
      double tail = 0.0;
      for (int q = std::max(0, deg - 8); q <= deg; ++q) tail = std::max(tail, std::fabs(h[q]));
      if (tail <= 1e-16 * amax) {
        // drop the negligible end of the series
        int last = deg;
        while (last > 1 && std::fabs(h[last]) <= 1e-17 * amax) --last;
        deg = last;
        break;
      }
      GK_REQUIRE(deg < 32768, GK_EUNSUPPORTED,
                 "the Chebyshev series of this spline needs more than 32768 terms on [0, Lambda]");
      deg = std::min(32768, 2 * deg);
    }
    const size_t tot = (size_t)m * s * s;
    double* Y0 = J.ar.get<double>(tot);
    double* Y1 = J.ar.get<double>(tot);
    double* Y2 = J.ar.get<double>(tot);
    launch_cheb_series(m, s, Hd, Bd, 0.0, Lam, deg, coef, Y0, Y1, Y2, U, J.st);
    launch_store_H(U, s, s, K, J.st);          // K = sym(U[0:s, :])
    J.phi_method = 2;
    return;
  }
  // spectral decomposition H_m = S Theta S^T (Sec. 7, Table 1 row phi(H_m))
  double* T = J.ar.get<double>((size_t)ms * ms);
  double* S = J.ar.get<double>((size_t)ms * ms);
  double* th = J.ar.get<double>(ms);
  double* fv = J.ar.get<double>(ms);
  int* ord = J.ar.get<int>(eig_order_elems(ms, 1));
  double* cs = J.ar.get<double>(eig_order_elems(ms, 1));
  launch_assemble_T(m, s, Hd, Bd, T, ms, J.st);
  launch_sym_eig(ms, T, ms, S, ms, th, 1, 0, 0, 0, ord, cs, J.st);
  launch_phi_values(ms, th, J.phi, J.poly_dev, fv, false, J.dflags + 0, J.st);
  launch_phi_apply(ms, s, S, ms, fv, U, s, 1.0, J.st);
  if (J.phi.kind != GK_PHI_POLYNOMIAL) {
    double* g = J.ar.get<double>(ms);
    launch_phi_values(ms, th, J.phi, J.poly_dev, g, true, J.dflags + 0, J.st);
    launch_kww_gram(ms, s, S, ms, g, K, J.st);  // SPD by construction (Theorem 3.1)
  } else {
    launch_store_H(U, s, s, K, J.st);
  }
  J.phi_method = 0;
}

// ---------------------------------------------------------------- cbl
// Classical block Lanczos as a resumable sequence of phases, so that a
// serving loop can advance many requests in lockstep (one grouped SpMM per
// graph, one batched launch of their CholQR factors) with exactly the
// launches, operands and order of a lone call:
//   setup; for k: spmm(k), local(k), [k+1 < m: qr1(k), mid(k), qr2(k)],
//   write(k); finish.
struct CblRun {
  Job& J;
  gk_graph* g;
  int64_t n;
  int ld, m, s;
  int64_t blk;
  size_t l2;
  bool mixed, full, no_reorth, two, pan, wave, widek, pro;
  hipStream_t st;
  double* Vb = nullptr;     // FP64 basis (GK_FP64)
  double* ring = nullptr;   // 3 FP64 recurrence blocks (GK_MIXED, two-pass)
  float* Va = nullptr;      // FP32 archive (GK_MIXED)
  double *X = nullptr, *Y = nullptr, *part = nullptr, *C = nullptr, *G = nullptr, *W = nullptr;
  double *R1 = nullptr, *R1i = nullptr, *R2 = nullptr, *R2i = nullptr, *R12i = nullptr, *d1 = nullptr,
         *d2 = nullptr, *Hd = nullptr, *Bd = nullptr, *Cst = nullptr, *Rst = nullptr, *ppart = nullptr;
  double* Wr[3] = {nullptr, nullptr, nullptr};
  double *est_part = nullptr, *om_rhs = nullptr, *part_all = nullptr, *part_arch = nullptr;
  int *fr = nullptr, *forced = nullptr;
  // GK_MIXED on the single-workgroup factorisations, one entry per step: the
  // first CholQR pass sets gate[k] = 0 when its factor is final, the archive
  // projection sets it back to 1; the Gram of X R1^-1 and the second pass run
  // only at 1
  int* gate = nullptr;
  int* gk(int k) const { return gate ? gate + k : nullptr; }
  // tolerances of the estimate: threshold, floor after a reorthogonalisation
  // against the float32 archive, floor of the two explicitly orthogonalised
  // neighbours, and the per-step rounding model.  The threshold is 2^-16:
  // semi-orthogonality (2^-12, the square root of the archive's unit
  // roundoff) keeps the Ritz values, but on hub-dominated graphs it let the
  // kernel columns drift to 1.7e-5 from the float64 path; 2^-16 keeps them
  // within 5e-7 there
  double om_tau = 0x1p-16, om_floor_re = 2e-8, om_floor_loc = 1e-14, om_nu = 0;

  explicit CblRun(Job& j) : J(j) {}
  double* V64(int k) const { return (mixed || two) ? ring + (int64_t)(k % 3) * blk : Vb + (int64_t)k * blk; }
  // CholQR pass p (1 or 2) of step k on the single-workgroup kernels (kind 0:
  // blocks up to 64 wide, 1: 65..512) or the generic factorisation (kind 2)
  int qr_kind() const { return wave ? 0 : (widek ? 1 : 2); }

  void setup() {
    g = J.g;
    n = g->n;
    ld = J.ld;
    m = J.m;
    s = J.s;
    blk = n * ld;
    l2 = (size_t)ld * ld;
    mixed = J.mixed();
    full = J.full_reorth();
    no_reorth = (J.flags & GK_NO_REORTH) != 0;
    // memory-lean two-pass form (GK_FP64): pass 1 keeps three blocks and the
    // coefficients of every step; pass 2 regenerates the basis from them
    two = (J.flags & GK_TWO_PASS) != 0;
    st = J.st;
    if (!mixed) {
      if (two) ring = J.ar.get<double>((size_t)3 * blk);
      else Vb = J.ar.get<double>((size_t)m * blk);
    } else {
      ring = J.ar.get<double>((size_t)3 * blk);
      Va = J.ar.get<float>((size_t)m * blk);
    }
    X = J.ar.get<double>(blk);
    Y = J.ar.get<double>(blk);
    // scratch for every block count the Gram launches use (1 .. m)
    size_t pe = 0;
    for (int nb = 1; nb <= (full ? m : 2); ++nb) pe = std::max(pe, gram_scratch_elems(n, nb, ld));
    part = J.ar.get<double>(pe);
    C = J.ar.get<double>((size_t)m * ld * ld);
    wave = small_wave_ok(ld);
    widek = wide_ok(ld);
    G = J.ar.get<double>(l2);
    W = J.ar.get<double>(widek ? cholqr_wide_scratch_elems(ld) : l2);
    R1 = J.ar.get<double>(l2);
    R1i = J.ar.get<double>(l2);
    R2 = J.ar.get<double>(l2);
    R2i = J.ar.get<double>(l2);
    R12i = J.ar.get<double>(l2);
    d1 = J.ar.get<double>(ld);
    d2 = J.ar.get<double>(ld);
    Hd = J.ar.get<double>((size_t)m * s * s);
    Bd = J.ar.get<double>((size_t)m * s * s);
    launch_zero(Bd, (size_t)m * s * s * sizeof(double), st);
    // two-pass: the local coefficients of both Gram-Schmidt passes and the
    // normalisation R1^-1 R2^-1 of every step, kept for the replay
    if (two) {
      Cst = J.ar.get<double>((size_t)m * 4 * l2);
      Rst = J.ar.get<double>((size_t)m * l2);
    }
    // start block Q_1 = E_W (Alg. 1)
    launch_start_block(n, ld, s, J.samp, 1.0, V64(0), mixed ? Va : nullptr, st);
    pan = panel_ok(ld);
    if (pan) ppart = J.ar.get<double>(pass_scratch_elems(n, ld));
    if (mixed && (wave || widek)) gate = J.ar.get<int>(m);
    // partial reorthogonalisation (GK_MIXED, s <= 512): block omega estimate,
    // reorthogonalisation against the float32 archive only when it is needed
    pro = mixed && !full && !no_reorth && (wave || widek) && m > 2;
    if (pro) {
      for (int i = 0; i < 3; ++i) {
        Wr[i] = J.ar.get<double>((size_t)m * s * s);
        launch_zero(Wr[i], (size_t)m * s * s * sizeof(double), st);
      }
      est_part = J.ar.get<double>((size_t)m * omega_est_per_block(s));
      if (widek) om_rhs = J.ar.get<double>(omega_wide_scratch_elems(m, s));
      fr = J.ar.get<int>(m);
      forced = J.ar.get<int>(m + 1);
      launch_zero(forced, sizeof(int) * (m + 1), st);
      if (arch_ok(ld)) part_arch = J.ar.get<double>(arch_scratch_elems(n, m, ld));
      else {
        size_t pe_all = 0;
        for (int nb = 1; nb <= m; ++nb) pe_all = std::max(pe_all, gram_scratch_elems(n, nb, ld));
        part_all = J.ar.get<double>(pe_all);
      }
    }
    om_nu = 1.1102230246251565e-16 * g->lambda_max * std::sqrt((double)s);
  }

  // X = L Q_k.  GK_MIXED at ld = 64 forms Q_k^T X in the same pass (the
  // Gram of the recurrence form below; block 1 of C at k > 0, block 0 at k = 0)
  // on graphs without hub rows: the fused pass walks a hub row with one lane
  // group inside its row tiles (BA 600k at s = 64: 994 us fused against
  // 401 + 127 us for the product with hub workgroups and the Gram pass)
  bool fused = false;
  bool fusable() const { return mixed && pan && ld == 64 && g->nhub == 0; }
  void spmm(int k) {
    J.tm.begin(PH_SPMM);
    fused = fusable();
    if (fused) launch_spmm_gram64(g, mixed, V64(k), X, ppart, k > 0 ? C + l2 : C, st);
    else launch_spmm(g, mixed, ld, V64(k), nullptr, X, 1.0, 0.0, 0.0, nullptr, 0.0, nullptr, st);
  }

  // local block [Q_{k-1}, Q_k]:  C = local^T X;  H_kk = sym(C_k);  X -= local C
  // (the Q_{k-1} part realises the three-term recurrence of Alg. 1), then the
  // reorthogonalisation against the whole basis where it is done every step,
  // and G = X^T X
  void local(int k) {
    double* Vk = V64(k);
    double* Vkm1 = k > 0 ? V64(k - 1) : nullptr;
    const int nbv = k > 0 ? 2 : 1;
    J.tm.begin(PH_ORTH);
    BlockList loc = (k > 0) ? BlockList{Vkm1, (int64_t)(Vk - Vkm1), 2, false} : BlockList{Vk, blk, 1, false};
    const double* V0 = k > 0 ? Vkm1 : Vk;
    const double* V1 = k > 0 ? Vk : nullptr;
    const int local_passes = mixed ? 1 : 2;
    // GK_MIXED (block widths up to 512) takes the recurrence as written in
    // Alg. 1: X = L Q_k - Q_{k-1} H_{k-1,k} with H_{k-1,k} = B_{k-1}^T from the
    // previous QR (coefficient block 0 of C, stored by the second CholQR pass),
    // and H_kk = Q_k^T L Q_k, so the Gram pass projects onto Q_k alone.
    // GK_FP64 projects onto both local blocks twice (classical Gram-Schmidt,
    // twice).
    const bool rec = mixed && (pan || widek) && k > 0;
    for (int pass = 0; pass < local_passes; ++pass) {
      if (rec && pan) {
        if (!fused)
          launch_panel(PM_GRAMV, n, ld, 1, X, nullptr, nullptr, Vk, nullptr, nullptr, nullptr, ppart, C + l2, st);
        launch_panel(PM_UPDATE_SELF, n, ld, 2, X, X, nullptr, Vkm1, Vk, C, nullptr, ppart, G, st,
                     Hd + (int64_t)k * s * s, s, true);
      } else if (rec) {
        launch_gram(n, ld, BlockList{Vk, blk, 1, false}, X, C + l2, part, nullptr, st);
        launch_store_H(C + l2, ld, s, Hd + (int64_t)k * s * s, st);
        launch_tsgemm(n, ld, loc, C, X, X, nullptr, -1.0, 1.0, nullptr, st, false, true);
      } else if (pan) {
        double* Cp = two ? Cst + ((int64_t)k * 2 + pass) * 2 * l2 : C;
        if (!(fused && pass == 0))
          launch_panel(PM_GRAMV, n, ld, nbv, X, nullptr, nullptr, V0, V1, nullptr, nullptr, ppart, Cp, st);
        // the update pass also stores H_kk = sym(C_k) on the first pass
        launch_panel(PM_UPDATE_SELF, n, ld, nbv, X, X, nullptr, V0, V1, Cp, nullptr, ppart, G, st,
                     pass == 0 ? Hd + (int64_t)k * s * s : nullptr, s);
      } else {
        double* Cp = two ? Cst + ((int64_t)k * 2 + pass) * 2 * l2 : C;
        launch_gram(n, ld, loc, X, Cp, part, nullptr, st);
        if (pass == 0) launch_store_H(Cp + (int64_t)(loc.nb - 1) * l2, ld, s, Hd + (int64_t)k * s * s, st);
        launch_tsgemm(n, ld, loc, Cp, X, X, nullptr, -1.0, 1.0, nullptr, st);
      }
    }
    J.tm.begin(PH_REORTH);
    bool g_ready = pan;   // the panel update already produced G = X^T X
    // Against the stored basis.  The float32 archive copies of the two local
    // blocks differ from their float64 recurrence blocks by the float32
    // rounding; projecting against them would put that rounding back into X,
    // so the mixed path stops at block k-2 (the local blocks were handled
    // exactly in float64 above).
    const int nb_re = mixed ? k - 1 : k + 1;
    if (!no_reorth && full && k >= 1 && nb_re >= 1) {
      BlockList all = mixed ? BlockList{Va, blk, nb_re, true} : BlockList{Vb, blk, nb_re, false};
      for (int pass = 0; pass < 2; ++pass) {
        launch_gram(n, ld, all, X, C, part, nullptr, st);
        launch_tsgemm(n, ld, all, C, X, X, nullptr, -1.0, 1.0, nullptr, st);
      }
      g_ready = false;
    }
    J.tm.begin(PH_ORTH);
    BlockList xl{X, blk, 1, false};
    if (!g_ready) launch_gram(n, ld, xl, X, G, part, nullptr, st);
  }

  // CholQR2: X = Q_{k+1} H_{k+1,k}; pass 1 factors G = X^T X (with the gate,
  // it also writes the final factors when the second pass is not needed)
  CholqrArgs qr1_args(int k) const {
    double* R12k = two ? Rst + (int64_t)k * l2 : R12i;
    double* BT = (mixed && (pan || widek)) ? C : nullptr;
    if (!gate) return CholqrArgs{G, ld, s, 1, nullptr, J.thr(), W, R1, R1i, d1};
    return CholqrArgs{G,       ld,      s,       1, nullptr, J.thr(), W, R1, R1i, d1, nullptr, nullptr, nullptr, R12k,
                      Bd + (int64_t)k * s * s, BT, gk(k)};
  }
  // pass 2 factors the Gram of X R1^-1; the mixed recurrence takes
  // H_{k,k+1} = B_k^T of the next step from C
  CholqrArgs qr2_args(int k) const {
    double* R12k = two ? Rst + (int64_t)k * l2 : R12i;
    double* BT = (mixed && (pan || widek)) ? C : nullptr;
    return CholqrArgs{G, ld, s, 2, d1, J.thr(), W, nullptr, nullptr, d2, J.dflags + 1, R1, R1i, R12k,
                      Bd + (int64_t)k * s * s, BT, gk(k)};
  }
  void qr1(int k) {
    if (wave) launch_cholqr_reg_batched(&qr1_args_storage(k), 1, st);
    else if (widek) launch_cholqr_wide_batched(&qr1_args_storage(k), 1, st);
    else launch_cholqr_factor(G, ld, s, 1, nullptr, J.thr(), W, R1, R1i, d1, nullptr, st);
  }
  void qr2(int k) {
    if (wave || widek) {
      qa_ = qr2_args(k);
      if (wave) launch_cholqr_reg_batched(&qa_, 1, st);
      else launch_cholqr_wide_batched(&qa_, 1, st);
      return;
    }
    double* R12k = two ? Rst + (int64_t)k * l2 : R12i;
    launch_cholqr_factor(G, ld, s, 2, d1, J.thr(), W, R2, R2i, d2, J.dflags + 1, st);
    launch_small_gemm(ld, ld, ld, R1i, ld, false, R2i, ld, false, R12k, ld, 1.0, 0.0, st);
    launch_small_gemm(s, s, s, R2, ld, false, R1, ld, false, Bd + (int64_t)k * s * s, s, 1.0, 0.0, st);
  }
  CholqrArgs qa_{};
  const CholqrArgs& qr1_args_storage(int k) {
    qa_ = qr1_args(k);
    return qa_;
  }

  // between the two CholQR passes: the orthogonality estimate, the flagged
  // projection against the archive, and the Gram of X R1^-1
  void mid(int k) {
    if (pro && k >= 1) {
      // Orthogonality estimate of the new block, taken after the first
      // CholQR pass with B_k^{-1} ~ R1^{-1} (B_k = R2 R1, R2 = I + O(u)), so
      // a flagged X is projected against the archive blocks 0..k-2 before
      // it is normalised (the local blocks were handled exactly in float64
      // above).  The second pass then absorbs the change: Y = X R1^{-1} has
      // moved by |V_a^T Y| ~ tau, and CholQR of Y restores orthonormality.
      // One projection suffices: from a loss of at most tau it reaches the
      // floor set by the float32 archive.  At k = 1 the estimate has no
      // block to act on.
      const int* fk = fr + k;
      // with the archive projection to follow, its first launch takes the
      // decision (no launch of its own)
      const bool defer = k >= 2 && part_arch;
      OmegaDecide dec{};
      launch_omega(k, s, ld, Wr[k % 3], Wr[(k + 2) % 3], Wr[(k + 1) % 3], Hd, Bd, R1i, om_nu, om_tau, om_floor_re,
                   om_floor_loc, est_part, fr, forced, J.dscal + 1, J.dflags + 3, om_rhs, st, defer ? &dec : nullptr,
                   gk(k));
      if (k >= 2) {
        J.tm.begin(PH_REORTH);
        BlockList all{Va, blk, k - 1, true};
        if (part_arch) {
          launch_arch_reorth(n, ld, all, X, C, part_arch, fk, st, &dec);
        } else {
          launch_gram(n, ld, all, X, C, part_all, fk, st);
          launch_tsgemm(n, ld, all, C, X, X, nullptr, -1.0, 1.0, fk, st);
        }
        J.tm.begin(PH_ORTH);
      }
    }
    if (pan) {
      launch_panel(PM_APPLY_SELF, n, ld, 0, X, nullptr, nullptr, nullptr, nullptr, nullptr, R1i, ppart, G, st,
                   nullptr, 0, false, gk(k));
    } else {
      BlockList xl{X, blk, 1, false};
      launch_tsgemm(n, ld, xl, R1i, nullptr, Y, nullptr, 1.0, 0.0, gk(k), st, true);
      BlockList yl{Y, blk, 1, false};
      launch_gram(n, ld, yl, Y, G, part, gk(k), st);
    }
  }

  // Q_{k+1} = X R1^-1 R2^-1 (float32 archive copy when mixed); at k = m-1
  // ||X_m||_F as the residual indicator (the unused H_{m+1,m})
  void write(int k) {
    if (k + 1 < m) {
      double* R12k = two ? Rst + (int64_t)k * l2 : R12i;
      float* arch32 = mixed ? Va + (int64_t)(k + 1) * blk : nullptr;
      if (pan)
        launch_panel(PM_APPLY_WRITE, n, ld, 0, X, V64(k + 1), arch32, nullptr, nullptr, nullptr, R12k, ppart,
                     nullptr, st);
      else
        launch_tsgemm(n, ld, BlockList{X, blk, 1, false}, R12k, nullptr, V64(k + 1), arch32, 1.0, 0.0, nullptr, st,
                      true);
    } else {
      hipLaunchKernelGGL(trace_sqrt_kernel, dim3(1), dim3(256), 0, st, G, ld, s, J.dscal);
      GK_HIP(hipGetLastError());
    }
  }

  // phi of the projected matrix and the coefficients of the assembly
  void finish() {
    J.tm.begin(PH_PHI);
    double* U = J.ar.get<double>((size_t)m * s * s);
    J.K = J.ar.get<double>((size_t)s * s);
    phi_stage_block(J, Hd, Bd, U, J.K);
    if (two) {
      // Pass 2: regenerate Q_1 .. Q_m with the stored coefficients (the same
      // kernels on the same operands, so the same blocks bit for bit) and
      // accumulate P = sum_k Q_k U_k (Alg. 1 output) as they appear.
      J.tm.begin(PH_ASM);
      double* Pacc = J.ar.get<double>(blk);
      double* Uk = J.ar.get<double>(l2);
      launch_zero(Pacc, (size_t)blk * sizeof(double), st);
      launch_start_block(n, ld, s, J.samp, 1.0, V64(0), nullptr, st);
      for (int k = 0; k < m; ++k) {
        double* Vk = V64(k);
        hipLaunchKernelGGL(pad_block_kernel, dim3(nblk((int64_t)l2)), dim3(256), 0, st, k, s, ld, U, Uk);
        GK_HIP(hipGetLastError());
        launch_tsgemm(n, ld, BlockList{Vk, blk, 1, false}, Uk, Pacc, Pacc, nullptr, 1.0, 1.0, nullptr, st);
        if (k + 1 == m) break;
        double* Vkm1 = k > 0 ? V64(k - 1) : nullptr;
        const int nbv = k > 0 ? 2 : 1;
        BlockList loc = (k > 0) ? BlockList{Vkm1, (int64_t)(Vk - Vkm1), 2, false} : BlockList{Vk, blk, 1, false};
        const double* V0 = k > 0 ? Vkm1 : Vk;
        const double* V1 = k > 0 ? Vk : nullptr;
        launch_spmm(g, false, ld, Vk, nullptr, X, 1.0, 0.0, 0.0, nullptr, 0.0, nullptr, st);
        for (int pass = 0; pass < 2; ++pass) {
          const double* Cp = Cst + ((int64_t)k * 2 + pass) * 2 * l2;
          if (pan)
            launch_panel(PM_UPDATE_SELF, n, ld, nbv, X, X, nullptr, V0, V1, Cp, nullptr, ppart, G, st, nullptr, s);
          else
            launch_tsgemm(n, ld, loc, Cp, X, X, nullptr, -1.0, 1.0, nullptr, st);
        }
        const double* R12k = Rst + (int64_t)k * l2;
        if (pan)
          launch_panel(PM_APPLY_WRITE, n, ld, 0, X, V64(k + 1), nullptr, nullptr, nullptr, nullptr, R12k, ppart,
                       nullptr, st);
        else
          launch_tsgemm(n, ld, BlockList{X, blk, 1, false}, R12k, nullptr, V64(k + 1), nullptr, 1.0, 0.0, nullptr,
                        st, true);
      }
      // P and the predictor now come from the one accumulated block
      J.Upad = J.ar.get<double>((size_t)ld * s);
      hipLaunchKernelGGL(ident_rows_kernel, dim3(nblk((int64_t)ld * s)), dim3(256), 0, st, s, ld, J.Upad);
      GK_HIP(hipGetLastError());
      J.arch = BlockList{Pacc, blk, 1, false};
      J.spd = J.phi.kind != GK_PHI_POLYNOMIAL;
      J.tm.end();
      return;
    }
    J.Upad = J.ar.get<double>((size_t)m * ld * s);
    hipLaunchKernelGGL(pad_rows_kernel, dim3(nblk((int64_t)m * ld * s)), dim3(256), 0, st, m, s, ld, U, J.Upad);
    GK_HIP(hipGetLastError());
    J.arch = mixed ? BlockList{Va, blk, m, true} : BlockList{Vb, blk, m, false};
    J.spd = J.phi.kind != GK_PHI_POLYNOMIAL;
    J.tm.end();
  }
};

static void run_cbl(Job& J) {
  CblRun R(J);
  R.setup();
  for (int k = 0; k < R.m; ++k) {
    R.spmm(k);
    R.local(k);
    if (k + 1 < R.m) {
      R.qr1(k);
      R.mid(k);
      R.qr2(k);
    }
    R.write(k);
  }
  R.finish();
}

// ---------------------------------------------------------------- gbl / sbl
static void run_scalar_lanczos(Job& J, bool global) {
  gk_graph* g = J.g;
  const int64_t n = g->n;
  const int ld = J.ld, m = J.m, s = J.s;
  const int64_t blk = n * ld;
  const bool mixed = J.mixed();
  const bool full = J.full_reorth();
  const bool no_reorth = (J.flags & GK_NO_REORTH) != 0;
  hipStream_t st = J.st;
  double* Vb = nullptr;
  double* ring = nullptr;
  float* Va = nullptr;
  if (!mixed) Vb = J.ar.get<double>((size_t)m * blk);
  else {
    ring = J.ar.get<double>((size_t)3 * blk);
    Va = J.ar.get<float>((size_t)m * blk);
  }
  double* X = J.ar.get<double>(blk);
  double* part = J.ar.get<double>(coldots_scratch_elems(n, m, ld));
  double* cd = J.ar.get<double>((size_t)m * ld);
  double* D = J.ar.get<double>((size_t)m * ld);
  double* scale = J.ar.get<double>(ld);
  // alpha / beta: global -> m scalars; sequential -> m x s
  const int ab = global ? 1 : s;
  double* alpha = J.ar.get<double>((size_t)m * ab);
  double* beta = J.ar.get<double>((size_t)m * ab);
  launch_zero(beta, (size_t)m * ab * sizeof(double), st);
  double* resid = J.ar.get<double>(ab);
  auto V64 = [&](int k) -> double* { return mixed ? ring + (int64_t)(k % 3) * blk : Vb + (int64_t)k * blk; };
  // partial reorthogonalisation (GK_MIXED): scalar omega recurrences, one per
  // Lanczos run (nw = 1 for gbl, s for sbl), ring of three estimate rows
  const bool pro = mixed && !full && !no_reorth && m > 2;
  const int nw = global ? 1 : s;
  double* Om[3] = {nullptr, nullptr, nullptr};
  int* fr = nullptr;
  int* forced = nullptr;
  if (pro) {
    for (int i = 0; i < 3; ++i) {
      Om[i] = J.ar.get<double>((size_t)m * nw);
      launch_zero(Om[i], (size_t)m * nw * sizeof(double), st);
    }
    fr = J.ar.get<int>(m);
    forced = J.ar.get<int>(m + 1);
    launch_zero(forced, sizeof(int) * (m + 1), st);
  }
  // thresholds as for the block estimate of cbl; the rounding term is the
  // local error of one step, 2 u_64 Lambda
  const double om_tau = 0x1p-12, om_floor_re = 2e-8, om_floor_loc = 1e-14;
  const double om_nu = 2.0 * 1.1102230246251565e-16 * g->lambda_max;
  // Q_1 = E_W / sqrt(N) (Alg. 2) or E_W (sequential, each column a unit vector)
  launch_start_block(n, ld, s, J.samp, global ? 1.0 / std::sqrt((double)s) : 1.0, V64(0),
                     mixed ? Va : nullptr, st);
  for (int k = 0; k < m; ++k) {
    double* Vk = V64(k);
    J.tm.begin(PH_SPMM);
    launch_spmm(g, mixed, ld, Vk, nullptr, X, 1.0, 0.0, 0.0, nullptr, 0.0, nullptr, st);
    J.tm.begin(PH_ORTH);
    BlockList loc = (k > 0) ? BlockList{V64(k - 1), (int64_t)(Vk - V64(k - 1)), 2, false}
                            : BlockList{Vk, blk, 1, false};
    for (int pass = 0; pass < 2; ++pass) {
      launch_coldots(n, ld, loc, X, cd, part, nullptr, st);
      if (global) {
        hipLaunchKernelGGL(frob_coef_kernel, dim3(loc.nb), dim3(256), 0, st, loc.nb, s, ld, cd, D,
                           pass == 0 ? alpha + k : (double*)nullptr, (const int*)nullptr);
      } else {
        // per-column coefficients are the dots themselves; alpha_k = D of Q_k
        GK_HIP(hipMemcpyAsync(D, cd, sizeof(double) * loc.nb * ld, hipMemcpyDeviceToDevice, st));
        if (pass == 0)
          GK_HIP(hipMemcpyAsync(alpha + (int64_t)k * s, cd + (int64_t)(loc.nb - 1) * ld, sizeof(double) * s,
                                hipMemcpyDeviceToDevice, st));
      }
      GK_HIP(hipGetLastError());
      launch_axpy_diag(n, ld, loc, D, X, nullptr, st);
    }
    J.tm.begin(PH_REORTH);
    // against the stored basis; the mixed path stops at block k-2 (see run_cbl)
    const int nb_re = mixed ? k - 1 : k + 1;
    if (!no_reorth && full && k >= 1 && nb_re >= 1) {
      BlockList all = mixed ? BlockList{Va, blk, nb_re, true} : BlockList{Vb, blk, nb_re, false};
      for (int pass = 0; pass < 2; ++pass) {
        launch_coldots(n, ld, all, X, cd, part, nullptr, st);
        if (global)
          hipLaunchKernelGGL(frob_coef_kernel, dim3(all.nb), dim3(256), 0, st, all.nb, s, ld, cd, D,
                             (double*)nullptr, (const int*)nullptr);
        else
          GK_HIP(hipMemcpyAsync(D, cd, sizeof(double) * all.nb * ld, hipMemcpyDeviceToDevice, st));
        launch_axpy_diag(n, ld, all, D, X, nullptr, st);
      }
    }
    J.tm.begin(PH_ORTH);
    BlockList xl{X, blk, 1, false};
    launch_coldots(n, ld, xl, X, cd, part, nullptr, st);
    if (pro && k >= 1 && k + 1 < m) {
      // partial reorthogonalisation: estimate from the norm of X, then (when
      // flagged) one projection against the float32 archive blocks 0..k-2 and
      // the norm again
      hipLaunchKernelGGL(omega_scalar_kernel, dim3(1), dim3(1024), 0, st, k, nw, s, global ? 1 : 0, alpha, beta, cd,
                         J.thr(), om_nu, om_tau, om_floor_re, om_floor_loc, Om[(k + 2) % 3], Om[k % 3],
                         Om[(k + 1) % 3], fr, forced, J.dscal + 1, J.dflags + 3);
      GK_HIP(hipGetLastError());
      if (k >= 2) {
        J.tm.begin(PH_REORTH);
        const int* fk = fr + k;
        BlockList arc{Va, blk, k - 1, true};
        launch_coldots(n, ld, arc, X, cd, part, fk, st);
        if (global) {
          hipLaunchKernelGGL(frob_coef_kernel, dim3(arc.nb), dim3(256), 0, st, arc.nb, s, ld, cd, D,
                             (double*)nullptr, fk);
          GK_HIP(hipGetLastError());
        }
        launch_axpy_diag(n, ld, arc, global ? D : cd, X, fk, st);
        launch_coldots(n, ld, xl, X, cd, part, fk, st);
        J.tm.begin(PH_ORTH);
      }
    }
    if (global)
      hipLaunchKernelGGL(frob_norm_kernel, dim3(1), dim3(256), 0, st, s, ld, cd, J.thr(),
                         (k + 1 < m) ? beta + k : (double*)nullptr, scale, resid);
    else
      hipLaunchKernelGGL(col_norm_kernel, dim3(nblk(ld)), dim3(256), 0, st, s, ld, cd, J.thr(),
                         (k + 1 < m) ? beta + (int64_t)k * s : (double*)nullptr, scale, resid);
    GK_HIP(hipGetLastError());
    if (k + 1 < m) launch_colscale(n, ld, X, scale, V64(k + 1), mixed ? Va + (int64_t)(k + 1) * blk : nullptr, st);
  }
  J.tm.begin(PH_PHI);
  // tridiagonal H_m (global) or s tridiagonal H_m^(w) (sequential): eigh
  const int batch = global ? 1 : s;
  const int64_t mm = (int64_t)m * m;
  double* T = J.ar.get<double>((size_t)mm * batch);
  double* S = J.ar.get<double>((size_t)mm * batch);
  double* th = J.ar.get<double>((size_t)m * batch);
  double* fv = J.ar.get<double>((size_t)m * batch);
  int* ord = J.ar.get<int>(eig_order_elems(m, batch));
  double* cs = J.ar.get<double>(eig_order_elems(m, batch));
  hipLaunchKernelGGL(tridiag_dense_kernel, dim3(nblk(mm * batch)), dim3(256), 0, st, m, batch, ab, alpha, beta, T);
  GK_HIP(hipGetLastError());
  launch_sym_eig(m, T, m, S, m, th, batch, mm, mm, m, ord, cs, st);
  launch_phi_values(m * batch, th, J.phi, J.poly_dev, fv, false, J.dflags + 0, st);
  J.D = J.ar.get<double>((size_t)m * ld);
  if (global) {
    double* u = J.ar.get<double>(m);
    launch_phi_apply(m, 1, S, m, fv, u, 1, std::sqrt((double)s), st);   // u = sqrt(N) phi(H_m) f_1
    hipLaunchKernelGGL(bcast_coef_kernel, dim3(nblk((int64_t)m * ld)), dim3(256), 0, st, m, s, ld, u, J.D);
  } else {
    hipLaunchKernelGGL(seq_coef_kernel, dim3(nblk((int64_t)m * ld)), dim3(256), 0, st, m, s, ld, S, fv, J.D);
  }
  GK_HIP(hipGetLastError());
  J.arch = mixed ? BlockList{Va, blk, m, true} : BlockList{Vb, blk, m, false};
  J.K = J.ar.get<double>((size_t)s * s);
  launch_gather_diag(n, ld, s, J.arch, J.D, J.samp, J.K, st);   // K = E_W^T P
  J.spd = false;
  J.phi_method = 0;
  J.tm.end();
}

// ------------------------------------------------------------- Chebyshev
static void run_cheb(Job& J, bool squared) {
  gk_graph* g = J.g;
  const int64_t n = g->n;
  const int ld = J.ld, s = J.s;
  const int64_t blk = n * ld;
  const bool mixed = J.mixed();
  hipStream_t st = J.st;
  const double Lam = g->lambda_max;
  const int deg = squared ? std::max(J.m / 2, 1) : J.m;
  double* a = J.ar.get<double>(deg + 1);
  hipLaunchKernelGGL(cheb_coef_kernel, dim3(nblk(deg + 1)), dim3(256), 0, st, deg, Lam, J.phi.kind, J.phi.t,
                     J.phi.eps, J.phi.k, J.poly_dev, J.phi.poly_len, squared ? 1 : 0, a, J.dflags + 0);
  GK_HIP(hipGetLastError());
  double* ring = J.ar.get<double>((size_t)3 * blk);
  double* acc = J.ar.get<double>(blk);
  double* acc2 = squared ? J.ar.get<double>(blk) : nullptr;
  auto Yb = [&](int k) -> double* { return ring + (int64_t)(k % 3) * blk; };
  launch_start_block(n, ld, s, J.samp, 1.0, Yb(0), nullptr, st);
  for (int rep = 0; rep < (squared ? 2 : 1); ++rep) {
    double* out = (rep == 0) ? acc : acc2;
    if (rep == 1) GK_HIP(hipMemcpyAsync(Yb(0), acc, sizeof(double) * blk, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(scale_copy_kernel, dim3(nblk(blk)), dim3(256), 0, st, blk, a, Yb(0), out);
    GK_HIP(hipGetLastError());
    J.tm.begin(PH_SPMM);
    // T_1(x) = x with x = I - (2/Lam) L ; T_{k+1} = 2 x T_k - T_{k-1}
    if (deg >= 1) launch_spmm(g, mixed, ld, Yb(0), nullptr, Yb(1), -2.0 / Lam, 1.0, 0.0, out, 0.0, a + 1, st);
    for (int k = 1; k < deg; ++k)
      launch_spmm(g, mixed, ld, Yb(k), Yb(k - 1), Yb(k + 1), -4.0 / Lam, 2.0, -1.0, out, 0.0, a + k + 1, st);
    J.tm.end();
  }
  double* P = squared ? acc2 : acc;
  J.arch = BlockList{P, blk, 1, false};
  J.D = J.ar.get<double>(ld);
  hipLaunchKernelGGL(fill_kernel, dim3(nblk(ld)), dim3(256), 0, st, J.D, ld, 1.0);
  GK_HIP(hipGetLastError());
  J.K = J.ar.get<double>((size_t)s * s);
  launch_gather_diag(n, ld, s, J.arch, J.D, J.samp, J.K, st);
  J.spd = false;
  J.phi_method = 2;
}

// ----------------------------------------------------------- call wrapper
uint64_t footprint_bytes(int64_t n, int s, int m, int variant, int precision, uint32_t flags) {
  const int ld = block_ld(s);
  const double blk8 = (double)n * ld * 8.0;
  double b = 0;
  const bool mixed = precision == GK_MIXED;
  if ((flags & GK_TWO_PASS) && variant == GK_CBL && !mixed) {
    // three recurrence blocks, X, Y, the accumulated columns, the stored
    // coefficients, the Gram partials of the local passes, the projected
    // matrix and the phi stage
    const double l2 = (double)ld * ld * 8.0, ms = (double)m * s;
    size_t pe = 0;
    for (int nb = 1; nb <= 2; ++nb) pe = std::max(pe, gram_scratch_elems(n, nb, ld));
    b = 6 * blk8 + 5.0 * m * l2 + 8.0 * pe + 2 * ms * ms * 8.0 + 8.0 * l2 + 4.0 * m * s * s * 8.0;
    if (panel_ok(ld)) b += 8.0 * pass_scratch_elems(n, ld);
    if (small_wave_ok(s)) b += 8.0 * bcr_work_elems(m, s);
    if (wide_ok(ld)) b += 8.0 * cholqr_wide_scratch_elems(ld);
    b += (double)n * s * 8.0 + 64.0 * (1 << 20);
    return (uint64_t)b;
  }
  if (variant == GK_CHEB || variant == GK_CHEB2) {
    b = blk8 * (variant == GK_CHEB2 ? 5 : 4);
  } else {
    b = mixed ? (3 * blk8 + m * blk8 / 2) : m * blk8;
    b += 2 * blk8;   // X, Y
    const double ms = (double)m * s;
    if (variant == GK_GBL || variant == GK_SBL) {
      // column-dot partials, coefficients, tridiagonal coefficients, the
      // eigendecompositions of the tridiagonal matrices, and the estimates
      const double nw = variant == GK_GBL ? 1.0 : (double)s;
      b += 8.0 * coldots_scratch_elems(n, m, ld) + 2.0 * m * ld * 8.0 + 2.0 * m * nw * 8.0 + 3.0 * nw * 8.0;
      b += nw * (2.0 * m * m + 2.0 * m) * 8.0 + 8.0 * 2.0 * eig_order_elems(m, (int)nw);
      b += 3.0 * m * nw * 8.0 + 8.0 * m * ld;
    }
    if (variant == GK_CBL) {
      b += 2 * ms * ms * 8.0 + (double)m * ld * ld * 8.0 + 4.0 * m * s * s * 8.0;
      if (small_wave_ok(s)) b += 8.0 * bcr_work_elems(m, s);   // spline by cyclic reduction
      // Gram partials of the orthogonalisation passes
      const bool full = !mixed || (variant == GK_CBL && !(small_wave_ok(ld) || wide_ok(ld)));
      size_t pe = 0;
      for (int nb = 1; nb <= (full ? m : 2); ++nb) pe = std::max(pe, gram_scratch_elems(n, nb, ld));
      b += 8.0 * pe;
      if (panel_ok(ld)) b += 8.0 * pass_scratch_elems(n, ld);
      if (mixed) {
        // partial reorthogonalisation: estimate blocks and archive partials
        b += 3.0 * m * s * s * 8.0;
        if (wide_ok(ld)) b += 8.0 * (omega_wide_scratch_elems(m, s) + cholqr_wide_scratch_elems(ld));
        if (arch_ok(ld)) {
          b += 8.0 * arch_scratch_elems(n, m, ld);
        } else {
          size_t pa = 0;
          for (int nb = 1; nb <= m; ++nb) pa = std::max(pa, gram_scratch_elems(n, nb, ld));
          b += 8.0 * pa;
        }
      }
    }
  }
  b += (double)n * s * 8.0 + 64.0 * (1 << 20);   // output staging + small scratch
  return (uint64_t)b;
}

static void validate_common(const CallArgs& a) {
  GK_REQUIRE(a.g, GK_EINVAL, "graph is NULL");
  GK_REQUIRE(a.s >= 1 && a.s <= 1024, GK_EINVAL, "s must be in [1, 1024]");
  GK_REQUIRE(a.m >= 1 && a.m <= 4096, GK_EINVAL, "m must be in [1, 4096]");
  GK_REQUIRE(a.phi, GK_EINVAL, "phi is NULL");
  GK_REQUIRE(a.samples, GK_EINVAL, "samples is NULL");
  GK_REQUIRE(a.variant >= GK_CBL && a.variant <= GK_CHEB2, GK_EINVAL, "unknown variant");
  GK_REQUIRE(a.precision == GK_FP64 || a.precision == GK_MIXED, GK_EINVAL, "unknown precision");
  GK_REQUIRE((a.flags & ~(GK_IO_DEVICE | GK_FULL_REORTH | GK_PHI_EIG | GK_TIMING | GK_NO_REORTH | GK_TWO_PASS)) == 0,
             GK_EINVAL, "unknown flag bits");
  if (a.flags & GK_TWO_PASS)
    GK_REQUIRE(a.variant == GK_CBL && a.precision == GK_FP64, GK_EUNSUPPORTED,
               "the two-pass form is built for classical block Lanczos in float64");
  phi_check(*a.phi);
  if (a.fit) {
    GK_REQUIRE(a.y, GK_EINVAL, "y is NULL");
    GK_REQUIRE(std::isfinite(a.gamma) && a.gamma >= 0.0, GK_EINVAL, "gamma must be finite and >= 0");
  }
  const int64_t ms = (int64_t)a.m * a.s;
  const bool banded_ok = a.phi->kind == GK_PHI_SPLINE && a.phi->k == std::floor(a.phi->k) && a.phi->k <= 16;
  const bool cheb_ok = a.phi->kind == GK_PHI_DIFFUSION;
  // beyond kEigMaxOrder splines and polynomials take the Chebyshev series;
  // the spectral decomposition itself (GK_PHI_EIG) stays one workgroup
  if (a.variant == GK_CBL && (a.flags & GK_PHI_EIG))
    GK_REQUIRE(ms <= kEigMaxOrder, GK_EUNSUPPORTED,
               "the single-workgroup spectral decomposition is limited to m*s <= 4096");
  (void)banded_ok;
  (void)cheb_ok;
}

static void check_samples_host(const int64_t* h, int s, int64_t n) {
  std::vector<int64_t> v(h, h + s);
  for (int64_t x : v) GK_REQUIRE(x >= 0 && x < n, GK_ERANGE, "sample " + std::to_string(x) + " out of range");
  std::sort(v.begin(), v.end());
  for (int i = 1; i < s; ++i) GK_REQUIRE(v[i] != v[i - 1], GK_EDUPSAMPLE, "duplicate sample " + std::to_string(v[i]));
}

// One call: validation and set-up, the Krylov stage, the outputs, completion.
// The lone entry points run the phases back to back; the serving loop
// advances several classical block Lanczos calls in lockstep between
// call_prepare and call_outputs (BatchCall below).
struct CallState {
  CallArgs a;
  Job J;
  bool dev_io = false;
  std::vector<int64_t> hs;   // samples on the host (uploaded asynchronously)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int hflags[8] = {0};
  double hscal[8] = {0};
  double* hcols = nullptr;
  double* hK = nullptr;
  double* coef = nullptr;
  double* pred = nullptr;
  explicit CallState(const CallArgs& args) : a(args) {}
  ~CallState() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

// validation, device set-up of the job and the samples (enqueued on stream)
static void call_prepare(CallState& S, hipStream_t stream, bool timers) {
  const CallArgs& a = S.a;
  validate_common(a);
  // a status left by the caller's own earlier HIP calls is not this call's
  (void)hipGetLastError();
  gk_graph* g = a.g;
  S.dev_io = (a.flags & GK_IO_DEVICE) != 0;
  // samples: validate on the host
  std::vector<int64_t>& hs = S.hs;
  hs.resize(a.s);
  if (S.dev_io) GK_HIP(hipMemcpy(hs.data(), a.samples, sizeof(int64_t) * a.s, hipMemcpyDeviceToHost));
  else std::memcpy(hs.data(), a.samples, sizeof(int64_t) * a.s);
  check_samples_host(hs.data(), a.s, g->n);
  GK_HIP(hipSetDevice(g->device));

  Job& J = S.J;
  J.ar.pool = static_cast<char*>(a.pool);
  J.ar.pool_cap = a.pool_cap;
  J.g = g;
  J.s = a.s;
  J.ld = block_ld(a.s);
  J.m = a.m;
  J.variant = a.variant;
  J.precision = a.precision;
  J.flags = a.flags;
  J.phi = *a.phi;
  J.st = stream;
  J.tm.on = timers && (a.flags & GK_TIMING) != 0;
  J.tm.st = stream;
  if (timers) kt_start(J.tm.on);
  if (J.tm.on) {
    GK_HIP(hipEventCreate(&S.ev0));
    GK_HIP(hipEventCreate(&S.ev1));
    GK_HIP(hipEventRecord(S.ev0, stream));
  }
  J.dflags = J.ar.get<int>(8);
  launch_zero(J.dflags, 256, stream);
  J.dscal = J.ar.get<double>(8);
  launch_zero(J.dscal, 256, stream);
  if (a.phi->kind == GK_PHI_POLYNOMIAL) {
    J.poly_dev = J.ar.get<double>(a.phi->poly_len);
    GK_HIP(hipMemcpyAsync(J.poly_dev, a.phi->poly, sizeof(double) * a.phi->poly_len, hipMemcpyHostToDevice, stream));
  }
  // samples in device numbering
  int64_t* samp_in = J.ar.get<int64_t>(a.s);
  GK_HIP(hipMemcpyAsync(samp_in, hs.data(), sizeof(int64_t) * a.s, hipMemcpyHostToDevice, stream));
  J.samp = J.ar.get<int64_t>(a.s);
  hipLaunchKernelGGL(map_samples_kernel, dim3(nblk(a.s)), dim3(256), 0, stream, a.s, samp_in,
                     g->reordered ? g->d_iperm : (const int64_t*)nullptr, J.samp);
  GK_HIP(hipGetLastError());
}

// assembly of the columns, K_WW, the fit and the predictor, and (copies)
// the copies back, all enqueued on J.st
static void call_outputs(CallState& S, bool copies = true) {
  const CallArgs& a = S.a;
  Job& J = S.J;
  gk_graph* g = a.g;
  hipStream_t stream = J.st;
  const int64_t n = g->n;
  const int s = a.s, ld = J.ld;
  const int64_t* perm = g->reordered ? g->d_perm : nullptr;
  J.tm.begin(PH_ASM);
  if (a.cols_out) {
    double* P = S.dev_io ? a.cols_out : J.ar.get<double>((size_t)n * s);
    if (J.Upad) {
      // [Q_1..Q_m] U (Alg. 1)
      if (J.arch.f32 && J.arch.stride > 0 && arch_ok(ld))
        launch_arch_assemble(n, ld, s, J.arch, J.Upad, P, perm, stream);
      else
        launch_assemble(n, ld, s, J.arch, J.Upad, s, P, perm, stream);
    } else {
      launch_assemble_diag(n, ld, s, J.arch, J.D, P, perm, true, stream);   // sum_k u_k Q_k (Alg. 2)
    }
    S.hcols = P;
  }
  J.tm.end();
  if (a.kww_out) {   // K is row-major internally; the ABI hands out column-major
    S.hK = J.ar.get<double>((size_t)s * s);
    hipLaunchKernelGGL(transpose_kernel, dim3(nblk((int64_t)s * s)), dim3(256), 0, stream, s, J.K, S.hK);
    GK_HIP(hipGetLastError());
  }
  if (a.fit) {
    J.tm.begin(PH_FIT);
    const double* y = a.y;
    if (!S.dev_io) {
      double* yd = J.ar.get<double>(s);
      GK_HIP(hipMemcpyAsync(yd, a.y, sizeof(double) * s, hipMemcpyHostToDevice, stream));
      y = yd;
    }
    S.coef = (S.dev_io && a.coef_out) ? a.coef_out : J.ar.get<double>(s);
    double* wk = J.ar.get<double>((size_t)s * s);
    int* piv = J.ar.get<int>(s);
    // K gathered from the float32 archive (mixed gbl / sbl) carries float32
    // rounding; elsewhere it is formed in float64
    const double piv_rel = (J.arch.f32 && !J.Upad) ? 0x1p-20 : 0x1p-40;
    launch_small_solve(s, J.K, a.gamma, y, S.coef, wk, piv, J.spd, piv_rel, J.dflags + 2, stream);
    J.tm.begin(PH_ASM);
    if (a.pred_out) {
      const int nbk = J.arch.nb;
      double* z = J.ar.get<double>((size_t)nbk * ld);
      if (J.Upad)   // z = phi(H_m) F_1 c  (Corollary 1)
        launch_small_gemm(nbk * ld, 1, s, J.Upad, s, false, S.coef, 1, false, z, 1, 1.0, 0.0, stream);
      else
        hipLaunchKernelGGL(zdiag_kernel, dim3(nblk((int64_t)nbk * ld)), dim3(256), 0, stream, nbk, s, ld, J.D, S.coef,
                           z);
      GK_HIP(hipGetLastError());
      S.pred = S.dev_io ? a.pred_out : J.ar.get<double>(n);
      launch_predict(n, ld, J.arch, z, S.pred, perm, stream);
    }
    J.tm.end();
  }
  if (J.tm.on) GK_HIP(hipEventRecord(S.ev1, stream));
  if (!copies) return;
  // copy back
  GK_HIP(hipMemcpyAsync(S.hflags, J.dflags, sizeof(S.hflags), hipMemcpyDeviceToHost, stream));
  GK_HIP(hipMemcpyAsync(S.hscal, J.dscal, sizeof(S.hscal), hipMemcpyDeviceToHost, stream));
  if (!S.dev_io) {
    if (a.cols_out)
      GK_HIP(hipMemcpyAsync(a.cols_out, S.hcols, sizeof(double) * n * s, hipMemcpyDeviceToHost, stream));
    if (a.coef_out && S.coef)
      GK_HIP(hipMemcpyAsync(a.coef_out, S.coef, sizeof(double) * s, hipMemcpyDeviceToHost, stream));
    if (a.pred_out && S.pred)
      GK_HIP(hipMemcpyAsync(a.pred_out, S.pred, sizeof(double) * n, hipMemcpyDeviceToHost, stream));
  }
  if (a.kww_out) {
    GK_HIP(hipMemcpyAsync(a.kww_out, S.hK, sizeof(double) * s * s,
                          S.dev_io ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, stream));
  }
}

// after the stream has completed the call's work: statistics and status
static int call_complete(CallState& S, bool timers) {
  const CallArgs& a = S.a;
  Job& J = S.J;
  gk_graph* g = a.g;
  const int64_t n = g->n;
  const int ld = J.ld;
  if (timers) kt_finish();
  if (a.st) {
    std::memset(a.st, 0, sizeof(gk_stats));
    J.tm.collect(a.st);
    if (S.ev0 && S.ev1) {
      float ms = 0;
      GK_HIP(hipEventElapsedTime(&ms, S.ev0, S.ev1));
      a.st->t_total_ms = ms;
    }
    a.st->n_deflated = S.hflags[1];
    a.st->n_qr2_series = S.hflags[5];
    a.st->n_qr2_skipped = S.hflags[6];
    a.st->resid_norm = S.hscal[0];
    a.st->phi_method = J.phi_method;
    a.st->footprint_bytes = J.ar.bytes;
    a.st->n_reorth = (J.variant <= GK_SBL && J.full_reorth() && !(J.flags & GK_NO_REORTH)) ? std::max(J.m - 1, 0)
                                                                                           : S.hflags[3];
    a.st->orth_est = S.hscal[1];
    const double wb = g->unit ? 0.0 : (J.mixed() ? 4.0 : 8.0);
    a.st->bytes_spmm = a.st->spmm_launches * (4.0 * (n + 1) + g->nnz * (4.0 + wb) + 8.0 * n + 2.0 * 8.0 * n * ld);
  }
  if (S.hflags[0] == 1) throw Error{GK_EINVAL, "eps + theta <= 0 for a Ritz value theta"};
  if (S.hflags[0] == 3) throw Error{GK_ENOTSPD, "eps I + H_m not positive definite"};
  if (S.hflags[2]) throw Error{GK_ENOTSPD, "(K_W + gamma I) c = y not solvable"};
  return GK_OK;
}

int run_call(const CallArgs& a, hipStream_t stream) {
  CallState S(a);
  call_prepare(S, stream, true);
  Job& J = S.J;
  switch (a.variant) {
    case GK_CBL: run_cbl(J); break;
    case GK_GBL: run_scalar_lanczos(J, true); break;
    case GK_SBL: run_scalar_lanczos(J, false); break;
    case GK_CHEB: run_cheb(J, false); break;
    case GK_CHEB2: run_cheb(J, true); break;
  }
  call_outputs(S);
  GK_HIP(hipStreamSynchronize(stream));
  J.ar.settled = true;   // its blocks are idle: cached without reuse events
  return call_complete(S, true);
}

// ------------------------------------------------ lockstep serving support
// A classical block Lanczos call that the serving loop advances one Lanczos
// step at a time together with other calls: one grouped SpMM per graph and
// one batched launch of each CholQR pass per step (same kernels, operands
// and order as a lone call, so the same results bit for bit).
struct BatchCall {
  CallState S;
  std::unique_ptr<CblRun> R;
  int k = 0;
  hipEvent_t done = nullptr;
  explicit BatchCall(const CallArgs& a) : S(a) {}
  ~BatchCall() {
    if (done) (void)hipEventDestroy(done);
  }
};

bool batch_eligible(const CallArgs& a) {
  return a.variant == GK_CBL && !(a.flags & (GK_TWO_PASS | GK_IO_DEVICE | GK_TIMING));
}

BatchCall* batch_begin(const CallArgs& a, hipStream_t step_stream) {
  std::unique_ptr<BatchCall> B(new BatchCall(a));
  call_prepare(B->S, step_stream, false);
  B->R.reset(new CblRun(B->S.J));
  B->R->setup();
  return B.release();
}

bool batch_stepping(const BatchCall* B) { return B->k < B->R->m; }

void batch_step(std::vector<BatchCall*>& calls, hipStream_t st) {
  for (BatchCall* B : calls) {
    B->R->st = st;
    B->S.J.st = st;
    B->S.J.tm.st = st;
  }
  // grouped SpMM: one launch per graph and weight precision; 64-wide mixed
  // calls take their own product with the Gram fused (the arithmetic of
  // their lone run)
  std::vector<char> done(calls.size(), 0);
  for (size_t i = 0; i < calls.size(); ++i) {
    calls[i]->R->fused = false;
    if (calls[i]->R->fusable()) {
      calls[i]->R->spmm(calls[i]->k);
      done[i] = 1;
    }
  }
  for (size_t i = 0; i < calls.size(); ++i) {
    if (done[i]) continue;
    const CblRun& Ri = *calls[i]->R;
    std::vector<int> ld;
    std::vector<const double*> V;
    std::vector<double*> X;
    for (size_t j = i; j < calls.size(); ++j) {
      const CblRun& Rj = *calls[j]->R;
      if (done[j] || Rj.g != Ri.g || Rj.mixed != Ri.mixed) continue;
      done[j] = 1;
      ld.push_back(Rj.ld);
      V.push_back(Rj.V64(calls[j]->k));
      X.push_back(Rj.X);
    }
    launch_spmm_group(Ri.g, Ri.mixed, (int)ld.size(), ld.data(), V.data(), X.data(), st);
  }
  for (BatchCall* B : calls) B->R->local(B->k);
  // the first CholQR pass of every call that normalises a new block
  std::vector<CholqrArgs> wave, wide;
  for (BatchCall* B : calls) {
    if (B->k + 1 >= B->R->m) continue;
    if (B->R->qr_kind() == 0) wave.push_back(B->R->qr1_args(B->k));
    else if (B->R->qr_kind() == 1) wide.push_back(B->R->qr1_args(B->k));
    else B->R->qr1(B->k);
  }
  if (!wave.empty()) launch_cholqr_reg_batched(wave.data(), (int)wave.size(), st);
  if (!wide.empty()) launch_cholqr_wide_batched(wide.data(), (int)wide.size(), st);
  for (BatchCall* B : calls)
    if (B->k + 1 < B->R->m) B->R->mid(B->k);
  wave.clear();
  wide.clear();
  for (BatchCall* B : calls) {
    if (B->k + 1 >= B->R->m) continue;
    if (B->R->qr_kind() == 0) wave.push_back(B->R->qr2_args(B->k));
    else if (B->R->qr_kind() == 1) wide.push_back(B->R->qr2_args(B->k));
    else B->R->qr2(B->k);
  }
  if (!wave.empty()) launch_cholqr_reg_batched(wave.data(), (int)wave.size(), st);
  if (!wide.empty()) launch_cholqr_wide_batched(wide.data(), (int)wide.size(), st);
  for (BatchCall* B : calls) {
    B->R->write(B->k);
    B->k++;
  }
}

// phi stage and outputs of a call whose steps are done, on stream fin (after
// the work already enqueued on the step stream); records the completion event
void batch_finish(BatchCall* B, hipStream_t step_stream, hipStream_t fin) {
  hipEvent_t ev;
  GK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  GK_HIP(hipEventRecord(ev, step_stream));
  GK_HIP(hipStreamWaitEvent(fin, ev, 0));
  GK_HIP(hipEventDestroy(ev));
  B->S.J.st = fin;
  B->S.J.tm.st = fin;
  B->R->st = fin;
  B->R->finish();
  call_outputs(B->S, false);
  GK_HIP(hipEventCreateWithFlags(&B->done, hipEventDisableTiming));
  GK_HIP(hipEventRecord(B->done, fin));
}

// waits for the call's work, then copies its results to the host buffers
// (synchronous copies here keep the thread that enqueues the steps from
// ever blocking on a transfer)
int batch_complete(BatchCall* B) {
  GK_HIP(hipEventSynchronize(B->done));
  CallState& S = B->S;
  const CallArgs& a = S.a;
  const int64_t n = a.g->n;
  GK_HIP(hipMemcpy(S.hflags, S.J.dflags, sizeof(S.hflags), hipMemcpyDeviceToHost));
  GK_HIP(hipMemcpy(S.hscal, S.J.dscal, sizeof(S.hscal), hipMemcpyDeviceToHost));
  if (a.cols_out) GK_HIP(hipMemcpy(a.cols_out, S.hcols, sizeof(double) * n * a.s, hipMemcpyDeviceToHost));
  if (a.coef_out && S.coef) GK_HIP(hipMemcpy(a.coef_out, S.coef, sizeof(double) * a.s, hipMemcpyDeviceToHost));
  if (a.pred_out && S.pred) GK_HIP(hipMemcpy(a.pred_out, S.pred, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (a.kww_out) GK_HIP(hipMemcpy(a.kww_out, S.hK, sizeof(double) * a.s * a.s, hipMemcpyDeviceToHost));
  return call_complete(S, false);
}

void batch_free(BatchCall* B) { delete B; }

}  // namespace gk

// ------------------------------------------------- static scratch (no-alloc)
namespace gk {
namespace {
// Device scratch of the allocation-free entry point: one copy per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel or copy (on the host the name is a stand-in, not a device address);
// it uses the address hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[GK_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on device `dev`, looked up once per device with that
// device current.
void* scratch_on(int dev) {
  GK_REQUIRE(dev >= 0 && dev < kMaxDevices, GK_EDEVICE, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    GK_HIP(hipGetDevice(&cur));
    GK_HIP(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    const hipError_t e2 = hipSetDevice(cur);
    GK_REQUIRE(e == hipSuccess && ptr, GK_EDEVICE,
               std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    GK_HIP(e2);
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace
}  // namespace gk

// ------------------------------------------------------------------ ABI
extern "C" {

static int guarded(const gk::CallArgs& a) {
  try {
    return gk::run_call(a, gk::current_stream());
  } catch (const gk::Error& e) {
    gk::set_detail(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    gk::set_detail("host allocation failed");
    return GK_ENOMEM;
  }
}

int krylov_kernel_columns(gk_graph* g, const int64_t* samples, int32_t s, const gk_phi* phi, int32_t m,
                          int32_t variant, int32_t precision, uint32_t flags, double* cols_out,
                          double* kww_out, gk_stats* st) {
  gk::CallArgs a{g, samples, s, phi, m, variant, precision, flags, nullptr, 0.0, cols_out, kww_out,
                 nullptr, nullptr, st, false};
  return guarded(a);
}

int krylov_kernel_columns_noalloc(gk_graph* g, const int64_t* samples, int32_t s, const gk_phi* phi, int32_t m,
                                  int32_t variant, int32_t precision, uint32_t flags, double* cols_out,
                                  double* kww_out, gk_stats* st) {
  try {
    GK_REQUIRE(g, GK_EINVAL, "graph is NULL");
    GK_REQUIRE((flags & GK_IO_DEVICE) != 0, GK_EINVAL,
               "krylov_kernel_columns_noalloc needs GK_IO_DEVICE (device samples and outputs)");
    GK_REQUIRE(s >= 1 && s <= 1024 && m >= 1 && m <= 4096, GK_EINVAL, "s or m out of range");
    GK_REQUIRE(variant >= GK_CBL && variant <= GK_CHEB2 && (precision == GK_FP64 || precision == GK_MIXED),
               GK_EINVAL, "unknown variant or precision");
    // The request's own buffers (footprint without the host staging of the
    // columns and the general small-buffer allowance) must fit the scratch;
    // the carving itself enforces the exact limit.
    const double need = (double)gk::footprint_bytes(g->n, s, m, variant, precision, flags) -
                        (double)g->n * s * 8.0 - 64.0 * (1 << 20);
    GK_REQUIRE(need <= (double)GK_STATIC_SCRATCH_BYTES, GK_ENOMEM,
               "request needs about " + std::to_string((uint64_t)need) + " bytes, more than the " +
                   std::to_string((uint64_t)GK_STATIC_SCRATCH_BYTES) + " bytes of static device scratch");
    gk::CallArgs a{g, samples, s, phi, m, variant, precision, flags, nullptr, 0.0, cols_out, kww_out,
                   nullptr, nullptr, st, false};
    a.pool = gk::scratch_on(g->device);
    a.pool_cap = GK_STATIC_SCRATCH_BYTES;
    return guarded(a);
  } catch (const gk::Error& e) {
    gk::set_detail(e.msg);
    return e.code;
  }
}

int kernel_machine_fit_predict(gk_graph* g, const int64_t* samples, int32_t s, const double* y,
                               const gk_phi* phi, int32_t m, int32_t variant, int32_t precision,
                               uint32_t flags, double gamma, double* coef_out, double* pred_out,
                               gk_stats* st) {
  gk::CallArgs a{g, samples, s, phi, m, variant, precision, flags, y, gamma, nullptr, nullptr,
                 coef_out, pred_out, st, true};
  return guarded(a);
}

int gk_request_footprint(int64_t n, int32_t s, int32_t m, int32_t variant, int32_t precision, uint32_t flags,
                         uint64_t* bytes) {
  if (!bytes || n < 1 || s < 1 || s > 1024 || m < 1 || m > 4096 || variant < GK_CBL || variant > GK_CHEB2 ||
      (precision != GK_FP64 && precision != GK_MIXED))
    return GK_EINVAL;
  *bytes = gk::footprint_bytes(n, s, m, variant, precision, flags);
  return GK_OK;
}

}  // extern "C"
