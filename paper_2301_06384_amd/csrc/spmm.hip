// CSR SpMM with the Laplacian in difference form, fused three-term epilogue.
//
// The products L*Q_k of Alg. 1 / Alg. 2 (and T_k(I - 2L/Lambda) E_W of the
// Chebyshev recurrence, Sec. 3.4) are the block matrix-vector products
// counted in Table 1.  Blocks are row-major n x ld (ld >= s, zero padded),
// so a neighbour's row is one contiguous ld*8-byte segment: each row of the
// output is owned by ld/VPT consecutive lanes that read VPT doubles of every
// neighbour row as 16-byte vector loads (coalesced gathers).
//
// (L v)_i = d_i v_i - sum_{j != i} w_ij v_j with d_i = sum_j w_ij + c_i
// accumulated in float64; with float32 weights d_i is the float64 sum of the
// rounded weights, so L 1 = c holds for the rounded operator too.
#include "gk_internal.h"

namespace gk {

enum { W_UNIT = 0, W_F64 = 1, W_F32 = 2 };

// A lane moves VPT doubles of a row as VPT / 2 16-byte chunks; chunk q of the
// lane with index r within its row sits at column 2 r + q * cs (cs = twice the
// lanes per row), so each chunk instruction of the row's lanes covers one
// contiguous stretch of the row (whole cache lines) instead of every other
// 16 bytes of all of it.
template <int VPT>
__device__ __forceinline__ void load_row(const double* p, int cs, double (&v)[VPT]) {
#pragma unroll
  for (int q = 0; q < VPT / 2; ++q) {
    const double2 t = *reinterpret_cast<const double2*>(p + q * cs);
    v[2 * q] = t.x;
    v[2 * q + 1] = t.y;
  }
}
template <int VPT>
__device__ __forceinline__ void store_row(double* p, int cs, const double (&v)[VPT]) {
#pragma unroll
  for (int q = 0; q < VPT / 2; ++q) *reinterpret_cast<double2*>(p + q * cs) = make_double2(v[2 * q], v[2 * q + 1]);
}

// Rows of workgroup `bid` of a grid of G workgroups (block index and grid
// size are those of the request's own launch, also inside a grouped launch).
template <int VPT, int WM, bool SHFL>
__device__ __forceinline__ void
spmm_diff_body(unsigned bid, unsigned G, int64_t n, int ld, const int32_t* __restrict__ rp,
               const int32_t* __restrict__ ci, const double* __restrict__ w64, const float* __restrict__ w32,
               const double* __restrict__ d, const double* __restrict__ V, const double* __restrict__ Vprev,
               double* __restrict__ out, double a, double b, double gm, double* __restrict__ acc, double e,
               const double* __restrict__ e_dev) {
  const int slots = ld / VPT;
  // Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
  // Renumber them so that every XCD walks one contiguous range of rows: with
  // a locality ordering of the nodes, the neighbour rows it gathers are then
  // mostly fetched into one L2 instead of several.
  const unsigned q8 = G >> 3, r8 = G & 7;
  const unsigned x = bid & 7, k = bid >> 3;
  const unsigned lb = x * q8 + (x < r8 ? x : r8) + k;
  const int64_t t = (int64_t)lb * blockDim.x + threadIdx.x;
  const int64_t row = t / slots;
  if (row >= n) return;
  const int lr = (int)(t - row * slots);   // lane index within the row
  const int c0 = 2 * lr, cs = 2 * slots;
  double s[VPT];
#pragma unroll
  for (int q = 0; q < VPT; ++q) s[q] = 0.0;
  const int p0 = rp[row], p1 = rp[row + 1];
  if (SHFL) {
    // The lanes of a row (a power of two dividing 64, so a row never straddles
    // wavefronts) load `slots` column indices and weights at once, then walk
    // them with lane shuffles, four gathers in flight.
    const int gbase = (int)(threadIdx.x & 63) - lr;
    for (int pc = p0; pc < p1; pc += slots) {
      const int pp = pc + lr;
      int myj = 0;
      double myw = 0.0;
      if (pp < p1) {
        myj = ci[pp];
        myw = (WM == W_F64) ? w64[pp] : (WM == W_F32 ? (double)w32[pp] : 1.0);
      }
      const int cnt = min(slots, p1 - pc);
      int k = 0;
      for (; k + 3 < cnt; k += 4) {
        int j[4];
        double w[4], v[4][VPT];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          j[u] = __shfl(myj, gbase + k + u);
          w[u] = __shfl(myw, gbase + k + u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) load_row<VPT>(V + (int64_t)j[u] * ld + c0, cs, v[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int q = 0; q < VPT; ++q) s[q] = fma(w[u], v[u][q], s[q]);
      }
      for (; k < cnt; ++k) {
        const int j0 = __shfl(myj, gbase + k);
        const double w0 = __shfl(myw, gbase + k);
        double v0[VPT];
        load_row<VPT>(V + (int64_t)j0 * ld + c0, cs, v0);
#pragma unroll
        for (int q = 0; q < VPT; ++q) s[q] = fma(w0, v0[q], s[q]);
      }
    }
  } else {
    int p = p0;
    // two neighbours per iteration to keep two gathers in flight
    for (; p + 1 < p1; p += 2) {
      const int j0 = ci[p], j1 = ci[p + 1];
      double w0 = 1.0, w1 = 1.0;
      if (WM == W_F64) { w0 = w64[p]; w1 = w64[p + 1]; }
      if (WM == W_F32) { w0 = (double)w32[p]; w1 = (double)w32[p + 1]; }
      double v0[VPT], v1[VPT];
      load_row<VPT>(V + (int64_t)j0 * ld + c0, cs, v0);
      load_row<VPT>(V + (int64_t)j1 * ld + c0, cs, v1);
#pragma unroll
      for (int q = 0; q < VPT; ++q) s[q] = fma(w0, v0[q], fma(w1, v1[q], s[q]));
    }
    if (p < p1) {
      const int j0 = ci[p];
      double w0 = 1.0;
      if (WM == W_F64) w0 = w64[p];
      if (WM == W_F32) w0 = (double)w32[p];
      double v0[VPT];
      load_row<VPT>(V + (int64_t)j0 * ld + c0, cs, v0);
#pragma unroll
      for (int q = 0; q < VPT; ++q) s[q] = fma(w0, v0[q], s[q]);
    }
  }
  double vi[VPT], o[VPT];
  load_row<VPT>(V + row * ld + c0, cs, vi);
  const double di = d[row];
#pragma unroll
  for (int q = 0; q < VPT; ++q) o[q] = a * (di * vi[q] - s[q]) + b * vi[q];
  if (Vprev) {
    double vp[VPT];
    load_row<VPT>(Vprev + row * ld + c0, cs, vp);
#pragma unroll
    for (int q = 0; q < VPT; ++q) o[q] += gm * vp[q];
  }
  store_row<VPT>(out + row * ld + c0, cs, o);
  if (acc) {
    if (e_dev) e = *e_dev;
    double ac[VPT];
    load_row<VPT>(acc + row * ld + c0, cs, ac);
#pragma unroll
    for (int q = 0; q < VPT; ++q) ac[q] = fma(e, o[q], ac[q]);
    store_row<VPT>(acc + row * ld + c0, cs, ac);
  }
}

template <int VPT, int WM, bool SHFL>
__global__ void __launch_bounds__(256)
spmm_diff_kernel(int64_t n, int ld, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                 const double* __restrict__ w64, const float* __restrict__ w32,
                 const double* __restrict__ d, const double* __restrict__ V,
                 const double* __restrict__ Vprev, double* __restrict__ out, double a, double b,
                 double gm, double* __restrict__ acc, double e, const double* __restrict__ e_dev) {
  spmm_diff_body<VPT, WM, SHFL>(blockIdx.x, gridDim.x, n, ld, rp, ci, w64, w32, d, V, Vprev, out, a, b, gm, acc,
                                e, e_dev);
}

// Lane layout of a block width: VPT doubles per lane (ld/VPT lanes per row),
// and whether the row's lanes walk the neighbour list with shuffles.
static inline int spmm_vpt(int ld) { return ld <= 32 ? 2 : (ld <= 256 ? 4 : 8); }
static inline bool spmm_shfl(int ld) {
  const int slots = ld / spmm_vpt(ld);
  return slots <= 64 && (64 % slots) == 0;
}
static inline int64_t spmm_grid(int64_t n, int ld) { return (n * (ld / spmm_vpt(ld)) + 255) / 256; }

// One launch for the products X_r = L V_r of several requests on the same
// graph (their blocks side by side: the concatenated column segments).
// Workgroups [start_r, start_{r+1}) belong to request r and run exactly the
// workgroups of its lone launch, with its own lane layout.
struct SpmmGroupArgs {
  int count;
  int start[kSpmmGroup + 1];
  int ld[kSpmmGroup];
  const double* V[kSpmmGroup];
  double* X[kSpmmGroup];
};
template <int WM>
__global__ void __launch_bounds__(256)
spmm_group_kernel(SpmmGroupArgs ga, int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                  const double* __restrict__ w64, const float* __restrict__ w32, const double* __restrict__ d) {
  int r = 0;
  while (r + 1 < ga.count && (int)blockIdx.x >= ga.start[r + 1]) ++r;
  const unsigned bid = blockIdx.x - ga.start[r], G = ga.start[r + 1] - ga.start[r];
  const int ld = ga.ld[r];
  const int vpt = ld <= 32 ? 2 : (ld <= 256 ? 4 : 8);
  const int slots = ld / vpt;
  const bool sh = slots <= 64 && (64 % slots) == 0;
#define GK_SPB(V_, S_)                                                                                            \
  spmm_diff_body<V_, WM, S_>(bid, G, n, ld, rp, ci, w64, w32, d, ga.V[r], nullptr, ga.X[r], 1.0, 0.0, 0.0, nullptr, \
                             0.0, nullptr)
  if (vpt == 2) {
    if (sh) GK_SPB(2, true); else GK_SPB(2, false);
  } else if (vpt == 4) {
    if (sh) GK_SPB(4, true); else GK_SPB(4, false);
  } else {
    if (sh) GK_SPB(8, true); else GK_SPB(8, false);
  }
#undef GK_SPB
}

void launch_spmm_group(const gk_graph* g, bool fp32_weights, int count, const int* ld, const double* const* V,
                       double* const* X, hipStream_t st) {
  const double wb = g->unit ? 0.0 : (fp32_weights ? 4.0 : 8.0);
  const double* d = fp32_weights ? g->d32 : g->d64;
  for (int c0 = 0; c0 < count; c0 += kSpmmGroup) {
    SpmmGroupArgs ga{};
    ga.count = std::min(kSpmmGroup, count - c0);
    double bytes = 0, flops = 0;
    int64_t tot = 0;
    for (int i = 0; i < ga.count; ++i) {
      ga.start[i] = (int)tot;
      ga.ld[i] = ld[c0 + i];
      ga.V[i] = V[c0 + i];
      ga.X[i] = X[c0 + i];
      tot += spmm_grid(g->n, ld[c0 + i]);
      bytes += 4.0 * (g->n + 1) + (double)g->nnz * (4.0 + wb) + 8.0 * g->n + 16.0 * (double)g->n * ld[c0 + i];
      flops += 2.0 * ((double)g->nnz + g->n) * ld[c0 + i];
    }
    ga.start[ga.count] = (int)tot;
    kt_begin(KC_SPMM, st);
    if (g->unit)
      hipLaunchKernelGGL(spmm_group_kernel<W_UNIT>, dim3((unsigned)tot), dim3(256), 0, st, ga, g->n, g->rp, g->ci,
                         g->w64, g->w32, d);
    else if (fp32_weights)
      hipLaunchKernelGGL(spmm_group_kernel<W_F32>, dim3((unsigned)tot), dim3(256), 0, st, ga, g->n, g->rp, g->ci,
                         g->w64, g->w32, d);
    else
      hipLaunchKernelGGL(spmm_group_kernel<W_F64>, dim3((unsigned)tot), dim3(256), 0, st, ga, g->n, g->rp, g->ci,
                         g->w64, g->w32, d);
    GK_HIP(hipGetLastError());
    kt_end(st, bytes, flops);
  }
}

template <int VPT>
static void spmm_dispatch_w(const gk_graph* g, bool fp32w, int ld, const double* V, const double* Vp,
                            double* out, double a, double b, double gm, double* acc, double e,
                            const double* e_dev, hipStream_t st) {
  const int slots = ld / VPT;
  const int64_t threads = g->n * slots;
  const int bs = 256;
  const int64_t grid = (threads + bs - 1) / bs;
  const double* d = fp32w ? g->d32 : g->d64;
  const bool shfl = slots <= 64 && (64 % slots) == 0;
#define GK_SPMM(WM_, SH_)                                                                                   \
  hipLaunchKernelGGL((spmm_diff_kernel<VPT, WM_, SH_>), dim3((unsigned)grid), dim3(bs), 0, st, g->n, ld, g->rp, \
                     g->ci, g->w64, g->w32, d, V, Vp, out, a, b, gm, acc, e, e_dev)
  if (g->unit) {
    if (shfl) GK_SPMM(W_UNIT, true); else GK_SPMM(W_UNIT, false);
  } else if (fp32w) {
    if (shfl) GK_SPMM(W_F32, true); else GK_SPMM(W_F32, false);
  } else {
    if (shfl) GK_SPMM(W_F64, true); else GK_SPMM(W_F64, false);
  }
#undef GK_SPMM
  GK_HIP(hipGetLastError());
}

void launch_spmm(const gk_graph* g, bool fp32_weights, int ld, const double* V, const double* Vprev,
                 double* out, double a, double b, double gmul, double* acc, double e, const double* e_dev,
                 hipStream_t st) {
  // algorithmic traffic: CSR structure, weights, diagonal, V (and V_prev) in, out
  const double wb = g->unit ? 0.0 : (fp32_weights ? 4.0 : 8.0);
  const double vb = 8.0 * (double)g->n * ld;
  kt_begin(KC_SPMM, st);
  // lanes per row: at most 64 (one wavefront), VPT doubles each
  // (16 lanes per row at ld = 64: 4 doubles each measured faster than 2 or 8)
  if (ld <= 32) {
    spmm_dispatch_w<2>(g, fp32_weights, ld, V, Vprev, out, a, b, gmul, acc, e, e_dev, st);
  } else if (ld <= 256) {
    spmm_dispatch_w<4>(g, fp32_weights, ld, V, Vprev, out, a, b, gmul, acc, e, e_dev, st);
  } else {
    // ld is a multiple of 16; 8 doubles per lane
    spmm_dispatch_w<8>(g, fp32_weights, ld, V, Vprev, out, a, b, gmul, acc, e, e_dev, st);
  }
  kt_end(st, 4.0 * (g->n + 1) + (double)g->nnz * (4.0 + wb) + 8.0 * g->n + vb * (Vprev ? 3.0 : 2.0),
         2.0 * ((double)g->nnz + g->n) * ld);
}

}  // namespace gk
