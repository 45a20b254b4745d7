// CSR SpMM with the Laplacian in difference form, fused three-term epilogue.
//
// The products L*Q_k of Alg. 1 / Alg. 2 (and T_k(I - 2L/Lambda) E_W of the
// Chebyshev recurrence, Sec. 3.4) are the block matrix-vector products
// counted in Table 1.  Blocks are row-major n x ld (ld >= s, zero padded),
// so a neighbour's row is one contiguous ld*8-byte segment.  The product is
// formed over column strips of width ws (ld, or 64 for wider blocks that are
// multiples of 64, one strip after the other): each row of a strip is owned
// by ws/VPT consecutive lanes that read VPT doubles of every neighbour's
// segment as 16-byte vector loads (coalesced gathers).  The rows are split
// among the 8 XCDs by cost, and rows with very many entries (hub rows) are
// summed by a workgroup of their own.
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

// The graph's row split and hub rows, passed by value to the product kernels.
struct SpmmGraph {
  int64_t r[9];           // rows [r[x], r[x+1]) are XCD x's (gk_graph::xr)
  const int32_t* hub;     // rows with more than hub_min off-diagonal entries
  int nhub, hub_min;
};
static inline SpmmGraph spmm_graph(const gk_graph* g) {
  SpmmGraph s;
  for (int i = 0; i < 9; ++i) s.r[i] = g->xr[i];
  s.hub = g->hub;
  s.nhub = (int)g->nhub;
  s.hub_min = g->hub_min;
  return s;
}
// Workgroups per XCD for `rows_per_unit` rows each: the widest range decides.
static inline int64_t xcd_units(const gk_graph* g, int64_t rows_per_unit) {
  int64_t u = 0;
  for (int x = 0; x < 8; ++x) u = std::max(u, (g->xr[x + 1] - g->xr[x] + rows_per_unit - 1) / rows_per_unit);
  return u;
}

// Lane layout of a (strip) width: VPT doubles per lane (ws/VPT lanes per
// row), and whether the row's lanes walk the neighbour list with shuffles.
__host__ __device__ inline int spmm_vpt(int ws) { return ws <= 32 ? 2 : (ws <= 256 ? 4 : 8); }
__host__ __device__ inline bool spmm_shfl(int ws) {
  const int slots = ws / spmm_vpt(ws);
  return slots <= 64 && (64 % slots) == 0;
}
// Strip width of the product: blocks wider than 64 (multiples of 64) are
// computed in 64-column strips with the 16-lane layout of a 64-wide block,
// one strip after the other over the whole graph.  Four rows per wavefront
// gather 512-byte segments instead of one row gathering 2-4 KB ones; the
// bytes fetched stay the same (the strips' CSR re-reads aside).
static inline int spmm_strip(int ld) { return (ld > 64 && ld % 64 == 0) ? 64 : ld; }

// Launch shape of the product of one block: strip width ws (ld / ws strips);
// per strip, hub8 workgroups for the hub rows (one each; the hub count
// rounded up to a multiple of 8) and then 8 * units workgroups for the other
// rows, per_strip in all.
struct SpmmShape {
  int ld, ws, hub8, per_strip;
};
constexpr int64_t kMaxSpmmGrid = int64_t(1) << 24;   // workgroups of 256 lanes: < 2^32 lanes
static inline int64_t spmm_workgroups(const SpmmShape& s) { return (int64_t)s.per_strip * (s.ld / s.ws); }
static inline SpmmShape spmm_shape(const gk_graph* g, int ld) {
  SpmmShape s;
  s.ld = ld;
  s.hub8 = (int)((g->nhub + 7) / 8 * 8);
  for (int ws : {spmm_strip(ld), ld}) {   // whole rows if strips would not fit one grid
    s.ws = ws;
    s.per_strip = (int)std::min<int64_t>(kMaxSpmmGrid, s.hub8 + 8 * xcd_units(g, 256 / (ws / spmm_vpt(ws))));
    if (spmm_workgroups(s) < kMaxSpmmGrid) break;
  }
  GK_REQUIRE(spmm_workgroups(s) < kMaxSpmmGrid, GK_EUNSUPPORTED, "graph too large for one product launch");
  return s;
}

// s[q] += w_ij V[j, c0 + ...] over the entries [pa, pb) of a row's
// neighbour list, in list order, by the row's slots lanes (lane lr; gbase is
// the wavefront lane of the row's lane 0).
template <int VPT, int WM, bool SHFL>
__device__ __forceinline__ void gather_sum(int pa, int pb, int slots, int lr, int gbase, int ld, int c0, int cs,
                                           const int32_t* __restrict__ ci, const double* __restrict__ w64,
                                           const float* __restrict__ w32, const double* __restrict__ V,
                                           double (&s)[VPT]) {
  if (SHFL) {
    // The lanes of a row (a power of two dividing 64, so a row never straddles
    // wavefronts) load `slots` column indices and weights at once, then walk
    // them with lane shuffles, four gathers in flight.
    for (int pc = pa; pc < pb; pc += slots) {
      const int pp = pc + lr;
      int myj = 0;
      double myw = 0.0;
      if (pp < pb) {
        myj = ci[pp];
        myw = (WM == W_F64) ? w64[pp] : (WM == W_F32 ? (double)w32[pp] : 1.0);
      }
      const int cnt = min(slots, pb - pc);
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
    int p = pa;
    // two neighbours per iteration to keep two gathers in flight
    for (; p + 1 < pb; p += 2) {
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
    if (p < pb) {
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
}

// out = a (d_i v_i - s) + b v_i (+ gm vprev_i), acc += e out, for the lane's
// columns of row `row`.
template <int VPT>
__device__ __forceinline__ void spmm_epilogue(int64_t row, int ld, int c0, int cs, const double (&s)[VPT],
                                              const double* __restrict__ d, const double* __restrict__ V,
                                              const double* __restrict__ Vprev, double* __restrict__ out, double a,
                                              double b, double gm, double* __restrict__ acc, double e,
                                              const double* __restrict__ e_dev) {
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

// Ordinary rows of workgroup `bid` of a strip.  Workgroups are dealt
// round-robin to the 8 XCDs, each with its own L2: workgroup bid runs on XCD
// bid % 8 and takes the (bid / 8)-th run of rows of that XCD's range, so
// every XCD walks one contiguous, cost-balanced range of rows and, with a
// locality ordering of the nodes, gathers mostly through its own L2.  A row's
// slots lanes never straddle workgroups (256 / slots rows per workgroup;
// lanes beyond them idle).  Columns [cb, cb + ws) of rows of stride ld.
// Each output element is the float64 sum over the row's entries in CSR
// order, whatever ws and cb are.  Hub rows are left to their workgroups.
template <int VPT, int WM, bool SHFL>
__device__ __forceinline__ void
spmm_rows_body(unsigned bid, const SpmmGraph& sg, int ld, int ws, int cb, const int32_t* __restrict__ rp,
               const int32_t* __restrict__ ci, const double* __restrict__ w64, const float* __restrict__ w32,
               const double* __restrict__ d, const double* __restrict__ V, const double* __restrict__ Vprev,
               double* __restrict__ out, double a, double b, double gm, double* __restrict__ acc, double e,
               const double* __restrict__ e_dev) {
  const int slots = ws / VPT;
  const int rpw = (int)blockDim.x / slots;
  const int rin = (int)threadIdx.x / slots;
  const unsigned x = bid & 7, k = bid >> 3;
  const int64_t row = sg.r[x] + (int64_t)k * rpw + rin;
  if (rin >= rpw || row >= sg.r[x + 1]) return;
  const int p0 = rp[row], p1 = rp[row + 1];
  if (p1 - p0 > sg.hub_min) return;
  const int lr = (int)threadIdx.x - rin * slots;   // lane index within the row
  const int c0 = cb + 2 * lr, cs = 2 * slots;
  double s[VPT];
#pragma unroll
  for (int q = 0; q < VPT; ++q) s[q] = 0.0;
  gather_sum<VPT, WM, SHFL>(p0, p1, slots, lr, (int)(threadIdx.x & 63) - lr, ld, c0, cs, ci, w64, w32, V, s);
  spmm_epilogue<VPT>(row, ld, c0, cs, s, d, V, Vprev, out, a, b, gm, acc, e, e_dev);
}

// Hub row h (more than hub_min entries) of a strip, by a whole workgroup:
// its G = 256 / slots lane groups take consecutive equal segments of the
// neighbour list, and the segment sums are added in segment order through
// LDS (a fixed order: the result depends on the strip width only).
template <int VPT, int WM, bool SHFL>
__device__ __forceinline__ void
spmm_hub_body(unsigned h, const SpmmGraph& sg, int ld, int ws, int cb, const int32_t* __restrict__ rp,
              const int32_t* __restrict__ ci, const double* __restrict__ w64, const float* __restrict__ w32,
              const double* __restrict__ d, const double* __restrict__ V, const double* __restrict__ Vprev,
              double* __restrict__ out, double a, double b, double gm, double* __restrict__ acc, double e,
              const double* __restrict__ e_dev) {
  __shared__ double red[256 * VPT];
  if ((int)h >= sg.nhub) return;   // the whole workgroup
  const int slots = ws / VPT, G = (int)blockDim.x / slots;
  const int grp = (int)threadIdx.x / slots, lr = (int)threadIdx.x - grp * slots;
  const int64_t row = sg.hub[h];
  const int p0 = rp[row], p1 = rp[row + 1];
  const int seg = (p1 - p0 + G - 1) / G;
  const int c0 = cb + 2 * lr, cs = 2 * slots;
  if (grp < G) {
    double s[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) s[q] = 0.0;
    const int pa = min(p1, p0 + grp * seg), pb = min(p1, pa + seg);
    gather_sum<VPT, WM, SHFL>(pa, pb, slots, lr, (int)(threadIdx.x & 63) - lr, ld, c0, cs, ci, w64, w32, V, s);
#pragma unroll
    for (int q = 0; q < VPT; ++q) red[(grp * slots + lr) * VPT + q] = s[q];
  }
  __syncthreads();
  if (grp == 0) {
    double t[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) t[q] = red[lr * VPT + q];
    for (int g = 1; g < G; ++g)
#pragma unroll
      for (int q = 0; q < VPT; ++q) t[q] += red[(g * slots + lr) * VPT + q];
    spmm_epilogue<VPT>(row, ld, c0, cs, t, d, V, Vprev, out, a, b, gm, acc, e, e_dev);
  }
}

// Workgroup w of the product of one block (index within the block's own
// launch, also inside a grouped launch): strip w / per_strip, hub rows first.
// per_strip and hub8 are multiples of 8, so the XCD of w (w % 8) is the XCD
// of its run of rows.
template <int VPT, int WM, bool SHFL>
__device__ __forceinline__ void
spmm_block_wg(unsigned w, const SpmmShape& sh, const SpmmGraph& sg, const int32_t* __restrict__ rp,
              const int32_t* __restrict__ ci, const double* __restrict__ w64, const float* __restrict__ w32,
              const double* __restrict__ d, const double* __restrict__ V, const double* __restrict__ Vprev,
              double* __restrict__ out, double a, double b, double gm, double* __restrict__ acc, double e,
              const double* __restrict__ e_dev) {
  const unsigned strip = w / (unsigned)sh.per_strip, u = w - strip * (unsigned)sh.per_strip;
  const int cb = (int)strip * sh.ws;
  if ((int)u < sh.hub8)
    spmm_hub_body<VPT, WM, SHFL>(u, sg, sh.ld, sh.ws, cb, rp, ci, w64, w32, d, V, Vprev, out, a, b, gm, acc, e,
                                 e_dev);
  else
    spmm_rows_body<VPT, WM, SHFL>(u - sh.hub8, sg, sh.ld, sh.ws, cb, rp, ci, w64, w32, d, V, Vprev, out, a, b, gm,
                                  acc, e, e_dev);
}

template <int VPT, int WM, bool SHFL>
__global__ void __launch_bounds__(256)
spmm_diff_kernel(SpmmShape sh, SpmmGraph sg, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                 const double* __restrict__ w64, const float* __restrict__ w32,
                 const double* __restrict__ d, const double* __restrict__ V,
                 const double* __restrict__ Vprev, double* __restrict__ out, double a, double b,
                 double gm, double* __restrict__ acc, double e, const double* __restrict__ e_dev) {
  spmm_block_wg<VPT, WM, SHFL>(blockIdx.x, sh, sg, rp, ci, w64, w32, d, V, Vprev, out, a, b, gm, acc, e, e_dev);
}

// One launch for the products X_r = L V_r of several requests on the same
// graph (their blocks side by side: the concatenated column segments).
// Workgroups [start_r, start_{r+1}) belong to request r and run exactly the
// workgroups of its lone launch, with its own shape.
struct SpmmGroupArgs {
  int count;
  int start[kSpmmGroup + 1];
  SpmmShape sh[kSpmmGroup];
  const double* V[kSpmmGroup];
  double* X[kSpmmGroup];
};
template <int WM>
__global__ void __launch_bounds__(256)
spmm_group_kernel(SpmmGroupArgs ga, SpmmGraph sg, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                  const double* __restrict__ w64, const float* __restrict__ w32, const double* __restrict__ d) {
  int r = 0;
  while (r + 1 < ga.count && (int)blockIdx.x >= ga.start[r + 1]) ++r;
  const unsigned w = blockIdx.x - ga.start[r];
  const SpmmShape sh = ga.sh[r];
  const int vpt = spmm_vpt(sh.ws);
  const bool shf = spmm_shfl(sh.ws);
#define GK_SPB(V_, S_) \
  spmm_block_wg<V_, WM, S_>(w, sh, sg, rp, ci, w64, w32, d, ga.V[r], nullptr, ga.X[r], 1.0, 0.0, 0.0, nullptr, 0.0, nullptr)
  if (vpt == 2) {
    if (shf) GK_SPB(2, true); else GK_SPB(2, false);
  } else if (vpt == 4) {
    if (shf) GK_SPB(4, true); else GK_SPB(4, false);
  } else {
    if (shf) GK_SPB(8, true); else GK_SPB(8, false);
  }
#undef GK_SPB
}

void launch_spmm_group(const gk_graph* g, bool fp32_weights, int count, const int* ld, const double* const* V,
                       double* const* X, hipStream_t st) {
  const double wb = g->unit ? 0.0 : (fp32_weights ? 4.0 : 8.0);
  const double* d = fp32_weights ? g->d32 : g->d64;
  const SpmmGraph sg = spmm_graph(g);
  for (int c0 = 0; c0 < count; c0 += kSpmmGroup) {
    SpmmGroupArgs ga{};
    ga.count = std::min(kSpmmGroup, count - c0);
    double bytes = 0, flops = 0;
    int64_t tot = 0;
    for (int i = 0; i < ga.count; ++i) {
      ga.start[i] = (int)tot;
      ga.sh[i] = spmm_shape(g, ld[c0 + i]);
      ga.V[i] = V[c0 + i];
      ga.X[i] = X[c0 + i];
      tot += spmm_workgroups(ga.sh[i]);
      bytes += 4.0 * (g->n + 1) + (double)g->nnz * (4.0 + wb) + 8.0 * g->n + 16.0 * (double)g->n * ld[c0 + i];
      flops += 2.0 * ((double)g->nnz + g->n) * ld[c0 + i];
    }
    GK_REQUIRE(tot < kMaxSpmmGrid, GK_EUNSUPPORTED, "grouped product too large for one launch");
    ga.start[ga.count] = (int)tot;
    kt_begin(KC_SPMM, st);
    if (g->unit)
      hipLaunchKernelGGL(spmm_group_kernel<W_UNIT>, dim3((unsigned)tot), dim3(256), 0, st, ga, sg, g->rp, g->ci,
                         g->w64, g->w32, d);
    else if (fp32_weights)
      hipLaunchKernelGGL(spmm_group_kernel<W_F32>, dim3((unsigned)tot), dim3(256), 0, st, ga, sg, g->rp, g->ci,
                         g->w64, g->w32, d);
    else
      hipLaunchKernelGGL(spmm_group_kernel<W_F64>, dim3((unsigned)tot), dim3(256), 0, st, ga, sg, g->rp, g->ci,
                         g->w64, g->w32, d);
    GK_HIP(hipGetLastError());
    kt_end(st, bytes, flops);
  }
}

// ------------------------------------------- X = L V with C = V^T X fused
// For 64-wide blocks: the product X = L V (as spmm_diff_body, 16 lanes per
// row, 4 doubles each, the same summation order) and the Gram C = V^T X of
// the three-term recurrence (H_kk = Q_k^T L Q_k, symmetric, so only its
// 16 x 16 tiles on and above the diagonal) in one pass: each workgroup
// computes 32 rows of X at a time, writes them out and stages them with the
// rows of V (already loaded for the diagonal term) in LDS, and its eight
// wavefronts accumulate the ten upper tiles of C on FP64 matrix cores
// (v_mfma_f64_16x16x4f64: lane l = i + 16 k holds A[i][k] and B[k][i],
// accumulator register r holds D[4 r + k][i]).  Partials: one 64 x 64
// upper-tile set per workgroup, reduced (and mirrored) in float64 in a fixed
// order by launch_reduce_parts.  (Walking two rows per lane group doubles
// the gathers in flight per wavefront but, at 152 VGPRs, halves the
// wavefronts per CU: no faster.)
constexpr int SG_THREADS = 512;   // 32 rows of 16 lanes
constexpr int SG_ROWS = 32;
constexpr int SG_P = 66;          // LDS pitch (doubles)
constexpr int SG_MAXGRID = 512;   // two workgroups per CU
typedef double sg_d4 __attribute__((ext_vector_type(4)));

template <int WM>
__device__ __forceinline__ double sg_weight(const double* __restrict__ w64, const float* __restrict__ w32, int p) {
  return (WM == W_F64) ? w64[p] : (WM == W_F32 ? (double)w32[p] : 1.0);
}

template <int WM>
__global__ void __launch_bounds__(SG_THREADS, 2)
spmm_gram64_kernel(int64_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                   const double* __restrict__ w64, const float* __restrict__ w32, const double* __restrict__ d,
                   const double* __restrict__ V, double* __restrict__ out, double* __restrict__ part, SpmmGraph xr) {
  constexpr int LD = 64, VPT = 4, SLOTS = 16, CS = 32;
  __shared__ __align__(16) double sX[SG_ROWS * SG_P];
  __shared__ __align__(16) double sV[SG_ROWS * SG_P];
  const int tid = threadIdx.x;
  const int g = tid >> 4, lr = tid & 15;
  const int c0 = 2 * lr;
  const int gbase = (tid & 63) - lr;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  // upper tiles (gi <= xj) of the 4 x 4 tile grid: wavefront w owns tile w
  // and, for w < 2, tile w + 8
  int tgi[2] = {-1, -1}, txj[2] = {-1, -1};
  {
    int cnt = 0;
    for (int i = 0; i < 4; ++i)
      for (int j = i; j < 4; ++j) {
        if (cnt == w) { tgi[0] = i; txj[0] = j; }
        if (cnt == w + 8) { tgi[1] = i; txj[1] = j; }
        ++cnt;
      }
  }
  sg_d4 acc[2] = {sg_d4{0.0, 0.0, 0.0, 0.0}, sg_d4{0.0, 0.0, 0.0, 0.0}};
  // each XCD (workgroups are dealt round-robin to the 8 XCDs; the grid is a
  // multiple of 8) walks the row tiles of its own range of the graph's
  // cost-balanced split, as the plain product does
  const unsigned x = blockIdx.x & 7, kx = blockIdx.x >> 3, gx = gridDim.x >> 3;
  const int64_t rb = xr.r[x], re = xr.r[x + 1];
  const int64_t ntiles = (re - rb + SG_ROWS - 1) / SG_ROWS;
  for (int64_t tile = kx; tile < ntiles; tile += gx) {
    const int64_t row = rb + tile * SG_ROWS + g;
    double o[VPT], vi[VPT];
    if (row < re) {
      double sacc[VPT];
#pragma unroll
      for (int q = 0; q < VPT; ++q) sacc[q] = 0.0;
      const int p0 = rp[row], p1 = rp[row + 1];
      for (int pc = p0; pc < p1; pc += SLOTS) {
        const int pp = pc + lr;
        int myj = 0;
        double myw = 0.0;
        if (pp < p1) {
          myj = ci[pp];
          myw = sg_weight<WM>(w64, w32, pp);
        }
        const int cnt = min(SLOTS, p1 - pc);
        int k = 0;
        for (; k + 3 < cnt; k += 4) {
          int j[4];
          double wv[4], v[4][VPT];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            j[u] = __shfl(myj, gbase + k + u);
            wv[u] = __shfl(myw, gbase + k + u);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) load_row<VPT>(V + (int64_t)j[u] * LD + c0, CS, v[u]);
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int q = 0; q < VPT; ++q) sacc[q] = fma(wv[u], v[u][q], sacc[q]);
        }
        for (; k < cnt; ++k) {
          const int j0 = __shfl(myj, gbase + k);
          const double w0 = __shfl(myw, gbase + k);
          double v0[VPT];
          load_row<VPT>(V + (int64_t)j0 * LD + c0, CS, v0);
#pragma unroll
          for (int q = 0; q < VPT; ++q) sacc[q] = fma(w0, v0[q], sacc[q]);
        }
      }
      load_row<VPT>(V + row * LD + c0, CS, vi);
      const double di = d[row];
#pragma unroll
      for (int q = 0; q < VPT; ++q) o[q] = di * vi[q] - sacc[q];
      store_row<VPT>(out + row * LD + c0, CS, o);
    } else {
#pragma unroll
      for (int q = 0; q < VPT; ++q) o[q] = vi[q] = 0.0;
    }
    // lane lr of row g holds columns 2 lr, 2 lr + 1, 2 lr + 32, 2 lr + 33
#pragma unroll
    for (int q = 0; q < VPT / 2; ++q) {
      *reinterpret_cast<double2*>(&sX[g * SG_P + c0 + q * CS]) = make_double2(o[2 * q], o[2 * q + 1]);
      *reinterpret_cast<double2*>(&sV[g * SG_P + c0 + q * CS]) = make_double2(vi[2 * q], vi[2 * q + 1]);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int gi = tgi[t], xj = txj[t];
      if (gi >= 0) {
#pragma unroll
        for (int k0 = 0; k0 < SG_ROWS; k0 += 4) {
          // rows read together by half a wavefront are 8 apart (as in the
          // panel kernels): 8 SG_P = 16 mod 32 double banks
          const int rr = (k0 & ~15) + ((k0 & 15) >> 2) + 8 * (lk & 1) + 4 * (lk >> 1);
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(sV[rr * SG_P + 16 * gi + li], sX[rr * SG_P + 16 * xj + li],
                                                        acc[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  double* P0 = part + (int64_t)blockIdx.x * LD * LD;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int gi = tgi[t], xj = txj[t];
    if (gi >= 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) P0[(16 * gi + 4 * r + lk) * LD + 16 * xj + li] = acc[t][r];
    }
  }
}

int spmm_gram64_grid(const gk_graph* g) {
  return (int)std::min<int64_t>(8 * xcd_units(g, SG_ROWS), SG_MAXGRID);
}
size_t spmm_gram64_scratch_elems(int64_t n) {
  // a range of the split holds at most n rows
  return (size_t)std::min<int64_t>(8 * ((n + SG_ROWS - 1) / SG_ROWS), SG_MAXGRID) * 64 * 64;
}

void launch_spmm_gram64(const gk_graph* g, bool fp32_weights, const double* V, double* X, double* part, double* C,
                        hipStream_t st) {
  const int grid = spmm_gram64_grid(g);
  const SpmmGraph xr = spmm_graph(g);
  const double wb = g->unit ? 0.0 : (fp32_weights ? 4.0 : 8.0);
  const double* d = fp32_weights ? g->d32 : g->d64;
  kt_begin(KC_SPMM, st);
  if (g->unit)
    hipLaunchKernelGGL(spmm_gram64_kernel<W_UNIT>, dim3(grid), dim3(SG_THREADS), 0, st, g->n, g->rp, g->ci, g->w64,
                       g->w32, d, V, X, part, xr);
  else if (fp32_weights)
    hipLaunchKernelGGL(spmm_gram64_kernel<W_F32>, dim3(grid), dim3(SG_THREADS), 0, st, g->n, g->rp, g->ci, g->w64,
                       g->w32, d, V, X, part, xr);
  else
    hipLaunchKernelGGL(spmm_gram64_kernel<W_F64>, dim3(grid), dim3(SG_THREADS), 0, st, g->n, g->rp, g->ci, g->w64,
                       g->w32, d, V, X, part, xr);
  GK_HIP(hipGetLastError());
  // the product's own traffic (the Gram reads nothing more); flops of both
  kt_end(st, 4.0 * (g->n + 1) + (double)g->nnz * (4.0 + wb) + 8.0 * g->n + 2.0 * 8.0 * g->n * 64,
         2.0 * ((double)g->nnz + g->n) * 64 + (double)g->n * 64 * 65);
  launch_reduce_parts((int64_t)64 * 64, grid, part, C, nullptr, st, 64, 16);
}

template <int VPT>
static void spmm_dispatch_w(const gk_graph* g, bool fp32w, const SpmmShape& sh, const double* V, const double* Vp,
                            double* out, double a, double b, double gm, double* acc, double e,
                            const double* e_dev, hipStream_t st) {
  const int64_t grid = spmm_workgroups(sh);
  if (grid == 0) return;
  const SpmmGraph sg = spmm_graph(g);
  const double* d = fp32w ? g->d32 : g->d64;
  const bool shfl = spmm_shfl(sh.ws);
#define GK_SPMM(WM_, SH_)                                                                                         \
  hipLaunchKernelGGL((spmm_diff_kernel<VPT, WM_, SH_>), dim3((unsigned)grid), dim3(256), 0, st, sh, sg, g->rp, \
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
  // (16 lanes per row at width 64: 4 doubles each measured faster than 2 or 8)
  const SpmmShape sh = spmm_shape(g, ld);
  if (sh.ws <= 32) {
    spmm_dispatch_w<2>(g, fp32_weights, sh, V, Vprev, out, a, b, gmul, acc, e, e_dev, st);
  } else if (sh.ws <= 256) {
    spmm_dispatch_w<4>(g, fp32_weights, sh, V, Vprev, out, a, b, gmul, acc, e, e_dev, st);
  } else {
    // ws is a multiple of 16; 8 doubles per lane
    spmm_dispatch_w<8>(g, fp32_weights, sh, V, Vprev, out, a, b, gmul, acc, e, e_dev, st);
  }
  // (the strips' extra CSR reads are not part of the algorithmic bytes)
  kt_end(st, 4.0 * (g->n + 1) + (double)g->nnz * (4.0 + wb) + 8.0 * g->n + vb * (Vprev ? 3.0 : 2.0),
         2.0 * ((double)g->nnz + g->n) * ld);
}

}  // namespace gk
