// Internal declarations of the block-Krylov graph-kernel library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "gk/graph_kernel.h"

namespace gk {

// ------------------------------------------------------------------ errors
void set_detail(const std::string& msg);

struct Error {
  int code;
  std::string msg;
};

#define GK_HIP(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::gk::Error{GK_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define GK_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) throw ::gk::Error{(code), (msg)}; \
  } while (0)

// ------------------------------------------------------------- allocation
// The free hook of the allocator that made a block (null: the library's own
// cache), kept with the block so that it goes back there even when another
// allocator has been installed since.
struct FreeHook {
  void (*fn)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
void* dev_alloc(size_t bytes, FreeHook* made_by);
// settled: the stream that used the block has completed all its work, so the
// cache may hand it out again at once (no reuse event)
void dev_free(void* p, const FreeHook& made_by, bool settled = false);
hipStream_t current_stream();
// Wait for and drop the reuse events of every cached block (before the
// streams they were recorded on are destroyed).
void cache_settle();
// Return every cached free block to HIP; bytes released.
uint64_t cache_trim();

// A set of device buffers released together (RAII).  With `pool` set, the
// buffers are carved in order out of that caller-provided device range
// (pool_cap bytes) instead of allocated, and a request beyond it fails with
// GK_ENOMEM.
struct Arena {
  std::vector<void*> ptrs;
  std::vector<FreeHook> hooks;
  uint64_t bytes = 0;
  char* pool = nullptr;
  size_t pool_cap = 0;
  template <typename T>
  T* get(size_t count) {
    size_t b = ((count * sizeof(T) + 255) / 256) * 256;
    if (b == 0) b = 256;
    if (pool) {
      if (bytes + b > pool_cap)
        throw Error{GK_ENOMEM, "request needs more than the " + std::to_string(pool_cap) +
                                   " bytes of static device scratch"};
      void* q = pool + bytes;
      bytes += b;
      return static_cast<T*>(q);
    }
    FreeHook h;
    void* p = dev_alloc(b, &h);
    if (!p) throw Error{GK_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed"};
    ptrs.push_back(p);
    hooks.push_back(h);
    bytes += b;
    return static_cast<T*>(p);
  }
  // set once the stream of the arena's work has been synchronised
  bool settled = false;
  ~Arena() {
    for (size_t i = 0; i < ptrs.size(); ++i) dev_free(ptrs[i], hooks[i], settled);
  }
};

// ------------------------------------------------------------------ graph
}  // namespace gk

struct gk_graph {
  int64_t n = 0;
  int64_t nnz = 0;          // off-diagonal nonzeros (both triangles)
  int device = 0;
  bool unit = false;
  double lambda_max = 0;    // Gershgorin bound of spec(L)
  int max_row = 0;          // max off-diagonal entries of a row
  // Rows [xr[x], xr[x+1]) are the product's share of XCD x (workgroups are
  // dealt round-robin to the 8 XCDs): contiguous ranges of about equal cost
  // (off-diagonal entries + 3 row accesses), so a degree skew over the node
  // order does not load one XCD's L2 and fabric link with most gathers.
  int64_t xr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  // Hub rows: rows with more than hub_min off-diagonal entries, each summed
  // by a workgroup of its own in the products (a heavy-tailed degree
  // distribution puts a few very long rows on otherwise short critical paths)
  int hub_min = 256;
  int64_t nhub = 0;
  int32_t* hub = nullptr;   // nhub row indices (device order)
  // device arrays (node order of the device, see perm)
  int32_t* rp = nullptr;    // n+1
  int32_t* ci = nullptr;    // nnz
  double* w64 = nullptr;    // nnz (null for unit weights)
  float* w32 = nullptr;     // nnz (null for unit weights)
  double* d64 = nullptr;    // n: sum_j w64_ij + c_i
  double* d32 = nullptr;    // n: sum_j (double) w32_ij + c_i
  // node relabelling: device node i is caller node perm[i]
  bool reordered = false;
  int64_t* d_perm = nullptr;   // n (device -> caller)
  int64_t* d_iperm = nullptr;  // n (caller -> device)
  std::vector<int64_t> h_iperm;
  std::mutex mu;               // serialises calls that share per-graph scratch
};

namespace gk {

// block leading dimension for block width s (rows of an n x s block are
// stored with stride ld; columns s..ld-1 are zero)
inline int block_ld(int s) { return s <= 8 ? 8 : ((s + 15) / 16) * 16; }

// ----------------------------------------------------------- kernel launchers
// spmm.hip
// out[i,c] = a*(L v)_i,c + b*V[i,c] + g*Vprev[i,c]  (difference form), and
// acc[i,c] += e*out[i,c] if acc != null (e read from e_dev when non-null).
void launch_spmm(const gk_graph* g, bool fp32_weights, int ld, const double* V, const double* Vprev,
                 double* out, double a, double b, double gmul, double* acc, double e, const double* e_dev,
                 hipStream_t st);
// X_r = L V_r for `count` blocks on the same graph (widths ld[r]) in one
// launch per kSpmmGroup blocks; each block gets the arithmetic of its lone
// launch_spmm(.., V_r, null, X_r, 1, 0, 0, null, ..)
constexpr int kSpmmGroup = 16;
// 64-wide blocks: X = L V (a = 1, b = 0) and C = V^T X (64 x 64, from its
// upper tiles, mirrored) in one pass; part: spmm_gram64_grid(g) * 64 * 64
// doubles, at most spmm_gram64_scratch_elems(n) for any graph of n nodes
int spmm_gram64_grid(const gk_graph* g);
size_t spmm_gram64_scratch_elems(int64_t n);
void launch_spmm_gram64(const gk_graph* g, bool fp32_weights, const double* V, double* X, double* part, double* C,
                        hipStream_t st);
void launch_spmm_group(const gk_graph* g, bool fp32_weights, int count, const int* ld, const double* const* V,
                       double* const* X, hipStream_t st);

// ortho.hip -- tall-skinny products over a list of equally shaped blocks.
struct BlockList {
  const void* base = nullptr;   // first block
  int64_t stride = 0;           // elements between consecutive blocks (may be negative)
  int nb = 0;                   // number of blocks
  bool f32 = false;             // element type float (else double)
};
size_t gram_scratch_elems(int64_t n, int nb, int ld);
// C (nb*ld x ld) = A^T B,  B = n x ld double block; `part` scratch
void launch_gram(int64_t n, int ld, BlockList A, const double* B, double* C, double* part,
                 const int* flag, hipStream_t st);
// out = beta*in + alpha*(A * C), C (nb*ld x ld); optional float copy of out.
// upper: C (one block) is upper triangular with zeros stored below the
// diagonal, and the contraction stops at each column tile's diagonal.
// tri0 (accounting only): the first coefficient block is triangular.
void launch_tsgemm(int64_t n, int ld, BlockList A, const double* C, const double* in, double* out,
                   float* out32, double alpha, double beta, const int* flag, hipStream_t st, bool upper = false,
                   bool tri0 = false);
// column-major n x s output P[perm(i), c] = sum_a A[i,a] U[a,c]
void launch_assemble(int64_t n, int ld, int s, BlockList A, const double* U, int ldu, double* P,
                     const int64_t* perm, hipStream_t st);
// P[perm(i), c] = sum_k D[k*ld + c] * A_k[i, c]
// out[perm[r]] = sum_k A_k[r, :] z[k ld : (k+1) ld] (kernel machine predictor)
void launch_predict(int64_t n, int ld, BlockList A, const double* z, double* out, const int64_t* perm,
                    hipStream_t st);
void launch_assemble_diag(int64_t n, int ld, int s, BlockList A, const double* D, double* P,
                          const int64_t* perm, bool colmajor, hipStream_t st);
size_t coldots_scratch_elems(int64_t n, int nb, int ld);
// out[k*ld + c] = sum_i A_k[i,c] * B[i,c]
void launch_coldots(int64_t n, int ld, BlockList A, const double* B, double* out, double* part,
                    const int* flag, hipStream_t st);
// X[i,c] -= sum_k D[k*ld + c] * A_k[i,c]
void launch_axpy_diag(int64_t n, int ld, BlockList A, const double* D, double* X, const int* flag,
                      hipStream_t st);
// Y[i,c] = X[i,c] * scale[c] (and optional float copy)
void launch_colscale(int64_t n, int ld, const double* X, const double* scale, double* Y, float* Y32,
                     hipStream_t st);
// out[r*s + c] = sum_k D[k*ld + c] * A_k[rows[r], c]
void launch_gather_diag(int64_t n, int ld, int s, BlockList A, const double* D, const int64_t* rows,
                        double* out, hipStream_t st);
void launch_start_block(int64_t n, int ld, int s, const int64_t* dev_samples, double value, double* V,
                        float* V32, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);
void launch_copy_f64_to_f32(const double* a, float* b, size_t count, hipStream_t st);

// small.hip -- small dense FP64 work in one workgroup
void launch_cholqr_factor(const double* G, int ld, int s, int pass, const double* diag_prev, double thr,
                          double* W, double* R, double* Rinv, double* diag_out, int* n_defl,
                          hipStream_t st);
void launch_small_gemm(int M, int N, int K, const double* A, int lda, bool ta, const double* B, int ldb,
                       bool tb, double* C, int ldc, double alpha, double beta, hipStream_t st);
void launch_store_H(const double* C, int ld, int s, double* Hk, hipStream_t st);
void launch_assemble_T(int m, int s, const double* Hd, const double* Bd, double* T, int ldt,
                       hipStream_t st);
void launch_sym_eig(int n, double* A, int lda, double* V, int ldv, double* theta, int batch,
                    int64_t strideA, int64_t strideV, int64_t strideTheta, int* order_ws, double* cs_ws,
                    hipStream_t st);
size_t eig_order_elems(int n, int batch);
void launch_phi_values(int n, const double* theta, const gk_phi& phi, const double* poly_dev, double* fv,
                       bool use_sqrt, int* bad, hipStream_t st);
void launch_phi_apply(int n, int s, const double* S, int lds, const double* fv, double* U, int ldu,
                      double outer, hipStream_t st);
void launch_kww_gram(int n, int s, const double* S, int lds, const double* g, double* K, hipStream_t st);
size_t banded_work_elems(int m, int s);
void launch_banded_spline(int m, int s, const double* Hd, const double* Bd, double eps, int k,
                          double* work, double* U, int* bad, hipStream_t st);
bool small_wave_ok(int ld);
void launch_cholqr_wave(const double* G, int ld, int s, int pass, const double* diag_prev, double thr, double* R,
                        double* Rinv, double* diag_out, int* n_defl, const double* R1, const double* R1inv,
                        double* Rc, double* Bout, hipStream_t st);
void launch_banded_spline_wave(int m, int s, const double* Hd, const double* Bd, double eps, int k, double* work,
                               double* U, int* bad, hipStream_t st);
// BT (pass 2, may be null): B^T zero padded to ld x ld
void launch_cholqr_reg(const double* G, int ld, int s, int pass, const double* diag_prev, double thr, double* R,
                       double* Rinv, double* diag_out, int* n_defl, const double* R1, const double* R1inv, double* Rc,
                       double* Bout, double* BT, hipStream_t st);
// Arguments of one CholQR factorisation (see launch_cholqr_reg); wk is the
// ld x ld scratch pair of the 65..512 kernel.
struct CholqrArgs {
  const double* G;
  int ld, s, pass;
  const double* diag_prev;
  double thr;
  double* wk;
  double* R;
  double* Rinv;
  double* diag_out;
  int* n_defl;
  const double* R1;
  const double* R1inv;
  double* Rc;
  double* Bout;
  double* BT;
  // Pass 1 with gate set (GK_MIXED): when the factor is well conditioned and
  // no column was clamped, pass 1 completes the factorisation itself (Rc =
  // R1inv, B = R1) and writes 0 to *gate, else 1.  Pass 2 does nothing when
  // *gate == 0.  Null: pass 2 always runs.
  int* gate;
};
constexpr int kCholqrBatch = 16;   // factorisations per batched launch (one workgroup each)
// count factorisations in as few launches as possible; every one runs the
// same arithmetic as a lone launch
void launch_cholqr_reg_batched(const CholqrArgs* a, int count, hipStream_t st);    // ld <= 64
void launch_cholqr_wide_batched(const CholqrArgs* a, int count, hipStream_t st);   // 64 < ld <= 512
// bcr.hip -- (eps I + H_m)^{-k} F_1 by block cyclic reduction (s <= 64);
// work holds bcr_work_elems(m, s) doubles
size_t bcr_work_elems(int m, int s);
void launch_banded_spline_reg(int m, int s, const double* Hd, const double* Bd, double eps, int k, double* work,
                              double* U, int* bad, hipStream_t st);
// Arguments of the reorthogonalisation decision of step k (decide.h): the
// per-slice estimates, the threshold and floors, the next estimate block set
// W_{k+1,*} (s x s blocks) and the decision records.
struct OmegaDecide {
  int k, s, nj, ne;
  const double* est_part;
  double tau, floor_re, floor_loc;
  double* Wk1;
  int* fr;
  int* forced;
  double* est_out;
  int* nre;
  int* gate;   // second CholQR pass needed (set when X is projected), or null
};
// Block orthogonality estimate (partial reorthogonalisation) for s <= 512.
// est_part holds m * omega_est_per_block(s) entries; rhs_wide is null for
// s <= 64 and omega_wide_scratch_elems(m, s) doubles otherwise.  With defer
// non-null the decision is not launched: its arguments go to *defer for the
// archive projection to take (launch_arch_reorth).
void launch_omega(int k, int s, int ld, const double* Wk, const double* Wkm1, double* Wk1, const double* Hd,
                  const double* Bd, const double* Rc, double nu, double tau, double floor_re, double floor_loc,
                  double* est_part, int* fr, int* forced, double* est_out, int* nre, double* rhs_wide,
                  hipStream_t st, OmegaDecide* defer = nullptr, int* gate = nullptr);
int omega_est_per_block(int s);
// Small kernels for widths 65..512 (tiles of 64, one workgroup each).
bool wide_ok(int ld);
size_t cholqr_wide_scratch_elems(int ld);
void launch_cholqr_wide(const double* G, int ld, int s, int pass, const double* diag_prev, double thr, double* wk,
                        double* R, double* Rinv, double* diag_out, int* n_defl, const double* R1, const double* R1inv,
                        double* Rc, double* Bout, double* BT, hipStream_t st);
size_t omega_wide_scratch_elems(int m, int s);
void launch_omega_wide(int k, int s, int ld, const double* Wk, const double* Wkm1, double* Wk1, const double* Hd,
                       const double* Bd, const double* Rc, double nu, double* rhs, double* est_part, hipStream_t st);
size_t banded_wide_work_elems(int m, int s);
void launch_banded_spline_wide(int m, int s, const double* Hd, const double* Bd, double eps, int k, double* work,
                               double* U, int* bad, hipStream_t st);
int cheb_diffusion_degree(double t, double Lam);
// one Chebyshev series term through the block tridiagonal H_m (s <= 512)
void launch_btd_cheb_tile(int m, int s, const double* Hd, const double* Bd, const double* Y, const double* Yp,
                          double* out, double alpha, double beta, double gamma, double* acc, const double* coef,
                          int kk, hipStream_t st);
// U (m s x s) = sum_{k <= deg} coef[k] T_k(I - 2 H_m / Lam) F_1 (Chebyshev
// series through the block tridiagonal H_m; t is not used)
void launch_cheb_series(int m, int s, const double* Hd, const double* Bd, double t, double Lam, int deg,
                        const double* coef, double* Y0, double* Y1, double* Y2, double* U, hipStream_t st);
// largest projected matrix (m s) the one-workgroup spectral decomposition takes
constexpr int kEigMaxOrder = 4096;
// Chebyshev-Lobatto coefficients of a spline or polynomial phi of degree deg
// on [0, Lam]: f at the points, then the cosine sums (angles reduced exactly)
void launch_cheb_coef_phi(int deg, double Lam, const gk_phi& phi, const double* poly_dev, double* fv, double* a,
                          hipStream_t st);
// deterministic sum of nparts equally long partial vectors: out[i] = sum_c part[c*len + i]
// sym_ld > 0: the parts hold the sym_t x sym_t tiles on and above the diagonal
// of a symmetric sym_ld x sym_ld matrix; out receives the whole matrix
void launch_reduce_parts(int64_t len, int nparts, const double* part, double* out, const int* flag, hipStream_t st,
                         int sym_ld = 0, int sym_t = 64);
// piv_rel: LU pivots at or below piv_rel * max|K + gamma I| count as singular
void launch_small_solve(int s, const double* K, double gamma, const double* y, double* c, double* work,
                        int* piv, bool spd, double piv_rel, int* bad, hipStream_t st);

// panel.hip -- fused row-panel MFMA passes (ld in {16, 32, 48, 64})
enum { PM_GRAMV = 0, PM_UPDATE_SELF = 1, PM_APPLY_SELF = 2, PM_APPLY_WRITE = 3 };
bool panel_ok(int ld);
// arch.hip -- projection against the float32 archive on FP32 matrix cores
bool arch_ok(int ld);
size_t arch_scratch_elems(int64_t n, int nb_max, int ld);
// flag gates the three launches; with dec non-null the first one takes the
// reorthogonalisation decision itself (it writes the flag, dec->fr + dec->k).
void launch_arch_reorth(int64_t n, int ld, BlockList A, double* X, double* C, double* part, const int* flag,
                        hipStream_t st, const OmegaDecide* dec = nullptr);
void launch_arch_assemble(int64_t n, int ld, int s, BlockList A, const double* U, double* P, const int64_t* perm,
                          hipStream_t st);
// X -= A C on the BF16 matrix cores (three-part split of every float32
// operand) for a float32 archive and ld % 64 == 0; C is nb*ld x ld row-major.
bool update_bf3_ok(int ld);
void launch_update_bf3(int64_t n, int ld, BlockList A, const double* C, double* X, const int* flag, hipStream_t st);
size_t panel_scratch_elems(int64_t n, int ld);
// flag: the pass and its reduction do nothing when *flag == 0
void launch_panel(int mode, int64_t n, int ld, int nbv, const double* X, double* Xout, float* X32,
                  const double* V0, const double* V1, const double* Cupd, const double* Rm, double* part,
                  double* Cout, hipStream_t st, double* H = nullptr, int hs = 0, bool tri0 = false,
                  const int* flag = nullptr);

// krylov.hip -- one call of the compute entry points
struct CallArgs {
  gk_graph* g;
  const int64_t* samples;
  int32_t s;
  const gk_phi* phi;
  int32_t m, variant, precision;
  uint32_t flags;
  const double* y;        // fit only
  double gamma;
  double* cols_out;
  double* kww_out;
  double* coef_out;
  double* pred_out;
  gk_stats* st;
  bool fit;
  void* pool = nullptr;     // device range all buffers are carved from (no allocation), or null
  size_t pool_cap = 0;
};
int run_call(const CallArgs& a, hipStream_t stream);
// Lockstep serving of classical block Lanczos calls (krylov.hip): begin
// (validation, set-up, start block on step_stream), one Lanczos step for a
// set of calls (grouped SpMM, batched CholQR; all on stream st), finish (phi
// stage and outputs on fin after the step stream), complete (wait, copy the
// results to the host, statistics; throws on a failed call), free.
struct BatchCall;
bool batch_eligible(const CallArgs& a);
BatchCall* batch_begin(const CallArgs& a, hipStream_t step_stream);
bool batch_stepping(const BatchCall* B);
void batch_step(std::vector<BatchCall*>& calls, hipStream_t st);
void batch_finish(BatchCall* B, hipStream_t step_stream, hipStream_t fin);
int batch_complete(BatchCall* B);
void batch_free(BatchCall* B);
uint64_t footprint_bytes(int64_t n, int s, int m, int variant, int precision, uint32_t flags = 0);
void set_thread_stream(hipStream_t s);

// ------------------------------------------------------------- timing
struct PhaseTimer {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  int cur = -1;
  hipEvent_t cur_start = nullptr;
  void begin(int phase);
  void end();
  void collect(gk_stats* s);
  ~PhaseTimer();
};
enum Phase { PH_SPMM = 0, PH_ORTH, PH_REORTH, PH_PHI, PH_ASM, PH_FIT, PH_TOTAL };

// Per-kernel timing of timed calls (GK_TIMING): launchers bracket their main
// kernel with kt_begin / kt_end (events on the launch stream) and state the
// algorithmic bytes and flops of that launch.  kt_start / kt_finish bracket a
// call on the calling thread; gk_kernel_timings returns the aggregate.
enum KernelClass {
  KC_SPMM = 0, KC_PANEL_GRAMV, KC_PANEL_UPDATE_SELF, KC_PANEL_APPLY_SELF, KC_PANEL_APPLY_WRITE,
  KC_GRAM, KC_TSGEMM, KC_ARCH_GRAM, KC_ARCH_UPDATE, KC_REDUCE, KC_CHOLQR, KC_OMEGA, KC_BANDED_FACTOR,
  KC_BANDED_SOLVE, KC_CHEB, KC_EIG, KC_ASSEMBLE, KC_PREDICT, KC_COUNT
};
void kt_start(bool on);
void kt_finish();
void kt_begin(int cls, hipStream_t st);
void kt_end(hipStream_t st, double bytes, double flops, const int* flag = nullptr);

}  // namespace gk
