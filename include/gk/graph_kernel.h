/*
 * graph_kernel.h -- C ABI of the MI355X (gfx950) block-Krylov graph-kernel
 * library.
 *
 * The library approximates kernel columns phi(L) E_W of a sparse graph
 * Laplacian L (Erb, "Krylov subspace methods to accelerate kernel machines
 * on graphs", arXiv 2301.06384, Sec. 3, the block phi(L) E_W) by classical
 * block Lanczos (Alg. 1), global block Lanczos (Alg. 2), sequential Lanczos
 * (Sec. 3.3) and the Chebyshev methods (Sec. 3.4), and fits / evaluates the
 * regularised least-squares kernel machine (Sec. 2.3, Alg. 3).
 *
 * Conventions shared by every entry point
 *   - Return value: GK_OK (0) or a negative gk_status code.  No exception
 *     crosses the ABI.  gk_strerror() maps a code to static text;
 *     gk_last_error_detail() gives a thread-local detail message.
 *   - Node indices are 0-based.  The block width s is the number of sample
 *     nodes (the paper's N); the graph order n is the paper's n.
 *   - Host buffers are owned by the caller and never retained after return
 *     (serving requests: until gk_poll reports completion).  Device memory is
 *     owned by the library; it is taken from the allocator installed with
 *     gk_set_allocator (default hipMalloc / hipFree).
 *   - With GK_IO_DEVICE in `flags`, the samples / y inputs and all outputs
 *     are device pointers on the current HIP device; otherwise host pointers.
 *   - Work is enqueued on the stream installed with gk_set_stream (default:
 *     the null stream of the current device).  Calls return after the
 *     results are complete, for host and device outputs alike (the call
 *     synchronises that stream before returning).
 *   - Results are deterministic: for fixed inputs, precision and flags the
 *     outputs are bitwise identical from run to run, alone or while other
 *     requests run (no atomics in any reduction; fixed reduction order).
 */
#ifndef GK_GRAPH_KERNEL_H
#define GK_GRAPH_KERNEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
typedef enum {
  GK_OK = 0,
  GK_EINVAL = -1,        /* bad argument: n<1, s<1, m<1, bad CSR, t<0, eps<=0, k<=0, non-finite value */
  GK_ENOTSYM = -2,       /* CSR not symmetric (|L_ij - L_ji| > 1e-14 max|L|) */
  GK_ENOTLAP = -3,       /* an off-diagonal entry > 0 (Sec. 2.1 needs L_ij < 0 on edges), or
                            negative diagonal excess without GK_ASSUME_PSD */
  GK_EDUPSAMPLE = -4,    /* sample nodes not distinct (E_W needs distinct unit columns, Sec. 3) */
  GK_ERANGE = -5,        /* sample index outside [0, n) */
  GK_ENOMEM = -6,        /* request refused by HBM admission, or allocation failed */
  GK_ENOTSPD = -7,       /* kernel system (K_W + gamma I) not solvable (cbl: not SPD; gbl/sbl/cheb:
                            singular), cf. Sec. 8.3 */
  GK_EDEVICE = -8,       /* HIP runtime error or no usable gfx950 device */
  GK_EUNSUPPORTED = -9,  /* combination not implemented */
  GK_EAGAIN = -10,       /* gk_poll: request not finished yet */
  GK_ESHUTDOWN = -11     /* serving loop stopped */
} gk_status;

/* ----------------------------------------------------------- graph object */
typedef struct gk_graph gk_graph;   /* opaque; owns the device-resident Laplacian */

/* graph_kernel_init flags */
#define GK_UNIT_WEIGHTS 0x1u   /* vals may be NULL: L = D - A with unit edge weights */
#define GK_ASSUME_PSD   0x2u   /* accept negative diagonal excess c_i = L_ii - sum_j |L_ij| */
#define GK_REORDER      0x4u   /* relabel nodes on the device for gather locality (BFS order);
                                  transparent to the caller: samples and outputs keep caller order */

/* --------------------------------------------------------------- phi spec */
typedef enum {
  GK_PHI_DIFFUSION = 0,   /* phi(lam) = exp(-t lam), t >= 0          (Sec. 2.4) */
  GK_PHI_SPLINE = 1,      /* phi(lam) = (eps + lam)^(-k), eps>0, k>0 (Sec. 2.4) */
  GK_PHI_POLYNOMIAL = 2   /* phi(lam) = sum_j poly[j] lam^j (exactness checks, Lemma 4.1) */
} gk_phi_kind;

typedef struct {
  int32_t kind;          /* gk_phi_kind */
  double t;              /* diffusion time */
  double eps;            /* spline shift */
  double k;              /* spline exponent (the paper's s) */
  const double* poly;    /* host pointer, poly_len coefficients, lowest degree first */
  int32_t poly_len;
} gk_phi;

/* ------------------------------------------------------ method selectors */
typedef enum {
  GK_CBL = 0,    /* classical block Lanczos, Alg. 1 */
  GK_GBL = 1,    /* global block Lanczos, Alg. 2 */
  GK_SBL = 2,    /* sequential Lanczos, Sec. 3.3 */
  GK_CHEB = 3,   /* Chebyshev interpolation, Sec. 3.4 */
  GK_CHEB2 = 4   /* squared Chebyshev, Sec. 3.4.1 */
} gk_variant;

typedef enum {
  GK_FP64 = 0,   /* every step in float64, full two-pass reorthogonalisation */
  GK_MIXED = 1   /* float64 three-term recurrence and small factors; float32 weights and
                    float32 basis archive for reorthogonalisation and assembly; partial
                    reorthogonalisation driven by an orthogonality estimate */
} gk_precision;

/* krylov_kernel_columns / kernel_machine_fit_predict / gk_submit flags */
#define GK_IO_DEVICE     0x1u   /* samples, y and outputs are device pointers */
#define GK_FULL_REORTH   0x2u   /* GK_MIXED: reorthogonalise against the whole basis every step */
#define GK_PHI_EIG       0x4u   /* form phi(H_m) F_1 through the spectral decomposition of H_m even
                                   where an exact banded evaluation exists */
#define GK_TIMING        0x8u   /* record per-phase device times into gk_stats (adds events) */
#define GK_NO_REORTH     0x10u  /* diagnostic: no reorthogonalisation against the stored basis (local
                                   orthogonalisation only, Alg. 1 / Alg. 2 as printed), to study the
                                   loss of orthogonality; the results lose accuracy once Ritz values
                                   converge */
#define GK_TWO_PASS      0x20u  /* memory-lean classical block Lanczos in float64 (GK_CBL, GK_FP64 only,
                                   else GK_EUNSUPPORTED): the basis storage m*n*N of Table 2 is replaced
                                   by three blocks.  Pass 1 runs Alg. 1 keeping the projected matrix and
                                   the coefficients of every step; pass 2 regenerates the basis from
                                   them (bit for bit) and accumulates the columns.  With no stored basis
                                   there is no reorthogonalisation against older blocks: the result is
                                   Alg. 1 with local (two-pass Gram-Schmidt) orthogonalisation */
/* Any other flag bit is rejected with GK_EINVAL. */

/* ------------------------------------------------------------- statistics */
typedef struct {
  double t_total_ms;      /* wall time of the call on the device (events), GK_TIMING only */
  double t_spmm_ms;       /* SpMM L*V (sum over steps) */
  double t_orth_ms;       /* local orthogonalisation + QR */
  double t_reorth_ms;     /* reorthogonalisation against the stored basis */
  double t_phi_ms;        /* phi(H_m) F_1 (eigendecomposition or banded evaluation) */
  double t_asm_ms;        /* assembly [V_1..V_m] U / predictor */
  double t_fit_ms;        /* small solve (K_W + gamma I) c = y */
  double spmm_launches;   /* number of SpMM launches timed */
  double bytes_spmm;      /* algorithmic bytes of all SpMM launches */
  double resid_norm;      /* ||X_m||_F of the last iteration (unused H_{m+1,m}) */
  double orth_est;        /* final orthogonality estimate (GK_MIXED) */
  int32_t n_reorth;       /* steps with reorthogonalisation against the stored basis */
  int32_t n_deflated;     /* basis columns deflated (rank-deficient QR) */
  int32_t phi_method;     /* 0 eigendecomposition, 1 banded Cholesky, 2 Chebyshev-on-H, 3 Horner */
  int32_t n_qr2_series;   /* second CholQR passes taken by the series expansion of chol(I + E) */
  int32_t n_qr2_skipped;  /* GK_MIXED: second CholQR passes left out (first factor final, no projection) */
  uint64_t footprint_bytes; /* device bytes the call held */
} gk_stats;

/* ------------------------------------------------------------------- calls */

/* Build a device-resident Laplacian (Sec. 2.1, eq. of the generalised Laplacian).
 *   n        graph order (n >= 1)
 *   row_ptr  host, n+1 int64 offsets, row_ptr[0] = 0, nondecreasing
 *   col_idx  host, row_ptr[n] int32 column indices, sorted within each row,
 *            full symmetric storage (both triangles), diagonal entry allowed
 *   vals     host, row_ptr[n] float64 values (NULL with GK_UNIT_WEIGHTS)
 * Checks symmetry (GK_ENOTSYM), L_ij <= 0 off the diagonal (GK_ENOTLAP),
 * finiteness and index range (GK_EINVAL).  Stored internally in difference
 * form: w_ij = -L_ij > 0 and the diagonal excess c_i = L_ii - sum_j w_ij, so
 * that (L v)_i = sum_j w_ij (v_i - v_j) + c_i v_i and L 1 = c exactly, also
 * with float32 weights.  The caller may free the CSR after return.  The
 * graph holds its device memory until graph_kernel_release. */
int graph_kernel_init(int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                      const double* vals, uint32_t flags, gk_graph** out);

/* Release a graph and its device memory.  NULL is accepted. */
void graph_kernel_release(gk_graph* g);

/* Query graph properties: order, off-diagonal nonzeros, spectral bound
 * Lambda (Gershgorin, max_i sum_j |L_ij|).  Any pointer may be NULL. */
int gk_graph_info(const gk_graph* g, int64_t* n, int64_t* nnz_offdiag, double* lambda_max);

/* Kernel columns p_{phi,m-1}(L) E_W ~ phi(L) E_W (Alg. 1 and 2, Sec. 3.3, 3.4).
 *   samples   s distinct node indices (host, or device with GK_IO_DEVICE)
 *   s         block width (number of samples), 1 <= s <= 1024
 *   phi       kernel function (host struct)
 *   m         number of Krylov blocks (Lanczos: m blocks, degree m-1; Chebyshev:
 *             degree m), 1 <= m <= 4096
 *   variant   gk_variant; precision gk_precision; flags GK_* call flags
 *   cols_out  n*s float64, column-major with leading dimension n; column j
 *             belongs to samples[j]; may be NULL
 *   kww_out   s*s float64 column-major sampled block K_W = E_W^T P; for cbl
 *             formed as F_1^T phi(H_m) F_1 (Theorem 3.1, SPD); may be NULL
 *   st        statistics, may be NULL
 * Errors: GK_EINVAL, GK_ERANGE, GK_EDUPSAMPLE, GK_ENOMEM, GK_EDEVICE,
 * GK_EUNSUPPORTED. */
int krylov_kernel_columns(gk_graph* g, const int64_t* samples, int32_t s, const gk_phi* phi,
                          int32_t m, int32_t variant, int32_t precision, uint32_t flags,
                          double* cols_out, double* kww_out, gk_stats* st);

/* krylov_kernel_columns without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and results as
 * krylov_kernel_columns, with GK_IO_DEVICE required: samples, cols_out and
 * kww_out are device pointers.  Every work buffer of the call is carved from
 * a static device array of GK_STATIC_SCRATCH_BYTES per GPU, held from the
 * first call on that GPU until the process ends; the call makes no
 * hipMalloc / hipFree and no allocator-hook call.  A request whose buffers
 * exceed the array fails with GK_ENOMEM (gk_request_footprint minus the
 * n*s*8 output staging and a 64 MiB allowance gives the estimate checked
 * first).  All calls on one GPU share its array: calls that overlap in time
 * on the same GPU (other threads, other streams) race and must be
 * serialised by the caller.  Errors as krylov_kernel_columns, plus
 * GK_EINVAL without GK_IO_DEVICE. */
#define GK_STATIC_SCRATCH_BYTES (128u << 20)
int krylov_kernel_columns_noalloc(gk_graph* g, const int64_t* samples, int32_t s, const gk_phi* phi,
                                  int32_t m, int32_t variant, int32_t precision, uint32_t flags,
                                  double* cols_out, double* kww_out, gk_stats* st);

/* Kernel RLS machine (Sec. 2.3; Alg. 3 for cbl, Sec. 5 system for the others).
 *   y         s labels at the samples (host or device)
 *   gamma     total diagonal shift >= 0 (the paper's gamma * N)
 *   coef_out  s coefficients c solving (K_W + gamma I) c = y; may be NULL
 *   pred_out  n predictions y(v) = sum_i c_i p(L) e_{w_i} (v); may be NULL
 * cbl never forms the n x s block: prediction = [V_1..V_m] (phi(H_m) F_1 c)
 * (Corollary 1).  Errors as above plus GK_ENOTSPD. */
int kernel_machine_fit_predict(gk_graph* g, const int64_t* samples, int32_t s, const double* y,
                               const gk_phi* phi, int32_t m, int32_t variant, int32_t precision,
                               uint32_t flags, double gamma, double* coef_out, double* pred_out,
                               gk_stats* st);

/* Device bytes a request would hold (basis archive, recurrence blocks,
 * projected matrix, workspaces) for the call flags `flags` (GK_TWO_PASS
 * changes the storage); pure arithmetic, callable without a GPU. */
int gk_request_footprint(int64_t n, int32_t s, int32_t m, int32_t variant, int32_t precision,
                         uint32_t flags, uint64_t* bytes);

/* -------------------------------------------------------------- serving
 * Continuous batching: requests are admitted while a slot is free and the
 * sum of admitted footprints stays within the HBM budget; admitted requests
 * run concurrently on a pool of streams, and a request arriving while others
 * run starts as soon as a slot and memory free up.  Each result is bitwise
 * identical to the same request run alone (same kernels, same tiling). */
typedef struct {
  gk_graph* graph;
  const int64_t* samples;   /* host, s entries; copied at submit */
  int32_t s;
  const double* y;          /* host, s labels; copied at submit */
  gk_phi phi;               /* poly copied at submit */
  int32_t m;
  int32_t variant;
  int32_t precision;
  uint32_t flags;           /* GK_IO_DEVICE is not accepted here */
  double gamma;
  double* coef_out;         /* host, s; written before completion is reported; may be NULL */
  double* pred_out;         /* host, n; may be NULL */
} gk_request;

typedef struct {
  int32_t status;           /* gk_status of the request */
  int32_t reserved;
  double t_submit_ms;       /* host clock (ms since server start) at gk_submit */
  double t_start_ms;        /* admission time */
  double t_complete_ms;     /* results visible on the host */
  gk_stats stats;
} gk_result;

/* Configure (and start) the serving loop: up to max_active concurrent
 * requests (1..64), admission budget in bytes (0 = 90% of free device
 * memory), n_streams streams (1..16, default priority). */
int gk_serve_start(int32_t max_active, uint64_t hbm_budget_bytes, int32_t n_streams);
/* Submit a request; returns a ticket.  Host inputs are copied. */
int gk_submit(const gk_request* r, uint64_t* ticket);
/* Wait up to timeout_us (0: poll, <0: forever) for a ticket; GK_EAGAIN if
 * not done.  A completed ticket is consumed by a successful gk_poll. */
int gk_poll(uint64_t ticket, int64_t timeout_us, gk_result* res);
/* Drain and stop the serving loop. */
int gk_serve_stop(void);

/* ---------------------------------------------------------------- plumbing */
const char* gk_strerror(int code);
const char* gk_last_error_detail(void);
/* Device memory hooks (e.g. a framework's caching allocator).  alloc must
 * return device memory of the current device aligned to 256 bytes, or NULL.
 * Both hooks or neither (NULL, NULL: the library's own cache again);
 * otherwise GK_EINVAL.  Calls and serving requests started afterwards
 * allocate through the new hooks; every block is returned to the allocator
 * that made it, also when the hooks change while it is in use. */
int gk_set_allocator(void* (*alloc_fn)(size_t bytes, void* ctx), void (*free_fn)(void* ptr, void* ctx),
                     void* ctx);
/* Return the device blocks the library's own cache keeps for reuse (freed
 * by finished calls) to HIP, after the work that last used them has
 * completed; *released_bytes (may be NULL) receives their size.  Blocks of
 * calls still running, and blocks of an allocator installed with
 * gk_set_allocator, are untouched. */
int gk_trim(uint64_t* released_bytes);
/* Stream used by the synchronous calls of the calling thread (hipStream_t). */
int gk_set_stream(void* hip_stream);
/* Library version string. */
const char* gk_version(void);

/* Per-kernel device times of the calling thread's most recent call made with
 * GK_TIMING: one record per kernel class (SpMM, each orthogonalisation pass,
 * archive projection, small factorisations, phi evaluation, assembly), each
 * with its launch count, summed time between HIP events recorded on the
 * call's stream around the launches, and the algorithmic bytes and flops of
 * those launches (operand sizes of the method, not hardware counters).
 * Writes min(cap, *count) records to `out` and the number of classes to
 * *count.  Returns GK_EINVAL for a NULL count or a NULL out with cap > 0. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double alg_bytes;
  double alg_flops;
} gk_kernel_timing;
int gk_kernel_timings(gk_kernel_timing* out, int32_t cap, int32_t* count);

#ifdef __cplusplus
}
#endif
#endif /* GK_GRAPH_KERNEL_H */
