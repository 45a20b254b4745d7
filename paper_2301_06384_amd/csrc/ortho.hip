// Tall-skinny block products: Gram matrices A^T B, block updates X -= A C,
// kernel-column assembly [Q_1..Q_m] U, and the column-wise (Frobenius /
// sequential) variants.
//
// These realise the DOT and AXPY work of Table 1: H_kk = Q_k^T X (Alg. 1),
// the projections that keep the basis orthonormal (Sec. 3.1), the QR of X,
// tr(Q_k^T X) and ||X||_F (Alg. 2), and the final [Q_1..Q_m] U (Alg. 1, 2).
// A "block list" is nb equally shaped n x ld row-major blocks, float or
// double, seen as one n x (nb*ld) matrix.  All accumulation is float64.
// Reductions over rows are split in fixed chunks whose partial results are
// summed in a fixed order by a second kernel: no atomics, so results are
// bitwise reproducible and independent of other work on the device.
#include "gk_internal.h"

namespace gk {

template <bool F32>
__device__ __forceinline__ double ldA(const void* base, int64_t off) {
  if (F32) return (double)static_cast<const float*>(base)[off];
  return static_cast<const double*>(base)[off];
}

// ------------------------------------------------------------------ Gram
constexpr int G_TA = 64, G_TB = 64, G_RS = 16;

template <bool F32>
__global__ void __launch_bounds__(256)
gram_kernel(int64_t n, int ld, const void* __restrict__ Abase, int64_t astride, int nb,
            const double* __restrict__ B, double* __restrict__ part, int64_t rows_per_chunk,
            const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  __shared__ double sA[G_RS][G_TA + 1];
  __shared__ double sB[G_RS][G_TB + 1];
  const int pa = nb * ld;
  const int a0 = blockIdx.x * G_TA;
  const int b0 = blockIdx.y * G_TB;
  const int64_t r_begin = (int64_t)blockIdx.z * rows_per_chunk;
  const int64_t r_end = min(n, r_begin + rows_per_chunk);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += G_RS) {
    for (int q = threadIdx.x; q < G_RS * G_TA; q += 256) {
      const int rr = q / G_TA, cc = q % G_TA;
      const int64_t r = r0 + rr;
      const int a = a0 + cc, b = b0 + cc;
      double va = 0.0, vb = 0.0;
      if (r < r_end) {
        if (a < pa) {
          const int blk = a / ld, col = a - blk * ld;
          va = ldA<F32>(Abase, (int64_t)blk * astride + r * ld + col);
        }
        if (b < ld) vb = B[r * ld + b];
      }
      sA[rr][cc] = va;
      sB[rr][cc] = vb;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < G_RS; ++rr) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[rr][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[rr][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* P = part + (int64_t)blockIdx.z * pa * ld;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + ty * 4 + i, b = b0 + tx * 4 + j;
      if (a < pa && b < ld) P[(int64_t)a * ld + b] = acc[i][j];
    }
}

// out[i] = sum_{c < nparts} part[c*len + i] in a fixed order: block b owns
// outputs [16b, 16b+16); its 16 thread groups sum interleaved parts (eight
// running sums per thread, so eight loads are in flight, combined pairwise),
// then the 16 group sums are added in group order.  sym_ld > 0: the parts
// hold only the sym_t x sym_t tiles on and above the diagonal of a symmetric
// sym_ld x sym_ld matrix (sym_ld and sym_t multiples of 16, so a block's
// outputs lie in one row of one tile); blocks below the diagonal return at
// once and those above it also write the mirrored entries.
__global__ void __launch_bounds__(256)
reduce_parts_kernel(int64_t len, int nparts, const double* __restrict__ part, double* __restrict__ out,
                    const int* __restrict__ flag, int sym_ld, int sym_t) {
  if (flag && *flag == 0) return;
  __shared__ double red[16][17];
  const int o = threadIdx.x & 15, g = threadIdx.x >> 4;
  // groups of 16 outputs, taken in turn by the workgroups of a capped grid
  // (a gated launch that has nothing to do then dispatches few workgroups)
  const int64_t ngrp = (len + 15) / 16;
  for (int64_t gb = blockIdx.x; gb < ngrp; gb += gridDim.x) {
    const int64_t i = gb * 16 + o;
    const int64_t src = i;
    int64_t mirror = -1;
    if (sym_ld > 0) {
      const int64_t r = (gb * 16) / sym_ld, c = i - r * sym_ld;
      const int64_t tr = r / sym_t, tc = (gb * 16 - r * sym_ld) / sym_t;
      if (tr > tc) continue;   // the whole group: lower tiles come from their mirror
      if (tr < tc) mirror = c * sym_ld + r;
    }
    double s = 0.0;
    if (i < len) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = 0.0;
      int c = g;
      for (; c + 16 * 7 < nparts; c += 16 * 8)
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += part[(int64_t)(c + 16 * u) * len + src];
      for (; c < nparts; c += 16) a[0] += part[(int64_t)c * len + src];
      s = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    }
    red[g][o] = s;
    __syncthreads();
    if (g == 0 && i < len) {
      double t = 0.0;
      for (int q = 0; q < 16; ++q) t += red[q][o];
      out[i] = t;
      if (mirror >= 0) out[mirror] = t;
    }
    __syncthreads();
  }
}

void launch_reduce_parts(int64_t len, int nparts, const double* part, double* out, const int* flag, hipStream_t st,
                        int sym_ld, int sym_t) {
  // entries read per part: the whole vector, or the tiles on and above the diagonal
  double rd = (double)len;
  if (sym_ld > 0) {
    const double nt = sym_ld / sym_t;
    rd = nt * (nt + 1) / 2 * sym_t * sym_t;
  }
  kt_begin(KC_REDUCE, st);
  const int64_t ngrp = (len + 15) / 16;
  hipLaunchKernelGGL(reduce_parts_kernel, dim3((unsigned)std::min<int64_t>(ngrp, 1024)), dim3(256), 0, st, len, nparts,
                     part, out, flag, sym_ld, sym_t);
  GK_HIP(hipGetLastError());
  kt_end(st, 8.0 * (rd * nparts + len), rd * nparts, flag);
}

// Blocks 64 and wider use the FP64 matrix-core kernels below (rows staged
// 32 at a time, 64-wide output tiles); narrower ones the vector kernel above.
static bool mfma_ok(int ld) { return ld >= 64 && ld % 16 == 0; }
constexpr int MG_T = 64, MG_RS = 32, MG_P = MG_T + 2;

static void gram_geometry(int64_t n, int nb, int ld, int* nx, int* ny, int* nch, int64_t* rpc) {
  const int rs = mfma_ok(ld) ? MG_RS : G_RS;
  const int pa = nb * ld;
  *nx = (pa + G_TA - 1) / G_TA;
  *ny = (ld + G_TB - 1) / G_TB;
  int64_t want = (2048 + (*nx) * (*ny) - 1) / ((*nx) * (*ny));
  int64_t maxc = (n + 255) / 256;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  if (want > 1024) want = 1024;
  // a multiple of 8 chunks, so that every XCD gets the same number of them
  // (the MFMA Gram kernels run each chunk's tiles on one XCD); chunks past
  // the last row are empty and contribute zero partials
  want = (want + 7) / 8 * 8;
  int64_t r = (n + want - 1) / want;
  r = ((r + rs - 1) / rs) * rs;
  *rpc = r;
  *nch = (int)want;
}

// Workgroup order of the MFMA tile kernels (one-dimensional grids).
// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// Gram (tiles nx x ny per row chunk): the nx ny tiles of chunk c are
// consecutive workgroups of XCD c % 8, so the rows of a chunk are fetched
// into one L2 and read there by all its tiles, not once per tile.
__device__ __forceinline__ void gram_tile(int nx, int ny, int& ta, int& tb, int& tc) {
  const unsigned L = blockIdx.x, x = L & 7, j = L >> 3, T = (unsigned)(nx * ny);
  const unsigned t = j % T;
  tc = (int)((j / T) * 8 + x);
  ta = (int)(t % (unsigned)nx);
  tb = (int)(t / (unsigned)nx);
}
// Row-tile products (row tiles x ny column tiles): the ny column tiles of
// row tile rt are consecutive workgroups of XCD rt % 8, so the rows they all
// read come from one L2.  False past the last row tile.
__device__ __forceinline__ bool row_tile(int64_t nrt, int ny, int64_t& rt, int& tb) {
  const unsigned L = blockIdx.x, x = L & 7, j = L >> 3;
  tb = (int)(j % (unsigned)ny);
  rt = (int64_t)(j / (unsigned)ny) * 8 + x;
  return rt < nrt;
}
static inline unsigned row_tile_grid(int64_t nrt, int ny) { return (unsigned)(8 * ((nrt + 7) / 8) * ny); }

size_t gram_scratch_elems(int64_t n, int nb, int ld) {
  int nx, ny, nch;
  int64_t rpc;
  gram_geometry(n, nb, ld, &nx, &ny, &nch, &rpc);
  return (size_t)nch * nb * ld * ld;
}

// ------------------------------------------- FP64 matrix-core Gram / update
typedef double d4v __attribute__((ext_vector_type(4)));

// Eight consecutive elements (16-byte aligned) held as loaded: the float to
// double conversion happens only when they are stored to LDS, so a prefetch
// does not wait for its own loads.
template <bool F32>
struct Raw8 {
  float4 f[2];
  __device__ __forceinline__ void load(const void* __restrict__ base, int64_t off) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(base) + off);
    f[0] = p[0];
    f[1] = p[1];
  }
  __device__ __forceinline__ void zero() { f[0] = f[1] = make_float4(0.f, 0.f, 0.f, 0.f); }
  __device__ __forceinline__ double get(int q) const {
    const float4& t = f[q >> 2];
    const int e = q & 3;
    return (double)(e == 0 ? t.x : e == 1 ? t.y : e == 2 ? t.z : t.w);
  }
};
template <>
struct Raw8<false> {
  double2 d[4];
  __device__ __forceinline__ void load(const void* __restrict__ base, int64_t off) {
    const double2* p = reinterpret_cast<const double2*>(static_cast<const double*>(base) + off);
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = p[q];
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = make_double2(0.0, 0.0);
  }
  __device__ __forceinline__ double get(int q) const { return (q & 1) ? d[q >> 1].y : d[q >> 1].x; }
};

// part[z] (pa x ld) = A^T B over the rows of chunk z, one 64 x 64 output tile
// per workgroup.  Wave w owns a 32 x 32 quarter as 2 x 2 tiles of
// v_mfma_f64_16x16x4f64 (lane l = i + 16 k: A operand A[r0+k][a+i], B operand
// B[r0+k][b+i]; accumulator register q holds output row 4q + k, column i).
// The next 32 rows are fetched into registers while the current ones are
// multiplied.
__global__ void __launch_bounds__(256)
gram_mfma_kernel(int64_t n, int ld, const double* __restrict__ Abase, int64_t astride, int nb,
                 const double* __restrict__ B, double* __restrict__ part, int64_t rows_per_chunk,
                 const int* __restrict__ flag, int sym) {
  if (flag && *flag == 0) return;
  const int pa = nb * ld;
  int ta, tb, tc;
  gram_tile((pa + MG_T - 1) / MG_T, (ld + MG_T - 1) / MG_T, ta, tb, tc);
  if (sym && ta > tb) return;   // B^T B: the tiles below the diagonal are mirrors
  __shared__ __align__(16) double sA[MG_RS][MG_P];
  __shared__ __align__(16) double sB[MG_RS][MG_P];
  const int a0 = ta * MG_T, b0 = tb * MG_T;
  const int64_t rb = (int64_t)tc * rows_per_chunk;
  const int64_t re = min(n, rb + rows_per_chunk);
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int wa = 32 * (w >> 1), wb = 32 * (w & 1);
  // staging: row sr; lane sj / 2 of the row's 8 moves the 16-byte chunks at
  // columns sj + 16 q (q = 0..3), so each load and each LDS store
  // instruction of the 8 lanes covers 128 contiguous bytes (a chunk never
  // crosses a block: ld % 16 == 0)
  const int sr = tid >> 3, sj = 2 * (tid & 7);
  int64_t aoff[4];
  bool aok[4], bok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ga = a0 + sj + 16 * q;
    aok[q] = ga < pa;
    const int blk = aok[q] ? ga / ld : 0;
    aoff[q] = (int64_t)blk * astride + (ga - blk * ld);
    bok[q] = b0 + sj + 16 * q < ld;
  }
  d4v acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = d4v{0.0, 0.0, 0.0, 0.0};
  double2 va[4], vb[4];
  auto fetch = [&](int64_t r0) {
    const int64_t r = r0 + sr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      va[q] = (r < re && aok[q]) ? *reinterpret_cast<const double2*>(Abase + aoff[q] + r * ld) : make_double2(0.0, 0.0);
      vb[q] = (r < re && bok[q]) ? *reinterpret_cast<const double2*>(B + r * ld + b0 + sj + 16 * q)
                                 : make_double2(0.0, 0.0);
    }
  };
  fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += MG_RS) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      *reinterpret_cast<double2*>(&sA[sr][sj + 16 * q]) = va[q];
      *reinterpret_cast<double2*>(&sB[sr][sj + 16 * q]) = vb[q];
    }
    __syncthreads();
    if (r0 + MG_RS < re) fetch(r0 + MG_RS);
#pragma unroll
    for (int ks = 0; ks < MG_RS / 4; ++ks) {
      double av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = sA[4 * ks + lk][wa + 16 * t + li];
        bv[t] = sB[4 * ks + lk][wb + 16 * t + li];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
  }
  double* P = part + (int64_t)tc * pa * ld;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = a0 + wa + 16 * ti + 4 * q + lk, b = b0 + wb + 16 * tj + li;
        if (a < pa && b < ld) P[(int64_t)a * ld + b] = acc[ti][tj][q];
      }
}

// out[r, b] = beta in[r, b] + alpha sum_a A[r, a] C[a, b], one 64-row x
// 64-column tile per workgroup, 32 contraction indices per stage; A is
// staged transposed so both operands are read along their contiguous LDS
// rows.  Row-major: ld columns, C with leading dimension ld.  COLMAJ (the
// assembly P = [Q_1 .. Q_nb] U): columns b < ncols written column-major
// (leading dimension ldo, row r to perm[r]) through an LDS transpose, C with
// leading dimension ldc, no in / out32.
constexpr int MT_R = 64, MT_C = 64, MT_K = 32;
// The transposed staging writes contraction index k of tile row r at column
// (r + tsw(k)) mod 64 of LDS row k.  One store instruction writes rows
// k = 8 g + q (g = 0..3 by lane, q fixed): unrotated, the four g fell on the
// same banks.  LDS serves 32-bit accesses 32 lanes at a time and 64-bit ones
// 16 lanes at a time over 32 four-byte banks, so floats are rotated by 8 g
// columns and doubles by 4 g, which spreads each group over all banks.  The
// product loop reads four consecutive k at once, which share one rotation.
template <typename T>
__device__ __forceinline__ int tsw(int k) { return (sizeof(T) == 8 ? 4 : 8) * ((k >> 3) & 3); }
// Coefficient staging: lane j of a row's 8 holds the elements q = 0..7 at
// columns cpos(j, q), pairs 16 columns apart, so each pair-wide load or
// store instruction of the 8 lanes covers one contiguous stretch of the row.
__device__ __forceinline__ int cpos(int j, int q) { return 2 * j + 16 * (q >> 1) + (q & 1); }
template <bool F32, bool COLMAJ>
__global__ void __launch_bounds__(256)
tsgemm_mfma_kernel(int64_t n, int ld, const void* __restrict__ Abase, int64_t astride, int nb,
                   const double* __restrict__ C, int ldc, int ncols, const double* __restrict__ in,
                   double* __restrict__ out, float* __restrict__ out32, double alpha, double beta, int64_t ldo,
                   const int64_t* __restrict__ perm, const int* __restrict__ flag, int upper) {
  if (flag && *flag == 0) return;
  __shared__ __align__(16) double sAT[MT_K][MT_R + 2];
  __shared__ __align__(16) double sC[MT_K][MT_C + 2];
  __shared__ double sO[COLMAJ ? MT_C : 1][MT_R + 1];
  const int pa = nb * ld;
  int64_t rt;
  int tb;
  if (!row_tile((n + MT_R - 1) / MT_R, ((COLMAJ ? ncols : ld) + MT_C - 1) / MT_C, rt, tb)) return;
  const int64_t r0 = rt * MT_R;
  const int b0 = tb * MT_C;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  const int ar = tid >> 2, ak = 8 * (tid & 3);     // A staging: row, 8 contraction indices
  const int cr = tid >> 3, cj = tid & 7;           // C staging: row, lane of the row (columns cpos)
  const int64_t arow = r0 + ar;
  double vcs[COLMAJ ? 8 : 1];   // column-major case: scalar coefficient loads (ldc need not be even)
  double2 vcp[COLMAJ ? 1 : 4];
  d4v acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = d4v{0.0, 0.0, 0.0, 0.0};
  Raw8<F32> va;
  auto fetch = [&](int a0) {
    const int ga = a0 + ak;
    if (arow < n && ga < pa) {
      const int blk = ga / ld;
      va.load(Abase, (int64_t)blk * astride + arow * ld + (ga - blk * ld));
    } else {
      va.zero();
    }
    const int gc = a0 + cr;
    if (COLMAJ) {
      const int gcc = gc < pa ? gc : pa - 1;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int col = b0 + cpos(cj, q);
        vcs[q] = C[(int64_t)gcc * ldc + (col < ncols ? col : ncols - 1)];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = b0 + 2 * cj + 16 * q;
        vcp[q] = (gc < pa && col < ld) ? *reinterpret_cast<const double2*>(C + (int64_t)gc * ld + col)
                                       : make_double2(0.0, 0.0);
      }
    }
  };
  // upper triangular C (one block): rows past the column tile are zero
  const int aend = upper ? min(pa, b0 + MT_C) : pa;
  fetch(0);
  for (int a0 = 0; a0 < aend; a0 += MT_K) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) sAT[ak + q][(ar + tsw<double>(ak)) & 63] = va.get(q);
    if (COLMAJ) {
      const bool rin = a0 + cr < pa;
#pragma unroll
      for (int q = 0; q < 8; ++q) sC[cr][cpos(cj, q)] = (rin && b0 + cpos(cj, q) < ncols) ? vcs[q] : 0.0;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) *reinterpret_cast<double2*>(&sC[cr][2 * cj + 16 * q]) = vcp[q];
    }
    __syncthreads();
    if (a0 + MT_K < aend) fetch(a0 + MT_K);
#pragma unroll
    for (int ks = 0; ks < MT_K / 4; ++ks) {
      double av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = sAT[4 * ks + lk][(wr + 16 * t + li + tsw<double>(4 * ks)) & 63];
        bv[t] = sC[4 * ks + lk][wc + 16 * t + li];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
  }
  if (COLMAJ) {
    // transpose through LDS: each column is then written as contiguous rows
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int q = 0; q < 4; ++q) sO[wc + 16 * tj + li][wr + 16 * ti + 4 * q + lk] = alpha * acc[ti][tj][q];
    __syncthreads();
    for (int q = tid; q < MT_C * MT_R; q += 256) {
      const int cc2 = q / MT_R, rr = q - cc2 * MT_R;
      const int64_t r = r0 + rr;
      const int b = b0 + cc2;
      if (r < n && b < ncols) out[(int64_t)b * ldo + (perm ? perm[r] : r)] = sO[cc2][rr];
    }
    return;
  }
  // epilogue: the 16 `in` values of this thread are loaded together (rows
  // and columns out of range read element 0 and are not stored)
  double inv[2][2][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + wr + 16 * ti + 4 * q + lk;
        const int b = b0 + wc + 16 * tj + li;
        inv[ti][tj][q] = (beta != 0.0) ? in[(r < n && b < ld) ? r * ld + b : 0] : 0.0;
      }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + wr + 16 * ti + 4 * q + lk;
        const int b = b0 + wc + 16 * tj + li;
        if (r < n && b < ld) {
          const double v = alpha * acc[ti][tj][q] + beta * inv[ti][tj][q];
          out[r * ld + b] = v;
          if (out32) out32[r * ld + b] = (float)v;
        }
      }
}

// ---------------------------- FP32 matrix-core products with the archive
// The float32 basis archive against a float64 block (reorthogonalisation
// coefficients C = Q^T X and the update X -= Q C), on v_mfma_f32_16x16x4f32:
// the coefficients only need the accuracy of the archive itself (unit
// roundoff 2^-24 relative to |Q||X|), so X and C are rounded to float in
// LDS, and the float accumulators are added into float64 every 32 terms.
// Same tiles as the FP64 kernels above; operand layout of the float MFMA:
// lane l = i + 16 k holds A[i][k] and B[k][i], accumulator register r holds
// D[4 k + r][i].  LDS pitch 80 floats (16 mod 32): the four 16-lane rows of
// an operand read fall in distinct bank halves.
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int FP = 80;

// 64 archive columns x 128 columns of X per workgroup of 8 wavefronts (wave
// w owns the 32 x 32 quarter (w % 2, w / 2)): each staged archive tile
// serves two 64-column halves of X, so the archive rows of a chunk are read
// by half as many workgroups as with 64 x 64 tiles.
constexpr int MG_TB2 = 128, FPB = MG_TB2 + 16;   // LDS pitch 144 floats (16 mod 32)
__global__ void __launch_bounds__(512)
gram_f32mma_kernel(int64_t n, int ld, const float* __restrict__ Abase, int64_t astride, int nb,
                   const double* __restrict__ B, double* __restrict__ part, int64_t rows_per_chunk,
                   const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  __shared__ __align__(16) float sA[MG_RS][FP];
  __shared__ __align__(16) float sB[MG_RS][FPB];
  const int pa = nb * ld;
  int ta, tb, tc;
  gram_tile((pa + MG_T - 1) / MG_T, (ld + MG_TB2 - 1) / MG_TB2, ta, tb, tc);
  const int a0 = ta * MG_T, b0 = tb * MG_TB2;
  const int64_t rb = (int64_t)tc * rows_per_chunk;
  const int64_t re = min(n, rb + rows_per_chunk);
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int wa = 32 * (w & 1), wb = 32 * (w >> 1);
  // staging: row sr; lane sj of the row's 16 moves the archive's 16-byte
  // chunk at column 4 sj and X's at columns 2 sj + 32 q (q = 0..3), so each
  // load and LDS store instruction of the 16 lanes covers a contiguous
  // stretch of the row (a chunk never crosses a block: ld % 16 == 0)
  const int sr = tid >> 4, sj = tid & 15;
  const int ga = a0 + 4 * sj;
  const bool aok = ga < pa;
  int64_t aoff = 0;
  if (aok) {
    const int blk = ga / ld;
    aoff = (int64_t)blk * astride + (ga - blk * ld);
  }
  bool bok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) bok[q] = b0 + 2 * sj + 32 * q < ld;
  f4v acc[2][2];
  double a64[2][2][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      acc[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) a64[ti][tj][q] = 0.0;
    }
  float4 va;
  double2 vb[4];
  auto fetch = [&](int64_t r0) {
    const int64_t r = r0 + sr;
    va = (r < re && aok) ? *reinterpret_cast<const float4*>(Abase + aoff + r * ld) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      vb[q] = (r < re && bok[q]) ? *reinterpret_cast<const double2*>(B + r * ld + b0 + 2 * sj + 32 * q)
                                 : make_double2(0.0, 0.0);
  };
  fetch(rb);
  for (int64_t r0 = rb; r0 < re; r0 += MG_RS) {
    __syncthreads();
    *reinterpret_cast<float4*>(&sA[sr][4 * sj]) = va;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<float2*>(&sB[sr][2 * sj + 32 * q]) = make_float2((float)vb[q].x, (float)vb[q].y);
    __syncthreads();
    if (r0 + MG_RS < re) fetch(r0 + MG_RS);
#pragma unroll
    for (int ks = 0; ks < MG_RS / 4; ++ks) {
      float av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = sA[4 * ks + lk][wa + 16 * t + li];
        bv[t] = sB[4 * ks + lk][wb + 16 * t + li];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a64[ti][tj][q] += (double)acc[ti][tj][q];
        acc[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
      }
  }
  double* P = part + (int64_t)tc * pa * ld;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = a0 + wa + 16 * ti + 4 * lk + q, b = b0 + wb + 16 * tj + li;
        if (a < pa && b < ld) P[(int64_t)a * ld + b] = a64[ti][tj][q];
      }
}

// out[r, b] = beta in[r, b] + alpha sum_a Q[r, a] C[a, b] (row-major, ld
// columns), one 64-row x 64-column tile per workgroup, 32 contraction
// indices per stage (the archive rows staged transposed).
__global__ void __launch_bounds__(256)
tsgemm_f32mma_kernel(int64_t n, int ld, const float* __restrict__ Abase, int64_t astride, int nb,
                     const double* __restrict__ C, const double* __restrict__ in, double* __restrict__ out,
                     double alpha, double beta, const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  __shared__ __align__(16) float sAT[MT_K][FP];
  __shared__ __align__(16) float sC[MT_K][FP];
  const int pa = nb * ld;
  int64_t rt;
  int tb;
  if (!row_tile((n + MT_R - 1) / MT_R, (ld + MT_C - 1) / MT_C, rt, tb)) return;
  const int64_t r0 = rt * MT_R;
  const int b0 = tb * MT_C;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  const int ar = tid >> 2, ak = 8 * (tid & 3);     // archive staging: row, 8 contraction indices
  const int cr = tid >> 3, cj = tid & 7;           // coefficient staging: row, lane of the row
  const int64_t arow = r0 + ar;
  f4v acc[2][2];
  double a64[2][2][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      acc[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) a64[ti][tj][q] = 0.0;
    }
  Raw8<true> va;
  double2 vcp[4];
  auto fetch = [&](int a0) {
    const int ga = a0 + ak;
    if (arow < n && ga < pa) {
      const int blk = ga / ld;
      va.load(Abase, (int64_t)blk * astride + arow * ld + (ga - blk * ld));
    } else {
      va.zero();
    }
    const int gc = a0 + cr;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = b0 + 2 * cj + 16 * q;
      vcp[q] = (gc < pa && col < ld) ? *reinterpret_cast<const double2*>(C + (int64_t)gc * ld + col)
                                     : make_double2(0.0, 0.0);
    }
  };
  fetch(0);
  for (int a0 = 0; a0 < pa; a0 += MT_K) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) sAT[ak + q][(ar + tsw<float>(ak)) & 63] = (float)va.get(q);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<float2*>(&sC[cr][2 * cj + 16 * q]) = make_float2((float)vcp[q].x, (float)vcp[q].y);
    __syncthreads();
    if (a0 + MT_K < pa) fetch(a0 + MT_K);
#pragma unroll
    for (int ks = 0; ks < MT_K / 4; ++ks) {
      float av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = sAT[4 * ks + lk][(wr + 16 * t + li + tsw<float>(4 * ks)) & 63];
        bv[t] = sC[4 * ks + lk][wc + 16 * t + li];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a64[ti][tj][q] += (double)acc[ti][tj][q];
        acc[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
      }
  }
  // the 16 `in` values of this thread are loaded together (rows and columns
  // out of range read element 0 and are not stored)
  double inv[2][2][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + wr + 16 * ti + 4 * lk + q;
        const int b = b0 + wc + 16 * tj + li;
        inv[ti][tj][q] = (beta != 0.0) ? in[(r < n && b < ld) ? r * ld + b : 0] : 0.0;
      }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = r0 + wr + 16 * ti + 4 * lk + q;
        const int b = b0 + wc + 16 * tj + li;
        if (r < n && b < ld) out[r * ld + b] = alpha * a64[ti][tj][q] + beta * inv[ti][tj][q];
      }
}

// Assembly P[perm(r), c] = sum_a Q[r, a] U[a, c] (c < ncols) from the
// float32 archive on FP32 matrix cores, U rounded to float (the accuracy of
// the archive itself, as for the 64-wide assembly of arch.hip); float
// accumulators added into float64 after every 32 contraction indices;
// column-major output (leading dimension ldo) written through an LDS
// transpose, each column as contiguous rows.
__global__ void __launch_bounds__(256)
assemble_f32mma_kernel(int64_t n, int ld, const float* __restrict__ Abase, int64_t astride, int nb,
                       const double* __restrict__ U, int ldu, int ncols, double* __restrict__ out, int64_t ldo,
                       const int64_t* __restrict__ perm) {
  __shared__ __align__(16) float sAT[MT_K][FP];
  __shared__ __align__(16) float sC[MT_K][FP];
  __shared__ double sO[MT_C][MT_R + 1];
  const int pa = nb * ld;
  int64_t rt;
  int tb;
  if (!row_tile((n + MT_R - 1) / MT_R, (ncols + MT_C - 1) / MT_C, rt, tb)) return;
  const int64_t r0 = rt * MT_R;
  const int b0 = tb * MT_C;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  const int ar = tid >> 2, ak = 8 * (tid & 3);     // archive staging: row, 8 contraction indices
  const int cr = tid >> 3, cj = tid & 7;           // coefficient staging: row, lane of the row
  const int64_t arow = r0 + ar;
  f4v acc[2][2];
  double a64[2][2][4];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj) {
      acc[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) a64[ti][tj][q] = 0.0;
    }
  Raw8<true> va;
  double vcs[8];   // scalar coefficient loads (ldu need not be even)
  auto fetch = [&](int a0) {
    const int ga = a0 + ak;
    if (arow < n && ga < pa) {
      const int blk = ga / ld;
      va.load(Abase, (int64_t)blk * astride + arow * ld + (ga - blk * ld));
    } else {
      va.zero();
    }
    const int gc = a0 + cr;
    const int gcc = gc < pa ? gc : pa - 1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int col = b0 + cpos(cj, q);
      vcs[q] = U[(int64_t)gcc * ldu + (col < ncols ? col : ncols - 1)];
    }
  };
  fetch(0);
  for (int a0 = 0; a0 < pa; a0 += MT_K) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) sAT[ak + q][(ar + tsw<float>(ak)) & 63] = (float)va.get(q);
    {
      const bool rin = a0 + cr < pa;
#pragma unroll
      for (int q = 0; q < 8; ++q) sC[cr][cpos(cj, q)] = (rin && b0 + cpos(cj, q) < ncols) ? (float)vcs[q] : 0.f;
    }
    __syncthreads();
    if (a0 + MT_K < pa) fetch(a0 + MT_K);
#pragma unroll
    for (int ks = 0; ks < MT_K / 4; ++ks) {
      float av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = sAT[4 * ks + lk][(wr + 16 * t + li + tsw<float>(4 * ks)) & 63];
        bv[t] = sC[4 * ks + lk][wc + 16 * t + li];
      }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a64[ti][tj][q] += (double)acc[ti][tj][q];
        acc[ti][tj] = f4v{0.f, 0.f, 0.f, 0.f};
      }
  }
  // D[4 k + r][i]: row wr + 16 ti + 4 lk + r, column wc + 16 tj + li
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int q = 0; q < 4; ++q) sO[wc + 16 * tj + li][wr + 16 * ti + 4 * lk + q] = a64[ti][tj][q];
  __syncthreads();
  for (int q = tid; q < MT_C * MT_R; q += 256) {
    const int cc2 = q / MT_R, rr = q - cc2 * MT_R;
    const int64_t r = r0 + rr;
    const int b = b0 + cc2;
    if (r < n && b < ncols) out[(int64_t)b * ldo + (perm ? perm[r] : r)] = sO[cc2][rr];
  }
}

void launch_gram(int64_t n, int ld, BlockList A, const double* B, double* C, double* part,
                 const int* flag, hipStream_t st) {
  int nx, ny, nch;
  int64_t rpc;
  gram_geometry(n, A.nb, ld, &nx, &ny, &nch, &rpc);
  dim3 grid(nx, ny, nch);
  // the Gram of a block with itself is symmetric: only the tiles on and
  // above the diagonal are formed
  const bool sym = mfma_ok(ld) && A.nb == 1 && !A.f32 && A.base == (const void*)B;
  // the float32 archive (reorthogonalisation coefficients) on the FP32
  // matrix cores
  const bool f32mma = mfma_ok(ld) && A.f32;
  kt_begin(f32mma ? KC_ARCH_GRAM : KC_GRAM, st);
  if (mfma_ok(ld)) {
    const dim3 g1((unsigned)(nx * ny * nch));   // chunk-major per XCD (gram_tile)
    if (A.f32)   // 64 x 128 tiles: the chunk count of the 64 x 64 geometry
      hipLaunchKernelGGL(gram_f32mma_kernel, dim3((unsigned)(nx * ((ld + MG_TB2 - 1) / MG_TB2) * nch)), dim3(512), 0,
                         st, n, ld, (const float*)A.base, A.stride, A.nb, B, part, rpc, flag);
    else
      hipLaunchKernelGGL(gram_mfma_kernel, g1, dim3(256), 0, st, n, ld, (const double*)A.base, A.stride, A.nb, B,
                         part, rpc, flag, sym ? 1 : 0);
  } else if (A.f32)
    hipLaunchKernelGGL(gram_kernel<true>, grid, dim3(256), 0, st, n, ld, A.base, A.stride, A.nb, B,
                       part, rpc, flag);
  else
    hipLaunchKernelGGL(gram_kernel<false>, grid, dim3(256), 0, st, n, ld, A.base, A.stride, A.nb, B,
                       part, rpc, flag);
  GK_HIP(hipGetLastError());
  // method's own work: the Gram of a block with itself reads it once and
  // forms one triangle
  const bool self_gram = A.nb == 1 && A.base == (const void*)B;
  kt_end(st, self_gram ? 8.0 * n * ld : (double)n * ld * ((A.f32 ? 4.0 : 8.0) * A.nb + 8.0),
         self_gram ? (double)n * ld * (ld + 1) : 2.0 * (double)n * ld * ld * A.nb, flag);
  launch_reduce_parts((int64_t)A.nb * ld * ld, nch, part, C, flag, st, sym ? ld : 0);
}

// ------------------------------------------------------- tall-skinny GEMM
constexpr int T_TR = 64, T_TB = 64, T_KS = 16;

// out[r,b] = beta*in[r,b] + alpha*sum_a A[r,a] C[a,b]   (b < ncols)
// row-major output (ld) or column-major output (ld_out rows, optional perm)
template <bool F32, bool COLMAJ>
__global__ void __launch_bounds__(256)
tsgemm_kernel(int64_t n, int ld, int ncols, const void* __restrict__ Abase, int64_t astride, int nb,
              const double* __restrict__ C, int ldc, const double* __restrict__ in,
              double* __restrict__ out, float* __restrict__ out32, double alpha, double beta,
              int64_t ldo, const int64_t* __restrict__ perm, const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  __shared__ double sA[T_TR][T_KS + 1];
  __shared__ double sC[T_KS][T_TB + 1];
  const int pa = nb * ld;
  const int64_t r0 = (int64_t)blockIdx.x * T_TR;
  const int b0 = blockIdx.y * T_TB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int a0 = 0; a0 < pa; a0 += T_KS) {
    for (int q = threadIdx.x; q < T_TR * T_KS; q += 256) {
      const int rr = q / T_KS, kk = q % T_KS;
      const int64_t r = r0 + rr;
      const int a = a0 + kk;
      double v = 0.0;
      if (r < n && a < pa) {
        const int blk = a / ld, col = a - blk * ld;
        v = ldA<F32>(Abase, (int64_t)blk * astride + r * ld + col);
      }
      sA[rr][kk] = v;
    }
    for (int q = threadIdx.x; q < T_KS * T_TB; q += 256) {
      const int kk = q / T_TB, cc = q % T_TB;
      const int a = a0 + kk, b = b0 + cc;
      sC[kk][cc] = (a < pa && b < ncols) ? C[(int64_t)a * ldc + b] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < T_KS; ++kk) {
      double av[4], cv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[ty * 4 + i][kk];
#pragma unroll
      for (int j = 0; j < 4; ++j) cv[j] = sC[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], cv[j], acc[i][j]);
    }
    __syncthreads();
  }
  if (!COLMAJ) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = r0 + ty * 4 + i;
      if (r >= n) continue;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int b = b0 + tx * 4 + j;
        if (b >= ld) continue;
        double v = alpha * acc[i][j];
        if (beta != 0.0) v += beta * in[r * ld + b];
        if (b >= ncols) v = (beta != 0.0) ? beta * in[r * ld + b] : 0.0;
        out[r * ld + b] = v;
        if (out32) out32[r * ld + b] = (float)v;
      }
    }
  } else {
    // stage through LDS so that each column is written as contiguous rows
    __shared__ double sO[T_TB][T_TR + 1];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) sO[tx * 4 + j][ty * 4 + i] = alpha * acc[i][j];
    __syncthreads();
    for (int q = threadIdx.x; q < T_TB * T_TR; q += 256) {
      const int cc = q / T_TR, rr = q % T_TR;
      const int64_t r = r0 + rr;
      const int b = b0 + cc;
      if (r < n && b < ncols) {
        const int64_t orow = perm ? perm[r] : r;
        out[(int64_t)b * ldo + orow] = sO[cc][rr];
      }
    }
  }
}

void launch_tsgemm(int64_t n, int ld, BlockList A, const double* C, const double* in, double* out,
                   float* out32, double alpha, double beta, const int* flag, hipStream_t st, bool upper,
                   bool tri0) {
  const int up = (upper && A.nb == 1) ? 1 : 0;
  // X -= A C against the float32 archive at widths 64 k: BF16 matrix cores
  if (A.f32 && !up && !out32 && !tri0 && in == out && alpha == -1.0 && beta == 1.0 && update_bf3_ok(ld)) {
    launch_update_bf3(n, ld, A, C, out, flag, st);
    return;
  }
  dim3 grid((unsigned)((n + T_TR - 1) / T_TR), (ld + T_TB - 1) / T_TB);
  // the float32 archive (reorthogonalisation update) on the FP32 matrix
  // cores; a triangular coefficient block or a float copy of the output
  // keeps the float64 kernel
  const bool f32mma = mfma_ok(ld) && A.f32 && !up && !out32;
  kt_begin(f32mma ? KC_ARCH_UPDATE : KC_TSGEMM, st);
  if (mfma_ok(ld)) {
    static_assert(MT_R == T_TR && MT_C == T_TB, "same tile grid");
    const dim3 g1(row_tile_grid((n + MT_R - 1) / MT_R, (ld + MT_C - 1) / MT_C));   // row_tile order
    if (f32mma)
      hipLaunchKernelGGL(tsgemm_f32mma_kernel, g1, dim3(256), 0, st, n, ld, (const float*)A.base, A.stride, A.nb, C,
                         in, out, alpha, beta, flag);
    else if (A.f32)
      hipLaunchKernelGGL((tsgemm_mfma_kernel<true, false>), g1, dim3(256), 0, st, n, ld, A.base, A.stride, A.nb, C,
                         ld, ld, in, out, out32, alpha, beta, (int64_t)ld, (const int64_t*)nullptr, flag, up);
    else
      hipLaunchKernelGGL((tsgemm_mfma_kernel<false, false>), g1, dim3(256), 0, st, n, ld, A.base, A.stride, A.nb,
                         C, ld, ld, in, out, out32, alpha, beta, (int64_t)ld, (const int64_t*)nullptr, flag, up);
  } else if (A.f32)
    hipLaunchKernelGGL((tsgemm_kernel<true, false>), grid, dim3(256), 0, st, n, ld, ld, A.base, A.stride,
                       A.nb, C, ld, in, out, out32, alpha, beta, (int64_t)ld, (const int64_t*)nullptr,
                       flag);
  else
    hipLaunchKernelGGL((tsgemm_kernel<false, false>), grid, dim3(256), 0, st, n, ld, ld, A.base,
                       A.stride, A.nb, C, ld, in, out, out32, alpha, beta, (int64_t)ld,
                       (const int64_t*)nullptr, flag);
  GK_HIP(hipGetLastError());
  // method's own flops: a triangular coefficient block (R^-1, or B_{k-1}^T
  // of the recurrence) costs n ld (ld + 1)
  const int ntri = (up || tri0) ? 1 : 0;
  kt_end(st, (double)n * ld * ((A.f32 ? 4.0 : 8.0) * A.nb + (beta != 0.0 ? 16.0 : 8.0) + (out32 ? 4.0 : 0.0)),
         2.0 * (double)n * ld * ld * (A.nb - ntri) + ntri * (double)n * ld * (ld + 1), flag);
}

void launch_assemble(int64_t n, int ld, int s, BlockList A, const double* U, int ldu, double* P,
                     const int64_t* perm, hipStream_t st) {
  dim3 grid((unsigned)((n + T_TR - 1) / T_TR), (s + T_TB - 1) / T_TB);
  kt_begin(KC_ASSEMBLE, st);
  if (mfma_ok(ld)) {
    const dim3 g1(row_tile_grid((n + MT_R - 1) / MT_R, (s + MT_C - 1) / MT_C));   // row_tile order
    if (A.f32)
      hipLaunchKernelGGL(assemble_f32mma_kernel, g1, dim3(256), 0, st, n, ld, (const float*)A.base, A.stride, A.nb,
                         U, ldu, s, P, n, perm);
    else
      hipLaunchKernelGGL((tsgemm_mfma_kernel<false, true>), g1, dim3(256), 0, st, n, ld, A.base, A.stride, A.nb, U,
                         ldu, s, (const double*)nullptr, P, (float*)nullptr, 1.0, 0.0, n, perm, (const int*)nullptr,
                         0);
  } else if (A.f32)
    hipLaunchKernelGGL((tsgemm_kernel<true, true>), grid, dim3(256), 0, st, n, ld, s, A.base, A.stride,
                       A.nb, U, ldu, (const double*)nullptr, P, (float*)nullptr, 1.0, 0.0, n, perm,
                       (const int*)nullptr);
  else
    hipLaunchKernelGGL((tsgemm_kernel<false, true>), grid, dim3(256), 0, st, n, ld, s, A.base, A.stride,
                       A.nb, U, ldu, (const double*)nullptr, P, (float*)nullptr, 1.0, 0.0, n, perm,
                       (const int*)nullptr);
  GK_HIP(hipGetLastError());
  kt_end(st, (double)n * ((A.f32 ? 4.0 : 8.0) * ld * A.nb + 8.0 * s), 2.0 * (double)n * ld * s * A.nb);
}

// ------------------------------------------------------------- predictor
// out[perm[r]] = sum_k sum_c A_k[r, c] z[k ld + c] (the GEMV of the kernel
// machine predictor, HBM-bound): q lanes per row (a power of two with
// 16 q >= ld), lane j reading float4 / double4 groups j, j + q, .. of each
// block row (contiguous across the lanes of a row), float64 accumulation,
// butterfly reduction over the q lanes.
template <bool F32>
__global__ void __launch_bounds__(256)
predict_kernel(int64_t n, int ld, int q, const void* __restrict__ Abase, int64_t astride, int nb,
               const double* __restrict__ z, double* __restrict__ out, const int64_t* __restrict__ perm) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r = t / q;
  const int j = (int)(t - r * q);
  double acc = 0.0;
  if (r < n) {
    for (int k = 0; k < nb; ++k) {
      const int64_t base = (int64_t)k * astride + r * ld;
      const double* zk = z + (int64_t)k * ld;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = 4 * (j + q * u);
        if (c < ld) {
          double a0, a1, a2, a3;
          if (F32) {
            const float4 v = *reinterpret_cast<const float4*>(static_cast<const float*>(Abase) + base + c);
            a0 = v.x; a1 = v.y; a2 = v.z; a3 = v.w;
          } else {
            const double2* p = reinterpret_cast<const double2*>(static_cast<const double*>(Abase) + base + c);
            const double2 v0 = p[0], v1 = p[1];
            a0 = v0.x; a1 = v0.y; a2 = v1.x; a3 = v1.y;
          }
          acc = fma(a0, zk[c], acc);
          acc = fma(a1, zk[c + 1], acc);
          acc = fma(a2, zk[c + 2], acc);
          acc = fma(a3, zk[c + 3], acc);
        }
      }
    }
  }
  for (int o = q >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (r < n && j == 0) out[perm ? perm[r] : r] = acc;
}

void launch_predict(int64_t n, int ld, BlockList A, const double* z, double* out, const int64_t* perm,
                    hipStream_t st) {
  int q = 1;
  while (16 * q < ld) q <<= 1;
  GK_REQUIRE(q <= 64 && ld % 4 == 0, GK_EINVAL, "predictor: unsupported block width");
  const int64_t tot = n * q;
  kt_begin(KC_PREDICT, st);
  if (A.f32)
    hipLaunchKernelGGL(predict_kernel<true>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, ld, q, A.base,
                       A.stride, A.nb, z, out, perm);
  else
    hipLaunchKernelGGL(predict_kernel<false>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, ld, q,
                       A.base, A.stride, A.nb, z, out, perm);
  GK_HIP(hipGetLastError());
  kt_end(st, (double)n * ld * A.nb * (A.f32 ? 4.0 : 8.0) + 8.0 * n, 2.0 * (double)n * ld * A.nb);
}

// ------------------------------------------------- column-wise operations
// out[i, c] = sum_k D[k*ld + c] * A_k[i, c]
template <bool F32, bool COLMAJ>
__global__ void assemble_diag_kernel(int64_t n, int ld, int s, const void* __restrict__ Abase,
                                     int64_t astride, int nb, const double* __restrict__ D,
                                     double* __restrict__ P, const int64_t* __restrict__ perm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / ld;
  const int c = (int)(t - i * ld);
  if (i >= n || c >= s) return;
  double acc = 0.0;
  for (int k = 0; k < nb; ++k) acc = fma(D[k * ld + c], ldA<F32>(Abase, (int64_t)k * astride + i * ld + c), acc);
  const int64_t orow = perm ? perm[i] : i;
  if (COLMAJ)
    P[(int64_t)c * n + orow] = acc;
  else
    P[orow * ld + c] = acc;
}

void launch_assemble_diag(int64_t n, int ld, int s, BlockList A, const double* D, double* P,
                          const int64_t* perm, bool colmajor, hipStream_t st) {
  const int64_t tot = n * ld;
  dim3 grid((unsigned)((tot + 255) / 256));
#define GK_AD(F, CM)                                                                              \
  hipLaunchKernelGGL((assemble_diag_kernel<F, CM>), grid, dim3(256), 0, st, n, ld, s, A.base, A.stride, \
                     A.nb, D, P, perm)
  if (A.f32) {
    if (colmajor) GK_AD(true, true); else GK_AD(true, false);
  } else {
    if (colmajor) GK_AD(false, true); else GK_AD(false, false);
  }
#undef GK_AD
  GK_HIP(hipGetLastError());
}

// part[chunk][k*ld + c] = sum_{i in chunk} A_k[i,c] * B[i,c]
template <bool F32>
__global__ void __launch_bounds__(256)
coldots_kernel(int64_t n, int ld, const void* __restrict__ Abase, int64_t astride, int nb,
               const double* __restrict__ B, double* __restrict__ part, int64_t rows_per_chunk,
               const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  __shared__ double red[256];
  const int cols = ld < 256 ? ld : 256;
  const int groups = 256 / cols;
  const int64_t r_begin = (int64_t)blockIdx.x * rows_per_chunk;
  const int64_t r_end = min(n, r_begin + rows_per_chunk);
  const int tid = threadIdx.x;
  const int cl = tid % cols, gr = tid / cols;
  double* P = part + (int64_t)blockIdx.x * nb * ld;
  for (int cb = 0; cb < ld; cb += cols) {
    const int c = cb + cl;
    for (int k = 0; k < nb; ++k) {
      double sacc = 0.0;
      if (gr < groups && c < ld)
        for (int64_t r = r_begin + gr; r < r_end; r += groups)
          sacc = fma(ldA<F32>(Abase, (int64_t)k * astride + r * ld + c), B[r * ld + c], sacc);
      red[tid] = sacc;
      __syncthreads();
      if (tid < cols && c < ld) {
        double t = 0.0;
        for (int q = 0; q < groups; ++q) t += red[q * cols + tid];
        P[k * ld + c] = t;
      }
      __syncthreads();
    }
  }
}

static void coldots_geometry(int64_t n, int* nch, int64_t* rpc) {
  int64_t want = 512;
  int64_t maxc = (n + 63) / 64;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  int64_t r = (n + want - 1) / want;
  *rpc = r;
  *nch = (int)((n + r - 1) / r);
}

size_t coldots_scratch_elems(int64_t n, int nb, int ld) {
  int nch;
  int64_t rpc;
  coldots_geometry(n, &nch, &rpc);
  return (size_t)nch * nb * ld;
}

void launch_coldots(int64_t n, int ld, BlockList A, const double* B, double* out, double* part,
                    const int* flag, hipStream_t st) {
  int nch;
  int64_t rpc;
  coldots_geometry(n, &nch, &rpc);
  if (A.f32)
    hipLaunchKernelGGL(coldots_kernel<true>, dim3(nch), dim3(256), 0, st, n, ld, A.base, A.stride, A.nb,
                       B, part, rpc, flag);
  else
    hipLaunchKernelGGL(coldots_kernel<false>, dim3(nch), dim3(256), 0, st, n, ld, A.base, A.stride, A.nb,
                       B, part, rpc, flag);
  GK_HIP(hipGetLastError());
  launch_reduce_parts((int64_t)A.nb * ld, nch, part, out, flag, st);
}

template <bool F32>
__global__ void axpy_diag_kernel(int64_t n, int ld, const void* __restrict__ Abase, int64_t astride,
                                 int nb, const double* __restrict__ D, double* __restrict__ X,
                                 const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ld) return;
  const int c = (int)(t % ld);
  double x = X[t];
  for (int k = 0; k < nb; ++k) x = fma(-D[k * ld + c], ldA<F32>(Abase, (int64_t)k * astride + t), x);
  X[t] = x;
}

void launch_axpy_diag(int64_t n, int ld, BlockList A, const double* D, double* X, const int* flag,
                      hipStream_t st) {
  const int64_t tot = n * ld;
  dim3 grid((unsigned)((tot + 255) / 256));
  if (A.f32)
    hipLaunchKernelGGL(axpy_diag_kernel<true>, grid, dim3(256), 0, st, n, ld, A.base, A.stride, A.nb, D,
                       X, flag);
  else
    hipLaunchKernelGGL(axpy_diag_kernel<false>, grid, dim3(256), 0, st, n, ld, A.base, A.stride, A.nb, D,
                       X, flag);
  GK_HIP(hipGetLastError());
}

__global__ void colscale_kernel(int64_t n, int ld, const double* __restrict__ X,
                                const double* __restrict__ scale, double* __restrict__ Y,
                                float* __restrict__ Y32) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * ld) return;
  const double v = X[t] * scale[t % ld];
  Y[t] = v;
  if (Y32) Y32[t] = (float)v;
}

void launch_colscale(int64_t n, int ld, const double* X, const double* scale, double* Y, float* Y32,
                     hipStream_t st) {
  const int64_t tot = n * ld;
  hipLaunchKernelGGL(colscale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, ld, X,
                     scale, Y, Y32);
  GK_HIP(hipGetLastError());
}

// out[r*s + c] = sum_k D[k*ld + c] * A_k[rows[r], c]   (D == null: single block, weight 1)
template <bool F32>
__global__ void gather_rows_kernel(int ld, int s, const void* __restrict__ Abase, int64_t astride,
                                   int nb, const double* __restrict__ D, const int64_t* __restrict__ rows,
                                   double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= s * s) return;
  const int r = t / s, c = t % s;
  const int64_t i = rows[r];
  double acc = 0.0;
  for (int k = 0; k < nb; ++k) {
    const double w = D ? D[k * ld + c] : 1.0;
    acc = fma(w, ldA<F32>(Abase, (int64_t)k * astride + i * ld + c), acc);
  }
  out[t] = acc;
}

void launch_gather_diag(int64_t n, int ld, int s, BlockList A, const double* D, const int64_t* rows,
                        double* out, hipStream_t st) {
  (void)n;
  const int tot = s * s;
  if (A.f32)
    hipLaunchKernelGGL(gather_rows_kernel<true>, dim3((tot + 255) / 256), dim3(256), 0, st, ld, s, A.base,
                       A.stride, A.nb, D, rows, out);
  else
    hipLaunchKernelGGL(gather_rows_kernel<false>, dim3((tot + 255) / 256), dim3(256), 0, st, ld, s,
                       A.base, A.stride, A.nb, D, rows, out);
  GK_HIP(hipGetLastError());
}

// ------------------------------------------------------------ misc
__global__ void start_block_kernel(int64_t n, int ld, int s, const int64_t* __restrict__ samples,
                                   double value, double* __restrict__ V, float* __restrict__ V32) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= s) return;
  const int64_t w = samples[j];
  V[w * ld + j] = value;
  if (V32) V32[w * ld + j] = (float)value;
}

__global__ void zero_kernel(uint64_t* __restrict__ p, size_t words) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < words; i += stride) p[i] = 0;
}

void launch_zero(void* p, size_t bytes, hipStream_t st) {
  // buffers come from the arena and are multiples of 256 bytes
  const size_t words = (bytes + 7) / 8;
  size_t blocks = (words + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (uint64_t*)p, words);
  GK_HIP(hipGetLastError());
}

void launch_start_block(int64_t n, int ld, int s, const int64_t* dev_samples, double value, double* V,
                        float* V32, hipStream_t st) {
  launch_zero(V, (size_t)n * ld * sizeof(double), st);
  if (V32) launch_zero(V32, (size_t)n * ld * sizeof(float), st);
  hipLaunchKernelGGL(start_block_kernel, dim3((s + 255) / 256), dim3(256), 0, st, n, ld, s, dev_samples,
                     value, V, V32);
  GK_HIP(hipGetLastError());
}

__global__ void f64_to_f32_kernel(const double* __restrict__ a, float* __restrict__ b, size_t cnt) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) b[i] = (float)a[i];
}

void launch_copy_f64_to_f32(const double* a, float* b, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, a, b,
                     count);
  GK_HIP(hipGetLastError());
}

}  // namespace gk
