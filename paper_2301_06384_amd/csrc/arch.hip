// Reorthogonalisation of a block against the float32 basis archive on FP32
// matrix cores (mixed precision, block widths ld in {16, 32, 48, 64}):
//
//   C = Q^T X      (Q = [Q_1 .. Q_nb] archived blocks, X the new block)
//   X -= Q C
//
// The orthonormality of the Krylov basis assumed in Sec. 3 (and used by
// Theorem 3.1) is restored by this projection.  Coefficients only need the
// accuracy of the archive itself (unit roundoff 2^-24 relative to |Q||X|), so
// the products run as v_mfma_f32_16x16x4f32 with float accumulation over short
// row runs that are added into float64; partial sums are reduced in float64 in
// a fixed order (bitwise reproducible, no atomics).  The update at widths
// that are multiples of 64 (update_bf3_kernel, also used for the wide blocks)
// forms the same float32-accurate product on the BF16 matrix cores from a
// three-part split of its operands.
//
// v_mfma_f32_16x16x4f32 operand layout (lane l of 64, i = l % 16, k = l / 16):
//   A (16 x 4):  lane l holds A[i][k]
//   B (4 x 16):  lane l holds B[k][i]
//   D (16 x 16): register r of lane l holds D[4 k + r][i]
#include "gk_internal.h"
#include "decide.h"

namespace gk {

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------- Gram C = Q^T X
// Workgroup = 16 wavefronts over BPW = 16 / NT archive blocks and the row
// range of blockIdx.y; wavefront w owns column tile t = w % NT of block
// j = BPW bx + w / NT and accumulates C_j[:, 16t .. 16t+15] (NT row tiles).
// Rows go through LDS in rounds of AG_ROWS: every archive and X element is
// loaded once per workgroup (the NT wavefronts of a block share its rows),
// and the next round's loads are issued into registers before the current
// round's products, so a full round of products covers their latency.  X is
// staged as float.  The float MFMA accumulators are added into float64
// registers every 32 rows, which keeps the accumulation error of C at the
// level of a 32-term float sum.
constexpr int AG_WAVES = 16;
constexpr int AG_THREADS = 64 * AG_WAVES;
constexpr int AG_ROWS = 64;       // rows staged per LDS round
constexpr int AG_FLUSH = 8;       // 4-row steps between float64 flushes
constexpr int AG_TARGET_WG = 256; // one workgroup per compute unit

constexpr int ag_blocks(int nt) { return AG_WAVES / nt; }

template <int NT>
__global__ void __launch_bounds__(AG_THREADS, 1)
arch_gram_kernel(int64_t n, const float* __restrict__ Q, int64_t qstride, int nb, const double* __restrict__ X,
                 double* __restrict__ part, int64_t rpc, const int* __restrict__ flag, OmegaDecide dec) {
  if (dec.fr) {
    // the reorthogonalisation decision, taken by every workgroup (no launch
    // of its own on the steps that do not project)
    __shared__ double dred[AG_THREADS / 64];
    if (!omega_decide(dec, blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y, dred)) return;
  } else if (flag && *flag == 0) {
    return;
  }
  constexpr int LD = 16 * NT;
  constexpr int P = LD + 16;                 // LDS pitch (floats): the 4-row operand reads avoid bank conflicts
  constexpr int BPW = ag_blocks(NT);
  constexpr int Q4 = BPW * AG_ROWS * LD / 4; // float4 of archive rows per round
  constexpr int QV = (Q4 + AG_THREADS - 1) / AG_THREADS;
  constexpr int XE = AG_ROWS * LD / AG_THREADS;
  static_assert(XE * AG_THREADS == AG_ROWS * LD, "whole X rows per round");
  __shared__ __align__(16) float sQ[BPW * AG_ROWS * P];
  __shared__ float sX[AG_ROWS * P];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int wb = w / NT, t = w - wb * NT;
  const int j0 = blockIdx.x * BPW;
  const bool active = wb < BPW && j0 + wb < nb;
  const int64_t rb = (int64_t)blockIdx.y * rpc;
  const int64_t re = min(n, rb + rpc);

  f4 acc[NT];
  double a64[NT][4];
#pragma unroll
  for (int e = 0; e < NT; ++e) {
    acc[e] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 4; ++r) a64[e][r] = 0.0;
  }

  // Loads never sit behind a branch: rows past the range read row re - 1,
  // blocks past nb read block nb - 1 and entries past the round repeat the
  // last one; X rows past the range are zeroed in LDS, which cancels them.
  f4 qv[QV];
  double xv[XE];
  auto load_round = [&](int64_t r0) {
#pragma unroll
    for (int e = 0; e < QV; ++e) {
      const int q = min(tid + e * AG_THREADS, Q4 - 1) * 4;
      const int b = q / (AG_ROWS * LD), rem = q - b * (AG_ROWS * LD);
      const int rr = rem / LD, cc = rem - rr * LD;
      const int64_t r = min(r0 + rr, re - 1);
      const int jb = min(j0 + b, nb - 1);
      qv[e] = *reinterpret_cast<const f4*>(Q + (int64_t)jb * qstride + r * LD + cc);
    }
#pragma unroll
    for (int e = 0; e < XE; ++e) {
      const int q = tid + e * AG_THREADS;
      const int rr = q / LD, cc = q - rr * LD;
      xv[e] = X[min(r0 + rr, re - 1) * LD + cc];
    }
  };
  auto store_round = [&](int64_t r0) {
#pragma unroll
    for (int e = 0; e < QV; ++e) {
      const int q4 = tid + e * AG_THREADS;
      const int q = q4 * 4;
      const int b = q / (AG_ROWS * LD), rem = q - b * (AG_ROWS * LD);
      const int rr = rem / LD, cc = rem - rr * LD;
      if (q4 < Q4) *reinterpret_cast<f4*>(&sQ[(b * AG_ROWS + rr) * P + cc]) = qv[e];
    }
#pragma unroll
    for (int e = 0; e < XE; ++e) {
      const int q = tid + e * AG_THREADS;
      const int rr = q / LD, cc = q - rr * LD;
      sX[rr * P + cc] = r0 + rr < re ? (float)xv[e] : 0.f;
    }
  };

  load_round(rb);
  const float* sQw = sQ + wb * AG_ROWS * P;
  for (int64_t r0 = rb; r0 < re; r0 += AG_ROWS) {
    store_round(r0);
    __syncthreads();
    load_round(r0 + AG_ROWS);   // past the range at the end: clamped, unused
    if (active) {
#pragma unroll
      for (int h = 0; h < AG_ROWS / (4 * AG_FLUSH); ++h) {
#pragma unroll
        for (int s8 = 0; s8 < AG_FLUSH; ++s8) {
          const int rr = 4 * (h * AG_FLUSH + s8) + lk;
          // B (4 x 16) = X[rows][16 t ..], A (16 x 4) = Q_j[rows][16 a ..]^T
          const float b = sX[rr * P + 16 * t + li];
#pragma unroll
          for (int a = 0; a < NT; ++a) acc[a] = mfma32(sQw[rr * P + 16 * a + li], b, acc[a]);
        }
#pragma unroll
        for (int a = 0; a < NT; ++a) {
#pragma unroll
          for (int q = 0; q < 4; ++q) a64[a][q] += (double)acc[a][q];
          acc[a] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
    __syncthreads();
  }
  if (active) {
    // D_a[4k + r][i] = C_j[16 a + 4 k + r][16 t + i]
    double* P0 = part + ((int64_t)blockIdx.y * nb + j0 + wb) * LD * LD;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) P0[(16 * a + 4 * lk + r) * LD + 16 * t + li] = a64[a][r];
  }
}

// ---------------------------------------------------------- update X -= Q C
// Workgroup = 4 wavefronts over 128 rows; wavefront w owns rows 32 w .. 32 w + 31
// as two groups of 16.  The product is formed transposed, D = C^T Q^T, so
// that the archive rows are the B operand: lane (i, k) loads the LD/4
// consecutive floats Q_j[row i][k LD/4 .. (k+1) LD/4 - 1] (float4 loads), and
// operand e contracts over the columns {k LD/4 + e}.  The coefficient block
// C_j (float64) is staged in LDS as float, double buffered over j.
constexpr int AU_ROWS = 128;
// Pitch (floats) of the coefficients staged for the update and the assembly:
// a product step reads rows lk KQ + e (KQ = 4 NT) at 16 consecutive columns
// per lane group lk, and LDS serves 32-bit reads 32 lanes at a time over 32
// banks, so KQ PC = 16 (mod 32) puts groups lk = 0, 1 (and 2, 3) on disjoint
// bank halves.
constexpr int arch_pc(int nt) { return 16 * nt + (nt == 4 ? 1 : (nt == 2 ? 2 : 4)); }
static_assert((4 * arch_pc(1)) % 32 == 16 && (8 * arch_pc(2)) % 32 == 16 && (12 * arch_pc(3)) % 32 == 16 &&
                  (16 * arch_pc(4)) % 32 == 16,
              "coefficient pitch");

template <int NT>
__global__ void __launch_bounds__(256, 2)
arch_update_kernel(int64_t n, const float* __restrict__ Q, int64_t qstride, int nb, const double* __restrict__ C,
                   double* __restrict__ X, const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  constexpr int LD = 16 * NT;
  constexpr int KQ = LD / 4;                 // floats per lane per block row
  constexpr int PC = arch_pc(NT);            // LDS pitch of the staged coefficients
  __shared__ float sC[2][LD * PC];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int64_t R0 = (int64_t)blockIdx.x * AU_ROWS + 32 * w;

  f4 acc[2][NT];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[g][t] = f4{0.f, 0.f, 0.f, 0.f};

  // coefficient block jb -> registers (all loads issued together) -> LDS
  constexpr int CE = LD * LD / 256;
  auto fetch_c = [&](int jb, double (&cv)[CE]) {
    const double* Cj = C + (int64_t)jb * LD * LD;
#pragma unroll
    for (int e = 0; e < CE; ++e) cv[e] = Cj[tid + 256 * e];
  };
  auto put_c = [&](int buf, const double (&cv)[CE]) {
#pragma unroll
    for (int e = 0; e < CE; ++e) {
      const int q = tid + 256 * e;
      const int a = q / LD, b = q - a * LD;
      sC[buf][a * PC + b] = (float)cv[e];
    }
  };
  auto load_q = [&](int jb, float (&qv)[2][KQ]) {
    const float* Qj = Q + (int64_t)jb * qstride;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      // rows past n read row n - 1: their results are never stored
      const int64_t r = R0 + 16 * g + li;
      const int64_t rc = r < n ? r : n - 1;
#pragma unroll
      for (int v = 0; v < KQ / 4; ++v) {
        const f4 x = *reinterpret_cast<const f4*>(Qj + rc * LD + lk * KQ + 4 * v);
        qv[g][4 * v] = x[0];
        qv[g][4 * v + 1] = x[1];
        qv[g][4 * v + 2] = x[2];
        qv[g][4 * v + 3] = x[3];
      }
    }
  };

  // One archive block per step.  The loads of the next block (at the end the
  // last block again, unused) are issued unconditionally before the
  // products, so the wait in front of the first product covers only the
  // current block's operands; the two register sets alternate.
  auto step = [&](int jb, const float (&qc)[2][KQ], float (&qn)[2][KQ]) {
    const int jn = jb + 1 < nb ? jb + 1 : nb - 1;
    double cnext[CE];
    fetch_c(jn, cnext);
    load_q(jn, qn);
    if (jb < nb) {
      const float* sc = sC[jb & 1];
#pragma unroll
      for (int e = 0; e < KQ; ++e) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float cv = sc[(lk * KQ + e) * PC + 16 * t + li];
#pragma unroll
          for (int g = 0; g < 2; ++g) acc[g][t] = mfma32(cv, qc[g][e], acc[g][t]);
        }
      }
    }
    if (jb + 1 < nb) put_c((jb & 1) ^ 1, cnext);
    __syncthreads();
  };
  float q0[2][KQ], q1[2][KQ];
  {
    double c0[CE];
    fetch_c(0, c0);
    put_c(0, c0);
  }
  load_q(0, q0);
  __syncthreads();
  for (int jb = 0; jb < nb; jb += 2) {
    step(jb, q0, q1);
    step(jb + 1, q1, q0);
  }
  // D_{g,t}[4k + r][i] = (Q C)[row 16 g + i][16 t + 4 k + r]
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int64_t r = R0 + 16 * g + li;
    if (r >= n) continue;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double* xp = X + r * LD + 16 * t + 4 * lk;
#pragma unroll
      for (int q = 0; q < 4; ++q) xp[q] -= (double)acc[g][t][q];
    }
  }
}

// ------------------------------------- update X -= Q C on BF16 matrix cores
// For ld a multiple of 64: the same product as above on the BF16 matrix
// cores, which issue sixteen times the FP32 rate.  Every float32 operand x is
// cut into three bfloat16 parts by truncation, x0 = the upper 16 bits of x,
// x1 = those of x - x0 and x2 = x - x0 - x1; the cut is exact, each part
// carrying 8 of the 24 significand bits (|x1| < 2^-7 |x|, |x2| < 2^-15 |x|).
// Of the nine part products of q c the six with i + j <= 2 are formed; the
// other three are together below 2^-21 |q| |c|, a few float32 rounding units.
// Each part product is exact in the float accumulator.  The update is a
// small correction of X (it runs when the estimated loss of orthogonality
// reaches 2^-16 in cbl, 2^-12 in gbl and sbl), so this error is far below the
// float32 rounding of the archive itself.
//
// v_mfma_f32_16x16x32_bf16 operand layout (lane l, i = l % 16, k = l / 16):
//   A (16 x 32): lane l holds A[i][8 k .. 8 k + 7]
//   B (32 x 16): lane l holds B[8 k .. 8 k + 7][i]
//   D (16 x 16): register r of lane l holds D[4 k + r][i]
//
// Workgroup = 4 wavefronts over 128 rows and 64 columns of X (column tile
// tb); wavefront w owns rows 32 w .. 32 w + 31 as two groups of 16.  The
// contraction runs over the archive columns in chunks of 64 (a chunk never
// crosses an archive block since ld % 64 == 0).  Per chunk, a lane splits its
// archive entries Q[row][32 h + 8 k .. + 7] (h = 0, 1) into the B operands,
// and the workgroup splits the 64 x 64 coefficient tile once into three
// planes in LDS.  A plane is stored per X column as 32 dwords of contraction
// index pairs, its 16-byte chunks XOR-swizzled by the column, so that the
// 128-bit operand reads and stores (eight lanes at a time) spread over all
// 32 banks.  The float accumulators run over the whole contraction.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma_bf3(u4 a, u4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// the three parts of x in the lower halves, of y in the upper halves
__device__ __forceinline__ void split3(float x, float y, unsigned& h, unsigned& m, unsigned& l) {
  const unsigned xb = __float_as_uint(x), yb = __float_as_uint(y);
  const float xr = x - __uint_as_float(xb & 0xffff0000u), yr = y - __uint_as_float(yb & 0xffff0000u);
  const unsigned xrb = __float_as_uint(xr), yrb = __float_as_uint(yr);
  const float xl = xr - __uint_as_float(xrb & 0xffff0000u), yl = yr - __uint_as_float(yrb & 0xffff0000u);
  h = __builtin_amdgcn_perm(yb, xb, 0x07060302u);
  m = __builtin_amdgcn_perm(yrb, xrb, 0x07060302u);
  l = __builtin_amdgcn_perm(__float_as_uint(yl), __float_as_uint(xl), 0x07060302u);
}

constexpr int UB_PLANE = 64 * 32;   // dwords per coefficient plane

__global__ void __launch_bounds__(256, 3)
update_bf3_kernel(int64_t n, int ld, const float* __restrict__ Q, int64_t qstride, int nb,
                  const double* __restrict__ C, double* __restrict__ X, const int* __restrict__ flag) {
  if (flag && *flag == 0) return;
  // tiles: the column tiles of row tile rt are consecutive workgroups of XCD
  // rt % 8, so the archive rows they share come from one L2
  const int nct = ld >> 6;
  const int64_t nrt = (n + AU_ROWS - 1) / AU_ROWS;
  const unsigned L = blockIdx.x, xcd = L & 7, jt = L >> 3;
  const int tb = (int)(jt % (unsigned)nct);
  const int64_t rt = (int64_t)(jt / (unsigned)nct) * 8 + xcd;
  if (rt >= nrt) return;
  const int b0 = 64 * tb;
  const int nch = nb * nct;   // 64-index chunks of the contraction
  __shared__ __align__(16) unsigned sC[2][3 * UB_PLANE];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int64_t R0 = rt * AU_ROWS + 32 * w;

  f4 acc[2][4];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[g][t] = f4{0.f, 0.f, 0.f, 0.f};

  // coefficient staging: wavefront w stages rows 16 w .. 16 w + 15 of the
  // 64 x 64 tile, lane l column l (64 consecutive doubles per load), and
  // stores them as the 16-byte chunks 2 w and 2 w + 1 of column l
  const int wu = __builtin_amdgcn_readfirstlane(w);
  auto fetch_c = [&](int jc, double (&cv)[16]) {
    const double* Cj = C + ((int64_t)jc * 64 + 16 * wu) * ld + b0;
#pragma unroll
    for (int j = 0; j < 16; ++j) cv[j] = Cj[(int64_t)j * ld + l];
  };
  auto put_c = [&](int buf, const double (&cv)[16]) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      u4 h, m, lo;
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        unsigned x0, x1, x2;
        split3((float)cv[8 * e + 2 * p], (float)cv[8 * e + 2 * p + 1], x0, x1, x2);
        h[p] = x0;
        m[p] = x1;
        lo[p] = x2;
      }
      const int o = l * 32 + (((2 * wu + e) ^ (l & 7)) << 2);
      *reinterpret_cast<u4*>(&sC[buf][o]) = h;
      *reinterpret_cast<u4*>(&sC[buf][UB_PLANE + o]) = m;
      *reinterpret_cast<u4*>(&sC[buf][2 * UB_PLANE + o]) = lo;
    }
  };
  // lane (i, k) of row group g: Q[row][32 h + 8 k .. 32 h + 8 k + 7] of the chunk
  auto load_q = [&](int jc, float (&qv)[2][16]) {
    const int blk = jc / nct;
    const float* Qj = Q + (int64_t)blk * qstride + 64 * (jc - blk * nct);
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      // rows past n read row n - 1: their results are never stored
      const int64_t r = R0 + 16 * g + li;
      const int64_t rc = r < n ? r : n - 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const f4 x = *reinterpret_cast<const f4*>(Qj + rc * ld + 32 * (v >> 1) + 8 * lk + 4 * (v & 1));
        qv[g][4 * v] = x[0];
        qv[g][4 * v + 1] = x[1];
        qv[g][4 * v + 2] = x[2];
        qv[g][4 * v + 3] = x[3];
      }
    }
  };

  // One chunk per step.  The next chunk's archive rows (at the end the last
  // chunk again, unused) are loaded before the products; its coefficients,
  // read from L2, once half the archive operands are spent (registers).
  auto step = [&](int jc, const float (&qc)[2][16], float (&qn)[2][16]) {
    const int jn = jc + 1 < nch ? jc + 1 : nch - 1;
    double cnext[16];
    load_q(jn, qn);
    const unsigned* sc = sC[jc & 1];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (h == 1) fetch_c(jn, cnext);
      if (jc >= nch) continue;
      u4 bh[2], bm[2], bl[2];
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          unsigned x0, x1, x2;
          split3(qc[g][8 * h + 2 * p], qc[g][8 * h + 2 * p + 1], x0, x1, x2);
          bh[g][p] = x0;
          bm[g][p] = x1;
          bl[g][p] = x2;
        }
      const int ch = ((4 * h + lk) ^ (li & 7)) << 2;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const unsigned* base = sc + (16 * t + li) * 32 + ch;
        const u4 ah = *reinterpret_cast<const u4*>(base);
        const u4 am = *reinterpret_cast<const u4*>(base + UB_PLANE);
        const u4 al = *reinterpret_cast<const u4*>(base + 2 * UB_PLANE);
        // smallest part products first
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[g][t] = mfma_bf3(al, bh[g], acc[g][t]);
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[g][t] = mfma_bf3(am, bm[g], acc[g][t]);
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[g][t] = mfma_bf3(ah, bl[g], acc[g][t]);
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[g][t] = mfma_bf3(am, bh[g], acc[g][t]);
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[g][t] = mfma_bf3(ah, bm[g], acc[g][t]);
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[g][t] = mfma_bf3(ah, bh[g], acc[g][t]);
      }
    }
    if (jc + 1 < nch) put_c((jc & 1) ^ 1, cnext);
    __syncthreads();
  };
  float q0[2][16], q1[2][16];
  {
    double c0[16];
    fetch_c(0, c0);
    put_c(0, c0);
  }
  load_q(0, q0);
  __syncthreads();
  for (int jc = 0; jc < nch; jc += 2) {
    step(jc, q0, q1);
    step(jc + 1, q1, q0);
  }
  // D_{g,t}[4k + r][i] = (Q C)[row 16 g + i][b0 + 16 t + 4 k + r]
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int64_t r = R0 + 16 * g + li;
    if (r >= n) continue;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      double* xp = X + r * ld + b0 + 16 * t + 4 * lk;
#pragma unroll
      for (int q = 0; q < 4; ++q) xp[q] -= (double)acc[g][t][q];
    }
  }
}

// ------------------------------------------------------- assembly P = Q U
// P[perm(r), c] = sum_j Q_j[r, :] U_j[:, c] for c < s (Alg. 1 output
// [Q_1 .. Q_m] phi(H_m) F_1): float32 archive and coefficients rounded to
// float on matrix cores, same operand scheme as the update kernel; the float
// accumulators are added into float64 after every archive block.  Output
// column-major n x s in caller node order (perm may be null).
template <int NT>
__global__ void __launch_bounds__(256, 2)
arch_assemble_kernel(int64_t n, const float* __restrict__ Q, int64_t qstride, int nb, const double* __restrict__ U,
                     int s, double* __restrict__ P, const int64_t* __restrict__ perm) {
  constexpr int LD = 16 * NT;
  constexpr int KQ = LD / 4;
  constexpr int PC = arch_pc(NT);
  __shared__ float sC[2][LD * PC];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, li = l & 15, lk = l >> 4;
  const int64_t R0 = (int64_t)blockIdx.x * AU_ROWS + 32 * w;

  f4 acc[2][NT];
  double a64[2][NT][4];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[g][t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) a64[g][t][q] = 0.0;
    }

  // coefficient block jb -> LDS as float, NT loads in flight per thread
  // (columns past s read column s - 1 and are zeroed)
  constexpr int CE = LD * LD / 256;   // = NT * NT
  auto stage = [&](int jb, int buf) {
    const double* Uj = U + (int64_t)jb * LD * s;
    constexpr int G4 = NT;
#pragma unroll
    for (int e0 = 0; e0 < CE; e0 += G4) {
      double cv[G4];
#pragma unroll
      for (int e = 0; e < G4; ++e) {
        const int q = tid + 256 * (e0 + e);
        const int a = q / LD, b = q - a * LD;
        cv[e] = Uj[(int64_t)a * s + (b < s ? b : s - 1)];
      }
#pragma unroll
      for (int e = 0; e < G4; ++e) {
        const int q = tid + 256 * (e0 + e);
        const int a = q / LD, b = q - a * LD;
        sC[buf][a * PC + b] = b < s ? (float)cv[e] : 0.f;
      }
    }
  };

  auto load_q = [&](int jb, float (&qv)[2][KQ]) {
    const float* Qj = Q + (int64_t)jb * qstride;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      // rows past n read row n - 1: their results are never stored
      const int64_t r = R0 + 16 * g + li;
      const int64_t rc = r < n ? r : n - 1;
#pragma unroll
      for (int v = 0; v < KQ / 4; ++v) {
        const f4 x = *reinterpret_cast<const f4*>(Qj + rc * LD + lk * KQ + 4 * v);
        qv[g][4 * v] = x[0];
        qv[g][4 * v + 1] = x[1];
        qv[g][4 * v + 2] = x[2];
        qv[g][4 * v + 3] = x[3];
      }
    }
  };

  // The next block's archive rows are loaded before the products
  // (unconditionally, the last block again at the end), so the wait in front
  // of the first product covers only the current block.  The next coefficient
  // block is staged after the products: the float64 accumulators leave no
  // registers to hold it across them.
  float qcur[2][KQ];
  stage(0, 0);
  load_q(0, qcur);
  __syncthreads();
  for (int jb = 0; jb < nb; ++jb) {
    float qnext[2][KQ];
    load_q(jb + 1 < nb ? jb + 1 : nb - 1, qnext);
    __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of the products
    const float* sc = sC[jb & 1];
#pragma unroll
    for (int e = 0; e < KQ; ++e) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const float c = sc[(lk * KQ + e) * PC + 16 * t + li];
#pragma unroll
        for (int g = 0; g < 2; ++g) acc[g][t] = mfma32(c, qcur[g][e], acc[g][t]);
      }
    }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a64[g][t][q] += (double)acc[g][t][q];
        acc[g][t] = f4{0.f, 0.f, 0.f, 0.f};
      }
    if (jb + 1 < nb) stage(jb + 1, (jb & 1) ^ 1);
    __syncthreads();
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int e = 0; e < KQ; ++e) qcur[g][e] = qnext[g][e];
  }
  // D_{g,t}[4k + r][i] = P[row 16 g + i][16 t + 4 k + r]
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int64_t r = R0 + 16 * g + li;
    if (r >= n) continue;
    const int64_t orow = perm ? perm[r] : r;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = 16 * t + 4 * lk + q;
        if (c < s) P[(int64_t)c * n + orow] = a64[g][t][q];
      }
  }
}

// ------------------------------------------------------------------ launchers
bool arch_ok(int ld) { return ld == 16 || ld == 32 || ld == 48 || ld == 64; }

bool update_bf3_ok(int ld) { return ld >= 64 && ld % 64 == 0; }

void launch_update_bf3(int64_t n, int ld, BlockList A, const double* C, double* X, const int* flag, hipStream_t st) {
  GK_REQUIRE(A.f32 && A.stride > 0 && A.nb >= 1 && update_bf3_ok(ld) && n >= 1, GK_EUNSUPPORTED,
             "the BF16 archive update needs a float32 archive and ld % 64 == 0");
  const int64_t nrt = (n + AU_ROWS - 1) / AU_ROWS;
  const int64_t grid = 8 * ((nrt + 7) / 8) * (ld / 64);
  GK_REQUIRE(grid <= 0x7fffffff, GK_EUNSUPPORTED, "archive update grid too large");
  kt_begin(KC_ARCH_UPDATE, st);
  hipLaunchKernelGGL(update_bf3_kernel, dim3((unsigned)grid), dim3(256), 0, st, n, ld,
                     static_cast<const float*>(A.base), A.stride, A.nb, C, X, flag);
  GK_HIP(hipGetLastError());
  kt_end(st, 4.0 * (double)n * ld * A.nb + 16.0 * (double)n * ld, 2.0 * (double)n * ld * ld * A.nb, flag);
}

static void arch_gram_geometry(int64_t n, int nb, int ld, int* ngroups, int* nchunks, int64_t* rpc) {
  const int bpw = ag_blocks(ld / 16);
  *ngroups = (nb + bpw - 1) / bpw;
  int64_t want = AG_TARGET_WG / *ngroups;    // at most one round of workgroups
  const int64_t maxc = (n + AG_ROWS - 1) / AG_ROWS;
  if (want > maxc) want = maxc;
  if (want < 1) want = 1;
  int64_t r = (n + want - 1) / want;
  r = ((r + AG_ROWS - 1) / AG_ROWS) * AG_ROWS;
  *rpc = r;
  *nchunks = (int)((n + r - 1) / r);
}

size_t arch_scratch_elems(int64_t n, int nb_max, int ld) {
  size_t mx = 0;
  for (int nb = 1; nb <= nb_max; ++nb) {
    int ng, nc;
    int64_t rpc;
    arch_gram_geometry(n, nb, ld, &ng, &nc, &rpc);
    mx = std::max(mx, (size_t)nc * nb * ld * ld);
  }
  return mx;
}

template <int NT>
static void arch_launch(int64_t n, BlockList A, double* X, double* C, double* part, const int* flag, hipStream_t st,
                        const OmegaDecide* dec) {
  const float* Q = static_cast<const float*>(A.base);
  int ng, nc;
  int64_t rpc;
  arch_gram_geometry(n, A.nb, 16 * NT, &ng, &nc, &rpc);
  const double qb = 4.0 * (double)n * 16 * NT * A.nb, xb = 8.0 * (double)n * 16 * NT;
  const double fl = 2.0 * (double)n * 16 * NT * 16 * NT * A.nb;
  kt_begin(KC_ARCH_GRAM, st);
  const OmegaDecide dv = dec ? *dec : OmegaDecide{};
  hipLaunchKernelGGL(arch_gram_kernel<NT>, dim3(ng, nc), dim3(AG_THREADS), 0, st, n, Q, A.stride, A.nb,
                     (const double*)X, part, rpc, flag, dv);
  GK_HIP(hipGetLastError());
  kt_end(st, qb + xb, fl, flag);
  const int64_t len = (int64_t)A.nb * 16 * NT * 16 * NT;
  launch_reduce_parts(len, nc, part, C, flag, st);
  if constexpr (NT == 4) {
    launch_update_bf3(n, 64, A, C, X, flag, st);
  } else {
    kt_begin(KC_ARCH_UPDATE, st);
    hipLaunchKernelGGL(arch_update_kernel<NT>, dim3((unsigned)((n + AU_ROWS - 1) / AU_ROWS)), dim3(256), 0, st, n,
                       Q, A.stride, A.nb, (const double*)C, X, flag);
    GK_HIP(hipGetLastError());
    kt_end(st, qb + 2.0 * xb, fl, flag);
  }
}

// One projection X -= Q (Q^T X) against the float32 archive A (A.f32, A.stride
// > 0, blocks n x ld row-major).  C receives the nb*ld x ld coefficients.  The
// Gram launch takes the decision dec when given (its workgroups return at
// once when it is negative) and otherwise tests the flag.
void launch_arch_reorth(int64_t n, int ld, BlockList A, double* X, double* C, double* part, const int* flag,
                        hipStream_t st, const OmegaDecide* dec) {
  GK_REQUIRE(A.f32 && A.stride > 0 && A.nb >= 1, GK_EUNSUPPORTED, "archive projection needs a float32 archive");
  GK_REQUIRE(!dec || (dec->fr && flag == dec->fr + dec->k), GK_EINVAL, "the decision must write the gating flag");
  switch (ld) {
    case 16: arch_launch<1>(n, A, X, C, part, flag, st, dec); break;
    case 32: arch_launch<2>(n, A, X, C, part, flag, st, dec); break;
    case 48: arch_launch<3>(n, A, X, C, part, flag, st, dec); break;
    case 64: arch_launch<4>(n, A, X, C, part, flag, st, dec); break;
    default: throw Error{GK_EUNSUPPORTED, "archive projection needs ld in {16,32,48,64}"};
  }
}

}  // namespace gk

namespace gk {

template <int NT>
static void arch_assemble_launch(int64_t n, int s, BlockList A, const double* U, double* P, const int64_t* perm,
                                 hipStream_t st) {
  kt_begin(KC_ASSEMBLE, st);
  hipLaunchKernelGGL(arch_assemble_kernel<NT>, dim3((unsigned)((n + AU_ROWS - 1) / AU_ROWS)), dim3(256), 0, st, n,
                     static_cast<const float*>(A.base), A.stride, A.nb, U, s, P, perm);
  GK_HIP(hipGetLastError());
  kt_end(st, (double)n * (4.0 * 16 * NT * A.nb + 8.0 * s), 2.0 * (double)n * 16 * NT * s * A.nb);
}

// P (column-major n x s, caller order through perm) = [A_1 .. A_nb] U with U
// (nb*ld x s, row-major) for a float32 archive with ld in {16, 32, 48, 64}.
void launch_arch_assemble(int64_t n, int ld, int s, BlockList A, const double* U, double* P, const int64_t* perm,
                          hipStream_t st) {
  GK_REQUIRE(A.f32 && A.stride > 0 && A.nb >= 1 && s >= 1 && s <= ld, GK_EUNSUPPORTED,
             "archive assembly needs a float32 archive and s <= ld");
  switch (ld) {
    case 16: arch_assemble_launch<1>(n, s, A, U, P, perm, st); break;
    case 32: arch_assemble_launch<2>(n, s, A, U, P, perm, st); break;
    case 48: arch_assemble_launch<3>(n, s, A, U, P, perm, st); break;
    case 64: arch_assemble_launch<4>(n, s, A, U, P, perm, st); break;
    default: throw Error{GK_EUNSUPPORTED, "archive assembly needs ld in {16,32,48,64}"};
  }
}

}  // namespace gk
