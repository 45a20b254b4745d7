// Fused row-panel kernels on FP64 matrix cores for the local block
// orthogonalisation of classical block Lanczos (Alg. 1: H_kk = Q_k^T X,
// X -= Q_k H_kk, QR of X) with block widths ld in {16, 32, 48, 64}.
//
// A workgroup (4 wavefronts) walks over row tiles of the n x ld blocks (32
// rows; 16 for the two-block update at ld >= 48).
// Per tile it stages the rows of X and of the local basis blocks in LDS, forms
// the updated rows X_new (X - V C, or X R) on MFMA, optionally writes them,
// and accumulates Gram products G^T X_new (G = basis blocks and/or X_new
// itself) in registers across all its tiles.  Per-workgroup Gram partials are
// summed afterwards in a fixed order (no atomics: bitwise reproducible).
//
// v_mfma_f64_16x16x4f64 operand layout (lane l of 64):
//   A (16 x 4):  A[l % 16][l / 16]
//   B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): register r of lane l holds D[4 r + l / 16][l % 16]
#include "gk_internal.h"

namespace gk {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int PT_ROWS = 32;      // rows per tile
constexpr int PT_THREADS = 256;  // 4 wavefronts
constexpr int PT_MAXGRID = 512;  // two workgroups per CU

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

struct PanelArgs {
  int64_t n;
  const double* X;       // n x ld input
  double* Xout;          // n x ld output (WRITE)
  float* X32;            // n x ld float copy (W32)
  const double* V0;      // local basis blocks (n x ld)
  const double* V1;
  const double* C;       // (nbv*ld) x ld update coefficients (UPDATE)
  const double* Rm;      // ld x ld upper triangular right factor (APPLY)
  double* part;          // [gridDim.x][ngb*ld][ld] Gram partials
  double* H;             // UPDATE: when non-null, H = sym of the last coefficient block (hs x hs)
  int hs;
  const int* flag;       // non-null: the pass does nothing when *flag == 0
};

// NT: ld / 16.  NBV: local blocks staged.  UPDATE: X_new = X - [V] C.
// APPLY: X_new = X Rm.  GRAMV: Gram [V]^T X_new.  SELF: Gram X_new^T X_new
// (symmetric: only tiles gi <= xj are formed and written to the partial; the
// reduction mirrors them).
template <int NT, int NBV, bool UPDATE, bool APPLY, bool GRAMV, bool SELF, bool WRITE, bool W32>
__global__ void __launch_bounds__(PT_THREADS, APPLY ? 3 : 2) panel_kernel(PanelArgs p) {
  constexpr int LD = NT * 16;
  // LDS row pitch (doubles): odd.  A 64-bit LDS access is served 16 lanes
  // at a time over 32 four-byte banks; the 16 rows that one matrix-core
  // operand read takes down a column then fall in 16 distinct bank pairs
  // (an even pitch pairs rows 8 apart on the same banks: measured 0.96
  // conflict cycles per busy cycle in the update pass against 0.06)
  constexpr int P = LD + 1;
  constexpr int KS = LD / 4;                     // MFMA k-steps over ld
  constexpr int NGB = (GRAMV ? NBV : 0) + (SELF ? 1 : 0);
  constexpr bool SYM = SELF && !GRAMV;
  constexpr int NPAIR = SYM ? NT * (NT + 1) / 2 : NGB * NT * NT;
  constexpr int TPW = (NPAIR + 3) / 4;           // Gram tiles per wavefront
  constexpr bool NEED_V = NBV > 0 && (UPDATE || GRAMV);
  constexpr int NBC = UPDATE ? NBV : (APPLY ? 1 : 0);   // coefficient blocks in registers
  // rows per tile: 16 for the two-block update at ld >= 48, whose
  // coefficients fill half the registers, so that the next tile's rows still
  // fit in registers while the current tile is processed
  constexpr bool HALF = UPDATE && NBV > 1 && NT > 2;
  constexpr int TR = HALF ? 16 : PT_ROWS;
  __shared__ double sX[TR * P];
  __shared__ double sV[(NEED_V ? NBV : 1) * TR * P];

  if (p.flag && *p.flag == 0) return;
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int l = tid & 63;
  const int li = l & 15;
  const int lk = l >> 4;
  if (UPDATE && p.H && blockIdx.x == 0) {
    // H_kk of the three-term recurrence: the coefficient block of the newest
    // basis block, symmetrised
    const double* Cl = p.C + (int64_t)(NBV - 1) * LD * LD;
    for (int q = tid; q < p.hs * p.hs; q += PT_THREADS) {
      const int i = q / p.hs, c = q - i * p.hs;
      p.H[q] = 0.5 * (Cl[i * LD + c] + Cl[c * LD + i]);
    }
  }

  // Update / apply product: wavefront w owns one 16-column tile (unt) of X_new
  // over UP slabs of 16 rows; its right operands stay in registers for the
  // whole kernel.
  constexpr int UP = NT >= 3 ? TR / 16 : 1;
  const int unt = NT >= 3 ? w : (w >> 1);
  const int us0 = NT >= 3 ? 0 : (w & 1);
  const bool uact = unt < NT;
  double creg[NBC > 0 ? NBC : 1][KS];
  if (NBC > 0) {
#pragma unroll
    for (int b = 0; b < (NBC > 0 ? NBC : 1); ++b)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        double v = 0.0;
        if (uact) {
          const double* src = UPDATE ? p.C : p.Rm;
          v = src[(int64_t)(b * LD + 4 * ks + lk) * LD + 16 * unt + li];
        }
        creg[b][ks] = v;
      }
  }
  // Gram tile list of this wavefront
  int tgi[TPW > 0 ? TPW : 1], txj[TPW > 0 ? TPW : 1];
#pragma unroll
  for (int t = 0; t < (TPW > 0 ? TPW : 1); ++t) {
    const int tt = w + 4 * t;
    int gi = -1, xj = -1;
    if (tt < NPAIR) {
      if (SYM) {
        int cnt = 0;
        for (int i = 0; i < NT; ++i)
          for (int j = i; j < NT; ++j) {
            if (cnt == tt) { gi = i; xj = j; }
            ++cnt;
          }
      } else {
        gi = tt / NT;
        xj = tt - gi * NT;
      }
    }
    tgi[t] = gi;
    txj[t] = xj;
  }
  d4 gacc[TPW > 0 ? TPW : 1];
#pragma unroll
  for (int t = 0; t < (TPW > 0 ? TPW : 1); ++t) gacc[t] = d4{0.0, 0.0, 0.0, 0.0};

  const int64_t ntiles = (p.n + TR - 1) / TR;
  // Tile rows go through registers: loads of the next tile are issued right
  // after the current one is in LDS, so they are in flight during its
  // products (rows past n read row n - 1 and are zeroed at the LDS store).
  constexpr int SQ = TR * LD / PT_THREADS;
  double lx[SQ], l0[NEED_V ? SQ : 1], l1[NEED_V && NBV > 1 ? SQ : 1];
  auto fetch_tile = [&](int64_t r0) {
#pragma unroll
    for (int e = 0; e < SQ; ++e) {
      const int q = e * PT_THREADS + tid;
      const int rr = q / LD, cc = q - rr * LD;
      const int64_t r = r0 + rr;
      const int64_t off = (r < p.n ? r : p.n - 1) * LD + cc;
      lx[e] = p.X[off];
      if (NEED_V) {
        l0[e] = p.V0[off];
        if (NBV > 1) l1[e] = p.V1[off];
      }
    }
  };
  if ((int64_t)blockIdx.x < ntiles) fetch_tile((int64_t)blockIdx.x * TR);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = tile * TR;
#pragma unroll
    for (int e = 0; e < SQ; ++e) {
      const int q = e * PT_THREADS + tid;
      const int rr = q / LD, cc = q - rr * LD;
      const bool in = r0 + rr < p.n;
      sX[rr * P + cc] = in ? lx[e] : 0.0;
      if (NEED_V) {
        sV[rr * P + cc] = in ? l0[e] : 0.0;
        if (NBV > 1) sV[TR * P + rr * P + cc] = in ? l1[e] : 0.0;
      }
    }
    __syncthreads();
    if (tile + gridDim.x < ntiles) fetch_tile((tile + gridDim.x) * TR);
    // ---- X_new for the (slabs, column tile) of this wavefront
    if (UPDATE || APPLY) {
      d4 acc[UP];
#pragma unroll
      for (int u = 0; u < UP; ++u) {
        const int rs = 16 * (us0 + u);
        acc[u] = d4{0.0, 0.0, 0.0, 0.0};
        if (UPDATE && uact) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[u][r] = sX[(rs + 4 * r + lk) * P + 16 * unt + li];
        }
      }
      if (uact) {
        if (UPDATE) {
#pragma unroll
          for (int b = 0; b < (NBV > 0 ? NBV : 1); ++b) {
            const double* sv = sV + b * TR * P;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
              for (int u = 0; u < UP; ++u) {
                const double a = -sv[(16 * (us0 + u) + li) * P + 4 * ks + lk];
                acc[u] = mfma64(a, creg[b][ks], acc[u]);
              }
            }
          }
        } else {
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            // Rm is upper triangular: rows 4ks.. of column tile unt vanish once 4ks >= 16(unt+1)
            if (4 * ks < 16 * (unt + 1)) {
#pragma unroll
              for (int u = 0; u < UP; ++u) {
                const double a = sX[(16 * (us0 + u) + li) * P + 4 * ks + lk];
                acc[u] = mfma64(a, creg[0][ks], acc[u]);
              }
            }
          }
        }
      }
      __syncthreads();   // every wavefront has read its sX rows
      if (uact) {
#pragma unroll
        for (int u = 0; u < UP; ++u) {
          const int rs = 16 * (us0 + u);
#pragma unroll
          for (int r = 0; r < 4; ++r) sX[(rs + 4 * r + lk) * P + 16 * unt + li] = acc[u][r];
        }
      }
      __syncthreads();
      if (WRITE || W32) {
#pragma unroll
        for (int q0 = 0; q0 < TR * LD; q0 += PT_THREADS) {
          const int q = q0 + tid;
          const int rr = q / LD, cc = q - rr * LD;
          const int64_t r = r0 + rr;
          if (r < p.n) {
            const double v = sX[rr * P + cc];
            if (WRITE) p.Xout[r * LD + cc] = v;
            if (W32) p.X32[r * LD + cc] = (float)v;
          }
        }
      }
    }
    // ---- Gram accumulation over the 32 rows of the tile
    if (NPAIR > 0) {
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        const int gi = tgi[t], xj = txj[t];
        if (gi >= 0) {
          const int gb = gi / NT, gc0 = 16 * (gi - gb * NT);
          const double* gsrc = (GRAMV && gb < NBV) ? (sV + gb * TR * P) : sX;
          d4 a4 = gacc[t];
#pragma unroll
          for (int k0 = 0; k0 < TR; k0 += 4) {
            // step k0 of a 16-row block takes rows t, t + 8, t + 4, t + 12
            // (t = k0 / 4 within the block): rows read together by half a
            // wavefront are 8 apart, 8 P = 16 mod 32 double banks
            const int row = (k0 & ~15) + ((k0 & 15) >> 2) + 8 * (lk & 1) + 4 * (lk >> 1);
            const double a = gsrc[row * P + gc0 + li];
            const double b = sX[row * P + 16 * xj + li];
            a4 = mfma64(a, b, a4);
          }
          gacc[t] = a4;
        }
      }
    }
    __syncthreads();
  }
  // ---- write the Gram partial of this workgroup
  if (NPAIR > 0) {
    double* P0 = p.part + (int64_t)blockIdx.x * NGB * LD * LD;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int gi = tgi[t], xj = txj[t];
      if (gi >= 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * gi + 4 * r + lk, col = 16 * xj + li;
          P0[(int64_t)row * LD + col] = gacc[t][r];
        }
      }
    }
  }
}

bool panel_ok(int ld) { return ld == 16 || ld == 32 || ld == 48 || ld == 64; }

int panel_grid(int64_t n) {
  const int64_t nt = (n + PT_ROWS - 1) / PT_ROWS;
  return (int)std::min<int64_t>(nt, PT_MAXGRID);
}

// Room for the largest set of Gram partials: two blocks over panel_grid(n)
// workgroups, or one block over up to 3/2 as many (the passes that run three
// workgroups per CU).
size_t panel_scratch_elems(int64_t n, int ld) { return (size_t)panel_grid(n) * 3 * ld * ld; }

typedef int PanelMode;

template <int NT>
static void panel_dispatch(PanelMode mode, int nbv, const PanelArgs& a, int grid, hipStream_t st) {
  dim3 g(grid), b(PT_THREADS);
#define GK_PK(NBV, U, AP, GV, SF, WR, W3) \
  hipLaunchKernelGGL((panel_kernel<NT, NBV, U, AP, GV, SF, WR, W3>), g, b, 0, st, a)
  switch (mode) {
    case PM_GRAMV:
      if (nbv == 1) GK_PK(1, false, false, true, false, false, false);
      else GK_PK(2, false, false, true, false, false, false);
      break;
    case PM_UPDATE_SELF:
      if (nbv == 1) GK_PK(1, true, false, false, true, true, false);
      else GK_PK(2, true, false, false, true, true, false);
      break;
    case PM_APPLY_SELF:
      GK_PK(0, false, true, false, true, false, false);
      break;
    case PM_APPLY_WRITE:
      if (a.X32) GK_PK(0, false, true, false, false, true, true);
      else GK_PK(0, false, true, false, false, true, false);
      break;
  }
#undef GK_PK
  GK_HIP(hipGetLastError());
}

// Launch one panel pass and (when it produces a Gram) reduce it into C.
void launch_panel(int mode, int64_t n, int ld, int nbv, const double* X, double* Xout, float* X32,
                  const double* V0, const double* V1, const double* Cupd, const double* Rm, double* part,
                  double* Cout, hipStream_t st, double* H, int hs, bool tri0, const int* flag) {
  PanelArgs a{n, X, Xout, X32, V0, V1, Cupd, Rm, part, H, hs, flag};
  const PanelMode pm = (PanelMode)mode;
  // the apply passes fit three workgroups per CU (their at most one Gram
  // block of partials stays within the scratch of panel_scratch_elems)
  const bool three = pm == PM_APPLY_WRITE || pm == PM_APPLY_SELF;
  const int grid = three ? (int)std::min<int64_t>((n + PT_ROWS - 1) / PT_ROWS, 3 * PT_MAXGRID / 2) : panel_grid(n);
  // algorithmic bytes / flops of the pass (block = n x ld float64)
  const double blk = 8.0 * (double)n * ld, nl2 = (double)n * ld * ld, self = (double)n * ld * (ld + 1);
  static const int kc[4] = {KC_PANEL_GRAMV, KC_PANEL_UPDATE_SELF, KC_PANEL_APPLY_SELF, KC_PANEL_APPLY_WRITE};
  double kb = 0, kf = 0;
  switch (pm) {
    case PM_GRAMV: kb = blk * (1 + nbv); kf = 2.0 * nl2 * nbv; break;
    // tri0: the first coefficient block is triangular (B_{k-1}^T of the recurrence)
    case PM_UPDATE_SELF: kb = blk * (2 + nbv); kf = 2.0 * nl2 * (nbv - (tri0 ? 1 : 0)) + (tri0 ? self : 0.0) + self; break;
    case PM_APPLY_SELF: kb = blk; kf = 2.0 * self; break;
    case PM_APPLY_WRITE: kb = blk * (X32 ? 2.5 : 2.0); kf = self; break;
  }
  kt_begin(kc[pm], st);
  switch (ld) {
    case 16: panel_dispatch<1>(pm, nbv, a, grid, st); break;
    case 32: panel_dispatch<2>(pm, nbv, a, grid, st); break;
    case 48: panel_dispatch<3>(pm, nbv, a, grid, st); break;
    case 64: panel_dispatch<4>(pm, nbv, a, grid, st); break;
    default: throw Error{GK_EUNSUPPORTED, "panel kernel needs ld in {16,32,48,64}"};
  }
  kt_end(st, kb, kf, flag);
  int ngb = 0;
  if (pm == PM_GRAMV) ngb = nbv;
  if (pm == PM_UPDATE_SELF || pm == PM_APPLY_SELF) ngb = 1;
  if (ngb > 0) {
    // the symmetric Gram's partials hold only its 16 x 16 tiles on and above the diagonal
    const bool sym = pm == PM_UPDATE_SELF || pm == PM_APPLY_SELF;
    launch_reduce_parts((int64_t)ngb * ld * ld, grid, part, Cout, flag, st, sym ? ld : 0, 16);
  }
}

}  // namespace gk
