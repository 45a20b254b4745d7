// Reorthogonalisation decision after the orthogonality estimate of a Lanczos
// step (partial reorthogonalisation driven by the block omega recurrence).
#pragma once
#include "gk_internal.h"

namespace gk {

// Reorthogonalise when the estimate exceeds tau, and once more on the next
// step (the three-term coupling carries the lost orthogonality one block
// further).  After a reorthogonalisation the estimates restart from floor_re
// (the float32 archive limits the attainable orthogonality); the two local
// blocks are always at floor_loc.
//
// Evaluated by each of nwg workgroups of a grid (the same maximum of the
// per-slice estimates, so the same decision, in each); workgroup wg = 0
// records it and the resets of W_{k+1,j} are shared out.  red: LDS for
// blockDim.x / 64 doubles.  Contains barriers: the whole workgroup calls it.
__device__ __forceinline__ bool omega_decide(const OmegaDecide& d, int wg, int nwg, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t ss = (int64_t)d.s * d.s;
  double e = 0.0;
  for (int j = tid; j < d.ne; j += nt) e = fmax(e, d.est_part[j]);
  for (int o = 32; o > 0; o >>= 1) e = fmax(e, __shfl_xor(e, o));
  if ((tid & 63) == 0) red[tid >> 6] = e;
  __syncthreads();
  e = 0.0;
  for (int q = 0; q < nt / 64; ++q) e = fmax(e, red[q]);
  __syncthreads();   // red is free again for the caller
  const int f = d.forced[d.k];
  const bool go = e > d.tau || f;
  if (wg == 0 && tid == 0) {
    d.fr[d.k] = go ? 1 : 0;
    d.forced[d.k + 1] = (go && !f) ? 1 : 0;
    if (go) *d.nre += 1;
    // a projected X needs the second CholQR pass
    if (go && d.gate) *d.gate = 1;
    *d.est_out = fmax(*d.est_out, go ? d.floor_re : e);
  }
  const int64_t q0 = (int64_t)wg * nt + tid, qs = (int64_t)nwg * nt;
  if (go)
    for (int64_t q = q0; q < d.nj * ss; q += qs) d.Wk1[q] = d.floor_re;
  for (int64_t q = q0; q < 2 * ss; q += qs) {
    const int64_t jj = d.k - 1 + q / ss;
    if (jj >= 0) d.Wk1[jj * ss + q % ss] = d.floor_loc;
  }
  return go;
}

}  // namespace gk
