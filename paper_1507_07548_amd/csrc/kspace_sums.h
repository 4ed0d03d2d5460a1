// The reciprocal-space sums of one slot (Sec. 4): sum_a d_a . F_a over the
// force kernel's per-(chunk, molecule-tile) partials, and the per-k energy
// and atomic-virial terms of the structure-factor reduction over k; each of
// the block's 256 threads a contiguous run, then a tree (a fixed order).
// U_recip, the molecular virial W_atomic - sum d.F and its dU/ds share are
// ADDED to the slot's sums.  Every thread of the 256-thread block calls it.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ms2 {

constexpr double kTwoPi = 6.283185307179586476925286766559;

__device__ __forceinline__ void kspace_sums_block(const SlotDev& sd, const SysParams& P, double* __restrict__ s_d,
                                                  double* __restrict__ s_u, double* __restrict__ s_w) {
  const int tid = threadIdx.x;
  const int nr = sd.kchunks * sd.mtiles;
  const int per = (nr + 255) / 256;
  double d = 0.0;
  {
    const int t1 = min(nr, (tid + 1) * per);
    int t = tid * per;
    for (; t + 4 <= t1; t += 4) {            // four loads before their additions, same order
      const double x0 = sd.kred[t], x1 = sd.kred[t + 1], x2 = sd.kred[t + 2], x3 = sd.kred[t + 3];
      d += x0;
      d += x1;
      d += x2;
      d += x3;
    }
    for (; t < t1; ++t) d += sd.kred[t];
  }
  const int perk = (sd.nk + 255) / 256;
  double u = 0.0, w = 0.0;
  for (int k = tid * perk; k < min(sd.nk, (tid + 1) * perk); ++k) {
    u += sd.sk_part[2 * k];
    w += sd.sk_part[2 * k + 1];
  }
  s_d[tid] = d;
  s_u[tid] = u;
  s_w[tid] = w;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      s_d[tid] += s_d[tid + h];
      s_u[tid] += s_u[tid + h];
      s_w[tid] += s_w[tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double pre = 2.0 * P.ke * kTwoPi / P.V;  // 2 pi k_e / V, doubled for the half space
    const double u_recip = pre * s_u[0], w_atomic = pre * s_w[0];
    sd.ksum[0] = u_recip;
    sd.ksum[1] = w_atomic;
    const double w_mol = w_atomic - s_d[0];  // molecular virial: W_atomic - sum d.F
    sd.sums[MS2_SUM_U_RECIP] += u_recip;
    sd.sums[MS2_SUM_VIRIAL] += w_mol;
    sd.sums[MS2_SUM_US] -= w_mol;
  }
}

// Sum over the force kernel's k-chunk partials of one (component c,
// molecule i) entry, in chunk order (four loads before their additions).
__device__ __forceinline__ double kspace_force_sum(const SlotDev& sd, int c, int i) {
  const int np = sd.npad;
  const double* fk = sd.fk + (size_t)c * np + i;
  const size_t stride = (size_t)6 * np;
  double v = 0.0;
  int kc = 0;
  for (; kc + 4 <= sd.kchunks; kc += 4) {
    const double a = fk[kc * stride], b = fk[(kc + 1) * stride];
    const double e = fk[(kc + 2) * stride], f = fk[(kc + 3) * stride];
    v += a;
    v += b;
    v += e;
    v += f;
  }
  for (; kc < sd.kchunks; ++kc) v += fk[kc * stride];
  return v;
}

}  // namespace ms2
