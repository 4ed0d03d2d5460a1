// Lab-frame site records of one molecule: d = A(q) b and e = A(q) ehat for
// every site (Real), the FP64 LJ-site offsets of the site-site cut-off, and
// the heat flux's lab velocities.  Shared by the site-frame kernel of the
// force path and the step kernel that runs the predictor and the site frame
// in one launch.
// Record layout per class: [lj 3*NLJ][ch 3*NCH][dp 6*NDP][qd 6*NQD], each
// real stored as a row of length npad (structure of arrays).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"
#include "quat.h"

namespace ms2 {

// One component of A b, rounded exactly as written (no fused multiply-add):
// equal bit for bit to a plain FP64 evaluation of the same sum.
__device__ __forceinline__ double rotate_row(const double* a, const double* b) {
#pragma clang fp contract(off)
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <typename Real, int C>
__device__ __forceinline__ void site_frame_molecule(const SlotDev& sd, const SpeciesTable* __restrict__ tab,
                                                    int i) {
  constexpr ClassShape S = kClassShapes[C];
  const int ld = sd.com_ld, np = sd.npad;
  Real* out = reinterpret_cast<Real*>(sd.sites);
  const SpeciesDev& D = tab->sp[clamp_species(sd.species[i], tab->nsp)];
  double A[3][3];
  quat_matrix(sd.quat[i], sd.quat[ld + i], sd.quat[2 * ld + i], sd.quat[3 * ld + i], A);
  int k = 0;
  auto put = [&](const double* b, int valid) {
    for (int c = 0; c < 3; ++c) {
      double v = valid ? rotate_row(A[c], b) : 0.0;
      out[(k + c) * np + i] = (Real)v;
    }
    k += 3;
  };
#pragma unroll
  for (int a = 0; a < S.lj; ++a) put(D.lj_pos[a < D.nlj ? a : 0], a < D.nlj);
  if (sd.lj64) {
    // site-site cut-off: the LJ-site offsets in FP64 as well, for the
    // decision r_ab^2 < rc^2 (taken in FP64 whatever the pair precision)
#pragma unroll
    for (int a = 0; a < S.lj; ++a)
      for (int c = 0; c < 3; ++c)
        sd.lj64[(3 * a + c) * np + i] = a < D.nlj ? rotate_row(A[c], D.lj_pos[a]) : 0.0;
  }
#pragma unroll
  for (int a = 0; a < S.ch; ++a) put(D.ch_pos[a < D.nch ? a : 0], a < D.nch);
#pragma unroll
  for (int a = 0; a < S.dp; ++a) {
    put(D.dp_pos[a < D.ndp ? a : 0], a < D.ndp);
    put(D.dp_axis[a < D.ndp ? a : 0], a < D.ndp);
  }
#pragma unroll
  for (int a = 0; a < S.qd; ++a) {
    put(D.qd_pos[a < D.nqd ? a : 0], a < D.nqd);
    put(D.qd_axis[a < D.nqd ? a : 0], a < D.nqd);
  }
  if (sd.hf_kin) {
    // lab-frame velocity and angular velocity of the state the forces are
    // evaluated at (heat flux)
    Real* kin = reinterpret_cast<Real*>(sd.hf_kin);
    double wb[3] = {0.0, 0.0, 0.0};
    if (sd.hf_w)
      for (int c = 0; c < 3; ++c) wb[c] = sd.hf_w[c * ld + i];
    for (int c = 0; c < 3; ++c) {
      kin[c * np + i] = (Real)(sd.hf_v[c * ld + i] * sd.hf_vscale);
      kin[(3 + c) * np + i] = (Real)(A[c][0] * wb[0] + A[c][1] * wb[1] + A[c][2] * wb[2]);
    }
  }
}

}  // namespace ms2
