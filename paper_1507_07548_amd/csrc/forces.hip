// Force/energy/virial hot path on gfx950: lab-frame site records, the
// molecule-pair kernel and its fixed-order reductions.
//
// Mapping (one block = 64*W lanes, W waves):
//   * every lane owns one molecule i of an i-tile of 64*W molecules and
//     accumulates everything acting on i in registers (row-owned: each pair
//     is evaluated from both sides, so no lane ever writes another lane's
//     molecule and no atomics are needed; the paper's Sec. 2 avoids the same
//     write race with per-interaction lists summed afterwards);
//   * j molecules stream through LDS in tiles of 64*W records (coalesced
//     structure-of-arrays loads);
//   * per tile, phase 1 tests every (i, j) pair against the molecule-centre
//     cut-off in FP64 and keeps one bit per accepted pair; phase 2 walks each
//     lane's own set bits, so the ~54 % of rejected pairs cost one FP64 test
//     and no site arithmetic (per-lane compaction instead of masked lanes);
//   * site-pair arithmetic runs in Real (float or double); force partials of
//     one j tile are folded into FP64 per-molecule accumulators; energies and
//     volume-derivative sums are accumulated per molecule pair in FP64.
// A work item is (system, i-tile, j-range); its per-molecule partials go to
// a slot-private buffer and are summed over j-ranges in a fixed order by
// reduce_pair_kernel, so results do not depend on launch order or on other
// systems sharing the launch.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ms2 {

// FP32 reciprocal and reciprocal square root: the hardware approximations
// (1 ulp) followed by one Newton step.  Without the step their rounding is
// biased in one direction, and r^-6, r^-12 turn that bias into a coherent
// relative error of the summed energy.
template <typename Real> __device__ __forceinline__ Real rcp_(Real x);
template <> __device__ __forceinline__ float rcp_<float>(float x) {
  const float y = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(y, __builtin_fmaf(-x, y, 1.0f), y);
}
template <> __device__ __forceinline__ double rcp_<double>(double x) { return 1.0 / x; }
template <typename Real> __device__ __forceinline__ Real rsq_(Real x);
template <> __device__ __forceinline__ float rsq_<float>(float x) {
  const float y = __builtin_amdgcn_rsqf(x);
  const float h = 0.5f * x * y;
  return __builtin_fmaf(y, __builtin_fmaf(-h, y, 0.5f), y);
}
template <> __device__ __forceinline__ double rsq_<double>(double x) { return 1.0 / sqrt(x); }
template <typename Real> __device__ __forceinline__ Real erfc_(Real x);
template <> __device__ __forceinline__ float erfc_<float>(float x) { return erfcf(x); }
template <> __device__ __forceinline__ double erfc_<double>(double x) { return erfc(x); }
template <typename Real> __device__ __forceinline__ Real exp_(Real x);
template <> __device__ __forceinline__ float exp_<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double exp_<double>(double x) { return exp(x); }

// Minimum-image centre difference, rounded exactly as written (no
// contraction) so that the accept decision is reproducible bit for bit.
__device__ __forceinline__ void min_image(double xi, double yi, double zi, double xj, double yj,
                                          double zj, double L, double invL, double& dx,
                                          double& dy, double& dz, double& r2) {
#pragma clang fp contract(off)
  dx = xi - xj;
  dy = yi - yj;
  dz = zi - zj;
  dx = dx - L * rint(dx * invL);
  dy = dy - L * rint(dy * invL);
  dz = dz - L * rint(dz * invL);
  r2 = dx * dx + dy * dy + dz * dz;
}

// ---------------------------------------------------------------------------
// Site frame: d = A(q) b and e = A(q) ehat for every site of every molecule.
// Record layout per class: [lj 3*NLJ][ch 3*NCH][dp 6*NDP][qd 6*NQD], each
// real stored as a row of length npad (structure of arrays).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rot_matrix(double w, double x, double y, double z, double A[3][3]) {
  A[0][0] = 1.0 - 2.0 * (y * y + z * z);
  A[0][1] = 2.0 * (x * y - w * z);
  A[0][2] = 2.0 * (x * z + w * y);
  A[1][0] = 2.0 * (x * y + w * z);
  A[1][1] = 1.0 - 2.0 * (x * x + z * z);
  A[1][2] = 2.0 * (y * z - w * x);
  A[2][0] = 2.0 * (x * z - w * y);
  A[2][1] = 2.0 * (y * z + w * x);
  A[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

template <typename Real, int C>
__global__ __launch_bounds__(256) void site_frame_kernel(const SlotDev* __restrict__ slots,
                                                         const SysParams* __restrict__ prm,
                                                         const SpeciesTable* __restrict__ tab) {
  constexpr ClassShape S = kClassShapes[C];
  const SlotDev& sd = slots[blockIdx.y];
  if (!sd.active) return;
  if (prm[blockIdx.y].precision != (sizeof(Real) == 4 ? MS2_FP32 : MS2_FP64)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= sd.n) return;
  const int ld = sd.com_ld, np = sd.npad;
  Real* out = reinterpret_cast<Real*>(sd.sites);
  const SpeciesDev& D = tab->sp[clamp_species(sd.species[i], tab->nsp)];
  double A[3][3];
  rot_matrix(sd.quat[i], sd.quat[ld + i], sd.quat[2 * ld + i], sd.quat[3 * ld + i], A);
  int k = 0;
  auto put = [&](const double* b, int valid) {
    for (int c = 0; c < 3; ++c) {
      double v = valid ? A[c][0] * b[0] + A[c][1] * b[1] + A[c][2] * b[2] : 0.0;
      out[(k + c) * np + i] = (Real)v;
    }
    k += 3;
  };
#pragma unroll
  for (int a = 0; a < S.lj; ++a) put(D.lj_pos[a < D.nlj ? a : 0], a < D.nlj);
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
}

// ---------------------------------------------------------------------------
// Orientation-dependent Coulomb terms of point multipoles.
// u = K * P(ca, cb, cab) * r^-p with ca = ea.n, cb = eb.n, cab = ea.eb and n
// the unit vector from site b (on j) to site a (on i).  P and its partial
// derivatives (d/dca, d/dcb, d/dcab, d2/dca2, d2/dcb2, d2/dca dcb).
// Types: 1 charge, 2 dipole, 3 quadrupole.
// ---------------------------------------------------------------------------
template <typename Real>
struct Poly {
  Real P, Pa, Pb, Pc, Paa, Pbb, Pab;
};

template <int TA, int TB> struct MpPower;
template <> struct MpPower<1, 2> { static constexpr int p = 2; };
template <> struct MpPower<2, 1> { static constexpr int p = 2; };
template <> struct MpPower<1, 3> { static constexpr int p = 3; };
template <> struct MpPower<3, 1> { static constexpr int p = 3; };
template <> struct MpPower<2, 2> { static constexpr int p = 3; };
template <> struct MpPower<2, 3> { static constexpr int p = 4; };
template <> struct MpPower<3, 2> { static constexpr int p = 4; };
template <> struct MpPower<3, 3> { static constexpr int p = 5; };

template <typename Real, int TA, int TB>
__device__ __forceinline__ Poly<Real> mp_poly(Real ca, Real cb, Real cab) {
  Poly<Real> q{0, 0, 0, 0, 0, 0, 0};
  if constexpr (TA == 1 && TB == 2) {          // charge . dipole field
    q.P = cb; q.Pb = 1;
  } else if constexpr (TA == 2 && TB == 1) {
    q.P = -ca; q.Pa = -1;
  } else if constexpr (TA == 1 && TB == 3) {   // charge in a quadrupole field: P2(cb)
    q.P = Real(1.5) * cb * cb - Real(0.5); q.Pb = Real(3) * cb; q.Pbb = Real(3);
  } else if constexpr (TA == 3 && TB == 1) {
    q.P = Real(1.5) * ca * ca - Real(0.5); q.Pa = Real(3) * ca; q.Paa = Real(3);
  } else if constexpr (TA == 2 && TB == 2) {
    q.P = cab - Real(3) * ca * cb; q.Pa = Real(-3) * cb; q.Pb = Real(-3) * ca;
    q.Pc = 1; q.Pab = -3;
  } else if constexpr (TA == 2 && TB == 3) {   // dipole a in the field gradient of quadrupole b
    const Real cb2 = cb * cb;
    q.P = Real(1.5) * ca - Real(7.5) * ca * cb2 + Real(3) * cb * cab;
    q.Pa = Real(1.5) - Real(7.5) * cb2;
    q.Pb = Real(3) * cab - Real(15) * ca * cb;
    q.Pc = Real(3) * cb;
    q.Pbb = Real(-15) * ca;
    q.Pab = Real(-15) * cb;
  } else if constexpr (TA == 3 && TB == 2) {
    const Real ca2 = ca * ca;
    q.P = Real(-1.5) * cb + Real(7.5) * ca2 * cb - Real(3) * ca * cab;
    q.Pb = Real(-1.5) + Real(7.5) * ca2;
    q.Pa = Real(15) * ca * cb - Real(3) * cab;
    q.Pc = Real(-3) * ca;
    q.Paa = Real(15) * cb;
    q.Pab = Real(15) * ca;
  } else {                                      // quadrupole-quadrupole
    const Real ca2 = ca * ca, cb2 = cb * cb, cc = ca * cb;
    q.P = Real(0.75) + Real(-3.75) * (ca2 + cb2) + Real(26.25) * ca2 * cb2 + Real(1.5) * cab * cab -
          Real(15) * cc * cab;
    q.Pa = Real(-7.5) * ca + Real(52.5) * ca * cb2 - Real(15) * cb * cab;
    q.Pb = Real(-7.5) * cb + Real(52.5) * ca2 * cb - Real(15) * ca * cab;
    q.Pc = Real(3) * cab - Real(15) * cc;
    q.Paa = Real(-7.5) + Real(52.5) * cb2;
    q.Pbb = Real(-7.5) + Real(52.5) * ca2;
    q.Pab = Real(105) * cc - Real(15) * cab;
  }
  return q;
}

template <typename Real, int P>
__device__ __forceinline__ Real ipow(Real x) {
  Real r = x;
#pragma unroll
  for (int k = 1; k < P; ++k) r *= x;
  return r;
}

// Per molecule-pair accumulators (Real) of the current (i, j) pair.
template <typename Real>
struct PairAcc {
  Real ulj, uel, uss;
  Real fx, fy, fz;
};

// One multipole site pair.  pa/ea: site a of i (offset, axis); pb/eb: site b
// of j.  Adds the force on a to fs, -du/dea to gs (when a is oriented).
// CENTRAL: both sites at their molecules' centres, so r = R and the
// volume-derivative terms follow from homogeneity (u ~ r^-p).
template <typename Real, int TA, int TB, bool CENTRAL_CLASS>
__device__ __forceinline__ void mp_site_pair(Real K, const Real* pa, const Real* ea, const Real* pb,
                                             const Real* eb, Real Rx, Real Ry, Real Rz, Real R2,
                                             PairAcc<Real>& acc, Real* fs, Real* gs, bool rf_dd,
                                             Real krf) {
  constexpr int p = MpPower<TA, TB>::p;
  // the class guarantees centred dipoles/quadrupoles, not centred charges
  constexpr bool CENTRAL = CENTRAL_CLASS && TA != 1 && TB != 1;
  Real rx = Rx, ry = Ry, rz = Rz, r2 = R2;
  if constexpr (!CENTRAL) {
    rx += pa[0] - pb[0];
    ry += pa[1] - pb[1];
    rz += pa[2] - pb[2];
    r2 = rx * rx + ry * ry + rz * rz;
  }
  const Real ir = rsq_(r2), ir2 = ir * ir;
  const Real nx = rx * ir, ny = ry * ir, nz = rz * ir;
  Real ca = 0, cb = 0, cab = 0;
  if constexpr (TA != 1) ca = ea[0] * nx + ea[1] * ny + ea[2] * nz;
  if constexpr (TB != 1) cb = eb[0] * nx + eb[1] * ny + eb[2] * nz;
  if constexpr (TA != 1 && TB != 1) cab = ea[0] * eb[0] + ea[1] * eb[1] + ea[2] * eb[2];
  const Poly<Real> q = mp_poly<Real, TA, TB>(ca, cb, cab);
  const Real Kp = K * ipow<Real, p>(ir);
  const Real u = Kp * q.P;
  acc.uel += u;
  // force on a = -grad_r u = (K r^-p / r) [(p P + Pa ca + Pb cb) n - Pa ea - Pb eb]
  const Real A = Kp * ir;
  Real sdot = Real(p) * q.P;
  if constexpr (TA != 1) sdot += q.Pa * ca;
  if constexpr (TB != 1) sdot += q.Pb * cb;
  Real fx = sdot * nx, fy = sdot * ny, fz = sdot * nz;
  if constexpr (TA != 1) { fx -= q.Pa * ea[0]; fy -= q.Pa * ea[1]; fz -= q.Pa * ea[2]; }
  if constexpr (TB != 1) { fx -= q.Pb * eb[0]; fy -= q.Pb * eb[1]; fz -= q.Pb * eb[2]; }
  fx *= A; fy *= A; fz *= A;
  fs[0] += fx; fs[1] += fy; fs[2] += fz;
  acc.fx += fx; acc.fy += fy; acc.fz += fz;
  if constexpr (TA != 1) {
    Real gx = q.Pa * nx, gy = q.Pa * ny, gz = q.Pa * nz;
    if constexpr (TB != 1) { gx += q.Pc * eb[0]; gy += q.Pc * eb[1]; gz += q.Pc * eb[2]; }
    gs[0] -= Kp * gx; gs[1] -= Kp * gy; gs[2] -= Kp * gz;
  }
  if constexpr (CENTRAL) {
    acc.uss += Real(p * (p + 1)) * u;
  } else {
    // second derivative of u(r + t R) at t = 0
    const Real beta = nx * Rx + ny * Ry + nz * Rz;
    const Real w = R2 - beta * beta;
    Real F1 = 0, F2 = 0;
    Real ca1 = 0, cb1 = 0;
    if constexpr (TA != 1) {
      ca1 = ((ea[0] * Rx + ea[1] * Ry + ea[2] * Rz) - ca * beta) * ir;
      const Real ca2 = -(Real(2) * ca1 * beta + ca * w * ir) * ir;
      F1 += q.Pa * ca1;
      F2 += q.Paa * ca1 * ca1 + q.Pa * ca2;
    }
    if constexpr (TB != 1) {
      cb1 = ((eb[0] * Rx + eb[1] * Ry + eb[2] * Rz) - cb * beta) * ir;
      const Real cb2 = -(Real(2) * cb1 * beta + cb * w * ir) * ir;
      F1 += q.Pb * cb1;
      F2 += q.Pbb * cb1 * cb1 + q.Pb * cb2;
    }
    if constexpr (TA != 1 && TB != 1) F2 += Real(2) * q.Pab * ca1 * cb1;
    const Real f1 = -Real(p) * ir * beta;
    const Real f2 = ir2 * (Real(p * (p + 1)) * beta * beta - Real(p) * w);
    acc.uss += Kp * (F2 + Real(2) * F1 * f1 + q.P * f2);
  }
  if constexpr (TA == 2 && TB == 2) {
    if (rf_dd) {  // Barker-Watts reaction field: -2 kRF K (ea.eb); no force, no volume terms
      acc.uel -= Real(2) * krf * K * cab;
      gs[0] += Real(2) * krf * K * eb[0];
      gs[1] += Real(2) * krf * K * eb[1];
      gs[2] += Real(2) * krf * K * eb[2];
    }
  }
}

// ---------------------------------------------------------------------------
// The pair kernel.
// ---------------------------------------------------------------------------
template <typename Real, int C, int W>
__global__ __launch_bounds__(64 * W) void pair_kernel(const WorkItem* __restrict__ items,
                                                      int item_base,
                                                      const SlotDev* __restrict__ slots,
                                                      const SysParams* __restrict__ prm,
                                                      const SpeciesTable* __restrict__ tab) {
  constexpr ClassShape S = kClassShapes[C];
  constexpr int NR = class_reals(C);
  constexpr int TJ = 64 * W;
  constexpr int NLJ = S.lj > 0 ? S.lj : 1;
  constexpr int NCH = S.ch > 0 ? S.ch : 1;
  constexpr int NDP = S.dp > 0 ? S.dp : 1;
  constexpr int NQD = S.qd > 0 ? S.qd : 1;
  constexpr int OFF_CH = 3 * S.lj, OFF_DP = OFF_CH + 3 * S.ch, OFF_QD = OFF_DP + 6 * S.dp;
  constexpr bool CENTRAL = S.central != 0;

  __shared__ double s_com[3][TJ];
  __shared__ int s_sp[TJ];
  __shared__ Real s_site[NR][TJ];
  __shared__ Real s_c6[kMaxSp * NLJ][kMaxSp * NLJ];
  __shared__ Real s_c12[kMaxSp * NLJ][kMaxSp * NLJ];
  __shared__ int s_cnt[kMaxSp][4];
  __shared__ Real s_mch[kMaxSp][NCH], s_mdp[kMaxSp][NDP], s_mqd[kMaxSp][NQD];
  __shared__ int s_nsite[kMaxSp][kMaxSp];
  __shared__ double s_red[kNumBlockSums][TJ];

  const int gitem = item_base + blockIdx.x;
  const WorkItem it = items[gitem];
  const SlotDev& sd = slots[it.slot];
  if (!sd.active) return;
  const SysParams& P = prm[it.slot];
  const int tid = threadIdx.x;
  const int nsp = P.nsp;

  // tables of this system's species
  for (int e = tid; e < nsp * NLJ * nsp * NLJ; e += TJ) {
    const int A = e / (NLJ * nsp * NLJ), r = e % (NLJ * nsp * NLJ);
    const int a = r / (nsp * NLJ), r2 = r % (nsp * NLJ);
    const int B = r2 / NLJ, b = r2 % NLJ;
    s_c6[A * NLJ + a][B * NLJ + b] = (Real)tab->c6[A][a][B][b];
    s_c12[A * NLJ + a][B * NLJ + b] = (Real)tab->c12[A][a][B][b];
  }
  for (int e = tid; e < nsp; e += TJ) {
    const SpeciesDev& D = tab->sp[e];
    s_cnt[e][0] = D.nlj; s_cnt[e][1] = D.nch; s_cnt[e][2] = D.ndp; s_cnt[e][3] = D.nqd;
    for (int a = 0; a < NCH; ++a) s_mch[e][a] = (Real)(P.ke * D.ch_q[a]);
    for (int a = 0; a < NDP; ++a) s_mdp[e][a] = (Real)(P.ke * D.dp_mu[a]);
    for (int a = 0; a < NQD; ++a) s_mqd[e][a] = (Real)(P.ke * D.qd_Q[a]);
    for (int b = 0; b < nsp; ++b) s_nsite[e][b] = tab->nsite_pair[e][b];
  }

  const int n = sd.n, ld = sd.com_ld, np = sd.npad;
  const double L = P.L, invL = P.invL, rc2 = P.rc2;
  const int elec = P.elec;
  const Real krf = (Real)P.krf, crf = (Real)P.crf;
  const Real alpha = (Real)P.alpha, alpha2 = (Real)P.alpha2, gpref = (Real)P.gpref;
  const Real* __restrict__ gsite = reinterpret_cast<const Real*>(sd.sites);

  const int i = it.i0 + tid;
  const bool iv = i < n;
  const int ic = iv ? i : 0;
  const double xi = sd.com[ic], yi = sd.com[ld + ic], zi = sd.com[2 * ld + ic];
  const int spi = iv ? clamp_species(sd.species[ic], nsp) : 0;
  Real rec[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rec[k] = gsite[k * np + ic];

  // accumulators
  double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  double a_ulj = 0, a_uel = 0, a_us = 0, a_uss = 0;
  int a_np = 0, a_ns = 0;
  Real fl[NLJ][3], fc[NCH][3], fd[NDP][3], gd[NDP][3], fq[NQD][3], gq[NQD][3];
  auto zero_site_acc = [&]() {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int a = 0; a < NLJ; ++a) fl[a][c] = 0;
#pragma unroll
      for (int a = 0; a < NCH; ++a) fc[a][c] = 0;
#pragma unroll
      for (int a = 0; a < NDP; ++a) { fd[a][c] = 0; gd[a][c] = 0; }
#pragma unroll
      for (int a = 0; a < NQD; ++a) { fq[a][c] = 0; gq[a][c] = 0; }
    }
  };
  zero_site_acc();
  __syncthreads();
  const int nlj_i = s_cnt[spi][0], nch_i = s_cnt[spi][1], ndp_i = s_cnt[spi][2], nqd_i = s_cnt[spi][3];

  for (int jt = it.j0; jt < it.j1; jt += TJ) {
    __syncthreads();
    {
      const int j = jt + tid;
      const bool jv = j < it.j1 && j < n;
      const int jc = jv ? j : 0;
      s_com[0][tid] = sd.com[jc];
      s_com[1][tid] = sd.com[ld + jc];
      s_com[2][tid] = sd.com[2 * ld + jc];
      s_sp[tid] = jv ? clamp_species(sd.species[jc], nsp) : -1;
#pragma unroll
      for (int k = 0; k < NR; ++k) s_site[k][tid] = gsite[k * np + jc];
    }
    __syncthreads();

    // phase 1: cut-off bits, one 64-bit word per 64 j molecules
    const int nvalid = min(TJ, min(it.j1, n) - jt);   // uniform over the block
    const int iself = i - jt;                          // lane's own molecule in this tile, if any
    unsigned long long mask[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      unsigned long long m = 0;
      for (int b = 0; b < 64; ++b) {
        const int jj = w * 64 + b;
        double dx, dy, dz, r2;
        min_image(xi, yi, zi, s_com[0][jj], s_com[1][jj], s_com[2][jj], L, invL, dx, dy, dz, r2);
        const unsigned ok = (unsigned)(r2 < rc2) & (unsigned)(jj < nvalid) & (unsigned)(jj != iself);
        m |= (unsigned long long)ok << b;
      }
      mask[w] = iv ? m : 0ull;
    }

    // phase 2: accepted pairs of this lane
    int w = 0;
    unsigned long long m = mask[0];
    while (true) {
      while (m == 0ull && w < W - 1) {
        ++w;
#pragma unroll
        for (int x = 1; x < W; ++x)
          if (x == w) m = mask[x];
      }
      if (m == 0ull) break;
      const int jj = w * 64 + __builtin_ctzll(m);
      m &= m - 1ull;

      const int spj = s_sp[jj];
      double dx, dy, dz, r2d;
      min_image(xi, yi, zi, s_com[0][jj], s_com[1][jj], s_com[2][jj], L, invL, dx, dy, dz, r2d);
      const Real Rx = (Real)dx, Ry = (Real)dy, Rz = (Real)dz;
      const Real R2 = Rx * Rx + Ry * Ry + Rz * Rz;
      PairAcc<Real> acc{0, 0, 0, 0, 0, 0};
      const int nlj_j = s_cnt[spj][0], nch_j = s_cnt[spj][1], ndp_j = s_cnt[spj][2], nqd_j = s_cnt[spj][3];

      // Lennard-Jones site pairs
#pragma unroll
      for (int a = 0; a < S.lj; ++a) {
        if (a >= nlj_i) break;
#pragma unroll
        for (int b = 0; b < S.lj; ++b) {
          if (b >= nlj_j) break;
          const Real rx = Rx + rec[3 * a] - s_site[3 * b][jj];
          const Real ry = Ry + rec[3 * a + 1] - s_site[3 * b + 1][jj];
          const Real rz = Rz + rec[3 * a + 2] - s_site[3 * b + 2][jj];
          const Real r2 = rx * rx + ry * ry + rz * rz;
          const Real ir2 = rcp_(r2);
          const Real ir6 = ir2 * ir2 * ir2;
          const Real t6 = s_c6[spi * NLJ + a][spj * NLJ + b] * ir6;
          const Real t12 = s_c12[spi * NLJ + a][spj * NLJ + b] * ir6 * ir6;
          const Real dur = (Real(6) * t6 - Real(12) * t12) * ir2;       // u'/r
          const Real d2u = (Real(156) * t12 - Real(42) * t6) * ir2;     // u''
          const Real rR = rx * Rx + ry * Ry + rz * Rz;
          acc.ulj += t12 - t6;
          acc.uss += (d2u - dur) * (rR * rR * ir2) + dur * R2;
          const Real fx = -dur * rx, fy = -dur * ry, fz = -dur * rz;
          fl[a][0] += fx; fl[a][1] += fy; fl[a][2] += fz;
          acc.fx += fx; acc.fy += fy; acc.fz += fz;
        }
      }
      // charge-charge site pairs
      if constexpr (S.ch > 0) {
#pragma unroll
        for (int a = 0; a < S.ch; ++a) {
          if (a >= nch_i) break;
#pragma unroll
          for (int b = 0; b < S.ch; ++b) {
            if (b >= nch_j) break;
            const Real K = s_mch[spi][a] * s_mch[spj][b] * (Real)(1.0 / P.ke);
            const Real rx = Rx + rec[OFF_CH + 3 * a] - s_site[OFF_CH + 3 * b][jj];
            const Real ry = Ry + rec[OFF_CH + 3 * a + 1] - s_site[OFF_CH + 3 * b + 1][jj];
            const Real rz = Rz + rec[OFF_CH + 3 * a + 2] - s_site[OFF_CH + 3 * b + 2][jj];
            const Real r2 = rx * rx + ry * ry + rz * rz;
            const Real ir = rsq_(r2), ir2 = ir * ir;
            Real u, dur, d2u;
            if (elec == MS2_ELEC_EWALD) {
              const Real r = r2 * ir;
              const Real e = erfc_(alpha * r);
              const Real gs = gpref * exp_(-alpha2 * r2);
              u = K * e * ir;
              dur = -K * (e * ir + gs) * ir2;
              d2u = K * (Real(2) * e * ir * ir2 + gs * (Real(2) * ir2 + Real(2) * alpha2));
            } else if (elec == MS2_ELEC_RF) {
              u = K * (ir + krf * r2 - crf);
              dur = K * (Real(2) * krf - ir * ir2);
              d2u = K * (Real(2) * ir * ir2 + Real(2) * krf);
            } else {
              u = K * ir;
              dur = -K * ir * ir2;
              d2u = Real(2) * K * ir * ir2;
            }
            const Real rR = rx * Rx + ry * Ry + rz * Rz;
            acc.uel += u;
            acc.uss += (d2u - dur) * (rR * rR * ir2) + dur * R2;
            const Real fx = -dur * rx, fy = -dur * ry, fz = -dur * rz;
            fc[a][0] += fx; fc[a][1] += fy; fc[a][2] += fz;
            acc.fx += fx; acc.fy += fy; acc.fz += fz;
          }
        }
      }
      // point multipoles (charges x dipoles x quadrupoles, not charge-charge)
      if constexpr (S.dp > 0 || S.qd > 0) {
        const bool rf_dd = elec == MS2_ELEC_RF;
        const Real kk = (Real)(1.0 / P.ke);
        const Real zero3[3] = {0, 0, 0};
        // a = charge on i
        if constexpr (S.ch > 0) {
#pragma unroll
          for (int a = 0; a < S.ch; ++a) {
            if (a >= nch_i) break;
            const Real* pa = &rec[OFF_CH + 3 * a];
            if constexpr (S.dp > 0) {
#pragma unroll
              for (int b = 0; b < S.dp; ++b) {
                if (b >= ndp_j) break;
                const Real pb[3] = {s_site[OFF_DP + 6 * b][jj], s_site[OFF_DP + 6 * b + 1][jj], s_site[OFF_DP + 6 * b + 2][jj]};
                const Real eb[3] = {s_site[OFF_DP + 6 * b + 3][jj], s_site[OFF_DP + 6 * b + 4][jj], s_site[OFF_DP + 6 * b + 5][jj]};
                Real gdummy[3] = {0, 0, 0};
                mp_site_pair<Real, 1, 2, CENTRAL>(s_mch[spi][a] * s_mdp[spj][b] * kk, pa, zero3, pb, eb, Rx, Ry, Rz, R2, acc, fc[a], gdummy, false, krf);
              }
            }
            if constexpr (S.qd > 0) {
#pragma unroll
              for (int b = 0; b < S.qd; ++b) {
                if (b >= nqd_j) break;
                const Real pb[3] = {s_site[OFF_QD + 6 * b][jj], s_site[OFF_QD + 6 * b + 1][jj], s_site[OFF_QD + 6 * b + 2][jj]};
                const Real eb[3] = {s_site[OFF_QD + 6 * b + 3][jj], s_site[OFF_QD + 6 * b + 4][jj], s_site[OFF_QD + 6 * b + 5][jj]};
                Real gdummy[3] = {0, 0, 0};
                mp_site_pair<Real, 1, 3, CENTRAL>(s_mch[spi][a] * s_mqd[spj][b] * kk, pa, zero3, pb, eb, Rx, Ry, Rz, R2, acc, fc[a], gdummy, false, krf);
              }
            }
          }
        }
        // a = dipole on i
        if constexpr (S.dp > 0) {
#pragma unroll
          for (int a = 0; a < S.dp; ++a) {
            if (a >= ndp_i) break;
            const Real* pa = &rec[OFF_DP + 6 * a];
            const Real* ea = &rec[OFF_DP + 6 * a + 3];
            if constexpr (S.ch > 0) {
#pragma unroll
              for (int b = 0; b < S.ch; ++b) {
                if (b >= nch_j) break;
                const Real pb[3] = {s_site[OFF_CH + 3 * b][jj], s_site[OFF_CH + 3 * b + 1][jj], s_site[OFF_CH + 3 * b + 2][jj]};
                mp_site_pair<Real, 2, 1, CENTRAL>(s_mdp[spi][a] * s_mch[spj][b] * kk, pa, ea, pb, zero3, Rx, Ry, Rz, R2, acc, fd[a], gd[a], false, krf);
              }
            }
#pragma unroll
            for (int b = 0; b < S.dp; ++b) {
              if (b >= ndp_j) break;
              const Real pb[3] = {s_site[OFF_DP + 6 * b][jj], s_site[OFF_DP + 6 * b + 1][jj], s_site[OFF_DP + 6 * b + 2][jj]};
              const Real eb[3] = {s_site[OFF_DP + 6 * b + 3][jj], s_site[OFF_DP + 6 * b + 4][jj], s_site[OFF_DP + 6 * b + 5][jj]};
              mp_site_pair<Real, 2, 2, CENTRAL>(s_mdp[spi][a] * s_mdp[spj][b] * kk, pa, ea, pb, eb, Rx, Ry, Rz, R2, acc, fd[a], gd[a], rf_dd, krf);
            }
            if constexpr (S.qd > 0) {
#pragma unroll
              for (int b = 0; b < S.qd; ++b) {
                if (b >= nqd_j) break;
                const Real pb[3] = {s_site[OFF_QD + 6 * b][jj], s_site[OFF_QD + 6 * b + 1][jj], s_site[OFF_QD + 6 * b + 2][jj]};
                const Real eb[3] = {s_site[OFF_QD + 6 * b + 3][jj], s_site[OFF_QD + 6 * b + 4][jj], s_site[OFF_QD + 6 * b + 5][jj]};
                mp_site_pair<Real, 2, 3, CENTRAL>(s_mdp[spi][a] * s_mqd[spj][b] * kk, pa, ea, pb, eb, Rx, Ry, Rz, R2, acc, fd[a], gd[a], false, krf);
              }
            }
          }
        }
        // a = quadrupole on i
        if constexpr (S.qd > 0) {
#pragma unroll
          for (int a = 0; a < S.qd; ++a) {
            if (a >= nqd_i) break;
            const Real* pa = &rec[OFF_QD + 6 * a];
            const Real* ea = &rec[OFF_QD + 6 * a + 3];
            if constexpr (S.ch > 0) {
#pragma unroll
              for (int b = 0; b < S.ch; ++b) {
                if (b >= nch_j) break;
                const Real pb[3] = {s_site[OFF_CH + 3 * b][jj], s_site[OFF_CH + 3 * b + 1][jj], s_site[OFF_CH + 3 * b + 2][jj]};
                mp_site_pair<Real, 3, 1, CENTRAL>(s_mqd[spi][a] * s_mch[spj][b] * kk, pa, ea, pb, zero3, Rx, Ry, Rz, R2, acc, fq[a], gq[a], false, krf);
              }
            }
            if constexpr (S.dp > 0) {
#pragma unroll
              for (int b = 0; b < S.dp; ++b) {
                if (b >= ndp_j) break;
                const Real pb[3] = {s_site[OFF_DP + 6 * b][jj], s_site[OFF_DP + 6 * b + 1][jj], s_site[OFF_DP + 6 * b + 2][jj]};
                const Real eb[3] = {s_site[OFF_DP + 6 * b + 3][jj], s_site[OFF_DP + 6 * b + 4][jj], s_site[OFF_DP + 6 * b + 5][jj]};
                mp_site_pair<Real, 3, 2, CENTRAL>(s_mqd[spi][a] * s_mdp[spj][b] * kk, pa, ea, pb, eb, Rx, Ry, Rz, R2, acc, fq[a], gq[a], false, krf);
              }
            }
#pragma unroll
            for (int b = 0; b < S.qd; ++b) {
              if (b >= nqd_j) break;
              const Real pb[3] = {s_site[OFF_QD + 6 * b][jj], s_site[OFF_QD + 6 * b + 1][jj], s_site[OFF_QD + 6 * b + 2][jj]};
              const Real eb[3] = {s_site[OFF_QD + 6 * b + 3][jj], s_site[OFF_QD + 6 * b + 4][jj], s_site[OFF_QD + 6 * b + 5][jj]};
              mp_site_pair<Real, 3, 3, CENTRAL>(s_mqd[spi][a] * s_mqd[spj][b] * kk, pa, ea, pb, eb, Rx, Ry, Rz, R2, acc, fq[a], gq[a], false, krf);
            }
          }
        }
      }
      a_ulj += (double)acc.ulj;
      a_uel += (double)acc.uel;
      a_uss += (double)acc.uss;
      a_us -= (double)(Rx * acc.fx + Ry * acc.fy + Rz * acc.fz);
      a_np += 1;
      a_ns += s_nsite[spi][spj];
    }

    // fold this tile's site forces into FP64 force and torque (tau = d x f + e x g)
    auto fold = [&](const Real* d, Real* f) {
      const double fx = f[0], fy = f[1], fz = f[2];
      F[0] += fx; F[1] += fy; F[2] += fz;
      T[0] += (double)d[1] * fz - (double)d[2] * fy;
      T[1] += (double)d[2] * fx - (double)d[0] * fz;
      T[2] += (double)d[0] * fy - (double)d[1] * fx;
    };
    auto fold_g = [&](const Real* e, Real* g) {
      T[0] += (double)e[1] * g[2] - (double)e[2] * g[1];
      T[1] += (double)e[2] * g[0] - (double)e[0] * g[2];
      T[2] += (double)e[0] * g[1] - (double)e[1] * g[0];
    };
#pragma unroll
    for (int a = 0; a < S.lj; ++a) fold(&rec[3 * a], fl[a]);
#pragma unroll
    for (int a = 0; a < S.ch; ++a) fold(&rec[OFF_CH + 3 * a], fc[a]);
#pragma unroll
    for (int a = 0; a < S.dp; ++a) { fold(&rec[OFF_DP + 6 * a], fd[a]); fold_g(&rec[OFF_DP + 6 * a + 3], gd[a]); }
#pragma unroll
    for (int a = 0; a < S.qd; ++a) { fold(&rec[OFF_QD + 6 * a], fq[a]); fold_g(&rec[OFF_QD + 6 * a + 3], gq[a]); }
    zero_site_acc();
  }

  // per-molecule partials of this j range
  if (iv) {
    double* pf = sd.pf + (size_t)it.part * 6 * np;
    pf[0 * np + i] = F[0]; pf[1 * np + i] = F[1]; pf[2 * np + i] = F[2];
    pf[3 * np + i] = T[0]; pf[4 * np + i] = T[1]; pf[5 * np + i] = T[2];
  }
  // block sums in a fixed tree order
  __syncthreads();
  s_red[0][tid] = a_ulj; s_red[1][tid] = a_uel; s_red[2][tid] = a_us; s_red[3][tid] = a_uss;
  s_red[4][tid] = (double)a_np; s_red[5][tid] = (double)a_ns;
  __syncthreads();
  for (int h = TJ / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int k = 0; k < kNumBlockSums; ++k) s_red[k][tid] += s_red[k][tid + h];
    __syncthreads();
  }
  if (tid < kNumBlockSums) sd.bsum[(size_t)it.local * kNumBlockSums + tid] = s_red[tid][0];
}

// ---------------------------------------------------------------------------
// Fixed-order reductions of the pair partials.
//  reduce_force_kernel: one thread per molecule sums its j-range partials in
//    order; grid (molecule blocks, slots).  OVERWRITES force and torque.
//  reduce_sums_kernel: one block per slot; item sums (each thread a
//    contiguous run, then a tree), species counts, Ewald constants and the LJ
//    tail.  OVERWRITES sums.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_force_kernel(const SlotDev* __restrict__ slots) {
  const SlotDev& sd = slots[blockIdx.y];
  if (!sd.active) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= sd.n) return;
  const int np = sd.npad, ld = sd.com_ld;
  double v[6] = {0, 0, 0, 0, 0, 0};
  for (int p = 0; p < sd.jsplits; ++p)
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] += sd.pf[((size_t)p * 6 + c) * np + i];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    sd.force[c * ld + i] = v[c];
    sd.torque[c * ld + i] = v[3 + c];
  }
}

__global__ __launch_bounds__(256) void reduce_sums_kernel(const SlotDev* __restrict__ slots,
                                                          const SysParams* __restrict__ prm) {
  __shared__ double s_red[kNumBlockSums][256];
  __shared__ int s_cnt[kMaxSp][256];
  const SlotDev& sd = slots[blockIdx.x];
  if (!sd.active) return;
  const SysParams& P = prm[blockIdx.x];
  const int tid = threadIdx.x, n = sd.n;
  int cnt[kMaxSp];
#pragma unroll
  for (int s = 0; s < kMaxSp; ++s) cnt[s] = 0;
  for (int i = tid; i < n; i += 256) {
    const int s = clamp_species(sd.species[i], P.nsp);
#pragma unroll
    for (int x = 0; x < kMaxSp; ++x) cnt[x] += (s == x);
  }
  const int ni = sd.nitems;
  const int per = (ni + 255) / 256;
  double acc[kNumBlockSums] = {0, 0, 0, 0, 0, 0};
  for (int t = tid * per; t < min(ni, (tid + 1) * per); ++t)
#pragma unroll
    for (int k = 0; k < kNumBlockSums; ++k) acc[k] += sd.bsum[(size_t)t * kNumBlockSums + k];
#pragma unroll
  for (int k = 0; k < kNumBlockSums; ++k) s_red[k][tid] = acc[k];
#pragma unroll
  for (int x = 0; x < kMaxSp; ++x) s_cnt[x][tid] = cnt[x];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      for (int k = 0; k < kNumBlockSums; ++k) s_red[k][tid] += s_red[k][tid + h];
      for (int x = 0; x < kMaxSp; ++x) s_cnt[x][tid] += s_cnt[x][tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* out = sd.sums;
    // every pair was evaluated from both sides
    out[MS2_SUM_U_LJ] = 0.5 * s_red[0][0];
    out[MS2_SUM_U_ELEC] = 0.5 * s_red[1][0];
    out[MS2_SUM_US] = 0.5 * s_red[2][0];
    out[MS2_SUM_VIRIAL] = -0.5 * s_red[2][0];
    out[MS2_SUM_USS] = 0.5 * s_red[3][0];
    out[MS2_SUM_NPAIR] = 0.5 * s_red[4][0];
    out[MS2_SUM_NSITE] = 0.5 * s_red[5][0];
    out[MS2_SUM_U_RECIP] = 0.0;
    double uc = 0.0, ul = 0.0, usl = 0.0, ussl = 0.0;
    for (int a = 0; a < P.nsp; ++a) {
      const double na = (double)s_cnt[a][0];
      if (P.elec == MS2_ELEC_EWALD) uc += na * P.ew_const[a];
      if (P.lrc)
        for (int b = 0; b < P.nsp; ++b) {
          const double nab = na * (double)s_cnt[b][0];
          ul += nab * P.lrc_u[a][b];
          usl += nab * P.lrc_us[a][b];
          ussl += nab * P.lrc_uss[a][b];
        }
    }
    out[MS2_SUM_U_CONST] = uc;
    out[MS2_SUM_U_LRC] = ul;
    out[MS2_SUM_US_LRC] = usl;
    out[MS2_SUM_USS_LRC] = ussl;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename Real, int C>
static hipError_t launch_frame_c(const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                                 int nslots, int max_n, hipStream_t st) {
  dim3 grid((max_n + 255) / 256, nslots);
  hipLaunchKernelGGL((site_frame_kernel<Real, C>), grid, dim3(256), 0, st, slots, prm, tab);
  return hipGetLastError();
}

hipError_t launch_site_frame(int cls, int precision, const SlotDev* slots, const SysParams* prm,
                             const SpeciesTable* tab, int nslots, int max_n, hipStream_t st) {
#define MS2_FRAME_CASE(C)                                                                       \
  case C:                                                                                       \
    return precision == MS2_FP32 ? launch_frame_c<float, C>(slots, prm, tab, nslots, max_n, st) \
                                 : launch_frame_c<double, C>(slots, prm, tab, nslots, max_n, st);
  switch (cls) {
    MS2_FRAME_CASE(0)
    MS2_FRAME_CASE(1)
    MS2_FRAME_CASE(2)
    MS2_FRAME_CASE(3)
    MS2_FRAME_CASE(4)
    MS2_FRAME_CASE(5)
  }
#undef MS2_FRAME_CASE
  return hipErrorInvalidValue;
}

template <typename Real, int C, int W>
static hipError_t launch_pair_cw(const WorkItem* items, int base, int count, const SlotDev* slots,
                                 const SysParams* prm, const SpeciesTable* tab, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((pair_kernel<Real, C, W>), dim3(count), dim3(64 * W), 0, st, items, base, slots,
                     prm, tab);
  return hipGetLastError();
}

template <typename Real, int C>
static hipError_t launch_pair_c(int waves, const WorkItem* items, int base, int count,
                                const SlotDev* slots, const SysParams* prm,
                                const SpeciesTable* tab, hipStream_t st) {
  if constexpr (C <= 3) {
    if (waves == 4) return launch_pair_cw<Real, C, 4>(items, base, count, slots, prm, tab, st);
  }
  return launch_pair_cw<Real, C, 1>(items, base, count, slots, prm, tab, st);
}

hipError_t launch_pair(int cls, int precision, int waves, const WorkItem* items, int base,
                       int count, const SlotDev* slots, const SysParams* prm,
                       const SpeciesTable* tab, hipStream_t st) {
#define MS2_PAIR_CASE(C)                                                                        \
  case C:                                                                                       \
    return precision == MS2_FP32                                                                \
               ? launch_pair_c<float, C>(waves, items, base, count, slots, prm, tab, st)        \
               : launch_pair_c<double, C>(waves, items, base, count, slots, prm, tab, st);
  switch (cls) {
    MS2_PAIR_CASE(0)
    MS2_PAIR_CASE(1)
    MS2_PAIR_CASE(2)
    MS2_PAIR_CASE(3)
    MS2_PAIR_CASE(4)
    MS2_PAIR_CASE(5)
  }
#undef MS2_PAIR_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_pair(const SlotDev* slots, const SysParams* prm, int nslots, int max_n,
                              hipStream_t st) {
  hipLaunchKernelGGL(reduce_force_kernel, dim3((max_n + 255) / 256, nslots), dim3(256), 0, st, slots);
  hipLaunchKernelGGL(reduce_sums_kernel, dim3(nslots), dim3(256), 0, st, slots, prm);
  return hipGetLastError();
}

}  // namespace ms2
