// Device arithmetic shared by the pair kernels (row-owned and symmetric):
// approximate reciprocals with a Newton step, the minimum-image centre
// difference, and the point-multipole site-pair terms.
#pragma once
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

// Squared minimum-image distance only, for centres wrapped into [0, L): a
// component difference d lies in (-L, L) and its minimum-image magnitude is
// min(|d|, L - |d|), with L - |d| rounded exactly as |d - L sign(d)|.  The
// value equals min_image's r2 bit for bit wherever the nearest image is
// unique (|d| not within rounding of L/2, where the component alone exceeds
// any admissible cut-off).
__device__ __forceinline__ double min_image_r2(double xi, double yi, double zi, double xj, double yj,
                                               double zj, double L) {
#pragma clang fp contract(off)
  const double ax = fabs(xi - xj), ay = fabs(yi - yj), az = fabs(zi - zj);
  const double mx = fmin(ax, L - ax), my = fmin(ay, L - ay), mz = fmin(az, L - az);
  return mx * mx + my * my + mz * mz;
}

// Separation of a site pair, r = R + delta, from the molecules' centre
// difference R (components, and |R|^2 rounded once from FP64) and the
// difference delta = d_a - d_b of the sites' lab offsets:
//   |r|^2 = |R|^2 + (2 R.delta + delta.delta),   r.R = |R|^2 + R.delta.
// The rounding of R's components enters only through the small terms (it
// is scaled by |delta|), so in FP32 |r|^2 carries about one rounding of its
// own instead of the roundings of three sums of a large and a small term
// This holds for r comparable to R: the error of |R|^2 grows as R^2 / r^2
// when r << R.  The pair kernels take it for the LJ sites of the model
// classes whose sites sit close to the centre (LJ fluids, two-centre LJ +
// quadrupole, water-like models, Stockmayer), where LJ repulsion keeps r
// near R; charges, which approach closer, and the classes with sites far
// off the centre take site_direct.
template <typename Real>
__device__ __forceinline__ void site_separation(Real Rx, Real Ry, Real Rz, Real R2, Real dx, Real dy, Real dz,
                                                Real& rx, Real& ry, Real& rz, Real& r2, Real& rR) {
  const Real Rd = Rx * dx + Ry * dy + Rz * dz;
  const Real dd = dx * dx + dy * dy + dz * dz;
  r2 = R2 + (Real(2) * Rd + dd);
  rR = R2 + Rd;
  rx = Rx + dx;
  ry = Ry + dy;
  rz = Rz + dz;
}

// The same separation formed directly: r = R + delta component by component.
template <typename Real>
__device__ __forceinline__ void site_direct(Real Rx, Real Ry, Real Rz, Real dx, Real dy, Real dz, Real& rx,
                                            Real& ry, Real& rz, Real& r2, Real& rR) {
  rx = Rx + dx;
  ry = Ry + dy;
  rz = Rz + dz;
  r2 = rx * rx + ry * ry + rz * rz;
  rR = rx * Rx + ry * Ry + rz * Rz;
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
// of j.  Adds the force on a to fs, -du/dea to gs (when a is oriented) and,
// with JSIDE, -du/deb to gsb (when b is oriented); the force on b is -f.
// CENTRAL: both sites at their molecules' centres, so r = R and the
// volume-derivative terms follow from homogeneity (u ~ r^-p).
template <typename Real, int TA, int TB, bool CENTRAL_CLASS, bool JSIDE = false>
__device__ __forceinline__ void mp_site_pair(Real K, const Real* pa, const Real* ea, const Real* pb,
                                             const Real* eb, Real Rx, Real Ry, Real Rz, Real R2,
                                             PairAcc<Real>& acc, Real* fs, Real* gs, bool rf_dd,
                                             Real krf, Real* gsb = nullptr) {
  constexpr int p = MpPower<TA, TB>::p;
  // the class guarantees centred dipoles/quadrupoles, not centred charges
  constexpr bool CENTRAL = CENTRAL_CLASS && TA != 1 && TB != 1;
  // off-centre multipoles may approach much closer than their centres
  // (r << R), where the expansion of site_separation loses what it gains
  // elsewhere: r is formed directly
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
  if constexpr (JSIDE && TB != 1) {
    Real gx = q.Pb * nx, gy = q.Pb * ny, gz = q.Pb * nz;
    if constexpr (TA != 1) { gx += q.Pc * ea[0]; gy += q.Pc * ea[1]; gz += q.Pc * ea[2]; }
    gsb[0] -= Kp * gx; gsb[1] -= Kp * gy; gsb[2] -= Kp * gz;
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
      if constexpr (JSIDE) {
        gsb[0] += Real(2) * krf * K * ea[0];
        gsb[1] += Real(2) * krf * K * ea[1];
        gsb[2] += Real(2) * krf * K * ea[2];
      }
    }
  }
}


// Compile-time tag of a site-type pair (1 charge, 2 dipole, 3 quadrupole).
template <int A, int B>
struct SitePairTag {
  static constexpr int a = A, b = B;
};

// Per-site force (and orientation-gradient) accumulators of one molecule.
template <typename Real, int C>
struct SiteAcc {
  static constexpr ClassShape S = kClassShapes[C];
  static constexpr int NLJ = S.lj > 0 ? S.lj : 1, NCH = S.ch > 0 ? S.ch : 1;
  static constexpr int NDP = S.dp > 0 ? S.dp : 1, NQD = S.qd > 0 ? S.qd : 1;
  Real fl[NLJ][3], fc[NCH][3], fd[NDP][3], gd[NDP][3], fq[NQD][3], gq[NQD][3];
  // Sums start at -0: -0 + x is x for every x, so the compiler drops the
  // first addition and the zeroing move (it may not drop +0 + x, which
  // turns -0 into +0).
  __device__ __forceinline__ void zero() {
    constexpr Real z = -Real(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int a = 0; a < NLJ; ++a) fl[a][c] = z;
#pragma unroll
      for (int a = 0; a < NCH; ++a) fc[a][c] = z;
#pragma unroll
      for (int a = 0; a < NDP; ++a) { fd[a][c] = z; gd[a][c] = z; }
#pragma unroll
      for (int a = 0; a < NQD; ++a) { fq[a][c] = z; gq[a][c] = z; }
    }
  }
};

// LDS tables of the species of one system, as the pair kernels stage them,
// for up to MAXSP species (1 in the single-species form).
template <typename Real, int C, int MAXSP = kMaxSp>
struct PairTables {
  static constexpr ClassShape S = kClassShapes[C];
  static constexpr int NLJ = S.lj > 0 ? S.lj : 1, NCH = S.ch > 0 ? S.ch : 1;
  static constexpr int NDP = S.dp > 0 ? S.dp : 1, NQD = S.qd > 0 ? S.qd : 1;
  Real c6[MAXSP * NLJ][MAXSP * NLJ];
  Real c12[MAXSP * NLJ][MAXSP * NLJ];
  int cnt[MAXSP][4];
  // k_e * magnitude, in FP64: the prefactor k_e m_a m_b of an electrostatic
  // site pair is formed in FP64 and rounded to Real once (kprod), so that
  // every pair of a kind carries the same single rounding of it at most
  double mch[MAXSP][NCH], mdp[MAXSP][NDP], mqd[MAXSP][NQD];
  int nsite[MAXSP][MAXSP];

  // nsp: the species in use (1 when every molecule is species 0, whatever
  // the context holds; at most MAXSP).  The LJ tables are walked over their
  // full size with compile-time divisors; entries of unused species are left
  // unset.
  __device__ void load(const SpeciesTable* tab, const SysParams& P, int nsp, int tid, int nthreads) {
    nsp = min(nsp, MAXSP);
    constexpr int W = MAXSP * NLJ;
    for (int e = tid; e < W * W; e += nthreads) {
      const int r = e / W, c = e % W;
      const int A = r / NLJ, a = r % NLJ, B = c / NLJ, b = c % NLJ;
      if (A < nsp && B < nsp) {
        c6[r][c] = (Real)tab->c6[A][a][B][b];
        c12[r][c] = (Real)tab->c12[A][a][B][b];
      }
    }
    for (int e = tid; e < nsp; e += nthreads) {
      const SpeciesDev& D = tab->sp[e];
      cnt[e][0] = D.nlj; cnt[e][1] = D.nch; cnt[e][2] = D.ndp; cnt[e][3] = D.nqd;
      for (int a = 0; a < NCH; ++a) mch[e][a] = P.ke * D.ch_q[a];
      for (int a = 0; a < NDP; ++a) mdp[e][a] = P.ke * D.dp_mu[a];
      for (int a = 0; a < NQD; ++a) mqd[e][a] = P.ke * D.qd_Q[a];
      for (int b = 0; b < nsp; ++b) nsite[e][b] = tab->nsite_pair[e][b];
    }
  }
};

// Electrostatic mode constants in the pair's precision.
template <typename Real>
struct ElecParams {
  int elec;
  Real krf, crf, alpha, alpha2, gpref;
  double inv_ke;
};

// k_e m_a m_b from the FP64 magnitudes (each k_e m), rounded once.
template <typename Real>
__device__ __forceinline__ Real kprod(double ma, double mb, double inv_ke) {
  return (Real)(ma * mb * inv_ke);
}

// The FP64 decision of the site-site cut-off for LJ site pair (a, b):
// r = (R + d_a) - d_b from the FP64 minimum-image centre difference R and
// the FP64 lab offsets of the two sites (component k of site a at
// li[3 a + k] times the stride), |r|^2 summed in the order x, y, z, each
// operation rounded as written, accepted iff |r|^2 < rc^2 -- the same
// arithmetic, so the same decision, as a plain FP64 evaluation.
struct SiteCut {
  const double* R = nullptr;    // [3]
  const double* li = nullptr;   // LJ offsets of molecule i
  const double* lj = nullptr;   // LJ offsets of molecule j
  double rc2 = 0.0;
  __device__ __forceinline__ bool inside(int a, int b, int stride) const {
#pragma clang fp contract(off)
    const double x = (R[0] + li[(3 * a) * stride]) - lj[(3 * b) * stride];
    const double y = (R[1] + li[(3 * a + 1) * stride]) - lj[(3 * b + 1) * stride];
    const double z = (R[2] + li[(3 * a + 2) * stride]) - lj[(3 * b + 2) * stride];
    double r2 = x * x;
    r2 = r2 + y * y;
    r2 = r2 + z * z;
    return r2 < rc2;
  }
};

// All site pairs of one accepted molecule pair (i, j) with centre difference
// R = R_i - R_j (components Rx, Ry, Rz and R2 = |R|^2, each rounded once
// from the FP64 minimum-image difference).  rec: the site record of i (registers); sj: the record of j,
// component k at sj[k * STRIDE] (LDS).  Forces and orientation gradients on
// i's sites go to ai; with JSIDE those on j's sites go to aj (force on a j
// site is minus the force on its partner).  acc collects the pair's energy,
// total force on i and d2U/ds2.
// ONE: the system has one species (spi = spj = 0); its site counts are then
// wave-uniform and the site loops branch on scalars.
// SITE: the site-site cut-off mode.  An LJ site pair then interacts only
// when its own squared distance is below rc^2, decided in FP64 by `cut`
// (and adds one to *nlj_in), and the electrostatic site pairs only when
// elec_in (the centres inside the cut-off).  Without SITE every site pair of
// the molecule pair interacts.
template <typename Real, int C, bool JSIDE, int STRIDE, bool SITE = false, bool ONE = false>
__device__ __forceinline__ void eval_molecule_pair(const Real* rec, const Real* sj, int spi, int spj,
                                                   const PairTables<Real, C, ONE ? 1 : kMaxSp>& T,
                                                   const ElecParams<Real>& E, Real Rx, Real Ry,
                                                   Real Rz, Real R2, SiteAcc<Real, C>& ai,
                                                   SiteAcc<Real, C>& aj, PairAcc<Real>& acc,
                                                   SiteCut cut = SiteCut{}, bool elec_in = true,
                                                   int* nlj_in = nullptr) {
  constexpr ClassShape S = kClassShapes[C];
  constexpr int NLJ = SiteAcc<Real, C>::NLJ;
  constexpr int OFF_CH = 3 * S.lj, OFF_DP = OFF_CH + 3 * S.ch, OFF_QD = OFF_DP + 6 * S.dp;
  constexpr bool CENTRAL = S.central != 0;
  auto count = [&](int sp, int k) {
    return ONE ? __builtin_amdgcn_readfirstlane(T.cnt[0][k]) : T.cnt[sp][k];
  };
  const int nlj_i = count(spi, 0), nch_i = count(spi, 1), ndp_i = count(spi, 2), nqd_i = count(spi, 3);
  const int nlj_j = count(spj, 0), nch_j = count(spj, 1), ndp_j = count(spj, 2), nqd_j = count(spj, 3);
  if constexpr (ONE) {
    // the single-species form is taken only for a species with at least one
    // site of every kind its class holds: the first site pair of each kind
    // always runs, so its sums start from it instead of from -0
    if constexpr (S.lj > 0) __builtin_assume(nlj_i >= 1 && nlj_j >= 1);
    if constexpr (S.ch > 0) __builtin_assume(nch_i >= 1 && nch_j >= 1);
    if constexpr (S.dp > 0) __builtin_assume(ndp_i >= 1 && ndp_j >= 1);
    if constexpr (S.qd > 0) __builtin_assume(nqd_i >= 1 && nqd_j >= 1);
  }
  auto J = [&](int k) { return sj[k * STRIDE]; };

  // Lennard-Jones site pairs; d2U/ds2 takes (u'' - u'/r) (r.R)^2 / r^2 =
  // (168 t12 - 48 t6) (r.R / r^2)^2 per site pair and the (u'/r) R^2 part of
  // all of them at once
  Real lj_dur = -Real(0);
#pragma unroll
  for (int a = 0; a < S.lj; ++a) {
    if (a >= nlj_i) break;
#pragma unroll
    for (int b = 0; b < S.lj; ++b) {
      if (b >= nlj_j) break;
      Real rx, ry, rz, r2, rR;
      if constexpr (CENTRAL) {
        site_separation(Rx, Ry, Rz, R2, rec[3 * a] - J(3 * b), rec[3 * a + 1] - J(3 * b + 1),
                        rec[3 * a + 2] - J(3 * b + 2), rx, ry, rz, r2, rR);
      } else {
        site_direct(Rx, Ry, Rz, rec[3 * a] - J(3 * b), rec[3 * a + 1] - J(3 * b + 1),
                    rec[3 * a + 2] - J(3 * b + 2), rx, ry, rz, r2, rR);
      }
      const Real ir2 = rcp_(r2);
      const Real ir6 = ir2 * ir2 * ir2;
      Real t6 = T.c6[spi * NLJ + a][spj * NLJ + b] * ir6;
      Real t12 = T.c12[spi * NLJ + a][spj * NLJ + b] * ir6 * ir6;
      if constexpr (SITE) {
        const bool in = cut.inside(a, b, STRIDE);
        *nlj_in += in ? 1 : 0;
        t6 = in ? t6 : Real(0);
        t12 = in ? t12 : Real(0);
      }
      const Real dur = (Real(6) * t6 - Real(12) * t12) * ir2;       // u'/r
      const Real p = rR * ir2;
      acc.ulj += t12 - t6;
      acc.uss += (Real(168) * t12 - Real(48) * t6) * (p * p);
      lj_dur += dur;
      const Real fx = -dur * rx, fy = -dur * ry, fz = -dur * rz;
      ai.fl[a][0] += fx; ai.fl[a][1] += fy; ai.fl[a][2] += fz;
      if constexpr (JSIDE) { aj.fl[b][0] -= fx; aj.fl[b][1] -= fy; aj.fl[b][2] -= fz; }
      acc.fx += fx; acc.fy += fy; acc.fz += fz;
    }
  }
  acc.uss += lj_dur * R2;
  if (SITE && !elec_in) return;
  // charge-charge site pairs
  if constexpr (S.ch > 0) {
#pragma unroll
    for (int a = 0; a < S.ch; ++a) {
      if (a >= nch_i) break;
#pragma unroll
      for (int b = 0; b < S.ch; ++b) {
        if (b >= nch_j) break;
        const Real K = kprod<Real>(T.mch[spi][a], T.mch[spj][b], E.inv_ke);
        Real rx, ry, rz, r2, rR;
        site_direct(Rx, Ry, Rz, rec[OFF_CH + 3 * a] - J(OFF_CH + 3 * b),
                    rec[OFF_CH + 3 * a + 1] - J(OFF_CH + 3 * b + 1),
                    rec[OFF_CH + 3 * a + 2] - J(OFF_CH + 3 * b + 2), rx, ry, rz, r2, rR);
        const Real ir = rsq_(r2), ir2 = ir * ir;
        Real u, dur, d2u;
        if (E.elec == MS2_ELEC_EWALD) {
          const Real r = r2 * ir;
          const Real e = erfc_(E.alpha * r);
          const Real gs = E.gpref * exp_(-E.alpha2 * r2);
          u = K * e * ir;
          dur = -K * (e * ir + gs) * ir2;
          d2u = K * (Real(2) * e * ir * ir2 + gs * (Real(2) * ir2 + Real(2) * E.alpha2));
        } else if (E.elec == MS2_ELEC_RF) {
          u = K * (ir + E.krf * r2 - E.crf);
          dur = K * (Real(2) * E.krf - ir * ir2);
          d2u = K * (Real(2) * ir * ir2 + Real(2) * E.krf);
        } else {
          u = K * ir;
          dur = -K * ir * ir2;
          d2u = Real(2) * K * ir * ir2;
        }
        acc.uel += u;
        acc.uss += (d2u - dur) * (rR * rR * ir2) + dur * R2;
        const Real fx = -dur * rx, fy = -dur * ry, fz = -dur * rz;
        ai.fc[a][0] += fx; ai.fc[a][1] += fy; ai.fc[a][2] += fz;
        if constexpr (JSIDE) { aj.fc[b][0] -= fx; aj.fc[b][1] -= fy; aj.fc[b][2] -= fz; }
        acc.fx += fx; acc.fy += fy; acc.fz += fz;
      }
    }
  }
  // point multipoles (all pairs involving a dipole or quadrupole)
  if constexpr (S.dp > 0 || S.qd > 0) {
    const bool rf_dd = E.elec == MS2_ELEC_RF;
    const Real zero3[3] = {0, 0, 0};
    Real gdummy[3] = {0, 0, 0};
    auto jrec = [&](int off, Real* p) { p[0] = J(off); p[1] = J(off + 1); p[2] = J(off + 2); };
    auto sub_f = [&](Real* dst, Real fx0, Real fy0, Real fz0) { dst[0] -= fx0; dst[1] -= fy0; dst[2] -= fz0; };
    // each call adds the force on i's site to `fa`; the j-site force is the
    // change of acc.f, so it is taken as a difference
    auto pair = [&](auto ta_tb, Real K, const Real* pa, const Real* ea, const Real* pb, const Real* eb,
                    Real* fa, Real* ga, Real* fb, Real* gb) {
      constexpr int TA = decltype(ta_tb)::a, TB = decltype(ta_tb)::b;
      const Real f0x = acc.fx, f0y = acc.fy, f0z = acc.fz;
      mp_site_pair<Real, TA, TB, CENTRAL, JSIDE>(K, pa, ea, pb, eb, Rx, Ry, Rz, R2, acc, fa, ga,
                                                  TA == 2 && TB == 2 && rf_dd, E.krf, gb);
      if constexpr (JSIDE) sub_f(fb, acc.fx - f0x, acc.fy - f0y, acc.fz - f0z);
    };
    if constexpr (S.ch > 0) {
#pragma unroll
      for (int a = 0; a < S.ch; ++a) {
        if (a >= nch_i) break;
        const Real* pa = &rec[OFF_CH + 3 * a];
        if constexpr (S.dp > 0) {
#pragma unroll
          for (int b = 0; b < S.dp; ++b) {
            if (b >= ndp_j) break;
            Real pb[3], eb[3];
            jrec(OFF_DP + 6 * b, pb);
            jrec(OFF_DP + 6 * b + 3, eb);
            pair(SitePairTag<1, 2>{}, kprod<Real>(T.mch[spi][a], T.mdp[spj][b], E.inv_ke), pa, zero3, pb, eb, ai.fc[a], gdummy,
                 aj.fd[b], aj.gd[b]);
          }
        }
        if constexpr (S.qd > 0) {
#pragma unroll
          for (int b = 0; b < S.qd; ++b) {
            if (b >= nqd_j) break;
            Real pb[3], eb[3];
            jrec(OFF_QD + 6 * b, pb);
            jrec(OFF_QD + 6 * b + 3, eb);
            pair(SitePairTag<1, 3>{}, kprod<Real>(T.mch[spi][a], T.mqd[spj][b], E.inv_ke), pa, zero3, pb, eb, ai.fc[a], gdummy,
                 aj.fq[b], aj.gq[b]);
          }
        }
      }
    }
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
            Real pb[3];
            jrec(OFF_CH + 3 * b, pb);
            pair(SitePairTag<2, 1>{}, kprod<Real>(T.mdp[spi][a], T.mch[spj][b], E.inv_ke), pa, ea, pb, zero3, ai.fd[a], ai.gd[a],
                 aj.fc[b], gdummy);
          }
        }
#pragma unroll
        for (int b = 0; b < S.dp; ++b) {
          if (b >= ndp_j) break;
          Real pb[3], eb[3];
          jrec(OFF_DP + 6 * b, pb);
          jrec(OFF_DP + 6 * b + 3, eb);
          pair(SitePairTag<2, 2>{}, kprod<Real>(T.mdp[spi][a], T.mdp[spj][b], E.inv_ke), pa, ea, pb, eb, ai.fd[a], ai.gd[a],
               aj.fd[b], aj.gd[b]);
        }
        if constexpr (S.qd > 0) {
#pragma unroll
          for (int b = 0; b < S.qd; ++b) {
            if (b >= nqd_j) break;
            Real pb[3], eb[3];
            jrec(OFF_QD + 6 * b, pb);
            jrec(OFF_QD + 6 * b + 3, eb);
            pair(SitePairTag<2, 3>{}, kprod<Real>(T.mdp[spi][a], T.mqd[spj][b], E.inv_ke), pa, ea, pb, eb, ai.fd[a], ai.gd[a],
                 aj.fq[b], aj.gq[b]);
          }
        }
      }
    }
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
            Real pb[3];
            jrec(OFF_CH + 3 * b, pb);
            pair(SitePairTag<3, 1>{}, kprod<Real>(T.mqd[spi][a], T.mch[spj][b], E.inv_ke), pa, ea, pb, zero3, ai.fq[a], ai.gq[a],
                 aj.fc[b], gdummy);
          }
        }
        if constexpr (S.dp > 0) {
#pragma unroll
          for (int b = 0; b < S.dp; ++b) {
            if (b >= ndp_j) break;
            Real pb[3], eb[3];
            jrec(OFF_DP + 6 * b, pb);
            jrec(OFF_DP + 6 * b + 3, eb);
            pair(SitePairTag<3, 2>{}, kprod<Real>(T.mqd[spi][a], T.mdp[spj][b], E.inv_ke), pa, ea, pb, eb, ai.fq[a], ai.gq[a],
                 aj.fd[b], aj.gd[b]);
          }
        }
#pragma unroll
        for (int b = 0; b < S.qd; ++b) {
          if (b >= nqd_j) break;
          Real pb[3], eb[3];
          jrec(OFF_QD + 6 * b, pb);
          jrec(OFF_QD + 6 * b + 3, eb);
          pair(SitePairTag<3, 3>{}, kprod<Real>(T.mqd[spi][a], T.mqd[spj][b], E.inv_ke), pa, ea, pb, eb, ai.fq[a], ai.gq[a],
               aj.fq[b], aj.gq[b]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Linear two-centre LJ + quadrupole molecules (one species): both LJ sites on
// the quadrupole's axis, at +d and -d from the centre (the site frame gives
// the second offset as the exact negation of the first), equal LJ
// coefficients, the quadrupole at the centre.  With d_i, d_j the lab offsets
// of the first LJ site of each molecule, the four LJ site pairs have
// separations R + delta, delta = +-(d_i - d_j) or +-(d_i + d_j), so two
// difference vectors give every |r|^2 = |R|^2 + (2 R.delta + delta.delta)
// and r.R = |R|^2 + R.delta -- the same values, bit for bit, as
// site_separation forms from the four site pairs one by one.  The pairs'
// forces and torques collapse onto the vectors R, d_i, d_j:
//   F_i   = -(sum u'/r) R - (E_m + E_p) d_i + (E_m - E_p) d_j
//   tau_i = d_i x (sum_a s_a f_a) = -(E_m + E_p) (d_i x R) + (S_m - S_p) (d_i x d_j)
// with E_m = u'/r(++) - u'/r(--), S_m = u'/r(++) + u'/r(--) and E_p, S_p
// the same for (+-), (-+).  The quadrupole pair (r = R, n = R / |R|,
// c_a = e_i.n, c_b = e_j.n, c_ab = e_i.e_j) adds
// A [(5 P + P_a c_a + P_b c_b) n - P_a e_i - P_b e_j] (A = K |R|^-6) to F_i
// and e_i x g_i, g_i = -K |R|^-5 (P_a n + P_c e_j), to tau_i.  No constant of
// the geometry (h) enters: every rounding is per molecule, as in the general
// form.  The caller takes tau_j from tau_i + tau_j + R x F_i = 0.
template <typename Real>
struct LinearModel {
  Real c6, c12, K;   // LJ coefficients, k_e Q^2
};

// ri, rj: the staged record of each molecule, [d (first LJ site), e (axis)]
template <typename Real>
__device__ __forceinline__ void eval_linear_pair(const Real* ri, const Real* rj, Real Rx, Real Ry, Real Rz,
                                                 Real R2, const LinearModel<Real>& M, PairAcc<Real>& acc,
                                                 Real* F, Real* T) {
  const Real* di = ri;
  const Real* ei = ri + 3;
  const Real* dj = rj;
  const Real* ej = rj + 3;
  const Real mx = di[0] - dj[0], my = di[1] - dj[1], mz = di[2] - dj[2];   // delta(++)
  const Real px = di[0] + dj[0], py = di[1] + dj[1], pz = di[2] + dj[2];   // delta(+-)
  const Real Rm = Rx * mx + Ry * my + Rz * mz, mm = mx * mx + my * my + mz * mz;
  const Real Rp = Rx * px + Ry * py + Rz * pz, pp = px * px + py * py + pz * pz;
  // (s_a, s_b) = (+,+), (-,-), (+,-), (-,+)
  const Real Rd[4] = {Rm, -Rm, Rp, -Rp};
  const Real dd[4] = {mm, mm, pp, pp};
  constexpr Real z = -Real(0);
  Real dur[4], ulj = z, uss = z;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const Real r2 = R2 + (Real(2) * Rd[k] + dd[k]);
    const Real rR = R2 + Rd[k];                                   // r . R
    const Real ir2 = rcp_(r2);
    const Real ir6 = ir2 * ir2 * ir2;
    const Real t6 = M.c6 * ir6;
    const Real t12 = M.c12 * ir6 * ir6;
    dur[k] = (Real(6) * t6 - Real(12) * t12) * ir2;               // u'/r
    // (u'' - u'/r) (r.R)^2 / r^2 = (168 t12 - 48 t6) (r.R / r^2)^2;
    // the (u'/r) R^2 part of every site pair is added once below
    const Real p = rR * ir2;
    ulj += t12 - t6;
    uss += (Real(168) * t12 - Real(48) * t6) * (p * p);
  }
  const Real Em = dur[0] - dur[1], Sm = dur[0] + dur[1];
  const Real Ep = dur[2] - dur[3], Sp = dur[2] + dur[3];
  uss += (Sm + Sp) * R2;

  const Real ir = rsq_(R2);
  const Real ca = (Rx * ei[0] + Ry * ei[1] + Rz * ei[2]) * ir;
  const Real cb = (Rx * ej[0] + Ry * ej[1] + Rz * ej[2]) * ir;
  const Real cab = ei[0] * ej[0] + ei[1] * ej[1] + ei[2] * ej[2];
  const Poly<Real> q = mp_poly<Real, 3, 3>(ca, cb, cab);
  const Real irr = ir * ir;
  const Real Kp = M.K * (irr * irr * ir);                         // K |R|^-5
  const Real uq = Kp * q.P;
  const Real A = Kp * ir;
  const Real sdot = Real(5) * q.P + q.Pa * ca + q.Pb * cb;
  acc.ulj = ulj;
  acc.uel = uq;
  acc.uss = uss + Real(30) * uq;
  // F_i = cR R + cd_i d_i + cd_j d_j - A P_a e_i - A P_b e_j
  const Real cR = A * sdot * ir - (Sm + Sp);
  const Real cdi = -(Em + Ep), cdj = Em - Ep;
  const Real cei = -A * q.Pa, cej = -A * q.Pb;
  F[0] = cR * Rx + cdi * di[0] + cdj * dj[0] + cei * ei[0] + cej * ej[0];
  F[1] = cR * Ry + cdi * di[1] + cdj * dj[1] + cei * ei[1] + cej * ej[1];
  F[2] = cR * Rz + cdi * di[2] + cdj * dj[2] + cei * ei[2] + cej * ej[2];
  acc.fx = F[0];
  acc.fy = F[1];
  acc.fz = F[2];
  // tau_i = d_i x V + e_i x W, V = -(E_m + E_p) R + (S_m - S_p) d_j,
  // W = -K |R|^-5 (P_a R / |R| + P_c e_j)
  const Real vs = Sm - Sp;
  const Real Vx = cdi * Rx + vs * dj[0], Vy = cdi * Ry + vs * dj[1], Vz = cdi * Rz + vs * dj[2];
  const Real wa = -Kp * q.Pa * ir, wc = -Kp * q.Pc;
  const Real Wx = wa * Rx + wc * ej[0], Wy = wa * Ry + wc * ej[1], Wz = wa * Rz + wc * ej[2];
  T[0] = (di[1] * Vz - di[2] * Vy) + (ei[1] * Wz - ei[2] * Wy);
  T[1] = (di[2] * Vx - di[0] * Vz) + (ei[2] * Wx - ei[0] * Wz);
  T[2] = (di[0] * Vy - di[1] * Vx) + (ei[0] * Wy - ei[1] * Wx);
}

// Force and torque of one molecule from its per-site accumulators:
// F = sum f, tau = sum d x f + e x g (d, e from the molecule's record, read
// with stride STRIDE).  Accumulates into F and T, of type Out.
template <typename Real, int C, int STRIDE, typename Out = double>
__device__ __forceinline__ void fold_sites(const Real* rec, const SiteAcc<Real, C>& a, Out* F, Out* T) {
  constexpr ClassShape S = kClassShapes[C];
  constexpr int OFF_CH = 3 * S.lj, OFF_DP = OFF_CH + 3 * S.ch, OFF_QD = OFF_DP + 6 * S.dp;
  auto R = [&](int k) { return (Out)rec[k * STRIDE]; };
  auto fold = [&](int off, const Real* f) {
    const Out fx = f[0], fy = f[1], fz = f[2];
    F[0] += fx; F[1] += fy; F[2] += fz;
    T[0] += R(off + 1) * fz - R(off + 2) * fy;
    T[1] += R(off + 2) * fx - R(off) * fz;
    T[2] += R(off) * fy - R(off + 1) * fx;
  };
  auto fold_g = [&](int off, const Real* g) {
    T[0] += R(off + 1) * (Out)g[2] - R(off + 2) * (Out)g[1];
    T[1] += R(off + 2) * (Out)g[0] - R(off) * (Out)g[2];
    T[2] += R(off) * (Out)g[1] - R(off + 1) * (Out)g[0];
  };
#pragma unroll
  for (int k = 0; k < S.lj; ++k) fold(3 * k, a.fl[k]);
#pragma unroll
  for (int k = 0; k < S.ch; ++k) fold(OFF_CH + 3 * k, a.fc[k]);
  // dipoles and quadrupoles of a central class sit at the centre: their
  // forces exert no torque about it
  auto fold_mp = [&](int off, const Real* f) {
    if constexpr (S.central) {
      F[0] += (Out)f[0]; F[1] += (Out)f[1]; F[2] += (Out)f[2];
    } else {
      fold(off, f);
    }
  };
#pragma unroll
  for (int k = 0; k < S.dp; ++k) { fold_mp(OFF_DP + 6 * k, a.fd[k]); fold_g(OFF_DP + 6 * k + 3, a.gd[k]); }
#pragma unroll
  for (int k = 0; k < S.qd; ++k) { fold_mp(OFF_QD + 6 * k, a.fq[k]); fold_g(OFF_QD + 6 * k + 3, a.gq[k]); }
}

}  // namespace ms2
