// Residual Massieu-potential derivatives A^r_mn (Sec. 3, Eq. 1) from the
// moment sums the device samplers accumulate, and the properties that follow
// from them.  Host arithmetic on a handful of doubles.
//
// With phi(beta, V) = ln INT exp(-beta U(s; V)) ds (scaled centres s fixed),
// F^r/(N k T) = -phi/N.  Differentiating the canonical average,
// d<A>/d beta = -cov(A, U) and d<A>/dV = <dA/dV> - beta cov(A, dU/dV); the
// density operators are rho d/d rho = -V d/dV and
// rho^2 d^2/d rho^2 = 2V d/dV + V^2 d^2/dV^2.
#include <cmath>

#include "batch.h"

using namespace ms2;

namespace {

// Canonical averages of the sampled observables (X = U - u0, Y = dU/dV,
// Z = d2U/dV2) and their central/joint cumulants.
struct Cumulants {
  double x, y, z;                // means
  double xx, xy, yy, xz;         // second order
  double xxx, xxy, xyy;          // third order
};

Cumulants cumulants(const double* s) {
  const double inv = 1.0 / s[0];
  const double x = s[1] * inv, x2 = s[2] * inv, x3 = s[3] * inv;
  const double y = s[4] * inv, xy = s[5] * inv, x2y = s[6] * inv;
  const double y2 = s[7] * inv, xy2 = s[8] * inv;
  const double z = s[9] * inv, xz = s[10] * inv;
  Cumulants c;
  c.x = x;
  c.y = y;
  c.z = z;
  c.xx = x2 - x * x;
  c.xy = xy - x * y;
  c.yy = y2 - y * y;
  c.xz = xz - x * z;
  // third-order joint cumulants: E[abc] - E[ab]E[c] - E[ac]E[b] - E[bc]E[a] + 2E[a]E[b]E[c]
  c.xxx = x3 - 3.0 * x2 * x + 2.0 * x * x * x;
  c.xxy = x2y - x2 * y - 2.0 * xy * x + 2.0 * x * x * y;
  c.xyy = xy2 - y2 * x - 2.0 * xy * y + 2.0 * x * y * y;
  return c;
}

}  // namespace

extern "C" ms2_status ms2_massieu(const double* h_moments, double u0, double temperature, double volume,
                                  int32_t n_mol, double* h_ar) {
  if (!h_moments || !h_ar) return set_error(MS2_EINVAL, "null pointer");
  if (!(h_moments[0] > 0.0)) return set_error(MS2_EINVAL, "no samples in the moment sums");
  if (!(temperature > 0.0) || !(volume > 0.0) || n_mol <= 0)
    return set_error(MS2_EINVAL, "temperature, volume and n_mol must be positive");
  const Cumulants c = cumulants(h_moments);
  const double b = 1.0 / temperature, V = volume, inv_n = 1.0 / (double)n_mol;
  const double u_mean = u0 + c.x;
  // derivatives of phi
  const double p_b = -u_mean, p_bb = c.xx, p_bbb = -c.xxx;
  const double p_v = -b * c.y;
  const double p_vv = b * b * c.yy - b * c.z;
  const double p_bv = b * c.xy - c.y;
  const double p_bbv = 2.0 * c.xy - b * c.xxy;
  const double p_bvv = b * c.xz - c.z + 2.0 * b * c.yy - b * b * c.xyy;
  // A^r = -phi/N under beta^m d^m/d beta^m and the density operators
  h_ar[MS2_AR_10] = -b * p_b * inv_n;
  h_ar[MS2_AR_20] = -b * b * p_bb * inv_n;
  h_ar[MS2_AR_30] = -b * b * b * p_bbb * inv_n;
  h_ar[MS2_AR_01] = V * p_v * inv_n;
  h_ar[MS2_AR_02] = -(2.0 * V * p_v + V * V * p_vv) * inv_n;
  h_ar[MS2_AR_11] = b * V * p_bv * inv_n;
  h_ar[MS2_AR_21] = b * b * V * p_bbv * inv_n;
  h_ar[MS2_AR_12] = -b * (2.0 * V * p_bv + V * V * p_bvv) * inv_n;
  return MS2_OK;
}

extern "C" ms2_status ms2_massieu_properties(const double* h_ar, double dof, double* h_props) {
  if (!h_ar || !h_props) return set_error(MS2_EINVAL, "null pointer");
  if (!(dof > 0.0)) return set_error(MS2_EINVAL, "dof must be positive");
  // total derivatives: ideal part of classical rigid molecules + residual
  const double a10 = 0.5 * dof + h_ar[MS2_AR_10];
  const double a20 = -0.5 * dof + h_ar[MS2_AR_20];
  const double a01 = 1.0 + h_ar[MS2_AR_01];
  const double a02 = -1.0 + h_ar[MS2_AR_02];
  const double a11 = h_ar[MS2_AR_11];
  const double dpdrho = 2.0 * a01 + a02;      // (dp/drho)_T / kT
  const double dpdt = a01 - a11;              // (dp/dT)_rho / (rho k)
  const double cv = -a20;
  const double cp = cv + dpdt * dpdt / dpdrho;
  h_props[MS2_PROP_Z] = a01;
  h_props[MS2_PROP_U_KT] = a10;
  h_props[MS2_PROP_CV] = cv;
  h_props[MS2_PROP_CP] = cp;
  h_props[MS2_PROP_DPDRHO] = dpdrho;
  h_props[MS2_PROP_DPDT] = dpdt;
  h_props[MS2_PROP_W2] = cp / cv * dpdrho;
  h_props[MS2_PROP_KAPPA_T] = 1.0 / dpdrho;
  return MS2_OK;
}
