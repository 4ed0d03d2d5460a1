/*
 * ms2_oracle.c -- plain, sequential FP64 reference for the rigid multi-site
 * MD hot path of ms2 2.0 (arXiv 1507.07548).  TEST INFRASTRUCTURE ONLY:
 * the product library never includes, links or calls it.
 *
 * Written for a reader checking it against the paper by eye: one i<j loop
 * over molecules (Sec. 2: partner search, energy and force are loops over
 * molecules), each accepted pair summed into both molecules (Newton's third
 * law; Sec. 2 notes every force is written to both partners), explicit k
 * loop over the whole sphere for Ewald (Sec. 4), textbook Gear integrator.
 * No blocking, fusion or reordering.
 *
 * Readings where the paper defers to the literature (listed with reasons
 * in the design notes of the repository):
 *  - LJ 12-6 with Lorentz-Berthelot combining; truncated, not shifted.
 *  - Molecule-centre cut-off: a molecule pair interacts iff the squared
 *    minimum-image distance of the centres is < rc^2; every site pair of
 *    an accepted pair uses the same image shift (Sec. 3 names both the
 *    site-site and the centre-of-mass cut-off modes).
 *  - Point dipoles / linear quadrupoles interact through the standard
 *    multipole expansion of the Coulomb energy.
 *  - Reaction field (Sec. 3): site RF for charge pairs
 *    k qa qb (1/r + kRF r^2 - cRF); Barker-Watts term for dipole pairs
 *    -2 kRF k mua mub (ea.eb); kRF = (eRF-1)/((2 eRF+1) rc^3),
 *    cRF = 1/rc + kRF rc^2; no RF term for other pairs.
 *  - Ewald (Sec. 4): Gaussian split, tin-foil boundary, real space under
 *    the molecule-centre cut-off, self and intramolecular constants.
 *  - Volume derivatives (Sec. 3): molecular scaling of the centres with
 *    rigid bodies, rc and alpha held fixed.  U_s = dU/ds, U_ss = d2U/ds2
 *    at s = 1, so dU/dV = U_s/(3V) and d2U/dV2 = (U_ss - 2 U_s)/(9 V^2).
 *  - LJ long-range correction, centre-of-mass mode, zeroth order: every LJ
 *    site pair treated as separated by the centre distance, g = 1 beyond rc.
 *
 * Build with -ffp-contract=off so that the cut-off expression is rounded
 * exactly as written.
 */
#include "ms2_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Rotation matrix (body -> lab) of the unit quaternion q = (w,x,y,z). */
static void quat_matrix(const double* q, double A[3][3]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
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

static void mat_vec(double A[3][3], const double* b, double* out) {
  for (int k = 0; k < 3; ++k) out[k] = A[k][0] * b[0] + A[k][1] * b[1] + A[k][2] * b[2];
}

/* Lab-frame site offsets d_a = A b_a and axes e_a = A ehat_a of one molecule. */
typedef struct {
  double d[OR_MAXS][3];
  double e[OR_MAXS][3];
} lab_t;

static void lab_sites(const or_species* s, const double* q, lab_t* out) {
  double A[3][3];
  quat_matrix(q, A);
  for (int a = 0; a < s->n_sites; ++a) {
    mat_vec(A, s->pos[a], out->d[a]);
    mat_vec(A, s->axis[a], out->e[a]);
  }
}

static int is_elec(int t) { return t == OR_CHARGE || t == OR_DIPOLE || t == OR_QUAD; }

/* ------------------------------------------------------------------ */
/* argument checks                                                     */
/* ------------------------------------------------------------------ */
/* largest distance of an LJ site from its molecule's centre */
static double lj_dmax(const or_species* sp, int nsp) {
  double d = 0.0;
  for (int s = 0; s < nsp; ++s)
    for (int a = 0; a < sp[s].n_sites; ++a)
      if (sp[s].type[a] == OR_LJ) {
        double r = sqrt(sp[s].pos[a][0] * sp[s].pos[a][0] + sp[s].pos[a][1] * sp[s].pos[a][1] +
                        sp[s].pos[a][2] * sp[s].pos[a][2]);
        if (r > d) d = r;
      }
  return d;
}

int or_check(const or_species* sp, int32_t nsp, const or_params* p) {
  if (!sp || !p || nsp <= 0) return -1;
  if (!(p->box > 0.0) || !(p->rc > 0.0) || !(2.0 * p->rc < p->box)) return -2;
  if (p->elec < OR_ELEC_NONE || p->elec > OR_ELEC_EWALD) return -3;
  if (p->elec == OR_ELEC_RF && !(p->eps_rf >= 1.0)) return -4;
  if (p->elec == OR_ELEC_EWALD && (!(p->alpha > 0.0) || p->kmax2 < 1)) return -5;
  if (p->cutoff_mode != OR_CUT_COM && p->cutoff_mode != OR_CUT_SITE) return -9;
  if (p->cutoff_mode == OR_CUT_SITE && !(2.0 * (p->rc + 2.0 * lj_dmax(sp, nsp)) < p->box)) return -2;
  for (int s = 0; s < nsp; ++s) {
    if (sp[s].n_sites < 1 || sp[s].n_sites > OR_MAXS) return -6;
    for (int a = 0; a < sp[s].n_sites; ++a) {
      int t = sp[s].type[a];
      if (t < OR_LJ || t > OR_QUAD) return -7;
      if (p->elec == OR_ELEC_EWALD && (t == OR_DIPOLE || t == OR_QUAD)) return -8;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* site-pair physics                                                   */
/* ------------------------------------------------------------------ */
typedef struct {
  double u_lj, u_el;      /* energies                                */
  double us, uss;         /* dU/ds, d2U/ds2 under molecular scaling   */
  double f[3];            /* force on molecule i from j               */
  double ti[3], tj[3];    /* torques on i and on j                    */
  double nsite;           /* interacting site pairs                   */
} pair_acc;

typedef struct {
  double k_rf, c_rf;      /* reaction-field constants                 */
} rf_t;

/* Central potential u(r) with first and second radial derivatives.
 * rv = r_a - r_b (site b on j to site a on i), R = centre difference. */
static void add_central(double u, double du, double d2u, const double* rv, double r,
                        const double* R, const double* da, const double* db,
                        int is_lj, pair_acc* o) {
  double n[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
  double f[3] = {-du * n[0], -du * n[1], -du * n[2]};  /* force on site a */
  double nR = dot3(n, R);
  double RR = dot3(R, R);
  if (is_lj) o->u_lj += u; else o->u_el += u;
  o->us += du * nR;
  o->uss += d2u * nR * nR + (du / r) * (RR - nR * nR);
  double c[3], mf[3] = {-f[0], -f[1], -f[2]};
  for (int k = 0; k < 3; ++k) o->f[k] += f[k];
  cross3(da, f, c);
  for (int k = 0; k < 3; ++k) o->ti[k] += c[k];
  cross3(db, mf, c);
  for (int k = 0; k < 3; ++k) o->tj[k] += c[k];
}

/* Orientation-dependent term u = K F(ca, cb, cab) / r^p with
 * ca = ea.n, cb = eb.n, cab = ea.eb and n = rv/r.  The caller supplies F
 * and its partial derivatives Fa, Fb, Fc (w.r.t. cab), Faa, Fbb, Fab. */
typedef struct {
  double F, Fa, Fb, Fc, Faa, Fbb, Fab;
} angf_t;

static void add_angular(double K, int p, const angf_t* g, const double* rv, double r,
                        const double* ea, const double* eb, const double* R,
                        const double* da, const double* db, pair_acc* o) {
  double n[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
  double ca = dot3(ea, n), cb = dot3(eb, n);
  double rp = pow(r, -p);
  double u = K * g->F * rp;
  o->u_el += u;
  /* gradient of u with respect to rv:
   *   d ca / d rv = (ea - ca n)/r,  d r^-p / d rv = -p r^-p-1 n          */
  double grad[3];
  for (int k = 0; k < 3; ++k)
    grad[k] = K * rp * (g->Fa * (ea[k] - ca * n[k]) / r + g->Fb * (eb[k] - cb * n[k]) / r) -
              p * K * g->F * rp / r * n[k];
  double f[3] = {-grad[0], -grad[1], -grad[2]};
  /* g_a = -du/d ea, g_b = -du/d eb with rv held fixed */
  double ga[3], gb[3];
  for (int k = 0; k < 3; ++k) {
    ga[k] = -K * rp * (g->Fa * n[k] + g->Fc * eb[k]);
    gb[k] = -K * rp * (g->Fb * n[k] + g->Fc * ea[k]);
  }
  /* first and second derivatives of u(rv + t R) at t = 0 */
  double beta = dot3(n, R), RR = dot3(R, R);
  double aa = dot3(ea, R), ab = dot3(eb, R);
  double ca1 = (aa - ca * beta) / r, cb1 = (ab - cb * beta) / r;
  double ca2 = (-2.0 * ca1 * beta * r - ca * (RR - beta * beta)) / (r * r);
  double cb2 = (-2.0 * cb1 * beta * r - cb * (RR - beta * beta)) / (r * r);
  double f0 = rp;
  double f1 = -p * rp / r * beta;
  double f2 = rp / (r * r) * (p * (p + 1.0) * beta * beta - p * (RR - beta * beta));
  double F1 = g->Fa * ca1 + g->Fb * cb1;
  double F2 = g->Faa * ca1 * ca1 + 2.0 * g->Fab * ca1 * cb1 + g->Fbb * cb1 * cb1 +
              g->Fa * ca2 + g->Fb * cb2;
  o->us += K * (F1 * f0 + g->F * f1);
  o->uss += K * (F2 * f0 + 2.0 * F1 * f1 + g->F * f2);
  double c[3], mf[3] = {-f[0], -f[1], -f[2]};
  for (int k = 0; k < 3; ++k) o->f[k] += f[k];
  cross3(da, f, c);
  for (int k = 0; k < 3; ++k) o->ti[k] += c[k];
  cross3(ea, ga, c);
  for (int k = 0; k < 3; ++k) o->ti[k] += c[k];
  cross3(db, mf, c);
  for (int k = 0; k < 3; ++k) o->tj[k] += c[k];
  cross3(eb, gb, c);
  for (int k = 0; k < 3; ++k) o->tj[k] += c[k];
}

/* Multipole expansion of the Coulomb energy between two point sites of
 * type ta (on i) and tb (on j); n points from b to a. */
static void multipole_terms(int ta, int tb, double ca, double cb, double cab,
                            int* p, angf_t* g) {
  memset(g, 0, sizeof(*g));
  if (ta == OR_CHARGE && tb == OR_CHARGE) {          /* q q / r           */
    *p = 1; g->F = 1.0;
  } else if (ta == OR_CHARGE && tb == OR_DIPOLE) {   /* q mu cb / r^2     */
    *p = 2; g->F = cb; g->Fb = 1.0;
  } else if (ta == OR_DIPOLE && tb == OR_CHARGE) {   /* -q mu ca / r^2    */
    *p = 2; g->F = -ca; g->Fa = -1.0;
  } else if (ta == OR_CHARGE && tb == OR_QUAD) {     /* q Q P2(cb) / r^3  */
    *p = 3; g->F = 0.5 * (3.0 * cb * cb - 1.0); g->Fb = 3.0 * cb; g->Fbb = 3.0;
  } else if (ta == OR_QUAD && tb == OR_CHARGE) {
    *p = 3; g->F = 0.5 * (3.0 * ca * ca - 1.0); g->Fa = 3.0 * ca; g->Faa = 3.0;
  } else if (ta == OR_DIPOLE && tb == OR_DIPOLE) {   /* (cab - 3 ca cb)/r^3 */
    *p = 3; g->F = cab - 3.0 * ca * cb; g->Fa = -3.0 * cb; g->Fb = -3.0 * ca;
    g->Fc = 1.0; g->Fab = -3.0;
  } else if (ta == OR_DIPOLE && tb == OR_QUAD) {
    /* mu_a . grad phi_Q(r_a): (3/2)[ca (1 - 5 cb^2) + 2 cb cab] / r^4 */
    *p = 4;
    g->F = 1.5 * (ca * (1.0 - 5.0 * cb * cb) + 2.0 * cb * cab);
    g->Fa = 1.5 * (1.0 - 5.0 * cb * cb);
    g->Fb = 1.5 * (-10.0 * ca * cb + 2.0 * cab);
    g->Fc = 3.0 * cb;
    g->Fbb = -15.0 * ca;
    g->Fab = -15.0 * cb;
  } else if (ta == OR_QUAD && tb == OR_DIPOLE) {
    /* the same with the roles of a and b exchanged and n reversed */
    *p = 4;
    g->F = -1.5 * (cb * (1.0 - 5.0 * ca * ca) + 2.0 * ca * cab);
    g->Fb = -1.5 * (1.0 - 5.0 * ca * ca);
    g->Fa = -1.5 * (-10.0 * ca * cb + 2.0 * cab);
    g->Fc = -3.0 * ca;
    g->Faa = 15.0 * cb;
    g->Fab = 15.0 * ca;
  } else { /* QUAD-QUAD: (3/4)[1 - 5ca^2 - 5cb^2 - 15 ca^2 cb^2 + 2 (cab - 5 ca cb)^2] / r^5 */
    *p = 5;
    double t = cab - 5.0 * ca * cb;
    g->F = 0.75 * (1.0 - 5.0 * ca * ca - 5.0 * cb * cb - 15.0 * ca * ca * cb * cb + 2.0 * t * t);
    g->Fa = 0.75 * (-10.0 * ca + 70.0 * ca * cb * cb - 20.0 * cb * cab);
    g->Fb = 0.75 * (-10.0 * cb + 70.0 * ca * ca * cb - 20.0 * ca * cab);
    g->Fc = 3.0 * cab - 15.0 * ca * cb;
    g->Faa = 0.75 * (-10.0 + 70.0 * cb * cb);
    g->Fbb = 0.75 * (-10.0 + 70.0 * ca * ca);
    g->Fab = 0.75 * (140.0 * ca * cb - 20.0 * cab);
  }
}

/* One site pair (a on molecule i, b on molecule j) of an accepted pair. */
/* One site pair of an accepted molecule pair.  elec_in: the molecule
 * centres are inside the cut-off (electrostatic site pairs interact only
 * then); in the site-site mode an LJ site pair interacts only when its own
 * distance is inside the cut-off. */
static void site_pair(const or_species* si, int a, const or_species* sj, int b,
                      const lab_t* li, const lab_t* lj, const double* R,
                      const or_params* p, const rf_t* rf, int elec_in, pair_acc* o) {
  int ta = si->type[a], tb = sj->type[b];
  const double* da = li->d[a];
  const double* db = lj->d[b];
  double rv[3];
  for (int k = 0; k < 3; ++k) rv[k] = R[k] + da[k] - db[k];
  double r2s = rv[0] * rv[0];
  r2s = r2s + rv[1] * rv[1];
  r2s = r2s + rv[2] * rv[2];
  if (ta == OR_LJ && tb == OR_LJ && p->cutoff_mode == OR_CUT_SITE && !(r2s < p->rc * p->rc)) return;
  if (is_elec(ta) && is_elec(tb) && !elec_in) return;
  double r = sqrt(dot3(rv, rv));

  if (ta == OR_LJ && tb == OR_LJ) {
    double sig = 0.5 * (si->sigma[a] + sj->sigma[b]);
    double eps = sqrt(si->eps[a] * sj->eps[b]);
    double s6 = pow(sig / r, 6.0), s12 = s6 * s6;
    double u = 4.0 * eps * (s12 - s6);
    double du = 4.0 * eps * (-12.0 * s12 + 6.0 * s6) / r;
    double d2u = 4.0 * eps * (156.0 * s12 - 42.0 * s6) / (r * r);
    add_central(u, du, d2u, rv, r, R, da, db, 1, o);
    o->nsite += 1.0;
    return;
  }
  if (!is_elec(ta) || !is_elec(tb)) return; /* LJ and electrostatic sites do not interact */

  double K = p->coulomb_k * si->mag[a] * sj->mag[b];
  o->nsite += 1.0;
  if (p->elec == OR_ELEC_EWALD) { /* charges only: k qa qb erfc(alpha r)/r */
    double al = p->alpha;
    double ec = erfc(al * r), gs = 2.0 * al / sqrt(OR_PI) * exp(-al * al * r * r);
    double u = K * ec / r;
    double du = -K * (ec / (r * r) + gs / r);
    double d2u = K * (2.0 * ec / (r * r * r) + gs * (2.0 / (r * r) + 2.0 * al * al));
    add_central(u, du, d2u, rv, r, R, da, db, 0, o);
    return;
  }
  if (p->elec == OR_ELEC_RF && ta == OR_CHARGE && tb == OR_CHARGE) {
    double u = K * (1.0 / r + rf->k_rf * r * r - rf->c_rf);
    double du = K * (-1.0 / (r * r) + 2.0 * rf->k_rf * r);
    double d2u = K * (2.0 / (r * r * r) + 2.0 * rf->k_rf);
    add_central(u, du, d2u, rv, r, R, da, db, 0, o);
    return;
  }
  const double* ea = li->e[a];
  const double* eb = lj->e[b];
  double n[3] = {rv[0] / r, rv[1] / r, rv[2] / r};
  int pw;
  angf_t g;
  multipole_terms(ta, tb, dot3(ea, n), dot3(eb, n), dot3(ea, eb), &pw, &g);
  add_angular(K, pw, &g, rv, r, ea, eb, R, da, db, o);
  if (p->elec == OR_ELEC_RF && ta == OR_DIPOLE && tb == OR_DIPOLE) {
    angf_t h;
    memset(&h, 0, sizeof(h));
    h.F = -2.0 * rf->k_rf * dot3(ea, eb);
    h.Fc = -2.0 * rf->k_rf;
    add_angular(K, 0, &h, rv, r, ea, eb, R, da, db, o);
  }
}

/* ------------------------------------------------------------------ */
/* LJ long-range correction, centre-of-mass cut-off, zeroth order       */
/* ------------------------------------------------------------------ */
/* Integrals over rc..inf of r^2 u, r^3 u' and r^4 u'' for the 12-6
 * potential, times 2 pi N_A N_B / V, summed over LJ site pairs. */
static void lj_tail(const or_species* sp, int nsp, const long* count, const or_params* p,
                    double* u_lrc, double* us_lrc, double* uss_lrc) {
  double V = p->box * p->box * p->box;
  *u_lrc = *us_lrc = *uss_lrc = 0.0;
  for (int A = 0; A < nsp; ++A)
    for (int B = 0; B < nsp; ++B) {
      double pre = 2.0 * OR_PI * (double)count[A] * (double)count[B] / V;
      for (int a = 0; a < sp[A].n_sites; ++a)
        for (int b = 0; b < sp[B].n_sites; ++b) {
          if (sp[A].type[a] != OR_LJ || sp[B].type[b] != OR_LJ) continue;
          double sig = 0.5 * (sp[A].sigma[a] + sp[B].sigma[b]);
          double eps = sqrt(sp[A].eps[a] * sp[B].eps[b]);
          double x = sig / p->rc, x3 = x * x * x, x9 = x3 * x3 * x3;
          double c = 4.0 * eps * sig * sig * sig * pre;
          *u_lrc += c * (x9 / 9.0 - x3 / 3.0);
          *us_lrc += c * (-4.0 / 3.0 * x9 + 2.0 * x3);
          *uss_lrc += c * (52.0 / 3.0 * x9 - 14.0 * x3);
        }
    }
}

/* ------------------------------------------------------------------ */
/* explicit pair sum: partner search + energy + forces (Sec. 2, Sec. 3) */
/* ------------------------------------------------------------------ */
int or_forces(const or_species* sp, int32_t nsp, const or_params* p, int32_t n,
              const int32_t* species, const double* com, const double* quat,
              double* force, double* torque, double* sums) {
  int rc_ok = or_check(sp, nsp, p);
  if (rc_ok) return rc_ok;
  if (n < 1 || !species || !com || !quat || !force || !torque || !sums) return -10;
  for (int i = 0; i < n; ++i)
    if (species[i] < 0 || species[i] >= nsp) return -11;

  double L = p->box, rc2 = p->rc * p->rc;
  int site_mode = p->cutoff_mode == OR_CUT_SITE;
  double rs = p->rc + 2.0 * lj_dmax(sp, nsp), rs2 = rs * rs;
  rf_t rf = {0.0, 0.0};
  if (p->elec == OR_ELEC_RF) {
    rf.k_rf = isinf(p->eps_rf) ? 1.0 / (2.0 * p->rc * p->rc * p->rc)
                               : (p->eps_rf - 1.0) / ((2.0 * p->eps_rf + 1.0) * p->rc * p->rc * p->rc);
    rf.c_rf = 1.0 / p->rc + rf.k_rf * p->rc * p->rc;
  }

  lab_t* lab = (lab_t*)malloc(sizeof(lab_t) * (size_t)n);
  if (!lab) return -12;
  for (int i = 0; i < n; ++i) lab_sites(&sp[species[i]], quat + 4 * i, &lab[i]);

  memset(force, 0, sizeof(double) * 3 * (size_t)n);
  memset(torque, 0, sizeof(double) * 3 * (size_t)n);
  for (int k = 0; k < OR_NSUM; ++k) sums[k] = 0.0;

  for (int i = 0; i < n; ++i) {
    for (int j = i + 1; j < n; ++j) {
      double R[3];
      for (int k = 0; k < 3; ++k) {
        double d = com[3 * i + k] - com[3 * j + k];
        R[k] = d - L * rint(d / L);           /* minimum image */
      }
      double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      int elec_in = r2 < rc2;                  /* molecule-centre cut-off */
      if (!site_mode && !elec_in) continue;
      if (site_mode && !(r2 < rs2)) continue;   /* no LJ site pair can reach */
      pair_acc o;
      memset(&o, 0, sizeof(o));
      const or_species* si = &sp[species[i]];
      const or_species* sj = &sp[species[j]];
      for (int a = 0; a < si->n_sites; ++a)
        for (int b = 0; b < sj->n_sites; ++b)
          site_pair(si, a, sj, b, &lab[i], &lab[j], R, p, &rf, elec_in, &o);
      if (site_mode && o.nsite == 0.0) continue;  /* no site pair interacts */
      for (int k = 0; k < 3; ++k) {
        force[3 * i + k] += o.f[k];
        force[3 * j + k] -= o.f[k];
        torque[3 * i + k] += o.ti[k];
        torque[3 * j + k] += o.tj[k];
      }
      sums[OR_U_LJ] += o.u_lj;
      sums[OR_U_ELEC] += o.u_el;
      sums[OR_VIRIAL] += dot3(R, o.f);
      sums[OR_US] += o.us;
      sums[OR_USS] += o.uss;
      sums[OR_NPAIR] += 1.0;
      sums[OR_NSITE] += o.nsite;
    }
  }

  /* Ewald constants: self energy and intramolecular erf exclusion */
  if (p->elec == OR_ELEC_EWALD) {
    double al = p->alpha, uc = 0.0;
    for (int i = 0; i < n; ++i) {
      const or_species* s = &sp[species[i]];
      for (int a = 0; a < s->n_sites; ++a) {
        if (s->type[a] != OR_CHARGE) continue;
        uc -= p->coulomb_k * al / sqrt(OR_PI) * s->mag[a] * s->mag[a];
        for (int b = a + 1; b < s->n_sites; ++b) {
          if (s->type[b] != OR_CHARGE) continue;
          double dv[3];
          for (int k = 0; k < 3; ++k) dv[k] = s->pos[a][k] - s->pos[b][k];
          double r = sqrt(dot3(dv, dv));
          uc -= p->coulomb_k * s->mag[a] * s->mag[b] * erf(al * r) / r;
        }
      }
    }
    sums[OR_U_CONST] = uc;
  }

  if (p->lj_lrc) {
    long* count = (long*)calloc((size_t)nsp, sizeof(long));
    if (!count) { free(lab); return -12; }
    for (int i = 0; i < n; ++i) count[species[i]]++;
    lj_tail(sp, nsp, count, p, &sums[OR_U_LRC], &sums[OR_US_LRC], &sums[OR_USS_LRC]);
    free(count);
  }
  free(lab);
  return 0;
}

/* ------------------------------------------------------------------ */
/* heat flux (Sec. 5, Eq. 6); the energy moment sum_k R_k e_k with       */
/* e_k = kinetic energy + half of k's pair energies changes at this rate */
/* ------------------------------------------------------------------ */
int or_heat_flux(const or_species* sp, int32_t nsp, const or_params* p, int32_t n,
                 const int32_t* species, const double* com, const double* quat,
                 const double* vel, const double* omega, const double* h_partial, double* jq) {
  int rc_ok = or_check(sp, nsp, p);
  if (rc_ok) return rc_ok;
  if (p->elec == OR_ELEC_EWALD) return -40;
  if (n < 1 || !species || !com || !quat || !vel || !omega || !jq) return -10;
  double L = p->box, rc2 = p->rc * p->rc;
  rf_t rf = {0.0, 0.0};
  if (p->elec == OR_ELEC_RF) {
    rf.k_rf = isinf(p->eps_rf) ? 1.0 / (2.0 * p->rc * p->rc * p->rc)
                               : (p->eps_rf - 1.0) / ((2.0 * p->eps_rf + 1.0) * p->rc * p->rc * p->rc);
    rf.c_rf = 1.0 / p->rc + rf.k_rf * p->rc * p->rc;
  }
  lab_t* lab = (lab_t*)malloc(sizeof(lab_t) * (size_t)n);
  double* wlab = (double*)malloc(sizeof(double) * 3 * (size_t)n);
  if (!lab || !wlab) { free(lab); free(wlab); return -12; }
  for (int k = 0; k < 3; ++k) jq[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    const or_species* s = &sp[species[i]];
    lab_sites(s, quat + 4 * i, &lab[i]);
    double A[3][3];
    quat_matrix(quat + 4 * i, A);
    mat_vec(A, omega + 3 * i, wlab + 3 * i);
    double e = 0.5 * s->mass * dot3(vel + 3 * i, vel + 3 * i);
    for (int k = 0; k < 3; ++k) e += 0.5 * s->inertia[k] * omega[3 * i + k] * omega[3 * i + k];
    if (h_partial) e -= h_partial[species[i]];
    for (int k = 0; k < 3; ++k) jq[k] += e * vel[3 * i + k];
  }
  for (int i = 0; i < n; ++i) {
    for (int j = i + 1; j < n; ++j) {
      double R[3];
      for (int k = 0; k < 3; ++k) {
        double d = com[3 * i + k] - com[3 * j + k];
        R[k] = d - L * rint(d / L);
      }
      double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      int elec_in = r2 < rc2;
      if (p->cutoff_mode == OR_CUT_COM && !elec_in) continue;
      pair_acc o;
      memset(&o, 0, sizeof(o));
      const or_species* si = &sp[species[i]];
      const or_species* sj = &sp[species[j]];
      for (int a = 0; a < si->n_sites; ++a)
        for (int b = 0; b < sj->n_sites; ++b)
          site_pair(si, a, sj, b, &lab[i], &lab[j], R, p, &rf, elec_in, &o);
      double u = o.u_lj + o.u_el, vs[3];
      for (int k = 0; k < 3; ++k) vs[k] = vel[3 * i + k] + vel[3 * j + k];
      double power = dot3(o.f, vs) + dot3(o.ti, wlab + 3 * i) - dot3(o.tj, wlab + 3 * j);
      for (int k = 0; k < 3; ++k) jq[k] += 0.5 * u * vs[k] + 0.5 * R[k] * power;
    }
  }
  free(lab);
  free(wlab);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Ewald reciprocal space, explicit loop over the full k sphere (Sec. 4) */
/* ------------------------------------------------------------------ */
int or_kspace(const or_species* sp, int32_t nsp, const or_params* p, int32_t n,
              const int32_t* species, const double* com, const double* quat,
              double* force, double* torque, double* sums) {
  int rc_ok = or_check(sp, nsp, p);
  if (rc_ok) return rc_ok;
  if (p->elec != OR_ELEC_EWALD) return -20;
  if (n < 1 || !species || !com || !quat || !force || !torque || !sums) return -10;
  for (int i = 0; i < n; ++i)
    if (species[i] < 0 || species[i] >= nsp) return -11;

  /* gather the charges: absolute position, lab offset, charge, molecule */
  int nq = 0;
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < sp[species[i]].n_sites; ++a)
      if (sp[species[i]].type[a] == OR_CHARGE) nq++;
  double* pos = (double*)malloc(sizeof(double) * 3 * (size_t)(nq ? nq : 1));
  double* off = (double*)malloc(sizeof(double) * 3 * (size_t)(nq ? nq : 1));
  double* q = (double*)malloc(sizeof(double) * (size_t)(nq ? nq : 1));
  int* mol = (int*)malloc(sizeof(int) * (size_t)(nq ? nq : 1));
  double* fq = (double*)calloc((size_t)(nq ? nq : 1) * 3, sizeof(double));
  if (!pos || !off || !q || !mol || !fq) return -12;
  int c = 0;
  for (int i = 0; i < n; ++i) {
    lab_t lb;
    const or_species* s = &sp[species[i]];
    lab_sites(s, quat + 4 * i, &lb);
    for (int a = 0; a < s->n_sites; ++a) {
      if (s->type[a] != OR_CHARGE) continue;
      for (int k = 0; k < 3; ++k) {
        off[3 * c + k] = lb.d[a][k];
        pos[3 * c + k] = com[3 * i + k] + lb.d[a][k];
      }
      q[c] = s->mag[a];
      mol[c] = i;
      c++;
    }
  }

  double L = p->box, V = L * L * L, al = p->alpha;
  int nmax = (int)floor(sqrt((double)p->kmax2));
  double u_rec = 0.0, w_atomic = 0.0;
  for (int nx = -nmax; nx <= nmax; ++nx)
    for (int ny = -nmax; ny <= nmax; ++ny)
      for (int nz = -nmax; nz <= nmax; ++nz) {
        int n2 = nx * nx + ny * ny + nz * nz;
        if (n2 == 0 || n2 > p->kmax2) continue;
        double kv[3] = {2.0 * OR_PI * nx / L, 2.0 * OR_PI * ny / L, 2.0 * OR_PI * nz / L};
        double k2 = dot3(kv, kv);
        double gk = exp(-k2 / (4.0 * al * al)) / k2;
        double sre = 0.0, sim = 0.0;           /* S(k) = sum q e^{i k.r} */
        for (int a = 0; a < nq; ++a) {
          double th = dot3(kv, pos + 3 * a);
          sre += q[a] * cos(th);
          sim += q[a] * sin(th);
        }
        double s2 = sre * sre + sim * sim;
        u_rec += gk * s2;
        w_atomic += gk * s2 * (1.0 - k2 / (2.0 * al * al));
        /* F_a = k 4 pi q_a / V  g(k) k Im(e^{i k.r_a} S(k)*) */
        for (int a = 0; a < nq; ++a) {
          double th = dot3(kv, pos + 3 * a);
          double im = sin(th) * sre - cos(th) * sim;
          double pre = p->coulomb_k * 4.0 * OR_PI / V * q[a] * gk * im;
          for (int k = 0; k < 3; ++k) fq[3 * a + k] += pre * kv[k];
        }
      }
  u_rec *= p->coulomb_k * 2.0 * OR_PI / V;
  w_atomic *= p->coulomb_k * 2.0 * OR_PI / V;

  double dF = 0.0; /* sum_a d_a . F_a (molecular-virial correction) */
  for (int a = 0; a < nq; ++a) {
    int i = mol[a];
    double t[3];
    cross3(off + 3 * a, fq + 3 * a, t);
    for (int k = 0; k < 3; ++k) {
      force[3 * i + k] += fq[3 * a + k];
      torque[3 * i + k] += t[k];
    }
    dF += dot3(off + 3 * a, fq + 3 * a);
  }
  double w_mol = w_atomic - dF;
  sums[OR_U_RECIP] += u_rec;
  sums[OR_VIRIAL] += w_mol;
  sums[OR_US] -= w_mol;
  free(pos); free(off); free(q); free(mol); free(fq);
  return 0;
}

/* ------------------------------------------------------------------ */
/* molecular dynamics: integrators, thermostat and sampling             */
/* ------------------------------------------------------------------ */
int or_rdf_ntypes(const or_species* sp, int32_t nsp) {
  int t = 0;
  for (int s = 0; s < nsp; ++s)
    for (int a = 0; a < sp[s].n_sites; ++a)
      if (sp[s].type[a] == OR_LJ) t++;
  return t;
}


/* LJ site type of (species s, site a) in the order species-major, site-minor;
 * -1 if the site is not an LJ site. */
static int lj_type(const or_species* sp, int s, int a) {
  if (sp[s].type[a] != OR_LJ) return -1;
  int t = 0;
  for (int u = 0; u < s; ++u)
    for (int b = 0; b < sp[u].n_sites; ++b)
      if (sp[u].type[b] == OR_LJ) t++;
  for (int b = 0; b < a; ++b)
    if (sp[s].type[b] == OR_LJ) t++;
  return t;
}

/* index of the unordered type pair (t1 <= t2) among T types */
static int type_pair(int t1, int t2, int T) {
  if (t1 > t2) { int x = t1; t1 = t2; t2 = x; }
  return t1 * T - t1 * (t1 - 1) / 2 + (t2 - t1);
}

static double u_total(const double* s) {
  return s[OR_U_LJ] + s[OR_U_ELEC] + s[OR_U_RECIP] + s[OR_U_CONST] + s[OR_U_LRC];
}

static int evaluate(const or_species* sp, int nsp, const or_params* p, int n,
                    const int32_t* species, const double* com, const double* quat,
                    double* F, double* T, double* sums) {
  int e = or_forces(sp, nsp, p, n, species, com, quat, F, T, sums);
  if (e) return e;
  if (p->elec == OR_ELEC_EWALD) e = or_kspace(sp, nsp, p, n, species, com, quat, F, T, sums);
  return e;
}

/* quaternion product c = a (x) b, components (w,x,y,z) */
static void qmul(const double* a, const double* b, double* c) {
  c[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  c[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  c[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  c[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

/* dq/dt = 1/2 q (x) (0, omega_body) */
static void qdot(const double* q, const double* w, double* out) {
  double pw[4] = {0.0, w[0], w[1], w[2]}, t[4];
  qmul(q, pw, t);
  for (int k = 0; k < 4; ++k) out[k] = 0.5 * t[k];
}

/* Euler's equations in the principal body frame; a zero moment of inertia
 * (linear or point molecule) freezes that component. */
static void euler_rhs(const double* I, const double* tb, const double* w, double* wd) {
  wd[0] = I[0] > 0.0 ? (tb[0] + (I[1] - I[2]) * w[1] * w[2]) / I[0] : 0.0;
  wd[1] = I[1] > 0.0 ? (tb[1] + (I[2] - I[0]) * w[2] * w[0]) / I[1] : 0.0;
  wd[2] = I[2] > 0.0 ? (tb[2] + (I[0] - I[1]) * w[0] * w[1]) / I[2] : 0.0;
}

/* body-frame torque: A^T tau */
static void to_body(const double* q, const double* t, double* tb) {
  double A[3][3];
  quat_matrix(q, A);
  for (int k = 0; k < 3; ++k) tb[k] = A[0][k] * t[0] + A[1][k] * t[1] + A[2][k] * t[2];
}

/* Pascal-triangle prediction of a 5-value Gear vector of width m */
static void gear_predict(double* y[5], int m) {
  for (int c = 0; c < m; ++c) {
    double y0 = y[0][c], y1 = y[1][c], y2 = y[2][c], y3 = y[3][c], y4 = y[4][c];
    y[0][c] = y0 + y1 + y2 + y3 + y4;
    y[1][c] = y1 + 2.0 * y2 + 3.0 * y3 + 4.0 * y4;
    y[2][c] = y2 + 3.0 * y3 + 6.0 * y4;
    y[3][c] = y3 + 4.0 * y4;
    y[4][c] = y4;
  }
}

typedef struct {
  int n, nlag, every, origin_every, max_live, n_origins;
  int* t0;
  double* v0;  /* [max_live][n][3] */
  double* j0;  /* [max_live][3]    */
} acf_t;

static double mol_charge(const or_species* s) {
  double q = 0.0;
  for (int a = 0; a < s->n_sites; ++a)
    if (s->type[a] == OR_CHARGE) q += s->mag[a];
  return q;
}

/* One sample of the velocity and electric-current autocorrelation functions
 * at step s; the electric current is j_e = sum over ions of q_k v_k
 * (Sec. 5, Eq. 4), molecules without net charge do not contribute. */
static void acf_sample(acf_t* A, int s, const double* vel, const or_species* sp,
                       const int32_t* species, double* acf_v, double* acf_j, double* acf_cnt) {
  int n = A->n;
  double j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < n; ++i) {
    double q = mol_charge(&sp[species[i]]);
    for (int k = 0; k < 3; ++k) j[k] += q * vel[3 * i + k];
  }
  if (s % A->origin_every == 0) {
    int slot = A->n_origins % A->max_live;
    A->t0[slot] = s;
    memcpy(A->v0 + (size_t)slot * 3 * n, vel, sizeof(double) * 3 * (size_t)n);
    for (int k = 0; k < 3; ++k) A->j0[3 * slot + k] = j[k];
    A->n_origins++;
  }
  int live = A->n_origins < A->max_live ? A->n_origins : A->max_live;
  for (int o = 0; o < live; ++o) {
    int lag = (s - A->t0[o]) / A->every;
    if (s < A->t0[o] || lag >= A->nlag) continue;
    double cv = 0.0;
    for (int i = 0; i < 3 * n; ++i) cv += A->v0[(size_t)o * 3 * n + i] * vel[i];
    if (acf_v) acf_v[lag] += cv / n;
    if (acf_j) acf_j[lag] += dot3(A->j0 + 3 * o, j);
    if (acf_cnt) acf_cnt[lag] += 1.0;
  }
}

/* Residence time and solvation number (Sec. 5, Eqs. 7-8).  A solvent
 * molecule k belongs to the shell of solute i while their centres are closer
 * than the radius.  At every time origin (the ACF origins) the molecules in
 * each solute's shell are recorded; at a later sample, molecule k still
 * counts for that origin while it is in the shell, unless it has at some
 * point been outside for more than `tol` consecutive samples (the allowance
 * of Impey et al. for short excursions).  The correlation at a lag is the
 * counted fraction of the shell at the origin. */
typedef struct {
  int on, tol, nlag, every, origin_every, max_live, n_origins;
  int nu, nv;
  int* solute;         /* molecule indices of the central molecules      */
  int* solvent;        /* molecule indices of the counted molecules      */
  double r2;
  int* t0;             /* [max_live] origin steps                         */
  int* n0;             /* [max_live][nu] shell population at the origin   */
  int* away;           /* [max_live][nu][nv]: -1 = does not count for this
                          origin, else consecutive samples spent outside  */
} res_t;

static int in_shell(const res_t* R, const double* com, double L, int i, int k) {
  if (i == k) return 0;
  double d[3];
  for (int c = 0; c < 3; ++c) {
    d[c] = com[3 * i + c] - com[3 * k + c];
    d[c] = d[c] - L * rint(d[c] / L);
  }
  double r2 = d[0] * d[0];
  r2 = r2 + d[1] * d[1];
  r2 = r2 + d[2] * d[2];
  return r2 < R->r2;
}

static void residence_sample(res_t* R, int s, const double* com, double L, double* res_acf,
                             double* res_cnt, double* solvation) {
  int nu = R->nu, nv = R->nv;
  if (solvation) {
    for (int a = 0; a < nu; ++a)
      for (int b = 0; b < nv; ++b) solvation[0] += in_shell(R, com, L, R->solute[a], R->solvent[b]);
    solvation[1] += nu;
  }
  if (s % R->origin_every == 0) {
    int o = R->n_origins % R->max_live;
    R->t0[o] = s;
    for (int a = 0; a < nu; ++a) {
      int pop = 0;
      for (int b = 0; b < nv; ++b) {
        int in = in_shell(R, com, L, R->solute[a], R->solvent[b]);
        R->away[((size_t)o * nu + a) * nv + b] = in ? 0 : -1;
        pop += in;
      }
      R->n0[(size_t)o * nu + a] = pop;
    }
    R->n_origins++;
  }
  int live = R->n_origins < R->max_live ? R->n_origins : R->max_live;
  for (int o = 0; o < live; ++o) {
    if (s < R->t0[o]) continue;
    int lag = (s - R->t0[o]) / R->every;
    if (lag >= R->nlag) continue;
    for (int a = 0; a < nu; ++a) {
      int pop0 = R->n0[(size_t)o * nu + a];
      if (pop0 == 0) continue;
      int resident = 0;
      for (int b = 0; b < nv; ++b) {
        int* w = &R->away[((size_t)o * nu + a) * nv + b];
        int in = in_shell(R, com, L, R->solute[a], R->solvent[b]);
        if (lag > 0 && *w >= 0) {
          *w = in ? 0 : *w + 1;
          if (*w > R->tol) *w = -1;
        }
        if (*w >= 0 && in) resident++;
      }
      if (res_acf) res_acf[lag] += (double)resident / (double)pop0;
      if (res_cnt) res_cnt[lag] += 1.0;
    }
  }
}

/* Heat-flux autocorrelation (Sec. 5, Eq. 5) on the ACF schedule: the flux
 * is evaluated with each step's force evaluation (Gear: predicted state;
 * velocity Verlet: after the drift, with the half-step velocities); the
 * initial state has none, so an origin at step 0 carries no flux. */
typedef struct {
  int on, nlag, every, origin_every, max_live, n_origins;
  int* t0;
  int* valid;
  double* j0;   /* [max_live][3] */
} hf_t;

static void heat_acf_sample(hf_t* H, int s, const double* jq, int have, double* acf_q, double* acf_q_cnt) {
  if (s % H->origin_every == 0) {
    int o = H->n_origins % H->max_live;
    H->t0[o] = s;
    H->valid[o] = have;
    for (int k = 0; k < 3; ++k) H->j0[3 * o + k] = have ? jq[k] : 0.0;
    H->n_origins++;
  }
  if (!have) return;
  int live = H->n_origins < H->max_live ? H->n_origins : H->max_live;
  for (int o = 0; o < live; ++o) {
    if (!H->valid[o] || s < H->t0[o]) continue;
    int lag = (s - H->t0[o]) / H->every;
    if (lag >= H->nlag) continue;
    if (acf_q) acf_q[lag] += dot3(H->j0 + 3 * o, jq);
    if (acf_q_cnt) acf_q_cnt[lag] += 1.0;
  }
}

/* RDF histogram between all LJ sites (Sec. 5, Eq. 2): unordered site pairs of
 * distinct molecules, site distance from the minimum-image centre shift;
 * bin = (int)(r * bins / rmax). */
static void rdf_sample(const or_species* sp, int nsp, const or_params* p, const or_md_cfg* cfg,
                       int n, const int32_t* species, const double* com, const double* quat,
                       double* rdf) {
  int T = or_rdf_ntypes(sp, nsp);
  double L = p->box, inv_dr = (double)cfg->rdf_bins / cfg->rdf_rmax;
  lab_t li, lj;
  for (int i = 0; i < n; ++i) {
    lab_sites(&sp[species[i]], quat + 4 * i, &li);
    for (int j = i + 1; j < n; ++j) {
      lab_sites(&sp[species[j]], quat + 4 * j, &lj);
      double R[3];
      for (int k = 0; k < 3; ++k) {
        double d = com[3 * i + k] - com[3 * j + k];
        R[k] = d - L * rint(d / L);
      }
      const or_species* si = &sp[species[i]];
      const or_species* sj = &sp[species[j]];
      for (int a = 0; a < si->n_sites; ++a) {
        int ta = lj_type(sp, species[i], a);
        if (ta < 0) continue;
        for (int b = 0; b < sj->n_sites; ++b) {
          int tb = lj_type(sp, species[j], b);
          if (tb < 0) continue;
          double rv[3];
          for (int k = 0; k < 3; ++k) rv[k] = R[k] + li.d[a][k] - lj.d[b][k];
          double r = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
          if (!(r < cfg->rdf_rmax)) continue;
          int bin = (int)(r * inv_dr);
          if (bin >= cfg->rdf_bins) continue;
          rdf[(size_t)type_pair(ta, tb, T) * cfg->rdf_bins + bin] += 1.0;
        }
      }
    }
  }
}

static void moment_sample(const double* sums, double V, double u0, double* m) {
  double X = u_total(sums) - u0;
  double us = sums[OR_US] + sums[OR_US_LRC];
  double uss = sums[OR_USS] + sums[OR_USS_LRC];
  double Y = us / (3.0 * V);                        /* dU/dV   */
  double Z = (uss - 2.0 * us) / (9.0 * V * V);      /* d2U/dV2 */
  m[OR_M_N] += 1.0;
  m[OR_M_X] += X;
  m[OR_M_XX] += X * X;
  m[OR_M_XXX] += X * X * X;
  m[OR_M_Y] += Y;
  m[OR_M_XY] += X * Y;
  m[OR_M_XXY] += X * X * Y;
  m[OR_M_YY] += Y * Y;
  m[OR_M_XYY] += X * Y * Y;
  m[OR_M_Z] += Z;
  m[OR_M_XZ] += X * Z;
}

/* One row of the energy log: U, K_trans, K_rot, W, and the two volume
 * derivatives in s (explicit + tail), from which dU/dV and d2U/dV2 follow
 * (Sec. 3). */
static void log_row(double* row, const double* sums, double ktr, double krot) {
  row[0] = u_total(sums);
  row[1] = ktr;
  row[2] = krot;
  row[3] = sums[OR_VIRIAL];
  row[4] = sums[OR_US] + sums[OR_US_LRC];
  row[5] = sums[OR_USS] + sums[OR_USS_LRC];
}

static void wrap_box(double* x, int n3, double L) {
  for (int c = 0; c < n3; ++c) x[c] -= L * floor(x[c] / L);
}

int or_md(const or_species* sp, int32_t nsp, const or_params* p, const or_md_cfg* cfg,
          int32_t n, const int32_t* species, double* com, double* quat, double* vel,
          double* omega, double* energy_log, double* moments, double* rdf, double* acf_v,
          double* acf_j, double* acf_cnt, double* res_acf, double* res_cnt, double* solvation,
          double* acf_q, double* acf_q_cnt) {
  int e = or_check(sp, nsp, p);
  if (e) return e;
  if (!cfg || n < 2 || cfg->n_steps < 0 || !(cfg->dt > 0.0)) return -30;
  if (cfg->rdf_every > 0 && (cfg->rdf_bins < 1 || !(cfg->rdf_rmax > 0.0))) return -31;
  if (cfg->acf_every > 0 &&
      (cfg->acf_nlag < 1 || cfg->acf_origin_every < cfg->acf_every ||
       cfg->acf_origin_every % cfg->acf_every != 0))
    return -32;
  int rotating = 0;
  for (int s = 0; s < nsp; ++s)
    for (int k = 0; k < 3; ++k)
      if (sp[s].inertia[k] > 0.0) rotating = 1;
  if (cfg->integrator == OR_VV && rotating) return -33;
  /* Massieu moments need d2U/dV2, which the reciprocal sum does not supply;
   * the paper does not combine them with Ewald summation (Sec. 4) */
  if (cfg->sample_every > 0 && p->elec == OR_ELEC_EWALD) return -36;

  double L = p->box, V = L * L * L, dt = cfg->dt;
  size_t n3 = 3 * (size_t)n, n4 = 4 * (size_t)n;
  double *F = calloc(n3, sizeof(double)), *Tq = calloc(n3, sizeof(double));
  double sums[OR_NSUM];
  acf_t acf;
  memset(&acf, 0, sizeof(acf));
  if (cfg->acf_every > 0) {
    acf.n = n;
    acf.nlag = cfg->acf_nlag;
    acf.every = cfg->acf_every;
    acf.origin_every = cfg->acf_origin_every;
    acf.max_live = cfg->acf_nlag * cfg->acf_every / cfg->acf_origin_every + 2;
    acf.t0 = calloc((size_t)acf.max_live, sizeof(int));
    acf.v0 = calloc((size_t)acf.max_live * n3, sizeof(double));
    acf.j0 = calloc((size_t)acf.max_live * 3, sizeof(double));
  }
  hf_t hf;
  memset(&hf, 0, sizeof(hf));
  double jq[3] = {0.0, 0.0, 0.0};
  if (cfg->heat_flux) {
    if (cfg->acf_every <= 0 || p->elec == OR_ELEC_EWALD) {
      free(F); free(Tq); free(acf.t0); free(acf.v0); free(acf.j0);
      return -35;
    }
    hf.on = 1;
    hf.nlag = cfg->acf_nlag;
    hf.every = cfg->acf_every;
    hf.origin_every = cfg->acf_origin_every;
    hf.max_live = acf.max_live;
    hf.t0 = calloc((size_t)hf.max_live, sizeof(int));
    hf.valid = calloc((size_t)hf.max_live, sizeof(int));
    hf.j0 = calloc((size_t)hf.max_live * 3, sizeof(double));
  }
  res_t res;
  memset(&res, 0, sizeof(res));
  if (cfg->res_solute >= 0) {
    if (cfg->acf_every <= 0 || cfg->res_solute >= nsp || cfg->res_solvent < 0 || cfg->res_solvent >= nsp ||
        !(cfg->res_radius > 0.0) || !(cfg->res_radius < 0.5 * p->box) || cfg->res_tolerance < 0) {
      free(F); free(Tq); free(acf.t0); free(acf.v0); free(acf.j0);
      return -34;
    }
    res.on = 1;
    res.tol = cfg->res_tolerance;
    res.nlag = cfg->acf_nlag;
    res.every = cfg->acf_every;
    res.origin_every = cfg->acf_origin_every;
    res.max_live = acf.max_live;
    res.r2 = cfg->res_radius * cfg->res_radius;
    res.solute = malloc(sizeof(int) * (size_t)n);
    res.solvent = malloc(sizeof(int) * (size_t)n);
    for (int i = 0; i < n; ++i) {
      if (species[i] == cfg->res_solute) res.solute[res.nu++] = i;
      if (species[i] == cfg->res_solvent) res.solvent[res.nv++] = i;
    }
    res.t0 = calloc((size_t)res.max_live, sizeof(int));
    res.n0 = calloc((size_t)res.max_live * (res.nu + 1), sizeof(int));
    res.away = calloc((size_t)res.max_live * (res.nu + 1) * (res.nv + 1), sizeof(int));
  }
  /* translational and rotational degrees of freedom (isokinetic NVT) */
  double f_tr = 3.0 * n - 3.0, f_rot = 0.0;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k)
      if (sp[species[i]].inertia[k] > 0.0) f_rot += 1.0;

  wrap_box(com, (int)n3, L);
  e = evaluate(sp, nsp, p, n, species, com, quat, F, Tq, sums);
  if (e) goto done;

  if (cfg->integrator == OR_VV) {
    /* velocity Verlet, point molecules */
    double ktr = 0.0;
    for (int i = 0; i < n; ++i) ktr += 0.5 * sp[species[i]].mass * dot3(vel + 3 * i, vel + 3 * i);
    if (energy_log) {
      log_row(energy_log, sums, ktr, 0.0);
    }
    if (acf.n) acf_sample(&acf, 0, vel, sp, species, acf_v, acf_j, acf_cnt);
    if (res.on) residence_sample(&res, 0, com, L, res_acf, res_cnt, solvation);
    if (hf.on) heat_acf_sample(&hf, 0, jq, 0, acf_q, acf_q_cnt);
    for (int s = 1; s <= cfg->n_steps; ++s) {
      for (int i = 0; i < n; ++i) {
        double m = sp[species[i]].mass;
        for (int k = 0; k < 3; ++k) {
          vel[3 * i + k] += 0.5 * dt / m * F[3 * i + k];
          com[3 * i + k] += dt * vel[3 * i + k];
        }
      }
      wrap_box(com, (int)n3, L);
      e = evaluate(sp, nsp, p, n, species, com, quat, F, Tq, sums);
      if (e) goto done;
      if (hf.on && s % cfg->acf_every == 0) {
        e = or_heat_flux(sp, nsp, p, n, species, com, quat, vel, omega, cfg->h_partial, jq);
        if (e) goto done;
      }
      for (int i = 0; i < n; ++i) {
        double m = sp[species[i]].mass;
        for (int k = 0; k < 3; ++k) vel[3 * i + k] += 0.5 * dt / m * F[3 * i + k];
      }
      double k2 = 0.0;
      for (int i = 0; i < n; ++i) k2 += sp[species[i]].mass * dot3(vel + 3 * i, vel + 3 * i);
      if (cfg->temperature > 0.0) {
        double fac = sqrt(cfg->temperature * f_tr / k2);
        for (size_t c = 0; c < n3; ++c) vel[c] *= fac;
        k2 = 0.0;
        for (int i = 0; i < n; ++i) k2 += sp[species[i]].mass * dot3(vel + 3 * i, vel + 3 * i);
      }
      if (energy_log) {
        log_row(energy_log + OR_LOG_COLS * s, sums, 0.5 * k2, 0.0);
      }
      if (moments && cfg->sample_every > 0 && s % cfg->sample_every == 0)
        moment_sample(sums, V, cfg->u0, moments);
      if (rdf && cfg->rdf_every > 0 && s % cfg->rdf_every == 0)
        rdf_sample(sp, nsp, p, cfg, n, species, com, quat, rdf);
      if (acf.n && s % cfg->acf_every == 0) acf_sample(&acf, s, vel, sp, species, acf_v, acf_j, acf_cnt);
      if (res.on && s % cfg->acf_every == 0) residence_sample(&res, s, com, L, res_acf, res_cnt, solvation);
      if (hf.on && s % cfg->acf_every == 0) heat_acf_sample(&hf, s, jq, 1, acf_q, acf_q_cnt);
    }
    goto done;
  }

  /* ---- 5-value Gear predictor-corrector with quaternions ---- */
  {
    const double ct[5] = {19.0 / 120.0, 3.0 / 4.0, 1.0, 1.0 / 2.0, 1.0 / 12.0};
    const double cr[5] = {251.0 / 720.0, 1.0, 11.0 / 12.0, 1.0 / 3.0, 1.0 / 24.0};
    double *r[5], *q[5], *w[5];
    for (int k = 0; k < 5; ++k) {
      r[k] = calloc(n3, sizeof(double));
      q[k] = calloc(n4, sizeof(double));
      w[k] = calloc(n3, sizeof(double));
    }
    double* vtmp = calloc(n3, sizeof(double));
    /* initial scaled derivatives: r1 = dt v, r2 = dt^2 a / 2, q1 = dt dq/dt,
     * w1 = dt domega/dt; higher ones start at zero */
    memcpy(r[0], com, n3 * sizeof(double));
    memcpy(q[0], quat, n4 * sizeof(double));
    memcpy(w[0], omega, n3 * sizeof(double));
    for (int i = 0; i < n; ++i) {
      const or_species* s = &sp[species[i]];
      double tb[3], wd[3], qd[4];
      for (int k = 0; k < 3; ++k) {
        r[1][3 * i + k] = dt * vel[3 * i + k];
        r[2][3 * i + k] = 0.5 * dt * dt * F[3 * i + k] / s->mass;
      }
      to_body(quat + 4 * i, Tq + 3 * i, tb);
      euler_rhs(s->inertia, tb, omega + 3 * i, wd);
      qdot(quat + 4 * i, omega + 3 * i, qd);
      for (int k = 0; k < 3; ++k) w[1][3 * i + k] = dt * wd[k];
      for (int k = 0; k < 4; ++k) q[1][4 * i + k] = dt * qd[k];
    }
    if (energy_log) {
      double ktr = 0.0, krot = 0.0;
      for (int i = 0; i < n; ++i) {
        const or_species* s = &sp[species[i]];
        ktr += 0.5 * s->mass * dot3(vel + 3 * i, vel + 3 * i);
        for (int k = 0; k < 3; ++k) krot += 0.5 * s->inertia[k] * omega[3 * i + k] * omega[3 * i + k];
      }
      log_row(energy_log, sums, ktr, krot);
    }
    if (acf.n) acf_sample(&acf, 0, vel, sp, species, acf_v, acf_j, acf_cnt);
    if (res.on) residence_sample(&res, 0, com, L, res_acf, res_cnt, solvation);
    if (hf.on) heat_acf_sample(&hf, 0, jq, 0, acf_q, acf_q_cnt);

    for (int s = 1; s <= cfg->n_steps && !e; ++s) {
      gear_predict(r, (int)n3);
      if (rotating) {
        gear_predict(q, (int)n4);
        gear_predict(w, (int)n3);
        for (int i = 0; i < n; ++i) { /* unit quaternion for the force evaluation */
          double* qi = q[0] + 4 * i;
          double nq = sqrt(qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]);
          for (int k = 0; k < 4; ++k) qi[k] /= nq;
        }
      }
      e = evaluate(sp, nsp, p, n, species, r[0], q[0], F, Tq, sums);
      if (e) break;
      if (hf.on && s % cfg->acf_every == 0) {   /* flux at the predicted state */
        for (size_t c = 0; c < n3; ++c) vtmp[c] = r[1][c] / dt;
        e = or_heat_flux(sp, nsp, p, n, species, r[0], q[0], vtmp, w[0], cfg->h_partial, jq);
        if (e) break;
      }
      for (int i = 0; i < n; ++i) {
        const or_species* sx = &sp[species[i]];
        for (int k = 0; k < 3; ++k) {
          int c = 3 * i + k;
          double delta = 0.5 * dt * dt * F[c] / sx->mass - r[2][c];
          for (int d = 0; d < 5; ++d) r[d][c] += ct[d] * delta;
        }
        if (!rotating) continue;
        double tb[3], wd[3], qd[4];
        to_body(q[0] + 4 * i, Tq + 3 * i, tb);
        euler_rhs(sx->inertia, tb, w[0] + 3 * i, wd);
        qdot(q[0] + 4 * i, w[0] + 3 * i, qd);
        for (int k = 0; k < 3; ++k) {
          int c = 3 * i + k;
          double delta = dt * wd[k] - w[1][c];
          for (int d = 0; d < 5; ++d) w[d][c] += cr[d] * delta;
        }
        for (int k = 0; k < 4; ++k) {
          int c = 4 * i + k;
          double delta = dt * qd[k] - q[1][c];
          for (int d = 0; d < 5; ++d) q[d][c] += cr[d] * delta;
        }
        double* qi = q[0] + 4 * i;
        double nq = sqrt(qi[0] * qi[0] + qi[1] * qi[1] + qi[2] * qi[2] + qi[3] * qi[3]);
        for (int k = 0; k < 4; ++k) qi[k] /= nq;
      }
      wrap_box(r[0], (int)n3, L);
      /* isokinetic NVT: scale dt*v, and omega together with dt*dq/dt */
      double k2 = 0.0, kr2 = 0.0;
      for (int i = 0; i < n; ++i) {
        const or_species* sx = &sp[species[i]];
        for (int k = 0; k < 3; ++k) {
          double v = r[1][3 * i + k] / dt;
          k2 += sx->mass * v * v;
          kr2 += sx->inertia[k] * w[0][3 * i + k] * w[0][3 * i + k];
        }
      }
      if (cfg->temperature > 0.0) {
        double ft = sqrt(cfg->temperature * f_tr / k2);
        for (size_t c = 0; c < n3; ++c) r[1][c] *= ft;
        k2 *= ft * ft;
        if (f_rot > 0.0 && kr2 > 0.0) {
          double fr = sqrt(cfg->temperature * f_rot / kr2);
          for (size_t c = 0; c < n3; ++c) w[0][c] *= fr;
          for (size_t c = 0; c < n4; ++c) q[1][c] *= fr;
          kr2 *= fr * fr;
        }
      }
      if (energy_log) {
        log_row(energy_log + OR_LOG_COLS * s, sums, 0.5 * k2, 0.5 * kr2);
      }
      if (moments && cfg->sample_every > 0 && s % cfg->sample_every == 0)
        moment_sample(sums, V, cfg->u0, moments);
      if (rdf && cfg->rdf_every > 0 && s % cfg->rdf_every == 0)
        rdf_sample(sp, nsp, p, cfg, n, species, r[0], q[0], rdf);
      if (acf.n && s % cfg->acf_every == 0) {
        for (size_t c = 0; c < n3; ++c) vtmp[c] = r[1][c] / dt;
        acf_sample(&acf, s, vtmp, sp, species, acf_v, acf_j, acf_cnt);
      }
      if (res.on && s % cfg->acf_every == 0) residence_sample(&res, s, r[0], L, res_acf, res_cnt, solvation);
      if (hf.on && s % cfg->acf_every == 0) heat_acf_sample(&hf, s, jq, 1, acf_q, acf_q_cnt);
    }
    memcpy(com, r[0], n3 * sizeof(double));
    memcpy(quat, q[0], n4 * sizeof(double));
    memcpy(omega, w[0], n3 * sizeof(double));
    for (size_t c = 0; c < n3; ++c) vel[c] = r[1][c] / dt;
    for (int k = 0; k < 5; ++k) { free(r[k]); free(q[k]); free(w[k]); }
    free(vtmp);
  }
done:
  free(F); free(Tq);
  free(acf.t0); free(acf.v0); free(acf.j0);
  free(res.solute); free(res.solvent); free(res.t0); free(res.n0); free(res.away);
  free(hf.t0); free(hf.valid); free(hf.j0);
  return e;
}
