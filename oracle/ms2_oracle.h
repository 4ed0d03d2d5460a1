/*
 * ms2_oracle.h -- plain, slow, sequential FP64 CPU oracle for the rigid
 * multi-site molecular dynamics hot path of ms2 2.0 (arXiv 1507.07548).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes,
 * links or calls this code; only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no header, helper,
 * table or constant with the GPU path: every declaration below is its own.
 *
 * What it computes (each function cites the passage it follows):
 *   or_forces      -- partner search, site-site energy/force/torque, virial,
 *                     volume-derivative sums, LJ long-range correction and
 *                     the Ewald constant terms   (Sec. 2 three molecule loops;
 *                     Sec. 3 dU/dV, d2U/dV2 and LRC; Sec. 4 Ewald)
 *   or_kspace      -- Ewald reciprocal-space energy, forces, torques and
 *                     molecular virial, summed over the full k sphere (Sec. 4)
 *   or_md          -- velocity Verlet or 5-value Gear predictor-corrector
 *                     with quaternions and isokinetic NVT, plus on-the-fly
 *                     sampling: Lustig moments (Sec. 3, Eq. 1), RDF (Sec. 5,
 *                     Eq. 2), velocity and electric-current autocorrelation
 *                     functions on an extended time step (Sec. 4; Sec. 5,
 *                     Eqs. 3-4)
 *
 * Layout: arrays of structures, molecule-major: com[n][3], quat[n][4]
 * (w,x,y,z; body -> lab), force[n][3], torque[n][3] (lab frame).
 * All functions return 0 on success and a negative code on bad arguments.
 */
#ifndef MS2_ORACLE_H
#define MS2_ORACLE_H
#include <stdint.h>

#define OR_MAXS 8

enum { OR_LJ = 0, OR_CHARGE = 1, OR_DIPOLE = 2, OR_QUAD = 3 };
enum { OR_ELEC_NONE = 0, OR_ELEC_RF = 1, OR_ELEC_EWALD = 2 };
enum { OR_VV = 0, OR_GEAR = 1 };

/* sums[] slots written by or_forces / accumulated by or_kspace */
enum {
  OR_U_LJ = 0,     /* explicit Lennard-Jones energy                      */
  OR_U_ELEC = 1,   /* explicit electrostatics (Coulomb/RF/multipole/erfc) */
  OR_U_RECIP = 2,  /* Ewald reciprocal energy                            */
  OR_U_CONST = 3,  /* Ewald self + intramolecular constant               */
  OR_U_LRC = 4,    /* LJ tail energy                                     */
  OR_VIRIAL = 5,   /* molecular virial W = sum R_ij . F_ij (+ recip)     */
  OR_US = 6,       /* sum dU/ds under molecular scaling (explicit+recip) */
  OR_USS = 7,      /* sum d2U/ds2 (explicit pairs only)                  */
  OR_US_LRC = 8,   /* LJ tail of U_s                                     */
  OR_USS_LRC = 9,  /* LJ tail of U_ss                                    */
  OR_NPAIR = 10,   /* accepted molecule pairs                            */
  OR_NSITE = 11,   /* interacting site pairs in accepted molecule pairs  */
  OR_NSUM = 12
};

typedef struct {
  int32_t n_sites;
  int32_t type[OR_MAXS];
  double pos[OR_MAXS][3];   /* body frame, relative to the centre of mass */
  double axis[OR_MAXS][3];  /* body frame unit axis of dipole/quadrupole  */
  double sigma[OR_MAXS];
  double eps[OR_MAXS];
  double mag[OR_MAXS];      /* charge q, dipole mu or quadrupole Q        */
  double mass;
  double inertia[3];        /* principal moments; 0 about a linear axis   */
} or_species;

typedef struct {
  double box;        /* cubic edge L                           */
  double rc;         /* molecule-centre cut-off, rc < L/2      */
  double eps_rf;     /* reaction-field permittivity (inf ok)   */
  double alpha;      /* Ewald splitting parameter              */
  double coulomb_k;  /* 1/(4 pi eps0) in the caller's units    */
  int32_t elec;      /* OR_ELEC_*                              */
  int32_t kmax2;     /* Ewald: integer vectors 0 < n^2 <= kmax2 */
  int32_t lj_lrc;    /* 1: add the LJ long-range correction    */
  int32_t cutoff_mode; /* OR_CUT_COM: every site pair of molecules whose
                          centres are closer than rc; OR_CUT_SITE: LJ site
                          pairs closer than rc themselves, electrostatic
                          site pairs of molecules closer than rc (needs
                          rc + 2 dmax < L/2, dmax = largest LJ-site offset) */
} or_params;

enum { OR_CUT_COM = 0, OR_CUT_SITE = 1 };

typedef struct {
  int32_t integrator;       /* OR_VV (point molecules only) or OR_GEAR */
  int32_t n_steps;
  double dt;
  double temperature;       /* > 0: isokinetic NVT at this T; <= 0: NVE */
  int32_t sample_every;     /* Lustig moments every k steps (0 = off)   */
  int32_t rdf_every;        /* RDF every k steps (0 = off)              */
  int32_t rdf_bins;
  int32_t acf_every;        /* extended time step n (0 = off)           */
  int32_t acf_origin_every; /* steps between new time origins           */
  int32_t acf_nlag;         /* lags per origin (window / n)             */
  double rdf_rmax;
  double u0;                /* shift of U inside the moment sums        */
  int32_t res_solute;       /* residence time (Sec. 5, Eqs. 7-8): species of
                               the central molecules, -1 = off          */
  int32_t res_solvent;      /* species counted around them              */
  double res_radius;        /* shell radius between molecule centres    */
  int32_t res_tolerance;    /* samples a molecule may stay outside and
                               still count as resident                  */
  int32_t heat_flux;        /* 1: heat-flux ACF on the ACF schedule     */
  const double* h_partial;  /* [nsp] partial molar enthalpy per molecule
                               of each species (NULL = 0)               */
} or_md_cfg;

/* moments[] slots: sums over samples of powers and products of
 * X = U - u0 (shifted potential energy), Y = dU/dV and Z = d2U/dV2 */
enum {
  OR_M_N = 0, OR_M_X, OR_M_XX, OR_M_XXX, OR_M_Y, OR_M_XY, OR_M_XXY,
  OR_M_YY, OR_M_XYY, OR_M_Z, OR_M_XZ, OR_NMOM
};

/* columns of one row of or_md's energy log */
#define OR_LOG_COLS 6

#ifdef __cplusplus
extern "C" {
#endif

int or_check(const or_species* sp, int32_t nsp, const or_params* p);

int or_forces(const or_species* sp, int32_t nsp, const or_params* p,
              int32_t n, const int32_t* species, const double* com,
              const double* quat, double* force, double* torque,
              double* sums);

int or_kspace(const or_species* sp, int32_t nsp, const or_params* p,
              int32_t n, const int32_t* species, const double* com,
              const double* quat, double* force, double* torque,
              double* sums);

/* Runs cfg->n_steps steps in place on com/quat/vel/omega (vel lab frame,
 * omega body frame).  energy_log[(n_steps+1)*OR_LOG_COLS] receives, per step
 * and for the initial state, (U_total, K_trans, K_rot, W, U_s + U_s,lrc,
 * U_ss + U_ss,lrc).  moments[OR_NMOM];
 * rdf[npairtypes*rdf_bins] (counts as doubles, unordered site pairs);
 * acf_v[acf_nlag], acf_j[acf_nlag], acf_cnt[acf_nlag]: raw sums over
 * origins of (1/N) sum_i v_i(t0).v_i(t0+l n), of j_e(t0).j_e(t0+l n), and
 * the number of origins contributing to each lag.  Residence sampling (on
 * the ACF schedule): res_acf[acf_nlag] sums over (origin, solute with a
 * non-empty shell at the origin) of the fraction of its initial shell still
 * resident, res_cnt[acf_nlag] the number of such terms, solvation[2] = (sum
 * over samples and solutes of the shell population, number of terms).  Any
 * output may be NULL. */
int or_md(const or_species* sp, int32_t nsp, const or_params* p,
          const or_md_cfg* cfg, int32_t n, const int32_t* species,
          double* com, double* quat, double* vel, double* omega,
          double* energy_log, double* moments, double* rdf,
          double* acf_v, double* acf_j, double* acf_cnt,
          double* res_acf, double* res_cnt, double* solvation,
          double* acf_q, double* acf_q_cnt);

/* Microscopic heat flux of rigid molecules (Sec. 5, Eq. 6) at one state:
 *   J_q = sum_k (m_k v_k^2 / 2 + w_k.I_k.w_k / 2 - h_k) v_k
 *       + sum over pairs k < l inside the cut-off of
 *         u_kl (v_k + v_l) / 2
 *         + R_kl (F_kl.(v_k + v_l) + tau_kl.w_k - tau_lk.w_l) / 2
 * with R_kl = R_k - R_l (minimum image), F_kl the force on k from l,
 * tau_kl the torque on k from l about its centre, w the lab angular
 * velocity and h_k the partial enthalpy per molecule of k's species.
 * vel[n][3] lab frame, omega[n][3] body frame (as in or_md), h_partial[nsp]
 * or NULL.  Reaction field or no electrostatics only (Ewald: -40). */
int or_heat_flux(const or_species* sp, int32_t nsp, const or_params* p, int32_t n,
                 const int32_t* species, const double* com, const double* quat,
                 const double* vel, const double* omega, const double* h_partial, double* jq);

/* Number of LJ site types (one per LJ site of each species) used by the
 * RDF; histograms are stored for every unordered type pair (t1 <= t2). */
int or_rdf_ntypes(const or_species* sp, int32_t nsp);

#ifdef __cplusplus
}
#endif
#endif
