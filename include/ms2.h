/*
 * ms2.h -- C ABI of the MI355X (gfx950) force/energy/virial hot path of the
 * rigid multi-site molecular dynamics method of ms2 2.0 (arXiv 1507.07548).
 *
 * One system is ~10^3 rigid molecules in a cubic periodic box.  Each
 * molecule carries Lennard-Jones sites, point charges, point dipoles and
 * linear point quadrupoles.  Pairs interact when their centres of mass lie
 * within the cut-off rc < L/2 under minimum image (the paper's Sec. 2 notes
 * rc is of the order of L/2, which rules out domain decomposition).
 * Electrostatics: plain truncated, reaction field (Sec. 3) or Ewald (Sec. 4).
 *
 * Conventions shared by every entry point
 *   - Plain C types only.  Device pointers (prefix d_) are HIP device
 *     memory owned by the caller, who keeps them alive until the stream has
 *     completed the call.  Host pointers (prefix h_) are read before return.
 *   - Device arrays are structure-of-arrays with row length n_mol:
 *       com   double[3][n]  centre of mass x,y,z (ideally wrapped to [0,L))
 *       quat  double[4][n]  unit quaternion w,x,y,z rotating body -> lab
 *       force double[3][n], torque double[3][n] (lab frame)
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls are stream-ordered and asynchronous unless stated otherwise.
 *   - Every call returns ms2_status.  Argument errors are detected on the
 *     host before anything is enqueued and leave outputs untouched;
 *     ms2_last_error() returns a thread-local message for the last failure.
 *   - Units are the caller's; k_B = 1 in the energy unit, coulomb_k is
 *     1/(4 pi eps0) in the caller's units.
 */
#ifndef MS2_H
#define MS2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MS2_MAX_SITES 8      /* sites per species            */
#define MS2_MAX_SPECIES 8    /* species per context          */
#define MS2_NOALLOC_MAX_MOL 4096  /* molecules per ms2_forces_noalloc call */

typedef enum {
  MS2_OK = 0,
  MS2_EINVAL = 1,      /* bad argument (synchronous)                     */
  MS2_ENOMEM = 2,      /* device allocation failed / HBM budget exceeded */
  MS2_EDEVICE = 3,     /* HIP runtime error                              */
  MS2_ENONFINITE = 4,  /* a slot produced a non-finite force or energy   */
  MS2_EFULL = 5        /* no free slot in the batch                      */
} ms2_status;

enum { MS2_SITE_LJ = 0, MS2_SITE_CHARGE = 1, MS2_SITE_DIPOLE = 2, MS2_SITE_QUAD = 3 };
enum { MS2_ELEC_NONE = 0, MS2_ELEC_RF = 1, MS2_ELEC_EWALD = 2 };
enum { MS2_FP64 = 0, MS2_FP32 = 1 };           /* pair arithmetic precision */
enum { MS2_CUT_COM = 0, MS2_CUT_SITE = 1 };    /* ms2_params.cutoff_mode    */
enum { MS2_VV = 0, MS2_GEAR = 1 };

/* Slots of the double sums[MS2_NSUM] output.
 * Energies: U = U_LJ + U_ELEC + U_RECIP + U_CONST + U_LRC.
 * Volume derivatives (Sec. 3; molecular scaling of the centres, rigid
 * bodies, rc and alpha fixed):
 *   dU/dV   = (US + US_LRC) / (3 V)
 *   d2U/dV2 = (USS + USS_LRC - 2 (US + US_LRC)) / (9 V^2)
 * USS excludes the Ewald reciprocal part (Massieu sampling is not offered
 * together with Ewald, Sec. 4). */
enum {
  MS2_SUM_U_LJ = 0,      /* explicit LJ energy                              */
  MS2_SUM_U_ELEC = 1,    /* explicit electrostatics (Coulomb/RF/multipole/erfc) */
  MS2_SUM_U_RECIP = 2,   /* Ewald reciprocal energy (ms2_ewald_kspace)      */
  MS2_SUM_U_CONST = 3,   /* Ewald self + intramolecular constants           */
  MS2_SUM_U_LRC = 4,     /* LJ long-range correction                        */
  MS2_SUM_VIRIAL = 5,    /* molecular virial W = sum_{i<j} R_ij . F_ij (+recip) */
  MS2_SUM_US = 6,        /* dU/ds at s = 1 (explicit + reciprocal)          */
  MS2_SUM_USS = 7,       /* d2U/ds2 at s = 1 (explicit pairs)               */
  MS2_SUM_US_LRC = 8,
  MS2_SUM_USS_LRC = 9,
  MS2_SUM_NPAIR = 10,    /* accepted molecule pairs                         */
  MS2_SUM_NSITE = 11,    /* interacting site pairs of accepted pairs        */
  MS2_NSUM = 12
};

/* One molecular species, host memory, copied by ms2_create.
 * Sites are given in the principal body frame relative to the centre of
 * mass.  A site is one of MS2_SITE_*; an LJ site and a charge at the same
 * place are two sites.  LJ: sigma, eps (Lorentz-Berthelot mixing).
 * CHARGE: mag = q.  DIPOLE: mag = mu along axis.  QUAD: mag = Q (linear
 * quadrupole, Q = sum q z^2) along axis.  inertia[k] = 0 freezes rotation
 * about body axis k (linear or point molecules). */
typedef struct {
  int32_t n_sites;
  int32_t type[MS2_MAX_SITES];
  double pos[MS2_MAX_SITES][3];
  double axis[MS2_MAX_SITES][3];
  double sigma[MS2_MAX_SITES];
  double eps[MS2_MAX_SITES];
  double mag[MS2_MAX_SITES];
  double mass;
  double inertia[3];
} ms2_species;

/* Per-system physical parameters (host memory, read before return). */
typedef struct {
  double box;        /* cubic edge L                                        */
  double rc;         /* cut-off radius, 0 < rc < L/2 (see cutoff_mode)      */
  double eps_rf;     /* reaction-field permittivity, >= 1, INFINITY allowed */
  double alpha;      /* Ewald splitting parameter (> 0 with Ewald)          */
  double coulomb_k;  /* 1/(4 pi eps0)                                       */
  int32_t elec;      /* MS2_ELEC_*; Ewald admits LJ and charge sites only   */
  int32_t kmax2;     /* Ewald k set: integer n with 0 < |n|^2 <= kmax2      */
  int32_t lj_lrc;    /* 1: LJ long-range correction (Sec. 3)                */
  int32_t precision; /* MS2_FP64 or MS2_FP32 (FP32 pairs, FP64 sums)         */
  int32_t cutoff_mode; /* MS2_CUT_COM: a molecule pair interacts (all its site
                          pairs) when its centres are closer than rc.
                          MS2_CUT_SITE: an LJ site pair interacts when its
                          own distance is below rc; electrostatic site pairs
                          still follow the centre distance; needs
                          rc + 2 d_max < L/2, d_max the largest LJ-site
                          distance from a centre (Sec. 3).  The LJ long-range
                          correction is the same in both modes.            */
  int32_t pad;       /* set to 0                                           */
} ms2_params;

typedef struct ms2_ctx ms2_ctx;
typedef struct ms2_batch ms2_batch;

/* Creates a context on HIP device `device` holding the species table.
 * Errors: MS2_EINVAL (bad species), MS2_EDEVICE, MS2_ENOMEM. */
ms2_status ms2_create(ms2_ctx** out, const ms2_species* h_species, int32_t n_species,
                      int32_t device);
/* Releases every device buffer the context owns; waits for the device. */
void ms2_destroy(ms2_ctx* ctx);

/* Explicit pair part of one force/energy evaluation (Sec. 2: partner search,
 * energy and force loops over molecules; Sec. 3: dU/dV, d2U/dV2, LJ LRC and
 * reaction field; Sec. 4: Ewald real space and constants).
 * For every molecule pair whose minimum-image centre distance R satisfies
 * |R|^2 < rc^2, all site pairs interact with that image shift.
 * OVERWRITES d_force, d_torque (double[3][n_mol]) and d_sums
 * (double[MS2_NSUM]) with the explicit terms, the LJ tail and the Ewald
 * constants.  d_species: int32[n_mol] species indices; d_com double[3][n];
 * d_quat double[4][n].  Scratch is owned by the context and grows on the
 * first call at a larger n_mol (that call allocates; later ones do not).
 * Errors: MS2_EINVAL (n_mol < 2, rc >= L/2, Ewald with multipoles, NULL
 * pointers, ...), MS2_ENOMEM, MS2_EDEVICE.  A species index outside
 * [0, n_species) in d_species is found on the device, where the call cannot
 * return it: that molecule's force and torque and every energy, virial and
 * volume-derivative sum of the call become NaN, and ms2_device_errors
 * reports MS2_EINVAL. */
ms2_status ms2_forces(ms2_ctx* ctx, const ms2_params* h_params, int32_t n_mol,
                      const int32_t* d_species, const double* d_com, const double* d_quat,
                      double* d_force, double* d_torque, double* d_sums, void* stream);

/* ms2_forces for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, outputs, errors and device-side species check as
 * ms2_forces, and the same result bit for bit as ms2_forces with its untuned
 * default tile shape (symmetric 64 x 64 tile pairs, 1, 2 or 4 items per
 * tile pair by the system size; this call always takes that shape).  It calls no hipMalloc/hipFree and allocates nothing: its scratch
 * (site records, pair partials, block sums, work items; under 16 MiB) is a
 * static device array that each GPU the library runs on holds until the
 * process ends.  Limit: 2 <= n_mol <= MS2_NOALLOC_MAX_MOL, otherwise
 * MS2_EINVAL before anything is enqueued.  Every call on one GPU shares that
 * GPU's array: calls that overlap on the same GPU (other streams, threads or
 * contexts) race and must be serialized by the caller. */
ms2_status ms2_forces_noalloc(ms2_ctx* ctx, const ms2_params* h_params, int32_t n_mol,
                              const int32_t* d_species, const double* d_com, const double* d_quat,
                              double* d_force, double* d_torque, double* d_sums, void* stream);

/* Ewald reciprocal-space part (Sec. 4): k = 2 pi n / L over the half space
 * of integer n with 0 < |n|^2 <= kmax2; S(k) = sum_a q_a exp(i k.r_a)
 * accumulated in FP64; tin-foil boundary.  ACCUMULATES (+=) reciprocal
 * forces and torques into d_force/d_torque and U_RECIP, VIRIAL (molecular)
 * and US into d_sums, so call it after ms2_forces on the same stream.
 * Errors: MS2_EINVAL if elec != MS2_ELEC_EWALD or arguments are bad.  A
 * species index outside [0, n_species) makes S(k), and with it every
 * reciprocal force, torque and sum of the call, NaN, and is reported by
 * ms2_device_errors. */
ms2_status ms2_ewald_kspace(ms2_ctx* ctx, const ms2_params* h_params, int32_t n_mol,
                            const int32_t* d_species, const double* d_com,
                            const double* d_quat, double* d_force, double* d_torque,
                            double* d_sums, void* stream);

/* Argument errors that only the device can see (a species index outside
 * the table in the arrays of ms2_forces / ms2_ewald_kspace).  Synchronizes
 * `stream`, then returns MS2_EINVAL if any call on this context recorded
 * such an error since the last ms2_device_errors, and clears the record;
 * MS2_OK otherwise.  Batch slots validate their species at admission and
 * never record one. */
ms2_status ms2_device_errors(ms2_ctx* ctx, void* stream);

/* ----------------------------------------------------------------------- */
/* Batched, device-resident simulation (many independent systems)          */
/* ----------------------------------------------------------------------- */

/* Host description of one simulation request, copied at admission.
 * Host arrays use the same structure-of-arrays layout as the device ones. */
typedef struct {
  ms2_params params;
  int32_t n_mol;
  int32_t integrator;        /* MS2_VV (point molecules only) or MS2_GEAR  */
  int64_t n_steps;           /* steps this slot runs before it stops       */
  double dt;
  double temperature;        /* > 0: isokinetic NVT at T; <= 0: NVE        */
  int32_t sample_every;      /* Lustig moment sample every k steps, 0 off  */
  int32_t rdf_every;         /* RDF sample every k steps, 0 off            */
  int32_t rdf_bins;
  int32_t acf_every;         /* extended time step n (Sec. 4), 0 off       */
  int32_t acf_origin_every;  /* steps between ACF time origins (multiple of n) */
  int32_t acf_nlag;          /* lags per origin                            */
  double rdf_rmax;
  double u0;                 /* energy shift inside the moment sums        */
  int32_t res_enable;        /* 1: residence time and solvation number
                                (Sec. 5, Eqs. 7-8), sampled with the ACFs;
                                0: off (a zero-filled struct samples none) */
  int32_t res_solute;        /* species of the central molecules           */
  int32_t res_solvent;       /* species of the molecules counted around them */
  int32_t res_tolerance;     /* samples a molecule may spend outside the shell
                                and still count as resident (Impey et al.) */
  double res_radius;         /* shell radius between molecule centres (< box/2) */
  int32_t heat_flux;         /* 1: heat-flux ACF (Sec. 5, Eqs. 5-6) sampled with
                                the ACFs; reaction field or no electrostatics */
  int32_t hf_pad;
  double h_partial[MS2_MAX_SPECIES]; /* partial molar enthalpy per molecule of
                                each species (energy units of the potential) */
  const int32_t* h_species;  /* [n]    */
  const double* h_com;       /* [3][n] */
  const double* h_quat;      /* [4][n] */
  const double* h_vel;       /* [3][n] lab frame  */
  const double* h_omega;     /* [3][n] body frame */
} ms2_system;

/* Batch flags */
enum {
  MS2_BATCH_PLAIN_TILES = 1  /* tile shapes of the one-system-per-launch path
                                (many small work items per system) instead of
                                the batched shapes (fewer, larger items)      */
};

/* Creates a batch of at most max_slots concurrently resident systems whose
 * device state may use at most hbm_budget bytes (0 = no limit). */
ms2_status ms2_batch_create(ms2_ctx* ctx, int32_t max_slots, size_t hbm_budget, int32_t flags,
                            ms2_batch** out);
void ms2_batch_destroy(ms2_batch* batch);

/* Device bytes a slot for this system would occupy (state, scratch and
 * sampling buffers).  Pure host computation. */
ms2_status ms2_slot_footprint(ms2_ctx* ctx, const ms2_system* h_sys, size_t* bytes);

/* Admits a system into a free slot: allocates its device state, uploads
 * it on `stream` and evaluates its initial forces.  Returns MS2_EFULL when
 * no slot is free and MS2_ENOMEM when the HBM budget would be exceeded;
 * in both cases nothing changes. */
ms2_status ms2_slot_admit(ms2_batch* batch, const ms2_system* h_sys, int32_t* slot,
                          void* stream);

/* Frees a slot (waits for the stream the batch last ran on). */
ms2_status ms2_slot_retire(ms2_batch* batch, int32_t slot);

/* Step flags */
enum {
  MS2_STEP_GRAPH = 1,   /* capture the n_steps launches in a hipGraph and replay it */
  MS2_STEP_TIMING = 2,  /* record HIP events around the pair-kernel launches of
                           every step (inside the graph when captured)       */
  MS2_STEP_PREPARE = 4  /* with MS2_STEP_GRAPH: capture and instantiate the
                           graph for these n_steps and flags, run nothing    */
};

/* Advances every active slot by up to n_steps MD steps on the device: per
 * step a predictor (Gear) or drift (VV), the force path of ms2_forces and
 * ms2_ewald_kspace for all slots at once (Sec. 2: the partner search, energy
 * and force loops over molecules that dominate each step), the corrector,
 * the isokinetic thermostat and the samplers: Lustig moments every
 * sample_every steps (Sec. 3, Eq. 1), the RDF (Sec. 5, Eq. 2) and the
 * autocorrelation functions on the extended time step of acf_every MD steps
 * (Sec. 4, transport properties).  Integrators: velocity Verlet for point
 * molecules; for rigid molecules a 5-value Gear predictor-corrector of the
 * centres and of the quaternions with the body-frame Euler equations (the
 * paper leaves the integrator to its predecessor release; this is the
 * textbook scheme).  A slot whose own step budget runs out stops advancing.
 * Asynchronous; nothing is copied to the host.  Errors: MS2_EINVAL (NULL
 * batch, n_steps < 0), MS2_EDEVICE. */
ms2_status ms2_step(ms2_batch* batch, int32_t n_steps, int32_t flags, void* stream);

/* Elapsed time of the pair-kernel launches of the last ms2_step call made
 * with MS2_STEP_TIMING, summed over its steps (HIP events on that call's
 * stream), and the number of steps timed.  Synchronizes that stream. */
ms2_status ms2_batch_timing(ms2_batch* batch, double* pair_ms, int32_t* n_steps);

/* Samples copied out of a slot (host memory owned by the caller). */
typedef struct {
  int64_t steps_done;
  int32_t status;            /* MS2_OK or MS2_ENONFINITE                  */
  int32_t rdf_ntypes;        /* LJ site types; histograms for t1 <= t2    */
  double sums[MS2_NSUM];     /* force-path sums of the last step          */
  double ekin_trans, ekin_rot;
  double pairs_total;        /* accepted molecule pairs summed over all steps   */
  double site_pairs_total;   /* interacting site pairs summed over all steps    */
  double moments[11];        /* sums of X, X^2, X^3, Y, XY, X^2Y, Y^2, XY^2, Z, XZ
                                (slot 0 = number of samples); X = U - u0,
                                Y = dU/dV, Z = d2U/dV2                     */
  double solvation_sum;      /* sum over samples and solutes of the number of
                                solvent molecules inside the shell         */
  double solvation_cnt;      /* number of (sample, solute) terms in it     */
  double* h_rdf;             /* [npairtypes][rdf_bins] counts, or NULL     */
  double* h_acf_v;           /* [acf_nlag] sum over origins of (1/N) sum v(t0).v(t0+l n) */
  double* h_acf_j;           /* [acf_nlag] sum over origins of j_e(t0).j_e(t0+l n) */
  double* h_acf_cnt;         /* [acf_nlag] origins per lag                 */
  double* h_res_acf;         /* [acf_nlag] sum over (origin, solute) with a
                                non-empty shell at t0 of the fraction of its
                                initial shell still resident at lag l      */
  double* h_res_cnt;         /* [acf_nlag] number of those terms per lag   */
  double* h_acf_q;           /* [acf_nlag] sum over origins of J_q(t0).J_q(t0+l n) */
  double* h_acf_q_cnt;       /* [acf_nlag] origins per lag (an origin at step 0
                                carries no flux)                           */
  double* h_com;             /* optional [3][n] current state              */
  double* h_quat;            /* optional [4][n]                            */
  double* h_vel;             /* optional [3][n]                            */
  double* h_omega;           /* optional [3][n]                            */
  double* h_force;           /* optional [3][n] last force evaluation      */
  double* h_torque;          /* optional [3][n]                            */
} ms2_samples;

/* Copies a slot's accumulated samples and (optionally) its state to host
 * memory; synchronizes `stream`.  Lustig moments (Sec. 3, Eq. 1), RDF
 * (Sec. 5, Eq. 2), velocity and electric-current ACFs (Sec. 5, Eqs. 3-4),
 * residence-time correlation and solvation-number sums (Sec. 5, Eqs. 7-8),
 * heat-flux autocorrelation (Sec. 5, Eqs. 5-6).  The heat flux of rigid
 * molecules, J_q = sum_k (m v^2/2 + w.I.w/2 - h_k) v_k + sum over pairs of
 * u (v_k + v_l)/2 + R_kl (F_kl.(v_k + v_l) + tau_kl.w_k - tau_lk.w_l)/2, is
 * evaluated with each step's force evaluation (Gear: predicted state;
 * velocity Verlet: half-step velocities); lambda = (1/(3 V k T^2)) x the
 * integral of h_acf_q / h_acf_q_cnt.
 * Residence: at a time origin t0 every solvent molecule inside the shell of
 * a solute is tracked; it counts at lag l while inside the shell, unless it
 * has been outside for more than res_tolerance consecutive samples since t0
 * (then it never counts again for that origin).  tau = (sum of the lag means
 * of h_res_acf / h_res_cnt) x acf_every x dt by the trapezoid rule; the
 * solvation number is solvation_sum / solvation_cnt. */
ms2_status ms2_sample(ms2_batch* batch, int32_t slot, ms2_samples* h_out, void* stream);

/* Per-slot progress without copying samples: steps done, status. */
ms2_status ms2_slot_status(ms2_batch* batch, int32_t slot, int64_t* steps_done,
                           int32_t* status, void* stream);

/* Pair-kernel tile shape for n molecules: wave_rows waves of 64 molecules i
 * per block, j_chunk molecules j per work item (row-owned: every pair is
 * evaluated from both sides), or wave_rows = 0: symmetric items of 64 x 64
 * tile pairs, every pair evaluated once, with j_chunk = 64 / S for S = 1, 2
 * or 4 items per tile pair, each taking every S-th 64-pair chunk of the
 * pair's list (S > 1 puts more workgroups in flight for small systems, at
 * the price of S cut-off tests per tile pair).  The shape depends only on
 * the context's model class, the precision, the launch mode (0: one system
 * per launch, 1: batched) and the size bucket floor(log2 n) -- never on which
 * other systems share a launch.  Until ms2_autotune or ms2_set_tile_config
 * sets a bucket, both modes use symmetric items. */
ms2_status ms2_tile_config(ms2_ctx* ctx, int32_t mode, int32_t n_mol, int32_t precision,
                           int32_t* wave_rows, int32_t* j_chunk);
ms2_status ms2_set_tile_config(ms2_ctx* ctx, int32_t mode, int32_t n_mol, int32_t precision,
                               int32_t wave_rows, int32_t j_chunk);

/* Autotuner: for every size bucket between n_lo and n_hi and both launch
 * modes, times candidate tile shapes on the device with a synthetic lattice
 * system of species 0 (mode 1: a batch of copies filling the GPU) and keeps
 * the fastest.  Allocates and synchronizes; call before admitting systems.
 * h_report (optional, host) receives up to max_report rows of
 * (mode, bucket n, wave_rows, j_chunk, microseconds per system evaluation)
 * for every candidate timed; *n_report is set to the number of rows. */
ms2_status ms2_autotune(ms2_ctx* ctx, int32_t precision, int32_t n_lo, int32_t n_hi,
                        double* h_report, int32_t max_report, int32_t* n_report, void* stream);

/* Residual Massieu-potential derivatives (Sec. 3, Eq. 1):
 * A^r_mn = beta^m rho^n d^(m+n)(F^r/(N k T)) / d beta^m d rho^n, beta = 1/T,
 * rho = N/V, for the eight (m, n) the paper samples, from the moment sums of
 * one NVT run (ms2_samples.moments, shifted by u0 as in ms2_system.u0).
 * Molecular scaling: centres scale with the box, bodies stay rigid.  The
 * estimators are the canonical fluctuation formulas of
 * phi = ln INT exp(-beta U(s; V)) ds over the sampled configurations:
 * cumulants of U, dU/dV, d2U/dV2 up to third order.
 *   h_moments    host [11] sums (count, X, X^2, X^3, Y, XY, X^2Y, Y^2, XY^2, Z, XZ)
 *   u0           the shift X = U - u0 used while sampling
 *   temperature  k T (energy units of U), volume V, n_mol N
 *   h_ar         host [MS2_NAR] out, order MS2_AR_10 ... MS2_AR_12
 * Host arithmetic only (no device work).  MS2_EINVAL on a null pointer, no
 * samples, or a non-positive temperature, volume or N. */
enum { MS2_AR_10 = 0, MS2_AR_01, MS2_AR_20, MS2_AR_11, MS2_AR_02, MS2_AR_30, MS2_AR_21, MS2_AR_12,
       MS2_NAR };
ms2_status ms2_massieu(const double* h_moments, double u0, double temperature, double volume,
                       int32_t n_mol, double* h_ar);

/* Properties per molecule (k = 1) from A_mn = A^i_mn + A^r_mn, the ideal part
 * of classical rigid molecules with `dof` quadratic degrees of freedom
 * (3 translational + 0, 2 or 3 rotational): A^i_10 = dof/2, A^i_20 = -dof/2,
 * A^i_30 = dof, A^i_01 = 1, A^i_02 = -1, the mixed ones 0 (Sec. 3: for n > 0
 * the ideal part depends on the density only).
 *   h_ar     host [MS2_NAR] residual derivatives (ms2_massieu)
 *   h_props  host [MS2_NPROP] out: p/(rho k T); u/(k T); c_v/k; c_p/k;
 *            (dp/drho)_T/(k T); (dp/dT)_rho/(rho k); w^2 m/(k T) (speed of
 *            sound, m = molecular mass); rho k T kappa_T (isothermal
 *            compressibility)
 * MS2_EINVAL on a null pointer or dof <= 0. */
enum { MS2_PROP_Z = 0, MS2_PROP_U_KT, MS2_PROP_CV, MS2_PROP_CP, MS2_PROP_DPDRHO, MS2_PROP_DPDT,
       MS2_PROP_W2, MS2_PROP_KAPPA_T, MS2_NPROP };
ms2_status ms2_massieu_properties(const double* h_ar, double dof, double* h_props);

/* Thread-local message of the last failed call ("" if none). */
const char* ms2_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
