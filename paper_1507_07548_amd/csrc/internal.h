// Internal layout of the MI355X force/energy path: device tables, per-system
// parameters, per-slot buffer descriptors and pair-kernel work items.
// Shared by the HIP kernels and the host side of the C ABI only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ms2.h"

namespace ms2 {

// Half-space integer k vectors: n_x > 0, or n_x == 0 and n_y > 0, or
// n_x == n_y == 0 and n_z > 0, with 0 < |n|^2 <= kmax2.
struct KVec { int nx, ny, nz, n2; };

constexpr int kMaxSp = MS2_MAX_SPECIES;
constexpr int kMaxS = MS2_MAX_SITES;
constexpr int kNumBlockSums = 9;  // u_lj, u_el, us, uss, npair, nsite, J_q pair part (x, y, z) per work item
// Ewald blocks are single waves running long FP64 chains: short chunks give
// small systems enough waves in flight.
constexpr int kKChunk = 32;       // k vectors per reciprocal-force block
constexpr int kMolTile = 16;      // molecules per structure-factor block (16 x 4 charge slots = one wave)
constexpr int kMaxRdfTypes = 16;

// Model classes: compile-time upper bounds on the sites of each type per
// molecule, and whether every dipole/quadrupole sits at the centre of mass
// (then a multipole pair depends on R only through its direction and
// magnitude: r = R, and U_s = -p u, U_ss = p (p+1) u for u ~ r^-p).  Each
// class is one instantiation of the pair kernel; a context runs in the first
// class that covers all of its species.
struct ClassShape { int lj, ch, dp, qd, central; };
constexpr int kNumClasses = 6;
constexpr ClassShape kClassShapes[kNumClasses] = {
    {1, 0, 0, 0, 1},   // one-centre LJ
    {2, 0, 0, 1, 1},   // two-centre LJ + linear quadrupole at the centre
    {1, 3, 0, 0, 1},   // LJ + up to three charges (water-like, ions)
    {1, 0, 1, 0, 1},   // Stockmayer (dipole at the centre)
    {2, 2, 1, 1, 0},   // small mixed, multipoles anywhere
    {4, 4, 2, 2, 0},   // general
};
__host__ __device__ constexpr int class_lj(int c) { return kClassShapes[c].lj; }
__host__ __device__ constexpr int class_reals(int c) {
  return 3 * (kClassShapes[c].lj + kClassShapes[c].ch) + 6 * (kClassShapes[c].dp + kClassShapes[c].qd);
}

// Species table, grouped by site type (order within a type kept).
struct SpeciesDev {
  int nlj, nch, ndp, nqd;
  int rot_dof;      // number of non-zero principal moments
  int lj_type0;     // first RDF LJ-site type index of this species
  double mass;
  double inertia[3];
  double net_charge;
  double lj_pos[kMaxS][3];
  double ch_pos[kMaxS][3];
  double dp_pos[kMaxS][3], dp_axis[kMaxS][3];
  double qd_pos[kMaxS][3], qd_axis[kMaxS][3];
  double ch_q[kMaxS], dp_mu[kMaxS], qd_Q[kMaxS];
  double lj_sigma[kMaxS], lj_eps[kMaxS];
};

struct SpeciesTable {
  int nsp;
  int n_lj_types;
  int nsite_pair[kMaxSp][kMaxSp];                  // interacting site pairs per molecule pair
  SpeciesDev sp[kMaxSp];
  // 4 eps sigma^6 and 4 eps sigma^12 for LJ site a of A and b of B
  double c6[kMaxSp][kMaxS][kMaxSp][kMaxS];
  double c12[kMaxSp][kMaxS][kMaxSp][kMaxS];
};

// Per-system constants derived on the host from ms2_params.
struct SysParams {
  double L, invL, rc, rc2, V;
  double ke, inv_ke, krf, crf;                     // inv_ke = 1 / ke
  double alpha, alpha2, gpref;                     // gpref = 2 alpha / sqrt(pi)
  int elec, kmax2, nk, lrc;
  int precision, cls, nsp;
  int site_cut;                                    // 1: LJ site pairs cut at their own distance
  double rc2_search;                               // squared centre distance a pair needs to be listed
  // LJ tail per species pair: multiply by N_A N_B (already includes 2 pi / V)
  double lrc_u[kMaxSp][kMaxSp], lrc_us[kMaxSp][kMaxSp], lrc_uss[kMaxSp][kMaxSp];
  double ew_const[kMaxSp];                         // self + intramolecular per molecule
};

// Per-slot buffers (device pointers) and bookkeeping.
struct SlotDev {
  int n, npad;
  int jsplits, nitems;
  int active;                 // 0: skipped by every kernel
  int kchunks, mchunks;       // Ewald force / structure-factor partial counts
  int com_ld;                 // row length of com/quat/force/torque (and slot state) arrays
  int symmetric;              // 1: symmetric tile-pair items (each pair once)
  int pf_single;              // 1: pair partials in FP32 (the FP32 form), 0: FP64
  int heat_flux;              // 1: the pair kernel adds the pair part of the heat flux
  int pad_hf;
  const double* hf_v;         // [3][com_ld] velocity source (x hf_vscale), heat flux only
  const double* hf_w;         // [3][com_ld] body angular velocity, or NULL
  double hf_vscale;
  void* hf_kin;               // [6][npad] Real: lab v and w at the force evaluation
  double* jq;                 // [3] pair part of the heat flux of the last evaluation
  const int* species;
  const double* com;          // [3][com_ld]
  const double* quat;         // [4][com_ld]
  void* sites;                // [class_reals][npad] Real
  double* lj64;               // site-site cut-off: [3 * class LJ sites][npad] FP64 LJ-site offsets, else NULL
  void* pf;                   // [jsplits][6][npad] pair partial F, tau, in the slot's Real
  double* bsum;               // [nitems][kNumBlockSums]
  double* force;              // [3][com_ld]
  double* torque;             // [3][com_ld]
  double* sums;               // [MS2_NSUM]
  double* sk_part;            // [mchunks][nk][2] structure-factor partials
  double* sk;                 // [nk][2]
  double* fk;                 // [kchunks][6][npad] reciprocal partial F, tau
  double* kred;               // [kchunks][kblocks_m] sum_a d_a . F_a partials + [2] U, W_atomic
  double* ksum;               // [4]: U_recip, W_atomic, sum d.F, spare
  const struct KVec* kvec;    // [nk] half-space integer vectors
  int nk, mtiles;             // k vectors; kMolTile-molecule tiles of the reciprocal-force kernel
  int* err;                   // device error word (1: a species index outside the table), or NULL
};

// Forms of the symmetric pair kernel, chosen per context (never per batch
// mix): any species; one species with a site of every kind its class holds;
// one linear two-centre LJ + quadrupole species (both LJ sites, equal, on
// the quadrupole's axis at +-h, the quadrupole at the centre).
enum PairForm { kFormGeneral = 0, kFormOneSpecies = 1, kFormLinear = 2 };

// Species indices come from caller memory.  Every load clamps them into the
// table so a bad index can never address outside it; the kernels that end
// a call (the force and sum reductions, the structure factor) also test them
// and turn a bad index into NaN outputs and the slot's error word.
__host__ __device__ inline int clamp_species(int s, int nsp) {
  return s < 0 ? 0 : (s >= nsp ? nsp - 1 : s);
}
__host__ __device__ inline bool species_ok(int s, int nsp) { return (unsigned)s < (unsigned)nsp; }

// A pair-kernel work item: molecules [i0, i0 + 64 W) of a slot against
// j in [j0, j1); `part` selects the per-molecule partial buffer of the i
// side, `part_j` that of the j side (symmetric items), `local` the item's
// block-sum row within its slot.  `split` (symmetric items): a tile pair's
// pair list may be dealt to S items, this one taking its chunks s, s + S,
// ...; split = s + 256 S, and 0 stands for s = 0, S = 1.
struct WorkItem {
  int slot, i0, j0, j1, part, local, part_j, split;
};
__host__ __device__ inline int split_count(int split) { return split >> 8 > 1 ? split >> 8 : 1; }
__host__ __device__ inline int split_index(int split) { return split & 255; }
constexpr int kMaxSplits = 4;   // symmetric items per tile pair

constexpr int kNumMoments = 11;   // N, X, X^2, X^3, Y, XY, X^2Y, Y^2, XY^2, Z, XZ
constexpr int kMdThreads = 1024;  // one block per slot for the per-system passes of the MD step
constexpr int kMdBlock = 256;     // threads per block of the per-molecule MD kernels

// Per-slot integrator and sampler state (device memory).
struct MDDev {
  int active;            // 1 while steps_done < steps_target and status == OK
  int integrator;        // MS2_VV or MS2_GEAR
  int rotating;          // any species with a non-zero moment of inertia
  int status;            // MS2_OK or MS2_ENONFINITE
  long long steps_done, steps_target;
  double dt, temperature;
  double f_tr, f_rot;    // translational / rotational degrees of freedom
  int sample_every, rdf_every, rdf_bins, rdf_due;
  int acf_every, acf_origin_every, acf_nlag, acf_max_live;
  int n_origins, rdf_ntp, pad0, pad1;
  double rdf_rmax, rdf_inv_dr, rdf_reach2, u0;
  double ekin_tr, ekin_rot;
  double scale_tr, scale_rot;  // this step's isokinetic factors (1 without a thermostat)
  double pairs_total, site_pairs_total;
  double* r;             // Gear translation [5][3][n] (r, dt v, dt^2 a/2, ...); VV: r[0]
  double* q;             // Gear quaternion  [5][4][n]
  double* w;             // Gear body angular velocity [5][3][n]
  double* vel;           // velocities [3][n] (VV state; Gear: r1/dt for the samplers)
  double* moments;       // [kNumMoments]
  double* md_part;       // [ceil(n / kMdBlock)][8] per-block partial sums of the step's end
  unsigned long long* rdf;  // [rdf_ntp][rdf_bins] counts
  double* acf_v;         // [acf_nlag]
  double* acf_j;         // [acf_nlag]
  double* acf_cnt;       // [acf_nlag]
  double* origin_v;      // [acf_max_live][3][n]
  double* origin_j;      // [acf_max_live][3]
  long long* origin_t0;  // [acf_max_live]
  // residence time and solvation number, on the ACF schedule
  int res_on, res_tol, n_solute, n_solvent;
  int res_due, pad2;     // res_due: a residence sample is pending for step res_step
  long long res_step;
  double res_r2;
  double res_solv_sum, res_solv_cnt;
  const int* res_solute_idx;   // [n_solute] molecule indices
  const int* res_solvent_idx;  // [n_solvent]
  unsigned short* res_state;   // [acf_max_live][n_solute][n_solvent]
  int* res_n0;                 // [acf_max_live][n_solute] shell population at the origin
  double* res_part;            // [n_solute][acf_max_live] per-solute fraction (staging)
  int* res_inside;             // [n_solute] shell population now (staging)
  double* res_acf;             // [acf_nlag]
  double* res_cnt;             // [acf_nlag]
  // heat-flux autocorrelation, on the ACF schedule
  int hf_on, pad3;
  double h_partial[kMaxSp];    // partial enthalpy per molecule of each species
  double jq_now[3];            // J_q of this step's force evaluation
  double* acf_q;               // [acf_nlag]
  double* acf_q_cnt;           // [acf_nlag]
  double* origin_jq;           // [acf_max_live][3]
  int* origin_jq_valid;        // [acf_max_live]
};

// residence state word: the pair no longer counts for this origin
constexpr unsigned short kResDead = 0xFFFF;
constexpr int kResMaxLive = 64;    // live ACF origins supported with residence sampling


}  // namespace ms2
