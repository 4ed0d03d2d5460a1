// Device-resident MD step for many independent systems (slots) at once:
// integrators, isokinetic thermostat and the on-the-fly samplers.
//
//   md_wrap_kernel     wrap the uploaded centres into [0, L)
//   md_init_kernel     Gear start-up derivatives from the first force
//                      evaluation; kinetic energies; ACF sample at t = 0
//   md_begin_frame_kernel
//                      Gear predictor (Pascal triangle) and unit-quaternion
//                      projection, or the first velocity-Verlet kick + drift;
//                      then the site frame of the predicted state
//   md_correct_kernel, md_finish_kernel
//                      the step's end: Gear corrector (5-value coefficients
//                      for second-order translation and first-order
//                      quaternion/Euler systems) or the second kick;
//                      isokinetic rescaling; Lustig moment sums (the paper's
//                      Sec. 3, Eq. 1 needs averages of U, dU/dV, d2U/dV2 and
//                      their products); velocity and electric-current
//                      autocorrelation on the extended time step (Sec. 4;
//                      Sec. 5, Eqs. 3-4)
//   rdf_kernel         site-site radial distribution histogram between LJ
//                      sites (Sec. 5, Eq. 2), FP64 distances, integer counts
//   residence_kernel   residence-time correlation and solvation number
//                      (Sec. 5, Eqs. 7-8) on the extended time step
// Every reduction (kinetic energy, ACF dot products) is a fixed-order tree:
// in-block for the per-system passes (one 1024-thread block per slot), block
// partials summed in block order for the per-molecule kernels.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "quat.h"
#include "site_frame.h"

namespace ms2 {

// d/dt of the quaternion for a body-frame angular velocity: (1/2) q (x) (0, w)
__device__ __forceinline__ void quat_rate(const double* q, const double* w, double* out) {
  out[0] = 0.5 * (-q[1] * w[0] - q[2] * w[1] - q[3] * w[2]);
  out[1] = 0.5 * (q[0] * w[0] + q[2] * w[2] - q[3] * w[1]);
  out[2] = 0.5 * (q[0] * w[1] - q[1] * w[2] + q[3] * w[0]);
  out[3] = 0.5 * (q[0] * w[2] + q[1] * w[1] - q[2] * w[0]);
}

// Euler's equations in the principal frame; a zero moment freezes its axis
__device__ __forceinline__ void euler_rate(const double* I, const double* tb, const double* w,
                                           double* wd) {
  wd[0] = I[0] > 0.0 ? (tb[0] + (I[1] - I[2]) * w[1] * w[2]) / I[0] : 0.0;
  wd[1] = I[1] > 0.0 ? (tb[1] + (I[2] - I[0]) * w[2] * w[0]) / I[1] : 0.0;
  wd[2] = I[2] > 0.0 ? (tb[2] + (I[0] - I[1]) * w[0] * w[1]) / I[2] : 0.0;
}

// body-frame torque A^T tau
__device__ __forceinline__ void body_torque(const double A[3][3], const double* t, double* tb) {
  for (int k = 0; k < 3; ++k) tb[k] = A[0][k] * t[0] + A[1][k] * t[1] + A[2][k] * t[2];
}

__device__ __forceinline__ double wrap(double x, double L, double invL) {
  return x - L * floor(x * invL);
}

// block-wide fixed-order sum over kMdThreads threads
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  __syncthreads();
  red[tid] = v;
  __syncthreads();
  for (int h = kMdThreads / 2; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// wraps the uploaded centres of one slot into [0, L)
__global__ __launch_bounds__(256) void md_wrap_kernel(MDDev* md, const SysParams* prm, int slot, int n) {
  const MDDev& m = md[slot];
  const SysParams& P = prm[slot];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < 3; ++c) m.r[c * n + i] = wrap(m.r[c * n + i], P.L, P.invL);
}

// ACF sample at the current state: v is [3][npad].  have_jq: m.jq_now holds
// this step's heat flux (there is none for the initial state).
__device__ void acf_sample(MDDev& m, const SpeciesTable* tab, const SlotDev& sd, const double* v,
                           int npad, long long s, double* red, bool have_jq) {
  const int tid = threadIdx.x, n = sd.n;
  double jl[3] = {0, 0, 0};
  for (int i = tid; i < n; i += kMdThreads) {
    const double q = tab->sp[clamp_species(sd.species[i], tab->nsp)].net_charge;
    for (int c = 0; c < 3; ++c) jl[c] += q * v[c * npad + i];
  }
  double j[3];
  for (int c = 0; c < 3; ++c) j[c] = block_sum(jl[c], red);
  if (s % m.acf_origin_every == 0) {
    const int slot_o = m.n_origins % m.acf_max_live;
    double* ov = m.origin_v + (size_t)slot_o * 3 * npad;
    for (int i = tid; i < n; i += kMdThreads)
      for (int c = 0; c < 3; ++c) ov[c * npad + i] = v[c * npad + i];
    if (tid == 0) {
      m.origin_t0[slot_o] = s;
      for (int c = 0; c < 3; ++c) m.origin_j[3 * slot_o + c] = j[c];
      if (m.hf_on) {
        m.origin_jq_valid[slot_o] = have_jq ? 1 : 0;
        for (int c = 0; c < 3; ++c) m.origin_jq[3 * slot_o + c] = have_jq ? m.jq_now[c] : 0.0;
      }
    }
    __syncthreads();
    if (tid == 0) m.n_origins += 1;
    __syncthreads();
  }
  const int live = m.n_origins < m.acf_max_live ? m.n_origins : m.acf_max_live;
  for (int o = 0; o < live; ++o) {
    const long long t0 = m.origin_t0[o];
    if (s < t0) continue;
    const long long lag = (s - t0) / m.acf_every;
    if (lag >= m.acf_nlag) continue;
    const double* ov = m.origin_v + (size_t)o * 3 * npad;
    double d = 0.0;
    for (int i = tid; i < n; i += kMdThreads)
      for (int c = 0; c < 3; ++c) d += ov[c * npad + i] * v[c * npad + i];
    d = block_sum(d, red);
    if (tid == 0) {
      m.acf_v[lag] += d / n;
      m.acf_j[lag] += m.origin_j[3 * o] * j[0] + m.origin_j[3 * o + 1] * j[1] +
                      m.origin_j[3 * o + 2] * j[2];
      m.acf_cnt[lag] += 1.0;
      if (m.hf_on && have_jq && m.origin_jq_valid[o]) {
        m.acf_q[lag] += m.origin_jq[3 * o] * m.jq_now[0] + m.origin_jq[3 * o + 1] * m.jq_now[1] +
                        m.origin_jq[3 * o + 2] * m.jq_now[2];
        m.acf_q_cnt[lag] += 1.0;
      }
    }
  }
}

// translational and rotational kinetic sums: sum m v^2, sum I w^2
__device__ void kinetic(const MDDev& m, const SpeciesTable* tab, const SlotDev& sd, const double* v,
                        int npad, double* red, double& k2, double& kr2) {
  const int tid = threadIdx.x, n = sd.n;
  double a = 0.0, b = 0.0;
  for (int i = tid; i < n; i += kMdThreads) {
    const SpeciesDev& D = tab->sp[clamp_species(sd.species[i], tab->nsp)];
    for (int c = 0; c < 3; ++c) {
      a += D.mass * v[c * npad + i] * v[c * npad + i];
      if (m.rotating) b += D.inertia[c] * m.w[c * npad + i] * m.w[c * npad + i];
    }
  }
  k2 = block_sum(a, red);
  kr2 = block_sum(b, red);
}

// one block per slot, launched for a single slot after its first force evaluation
__global__ __launch_bounds__(kMdThreads) void md_init_kernel(SlotDev* slots, MDDev* md,
                                                             const SpeciesTable* __restrict__ tab,
                                                             int slot) {
  __shared__ double red[kMdThreads];
  SlotDev& sd = slots[slot];
  MDDev& m = md[slot];
  const int tid = threadIdx.x, n = sd.n, np = sd.com_ld;
  const double dt = m.dt;
  double* vnow;
  if (m.integrator == MS2_GEAR) {
    // r1 holds the uploaded velocity; w0 the uploaded body angular velocity
    for (int i = tid; i < n; i += kMdThreads) {
      const SpeciesDev& D = tab->sp[clamp_species(sd.species[i], tab->nsp)];
      for (int c = 0; c < 3; ++c) {
        const double v = m.r[(1 * 3 + c) * np + i];
        m.r[(1 * 3 + c) * np + i] = dt * v;
        m.r[(2 * 3 + c) * np + i] = 0.5 * dt * dt * sd.force[c * sd.com_ld + i] / D.mass;
        m.r[(3 * 3 + c) * np + i] = 0.0;
        m.r[(4 * 3 + c) * np + i] = 0.0;
        if (m.vel) m.vel[c * np + i] = v;
      }
      if (m.rotating) {
        double q[4], w[3], tq[3], tb[3], wd[3], qd[4], A[3][3];
        for (int c = 0; c < 4; ++c) q[c] = m.q[c * np + i];
        for (int c = 0; c < 3; ++c) {
          w[c] = m.w[c * np + i];
          tq[c] = sd.torque[c * sd.com_ld + i];
        }
        quat_matrix(q[0], q[1], q[2], q[3], A);
        body_torque(A, tq, tb);
        euler_rate(D.inertia, tb, w, wd);
        quat_rate(q, w, qd);
        for (int c = 0; c < 3; ++c) {
          m.w[(1 * 3 + c) * np + i] = dt * wd[c];
          m.w[(2 * 3 + c) * np + i] = 0.0;
          m.w[(3 * 3 + c) * np + i] = 0.0;
          m.w[(4 * 3 + c) * np + i] = 0.0;
        }
        for (int c = 0; c < 4; ++c) {
          m.q[(1 * 4 + c) * np + i] = dt * qd[c];
          m.q[(2 * 4 + c) * np + i] = 0.0;
          m.q[(3 * 4 + c) * np + i] = 0.0;
          m.q[(4 * 4 + c) * np + i] = 0.0;
        }
      }
    }
    vnow = m.vel;   // scratch copy of the velocities for the samplers
  } else {
    vnow = m.vel;
  }
  __syncthreads();
  double k2, kr2;
  kinetic(m, tab, sd, vnow, np, red, k2, kr2);
  if (tid == 0) {
    m.ekin_tr = 0.5 * k2;
    m.ekin_rot = 0.5 * kr2;
  }
  if (m.acf_every > 0) acf_sample(m, tab, sd, vnow, np, 0, red, false);
  if (tid == 0 && m.res_on) {
    m.res_due = 1;
    m.res_step = 0;
  }
}

// ---------------------------------------------------------------------------
// Gear predictor on the scaled derivatives y_d = dt^d y^(d) / d! of each
// component: y_d <- sum over e >= d of C(e, d) y_e (Pascal triangle)
template <int NC>
__device__ __forceinline__ void gear_predict(double (&a)[5][NC]) {
  for (int c = 0; c < NC; ++c) {
    const double y0 = a[0][c], y1 = a[1][c], y2 = a[2][c], y3 = a[3][c], y4 = a[4][c];
    a[0][c] = y0 + y1 + y2 + y3 + y4;
    a[1][c] = y1 + 2.0 * y2 + 3.0 * y3 + 4.0 * y4;
    a[2][c] = y2 + 3.0 * y3 + 6.0 * y4;
    a[3][c] = y3 + 4.0 * y4;
  }
}

// Predictor (Gear) or first kick and drift (velocity Verlet) of molecule i.
__device__ __forceinline__ void md_begin_molecule(const SlotDev& sd, const MDDev& m, const SysParams& P,
                                                  const SpeciesTable* __restrict__ tab, int i) {
  const int np = sd.com_ld;
  if (m.integrator == MS2_GEAR) {
    // every load of the molecule's state is issued before the first store
    // (the rows of an array lie np apart, which the compiler cannot prove
    // non-zero); Pascal-triangle predictor on the 5 scaled derivatives of
    // each component; row 4 is unchanged
    const bool rotating = m.rotating;
    double* __restrict__ const r = m.r;
    double* __restrict__ const w = m.w;
    double* __restrict__ const q = m.q;
    double R[5][3], W[5][3], Q[5][4];
    for (int d = 0; d < 5; ++d)
      for (int c = 0; c < 3; ++c) R[d][c] = r[(d * 3 + c) * np + i];
    if (rotating)
      for (int d = 0; d < 5; ++d) {
        for (int c = 0; c < 3; ++c) W[d][c] = w[(d * 3 + c) * np + i];
        for (int c = 0; c < 4; ++c) Q[d][c] = q[(d * 4 + c) * np + i];
      }
    gear_predict(R);
    for (int d = 0; d < 4; ++d)
      for (int c = 0; c < 3; ++c) r[(d * 3 + c) * np + i] = R[d][c];
    if (rotating) {
      gear_predict(W);
      gear_predict(Q);
      // the force evaluation uses the predicted orientation projected onto |q| = 1
      const double nq = sqrt(Q[0][0] * Q[0][0] + Q[0][1] * Q[0][1] + Q[0][2] * Q[0][2] + Q[0][3] * Q[0][3]);
      for (int c = 0; c < 4; ++c) Q[0][c] = Q[0][c] / nq;
      for (int d = 0; d < 4; ++d) {
        for (int c = 0; c < 3; ++c) w[(d * 3 + c) * np + i] = W[d][c];
        for (int c = 0; c < 4; ++c) q[(d * 4 + c) * np + i] = Q[d][c];
      }
    }
  } else {
    const double h = 0.5 * m.dt / tab->sp[clamp_species(sd.species[i], tab->nsp)].mass;
    for (int c = 0; c < 3; ++c) {
      const double v = m.vel[c * np + i] + h * sd.force[c * sd.com_ld + i];
      m.vel[c * np + i] = v;
      m.r[c * np + i] = wrap(m.r[c * np + i] + m.dt * v, P.L, P.invL);
    }
  }
}

// Start of a step in one launch per precision: the predictor of each
// molecule, then the site frame of the predicted state (the force path's
// first kernel), by the same thread.  Slots of the other precision are left
// to the other launch.
template <typename Real, int C>
__global__ __launch_bounds__(256) void md_begin_frame_kernel(const SlotDev* __restrict__ slots, MDDev* md,
                                                             const SysParams* __restrict__ prm,
                                                             const SpeciesTable* __restrict__ tab) {
  const SlotDev& sd = slots[blockIdx.y];
  const MDDev& m = md[blockIdx.y];
  const SysParams& P = prm[blockIdx.y];
  if (P.precision != (sizeof(Real) == 4 ? MS2_FP32 : MS2_FP64)) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= sd.n) return;
  if (m.active) md_begin_molecule(sd, m, P, tab, i);
  // the site frame reads the predicted centre and quaternion this thread
  // has just stored: no reordering of memory accesses across this point
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if (sd.active) site_frame_molecule<Real, C>(sd, tab, i);
}

// ---------------------------------------------------------------------------
// End of the step, in two launches:
//   md_correct_kernel  (molecule blocks x slots) heat-flux kinetic part of the
//                      predicted state when due, corrector (or second kick),
//                      per-block fixed-order partials of sum m v^2, sum I w^2
//                      and the heat-flux part
//   md_finish_kernel   (one block per slot) the partials summed in block
//                      order; isokinetic factors; kinetic energies, totals,
//                      Lustig moments, RDF flag, status; the factors applied
//                      to every molecule; ACF sample when due; step count,
//                      end of run
// ---------------------------------------------------------------------------

// fixed-order sums of NV values over the kMdBlock threads of a block; every
// thread gets the sums
template <int NV>
__device__ void block_sums(double* v, double (*red)[kMdBlock]) {
  const int tid = threadIdx.x;
  for (int k = 0; k < NV; ++k) red[k][tid] = v[k];
  __syncthreads();
  for (int h = kMdBlock / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int k = 0; k < NV; ++k) red[k][tid] += red[k][tid + h];
    __syncthreads();
  }
  for (int k = 0; k < NV; ++k) v[k] = red[k][0];
}

__device__ __forceinline__ bool hf_due(const MDDev& m) {
  return m.hf_on && m.acf_every > 0 && (m.steps_done + 1) % m.acf_every == 0;
}

// Gear corrector of molecule i (5-value coefficients ct for the second-order
// translation, cr for the first-order quaternion and Euler systems; the
// state arrays are distinct allocations, passed as restrict pointers so that
// loads may pass stores), or the second velocity-Verlet kick.  Returns the
// corrected velocity and (rotating Gear) body angular velocity in vo, wo.
__device__ __forceinline__ void correct_molecule(const MDDev& m, const SpeciesDev& D, const SysParams& P, int i,
                                                 int np, int ld, double* __restrict__ gr, double* __restrict__ gw,
                                                 double* __restrict__ gq, double* __restrict__ gv,
                                                 const double* __restrict__ gf, const double* __restrict__ gt,
                                                 double* vo, double* wo) {
  const double dt = m.dt;
  const double ct[5] = {19.0 / 120.0, 3.0 / 4.0, 1.0, 1.0 / 2.0, 1.0 / 12.0};
  const double cr[5] = {251.0 / 720.0, 1.0, 11.0 / 12.0, 1.0 / 3.0, 1.0 / 24.0};
  if (m.integrator == MS2_GEAR) {
    // the whole state of the molecule is loaded before the first store: the
    // rows of one array lie np apart, a distance the compiler cannot prove
    // non-zero, so updates in place would chain each load behind the
    // previous store
    const bool rotating = m.rotating;
    const double mass = D.mass, L = P.L, invL = P.invL;
    double R[5][3], F[3], W[5][3], Q[5][4], T[3];
    for (int d = 0; d < 5; ++d)
      for (int c = 0; c < 3; ++c) R[d][c] = gr[(d * 3 + c) * np + i];
    for (int c = 0; c < 3; ++c) F[c] = gf[c * ld + i];
    if (rotating) {
      for (int d = 0; d < 5; ++d) {
        for (int c = 0; c < 3; ++c) W[d][c] = gw[(d * 3 + c) * np + i];
        for (int c = 0; c < 4; ++c) Q[d][c] = gq[(d * 4 + c) * np + i];
      }
      for (int c = 0; c < 3; ++c) T[c] = gt[c * ld + i];
    }
    for (int c = 0; c < 3; ++c) {
      const double delta = 0.5 * dt * dt * F[c] / mass - R[2][c];
      for (int d = 0; d < 5; ++d) R[d][c] += ct[d] * delta;
    }
    if (rotating) {
      double wd[3], qd[4], tb[3], A[3][3];
      quat_matrix(Q[0][0], Q[0][1], Q[0][2], Q[0][3], A);
      body_torque(A, T, tb);
      euler_rate(D.inertia, tb, W[0], wd);
      quat_rate(Q[0], W[0], qd);
      for (int c = 0; c < 3; ++c) {
        const double delta = dt * wd[c] - W[1][c];
        for (int d = 0; d < 5; ++d) W[d][c] = W[d][c] + cr[d] * delta;
        wo[c] = W[0][c];
      }
      for (int c = 0; c < 4; ++c) {
        const double delta = dt * qd[c] - Q[1][c];
        for (int d = 0; d < 5; ++d) Q[d][c] += cr[d] * delta;
      }
      const double nq = sqrt(Q[0][0] * Q[0][0] + Q[0][1] * Q[0][1] + Q[0][2] * Q[0][2] + Q[0][3] * Q[0][3]);
      for (int c = 0; c < 4; ++c) Q[0][c] = Q[0][c] / nq;
      for (int d = 0; d < 5; ++d) {
        for (int c = 0; c < 3; ++c) gw[(d * 3 + c) * np + i] = W[d][c];
        for (int c = 0; c < 4; ++c) gq[(d * 4 + c) * np + i] = Q[d][c];
      }
    }
    for (int c = 0; c < 3; ++c) {
      R[0][c] = wrap(R[0][c], L, invL);
      vo[c] = R[1][c] / dt;
    }
    for (int d = 0; d < 5; ++d)
      for (int c = 0; c < 3; ++c) gr[(d * 3 + c) * np + i] = R[d][c];
    for (int c = 0; c < 3; ++c) gv[c * np + i] = vo[c];
  } else {
    const double h = 0.5 * dt / D.mass;
    for (int c = 0; c < 3; ++c) {
      vo[c] = gv[c * np + i] + h * gf[c * ld + i];
      gv[c * np + i] = vo[c];
    }
  }
}

__global__ __launch_bounds__(kMdBlock) void md_correct_kernel(SlotDev* slots, MDDev* md,
                                                              const SysParams* __restrict__ prm,
                                                              const SpeciesTable* __restrict__ tab) {
  __shared__ double red[5][kMdBlock];
  SlotDev& sd = slots[blockIdx.y];
  MDDev& m = md[blockIdx.y];
  const int n = sd.n;
  if (!m.active || (int)blockIdx.x * kMdBlock >= n) return;   // uniform over the block
  const SysParams& P = prm[blockIdx.y];
  const int i = blockIdx.x * kMdBlock + threadIdx.x, np = sd.com_ld, ld = sd.com_ld;
  double part[5] = {0.0, 0.0, 0.0, 0.0, 0.0};   // sum m v^2, sum I w^2, heat-flux kinetic part
  if (i < n) {
    const int spi = clamp_species(sd.species[i], tab->nsp);
    const SpeciesDev& D = tab->sp[spi];
    double* v = m.vel;
    if (hf_due(m)) {
      // heat flux of this step's force evaluation (still the predicted
      // state): (m v^2/2 + w.I.w/2 - h_k) v_k of the molecule
      double vi[3], e = 0.0;
      for (int c = 0; c < 3; ++c) {
        vi[c] = m.integrator == MS2_GEAR ? m.r[(1 * 3 + c) * np + i] / m.dt : v[c * np + i];
        e += 0.5 * D.mass * vi[c] * vi[c];
      }
      if (m.integrator == MS2_GEAR && m.rotating)
        for (int c = 0; c < 3; ++c) e += 0.5 * D.inertia[c] * m.w[c * np + i] * m.w[c * np + i];
      e -= m.h_partial[spi];
      for (int c = 0; c < 3; ++c) part[2 + c] = e * vi[c];
    }
    double vo[3], wo[3];
    correct_molecule(m, D, P, i, np, ld, m.r, m.w, m.q, v, sd.force, sd.torque, vo, wo);
    if (m.rotating && m.integrator != MS2_GEAR)
      for (int c = 0; c < 3; ++c) wo[c] = m.w[c * np + i];
    for (int c = 0; c < 3; ++c) {
      part[0] += D.mass * vo[c] * vo[c];
      if (m.rotating) part[1] += D.inertia[c] * wo[c] * wo[c];
    }
  }
  block_sums<5>(part, red);
  if (threadIdx.x == 0) {
    double* o = m.md_part + (size_t)blockIdx.x * 8;
    for (int k = 0; k < 5; ++k) o[k] = part[k];
  }
}

// The thermostat's tail (one thread): the kinetic sums v (m v^2, I w^2, the
// heat flux's kinetic part) give the isokinetic factors, kinetic energies,
// Lustig moments, the RDF flag and the status.
__device__ void thermo_tail(SlotDev& sd, MDDev& m, const SysParams& P, const double* v) {
  if (hf_due(m))
    for (int c = 0; c < 3; ++c) m.jq_now[c] = v[2 + c] + sd.jq[c];
  double k2 = v[0], kr2 = v[1], ft = 1.0, fr = 1.0;
  if (m.temperature > 0.0) {
    ft = sqrt(m.temperature * m.f_tr / k2);
    fr = (m.f_rot > 0.0 && kr2 > 0.0) ? sqrt(m.temperature * m.f_rot / kr2) : 1.0;
    k2 *= ft * ft;
    kr2 *= fr * fr;
  }
  m.scale_tr = ft;
  m.scale_rot = fr;
  const long long s = m.steps_done + 1;
  m.ekin_tr = 0.5 * k2;
  m.ekin_rot = 0.5 * kr2;
  const double* su = sd.sums;
  m.pairs_total += su[MS2_SUM_NPAIR];
  m.site_pairs_total += su[MS2_SUM_NSITE];
  const double U = su[MS2_SUM_U_LJ] + su[MS2_SUM_U_ELEC] + su[MS2_SUM_U_RECIP] + su[MS2_SUM_U_CONST] +
                   su[MS2_SUM_U_LRC];
  const bool ok = isfinite(U) && isfinite(k2) && isfinite(su[MS2_SUM_VIRIAL]);
  if (m.sample_every > 0 && s % m.sample_every == 0) {
    const double X = U - m.u0;
    const double us = su[MS2_SUM_US] + su[MS2_SUM_US_LRC];
    const double uss = su[MS2_SUM_USS] + su[MS2_SUM_USS_LRC];
    const double Y = us / (3.0 * P.V);
    const double Z = (uss - 2.0 * us) / (9.0 * P.V * P.V);
    double* mo = m.moments;
    mo[0] += 1.0;
    mo[1] += X;
    mo[2] += X * X;
    mo[3] += X * X * X;
    mo[4] += Y;
    mo[5] += X * Y;
    mo[6] += X * X * Y;
    mo[7] += Y * Y;
    mo[8] += X * Y * Y;
    mo[9] += Z;
    mo[10] += X * Z;
  }
  m.rdf_due = (m.rdf_every > 0 && s % m.rdf_every == 0) ? 1 : 0;
  if (!ok) m.status = MS2_ENONFINITE;
}

// The isokinetic factors applied to molecule i (velocities, the Gear
// state's first derivatives).
__device__ __forceinline__ void rescale_molecule(MDDev& m, int np, int i, double ft, double fr) {
  const bool gear = m.integrator == MS2_GEAR, rot = m.rotating && fr != 1.0;
  double* __restrict__ const gv = m.vel;
  double* __restrict__ const gr = m.r;
  double* __restrict__ const gw = m.w;
  double* __restrict__ const gq = m.q;
  // all loads before the first store (see md_begin_molecule)
  double v[3], r1[3], w1[3], q1[4];
  for (int c = 0; c < 3; ++c) {
    v[c] = gv[c * np + i];
    if (gear) r1[c] = gr[(1 * 3 + c) * np + i];
  }
  if (rot) {
    for (int c = 0; c < 3; ++c) w1[c] = gw[c * np + i];
    for (int c = 0; c < 4; ++c) q1[c] = gq[(1 * 4 + c) * np + i];
  }
  for (int c = 0; c < 3; ++c) {
    gv[c * np + i] = v[c] * ft;
    if (gear) gr[(1 * 3 + c) * np + i] = r1[c] * ft;
  }
  if (rot) {
    for (int c = 0; c < 3; ++c) gw[c * np + i] = w1[c] * fr;
    for (int c = 0; c < 4; ++c) gq[(1 * 4 + c) * np + i] = q1[c] * fr;
  }
}

// thermostat, rescale and samplers of one slot in one block of kMdThreads
// threads; the thermostat's sums use the first kMdBlock threads in the
// order of md_correct_kernel's block partials (the same bits as a block of
// kMdBlock threads)
__global__ __launch_bounds__(kMdThreads) void md_finish_kernel(SlotDev* slots, MDDev* md,
                                                               const SysParams* __restrict__ prm,
                                                               const SpeciesTable* __restrict__ tab) {
  __shared__ double red5[5][kMdBlock];
  __shared__ double red[kMdThreads];
  __shared__ double s_scale[2];
  SlotDev& sd = slots[blockIdx.x];
  MDDev& m = md[blockIdx.x];
  const int tid = threadIdx.x;
  if (!m.active) {
    // a finished slot samples nothing more (its last RDF sample was taken
    // right after the step that ended it)
    if (tid == 0) m.rdf_due = 0;
    return;
  }
  const SysParams& P = prm[blockIdx.x];
  // 1. block partials: each of the first kMdBlock threads a contiguous run,
  //    then the tree
  {
    const int nb = (sd.n + kMdBlock - 1) / kMdBlock, per = (nb + kMdBlock - 1) / kMdBlock;
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (tid < kMdBlock) {
      for (int b = tid * per; b < min(nb, (tid + 1) * per); ++b)
        for (int k = 0; k < 5; ++k) v[k] += m.md_part[(size_t)b * 8 + k];
      for (int k = 0; k < 5; ++k) red5[k][tid] = v[k];
    }
    __syncthreads();
    for (int h = kMdBlock / 2; h > 0; h >>= 1) {
      if (tid < h)
        for (int k = 0; k < 5; ++k) red5[k][tid] += red5[k][tid + h];
      __syncthreads();
    }
    if (tid == 0) {
      for (int k = 0; k < 5; ++k) v[k] = red5[k][0];
      thermo_tail(sd, m, P, v);
      s_scale[0] = m.scale_tr;
      s_scale[1] = m.scale_rot;
    }
    __syncthreads();
  }
  // 2. the isokinetic factors applied to every molecule
  if (m.temperature > 0.0) {
    const int np = sd.com_ld, n = sd.n;
    const double ft = s_scale[0], fr = s_scale[1];
    for (int i = tid; i < n; i += kMdThreads) rescale_molecule(m, np, i, ft, fr);
  }
  __syncthreads();
  // 3. samplers and the step count
  const long long s = m.steps_done + 1;
  if (m.acf_every > 0 && s % m.acf_every == 0) {
    acf_sample(m, tab, sd, m.vel, sd.com_ld, s, red, true);
    if (tid == 0 && m.res_on) {
      m.res_due = 1;
      m.res_step = s;
    }
  }
  __syncthreads();
  if (tid == 0) {
    m.steps_done = s;
    if (s >= m.steps_target || m.status != MS2_OK) {
      m.active = 0;
      sd.active = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// RDF: the pair kernel's work items; only pairs with j > i count.
// ---------------------------------------------------------------------------
constexpr int kRdfLj = 4;   // LJ sites per species in the largest model class

template <int W>
__global__ __launch_bounds__(64 * W) void rdf_kernel(const WorkItem* __restrict__ items, int item_base,
                                                     const SlotDev* __restrict__ slots,
                                                     const MDDev* __restrict__ md,
                                                     const SysParams* __restrict__ prm,
                                                     const SpeciesTable* __restrict__ tab) {
  constexpr int TJ = 64 * W;
  constexpr int kLds = W == 4 ? 4096 : 8192;
  __shared__ double s_com[3][TJ];
  __shared__ double s_lj[kRdfLj][3][TJ];
  __shared__ int s_sp[TJ];
  __shared__ unsigned int s_hist[kLds];
  const WorkItem it = items[item_base + blockIdx.x];
  const SlotDev& sd = slots[it.slot];
  const MDDev& m = md[it.slot];
  // a tile pair dealt to several symmetric items is histogrammed by the first
  if (!m.rdf_due || split_index(it.split) != 0) return;
  const SysParams& P = prm[it.slot];
  const int tid = threadIdx.x, n = sd.n, ld = sd.com_ld, nsp = tab->nsp;
  const int bins = m.rdf_bins, T = tab->n_lj_types;
  const bool use_lds = m.rdf_ntp * bins <= kLds;
  if (use_lds)
    for (int e = tid; e < m.rdf_ntp * bins; e += TJ) s_hist[e] = 0u;
  const int i = it.i0 + tid;
  const bool iv = i < n;
  const int ic = iv ? i : 0;
  const int spi = clamp_species(sd.species[ic], nsp);
  const SpeciesDev& Di = tab->sp[spi];
  double A[3][3];
  quat_matrix(sd.quat[ic], sd.quat[ld + ic], sd.quat[2 * ld + ic], sd.quat[3 * ld + ic], A);
  double di[kRdfLj][3];
#pragma unroll
  for (int a = 0; a < kRdfLj; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      di[a][c] = a < Di.nlj ? A[c][0] * Di.lj_pos[a][0] + A[c][1] * Di.lj_pos[a][1] +
                                  A[c][2] * Di.lj_pos[a][2]
                            : 0.0;
  const double xi = sd.com[ic], yi = sd.com[ld + ic], zi = sd.com[2 * ld + ic];
  unsigned long long* ghist = m.rdf;
  for (int jt = it.j0; jt < it.j1; jt += TJ) {
    __syncthreads();
    {
      const int j = jt + tid;
      const bool jv = j < it.j1 && j < n;
      const int jc = jv ? j : 0;
      const int spj = clamp_species(sd.species[jc], nsp);
      const SpeciesDev& Dj = tab->sp[spj];
      double B[3][3];
      quat_matrix(sd.quat[jc], sd.quat[ld + jc], sd.quat[2 * ld + jc], sd.quat[3 * ld + jc], B);
      s_com[0][tid] = sd.com[jc];
      s_com[1][tid] = sd.com[ld + jc];
      s_com[2][tid] = sd.com[2 * ld + jc];
      s_sp[tid] = jv ? spj : -1;
      for (int a = 0; a < kRdfLj; ++a)
        for (int c = 0; c < 3; ++c)
          s_lj[a][c][tid] = a < Dj.nlj ? B[c][0] * Dj.lj_pos[a][0] + B[c][1] * Dj.lj_pos[a][1] +
                                             B[c][2] * Dj.lj_pos[a][2]
                                       : 0.0;
    }
    __syncthreads();
    if (!iv) continue;
    for (int jj = 0; jj < TJ; ++jj) {
      const int j = jt + jj;
      const int spj = s_sp[jj];
      if (spj < 0 || j <= i) continue;
      double R[3];
      {
#pragma clang fp contract(off)
        const double dx = xi - s_com[0][jj], dy = yi - s_com[1][jj], dz = zi - s_com[2][jj];
        R[0] = dx - P.L * rint(dx * P.invL);
        R[1] = dy - P.L * rint(dy * P.invL);
        R[2] = dz - P.L * rint(dz * P.invL);
      }
      if (R[0] * R[0] + R[1] * R[1] + R[2] * R[2] >= m.rdf_reach2) continue;
      const SpeciesDev& Dj = tab->sp[spj];
#pragma unroll
      for (int a = 0; a < kRdfLj; ++a) {
        if (a >= Di.nlj) break;
        for (int b = 0; b < Dj.nlj; ++b) {
          double r;
          {
#pragma clang fp contract(off)
            const double rx = R[0] + di[a][0] - s_lj[b][0][jj];
            const double ry = R[1] + di[a][1] - s_lj[b][1][jj];
            const double rz = R[2] + di[a][2] - s_lj[b][2][jj];
            r = sqrt(rx * rx + ry * ry + rz * rz);
          }
          if (!(r < m.rdf_rmax)) continue;
          const int bin = (int)(r * m.rdf_inv_dr);
          if (bin >= bins) continue;
          int t1 = Di.lj_type0 + a, t2 = Dj.lj_type0 + b;
          if (t1 > t2) { const int x = t1; t1 = t2; t2 = x; }
          const int tp = t1 * T - t1 * (t1 - 1) / 2 + (t2 - t1);
          if (use_lds)
            atomicAdd(&s_hist[tp * bins + bin], 1u);
          else
            atomicAdd(&ghist[(size_t)tp * bins + bin], 1ull);
        }
      }
    }
  }
  __syncthreads();
  if (use_lds)
    for (int e = tid; e < m.rdf_ntp * bins; e += TJ)
      if (s_hist[e]) atomicAdd(&ghist[e], (unsigned long long)s_hist[e]);
}

// ---------------------------------------------------------------------------
// Residence time and solvation number (Sec. 5, Eqs. 7-8), sampled with the
// ACFs.  residence_kernel: one block per (solute, slot).  A solvent molecule
// is inside the shell when the centres are closer than the radius (FP64,
// minimum image, no contraction).  Per live origin o, the state word of the
// pair (solute, solvent) is kResDead (outside the shell at t0, or outside for
// more than res_tol consecutive samples since: it never counts again for o)
// or the number of consecutive samples spent outside; the pair counts at a
// lag while not dead and inside (the tolerance of Impey et al.).  Counts are
// wave ballots added per wave and then in wave order.  The solute's fraction
// of its initial shell still resident, per origin, and its shell population
// now go to staging arrays; residence_reduce_kernel adds them up over the
// solutes in a fixed order and clears the pending flag.
// ---------------------------------------------------------------------------
constexpr int kResThreads = 256;

__global__ __launch_bounds__(kResThreads) void residence_kernel(const SlotDev* __restrict__ slots, MDDev* md,
                                                                const SysParams* __restrict__ prm,
                                                                int slot_base) {
  constexpr int NW = kResThreads / 64;
  __shared__ int s_lag[kResMaxLive];
  __shared__ int s_cnt[NW][kResMaxLive];
  __shared__ int s_in[NW];
  const int slot = slot_base + blockIdx.y;
  const MDDev& m = md[slot];
  if (!m.res_due || (int)blockIdx.x >= m.n_solute) return;
  const SlotDev& sd = slots[slot];
  const SysParams& P = prm[slot];
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid / 64);
  const int live = m.n_origins < m.acf_max_live ? m.n_origins : m.acf_max_live;
  const long long step = m.res_step;
  for (int o = tid; o < kResMaxLive; o += kResThreads) {
    int lag = -1;
    if (o < live && step >= m.origin_t0[o]) {
      const long long l = (step - m.origin_t0[o]) / m.acf_every;
      if (l < m.acf_nlag) lag = (int)l;
    }
    s_lag[o] = lag;
    for (int w = 0; w < NW; ++w) s_cnt[w][o] = 0;
  }
  if (tid < NW) s_in[tid] = 0;
  __syncthreads();
  const int a = blockIdx.x, ns = m.n_solvent, nu = m.n_solute, ld = sd.com_ld;
  const int ia = m.res_solute_idx[a];
  const double xa = sd.com[ia], ya = sd.com[ld + ia], za = sd.com[2 * ld + ia];
  for (int b0 = wv * 64; b0 < ns; b0 += kResThreads) {
    const int b = b0 + lane;
    bool in = false;
    if (b < ns) {
      const int ib = m.res_solvent_idx[b];
      double r2;
      {
#pragma clang fp contract(off)
        double dx = xa - sd.com[ib], dy = ya - sd.com[ld + ib], dz = za - sd.com[2 * ld + ib];
        dx = dx - P.L * rint(dx * P.invL);
        dy = dy - P.L * rint(dy * P.invL);
        dz = dz - P.L * rint(dz * P.invL);
        r2 = dx * dx + dy * dy + dz * dz;
      }
      in = ib != ia && r2 < m.res_r2;
    }
    const unsigned long long win = __builtin_amdgcn_ballot_w64(in);
    if (lane == 0) s_in[wv] += __popcll(win);
    for (int o = 0; o < live; ++o) {
      const int lag = s_lag[o];
      if (lag < 0) continue;
      bool counts = false;
      if (b < ns) {
        unsigned short* stp = m.res_state + ((size_t)o * nu + a) * ns + b;
        unsigned short v = *stp;
        if (lag == 0) {
          v = in ? 0 : kResDead;
        } else if (v != kResDead) {
          v = in ? 0 : (unsigned short)(v + 1);
          if (v != kResDead && (int)v > m.res_tol) v = kResDead;
        }
        *stp = v;
        counts = in && v != kResDead;
      }
      const unsigned long long wc = __builtin_amdgcn_ballot_w64(counts);
      if (lane == 0) s_cnt[wv][o] += __popcll(wc);
    }
  }
  __syncthreads();
  for (int o = tid; o < m.acf_max_live; o += kResThreads) {
    double frac = -1.0;
    if (o < live && s_lag[o] >= 0) {
      int c = 0;
      for (int w = 0; w < NW; ++w) c += s_cnt[w][o];
      int* n0p = m.res_n0 + (size_t)o * nu + a;
      if (s_lag[o] == 0) *n0p = c;      // at the origin every molecule inside counts
      const int n0 = s_lag[o] == 0 ? c : *n0p;
      if (n0 > 0) frac = (double)c / (double)n0;
    }
    m.res_part[(size_t)a * m.acf_max_live + o] = frac;
  }
  if (tid == 0) {
    int t = 0;
    for (int w = 0; w < NW; ++w) t += s_in[w];
    m.res_inside[a] = t;
  }
}

__global__ __launch_bounds__(64) void residence_reduce_kernel(MDDev* md, int slot_base) {
  MDDev& m = md[slot_base + blockIdx.x];
  if (!m.res_due) return;
  const int lane = threadIdx.x, nu = m.n_solute, ml = m.acf_max_live;
  const int live = m.n_origins < ml ? m.n_origins : ml;
  const long long step = m.res_step;
  for (int o = 0; o < live; ++o) {
    if (step < m.origin_t0[o]) continue;
    const long long lag = (step - m.origin_t0[o]) / m.acf_every;
    if (lag >= m.acf_nlag) continue;
    double sum = 0.0;
    int cnt = 0;
    for (int a = lane; a < nu; a += 64) {
      const double f = m.res_part[(size_t)a * ml + o];
      if (f >= 0.0) {
        sum += f;
        cnt += 1;
      }
    }
    for (int h = 32; h > 0; h >>= 1) {
      sum += __shfl_xor(sum, h, 64);
      cnt += __shfl_xor(cnt, h, 64);
    }
    if (lane == 0) {
      m.res_acf[lag] += sum;
      m.res_cnt[lag] += (double)cnt;
    }
  }
  int inside = 0;
  for (int a = lane; a < nu; a += 64) inside += m.res_inside[a];
  for (int h = 32; h > 0; h >>= 1) inside += __shfl_xor(inside, h, 64);
  if (lane == 0) {
    m.res_solv_sum += (double)inside;
    m.res_solv_cnt += (double)nu;
    m.res_due = 0;
  }
}

// ---------------------------------------------------------------------------
hipError_t launch_residence(const SlotDev* slots, MDDev* md, const SysParams* prm, int slot_base,
                            int nslots, int max_solute, hipStream_t st) {
  if (nslots <= 0 || max_solute <= 0) return hipSuccess;
  hipLaunchKernelGGL(residence_kernel, dim3(max_solute, nslots), dim3(kResThreads), 0, st, slots, md, prm,
                     slot_base);
  hipLaunchKernelGGL(residence_reduce_kernel, dim3(nslots), dim3(64), 0, st, md, slot_base);
  return hipGetLastError();
}

hipError_t launch_md_wrap(MDDev* md, const SysParams* prm, int slot, int n, hipStream_t st) {
  hipLaunchKernelGGL(md_wrap_kernel, dim3((n + 255) / 256), dim3(256), 0, st, md, prm, slot, n);
  return hipGetLastError();
}

hipError_t launch_md_init(SlotDev* slots, MDDev* md, const SpeciesTable* tab, int slot, hipStream_t st) {
  hipLaunchKernelGGL(md_init_kernel, dim3(1), dim3(kMdThreads), 0, st, slots, md, tab, slot);
  return hipGetLastError();
}

hipError_t launch_md_end(SlotDev* slots, MDDev* md, const SysParams* prm, const SpeciesTable* tab,
                         int nslots, int max_n, hipStream_t st) {
  const int mb = (max_n + kMdBlock - 1) / kMdBlock;
  hipLaunchKernelGGL(md_correct_kernel, dim3(mb, nslots), dim3(kMdBlock), 0, st, slots, md, prm, tab);
  hipLaunchKernelGGL(md_finish_kernel, dim3(nslots), dim3(kMdThreads), 0, st, slots, md, prm, tab);
  return hipGetLastError();
}

template <typename Real, int C>
static hipError_t launch_begin_frame_c(const SlotDev* slots, MDDev* md, const SysParams* prm,
                                       const SpeciesTable* tab, int nslots, int max_n, hipStream_t st) {
  hipLaunchKernelGGL((md_begin_frame_kernel<Real, C>), dim3((max_n + 255) / 256, nslots), dim3(256), 0, st, slots,
                     md, prm, tab);
  return hipGetLastError();
}

hipError_t launch_md_begin_frame(int cls, int precision, const SlotDev* slots, MDDev* md, const SysParams* prm,
                                 const SpeciesTable* tab, int nslots, int max_n, hipStream_t st) {
#define MS2_BEGIN_CASE(C)                                                                             \
  case C:                                                                                             \
    return precision == MS2_FP32 ? launch_begin_frame_c<float, C>(slots, md, prm, tab, nslots, max_n, st) \
                                 : launch_begin_frame_c<double, C>(slots, md, prm, tab, nslots, max_n, st);
  switch (cls) {
    MS2_BEGIN_CASE(0)
    MS2_BEGIN_CASE(1)
    MS2_BEGIN_CASE(2)
    MS2_BEGIN_CASE(3)
    MS2_BEGIN_CASE(4)
    MS2_BEGIN_CASE(5)
  }
#undef MS2_BEGIN_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_rdf(int waves, const WorkItem* items, int base, int count, const SlotDev* slots,
                      const MDDev* md, const SysParams* prm, const SpeciesTable* tab, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (waves == 4)
    hipLaunchKernelGGL(rdf_kernel<4>, dim3(count), dim3(256), 0, st, items, base, slots, md, prm, tab);
  else
    hipLaunchKernelGGL(rdf_kernel<1>, dim3(count), dim3(64), 0, st, items, base, slots, md, prm, tab);
  return hipGetLastError();
}

}  // namespace ms2
