// Ewald reciprocal space on gfx950 (the paper's Sec. 4: the long-range part
// of the Coulomb sum is done in Fourier space).  Everything here is FP64:
// charge positions are rebuilt from the centre and the quaternion in FP64,
// phases are reduced to [-pi, pi] exactly via the integer period of the k
// lattice, and S(k) is accumulated in FP64.
//
//   sk_kernel          (k block of 64) x (molecule tile): partial S(k)
//   sk_reduce_kernel   64 k per block: S(k) over tiles in fixed order and
//                      the k's energy and atomic-virial terms
//   kforce_kernel      (64-molecule tile) x (k chunk): per-molecule force,
//                      torque and sum d.F partials
//   reduce_kforce_kernel, reduce_ksums_kernel: add the force partials and the
//                      per-k terms (fixed order) into the caller's force,
//                      torque and sums
// The k set is a half space (k and -k give equal contributions), so every
// reciprocal term is doubled.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace ms2 {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.14159265358979323846264338328;

__device__ __forceinline__ void quat_rot(const double* q, int ld, int i, double A[3][3]) {
  const double w = q[i], x = q[ld + i], y = q[2 * ld + i], z = q[3 * ld + i];
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

// exp(i 2 pi t) with t reduced by its nearest integer first
__device__ __forceinline__ void phase(double t, double& c, double& s) {
  t -= rint(t);
  sincospi(2.0 * t, &s, &c);
}

__global__ __launch_bounds__(64) void sk_kernel(const SlotDev* __restrict__ slots,
                                                const SysParams* __restrict__ prm,
                                                const SpeciesTable* __restrict__ tab) {
  __shared__ double s_x[kMolTile * kMaxS], s_y[kMolTile * kMaxS], s_z[kMolTile * kMaxS],
      s_q[kMolTile * kMaxS];
  const SlotDev& sd = slots[blockIdx.z];
  const SysParams& P = prm[blockIdx.z];
  if (!sd.active || P.elec != MS2_ELEC_EWALD) return;
  const int mc = blockIdx.y;
  if (mc >= sd.mchunks || (int)blockIdx.x * 64 >= sd.nk) return;
  const int tid = threadIdx.x, ld = sd.com_ld;
  const int m0 = mc * kMolTile, m1 = min(sd.n, m0 + kMolTile);
  int maxq = 0;
  for (int s = 0; s < P.nsp; ++s) maxq = max(maxq, tab->sp[s].nch);
  if (tid < kMolTile) {
    const int i = m0 + tid;
    for (int a = 0; a < maxq; ++a) s_q[tid * kMaxS + a] = 0.0;
    if (i < m1) {
      const SpeciesDev& D = tab->sp[clamp_species(sd.species[i], P.nsp)];
      double A[3][3];
      quat_rot(sd.quat, ld, i, A);
      const double cx = sd.com[i], cy = sd.com[ld + i], cz = sd.com[2 * ld + i];
      for (int a = 0; a < D.nch; ++a) {
        const double* b = D.ch_pos[a];
        s_x[tid * kMaxS + a] = cx + A[0][0] * b[0] + A[0][1] * b[1] + A[0][2] * b[2];
        s_y[tid * kMaxS + a] = cy + A[1][0] * b[0] + A[1][1] * b[1] + A[1][2] * b[2];
        s_z[tid * kMaxS + a] = cz + A[2][0] * b[0] + A[2][1] * b[1] + A[2][2] * b[2];
        s_q[tid * kMaxS + a] = D.ch_q[a];
      }
    }
  }
  __syncthreads();
  const int k = blockIdx.x * 64 + tid;
  if (k >= sd.nk) return;
  const KVec kv = sd.kvec[k];
  const double invL = P.invL;
  double re = 0.0, im = 0.0;
  for (int m = 0; m < m1 - m0; ++m)
    for (int a = 0; a < maxq; ++a) {
      const int e = m * kMaxS + a;
      const double q = s_q[e];
      if (q == 0.0) continue;
      double c, s;
      phase((kv.nx * s_x[e] + kv.ny * s_y[e] + kv.nz * s_z[e]) * invL, c, s);
      re += q * c;
      im += q * s;
    }
  double* out = sd.sk_part + ((size_t)mc * sd.nk + k) * 2;
  out[0] = re;
  out[1] = im;
}

// S(k) summed over the molecule tiles in a fixed order: a block holds 64 k,
// and its four waves each sum one consecutive run of the tiles (loads of four
// partials issued before their additions); the run sums are added in run
// order.  Then the k's terms of the reciprocal energy and atomic virial,
// g(k) |S(k)|^2 and g(k) |S(k)|^2 (1 - k^2 / (2 alpha^2)) with
// g(k) = exp(-k^2 / (4 alpha^2)) / k^2, for a fixed-order sum over k in
// reduce_ksums_kernel.  The terms overwrite the tile-0 partial of the same
// k, which only this block reads.
__global__ __launch_bounds__(256) void sk_reduce_kernel(const SlotDev* __restrict__ slots,
                                                        const SysParams* __restrict__ prm) {
  __shared__ double s_re[4][64], s_im[4][64];
  const SlotDev& sd = slots[blockIdx.y];
  const SysParams& P = prm[blockIdx.y];
  if (!sd.active || P.elec != MS2_ELEC_EWALD) return;
  const int kl = threadIdx.x & 63, run = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + kl;
  const bool kin = k < sd.nk;
  const int len = (sd.mchunks + 3) / 4, t0 = min(sd.mchunks, run * len), t1 = min(sd.mchunks, t0 + len);
  double re = 0.0, im = 0.0;
  if (kin) {
    const double2* part = reinterpret_cast<const double2*>(sd.sk_part) + k;
    const size_t stride = (size_t)sd.nk;
    int t = t0;
    for (; t + 4 <= t1; t += 4) {
      const double2 a = part[t * stride], b = part[(t + 1) * stride];
      const double2 c = part[(t + 2) * stride], d = part[(t + 3) * stride];
      re += a.x; im += a.y;
      re += b.x; im += b.y;
      re += c.x; im += c.y;
      re += d.x; im += d.y;
    }
    for (; t < t1; ++t) {
      const double2 a = part[t * stride];
      re += a.x; im += a.y;
    }
  }
  s_re[run][kl] = re;
  s_im[run][kl] = im;
  __syncthreads();
  if (run != 0 || !kin) return;
  re = ((s_re[0][kl] + s_re[1][kl]) + s_re[2][kl]) + s_re[3][kl];
  im = ((s_im[0][kl] + s_im[1][kl]) + s_im[2][kl]) + s_im[3][kl];
  sd.sk[2 * k] = re;
  sd.sk[2 * k + 1] = im;
  const double k2s = (kTwoPi * P.invL) * (kTwoPi * P.invL);
  const double k2 = k2s * sd.kvec[k].n2;
  const double g = exp(-k2 / (4.0 * P.alpha2)) / k2;
  const double s2 = re * re + im * im;
  sd.sk_part[2 * k] = g * s2;
  sd.sk_part[2 * k + 1] = g * s2 * (1.0 - k2 / (2.0 * P.alpha2));
}

__global__ __launch_bounds__(64) void kforce_kernel(const SlotDev* __restrict__ slots,
                                                    const SysParams* __restrict__ prm,
                                                    const SpeciesTable* __restrict__ tab) {
  __shared__ double s_re[kKChunk], s_im[kKChunk], s_g[kKChunk];
  __shared__ int s_n[kKChunk][3];
  __shared__ int s_next[kKChunk];   // 1: k is k - 1 of the chunk plus one step in n_z
  __shared__ double s_red[64];
  const SlotDev& sd = slots[blockIdx.z];
  const SysParams& P = prm[blockIdx.z];
  if (!sd.active || P.elec != MS2_ELEC_EWALD) return;
  const int kc = blockIdx.y;
  if (kc >= sd.kchunks || (int)blockIdx.x >= sd.mtiles) return;
  const int tid = threadIdx.x, ld = sd.com_ld, np = sd.npad;
  const int k0 = kc * kKChunk, nkc = min(kKChunk, sd.nk - k0);
  const double k2s = (kTwoPi * P.invL) * (kTwoPi * P.invL);
  for (int e = tid; e < nkc; e += 64) {
    const KVec kv = sd.kvec[k0 + e];
    s_re[e] = sd.sk[2 * (k0 + e)];
    s_im[e] = sd.sk[2 * (k0 + e) + 1];
    const double k2 = k2s * kv.n2;
    s_g[e] = exp(-k2 / (4.0 * P.alpha2)) / k2;
    s_n[e][0] = kv.nx;
    s_n[e][1] = kv.ny;
    s_n[e][2] = kv.nz;
    int next = 0;
    if (e > 0) {
      const KVec kp = sd.kvec[k0 + e - 1];
      next = kp.nx == kv.nx && kp.ny == kv.ny && kp.nz + 1 == kv.nz;
    }
    s_next[e] = next;
  }
  __syncthreads();
  const int i = blockIdx.x * 64 + tid;
  double dF = 0.0;
  if (i < sd.n) {
    const SpeciesDev& D = tab->sp[clamp_species(sd.species[i], P.nsp)];
    double A[3][3];
    quat_rot(sd.quat, ld, i, A);
    const double cx = sd.com[i], cy = sd.com[ld + i], cz = sd.com[2 * ld + i];
    double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
    // F_a = (4 pi k_e q_a / V) sum_k g(k) k Im(e^{i k.r_a} S(k)^*), doubled
    const double pre = 2.0 * P.ke * 4.0 * kPi / P.V;
    for (int a = 0; a < D.nch; ++a) {
      const double* b = D.ch_pos[a];
      const double d[3] = {A[0][0] * b[0] + A[0][1] * b[1] + A[0][2] * b[2],
                           A[1][0] * b[0] + A[1][1] * b[1] + A[1][2] * b[2],
                           A[2][0] * b[0] + A[2][1] * b[1] + A[2][2] * b[2]};
      const double x = cx + d[0], y = cy + d[1], z = cz + d[2];
      double sx = 0.0, sy = 0.0, sz = 0.0;
      // along a line of the k set (n_x, n_y fixed, n_z rising by one) the
      // phase advances by exp(i 2 pi z / L): one complex product; a line's
      // first k takes the phase directly
      double ezc, ezs;
      phase(z * P.invL, ezc, ezs);
      double c = 1.0, s = 0.0;
      for (int e = 0; e < nkc; ++e) {
        if (s_next[e]) {
          const double c1 = c * ezc - s * ezs;
          s = c * ezs + s * ezc;
          c = c1;
        } else {
          phase((s_n[e][0] * x + s_n[e][1] * y + s_n[e][2] * z) * P.invL, c, s);
        }
        const double t = s_g[e] * (s * s_re[e] - c * s_im[e]);
        sx += t * s_n[e][0];
        sy += t * s_n[e][1];
        sz += t * s_n[e][2];
      }
      const double f = pre * D.ch_q[a] * kTwoPi * P.invL;
      const double fa[3] = {f * sx, f * sy, f * sz};
      F[0] += fa[0]; F[1] += fa[1]; F[2] += fa[2];
      T[0] += d[1] * fa[2] - d[2] * fa[1];
      T[1] += d[2] * fa[0] - d[0] * fa[2];
      T[2] += d[0] * fa[1] - d[1] * fa[0];
      dF += d[0] * fa[0] + d[1] * fa[1] + d[2] * fa[2];
    }
    double* out = sd.fk + (size_t)kc * 6 * np;
    for (int c = 0; c < 3; ++c) {
      out[c * np + i] = F[c];
      out[(3 + c) * np + i] = T[c];
    }
  }
  s_red[tid] = dF;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (tid < h) s_red[tid] += s_red[tid + h];
    __syncthreads();
  }
  if (tid == 0) sd.kred[(size_t)kc * sd.mtiles + blockIdx.x] = s_red[0];
}

// One thread per (component, molecule): the grid's x holds six runs of
// molecule blocks, one per force/torque component; the chunk partials are
// added in chunk order (the loads of four chunks issued before their
// additions).
__global__ __launch_bounds__(256) void reduce_kforce_kernel(const SlotDev* __restrict__ slots,
                                                            const SysParams* __restrict__ prm) {
  const SlotDev& sd = slots[blockIdx.y];
  const SysParams& P = prm[blockIdx.y];
  if (!sd.active || P.elec != MS2_ELEC_EWALD) return;
  const int mb = gridDim.x / 6, c = blockIdx.x / mb;
  const int i = (blockIdx.x - c * mb) * 256 + threadIdx.x;
  if (i >= sd.n) return;
  const int np = sd.npad, ld = sd.com_ld;
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
  if (c < 3)
    sd.force[c * ld + i] += v;
  else
    sd.torque[(c - 3) * ld + i] += v;
}

__global__ __launch_bounds__(256) void reduce_ksums_kernel(const SlotDev* __restrict__ slots,
                                                           const SysParams* __restrict__ prm) {
  __shared__ double s_d[256], s_u[256], s_w[256];
  const SlotDev& sd = slots[blockIdx.x];
  const SysParams& P = prm[blockIdx.x];
  if (!sd.active || P.elec != MS2_ELEC_EWALD) return;
  const int tid = threadIdx.x;
  // sum_a d_a . F_a over the force partials, and the per-k energy and virial
  // terms over k: each thread a contiguous run, then a tree (fixed order)
  const int nr = sd.kchunks * sd.mtiles;
  const int per = (nr + 255) / 256;
  double d = 0.0;
  for (int t = tid * per; t < min(nr, (tid + 1) * per); ++t) d += sd.kred[t];
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

hipError_t launch_kspace(const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                         int nslots, int max_kblocks, int max_mchunks, int max_mtiles,
                         int max_kchunks, hipStream_t st) {
  hipLaunchKernelGGL(sk_kernel, dim3(max_kblocks, max_mchunks, nslots), dim3(64), 0, st, slots,
                     prm, tab);
  hipLaunchKernelGGL(sk_reduce_kernel, dim3(max_kblocks, nslots), dim3(256), 0, st, slots, prm);
  hipLaunchKernelGGL(kforce_kernel, dim3(max_mtiles, max_kchunks, nslots), dim3(64), 0, st, slots,
                     prm, tab);
  hipLaunchKernelGGL(reduce_kforce_kernel, dim3(6 * ((64 * max_mtiles + 255) / 256), nslots), dim3(256), 0,
                     st, slots, prm);
  hipLaunchKernelGGL(reduce_ksums_kernel, dim3(nslots), dim3(256), 0, st, slots, prm);
  return hipGetLastError();
}

}  // namespace ms2
