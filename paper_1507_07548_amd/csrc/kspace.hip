// Ewald reciprocal space on gfx950 (the paper's Sec. 4: the long-range part
// of the Coulomb sum is done in Fourier space).  Everything here is FP64:
// charge positions are rebuilt from the centre and the quaternion in FP64;
// a charge's phase is taken from sincospi (its argument reduced by the
// nearest integer first, exact for the integer k lattice) at the first k of
// each line of the k set and carried along the line by complex products;
// S(k) is accumulated in FP64.
//
//   sk_kernel          (k block of 64) x (16-molecule tile): partial S(k),
//                      phases carried along the k lines per charge
//   sk_reduce_kernel   64 k per block: S(k) over tiles in fixed order and
//                      the k's energy and atomic-virial terms
//   kforce_kernel      (16-molecule tile) x (k chunk): per-molecule force,
//                      torque and sum d.F partials
//   reduce_kforce_kernel, reduce_ksums_kernel: add the force partials and the
//                      per-k terms (fixed order) into the caller's force,
//                      torque and sums
// The k set is a half space (k and -k give equal contributions), so every
// reciprocal term is doubled.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kspace_sums.h"
#include "quat.h"

namespace ms2 {

constexpr double kPi = 3.14159265358979323846264338328;

__device__ __forceinline__ void quat_rot(const double* q, int ld, int i, double A[3][3]) {
  quat_matrix(q[i], q[ld + i], q[2 * ld + i], q[3 * ld + i], A);
}

// exp(i 2 pi t) with t reduced by its nearest integer first
__device__ __forceinline__ void phase(double t, double& c, double& s) {
  t -= rint(t);
  sincospi(2.0 * t, &s, &c);
}

// Partial S(k) of one tile of kMolTile = 16 molecules for kSkK k vectors.  A
// block is one wave; lane l owns charge l mod 4 of molecule l / 4 of the
// tile (every model class has at most four charges per molecule) and carries
// its phase exp(2 pi i n.r / L) from k to k: inside a line of the k set
// (n_x, n_y fixed, n_z rising by one) by one complex product with
// exp(2 pi i z / L), from sincospi at a line's or the block's first k.
// Batches of 8 k go through LDS: lane l adds the 8 charges of segment l / 8
// for the k l mod 8 of the batch, and the eight segment sums are added in
// segment order (8 KB of LDS per block, so that ~4 waves per SIMD fit).
constexpr int kChargeSlots = 4;
static_assert(kMolTile * kChargeSlots == 64, "one charge slot per lane");
// k vectors per structure-factor block (a multiple of 8, at most 64): 32
// puts twice the waves of 64 in flight for the phase chains, at the price of
// more line-start sincospi (water + ions, N = 1000, lone MD step: 64 / 32 /
// 16 k: 98.0 / 93.7 / 93.3 us)
constexpr int kSkK = 32;
static_assert(kSkK % 8 == 0 && kSkK <= 64, "k batches of 8, one k vector per lane at most");

constexpr int max_class_charges() {
  int m = 0;
  for (int c = 0; c < kNumClasses; ++c) m = kClassShapes[c].ch > m ? kClassShapes[c].ch : m;
  return m;
}
static_assert(max_class_charges() <= kChargeSlots, "every charge of every model class needs a slot");

__global__ __launch_bounds__(64) void sk_kernel(const SlotDev* __restrict__ slots,
                                                const SysParams* __restrict__ prm,
                                                const SpeciesTable* __restrict__ tab) {
  __shared__ double2 s_c[8][65];        // q exp(i k.r) per (k of the batch, lane); padded rows
  __shared__ double2 s_seg[8][8];
  __shared__ int s_n[kSkK][3];
  __shared__ int s_next[kSkK];          // 1: k continues the line of the previous k
  const SlotDev& sd = slots[blockIdx.z];
  const SysParams& P = prm[blockIdx.z];
  if (!sd.active || P.elec != MS2_ELEC_EWALD) return;
  const int mc = blockIdx.y;
  if (mc >= sd.mchunks || (int)blockIdx.x * kSkK >= sd.nk) return;
  const int lane = threadIdx.x, ld = sd.com_ld;
  const int k0 = blockIdx.x * kSkK, nkb = min(kSkK, sd.nk - k0);
  if (lane < nkb) {
    const KVec kv = sd.kvec[k0 + lane];
    s_n[lane][0] = kv.nx;
    s_n[lane][1] = kv.ny;
    s_n[lane][2] = kv.nz;
    int next = 0;
    if (lane > 0) {
      const KVec kp = sd.kvec[k0 + lane - 1];
      next = kp.nx == kv.nx && kp.ny == kv.ny && kp.nz + 1 == kv.nz;
    }
    s_next[lane] = next;
  }
  const int i = mc * kMolTile + (lane >> 2), a = lane & (kChargeSlots - 1);
  double q = 0.0, x = 0.0, y = 0.0, z = 0.0;
  if (i < sd.n) {
    const int spr = sd.species[i];
    const SpeciesDev& D = tab->sp[clamp_species(spr, P.nsp)];
    if (a < min(D.nch, kChargeSlots)) {
      double A[3][3];
      quat_rot(sd.quat, ld, i, A);
      const double* b = D.ch_pos[a];
      x = sd.com[i] + A[0][0] * b[0] + A[0][1] * b[1] + A[0][2] * b[2];
      y = sd.com[ld + i] + A[1][0] * b[0] + A[1][1] * b[1] + A[1][2] * b[2];
      z = sd.com[2 * ld + i] + A[2][0] * b[0] + A[2][1] * b[1] + A[2][2] * b[2];
      q = D.ch_q[a];
    }
    if (!species_ok(spr, P.nsp)) {
      // an argument error found on the device: S(k), and with it every
      // reciprocal result of the call, becomes NaN
      q = __builtin_nan("");
      if (a == 0 && sd.err) *sd.err = 1;
    }
  }
  __syncthreads();
  const double invL = P.invL;
  double ezc, ezs;
  phase(z * invL, ezc, ezs);
  double c = 1.0, s = 0.0;
  double* out = sd.sk_part + ((size_t)mc * sd.nk + k0) * 2;
  for (int b0 = 0; b0 < nkb; b0 += 8) {
    for (int j = 0; j < 8; ++j) {
      const int e = b0 + j;
      double2 v = make_double2(0.0, 0.0);
      if (e < nkb) {
        if (s_next[e]) {
          const double c1 = c * ezc - s * ezs;
          s = c * ezs + s * ezc;
          c = c1;
        } else {
          phase((s_n[e][0] * x + s_n[e][1] * y + s_n[e][2] * z) * invL, c, s);
        }
        v = make_double2(q * c, q * s);
      }
      s_c[j][lane] = v;
    }
    __syncthreads();
    {
      const int j = lane & 7, seg = lane >> 3;
      double re = 0.0, im = 0.0;
      for (int t = 0; t < 8; ++t) {
        const double2 v = s_c[j][8 * seg + t];
        re += v.x;
        im += v.y;
      }
      s_seg[seg][j] = make_double2(re, im);
    }
    __syncthreads();
    if (lane < 8 && b0 + lane < nkb) {
      double re = s_seg[0][lane].x, im = s_seg[0][lane].y;
      for (int g = 1; g < 8; ++g) {
        re += s_seg[g][lane].x;
        im += s_seg[g][lane].y;
      }
      out[2 * (b0 + lane)] = re;
      out[2 * (b0 + lane) + 1] = im;
    }
    __syncthreads();
  }
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

// Reciprocal forces: a block is one wave over a tile of kMolTile molecules
// and a chunk of kKChunk k vectors; lane l owns charge l mod 4 of molecule
// l / 4 and walks the chunk with its phase carried along the n_z lines (one
// complex product per k, sincospi at a line's or the chunk's first k).  Each
// molecule's force, torque and d.F are the sums of its four slots in charge
// order; lane 4m writes them.
__global__ __launch_bounds__(64) void kforce_kernel(const SlotDev* __restrict__ slots,
                                                    const SysParams* __restrict__ prm,
                                                    const SpeciesTable* __restrict__ tab) {
  // per k: (g(k) Re S(k), g(k) Im S(k)) and (n_x, n_y, n_z, 1 if k continues the
  // previous k's line else 0), as doubles: two 16-byte LDS reads per k
  __shared__ double2 s_gs[kKChunk];
  __shared__ double4 s_nk[kKChunk];
  __shared__ double s_v[7][64];     // per slot: force, torque, d.F
  __shared__ double s_red[kMolTile];
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
    const double k2 = k2s * kv.n2;
    const double g = exp(-k2 / (4.0 * P.alpha2)) / k2;
    s_gs[e] = make_double2(g * sd.sk[2 * (k0 + e)], g * sd.sk[2 * (k0 + e) + 1]);
    int next = 0;
    if (e > 0) {
      const KVec kp = sd.kvec[k0 + e - 1];
      next = kp.nx == kv.nx && kp.ny == kv.ny && kp.nz + 1 == kv.nz;
    }
    s_nk[e] = make_double4(kv.nx, kv.ny, kv.nz, next);
  }
  __syncthreads();
  const int mloc = tid >> 2, a = tid & (kChargeSlots - 1);
  const int i = blockIdx.x * kMolTile + mloc;
  double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // F, tau, d.F of this slot's charge
  if (i < sd.n) {
    const SpeciesDev& D = tab->sp[clamp_species(sd.species[i], P.nsp)];
    if (a < min(D.nch, kChargeSlots)) {
      double A[3][3];
      quat_rot(sd.quat, ld, i, A);
      const double* b = D.ch_pos[a];
      const double d[3] = {A[0][0] * b[0] + A[0][1] * b[1] + A[0][2] * b[2],
                           A[1][0] * b[0] + A[1][1] * b[1] + A[1][2] * b[2],
                           A[2][0] * b[0] + A[2][1] * b[1] + A[2][2] * b[2]};
      const double x = sd.com[i] + d[0], y = sd.com[ld + i] + d[1], z = sd.com[2 * ld + i] + d[2];
      // F_a = (4 pi k_e q_a / V) sum_k g(k) k Im(e^{i k.r_a} S(k)^*), doubled
      double sx = 0.0, sy = 0.0, sz = 0.0;
      double ezc, ezs;
      phase(z * P.invL, ezc, ezs);
      double c = 1.0, s = 0.0;
      for (int e = 0; e < nkc; ++e) {
        const double4 nk = s_nk[e];
        const double2 gs = s_gs[e];
        if (nk.w != 0.0) {
          const double c1 = c * ezc - s * ezs;
          s = c * ezs + s * ezc;
          c = c1;
        } else {
          phase((nk.x * x + nk.y * y + nk.z * z) * P.invL, c, s);
        }
        const double t = s * gs.x - c * gs.y;
        sx += t * nk.x;
        sy += t * nk.y;
        sz += t * nk.z;
      }
      const double pre = 2.0 * P.ke * 4.0 * kPi / P.V;
      const double f = pre * D.ch_q[a] * kTwoPi * P.invL;
      const double fa[3] = {f * sx, f * sy, f * sz};
      v[0] = fa[0];
      v[1] = fa[1];
      v[2] = fa[2];
      v[3] = d[1] * fa[2] - d[2] * fa[1];
      v[4] = d[2] * fa[0] - d[0] * fa[2];
      v[5] = d[0] * fa[1] - d[1] * fa[0];
      v[6] = d[0] * fa[0] + d[1] * fa[1] + d[2] * fa[2];
    }
  }
  for (int k = 0; k < 7; ++k) s_v[k][tid] = v[k];
  __syncthreads();
  if (a == 0) {
    double w[7];
    for (int k = 0; k < 7; ++k)
      w[k] = ((s_v[k][tid] + s_v[k][tid + 1]) + s_v[k][tid + 2]) + s_v[k][tid + 3];
    if (i < sd.n) {
      double* out = sd.fk + (size_t)kc * 6 * np;
      for (int c = 0; c < 6; ++c) out[c * np + i] = w[c];
    }
    s_red[mloc] = w[6];
  }
  __syncthreads();
  if (tid == 0) {
    double dF = 0.0;
    for (int m = 0; m < kMolTile; ++m) dF += s_red[m];
    sd.kred[(size_t)kc * sd.mtiles + blockIdx.x] = dF;
  }
}

// One thread per (component, molecule): the grid's x holds six runs of
// molecule blocks, one per force/torque component; the chunk partials are
// added in chunk order (kspace_force_sum).
__global__ __launch_bounds__(256) void reduce_kforce_kernel(const SlotDev* __restrict__ slots,
                                                            const SysParams* __restrict__ prm) {
  const SlotDev& sd = slots[blockIdx.y];
  const SysParams& P = prm[blockIdx.y];
  if (!sd.active || P.elec != MS2_ELEC_EWALD) return;
  const int mb = gridDim.x / 6, c = blockIdx.x / mb;
  const int i = (blockIdx.x - c * mb) * 256 + threadIdx.x;
  if (i >= sd.n) return;
  const int ld = sd.com_ld;
  const double v = kspace_force_sum(sd, c, i);
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
  kspace_sums_block(sd, P, s_d, s_u, s_w);
}

// The structure factor and the reciprocal force partials: everything but
// the two reductions, which reduce_pair_kernel can take over in the MD step.
hipError_t launch_kspace_partials(const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                                  int nslots, int max_kblocks, int max_mchunks, int max_mtiles,
                                  int max_kchunks, hipStream_t st) {
  // max_kblocks counts blocks of 64 k vectors
  hipLaunchKernelGGL(sk_kernel, dim3(max_kblocks * (64 / kSkK), max_mchunks, nslots), dim3(64), 0, st, slots,
                     prm, tab);
  hipLaunchKernelGGL(sk_reduce_kernel, dim3(max_kblocks, nslots), dim3(256), 0, st, slots, prm);
  hipLaunchKernelGGL(kforce_kernel, dim3(max_mtiles, max_kchunks, nslots), dim3(64), 0, st, slots,
                     prm, tab);
  return hipGetLastError();
}

hipError_t launch_kspace(const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                         int nslots, int max_kblocks, int max_mchunks, int max_mtiles,
                         int max_kchunks, hipStream_t st) {
  const hipError_t e = launch_kspace_partials(slots, prm, tab, nslots, max_kblocks, max_mchunks, max_mtiles,
                                              max_kchunks, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_kforce_kernel, dim3(6 * ((kMolTile * max_mtiles + 255) / 256), nslots), dim3(256),
                     0, st, slots, prm);
  hipLaunchKernelGGL(reduce_ksums_kernel, dim3(nslots), dim3(256), 0, st, slots, prm);
  return hipGetLastError();
}

}  // namespace ms2
