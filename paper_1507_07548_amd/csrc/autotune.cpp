// Tile-shape autotuner of the pair kernel.
//
// For each size bucket floor(log2 n) in [n_lo, n_hi] and each launch mode it
// builds a synthetic system of species 0 (molecules on a cubic lattice whose
// spacing clears the LJ diameters, deterministic orientations, rc = 0.48 L),
// times every candidate tile shape with HIP events around the pair-kernel
// launches of a few MD steps, and keeps the fastest per system evaluation.
//   mode 0 (one system per launch): a single-slot batch with plain tiles;
//   mode 1 (batched): a batch of enough copies to fill the GPU.
// The chosen shape depends only on (model class, precision, mode, bucket).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "batch.h"

using namespace ms2;

namespace {

struct Synthetic {
  std::vector<int32_t> species;
  std::vector<double> com, quat, vel, omega;
  ms2_system sys;
};

void make_synthetic(const ms2_ctx* ctx, int n, int precision, Synthetic& s) {
  const SpeciesDev& d = ctx->tab.sp[0];
  double sig = 1.0, ext = 0.0;
  for (int a = 0; a < d.nlj; ++a) sig = std::max(sig, d.lj_sigma[a]);
  auto extent = [&](const double* p) { return std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]); };
  for (int a = 0; a < d.nlj; ++a) ext = std::max(ext, extent(d.lj_pos[a]));
  for (int a = 0; a < d.nch; ++a) ext = std::max(ext, extent(d.ch_pos[a]));
  int m = 1;
  while (m * m * m < n) ++m;
  const double a = 1.15 * sig + 2.0 * ext;
  const double L = a * m;
  s.species.assign(n, 0);
  s.com.resize(3 * n);
  s.quat.resize(4 * n);
  s.vel.assign(3 * n, 0.0);
  s.omega.assign(3 * n, 0.0);
  uint64_t h = 0x9e3779b97f4a7c15ull;
  auto rnd = [&]() {  // splitmix64 -> [0, 1)
    h += 0x9e3779b97f4a7c15ull;
    uint64_t z = h;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (double)((z ^ (z >> 31)) >> 11) * (1.0 / 9007199254740992.0);
  };
  for (int i = 0; i < n; ++i) {
    const int ix = i % m, iy = (i / m) % m, iz = i / (m * m);
    s.com[i] = (ix + 0.5 + 0.1 * (rnd() - 0.5)) * a;
    s.com[n + i] = (iy + 0.5 + 0.1 * (rnd() - 0.5)) * a;
    s.com[2 * n + i] = (iz + 0.5 + 0.1 * (rnd() - 0.5)) * a;
    double q[4] = {rnd() - 0.5, rnd() - 0.5, rnd() - 0.5, rnd() - 0.5};
    const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) + 1e-300;
    for (int c = 0; c < 4; ++c) s.quat[c * n + i] = q[c] / nq;
  }
  std::memset(&s.sys, 0, sizeof(s.sys));
  s.sys.params.box = L;
  s.sys.params.rc = 0.48 * L;
  s.sys.params.eps_rf = INFINITY;
  s.sys.params.coulomb_k = 1.0;
  s.sys.params.elec = MS2_ELEC_NONE;
  s.sys.params.lj_lrc = 1;
  s.sys.params.precision = precision;
  s.sys.n_mol = n;
  s.sys.integrator = MS2_GEAR;
  s.sys.n_steps = 1 << 30;
  s.sys.dt = 1e-4;
  s.sys.h_species = s.species.data();
  s.sys.h_com = s.com.data();
  s.sys.h_quat = s.quat.data();
  s.sys.h_vel = s.vel.data();
  s.sys.h_omega = s.omega.data();
}

// microseconds of pair kernel per system evaluation, or a negative value on failure
double time_shape(ms2_ctx* ctx, const Synthetic& syn, int mode, int copies, hipStream_t st) {
  ms2_batch* b = nullptr;
  if (ms2_batch_create(ctx, copies, 0, mode == 0 ? MS2_BATCH_PLAIN_TILES : 0, &b) != MS2_OK) return -1.0;
  double us = -1.0;
  int32_t slot = 0;
  bool ok = true;
  for (int c = 0; c < copies && ok; ++c) ok = ms2_slot_admit(b, &syn.sys, &slot, st) == MS2_OK;
  const int steps = 3;
  if (ok) ok = ms2_step(b, 1, 0, st) == MS2_OK;
  if (ok) ok = ms2_step(b, steps, MS2_STEP_TIMING, st) == MS2_OK;
  double ms = 0.0;
  int32_t k = 0;
  if (ok) ok = ms2_batch_timing(b, &ms, &k) == MS2_OK;
  if (ok && k > 0) us = 1e3 * ms / (double)(k * copies);
  ms2_batch_destroy(b);
  return us;
}

}  // namespace

extern "C" ms2_status ms2_autotune(ms2_ctx* ctx, int32_t precision, int32_t n_lo, int32_t n_hi,
                                   double* h_report, int32_t max_report, int32_t* n_report,
                                   void* stream) {
  if (!ctx || n_lo < 2 || n_hi < n_lo || (precision != MS2_FP32 && precision != MS2_FP64))
    return set_error(MS2_EINVAL, "bad autotune arguments");
  hipStream_t st = (hipStream_t)stream;
  int rows = 0;
  for (int bucket = size_bucket(n_lo); bucket <= size_bucket(n_hi); ++bucket) {
    // representative size: the bucket's geometric middle, clipped to the range
    int n = (int)std::lround(std::ldexp(1.41421356, bucket));
    n = std::max(n_lo, std::min(n_hi, n));
    Synthetic syn;
    make_synthetic(ctx, n, precision, syn);
    for (int mode = 0; mode <= 1; ++mode) {
      std::vector<TileCfg> cand;
      for (int S = 1; S <= kMaxSplits; S *= 2) {
        TileCfg sym;   // symmetric 64 x 64 tile pairs, S items per tile pair
        sym.waves = 0;
        sym.jchunk = 64 / S;
        cand.push_back(sym);
      }
      const int wmax = (mode == 1 && ctx->cls <= 3) ? 4 : 1;
      for (int w = 1; w <= wmax; w *= 4)
        for (int j = 64 * w; j <= std::max(64 * w, 2 * n); j *= 2) {
          TileCfg c;
          c.waves = w;
          c.jchunk = j;
          cand.push_back(c);
          if (j >= n) break;  // one chunk covers every j
        }
      const int copies = mode == 0 ? 1 : std::max(1, std::min(256, (131072 + n - 1) / n));
      double best = 1e300;
      TileCfg best_cfg = tile_config(ctx, mode, precision, n);
      for (const TileCfg& c : cand) {
        ctx->tuned[std::make_tuple(mode, precision, bucket)] = c;
        const double us = time_shape(ctx, syn, mode, copies, st);
        if (h_report && rows < max_report) {
          double* r = h_report + 5 * rows;
          r[0] = mode;
          r[1] = n;
          r[2] = c.waves;
          r[3] = c.jchunk;
          r[4] = us;
        }
        rows++;
        if (us > 0.0 && us < best) {
          best = us;
          best_cfg = c;
        }
      }
      ctx->tuned[std::make_tuple(mode, precision, bucket)] = best_cfg;
    }
  }
  if (n_report) *n_report = std::min(rows, max_report);
  return MS2_OK;
}
