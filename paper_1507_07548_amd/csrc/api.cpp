// Host side of the C ABI: validation, per-system constants, device tables,
// scratch management and launch sequencing.  All arithmetic of the hot path
// runs in the HIP kernels; the host only derives constants (reaction-field
// coefficients, LJ tail coefficients, Ewald self/intramolecular terms, the
// k-vector list) and builds the work-item list of the pair kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "batch.h"
#include "internal.h"

namespace ms2 {
hipError_t launch_site_frame(int cls, int precision, const SlotDev* slots, const SysParams* prm,
                             const SpeciesTable* tab, int nslots, int max_n, hipStream_t st);
hipError_t launch_pair(int cls, int precision, int waves, bool heat_flux, bool site_cut, int form,
                       const WorkItem* items, int base, int count, const SlotDev* slots, const SysParams* prm,
                       const SpeciesTable* tab, hipStream_t st);
hipError_t launch_reduce_pair(const SlotDev* slots, const SysParams* prm, int nslots, int max_n,
                              hipStream_t st);
hipError_t launch_kspace(const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                         int nslots, int max_kblocks, int max_mchunks, int max_mtiles,
                         int max_kchunks, hipStream_t st);

static thread_local std::string g_last_error;

ms2_status set_error(ms2_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

ms2_status hip_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return MS2_OK;
  return set_error(e == hipErrorOutOfMemory ? MS2_ENOMEM : MS2_EDEVICE,
                   std::string(where) + ": " + hipGetErrorString(e));
}

#define MS2_HIP(call)                                           \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return hip_status(e_, #call);         \
  } while (0)

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

hipError_t DevBuf::ensure(size_t need) {
  if (need <= bytes) return hipSuccess;
  if (p) {
    hipError_t e = hipDeviceSynchronize();  // old contents may still be in use
    if (e != hipSuccess) return e;
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  size_t sz = std::max<size_t>(need, 256);
  hipError_t e = hipMalloc(&p, sz);
  if (e == hipSuccess) bytes = sz;
  return e;
}

// ---------------------------------------------------------------------------
// species table and model class
// ---------------------------------------------------------------------------
static ms2_status build_species_table(const ms2_species* in, int nsp, SpeciesTable& t) {
  std::memset(&t, 0, sizeof(t));
  t.nsp = nsp;
  int lj_types = 0;
  for (int s = 0; s < nsp; ++s) {
    const ms2_species& x = in[s];
    SpeciesDev& d = t.sp[s];
    if (x.n_sites < 1 || x.n_sites > MS2_MAX_SITES)
      return set_error(MS2_EINVAL, "species " + std::to_string(s) + ": n_sites out of range");
    if (!(x.mass > 0.0) || !std::isfinite(x.mass))
      return set_error(MS2_EINVAL, "species " + std::to_string(s) + ": mass must be > 0");
    d.mass = x.mass;
    d.rot_dof = 0;
    for (int k = 0; k < 3; ++k) {
      if (!(x.inertia[k] >= 0.0)) return set_error(MS2_EINVAL, "negative moment of inertia");
      d.inertia[k] = x.inertia[k];
      d.rot_dof += x.inertia[k] > 0.0;
    }
    d.lj_type0 = lj_types;
    for (int a = 0; a < x.n_sites; ++a) {
      const double* p = x.pos[a];
      const double* e = x.axis[a];
      switch (x.type[a]) {
        case MS2_SITE_LJ:
          if (!(x.sigma[a] >= 0.0) || !(x.eps[a] >= 0.0))
            return set_error(MS2_EINVAL, "LJ site with negative sigma or eps");
          std::memcpy(d.lj_pos[d.nlj], p, sizeof(double) * 3);
          d.lj_sigma[d.nlj] = x.sigma[a];
          d.lj_eps[d.nlj] = x.eps[a];
          d.nlj++;
          lj_types++;
          break;
        case MS2_SITE_CHARGE:
          std::memcpy(d.ch_pos[d.nch], p, sizeof(double) * 3);
          d.ch_q[d.nch] = x.mag[a];
          d.net_charge += x.mag[a];
          d.nch++;
          break;
        case MS2_SITE_DIPOLE:
        case MS2_SITE_QUAD: {
          const double nrm = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
          if (!(std::fabs(nrm - 1.0) < 1e-9))
            return set_error(MS2_EINVAL, "dipole/quadrupole axis must be a unit vector");
          if (x.type[a] == MS2_SITE_DIPOLE) {
            std::memcpy(d.dp_pos[d.ndp], p, sizeof(double) * 3);
            std::memcpy(d.dp_axis[d.ndp], e, sizeof(double) * 3);
            d.dp_mu[d.ndp] = x.mag[a];
            d.ndp++;
          } else {
            std::memcpy(d.qd_pos[d.nqd], p, sizeof(double) * 3);
            std::memcpy(d.qd_axis[d.nqd], e, sizeof(double) * 3);
            d.qd_Q[d.nqd] = x.mag[a];
            d.nqd++;
          }
          break;
        }
        default:
          return set_error(MS2_EINVAL, "unknown site type");
      }
    }
  }
  if (lj_types > kMaxRdfTypes) return set_error(MS2_EINVAL, "too many LJ site types");
  t.n_lj_types = lj_types;
  for (int A = 0; A < nsp; ++A)
    for (int B = 0; B < nsp; ++B) {
      const SpeciesDev &a = t.sp[A], &b = t.sp[B];
      const int ne_a = a.nch + a.ndp + a.nqd, ne_b = b.nch + b.ndp + b.nqd;
      t.nsite_pair[A][B] = a.nlj * b.nlj + ne_a * ne_b;
      for (int x = 0; x < a.nlj; ++x)
        for (int y = 0; y < b.nlj; ++y) {
          const double sig = 0.5 * (a.lj_sigma[x] + b.lj_sigma[y]);
          const double eps = std::sqrt(a.lj_eps[x] * b.lj_eps[y]);
          const double s6 = sig * sig * sig * sig * sig * sig;
          t.c6[A][x][B][y] = 4.0 * eps * s6;
          t.c12[A][x][B][y] = 4.0 * eps * s6 * s6;
        }
    }
  return MS2_OK;
}

static int pick_class(const SpeciesTable& t) {
  int lj = 0, ch = 0, dp = 0, qd = 0;
  bool central = true;
  auto at_centre = [](const double* p) { return p[0] == 0.0 && p[1] == 0.0 && p[2] == 0.0; };
  for (int s = 0; s < t.nsp; ++s) {
    const SpeciesDev& d = t.sp[s];
    lj = std::max(lj, d.nlj);
    ch = std::max(ch, d.nch);
    dp = std::max(dp, d.ndp);
    qd = std::max(qd, d.nqd);
    for (int a = 0; a < d.ndp; ++a) central &= at_centre(d.dp_pos[a]);
    for (int a = 0; a < d.nqd; ++a) central &= at_centre(d.qd_pos[a]);
  }
  for (int c = 0; c < kNumClasses; ++c)
    if (lj <= kClassShapes[c].lj && ch <= kClassShapes[c].ch && dp <= kClassShapes[c].dp &&
        qd <= kClassShapes[c].qd && (central || !kClassShapes[c].central || (dp + qd) == 0))
      return c;
  return -1;
}

// ---------------------------------------------------------------------------
// per-system constants
// ---------------------------------------------------------------------------
// largest distance of an LJ site from its molecule's centre
double lj_extent(const ms2_ctx* ctx) {
  double d = 0.0;
  for (int s = 0; s < ctx->tab.nsp; ++s)
    for (int a = 0; a < ctx->tab.sp[s].nlj; ++a) {
      const double* r = ctx->tab.sp[s].lj_pos[a];
      d = std::max(d, std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]));
    }
  return d;
}

ms2_status check_params(const ms2_ctx* ctx, const ms2_params* p) {
  if (!p) return set_error(MS2_EINVAL, "params is NULL");
  if (!(p->box > 0.0) || !std::isfinite(p->box)) return set_error(MS2_EINVAL, "box must be > 0");
  if (!(p->rc > 0.0) || !(2.0 * p->rc < p->box))
    return set_error(MS2_EINVAL, "cut-off must satisfy 0 < rc < box/2");
  if (p->elec < MS2_ELEC_NONE || p->elec > MS2_ELEC_EWALD)
    return set_error(MS2_EINVAL, "unknown electrostatics mode");
  if (p->precision != MS2_FP64 && p->precision != MS2_FP32)
    return set_error(MS2_EINVAL, "precision must be MS2_FP64 or MS2_FP32");
  if (!std::isfinite(p->coulomb_k)) return set_error(MS2_EINVAL, "coulomb_k must be finite");
  if (p->cutoff_mode != MS2_CUT_COM && p->cutoff_mode != MS2_CUT_SITE)
    return set_error(MS2_EINVAL, "cutoff_mode must be MS2_CUT_COM or MS2_CUT_SITE");
  if (p->cutoff_mode == MS2_CUT_SITE && !(2.0 * (p->rc + 2.0 * lj_extent(ctx)) < p->box))
    return set_error(MS2_EINVAL, "site-site cut-off needs rc + 2 d_max < box/2 (d_max: largest LJ-site offset)");
  if (p->elec == MS2_ELEC_RF && !(p->eps_rf >= 1.0))
    return set_error(MS2_EINVAL, "reaction field needs eps_rf >= 1");
  if (p->elec == MS2_ELEC_EWALD) {
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha))
      return set_error(MS2_EINVAL, "Ewald needs alpha > 0");
    if (p->kmax2 < 1 || p->kmax2 > 1600) return set_error(MS2_EINVAL, "Ewald kmax2 out of [1, 1600]");
    for (int s = 0; s < ctx->tab.nsp; ++s)
      if (ctx->tab.sp[s].ndp || ctx->tab.sp[s].nqd)
        return set_error(MS2_EINVAL, "Ewald supports LJ and charge sites only");
  }
  return MS2_OK;
}

void build_sys_params(const ms2_ctx* ctx, const ms2_params* p, int nk, SysParams& s) {
  std::memset(&s, 0, sizeof(s));
  s.L = p->box;
  s.invL = 1.0 / p->box;
  s.rc = p->rc;
  s.rc2 = p->rc * p->rc;
  s.V = p->box * p->box * p->box;
  s.ke = p->coulomb_k;
  s.inv_ke = p->coulomb_k != 0.0 ? 1.0 / p->coulomb_k : 0.0;   // k_e = 0: no electrostatics, not 0 * inf
  s.elec = p->elec;
  s.kmax2 = p->kmax2;
  s.nk = nk;
  s.lrc = p->lj_lrc ? 1 : 0;
  s.precision = p->precision;
  s.cls = ctx->cls;
  s.nsp = ctx->tab.nsp;
  s.site_cut = p->cutoff_mode == MS2_CUT_SITE ? 1 : 0;
  if (s.site_cut) {
    // no LJ site pair of centres farther apart than rc + 2 d_max can be
    // closer than rc
    const double rs = p->rc + 2.0 * lj_extent(ctx);
    s.rc2_search = rs * rs;
  } else {
    s.rc2_search = s.rc2;
  }
  const double rc3 = p->rc * p->rc * p->rc;
  if (p->elec == MS2_ELEC_RF) {
    s.krf = std::isinf(p->eps_rf) ? 0.5 / rc3 : (p->eps_rf - 1.0) / ((2.0 * p->eps_rf + 1.0) * rc3);
    s.crf = 1.0 / p->rc + s.krf * p->rc * p->rc;
  }
  if (p->elec == MS2_ELEC_EWALD) {
    s.alpha = p->alpha;
    s.alpha2 = p->alpha * p->alpha;
    s.gpref = 2.0 * p->alpha / std::sqrt(M_PI);
    for (int A = 0; A < ctx->tab.nsp; ++A) {
      const SpeciesDev& d = ctx->tab.sp[A];
      double c = 0.0;
      for (int a = 0; a < d.nch; ++a) {
        c -= p->coulomb_k * p->alpha / std::sqrt(M_PI) * d.ch_q[a] * d.ch_q[a];
        for (int b = a + 1; b < d.nch; ++b) {
          const double dx = d.ch_pos[a][0] - d.ch_pos[b][0], dy = d.ch_pos[a][1] - d.ch_pos[b][1],
                       dz = d.ch_pos[a][2] - d.ch_pos[b][2];
          const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
          c -= p->coulomb_k * d.ch_q[a] * d.ch_q[b] * std::erf(p->alpha * r) / r;
        }
      }
      s.ew_const[A] = c;
    }
  }
  // LJ tail integrals from rc to infinity of r^2 u, r^3 u', r^4 u'' with
  // u = c12 r^-12 - c6 r^-6, times 2 pi / V (multiplied by N_A N_B later)
  const double rc9 = rc3 * rc3 * rc3;
  for (int A = 0; A < ctx->tab.nsp; ++A)
    for (int B = 0; B < ctx->tab.nsp; ++B) {
      double u = 0, us = 0, uss = 0;
      for (int a = 0; a < ctx->tab.sp[A].nlj; ++a)
        for (int b = 0; b < ctx->tab.sp[B].nlj; ++b) {
          const double c6 = ctx->tab.c6[A][a][B][b], c12 = ctx->tab.c12[A][a][B][b];
          u += c12 / (9.0 * rc9) - c6 / (3.0 * rc3);
          us += -4.0 * c12 / (3.0 * rc9) + 2.0 * c6 / rc3;
          uss += 52.0 * c12 / (3.0 * rc9) - 14.0 * c6 / rc3;
        }
      const double pre = 2.0 * M_PI / s.V;
      s.lrc_u[A][B] = pre * u;
      s.lrc_us[A][B] = pre * us;
      s.lrc_uss[A][B] = pre * uss;
    }
}

ms2_status kvec_table(ms2_ctx* ctx, int kmax2, const KVec** d_out, int* nk) {
  auto it = ctx->kvecs.find(kmax2);
  if (it == ctx->kvecs.end()) {
    std::vector<KVec> v;
    const int m = (int)std::floor(std::sqrt((double)kmax2));
    for (int x = 0; x <= m; ++x)
      for (int y = -m; y <= m; ++y)
        for (int z = -m; z <= m; ++z) {
          const int n2 = x * x + y * y + z * z;
          if (n2 == 0 || n2 > kmax2) continue;
          if (x == 0 && (y < 0 || (y == 0 && z < 0))) continue;
          v.push_back(KVec{x, y, z, n2});
        }
    DevBuf b;
    MS2_HIP(b.ensure(v.size() * sizeof(KVec)));
    MS2_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(KVec), hipMemcpyHostToDevice));
    it = ctx->kvecs.emplace(kmax2, std::make_pair(b, (int)v.size())).first;
  }
  *d_out = reinterpret_cast<const KVec*>(it->second.first.p);
  *nk = it->second.second;
  return MS2_OK;
}

// ---------------------------------------------------------------------------
// tile shapes (per model class, precision, n and launch mode)
// ---------------------------------------------------------------------------
int size_bucket(int n) {
  int b = 0;
  while ((2 << b) <= n) ++b;
  return b;  // floor(log2 n)
}

TileCfg default_sym_shape(int n, int target) {
  const int nt = (n + 63) / 64, items = nt * (nt + 1) / 2;
  int S = 1;
  while (S < kMaxSplits && items * S < target) S *= 2;
  TileCfg c;
  c.waves = 0;
  c.jchunk = 64 / S;
  return c;
}

TileCfg default_shape(const ms2_ctx* ctx, int n) {
  // one item per CU for the light pair classes (LJ, 2CLJQ, Stockmayer); four
  // for classes with charges or off-centre multipoles, whose longer pair
  // evaluations leave the per-item work a smaller share (water + ions, lone
  // step, S = 1 / 2 / 4: N = 500: 106 / 88 / 79 us; N = 1000: 127 / 103 / 98;
  // N = 2000: 156 / 139 / 147)
  const bool heavy = ctx->cls == 2 || ctx->cls >= 4;
  return default_sym_shape(n, ctx->cus * (heavy ? 4 : 1));
}

TileCfg tile_config(const ms2_ctx* ctx, int mode, int precision, int n) {
  auto it = ctx->tuned.find(std::make_tuple(mode, precision, size_bucket(n)));
  if (it != ctx->tuned.end()) return it->second;
  // untuned: symmetric tile pairs, every pair evaluated once, in both launch
  // modes (one system per launch as well: 1.2-2.5x faster than row-owned
  // items from N = 500 to 8192 for the LJ, 2CLJQ and ionic models); small
  // systems deal each tile pair to 2 or 4 items so that they fill the
  // device (a lone 2CLJQ system, N = 256 / 1000: 42 -> 36 / 50 -> 43 us per
  // MD step; water + ions, N = 1000: 127 -> 98 us).  The shape depends on the
  // context's model class and n alone, so a system gets the same items alone
  // and in a mix.
  (void)mode;
  (void)precision;
  return default_shape(ctx, n);
}

static bool single_species_form(const ms2_ctx* ctx) {
  if (ctx->tab.nsp != 1) return false;
  const SpeciesDev& d = ctx->tab.sp[0];
  const ClassShape& S = kClassShapes[ctx->cls];
  return (S.lj == 0 || d.nlj >= 1) && (S.ch == 0 || d.nch >= 1) && (S.dp == 0 || d.ndp >= 1) &&
         (S.qd == 0 || d.nqd >= 1);
}

double linear_h(const ms2_ctx* ctx) {
  if (ctx->cls != 1 || !single_species_form(ctx)) return 0.0;
  const SpeciesDev& d = ctx->tab.sp[0];
  if (d.nlj != 2 || d.nqd != 1 || d.nch != 0 || d.ndp != 0) return 0.0;
  const double* a = d.lj_pos[0];
  const double* b = d.lj_pos[1];
  const double* e = d.qd_axis[0];
  const double* q = d.qd_pos[0];
  if (q[0] != 0.0 || q[1] != 0.0 || q[2] != 0.0) return 0.0;
  if (d.lj_sigma[0] != d.lj_sigma[1] || d.lj_eps[0] != d.lj_eps[1]) return 0.0;
  if (a[0] != -b[0] || a[1] != -b[1] || a[2] != -b[2]) return 0.0;   // symmetric about the centre
  const double h = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  if (!(h > 0.0)) return 0.0;
  // on the axis: a = +-h e to rounding
  const double cx = a[1] * e[2] - a[2] * e[1], cy = a[2] * e[0] - a[0] * e[2], cz = a[0] * e[1] - a[1] * e[0];
  if (std::sqrt(cx * cx + cy * cy + cz * cz) > 1e-12 * h) return 0.0;
  return h;
}

int pair_form(const ms2_ctx* ctx) {
  if (linear_h(ctx) > 0.0) return kFormLinear;
  return single_species_form(ctx) ? kFormOneSpecies : kFormGeneral;
}

int build_items(int n, const TileCfg& c, int slot, std::vector<WorkItem>& out, int* jsplits) {
  if (c.waves == 0) {  // symmetric: tile pairs (I, J >= I) of 64 molecules, S items each
    const int nt = (n + 63) / 64, S = sym_splits(c);
    int local = 0;
    for (int I = 0; I < nt; ++I)
      for (int J = I; J < nt; ++J)
        for (int sp = 0; sp < S; ++sp) {
          // partial index k S + sp of tile index k: each written by one item
          WorkItem w{};
          w.slot = slot;
          w.i0 = 64 * I;
          w.j0 = 64 * J;
          w.j1 = std::min(n, 64 * J + 64);
          w.part = J * S + sp;
          w.part_j = I * S + sp;
          w.local = local++;
          w.split = S > 1 ? sp + 256 * S : 0;
          out.push_back(w);
        }
    *jsplits = nt * S;
    return local;
  }
  const int it = 64 * c.waves;
  const int js = (n + c.jchunk - 1) / c.jchunk;
  int local = 0;
  for (int i0 = 0; i0 < n; i0 += it)
    for (int p = 0; p < js; ++p) {
      WorkItem w{};
      w.slot = slot;
      w.i0 = i0;
      w.j0 = p * c.jchunk;
      w.j1 = std::min(n, (p + 1) * c.jchunk);
      w.part = p;
      w.local = local++;
      out.push_back(w);
    }
  *jsplits = js;
  return local;
}

// ---------------------------------------------------------------------------
// single-system calls: parameters travel through a ring of pinned blocks
// ---------------------------------------------------------------------------
ms2_status ring_acquire(ms2_ctx* ctx, RingSlot** out) {
  RingSlot& r = ctx->ring[ctx->ring_pos];
  ctx->ring_pos = (ctx->ring_pos + 1) % kRing;
  if (r.used) MS2_HIP(hipEventSynchronize(r.ev));
  r.used = true;
  *out = &r;
  return MS2_OK;
}

static ms2_status single_setup(ms2_ctx* ctx, const ms2_params* p, int n, const int32_t* d_species,
                               const double* d_com, const double* d_quat, double* d_force,
                               double* d_torque, double* d_sums, bool kspace, hipStream_t st,
                               RingSlot** ring_out, TileCfg* cfg_out, int* nitems_out) {
  if (!ctx) return set_error(MS2_EINVAL, "context is NULL");
  if (n < 2) return set_error(MS2_EINVAL, "n_mol must be >= 2");
  if (!d_species || !d_com || !d_quat || !d_force || !d_torque || !d_sums)
    return set_error(MS2_EINVAL, "NULL device pointer");
  ms2_status s = check_params(ctx, p);
  if (s != MS2_OK) return s;
  if (kspace && p->elec != MS2_ELEC_EWALD)
    return set_error(MS2_EINVAL, "ms2_ewald_kspace needs elec == MS2_ELEC_EWALD");
  MS2_HIP(hipSetDevice(ctx->device));
  const int npad = (n + 63) & ~63;
  TileCfg cfg = tile_config(ctx, 0, p->precision, n);
  if (p->cutoff_mode == MS2_CUT_SITE && cfg.waves != 0) {   // the site-site cut-off runs on symmetric items only
    cfg.waves = 0;
    cfg.jchunk = 64;
  }
  const int rs = p->precision == MS2_FP32 ? 4 : 8;

  // items (cached per n and tile shape)
  auto key = std::make_tuple(n, cfg.waves, cfg.jchunk);
  auto ic = ctx->item_cache.find(key);
  if (ic == ctx->item_cache.end()) {
    std::vector<WorkItem> items;
    int js = 0;
    build_items(n, cfg, 0, items, &js);
    DevBuf b;
    MS2_HIP(b.ensure(items.size() * sizeof(WorkItem)));
    MS2_HIP(hipMemcpy(b.p, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice));
    ic = ctx->item_cache.emplace(key, CachedItems{b, (int)items.size(), js}).first;
  }
  const int nitems = ic->second.count, js = ic->second.jsplits;

  const KVec* kv = nullptr;
  int nk = 0;
  if (p->elec == MS2_ELEC_EWALD) {
    s = kvec_table(ctx, p->kmax2, &kv, &nk);
    if (s != MS2_OK) return s;
  }
  const int mchunks = (n + kMolTile - 1) / kMolTile;
  const int kchunks = (nk + kKChunk - 1) / kKChunk;
  const int mtiles = (n + kMolTile - 1) / kMolTile;
  MS2_HIP(ctx->s_sites.ensure((size_t)class_reals(ctx->cls) * npad * rs));
  if (p->cutoff_mode == MS2_CUT_SITE) MS2_HIP(ctx->s_lj64.ensure((size_t)3 * class_lj(ctx->cls) * npad * 8));
  MS2_HIP(ctx->s_pf.ensure((size_t)js * 6 * npad * 8));
  MS2_HIP(ctx->s_bsum.ensure((size_t)nitems * kNumBlockSums * 8));
  if (nk) {
    MS2_HIP(ctx->s_skp.ensure((size_t)mchunks * nk * 2 * 8));
    MS2_HIP(ctx->s_sk.ensure((size_t)nk * 2 * 8));
    MS2_HIP(ctx->s_fk.ensure((size_t)kchunks * 6 * npad * 8));
    MS2_HIP(ctx->s_kred.ensure((size_t)kchunks * mtiles * 8));
    MS2_HIP(ctx->s_ksum.ensure(4 * 8));
  }

  RingSlot* r = nullptr;
  s = ring_acquire(ctx, &r);
  if (s != MS2_OK) return s;
  build_sys_params(ctx, p, nk, *r->h_prm);
  SlotDev& d = *r->h_slot;
  std::memset(&d, 0, sizeof(d));
  d.n = n;
  d.npad = npad;
  d.jsplits = js;
  d.nitems = nitems;
  d.active = 1;
  d.symmetric = cfg.waves == 0 ? 1 : 0;
  d.kchunks = kchunks;
  d.mchunks = mchunks;
  d.com_ld = n;
  d.species = d_species;
  d.com = d_com;
  d.quat = d_quat;
  d.sites = ctx->s_sites.p;
  d.lj64 = p->cutoff_mode == MS2_CUT_SITE ? (double*)ctx->s_lj64.p : nullptr;
  d.pf = ctx->s_pf.p;
  d.pf_single = p->precision == MS2_FP32 ? 1 : 0;
  d.bsum = (double*)ctx->s_bsum.p;
  d.force = d_force;
  d.torque = d_torque;
  d.sums = d_sums;
  d.sk_part = (double*)ctx->s_skp.p;
  d.sk = (double*)ctx->s_sk.p;
  d.fk = (double*)ctx->s_fk.p;
  d.kred = (double*)ctx->s_kred.p;
  d.ksum = (double*)ctx->s_ksum.p;
  d.kvec = kv;
  d.nk = nk;
  d.mtiles = mtiles;
  d.err = ctx->d_err;
  MS2_HIP(hipMemcpyAsync(r->d_slot, r->h_slot, sizeof(SlotDev), hipMemcpyHostToDevice, st));
  MS2_HIP(hipMemcpyAsync(r->d_prm, r->h_prm, sizeof(SysParams), hipMemcpyHostToDevice, st));
  *ring_out = r;
  *cfg_out = cfg;
  *nitems_out = nitems;
  return MS2_OK;
}

}  // namespace ms2

using namespace ms2;

extern "C" {

const char* ms2_last_error(void) { return g_last_error.c_str(); }

ms2_status ms2_create(ms2_ctx** out, const ms2_species* h_species, int32_t n_species,
                      int32_t device) {
  if (!out) return set_error(MS2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!h_species || n_species < 1 || n_species > MS2_MAX_SPECIES)
    return set_error(MS2_EINVAL, "need 1..MS2_MAX_SPECIES species");
  int ndev = 0;
  MS2_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error(MS2_EINVAL, "no such HIP device");
  ms2_ctx* c = new ms2_ctx();
  c->device = device;
  ms2_status s = build_species_table(h_species, n_species, c->tab);
  if (s != MS2_OK) {
    delete c;
    return s;
  }
  c->cls = pick_class(c->tab);
  if (c->cls < 0) {
    delete c;
    return set_error(MS2_EINVAL, "site counts exceed every compiled model class");
  }
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess) e = hipMalloc(&c->d_tab, sizeof(SpeciesTable));
  if (e == hipSuccess) e = hipMemcpy(c->d_tab, &c->tab, sizeof(SpeciesTable), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&c->d_err, sizeof(int));
  if (e == hipSuccess) e = hipMemset(c->d_err, 0, sizeof(int));
  if (e == hipSuccess) e = noalloc_scratch_attach(device);
  for (int k = 0; k < kRing && e == hipSuccess; ++k) {
    RingSlot& r = c->ring[k];
    e = hipHostMalloc((void**)&r.h_slot, sizeof(SlotDev), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&r.h_prm, sizeof(SysParams), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc((void**)&r.d_slot, sizeof(SlotDev));
    if (e == hipSuccess) e = hipMalloc((void**)&r.d_prm, sizeof(SysParams));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r.ev, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    ms2_destroy(c);
    return hip_status(e, "ms2_create");
  }
  *out = c;
  return MS2_OK;
}

void ms2_destroy(ms2_ctx* c) {
  if (!c) return;
  while (!c->batches.empty()) ms2_batch_destroy(c->batches.back());   // unregisters itself
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (int k = 0; k < kRing; ++k) {
    RingSlot& r = c->ring[k];
    if (r.h_slot) (void)hipHostFree(r.h_slot);
    if (r.h_prm) (void)hipHostFree(r.h_prm);
    if (r.d_slot) (void)hipFree(r.d_slot);
    if (r.d_prm) (void)hipFree(r.d_prm);
    if (r.ev) (void)hipEventDestroy(r.ev);
  }
  if (c->d_tab) (void)hipFree(c->d_tab);
  if (c->d_err) (void)hipFree(c->d_err);
  c->s_sites.release();
  c->s_lj64.release();
  c->s_pf.release();
  c->s_bsum.release();
  c->s_skp.release();
  c->s_sk.release();
  c->s_fk.release();
  c->s_kred.release();
  c->s_ksum.release();
  for (auto& kv : c->kvecs) kv.second.first.release();
  for (auto& it : c->item_cache) it.second.buf.release();
  delete c;
}

ms2_status ms2_forces(ms2_ctx* ctx, const ms2_params* h_params, int32_t n_mol,
                      const int32_t* d_species, const double* d_com, const double* d_quat,
                      double* d_force, double* d_torque, double* d_sums, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  RingSlot* r = nullptr;
  TileCfg cfg;
  int nitems = 0;
  (void)hipGetLastError();   // launch checks below must not see an unrelated earlier error
  ms2_status s = single_setup(ctx, h_params, n_mol, d_species, d_com, d_quat, d_force, d_torque,
                              d_sums, false, st, &r, &cfg, &nitems);
  if (s != MS2_OK) return s;
  const ms2::CachedItems& ci = ctx->item_cache[std::make_tuple(n_mol, cfg.waves, cfg.jchunk)];
  MS2_HIP(launch_site_frame(ctx->cls, h_params->precision, r->d_slot, r->d_prm, ctx->d_tab, 1, n_mol, st));
  MS2_HIP(launch_pair(ctx->cls, h_params->precision, cfg.waves, false, h_params->cutoff_mode == MS2_CUT_SITE,
                      pair_form(ctx), (const WorkItem*)ci.buf.p, 0, nitems,
                      r->d_slot, r->d_prm, ctx->d_tab, st));
  MS2_HIP(launch_reduce_pair(r->d_slot, r->d_prm, 1, n_mol, st));
  MS2_HIP(hipEventRecord(r->ev, st));
  return MS2_OK;
}

ms2_status ms2_ewald_kspace(ms2_ctx* ctx, const ms2_params* h_params, int32_t n_mol,
                            const int32_t* d_species, const double* d_com, const double* d_quat,
                            double* d_force, double* d_torque, double* d_sums, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  RingSlot* r = nullptr;
  TileCfg cfg;
  int nitems = 0;
  (void)hipGetLastError();
  ms2_status s = single_setup(ctx, h_params, n_mol, d_species, d_com, d_quat, d_force, d_torque,
                              d_sums, true, st, &r, &cfg, &nitems);
  if (s != MS2_OK) return s;
  const SlotDev& d = *r->h_slot;
  MS2_HIP(launch_kspace(r->d_slot, r->d_prm, ctx->d_tab, 1, (d.nk + 63) / 64, d.mchunks, d.mtiles,
                        d.kchunks, st));
  MS2_HIP(hipEventRecord(r->ev, st));
  return MS2_OK;
}

ms2_status ms2_device_errors(ms2_ctx* ctx, void* stream) {
  if (!ctx) return set_error(MS2_EINVAL, "context is NULL");
  MS2_HIP(hipSetDevice(ctx->device));
  MS2_HIP(hipStreamSynchronize((hipStream_t)stream));
  int word = 0;
  MS2_HIP(hipMemcpy(&word, ctx->d_err, sizeof(int), hipMemcpyDeviceToHost));
  if (!word) return MS2_OK;
  const int zero = 0;
  MS2_HIP(hipMemcpy(ctx->d_err, &zero, sizeof(int), hipMemcpyHostToDevice));
  return set_error(MS2_EINVAL, "a device species array held an index outside [0, n_species): "
                               "the outputs of that call are NaN");
}

ms2_status ms2_tile_config(ms2_ctx* ctx, int32_t mode, int32_t n_mol, int32_t precision,
                           int32_t* wave_rows, int32_t* j_chunk) {
  if (!ctx || !wave_rows || !j_chunk || n_mol < 2 || (mode != 0 && mode != 1))
    return set_error(MS2_EINVAL, "bad arguments");
  TileCfg c = tile_config(ctx, mode, precision, n_mol);
  *wave_rows = c.waves;
  *j_chunk = c.jchunk;
  return MS2_OK;
}

ms2_status ms2_set_tile_config(ms2_ctx* ctx, int32_t mode, int32_t n_mol, int32_t precision,
                               int32_t wave_rows, int32_t j_chunk) {
  if (!ctx || n_mol < 2 || (mode != 0 && mode != 1) || (precision != MS2_FP32 && precision != MS2_FP64))
    return set_error(MS2_EINVAL, "bad arguments");
  if (!(wave_rows == 0 || wave_rows == 1 || (wave_rows == 4 && ctx->cls <= 3)))
    return set_error(MS2_EINVAL,
                     "wave_rows must be 0 (symmetric), 1, or 4 (first four model classes only)");
  if (wave_rows == 0 && j_chunk != 64 && j_chunk != 32 && j_chunk != 16)
    return set_error(MS2_EINVAL, "symmetric tiles use j_chunk = 64, 32 or 16 (1, 2 or 4 items per tile pair)");
  if (wave_rows > 0 && (j_chunk < 64 * wave_rows || j_chunk % (64 * wave_rows) != 0))
    return set_error(MS2_EINVAL, "j_chunk must be a positive multiple of 64 * wave_rows");
  TileCfg c;
  c.waves = wave_rows;
  c.jchunk = j_chunk;
  ctx->tuned[std::make_tuple(mode, precision, size_bucket(n_mol))] = c;
  return MS2_OK;
}

}  // extern "C"
