// Batched, device-resident simulation: slots, admission by HBM footprint,
// stepping many systems per launch (optionally replayed from a hipGraph) and
// copying samples out.
//
// Each slot owns one device allocation holding its state (Gear arrays,
// velocities, forces), its force-path scratch (site records, partials,
// Ewald buffers) and its sampler accumulators.  The batch owns the device
// tables indexed by slot (SlotDev, SysParams, MDDev) and the pair-kernel
// work-item list, rebuilt whenever the set of slots changes.  Fields that the
// device updates while stepping (step counters, status, active flags, ACF
// origins) are only ever written by the host for the slot being admitted or
// retired, so other slots keep running undisturbed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "batch.h"

namespace ms2 {
hipError_t launch_pair(int cls, int precision, int waves, bool heat_flux, bool site_cut, int form,
                       const WorkItem* items, int base, int count, const SlotDev* slots, const SysParams* prm,
                       const SpeciesTable* tab, hipStream_t st);
hipError_t launch_reduce_pair(const SlotDev* slots, const SysParams* prm, int nslots, int max_n,
                              hipStream_t st);
hipError_t launch_kspace(const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                         int nslots, int max_kblocks, int max_mchunks, int max_mtiles,
                         int max_kchunks, hipStream_t st);
hipError_t launch_kspace_partials(const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                                  int nslots, int max_kblocks, int max_mchunks, int max_mtiles,
                                  int max_kchunks, hipStream_t st);
hipError_t launch_reduce_pair_kspace(const SlotDev* slots, const SysParams* prm, int nslots, int max_n,
                                     hipStream_t st);
hipError_t launch_md_wrap(MDDev* md, const SysParams* prm, int slot, int n, hipStream_t st);
hipError_t launch_md_init(SlotDev* slots, MDDev* md, const SpeciesTable* tab, int slot,
                          hipStream_t st);
hipError_t launch_md_begin_frame(int cls, int precision, const SlotDev* slots, MDDev* md, const SysParams* prm,
                                 const SpeciesTable* tab, int nslots, int max_n, hipStream_t st);
hipError_t launch_residence(const SlotDev* slots, MDDev* md, const SysParams* prm, int slot_base,
                            int nslots, int max_solute, hipStream_t st);
hipError_t launch_md_end(SlotDev* slots, MDDev* md, const SysParams* prm, const SpeciesTable* tab,
                         int nslots, int max_n, hipStream_t st);
hipError_t launch_rdf(int waves, const WorkItem* items, int base, int count, const SlotDev* slots,
                      const MDDev* md, const SysParams* prm, const SpeciesTable* tab,
                      hipStream_t st);

// number of half-space k vectors with 0 < |n|^2 <= kmax2
int kvec_count(int kmax2) {
  const int m = (int)std::floor(std::sqrt((double)kmax2));
  int c = 0;
  for (int x = 0; x <= m; ++x)
    for (int y = -m; y <= m; ++y)
      for (int z = -m; z <= m; ++z) {
        const int n2 = x * x + y * y + z * z;
        if (n2 == 0 || n2 > kmax2) continue;
        if (x == 0 && (y < 0 || (y == 0 && z < 0))) continue;
        c++;
      }
  return c;
}
}  // namespace ms2

using namespace ms2;

#define MS2_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_status(e_, #call); \
  } while (0)

namespace {

// byte layout of one slot's allocation
struct SlotLayout {
  size_t species, sites, lj64, pf, bsum, force, torque, sums, r, q, w, vel;
  size_t skp, sk, fk, kred, ksum, moments, md_part, rdf, acf_v, acf_j, acf_cnt, origin_v, origin_j,
      origin_t0;
  size_t res_idx, res_state, res_n0, res_part, res_inside, res_acf, res_cnt;
  size_t hf_kin, hf_jq, acf_q, acf_q_cnt, origin_jq, origin_jq_valid;
  size_t total;
};

struct SlotShape {
  int n, npad, cls, precision, jsplits, nitems, waves, jchunk, mode, nk, kchunks, mchunks, mtiles;
  int rdf_ntp, rdf_bins, acf_nlag, acf_max_live;
  int n_solute, n_solvent;   // residence sampling (0 = off)
  int heat_flux;             // heat-flux ACF (symmetric items)
  int site_cut;              // site-site cut-off mode (symmetric items)
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

SlotLayout layout_of(const SlotShape& s) {
  SlotLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align256(std::max<size_t>(bytes, 8));
    return o;
  };
  const size_t n = s.n, np = s.npad, rs = s.precision == MS2_FP32 ? 4 : 8;
  L.species = take(n * 4);
  L.sites = take((size_t)class_reals(s.cls) * np * rs);
  L.lj64 = take(s.site_cut ? (size_t)3 * class_lj(s.cls) * np * 8 : 0);
  L.pf = take((size_t)s.jsplits * 6 * np * rs);
  L.bsum = take((size_t)s.nitems * kNumBlockSums * 8);
  L.force = take(3 * n * 8);
  L.torque = take(3 * n * 8);
  L.sums = take(MS2_NSUM * 8);
  L.r = take(5 * 3 * n * 8);
  L.q = take(5 * 4 * n * 8);
  L.w = take(5 * 3 * n * 8);
  L.vel = take(3 * n * 8);
  L.skp = take((size_t)s.mchunks * s.nk * 2 * 8);
  L.sk = take((size_t)s.nk * 2 * 8);
  L.fk = take((size_t)s.kchunks * 6 * np * 8);
  L.kred = take((size_t)s.kchunks * s.mtiles * 8);
  L.ksum = take(4 * 8);
  L.moments = take(kNumMoments * 8);
  L.md_part = take((n + kMdBlock - 1) / kMdBlock * 8 * 8);
  L.rdf = take((size_t)s.rdf_ntp * s.rdf_bins * 8);
  L.acf_v = take((size_t)s.acf_nlag * 8);
  L.acf_j = take((size_t)s.acf_nlag * 8);
  L.acf_cnt = take((size_t)s.acf_nlag * 8);
  L.origin_v = take((size_t)s.acf_max_live * 3 * n * 8);
  L.origin_j = take((size_t)s.acf_max_live * 3 * 8);
  L.origin_t0 = take((size_t)s.acf_max_live * 8);
  const size_t nu = s.n_solute, nv = s.n_solvent, ml = s.n_solute ? s.acf_max_live : 0;
  L.res_idx = take((nu + nv) * 4);
  L.res_state = take(ml * nu * nv * 2);
  L.res_n0 = take(ml * nu * 4);
  L.res_part = take(nu * ml * 8);
  L.res_inside = take(nu * 4);
  L.res_acf = take(s.n_solute ? (size_t)s.acf_nlag * 8 : 0);
  L.res_cnt = take(s.n_solute ? (size_t)s.acf_nlag * 8 : 0);
  const size_t hf = s.heat_flux ? 1 : 0;
  L.hf_kin = take(hf * 6 * np * rs);
  L.hf_jq = take(hf * 3 * 8);
  L.acf_q = take(hf * (size_t)s.acf_nlag * 8);
  L.acf_q_cnt = take(hf * (size_t)s.acf_nlag * 8);
  L.origin_jq = take(hf * (size_t)s.acf_max_live * 3 * 8);
  L.origin_jq_valid = take(hf * (size_t)s.acf_max_live * 4);
  L.total = off;
  return L;
}


}  // namespace

struct SlotHost {
  bool used = false;
  SlotShape shape{};
  SlotLayout lay{};
  ms2_params params{};
  DevBuf mem;
  SlotDev dev{};
  MDDev md{};
  SysParams prm{};
  const KVec* kvec = nullptr;
};

struct ms2_batch {
  ms2_ctx* ctx = nullptr;
  int max_slots = 0;
  size_t budget = 0, used_bytes = 0;
  std::vector<SlotHost> slots;
  // allocations of retired slots, kept for later admissions: hipFree waits
  // for the whole device, which would stall other batches' work in flight
  std::vector<DevBuf> pool;
  DevBuf d_slots, d_md, d_prm, d_items;
  // work items grouped by (precision, waves): [begin, end) into d_items
  struct Group { int precision, waves, begin, end; bool heat_flux, site_cut; };
  std::vector<Group> groups;
  bool dirty = true;
  int max_n = 2, max_kblocks = 1, max_mchunks = 1, max_mtiles = 1, max_kchunks = 1;
  bool any_ewald = false, any_rdf = false, any_res = false;
  int max_solute = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int graph_steps = 0, graph_flags = 0;
  hipStream_t last_stream = nullptr;
  int flags = 0;
  // pair-kernel timing events, one (begin, end) pair per step
  std::vector<hipEvent_t> ev_begin, ev_end;
  int timed_steps = 0;
};

namespace {

void drop_graph(ms2_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_steps = 0;
}

ms2_status shape_of(ms2_ctx* ctx, const ms2_system* sys, int mode, SlotShape& s) {
  if (!sys) return set_error(MS2_EINVAL, "system is NULL");
  ms2_status st = check_params(ctx, &sys->params);
  if (st != MS2_OK) return st;
  if (sys->n_mol < 2) return set_error(MS2_EINVAL, "n_mol must be >= 2");
  if (!sys->h_species || !sys->h_com || !sys->h_quat || !sys->h_vel || !sys->h_omega)
    return set_error(MS2_EINVAL, "NULL host array in system");
  if (!(sys->dt > 0.0) || !std::isfinite(sys->dt)) return set_error(MS2_EINVAL, "dt must be > 0");
  if (sys->n_steps < 0) return set_error(MS2_EINVAL, "n_steps must be >= 0");
  if (sys->integrator != MS2_VV && sys->integrator != MS2_GEAR)
    return set_error(MS2_EINVAL, "unknown integrator");
  bool rotating = false;
  double dmax = 0.0;
  for (int i = 0; i < sys->n_mol; ++i) {
    const int sp = sys->h_species[i];
    if (sp < 0 || sp >= ctx->tab.nsp) return set_error(MS2_EINVAL, "species index out of range");
  }
  for (int a = 0; a < ctx->tab.nsp; ++a) {
    const SpeciesDev& d = ctx->tab.sp[a];
    if (d.rot_dof) rotating = true;
    for (int k = 0; k < d.nlj; ++k)
      dmax = std::max(dmax, std::sqrt(d.lj_pos[k][0] * d.lj_pos[k][0] + d.lj_pos[k][1] * d.lj_pos[k][1] +
                                      d.lj_pos[k][2] * d.lj_pos[k][2]));
  }
  if (sys->integrator == MS2_VV && rotating)
    return set_error(MS2_EINVAL, "velocity Verlet supports point molecules only");
  s = SlotShape{};
  s.n = sys->n_mol;
  s.npad = (s.n + 63) & ~63;
  s.cls = ctx->cls;
  s.precision = sys->params.precision;
  s.mode = mode;
  TileCfg cfg = tile_config(ctx, mode, s.precision, s.n);
  s.site_cut = sys->params.cutoff_mode == MS2_CUT_SITE ? 1 : 0;
  if ((sys->heat_flux || s.site_cut) && cfg.waves != 0) {   // both are evaluated on symmetric items only
    cfg.waves = 0;
    cfg.jchunk = 64;
  }
  s.waves = cfg.waves;
  s.jchunk = cfg.jchunk;   // frozen at admission: the slot's buffers are sized for it
  if (cfg.waves == 0) {    // symmetric tile pairs, S items each
    const int nt = (s.n + 63) / 64, S = sym_splits(cfg);
    s.jsplits = nt * S;
    s.nitems = nt * (nt + 1) / 2 * S;
  } else {
    s.jsplits = (s.n + cfg.jchunk - 1) / cfg.jchunk;
    s.nitems = ((s.n + 64 * cfg.waves - 1) / (64 * cfg.waves)) * s.jsplits;
  }
  if (sys->params.elec == MS2_ELEC_EWALD) {
    s.nk = kvec_count(sys->params.kmax2);
    s.kchunks = (s.nk + kKChunk - 1) / kKChunk;
    s.mchunks = (s.n + kMolTile - 1) / kMolTile;
    s.mtiles = (s.n + kMolTile - 1) / kMolTile;
  }
  if (sys->rdf_every > 0) {
    if (sys->rdf_bins < 1 || !(sys->rdf_rmax > 0.0))
      return set_error(MS2_EINVAL, "RDF needs rdf_bins >= 1 and rdf_rmax > 0");
    if (!(sys->rdf_rmax + 2.0 * dmax < 0.5 * sys->params.box))
      return set_error(MS2_EINVAL, "RDF range plus LJ-site extent must stay below box/2");
    const int T = ctx->tab.n_lj_types;
    s.rdf_ntp = T * (T + 1) / 2;
    s.rdf_bins = sys->rdf_bins;
  }
  if (sys->acf_every > 0) {
    if (sys->acf_nlag < 1 || sys->acf_origin_every < sys->acf_every ||
        sys->acf_origin_every % sys->acf_every != 0)
      return set_error(MS2_EINVAL, "ACF needs nlag >= 1 and origins on multiples of acf_every");
    s.acf_nlag = sys->acf_nlag;
    s.acf_max_live = (int)((long long)sys->acf_nlag * sys->acf_every / sys->acf_origin_every + 2);
  }
  if (sys->sample_every > 0 && sys->params.elec == MS2_ELEC_EWALD)
    // the reciprocal part has no d2U/ds2 here, so Z = d2U/dV2 and the
    // derivatives built on it would be wrong; the paper does not combine
    // Massieu sampling with Ewald summation either (Sec. 4)
    return set_error(MS2_EINVAL, "Lustig moment sampling (sample_every > 0) is not offered with Ewald summation");
  if (sys->sample_every < 0) return set_error(MS2_EINVAL, "sample_every must be >= 0");
  if (sys->heat_flux) {
    if (sys->acf_every <= 0) return set_error(MS2_EINVAL, "the heat flux is sampled with the ACFs: acf_every > 0");
    if (sys->params.elec == MS2_ELEC_EWALD)
      return set_error(MS2_EINVAL, "heat flux with Ewald summation is not supported");
    s.heat_flux = 1;
  }
  if (sys->res_enable) {
    if (sys->acf_every <= 0) return set_error(MS2_EINVAL, "residence sampling runs on the ACF schedule: acf_every > 0");
    if (sys->res_solute < 0 || sys->res_solute >= ctx->tab.nsp || sys->res_solvent < 0 ||
        sys->res_solvent >= ctx->tab.nsp)
      return set_error(MS2_EINVAL, "residence solute/solvent species out of range");
    if (!(sys->res_radius > 0.0) || !(sys->res_radius < 0.5 * sys->params.box) || sys->res_tolerance < 0 ||
        sys->res_tolerance >= (int)kResDead - 1)
      return set_error(MS2_EINVAL, "residence needs 0 < radius < box/2 and 0 <= tolerance < 65534");
    if (s.acf_max_live > kResMaxLive)
      return set_error(MS2_EINVAL, "too many live ACF origins for residence sampling");
    for (int i = 0; i < s.n; ++i) {
      s.n_solute += sys->h_species[i] == sys->res_solute;
      s.n_solvent += sys->h_species[i] == sys->res_solvent;
    }
    if (s.n_solute == 0 || s.n_solvent == 0)
      return set_error(MS2_EINVAL, "residence solute or solvent species absent from the system");
  }
  return MS2_OK;
}

void rebuild_items(ms2_batch* b) {
  std::vector<WorkItem> all;
  b->groups.clear();
  b->max_n = 2;
  b->max_kblocks = b->max_mchunks = b->max_mtiles = b->max_kchunks = 1;
  b->any_ewald = b->any_rdf = b->any_res = false;
  b->max_solute = 0;
  for (int prec : {MS2_FP64, MS2_FP32})
    for (int hfv : {0, 1})
    for (int scv : {0, 1})
    for (int waves : {0, 1, 4}) {
      ms2_batch::Group g{prec, waves, (int)all.size(), 0, hfv == 1, scv == 1};
      for (int s = 0; s < b->max_slots; ++s) {
        const SlotHost& h = b->slots[s];
        if (!h.used || h.shape.precision != prec || h.shape.waves != waves || h.shape.heat_flux != hfv ||
            h.shape.site_cut != scv)
          continue;
        TileCfg c;
        c.waves = h.shape.waves;
        c.jchunk = h.shape.jchunk;
        int js = 0;
        build_items(h.shape.n, c, s, all, &js);
      }
      g.end = (int)all.size();
      if (g.end > g.begin) b->groups.push_back(g);
    }
  for (int s = 0; s < b->max_slots; ++s) {
    const SlotHost& h = b->slots[s];
    if (!h.used) continue;
    b->max_n = std::max(b->max_n, h.shape.n);
    if (h.params.elec == MS2_ELEC_EWALD) {
      b->any_ewald = true;
      b->max_kblocks = std::max(b->max_kblocks, (h.shape.nk + 63) / 64);
      b->max_mchunks = std::max(b->max_mchunks, h.shape.mchunks);
      b->max_mtiles = std::max(b->max_mtiles, h.shape.mtiles);
      b->max_kchunks = std::max(b->max_kchunks, h.shape.kchunks);
    }
    if (h.md.rdf_every > 0) b->any_rdf = true;
    if (h.shape.n_solute > 0) {
      b->any_res = true;
      b->max_solute = std::max(b->max_solute, h.shape.n_solute);
    }
  }
  if (!all.empty()) {
    // grown with headroom: a reallocation waits for the whole device
    size_t need = all.size() * sizeof(WorkItem);
    if (need > b->d_items.bytes) need += need / 2;
    (void)b->d_items.ensure(need);
    (void)hipMemcpy(b->d_items.p, all.data(), all.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
  }
  b->dirty = false;
}

// the force path for every slot of the batch after the site frame (pair
// part + reduction + k-space)
ms2_status enqueue_forces(ms2_batch* b, hipStream_t st, int timed_step) {
  ms2_ctx* ctx = b->ctx;
  const SlotDev* ds = (const SlotDev*)b->d_slots.p;
  const SysParams* dp = (const SysParams*)b->d_prm.p;
  const WorkItem* di = (const WorkItem*)b->d_items.p;
  if (timed_step >= 0) MS2_HIP(hipEventRecord(b->ev_begin[timed_step], st));
  for (auto& g : b->groups)
    MS2_HIP(launch_pair(ctx->cls, g.precision, g.waves, g.heat_flux, g.site_cut, pair_form(ctx), di, g.begin,
                        g.end - g.begin, ds, dp, ctx->d_tab, st));
  if (timed_step >= 0) MS2_HIP(hipEventRecord(b->ev_end[timed_step], st));
  if (b->any_ewald) {
    // reciprocal partials first; one reduction then adds pair and reciprocal
    // parts (the same bits as the pair reduction followed by the reciprocal ones)
    MS2_HIP(launch_kspace_partials(ds, dp, ctx->d_tab, b->max_slots, b->max_kblocks, b->max_mchunks,
                                   b->max_mtiles, b->max_kchunks, st));
    MS2_HIP(launch_reduce_pair_kspace(ds, dp, b->max_slots, b->max_n, st));
  } else {
    MS2_HIP(launch_reduce_pair(ds, dp, b->max_slots, b->max_n, st));
  }
  return MS2_OK;
}

ms2_status enqueue_step(ms2_batch* b, hipStream_t st, int timed_step) {
  ms2_ctx* ctx = b->ctx;
  SlotDev* ds = (SlotDev*)b->d_slots.p;
  MDDev* dm = (MDDev*)b->d_md.p;
  const SysParams* dp = (const SysParams*)b->d_prm.p;
  // predictor and site frame, one launch per precision in use
  for (int prec : {MS2_FP64, MS2_FP32}) {
    bool any = false;
    for (auto& g : b->groups) any |= g.precision == prec;
    if (any) MS2_HIP(launch_md_begin_frame(ctx->cls, prec, ds, dm, dp, ctx->d_tab, b->max_slots, b->max_n, st));
  }
  ms2_status s = enqueue_forces(b, st, timed_step);
  if (s != MS2_OK) return s;
  MS2_HIP(launch_md_end(ds, dm, dp, ctx->d_tab, b->max_slots, b->max_n, st));
  if (b->any_rdf)
    for (auto& g : b->groups)
      MS2_HIP(launch_rdf(g.waves, (const WorkItem*)b->d_items.p, g.begin, g.end - g.begin, ds, dm, dp,
                         ctx->d_tab, st));
  if (b->any_res) MS2_HIP(launch_residence(ds, dm, dp, 0, b->max_slots, b->max_solute, st));
  return MS2_OK;
}

}  // namespace

extern "C" {

ms2_status ms2_batch_create(ms2_ctx* ctx, int32_t max_slots, size_t hbm_budget, int32_t flags,
                            ms2_batch** out) {
  if (!out) return set_error(MS2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx || max_slots < 1 || max_slots > 65535) return set_error(MS2_EINVAL, "bad batch arguments");
  MS2_HIP(hipSetDevice(ctx->device));
  ms2_batch* b = new ms2_batch();
  b->ctx = ctx;
  b->max_slots = max_slots;
  b->budget = hbm_budget;
  b->flags = flags;
  b->slots.resize(max_slots);
  hipError_t e = b->d_slots.ensure(sizeof(SlotDev) * max_slots);
  if (e == hipSuccess) e = b->d_md.ensure(sizeof(MDDev) * max_slots);
  if (e == hipSuccess) e = b->d_prm.ensure(sizeof(SysParams) * max_slots);
  if (e == hipSuccess) {
    std::vector<SlotDev> zs(max_slots);
    std::vector<MDDev> zm(max_slots);
    std::vector<SysParams> zp(max_slots);
    std::memset(zs.data(), 0, sizeof(SlotDev) * max_slots);
    std::memset(zm.data(), 0, sizeof(MDDev) * max_slots);
    std::memset(zp.data(), 0, sizeof(SysParams) * max_slots);
    e = hipMemcpy(b->d_slots.p, zs.data(), sizeof(SlotDev) * max_slots, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_md.p, zm.data(), sizeof(MDDev) * max_slots, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_prm.p, zp.data(), sizeof(SysParams) * max_slots, hipMemcpyHostToDevice);
  }
  ctx->batches.push_back(b);
  if (e != hipSuccess) {
    ms2_batch_destroy(b);
    return hip_status(e, "ms2_batch_create");
  }
  *out = b;
  return MS2_OK;
}

void ms2_batch_destroy(ms2_batch* b) {
  if (!b) return;
  auto& reg = b->ctx->batches;
  reg.erase(std::remove(reg.begin(), reg.end(), b), reg.end());
  (void)hipSetDevice(b->ctx->device);
  (void)hipDeviceSynchronize();
  drop_graph(b);
  for (auto e : b->ev_begin) (void)hipEventDestroy(e);
  for (auto e : b->ev_end) (void)hipEventDestroy(e);
  for (auto& s : b->slots) s.mem.release();
  for (auto& m : b->pool) m.release();
  b->d_slots.release();
  b->d_md.release();
  b->d_prm.release();
  b->d_items.release();
  delete b;
}

ms2_status ms2_slot_footprint(ms2_ctx* ctx, const ms2_system* sys, size_t* bytes) {
  if (!ctx || !bytes) return set_error(MS2_EINVAL, "bad arguments");
  SlotShape s;
  ms2_status st = shape_of(ctx, sys, 1, s);
  if (st != MS2_OK) return st;
  *bytes = layout_of(s).total;
  return MS2_OK;
}

ms2_status ms2_slot_admit(ms2_batch* b, const ms2_system* sys, int32_t* slot_out, void* stream) {
  if (!b || !slot_out) return set_error(MS2_EINVAL, "bad arguments");
  ms2_ctx* ctx = b->ctx;
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  SlotShape shape;
  ms2_status s = shape_of(ctx, sys, (b->flags & MS2_BATCH_PLAIN_TILES) ? 0 : 1, shape);
  if (s != MS2_OK) return s;
  int slot = -1;
  for (int k = 0; k < b->max_slots; ++k)
    if (!b->slots[k].used) {
      slot = k;
      break;
    }
  if (slot < 0) return set_error(MS2_EFULL, "no free slot");
  const SlotLayout lay = layout_of(shape);
  if (b->budget && b->used_bytes + lay.total > b->budget)
    return set_error(MS2_ENOMEM, "HBM budget of the batch exceeded");
  MS2_HIP(hipSetDevice(ctx->device));
  SlotHost& h = b->slots[slot];
  {
    // the smallest pooled allocation that holds the slot, else a new one
    int best = -1;
    for (int k = 0; k < (int)b->pool.size(); ++k)
      if (b->pool[k].bytes >= lay.total && (best < 0 || b->pool[k].bytes < b->pool[best].bytes)) best = k;
    if (best >= 0) {
      h.mem = b->pool[best];
      b->pool.erase(b->pool.begin() + best);
    }
  }
  MS2_HIP(h.mem.ensure(lay.total));
  MS2_HIP(hipMemsetAsync(h.mem.p, 0, lay.total, st));
  char* base = (char*)h.mem.p;
  h.shape = shape;
  h.lay = lay;
  h.params = sys->params;
  const int n = shape.n;

  // upload: species, centres, quaternions, velocities, angular velocities
  std::vector<int32_t> sp(sys->h_species, sys->h_species + n);
  MS2_HIP(hipMemcpyAsync(base + lay.species, sp.data(), n * 4, hipMemcpyHostToDevice, st));
  MS2_HIP(hipMemcpyAsync(base + lay.r, sys->h_com, 3 * n * 8, hipMemcpyHostToDevice, st));
  MS2_HIP(hipMemcpyAsync(base + lay.q, sys->h_quat, 4 * n * 8, hipMemcpyHostToDevice, st));
  MS2_HIP(hipMemcpyAsync(base + lay.w, sys->h_omega, 3 * n * 8, hipMemcpyHostToDevice, st));
  MS2_HIP(hipMemcpyAsync(base + lay.vel, sys->h_vel, 3 * n * 8, hipMemcpyHostToDevice, st));
  if (sys->integrator == MS2_GEAR)  // r1 temporarily holds v; md_init_kernel scales it by dt
    MS2_HIP(hipMemcpyAsync(base + lay.r + 3 * n * 8, sys->h_vel, 3 * n * 8, hipMemcpyHostToDevice, st));

  int nk = 0;
  const KVec* kv = nullptr;
  if (sys->params.elec == MS2_ELEC_EWALD) {
    s = kvec_table(ctx, sys->params.kmax2, &kv, &nk);
    if (s != MS2_OK) return s;
  }
  build_sys_params(ctx, &sys->params, nk, h.prm);

  SlotDev& d = h.dev;
  std::memset(&d, 0, sizeof(d));
  d.n = n;
  d.npad = shape.npad;
  d.jsplits = shape.jsplits;
  d.nitems = shape.nitems;
  d.active = 1;
  d.symmetric = shape.waves == 0 ? 1 : 0;
  d.kchunks = shape.kchunks;
  d.mchunks = shape.mchunks;
  d.com_ld = n;
  d.species = (const int*)(base + lay.species);
  d.com = (const double*)(base + lay.r);
  d.quat = (const double*)(base + lay.q);
  d.sites = base + lay.sites;
  d.lj64 = shape.site_cut ? (double*)(base + lay.lj64) : nullptr;
  d.pf = base + lay.pf;
  d.pf_single = shape.precision == MS2_FP32 ? 1 : 0;
  if (shape.heat_flux) {
    // velocities as held during the force evaluation: Gear r1 = dt v
    // (predicted), or the velocity-Verlet half-step velocities
    d.heat_flux = 1;
    d.hf_kin = base + lay.hf_kin;
    d.jq = (double*)(base + lay.hf_jq);
    if (sys->integrator == MS2_GEAR) {
      d.hf_v = (const double*)(base + lay.r) + 3 * (size_t)n;
      d.hf_vscale = 1.0 / sys->dt;
      d.hf_w = (const double*)(base + lay.w);
    } else {
      d.hf_v = (const double*)(base + lay.vel);
      d.hf_vscale = 1.0;
      d.hf_w = nullptr;
    }
  }
  d.bsum = (double*)(base + lay.bsum);
  d.force = (double*)(base + lay.force);
  d.torque = (double*)(base + lay.torque);
  d.sums = (double*)(base + lay.sums);
  d.sk_part = (double*)(base + lay.skp);
  d.sk = (double*)(base + lay.sk);
  d.fk = (double*)(base + lay.fk);
  d.kred = (double*)(base + lay.kred);
  d.ksum = (double*)(base + lay.ksum);
  d.kvec = kv;
  d.nk = nk;
  d.mtiles = shape.mtiles;

  MDDev& m = h.md;
  std::memset(&m, 0, sizeof(m));
  m.active = sys->n_steps > 0 ? 1 : 0;
  m.integrator = sys->integrator;
  m.steps_target = sys->n_steps;
  m.dt = sys->dt;
  m.temperature = sys->temperature;
  m.f_tr = 3.0 * n - 3.0;
  double frot = 0.0;
  bool rotating = false;
  for (int a = 0; a < ctx->tab.nsp; ++a) rotating |= ctx->tab.sp[a].rot_dof > 0;
  for (int i = 0; i < n; ++i) frot += ctx->tab.sp[sys->h_species[i]].rot_dof;
  m.f_rot = frot;
  m.rotating = rotating ? 1 : 0;
  m.sample_every = sys->sample_every;
  m.rdf_every = sys->rdf_every;
  m.rdf_bins = shape.rdf_bins;
  m.rdf_ntp = shape.rdf_ntp;
  m.rdf_rmax = sys->rdf_rmax;
  m.rdf_inv_dr = sys->rdf_every > 0 ? (double)sys->rdf_bins / sys->rdf_rmax : 0.0;
  {
    double dmax = 0.0;
    for (int a = 0; a < ctx->tab.nsp; ++a)
      for (int k = 0; k < ctx->tab.sp[a].nlj; ++k) {
        const double* p = ctx->tab.sp[a].lj_pos[k];
        dmax = std::max(dmax, std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
      }
    const double reach = sys->rdf_rmax + 2.0 * dmax;
    m.rdf_reach2 = reach * reach;
  }
  m.acf_every = sys->acf_every;
  m.acf_origin_every = sys->acf_origin_every;
  m.acf_nlag = shape.acf_nlag;
  m.acf_max_live = shape.acf_max_live;
  m.u0 = sys->u0;
  m.r = (double*)(base + lay.r);
  m.q = (double*)(base + lay.q);
  m.w = (double*)(base + lay.w);
  m.vel = (double*)(base + lay.vel);
  m.moments = (double*)(base + lay.moments);
  m.md_part = (double*)(base + lay.md_part);
  m.rdf = (unsigned long long*)(base + lay.rdf);
  m.acf_v = (double*)(base + lay.acf_v);
  m.acf_j = (double*)(base + lay.acf_j);
  m.acf_cnt = (double*)(base + lay.acf_cnt);
  m.origin_v = (double*)(base + lay.origin_v);
  m.origin_j = (double*)(base + lay.origin_j);
  m.origin_t0 = (long long*)(base + lay.origin_t0);
  if (shape.heat_flux) {
    m.hf_on = 1;
    for (int a = 0; a < kMaxSp; ++a) m.h_partial[a] = sys->h_partial[a];
    m.acf_q = (double*)(base + lay.acf_q);
    m.acf_q_cnt = (double*)(base + lay.acf_q_cnt);
    m.origin_jq = (double*)(base + lay.origin_jq);
    m.origin_jq_valid = (int*)(base + lay.origin_jq_valid);
  }
  std::vector<int> res_idx;
  if (shape.n_solute > 0) {
    for (int i = 0; i < n; ++i)
      if (sys->h_species[i] == sys->res_solute) res_idx.push_back(i);
    for (int i = 0; i < n; ++i)
      if (sys->h_species[i] == sys->res_solvent) res_idx.push_back(i);
    m.res_on = 1;
    m.res_tol = sys->res_tolerance;
    m.n_solute = shape.n_solute;
    m.n_solvent = shape.n_solvent;
    m.res_r2 = sys->res_radius * sys->res_radius;
    m.res_solute_idx = (const int*)(base + lay.res_idx);
    m.res_solvent_idx = (const int*)(base + lay.res_idx) + shape.n_solute;
    m.res_state = (unsigned short*)(base + lay.res_state);
    m.res_n0 = (int*)(base + lay.res_n0);
    m.res_part = (double*)(base + lay.res_part);
    m.res_inside = (int*)(base + lay.res_inside);
    m.res_acf = (double*)(base + lay.res_acf);
    m.res_cnt = (double*)(base + lay.res_cnt);
    MS2_HIP(hipMemcpyAsync(base + lay.res_idx, res_idx.data(), res_idx.size() * sizeof(int),
                           hipMemcpyHostToDevice, st));
  }

  SlotDev* ds = (SlotDev*)b->d_slots.p;
  MDDev* dm = (MDDev*)b->d_md.p;
  SysParams* dp = (SysParams*)b->d_prm.p;
  MS2_HIP(hipMemcpyAsync(ds + slot, &d, sizeof(SlotDev), hipMemcpyHostToDevice, st));
  MS2_HIP(hipMemcpyAsync(dm + slot, &m, sizeof(MDDev), hipMemcpyHostToDevice, st));
  MS2_HIP(hipMemcpyAsync(dp + slot, &h.prm, sizeof(SysParams), hipMemcpyHostToDevice, st));
  MS2_HIP(launch_md_wrap(dm, dp, slot, n, st));
  // first force evaluation through the single-system path, on the slot's arrays
  s = ms2_forces(ctx, &sys->params, n, d.species, d.com, d.quat, d.force, d.torque, d.sums, st);
  if (s == MS2_OK && sys->params.elec == MS2_ELEC_EWALD)
    s = ms2_ewald_kspace(ctx, &sys->params, n, d.species, d.com, d.quat, d.force, d.torque, d.sums, st);
  if (s != MS2_OK) {
    (void)hipStreamSynchronize(st);
    h.mem.release();
    return s;
  }
  MS2_HIP(launch_md_init(ds, dm, ctx->d_tab, slot, st));
  if (shape.n_solute > 0) MS2_HIP(launch_residence(ds, dm, dp, slot, 1, shape.n_solute, st));
  MS2_HIP(hipStreamSynchronize(st));
  h.used = true;
  b->used_bytes += lay.total;
  b->dirty = true;
  drop_graph(b);
  b->last_stream = st;
  *slot_out = slot;
  return MS2_OK;
}

ms2_status ms2_slot_retire(ms2_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used)
    return set_error(MS2_EINVAL, "no such slot");
  MS2_HIP(hipSetDevice(b->ctx->device));
  MS2_HIP(hipStreamSynchronize(b->last_stream));
  SlotHost& h = b->slots[slot];
  SlotDev z{};
  MDDev zm{};
  std::memset(&z, 0, sizeof(z));
  std::memset(&zm, 0, sizeof(zm));
  MS2_HIP(hipMemcpy((SlotDev*)b->d_slots.p + slot, &z, sizeof(SlotDev), hipMemcpyHostToDevice));
  MS2_HIP(hipMemcpy((MDDev*)b->d_md.p + slot, &zm, sizeof(MDDev), hipMemcpyHostToDevice));
  b->used_bytes -= h.lay.total;
  // keep the allocation for a later admission; beyond one per slot of the
  // batch the smallest pooled one is freed
  b->pool.push_back(h.mem);
  h.mem = DevBuf{};
  if ((int)b->pool.size() > b->max_slots) {
    auto it = std::min_element(b->pool.begin(), b->pool.end(),
                               [](const DevBuf& x, const DevBuf& y) { return x.bytes < y.bytes; });
    it->release();
    b->pool.erase(it);
  }
  h.used = false;
  b->dirty = true;
  drop_graph(b);
  return MS2_OK;
}

ms2_status ms2_step(ms2_batch* b, int32_t n_steps, int32_t flags, void* stream) {
  if (!b || n_steps < 0) return set_error(MS2_EINVAL, "bad arguments");
  if (n_steps == 0) return MS2_OK;
  hipStream_t st = (hipStream_t)stream;
  MS2_HIP(hipSetDevice(b->ctx->device));
  (void)hipGetLastError();
  if (b->dirty) rebuild_items(b);
  b->last_stream = st;
  bool any = false;
  for (auto& s : b->slots) any |= s.used;
  if (!any) return MS2_OK;
  const bool timing = (flags & MS2_STEP_TIMING) != 0;
  if (timing) {
    while ((int)b->ev_begin.size() < n_steps) {
      hipEvent_t e0, e1;
      MS2_HIP(hipEventCreate(&e0));
      MS2_HIP(hipEventCreate(&e1));
      b->ev_begin.push_back(e0);
      b->ev_end.push_back(e1);
    }
    b->timed_steps = n_steps;
  }
  const bool graph = (flags & MS2_STEP_GRAPH) && st != nullptr;
  if (!graph) {
    for (int k = 0; k < n_steps; ++k) {
      ms2_status s = enqueue_step(b, st, timing ? k : -1);
      if (s != MS2_OK) return s;
    }
    return MS2_OK;
  }
  const int gflags = flags & ~MS2_STEP_PREPARE;
  if (!b->exec || b->graph_steps != n_steps || b->graph_flags != gflags) {
    drop_graph(b);
    MS2_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    ms2_status s = MS2_OK;
    for (int k = 0; k < n_steps && s == MS2_OK; ++k) s = enqueue_step(b, st, timing ? k : -1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != MS2_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    MS2_HIP(e);
    b->graph = g;
    MS2_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_steps = n_steps;
    b->graph_flags = gflags;
  }
  if (flags & MS2_STEP_PREPARE) return MS2_OK;
  MS2_HIP(hipGraphLaunch(b->exec, st));
  return MS2_OK;
}

ms2_status ms2_batch_timing(ms2_batch* b, double* pair_ms, int32_t* n_steps) {
  if (!b || !pair_ms) return set_error(MS2_EINVAL, "bad arguments");
  MS2_HIP(hipSetDevice(b->ctx->device));
  MS2_HIP(hipStreamSynchronize(b->last_stream));
  double tot = 0.0;
  for (int k = 0; k < b->timed_steps; ++k) {
    float ms = 0.0f;
    MS2_HIP(hipEventElapsedTime(&ms, b->ev_begin[k], b->ev_end[k]));
    tot += ms;
  }
  *pair_ms = tot;
  if (n_steps) *n_steps = b->timed_steps;
  return MS2_OK;
}

ms2_status ms2_slot_status(ms2_batch* b, int32_t slot, int64_t* steps_done, int32_t* status,
                           void* stream) {
  if (!b || slot < 0 || slot >= b->max_slots || !b->slots[slot].used)
    return set_error(MS2_EINVAL, "no such slot");
  hipStream_t st = (hipStream_t)stream;
  MS2_HIP(hipSetDevice(b->ctx->device));
  MDDev m;
  MS2_HIP(hipMemcpyAsync(&m, (MDDev*)b->d_md.p + slot, sizeof(MDDev), hipMemcpyDeviceToHost, st));
  MS2_HIP(hipStreamSynchronize(st));
  if (steps_done) *steps_done = m.steps_done;
  if (status) *status = m.status;
  return MS2_OK;
}

ms2_status ms2_sample(ms2_batch* b, int32_t slot, ms2_samples* out, void* stream) {
  if (!b || !out || slot < 0 || slot >= b->max_slots || !b->slots[slot].used)
    return set_error(MS2_EINVAL, "no such slot");
  hipStream_t st = (hipStream_t)stream;
  MS2_HIP(hipSetDevice(b->ctx->device));
  const SlotHost& h = b->slots[slot];
  const int n = h.shape.n;
  MDDev m;
  MS2_HIP(hipMemcpyAsync(&m, (MDDev*)b->d_md.p + slot, sizeof(MDDev), hipMemcpyDeviceToHost, st));
  MS2_HIP(hipMemcpyAsync(out->sums, h.dev.sums, MS2_NSUM * 8, hipMemcpyDeviceToHost, st));
  MS2_HIP(hipMemcpyAsync(out->moments, h.md.moments, kNumMoments * 8, hipMemcpyDeviceToHost, st));
  std::vector<unsigned long long> rdf;
  if (out->h_rdf && h.shape.rdf_ntp) {
    rdf.resize((size_t)h.shape.rdf_ntp * h.shape.rdf_bins);
    MS2_HIP(hipMemcpyAsync(rdf.data(), h.md.rdf, rdf.size() * 8, hipMemcpyDeviceToHost, st));
  }
  const size_t nl = (size_t)h.shape.acf_nlag * 8;
  if (nl && out->h_acf_v) MS2_HIP(hipMemcpyAsync(out->h_acf_v, h.md.acf_v, nl, hipMemcpyDeviceToHost, st));
  if (nl && out->h_acf_j) MS2_HIP(hipMemcpyAsync(out->h_acf_j, h.md.acf_j, nl, hipMemcpyDeviceToHost, st));
  if (nl && out->h_acf_cnt)
    MS2_HIP(hipMemcpyAsync(out->h_acf_cnt, h.md.acf_cnt, nl, hipMemcpyDeviceToHost, st));
  if (h.shape.heat_flux) {
    if (out->h_acf_q) MS2_HIP(hipMemcpyAsync(out->h_acf_q, h.md.acf_q, nl, hipMemcpyDeviceToHost, st));
    if (out->h_acf_q_cnt)
      MS2_HIP(hipMemcpyAsync(out->h_acf_q_cnt, h.md.acf_q_cnt, nl, hipMemcpyDeviceToHost, st));
  } else {
    if (out->h_acf_q) std::memset(out->h_acf_q, 0, nl);
    if (out->h_acf_q_cnt) std::memset(out->h_acf_q_cnt, 0, nl);
  }
  if (h.shape.n_solute > 0) {
    if (out->h_res_acf) MS2_HIP(hipMemcpyAsync(out->h_res_acf, h.md.res_acf, nl, hipMemcpyDeviceToHost, st));
    if (out->h_res_cnt) MS2_HIP(hipMemcpyAsync(out->h_res_cnt, h.md.res_cnt, nl, hipMemcpyDeviceToHost, st));
  } else {
    if (out->h_res_acf) std::memset(out->h_res_acf, 0, nl);
    if (out->h_res_cnt) std::memset(out->h_res_cnt, 0, nl);
  }
  if (out->h_com) MS2_HIP(hipMemcpyAsync(out->h_com, h.md.r, 3 * n * 8, hipMemcpyDeviceToHost, st));
  if (out->h_quat) MS2_HIP(hipMemcpyAsync(out->h_quat, h.md.q, 4 * n * 8, hipMemcpyDeviceToHost, st));
  if (out->h_vel) MS2_HIP(hipMemcpyAsync(out->h_vel, h.md.vel, 3 * n * 8, hipMemcpyDeviceToHost, st));
  if (out->h_omega) MS2_HIP(hipMemcpyAsync(out->h_omega, h.md.w, 3 * n * 8, hipMemcpyDeviceToHost, st));
  if (out->h_force) MS2_HIP(hipMemcpyAsync(out->h_force, h.dev.force, 3 * n * 8, hipMemcpyDeviceToHost, st));
  if (out->h_torque)
    MS2_HIP(hipMemcpyAsync(out->h_torque, h.dev.torque, 3 * n * 8, hipMemcpyDeviceToHost, st));
  MS2_HIP(hipStreamSynchronize(st));
  for (size_t k = 0; k < rdf.size(); ++k) out->h_rdf[k] = (double)rdf[k];
  out->steps_done = m.steps_done;
  out->status = m.status;
  out->rdf_ntypes = b->ctx->tab.n_lj_types;
  out->ekin_trans = m.ekin_tr;
  out->ekin_rot = m.ekin_rot;
  out->pairs_total = m.pairs_total;
  out->site_pairs_total = m.site_pairs_total;
  out->solvation_sum = m.res_solv_sum;
  out->solvation_cnt = m.res_solv_cnt;
  return MS2_OK;
}

}  // extern "C"
