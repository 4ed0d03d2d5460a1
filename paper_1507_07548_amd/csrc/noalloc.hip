// ms2_forces without device allocation.
//
// The explicit pair part of one force/energy evaluation needs scratch beyond
// the caller's inputs and outputs: the lab-frame site records (and, in the
// site-site cut-off mode, the FP64 LJ-site offsets), the per-tile
// force/torque partials, the per-item block sums and the work-item list.
// ms2_forces keeps them in context buffers that grow on the first call at a
// larger size (that call allocates).  Here they live in one file-scope
// device array, `scratch`, sized for MS2_NOALLOC_MAX_MOL molecules of the
// largest model class in FP64; every GPU the library runs on holds its own
// copy from the time the code object is loaded until the process ends.
//
// Host code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): ms2_create looks up the array's device
// address once per device, with that device current, and every launch takes
// that address.
//
// The work items are the symmetric 64 x 64 tile pairs of ms2_forces' untuned
// default shape (1, 2 or 4 items per tile pair by the system's size), written
// by a small kernel in the order the host list uses, so the result equals
// ms2_forces with that shape bit for bit.  Every scratch entry
// a kernel reads was written earlier in the same call (site records and
// partials of every molecule and tile index, block sums of every item), so
// nothing is cleared between calls.  All calls on one GPU share the array:
// calls that overlap on that GPU (two streams, two threads, two contexts)
// race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>

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

namespace {

constexpr int kNaTiles = MS2_NOALLOC_MAX_MOL / 64;
static_assert(MS2_NOALLOC_MAX_MOL % 64 == 0, "the molecule limit is a whole number of 64-molecule tiles");
constexpr int kNaItems = kNaTiles * (kNaTiles + 1) / 2;

constexpr int max_class_reals() {
  int m = 0;
  for (int c = 0; c < kNumClasses; ++c) m = class_reals(c) > m ? class_reals(c) : m;
  return m;
}
constexpr int max_class_lj() {
  int m = 0;
  for (int c = 0; c < kNumClasses; ++c) m = class_lj(c) > m ? class_lj(c) : m;
  return m;
}
constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// byte offsets of the four regions (sized for the limit, FP64 reals)
constexpr size_t kOffItems = 0;
constexpr size_t kOffBsum = align256(kOffItems + (size_t)kNaItems * sizeof(WorkItem));
constexpr size_t kOffSites = align256(kOffBsum + (size_t)kNaItems * kNumBlockSums * sizeof(double));
constexpr size_t kOffLj64 = align256(kOffSites + (size_t)max_class_reals() * MS2_NOALLOC_MAX_MOL * sizeof(double));
constexpr size_t kOffPf = align256(kOffLj64 + (size_t)3 * max_class_lj() * MS2_NOALLOC_MAX_MOL * sizeof(double));
constexpr size_t kScratchBytes = align256(kOffPf + (size_t)kNaTiles * 6 * MS2_NOALLOC_MAX_MOL * sizeof(double));
static_assert(kScratchBytes <= (size_t)16 << 20, "the no-allocation scratch stays under 16 MiB");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_ptr;   // device -> address of `scratch` on it

unsigned char* scratch_on(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// Symmetric tile pairs (I, J >= I) of ceil(n / 64) tiles, row-major in I,
// S items per tile pair: thread I writes row I, whose first tile pair is
// the number of pairs in rows 0 .. I-1, sum_{r < I} (nt - r).  Same items,
// same order as the host list of the default shape.
__global__ __launch_bounds__(64) void noalloc_items_kernel(WorkItem* __restrict__ items, int n, int S) {
  const int nt = (n + 63) / 64;
  const int I = threadIdx.x;
  if (I >= nt) return;
  int k = I * nt - I * (I - 1) / 2;
  for (int J = I; J < nt; ++J, ++k) {
    for (int sp = 0; sp < S; ++sp) {
      WorkItem w;
      w.slot = 0;
      w.i0 = 64 * I;
      w.j0 = 64 * J;
      w.j1 = min(n, 64 * J + 64);
      w.part = J * S + sp;
      w.local = k * S + sp;
      w.part_j = I * S + sp;
      w.split = S > 1 ? sp + 256 * S : 0;
      items[k * S + sp] = w;
    }
  }
}

}  // namespace

hipError_t noalloc_scratch_attach(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr.count(device)) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  return hipSuccess;
}

}  // namespace ms2

using namespace ms2;

extern "C" ms2_status ms2_forces_noalloc(ms2_ctx* ctx, const ms2_params* h_params, int32_t n_mol,
                                         const int32_t* d_species, const double* d_com, const double* d_quat,
                                         double* d_force, double* d_torque, double* d_sums, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();   // launch checks below must not see an unrelated earlier error
  if (!ctx) return set_error(MS2_EINVAL, "context is NULL");
  if (n_mol < 2) return set_error(MS2_EINVAL, "n_mol must be >= 2");
  if (n_mol > MS2_NOALLOC_MAX_MOL)
    return set_error(MS2_EINVAL, "ms2_forces_noalloc: n_mol exceeds MS2_NOALLOC_MAX_MOL (" +
                                     std::to_string(MS2_NOALLOC_MAX_MOL) + "); use ms2_forces");
  if (!d_species || !d_com || !d_quat || !d_force || !d_torque || !d_sums)
    return set_error(MS2_EINVAL, "NULL device pointer");
  ms2_status s = check_params(ctx, h_params);
  if (s != MS2_OK) return s;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_status(e, "hipSetDevice");
  unsigned char* base = scratch_on(ctx->device);
  if (!base) return set_error(MS2_EDEVICE, "no-allocation scratch was not attached on this device");

  const int n = n_mol, npad = (n + 63) & ~63, nt = npad / 64;
  // the default symmetric shape of ms2_forces (S items per tile pair), within
  // the scratch's item and partial capacity
  int S = sym_splits(default_shape(ctx, n));
  while (S > 1 && ((size_t)nt * (nt + 1) / 2 * S > (size_t)kNaItems || nt * S > kNaTiles)) S /= 2;
  const int nitems = nt * (nt + 1) / 2 * S;
  const int nk = h_params->elec == MS2_ELEC_EWALD ? kvec_count(h_params->kmax2) : 0;
  RingSlot* r = nullptr;
  s = ring_acquire(ctx, &r);
  if (s != MS2_OK) return s;
  build_sys_params(ctx, h_params, nk, *r->h_prm);
  SlotDev& d = *r->h_slot;
  std::memset(&d, 0, sizeof(d));
  d.n = n;
  d.npad = npad;
  d.jsplits = nt * S;
  d.nitems = nitems;
  d.active = 1;
  d.symmetric = 1;
  d.com_ld = n;
  d.species = d_species;
  d.com = d_com;
  d.quat = d_quat;
  d.sites = base + kOffSites;
  d.lj64 = h_params->cutoff_mode == MS2_CUT_SITE ? reinterpret_cast<double*>(base + kOffLj64) : nullptr;
  d.pf = base + kOffPf;
  d.pf_single = h_params->precision == MS2_FP32 ? 1 : 0;
  d.bsum = reinterpret_cast<double*>(base + kOffBsum);
  d.force = d_force;
  d.torque = d_torque;
  d.sums = d_sums;
  d.nk = nk;
  d.err = ctx->d_err;
  WorkItem* items = reinterpret_cast<WorkItem*>(base + kOffItems);
#define MS2_NA_HIP(call)                                   \
  do {                                                     \
    const hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_status(e_, #call);    \
  } while (0)
  MS2_NA_HIP(hipMemcpyAsync(r->d_slot, r->h_slot, sizeof(SlotDev), hipMemcpyHostToDevice, st));
  MS2_NA_HIP(hipMemcpyAsync(r->d_prm, r->h_prm, sizeof(SysParams), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(noalloc_items_kernel, dim3(1), dim3(64), 0, st, items, n, S);
  MS2_NA_HIP(hipGetLastError());
  MS2_NA_HIP(launch_site_frame(ctx->cls, h_params->precision, r->d_slot, r->d_prm, ctx->d_tab, 1, n, st));
  MS2_NA_HIP(launch_pair(ctx->cls, h_params->precision, 0, false, h_params->cutoff_mode == MS2_CUT_SITE,
                         pair_form(ctx), items, 0, nitems, r->d_slot, r->d_prm, ctx->d_tab, st));
  MS2_NA_HIP(launch_reduce_pair(r->d_slot, r->d_prm, 1, n, st));
  MS2_NA_HIP(hipEventRecord(r->ev, st));
#undef MS2_NA_HIP
  return MS2_OK;
}
