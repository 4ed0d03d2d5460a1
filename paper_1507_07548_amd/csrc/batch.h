// Host-side objects behind the opaque ms2_ctx / ms2_batch handles.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "internal.h"

namespace ms2 {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need);
  void release();
};

struct TileCfg {
  int waves = 1;    // waves per block (64 i molecules each); 0 = symmetric tile pairs
  int jchunk = 64;  // j molecules per work item; symmetric: 64 / S, S items per tile pair
};
// items per symmetric tile pair (1, 2 or 4); 1 for row-owned shapes
inline int sym_splits(const TileCfg& c) { return c.waves == 0 && c.jchunk > 0 ? 64 / c.jchunk : 1; }
// the untuned symmetric shape for n molecules: the fewest items per tile
// pair (1, 2, 4) that give the system at least `target` items
TileCfg default_sym_shape(int n, int target);
// the untuned shape of a context for n molecules (symmetric items)
TileCfg default_shape(const ms2_ctx* ctx, int n);

struct CachedItems {
  DevBuf buf;
  int count = 0;
  int jsplits = 0;
};

constexpr int kRing = 32;
struct RingSlot {
  SlotDev* h_slot = nullptr;
  SysParams* h_prm = nullptr;
  SlotDev* d_slot = nullptr;
  SysParams* d_prm = nullptr;
  hipEvent_t ev = nullptr;
  bool used = false;
};

ms2_status set_error(ms2_status s, const std::string& msg);
ms2_status hip_status(hipError_t e, const char* where);

}  // namespace ms2

struct ms2_ctx {
  int device = 0;
  int cls = 0;
  int cus = 256;           // compute units of the device (untuned tile shapes)
  ms2::SpeciesTable tab;
  ms2::SpeciesTable* d_tab = nullptr;
  int* d_err = nullptr;    // device error word of the single-system entry points
  // scratch of the single-system entry points
  ms2::DevBuf s_sites, s_lj64, s_pf, s_bsum, s_skp, s_sk, s_fk, s_kred, s_ksum;
  std::map<int, std::pair<ms2::DevBuf, int>> kvecs;            // kmax2 -> (table, count)
  std::map<std::tuple<int, int, int>, ms2::CachedItems> item_cache;
  std::map<std::tuple<int, int, int>, ms2::TileCfg> tuned;     // (mode, precision, log2 n) -> shape
  ms2::RingSlot ring[ms2::kRing];
  int ring_pos = 0;
  std::vector<ms2_batch*> batches;   // live batches; destroyed before the context
};

namespace ms2 {
ms2_status check_params(const ms2_ctx* ctx, const ms2_params* p);
void build_sys_params(const ms2_ctx* ctx, const ms2_params* p, int nk, SysParams& s);
ms2_status kvec_table(ms2_ctx* ctx, int kmax2, const KVec** d_out, int* nk);
TileCfg tile_config(const ms2_ctx* ctx, int mode, int precision, int n);
int size_bucket(int n);
int build_items(int n, const TileCfg& c, int slot, std::vector<WorkItem>& out, int* jsplits);
// the form of the symmetric pair kernel a context takes (PairForm): the
// single-species form needs one species with at least one site of every
// kind its model class holds; the linear form in addition a two-centre LJ +
// quadrupole molecule with both LJ sites (equal parameters) at +-h on the
// quadrupole's axis and the quadrupole at the centre
int pair_form(const ms2_ctx* ctx);
// h of the linear form, or 0 when the context's species is not of that shape
double linear_h(const ms2_ctx* ctx);
int kvec_count(int kmax2);
// next block of the context's ring of pinned parameter blocks (waits for
// the call that used it last)
ms2_status ring_acquire(ms2_ctx* ctx, RingSlot** out);
// device address of the no-allocation scratch array on the current device
// (looked up once per device; ms2_create calls it with its device current)
hipError_t noalloc_scratch_attach(int device);
}  // namespace ms2
