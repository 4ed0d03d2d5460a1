// Force/energy/virial hot path on gfx950: lab-frame site records, the
// molecule-pair kernel and its fixed-order reductions.
//
// Mapping (one block = 64*W lanes, W waves):
//   * every lane owns one molecule i of an i-tile of 64*W molecules and
//     accumulates everything acting on i in registers (row-owned: each pair
//     is evaluated from both sides, so no lane ever writes another lane's
//     molecule and no atomics are needed; the paper's Sec. 2 avoids the same
//     write race with per-interaction lists summed afterwards);
//   * j molecules stream through LDS in tiles of 64*W records (coalesced
//     structure-of-arrays loads);
//   * per tile, phase 1 tests every (i, j) pair against the molecule-centre
//     cut-off in FP64 and keeps one bit per accepted pair; phase 2 walks each
//     lane's own set bits, so the ~54 % of rejected pairs cost one FP64 test
//     and no site arithmetic (per-lane compaction instead of masked lanes);
//   * site-pair arithmetic runs in Real (float or double); force partials of
//     one j tile are folded into FP64 per-molecule accumulators; energies and
//     volume-derivative sums are accumulated per molecule pair in FP64.
// A work item is (system, i-tile, j-range); its per-molecule partials go to
// a slot-private buffer and are summed over j-ranges in a fixed order by
// reduce_pair_kernel, so results do not depend on launch order or on other
// systems sharing the launch.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "kspace_sums.h"
#include "pair_math.h"
#include "quat.h"
#include "site_frame.h"

namespace ms2 {

// ---------------------------------------------------------------------------
// Site frame of every molecule of every slot of this precision.
// ---------------------------------------------------------------------------
template <typename Real, int C>
__global__ __launch_bounds__(256) void site_frame_kernel(const SlotDev* __restrict__ slots,
                                                         const SysParams* __restrict__ prm,
                                                         const SpeciesTable* __restrict__ tab) {
  const SlotDev& sd = slots[blockIdx.y];
  if (!sd.active) return;
  if (prm[blockIdx.y].precision != (sizeof(Real) == 4 ? MS2_FP32 : MS2_FP64)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= sd.n) return;
  site_frame_molecule<Real, C>(sd, tab, i);
}

// ---------------------------------------------------------------------------
// Row-owned pair kernel: a lane owns molecule i and evaluates every accepted
// pair from its own side.
// ---------------------------------------------------------------------------
template <typename Real>
__device__ __forceinline__ ElecParams<Real> elec_params(const SysParams& P) {
  ElecParams<Real> E;
  E.elec = P.elec;
  E.krf = (Real)P.krf;
  E.crf = (Real)P.crf;
  E.alpha = (Real)P.alpha;
  E.alpha2 = (Real)P.alpha2;
  E.gpref = (Real)P.gpref;
  E.inv_ke = P.inv_ke;
  return E;
}

// Workgroups are dealt to the eight XCDs in turn (block b to XCD b mod 8),
// each with its own L2.  This maps the blocks of one XCD to a contiguous run
// of the n items, so that items sharing a tile (consecutive in the item list)
// meet in the same L2.  A bijection of [0, n) for any n.
__device__ __forceinline__ int xcd_local_item(int b, int n) {
  const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + k;
}

// fixed-order block sum of the six per-lane scalars; thread 0..5 write them
template <int NT>
__device__ __forceinline__ void block_sums(double (*s_red)[NT], const double* v, double* out) {
  const int tid = threadIdx.x;
  __syncthreads();
  for (int k = 0; k < kNumBlockSums; ++k) s_red[k][tid] = v[k];
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int k = 0; k < kNumBlockSums; ++k) s_red[k][tid] += s_red[k][tid + h];
    __syncthreads();
  }
  if (tid < kNumBlockSums) out[tid] = s_red[tid][0];
}

// Sums of v[k] over the 64 lanes of a wave in butterfly order (a fixed
// order; every lane ends with the same bits); lane k writes out[k].
__device__ __forceinline__ void wave_sums(double* v, double* out) {
#pragma unroll
  for (int h = 32; h > 0; h >>= 1) {
#pragma unroll
    for (int k = 0; k < kNumBlockSums; ++k) v[k] += __shfl_xor(v[k], h, 64);
  }
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kNumBlockSums; ++k)
    if (lane == k) out[k] = v[k];
}

template <typename Real, int C, int W>
__global__ __launch_bounds__(64 * W) void pair_kernel(const WorkItem* __restrict__ items,
                                                      int item_base,
                                                      const SlotDev* __restrict__ slots,
                                                      const SysParams* __restrict__ prm,
                                                      const SpeciesTable* __restrict__ tab) {
  constexpr int NR = class_reals(C);
  constexpr int TJ = 64 * W;

  __shared__ double s_com[3][TJ];
  __shared__ int s_sp[TJ];
  __shared__ Real s_site[NR][TJ];
  __shared__ PairTables<Real, C> s_tab;
  __shared__ double s_red[W > 1 ? kNumBlockSums : 1][W > 1 ? TJ : 1];

  const WorkItem it = items[item_base + xcd_local_item(blockIdx.x, gridDim.x)];
  const SlotDev& sd = slots[it.slot];
  if (!sd.active) return;
  const SysParams& P = prm[it.slot];
  const int tid = threadIdx.x;
  const int nsp = P.nsp;
  s_tab.load(tab, P, P.nsp, tid, TJ);

  const int n = sd.n, ld = sd.com_ld, np = sd.npad;
  const double L = P.L, invL = P.invL, rc2 = P.rc2;
  const ElecParams<Real> E = elec_params<Real>(P);
  const Real* __restrict__ gsite = reinterpret_cast<const Real*>(sd.sites);

  const int i = it.i0 + tid;
  const bool iv = i < n;
  const int ic = iv ? i : 0;
  const double xi = sd.com[ic], yi = sd.com[ld + ic], zi = sd.com[2 * ld + ic];
  const int spi = iv ? clamp_species(sd.species[ic], nsp) : 0;
  Real rec[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) rec[k] = gsite[k * np + ic];

  double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  double a_ulj = 0, a_uel = 0, a_us = 0, a_uss = 0;
  int a_np = 0, a_ns = 0;
  SiteAcc<Real, C> ai, unused;
  ai.zero();

  for (int jt = it.j0; jt < it.j1; jt += TJ) {
    __syncthreads();
    {
      const int j = jt + tid;
      const bool jv = j < it.j1 && j < n;
      const int jc = jv ? j : 0;
      s_com[0][tid] = sd.com[jc];
      s_com[1][tid] = sd.com[ld + jc];
      s_com[2][tid] = sd.com[2 * ld + jc];
      s_sp[tid] = jv ? clamp_species(sd.species[jc], nsp) : 0;
#pragma unroll
      for (int k = 0; k < NR; ++k) s_site[k][tid] = gsite[k * np + jc];
    }
    __syncthreads();

    // phase 1: cut-off bits, one 64-bit word per 64 j molecules
    const int nvalid = min(TJ, min(it.j1, n) - jt);   // uniform over the block
    const int iself = i - jt;                          // lane's own molecule in this tile, if any
    unsigned long long mask[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      unsigned long long m = 0;
      for (int b = 0; b < 64; ++b) {
        const int jj = w * 64 + b;
        double dx, dy, dz, r2;
        min_image(xi, yi, zi, s_com[0][jj], s_com[1][jj], s_com[2][jj], L, invL, dx, dy, dz, r2);
        const unsigned ok = (unsigned)(r2 < rc2) & (unsigned)(jj < nvalid) & (unsigned)(jj != iself);
        m |= (unsigned long long)ok << b;
      }
      mask[w] = iv ? m : 0ull;
    }

    // phase 2: accepted pairs of this lane
    int w = 0;
    unsigned long long m = mask[0];
    while (true) {
      while (m == 0ull && w < W - 1) {
        ++w;
#pragma unroll
        for (int x = 1; x < W; ++x)
          if (x == w) m = mask[x];
      }
      if (m == 0ull) break;
      const int jj = w * 64 + __builtin_ctzll(m);
      m &= m - 1ull;
      const int spj = s_sp[jj];
      double dx, dy, dz, r2d;
      min_image(xi, yi, zi, s_com[0][jj], s_com[1][jj], s_com[2][jj], L, invL, dx, dy, dz, r2d);
      const Real Rx = (Real)dx, Ry = (Real)dy, Rz = (Real)dz;
      const Real R2 = (Real)r2d;
      PairAcc<Real> acc{0, 0, 0, 0, 0, 0};
      eval_molecule_pair<Real, C, false, TJ>(rec, &s_site[0][jj], spi, spj, s_tab, E, Rx, Ry, Rz, R2, ai,
                                             unused, acc);
      a_ulj += (double)acc.ulj;
      a_uel += (double)acc.uel;
      a_uss += (double)acc.uss;
      a_us -= (double)(Rx * acc.fx + Ry * acc.fy + Rz * acc.fz);
      a_np += 1;
      a_ns += s_tab.nsite[spi][spj];
    }
    // fold this tile's site forces into the FP64 force and torque
    fold_sites<Real, C, 1>(rec, ai, F, T);
    ai.zero();
  }

  if (iv) {
    Real* pf = reinterpret_cast<Real*>(sd.pf) + (size_t)it.part * 6 * np;
    pf[0 * np + i] = (Real)F[0]; pf[1 * np + i] = (Real)F[1]; pf[2 * np + i] = (Real)F[2];
    pf[3 * np + i] = (Real)T[0]; pf[4 * np + i] = (Real)T[1]; pf[5 * np + i] = (Real)T[2];
  }
  double v[kNumBlockSums] = {a_ulj, a_uel, a_us, a_uss, (double)a_np, (double)a_ns, 0.0, 0.0, 0.0};
  if constexpr (W > 1)
    block_sums<TJ>(s_red, v, sd.bsum + (size_t)it.local * kNumBlockSums);
  else
    wave_sums(v, sd.bsum + (size_t)it.local * kNumBlockSums);
}

// ---------------------------------------------------------------------------
// Symmetric pair kernel: work items are 64 x 64 tile pairs (I, J >= I) and
// every accepted molecule pair is evaluated once, by one lane, with no
// atomics.  Four waves share one item (its tiles are staged once).
//  1. the cut-off bits of the 64 x 64 pairs (FP64, j > i on the diagonal
//     tile; each wave tests 16 columns of every row) are rotated right by
//     the row index l, so that bit d marks pair (l, l + d): "diagonal" d of
//     the tile.  Every wave transposes the 64 x 64 bits in registers (lane
//     swizzles, no shared memory, no barrier), so that lane d holds diagonal
//     d's 64-bit word; a wave scan of their counts gives each diagonal's
//     offset in the diagonal-major list of accepted pairs.
//  2. the list is processed 64 entries at a time, one pair per lane, the
//     chunks dealt to the waves in turn.  A chunk's diagonals follow from
//     two ballots over the offsets.  For each of them lane m holds row m's
//     entry index: the diagonal's offset plus the count of set bits below
//     bit m (mbcnt).  Lanes write their (row, diagonal) to those slots of a
//     per-wave list, from which each lane reads its pair, and keep the
//     entry indices of the chunk's first diagonals for step 3.
//  3. each lane stages its pair's force and torques in its wave's LDS area.
//     Lane m then gathers the entries of molecule m of tile I (as a row, at
//     its own entry index) and of tile J (as a column, at the index held by
//     row m - d): on each diagonal d of the chunk there is at most one of
//     each.  Sums stay in registers; there are no read-modify-writes of
//     shared memory.
//  4. the reaction on j follows from the pair's force and torque on i:
//     F_j = -F_i and, the pair energy being invariant under a rigid rotation
//     of both molecules, tau_j = -tau_i - R x F_i with R = R_i - R_j.
//  5. the four waves' partials are added in wave order.
// The schedule and the order of additions depend on the tile's data only.
// Partials: molecule m of tile T receives exactly one partial per tile index
// p -- the column side of item (p, T) for p < T, the row side of item (T, p)
// for p > T, and both sides of the diagonal item (T, T) -- so the
// fixed-order reduction over p is unchanged.
// ---------------------------------------------------------------------------
constexpr int kSymWaves = 4;
constexpr int kKeepDiags = 6;   // diagonals per chunk whose entry indices are kept for the gather

// Index in the chunk [q, q + 64) of this lane's row on a diagonal with word
// wd starting at offset o - q (all wave-uniform), or -1 if the row is not on
// it or its entry lies outside the chunk.
__device__ __forceinline__ int row_entry(unsigned long long wd, int o_rel) {
  const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(wd >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)wd, 0u));
  const int e = o_rel + rank;
  // wd is wave-uniform: its bits are the lane mask of the rows it holds
  const bool on = __builtin_amdgcn_inverse_ballot_w64(wd);
  return (on && (unsigned)e < 64u) ? e : -1;
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP row shifts:
// Hillis-Steele steps of 1, 2, 4 and 8 lanes inside each row of 16, then the
// last lane of row 0 (2) is added to row 1 (3) and lane 31 to rows 2 and 3.
// Lanes whose DPP source lies outside the row, or whose row the row mask
// leaves out, add 0.
__device__ __forceinline__ int wave_inclusive_sum(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
  return v;
}

__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int lane) {
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, lane);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

// One stage of the wave's 64 x 64 bit transpose (wave_bit_transpose): lane-
// index bit S trades places with bit-position bit S inside each 32-bit half.
// Lane l keeps its bits whose position agrees with l in bit S and takes the
// others from lane l ^ S (an LDS swizzle, no VALU), rotated by S the way
// that lands them in place: left where l has bit S clear, right where set.
template <int S>
__device__ __forceinline__ void bit_transpose_stage(unsigned& lo, unsigned& hi) {
  constexpr unsigned kLow = S == 16 ? 0x0000FFFFu : S == 8 ? 0x00FF00FFu : S == 4 ? 0x0F0F0F0Fu
                            : S == 2 ? 0x33333333u : 0x55555555u;   // positions with bit S clear
  constexpr unsigned long long kUp = S == 16 ? 0xFFFF0000FFFF0000ull : S == 8 ? 0xFF00FF00FF00FF00ull
                                     : S == 4 ? 0xF0F0F0F0F0F0F0F0ull : S == 2 ? 0xCCCCCCCCCCCCCCCCull
                                                                      : 0xAAAAAAAAAAAAAAAAull;   // lanes with bit S set
  constexpr int kXor = 0x1F | (S << 10);   // swizzle, bit-mask mode: lane (l & 31) ^ S of its half
  const bool up = __builtin_amdgcn_inverse_ballot_w64(kUp);
  const unsigned keep = kLow ^ (up ? ~0u : 0u);
  const unsigned amt = up ? S : 32 - S;
  const unsigned plo = (unsigned)__builtin_amdgcn_ds_swizzle((int)lo, kXor);
  const unsigned phi = (unsigned)__builtin_amdgcn_ds_swizzle((int)hi, kXor);
  lo = (lo & keep) | (__builtin_amdgcn_alignbit(plo, plo, amt) & ~keep);
  hi = (hi & keep) | (__builtin_amdgcn_alignbit(phi, phi, amt) & ~keep);
}

// 64 x 64 bit-matrix transpose held one row per lane: lane l passes word r
// (bit c: element (l, c)) and gets back the word whose bit c is element
// (c, l).  The six stages (lane-index bit s against bit-position bit s, s =
// 32, 16, ..., 1) commute; for s = 32 the 32-bit halves cross between lanes
// l and l ^ 32.  Registers and LDS swizzles only: no shared memory, no
// barrier.
__device__ __forceinline__ unsigned long long wave_bit_transpose(unsigned long long r) {
  unsigned lo = (unsigned)r, hi = (unsigned)(r >> 32);
  {
    const int lane = threadIdx.x & 63;
    const bool up = __builtin_amdgcn_inverse_ballot_w64(0xFFFFFFFF00000000ull);
    const unsigned recv = (unsigned)__builtin_amdgcn_ds_bpermute((lane ^ 32) << 2, (int)(up ? lo : hi));
    lo = up ? recv : lo;
    hi = up ? hi : recv;
  }
  bit_transpose_stage<16>(lo, hi);
  bit_transpose_stage<8>(lo, hi);
  bit_transpose_stage<4>(lo, hi);
  bit_transpose_stage<2>(lo, hi);
  bit_transpose_stage<1>(lo, hi);
  return ((unsigned long long)hi << 32) | lo;
}

// Orders this wave's LDS accesses before and after, for the wave's own
// lanes only: a wave's LDS operations are performed in issue order, so
// fences of wavefront scope suffice and cost no wait (workgroup scope would
// drain the wave's outstanding LDS operations at each call).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename Real, int NR, bool HF, int NL64>
struct SymTiles {
  // centres [xyz][molecule] of the columns, then the rows: phase 1 reads
  // three columns' components at offsets of one base address
  double comj[3][64];
  double comi[3][64];
  Real site[2][NR][64];
  Real stage[kSymWaves][9][64];         // F_i, tau_i, tau_j of each lane's pair
  unsigned char er[kSymWaves][kKeepDiags][64];  // row m's entry index on the chunk's k-th diagonal, or 255
  Real kin[HF ? 2 : 1][6][HF ? 64 : 1]; // heat flux: lab v and w of rows, columns
  double lj64[NL64 ? 2 : 1][NL64 ? NL64 : 1][NL64 ? 64 : 1];  // site-site cut-off: FP64 LJ offsets
};

template <typename Real>
struct SymFinal {
  Real part[kSymWaves][12][64];         // per wave: row F, tau; column F, tau
  double sums[kSymWaves][kNumBlockSums];
};

// Waves per SIMD the register allocation must allow: six for the FP32
// two-centre quadrupole kernel of the centre cut-off (it fits 80 registers
// without spilling, and the kernel hides its LDS latency better with six
// waves than with five); in FP64 four for the general single-species form
// and three for the linear form (150 VGPRs, no spills); the compiler's
// choice otherwise.
template <typename Real, int C, bool HF, bool SITE, bool LIN>
constexpr int kSymOccupancy = (sizeof(Real) == 4 && C == 1 && !HF && !SITE) ? 6
                              : (sizeof(Real) == 8 && C == 1 && !HF && !SITE) ? (LIN ? 3 : 4)
                                                                             : 1;

// ONE: every molecule of the system is species 0, a species with at least
// one site of every kind its class holds (instantiated for classes 0-3); the
// species reads and table indexing drop out, and the first site pair of each
// kind starts its sums.
// LIN (class 1, ONE, centre cut-off, no heat flux): the species is a
// linear two-centre LJ + quadrupole molecule (eval_linear_pair); only the
// first LJ site's offset and the quadrupole axis of each molecule are staged
// (278 instead of 319 VALU instructions in the pair loop; 4.37 -> 4.29 ms on
// the batched 2CLJQ workload).
template <typename Real, int C, bool HF, bool SITE, bool ONE, bool LIN = false>
__global__ __launch_bounds__(64 * kSymWaves) __attribute__((amdgpu_waves_per_eu(kSymOccupancy<Real, C, HF, SITE, LIN>)))
void pair_sym_kernel(const WorkItem* __restrict__ items,
                                                                  int item_base,
                                                                  const SlotDev* __restrict__ slots,
                                                                  const SysParams* __restrict__ prm,
                                                                  const SpeciesTable* __restrict__ tab) {
  static_assert(!LIN || (C == 1 && ONE && !HF && !SITE),
                "the linear form is a class-1 single-species form of the centre cut-off");
  // reals of the site record staged per molecule: all of them, or (LIN) the
  // first LJ site's offset (the record's first three) and the quadrupole
  // axis (its last three)
  constexpr int NR = LIN ? 6 : class_reals(C);
  constexpr int TJ = 64, NW = kSymWaves;
  static_assert(NW == 4 || NW == 8, "waves 0-3 stage the tiles and write the partials");

  constexpr int NL64 = SITE ? 3 * kClassShapes[C].lj : 0;
  __shared__ union {
    SymTiles<Real, NR, HF, NL64> t;
    SymFinal<Real> f;
  } u;
  __shared__ int s_sp[ONE ? 1 : 2][ONE ? 1 : TJ];   // species of rows, columns (not read when ONE)
  __shared__ PairTables<Real, C, ONE ? 1 : kMaxSp> s_tab;
  __shared__ unsigned s_mpart[NW][TJ];
  __shared__ int s_list[NW][TJ];          // per wave: row | diagonal << 6 of each entry of the chunk
  __shared__ int s_inbox[2];              // 1: every staged centre of the side lies in [0, L]

  const WorkItem it = items[item_base + xcd_local_item(blockIdx.x, gridDim.x)];
  const SlotDev& sd = slots[it.slot];
  if (!sd.active) return;
  const SysParams& P = prm[it.slot];
  // wave index made explicitly wave-uniform, so that the chunk loop and
  // the walks over diagonals run on scalar registers
  const int tid = threadIdx.x, lane = tid & (TJ - 1), wv = __builtin_amdgcn_readfirstlane(tid / TJ);
  const int nsp = P.nsp;
  s_tab.load(tab, P, ONE ? 1 : nsp, tid, TJ * NW);

  const int n = sd.n, ld = sd.com_ld, np = sd.npad;
  const double L = P.L, invL = P.invL, rc2 = P.rc2;
  // pairs are listed within the centre cut-off, or in the site-site mode
  // within the radius at which an LJ site pair can still reach
  const double rlist2 = SITE ? P.rc2_search : rc2;
  const ElecParams<Real> E = elec_params<Real>(P);
  LinearModel<Real> lin_model{};
  const Real* __restrict__ gsite = reinterpret_cast<const Real*>(sd.sites);
  const bool diag = it.i0 == it.j0;
  const int nrow = min(TJ, n - it.i0), ncol = min(TJ, n - it.j0);

  {
    // stage both tiles: waves 0/1 the centres and species of rows/columns,
    // waves 2/3 their site records; every global load before the LDS stores
    const int side = wv & 1;
    const int base = side ? it.j0 : it.i0, cnt = side ? ncol : nrow;
    const int mc = lane < cnt ? base + lane : 0;
    if (wv >= 4) {
      // further waves stage nothing
    } else if (wv < 2) {
      double c3[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) c3[c] = sd.com[c * ld + mc];
      const int sp = lane < cnt ? clamp_species(sd.species[mc], nsp) : 0;
      bool in = true;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        (side ? u.t.comj : u.t.comi)[c][lane] = c3[c];
        in = in && c3[c] >= 0.0 && c3[c] <= L;
      }
      if constexpr (!ONE) s_sp[side][lane] = sp;
      const bool all_in = __builtin_amdgcn_ballot_w64(!in) == 0ull;
      if (lane == 0) s_inbox[side] = all_in ? 1 : 0;
    } else {
      Real r[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) r[k] = gsite[(LIN && k >= 3 ? class_reals(C) - 6 + k : k) * np + mc];
#pragma unroll
      for (int k = 0; k < NR; ++k) u.t.site[side][k][lane] = r[k];
      if constexpr (SITE) {
        double l[NL64];
#pragma unroll
        for (int k = 0; k < NL64; ++k) l[k] = sd.lj64[k * np + mc];
#pragma unroll
        for (int k = 0; k < NL64; ++k) u.t.lj64[side][k][lane] = l[k];
      }
    }
    if constexpr (HF) {
      if (wv < 2) {
        const Real* kin = reinterpret_cast<const Real*>(sd.hf_kin);
        Real kv[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) kv[c] = kin[c * np + mc];
#pragma unroll
        for (int c = 0; c < 6; ++c) u.t.kin[side][c][lane] = kv[c];
      }
    }
    s_list[wv][lane] = 0;
  }
  __syncthreads();

  // 1. cut-off bits: wave wv tests columns [CW wv, CW wv + CW) of row `lane`
  //    (centres in [0, L], the usual case: the image-free form of the same r2)
  constexpr int CW = TJ / NW;               // columns (and diagonals) per wave
  constexpr unsigned kWaveBits = CW >= 32 ? 0xFFFFFFFFu : (1u << CW) - 1u;
  {
    const double xi = u.t.comi[0][lane], yi = u.t.comi[1][lane], zi = u.t.comi[2][lane];
    const bool inbox = __builtin_amdgcn_readfirstlane(s_inbox[0] & s_inbox[1]) != 0;
    // the columns this row may pair with, as bits of the wave's CW: inside
    // the tile, and on the diagonal item above the row
    const int j0 = CW * wv, nv = ncol - j0, s = lane - j0 + 1;
    unsigned valid = nv >= CW ? kWaveBits : nv > 0 ? (1u << nv) - 1u : 0u;
    if (diag) valid &= s <= 0 ? kWaveBits : s < CW ? (kWaveBits << s) & kWaveBits : 0u;
    const double* cj = &u.t.comj[0][j0];
    unsigned part = 0;
    if (inbox) {
      for (int b = 0; b < CW; ++b) {
        const double r2 = min_image_r2(xi, yi, zi, cj[b], cj[TJ + b], cj[2 * TJ + b], L);
        part |= (unsigned)(r2 < rlist2) << b;
      }
    } else {
      for (int b = 0; b < CW; ++b) {
        double dx, dy, dz, r2;
        min_image(xi, yi, zi, cj[b], cj[TJ + b], cj[2 * TJ + b], L, invL, dx, dy, dz, r2);
        part |= (unsigned)(r2 < rlist2) << b;
      }
    }
    s_mpart[wv][lane] = lane < nrow ? part & valid : 0u;
  }
  __syncthreads();
  // every wave: the row mask rotated so that bit d is column lane + d, then
  // transposed, so that lane d holds diagonal d's word (bit l: the pair (l,
  // l + d)) of every row l
  unsigned long long dword;
  {
    unsigned m0 = 0, m1 = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if (CW * w < 32) m0 |= s_mpart[w][lane] << (CW * w);
      else m1 |= s_mpart[w][lane] << (CW * w - 32);
    }
    // rotate right by lane: halves swapped for lanes 32-63, then a funnel
    // shift by lane & 31
    const bool swap = lane >= 32;
    const unsigned a = swap ? m1 : m0, b = swap ? m0 : m1;
    const unsigned lo = __builtin_amdgcn_alignbit(b, a, lane & 31), hi = __builtin_amdgcn_alignbit(a, b, lane & 31);
    dword = wave_bit_transpose(((unsigned long long)hi << 32) | lo);
  }
  const int cnt = __popcll(dword);
  const int incl = wave_inclusive_sum(cnt);
  const int doff = incl - cnt;               // lane d: offset of diagonal d
  const int total = __builtin_amdgcn_readlane(incl, TJ - 1);

  if constexpr (LIN) {
    lin_model.c6 = s_tab.c6[0][0];
    lin_model.c12 = s_tab.c12[0][0];
    lin_model.K = kprod<Real>(s_tab.mqd[0][0], s_tab.mqd[0][0], E.inv_ke);
  }
  // one species, centre cut-off: every listed pair counts, with the same
  // number of site pairs, so the item's pair counters follow from the list
  // length (no per-pair counting)
  constexpr bool COUNT_ALL = ONE && !SITE;
  // 2.-3. the diagonal-major list, one pair per lane, chunks dealt to waves
  double a_ulj = 0, a_uel = 0, a_us = 0, a_uss = 0;
  double a_jq[3] = {0, 0, 0};
  int a_np = 0, a_ns = 0;
  Real g_row[6] = {0, 0, 0, 0, 0, 0}, g_col[6] = {0, 0, 0, 0, 0, 0};
  Real(*stage)[TJ] = u.t.stage[wv];
  int* list = s_list[wv];
  unsigned char(*keep)[TJ] = u.t.er[wv];
  // this item's share of the list: chunks s, s + S, ... of the tile pair's
  // ceil(total / 64), dealt to the four waves in turn
  const int n_split = split_count(it.split), i_split = split_index(it.split);
  for (int q = (wv + NW * i_split) * TJ; q < total; q += NW * n_split * TJ) {
    const bool valid = q + lane < total;
    const int qend = min(q + TJ, total);
    // the chunk's diagonals (wave-uniform): from the first one ending after
    // q (it holds entry q) to the last one starting before the chunk's end
    const int dfirst = min((int)__popcll(__builtin_amdgcn_ballot_w64(incl <= q)), TJ - 1);
    const int dlast = (int)__popcll(__builtin_amdgcn_ballot_w64(doff < qend)) - 1;
    for (int dd = dfirst; dd <= dlast; ++dd) {
      const int er = row_entry(readlane64(dword, dd), __builtin_amdgcn_readlane(doff, dd) - q);
      if (er >= 0) list[er] = lane | (dd << 6);
      if (dd - dfirst < kKeepDiags) keep[dd - dfirst][lane] = (unsigned char)er;
    }
    wave_sync_lds();
    const int pr = list[lane];
    const int row = pr & (TJ - 1);
    const int col = (row + (pr >> 6)) & (TJ - 1);

    const int spi = ONE ? 0 : s_sp[0][row], spj = ONE ? 0 : s_sp[1][col];
    double dx, dy, dz, r2d;
    min_image(u.t.comi[0][row], u.t.comi[1][row], u.t.comi[2][row], u.t.comj[0][col], u.t.comj[1][col],
              u.t.comj[2][col], L, invL, dx, dy, dz, r2d);
    const Real Rx = (Real)dx, Ry = (Real)dy, Rz = (Real)dz;
    const Real R2 = (Real)r2d;
    Real rec[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) rec[k] = u.t.site[0][k][row];
    constexpr Real z = -Real(0);             // -0 + x is x: no zeroing, no first add
    PairAcc<Real> acc{z, z, z, z, z, z};
    Real Fi[3] = {z, z, z}, Ti[3] = {z, z, z};
    int ns = s_tab.nsite[spi][spj];
    if constexpr (LIN) {
      Real recj[NR];
#pragma unroll
      for (int k = 0; k < NR; ++k) recj[k] = u.t.site[1][k][col];
      eval_linear_pair(rec, recj, Rx, Ry, Rz, R2, lin_model, acc, Fi, Ti);
    } else {
      SiteAcc<Real, C> ai, unused;
      ai.zero();
      const bool elec_in = !SITE || r2d < rc2;
      int nlj_in = 0;
      const double R64[3] = {dx, dy, dz};
      eval_molecule_pair<Real, C, false, TJ, SITE, ONE>(rec, &u.t.site[1][0][col], spi, spj, s_tab, E, Rx, Ry,
                                                        Rz, R2, ai, unused, acc, SiteCut{R64, &u.t.lj64[0][0][row],
                                                        &u.t.lj64[1][0][col], rc2}, elec_in, &nlj_in);
      // interacting site pairs; in the site-site mode a listed pair counts
      // only when at least one of its site pairs interacts
      if constexpr (SITE) {
        const int nlj2 = s_tab.cnt[spi][0] * s_tab.cnt[spj][0];
        ns = nlj_in + (elec_in ? ns - nlj2 : 0);
      }
      fold_sites<Real, C, 1, Real>(rec, ai, Fi, Ti);
    }
    const Real Tj[3] = {-Ti[0] - (Ry * Fi[2] - Rz * Fi[1]), -Ti[1] - (Rz * Fi[0] - Rx * Fi[2]),
                        -Ti[2] - (Rx * Fi[1] - Ry * Fi[0])};
    if (valid) {
      a_ulj += (double)acc.ulj;
      a_uel += (double)acc.uel;
      a_uss += (double)acc.uss;
      a_us -= (double)(Rx * Fi[0] + Ry * Fi[1] + Rz * Fi[2]);
      if constexpr (!COUNT_ALL) {
        a_np += (!SITE || ns > 0) ? 1 : 0;
        a_ns += ns;
      }
      if constexpr (HF) {
        // pair part of the heat flux: u (v_i + v_j)/2 + R (F.(v_i + v_j) +
        // tau_i.w_i - tau_j.w_j)/2
        Real vs[3], pw = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          vs[c] = u.t.kin[0][c][row] + u.t.kin[1][c][col];
          pw += Fi[c] * vs[c] + Ti[c] * u.t.kin[0][3 + c][row] - Tj[c] * u.t.kin[1][3 + c][col];
        }
        const Real up = acc.ulj + acc.uel;
        a_jq[0] += 0.5 * ((double)(up * vs[0]) + (double)(Rx * pw));
        a_jq[1] += 0.5 * ((double)(up * vs[1]) + (double)(Ry * pw));
        a_jq[2] += 0.5 * ((double)(up * vs[2]) + (double)(Rz * pw));
      }
    }
    stage[0][lane] = Fi[0];
    stage[1][lane] = Fi[1];
    stage[2][lane] = Fi[2];
    stage[3][lane] = Ti[0];
    stage[4][lane] = Ti[1];
    stage[5][lane] = Ti[2];
    stage[6][lane] = Tj[0];
    stage[7][lane] = Tj[1];
    stage[8][lane] = Tj[2];
    wave_sync_lds();
    // gather: molecule `lane` of tile I at its own entry index; molecule
    // `lane` of tile J is the column of row lane - dd
    for (int dd = dfirst; dd <= dlast; ++dd) {
      unsigned er, ec;                       // entry index, or 64 and above for none
      if (dd - dfirst < kKeepDiags) {
        er = keep[dd - dfirst][lane];
        ec = keep[dd - dfirst][(lane - dd) & (TJ - 1)];
      } else {
        er = (unsigned)row_entry(readlane64(dword, dd), __builtin_amdgcn_readlane(doff, dd) - q);
        ec = (unsigned)__shfl((int)er, (lane - dd) & (TJ - 1), TJ);
      }
      if (er < (unsigned)TJ) {
#pragma unroll
        for (int c = 0; c < 6; ++c) g_row[c] += stage[c][er];
      }
      if (ec < (unsigned)TJ) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          g_col[c] -= stage[c][ec];
          g_col[3 + c] += stage[6 + c][ec];
        }
      }
    }
    wave_sync_lds();
  }

  // 5. the waves' partials, added in wave order
  double v[kNumBlockSums] = {a_ulj, a_uel, a_us, a_uss, (double)a_np, (double)a_ns, a_jq[0], a_jq[1], a_jq[2]};
  __syncthreads();                           // tiles and stages are dead from here
  wave_sums(v, u.f.sums[wv]);
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    u.f.part[wv][c][lane] = g_row[c];
    u.f.part[wv][6 + c][lane] = g_col[c];
  }
  __syncthreads();
  // wave w writes three of the twelve components (rows 0-2, rows 3-5,
  // columns 0-2, columns 3-5), each summed over the waves in wave order; on
  // the diagonal item the columns are the rows and waves 0/1 add both
  if (wv < 4) {
    const bool col_side = wv >= 2;
    const int c0 = 3 * (wv & 1);
    Real* pf = reinterpret_cast<Real*>(sd.pf);
    if (!(diag && col_side) && lane < (col_side ? ncol : nrow)) {
      Real* out = pf + (size_t)(col_side ? it.part_j : it.part) * 6 * np + (col_side ? it.j0 : it.i0) + lane;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int c = c0 + k, src = col_side ? 6 + c : c;
        double t = (double)u.f.part[0][src][lane];
#pragma unroll
        for (int w = 1; w < NW; ++w) t += (double)u.f.part[w][src][lane];
        if (diag) {
          double tc = (double)u.f.part[0][6 + c][lane];
#pragma unroll
          for (int w = 1; w < NW; ++w) tc += (double)u.f.part[w][6 + c][lane];
          t += tc;
        }
        out[(size_t)c * np] = (Real)t;
      }
    }
    if (wv == 3 && lane < kNumBlockSums) {
      double t = u.f.sums[0][lane];
#pragma unroll
      for (int w = 1; w < NW; ++w) t += u.f.sums[w][lane];
      // the first of a tile pair's items counts its whole list
      if (COUNT_ALL && lane == 4) t = i_split == 0 ? (double)total : 0.0;
      if (COUNT_ALL && lane == 5) t = i_split == 0 ? (double)total * (double)s_tab.nsite[0][0] : 0.0;
      sd.bsum[(size_t)it.local * kNumBlockSums + lane] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Fixed-order reductions of the pair partials.
//  forces: one thread per molecule and component sums its partials in
//    order, in FP64 (the partials are in the slot's Real: each is a sum of at
//    most one tile's pair terms).  OVERWRITES force and torque.
//  sums: one block per slot; item sums (each thread a contiguous run, then a
//    tree), species counts, Ewald constants and the LJ tail.  OVERWRITES sums.
//  One launch does both (reduce_pair_kernel).
// ---------------------------------------------------------------------------
// one thread per (component, molecule): block bx of the slot's 6 x mb force
// blocks, six runs of molecule blocks, one per force/torque component, so
// that the largest systems' serial chains are one component long
__device__ __forceinline__ void reduce_force_block(const SlotDev* __restrict__ slots,
                                                   const SysParams* __restrict__ prm, int bx, int mb, bool with_k) {
  const SlotDev& sd = slots[blockIdx.y];
  if (!sd.active) return;
  const int c = bx / mb;
  const int i = (bx - c * mb) * 256 + threadIdx.x;
  if (i >= sd.n) return;
  const int np = sd.npad, ld = sd.com_ld, nparts = sd.jsplits;
  const size_t stride = (size_t)6 * np;
  // a species index outside the table makes this molecule's result NaN
  double v = species_ok(sd.species[i], prm[blockIdx.y].nsp) ? 0.0 : __builtin_nan("");
  // the loads of four partials are issued before their additions, which
  // keep the order p = 0, 1, 2, ...
  auto reduce = [&](auto* __restrict__ pf) {
    int p = 0;
    for (; p + 4 <= nparts; p += 4) {
      const double x0 = (double)pf[(size_t)p * stride], x1 = (double)pf[(size_t)(p + 1) * stride];
      const double x2 = (double)pf[(size_t)(p + 2) * stride], x3 = (double)pf[(size_t)(p + 3) * stride];
      v += x0;
      v += x1;
      v += x2;
      v += x3;
    }
    for (; p < nparts; ++p) v += (double)pf[(size_t)p * stride];
  };
  if (sd.pf_single)
    reduce(reinterpret_cast<const float*>(sd.pf) + (size_t)c * np + i);
  else
    reduce(reinterpret_cast<const double*>(sd.pf) + (size_t)c * np + i);
  // the reciprocal part added to the stored pair sum, as its own reduction
  // would add it
  if (with_k && prm[blockIdx.y].elec == MS2_ELEC_EWALD) v = v + kspace_force_sum(sd, c, i);
  if (c < 3)
    sd.force[c * ld + i] = v;
  else
    sd.torque[(c - 3) * ld + i] = v;
}

__device__ __forceinline__ void reduce_sums_block(const SlotDev* __restrict__ slots,
                                                  const SysParams* __restrict__ prm, int slot, bool with_k) {
  // per-wave totals and the reciprocal sums' trees (6 KB): the launch's
  // force blocks share this kernel's static LDS size, so the sums keep it
  // small
  __shared__ double s_red[4][kNumBlockSums];
  __shared__ int s_cnt[4][kMaxSp];
  __shared__ double s_kd[256], s_ku[256], s_kw[256];
  const SlotDev& sd = slots[slot];
  if (!sd.active) return;
  const SysParams& P = prm[slot];
  const int tid = threadIdx.x, n = sd.n;
  int cnt[kMaxSp];
#pragma unroll
  for (int s = 0; s < kMaxSp; ++s) cnt[s] = 0;
  int bad = 0;                               // species indices outside the table
  // loads of four iterations are issued before their uses (the order of the
  // additions is unchanged)
  {
    int i = tid;
    for (; i + 3 * 256 < n; i += 4 * 256) {
      const int s0 = sd.species[i], s1 = sd.species[i + 256], s2 = sd.species[i + 512], s3 = sd.species[i + 768];
      for (const int sr : {s0, s1, s2, s3}) {
        bad += species_ok(sr, P.nsp) ? 0 : 1;
        const int sp = clamp_species(sr, P.nsp);
#pragma unroll
        for (int x = 0; x < kMaxSp; ++x) cnt[x] += (sp == x);
      }
    }
    for (; i < n; i += 256) {
      bad += species_ok(sd.species[i], P.nsp) ? 0 : 1;
      const int sp = clamp_species(sd.species[i], P.nsp);
#pragma unroll
      for (int x = 0; x < kMaxSp; ++x) cnt[x] += (sp == x);
    }
  }
  const int ni = sd.nitems;
  const int per = (ni + 255) / 256;
  double acc[kNumBlockSums] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  {
    const int t1 = min(ni, (tid + 1) * per);
    int t = tid * per;
    for (; t + 4 <= t1; t += 4) {
      double v[4][kNumBlockSums];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < kNumBlockSums; ++k) v[u][k] = sd.bsum[(size_t)(t + u) * kNumBlockSums + k];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < kNumBlockSums; ++k) acc[k] += v[u][k];
    }
    for (; t < t1; ++t)
#pragma unroll
      for (int k = 0; k < kNumBlockSums; ++k) acc[k] += sd.bsum[(size_t)t * kNumBlockSums + k];
  }
  // the 64 lanes of each wave in butterfly order (a fixed order), then the
  // four waves' totals in wave order
#pragma unroll
  for (int h = 32; h > 0; h >>= 1) {
#pragma unroll
    for (int k = 0; k < kNumBlockSums; ++k) acc[k] += __shfl_xor(acc[k], h, 64);
#pragma unroll
    for (int x = 0; x < kMaxSp; ++x) cnt[x] += __shfl_xor(cnt[x], h, 64);
  }
  const int wave = tid >> 6, lane = tid & 63;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kNumBlockSums; ++k) s_red[wave][k] = acc[k];
#pragma unroll
    for (int x = 0; x < kMaxSp; ++x) s_cnt[wave][x] = cnt[x];
  }
  const bool any_bad = __syncthreads_or(bad);
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < kNumBlockSums; ++k)
      s_red[0][k] = ((s_red[0][k] + s_red[1][k]) + s_red[2][k]) + s_red[3][k];
#pragma unroll
    for (int x = 0; x < kMaxSp; ++x) s_cnt[0][x] = s_cnt[0][x] + s_cnt[1][x] + s_cnt[2][x] + s_cnt[3][x];
  }
  if (tid == 0) {
    double* out = sd.sums;
    // row-owned items evaluate every pair from both sides; symmetric ones once
    const double h = sd.symmetric ? 1.0 : 0.5;
    out[MS2_SUM_U_LJ] = h * s_red[0][0];
    out[MS2_SUM_U_ELEC] = h * s_red[0][1];
    out[MS2_SUM_US] = h * s_red[0][2];
    out[MS2_SUM_VIRIAL] = -h * s_red[0][2];
    out[MS2_SUM_USS] = h * s_red[0][3];
    out[MS2_SUM_NPAIR] = h * s_red[0][4];
    out[MS2_SUM_NSITE] = h * s_red[0][5];
    out[MS2_SUM_U_RECIP] = 0.0;
    if (sd.jq)
      for (int c = 0; c < 3; ++c) sd.jq[c] = s_red[0][6 + c];
    double uc = 0.0, ul = 0.0, usl = 0.0, ussl = 0.0;
    for (int a = 0; a < P.nsp; ++a) {
      const double na = (double)s_cnt[0][a];
      if (P.elec == MS2_ELEC_EWALD) uc += na * P.ew_const[a];
      if (P.lrc)
        for (int b = 0; b < P.nsp; ++b) {
          const double nab = na * (double)s_cnt[0][b];
          ul += nab * P.lrc_u[a][b];
          usl += nab * P.lrc_us[a][b];
          ussl += nab * P.lrc_uss[a][b];
        }
    }
    out[MS2_SUM_U_CONST] = uc;
    out[MS2_SUM_U_LRC] = ul;
    out[MS2_SUM_US_LRC] = usl;
    out[MS2_SUM_USS_LRC] = ussl;
    if (any_bad) {
      // an argument error found on the device: no sum of this call is valid
      for (int k = 0; k < MS2_SUM_NPAIR; ++k) out[k] = __builtin_nan("");
      if (sd.err) *sd.err = 1;
    }
  }
  if (with_k && P.elec == MS2_ELEC_EWALD) {
    __syncthreads();
    kspace_sums_block(sd, P, s_kd, s_ku, s_kw);
  }
}

// Both reductions in one launch: grid (6 x molecule blocks + 1, slots); the
// last block of each slot's row sums its work items' block sums.  With
// with_k, Ewald slots also get their reciprocal forces, torques and sums
// (the structure factor and force partials must be complete), added after
// the pair sums as the reciprocal reductions would add them: the same bits
// in one launch instead of three.
__global__ __launch_bounds__(256) void reduce_pair_kernel(const SlotDev* __restrict__ slots,
                                                          const SysParams* __restrict__ prm, int with_k) {
  const int mb = (gridDim.x - 1) / 6;
  if ((int)blockIdx.x < 6 * mb)
    reduce_force_block(slots, prm, blockIdx.x, mb, with_k != 0);
  else
    reduce_sums_block(slots, prm, blockIdx.y, with_k != 0);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename Real, int C>
static hipError_t launch_frame_c(const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                                 int nslots, int max_n, hipStream_t st) {
  dim3 grid((max_n + 255) / 256, nslots);
  hipLaunchKernelGGL((site_frame_kernel<Real, C>), grid, dim3(256), 0, st, slots, prm, tab);
  return hipGetLastError();
}

hipError_t launch_site_frame(int cls, int precision, const SlotDev* slots, const SysParams* prm,
                             const SpeciesTable* tab, int nslots, int max_n, hipStream_t st) {
#define MS2_FRAME_CASE(C)                                                                       \
  case C:                                                                                       \
    return precision == MS2_FP32 ? launch_frame_c<float, C>(slots, prm, tab, nslots, max_n, st) \
                                 : launch_frame_c<double, C>(slots, prm, tab, nslots, max_n, st);
  switch (cls) {
    MS2_FRAME_CASE(0)
    MS2_FRAME_CASE(1)
    MS2_FRAME_CASE(2)
    MS2_FRAME_CASE(3)
    MS2_FRAME_CASE(4)
    MS2_FRAME_CASE(5)
  }
#undef MS2_FRAME_CASE
  return hipErrorInvalidValue;
}

template <typename Real, int C, int W>
static hipError_t launch_pair_cw(const WorkItem* items, int base, int count, const SlotDev* slots,
                                 const SysParams* prm, const SpeciesTable* tab, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((pair_kernel<Real, C, W>), dim3(count), dim3(64 * W), 0, st, items, base, slots,
                     prm, tab);
  return hipGetLastError();
}

template <typename Real, int C, bool HF, bool SITE>
static hipError_t launch_pair_sym(int form, const WorkItem* items, int base, int count,
                                  const SlotDev* slots, const SysParams* prm, const SpeciesTable* tab,
                                  hipStream_t st) {
  // the linear form; in FP64 it runs at three waves per SIMD (150 VGPRs: at
  // four it spills, 13.7 against 8.0 ms per batched step; at three, 8.13
  // against 8.22 ms for the general single-species form at four)
  if constexpr (C == 1 && !HF && !SITE) {
    if (form == kFormLinear) {
      hipLaunchKernelGGL((pair_sym_kernel<Real, C, HF, SITE, true, true>), dim3(count), dim3(64 * kSymWaves), 0,
                         st, items, base, slots, prm, tab);
      return hipGetLastError();
    }
  }
  if constexpr (C <= 3) {
    if (form != kFormGeneral) {
      hipLaunchKernelGGL((pair_sym_kernel<Real, C, HF, SITE, true>), dim3(count), dim3(64 * kSymWaves), 0, st,
                         items, base, slots, prm, tab);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((pair_sym_kernel<Real, C, HF, SITE, false>), dim3(count), dim3(64 * kSymWaves), 0, st,
                     items, base, slots, prm, tab);
  return hipGetLastError();
}

template <typename Real, int C>
static hipError_t launch_pair_c(int waves, bool heat_flux, bool site_cut, int form, const WorkItem* items,
                                int base, int count, const SlotDev* slots, const SysParams* prm,
                                const SpeciesTable* tab, hipStream_t st) {
  if (waves == 0) {  // symmetric tile pairs
    if (count <= 0) return hipSuccess;
    if (site_cut)
      return heat_flux ? launch_pair_sym<Real, C, true, true>(form, items, base, count, slots, prm, tab, st)
                       : launch_pair_sym<Real, C, false, true>(form, items, base, count, slots, prm, tab, st);
    return heat_flux ? launch_pair_sym<Real, C, true, false>(form, items, base, count, slots, prm, tab, st)
                     : launch_pair_sym<Real, C, false, false>(form, items, base, count, slots, prm, tab, st);
  }
  // the heat flux and the site-site cut-off run on symmetric items only
  if (heat_flux || site_cut) return hipErrorInvalidValue;
  if constexpr (C <= 3) {
    if (waves == 4) return launch_pair_cw<Real, C, 4>(items, base, count, slots, prm, tab, st);
  }
  return launch_pair_cw<Real, C, 1>(items, base, count, slots, prm, tab, st);
}

hipError_t launch_pair(int cls, int precision, int waves, bool heat_flux, bool site_cut, int form,
                       const WorkItem* items, int base, int count, const SlotDev* slots, const SysParams* prm,
                       const SpeciesTable* tab, hipStream_t st) {
#define MS2_PAIR_CASE(C)                                                                                       \
  case C:                                                                                                      \
    return precision == MS2_FP32                                                                               \
               ? launch_pair_c<float, C>(waves, heat_flux, site_cut, form, items, base, count, slots, prm, tab, st)  \
               : launch_pair_c<double, C>(waves, heat_flux, site_cut, form, items, base, count, slots, prm, tab, st);
  switch (cls) {
    MS2_PAIR_CASE(0)
    MS2_PAIR_CASE(1)
    MS2_PAIR_CASE(2)
    MS2_PAIR_CASE(3)
    MS2_PAIR_CASE(4)
    MS2_PAIR_CASE(5)
  }
#undef MS2_PAIR_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_pair(const SlotDev* slots, const SysParams* prm, int nslots, int max_n,
                              hipStream_t st) {
  hipLaunchKernelGGL(reduce_pair_kernel, dim3(6 * ((max_n + 255) / 256) + 1, nslots), dim3(256), 0, st, slots,
                     prm, 0);
  return hipGetLastError();
}

hipError_t launch_reduce_pair_kspace(const SlotDev* slots, const SysParams* prm, int nslots, int max_n,
                                     hipStream_t st) {
  hipLaunchKernelGGL(reduce_pair_kernel, dim3(6 * ((max_n + 255) / 256) + 1, nslots), dim3(256), 0, st, slots,
                     prm, 1);
  return hipGetLastError();
}

}  // namespace ms2
