// hesp_device.h -- device helpers shared by the gfx950 kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_core.h"
#include "hesp_internal.h"

namespace hesp {
namespace dev {

constexpr int64_t kInf = INT64_MAX;
constexpr uint32_t kNil = 0xFFFFFFFFu;
constexpr int kOK = 0, kEINVAL = -1, kECAP = -4;

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Loads of data this kernel writes go through the vector memory path.
template <class T>
__device__ __forceinline__ T vld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Arrays updated by atomic read-modify-writes (performed in L2, past the L1)
// are read at device scope so that no stale L1 line can be returned.
template <class T>
__device__ __forceinline__ T vld_l2(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every workgroup is a single wavefront, and the lanes of one wavefront share
// the compute unit's vector L1: global-memory accesses of the wavefront are
// coherent between its lanes without waiting on the memory counters.  Only the
// compiler must not move memory accesses across these points.
__device__ __forceinline__ void wave_order() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ int64_t rdl64(int64_t v, int l) {
  uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
  uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ int rdl32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// DPP lane moves of a 64-bit value (lanes left out by the row mask keep v).
// With every row enabled, the controls used here (quad permutations, row
// rotations) give each lane a source inside its row, so the destination's old
// value is never read and need not be a copy of v.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
  const int lo = (int)(uint32_t)(uint64_t)v, hi = (int)(uint32_t)((uint64_t)v >> 32);
  int rlo, rhi;
  if constexpr (ROWS == 0xF) {
    rlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, true);
    rhi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, true);
  } else {
    rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
    rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  }
  return (int64_t)(((uint64_t)(uint32_t)rhi << 32) | (uint32_t)rlo);
}
constexpr int kQuadSwap1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadSwap2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return b < a ? b : a; }
__device__ __forceinline__ int64_t max64(int64_t a, int64_t b) { return b > a ? b : a; }

// minimum of a 32-bit unsigned value over the 64 lanes, returned to every lane
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  auto mn = [](uint32_t a, int b) { return a < (uint32_t)b ? a : (uint32_t)b; };
  v = mn(v, __builtin_amdgcn_update_dpp(0, (int)v, kQuadSwap1, 0xF, 0xF, true));
  v = mn(v, __builtin_amdgcn_update_dpp(0, (int)v, kQuadSwap2, 0xF, 0xF, true));
  v = mn(v, __builtin_amdgcn_update_dpp(0, (int)v, kRowRor4, 0xF, 0xF, true));
  v = mn(v, __builtin_amdgcn_update_dpp(0, (int)v, kRowRor8, 0xF, 0xF, true));
  v = mn(v, __builtin_amdgcn_update_dpp((int)v, (int)v, kRowBcast15, 0xA, 0xF, false));
  v = mn(v, __builtin_amdgcn_update_dpp((int)v, (int)v, kRowBcast31, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, kWave - 1);
}

// maximum over aligned segments of 2^lg lanes (lg in {0, 2, 4, 5, 6}); the
// last lane of every segment holds its segment's maximum (all lanes for lg <= 4)
__device__ __forceinline__ int64_t seg_max64(int64_t v, int lg) {
  if (lg >= 2) {
    v = max64(v, dpp64<kQuadSwap1>(v));
    v = max64(v, dpp64<kQuadSwap2>(v));
  }
  if (lg >= 4) {
    v = max64(v, dpp64<kRowRor4>(v));
    v = max64(v, dpp64<kRowRor8>(v));
  }
  if (lg >= 5) v = max64(v, dpp64<kRowBcast15, 0xA>(v));
  if (lg >= 6) v = max64(v, dpp64<kRowBcast31, 0xC>(v));
  return v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = lane();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int y = __shfl_up(v, o, kWave);
    if (l >= o) v += y;
  }
  return v;
}

__device__ __forceinline__ uint64_t lanes_below() { return (1ull << lane()) - 1ull; }

struct Cand {
  int nt, dmax, n_top;
  const uint8_t* depth;
};

__device__ __forceinline__ Cand load_cand(const BatchView& b, int c) {
  Cand x;
  x.nt = b.nt_arr ? b.nt_arr[c] : b.nt;
  x.dmax = b.dmax_arr ? b.dmax_arr[c] : b.dmax;
  x.n_top = (int)tet3(x.nt);
  x.depth = b.depth + (b.off ? b.off[c] : (int64_t)c * x.n_top);
  return x;
}

// Visit every fine task, 64 top-level tasks at a time: fn(f, top, cell, d, K, I, J)
// with f counted from `first_fine` in the global numbering.  All lanes call fn
// (with valid=false beyond the end) so that fn may use cross-lane operations.
template <class Fn>
__device__ void for_each_fine(const Cand& c, Fn&& fn) {
  const int l = lane();
  int64_t carry = 0;
  for (int t0 = 0; t0 < c.n_top; t0 += kWave) {
    const int t = t0 + l;
    const bool vt = t < c.n_top;
    const uint32_t cell = vt ? top_cell(c.nt, t) : 0u;
    int d = vt ? (int)c.depth[t] : 0;
    d = d > c.dmax ? c.dmax : d;
    const int cnt = vt ? fine_count(kind_of(cell_k(cell), cell_i(cell), cell_j(cell)), d) : 0;
    const int incl = wave_incl_scan(cnt);
    const int total = rdl32(incl, kWave - 1);
    for (int r0 = 0; r0 < total; r0 += kWave) {
      const int rel = r0 + l;
      int lo = 0, hi = kWave - 1;  // owner lane: smallest with incl > rel
#pragma unroll
      for (int it = 0; it < 6; it++) {
        const int mid = (lo + hi) >> 1;
        const int v = __shfl(incl, mid, kWave);
        if (v > rel) hi = mid; else lo = mid + 1;
      }
      const int own = lo > kWave - 1 ? kWave - 1 : lo;
      const uint32_t ocell = (uint32_t)__shfl((int)cell, own, kWave);
      const int od = __shfl(d, own, kWave);
      const int ocnt = __shfl(cnt, own, kWave);
      const int oincl = __shfl(incl, own, kWave);
      const bool valid = rel < total;
      int K = 0, I = 0, J = 0;
      if (valid) {
        const int s = 1 << od;
        const int kind = kind_of(cell_k(ocell), cell_i(ocell), cell_j(ocell));
        int q, r, cc;
        local_coords(kind, s, rel - (oincl - ocnt), q, r, cc);
        K = cell_k(ocell) * s + q;
        I = cell_i(ocell) * s + r;
        J = cell_j(ocell) * s + cc;
      }
      fn(valid, carry + rel, (int64_t)(t0 + own), ocell, od, K, I, J);
    }
    carry += total;
  }
}

// finest block (atom) number of position (u, v) inside block (R, C) of level lvl
__device__ __forceinline__ int64_t atom_base(int nt, int dmax, int lvl, int R, int C) {
  const int tr = R >> lvl, tc = C >> lvl;
  const int w = 1 << (dmax - lvl);
  const int fr = (R & ((1 << lvl) - 1)) * w, fc = (C & ((1 << lvl) - 1)) * w;
  const int64_t tile = (int64_t)tr * nt - (int64_t)tr * (tr - 1) / 2 + (tc - tr);
  return (tile << (2 * dmax)) + ((int64_t)fr << dmax) + fc;
}

// ordering key of a ready task: fine indices scaled to the finest level
__device__ __forceinline__ uint32_t task_key_of(int dmax, int lvl, int K, int I, int J) {
  const int sh = dmax - lvl;
  return ((uint32_t)(K << sh) << 18) | ((uint32_t)(I << sh) << 9) | (uint32_t)(J << sh);
}
__device__ __forceinline__ uint32_t task_key(uint32_t dsc, int dmax) {
  return task_key_of(dmax, desc_level(dsc), desc_K(dsc), desc_I(dsc), desc_J(dsc));
}

// Dispatch word of a fine task, computed once by the preparation so that the
// event loop decodes nothing: the first finest block (atom) of each data block
// the task touches (reads first, the written block last), its level, kind and
// number of blocks:
//   atom0:18 | atom1:18 | atom2:18 | level:3 | kind:2 | blocks:2
// Eighteen bits hold every atom number: a candidate has at most F (F + 2^dmax) / 2
// finest blocks, F = nt 2^dmax <= kMaxFine.
static_assert((int64_t)kMaxFine * (kMaxFine + (1 << kMaxLevel)) / 2 <= (1 << 18), "atom numbers need 18 bits");
static_assert(kMaxLevel < 8, "levels need 3 bits");
__device__ __forceinline__ uint64_t dispatch_word(int nt, int dmax, int kind, int lvl, int K, int I, int J) {
  int br[3] = {0, 0, 0}, bc[3] = {0, 0, 0};
  const int nb = desc_blocks(pack_desc(kind, lvl, K, I, J), br, bc);
  // atom_base in 32-bit arithmetic (every atom number is below 2^18)
  const int w_l = 1 << (dmax - lvl), lmask = (1 << lvl) - 1;
  uint64_t w = 0;
  for (int b = 0; b < 3; b++) {
    const int tr = br[b] >> lvl, tc = bc[b] >> lvl;
    const int tile = tr * nt - ((tr * (tr - 1)) >> 1) + (tc - tr);
    const int atom = (tile << (2 * dmax)) + (((br[b] & lmask) * w_l) << dmax) + (bc[b] & lmask) * w_l;
    if (b < nb) w |= (uint64_t)(uint32_t)atom << (18 * b);
  }
  return w | ((uint64_t)lvl << 54) | ((uint64_t)kind << 57) | ((uint64_t)nb << 59);
}
__device__ __forceinline__ int dw_atom(uint64_t w, int b) { return (int)((w >> (18 * b)) & 0x3FFFFu); }
__device__ __forceinline__ int dw_level(uint64_t w) { return (int)((w >> 54) & 7u); }
__device__ __forceinline__ int dw_kind(uint64_t w) { return (int)((w >> 57) & 3u); }
__device__ __forceinline__ int dw_blocks(uint64_t w) { return (int)((w >> 59) & 3u); }
// A task with at most two successors keeps their numbers in its record in place
// of its edge range (kNil for an absent one); bit 61 of its dispatch word says so.
constexpr uint64_t kDwInline = 1ull << 61;
__device__ __forceinline__ bool dw_inline(uint64_t w) { return (w & kDwInline) != 0; }
// what a completion needs of the task: the written block's atom, the level and
// (bit 31) whether its successors are inline
__device__ __forceinline__ uint32_t completion_word(uint64_t w) {
  return (uint32_t)dw_atom(w, dw_blocks(w) - 1) | ((uint32_t)dw_level(w) << 18) | ((uint32_t)dw_inline(w) << 31);
}
__device__ __forceinline__ int cw_level(uint32_t cw) { return (int)((cw >> 18) & 7u); }
__device__ __forceinline__ bool cw_inline(uint32_t cw) { return (cw >> 31) != 0; }


// ---------------------------------------------------------------- lane groups
// A wavefront holds kWave / G independent groups of G lanes (G = 16, 32 or 64).
// Values that are uniform inside a group live in VGPRs; cross-lane operations
// only read lanes of the same group: DPP within 16-lane rows, ds_bpermute for
// broadcasts, and masked ballots.
template <int G>
struct Grp {
  static constexpr int NG = kWave / G;
  int l, g, gl, gbase;
  uint64_t gmask;
  __device__ __forceinline__ Grp() {
    l = lane();
    g = l / G;
    gl = l % G;
    gbase = g * G;
    gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << gbase);
  }
  // bits of the group's lanes, lane gl at bit gl
  __device__ __forceinline__ uint64_t ballot(bool p) const {
    const uint64_t b = __ballot(p) & gmask;
    return G == 64 ? b : (b >> gbase);
  }
  __device__ __forceinline__ uint64_t below() const { return (1ull << gl) - 1ull; }
  // broadcast from group lane j (j uniform inside the group); a whole-wave group
  // reads the lane into scalar registers
  __device__ __forceinline__ int bcast(int v, int j) const {
    if (G == 64) return __builtin_amdgcn_readlane(v, __builtin_amdgcn_readfirstlane(j));
    return __shfl(v, gbase + j, kWave);
  }
  __device__ __forceinline__ int64_t bcast64(int64_t v, int j) const {
    if (G == 64) return rdl64(v, __builtin_amdgcn_readfirstlane(j));
    return __shfl(v, gbase + j, kWave);
  }
  // the value of group lane j, j chosen per lane (all lanes of the group active)
  __device__ __forceinline__ int64_t read64(int64_t v, int j) const { return __shfl(v, gbase + j, kWave); }
  // a value known to be uniform inside the group (scalar for a whole-wave group)
  __device__ __forceinline__ int uni(int v) const { return G == 64 ? __builtin_amdgcn_readfirstlane(v) : v; }
  __device__ __forceinline__ int64_t uni64(int64_t v) const { return G == 64 ? rdl64(v, 0) : v; }
  // minimum over the group, returned to every lane of the group
  __device__ __forceinline__ int64_t min64all(int64_t v) const {
    v = min64(v, dpp64<kQuadSwap1>(v));
    v = min64(v, dpp64<kQuadSwap2>(v));
    v = min64(v, dpp64<kRowRor4>(v));
    v = min64(v, dpp64<kRowRor8>(v));
    if (G >= 32) v = min64(v, dpp64<kRowBcast15, 0xA>(v));
    if (G >= 64) v = min64(v, dpp64<kRowBcast31, 0xC>(v));
    if (G >= 32) v = bcast64(v, G - 1);
    return v;
  }
  // the same for a non-negative value that is kInf outside the group's first 16
  // lanes whenever lo16 (uniform) holds: the minimum of lanes 0..15 is then
  // taken on 32-bit halves inside the first row (the high words, then the low
  // words of the lanes holding the least high word; each step one DPP-fused
  // unsigned minimum) and broadcast from the group's lane 0
  __device__ __forceinline__ int64_t min64lo(int64_t v, bool lo16) const {
    if (G <= 16 || !lo16) return min64all(v);
    auto row_min = [](uint32_t x) {
      auto mn = [](uint32_t a, int b) { return a < (uint32_t)b ? a : (uint32_t)b; };
      x = mn(x, __builtin_amdgcn_update_dpp(0, (int)x, kQuadSwap1, 0xF, 0xF, true));
      x = mn(x, __builtin_amdgcn_update_dpp(0, (int)x, kQuadSwap2, 0xF, 0xF, true));
      x = mn(x, __builtin_amdgcn_update_dpp(0, (int)x, kRowRor4, 0xF, 0xF, true));
      x = mn(x, __builtin_amdgcn_update_dpp(0, (int)x, kRowRor8, 0xF, 0xF, true));
      return x;
    };
    const uint32_t hi = (uint32_t)((uint64_t)v >> 32), lo = (uint32_t)(uint64_t)v;
    const uint32_t mh = row_min(hi);
    const uint32_t ml = row_min(hi == mh ? lo : 0xFFFFFFFFu);
    const uint32_t bh = (uint32_t)bcast((int)mh, 0), bl = (uint32_t)bcast((int)ml, 0);
    return (int64_t)(((uint64_t)bh << 32) | bl);
  }
};

}  // namespace dev
}  // namespace hesp
