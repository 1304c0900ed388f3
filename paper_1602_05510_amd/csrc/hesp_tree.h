// hesp_tree.h -- device helpers for split-tree candidates (internal): the walk
// over a candidate's tasks in program order and the last-writer dependence scan.
// A split-tree candidate holds one flag per task of each uniform level-l tiling
// (nt 2^l tiles, Fig. 1 order, levels 0 .. dmax-1 concatenated).  A level-l
// task exists when its ancestors are split; a flagged one is replaced in place
// by the blocked algorithm of its kind on the 2 x 2 sub-tiling of its cell
// (section 2.1, "Recursive task partitioners", applied to any task).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_core.h"
#include "hesp_device.h"

namespace hesp {
namespace dev {

__device__ __forceinline__ int64_t tree_level_off(int nt, int l) {
  int64_t o = 0;
  for (int x = 0; x < l; x++) o += tet3((int64_t)nt << x);
  return o;
}

// Child x of a split task in the order of the Fig. 1 loop nest restricted to its
// 2 x 2 sub-tiling, as a local index: the same order except in a syrk cell,
// where each row step issues its gemm before its syrk.
__device__ __forceinline__ int fig1_child(int kind, int x) {
  if (kind != SYRK) return x;
  const int r = x % 3;
  return x - r + (r == 0 ? 1 : (r == 1 ? 0 : 2));
}

// The tasks (leaves) of a candidate of depth 4 or 5 in program order: a
// depth-first walk keeping, per level below the current task, the split task
// and its next child.
template <class Fn>
__device__ void walk_tree_deep(int nt, int dmax, const uint8_t* flags, Fn&& fn) {
  int64_t off[kMaxLevel];
  for (int l = 0; l < kMaxLevel; l++) off[l] = tree_level_off(nt, l);
  auto split = [&](int lv, int K, int I, int J) {
    return lv < dmax && flags[off[lv] + top_index(nt << lv, K, I, J)] != 0;
  };
  int pk[kMaxLevel], pK[kMaxLevel], pI[kMaxLevel], pJ[kMaxLevel], px[kMaxLevel];
  const int64_t n_top = tet3(nt);
  for (int64_t t = 0; t < n_top; t++) {
    const uint32_t cell = top_cell(nt, t);
    const int k0 = cell_k(cell), i0 = cell_i(cell), j0 = cell_j(cell), kd0 = kind_of(k0, i0, j0);
    if (!split(0, k0, i0, j0)) {
      fn(kd0, 0, k0, i0, j0);
      continue;
    }
    int sp = 0;
    pk[0] = kd0; pK[0] = k0; pI[0] = i0; pJ[0] = j0; px[0] = 0;
    while (sp >= 0) {
      if (px[sp] == fine_count(pk[sp], 1)) {
        sp--;
        continue;
      }
      int q, r, w;
      local_coords(pk[sp], 2, fig1_child(pk[sp], px[sp]), q, r, w);
      px[sp]++;
      const int k = 2 * pK[sp] + q, i = 2 * pI[sp] + r, j = 2 * pJ[sp] + w, kd = kind_of(k, i, j), lv = sp + 1;
      if (split(lv, k, i, j)) {   // lv < dmax <= kMaxLevel: sp + 1 stays inside the arrays
        sp++;
        pk[sp] = kd; pK[sp] = k; pI[sp] = i; pJ[sp] = j; px[sp] = 0;
      } else {
        fn(kd, lv, k, i, j);
      }
    }
  }
}

// The tasks (leaves) of a candidate in program order: fn(kind, level, K, I, J)
// with wave-uniform arguments.  Up to depth 3 the walk is unrolled (level-3
// tasks are leaves); deeper candidates take walk_tree_deep.
template <class Fn>
__device__ void walk_tree(int nt, int dmax, const uint8_t* flags, Fn&& fn) {
  if (dmax > 3) {
    walk_tree_deep(nt, dmax, flags, fn);
    return;
  }
  const int64_t n_top = tet3(nt);
  const int64_t off1 = tree_level_off(nt, 1), off2 = tree_level_off(nt, 2);
  auto split = [&](int lv, int64_t off, int K, int I, int J) {
    return lv < dmax && flags[off + top_index(nt << lv, K, I, J)] != 0;
  };
  for (int64_t t = 0; t < n_top; t++) {
    const uint32_t cell = top_cell(nt, t);
    const int k0 = cell_k(cell), i0 = cell_i(cell), j0 = cell_j(cell), kd0 = kind_of(k0, i0, j0);
    if (!split(0, 0, k0, i0, j0)) {
      fn(kd0, 0, k0, i0, j0);
      continue;
    }
    for (int x1 = 0; x1 < fine_count(kd0, 1); x1++) {
      int q, r, w;
      local_coords(kd0, 2, fig1_child(kd0, x1), q, r, w);
      const int k1 = 2 * k0 + q, i1 = 2 * i0 + r, j1 = 2 * j0 + w, kd1 = kind_of(k1, i1, j1);
      if (!split(1, off1, k1, i1, j1)) {
        fn(kd1, 1, k1, i1, j1);
        continue;
      }
      for (int x2 = 0; x2 < fine_count(kd1, 1); x2++) {
        local_coords(kd1, 2, fig1_child(kd1, x2), q, r, w);
        const int k2 = 2 * k1 + q, i2 = 2 * i1 + r, j2 = 2 * j1 + w, kd2 = kind_of(k2, i2, j2);
        if (!split(2, off2, k2, i2, j2)) {
          fn(kd2, 2, k2, i2, j2);
          continue;
        }
        for (int x3 = 0; x3 < fine_count(kd2, 1); x3++) {
          local_coords(kd2, 2, fig1_child(kd2, x3), q, r, w);
          const int k3 = 2 * k2 + q, i3 = 2 * i2 + r, j3 = 2 * j2 + w;
          fn(kind_of(k3, i3, j3), 3, k3, i3, j3);
        }
      }
    }
  }
}

// Dependences of task f from the last writer of every finest block it reads or
// writes (read-after-write and write-after-write; in this factorization a task
// reads only finalized blocks and its own output block, so write-after-read
// edges are implied by these): emit(p) once per distinct writer, smallest
// first, wave-uniform; then the blocks f writes record it.  Returns the count.
template <class EmitF>
__device__ __forceinline__ int scan_task(uint32_t* lw, int nt, int dmax, int kind, int lvl, int K, int I, int J,
                                         uint32_t f, EmitF&& emit) {
  const int l = lane();
  int br[3], bc[3];
  const int nb = desc_blocks(pack_desc(kind, lvl, K, I, J), br, bc);
  const int sh = dmax - lvl, lg = 2 * sh, wmask = (1 << sh) - 1;
  const int items = nb << lg;                       // 3 x 4^sh finest blocks at most
  auto atom_of = [&](int it) {
    const int b = it >> lg, a = it & ((1 << lg) - 1);
    const int R = b == 0 ? br[0] : (b == 1 ? br[1] : br[2]);
    const int C = b == 0 ? bc[0] : (b == 1 ? bc[1] : bc[2]);
    return atom_base(nt, dmax, lvl, R, C) + ((int64_t)(a >> sh) << dmax) + (a & wmask);
  };
  int n = 0;
  if (items <= 3 * kWave) {
    // up to three finest blocks per lane, held in registers
    uint32_t v0 = kNil, v1 = kNil, v2 = kNil;
    if (l < items) v0 = vld(&lw[atom_of(l)]);
    if (l + kWave < items) v1 = vld(&lw[atom_of(l + kWave)]);
    if (l + 2 * kWave < items) v2 = vld(&lw[atom_of(l + 2 * kWave)]);
    for (;;) {
      const uint32_t mine = v0 < v1 ? (v0 < v2 ? v0 : v2) : (v1 < v2 ? v1 : v2);
      const uint32_t m = wave_min_u32(mine);
      if (m == kNil) break;
      emit(m);
      n++;
      v0 = v0 == m ? kNil : v0;
      v1 = v1 == m ? kNil : v1;
      v2 = v2 == m ? kNil : v2;
    }
  } else {
    // blocks of side 16 and 32 (depths 4 and 5): each pass re-reads the blocks'
    // last writers and takes the smallest one above the previous
    uint32_t last = 0;
    for (;;) {
      uint32_t mine = kNil;
      for (int it = l; it < items; it += kWave) {
        const uint32_t v = vld(&lw[atom_of(it)]);
        if (v != kNil && (n == 0 || v > last) && v < mine) mine = v;
      }
      const uint32_t m = wave_min_u32(mine);
      if (m == kNil) break;
      emit(m);
      n++;
      last = m;
    }
  }
  wave_order();
  const int na = 1 << lg, bw = nb - 1;
  const int64_t wbase = atom_base(nt, dmax, lvl, br[bw], bc[bw]);
  for (int a0 = 0; a0 < na; a0 += kWave) {
    const int a = a0 + l;
    if (a < na) lw[wbase + ((int64_t)(a >> sh) << dmax) + (a & wmask)] = f;
  }
  wave_order();
  return n;
}

}  // namespace dev
}  // namespace hesp
