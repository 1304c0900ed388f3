// hesp_core.h -- structural expansion of a recursively partitioned tiled
// Cholesky task DAG (HeSP, Rey/Igual/Prieto-Matias, arXiv 1602.05510).
//
// Shared by the host entry point hesp_expand and the gfx950 kernels.
//
// The loop nest of Fig. 1 issues, for every k, chol(k), trsm(k,j) (j>k),
// gemm(k,i,j) (k<i<j) and syrk(k,i) (k<i).  A top-level task is identified by
// its cell (k,i,j) of the iteration space {k <= i <= j}: chol = (k,k,k),
// trsm = (k,k,j), syrk = (k,i,i), gemm = (k,i,j).  Splitting a task d times
// (partition parameter p = 2^-d, section 2.1 "Recursive task partitioners")
// replaces it by the blocked algorithm of its own kind on a 2^d x 2^d
// sub-tiling; those sub-tasks are exactly the fine-grain cells (K,I,J),
// K <= I <= J, of the loop nest at granularity b/2^d that fall inside the
// parent's cell, and the kind of each follows from its indices.
//
// Dependences (section 2.1: RaW, WaR, WaW) are derived structurally instead
// of by scanning data: every block is final before it is first read, so only
// two kinds of predecessor exist --
//   * the previous writer of the written block (the same cell at K-1, or the
//     last K of the previous top-level task that writes the same tile), and
//   * the finalising writer (chol or trsm) of every block the task reads.
// When neighbouring tasks were split to different depths, a coarse block
// covers several fine ones and every covering fine writer is a predecessor.
// Sub-blocks strictly below the diagonal of a diagonal block are skipped:
// whoever wrote them also wrote the diagonal sub-blocks, so those edges are
// implied by the ones kept (the DAG has the same transitive closure as a full
// atom-by-atom hazard scan, hence the same release times and critical times).
//
// Numbering: fine tasks are numbered top-level task by top-level task in
// Fig. 1 order, and inside a top-level task by increasing K, so every edge
// points from a lower to a higher number (the numbering is topological).
#pragma once
#include <stdint.h>

#ifndef HESP_HD
#if defined(__HIPCC__)
#define HESP_HD __host__ __device__ __forceinline__
#else
#define HESP_HD inline
#endif
#endif

namespace hesp {

enum : int { CHOL = 0, TRSM = 1, SYRK = 2, GEMM = 3 };

// fine coordinates are packed into 9 bits each
constexpr int kCoordBits = 9;
constexpr int kMaxFine = 1 << kCoordBits;     // nt * 2^dmax must not exceed this
constexpr int kMaxLevel = 5;                  // split depth 0..5 (b, b/2, ..., b/32)
constexpr int kMaxWaveLevel = 3;              // candidates simulated with 64 lanes: depth 0..3

HESP_HD int64_t tet3(int64_t n) { return n * (n + 1) * (n + 2) / 6; }
HESP_HD int tri2(int n) { return n * (n + 1) / 2; }

HESP_HD int kind_of(int k, int i, int j) {
  return k == i ? (i == j ? CHOL : TRSM) : (i == j ? SYRK : GEMM);
}

// number of fine tasks of a top-level task of kind `kind` split d times
HESP_HD int fine_count(int kind, int d) {
  int s = 1 << d;
  if (kind == CHOL) return s * (s + 1) * (s + 2) / 6;
  if (kind == GEMM) return s * s * s;
  return s * s * (s + 1) / 2;
}

// --- Fig. 1 numbering of top-level tasks --------------------------------------
// iteration k issues 1 + 2m + m(m-1)/2 tasks, m = nt-1-k;  F(M) sums the first M
// of those sizes counted from the last iteration.
HESP_HD int64_t iter_prefix(int64_t M) { return M + M * (M - 1) + M * (M - 1) * (M - 2) / 6; }
HESP_HD int64_t iter_offset(int nt, int k) { return iter_prefix(nt) - iter_prefix(nt - k); }

HESP_HD int64_t top_index(int nt, int k, int i, int j) {
  int64_t base = iter_offset(nt, k);
  int m = nt - 1 - k;
  if (i == k) return base + (j == k ? 0 : 1 + (j - k - 1));
  int q = i - k - 1;                                 // gemm/syrk groups before i
  int64_t gbase = base + 1 + m + (int64_t)q * m - (int64_t)q * (q - 1) / 2;
  return gbase + (i == j ? (nt - 1 - i) : (j - i - 1));
}

// inverse of top_index (k, i, j packed as 10-bit fields)
HESP_HD uint32_t pack_cell(int k, int i, int j) { return (uint32_t)k | ((uint32_t)i << 10) | ((uint32_t)j << 20); }
HESP_HD int cell_k(uint32_t c) { return (int)(c & 1023u); }
HESP_HD int cell_i(uint32_t c) { return (int)((c >> 10) & 1023u); }
HESP_HD int cell_j(uint32_t c) { return (int)((c >> 20) & 1023u); }

HESP_HD uint32_t top_cell(int nt, int64_t t) {
  int lo = 0, hi = nt - 1;                           // last k with iter_offset(k) <= t
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (iter_offset(nt, mid) <= t) lo = mid; else hi = mid - 1;
  }
  int k = lo, m = nt - 1 - k;
  int64_t r = t - iter_offset(nt, k);
  if (r == 0) return pack_cell(k, k, k);
  if (r <= m) return pack_cell(k, k, k + (int)r);
  int64_t r2 = r - 1 - m;
  int q = 0;                                         // group q holds nt-(k+1+q) tasks
  while (r2 >= nt - (k + 1 + q)) { r2 -= nt - (k + 1 + q); q++; }
  int i = k + 1 + q;
  int g = nt - 1 - i;                                // gemms before the syrk
  return r2 < g ? pack_cell(k, i, i + 1 + (int)r2) : pack_cell(k, i, i);
}

// --- numbering inside one top-level task ---------------------------------------
// position of (r,c), r <= c, in the row-major upper triangle of an s x s grid
HESP_HD int utri(int s, int r, int c) { return r * s - r * (r - 1) / 2 + (c - r); }
HESP_HD void utri_inv(int s, int x, int& r, int& c) {
  r = 0;
  while (x >= s - r) { x -= s - r; r++; }
  c = r + x;
}

// (q,r,c) are the fine indices relative to the cell origin (k*s, i*s, j*s)
HESP_HD int local_index(int kind, int s, int q, int r, int c) {
  switch (kind) {
    case GEMM: return (q * s + r) * s + c;
    case SYRK: return q * tri2(s) + utri(s, r, c);
    case TRSM: return utri(s, q, r) * s + c;
    default:   return (int)(tet3(s) - tet3(s - q)) + utri(s - q, r - q, c - q);
  }
}

HESP_HD void local_coords(int kind, int s, int x, int& q, int& r, int& c) {
  switch (kind) {
    case GEMM: c = x % s; r = (x / s) % s; q = x / (s * s); return;
    case SYRK: q = x / tri2(s); utri_inv(s, x % tri2(s), r, c); return;
    case TRSM: c = x % s; utri_inv(s, x / s, q, r); return;
    default: {
      q = 0;
      while (x >= tri2(s - q)) { x -= tri2(s - q); q++; }
      int rr, cc;
      utri_inv(s - q, x, rr, cc);
      r = q + rr; c = q + cc;
      return;
    }
  }
}

// --- packed descriptor of a fine task ------------------------------------------
// kind:2 | level:3 | K:9 | I:9 | J:9  (fine indices at the task's own level)
HESP_HD uint32_t pack_desc(int kind, int level, int K, int I, int J) {
  return (uint32_t)kind | ((uint32_t)level << 2) | ((uint32_t)K << 5) | ((uint32_t)I << 14) |
         ((uint32_t)J << 23);
}
HESP_HD int desc_kind(uint32_t d) { return (int)(d & 3u); }
HESP_HD int desc_level(uint32_t d) { return (int)((d >> 2) & 7u); }
HESP_HD int desc_K(uint32_t d) { return (int)((d >> 5) & 511u); }
HESP_HD int desc_I(uint32_t d) { return (int)((d >> 14) & 511u); }
HESP_HD int desc_J(uint32_t d) { return (int)((d >> 23) & 511u); }

// data blocks of a fine task: reads first, the written block last
HESP_HD int desc_blocks(uint32_t d, int* br, int* bc) {
  int K = desc_K(d), I = desc_I(d), J = desc_J(d);
  switch (desc_kind(d)) {
    case CHOL: br[0] = K; bc[0] = K; return 1;
    case TRSM: br[0] = K; bc[0] = K; br[1] = K; bc[1] = J; return 2;
    case SYRK: br[0] = K; bc[0] = I; br[1] = I; bc[1] = I; return 2;
    default:   br[0] = K; bc[0] = I; br[1] = K; bc[1] = J; br[2] = I; bc[2] = J; return 3;
  }
}

// --- predecessors ------------------------------------------------------------------
// View of one candidate: nt, the split depth of every top-level task and the
// number of the first fine task of every top-level task.
//   depth(t) -> int, first(t) -> int64
// emit(pred_number) is called once per distinct predecessor.
template <class DepthF, class FirstF, class EmitF>
HESP_HD int for_each_pred(int nt, const DepthF& depth, const FirstF& first, int64_t top, uint32_t cell,
                          int d, int K, int I, int J, EmitF&& emit) {
  const int k = cell_k(cell), i = cell_i(cell), j = cell_j(cell);
  const int kind = kind_of(k, i, j);
  const int s = 1 << d;
  const int64_t self = first(top);
  int n = 0;
  // (1) previous writer of the written block (I,J)
  if (K > k * s) {
    emit(self + local_index(kind, s, K - 1 - k * s, I - i * s, J - j * s));
    n++;
  } else if (k > 0) {
    const int64_t tu = top_index(nt, k - 1, i, j);
    const int du = depth(tu), su = 1 << du;
    const int ku = (i == j) ? SYRK : GEMM;
    const int64_t fu = first(tu);
    const int qu = su - 1;                            // last K of that task
    if (du <= d) {
      const int sh = d - du;
      emit(fu + local_index(ku, su, qu, (I >> sh) - i * su, (J >> sh) - j * su));
      n++;
    } else {
      const int sh = du - d, w = 1 << sh;
      for (int u = 0; u < w; u++)
        for (int v = 0; v < w; v++) {
          const int I2 = (I << sh) + u, J2 = (J << sh) + v;
          if (I2 > J2) continue;
          emit(fu + local_index(ku, su, qu, I2 - i * su, J2 - j * su));
          n++;
        }
    }
  }
  // (2) finalising writers of the blocks read: (K,K) for trsm, (K,I) for syrk,
  //     (K,I) and (K,J) for gemm
  int rc[2], nr = 0;
  const int fk = kind_of(K, I, J);                    // kind of the fine task itself
  if (fk == TRSM) { rc[0] = K; nr = 1; }
  else if (fk == SYRK) { rc[0] = I; nr = 1; }
  else if (fk == GEMM) { rc[0] = I; rc[1] = J; nr = 2; }
  int64_t last_coarse = -1;
  for (int x = 0; x < nr; x++) {
    const int R = K, C = rc[x];
    const int tc = C >> d;                            // tile column of the block read
    const int64_t tf = (tc == k) ? top_index(nt, k, k, k) : top_index(nt, k, k, tc);
    const int kf = (tc == k) ? CHOL : TRSM;
    if (tf == top) {                                  // finalised inside this cell
      emit(self + local_index(kind, s, R - k * s, R - i * s, C - j * s));
      n++;
      continue;
    }
    const int dfi = depth(tf), sf = 1 << dfi;
    const int64_t ff = first(tf);
    if (dfi <= d) {
      const int sh = d - dfi;
      const int R2 = R >> sh, C2 = C >> sh;
      const int64_t id = ff + local_index(kf, sf, R2 - k * sf, R2 - k * sf, C2 - tc * sf);
      if (id != last_coarse) { emit(id); n++; }
      last_coarse = id;
    } else {
      const int sh = dfi - d, w = 1 << sh;
      for (int u = 0; u < w; u++)
        for (int v = 0; v < w; v++) {
          const int R2 = (R << sh) + u, C2 = (C << sh) + v;
          if (R2 > C2) continue;
          emit(ff + local_index(kf, sf, R2 - k * sf, R2 - k * sf, C2 - tc * sf));
          n++;
        }
    }
  }
  return n;
}

}  // namespace hesp
