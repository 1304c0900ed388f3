// hesp_sim.hip -- the batched simulation on gfx950: layout, preparation and
// the lane-group event loop.
//
// For a chunk of candidates:
//   k_layout   prefix sums of the exact per-candidate sizes (tasks, edges,
//              finest-block validity words, top-level tasks) over the batch;
//   k_prepare  one wavefront per candidate: expansion of the Fig. 1 loop nest
//              by the candidate's split depths into fine tasks and a successor
//              CSR (section 2.1, "Recursive task partitioners"; RaW/WaW
//              dependences by data block), then critical times (sum of the task
//              time over all processors plus the largest critical time of a
//              successor; "Priority-List", section 2.1);
//   k_sim<G>   persistent: lane groups of G lanes, each running the event
//              simulation of its own candidate -- every task released at the
//              current time is mapped at once, in decreasing critical time (ties:
//              smaller fine indices), to the processor with the earliest finish
//              time counting the transfers it needs (EFT-P, ties: lowest
//              processor index); transfers start at mapping time; on completion
//              the written block becomes valid only in the executing processor's
//              memory space (write-back).  Completions at one instant are all
//              applied before any mapping at that instant.
// Inside a group, lane p < P is processor p; the readiness of a task's blocks
// is read with one lane per (memory space, block, finest block); successors are
// released one per lane.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_core.h"
#include "hesp_device.h"
#include "hesp_internal.h"
#include "hesp_tree.h"

namespace hesp {

namespace {

using namespace dev;

// ---------------------------------------------------------------- layout

// off_X[c] = sum over candidates before c; five columns at once (one workgroup):
// tasks, edges, validity words, top-level tasks and (when off_b is given) the
// bytes of the candidate's region (all its arrays in one block, 16-byte aligned)
// Candidates above a plan's task or edge capacity get no task or edge storage
// (k_prepare marks them HESP_ECAPACITY), so a chunk never needs more than
// (candidates x capacity).
__global__ void __launch_bounds__(1024) k_layout(BatchView b, int32_t n_mem, const int32_t* n_tasks,
                                                 const int64_t* n_edges, int64_t cap_t, int64_t cap_e,
                                                 int64_t* off_t, int64_t* off_e, int64_t* off_v, int64_t* off_top,
                                                 int64_t* off_b) {
  constexpr int Q = 5;
  __shared__ int64_t s_part[Q][16];
  __shared__ int64_t s_carry[Q];
  const int l = lane(), wv = threadIdx.x / kWave;
  if (threadIdx.x < Q) s_carry[threadIdx.x] = 0;
  __syncthreads();
  for (int base = 0; base < b.n_cand; base += 1024) {
    const int c = base + (int)threadIdx.x;
    int64_t x[Q] = {0, 0, 0, 0, 0};
    if (c < b.n_cand) {
      const int nt = b.nt_arr ? b.nt_arr[c] : b.nt;
      const int dmax = b.dmax_arr ? b.dmax_arr[c] : b.dmax;
      const bool ok = nt >= 1 && dmax >= 0 && dmax <= kMaxLevel && (nt << dmax) <= kMaxFine;
      const bool fits = (cap_t <= 0 || n_tasks[c] <= cap_t) && (cap_e <= 0 || n_edges[c] <= cap_e);
      x[0] = fits ? n_tasks[c] : 0;
      x[1] = fits ? n_edges[c] : 0;
      x[2] = ok ? ((int64_t)tri2(nt) << (2 * dmax)) * n_mem : 0;
      x[3] = ok ? tet3(nt) + 1 : 0;
      x[4] = region_bytes(x[0], x[1], x[2], x[3]);
    }
    int64_t incl[Q];
    for (int q = 0; q < Q; q++) {
      int64_t v = x[q];
      for (int o = 1; o < kWave; o <<= 1) {
        const int64_t y = __shfl_up(v, o, kWave);
        if (l >= o) v += y;
      }
      incl[q] = v;
      if (l == kWave - 1) s_part[q][wv] = v;
    }
    __syncthreads();
    for (int q = 0; q < Q; q++) {
      int64_t pre = s_carry[q];
      for (int w = 0; w < wv; w++) pre += s_part[q][w];
      int64_t* off = q == 0 ? off_t : (q == 1 ? off_e : (q == 2 ? off_v : (q == 3 ? off_top : off_b)));
      if (off && c < b.n_cand) off[c + 1] = pre + incl[q];
      if (off && c == 0) off[0] = 0;
    }
    __syncthreads();
    if (threadIdx.x < Q) {
      int64_t s = 0;
      for (int w = 0; w < 16; w++) s += s_part[threadIdx.x][w];
      s_carry[threadIdx.x] += s;
    }
    __syncthreads();
  }
  if (b.n_cand == 0 && threadIdx.x == 0) {
    off_t[0] = 0; off_e[0] = 0; off_v[0] = 0; off_top[0] = 0;
    if (off_b) off_b[0] = 0;
  }
}

// off_X at the chunk boundaries min(i * chunk, n): out[q * (n_chunks + 1) + i]
__global__ void k_bounds(const int64_t* off_t, const int64_t* off_e, const int64_t* off_v, const int64_t* off_top,
                         int32_t n, int32_t chunk, int32_t n_chunks, int64_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_chunks) return;
  const int64_t c = (int64_t)i * chunk < n ? (int64_t)i * chunk : n;
  out[0 * (n_chunks + 1) + i] = off_t[c];
  out[1 * (n_chunks + 1) + i] = off_e[c];
  out[2 * (n_chunks + 1) + i] = off_v[c];
  out[3 * (n_chunks + 1) + i] = off_top[c];
}

// ---------------------------------------------------------------- candidate views

struct CandPtrs {
  int64_t toff;        // first task of the candidate in the chunk's task arrays
  uint32_t* top_first;
  uint32_t* desc;
  uint32_t* indeg;
  uint32_t* cur;
  uint32_t* succ;
  int64_t* rec;        // per task: [critical time, descriptor | first edge << 32], plus one closing entry
  int64_t* fifo;       // per queued task: [finish, id | desc << 32, e0 | e1 << 32] of the task behind it
  uint32_t* ready;
  int64_t* sortbuf;
  int64_t* vf;         // [finest block][memory space] valid-from times
};

__device__ __forceinline__ CandPtrs cand_ptrs(const ChunkView& v, int c) {
  CandPtrs p;
  const int64_t t = v.task_off[c] - v.task_off[v.c0];
  const int64_t e = v.edge_off[c] - v.edge_off[v.c0];
  const int64_t f = v.vf_off[c] - v.vf_off[v.c0];
  const int64_t tp = v.top_off[c] - v.top_off[v.c0];
  p.toff = t;
  if (v.region) {
    // region mode: the candidate's arrays one after the other in its own block,
    // 8-byte elements first
    const int64_t T = v.task_off[c + 1] - v.task_off[c], E = v.edge_off[c + 1] - v.edge_off[c];
    const int64_t V = v.vf_off[c + 1] - v.vf_off[c], TP = v.top_off[c + 1] - v.top_off[c];
    uint8_t* r = v.region + (v.byte_off[c] - v.byte_off[v.c0]);
    p.rec = (int64_t*)r;        r += 16 * (T + 1);
    p.fifo = (int64_t*)r;       r += 24 * T;
    p.sortbuf = (int64_t*)r;    r += 32 * T;
    p.vf = (int64_t*)r;         r += 8 * V;
    p.desc = (uint32_t*)r;      r += 4 * T;
    p.indeg = (uint32_t*)r;     r += 4 * T;
    p.cur = (uint32_t*)r;       r += 4 * T;
    p.ready = (uint32_t*)r;     r += 4 * T;
    p.succ = (uint32_t*)r;      r += 4 * E;
    p.top_first = (uint32_t*)r;
    (void)TP;
    return p;
  }
  p.top_first = v.top_first + tp;
  p.desc = v.desc + t;
  p.indeg = v.indeg + t;
  p.cur = v.cur + t;
  p.succ = v.succ + e;
  p.rec = v.rec + 2 * (t + (c - v.c0));
  p.fifo = v.fifo + 3 * t;
  p.ready = v.ready + t;
  p.sortbuf = v.sortbuf + 4 * t;
  p.vf = v.vf + f;
  return p;
}

// a region-mode candidate whose block ends beyond the region gets no storage
__device__ __forceinline__ bool region_overflow(const ChunkView& v, int c) {
  return v.region && v.byte_off[c + 1] - v.byte_off[v.c0] > v.region_cap;
}

// ---------------------------------------------------------------- preparation, shared steps

// exclusive scan of the successor counts: afterwards cur[f] = first edge of f;
// returns the number of edges
__device__ __forceinline__ int64_t prep_scan_succ(const CandPtrs& sp, int64_t n_fine) {
  const int l = lane();
  int64_t ecarry = 0;
  for (int64_t f0 = 0; f0 < n_fine; f0 += kWave) {
    const int64_t f = f0 + l;
    const int v = f < n_fine ? (int)vld_l2(&sp.cur[f]) : 0;
    const int incl = wave_incl_scan(v);
    if (f < n_fine) sp.cur[f] = (uint32_t)(ecarry + incl - v);
    ecarry += rdl32(incl, kWave - 1);
  }
  wave_order();

  return ecarry;
}

// LDS of the critical-time pass: per task of the current chunk of 64, its critical
// time (rk), the largest critical time among its successors outside the chunk
// (ext), the sweep's running maximum (mx) and its first edge (e, e[64] = the
// chunk's end); the chunk's internal edges as (source << 6 | target), up to
// kPrepIn of them, or fewer when the plan says so (more are re-read from the
// successor lists in each sweep)
constexpr int kPrepIn = 1024;
struct PrepLds {
  int64_t rk[kWave], ext[kWave], mx[kWave];
  uint32_t e[kWave + 1];
  uint16_t in[kPrepIn];
};

// the task of the chunk that owns edge e (E0 <= e < E1): the last t with
// e[t] <= e, the first edges being non-decreasing
__device__ __forceinline__ int prep_owner(const PrepLds& s, uint32_t e) {
  int lo = 0;
  for (int step = kWave / 2; step > 0; step >>= 1)
    if (s.e[lo + step] <= e) lo += step;
  return lo;
}

// critical times, the closing record, initial validity and the first ready
// list; cur[f] = one past the last edge of f, successor lists filled
__device__ __forceinline__ void prep_finish(const ChunkView& cv, const OutView& out, int c, int nt, int dmax, int M,
                                            const CandPtrs& sp, int64_t n_fine, int64_t n_edges,
                                            const int64_t (*s_W)[kLevels], PrepLds& s) {
  const int l = lane();
  const int in_cap = cv.prep_in >= 1 && cv.prep_in <= kPrepIn ? cv.prep_in : kPrepIn;
  // R: critical times, last chunk of 64 tasks first.  The chunk's successor
  // lists form one contiguous edge range, read by all lanes together, four
  // edges per lane per round trip: a successor beyond the chunk is final, and its
  // critical time is gathered and folded into its source's ext with an LDS
  // maximum; one inside the chunk is kept as an internal edge.  The chunk's own
  // values are then iterated over the internal edges to their fixed point
  // (monotone from below).
  const int64_t n_chunks = (n_fine + kWave - 1) / kWave;
  for (int64_t ch = n_chunks - 1; ch >= 0; ch--) {
    const int64_t base = ch * kWave, lim = base + kWave;
    const int64_t f = base + l;
    const bool valid = f < n_fine;
    const int n_valid = (int)(n_fine - base < kWave ? n_fine - base : kWave);
    int64_t w = 0;
    uint32_t e0 = 0, e1 = 0, dsc = 0;
    if (valid) {
      dsc = vld(&sp.desc[f]);
      w = s_W[desc_kind(dsc)][desc_level(dsc)];
      e0 = f == 0 ? 0u : vld_l2(&sp.cur[f - 1]);
      e1 = vld_l2(&sp.cur[f]);
    }
    const uint32_t E0 = (uint32_t)rdl32((int)e0, 0), E1 = (uint32_t)rdl32((int)e1, n_valid - 1);
    s.e[l] = valid ? e0 : E1;
    if (l == 0) s.e[kWave] = E1;
    s.ext[l] = 0;
    __syncthreads();
    int n_in = 0;
    for (uint32_t eb = E0; eb < E1; eb += 4 * kWave) {
      uint32_t v[4];
      int64_t rv[4];
      int src[4];
      for (int q = 0; q < 4; q++) {
        const uint32_t e = eb + q * kWave + l;
        v[q] = e < E1 ? vld(&sp.succ[e]) : kNil;
      }
      for (int q = 0; q < 4; q++) rv[q] = (v[q] != kNil && v[q] >= lim) ? vld(&sp.rec[2 * v[q]]) : 0;
      for (int q = 0; q < 4; q++) src[q] = v[q] != kNil ? prep_owner(s, eb + q * kWave + l) : 0;
      for (int q = 0; q < 4; q++) {
        if (v[q] != kNil && v[q] >= lim) atomicMax((long long*)&s.ext[src[q]], (long long)rv[q]);
        const bool inner = v[q] != kNil && v[q] < lim;
        const uint64_t m = __ballot(inner);
        const int pos = n_in + __popcll(m & lanes_below());
        if (inner && pos < in_cap) s.in[pos] = (uint16_t)((src[q] << 6) | (int)(v[q] - base));
        n_in += __popcll(m);
      }
    }
    __syncthreads();
    const int64_t ext = s.ext[l];
    int64_t r = w + ext;
    for (int sweep = 0; n_in > 0 && sweep < kWave + 2; sweep++) {
      s.rk[l] = r;
      s.mx[l] = ext;
      __syncthreads();
      if (n_in <= in_cap) {
        for (int i = l; i < n_in; i += kWave) {
          const int u = s.in[i];
          atomicMax((long long*)&s.mx[u >> 6], (long long)s.rk[u & 63]);
        }
      } else {
        for (uint32_t e = E0 + l; e < E1; e += kWave) {
          const uint32_t vv = vld(&sp.succ[e]);
          if (vv < lim) atomicMax((long long*)&s.mx[prep_owner(s, e)], (long long)s.rk[vv - base]);
        }
      }
      __syncthreads();
      const int64_t nr = w + s.mx[l];
      const bool changed = valid && nr != r;
      r = nr;
      if (!__ballot(changed)) break;
    }
    if (valid) {
      sp.rec[2 * f] = r;
      sp.rec[2 * f + 1] = (int64_t)(dsc | ((uint64_t)e0 << 32));
    }
    __syncthreads();
  }
  if (l == 0) {
    sp.rec[2 * n_fine] = 0;
    sp.rec[2 * n_fine + 1] = (int64_t)((uint64_t)n_edges << 32);   // end of the last range
  }

  // initial validity: data valid on the host (space 0) only
  {
    const int64_t n_vf = ((int64_t)tri2(nt) << (2 * dmax)) * M;
    const int step = kWave % M;
    int m = l % M;
    for (int64_t e = l; e < n_vf; e += kWave) {
      sp.vf[e] = m == 0 ? 0 : kInf;
      m += step;
      m = m >= M ? m - M : m;
    }
  }
  // tasks without predecessors start the ready list
  int64_t n_src = 0;
  for (int64_t f0 = 0; f0 < n_fine; f0 += kWave) {
    const int64_t f = f0 + l;
    const bool src = f < n_fine && vld(&sp.indeg[f]) == 0u;
    const uint64_t m = __ballot(src);
    if (src) sp.ready[n_src + __popcll(m & lanes_below())] = (uint32_t)f;
    n_src += __popcll(m);
  }
  if (l == 0) {
    cv.nsrc[c - cv.c0] = (int32_t)n_src;
    out.status[c] = kOK;
    if (out.n_tasks) out.n_tasks[c] = (int32_t)n_fine;
  }
}

// ---------------------------------------------------------------- preparation

// eight waves per SIMD (64 VGPRs): the passes wait on memory most of the time
__global__ void __launch_bounds__(kWave, 8) k_prepare(SimTables tb, BatchView bv, ChunkView cv, OutView out) {
  __shared__ int64_t s_W[4][kLevels];
  __shared__ PrepLds s_p;
  const int l = lane();
  for (int x = l; x < 4 * kLevels; x += kWave) (&s_W[0][0])[x] = (&tb.W[0][0])[x];
  __syncthreads();

  const int c = cv.c0 + (int)blockIdx.x;
  if (c >= bv.n_cand) return;
  const Cand cd = load_cand(bv, c);
  const int nt = cd.nt, dmax = cd.dmax, M = tb.n_mem;
  int status = kOK;
  if (nt < 1 || dmax < 0 || dmax > kMaxLevel || dmax > tb.max_level || (nt << dmax) > kMaxFine) status = kEINVAL;
  if (status == kOK && ((cv.cap_tasks > 0 && cv.cnt_tasks[c] > cv.cap_tasks) ||
                        (cv.cap_edges > 0 && cv.cnt_edges[c] > cv.cap_edges) || region_overflow(cv, c)))
    status = kECAP;
  const int64_t n_tasks = cv.task_off[c + 1] - cv.task_off[c];
  const int64_t n_edges = cv.edge_off[c + 1] - cv.edge_off[c];
  const CandPtrs sp = cand_ptrs(cv, c);

  // pass A: first fine task of every top-level task; depths above dmax
  int64_t carry = 0;
  if (status == kOK) {
    bool bad = false;
    for (int t0 = 0; t0 < cd.n_top; t0 += kWave) {
      const int t = t0 + l;
      const bool vt = t < cd.n_top;
      const uint32_t cell = vt ? top_cell(nt, t) : 0u;
      const int d = vt ? (int)cd.depth[t] : 0;
      bad |= vt && d > dmax;
      const int cnt = vt ? fine_count(kind_of(cell_k(cell), cell_i(cell), cell_j(cell)), d > dmax ? dmax : d) : 0;
      const int incl = wave_incl_scan(cnt);
      if (vt) sp.top_first[t] = (uint32_t)(carry + incl - cnt);
      carry += rdl32(incl, kWave - 1);
    }
    if (l == 0) sp.top_first[cd.n_top] = (uint32_t)carry;
    if (__ballot(bad) || carry != n_tasks) status = kEINVAL;
  }
  if (status != kOK) {
    if (l == 0) {
      out.makespan[c] = -1;
      out.status[c] = status;
      if (out.n_tasks) out.n_tasks[c] = 0;
    }
    return;
  }
  const int64_t n_fine = n_tasks;
  for (int64_t f = l; f < n_fine; f += kWave) sp.cur[f] = 0u;
  wave_order();

  auto depth_of = [&](int64_t t) { return (int)cd.depth[t]; };
  auto first_of = [&](int64_t t) { return (int64_t)vld(&sp.top_first[t]); };

  // pass B: descriptors, predecessor counts, successor counts
  for_each_fine(cd, [&](bool valid, int64_t f, int64_t top, uint32_t cell, int d, int K, int I, int J) {
    if (!valid) return;
    sp.desc[f] = pack_desc(kind_of(K, I, J), d, K, I, J);
    const int np = for_each_pred(nt, depth_of, first_of, top, cell, d, K, I, J,
                                 [&](int64_t p) { atomicAdd(&sp.cur[p], 1u); });
    sp.indeg[f] = (uint32_t)np;
  });
  wave_order();

  prep_scan_succ(sp, n_fine);

  // pass D: fill successor lists; afterwards cur[f] = one past the last edge of f
  for_each_fine(cd, [&](bool valid, int64_t f, int64_t top, uint32_t cell, int d, int K, int I, int J) {
    if (!valid) return;
    // the first eight predecessors are collected (predicated register writes),
    // then their slots are claimed together and written together
    uint32_t pl[8];
    int np = 0;
    for_each_pred(nt, depth_of, first_of, top, cell, d, K, I, J, [&](int64_t p) {
      if (np < 8) {
        for (int q = 0; q < 8; q++) pl[q] = q == np ? (uint32_t)p : pl[q];
        np++;
      } else {
        const uint32_t pos = atomicAdd(&sp.cur[p], 1u);
        sp.succ[pos] = (uint32_t)f;
      }
    });
    uint32_t pos[8];
    for (int q = 0; q < 8; q++) pos[q] = q < np ? atomicAdd(&sp.cur[pl[q]], 1u) : 0u;
    for (int q = 0; q < 8; q++)
      if (q < np) sp.succ[pos[q]] = (uint32_t)f;
  });
  wave_order();

  prep_finish(cv, out, c, nt, dmax, M, sp, n_fine, n_edges, s_W, s_p);
}

// ---------------------------------------------------------------- split trees
// (the walk over a candidate's tasks and the last-writer scan: hesp_tree.h)

__device__ __forceinline__ bool tree_shape_ok(int nt, int dmax) {
  return nt >= 1 && dmax >= 0 && dmax <= kMaxLevel && (nt << dmax) <= kMaxFine;
}

// exact task and edge counts of every split-tree candidate
// both split-tree kernels run at eight waves per SIMD: their walks wait on memory
// per task, and the extra waves hide more than the spilled registers cost
__global__ void __launch_bounds__(kWave, 8) k_count_tree(BatchView bv, uint32_t* scratch, int32_t* n_tasks,
                                                      int64_t* n_edges) {
  const int c = blockIdx.x;
  if (c >= bv.n_cand) return;
  const int nt = bv.nt, dmax = bv.dmax, l = lane();
  if (!tree_shape_ok(nt, dmax)) {
    if (l == 0) { n_tasks[c] = 0; n_edges[c] = 0; }
    return;
  }
  const int64_t n_atoms = (int64_t)tri2(nt) << (2 * dmax);
  uint32_t* lw = scratch + (int64_t)c * n_atoms;
  for (int64_t a = l; a < n_atoms; a += kWave) lw[a] = kNil;
  wave_order();
  int64_t tasks = 0, edges = 0;
  walk_tree(nt, dmax, bv.depth + (int64_t)c * bv.tree_stride, [&](int kind, int lv, int K, int I, int J) {
    edges += scan_task(lw, nt, dmax, kind, lv, K, I, J, (uint32_t)tasks, [](uint32_t) {});
    tasks++;
  });
  if (l == 0) {
    n_tasks[c] = (int32_t)tasks;
    n_edges[c] = edges;
  }
}

// preparation of a split-tree candidate: descriptors and predecessor counts from
// the scan, successor offsets, a second scan filling the successor lists, then
// the steps shared with depth candidates (the last-writer table lives in the
// candidate's validity words until they are initialized)
__global__ void __launch_bounds__(kWave, 8) k_prepare_tree(SimTables tb, BatchView bv, ChunkView cv, OutView out) {
  __shared__ int64_t s_W[4][kLevels];
  __shared__ PrepLds s_p;
  const int l = lane();
  for (int x = l; x < 4 * kLevels; x += kWave) (&s_W[0][0])[x] = (&tb.W[0][0])[x];
  __syncthreads();

  const int c = cv.c0 + (int)blockIdx.x;
  if (c >= bv.n_cand) return;
  const int nt = bv.nt, dmax = bv.dmax, M = tb.n_mem;
  int status = kOK;
  if (!tree_shape_ok(nt, dmax) || dmax > tb.max_level) status = kEINVAL;
  if (status == kOK && ((cv.cap_tasks > 0 && cv.cnt_tasks[c] > cv.cap_tasks) ||
                        (cv.cap_edges > 0 && cv.cnt_edges[c] > cv.cap_edges) || region_overflow(cv, c)))
    status = kECAP;
  const uint8_t* flags = bv.depth + (int64_t)c * bv.tree_stride;
  if (status == kOK) {
    bool bad = false;
    const int64_t nf = tree_level_off(nt, dmax);
    for (int64_t x = l; x < nf; x += kWave) bad |= flags[x] > 1;
    if (__ballot(bad)) status = kEINVAL;
  }
  const int64_t n_fine = cv.task_off[c + 1] - cv.task_off[c];
  const int64_t n_edges = cv.edge_off[c + 1] - cv.edge_off[c];
  if (status != kOK) {
    if (l == 0) {
      out.makespan[c] = -1;
      out.status[c] = status;
      if (out.n_tasks) out.n_tasks[c] = 0;
    }
    return;
  }
  const CandPtrs sp = cand_ptrs(cv, c);
  const int64_t n_atoms = (int64_t)tri2(nt) << (2 * dmax);
  uint32_t* lw = reinterpret_cast<uint32_t*>(sp.vf);
  for (int64_t a = l; a < n_atoms; a += kWave) lw[a] = kNil;
  for (int64_t f = l; f < n_fine; f += kWave) sp.cur[f] = 0u;
  wave_order();

  // descriptors, predecessor counts, successor counts
  uint32_t nf_seen = 0;
  // A task's distinct last writers (at most 3 x 64: one per finest block it
  // reads) are dealt to the lanes as they are found, lane j holding writers j,
  // j + 64 and j + 128; their successor counters are then updated by all lanes
  // together instead of one writer at a time.
  walk_tree(nt, dmax, flags, [&](int kind, int lv, int K, int I, int J) {
    const uint32_t f = nf_seen++;
    uint32_t wr[3] = {kNil, kNil, kNil};
    int k = 0;
    const int np = scan_task(lw, nt, dmax, kind, lv, K, I, J, f, [&](uint32_t p) {
      for (int h = 0; h < 3; h++) wr[h] = k == l + h * kWave ? p : wr[h];
      k++;
    });
    for (int h = 0; h < 3; h++)
      if (wr[h] != kNil) atomicAdd(&sp.cur[wr[h]], 1u);
    if (l == 0 && f < n_fine) {            // the counts came from the same walk: always true
      sp.desc[f] = pack_desc(kind, lv, K, I, J);
      sp.indeg[f] = (uint32_t)np;
    }
  });
  wave_order();
  prep_scan_succ(sp, n_fine);

  // successor lists; afterwards cur[f] = one past the last edge of f
  for (int64_t a = l; a < n_atoms; a += kWave) lw[a] = kNil;
  wave_order();
  nf_seen = 0;
  walk_tree(nt, dmax, flags, [&](int kind, int lv, int K, int I, int J) {
    const uint32_t f = nf_seen++;
    uint32_t wr[3] = {kNil, kNil, kNil};
    int k = 0;
    scan_task(lw, nt, dmax, kind, lv, K, I, J, f, [&](uint32_t p) {
      for (int h = 0; h < 3; h++) wr[h] = k == l + h * kWave ? p : wr[h];
      k++;
    });
    uint32_t pos[3];
    for (int h = 0; h < 3; h++) pos[h] = wr[h] != kNil ? atomicAdd(&sp.cur[wr[h]], 1u) : 0u;
    for (int h = 0; h < 3; h++)
      if (wr[h] != kNil && pos[h] < n_edges) sp.succ[pos[h]] = f;
  });
  wave_order();
  prep_finish(cv, out, c, nt, dmax, M, sp, n_fine, n_edges, s_W, s_p);
}

// ---------------------------------------------------------------- event simulation

// SplitMix64 (Steele, Lea, Flood 2014): value idx+1 of the stream of purpose 8
// (random processor choices) of `seed`
__device__ __forceinline__ uint64_t choice_draw(uint64_t seed, uint64_t idx) {
  auto mix = [](uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const uint64_t g = 0x9E3779B97F4A7C15ull;
  return mix(mix(seed + g * 9ull) + g * (idx + 1));
}

// Instantiated per policy class so that the default policy carries no policy
// code: R-P / F-P map tasks only onto idle processors and may make them wait.
// The whole-wave variant is limited to 72 VGPRs, seven waves per SIMD: the event
// loop waits on memory between short bursts of issue, and a seventh wave hides
// more of it than the few spilled registers cost (-15% per launch measured); the
// 16- and 32-lane variants lose when squeezed and keep their registers.
template <int G, int POL>
__global__ void __launch_bounds__(kWave, G == 64 ? 7 : 1) k_sim(SimTables tb, BatchView bv, ChunkView cv, OutView out,
                                               uint32_t* counter) {
  // POL 0: Priority-List + EFT-P + write-back (no policy flags read); 1: the
  // other push policies (FCFS, EIT-P) and caching policies; 2: R-P / F-P
  constexpr bool PULL = POL == 2;
  const bool fcfs = POL != 0 && tb.fcfs;
  const int sel = POL == 0 ? 0 : tb.sel;
  const int cache = POL == 0 ? 0 : tb.cache;
  const bool bus = POL != 0 && tb.bus != 0;
  constexpr int NG = kWave / G;
  constexpr int LGG = G == 16 ? 4 : (G == 32 ? 5 : 6);
  __shared__ int64_t s_cost[kMaxPtypes][4][kLevels];
  __shared__ int64_t s_xfer[kXferLen];
  __shared__ int64_t s_fin[NG][4][kMaxMem];    // per (block, space): latest finite valid-from
  __shared__ int32_t s_miss[NG][4][kMaxMem];   // per (block, space): finest blocks missing
  // write-around: per (block, space), the latest host valid-from of the missing
  // finest blocks (their transfer cannot leave before)
  __shared__ int64_t s_src[POL == 0 ? 1 : NG][4][kMaxMem];
  __shared__ uint32_t s_rid[NG][G];            // ready list, first G entries, with records
  __shared__ int64_t s_rrank[NG][G];
  __shared__ uint32_t s_rdesc[NG][G];
  __shared__ uint32_t s_re0[NG][G];
  __shared__ uint32_t s_re1[NG][G];
  __shared__ uint8_t s_order[NG][G];

  const Grp<G> gp;
  const int l = gp.l, g = gp.g, gl = gp.gl;
  for (int x = l; x < kMaxPtypes * 4 * kLevels; x += kWave) (&s_cost[0][0][0])[x] = (&tb.cost[0][0][0])[x];
  for (int x = l; x < kXferLen; x += kWave) s_xfer[x] = tb.xfer[x];
  __syncthreads();

  const int P = tb.n_procs, M = tb.n_mem;
  const bool p16 = P <= 16;                    // processor lanes all in the group's first row
  const int pmem = gl < P ? tb.proc_mem[gl] : 0;
  const int ptype = gl < P ? tb.proc_type[gl] : 0;
  const bool want_sched = out.sched_off != nullptr;

  bool active = false, exhausted = false;
  int c = 0, nt = 0, dmax = 0;
  int64_t xs = 0, T = 0, n_ready = 0, sbase = 0;
  CandPtrs sp{};
  int64_t avail = 0, hfin = kInf;
  int64_t bus_free = 0;                       // shared interconnect: free from this time
  uint32_t hid = kNil, hdesc = 0, he0 = 0, he1 = 0, tail = kNil;

  auto push = [&](int64_t pos, uint32_t v, int64_t r0, int64_t r1, int64_t r3) {
    if (pos < G) {
      s_rid[g][pos] = v;
      s_rrank[g][pos] = r0;
      s_rdesc[g][pos] = (uint32_t)r1;
      s_re0[g][pos] = (uint32_t)((uint64_t)r1 >> 32);
      s_re1[g][pos] = (uint32_t)((uint64_t)r3 >> 32);
    } else {
      sp.ready[pos] = v;
    }
  };

  for (;;) {
    // groups without a candidate take the next one
    if (!active && !exhausted) {
      int cc = 0;
      if (gl == 0) cc = (int)atomicAdd(counter, 1u);
      cc = gp.bcast(cc, 0);
      if (cc >= cv.nc) {
        exhausted = true;
      } else {
        c = cv.c0 + (cv.order ? (int)cv.order[cc] : cc);
        if (out.status[c] == kOK) {
          const Cand cd = load_cand(bv, c);
          nt = cd.nt;
          dmax = cd.dmax;
          xs = (int64_t)1 << (2 * (tb.max_level - dmax));
          sp = cand_ptrs(cv, c);
          sbase = want_sched ? out.sched_off[c] : 0;
          T = 0;
          avail = 0;
          bus_free = 0;
          hfin = kInf;
          hid = kNil;
          tail = kNil;
          n_ready = cv.nsrc[c - cv.c0];
          // FCFS keeps minus the release time in the rank slot (sources: 0)
          for (int64_t x = gl; x < (fcfs || n_ready < G ? n_ready : G); x += G) {
            const uint32_t v = vld(&sp.ready[x]);
            if (fcfs) sp.rec[2 * v] = 0;
            if (x < G) push(x, v, fcfs ? 0 : vld(&sp.rec[2 * v]), vld(&sp.rec[2 * v + 1]), vld(&sp.rec[2 * v + 3]));
          }
          active = true;
        }
      }
    }
    if (__ballot(!exhausted) == 0) break;
    if (!active) continue;
    wave_order();

    // (i) map every released task, in priority order
    if (n_ready > 0) {
      const bool small = n_ready <= G;
      if (n_ready == 1) {
        if (gl == 0) s_order[g][0] = 0;
      } else if (small) {
        // position of each entry: decreasing critical time, then increasing key
        const bool v = gl < n_ready;
        const int64_t rk = v ? s_rrank[g][gl] : INT64_MIN;
        const uint32_t ky = v ? task_key(s_rdesc[g][gl], dmax) : 0u;
        int pos = 0;
        for (int j = 0; j < (int)n_ready; j++) {
          const int64_t rj = gp.bcast64(rk, j);
          const uint32_t kj = (uint32_t)gp.bcast((int)ky, j);
          pos += (rj > rk || (rj == rk && kj < ky)) ? 1 : 0;
        }
        if (v) s_order[g][pos] = (uint8_t)gl;
      } else {
        // bitonic sort of (critical time, key|id) pairs in the candidate's buffer
        int64_t n2 = 1;
        while (n2 < n_ready) n2 <<= 1;
        for (int64_t x = gl; x < n2; x += G) {
          if (x < n_ready) {
            uint32_t id, dsc;
            int64_t rk;
            if (x < G) {
              id = s_rid[g][x];
              rk = s_rrank[g][x];
              dsc = s_rdesc[g][x];
            } else {
              id = vld(&sp.ready[x]);
              rk = vld(&sp.rec[2 * id]);
              dsc = (uint32_t)vld(&sp.rec[2 * id + 1]);
            }
            sp.sortbuf[2 * x] = rk;
            sp.sortbuf[2 * x + 1] = ((int64_t)task_key(dsc, dmax) << 32) | id;
          } else {
            sp.sortbuf[2 * x] = INT64_MIN;
            sp.sortbuf[2 * x + 1] = INT64_MAX;
          }
        }
        wave_order();
        // R-P / F-P map at most one task per idle processor now: the entries are
        // selected one at a time below instead of sorted
        for (int64_t k2 = 2; k2 <= (PULL ? 1 : n2); k2 <<= 1) {
          for (int64_t j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
            for (int64_t x = gl; x < n2; x += G) {
              const int64_t y = x ^ j2;
              if (y > x) {
                const int64_t ra = vld(&sp.sortbuf[2 * x]), ka = vld(&sp.sortbuf[2 * x + 1]);
                const int64_t rb = vld(&sp.sortbuf[2 * y]), kb = vld(&sp.sortbuf[2 * y + 1]);
                // "a before b": larger rank, then smaller key
                const bool a_first = ra > rb || (ra == rb && ka < kb);
                const bool up = (x & k2) == 0;
                if (up != a_first) {
                  sp.sortbuf[2 * x] = rb;
                  sp.sortbuf[2 * x + 1] = kb;
                  sp.sortbuf[2 * y] = ra;
                  sp.sortbuf[2 * y + 1] = ka;
                }
              }
            }
            wave_order();
          }
        }
      }
      wave_order();
      int64_t r_stop = n_ready;
      for (int64_t r = 0; r < n_ready; r++) {
        // R-P / F-P map onto processors idle now; without one the rest wait
        uint64_t idle = 0;
        if (PULL) {
          idle = gp.ballot(gl < P && avail <= T);
          if (idle == 0) {
            r_stop = r;
            break;
          }
        }
        uint32_t t, dsc, e0, e1;
        if (small) {
          const int q = gp.uni(s_order[g][r]);
          t = s_rid[g][q];
          dsc = s_rdesc[g][q];
          e0 = s_re0[g][q];
          e1 = s_re1[g][q];
        } else {
          if (PULL) {
            // best remaining entry: largest rank, then smallest key; taken entries
            // have their key set to INT64_MAX
            int64_t br = INT64_MIN, bk = INT64_MAX;
            int bp = -1;
            for (int x = gl; x < n_ready; x += G) {
              const int64_t ra = vld(&sp.sortbuf[2 * x]), ka = vld(&sp.sortbuf[2 * x + 1]);
              if (ka != INT64_MAX && (bp < 0 || ra > br || (ra == br && ka < bk))) {
                br = ra;
                bk = ka;
                bp = x;
              }
            }
            const int64_t rbest = ~gp.min64all(bp >= 0 ? ~br : kInf);   // ~ reverses the order exactly
            const int64_t kbest = gp.min64all(bp >= 0 && br == rbest ? bk : kInf);
            const int owner = __ffsll((unsigned long long)gp.ballot(bp >= 0 && br == rbest && bk == kbest)) - 1;
            const int pos = gp.bcast(bp, owner);
            if (gl == owner) sp.sortbuf[2 * pos + 1] = INT64_MAX;
            t = (uint32_t)(kbest & 0xFFFFFFFFll);
          } else {
            t = (uint32_t)(vld(&sp.sortbuf[2 * r + 1]) & 0xFFFFFFFFll);
          }
          const int64_t r1 = vld(&sp.rec[2 * t + 1]);
          dsc = (uint32_t)r1;
          e0 = (uint32_t)((uint64_t)r1 >> 32);
          e1 = (uint32_t)((uint64_t)vld(&sp.rec[2 * t + 3]) >> 32);
        }
        t = (uint32_t)gp.uni((int)t);
        dsc = (uint32_t)gp.uni((int)dsc);
        e0 = (uint32_t)gp.uni((int)e0);
        e1 = (uint32_t)gp.uni((int)e1);
        const int kind = desc_kind(dsc), lvl = desc_level(dsc);
        const int sh = dmax - lvl;                 // a block is 2^sh x 2^sh finest blocks
        const int lg = 2 * sh;
        const int lgs = lg < LGG ? lg : LGG;      // lanes per segment chunk: 2^lgs
        const int wmask = (1 << sh) - 1;
        int br[3], bc[3];
        const int nb = desc_blocks(dsc, br, bc);
        // validity-table indices fit in 32 bits: at most 512 x 513 / 2 finest
        // blocks (nt * 2^dmax <= 512) times at most 16 memory spaces
        const int ab0 = (int)atom_base(nt, dmax, lvl, br[0], bc[0]);
        const int ab1 = nb > 1 ? (int)atom_base(nt, dmax, lvl, br[1], bc[1]) : 0;
        const int ab2 = nb > 2 ? (int)atom_base(nt, dmax, lvl, br[2], bc[2]) : 0;
        for (int x = gl; x < 4 * M; x += G) {
          (&s_fin[g][0][0])[(x >> 2) + (x & 3) * kMaxMem] = INT64_MIN;
          (&s_miss[g][0][0])[(x >> 2) + (x & 3) * kMaxMem] = 0;
          if (POL != 0) (&s_src[POL == 0 ? 0 : g][0][0])[(x >> 2) + (x & 3) * kMaxMem] = INT64_MIN;
        }
        wave_order();
        // one lane per (space m, block b, finest block a): it = ((m*4 + b) << lg) | a
        const int items = (M << 2) << lg;
        const bool one_pass = items <= G;
        int64_t my_x = 0;
        int my_addr = -1;
        int my_m = 0, my_b = 0;
        for (int i0 = 0; i0 < items; i0 += G) {
          const int it = i0 + gl;
          const int a = it & ((1 << lg) - 1);
          const int b = (it >> lg) & 3;
          const int m = it >> (lg + 2);
          const bool act = it < items && b < nb;
          const int abase = b == 0 ? ab0 : (b == 1 ? ab1 : ab2);
          const int addr = (abase + ((a >> sh) << dmax) + (a & wmask)) * M + m;
          const int64_t x = act ? vld(&sp.vf[addr]) : kInf;
          const uint64_t infm = gp.ballot(act && x == kInf);
          const int64_t fin = seg_max64((act && x != kInf) ? x : INT64_MIN, lgs);
          int64_t src = INT64_MIN;
          if (POL != 0 && cache == 2) {
            // write-around keeps a valid (possibly future) copy of every block on
            // the host, and no other copy is valid earlier
            const int64_t h = (act && x == kInf) ? vld(&sp.vf[addr - m]) : INT64_MIN;
            src = seg_max64(h, lgs);
          }
          if (act && (a & ((1 << lgs) - 1)) == (1 << lgs) - 1) {   // last lane of its segment chunk
            const uint64_t segm = lgs == 6 ? ~0ull : (((1ull << (1 << lgs)) - 1ull) << (gl + 1 - (1 << lgs)));
            s_fin[g][b][m] = max64(s_fin[g][b][m], fin);
            s_miss[g][b][m] += __popcll(infm & segm);
            if (POL != 0 && cache == 2) s_src[POL == 0 ? 0 : g][b][m] = max64(s_src[POL == 0 ? 0 : g][b][m], src);
          }
          if (one_pass) {
            my_x = x;
            my_addr = act ? addr : -1;
            my_m = m;
            my_b = b;
          }
        }
        wave_order();
        int64_t est = T > avail ? T : avail;
        if (gl < P) {
          int64_t lb = bus_free;                    // with a shared interconnect: the blocks in order
          for (int b = 0; b < nb; b++) {
            const int ms = s_miss[g][b][pmem];
            int64_t rdy = s_fin[g][b][pmem];
            int64_t go = T;
            if (POL != 0 && cache == 2) go = max64(T, s_src[POL == 0 ? 0 : g][b][pmem]);
            if (ms > 0) {
              if (bus) go = max64(go, lb);
              const int64_t arr = go + s_xfer[ms * xs];
              if (bus) lb = arr;
              rdy = max64(rdy, arr);
            }
            est = max64(est, rdy);
          }
        }
        const int64_t eft = est + s_cost[ptype][kind][lvl];
        int pstar;
        int64_t eft_star;
        if (PULL && sel == 2) {
          // R-P: the u-th idle processor in index order
          const int u = (int)(choice_draw(tb.seed, task_key(dsc, dmax)) % (uint64_t)__popcll(idle));
          const bool mine = ((idle >> gl) & 1ull) && __popcll(idle & gp.below()) == u;
          pstar = __ffsll((unsigned long long)gp.ballot(mine)) - 1;
          eft_star = gp.bcast64(eft, pstar);
        } else {
          // EFT-P: earliest finish; EIT-P: earliest idle time (an idle processor
          // from now); F-P: smallest task time among the idle processors
          int64_t score = eft;
          if (sel == 1) score = T > avail ? T : avail;
          if (PULL && sel == 3) score = ((idle >> gl) & 1ull) ? s_cost[ptype][kind][lvl] : (kInf >> 6);
          const int64_t key = gl < P ? ((score << 6) | gl) : kInf;
          const int64_t best = gp.min64lo(key, p16);
          pstar = (int)(best & 63);
          eft_star = sel == 0 ? best >> 6 : gp.bcast64(eft, pstar);
        }
        const int64_t est_star = gp.bcast64(est, pstar);
        const int mstar = gp.bcast(pmem, pstar);
        // transfers of the missing finest blocks start now
        auto leave = [&](int b) {   // when the transfer of block b's missing finest blocks can start
          return (POL != 0 && cache == 2) ? max64(T, s_src[POL == 0 ? 0 : g][b][mstar]) : T;
        };
        // arrival of each block's transfer (in block order on a shared interconnect)
        int64_t arr0 = 0, arr1 = 0, arr2 = 0;
        if constexpr (POL != 0) {
          int64_t lb = bus_free;
          for (int b = 0; b < nb; b++) {
            const int miss = s_miss[g][b][mstar];
            if (miss == 0) continue;
            int64_t go = leave(b);
            if (bus) go = max64(go, lb);
            const int64_t a = go + s_xfer[miss * xs];
            if (bus) lb = a;
            if (b == 0) arr0 = a;
            else if (b == 1) arr1 = a;
            else arr2 = a;
          }
          if (bus) bus_free = lb;
        }
        auto arrival = [&](int b) {
          if constexpr (POL == 0) return leave(b) + s_xfer[s_miss[g][b][mstar] * xs];
          return b == 0 ? arr0 : (b == 1 ? arr1 : arr2);
        };
        if (one_pass) {
          if (my_addr >= 0 && my_m == mstar && my_x == kInf) sp.vf[my_addr] = arrival(my_b);
        } else {
          for (int b = 0; b < nb; b++) {
            const int miss = s_miss[g][b][mstar];
            if (miss == 0) continue;
            const int64_t arrive = arrival(b);
            const int abase = b == 0 ? ab0 : (b == 1 ? ab1 : ab2);
            for (int a0 = 0; a0 < (1 << lg); a0 += G) {
              const int a = a0 + gl;
              if (a < (1 << lg)) {
                const int addr = (abase + ((a >> sh) << dmax) + (a & wmask)) * M + mstar;
                if (vld(&sp.vf[addr]) == kInf) sp.vf[addr] = arrive;
              }
            }
          }
        }
        // append to the chosen processor's queue
        if (gl == pstar) {
          avail = eft_star;
          if (hid == kNil) {
            hid = t;
            hfin = eft_star;
            hdesc = dsc;
            he0 = e0;
            he1 = e1;
          } else {
            sp.fifo[3 * tail] = eft_star;
            sp.fifo[3 * tail + 1] = (int64_t)(t | ((uint64_t)dsc << 32));
            sp.fifo[3 * tail + 2] = (int64_t)(e0 | ((uint64_t)e1 << 32));
          }
          tail = t;
        }
        if (want_sched && gl == 0) {
          out.proc[sbase + t] = pstar;
          out.start[sbase + t] = est_star;
          out.finish[sbase + t] = eft_star;
        }
        wave_order();
      }
      if (PULL && r_stop < n_ready) {
        // the tasks that found no idle processor stay released, in front
        const int rem = (int)(n_ready - r_stop);
        if (small) {
          uint32_t id = 0, d1 = 0, a0 = 0, a1 = 0;
          int64_t rk = 0;
          if (gl < rem) {
            const int q = s_order[g][r_stop + gl];
            id = s_rid[g][q];
            rk = s_rrank[g][q];
            d1 = s_rdesc[g][q];
            a0 = s_re0[g][q];
            a1 = s_re1[g][q];
          }
          wave_order();
          if (gl < rem) {
            s_rid[g][gl] = id;
            s_rrank[g][gl] = rk;
            s_rdesc[g][gl] = d1;
            s_re0[g][gl] = a0;
            s_re1[g][gl] = a1;
          }
        } else {
          // entries not taken by the selection, in buffer order (the next round
          // orders them again)
          int kept = 0;
          for (int x0 = 0; x0 < n_ready; x0 += G) {
            const int x = x0 + gl;
            int64_t ka = INT64_MAX;
            if (x < n_ready) ka = vld(&sp.sortbuf[2 * x + 1]);
            const bool keep = ka != INT64_MAX;
            const uint64_t km = gp.ballot(keep);
            const int at = kept + __popcll(km & gp.below());
            if (keep) {
              const uint32_t id = (uint32_t)(ka & 0xFFFFFFFFll);
              if (at < G) push(at, id, vld(&sp.rec[2 * id]), vld(&sp.rec[2 * id + 1]), vld(&sp.rec[2 * id + 3]));
              else sp.ready[at] = id;
            }
            kept += __popcll(km);
          }
        }
        n_ready = rem;
      } else {
        n_ready = 0;
      }
      wave_order();
    }

    // (ii) next event: the earliest queue head
    const int64_t Tn = gp.min64lo(gl < P ? hfin : kInf, p16);
    if (Tn == kInf) {
      if (gl == 0) out.makespan[c] = T;
      active = false;
      continue;
    }

    // (iii) completions at Tn; the next queue entries are fetched first
    const uint64_t cm = gp.ballot(gl < P && hfin == Tn);
    const bool adv = (cm >> gl) & 1ull;
    const bool has_next = adv && hid != tail;
    int64_t nf = kInf, nid = 0, ne = 0;
    if (has_next) {
      nf = vld(&sp.fifo[3 * hid]);
      nid = vld(&sp.fifo[3 * hid + 1]);
      ne = vld(&sp.fifo[3 * hid + 2]);
    }
    uint64_t rem = cm;
    while (rem) {
      const int p = __ffsll((unsigned long long)rem) - 1;
      rem &= rem - 1;
      const int ms = gp.bcast(pmem, p);
      const uint32_t dsc = (uint32_t)gp.bcast((int)hdesc, p);
      const uint32_t e0 = (uint32_t)gp.bcast((int)he0, p);
      const uint32_t e1 = (uint32_t)gp.bcast((int)he1, p);
      const int lvl = desc_level(dsc);
      const int sh = dmax - lvl, lg = 2 * sh, wmask = (1 << sh) - 1;
      int br[3], bc[3];
      const int nb = desc_blocks(dsc, br, bc);
      // write-back: the written block is valid only where it was computed;
      // write-through: also on the host, once the copy sent now has arrived;
      // write-around: on the host only, once that copy has arrived
      const int abase = (int)atom_base(nt, dmax, lvl, br[nb - 1], bc[nb - 1]);
      const int items = M << lg;
      int64_t host_at = (POL != 0 && cache != 0 && ms != 0) ? Tn + s_xfer[(1 << lg) * xs] : Tn;
      if (bus && cache != 0 && ms != 0) {         // the host copy queues on the interconnect
        host_at = max64(Tn, bus_free) + s_xfer[(1 << lg) * xs];
        bus_free = host_at;
      }
      for (int i0 = 0; i0 < items; i0 += G) {
        const int it = i0 + gl;
        if (it < items) {
          const int m = it >> lg, a = it & ((1 << lg) - 1);
          const int atom = abase + ((a >> sh) << dmax) + (a & wmask);
          int64_t x = (m == ms) ? Tn : kInf;
          if (POL != 0 && cache == 1) x = (m == ms) ? Tn : (m == 0 ? host_at : kInf);
          if (POL != 0 && cache == 2) x = (m == 0) ? host_at : kInf;
          sp.vf[atom * M + m] = x;
        }
      }
      // release successors (their records are fetched alongside the decrement)
      for (uint32_t e = e0; e < e1; e += G) {
        const uint32_t ee = e + gl;
        bool rel = false;
        uint32_t v = 0;
        int64_t r0 = 0, r1 = 0, r3 = 0;
        if (ee < e1) {
          v = vld(&sp.succ[ee]);
          r0 = vld(&sp.rec[2 * v]);
          r1 = vld(&sp.rec[2 * v + 1]);
          r3 = vld(&sp.rec[2 * v + 3]);
          rel = atomicSub(&sp.indeg[v], 1u) == 1u;
          if (fcfs) {
            r0 = -Tn;
            if (rel) sp.rec[2 * v] = -Tn;
          }
        }
        const uint64_t rm = gp.ballot(rel);
        if (rel) push(n_ready + __popcll(rm & gp.below()), v, r0, r1, r3);
        n_ready += __popcll(rm);
      }
    }
    if (adv) {
      if (has_next) {
        hid = (uint32_t)nid;
        hdesc = (uint32_t)((uint64_t)nid >> 32);
        hfin = nf;
        he0 = (uint32_t)ne;
        he1 = (uint32_t)((uint64_t)ne >> 32);
      } else {
        hid = kNil;
        hfin = kInf;
        tail = kNil;
      }
    }
    wave_order();
    T = Tn;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_layout(const BatchView& b, int32_t n_mem, const int32_t* n_tasks, const int64_t* n_edges,
                         int64_t cap_t, int64_t cap_e, int64_t* off_t, int64_t* off_e, int64_t* off_v,
                         int64_t* off_top, int64_t* off_b, hipStream_t s) {
  hipLaunchKernelGGL(k_layout, dim3(1), dim3(1024), 0, s, b, n_mem, n_tasks, n_edges, cap_t, cap_e, off_t, off_e,
                     off_v, off_top, off_b);
  return hipGetLastError();
}

hipError_t launch_bounds(const int64_t* off_t, const int64_t* off_e, const int64_t* off_v, const int64_t* off_top,
                         int32_t n, int32_t chunk, int32_t n_chunks, int64_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bounds, dim3((n_chunks + 1 + 255) / 256), dim3(256), 0, s, off_t, off_e, off_v, off_top, n,
                     chunk, n_chunks, out);
  return hipGetLastError();
}

hipError_t launch_prepare(const SimTables& t, const BatchView& b, const ChunkView& v, const OutView& o,
                          hipStream_t s) {
  if (v.nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prepare, dim3(v.nc), dim3(kWave), 0, s, t, b, v, o);
  return hipGetLastError();
}

hipError_t launch_count_tree(const BatchView& b, uint32_t* scratch, int32_t* n_tasks, int64_t* n_edges,
                             hipStream_t s) {
  if (b.n_cand <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count_tree, dim3(b.n_cand), dim3(kWave), 0, s, b, scratch, n_tasks, n_edges);
  return hipGetLastError();
}

hipError_t launch_prepare_tree(const SimTables& t, const BatchView& b, const ChunkView& v, const OutView& o,
                               hipStream_t s) {
  if (v.nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prepare_tree, dim3(v.nc), dim3(kWave), 0, s, t, b, v, o);
  return hipGetLastError();
}

hipError_t launch_sim(const SimTables& t, const BatchView& b, const ChunkView& v, const OutView& o, int32_t slots,
                      int32_t group, uint32_t* counter, hipStream_t s) {
  if (v.nc <= 0) return hipSuccess;
  if ((group != 16 && group != 32 && group != 64) || group < t.n_procs) return hipErrorInvalidValue;
  hipError_t e = launch_zero_u32(counter, s);
  if (e != hipSuccess) return e;
  const int G = group;
  const int per_wave = kWave / G;
  int waves = (v.nc + per_wave - 1) / per_wave;
  if (waves > slots) waves = slots;
  const int pol = t.sel >= 2 ? 2 : (t.sel == 1 || t.fcfs || t.cache != 0 || t.bus != 0 ? 1 : 0);
  const dim3 grid(waves), block(kWave);
#define HESP_SIM_LAUNCH(GG, PP) hipLaunchKernelGGL((k_sim<GG, PP>), grid, block, 0, s, t, b, v, o, counter)
  if (G == 16) {
    if (pol == 0) HESP_SIM_LAUNCH(16, 0);
    else if (pol == 1) HESP_SIM_LAUNCH(16, 1);
    else HESP_SIM_LAUNCH(16, 2);
  } else if (G == 32) {
    if (pol == 0) HESP_SIM_LAUNCH(32, 0);
    else if (pol == 1) HESP_SIM_LAUNCH(32, 1);
    else HESP_SIM_LAUNCH(32, 2);
  } else {
    if (pol == 0) HESP_SIM_LAUNCH(64, 0);
    else if (pol == 1) HESP_SIM_LAUNCH(64, 1);
    else HESP_SIM_LAUNCH(64, 2);
  }
#undef HESP_SIM_LAUNCH
  return hipGetLastError();
}

}  // namespace hesp
