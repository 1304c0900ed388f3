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

#include <type_traits>

#include "hesp_core.h"
#include "hesp_device.h"
#include "hesp_internal.h"
#include "hesp_tree.h"

namespace hesp {

namespace {

using namespace dev;

// ---------------------------------------------------------------- layout

// The five columns of candidate c: tasks, edges, validity words, top-level
// tasks and the bytes of its region (all its arrays in one block, 16-byte
// aligned).  Candidates above a plan's task or edge capacity get no task or edge
// storage (k_prepare marks them HESP_ECAPACITY), so a chunk never needs more than
// (candidates x capacity).
constexpr int kLayoutCols = 5;
__device__ __forceinline__ void layout_cols(const BatchView& b, int32_t n_mem, const int32_t* n_tasks,
                                            const int64_t* n_edges, int64_t cap_t, int64_t cap_e, int c,
                                            int64_t (&x)[kLayoutCols]) {
  for (int q = 0; q < kLayoutCols; q++) x[q] = 0;
  if (c >= b.n_cand) return;
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

// inclusive sums of the five columns over the 1,024 candidates of a workgroup
// (16 wavefronts: shuffles inside each, then the wavefront totals in s_part);
// returns, per column, the workgroup's total
__device__ __forceinline__ void layout_block_scan(int64_t (&x)[kLayoutCols], int64_t (*s_part)[16],
                                                  int64_t (&total)[kLayoutCols]) {
  const int l = lane(), wv = threadIdx.x / kWave;
  int64_t incl[kLayoutCols];
  for (int q = 0; q < kLayoutCols; q++) {
    int64_t v = x[q];
    for (int o = 1; o < kWave; o <<= 1) {
      const int64_t y = __shfl_up(v, o, kWave);
      if (l >= o) v += y;
    }
    incl[q] = v;
    if (l == kWave - 1) s_part[q][wv] = v;
  }
  __syncthreads();
  for (int q = 0; q < kLayoutCols; q++) {
    int64_t pre = 0, tot = 0;
    for (int w = 0; w < 16; w++) {
      pre += w < wv ? s_part[q][w] : 0;
      tot += s_part[q][w];
    }
    x[q] = pre + incl[q];
    total[q] = tot;
  }
  __syncthreads();
}

__device__ __forceinline__ int64_t* layout_out(int q, int64_t* off_t, int64_t* off_e, int64_t* off_v,
                                               int64_t* off_top, int64_t* off_b) {
  return q == 0 ? off_t : (q == 1 ? off_e : (q == 2 ? off_v : (q == 3 ? off_top : off_b)));
}

// off_X[c] = sum over candidates before c, the five columns at once; one
// workgroup walks the whole batch (small batches, and callers without scratch)
__global__ void __launch_bounds__(1024) k_layout(BatchView b, int32_t n_mem, const int32_t* n_tasks,
                                                 const int64_t* n_edges, int64_t cap_t, int64_t cap_e,
                                                 int64_t* off_t, int64_t* off_e, int64_t* off_v, int64_t* off_top,
                                                 int64_t* off_b) {
  __shared__ int64_t s_part[kLayoutCols][16];
  int64_t carry[kLayoutCols] = {0, 0, 0, 0, 0};
  for (int base = 0; base < b.n_cand; base += 1024) {
    const int c = base + (int)threadIdx.x;
    int64_t x[kLayoutCols], tot[kLayoutCols];
    layout_cols(b, n_mem, n_tasks, n_edges, cap_t, cap_e, c, x);
    layout_block_scan(x, s_part, tot);
    for (int q = 0; q < kLayoutCols; q++) {
      int64_t* off = layout_out(q, off_t, off_e, off_v, off_top, off_b);
      if (off && c < b.n_cand) off[c + 1] = carry[q] + x[q];
      carry[q] += tot[q];
    }
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < kLayoutCols; q++) {
      int64_t* off = layout_out(q, off_t, off_e, off_v, off_top, off_b);
      if (off) off[0] = 0;
    }
}

// the same over many workgroups: each scans its 1,024 candidates and leaves its
// totals in part[q][block]; k_layout_fix then adds the totals of the blocks before
__global__ void __launch_bounds__(1024) k_layout_part(BatchView b, int32_t n_mem, const int32_t* n_tasks,
                                                      const int64_t* n_edges, int64_t cap_t, int64_t cap_e,
                                                      int64_t* off_t, int64_t* off_e, int64_t* off_v,
                                                      int64_t* off_top, int64_t* off_b, int64_t* part) {
  __shared__ int64_t s_part[kLayoutCols][16];
  const int c = blockIdx.x * 1024 + (int)threadIdx.x;
  int64_t x[kLayoutCols], tot[kLayoutCols];
  layout_cols(b, n_mem, n_tasks, n_edges, cap_t, cap_e, c, x);
  layout_block_scan(x, s_part, tot);
  for (int q = 0; q < kLayoutCols; q++) {
    int64_t* off = layout_out(q, off_t, off_e, off_v, off_top, off_b);
    if (off && c < b.n_cand) off[c + 1] = x[q];
    if (threadIdx.x == 0) part[q * gridDim.x + blockIdx.x] = tot[q];
  }
}

__global__ void __launch_bounds__(1024) k_layout_fix(int32_t n, int64_t* off_t, int64_t* off_e, int64_t* off_v,
                                                     int64_t* off_top, int64_t* off_b, const int64_t* part) {
  __shared__ int64_t s_carry[kLayoutCols];
  if (threadIdx.x < kLayoutCols) {
    int64_t sum = 0;
    for (unsigned k = 0; k < blockIdx.x; k++) sum += part[threadIdx.x * gridDim.x + k];
    s_carry[threadIdx.x] = sum;
  }
  __syncthreads();
  const int c = blockIdx.x * 1024 + (int)threadIdx.x;
  for (int q = 0; q < kLayoutCols; q++) {
    int64_t* off = layout_out(q, off_t, off_e, off_v, off_top, off_b);
    if (!off) continue;
    if (c < n) off[c + 1] += s_carry[q];
    if (c == 0) off[0] = 0;
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

// Task record, four 8-byte words per task (32-byte aligned): the ordering key
// (low half) and first successor edge (high half), the dispatch word, the
// critical time (FCFS: minus the release time) and one past the last edge.  The
// event loop writes only the third word.
constexpr int kRecKE = 0, kRecW = 1, kRecRank = 2, kRecE1 = 3;
static_assert(kRecW == kRecKE + 1 && kRecE1 == kRecRank + 1 && kRecKE % 2 == 0 && kRecRank % 2 == 0,
              "records are read and written as aligned 16-byte pairs");

struct CandPtrs {
  int64_t toff;        // first task of the candidate in the chunk's task arrays
  uint32_t* top_first;
  uint32_t* desc;      // per task: packed descriptor (preparation only)
  uint32_t* indeg;
  uint32_t* cur;
  uint32_t* succ;
  int64_t* rec;        // per task: the record above
  int64_t* fifo;       // per queued task: [finish, id | completion word << 32, e0 | e1 << 32] of the task behind it
  uint32_t* ready;
  int64_t* sortbuf;
  int64_t* vf;         // [finest block][memory space] valid-from times
  int64_t* use;        // finite spaces: [finest block][space] latest mapping there of a task using it
  uint32_t* pin;       // finite spaces: [finest block][space] mapped tasks there not yet finished
};

// a candidate's arrays one after the other in one block of region_bytes(T, E, V, TP)
// bytes, 8-byte elements first
__device__ __forceinline__ CandPtrs carve(uint8_t* r, int64_t T, int64_t E, int64_t V) {
  CandPtrs p;
  p.toff = 0;
  p.use = nullptr;            // region mode has no finite spaces
  p.pin = nullptr;
  p.rec = (int64_t*)r;        r += 32 * T;
  p.fifo = (int64_t*)r;       r += 24 * T;
  p.sortbuf = (int64_t*)r;    r += 32 * T;
  p.vf = (int64_t*)r;         r += 8 * V;
  p.desc = (uint32_t*)r;      r += 4 * T;
  p.indeg = (uint32_t*)r;     r += 4 * T;
  p.cur = (uint32_t*)r;       r += 4 * T;
  p.ready = (uint32_t*)r;     r += 4 * T;
  p.succ = (uint32_t*)r;      r += 4 * E;
  p.top_first = (uint32_t*)r;
  return p;
}

__device__ __forceinline__ CandPtrs cand_ptrs(const ChunkView& v, int c) {
  CandPtrs p;
  const int64_t t = v.task_off[c] - v.task_off[v.c0];
  const int64_t e = v.edge_off[c] - v.edge_off[v.c0];
  const int64_t f = v.vf_off[c] - v.vf_off[v.c0];
  const int64_t tp = v.top_off[c] - v.top_off[v.c0];
  if (v.region) {
    // region mode: the candidate's own block at its byte offset
    const int64_t T = v.task_off[c + 1] - v.task_off[c], E = v.edge_off[c + 1] - v.edge_off[c];
    const int64_t V = v.vf_off[c + 1] - v.vf_off[c];
    p = carve(v.region + (v.byte_off[c] - v.byte_off[v.c0]), T, E, V);
    p.toff = t;
    return p;
  }
  p.toff = t;
  p.top_first = v.top_first + tp;
  p.desc = v.desc + t;
  p.indeg = v.indeg + t;
  p.cur = v.cur + t;
  p.succ = v.succ + e;
  p.rec = v.rec + 4 * t;
  p.fifo = v.fifo + 3 * t;
  p.ready = v.ready + t;
  p.sortbuf = v.sortbuf + 4 * t;
  p.vf = v.vf + f;
  p.use = v.use ? v.use + f : nullptr;
  p.pin = v.pin ? v.pin + f : nullptr;
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

// critical times and the task records, initial validity and the first ready
// list; cur[f] = one past the last edge of f, successor lists filled
// returns the number of tasks without predecessors (the first ready list)
__device__ __forceinline__ int prep_finish(int prep_in, const OutView& out, int c, int nt, int dmax, int M,
                                           const CandPtrs& sp, int64_t n_fine,
                                           const int64_t (*s_W)[kLevels], PrepLds& s) {
  const int l = lane();
  const int in_cap = prep_in >= 1 && prep_in <= kPrepIn ? prep_in : kPrepIn;
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
      for (int q = 0; q < 4; q++) rv[q] = (v[q] != kNil && v[q] >= lim) ? vld(&sp.rec[4 * v[q] + kRecRank]) : 0;
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
      // the whole record in two 16-byte stores
      const int kind = desc_kind(dsc), lvl = desc_level(dsc);
      const int K = desc_K(dsc), I = desc_I(dsc), J = desc_J(dsc);
      // at most two successors: their numbers replace the edge range
      const uint32_t deg = e1 - e0;
      uint64_t dwv = dispatch_word(nt, dmax, kind, lvl, K, I, J);
      uint32_t s0 = e0, s1 = e1;
      if (deg <= 2u) {
        s0 = deg >= 1u ? vld(&sp.succ[e0]) : kNil;
        s1 = deg == 2u ? vld(&sp.succ[e0 + 1]) : kNil;
        dwv |= kDwInline;
      }
      longlong2 kw, re;
      kw.x = (long long)(task_key_of(dmax, lvl, K, I, J) | ((uint64_t)s0 << 32));
      kw.y = (long long)dwv;
      re.x = r;
      re.y = (long long)s1;
      *reinterpret_cast<longlong2*>(&sp.rec[4 * f + kRecKE]) = kw;
      *reinterpret_cast<longlong2*>(&sp.rec[4 * f + kRecRank]) = re;
    }
    __syncthreads();
  }

  // initial validity: data valid on the host (space 0) only
  {
    const int64_t n_vf = ((int64_t)tri2(nt) << (2 * dmax)) * M;
    const int step = kWave % M;
    int m = l % M;
    for (int64_t e = l; e < n_vf; e += kWave) {
      sp.vf[e] = m == 0 ? 0 : kInf;
      if (sp.pin) {
        sp.pin[e] = 0u;
        sp.use[e] = 0;
      }
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
    out.status[c] = kOK;
    if (out.n_tasks) out.n_tasks[c] = (int32_t)n_fine;
  }
  return (int)n_src;
}

// ---------------------------------------------------------------- preparation

// Preparation of depth candidate c by one whole wavefront into the arrays sp
// (T tasks and E edges, the exact counts): status checks, A -- first fine task
// of every top-level task, B -- descriptors, predecessor counts, successor
// counts, C -- successor offsets, D -- successor lists, then critical times,
// initial validity and the first ready list.  cap: the candidate does not fit
// its storage (HESP_ECAPACITY).  Returns the status (written to the outputs,
// with makespan -1 when not OK); n_src gets the number of first ready tasks.
__device__ __forceinline__ int prepare_cand(const SimTables& tb, const BatchView& bv, const OutView& out, int c, const CandPtrs& sp,
                            int64_t n_tasks, int64_t n_edges, bool cap, int prep_in,
                            const int64_t (*s_W)[kLevels], PrepLds& s_p, int& n_src) {
  const int l = lane();
  const Cand cd = load_cand(bv, c);
  const int nt = cd.nt, dmax = cd.dmax, M = tb.n_mem;
  int status = kOK;
  // a ragged candidate above the batch's stated maxima is refused too (the
  // maxima choose the lanes per candidate)
  if (nt < 1 || dmax < 0 || dmax > kMaxLevel || dmax > tb.max_level || (nt << dmax) > kMaxFine || dmax > bv.dmax ||
      nt > bv.nt)
    status = kEINVAL;
  if (status == kOK && cap) status = kECAP;

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
    return status;
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

  n_src = prep_finish(prep_in, out, c, nt, dmax, M, sp, n_fine, s_W, s_p);
  return kOK;
}

// eight waves per SIMD (64 VGPRs): the passes wait on memory most of the time
__global__ void __launch_bounds__(kWave, 8) k_prepare(SimTables tb, BatchView bv, ChunkView cv, OutView out) {
  __shared__ int64_t s_W[4][kLevels];
  __shared__ PrepLds s_p;
  const int l = lane();
  for (int x = l; x < 4 * kLevels; x += kWave) (&s_W[0][0])[x] = (&tb.W[0][0])[x];
  __syncthreads();

  const int c = cv.c0 + (int)blockIdx.x;
  if (c >= bv.n_cand) return;
  const bool cap = (cv.cap_tasks > 0 && cv.cnt_tasks[c] > cv.cap_tasks) ||
                   (cv.cap_edges > 0 && cv.cnt_edges[c] > cv.cap_edges) || region_overflow(cv, c);
  const int64_t n_tasks = cv.task_off[c + 1] - cv.task_off[c];
  const int64_t n_edges = cv.edge_off[c + 1] - cv.edge_off[c];
  int n_src = 0;
  if (prepare_cand(tb, bv, out, c, cand_ptrs(cv, c), n_tasks, n_edges, cap, cv.prep_in, s_W, s_p, n_src) == kOK &&
      l == 0)
    cv.nsrc[c - cv.c0] = n_src;
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
  // A task's distinct last writers are dealt to the lanes as they are found,
  // lane j holding writers j, j + 64 and j + 128; their successor counters are
  // then updated by all lanes together instead of one writer at a time.  Writers
  // past the first 3 x 64 (blocks of side 16 or 32 only) are counted one at a
  // time as found.
  walk_tree(nt, dmax, flags, [&](int kind, int lv, int K, int I, int J) {
    const uint32_t f = nf_seen++;
    uint32_t wr[3] = {kNil, kNil, kNil};
    int k = 0;
    const int np = scan_task(lw, nt, dmax, kind, lv, K, I, J, f, [&](uint32_t p) {
      for (int h = 0; h < 3; h++) wr[h] = k == l + h * kWave ? p : wr[h];
      if (k >= 3 * kWave && l == 0) atomicAdd(&sp.cur[p], 1u);
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
      if (k >= 3 * kWave && l == 0) {
        const uint32_t q = atomicAdd(&sp.cur[p], 1u);
        if (q < n_edges) sp.succ[q] = f;
      }
      k++;
    });
    uint32_t pos[3];
    for (int h = 0; h < 3; h++) pos[h] = wr[h] != kNil ? atomicAdd(&sp.cur[wr[h]], 1u) : 0u;
    for (int h = 0; h < 3; h++)
      if (wr[h] != kNil && pos[h] < n_edges) sp.succ[pos[h]] = f;
  });
  wave_order();
  const int n_src = prep_finish(cv.prep_in, out, c, nt, dmax, M, sp, n_fine, s_W, s_p);
  if (l == 0) cv.nsrc[c - cv.c0] = n_src;
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

// Per-group LDS state of the event loop.
constexpr int kEvict = 256;   // finite spaces: evictable blocks gathered at once
template <int G, int POL>
struct SimLds {
  static constexpr int NG = kWave / G;
  int64_t fin[NG][4][kMaxMem];    // per (block, space): latest finite valid-from
  int32_t miss[NG][4][kMaxMem];   // per (block, space): finest blocks missing
  int64_t rdy[NG][kMaxMem];       // default policy: per space, when the task's data is ready there
  // write-around: per (block, space), the latest host valid-from of the missing
  // finest blocks (their transfer cannot leave before)
  int64_t src[POL == 0 ? 1 : NG][4][kMaxMem];
  // finite spaces (POL 3): per (block, space) the task's finest blocks pinned by no
  // other task; per space the candidate's capacity in finest blocks (-1:
  // unbounded), the finest blocks held and those pinned
  int32_t npin[POL == 3 ? NG : 1][4][kMaxMem];
  int64_t capm[POL == 3 ? NG : 1][kMaxMem];
  int32_t occ[POL == 3 ? NG : 1][kMaxMem];
  int32_t pinned[POL == 3 ? NG : 1][kMaxMem];
  int64_t ev[POL == 3 ? NG : 1][POL == 3 ? kEvict : 1];   // evictable blocks' keys, gathered per mapping
  uint32_t rid[NG][G];            // ready list, first G entries, with records
  int64_t rrank[NG][G];
  uint64_t rw[NG][G];             // dispatch words
  uint32_t rkey[NG][G];
  uint32_t re0[NG][G];
  uint32_t re1[NG][G];
  uint8_t order[NG][G];
};
// With the preparation fused in, a wave prepares its next candidate while the
// event loop's state is dead: the preparation's LDS overlays it.
template <int G, int POL>
union SimPrepLds {
  SimLds<G, POL> sim;
  PrepLds prep;
};

// Instantiated per policy class so that the default policy carries no policy
// code: R-P / F-P map tasks only onto idle processors and may make them wait.
// The whole-wave variant is limited to 80 VGPRs, six waves per SIMD: the event
// loop waits on memory and on its own dependent steps, and at six waves it needs
// no spill code (16x16-tile headline batch, per launch: 275 ms at six waves,
// 280 at seven with a few spills, 324 at eight, 285 at five and at four); the
// 16- and 32-lane variants lose when squeezed and keep their registers.
// FUSED (whole-wave groups only): each wave prepares the candidates it claims
// itself (prepare_cand) into its own slot of cv.slot_bytes bytes, so a batch
// needs neither the separate preparation launch nor memory chunks; the slot is
// slot blockIdx.x of cv.region (FUSED 1) or the workgroup's dynamic LDS (FUSED
// 2: the whole state of a small candidate, validity table, records, successor
// lists and queues, never leaves the compute unit; its LDS slot, not registers,
// bounds the waves per compute unit, so this variant keeps its registers).  FUSED
// 1 runs at four waves per SIMD (128 VGPRs): the preparation's live state spills
// at six (16x16-tile headline batch, per step: 401 ms at four, 598 at five, 658
// at six, 475 at three).  Finite spaces on deep tables: four (their LDS, with
// the six-level cost table, holds no more).
// DT: the platform's tables are deeper than kXferLevels levels (candidates of
// depth 4 and 5 among them): the rest of the transfer table is read from device
// memory, and whole-wave groups scan block sides up to 32 without the
// compile-time specialisation (blocks above 8 x 8 finest blocks span passes).
constexpr int sim_waves(int G, int POL, int FUSED, int DT) {
  return G != 64 ? 1 : FUSED == 2 ? 2 : FUSED == 1 ? 4 : (POL == 3 && DT) ? 4 : 6;
}
template <int G, int POL, int FUSED, int DT = 0>
__global__ void __launch_bounds__(kWave, sim_waves(G, POL, FUSED, DT)) k_sim(SimTables tb, BatchView bv, ChunkView cv, OutView out,
                                               uint32_t* counter) {
  static_assert(!FUSED || G == kWave, "the fused preparation needs whole-wave groups");
  // POL 0: Priority-List + EFT-P + write-back (no policy flags read); 1: the
  // other push policies (FCFS, EIT-P) and caching policies; 2: R-P / F-P; 3:
  // finite memory spaces (PL or FCFS, EFT-P, write-back, independent transfers)
  constexpr bool PULL = POL == 2;
  constexpr bool CAP = POL == 3;
  static_assert(!CAP || (G == kWave && !FUSED), "finite spaces run in whole-wave groups, unfused");
  const bool fcfs = POL != 0 && tb.fcfs;
  const int sel = (POL == 0 || CAP) ? 0 : tb.sel;
  const int cache = (POL == 0 || CAP) ? 0 : tb.cache;
  const bool bus = POL != 0 && !CAP && tb.bus != 0;
  constexpr int LGG = G == 16 ? 4 : (G == 32 ? 5 : 6);
  // task times of the levels the groups can meet (whole-wave groups: 0..3)
  constexpr int kSimLevels = G == kWave && !DT ? kMaxWaveLevel + 1 : kLevels;
  __shared__ int64_t s_cost[kMaxPtypes][4][kSimLevels];
  __shared__ int64_t s_xfer[kXferLen];
  __shared__ int64_t s_W[FUSED ? 4 : 1][kLevels];
  using Lds = std::conditional_t<(FUSED != 0), SimPrepLds<G, POL>, SimLds<G, POL>>;
  extern __shared__ __align__(16) uint8_t s_ws[];   // FUSED 2: the candidate's workspace
  __shared__ Lds s_l;
  SimLds<G, POL>& L = reinterpret_cast<SimLds<G, POL>&>(s_l);
  auto& s_fin = L.fin;
  auto& s_miss = L.miss;
  auto& s_rdy = L.rdy;
  auto& s_src = L.src;
  auto& s_npin = L.npin;
  auto& s_capm = L.capm;
  auto& s_occ = L.occ;
  auto& s_pinned = L.pinned;
  auto& s_ev = L.ev;
  auto& s_rid = L.rid;
  auto& s_rrank = L.rrank;
  auto& s_rw = L.rw;
  auto& s_rkey = L.rkey;
  auto& s_re0 = L.re0;
  auto& s_re1 = L.re1;
  auto& s_order = L.order;

  const Grp<G> gp;
  const int l = gp.l, g = gp.g, gl = gp.gl;
  for (int x = l; x < kMaxPtypes * 4 * kSimLevels; x += kWave)
    (&s_cost[0][0][0])[x] = tb.cost[x / (4 * kSimLevels)][(x / kSimLevels) % 4][x % kSimLevels];
  for (int x = l; x < kXferLen; x += kWave) s_xfer[x] = tb.xfer[x];
  // xf(m): transfer time of m of the candidate's finest blocks (side b / 2^dmax),
  // entry m xs of the platform's table (blocks of side b / 2^max_level): in LDS,
  // or past its first kXferLen entries (DT) in device memory
  const int64_t* const xdeep = tb.xfer_deep;
  int64_t xs = 0;
  auto xf = [&](int64_t m) -> int64_t {
    const int64_t i = m * xs;
    if constexpr (!DT) return s_xfer[i];
    return i < kXferLen ? s_xfer[i] : xdeep[i];
  };
  if (FUSED)
    for (int x = l; x < 4 * kLevels; x += kWave) (&s_W[0][0])[x] = (&tb.W[0][0])[x];
  __syncthreads();

  const int P = tb.n_procs, M = tb.n_mem;
  const bool p16 = P <= 16;                    // processor lanes all in the group's first row
  const int pmem = gl < P ? tb.proc_mem[gl] : 0;
  const int plink = gl < P ? tb.link[pmem] : 0;   // the link of the transfers into the lane's space
  const int hlink = tb.link[0];                   // and into the host's
  const int ptype = gl < P ? tb.proc_type[gl] : 0;
  const bool want_sched = out.sched_off != nullptr;

  int c = 0, dmax = 0;
  int64_t T = 0, n_ready = 0, sbase = 0;
  int64_t n_atoms = 0;                        // finite spaces: the candidate's finest blocks
  CandPtrs sp{};
  int64_t avail = 0, hfin = kInf;
  int64_t lfree = 0;                          // link contention: lane l < n_mem holds when link l is free
  // queue head of processor lane: task, finish, completion word, successor edges
  uint32_t hid = kNil, hcw = 0, he0 = 0, he1 = 0, tail = kNil;

  // entry pos of the ready list: task v with its rank, key | e0 << 32, dispatch
  // word and e1 (the first G entries in LDS, the rest by number only)
  auto push = [&](int64_t pos, uint32_t v, int64_t rank, int64_t ke, int64_t dw, int64_t e1) {
    if (pos < G) {
      s_rid[g][pos] = v;
      s_rrank[g][pos] = rank;
      s_rw[g][pos] = (uint64_t)dw;
      s_rkey[g][pos] = (uint32_t)ke;
      s_re0[g][pos] = (uint32_t)((uint64_t)ke >> 32);
      s_re1[g][pos] = (uint32_t)e1;
    } else {
      sp.ready[pos] = v;
    }
  };
  // the read-only words of task v's record: key | e0 << 32 and the dispatch word
  // in one 16-byte load, e1
  auto rec_ro = [&](uint32_t v, int64_t& ke, int64_t& dw, int64_t& e1) {
    const longlong2 kw = *reinterpret_cast<const longlong2*>(&sp.rec[4 * v + kRecKE]);
    ke = kw.x;
    dw = kw.y;
    e1 = sp.rec[4 * v + kRecE1];
  };

  if constexpr (!FUSED) {
    // groups without a candidate take the next one; the wave runs until every
    // group has found the candidates exhausted
    bool active = false, exhausted = false;
    for (;;) {
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
            dmax = cd.dmax;
            xs = (int64_t)1 << (2 * (tb.max_level - dmax));
            sp = cand_ptrs(cv, c);
            sbase = want_sched ? out.sched_off[c] : 0;
            T = 0;
            avail = 0;
            lfree = 0;
            hfin = kInf;
            hid = kNil;
            tail = kNil;
            if constexpr (CAP) {
              n_atoms = (int64_t)tri2(cd.nt) << (2 * dmax);
              if (gl < M) {
                const int64_t cb = tb.capacity[gl];
                s_capm[g][gl] = cb >= 0 ? cb >> (2 * (tb.max_level - dmax)) : -1;
                s_occ[g][gl] = 0;
                s_pinned[g][gl] = 0;
              }
            }
            n_ready = cv.nsrc[c - cv.c0];
            // FCFS keeps minus the release time in the rank slot (sources: 0)
            for (int64_t x = gl; x < (fcfs || n_ready < G ? n_ready : G); x += G) {
              const uint32_t v = vld(&sp.ready[x]);
              if (fcfs) sp.rec[4 * v + kRecRank] = 0;
              if (x < G) {
                int64_t ke, dw, e1;
                rec_ro(v, ke, dw, e1);
                push(x, v, fcfs ? 0 : vld(&sp.rec[4 * v + kRecRank]), ke, dw, e1);
              }
            }
            active = true;
          }
        }
      }
      if (__ballot(!exhausted) == 0) break;
      if (!active) continue;
      wave_order();
#define HESP_CANDIDATE_DONE \
  {                         \
    active = false;         \
    continue;               \
  }
#include "hesp_sim_round.inc"
#undef HESP_CANDIDATE_DONE
    }
  } else {
    // the wave prepares each candidate it takes into its own slot, then runs it
    // to completion (no event-loop state lives across the preparation)
    for (;;) {
      int cc = 0;
      if (l == 0) cc = (int)atomicAdd(counter, 1u);
      cc = __builtin_amdgcn_readfirstlane(cc);
      if (cc >= cv.nc) break;
      c = cv.c0 + (cv.order ? (int)cv.order[cc] : cc);
      {
        const Cand cq = load_cand(bv, c);
        const int64_t Tq = cv.cnt_tasks[c], Eq = cv.cnt_edges[c];
        const bool shape_ok = cq.nt >= 1 && cq.dmax >= 0 && cq.dmax <= kMaxLevel && (cq.nt << cq.dmax) <= kMaxFine;
        const int64_t Vq = shape_ok ? ((int64_t)tri2(cq.nt) << (2 * cq.dmax)) * M : 0;
        const bool cap = (cv.cap_tasks > 0 && Tq > cv.cap_tasks) || (cv.cap_edges > 0 && Eq > cv.cap_edges) ||
                         region_bytes(Tq, Eq, Vq, cq.n_top + 1) > cv.slot_bytes;
        sp = carve(FUSED == 2 ? s_ws : cv.region + (int64_t)blockIdx.x * cv.slot_bytes, Tq, Eq, Vq);
        int n_src = 0;
        const bool ok = prepare_cand(tb, bv, out, c, sp, Tq, Eq, cap, cv.prep_in, s_W, s_l.prep, n_src) == kOK;
        __syncthreads();   // the preparation's LDS is the event loop's from here
        if (!ok) continue;
        dmax = cq.dmax;
        n_ready = n_src;
      }
      xs = (int64_t)1 << (2 * (tb.max_level - dmax));
      sbase = want_sched ? out.sched_off[c] : 0;
      T = 0;
      avail = 0;
      lfree = 0;
      hfin = kInf;
      hid = kNil;
      tail = kNil;
      for (int64_t x = gl; x < (fcfs || n_ready < G ? n_ready : G); x += G) {
        const uint32_t v = vld(&sp.ready[x]);
        if (fcfs) sp.rec[4 * v + kRecRank] = 0;
        if (x < G) {
          int64_t ke, dw, e1;
          rec_ro(v, ke, dw, e1);
          push(x, v, fcfs ? 0 : vld(&sp.rec[4 * v + kRecRank]), ke, dw, e1);
        }
      }
      for (;;) {
        wave_order();
#define HESP_CANDIDATE_DONE break
#include "hesp_sim_round.inc"
#undef HESP_CANDIDATE_DONE
      }
      __syncthreads();   // and the next preparation's after the event loop
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_layout(const BatchView& b, int32_t n_mem, const int32_t* n_tasks, const int64_t* n_edges,
                         int64_t cap_t, int64_t cap_e, int64_t* off_t, int64_t* off_e, int64_t* off_v,
                         int64_t* off_top, int64_t* off_b, hipStream_t s, int64_t* part) {
  const int blocks = (b.n_cand + 1023) / 1024;
  if (!part || blocks <= 4) {
    hipLaunchKernelGGL(k_layout, dim3(1), dim3(1024), 0, s, b, n_mem, n_tasks, n_edges, cap_t, cap_e, off_t, off_e,
                       off_v, off_top, off_b);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_layout_part, dim3(blocks), dim3(1024), 0, s, b, n_mem, n_tasks, n_edges, cap_t, cap_e, off_t,
                     off_e, off_v, off_top, off_b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_layout_fix, dim3(blocks), dim3(1024), 0, s, b.n_cand, off_t, off_e, off_v, off_top, off_b,
                     part);
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
  const bool fused = v.slot_bytes > 0;
  if (fused && (group != 64 || (!v.region && !v.slot_lds) || b.tree_stride > 0)) return hipErrorInvalidValue;
  if (v.slot_lds && (!fused || v.slot_bytes > kLdsSlotMax)) return hipErrorInvalidValue;
  hipError_t e = launch_zero_u32(counter, s);
  if (e != hipSuccess) return e;
  const int G = group;
  const int per_wave = kWave / G;
  int waves = (v.nc + per_wave - 1) / per_wave;
  if (waves > slots) waves = slots;
  const int pol = t.capped ? 3 : (t.sel >= 2 ? 2 : (t.sel == 1 || t.fcfs || t.cache != 0 || t.bus != 0 ? 1 : 0));
  if (pol == 3 && (fused || G != 64 || !v.use || !v.pin)) return hipErrorInvalidValue;
  const bool dt = t.max_level > kXferLevels;
  if (dt && (fused || !t.xfer_deep)) return hipErrorInvalidValue;
  const dim3 grid(waves), block(kWave);
#define HESP_SIM_LAUNCH(GG, PP, FF, LDSB) \
  hipLaunchKernelGGL((k_sim<GG, PP, FF>), grid, block, LDSB, s, t, b, v, o, counter)
#define HESP_SIM_LAUNCH_N(GG, PP)                                                               \
  do {                                                                                          \
    if (dt) hipLaunchKernelGGL((k_sim<GG, PP, 0, 1>), grid, block, 0, s, t, b, v, o, counter);  \
    else hipLaunchKernelGGL((k_sim<GG, PP, 0, 0>), grid, block, 0, s, t, b, v, o, counter);     \
  } while (0)
  if (fused && v.slot_lds) {
    const size_t ws = (size_t)v.slot_bytes;
    if (pol == 0) HESP_SIM_LAUNCH(64, 0, 2, ws);
    else if (pol == 1) HESP_SIM_LAUNCH(64, 1, 2, ws);
    else HESP_SIM_LAUNCH(64, 2, 2, ws);
  } else if (fused) {
    if (pol == 0) HESP_SIM_LAUNCH(64, 0, 1, 0);
    else if (pol == 1) HESP_SIM_LAUNCH(64, 1, 1, 0);
    else HESP_SIM_LAUNCH(64, 2, 1, 0);
  } else if (G == 16) {
    if (pol == 0) HESP_SIM_LAUNCH_N(16, 0);
    else if (pol == 1) HESP_SIM_LAUNCH_N(16, 1);
    else HESP_SIM_LAUNCH_N(16, 2);
  } else if (G == 32) {
    if (pol == 0) HESP_SIM_LAUNCH_N(32, 0);
    else if (pol == 1) HESP_SIM_LAUNCH_N(32, 1);
    else HESP_SIM_LAUNCH_N(32, 2);
  } else {
    if (pol == 0) HESP_SIM_LAUNCH_N(64, 0);
    else if (pol == 1) HESP_SIM_LAUNCH_N(64, 1);
    else if (pol == 2) HESP_SIM_LAUNCH_N(64, 2);
    else HESP_SIM_LAUNCH_N(64, 3);
  }
#undef HESP_SIM_LAUNCH
#undef HESP_SIM_LAUNCH_N
  return hipGetLastError();
}

// largest region_bytes of a candidate of the batch (for the fused simulation's
// slots): out[0] = max over candidates (atomic maximum; out[0] zeroed first)
__global__ void k_max_region(BatchView b, int32_t n_mem, const int32_t* n_tasks, const int64_t* n_edges,
                             unsigned long long* out) {
  unsigned long long m = 0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < b.n_cand; c += gridDim.x * blockDim.x) {
    const int nt = b.nt_arr ? b.nt_arr[c] : b.nt;
    const int dmax = b.dmax_arr ? b.dmax_arr[c] : b.dmax;
    const bool ok = nt >= 1 && dmax >= 0 && dmax <= kMaxLevel && (nt << dmax) <= kMaxFine;
    if (!ok) continue;
    const int64_t V = ((int64_t)tri2(nt) << (2 * dmax)) * n_mem;
    const unsigned long long r = (unsigned long long)region_bytes(n_tasks[c], n_edges[c], V, tet3(nt) + 1);
    m = r > m ? r : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(m, o, kWave);
    m = y > m ? y : m;
  }
  if ((threadIdx.x & (kWave - 1)) == 0 && m) atomicMax(out, m);
}

hipError_t launch_max_region(const BatchView& b, int32_t n_mem, const int32_t* n_tasks, const int64_t* n_edges,
                             int64_t* out, hipStream_t s) {
  hipError_t e = launch_zero_u32(reinterpret_cast<uint32_t*>(out), s);
  if (e == hipSuccess) e = launch_zero_u32(reinterpret_cast<uint32_t*>(out) + 1, s);
  if (e != hipSuccess) return e;
  const int blocks = b.n_cand > 0 ? (b.n_cand + 255) / 256 < 1024 ? (b.n_cand + 255) / 256 : 1024 : 1;
  hipLaunchKernelGGL(k_max_region, dim3(blocks), dim3(256), 0, s, b, n_mem, n_tasks, n_edges,
                     reinterpret_cast<unsigned long long*>(out));
  return hipGetLastError();
}

}  // namespace hesp
