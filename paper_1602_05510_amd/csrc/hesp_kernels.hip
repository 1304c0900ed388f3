// hesp_kernels.hip -- gfx950 kernels of the batched HeSP simulator.
//
// k_simulate is a persistent kernel: one wavefront (64 lanes) per workgroup,
// each workgroup repeatedly takes the next candidate from an atomic counter and
// runs, for that candidate,
//   E  expansion of the Fig. 1 loop nest by the candidate's split depths into
//      fine tasks and a successor CSR (section 2.1, "Recursive task
//      partitioners"; dependences RaW/WaW by data block),
//   R  critical times: sum of the task time over all processors plus the largest
//      critical time among the successors ("Priority-List", section 2.1),
//   S  the event simulation: every task released at the current time is mapped
//      at once, in decreasing critical time (ties: smaller fine indices), to the
//      processor with the earliest finish time counting the transfers it needs
//      (EFT-P; ties: lowest processor index); transfers start at mapping time;
//      on completion the written block becomes valid only in the executing
//      processor's memory space (write-back).  Completions that happen at the
//      same instant are all applied before any mapping at that instant.
// The expansion and the rank pass are wave-parallel over tasks; the event loop
// is serial per candidate and wave-parallel inside a step: lanes evaluate the
// finish time on every processor at once (one lane per processor), read the
// validity of every finest block of a task in every memory space at once (one
// lane per block and space), and release successors in parallel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_core.h"
#include "hesp_internal.h"

namespace hesp {

namespace {

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

// DPP lane moves of a 64-bit value (lanes left out by the row mask keep v)
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
  const int lo = (int)(uint32_t)(uint64_t)v, hi = (int)(uint32_t)((uint64_t)v >> 32);
  const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false);
  const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false);
  return (int64_t)(((uint64_t)(uint32_t)rhi << 32) | (uint32_t)rlo);
}
constexpr int kQuadSwap1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadSwap2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kRowRor4 = 0x124, kRowRor8 = 0x128;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return b < a ? b : a; }
__device__ __forceinline__ int64_t max64(int64_t a, int64_t b) { return b > a ? b : a; }

// minimum over the 64 lanes, returned to every lane
__device__ __forceinline__ int64_t wave_min64(int64_t v) {
  v = min64(v, dpp64<kQuadSwap1>(v));
  v = min64(v, dpp64<kQuadSwap2>(v));
  v = min64(v, dpp64<kRowRor4>(v));
  v = min64(v, dpp64<kRowRor8>(v));
  v = min64(v, dpp64<kRowBcast15, 0xA>(v));
  v = min64(v, dpp64<kRowBcast31, 0xC>(v));
  return rdl64(v, kWave - 1);
}

// maximum over aligned segments of 4^k lanes (k = lg/2, lg even, 0..6); the
// last lane of every segment holds its segment's maximum
__device__ __forceinline__ int64_t seg_max64(int64_t v, int lg) {
  if (lg >= 2) {
    v = max64(v, dpp64<kQuadSwap1>(v));
    v = max64(v, dpp64<kQuadSwap2>(v));
  }
  if (lg >= 4) {
    v = max64(v, dpp64<kRowRor4>(v));
    v = max64(v, dpp64<kRowRor8>(v));
  }
  if (lg >= 6) {
    v = max64(v, dpp64<kRowBcast15, 0xA>(v));
    v = max64(v, dpp64<kRowBcast31, 0xC>(v));
  }
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

// The ready list: the first 64 entries live in LDS with the task's record
// (critical time, descriptor, successor range); the rest in the slot's buffer
// as bare task numbers.
struct Ready {
  uint32_t id[kWave];
  int64_t rank[kWave];
  uint32_t desc[kWave];
  uint32_t e0[kWave];
  uint32_t e1[kWave];
};

// ---------------------------------------------------------------- candidates

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

// ---------------------------------------------------------------- counting

__global__ void __launch_bounds__(kWave) k_count(BatchView b, int32_t* n_tasks, int64_t* n_edges) {
  const int c = blockIdx.x;
  if (c >= b.n_cand) return;
  const Cand cd = load_cand(b, c);
  if (cd.nt < 1 || cd.dmax < 0 || cd.dmax > kMaxLevel || (cd.nt << cd.dmax) > kMaxFine) {
    if (lane() == 0) {
      if (n_tasks) n_tasks[c] = 0;
      if (n_edges) n_edges[c] = 0;
    }
    return;
  }
  int64_t edges = 0, tasks = 0;
  auto depth_of = [&](int64_t t) { int d = cd.depth[t]; return d > cd.dmax ? cd.dmax : d; };
  auto first_of = [&](int64_t t) { return t << 32; };   // distinct per top-level task
  for_each_fine(cd, [&](bool valid, int64_t f, int64_t top, uint32_t cell, int d, int K, int I, int J) {
    (void)f;
    if (valid) {
      tasks++;
      edges += for_each_pred(cd.nt, depth_of, first_of, top, cell, d, K, I, J, [](int64_t) {});
    }
  });
  // wave sums
  for (int o = 32; o > 0; o >>= 1) {
    edges += __shfl_xor(edges, o, kWave);
    tasks += __shfl_xor(tasks, o, kWave);
  }
  if (lane() == 0) {
    if (n_tasks) n_tasks[c] = (int32_t)tasks;
    if (n_edges) n_edges[c] = edges;
  }
}

// ---------------------------------------------------------------- simulation

struct SlotPtrs {
  uint32_t* top_first;
  uint32_t* desc;
  int64_t* rec;        // per task: [critical time, descriptor | first successor edge << 32]
  uint32_t* indeg;
  uint32_t* cur;
  uint32_t* succ;
  int64_t* fifo;       // per queued task: [finish, id | desc << 32, e0 | e1 << 32] of the task behind it
  uint32_t* ready;
  int64_t* sortbuf;
  int64_t* vf;
};

__device__ __forceinline__ SlotPtrs slot_ptrs(const Workspace& w, int slot) {
  char* p = w.base + (int64_t)slot * w.stride;
  SlotPtrs s;
  s.top_first = (uint32_t*)(p + w.o_top_first);
  s.desc = (uint32_t*)(p + w.o_desc);
  s.rec = (int64_t*)(p + w.o_rec);
  s.indeg = (uint32_t*)(p + w.o_indeg);
  s.cur = (uint32_t*)(p + w.o_cur);
  s.succ = (uint32_t*)(p + w.o_succ);
  s.fifo = (int64_t*)(p + w.o_fifo);
  s.ready = (uint32_t*)(p + w.o_ready);
  s.sortbuf = (int64_t*)(p + w.o_sort);
  s.vf = (int64_t*)(p + w.o_vf);
  return s;
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
__device__ __forceinline__ uint32_t task_key(uint32_t dsc, int dmax) {
  const int sh = dmax - desc_level(dsc);
  return ((uint32_t)(desc_K(dsc) << sh) << 18) | ((uint32_t)(desc_I(dsc) << sh) << 9) |
         (uint32_t)(desc_J(dsc) << sh);
}

__global__ void __launch_bounds__(kWave) k_simulate(SimTables tb, BatchView bv, Workspace ws, OutView out,
                                                    uint32_t* counter) {
  __shared__ int64_t s_cost[kMaxPtypes][4][kLevels];
  __shared__ int64_t s_xfer[kXferLen];
  __shared__ int64_t s_W[4][kLevels];
  __shared__ uint32_t s_order[kWave];
  __shared__ int64_t s_rdy[4][kMaxMem];   // readiness of block b in space m (current task)
  __shared__ int32_t s_miss[4][kMaxMem];  // its finest blocks missing in space m
  __shared__ int64_t s_rk[kWave];          // critical times of one chunk
  __shared__ Ready s_ready;                // first 64 entries of the ready list

  const int l = lane();
  for (int x = l; x < kMaxPtypes * 4 * kLevels; x += kWave) (&s_cost[0][0][0])[x] = (&tb.cost[0][0][0])[x];
  for (int x = l; x < kXferLen; x += kWave) s_xfer[x] = tb.xfer[x];
  for (int x = l; x < 4 * kLevels; x += kWave) (&s_W[0][0])[x] = (&tb.W[0][0])[x];
  __syncthreads();

  const SlotPtrs sp = slot_ptrs(ws, blockIdx.x);
  const int P = tb.n_procs, M = tb.n_mem;
  const int my_ptype = l < P ? tb.proc_type[l] : 0;
  const int my_mem = l < P ? tb.proc_mem[l] : 0;

  for (;;) {
    int c = 0;
    if (l == 0) c = (int)atomicAdd(counter, 1u);
    c = rdl32(c, 0);
    if (c >= bv.n_cand) break;
    const Cand cd = load_cand(bv, c);
    const int nt = cd.nt, dmax = cd.dmax;
    int status = kOK;

    // ---------------- E: expansion -------------------------------------------
    // pass A: first fine task of every top-level task
    bool bad = false;
    int64_t carry = 0;
    if (nt < 1 || dmax < 0 || dmax > kMaxLevel || dmax > tb.max_level || (nt << dmax) > kMaxFine)
      status = kEINVAL;
    const int64_t n_atoms = status == kOK ? ((int64_t)tri2(nt) << (2 * dmax)) : 0;
    if (status == kOK && n_atoms * M > ws.cap_vf) status = kECAP;
    if (status == kOK && (int64_t)cd.n_top + 1 > ws.cap_tops) status = kECAP;
    if (status == kOK) {
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
      if (__ballot(bad)) status = kEINVAL;
      else if (carry > ws.cap_tasks) status = kECAP;
    }
    const int64_t n_fine = carry;
    if (l == 0 && out.n_tasks) out.n_tasks[c] = status == kOK ? (int32_t)n_fine : 0;
    if (status != kOK) {
      if (l == 0) {
        out.makespan[c] = -1;
        out.status[c] = status;
      }
      continue;
    }
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

    // pass C: exclusive scan of successor counts (cur[f] = first edge of f)
    int64_t ecarry = 0;
    for (int64_t f0 = 0; f0 < n_fine; f0 += kWave) {
      const int64_t f = f0 + l;
      const int v = f < n_fine ? (int)vld_l2(&sp.cur[f]) : 0;
      const int incl = wave_incl_scan(v);
      if (f < n_fine) sp.cur[f] = (uint32_t)(ecarry + incl - v);
      ecarry += rdl32(incl, kWave - 1);
    }
    const int64_t n_edges = ecarry;
    if (n_edges > ws.cap_edges) {
      if (l == 0) {
        out.makespan[c] = -1;
        out.status[c] = kECAP;
      }
      continue;
    }
    wave_order();

    // pass D: fill successor lists; afterwards cur[f] = one past the last edge of f
    for_each_fine(cd, [&](bool valid, int64_t f, int64_t top, uint32_t cell, int d, int K, int I, int J) {
      if (!valid) return;
      for_each_pred(nt, depth_of, first_of, top, cell, d, K, I, J, [&](int64_t p) {
        const uint32_t pos = atomicAdd(&sp.cur[p], 1u);
        sp.succ[pos] = (uint32_t)f;
      });
    });
    wave_order();

    // ---------------- R: critical times, last chunk first ---------------------
    // Successors always have larger numbers: those beyond the chunk are final
    // and read once; those inside it are resolved by iterating the chunk's 64
    // values in LDS to their fixed point (monotone from below).
    const int64_t n_chunks = (n_fine + kWave - 1) / kWave;
    for (int64_t ch = n_chunks - 1; ch >= 0; ch--) {
      const int64_t base = ch * kWave, lim = base + kWave;
      const int64_t f = base + l;
      const bool valid = f < n_fine;
      int64_t w = 0, ext = 0;
      uint64_t inl = 0;                       // up to 8 successor lanes inside the chunk
      int nin = 0;
      bool ovf = false;
      uint32_t e0 = 0, e1 = 0, dsc_f = 0;
      if (valid) {
        const uint32_t dsc = vld(&sp.desc[f]);
        dsc_f = dsc;
        w = s_W[desc_kind(dsc)][desc_level(dsc)];
        e0 = f == 0 ? 0u : vld_l2(&sp.cur[f - 1]);
        e1 = vld_l2(&sp.cur[f]);
        for (uint32_t e = e0; e < e1; e++) {
          const uint32_t v = vld(&sp.succ[e]);
          if (v >= lim) {
            ext = max64(ext, vld(&sp.rec[2 * v]));
          } else if (nin < 8) {
            inl |= (uint64_t)(v - base) << (6 * nin);
            nin++;
          } else {
            ovf = true;
          }
        }
      }
      int64_t r = w + ext;
      for (int sweep = 0; sweep < kWave + 2; sweep++) {
        s_rk[l] = r;
        __syncthreads();
        int64_t mx = ext;
        for (int j = 0; j < nin; j++) mx = max64(mx, s_rk[(inl >> (6 * j)) & 63]);
        if (ovf)
          for (uint32_t e = e0; e < e1; e++) {
            const uint32_t v = vld(&sp.succ[e]);
            if (v < lim) mx = max64(mx, s_rk[v - base]);
          }
        const int64_t nr = w + mx;
        const bool changed = valid && nr != r;
        r = nr;
        __syncthreads();
        if (!__ballot(changed)) break;
      }
      if (valid) {
        sp.rec[2 * f] = r;
        sp.rec[2 * f + 1] = (int64_t)(dsc_f | ((uint64_t)e0 << 32));
      }
    }
    if (l == 0) sp.rec[2 * n_fine + 1] = (int64_t)((uint64_t)n_edges << 32);   // end of the last range

    // ---------------- S: event simulation -------------------------------------
    {
      // data starts valid on the host (space 0) only
      const int step = kWave % M;
      int m = l % M;
      for (int64_t e = l; e < n_atoms * M; e += kWave) {
        sp.vf[e] = m == 0 ? 0 : kInf;
        m += step;
        m = m >= M ? m - M : m;
      }
    }
    // processor p lives in lane p: availability, its FIFO queue's head (with
    // the head's record) and tail
    int64_t avail = 0, hfin = kInf;
    uint32_t hid = kNil, hdesc = 0, he0 = 0, he1 = 0, tail = kNil;
    const int pmem = my_mem, ptype = my_ptype;

    const int64_t xs = (int64_t)1 << (2 * (tb.max_level - dmax));   // transfer index scale
    const bool want_sched = out.sched_off != nullptr;
    const int64_t sbase = want_sched ? out.sched_off[c] : 0;

    // release of task v at ready position pos; r0/r1/r3 are its record words
    auto push = [&](int64_t pos, uint32_t v, int64_t r0, int64_t r1, int64_t r3) {
      if (pos < kWave) {
        s_ready.id[pos] = v;
        s_ready.rank[pos] = r0;
        s_ready.desc[pos] = (uint32_t)r1;
        s_ready.e0[pos] = (uint32_t)((uint64_t)r1 >> 32);
        s_ready.e1[pos] = (uint32_t)((uint64_t)r3 >> 32);
      } else {
        sp.ready[pos] = v;
      }
    };

    int64_t n_ready = 0;
    for (int64_t f0 = 0; f0 < n_fine; f0 += kWave) {
      const int64_t f = f0 + l;
      const bool src = f < n_fine && vld_l2(&sp.indeg[f]) == 0u;
      int64_t r0 = 0, r1 = 0, r3 = 0;
      if (src) {
        r0 = vld(&sp.rec[2 * f]);
        r1 = vld(&sp.rec[2 * f + 1]);
        r3 = vld(&sp.rec[2 * f + 3]);
      }
      const uint64_t m = __ballot(src);
      if (src) push(n_ready + __popcll(m & lanes_below()), (uint32_t)f, r0, r1, r3);
      n_ready += __popcll(m);
    }
    __syncthreads();

    int64_t T = 0;
    for (;;) {
      // (i) map every released task, in priority order
      if (n_ready > 0) {
        const bool small = n_ready <= kWave;
        if (n_ready == 1) {
          s_order[0] = 0;
        } else if (small) {
          // position of each entry: decreasing critical time, then increasing key
          const bool v = l < n_ready;
          const int64_t rk = v ? s_ready.rank[l] : -1;
          const uint32_t ky = v ? task_key(s_ready.desc[l], dmax) : 0u;
          int pos = 0;
          for (int j = 0; j < (int)n_ready; j++) {
            const int64_t rj = rdl64(rk, j);
            const uint32_t kj = (uint32_t)rdl32((int)ky, j);
            pos += (rj > rk || (rj == rk && kj < ky)) ? 1 : 0;
          }
          if (v) s_order[pos] = (uint32_t)l;
        } else {
          // bitonic sort of (critical time, key|id) pairs in the slot's buffer
          int64_t n2 = 1;
          while (n2 < n_ready) n2 <<= 1;
          for (int64_t x = l; x < n2; x += kWave) {
            if (x < n_ready) {
              uint32_t id, dsc;
              int64_t rk;
              if (x < kWave) {
                id = s_ready.id[x];
                rk = s_ready.rank[x];
                dsc = s_ready.desc[x];
              } else {
                id = vld(&sp.ready[x]);
                rk = vld(&sp.rec[2 * id]);
                dsc = (uint32_t)vld(&sp.rec[2 * id + 1]);
              }
              sp.sortbuf[2 * x] = rk;
              sp.sortbuf[2 * x + 1] = ((int64_t)task_key(dsc, dmax) << 32) | id;
            } else {
              sp.sortbuf[2 * x] = -1;
              sp.sortbuf[2 * x + 1] = INT64_MAX;
            }
          }
          wave_order();
          for (int64_t k2 = 2; k2 <= n2; k2 <<= 1) {
            for (int64_t j2 = k2 >> 1; j2 > 0; j2 >>= 1) {
              for (int64_t x = l; x < n2; x += kWave) {
                const int64_t y = x ^ j2;
                if (y > x) {
                  const int64_t ra = vld(&sp.sortbuf[2 * x]), ka = vld(&sp.sortbuf[2 * x + 1]);
                  const int64_t rb = vld(&sp.sortbuf[2 * y]), kb = vld(&sp.sortbuf[2 * y + 1]);
                  // "a before b": larger rank, then smaller key
                  const bool a_first = ra > rb || (ra == rb && ka < kb);
                  const bool up = (x & k2) == 0;
                  if (up != a_first) {
                    sp.sortbuf[2 * x] = rb; sp.sortbuf[2 * x + 1] = kb;
                    sp.sortbuf[2 * y] = ra; sp.sortbuf[2 * y + 1] = ka;
                  }
                }
              }
              wave_order();
            }
          }
        }
        __syncthreads();
        for (int64_t r = 0; r < n_ready; r++) {
          uint32_t t, dsc, e0, e1;
          if (small) {
            const int q = (int)s_order[r];
            t = s_ready.id[q];
            dsc = s_ready.desc[q];
            e0 = s_ready.e0[q];
            e1 = s_ready.e1[q];
          } else {
            t = (uint32_t)(vld(&sp.sortbuf[2 * r + 1]) & 0xFFFFFFFFll);
            t = (uint32_t)rdl32((int)t, 0);
            const int64_t r1 = vld(&sp.rec[2 * t + 1]);
            dsc = (uint32_t)r1;
            e0 = (uint32_t)((uint64_t)r1 >> 32);
            e1 = (uint32_t)((uint64_t)vld(&sp.rec[2 * t + 3]) >> 32);
          }
          t = (uint32_t)rdl32((int)t, 0);
          dsc = (uint32_t)rdl32((int)dsc, 0);
          e0 = (uint32_t)rdl32((int)e0, 0);
          e1 = (uint32_t)rdl32((int)e1, 0);
          const int kind = desc_kind(dsc), lvl = desc_level(dsc);
          const int sh = dmax - lvl;                 // a block is 2^sh x 2^sh finest blocks
          const int lg = 2 * sh;
          const int wmask = (1 << sh) - 1;
          int br[3], bc[3];
          const int nb = desc_blocks(dsc, br, bc);
          const int64_t ab0 = atom_base(nt, dmax, lvl, br[0], bc[0]);
          const int64_t ab1 = nb > 1 ? atom_base(nt, dmax, lvl, br[1], bc[1]) : 0;
          const int64_t ab2 = nb > 2 ? atom_base(nt, dmax, lvl, br[2], bc[2]) : 0;
          // one lane per (space m, block b, finest block a): it = ((m*4 + b) << lg) | a
          const int items = (M << 2) << lg;
          const bool one_pass = items <= kWave;
          int64_t my_x = 0, my_addr = -1;
          int my_m = 0, my_b = 0;
          for (int i0 = 0; i0 < items; i0 += kWave) {
            const int it = i0 + l;
            const int a = it & ((1 << lg) - 1);
            const int b = (it >> lg) & 3;
            const int m = it >> (lg + 2);
            const bool act = it < items && b < nb;
            const int64_t abase = b == 0 ? ab0 : (b == 1 ? ab1 : ab2);
            const int64_t addr = (abase + ((int64_t)(a >> sh) << dmax) + (a & wmask)) * M + m;
            const int64_t x = act ? vld(&sp.vf[addr]) : kInf;
            const uint64_t infm = __ballot(act && x == kInf);
            const int64_t fin = seg_max64((act && x != kInf) ? x : INT64_MIN, lg);
            if (act && a == (1 << lg) - 1) {         // last lane of the (m, b) segment
              const uint64_t segm = lg == 6 ? ~0ull : (((1ull << (1 << lg)) - 1ull) << (l + 1 - (1 << lg)));
              const int miss = __popcll(infm & segm);
              int64_t rdy = fin;
              if (miss > 0) rdy = max64(rdy, T + s_xfer[miss * xs]);
              s_rdy[b][m] = rdy;
              s_miss[b][m] = miss;
            }
            if (one_pass) {
              my_x = x;
              my_addr = act ? addr : -1;
              my_m = m;
              my_b = b;
            }
          }
          __syncthreads();
          int64_t est = T > avail ? T : avail;
          if (l < P)
            for (int b = 0; b < nb; b++) est = max64(est, s_rdy[b][pmem]);
          const int64_t eft = est + s_cost[ptype][kind][lvl];
          const int64_t key = l < P ? ((eft << 6) | l) : kInf;
          const int64_t best = wave_min64(key);
          const int pstar = (int)(best & 63);
          const int64_t eft_star = best >> 6;
          const int64_t est_star = rdl64(est, pstar);
          const int mstar = rdl32(pmem, pstar);
          // transfers of the missing finest blocks start now
          if (one_pass) {
            if (my_addr >= 0 && my_m == mstar && my_x == kInf)
              sp.vf[my_addr] = T + s_xfer[s_miss[my_b][mstar] * xs];
          } else {
            for (int b = 0; b < nb; b++) {
              const int miss = s_miss[b][mstar];
              if (miss == 0) continue;
              const int64_t arrive = T + s_xfer[miss * xs];
              const int64_t abase = b == 0 ? ab0 : (b == 1 ? ab1 : ab2);
              for (int a0 = 0; a0 < (1 << lg); a0 += kWave) {
                const int a = a0 + l;
                if (a < (1 << lg)) {
                  const int64_t addr = (abase + ((int64_t)(a >> sh) << dmax) + (a & wmask)) * M + mstar;
                  if (vld(&sp.vf[addr]) == kInf) sp.vf[addr] = arrive;
                }
              }
            }
          }
          // append to the chosen processor's queue
          if (l == pstar) {
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
          if (want_sched && l == 0) {
            out.proc[sbase + t] = pstar;
            out.start[sbase + t] = est_star;
            out.finish[sbase + t] = eft_star;
          }
          __syncthreads();
        }
        n_ready = 0;
      }

      // (ii) next event: the earliest queue head
      const int64_t Tn = wave_min64(l < P ? hfin : kInf);
      if (Tn == kInf) break;

      // (iii) completions at Tn; the next queue entries are fetched first
      const uint64_t cm = __ballot(l < P && hfin == Tn);
      const bool adv = (cm >> l) & 1ull;
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
        const int ms = rdl32(pmem, p);
        const uint32_t dsc = (uint32_t)rdl32((int)hdesc, p);
        const uint32_t e0 = (uint32_t)rdl32((int)he0, p);
        const uint32_t e1 = (uint32_t)rdl32((int)he1, p);
        const int lvl = desc_level(dsc);
        const int sh = dmax - lvl, lg = 2 * sh, wmask = (1 << sh) - 1;
        int br[3], bc[3];
        const int nb = desc_blocks(dsc, br, bc);
        // write-back: the written block is valid only where it was computed
        const int64_t abase = atom_base(nt, dmax, lvl, br[nb - 1], bc[nb - 1]);
        const int items = M << lg;
        for (int i0 = 0; i0 < items; i0 += kWave) {
          const int it = i0 + l;
          if (it < items) {
            const int m = it >> lg, a = it & ((1 << lg) - 1);
            const int64_t atom = abase + ((int64_t)(a >> sh) << dmax) + (a & wmask);
            sp.vf[atom * M + m] = (m == ms) ? Tn : kInf;
          }
        }
        // release successors (their records are fetched alongside the decrement)
        for (uint32_t e = e0; e < e1; e += kWave) {
          const uint32_t ee = e + l;
          bool rel = false;
          uint32_t v = 0;
          int64_t r0 = 0, r1 = 0, r3 = 0;
          if (ee < e1) {
            v = vld(&sp.succ[ee]);
            r0 = vld(&sp.rec[2 * v]);
            r1 = vld(&sp.rec[2 * v + 1]);
            r3 = vld(&sp.rec[2 * v + 3]);
            rel = atomicSub(&sp.indeg[v], 1u) == 1u;
          }
          const uint64_t rm = __ballot(rel);
          if (rel) push(n_ready + __popcll(rm & lanes_below()), v, r0, r1, r3);
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
      __syncthreads();
      T = Tn;
    }
    if (l == 0) {
      out.makespan[c] = T;
      out.status[c] = kOK;
    }
  }
}

// ---------------------------------------------------------------- generation

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kPurposeDepth = 2, kPurposeShape = 3;

__device__ __forceinline__ uint64_t draw(uint64_t seed, int purpose, uint64_t idx) {
  const uint64_t s = mix64(seed + kGamma * (uint64_t)(purpose + 1));
  return mix64(s + kGamma * (idx + 1));
}

__device__ __forceinline__ uint8_t depth_of_draw(uint64_t u, uint32_t thr, int dmax) {
  int d = 0;
  for (int j = 0; j < 3 && d < dmax; j++) {
    const uint32_t ch = (uint32_t)((u >> (21 * j)) & 0x1FFFFFull);
    if (ch < thr) d++;
    else break;
  }
  return (uint8_t)d;
}

__global__ void k_gen_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t n_top, int32_t dmax,
                              uint32_t thr, uint8_t* depth) {
  const int64_t total = (int64_t)n_cand * n_top;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = x / n_top, t = x % n_top;
    const uint64_t u = draw(seed, kPurposeDepth, ((uint64_t)(first + c) << 24) | (uint64_t)t);
    depth[x] = depth_of_draw(u, thr, dmax);
  }
}

__global__ void k_gen_shape(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt_lo, int32_t nt_hi,
                            int32_t dmax_hi, int32_t* nt, int32_t* dmax, int64_t* tops) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cand) return;
  const uint64_t u = draw(seed, kPurposeShape, (uint64_t)(first + c));
  const int n = nt_lo + (int)(u % (uint64_t)(nt_hi - nt_lo + 1));
  nt[c] = n;
  dmax[c] = (int)((u >> 32) % (uint64_t)(dmax_hi + 1));
  tops[c] = tet3(n);
}

// single-workgroup exclusive scan: off[0] = 0, off[c+1] = off[c] + v[c]
__global__ void __launch_bounds__(1024) k_scan_excl(const int64_t* v, int32_t n, int64_t* off) {
  __shared__ int64_t s_part[16];
  __shared__ int64_t s_carry;
  if (threadIdx.x == 0) { s_carry = 0; off[0] = 0; }
  __syncthreads();
  const int l = lane(), wv = threadIdx.x / kWave;
  for (int base = 0; base < n; base += 1024) {
    const int i = base + threadIdx.x;
    int64_t x = i < n ? v[i] : 0;
    int64_t incl = x;
    for (int o = 1; o < kWave; o <<= 1) {
      int64_t y = __shfl_up(incl, o, kWave);
      if (l >= o) incl += y;
    }
    if (l == kWave - 1) s_part[wv] = incl;
    __syncthreads();
    int64_t pre = s_carry;
    for (int q = 0; q < wv; q++) pre += s_part[q];
    if (i < n) off[i + 1] = pre + incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t s = 0;
      for (int q = 0; q < 16; q++) s += s_part[q];
      s_carry += s;
    }
    __syncthreads();
  }
}

__global__ void k_gen_ragged_depth(uint64_t seed, int64_t first, BatchView b, uint32_t thr, uint8_t* depth) {
  const int c = blockIdx.x;
  if (c >= b.n_cand) return;
  const int nt = b.nt_arr[c], dmax = b.dmax_arr[c];
  const int64_t n_top = tet3(nt), o = b.off[c];
  for (int64_t t = threadIdx.x; t < n_top; t += blockDim.x) {
    const uint64_t u = draw(seed, kPurposeDepth, ((uint64_t)(first + c) << 24) | (uint64_t)t);
    depth[o + t] = depth_of_draw(u, thr, dmax);
  }
}

// ---------------------------------------------------------------- reductions

__global__ void __launch_bounds__(1024) k_argmin(const int64_t* v, int32_t n, int64_t* best) {
  __shared__ int64_t s_v[16];
  __shared__ int64_t s_i[16];
  int64_t bv = kInf, bi = -1;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int64_t x = v[i];
    if (x >= 0 && (x < bv || (x == bv && i < bi))) { bv = x; bi = i; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t ov = __shfl_xor(bv, o, kWave), oi = __shfl_xor(bi, o, kWave);
    if (oi >= 0 && (ov < bv || (ov == bv && (bi < 0 || oi < bi)))) { bv = ov; bi = oi; }
  }
  const int wv = threadIdx.x / kWave;
  if (lane() == 0) { s_v[wv] = bv; s_i[wv] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t rv = kInf, ri = -1;
    for (int q = 0; q < (int)(blockDim.x / kWave); q++)
      if (s_i[q] >= 0 && (s_v[q] < rv || (s_v[q] == rv && s_i[q] < ri))) { rv = s_v[q]; ri = s_i[q]; }
    best[0] = ri >= 0 ? rv : -1;
    best[1] = ri;
  }
}

__global__ void __launch_bounds__(1024) k_max2(const int32_t* a, const int64_t* b, int32_t n, int64_t* out2) {
  __shared__ int64_t s_a[16], s_b[16];
  int64_t ma = 0, mb = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    ma = a[i] > ma ? a[i] : ma;
    mb = b[i] > mb ? b[i] : mb;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t x = __shfl_xor(ma, o, kWave), y = __shfl_xor(mb, o, kWave);
    ma = x > ma ? x : ma;
    mb = y > mb ? y : mb;
  }
  const int wv = threadIdx.x / kWave;
  if (lane() == 0) { s_a[wv] = ma; s_b[wv] = mb; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t ra = 0, rb = 0;
    for (int q = 0; q < (int)(blockDim.x / kWave); q++) {
      ra = s_a[q] > ra ? s_a[q] : ra;
      rb = s_b[q] > rb ? s_b[q] : rb;
    }
    out2[0] = ra;
    out2[1] = rb;
  }
}

__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

}  // namespace

// ---------------------------------------------------------------- launchers

Workspace make_workspace_layout(int64_t cap_tasks, int64_t cap_edges, int64_t cap_tops, int64_t cap_vf) {
  Workspace w{};
  auto al = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
  int64_t o = 0;
  w.o_top_first = o; o = al(o + 4 * (cap_tops + 1));
  w.o_desc = o;      o = al(o + 4 * cap_tasks);
  w.o_rec = o;       o = al(o + 16 * (cap_tasks + 1));
  w.o_indeg = o;     o = al(o + 4 * cap_tasks);
  w.o_cur = o;       o = al(o + 4 * cap_tasks);
  w.o_succ = o;      o = al(o + 4 * (cap_edges > 0 ? cap_edges : 1));
  w.o_fifo = o;      o = al(o + 24 * cap_tasks);
  w.o_ready = o;     o = al(o + 4 * cap_tasks);
  int64_t n2 = 1;
  while (n2 < cap_tasks) n2 <<= 1;
  w.o_sort = o;      o = al(o + 16 * n2);
  w.o_vf = o;        o = al(o + 8 * cap_vf);
  w.stride = o;
  w.cap_tasks = cap_tasks;
  w.cap_edges = cap_edges;
  w.cap_tops = cap_tops;
  w.cap_vf = cap_vf;
  return w;
}

hipError_t launch_count(const BatchView& b, int32_t* n_tasks, int64_t* n_edges, hipStream_t s) {
  if (b.n_cand <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count, dim3(b.n_cand), dim3(kWave), 0, s, b, n_tasks, n_edges);
  return hipGetLastError();
}

hipError_t launch_simulate(const SimTables& t, const BatchView& b, const Workspace& w, const OutView& o,
                           int32_t slots, uint32_t* counter, hipStream_t s) {
  if (b.n_cand <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int g = slots < b.n_cand ? slots : b.n_cand;
  hipLaunchKernelGGL(k_simulate, dim3(g), dim3(kWave), 0, s, t, b, w, o, counter);
  return hipGetLastError();
}

hipError_t launch_gen_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt, int32_t dmax,
                              uint32_t thr, uint8_t* depth, hipStream_t s) {
  if (n_cand <= 0) return hipSuccess;
  const int64_t total = (int64_t)n_cand * tet3(nt);
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gen_uniform, dim3((unsigned)blocks), dim3(256), 0, s, seed, first, n_cand,
                     (int32_t)tet3(nt), dmax, thr, depth);
  return hipGetLastError();
}

hipError_t launch_gen_shape(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt_lo, int32_t nt_hi,
                            int32_t dmax_hi, int32_t* nt, int32_t* dmax, int64_t* off, hipStream_t s) {
  if (n_cand <= 0) {
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, (const int64_t*)nullptr, 0, off);
    return hipGetLastError();
  }
  // off[1..n] first holds tet(nt_c), then is scanned in place from a copy
  int64_t* tops = off + 1;
  hipLaunchKernelGGL(k_gen_shape, dim3((n_cand + 255) / 256), dim3(256), 0, s, seed, first, n_cand, nt_lo,
                     nt_hi, dmax_hi, nt, dmax, tops);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // in-place scan: each 1024-chunk reads its inputs before writing (one workgroup, ordered)
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, (const int64_t*)tops, n_cand, off);
  return hipGetLastError();
}

hipError_t launch_gen_ragged_depth(uint64_t seed, int64_t first, const BatchView& b, uint32_t thr,
                                   uint8_t* depth, hipStream_t s) {
  if (b.n_cand <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gen_ragged_depth, dim3(b.n_cand), dim3(256), 0, s, seed, first, b, thr, depth);
  return hipGetLastError();
}

hipError_t launch_argmin(const int64_t* v, int32_t n, int64_t* best, hipStream_t s) {
  hipLaunchKernelGGL(k_argmin, dim3(1), dim3(1024), 0, s, v, n, best);
  return hipGetLastError();
}

hipError_t launch_max_i32_i64(const int32_t* a, const int64_t* b, int32_t n, int64_t* out2, hipStream_t s) {
  hipLaunchKernelGGL(k_max2, dim3(1), dim3(1024), 0, s, a, b, n, out2);
  return hipGetLastError();
}

}  // namespace hesp
