// hesp_grain.hip -- grain batches: every top-level task of the Fig. 1 loop nest
// is split with its own integer factor f (partition parameter p = 1/f, section
// 2.1), so that the blocks of two tasks whose factors do not divide each other
// overlap partially (the intersection blocks of the data DAG, Fig. 4).
//
// Every tile is cut into L x L atoms, L = lcm of the factors; a block of factor
// f is the union of its (L/f)^2 atoms, and the intersection of two blocks is the
// set of atoms they share, so validity and dependences are kept per atom.
//
// One wavefront per candidate, in its own slot of the caller's workspace:
//   1. expansion and dependences: fine tasks in program order (top-level task
//      by top-level task, each by increasing K, Fig. 1 order inside), every
//      task linked to the last writer of each atom it touches (RaW and WaW;
//      every block is final before it is first read, so no WaR hazard exists,
//      and a violation is reported instead of being ignored);
//   2. successor lists (counting sort of the edges by source);
//   3. critical times (section 2.1, "Priority-List": task time summed over the
//      processors, longest path to an exit), reverse program order;
//   4. the event simulation of section 2.1: every released task is mapped at its
//      release in Priority-List or FCFS order (ties by the task's first atom),
//      onto the processor of earliest finish (EFT-P, counting the transfers of
//      the atoms missing in its memory space) or earliest idle time (EIT-P);
//      write-back, write-through or write-around caching of written blocks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp.h"

extern "C" int hesp_internal_fail(int code, const char* msg);

namespace {

constexpr int kGMaxFac = HESP_GRAIN_MAX_FAC;
constexpr int kGMaxMem = HESP_GRAIN_MAX_MEM;
constexpr int kGMaxProcs = HESP_MAX_PROCS;
constexpr int kGMaxPtypes = HESP_MAX_PTYPES;
constexpr int kGMaxL = HESP_GRAIN_MAX_ATOMS;
constexpr int64_t kInf = INT64_MAX;
constexpr int64_t kNegInf = INT64_MIN;
enum : int { CHOL = 0, TRSM = 1, SYRK = 2, GEMM = 3 };

struct GrainTables {
  int32_t nt, n_top, n_fac, L, n_procs, n_mem, fcfs, sel, cache;
  int32_t fac[kGMaxFac];
  int8_t proc_type[kGMaxProcs];
  int8_t proc_mem[kGMaxProcs];
  int64_t cost[kGMaxPtypes][4][kGMaxFac];   // task time, ns
  int64_t W[4][kGMaxFac];                   // task time summed over the processors
  const int64_t* xfer;                      // [L*L + 1]: transfer time of k atoms
};

// byte offsets of the arrays of one slot, and its capacities
struct SlotLayout {
  int64_t last_w, last_r, vf, rec, rank, finish, left, succ_ptr, cur, mark, next, ready, pred_ptr, pred, pred_v,
      succ, bytes;
  int64_t max_tasks, max_edges, atoms;
};

constexpr int64_t up256(int64_t x) { return (x + 255) & ~(int64_t)255; }

int64_t fine_count(int kind, int64_t f) {
  if (kind == CHOL) return f * (f + 1) * (f + 2) / 6;
  if (kind == GEMM) return f * f * f;
  return f * f * (f + 1) / 2;
}

int64_t gcd64(int64_t a, int64_t b) {
  while (b) { int64_t t = a % b; a = b; b = t; }
  return a;
}

// L = lcm(fac), or 0 when a factor or L is out of range
int atoms_per_side(int n_fac, const int32_t* fac) {
  if (n_fac < 1 || n_fac > kGMaxFac || !fac) return 0;
  int64_t L = 1;
  for (int g = 0; g < n_fac; g++) {
    if (fac[g] < 1 || fac[g] > kGMaxL) return 0;
    L = L / gcd64(L, fac[g]) * fac[g];
    if (L > kGMaxL) return 0;
  }
  return (int)L;
}

// capacities: tasks of the largest expansion; edges at most one per atom a task
// touches (each atom has one last writer)
SlotLayout layout(int nt, int n_fac, const int32_t* fac, int L, int n_mem) {
  SlotLayout s{};
  const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
  s.atoms = tiles * L * L;
  int64_t nk[4] = {nt, (int64_t)nt * (nt - 1) / 2, (int64_t)nt * (nt - 1) / 2, 0};
  nk[GEMM] = (int64_t)nt * (nt + 1) * (nt + 2) / 6 - nk[CHOL] - nk[TRSM] - nk[SYRK];
  for (int kind = 0; kind < 4; kind++) {
    int64_t bt = 0, be = 0;
    for (int g = 0; g < n_fac; g++) {
      const int64_t w = L / fac[g], n = fine_count(kind, fac[g]);
      if (n > bt) bt = n;
      if (3 * n * w * w > be) be = 3 * n * w * w;
    }
    s.max_tasks += nk[kind] * bt;
    s.max_edges += nk[kind] * be;
  }
  const int64_t n = s.max_tasks, e = s.max_edges;
  int64_t o = 0;
  auto take = [&](int64_t bytes) { int64_t at = o; o += up256(bytes); return at; };
  s.last_w = take(4 * s.atoms);
  s.last_r = take(4 * s.atoms);
  s.vf = take(8 * s.atoms * n_mem);
  s.rec = take(8 * n);
  s.rank = take(8 * n);
  s.finish = take(8 * n);
  s.left = take(4 * n);
  s.succ_ptr = take(4 * (n + 1));
  s.cur = take(4 * n);
  s.mark = take(4 * n);
  s.next = take(4 * n);
  s.ready = take(32 * n);
  s.pred_ptr = take(4 * (n + 1));
  s.pred = take(4 * e);
  s.pred_v = take(4 * e);
  s.succ = take(4 * e);
  s.bytes = o;
  return s;
}

// ---------------------------------------------------------------- device side

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// The arrays of a slot are written and read by the lanes of one wavefront (one
// workgroup); loads go through the vector path at workgroup scope, and arrays
// updated by atomics (performed in L2) are read at device scope.
template <class T>
__device__ __forceinline__ T ld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <class T>
__device__ __forceinline__ T ld2(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t wmax64(int64_t v) {
  for (int o = 32; o; o >>= 1) { int64_t u = __shfl_xor(v, o); v = u > v ? u : v; }
  return v;
}
__device__ __forceinline__ int64_t wmin64(int64_t v) {
  for (int o = 32; o; o >>= 1) { int64_t u = __shfl_xor(v, o); v = u < v ? u : v; }
  return v;
}
__device__ __forceinline__ int wsum(int v) {
  for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// task record: kind | grain << 2 | K << 5 | I << 17 | J << 29 (fine indices < 4096)
__device__ __forceinline__ uint64_t pack_rec(int kind, int g, int K, int I, int J) {
  return (uint64_t)kind | ((uint64_t)g << 2) | ((uint64_t)K << 5) | ((uint64_t)I << 17) | ((uint64_t)J << 29);
}
struct Task {
  int kind, g, K, I, J;
};
__device__ __forceinline__ Task unpack_rec(uint64_t r) {
  return Task{(int)(r & 3), (int)((r >> 2) & 7), (int)((r >> 5) & 4095), (int)((r >> 17) & 4095),
              (int)((r >> 29) & 4095)};
}

// data blocks of a fine task (row, col at its factor); the written one is last
__device__ __forceinline__ int task_blocks(const Task& t, int* br, int* bc) {
  switch (t.kind) {
    case CHOL: br[0] = t.K; bc[0] = t.K; return 1;
    case TRSM: br[0] = t.K; bc[0] = t.K; br[1] = t.K; bc[1] = t.J; return 2;
    case SYRK: br[0] = t.K; bc[0] = t.I; br[1] = t.I; bc[1] = t.I; return 2;
    default: br[0] = t.K; bc[0] = t.I; br[1] = t.K; bc[1] = t.J; br[2] = t.I; bc[2] = t.J; return 3;
  }
}

struct Slot {
  int32_t *last_w, *last_r;
  int64_t* vf;
  uint64_t* rec;
  int64_t *rank, *finish;
  uint32_t *left, *succ_ptr, *cur;
  int32_t *mark, *next;
  uint32_t *ready, *pred_ptr, *pred, *pred_v, *succ;
};

// atom (row, col) of the whole N x N atom grid: tiles of the upper triangle row
// by row, L x L atoms each, row-major inside the tile
__device__ __forceinline__ int64_t atom_of(int row, int col, int L, int nt) {
  const int tr = row / L, tc = col / L;
  const int64_t tile = (int64_t)tr * nt - (int64_t)tr * (tr - 1) / 2 + (tc - tr);
  return (tile * L + (row - tr * L)) * L + (col - tc * L);
}

// block bi's x-th atom (row-major inside the block of side w)
__device__ __forceinline__ int64_t block_atom(const int* br, const int* bc, int bi, int x, int w, int L, int nt) {
  const int u = x / w, v = x - u * w;
  return atom_of(br[bi] * w + u, bc[bi] * w + v, L, nt);
}

struct ScanState {
  uint32_t t;        // tasks emitted
  uint32_t ne;       // edges emitted
  int err;           // 0, or a status
};

constexpr int kSet = 256;   // LDS set of a task's distinct predecessors (when its atoms fit)

__device__ void visit(const GrainTables& tb, const SlotLayout& lay, const Slot& s, ScanState& st, int kind, int g,
                      int K, int I, int J, uint32_t* lds_cnt, int32_t* set) {
  const uint32_t t = st.t;
  if ((int64_t)t >= lay.max_tasks) { st.err = HESP_ECAPACITY; return; }
  const Task tk{kind, g, K, I, J};
  int br[3], bc[3];
  const int nb = task_blocks(tk, br, bc);
  const int w = tb.L / tb.fac[g], per = w * w;
  // at most kSet atoms: distinct predecessors found in an LDS hash set, else
  // through the per-task marks in memory
  const bool in_lds = nb * per <= kSet;
  if (lane() == 0) {
    *lds_cnt = 0;
    s.rec[t] = pack_rec(kind, g, K, I, J);
    s.pred_ptr[t] = st.ne;
    __hip_atomic_store(&s.mark[t], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (in_lds)
    for (int i = lane(); i < kSet; i += 64) set[i] = -1;
  __syncthreads();
  // one pass over the atoms of every block (blocks of one task are disjoint):
  // the last writer of each atom is a predecessor (once); a read marks the atom,
  // the written block takes the task as last writer, and a read of it since its
  // last write would be a WaR hazard
  int war = 0;
  for (int x = lane(); x < nb * per; x += 64) {
    const int bi = x / per;
    const int64_t a = block_atom(br, bc, bi, x - bi * per, w, tb.L, tb.nt);
    const int32_t lw = ld(&s.last_w[a]);
    const bool wr = bi == nb - 1;
    const int32_t lr = wr ? ld(&s.last_r[a]) : -1;
    if (lw >= 0 && (uint32_t)lw != t) {
      bool fresh;
      if (in_lds) {
        // open addressing; the set holds at most nb * per <= kSet keys
        uint32_t h = ((uint32_t)lw * 2654435761u) >> 24;
        for (;;) {
          const int32_t old = atomicCAS(&set[h], -1, lw);
          if (old == -1) { fresh = true; break; }
          if (old == lw) { fresh = false; break; }
          h = (h + 1) & (kSet - 1);
        }
      } else {
        fresh = atomicExch(&s.mark[lw], (int32_t)t) != (int32_t)t;
      }
      if (fresh) {
        const uint32_t pos = atomicAdd(lds_cnt, 1u);
        s.pred[st.ne + pos] = (uint32_t)lw;
        s.pred_v[st.ne + pos] = t;
      }
    }
    if (wr) {
      war |= lr >= 0 && (uint32_t)lr != t;
      s.last_r[a] = -1;
      s.last_w[a] = (int32_t)t;
    } else {
      s.last_r[a] = (int32_t)t;
    }
  }
  __syncthreads();
  const uint32_t np = *lds_cnt;
  if (wsum(war)) st.err = HESP_EINVAL;
  if (st.ne + np > lay.max_edges) st.err = HESP_ECAPACITY;
  if (lane() == 0) s.left[t] = np;
  st.ne += np;
  st.t = t + 1;
}

// the fine tasks of top-level cell (k, i, j) at factor f, in right-looking order
__device__ void emit_cell(const GrainTables& tb, const SlotLayout& lay, const Slot& s, ScanState& st, int g,
                          int k, int i, int j, uint32_t* lds_cnt, int32_t* set) {
  const int f = tb.fac[g];
  const int ks = k * f, is = i * f, js = j * f;
  for (int K = ks; K < ks + f && !st.err; K++) {
    const bool kin_i = K >= is && K < is + f, kin_j = K >= js && K < js + f;
    if (kin_i && kin_j) visit(tb, lay, s, st, CHOL, g, K, K, K, lds_cnt, set);
    if (kin_i)
      for (int J = (K + 1 > js ? K + 1 : js); J < js + f && !st.err; J++) visit(tb, lay, s, st, TRSM, g, K, K, J, lds_cnt, set);
    for (int I = (K + 1 > is ? K + 1 : is); I < is + f && !st.err; I++) {
      for (int J = (I + 1 > js ? I + 1 : js); J < js + f && !st.err; J++) visit(tb, lay, s, st, GEMM, g, K, I, J, lds_cnt, set);
      if (I >= js && I < js + f && !st.err) visit(tb, lay, s, st, SYRK, g, K, I, I, lds_cnt, set);
    }
  }
}

__device__ int expand_scan(const GrainTables& tb, const SlotLayout& lay, const Slot& s, const uint8_t* grain,
                           ScanState& st, uint32_t* lds_cnt, int32_t* set) {
  for (int64_t a = lane(); a < lay.atoms; a += 64) { s.last_w[a] = -1; s.last_r[a] = -1; }
  __syncthreads();
  st.t = 0; st.ne = 0; st.err = 0;
  int top = 0;
  auto cell = [&](int k, int i, int j) {
    const int g = grain[top++];
    if (g >= tb.n_fac) { st.err = HESP_EINVAL; return; }
    emit_cell(tb, lay, s, st, g, k, i, j, lds_cnt, set);
  };
  const int nt = tb.nt;
  for (int k = 0; k < nt && !st.err; k++) {
    cell(k, k, k);
    for (int j = k + 1; j < nt && !st.err; j++) cell(k, k, j);
    for (int i = k + 1; i < nt && !st.err; i++) {
      for (int j = i + 1; j < nt && !st.err; j++) cell(k, i, j);
      if (!st.err) cell(k, i, i);
    }
  }
  if (lane() == 0) s.pred_ptr[st.t] = st.ne;
  __syncthreads();
  return st.err;
}

// successor lists: count per source, exclusive scan, scatter
__device__ void successors(const Slot& s, uint32_t n, uint32_t ne) {
  for (uint32_t t = lane(); t < n; t += 64) s.cur[t] = 0;
  __syncthreads();
  for (uint32_t e = lane(); e < ne; e += 64) atomicAdd(&s.cur[ld(&s.pred[e])], 1u);
  __syncthreads();
  uint32_t run = 0;
  for (uint32_t t0 = 0; t0 < n; t0 += 64) {
    const uint32_t t = t0 + lane();
    const uint32_t c = t < n ? ld2(&s.cur[t]) : 0u;
    uint32_t inc = c;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t u = __shfl_up(inc, o);
      if (lane() >= o) inc += u;
    }
    if (t < n) {
      s.succ_ptr[t] = run + inc - c;
      __hip_atomic_store(&s.cur[t], run + inc - c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    run += __shfl(inc, 63);
  }
  if (lane() == 0) s.succ_ptr[n] = run;
  __syncthreads();
  for (uint32_t e = lane(); e < ne; e += 64) {
    const uint32_t u = ld(&s.pred[e]), v = ld(&s.pred_v[e]);
    const uint32_t pos = atomicAdd(&s.cur[u], 1u);
    s.succ[pos] = v;
  }
  __syncthreads();
}

// critical times, reverse program order (every edge points forward), 64 tasks
// at a time: their successor ranges and own times are loaded together, and the
// ranks computed in the chunk stay in the lanes' registers
__device__ void ranks(const GrainTables& tb, const Slot& s, uint32_t n) {
  for (int64_t hi = n; hi > 0; hi -= 64) {
    const int64_t lo = hi > 64 ? hi - 64 : 0;
    const int64_t tl = lo + lane();
    uint32_t ep0 = 0, ep1 = 0;
    int64_t wl = 0, myrank = 0;
    if (tl < hi) {
      ep0 = ld(&s.succ_ptr[tl]);
      ep1 = ld(&s.succ_ptr[tl + 1]);
      const Task tk = unpack_rec(ld(&s.rec[tl]));
      wl = tb.W[tk.kind][tk.g];
    }
    for (int64_t t = hi - 1; t >= lo; t--) {
      const int j = (int)(t - lo);
      const uint32_t e0 = __shfl(ep0, j), e1 = __shfl(ep1, j);
      int64_t best = 0;
      for (uint32_t eb = e0; eb < e1; eb += 64) {
        const uint32_t e = eb + lane();
        const int64_t sv = e < e1 ? (int64_t)ld(&s.succ[e]) : -1;
        const int inside = sv >= lo && sv < hi;
        const int64_t rin = __shfl(myrank, inside ? (int)(sv - lo) : 0);
        const int64_t r = sv < 0 ? 0 : (inside ? rin : ld(&s.rank[sv]));
        best = r > best ? r : best;
      }
      best = wmax64(best);
      const int64_t r = __shfl(wl, j) + best;
      if (lane() == j) myrank = r;
    }
    if (tl < hi) s.rank[tl] = myrank;
    __syncthreads();
  }
}

// ready-set order: larger key first, then the smaller first atom (K', I', J')
__device__ __forceinline__ uint32_t corner(const GrainTables& tb, const Task& tk) {
  const uint32_t w = (uint32_t)(tb.L / tb.fac[tk.g]);
  return ((uint32_t)tk.K * w << 18) | ((uint32_t)tk.I * w << 9) | ((uint32_t)tk.J * w);
}

// a released task: ordering key, (first atom << 32 | task), record
struct Entry {
  int64_t key;
  uint64_t cid, rec, pad;
};
__device__ __forceinline__ Entry load_entry(const Entry* p) {
  const uint64_t* q = (const uint64_t*)p;
  return Entry{(int64_t)ld(q), ld(q + 1), ld(q + 2), 0};
}
__device__ __forceinline__ void store_entry(Entry* p, const Entry& e) {
  uint64_t* q = (uint64_t*)p;
  q[0] = (uint64_t)e.key; q[1] = e.cid; q[2] = e.rec;
}
__device__ __forceinline__ Entry make_entry(const GrainTables& tb, const Slot& s, uint32_t v) {
  const uint64_t rec = ld(&s.rec[v]);
  const int64_t key = tb.fcfs ? 0 : ld(&s.rank[v]);
  return Entry{key, ((uint64_t)corner(tb, unpack_rec(rec)) << 32) | v, rec, 0};
}

__device__ int simulate(const GrainTables& tb, const Slot& s, uint32_t n, int64_t& makespan,
                        int* s_miss, int64_t* s_fin, int64_t* s_go) {
  const int P = tb.n_procs, M = tb.n_mem, L = tb.L, nt = tb.nt;
  Entry* ready = (Entry*)s.ready;
  for (int64_t a = lane(); a < (int64_t)nt * (nt + 1) / 2 * L * L; a += 64)
    for (int m = 0; m < M; m++) s.vf[a * M + m] = m == 0 ? 0 : kInf;   // data starts on the host
  // ready set: the tasks without predecessors
  uint32_t nb = 0;
  for (uint32_t t0 = 0; t0 < n; t0 += 64) {
    const uint32_t t = t0 + lane();
    const bool r = t < n && ld(&s.left[t]) == 0u;
    const uint64_t m = __ballot(r);
    if (r) store_entry(&ready[nb + __popcll(m & ((1ull << lane()) - 1))], make_entry(tb, s, t));
    nb += (uint32_t)__popcll(m);
  }
  __syncthreads();
  // processor lanes: queue head (task, finish, record) and tail, idle time
  const bool is_p = lane() < P;
  const int my_mem = is_p ? tb.proc_mem[lane()] : 0;
  const int my_type = is_p ? tb.proc_type[lane()] : 0;
  int64_t avail = 0, headfin = kInf;
  uint64_t headrec = 0;
  int32_t head = -1, tail = -1;
  int64_t T = 0;
  uint32_t done = 0;
  makespan = 0;
  for (;;) {
    // (i) map the released tasks, in order
    while (nb > 0) {
      int64_t bk = kNegInf;
      int64_t bcid = kInf;
      uint64_t brec = 0;
      uint32_t bi = 0;
      Entry le{0, 0, 0, 0};
      for (uint32_t i = lane(); i < nb; i += 64) {
        const Entry e = load_entry(&ready[i]);
        le = e;
        if (e.key > bk || (e.key == bk && (int64_t)e.cid < bcid)) { bk = e.key; bcid = (int64_t)e.cid; brec = e.rec; bi = i; }
      }
      const int64_t kmax = wmax64(bk);
      const int64_t cmin = wmin64(bk == kmax ? bcid : kInf);
      const int src = __ffsll((unsigned long long)__ballot(bk == kmax && bcid == cmin)) - 1;
      const uint32_t pick = __shfl(bi, src);
      const uint32_t t = (uint32_t)(uint64_t)cmin;
      const uint64_t rec = __shfl(brec, src);
      const int ll = (int)((nb - 1) & 63);
      const Entry last{__shfl(le.key, ll), __shfl(le.cid, ll), __shfl(le.rec, ll), 0};
      if (lane() == 0 && pick != nb - 1) store_entry(&ready[pick], last);
      nb--;
      const Task tk = unpack_rec(rec);
      int br[3], bc3[3];
      const int nbk = task_blocks(tk, br, bc3);
      const int w = L / tb.fac[tk.g], per = w * w;
      // per block and memory space: atoms missing, latest valid-from of those
      // present, latest time a missing atom has a copy somewhere
      if (lane() < 3 * kGMaxMem) { s_miss[lane()] = 0; s_fin[lane()] = kNegInf; s_go[lane()] = kNegInf; }
      __syncthreads();
      for (int x = lane(); x < nbk * per; x += 64) {
        const int b = x / per;
        const int64_t a = block_atom(br, bc3, b, x - b * per, w, L, nt);
        int64_t v[kGMaxMem], src_t = kInf;
#pragma unroll
        for (int m = 0; m < kGMaxMem; m++)
          if (m < M) { v[m] = ld(&s.vf[a * M + m]); src_t = v[m] < src_t ? v[m] : src_t; }
#pragma unroll
        for (int m = 0; m < kGMaxMem; m++)
          if (m < M) {
            if (v[m] == kInf) {
              atomicAdd(&s_miss[b * kGMaxMem + m], 1);
              if (src_t != kInf) atomicMax((long long*)&s_go[b * kGMaxMem + m], (long long)src_t);
            } else {
              atomicMax((long long*)&s_fin[b * kGMaxMem + m], (long long)v[m]);
            }
          }
      }
      __syncthreads();
      // every processor's estimate
      int64_t est = T > avail ? T : avail;
      for (int b = 0; b < nbk; b++) {
        const int ms = s_miss[b * kGMaxMem + my_mem];
        int64_t rdy = s_fin[b * kGMaxMem + my_mem];
        if (ms > 0) {
          int64_t g0 = s_go[b * kGMaxMem + my_mem];
          g0 = g0 > T ? g0 : T;
          const int64_t arr = g0 + tb.xfer[ms];
          rdy = arr > rdy ? arr : rdy;
        }
        est = rdy > est ? rdy : est;
      }
      const int64_t eft = est + tb.cost[my_type][tk.kind][tk.g];
      const int64_t sel = is_p ? (tb.sel ? (T > avail ? T : avail) : eft) : kInf;
      const int64_t smin = wmin64(sel);
      const int bp = __ffsll((unsigned long long)__ballot(is_p && sel == smin)) - 1;
      const int64_t beft = __shfl(eft, bp);
      const int bm = tb.proc_mem[bp];
      // commit: transfers of the missing atoms into the chosen space, issued now
      for (int x = lane(); x < nbk * per; x += 64) {
        const int b = x / per;
        const int ms = s_miss[b * kGMaxMem + bm];
        if (ms == 0) continue;
        int64_t g0 = s_go[b * kGMaxMem + bm];
        g0 = g0 > T ? g0 : T;
        const int64_t a = block_atom(br, bc3, b, x - b * per, w, L, nt);
        if (ld(&s.vf[a * M + bm]) == kInf) s.vf[a * M + bm] = g0 + tb.xfer[ms];
      }
      if (lane() == 0) { s.finish[t] = beft; s.next[t] = -1; }
      if (lane() == bp) {
        avail = beft;
        if (head < 0) { head = (int32_t)t; headfin = beft; headrec = rec; }
        else s.next[tail] = (int32_t)t;
        tail = (int32_t)t;
      }
      __syncthreads();
    }
    // (ii) the next event: the earliest completion at the head of a queue
    const int64_t Tn = wmin64(is_p && head >= 0 ? headfin : kInf);
    if (Tn == kInf) break;
    // (iii) every completion at Tn, processors in index order
    uint64_t fin_mask = __ballot(is_p && head >= 0 && headfin == Tn);
    while (fin_mask) {
      const int p = __ffsll((unsigned long long)fin_mask) - 1;
      fin_mask &= fin_mask - 1;
      const uint32_t t = (uint32_t)__shfl(head, p);
      const Task tk = unpack_rec(__shfl(headrec, p));
      if (lane() == p) {
        head = ld(&s.next[t]);
        if (head < 0) { tail = -1; headfin = kInf; }
        else { headfin = ld(&s.finish[head]); headrec = ld(&s.rec[head]); }
      }
      done++;
      int br[3], bc3[3];
      const int nbk = task_blocks(tk, br, bc3);
      const int w = L / tb.fac[tk.g], per = w * w, m = tb.proc_mem[p];
      // coherence of the written block: write-back keeps it where it was
      // computed; write-through there and on the host once its copy arrives;
      // write-around on the host only, once its copy arrives
      const int64_t host_at = m == 0 ? Tn : Tn + tb.xfer[per];
      for (int x = lane(); x < per; x += 64) {
        const int64_t a = block_atom(br, bc3, nbk - 1, x, w, L, nt);
        for (int mm = 0; mm < M; mm++) {
          int64_t v;
          if (tb.cache == 0) v = mm == m ? Tn : kInf;
          else if (tb.cache == 1) v = mm == m ? Tn : (mm == 0 ? host_at : kInf);
          else v = mm == 0 ? host_at : kInf;
          s.vf[a * M + mm] = v;
        }
      }
      // release the successors whose last predecessor this was
      const uint32_t e0 = ld(&s.succ_ptr[t]), e1 = ld(&s.succ_ptr[t + 1]);
      for (uint32_t e0c = e0; e0c < e1; e0c += 64) {
        const uint32_t e = e0c + lane();
        uint32_t v = 0;
        bool rel = false;
        if (e < e1) {
          v = ld(&s.succ[e]);
          rel = atomicSub(&s.left[v], 1u) == 1u;
        }
        const uint64_t mk = __ballot(rel);
        if (rel) store_entry(&ready[nb + __popcll(mk & ((1ull << lane()) - 1))], make_entry(tb, s, v));
        nb += (uint32_t)__popcll(mk);
      }
      __syncthreads();
    }
    T = Tn;
    makespan = Tn > makespan ? Tn : makespan;
  }
  return done == n ? HESP_OK : HESP_EINVAL;
}

__global__ __launch_bounds__(64) void k_grain(GrainTables tb, SlotLayout lay, const uint8_t* __restrict__ grain,
                                              int32_t n_cand, uint8_t* __restrict__ ws, int64_t* __restrict__ out_ms,
                                              int32_t* __restrict__ out_nt, int64_t* __restrict__ out_ne,
                                              int32_t* __restrict__ out_st) {
  __shared__ uint32_t lds_cnt;
  __shared__ int32_t set[kSet];
  __shared__ int s_miss[3 * kGMaxMem];
  __shared__ int64_t s_fin[3 * kGMaxMem], s_go[3 * kGMaxMem];
  uint8_t* base = ws + (int64_t)blockIdx.x * lay.bytes;
  Slot s;
  s.last_w = (int32_t*)(base + lay.last_w);
  s.last_r = (int32_t*)(base + lay.last_r);
  s.vf = (int64_t*)(base + lay.vf);
  s.rec = (uint64_t*)(base + lay.rec);
  s.rank = (int64_t*)(base + lay.rank);
  s.finish = (int64_t*)(base + lay.finish);
  s.left = (uint32_t*)(base + lay.left);
  s.succ_ptr = (uint32_t*)(base + lay.succ_ptr);
  s.cur = (uint32_t*)(base + lay.cur);
  s.mark = (int32_t*)(base + lay.mark);
  s.next = (int32_t*)(base + lay.next);
  s.ready = (uint32_t*)(base + lay.ready);
  s.pred_ptr = (uint32_t*)(base + lay.pred_ptr);
  s.pred = (uint32_t*)(base + lay.pred);
  s.pred_v = (uint32_t*)(base + lay.pred_v);
  s.succ = (uint32_t*)(base + lay.succ);
  for (int32_t c = blockIdx.x; c < n_cand; c += gridDim.x) {
    ScanState st;
    int rc = expand_scan(tb, lay, s, grain + (int64_t)c * tb.n_top, st, &lds_cnt, set);
    int64_t ms = -1;
    if (rc == HESP_OK) {
      successors(s, st.t, st.ne);
      ranks(tb, s, st.t);
      rc = simulate(tb, s, st.t, ms, s_miss, s_fin, s_go);
      if (rc != HESP_OK) ms = -1;
    }
    if (lane() == 0) {
      out_ms[c] = ms;
      if (out_nt) out_nt[c] = rc == HESP_OK ? (int32_t)st.t : 0;
      if (out_ne) out_ne[c] = rc == HESP_OK ? (int64_t)st.ne : 0;
      if (out_st) out_st[c] = rc;
    }
    __syncthreads();
  }
}

int64_t tet(int64_t n) { return n * (n + 1) * (n + 2) / 6; }

int check_batch(const hesp_grain_batch* gb, int& L) {
  if (!gb) return hesp_internal_fail(HESP_EINVAL, "grain batch: null batch");
  L = atoms_per_side(gb->n_fac, gb->fac);
  if (!L) return hesp_internal_fail(HESP_EINVAL, "grain batch: factors must be 1..64 with lcm <= 64, 1..8 of them");
  if (gb->nt < 1 || (int64_t)gb->nt * L > HESP_MAX_FINE)
    return hesp_internal_fail(HESP_EINVAL, "grain batch: nt * lcm(fac) must be 1..HESP_MAX_FINE");
  if (gb->n_cand < 0) return hesp_internal_fail(HESP_EINVAL, "grain batch: n_cand < 0");
  for (int g = 0; g < gb->n_fac; g++)
    if ((int64_t)gb->nt * gb->fac[g] > 4095) return hesp_internal_fail(HESP_EINVAL, "grain batch: nt * fac too large");
  return HESP_OK;
}

}  // namespace

extern "C" {

int hesp_grain_cost_tables(const hesp_cost_model* cm, int32_t n_fac, const int32_t* fac, int64_t* cost_ns,
                           int64_t* xfer_ns) {
  if (!cm || !cost_ns || !xfer_ns) return hesp_internal_fail(HESP_EINVAL, "hesp_grain_cost_tables: null argument");
  const int L = atoms_per_side(n_fac, fac);
  if (!L) return hesp_internal_fail(HESP_EINVAL, "hesp_grain_cost_tables: factors");
  if (cm->n_ptypes < 1 || cm->n_ptypes > HESP_MAX_PTYPES || !cm->rmax_mflops || !cm->h)
    return hesp_internal_fail(HESP_EINVAL, "hesp_grain_cost_tables: bad processor types");
  if (cm->b <= 0 || cm->b > (1 << 20) || cm->bw_bytes_per_ns <= 0 || cm->latency_ns < 0 || cm->elem_bytes <= 0)
    return hesp_internal_fail(HESP_EINVAL, "hesp_grain_cost_tables: block side or transfer model");
  static const int64_t c3[4] = {1, 3, 3, 6};  // flops * 3 / side^3
  for (int pt = 0; pt < cm->n_ptypes; pt++) {
    const int64_t h = cm->h[pt];
    if (h < 0 || h > (1 << 20)) return hesp_internal_fail(HESP_EINVAL, "hesp_grain_cost_tables: h");
    for (int ty = 0; ty < 4; ty++) {
      const int64_t rmax = cm->rmax_mflops[pt * 4 + ty];
      if (rmax <= 0) return hesp_internal_fail(HESP_EINVAL, "hesp_grain_cost_tables: rmax");
      for (int g = 0; g < n_fac; g++) {
        // side s = b/f: ceil((c/3) s^3 * 1000 (s^2 + h^2) / (rmax s^2)) in exact rationals
        const __int128 f = fac[g], b = cm->b;
        const __int128 num = (__int128)c3[ty] * 1000 * b * (b * b + f * f * h * h);
        const __int128 den = (__int128)3 * f * f * f * rmax;
        cost_ns[(pt * 4 + ty) * n_fac + g] = (int64_t)((num + den - 1) / den);
      }
    }
  }
  for (int64_t k = 0; k <= (int64_t)L * L; k++) {
    if (cm->shared_memory || k == 0) { xfer_ns[k] = 0; continue; }
    const __int128 num = (__int128)cm->elem_bytes * k * cm->b * cm->b, den = (__int128)L * L * cm->bw_bytes_per_ns;
    xfer_ns[k] = cm->latency_ns + (int64_t)((num + den - 1) / den);
  }
  return HESP_OK;
}

int hesp_grain_workspace(const hesp_grain_batch* gb, int32_t n_mem, int32_t slots, int64_t* bytes) {
  int L = 0;
  if (int rc = check_batch(gb, L)) return rc;
  if (!bytes || n_mem < 1 || n_mem > kGMaxMem || slots < 1)
    return hesp_internal_fail(HESP_EINVAL, "hesp_grain_workspace: n_mem, slots or bytes");
  const SlotLayout s = layout(gb->nt, gb->n_fac, gb->fac, L, n_mem);
  *bytes = up256(8 * ((int64_t)L * L + 1)) + (int64_t)slots * s.bytes;
  return HESP_OK;
}

int hesp_simulate_grain_batch(const hesp_platform* pf, hesp_policy policy, const hesp_grain_batch* gb,
                              int64_t* d_makespan, int32_t* d_n_tasks, int64_t* d_n_edges, int32_t* d_status,
                              void* d_ws, int64_t ws_bytes, int32_t slots, void* stream) {
  int L = 0;
  if (int rc = check_batch(gb, L)) return rc;
  if (!pf || !pf->proc_type || !pf->proc_mem || !pf->cost_ns || !pf->xfer_ns)
    return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: null argument");
  if (gb->n_cand > 0 && (!gb->grain || !d_makespan || !d_ws))
    return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: null grain, makespan or workspace");
  if (pf->n_procs < 1 || pf->n_procs > HESP_MAX_PROCS || pf->n_ptypes < 1 || pf->n_ptypes > HESP_MAX_PTYPES ||
      pf->n_mem < 1 || pf->n_mem > kGMaxMem)
    return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: processors, types or memory spaces");
  if (pf->max_level != gb->n_fac - 1)
    return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: cost table must have n_fac grains");
  for (int m = 1; pf->capacity && m < pf->n_mem; m++)
    if (pf->capacity[m] > 0) return hesp_internal_fail(HESP_EUNSUPPORTED, "grain batches: finite spaces");
  if (policy.order < 0 || policy.order > 1 || policy.select < 0 || policy.select > 1 || policy.cache < 0 ||
      policy.cache > 2 || policy.bus != 0)
    return hesp_internal_fail(HESP_EUNSUPPORTED,
                              "grain batches: Priority-List or FCFS, EFT-P or EIT-P, any caching, no contention");
  if (slots < 1) return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: slots");
  const SlotLayout lay = layout(gb->nt, gb->n_fac, gb->fac, L, pf->n_mem);
  const int64_t head = up256(8 * ((int64_t)L * L + 1));
  if (ws_bytes < head + (int64_t)slots * lay.bytes)
    return hesp_internal_fail(HESP_ECAPACITY, "hesp_simulate_grain_batch: workspace smaller than hesp_grain_workspace");
  if (lay.max_tasks >= (1ll << 31) || lay.max_edges >= (1ll << 32))
    return hesp_internal_fail(HESP_EUNSUPPORTED, "grain batches: more than 2^31 tasks or 2^32 edges per candidate");
  GrainTables tb{};
  tb.nt = gb->nt; tb.n_top = (int32_t)tet(gb->nt); tb.n_fac = gb->n_fac; tb.L = L;
  tb.n_procs = pf->n_procs; tb.n_mem = pf->n_mem;
  tb.fcfs = policy.order; tb.sel = policy.select; tb.cache = policy.cache;
  for (int g = 0; g < gb->n_fac; g++) tb.fac[g] = gb->fac[g];
  for (int p = 0; p < pf->n_procs; p++) {
    if (pf->proc_type[p] < 0 || pf->proc_type[p] >= pf->n_ptypes || pf->proc_mem[p] < 0 ||
        pf->proc_mem[p] >= pf->n_mem)
      return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: proc_type / proc_mem out of range");
    tb.proc_type[p] = (int8_t)pf->proc_type[p];
    tb.proc_mem[p] = (int8_t)pf->proc_mem[p];
  }
  for (int pt = 0; pt < pf->n_ptypes; pt++)
    for (int ty = 0; ty < 4; ty++)
      for (int g = 0; g < gb->n_fac; g++) {
        const int64_t c = pf->cost_ns[(pt * 4 + ty) * gb->n_fac + g];
        if (c < 1) return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: task times must be >= 1");
        tb.cost[pt][ty][g] = c;
      }
  for (int ty = 0; ty < 4; ty++)
    for (int g = 0; g < gb->n_fac; g++) {
      int64_t w = 0;
      for (int p = 0; p < pf->n_procs; p++) w += tb.cost[tb.proc_type[p]][ty][g];
      tb.W[ty][g] = w;
    }
  if (pf->xfer_ns[0] != 0) return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: xfer_ns[0] must be 0");
  for (int64_t k = 1; k <= (int64_t)L * L; k++)
    if (pf->xfer_ns[k] < pf->xfer_ns[k - 1])
      return hesp_internal_fail(HESP_EINVAL, "hesp_simulate_grain_batch: xfer_ns must not decrease");
  if (gb->n_cand == 0) return HESP_OK;
  hipStream_t st = (hipStream_t)stream;
  uint8_t* ws = (uint8_t*)d_ws;
  if (hipMemcpyAsync(ws, pf->xfer_ns, 8 * ((size_t)L * L + 1), hipMemcpyHostToDevice, st) != hipSuccess)
    return hesp_internal_fail(HESP_EHIP, "hesp_simulate_grain_batch: copy of the transfer table");
  tb.xfer = (const int64_t*)ws;
  const int grid = gb->n_cand < slots ? gb->n_cand : slots;
  hipLaunchKernelGGL(k_grain, dim3(grid), dim3(64), 0, st, tb, lay, gb->grain, gb->n_cand, ws + head, d_makespan,
                     d_n_tasks, d_n_edges, d_status);
  if (hipGetLastError() != hipSuccess) return hesp_internal_fail(HESP_EHIP, "hesp_simulate_grain_batch: launch");
  return HESP_OK;
}

}  // extern "C"
