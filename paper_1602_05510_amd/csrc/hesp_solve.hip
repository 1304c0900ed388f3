// hesp_solve.hip -- the partition stage of the iterative scheduler-partitioner
// (section 2.1, "Iterative solver") on gfx950, for many independent chains.
//
// One iteration of every chain: the batched simulation (hesp_simulate_batch)
// gives the schedule of the chain's current partition; then
//   k_sv_first   one workgroup per chain: first fine task of every top-level
//                task (a "cluster": the task of Fig. 1 and the fine tasks it was
//                split into);
//   k_sv_tasks   one lane per fine task: its cluster, the DAG predecessor that
//                finished last; cluster start/finish bounds and the chain's last
//                task (reduced in the wavefront, then atomics);
//   k_sv_part    one workgroup per chain: tasks running at every cluster's
//                start, the proposal of every candidate cluster (the other depth
//                with the largest score span - estimated time), the candidate
//                list (All / CP / Shallow), the Hard or Soft choice, the update.
// Scores and estimates are integers (nanoseconds), so every chain follows the
// same trajectory as an exact sequential implementation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_core.h"
#include "hesp_device.h"
#include "hesp_solve.h"
#include "hesp_tree.h"

namespace hesp {
namespace solve {

namespace {

constexpr int kPartThreads = 1024;
constexpr int kPerThread = kMaxTop / kPartThreads;   // clusters owned by one thread

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// SplitMix64 (Steele, Lea, Flood 2014): value idx+1 of the sequence that starts
// at mix(seed + gamma (purpose + 1))
__device__ __forceinline__ uint64_t sm_draw(uint64_t seed, uint64_t purpose, uint64_t idx) {
  const uint64_t g = 0x9E3779B97F4A7C15ull;
  return sm_mix(sm_mix(seed + g * (purpose + 1)) + g * (idx + 1));
}

// fine tasks of each kind (chol, trsm, syrk, gemm) in a cluster of `kind` split d times
__device__ __forceinline__ void kind_counts(int kind, int d, int64_t* n) {
  const int64_t s = 1 << d;
  n[0] = n[1] = n[2] = n[3] = 0;
  if (kind == CHOL) {
    n[0] = s; n[1] = s * (s - 1) / 2; n[2] = s * (s - 1) / 2; n[3] = s * (s - 1) * (s - 2) / 6;
  } else if (kind == TRSM) {
    n[1] = s * s; n[3] = s * s * (s - 1) / 2;
  } else if (kind == SYRK) {
    n[2] = s * s; n[3] = s * s * (s - 1) / 2;
  } else {
    n[3] = s * s * s;
  }
}

// packed (time, processor) keys: a processor runs one task at a time, so the
// pair names one task.  Start keys order by start, then lower processor; finish
// keys order by finish, then lower processor (the larger key wins).
__device__ __forceinline__ uint64_t start_key(int64_t t, int p) { return ((uint64_t)t << 6) | (uint64_t)p; }
__device__ __forceinline__ uint64_t finish_key(int64_t t, int p) {
  return ((uint64_t)t << 6) | (uint64_t)(kMaxP - 1 - p);
}

// ---------------------------------------------------------------- per chain: first tasks

__global__ void __launch_bounds__(256) k_sv_first(SolveView v) {
  __shared__ int s_part[256 / 64];
  __shared__ int s_carry;
  const int r = blockIdx.x;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const uint8_t* depth = v.depth + (int64_t)r * v.n_top;
  uint32_t* first = v.first + (int64_t)r * (v.n_top + 1);
  if (tid == 0) {
    s_carry = 0;
    v.lastkey[r] = 0;
  }
  __syncthreads();
  for (int base = 0; base < v.n_top; base += 256) {
    const int t = base + tid;
    int cnt = 0;
    if (t < v.n_top) {
      const uint32_t c = top_cell(v.nt, t);
      int d = depth[t];
      d = d > v.dmax ? v.dmax : d;
      cnt = fine_count(kind_of(cell_k(c), cell_i(c), cell_j(c)), d);
      v.t0key[(int64_t)r * v.n_top + t] = ~0ull;
      v.fin[(int64_t)r * v.n_top + t] = 0;
    }
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (l >= o) incl += y;
    }
    if (l == 63) s_part[w] = incl;
    __syncthreads();
    int pre = s_carry;
    for (int q = 0; q < w; q++) pre += s_part[q];
    if (t < v.n_top) first[t] = (uint32_t)(pre + incl - cnt);
    __syncthreads();
    if (tid == 0) {
      int s = 0;
      for (int q = 0; q < 256 / 64; q++) s += s_part[q];
      s_carry += s;
    }
    __syncthreads();
  }
  if (tid == 0) first[v.n_top] = (uint32_t)s_carry;
}

// ---------------------------------------------------------------- per task

// one fine task: its cluster and latest-finishing DAG predecessor; returns its
// finish key, its cluster and its start key
__device__ __forceinline__ uint64_t sv_task(const SolveView& v, int r, int64_t o, int64_t f, int& cl_out,
                                            uint64_t& sk_out, int64_t& fi_out) {
  const uint8_t* depth = v.depth + (int64_t)r * v.n_top;
  const uint32_t* first = v.first + (int64_t)r * (v.n_top + 1);
  // cluster of f: the last top-level task whose first fine task is <= f
  int lo = 0, hi = v.n_top - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((int64_t)first[mid] <= f) lo = mid; else hi = mid - 1;
  }
  const int t = lo;
  const uint32_t cell = top_cell(v.nt, t);
  const int d = depth[t];
  const int s = 1 << d;
  const int kind = kind_of(cell_k(cell), cell_i(cell), cell_j(cell));
  int q, rr, cc;
  local_coords(kind, s, (int)(f - first[t]), q, rr, cc);
  const int K = cell_k(cell) * s + q, I = cell_i(cell) * s + rr, J = cell_j(cell) * s + cc;

  const int p = v.proc[o + f];
  const int64_t fi = v.finish[o + f];
  cl_out = t;
  sk_out = start_key(v.start[o + f], p);
  fi_out = fi;

  uint64_t best = 0;
  int32_t bid = -1;
  auto depth_of = [&](int64_t x) { return (int)depth[x]; };
  auto first_of = [&](int64_t x) { return (int64_t)first[x]; };
  for_each_pred(v.nt, depth_of, first_of, (int64_t)t, cell, d, K, I, J, [&](int64_t u) {
    const uint64_t k = finish_key(v.finish[o + u], v.proc[o + u]);
    if (bid < 0 || k > best) {
      best = k;
      bid = (int32_t)u;
    }
  });
  v.par[o + f] = bid;
  v.cl[o + f] = t;
  return finish_key(fi, p);
}

__global__ void __launch_bounds__(256) k_sv_tasks(SolveView v) {
  const int r = blockIdx.y;
  if (v.status[r] != 0) return;
  const int64_t o = (int64_t)r * v.stride;
  const int64_t n = v.n_tasks[r];
  // the same trip count on every lane (n is uniform): the last-task key is
  // reduced over the wavefront, and the cluster bounds over each run of lanes
  // holding one cluster (a cluster's tasks are consecutive), before the atomics
  const int l = threadIdx.x & 63;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
    const int64_t f = base + threadIdx.x;
    int c = -1;
    uint64_t sk = ~0ull;
    int64_t fi = 0;
    uint64_t key = f < n ? sv_task(v, r, o, f, c, sk, fi) : 0;
    for (int off = 32; off >= 1; off >>= 1) {
      const uint64_t y = __shfl_xor(key, off, 64);
      key = y > key ? y : key;
    }
    if (l == 0 && key != 0) atomicMax((unsigned long long*)&v.lastkey[r], (unsigned long long)key);
    for (int off = 1; off < 64; off <<= 1) {
      const int c2 = __shfl_down(c, off, 64);
      const uint64_t sk2 = __shfl_down(sk, off, 64);
      const int64_t fi2 = __shfl_down(fi, off, 64);
      if (l + off < 64 && c2 == c) {
        sk = sk2 < sk ? sk2 : sk;
        fi = fi2 > fi ? fi2 : fi;
      }
    }
    const int cprev = __shfl_up(c, 1, 64);
    if (c >= 0 && (l == 0 || cprev != c)) {
      atomicMin((unsigned long long*)&v.t0key[(int64_t)r * v.n_top + c], (unsigned long long)sk);
      atomicMax((unsigned long long*)&v.fin[(int64_t)r * v.n_top + c], (unsigned long long)fi);
    }
  }
}

// ---------------------------------------------------------------- per chain: partition stage

__device__ __forceinline__ uint64_t block_max_u64(uint64_t x, uint64_t* s_red) {
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  __syncthreads();
  if (l == 0) s_red[w] = x;
  __syncthreads();
  uint64_t m = 0;
  for (int q = 0; q < kPartThreads / 64; q++) m = s_red[q] > m ? s_red[q] : m;
  return m;
}

// Tasks running at each cluster's start t0 (start <= t0 < finish), for the
// clusters tid * kPerThread + j (t0 = INT64_MAX for absent ones): the starts are
// sorted in LDS; a task adds one over the sorted range [first t0 >= its start,
// first t0 >= its finish), recorded as two differences, then one prefix sum.
// The task whose finish key is lastkey goes to *s_last.  Every thread calls it.
__device__ __forceinline__ void running_at_starts(int n_cl, const int64_t* t0, const int64_t* start,
                                                  const int64_t* finish, const int32_t* proc, int64_t n,
                                                  uint64_t lastkey, int64_t* s_q, int16_t* s_qc, int32_t* s_diff,
                                                  int64_t* s_red, int32_t* s_last, int* run) {
  const int tid = threadIdx.x, c0 = tid * kPerThread;
  int q2 = 1;
  while (q2 < n_cl) q2 <<= 1;
  for (int j = 0; j < kPerThread; j++) {
    const int c = c0 + j;
    if (c < q2) {
      s_q[c] = t0[j];
      s_qc[c] = (int16_t)c;
    }
  }
  for (int i = tid; i <= q2; i += kPartThreads) s_diff[i] = 0;
  __syncthreads();
  for (int k = 2; k <= q2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < q2; i += kPartThreads) {
        const int x = i ^ j;
        if (x > i) {
          const int64_t a = s_q[i], b = s_q[x];
          const int ca = s_qc[i], cb = s_qc[x];
          const bool gt = a > b || (a == b && ca > cb);
          if (((i & k) == 0) == gt) {
            s_q[i] = b; s_q[x] = a;
            s_qc[i] = (int16_t)cb; s_qc[x] = (int16_t)ca;
          }
        }
      }
      __syncthreads();
    }
  auto lower = [&](int64_t t) {          // first sorted position with s_q >= t
    int lo = 0, hi = q2;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_q[mid] < t) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  for (int64_t f = tid; f < n; f += kPartThreads) {
    const int64_t st = start[f], fi = finish[f];
    if (finish_key(fi, proc[f]) == lastkey) *s_last = (int32_t)f;
    const int a = lower(st), b = lower(fi);
    if (a < b) {
      atomicAdd(&s_diff[a], 1);
      atomicAdd(&s_diff[b], -1);
    }
  }
  __syncthreads();
  {
    // inclusive scan of the differences: thread tid owns sorted positions tid*4 .. tid*4+3
    int loc[kPerThread], sum = 0;
    for (int j = 0; j < kPerThread; j++) {
      const int i = tid * kPerThread + j;
      sum += i < q2 ? s_diff[i] : 0;
      loc[j] = sum;
    }
    const int l = tid & 63, w = tid >> 6;
    int incl = sum;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (l >= off) incl += y;
    }
    __syncthreads();
    if (l == 63) ((int*)s_red)[w] = incl;
    __syncthreads();
    int pre = incl - sum;
    for (int q = 0; q < w; q++) pre += ((int*)s_red)[q];
    __syncthreads();
    // counts back to the clusters (s_diff is reused: count of cluster c at c)
    for (int j = 0; j < kPerThread; j++) {
      const int i = tid * kPerThread + j;
      if (i < q2) loc[j] += pre;
    }
    __syncthreads();
    for (int j = 0; j < kPerThread; j++) {
      const int i = tid * kPerThread + j;
      if (i < q2) s_diff[s_qc[i]] = loc[j];
    }
    __syncthreads();
    for (int j = 0; j < kPerThread; j++)
      if (c0 + j < n_cl) run[j] = s_diff[c0 + j];
  }
  __syncthreads();

}

__global__ void __launch_bounds__(kPartThreads) k_sv_part(SolveView v, SolveTables tb) {
  __shared__ int64_t s_q[kMaxTop];        // cluster start times, sorted
  __shared__ int16_t s_qc[kMaxTop];       // their clusters
  __shared__ int32_t s_diff[kMaxTop + 1]; // running-count differences over the sorted starts
  __shared__ int64_t s_red[kPartThreads / 64];
  __shared__ uint32_t s_cp[kMaxTop / 32];
  __shared__ int32_t s_last;
  __shared__ int64_t s_pick[3];

  const int r = blockIdx.x;
  const int tid = threadIdx.x;
  const int it = v.iter;
  const int n_top = v.n_top;
  uint8_t* depth = v.depth + (int64_t)r * n_top;
  int64_t* trace = v.trace ? v.trace + (int64_t)r * v.iters : nullptr;
  int64_t* steps = v.steps ? v.steps + ((int64_t)r * v.iters + it) * 3 : nullptr;
  if (v.status[r] != 0) {
    if (tid == 0) {
      if (trace) trace[it] = -1;
      if (steps) { steps[0] = -1; steps[1] = -1; steps[2] = 0; }
    }
    return;
  }
  const int64_t ms = v.makespan[r];
  // best partition so far (the earliest on ties): taken before the update
  const bool better = it == 0 || ms < v.best_ms[r];
  __syncthreads();
  if (better) {
    uint8_t* bd = v.best_depth + (int64_t)r * n_top;
    for (int t = tid; t < n_top; t += kPartThreads) bd[t] = depth[t];
  }
  if (tid == 0) {
    if (trace) trace[it] = ms;
    if (better) v.best_ms[r] = ms;
  }

  // clusters tid * kPerThread + j, in Fig. 1 order along the threads
  int64_t t0[kPerThread], span[kPerThread];
  int run[kPerThread], pt[kPerThread];
  const int c0 = tid * kPerThread;
  const int64_t o = (int64_t)r * v.stride;
  const int64_t n = v.n_tasks[r];
  for (int j = 0; j < kPerThread; j++) {
    const int c = c0 + j;
    t0[j] = INT64_MAX;
    span[j] = 0;
    run[j] = 0;
    pt[j] = 0;
    if (c < n_top) {
      const uint64_t k = v.t0key[(int64_t)r * n_top + c];
      t0[j] = (int64_t)(k >> 6);
      span[j] = (int64_t)v.fin[(int64_t)r * n_top + c] - t0[j];
      pt[j] = tb.proc_type[(int)(k & 63)];
    }
  }
  for (int q = tid; q < kMaxTop / 32; q += kPartThreads) s_cp[q] = 0;
  if (tid == 0) s_last = -1;
  const uint64_t lastkey = v.lastkey[r];

  running_at_starts(n_top, t0, v.start + o, v.finish + o, v.proc + o, n, lastkey, s_q, s_qc, s_diff, s_red, &s_last,
                    run);

  // candidate list
  int dmin = 255;
  for (int j = 0; j < kPerThread; j++)
    if (c0 + j < n_top) dmin = min(dmin, (int)depth[c0 + j]);
  const int64_t shallow = -block_max_u64((uint64_t)(255 - dmin), (uint64_t*)s_red) + 255;
  if (v.list == 1 && tid == 0) {
    // critical path: from the last-finishing task along the latest-finishing
    // DAG predecessors (at most n steps)
    int32_t x = s_last;
    for (int64_t guard = 0; x >= 0 && guard < n; guard++) {
      const int c = v.cl[o + x];
      s_cp[c >> 5] |= 1u << (c & 31);
      x = v.par[o + x];
    }
  }
  __syncthreads();

  // proposals: the other depth with the largest score (the smallest on ties)
  int64_t score[kPerThread];
  int dnew[kPerThread];
  for (int j = 0; j < kPerThread; j++) {
    const int c = c0 + j;
    score[j] = 0;
    dnew[j] = -1;
    if (c >= n_top) continue;
    const int dc = depth[c];
    bool in = true;
    if (v.list == 1) in = (s_cp[c >> 5] >> (c & 31)) & 1u;
    if (v.list == 2) in = dc == (int)shallow;
    if (!in) continue;
    const uint32_t cell = top_cell(v.nt, c);
    const int kind = kind_of(cell_k(cell), cell_i(cell), cell_j(cell));
    const int64_t avail = (int64_t)tb.n_procs - run[j] + 1;
    bool have = false;
    int64_t top = 0;
    int td = -1;
    for (int dn = 0; dn <= v.dmax; dn++) {
      if (dn == dc) continue;
      int64_t cnt[4];
      kind_counts(kind, dn, cnt);
      int64_t work = 0;
      for (int k = 0; k < 4; k++) work += cnt[k] * tb.cost[pt[j]][k][dn];
      int64_t par = (cnt[0] + cnt[1] + cnt[2] + cnt[3]) >> dn;
      par = par < 1 ? 1 : par;
      const int64_t lanes = avail < par ? avail : par;
      const int64_t est = (work + lanes - 1) / lanes;
      const int64_t sc = span[j] - est;
      if (!have || sc > top) {
        have = true;
        top = sc;
        td = dn;
      }
    }
    if (have && top > 0) {
      score[j] = top;
      dnew[j] = td;
    }
  }

  // selection
  if (tid == 0) { s_pick[0] = -1; s_pick[1] = -1; s_pick[2] = 0; }
  if (v.sampling == 0) {
    uint64_t key = 0;   // score << 12 | (kMaxTop - 1 - cluster): largest score, then smallest cluster
    for (int j = 0; j < kPerThread; j++)
      if (dnew[j] >= 0) {
        const uint64_t k = ((uint64_t)score[j] << 12) | (uint64_t)(kMaxTop - 1 - (c0 + j));
        key = k > key ? k : key;
      }
    const uint64_t bestk = block_max_u64(key, (uint64_t*)s_red);
    if (bestk != 0) {
      const int c = kMaxTop - 1 - (int)(bestk & (kMaxTop - 1));
      if (c >= c0 && c < c0 + kPerThread) {
        s_pick[0] = c;
        s_pick[1] = dnew[c - c0];
        s_pick[2] = score[c - c0];
      }
    }
  } else {
    int64_t mine = 0;
    for (int j = 0; j < kPerThread; j++) mine += score[j];
    // exclusive prefix of the score sums in cluster order
    const int l = tid & 63, w = tid >> 6;
    int64_t incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(incl, off, 64);
      if (l >= off) incl += y;
    }
    __syncthreads();
    if (l == 63) s_red[w] = incl;
    __syncthreads();
    int64_t pre = 0, total = 0;
    for (int q = 0; q < kPartThreads / 64; q++) {
      if (q < w) pre += s_red[q];
      total += s_red[q];
    }
    pre += incl - mine;
    if (total > 0) {
      const int64_t u = (int64_t)(sm_draw(v.seed + (uint64_t)r, 10, (uint64_t)it) % (uint64_t)total);
      int64_t acc = pre;
      for (int j = 0; j < kPerThread; j++) {
        if (dnew[j] < 0) continue;
        if (acc <= u && u < acc + score[j]) {
          s_pick[0] = c0 + j;
          s_pick[1] = dnew[j];
          s_pick[2] = score[j];
        }
        acc += score[j];
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (steps) { steps[0] = s_pick[0]; steps[1] = s_pick[1]; steps[2] = s_pick[2]; }
    if (s_pick[0] >= 0) depth[s_pick[0]] = (uint8_t)s_pick[1];
  }
}

__global__ void k_sv_strided(int64_t stride, int32_t count, int64_t* off) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= count) off[c] = (int64_t)c * stride;
}


// ---------------------------------------------------------------- split-tree partitions

// node x: its level, cell and kind (levels from the flag offsets)
struct Node {
  int lv, K, I, J, kind;
};
__device__ __forceinline__ Node node_of(const TreeSolveView& v, int x) {
  Node d;
  d.lv = 0;
  while (d.lv + 1 < v.dmax && x >= v.level_off[d.lv + 1]) d.lv++;
  const uint32_t c = top_cell(v.nt << d.lv, x - v.level_off[d.lv]);
  d.K = cell_k(c);
  d.I = cell_i(c);
  d.J = cell_j(c);
  d.kind = kind_of(d.K, d.I, d.J);
  return d;
}
// flag index of the level-h ancestor (or self) of level-lv cell (K, I, J)
__device__ __forceinline__ int64_t node_at(const TreeSolveView& v, int h, int lv, int K, int I, int J) {
  const int sh = lv - h;
  return v.level_off[h] + top_index(v.nt << h, K >> sh, I >> sh, J >> sh);
}

__global__ void __launch_bounds__(256) k_svt_init(TreeSolveView v) {
  const int r = blockIdx.x;
  for (int x = threadIdx.x; x < v.n_nodes; x += 256) {
    v.t0key[(int64_t)r * v.n_nodes + x] = ~0ull;
    v.fin[(int64_t)r * v.n_nodes + x] = 0;
  }
  if (threadIdx.x == 0) v.lastkey[r] = 0;
}

// one wavefront per chain walks its tasks in program order: descriptor, the
// latest-finishing of the last writers of its blocks (a predecessor with the
// latest finish, as over the whole dependence graph), bounds of the nodes
// holding it, the last-finishing task and the smallest task level
__global__ void __launch_bounds__(kWave) k_svt_tasks(TreeSolveView v) {
  const int r = blockIdx.x;
  if (v.status[r] != 0) return;
  const int l = dev::lane();
  const int nt = v.nt, dmax = v.dmax;
  const int64_t o = (int64_t)r * v.stride;
  const int64_t n_atoms = (int64_t)tri2(nt) << (2 * dmax);
  uint32_t* lw = v.lw + (int64_t)r * n_atoms;
  for (int64_t a = l; a < n_atoms; a += kWave) lw[a] = dev::kNil;
  dev::wave_order();
  uint32_t f = 0;
  uint64_t last = 0;
  int lmin = 255;
  dev::walk_tree(nt, dmax, v.flags + (int64_t)r * v.n_nodes, [&](int kind, int lv, int K, int I, int J) {
    const uint32_t t = f++;
    if ((int64_t)t >= v.n_tasks[r]) return;            // the simulation counted the same tasks
    uint64_t best = 0;
    int32_t bid = -1;
    dev::scan_task(lw, nt, dmax, kind, lv, K, I, J, t, [&](uint32_t p) {
      const uint64_t k = finish_key(v.finish[o + p], v.proc[o + p]);
      if (bid < 0 || k > best) {
        best = k;
        bid = (int32_t)p;
      }
    });
    const int p = v.proc[o + t];
    const int64_t st = v.start[o + t], fi = v.finish[o + t];
    const uint64_t fk = finish_key(fi, p);
    last = fk > last ? fk : last;
    lmin = lv < lmin ? lv : lmin;
    if (l == 0) {
      v.par[o + t] = bid;
      v.desc[o + t] = pack_desc(kind, lv, K, I, J);
    }
    const int nh = (lv < dmax - 1 ? lv : dmax - 1) + 1;   // nodes holding it: levels 0 .. min(lv, dmax-1)
    if (l < nh) {
      const int64_t x = node_at(v, l, lv, K, I, J);
      atomicMin((unsigned long long*)&v.t0key[(int64_t)r * v.n_nodes + x], (unsigned long long)start_key(st, p));
      atomicMax((unsigned long long*)&v.fin[(int64_t)r * v.n_nodes + x], (unsigned long long)fi);
    }
  });
  if (l == 0) {
    v.lastkey[r] = last;
    v.lmin[r] = lmin;
  }
}

__global__ void __launch_bounds__(kPartThreads) k_svt_part(TreeSolveView v, SolveTables tb) {
  __shared__ int64_t s_q[kMaxTop];
  __shared__ int16_t s_qc[kMaxTop];
  __shared__ int32_t s_diff[kMaxTop + 1];
  __shared__ int64_t s_red[kPartThreads / 64];
  __shared__ uint32_t s_cp[kMaxTop / 32];
  __shared__ int32_t s_last;
  __shared__ int64_t s_pick[3];

  const int r = blockIdx.x;
  const int tid = threadIdx.x;
  const int it = v.iter;
  const int nn = v.n_nodes;
  uint8_t* flags = v.flags + (int64_t)r * nn;
  int64_t* trace = v.trace ? v.trace + (int64_t)r * v.iters : nullptr;
  int64_t* steps = v.steps ? v.steps + ((int64_t)r * v.iters + it) * 3 : nullptr;
  if (v.status[r] != 0) {
    if (tid == 0) {
      if (trace) trace[it] = -1;
      if (steps) { steps[0] = -1; steps[1] = -1; steps[2] = 0; }
    }
    return;
  }
  const int64_t ms = v.makespan[r];
  const bool better = it == 0 || ms < v.best_ms[r];
  __syncthreads();
  if (better)
    for (int x = tid; x < nn; x += kPartThreads) v.best_flags[(int64_t)r * nn + x] = flags[x];
  if (tid == 0) {
    if (trace) trace[it] = ms;
    if (better) v.best_ms[r] = ms;
  }

  // nodes tid * kPerThread + j
  int64_t t0[kPerThread], span[kPerThread];
  int run[kPerThread], pt[kPerThread], state[kPerThread];   // state: 0 absent, 1 leaf, 2 internal
  const int c0 = tid * kPerThread;
  for (int j = 0; j < kPerThread; j++) {
    const int x = c0 + j;
    t0[j] = INT64_MAX;
    span[j] = 0;
    run[j] = 0;
    pt[j] = 0;
    state[j] = 0;
    if (x < nn) {
      const Node d = node_of(v, x);
      bool ex = true;
      for (int h = 0; h < d.lv; h++) ex = ex && flags[node_at(v, h, d.lv, d.K, d.I, d.J)] == 1;
      if (ex) {
        state[j] = flags[x] == 1 ? 2 : 1;
        const uint64_t k = v.t0key[(int64_t)r * nn + x];
        t0[j] = (int64_t)(k >> 6);
        span[j] = (int64_t)v.fin[(int64_t)r * nn + x] - t0[j];
        pt[j] = tb.proc_type[(int)(k & 63)];
      }
    }
  }
  for (int q = tid; q < kMaxTop / 32; q += kPartThreads) s_cp[q] = 0;
  if (tid == 0) s_last = -1;
  const int64_t o = (int64_t)r * v.stride;
  const int64_t n = v.n_tasks[r];
  running_at_starts(nn, t0, v.start + o, v.finish + o, v.proc + o, n, v.lastkey[r], s_q, s_qc, s_diff, s_red,
                    &s_last, run);
  if (v.list == 1 && tid == 0) {
    // critical path: every node holding one of its tasks
    int32_t x = s_last;
    for (int64_t guard = 0; x >= 0 && guard < n; guard++) {
      const uint32_t d = v.desc[o + x];
      const int lv = desc_level(d), nh = (lv < v.dmax - 1 ? lv : v.dmax - 1) + 1;
      for (int h = 0; h < nh; h++) {
        const int64_t y = node_at(v, h, lv, desc_K(d), desc_I(d), desc_J(d));
        s_cp[y >> 5] |= 1u << (y & 31);
      }
      x = v.par[o + x];
    }
  }
  __syncthreads();

  // proposals: an internal node merges (its own task), a leaf one splits once
  const int lmin = v.lmin[r];
  int64_t score[kPerThread];
  int act[kPerThread];
  for (int j = 0; j < kPerThread; j++) {
    const int x = c0 + j;
    score[j] = 0;
    act[j] = -1;
    if (state[j] == 0) continue;
    const Node d = node_of(v, x);
    bool in = true;
    if (v.list == 1) in = (s_cp[x >> 5] >> (x & 31)) & 1u;
    if (v.list == 2) in = state[j] == 1 && d.lv == lmin;
    if (!in) continue;
    int64_t est;
    int a;
    if (state[j] == 2) {
      est = tb.cost[pt[j]][d.kind][d.lv];
      a = 0;
    } else {
      int64_t cnt[4];
      kind_counts(d.kind, 1, cnt);
      int64_t work = 0;
      for (int k = 0; k < 4; k++) work += cnt[k] * tb.cost[pt[j]][k][d.lv + 1];
      int64_t width = (cnt[0] + cnt[1] + cnt[2] + cnt[3]) >> 1;
      width = width < 1 ? 1 : width;
      const int64_t avail = (int64_t)tb.n_procs - run[j] + 1;
      const int64_t lanes = avail < width ? avail : width;
      est = (work + lanes - 1) / lanes;
      a = 1;
    }
    if (span[j] - est > 0) {
      score[j] = span[j] - est;
      act[j] = a;
    }
  }

  // selection (as for top-level clusters)
  if (tid == 0) { s_pick[0] = -1; s_pick[1] = -1; s_pick[2] = 0; }
  if (v.sampling == 0) {
    uint64_t key = 0;
    for (int j = 0; j < kPerThread; j++)
      if (act[j] >= 0) {
        const uint64_t k = ((uint64_t)score[j] << 12) | (uint64_t)(kMaxTop - 1 - (c0 + j));
        key = k > key ? k : key;
      }
    const uint64_t bestk = block_max_u64(key, (uint64_t*)s_red);
    if (bestk != 0) {
      const int x = kMaxTop - 1 - (int)(bestk & (kMaxTop - 1));
      if (x >= c0 && x < c0 + kPerThread) {
        s_pick[0] = x;
        s_pick[1] = act[x - c0];
        s_pick[2] = score[x - c0];
      }
    }
  } else {
    int64_t mine = 0;
    for (int j = 0; j < kPerThread; j++) mine += score[j];
    const int l = tid & 63, w = tid >> 6;
    int64_t incl = mine;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(incl, off, 64);
      if (l >= off) incl += y;
    }
    __syncthreads();
    if (l == 63) s_red[w] = incl;
    __syncthreads();
    int64_t pre = 0, total = 0;
    for (int q = 0; q < kPartThreads / 64; q++) {
      if (q < w) pre += s_red[q];
      total += s_red[q];
    }
    pre += incl - mine;
    if (total > 0) {
      const int64_t u = (int64_t)(sm_draw(v.seed + (uint64_t)r, 10, (uint64_t)it) % (uint64_t)total);
      int64_t acc = pre;
      for (int j = 0; j < kPerThread; j++) {
        if (act[j] < 0) continue;
        if (acc <= u && u < acc + score[j]) {
          s_pick[0] = c0 + j;
          s_pick[1] = act[j];
          s_pick[2] = score[j];
        }
        acc += score[j];
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (steps) { steps[0] = s_pick[0]; steps[1] = s_pick[1]; steps[2] = s_pick[2]; }
    if (s_pick[0] >= 0) {
      const int x = (int)s_pick[0];
      flags[x] = (uint8_t)s_pick[1];
      const Node d = node_of(v, x);
      if (s_pick[1] == 1 && d.lv + 1 < v.dmax)
        // the new children start as leaves
        for (int c = 0; c < fine_count(d.kind, 1); c++) {
          int q, rr, cc;
          local_coords(d.kind, 2, c, q, rr, cc);
          flags[node_at(v, d.lv + 1, d.lv + 1, 2 * d.K + q, 2 * d.I + rr, 2 * d.J + cc)] = 0;
        }
    }
  }
}

}  // namespace

hipError_t launch_strided(int64_t stride, int32_t count, int64_t* off, hipStream_t s) {
  hipLaunchKernelGGL(k_sv_strided, dim3((count + 256) / 256), dim3(256), 0, s, stride, count, off);
  return hipGetLastError();
}

hipError_t launch_first(const SolveView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_sv_first, dim3(v.n_chains), dim3(256), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_tasks(const SolveView& v, int64_t max_tasks, hipStream_t s) {
  // a few workgroups per chain, each striding over the chain's tasks
  int64_t nb = (max_tasks + 255) / 256;
  nb = nb < 8 ? nb : 8;
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sv_tasks, dim3((unsigned)nb, v.n_chains), dim3(256), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_tree_init(const TreeSolveView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_svt_init, dim3(v.n_chains), dim3(256), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_tree_tasks(const TreeSolveView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_svt_tasks, dim3(v.n_chains), dim3(kWave), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_tree_part(const TreeSolveView& v, const SolveTables& t, hipStream_t s) {
  hipLaunchKernelGGL(k_svt_part, dim3(v.n_chains), dim3(kPartThreads), 0, s, v, t);
  return hipGetLastError();
}

hipError_t launch_part(const SolveView& v, const SolveTables& t, hipStream_t s) {
  hipLaunchKernelGGL(k_sv_part, dim3(v.n_chains), dim3(kPartThreads), 0, s, v, t);
  return hipGetLastError();
}

}  // namespace solve
}  // namespace hesp
