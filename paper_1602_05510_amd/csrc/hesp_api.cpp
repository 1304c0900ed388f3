// hesp_api.cpp -- implementation of the C ABI declared in include/hesp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <map>
#include <tuple>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hesp.h"
#include "hesp_core.h"
#include "hesp_internal.h"
#include "hesp_search.h"

using namespace hesp;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int ok() { return HESP_OK; }

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(HESP_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int64_t pow4(int x) { return (int64_t)1 << (2 * x); }

void hfree(void* p) {
  if (p) (void)hipFree(p);
}

// exact ceil(a / b) for a >= 0, b > 0 with a 128-bit numerator
int64_t ceil_div128(__int128 a, __int128 b) { return (int64_t)((a + b - 1) / b); }

}  // namespace

// A device buffer that only grows.
struct DevBuf {
  void* p = nullptr;
  int64_t bytes = 0;
  hipError_t ensure(int64_t need) {
    if (need <= bytes) return hipSuccess;
    hfree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, (size_t)(need > 0 ? need : 1));
    if (e == hipSuccess) bytes = need;
    return e;
  }
  void release() {
    hfree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T>
  T* as() const { return (T*)p; }
};

// Workspace of one chunk of candidates.
struct WorkSet {
  DevBuf top_first, desc, indeg, cur, succ, rec, fifo, ready, sortbuf, vf, use, pin, nsrc, order_keys, order;
  std::vector<DevBuf*> all() {
    return {&top_first, &desc, &indeg, &cur, &succ, &rec, &fifo, &ready, &sortbuf, &vf, &use, &pin, &nsrc,
            &order_keys, &order};
  }
  int64_t bytes() const {
    return top_first.bytes + desc.bytes + indeg.bytes + cur.bytes + succ.bytes + rec.bytes + fifo.bytes +
           ready.bytes + sortbuf.bytes + vf.bytes + use.bytes + pin.bytes + nsrc.bytes + order_keys.bytes +
           order.bytes;
  }
};

struct hesp_plan {
  hesp_plan_opts opts{};
  int32_t slots = 0;          // waves of the persistent simulation kernel
  int32_t chunk = 0;          // candidates per chunk
  uint32_t* counter = nullptr;
  // per batch
  DevBuf cnt_tasks, cnt_edges, off_t, off_e, off_v, off_top, bounds, layout_part;
  DevBuf tree_lw;             // split-tree counts: last writer per finest block and candidate
  // transfer times of platforms deeper than kXferLevels: the device copy and the
  // host table it was made from
  DevBuf xfer_deep;
  std::vector<int64_t> xfer_host;
  // per chunk, two sets: chunk i+1 is prepared while chunk i is simulated
  WorkSet ws[2];
  hipStream_t s_prep = nullptr, s_sim = nullptr;
  std::vector<hipEvent_t> sync_ev;   // fork, then per chunk: prepared, simulated
  std::vector<int64_t> h_bounds;
  // autotuned lanes per candidate, by (processors, memory spaces, nt, dmax, ragged)
  std::map<std::tuple<int, int, int, int, int>, int> tuned;
  // fixed-capacity plans: chunk size chosen for (candidates, validity words, top-level tasks)
  std::tuple<int64_t, int64_t, int64_t> fixed_key{-1, -1, -1};
  int32_t fixed_chunk = 0;
  // fused pipeline: one slot per resident wave of the 64-lane event loop
  DevBuf arena;
  int32_t resident64 = 0;     // waves of the fused event loop resident at once (four per SIMD)
  std::tuple<int64_t, int64_t, int64_t> fused_key{-1, -1, -1};
  int32_t fused_waves = 0;
  // optional kernel timing of the last call: events around each launch
  bool timing = false;
  std::vector<hipEvent_t> ev;   // per chunk: prepare start and end, simulation start and end
  size_t ev_used = 0;
  int64_t held() const {
    return cnt_tasks.bytes + cnt_edges.bytes + off_t.bytes + off_e.bytes + off_v.bytes + off_top.bytes +
           bounds.bytes + layout_part.bytes + tree_lw.bytes + arena.bytes + xfer_deep.bytes + ws[0].bytes() +
           ws[1].bytes();
  }
  void release() {
    for (DevBuf* b : {&cnt_tasks, &cnt_edges, &off_t, &off_e, &off_v, &off_top, &bounds, &layout_part, &tree_lw, &arena,
                      &xfer_deep})
      b->release();
    xfer_host.clear();
    for (WorkSet& w : ws)
      for (DevBuf* d : w.all()) d->release();
  }
};

extern "C" {

int hesp_internal_fail(int code, const char* msg) {
  g_err = msg;
  return code;
}

// 1 when the plan limits the tasks or edges of a candidate (such candidates fail
// with HESP_ECAPACITY)
int hesp_internal_plan_capped(const hesp_plan* p) { return p && (p->opts.max_tasks > 0 || p->opts.max_edges > 0); }

const char* hesp_last_error(void) { return g_err.c_str(); }
const char* hesp_version(void) { return "hesp-mi355x 0.1 (gfx950)"; }

int hesp_cost_tables(const hesp_cost_model* cm, int64_t* cost_ns, int64_t* xfer_ns) {
  if (!cm || !cost_ns || !xfer_ns) return fail(HESP_EINVAL, "hesp_cost_tables: null argument");
  if (cm->n_ptypes < 1 || cm->n_ptypes > HESP_MAX_PTYPES || !cm->rmax_mflops || !cm->h)
    return fail(HESP_EINVAL, "hesp_cost_tables: bad processor types");
  if (cm->max_level < 0 || cm->max_level > HESP_MAX_LEVEL) return fail(HESP_EINVAL, "hesp_cost_tables: max_level");
  if (cm->b <= 0 || ((cm->b >> cm->max_level) << cm->max_level) != cm->b)
    return fail(HESP_EINVAL, "hesp_cost_tables: b must be a positive multiple of 2^max_level");
  if (cm->bw_bytes_per_ns <= 0 || cm->latency_ns < 0 || cm->elem_bytes <= 0)
    return fail(HESP_EINVAL, "hesp_cost_tables: transfer model");
  static const int64_t c3[4] = {1, 3, 3, 6};  // flops * 3 / bl^3
  const int L = cm->max_level + 1;
  for (int pt = 0; pt < cm->n_ptypes; pt++) {
    const int64_t h = cm->h[pt];
    if (h < 0) return fail(HESP_EINVAL, "hesp_cost_tables: h < 0");
    for (int k = 0; k < 4; k++) {
      const int64_t r = cm->rmax_mflops[pt * 4 + k];
      if (r <= 0) return fail(HESP_EINVAL, "hesp_cost_tables: rmax <= 0");
      for (int l = 0; l < L; l++) {
        const int64_t bl = cm->b >> l;
        // time = (c3 bl^3 / 3) / (r/1000 * bl^2/(bl^2+h^2)) = 1000 c3 bl (bl^2+h^2) / (3 r)
        const __int128 num = (__int128)1000 * c3[k] * bl * ((__int128)bl * bl + (__int128)h * h);
        cost_ns[(pt * 4 + k) * L + l] = ceil_div128(num, (__int128)3 * r);
      }
    }
  }
  const int64_t a = cm->b >> cm->max_level;
  for (int64_t k = 0; k <= pow4(cm->max_level); k++) {
    if (k == 0 || cm->shared_memory) xfer_ns[k] = 0;
    else xfer_ns[k] = cm->latency_ns + ceil_div128((__int128)cm->elem_bytes * k * a * a, cm->bw_bytes_per_ns);
  }
  return ok();
}

int hesp_expand(int32_t nt, int32_t dmax, const uint8_t* depth, int32_t* n_tasks, int64_t* n_edges,
                hesp_task* tasks, int64_t* succ_ptr, int32_t* succ_idx) {
  if (nt < 1 || dmax < 0 || dmax > HESP_MAX_LEVEL || (nt << dmax) > HESP_MAX_FINE)
    return fail(HESP_EINVAL, "hesp_expand: nt=%d dmax=%d outside 1 <= nt, 0 <= dmax <= %d, nt*2^dmax <= %d", nt,
                dmax, HESP_MAX_LEVEL, HESP_MAX_FINE);
  if (!depth || !n_tasks || !n_edges) return fail(HESP_EINVAL, "hesp_expand: null argument");
  const int64_t n_top = tet3(nt);
  for (int64_t t = 0; t < n_top; t++)
    if (depth[t] > dmax) return fail(HESP_EINVAL, "hesp_expand: depth[%lld]=%d > dmax", (long long)t, depth[t]);
  std::vector<int64_t> first(n_top + 1);
  std::vector<uint32_t> cells(n_top);
  first[0] = 0;
  for (int64_t t = 0; t < n_top; t++) {
    cells[t] = top_cell(nt, t);
    first[t + 1] = first[t] + fine_count(kind_of(cell_k(cells[t]), cell_i(cells[t]), cell_j(cells[t])), depth[t]);
  }
  const int64_t n = first[n_top];
  auto depth_of = [&](int64_t t) { return (int)depth[t]; };
  auto first_of = [&](int64_t t) { return first[t]; };
  // enumerate (task number, top, cell, d, K, I, J)
  auto each_task = [&](auto&& fn) {
    for (int64_t t = 0; t < n_top; t++) {
      const uint32_t cell = cells[t];
      const int d = depth[t], s = 1 << d;
      const int kind = kind_of(cell_k(cell), cell_i(cell), cell_j(cell));
      for (int64_t x = 0; x < first[t + 1] - first[t]; x++) {
        int q, r, c;
        local_coords(kind, s, (int)x, q, r, c);
        fn(first[t] + x, t, cell, d, cell_k(cell) * s + q, cell_i(cell) * s + r, cell_j(cell) * s + c);
      }
    }
  };
  std::vector<int64_t> cnt(n + 1, 0);
  int64_t m = 0;
  each_task([&](int64_t f, int64_t t, uint32_t cell, int d, int K, int I, int J) {
    (void)f;
    m += for_each_pred(nt, depth_of, first_of, t, cell, d, K, I, J, [&](int64_t p) { cnt[p + 1]++; });
  });
  if (n > INT32_MAX) return fail(HESP_EUNSUPPORTED, "hesp_expand: too many tasks");
  *n_tasks = (int32_t)n;
  *n_edges = m;
  if (!tasks && !succ_ptr && !succ_idx) return ok();
  if (!tasks || !succ_ptr || !succ_idx) return fail(HESP_EINVAL, "hesp_expand: give all or none of the arrays");
  for (int64_t f = 0; f < n; f++) cnt[f + 1] += cnt[f];
  for (int64_t f = 0; f <= n; f++) succ_ptr[f] = cnt[f];
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  each_task([&](int64_t f, int64_t t, uint32_t cell, int d, int K, int I, int J) {
    tasks[f] = hesp_task{kind_of(K, I, J), d, K, I, J};
    for_each_pred(nt, depth_of, first_of, t, cell, d, K, I, J,
                  [&](int64_t p) { succ_idx[pos[p]++] = (int32_t)f; });
  });
  return ok();
}

// ---- generation -------------------------------------------------------------

static int check_thr(uint32_t thr) {
  return thr <= (1u << 21) ? HESP_OK : fail(HESP_EINVAL, "split_thr must be <= 2^21");
}

int hesp_generate_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt, int32_t dmax,
                          uint32_t split_thr, uint8_t* d_depth, void* stream) {
  if (n_cand < 0 || nt < 1 || dmax < 0 || dmax > HESP_MAX_LEVEL || first < 0 || (!d_depth && n_cand > 0))
    return fail(HESP_EINVAL, "hesp_generate_uniform: bad argument");
  if (check_thr(split_thr)) return HESP_EINVAL;
  HIP_TRY(launch_gen_uniform(seed, first, n_cand, nt, dmax, split_thr, d_depth, (hipStream_t)stream));
  return ok();
}

int hesp_generate_ragged_shape(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt_lo, int32_t nt_hi,
                               int32_t dmax_hi, int32_t* d_nt, int32_t* d_dmax, int64_t* d_mask_off,
                               void* stream) {
  if (n_cand < 0 || nt_lo < 1 || nt_hi < nt_lo || dmax_hi < 0 || dmax_hi > HESP_MAX_LEVEL || first < 0 ||
      !d_mask_off || (n_cand > 0 && (!d_nt || !d_dmax)))
    return fail(HESP_EINVAL, "hesp_generate_ragged_shape: bad argument");
  HIP_TRY(launch_gen_shape(seed, first, n_cand, nt_lo, nt_hi, dmax_hi, d_nt, d_dmax, d_mask_off,
                           (hipStream_t)stream));
  return ok();
}

static int batch_view(const hesp_batch* b, BatchView& v, const char* who) {
  if (!b) return fail(HESP_EINVAL, "%s: null batch", who);
  if (b->n_cand < 0 || (b->n_cand > 0 && !b->d_depth)) return fail(HESP_EINVAL, "%s: bad batch", who);
  if ((b->d_nt == nullptr) != (b->d_dmax == nullptr))
    return fail(HESP_EINVAL, "%s: give both or neither of d_nt and d_dmax", who);
  if (b->d_nt && !b->d_mask_off) return fail(HESP_EINVAL, "%s: a ragged batch needs d_mask_off", who);
  if (b->nt < 1 || b->dmax < 0 || b->dmax > HESP_MAX_LEVEL || (b->nt << b->dmax) > HESP_MAX_FINE)
    return fail(HESP_EINVAL, "%s: nt=%d dmax=%d outside the supported range", who, b->nt, b->dmax);
  v.n_cand = b->n_cand;
  v.nt = b->nt;
  v.dmax = b->dmax;
  v.nt_arr = b->d_nt;
  v.dmax_arr = b->d_dmax;
  v.off = b->d_mask_off;
  v.depth = b->d_depth;
  v.tree_stride = 0;
  return HESP_OK;
}

static int tree_view(const hesp_tree_batch* b, BatchView& v, const char* who) {
  if (!b) return fail(HESP_EINVAL, "%s: null batch", who);
  if (b->n_cand < 0 || b->nt < 1 || b->dmax < 0 || b->dmax > HESP_MAX_LEVEL || (b->nt << b->dmax) > HESP_MAX_FINE)
    return fail(HESP_EINVAL, "%s: n_cand=%d nt=%d dmax=%d outside the supported range", who, b->n_cand, b->nt,
                b->dmax);
  const int64_t nf = hesp_tree_flag_count(b->nt, b->dmax);
  if (b->n_cand > 0 && nf > 0 && !b->d_flags) return fail(HESP_EINVAL, "%s: null flags", who);
  v.n_cand = b->n_cand;
  v.nt = b->nt;
  v.dmax = b->dmax;
  v.nt_arr = nullptr;
  v.dmax_arr = nullptr;
  v.off = nullptr;
  v.depth = b->d_flags;
  v.tree_stride = nf > 0 ? nf : 1;     // dmax = 0: no flags, the unsplit problem
  return HESP_OK;
}

int hesp_generate_ragged_depth(uint64_t seed, int64_t first, const hesp_batch* batch, uint32_t split_thr,
                               uint8_t* d_depth, void* stream) {
  BatchView v;
  hesp_batch b2 = batch ? *batch : hesp_batch{};
  b2.d_depth = d_depth;
  if (int r = batch_view(&b2, v, "hesp_generate_ragged_depth")) return r;
  if (!v.nt_arr) return fail(HESP_EINVAL, "hesp_generate_ragged_depth: needs d_nt, d_dmax, d_mask_off");
  if (check_thr(split_thr)) return HESP_EINVAL;
  HIP_TRY(launch_gen_ragged_depth(seed, first, v, split_thr, d_depth, (hipStream_t)stream));
  return ok();
}

int hesp_count_batch(const hesp_batch* batch, int32_t* d_n_tasks, int64_t* d_n_edges, void* stream) {
  BatchView v;
  if (int r = batch_view(batch, v, "hesp_count_batch")) return r;
  HIP_TRY(launch_count(v, d_n_tasks, d_n_edges, (hipStream_t)stream));
  return ok();
}

// ---- plans -------------------------------------------------------------------

int hesp_plan_create(hesp_plan** plan, const hesp_plan_opts* opts) {
  if (!plan) return fail(HESP_EINVAL, "hesp_plan_create: null plan");
  hesp_plan* p = new (std::nothrow) hesp_plan();
  if (!p) return fail(HESP_ENOMEM, "hesp_plan_create: out of host memory");
  if (opts) p->opts = *opts;
  if (p->opts.slots < 0 || p->opts.max_tasks < 0 || p->opts.max_edges < 0 || p->opts.chunks < 0 ||
      (p->opts.group != 0 && p->opts.group != 16 && p->opts.group != 32 && p->opts.group != 64) ||
      p->opts.prep_edges < 0 || p->opts.prep_edges > 1024 || p->opts.fuse < 0 || p->opts.fuse > 2 || (p->opts.fuse && p->opts.group != 0 && p->opts.group != 64)) {
    delete p;
    return fail(HESP_EINVAL, "hesp_plan_create: negative option");
  }
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) {
    delete p;
    return fail(HESP_EHIP, "hesp_plan_create: %s", hipGetErrorString(e));
  }
  p->slots = p->opts.slots ? p->opts.slots : 32 * cus;
  p->resident64 = std::min(p->slots, 16 * cus);
  p->chunk = 1 << 22;   // bounded by device memory below
  e = hipMalloc(&p->counter, sizeof(uint32_t));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->s_prep, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->s_sim, hipStreamNonBlocking);
  if (e != hipSuccess) {
    hfree(p->counter);
    if (p->s_prep) (void)hipStreamDestroy(p->s_prep);
    delete p;
    return fail(HESP_ENOMEM, "hesp_plan_create: %s", hipGetErrorString(e));
  }
  *plan = p;
  return ok();
}

int hesp_plan_destroy(hesp_plan* p) {
  if (!p) return ok();
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->sync_ev) (void)hipEventDestroy(e);
  if (p->s_prep) (void)hipStreamDestroy(p->s_prep);
  if (p->s_sim) (void)hipStreamDestroy(p->s_sim);
  p->release();
  hfree(p->counter);
  delete p;
  return ok();
}

int hesp_plan_bytes(const hesp_plan* p, int64_t* bytes) {
  if (!p || !bytes) return fail(HESP_EINVAL, "hesp_plan_bytes: null argument");
  *bytes = p->held();
  return ok();
}

int hesp_plan_timing(hesp_plan* p, int32_t enable) {
  if (!p) return fail(HESP_EINVAL, "hesp_plan_timing: null plan");
  p->timing = enable != 0;
  p->ev_used = 0;
  return ok();
}

int hesp_plan_last_ms(hesp_plan* p, double* ms) {
  if (!p || !ms) return fail(HESP_EINVAL, "hesp_plan_last_ms: null argument");
  ms[0] = ms[1] = ms[2] = 0.0;
  for (size_t i = 0; i + 4 <= p->ev_used; i += 4) {
    HIP_TRY(hipEventSynchronize(p->ev[i + 3]));
    HIP_TRY(hipEventSynchronize(p->ev[i + 1]));
    float a = 0.f, b = 0.f;
    HIP_TRY(hipEventElapsedTime(&a, p->ev[i], p->ev[i + 1]));
    HIP_TRY(hipEventElapsedTime(&b, p->ev[i + 2], p->ev[i + 3]));
    ms[0] += a;
    ms[1] += b;
    ms[2] += 1.0;
  }
  return ok();
}

static int build_tables(const hesp_platform* pf, SimTables& t) {
  if (!pf) return fail(HESP_EINVAL, "hesp_simulate_batch: null platform");
  if (pf->n_procs < 1 || pf->n_procs > HESP_MAX_PROCS || pf->n_ptypes < 1 || pf->n_ptypes > HESP_MAX_PTYPES ||
      pf->n_mem < 1 || pf->n_mem > HESP_MAX_MEM || pf->max_level < 0 || pf->max_level > HESP_MAX_LEVEL ||
      !pf->proc_type || !pf->proc_mem || !pf->cost_ns || !pf->xfer_ns)
    return fail(HESP_EINVAL, "hesp_simulate_batch: bad platform description");
  memset(&t, 0, sizeof t);
  t.n_procs = pf->n_procs;
  t.n_ptypes = pf->n_ptypes;
  t.n_mem = pf->n_mem;
  t.max_level = pf->max_level;
  const int L = pf->max_level + 1;
  for (int p = 0; p < pf->n_procs; p++) {
    if (pf->proc_type[p] < 0 || pf->proc_type[p] >= pf->n_ptypes || pf->proc_mem[p] < 0 ||
        pf->proc_mem[p] >= pf->n_mem)
      return fail(HESP_EINVAL, "hesp_simulate_batch: processor %d has a bad type or memory space", p);
    t.proc_type[p] = (int8_t)pf->proc_type[p];
    t.proc_mem[p] = (int8_t)pf->proc_mem[p];
  }
  for (int pt = 0; pt < pf->n_ptypes; pt++)
    for (int k = 0; k < 4; k++)
      for (int l = 0; l < L; l++) {
        const int64_t c = pf->cost_ns[(pt * 4 + k) * L + l];
        if (c < 1 || c > ((int64_t)1 << 40)) return fail(HESP_EINVAL, "hesp_simulate_batch: task time out of range");
        t.cost[pt][k][l] = c;
      }
  for (int p = 0; p < pf->n_procs; p++)
    for (int k = 0; k < 4; k++)
      for (int l = 0; l < L; l++) t.W[k][l] += t.cost[t.proc_type[p]][k][l];
  const int64_t nx = pow4(pf->max_level) + 1;
  if (pf->xfer_ns[0] != 0) return fail(HESP_EINVAL, "hesp_simulate_batch: xfer_ns[0] must be 0");
  for (int64_t k = 0; k < nx; k++) {
    if (pf->xfer_ns[k] < 0 || pf->xfer_ns[k] > ((int64_t)1 << 40) || (k > 0 && pf->xfer_ns[k] < pf->xfer_ns[k - 1]))
      return fail(HESP_EINVAL, "hesp_simulate_batch: xfer_ns must be non-decreasing and in range");
    if (k < kXferLen) t.xfer[k] = pf->xfer_ns[k];
  }
  t.xfer_deep = nullptr;   // set by the caller for tables deeper than kXferLevels
  for (int m = 0; m < kMaxMem; m++) {
    t.capacity[m] = (m > 0 && m < pf->n_mem && pf->capacity && pf->capacity[m] > 0) ? pf->capacity[m] : -1;
    if (t.capacity[m] >= 0) t.capped = 1;
  }
  for (int m = 0; m < pf->n_mem; m++) {
    if (pf->link && (pf->link[m] < 0 || pf->link[m] >= pf->n_mem))
      return fail(HESP_EINVAL, "hesp_simulate_batch: link[%d] must be in 0..n_mem-1", m);
    t.link[m] = pf->link ? (int8_t)pf->link[m] : 0;
  }
  return HESP_OK;
}

static OutView ov_of(const hesp_outputs* o) {
  return OutView{o->d_makespan, o->d_status, o->d_n_tasks, o->d_sched_off, o->d_proc, o->d_start, o->d_finish};
}

// argument checks and launch tables shared by the batch entry points (depth
// batches, or split-tree batches when tree is given)
int hesp_internal_batch_setup(const hesp_platform* pf, hesp_policy policy, const hesp_batch* batch,
                              const hesp_tree_batch* tree, const hesp_outputs* out, SimTables& tb, BatchView& bv) {
  if ((policy.order != HESP_ORDER_PL && policy.order != HESP_ORDER_FCFS) || policy.select < HESP_SELECT_EFT ||
      policy.select > HESP_SELECT_FP || policy.cache < HESP_CACHE_WB || policy.cache > HESP_CACHE_WA ||
      policy.bus < 0 || policy.bus > 1)
    return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch: PL or FCFS order, EFT-P, EIT-P, R-P or F-P selection, "
                                   "WB, WT or WA caching, bus 0 or 1");
  if (int r = build_tables(pf, tb)) return r;
  tb.fcfs = policy.order == HESP_ORDER_FCFS;
  tb.sel = policy.select;
  tb.seed = policy.seed;
  tb.cache = policy.cache;
  tb.bus = policy.bus;
  if (tb.capped && (tree || policy.cache != HESP_CACHE_WB || policy.select != HESP_SELECT_EFT || policy.bus))
    return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch: finite memory spaces take depth batches, write-back "
                                   "caching, EFT-P and independent transfers");
  if (int r = tree ? tree_view(tree, bv, "hesp_simulate_tree_batch") : batch_view(batch, bv, "hesp_simulate_batch"))
    return r;
  if (bv.dmax > pf->max_level) return fail(HESP_EINVAL, "hesp_simulate_batch: dmax above the platform's max_level");
  if (!out || !out->d_makespan || !out->d_status) return fail(HESP_EINVAL, "hesp_simulate_batch: null outputs");
  if (out->d_sched_off && (!out->d_proc || !out->d_start || !out->d_finish))
    return fail(HESP_EINVAL, "hesp_simulate_batch: schedule outputs need proc, start and finish");
  return HESP_OK;
}

// The pipeline with a separate preparation launch, on the first n candidates
// (their counts are in the plan): exact per-candidate layout, memory chunks,
// per chunk the preparation and the event loop with `group` lanes per candidate.
static int run_unfused(hesp_plan* plan, const SimTables& tb, BatchView bv, bool is_tree, const hesp_platform* pf,
                       const OutView& ov, hipStream_t s, int32_t n) {
  bv.n_cand = n;
  for (DevBuf* b : {&plan->off_t, &plan->off_e, &plan->off_v, &plan->off_top}) HIP_TRY(b->ensure(8 * ((int64_t)n + 1)));
  // the fused pipeline's arena is not given back to this path
  const int64_t held = plan->held() - plan->arena.bytes;
  auto prepare = [&](const ChunkView& cv, hipStream_t st) {
    return is_tree ? launch_prepare_tree(tb, bv, cv, ov, st) : launch_prepare(tb, bv, cv, ov, st);
  };
  HIP_TRY(plan->layout_part.ensure(8 * 5 * (((int64_t)n + 1023) / 1024)));
  HIP_TRY(launch_layout(bv, pf->n_mem, plan->cnt_tasks.as<int32_t>(), plan->cnt_edges.as<int64_t>(),
                        plan->opts.max_tasks, plan->opts.max_edges, plan->off_t.as<int64_t>(),
                        plan->off_e.as<int64_t>(), plan->off_v.as<int64_t>(), plan->off_top.as<int64_t>(), nullptr,
                        s, plan->layout_part.as<int64_t>()));

  // chunk boundaries: the largest chunk must fit the memory budget
  const bool fixed = plan->opts.max_tasks > 0 && plan->opts.max_edges > 0;
  int32_t chunk = std::min<int32_t>(plan->chunk, n);
  if (plan->opts.chunks > 1) chunk = std::min<int32_t>(chunk, (n + plan->opts.chunks - 1) / plan->opts.chunks);
  int32_t n_chunks = 0;
  int64_t mT = 0, mE = 0, mV = 0, mP = 0;
  if (fixed) {
    // fixed capacities: sizes follow from the plan and the batch shape alone, so
    // nothing is read back and nothing is allocated once the plan has seen a
    // batch of this shape and size (the call can be captured in a HIP graph)
    const int64_t cT = plan->opts.max_tasks, cE = plan->opts.max_edges;
    const int64_t cV = ((int64_t)tri2(bv.nt) << (2 * bv.dmax)) * pf->n_mem, cP = tet3(bv.nt) + 1;
    const int64_t per = 104 * cT + 4 * cE + (tb.capped ? 20 : 8) * cV + 4 * cP + 24 + 4;
    const auto key = std::make_tuple(n, cV, cP);
    if (plan->fixed_key != key) {
      size_t free_b = 0, total_b = 0;
      HIP_TRY(hipMemGetInfo(&free_b, &total_b));
      const int64_t budget = (int64_t)(free_b + (size_t)held) / 2;
      const int64_t want = plan->opts.chunks > 1 ? (n + plan->opts.chunks - 1) / plan->opts.chunks : n;
      plan->fixed_chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(want, budget / (2 * per)));
      plan->fixed_key = key;
    }
    chunk = plan->fixed_chunk;
    n_chunks = (n + chunk - 1) / chunk;
    mT = cT * chunk;
    mE = cE * chunk;
    mV = cV * chunk;
    mP = cP * chunk;
  }
  size_t free_b = 0, total_b = 0;
  if (!fixed) HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  const int64_t budget = (int64_t)(free_b + (size_t)held) / 2;
  for (; !fixed;) {
    n_chunks = (n + chunk - 1) / chunk;
    HIP_TRY(plan->bounds.ensure(4 * 8 * ((int64_t)n_chunks + 1)));
    HIP_TRY(launch_bounds(plan->off_t.as<int64_t>(), plan->off_e.as<int64_t>(), plan->off_v.as<int64_t>(),
                          plan->off_top.as<int64_t>(), n, chunk, n_chunks, plan->bounds.as<int64_t>(), s));
    plan->h_bounds.resize(4 * ((size_t)n_chunks + 1));
    HIP_TRY(hipMemcpyAsync(plan->h_bounds.data(), plan->bounds.p, 8 * plan->h_bounds.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int64_t* hb = plan->h_bounds.data();
    mT = mE = mV = mP = 0;
    for (int i = 0; i < n_chunks; i++) {
      mT = std::max(mT, hb[0 * (n_chunks + 1) + i + 1] - hb[0 * (n_chunks + 1) + i]);
      mE = std::max(mE, hb[1 * (n_chunks + 1) + i + 1] - hb[1 * (n_chunks + 1) + i]);
      mV = std::max(mV, hb[2 * (n_chunks + 1) + i + 1] - hb[2 * (n_chunks + 1) + i]);
      mP = std::max(mP, hb[3 * (n_chunks + 1) + i + 1] - hb[3 * (n_chunks + 1) + i]);
    }
    // two workspace sets when chunks overlap
    const int64_t bytes =
        (n_chunks > 1 ? 2 : 1) * (104 * mT + 4 * mE + (tb.capped ? 20 : 8) * mV + 4 * mP + 24 * (int64_t)chunk);
    if (bytes <= budget || chunk == 1) {
      if (bytes > budget) return fail(HESP_ENOMEM, "hesp_simulate_batch: one candidate needs %lld bytes", (long long)bytes);
      break;
    }
    chunk = (chunk + 1) / 2;
  }
  for (int k = 0; k < (n_chunks > 1 ? 2 : 1); k++) {
    WorkSet& w = plan->ws[k];
    HIP_TRY(w.top_first.ensure(4 * mP));
    HIP_TRY(w.desc.ensure(4 * mT));
    HIP_TRY(w.indeg.ensure(4 * mT));
    HIP_TRY(w.cur.ensure(4 * mT));
    HIP_TRY(w.succ.ensure(4 * mE));
    HIP_TRY(w.rec.ensure(32 * mT));
    HIP_TRY(w.fifo.ensure(24 * mT));
    HIP_TRY(w.ready.ensure(4 * mT));
    HIP_TRY(w.sortbuf.ensure(32 * mT));
    HIP_TRY(w.vf.ensure(8 * mV));
    if (tb.capped) {
      HIP_TRY(w.use.ensure(8 * mV));
      HIP_TRY(w.pin.ensure(4 * mV));
    }
    HIP_TRY(w.nsrc.ensure(4 * (int64_t)chunk));
    HIP_TRY(w.order_keys.ensure(8 * srch::sort_len(chunk)));
    HIP_TRY(w.order.ensure(4 * (int64_t)chunk));
  }

  auto chunk_view = [&](int32_t c0, int32_t nc, int set) {
    WorkSet& w = plan->ws[set];
    ChunkView cv{};
    cv.task_off = plan->off_t.as<int64_t>();
    cv.edge_off = plan->off_e.as<int64_t>();
    cv.vf_off = plan->off_v.as<int64_t>();
    cv.top_off = plan->off_top.as<int64_t>();
    cv.c0 = c0;
    cv.nc = nc;
    cv.cap_tasks = plan->opts.max_tasks;
    cv.cap_edges = plan->opts.max_edges;
    cv.prep_in = plan->opts.prep_edges;
    cv.top_first = w.top_first.as<uint32_t>();
    cv.desc = w.desc.as<uint32_t>();
    cv.indeg = w.indeg.as<uint32_t>();
    cv.cur = w.cur.as<uint32_t>();
    cv.succ = w.succ.as<uint32_t>();
    cv.rec = w.rec.as<int64_t>();
    cv.fifo = w.fifo.as<int64_t>();
    cv.ready = w.ready.as<uint32_t>();
    cv.sortbuf = w.sortbuf.as<int64_t>();
    cv.vf = w.vf.as<int64_t>();
    cv.use = tb.capped ? w.use.as<int64_t>() : nullptr;
    cv.pin = tb.capped ? w.pin.as<uint32_t>() : nullptr;
    cv.nsrc = w.nsrc.as<int32_t>();
    cv.cnt_tasks = plan->cnt_tasks.as<int32_t>();
    cv.cnt_edges = plan->cnt_edges.as<int64_t>();
    return cv;
  };


  // lanes per candidate: forced by the plan, or timed once per batch shape on a
  // sub-batch of the first chunk (outputs of that sub-batch are rewritten below)
  int group = plan->opts.group;
  if (tb.capped) {
    // finite spaces: the event loop keeps its per-space state in whole-wave groups
    if (group != 0 && group != 64)
      return fail(HESP_EINVAL, "hesp_simulate_batch: finite memory spaces take 64 lanes per candidate");
    group = 64;
  }
  if (group == 0) {
    const auto key = std::make_tuple(pf->n_procs, pf->n_mem, bv.nt, bv.dmax, (bv.nt_arr ? 1 : 0) | (is_tree ? 2 : 0));
    auto it = plan->tuned.find(key);
    if (it != plan->tuned.end()) {
      group = it->second;
    } else {
      // the timing calls synchronise the stream: a captured call takes the choice
      // an earlier call of the same shape made
      hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
      HIP_TRY(hipStreamIsCapturing(s, &cs));
      if (cs != hipStreamCaptureStatusNone)
        return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch: a captured call with group 0 needs an earlier call "
                                       "of the same batch shape (which chooses the lanes per candidate)");
      const int32_t sub = std::min<int32_t>(std::min(chunk, n), 8192);
      float best_ms = 0.f;
      hipEvent_t e0, e1;
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      for (int G : {16, 32, 64}) {
        if (G < pf->n_procs) continue;
        ChunkView cv = chunk_view(0, sub, 0);
        HIP_TRY(prepare(cv, s));
        HIP_TRY(hipEventRecord(e0, s));
        HIP_TRY(launch_sim(tb, bv, cv, ov, plan->slots, G, plan->counter, s));
        HIP_TRY(hipEventRecord(e1, s));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (group == 0 || ms < best_ms) {
          best_ms = ms;
          group = G;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      plan->tuned[key] = group;
    }
  } else if (group < pf->n_procs) {
    return fail(HESP_EINVAL, "hesp_simulate_batch: %d lanes per candidate < %d processors", group, pf->n_procs);
  }

  plan->ev_used = 0;
  if (plan->timing)
    while (plan->ev.size() < 4 * (size_t)n_chunks) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      plan->ev.push_back(e);
    }
  while (plan->sync_ev.size() < 2 + 2 * (size_t)n_chunks) {
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    plan->sync_ev.push_back(e);
  }
  // fork: preparation and simulation run on the plan's two streams, chunk i+1
  // being prepared (into the other workspace set) while chunk i is simulated;
  // the caller's stream then waits for the last operation of both streams.  A
  // call being captured into a graph keeps every chunk on the caller's stream
  // (stream order alone keeps a workspace set from being reused early): the
  // capture holds only kernel nodes, and no event recorded outside it.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  const bool timing = plan->timing && !capturing;
  // a single chunk has nothing to overlap: it stays on the caller's stream
  const bool fork = !capturing && n_chunks > 1;
  hipStream_t sp = fork ? plan->s_prep : s, ss = fork ? plan->s_sim : s;
  hipEvent_t* se = plan->sync_ev.data();
  if (fork) {
    HIP_TRY(hipEventRecord(se[0], s));
    HIP_TRY(hipStreamWaitEvent(sp, se[0], 0));
    HIP_TRY(hipStreamWaitEvent(ss, se[0], 0));
  }
  for (int i = 0; i < n_chunks; i++) {
    const int set = i & 1;
    ChunkView cv = chunk_view(i * chunk, std::min(chunk, n - i * chunk), set);
    if (fork && i >= 2) HIP_TRY(hipStreamWaitEvent(sp, se[2 + 2 * (i - 2)], 0));   // set free again
    if (timing) HIP_TRY(hipEventRecord(plan->ev[4 * i], sp));
    // largest candidates first, so that the persistent launch does not end on a long one
    HIP_TRY(srch::size_order(plan->cnt_tasks.as<int32_t>(), cv.c0, cv.nc, plan->ws[set].order_keys.as<uint64_t>(),
                             plan->ws[set].order.as<uint32_t>(), sp));
    cv.order = plan->ws[set].order.as<uint32_t>();
    HIP_TRY(prepare(cv, sp));
    if (timing) HIP_TRY(hipEventRecord(plan->ev[4 * i + 1], sp));
    if (fork) {
      HIP_TRY(hipEventRecord(se[1 + 2 * i], sp));
      HIP_TRY(hipStreamWaitEvent(ss, se[1 + 2 * i], 0));
    }
    if (timing) HIP_TRY(hipEventRecord(plan->ev[4 * i + 2], ss));
    HIP_TRY(launch_sim(tb, bv, cv, ov, plan->slots, group, plan->counter, ss));
    if (timing) HIP_TRY(hipEventRecord(plan->ev[4 * i + 3], ss));
    if (fork) HIP_TRY(hipEventRecord(se[2 + 2 * i], ss));
    if (timing) plan->ev_used = 4 * (size_t)(i + 1);
  }
  if (fork) {
    HIP_TRY(hipEventRecord(se[1 + 2 * n_chunks], sp));
    HIP_TRY(hipStreamWaitEvent(s, se[2 * n_chunks], 0));
    HIP_TRY(hipStreamWaitEvent(s, se[1 + 2 * n_chunks], 0));
  }
  return ok();
}

// The fused pipeline on the first n candidates (depth batches, 64 lanes per
// candidate): one launch of the persistent event loop, each wave preparing the
// candidates it takes into its own slot of the plan's arena.  The slot holds the
// largest candidate of the batch (read back: one synchronisation of `s`), or, in
// a fixed-capacity plan, the largest allowed by the capacities (no read-back, no
// allocation after the first call of a shape: capturable).  Waves: the ones that
// are resident at once, fewer if the arena would not fit half the free memory.
static int run_fused(hesp_plan* plan, const SimTables& tb, BatchView bv, const OutView& ov, hipStream_t s,
                     int32_t n) {
  bv.n_cand = n;
  const bool fixed = plan->opts.max_tasks > 0 && plan->opts.max_edges > 0;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(s, &cap));
  if (cap != hipStreamCaptureStatusNone && !fixed)
    return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch: a captured call needs a fixed-capacity plan");
  const int64_t V = ((int64_t)tri2(bv.nt) << (2 * bv.dmax)) * tb.n_mem, TP = tet3(bv.nt) + 1;
  int64_t slot = 0;
  int32_t waves = 0;
  if (fixed) {
    slot = region_bytes(plan->opts.max_tasks, plan->opts.max_edges, V, TP);
    const auto key = std::make_tuple((int64_t)n, slot, (int64_t)-2);
    if (plan->fused_key == key) waves = plan->fused_waves;
  } else {
    HIP_TRY(plan->bounds.ensure(64));
    HIP_TRY(launch_max_region(bv, tb.n_mem, plan->cnt_tasks.as<int32_t>(), plan->cnt_edges.as<int64_t>(),
                              plan->bounds.as<int64_t>(), s));
    int64_t mx = 0;
    HIP_TRY(hipMemcpyAsync(&mx, plan->bounds.p, sizeof mx, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    slot = mx;
  }
  slot = std::max<int64_t>(256, (slot + 255) & ~(int64_t)255);
  const bool in_lds = plan->opts.fuse == 2;
  // LDS slots: candidates whose workspace exceeds the largest slot get HESP_ECAPACITY
  if (in_lds) slot = std::min<int64_t>(slot, kLdsSlotMax);
  if (in_lds) waves = std::min<int32_t>(n, plan->resident64);
  if (waves == 0) {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const int64_t budget = (int64_t)(free_b + (size_t)plan->arena.bytes) / 2;
    waves = std::min<int32_t>(n, plan->resident64);
    while (waves > 1 && (int64_t)waves * slot > budget) waves = (waves + 1) / 2;
    if ((int64_t)waves * slot > budget)
      return fail(HESP_ENOMEM, "hesp_simulate_batch: one candidate needs %lld bytes", (long long)slot);
    if (fixed) {
      plan->fused_key = std::make_tuple((int64_t)n, slot, (int64_t)-2);
      plan->fused_waves = waves;
    }
  }
  if (!in_lds) HIP_TRY(plan->arena.ensure((int64_t)waves * slot));
  WorkSet& w = plan->ws[0];
  HIP_TRY(w.order_keys.ensure(8 * srch::sort_len(n)));
  HIP_TRY(w.order.ensure(4 * (int64_t)n));
  // largest candidates first, so that the persistent launch does not end on a long one
  HIP_TRY(srch::size_order(plan->cnt_tasks.as<int32_t>(), 0, n, w.order_keys.as<uint64_t>(), w.order.as<uint32_t>(), s));
  ChunkView cv{};
  cv.c0 = 0;
  cv.nc = n;
  cv.cap_tasks = plan->opts.max_tasks;
  cv.cap_edges = plan->opts.max_edges;
  cv.prep_in = plan->opts.prep_edges;
  cv.cnt_tasks = plan->cnt_tasks.as<int32_t>();
  cv.cnt_edges = plan->cnt_edges.as<int64_t>();
  cv.order = w.order.as<uint32_t>();
  cv.region = in_lds ? nullptr : plan->arena.as<uint8_t>();
  cv.slot_bytes = slot;
  cv.slot_lds = in_lds ? 1 : 0;
  plan->ev_used = 0;
  if (plan->timing)
    while (plan->ev.size() < 4) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      plan->ev.push_back(e);
    }
  if (plan->timing) {
    HIP_TRY(hipEventRecord(plan->ev[0], s));   // no separate preparation: an empty interval
    HIP_TRY(hipEventRecord(plan->ev[1], s));
    HIP_TRY(hipEventRecord(plan->ev[2], s));
  }
  HIP_TRY(launch_sim(tb, bv, cv, ov, waves, 64, plan->counter, s));
  if (plan->timing) {
    HIP_TRY(hipEventRecord(plan->ev[3], s));
    plan->ev_used = 4;
  }
  return ok();
}

// Transfer times beyond the first kXferLen entries (platforms deeper than
// kXferLevels): a device copy held by the plan, made on the call's stream and
// remade only when the table changes (after the stream has drained, so that no
// earlier copy still reads the host table).  A captured call finds the copy made
// by an earlier call on the same table, or fails.
static int deep_xfer(hesp_plan* plan, const hesp_platform* pf, SimTables& tb, hipStream_t s) {
  const int64_t nx = pow4(pf->max_level) + 1;
  if ((int64_t)plan->xfer_host.size() != nx ||
      memcmp(plan->xfer_host.data(), pf->xfer_ns, (size_t)nx * sizeof(int64_t)) != 0) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cap));
    if (cap != hipStreamCaptureStatusNone)
      return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch: a captured call on a platform with max_level above %d "
                                     "needs an earlier call with the same transfer table", kXferLevels);
    HIP_TRY(hipStreamSynchronize(s));
    plan->xfer_host.assign(pf->xfer_ns, pf->xfer_ns + nx);
    HIP_TRY(plan->xfer_deep.ensure(8 * (pow4(kMaxLevel) + 1)));
    HIP_TRY(hipMemcpyAsync(plan->xfer_deep.p, plan->xfer_host.data(), (size_t)nx * sizeof(int64_t),
                           hipMemcpyHostToDevice, s));
  }
  tb.xfer_deep = plan->xfer_deep.as<int64_t>();
  return HESP_OK;
}

// depth batches (batch) or split-tree batches (tree)
static int simulate_any(hesp_plan* plan, const hesp_platform* pf, hesp_policy policy, const hesp_batch* batch,
                        const hesp_tree_batch* tree, const hesp_outputs* out, void* stream) {
  if (!plan) return fail(HESP_EINVAL, "hesp_simulate_batch: null plan");
  SimTables tb;
  BatchView bv;
  if (int r = hesp_internal_batch_setup(pf, policy, batch, tree, out, tb, bv)) return r;
  const bool is_tree = tree != nullptr;
  const int n = bv.n_cand;
  if (n == 0) return ok();
  hipStream_t s = (hipStream_t)stream;
  const OutView ov = ov_of(out);
  if (tb.max_level > kXferLevels)
    if (int r = deep_xfer(plan, pf, tb, s)) return r;

  // exact sizes of every candidate
  HIP_TRY(plan->cnt_tasks.ensure(4 * (int64_t)n));
  HIP_TRY(plan->cnt_edges.ensure(8 * (int64_t)n));
  if (is_tree) {
    HIP_TRY(plan->tree_lw.ensure(4 * (int64_t)n * ((int64_t)tri2(bv.nt) << (2 * bv.dmax))));
    HIP_TRY(launch_count_tree(bv, plan->tree_lw.as<uint32_t>(), plan->cnt_tasks.as<int32_t>(),
                              plan->cnt_edges.as<int64_t>(), s));
  } else {
    HIP_TRY(launch_count(bv, plan->cnt_tasks.as<int32_t>(), plan->cnt_edges.as<int64_t>(), s));
  }

  // the fused pipeline on request (depth batches, 64 lanes per candidate), else
  // separate preparation and simulation launches per memory chunk
  if (plan->opts.fuse) {
    if (is_tree) return fail(HESP_EUNSUPPORTED, "hesp_simulate_tree_batch: the fused pipeline takes depth batches");
    if (tb.capped) return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch: the fused pipeline has no finite spaces");
    if (bv.dmax > kMaxWaveLevel || tb.max_level > kXferLevels)
      return fail(HESP_EUNSUPPORTED, "hesp_simulate_batch: the fused pipeline takes depths and platform levels up to "
                                     "%d", kMaxWaveLevel);
    if (pf->n_procs > 64) return fail(HESP_EINVAL, "hesp_simulate_batch: more than 64 processors");
    return run_fused(plan, tb, bv, ov, s, n);
  }
  return run_unfused(plan, tb, bv, is_tree, pf, ov, s, n);
}

int hesp_simulate_batch(hesp_plan* plan, const hesp_platform* pf, hesp_policy policy, const hesp_batch* batch,
                        const hesp_outputs* out, void* stream) {
  if (!batch) return fail(HESP_EINVAL, "hesp_simulate_batch: null batch");
  return simulate_any(plan, pf, policy, batch, nullptr, out, stream);
}

int hesp_simulate_tree_batch(hesp_plan* plan, const hesp_platform* pf, hesp_policy policy,
                             const hesp_tree_batch* batch, const hesp_outputs* out, void* stream) {
  if (!batch) return fail(HESP_EINVAL, "hesp_simulate_tree_batch: null batch");
  return simulate_any(plan, pf, policy, nullptr, batch, out, stream);
}

int64_t hesp_tree_flag_count(int32_t nt, int32_t dmax) {
  if (nt < 1 || dmax < 0 || dmax > HESP_MAX_LEVEL) return -1;
  int64_t n = 0;
  for (int l = 0; l < dmax; l++) n += tet3((int64_t)nt << l);
  return n;
}

int hesp_generate_tree_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt, int32_t dmax,
                               uint32_t split_thr, uint8_t* d_flags, void* stream) {
  const int64_t nf = hesp_tree_flag_count(nt, dmax);
  if (n_cand < 0 || nf < 0 || first < 0 || (nt << dmax) > HESP_MAX_FINE || (!d_flags && n_cand > 0 && nf > 0))
    return fail(HESP_EINVAL, "hesp_generate_tree_uniform: bad argument");
  if (check_thr(split_thr)) return HESP_EINVAL;
  HIP_TRY(launch_gen_tree(seed, first, n_cand, nf, split_thr, d_flags, (hipStream_t)stream));
  return ok();
}

int hesp_count_tree_batch(const hesp_tree_batch* batch, int32_t* d_n_tasks, int64_t* d_n_edges, void* stream) {
  BatchView bv;
  if (int r = tree_view(batch, bv, "hesp_count_tree_batch")) return r;
  if (bv.n_cand == 0) return ok();
  if (!d_n_tasks || !d_n_edges) return fail(HESP_EINVAL, "hesp_count_tree_batch: null outputs");
  hipStream_t s = (hipStream_t)stream;
  void* lw = nullptr;
  HIP_TRY(hipMalloc(&lw, 4 * (size_t)bv.n_cand * ((size_t)tri2(bv.nt) << (2 * bv.dmax))));
  hipError_t e = launch_count_tree(bv, (uint32_t*)lw, d_n_tasks, d_n_edges, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(lw);
  if (e != hipSuccess) return fail(HESP_EHIP, "hesp_count_tree_batch: %s", hipGetErrorString(e));
  return ok();
}

int hesp_argmin(const int64_t* d_makespan, int32_t n, int64_t* d_best, void* stream) {
  if (n < 0 || !d_best || (n > 0 && !d_makespan)) return fail(HESP_EINVAL, "hesp_argmin: bad argument");
  HIP_TRY(launch_argmin(d_makespan, n, d_best, (hipStream_t)stream));
  return ok();
}

}  // extern "C"
