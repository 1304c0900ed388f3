// hesp_solve_api.cpp -- C ABI of the iterative scheduler-partitioner
// (include/hesp.h, hesp_solve): the schedule stage is the batched simulation,
// the partition stage the kernels of hesp_solve.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "hesp.h"
#include "hesp_core.h"
#include "hesp_solve.h"

using namespace hesp;

extern "C" int hesp_internal_fail(int code, const char* msg);

namespace {

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return hesp_internal_fail(code, buf);
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return fail(HESP_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define RC_TRY(expr)        \
  do {                      \
    int r_ = (expr);        \
    if (r_) return r_;      \
  } while (0)

// device allocations of one call, freed on every exit path once the stream is idle
struct Scratch {
  hipStream_t s = nullptr;
  std::vector<void*> ptrs;
  ~Scratch() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(s);
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t get(T** out, int64_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)std::max<int64_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) {
      ptrs.push_back(p);
      *out = (T*)p;
    }
    return e;
  }
};

}  // namespace

extern "C" {

// argument checks and the cost tables shared by both solvers; n_cl = clusters per
// chain; depths and platform levels up to max_depth
static int solve_setup(hesp_plan* plan, const hesp_platform* pf, const hesp_solve_params* sp, int64_t n_cl,
                       const void* d_part, const void* d_best, const int64_t* d_best_makespan, const char* who,
                       int max_depth, solve::SolveTables& tb) {
  if (!plan || !pf || !sp) return fail(HESP_EINVAL, "%s: null plan, platform or parameters", who);
  const int B = sp->n_chains, nt = sp->nt, dmax = sp->dmax;
  if (B < 1 || B > 65535 || nt < 1 || dmax < 0 || dmax > max_depth || (nt << dmax) > kMaxFine || sp->iters < 1)
    return fail(HESP_EINVAL, "%s: need 1 <= n_chains <= 65535, nt >= 1, 0 <= dmax <= %d, iters >= 1", who,
                max_depth);
  if (sp->list < HESP_LIST_ALL || sp->list > HESP_LIST_SHALLOW || sp->sampling < HESP_SAMPLE_HARD ||
      sp->sampling > HESP_SAMPLE_SOFT)
    return fail(HESP_EINVAL, "%s: list must be ALL, CP or SHALLOW and sampling HARD or SOFT", who);
  if (n_cl > solve::kMaxTop) return fail(HESP_EUNSUPPORTED, "%s: more than %d clusters per chain", who, solve::kMaxTop);
  if (!d_part || !d_best || !d_best_makespan) return fail(HESP_EINVAL, "%s: null outputs", who);
  if (pf->n_procs < 1 || pf->n_procs > std::min<int>(HESP_MAX_PROCS, solve::kMaxP) || pf->n_ptypes < 1 ||
      pf->n_ptypes > std::min<int>(HESP_MAX_PTYPES, solve::kMaxTypes) || pf->max_level < dmax ||
      pf->max_level > max_depth || !pf->proc_type || !pf->cost_ns)
    return fail(HESP_EINVAL, "%s: bad platform description (or dmax above its max_level)", who);
  memset(&tb, 0, sizeof tb);
  tb.n_procs = pf->n_procs;
  for (int p = 0; p < pf->n_procs; p++) {
    if (pf->proc_type[p] < 0 || pf->proc_type[p] >= pf->n_ptypes)
      return fail(HESP_EINVAL, "%s: processor %d has a bad type", who, p);
    tb.proc_type[p] = (int8_t)pf->proc_type[p];
  }
  const int L = pf->max_level + 1;
  for (int t = 0; t < pf->n_ptypes; t++)
    for (int k = 0; k < 4; k++)
      for (int l = 0; l <= dmax; l++) tb.cost[t][k][l] = pf->cost_ns[(t * 4 + k) * L + l];
  return HESP_OK;
}


// the solver's partition stage reads every task's schedule, which a candidate
// failing on a finite memory space does not have
static bool finite_spaces(const hesp_platform* pf) {
  if (!pf || !pf->capacity) return false;
  for (int m = 1; m < pf->n_mem; m++)
    if (pf->capacity[m] > 0) return true;
  return false;
}

int hesp_solve(hesp_plan* plan, const hesp_platform* pf, hesp_policy policy, const hesp_solve_params* sp,
               uint8_t* d_depth, uint8_t* d_best_depth, int64_t* d_best_makespan, int64_t* d_trace,
               int64_t* d_steps, void* stream) {
  if (!sp) return fail(HESP_EINVAL, "hesp_solve: null parameters");
  if (finite_spaces(pf)) return fail(HESP_EUNSUPPORTED, "hesp_solve: finite memory spaces are not supported");
  const int B = sp->n_chains, nt = sp->nt, dmax = sp->dmax;
  const int64_t n_top = nt >= 1 ? tet3(nt) : 0;
  solve::SolveTables tb;
  RC_TRY(solve_setup(plan, pf, sp, n_top, d_depth, d_best_depth, d_best_makespan, "hesp_solve", kMaxLevel, tb));

  hipStream_t s = (hipStream_t)stream;
  const int64_t max_tasks = tet3((int64_t)nt << dmax);   // a chain split to dmax everywhere
  const int64_t tasks = (int64_t)B * max_tasks;
  Scratch sc;
  sc.s = s;
  int32_t *cnt, *status, *proc, *par, *cl;
  int64_t *off, *ms, *start, *finish;
  uint32_t* first;
  uint64_t *t0key, *fin, *lastkey;
  HIP_TRY(sc.get(&cnt, B));
  HIP_TRY(sc.get(&status, B));
  HIP_TRY(sc.get(&off, (int64_t)B + 1));
  HIP_TRY(sc.get(&ms, B));
  HIP_TRY(sc.get(&proc, tasks));
  HIP_TRY(sc.get(&start, tasks));
  HIP_TRY(sc.get(&finish, tasks));
  HIP_TRY(sc.get(&par, tasks));
  HIP_TRY(sc.get(&cl, tasks));
  HIP_TRY(sc.get(&first, (int64_t)B * (n_top + 1)));
  HIP_TRY(sc.get(&t0key, (int64_t)B * n_top));
  HIP_TRY(sc.get(&fin, (int64_t)B * n_top));
  HIP_TRY(sc.get(&lastkey, B));

  // a chain that never simulates successfully keeps makespan -1 and its input
  HIP_TRY(hipMemsetAsync(d_best_makespan, 0xFF, 8 * (size_t)B, s));
  HIP_TRY(hipMemcpyAsync(d_best_depth, d_depth, (size_t)B * n_top, hipMemcpyDeviceToDevice, s));

  solve::SolveView v{};
  v.n_chains = B;
  v.nt = nt;
  v.dmax = dmax;
  v.n_top = (int32_t)n_top;
  v.iters = sp->iters;
  v.list = sp->list;
  v.sampling = sp->sampling;
  v.seed = sp->seed;
  v.depth = d_depth;
  v.best_depth = d_best_depth;
  v.best_ms = d_best_makespan;
  v.trace = d_trace;
  v.steps = d_steps;
  v.stride = max_tasks;
  v.n_tasks = cnt;
  v.proc = proc;
  v.start = start;
  v.finish = finish;
  v.makespan = ms;
  v.status = status;
  v.first = first;
  v.t0key = t0key;
  v.fin = fin;
  v.par = par;
  v.cl = cl;
  v.lastkey = lastkey;

  hesp_batch hb{B, nt, dmax, nullptr, nullptr, nullptr, d_depth};
  // chain r's schedule at r * max_tasks: no per-iteration offsets needed
  HIP_TRY(solve::launch_strided(max_tasks, B, off, s));
  hesp_outputs out{ms, status, cnt, off, proc, start, finish};
  for (int it = 0; it < sp->iters; it++) {
    // schedule stage: exact simulation of every chain's partition, with the
    // processor, start and finish of every task
    RC_TRY(hesp_simulate_batch(plan, pf, policy, &hb, &out, s));
    // partition stage
    v.iter = it;
    HIP_TRY(solve::launch_first(v, s));
    HIP_TRY(solve::launch_tasks(v, max_tasks, s));
    HIP_TRY(solve::launch_part(v, tb, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return HESP_OK;
}

int hesp_solve_tree(hesp_plan* plan, const hesp_platform* pf, hesp_policy policy, const hesp_solve_params* sp,
                    uint8_t* d_flags, uint8_t* d_best_flags, int64_t* d_best_makespan, int64_t* d_trace,
                    int64_t* d_steps, void* stream) {
  if (!sp) return fail(HESP_EINVAL, "hesp_solve_tree: null parameters");
  const int B = sp->n_chains, nt = sp->nt, dmax = sp->dmax;
  if (dmax < 1 || nt < 1 || dmax > kMaxLevel)
    return fail(HESP_EINVAL, "hesp_solve_tree: need 1 <= dmax <= %d (the clusters are the tasks above the last level)",
                kMaxLevel);
  const int64_t nn = hesp_tree_flag_count(nt, dmax);
  solve::SolveTables tb;
  RC_TRY(solve_setup(plan, pf, sp, nn, d_flags, d_best_flags, d_best_makespan, "hesp_solve_tree", kMaxLevel, tb));

  hipStream_t s = (hipStream_t)stream;
  const int64_t max_tasks = tet3((int64_t)nt << dmax);
  const int64_t tasks = (int64_t)B * max_tasks;
  const int64_t n_atoms = (int64_t)tri2(nt) << (2 * dmax);
  Scratch sc;
  sc.s = s;
  int32_t *cnt, *status, *proc, *par, *lmin;
  int64_t *off, *ms, *start, *finish;
  uint32_t *lw, *desc;
  uint64_t *t0key, *fin, *lastkey;
  HIP_TRY(sc.get(&cnt, B));
  HIP_TRY(sc.get(&status, B));
  HIP_TRY(sc.get(&off, (int64_t)B + 1));
  HIP_TRY(sc.get(&ms, B));
  HIP_TRY(sc.get(&proc, tasks));
  HIP_TRY(sc.get(&start, tasks));
  HIP_TRY(sc.get(&finish, tasks));
  HIP_TRY(sc.get(&par, tasks));
  HIP_TRY(sc.get(&desc, tasks));
  HIP_TRY(sc.get(&lw, (int64_t)B * n_atoms));
  HIP_TRY(sc.get(&t0key, (int64_t)B * nn));
  HIP_TRY(sc.get(&fin, (int64_t)B * nn));
  HIP_TRY(sc.get(&lastkey, B));
  HIP_TRY(sc.get(&lmin, B));
  HIP_TRY(hipMemsetAsync(d_best_makespan, 0xFF, 8 * (size_t)B, s));
  HIP_TRY(hipMemcpyAsync(d_best_flags, d_flags, (size_t)B * nn, hipMemcpyDeviceToDevice, s));

  solve::TreeSolveView v{};
  v.n_chains = B;
  v.nt = nt;
  v.dmax = dmax;
  v.n_nodes = (int32_t)nn;
  v.iters = sp->iters;
  v.list = sp->list;
  v.sampling = sp->sampling;
  v.seed = sp->seed;
  for (int l = 0; l <= dmax; l++) v.level_off[l] = hesp_tree_flag_count(nt, l);
  v.flags = d_flags;
  v.best_flags = d_best_flags;
  v.best_ms = d_best_makespan;
  v.trace = d_trace;
  v.steps = d_steps;
  v.stride = max_tasks;
  v.n_tasks = cnt;
  v.proc = proc;
  v.start = start;
  v.finish = finish;
  v.makespan = ms;
  v.status = status;
  v.lw = lw;
  v.desc = desc;
  v.par = par;
  v.t0key = t0key;
  v.fin = fin;
  v.lastkey = lastkey;
  v.lmin = lmin;

  hesp_tree_batch hb{B, nt, dmax, d_flags};
  HIP_TRY(solve::launch_strided(max_tasks, B, off, s));
  hesp_outputs out{ms, status, cnt, off, proc, start, finish};
  for (int it = 0; it < sp->iters; it++) {
    RC_TRY(hesp_simulate_tree_batch(plan, pf, policy, &hb, &out, s));
    v.iter = it;
    HIP_TRY(solve::launch_tree_init(v, s));
    HIP_TRY(solve::launch_tree_tasks(v, s));
    HIP_TRY(solve::launch_tree_part(v, tb, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  return HESP_OK;
}

}  // extern "C"
