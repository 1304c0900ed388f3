// hesp_search_api.cpp -- C ABI of candidate enumeration, top-k selection,
// surrogate features and the partition search driver (include/hesp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "hesp.h"
#include "hesp_core.h"
#include "hesp_mlp.h"
#include "hesp_search.h"

using namespace hesp;

extern "C" int hesp_internal_fail(int code, const char* msg);
extern "C" int hesp_internal_plan_capped(const hesp_plan* p);

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

// device allocations of one call, freed on every exit path
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
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

// kind | (k >= nt/2) << 2 of every top-level task, in the order of Fig. 1
std::vector<uint8_t> top_info(int nt) {
  std::vector<uint8_t> v((size_t)tet3(nt));
  for (int64_t t = 0; t < (int64_t)v.size(); t++) {
    const uint32_t c = top_cell(nt, t);
    const int k = cell_k(c);
    v[t] = (uint8_t)(kind_of(k, cell_i(c), cell_j(c)) | ((2 * k >= nt) ? 4 : 0));
  }
  return v;
}

int topk_common(int64_t n, int32_t k, const int32_t* d_idx, const void* d_ws, int64_t ws_bytes, const char* who) {
  if (n < 0 || n > (1 << 24) || k < 0 || k > n || (k > 0 && !d_idx))
    return fail(HESP_EINVAL, "%s: need 0 <= k <= n <= 2^24", who);
  if (n > 0 && (!d_ws || ws_bytes < 8 * srch::sort_len(n)))
    return fail(HESP_EINVAL, "%s: workspace of %lld bytes needed", who, (long long)(8 * srch::sort_len(n)));
  return HESP_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

int hesp_generate_enumerate(int64_t first, int32_t n_cand, int32_t nt, int32_t dmax, uint8_t* d_depth, void* stream) {
  if (first < 0 || n_cand < 0 || nt < 1 || dmax < 0 || dmax > kMaxLevel || (nt << dmax) > kMaxFine ||
      (n_cand > 0 && !d_depth))
    return fail(HESP_EINVAL, "hesp_generate_enumerate: bad argument");
  if (n_cand == 0) return HESP_OK;
  HIP_TRY(srch::enumerate(first, n_cand, (int32_t)tet3(nt), dmax, d_depth, (hipStream_t)stream));
  return HESP_OK;
}

int64_t hesp_topk_workspace_bytes(int64_t n) { return 8 * srch::sort_len(n < 1 ? 1 : n); }

int hesp_topk_makespan(const int64_t* d_makespan, int32_t n, int32_t k, int32_t* d_idx, void* d_ws, int64_t ws_bytes,
                       void* stream) {
  RC_TRY(topk_common(n, k, d_idx, d_ws, ws_bytes, "hesp_topk_makespan"));
  if (n == 0 || k == 0) return HESP_OK;
  if (!d_makespan) return fail(HESP_EINVAL, "hesp_topk_makespan: null makespans");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n2 = srch::sort_len(n);
  uint64_t* keys = (uint64_t*)d_ws;
  HIP_TRY(srch::keys_ms(d_makespan, n, nullptr, 0, n2, keys, s));
  HIP_TRY(srch::sort(keys, n2, s));
  HIP_TRY(srch::key_index(keys, k, 0xFFFFFFull, d_idx, s));
  return HESP_OK;
}

int hesp_topk_score(const float* d_score, int32_t n, int32_t k, int32_t* d_idx, void* d_ws, int64_t ws_bytes,
                    void* stream) {
  RC_TRY(topk_common(n, k, d_idx, d_ws, ws_bytes, "hesp_topk_score"));
  if (n == 0 || k == 0) return HESP_OK;
  if (!d_score) return fail(HESP_EINVAL, "hesp_topk_score: null scores");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n2 = srch::sort_len(n);
  uint64_t* keys = (uint64_t*)d_ws;
  HIP_TRY(srch::keys_f32(d_score, n, n2, keys, s));
  HIP_TRY(srch::sort(keys, n2, s));
  HIP_TRY(srch::key_index(keys, k, 0xFFFFFFFFull, d_idx, s));
  return HESP_OK;
}

int hesp_mlp_rate_features(const hesp_cost_model* cm, float* out, int32_t n_out) {
  if (!cm || !out || !cm->rmax_mflops || cm->n_ptypes < 1 || cm->n_ptypes > HESP_MAX_PTYPES ||
      n_out < 4 * cm->n_ptypes)
    return fail(HESP_EINVAL, "hesp_mlp_rate_features: need 4 outputs per processor type");
  for (int p = 0; p < cm->n_ptypes; p++)
    for (int k = 0; k < 4; k++) {
      const int64_t r = cm->rmax_mflops[4 * p + k];
      if (r <= 0) return fail(HESP_EINVAL, "hesp_mlp_rate_features: rates must be positive");
      out[4 * p + k] = (float)(std::log2((double)r / 131072.0) / 4.0);
    }
  return HESP_OK;
}

int hesp_mlp_features_agg(const uint8_t* d_depth, int64_t n, int32_t nt, const float* d_rate, int32_t n_rate,
                          uint16_t* d_x, void* stream) {
  if (n < 0 || nt < 1 || nt > kMaxFine || n_rate < 0 || n_rate > mlp::kInDim - mlp::kAggFeatures ||
      (n > 0 && (!d_depth || !d_x)) || (n_rate > 0 && !d_rate))
    return fail(HESP_EINVAL, "hesp_mlp_features_agg: bad argument (at most %d rate features)",
                mlp::kInDim - mlp::kAggFeatures);
  if (n == 0) return HESP_OK;
  hipStream_t s = (hipStream_t)stream;
  const std::vector<uint8_t> info = top_info(nt);
  Scratch sc;
  uint8_t* d_info = nullptr;
  HIP_TRY(sc.get(&d_info, (int64_t)info.size()));
  HIP_TRY(hipMemcpyAsync(d_info, info.data(), info.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(mlp::features_agg(d_depth, n, (int)info.size(), d_info, d_rate, n_rate, d_x, s));
  HIP_TRY(hipStreamSynchronize(s));
  return HESP_OK;
}

int hesp_search(hesp_plan* plan, const hesp_platform* pf, hesp_policy policy, const hesp_search_params* sp,
                uint8_t* best_depth, int64_t* best_makespan, hesp_trace_point* trace, void* stream) {
  if (!plan || !pf || !sp || !best_depth || !best_makespan) return fail(HESP_EINVAL, "hesp_search: null argument");
  const int nt = sp->nt, dmax = sp->dmax;
  if (nt < 1 || dmax < 0 || dmax > kMaxLevel || dmax > pf->max_level || (nt << dmax) > kMaxFine)
    return fail(HESP_EINVAL, "hesp_search: bad problem shape (dmax <= %d)", kMaxLevel);
  if (sp->mode < HESP_SEARCH_RANDOM || sp->mode > HESP_SEARCH_SURROGATE)
    return fail(HESP_EINVAL, "hesp_search: unknown mode");
  if (sp->rounds < 1 || sp->batch < 1 || sp->warm_rounds < 1 || sp->warm_batch < 1 || sp->pool < 1 ||
      sp->split_thr > (1u << 21) || sp->mutate_thr > (1u << 21))
    return fail(HESP_EINVAL, "hesp_search: rounds, batch, warm_rounds, warm_batch and pool must be positive");
  const bool sur = sp->mode == HESP_SEARCH_SURROGATE;
  const int64_t n_top = tet3(nt);
  const int n_rate = sur ? sp->n_rate : 0;
  const bool raw = n_top + n_rate <= mlp::kInDim;
  if (sur) {
    if (!sp->mlp || sp->proposals < sp->batch || sp->train_batch < 512 || sp->train_batch % 512 ||
        sp->replay < sp->train_batch || sp->replay < std::max(sp->batch, sp->warm_batch) || sp->train_steps < 0 ||
        !(sp->lr > 0.f) || n_rate < 0 || (n_rate > 0 && !sp->d_rate))
      return fail(HESP_EINVAL, "hesp_search: surrogate mode needs mlp, proposals >= batch, train_batch a multiple "
                               "of 512 and replay >= train_batch, batch and warm_batch");
    if (!raw && n_rate > mlp::kInDim - mlp::kAggFeatures)
      return fail(HESP_EINVAL, "hesp_search: at most %d rate features", mlp::kInDim - mlp::kAggFeatures);
    if (sp->proposals > (1 << 24) || (int64_t)sp->pool + sp->batch > (1 << 24))
      return fail(HESP_EINVAL, "hesp_search: at most 2^24 proposals");
  }
  if ((int64_t)sp->pool + std::max(sp->batch, sp->warm_batch) > (1 << 24))
    return fail(HESP_EINVAL, "hesp_search: pool + batch above 2^24");
  // every proposal has depths within 0..dmax, so only a capacity limit could
  // fail one, and a failed candidate has no makespan to learn or keep
  if (hesp_internal_plan_capped(plan))
    return fail(HESP_EINVAL, "hesp_search: the plan must not limit tasks or edges per candidate");

  hipStream_t s = (hipStream_t)stream;
  const int32_t maxb = std::max(sp->batch, sp->warm_batch);
  const int32_t gen_n = std::max(maxb, sur ? sp->proposals : 0);
  Scratch sc;
  uint8_t *cand = nullptr, *sel = nullptr, *pool_d[2] = {nullptr, nullptr}, *d_info = nullptr;
  int64_t *ms = nullptr, *pool_ms[2] = {nullptr, nullptr}, *rep_ms = nullptr;
  int32_t *st = nullptr, *idx = nullptr;
  uint64_t* keys = nullptr;
  uint16_t *xp = nullptr, *rep_x = nullptr, *round_x = nullptr;
  int64_t* d_count = nullptr;
  float *yp = nullptr, *rep_t = nullptr;
  const int64_t n2 = srch::sort_len(std::max<int64_t>((int64_t)sp->pool + maxb, sur ? sp->proposals : 0));
  HIP_TRY(sc.get(&cand, (int64_t)gen_n * n_top));
  HIP_TRY(sc.get(&ms, maxb));
  HIP_TRY(sc.get(&st, maxb));
  HIP_TRY(sc.get(&pool_d[0], (int64_t)sp->pool * n_top));
  HIP_TRY(sc.get(&pool_d[1], (int64_t)sp->pool * n_top));
  HIP_TRY(sc.get(&pool_ms[0], sp->pool));
  HIP_TRY(sc.get(&pool_ms[1], sp->pool));
  HIP_TRY(sc.get(&keys, n2));
  if (sur) {
    HIP_TRY(sc.get(&sel, (int64_t)sp->batch * n_top));
    HIP_TRY(sc.get(&idx, sp->batch));
    HIP_TRY(sc.get(&xp, (int64_t)sp->proposals * mlp::kInDim));
    HIP_TRY(sc.get(&yp, sp->proposals));
    HIP_TRY(sc.get(&rep_x, sp->replay * mlp::kInDim));
    HIP_TRY(sc.get(&rep_ms, sp->replay));
    HIP_TRY(sc.get(&rep_t, sp->replay));
    HIP_TRY(sc.get(&round_x, (int64_t)maxb * mlp::kInDim));
    HIP_TRY(sc.get(&d_count, 1));
    if (!raw) {
      const std::vector<uint8_t> info = top_info(nt);
      HIP_TRY(sc.get(&d_info, n_top));
      HIP_TRY(hipMemcpyAsync(d_info, info.data(), info.size(), hipMemcpyHostToDevice, s));
    }
  }
  auto featurize = [&](const uint8_t* dep, int64_t n, uint16_t* x) -> hipError_t {
    if (raw) return mlp::features(dep, n, (int)n_top, sp->d_rate, n_rate, x, s);
    return mlp::features_agg(dep, n, (int)n_top, d_info, sp->d_rate, n_rate, x, s);
  };

  int cur = 0, pool_n = 0;
  int64_t first = 0, simulated = 0, proposed = 0, filled = 0, rep_pos = 0;
  float mu = 0.f, sigma = 1.f;
  HIP_TRY(hipStreamSynchronize(s));
  const double t0 = now_ms();
  for (int r = 0; r < sp->rounds; r++) {
    const bool warm = r < sp->warm_rounds;
    int32_t B;
    const uint8_t* sim = cand;
    if (warm || sp->mode == HESP_SEARCH_RANDOM) {
      B = warm ? sp->warm_batch : sp->batch;
      RC_TRY(hesp_generate_uniform(sp->seed, first, B, nt, dmax, sp->split_thr, cand, s));
      first += B;
      proposed += B;
    } else if (sp->mode == HESP_SEARCH_GREEDY) {
      B = sp->batch;
      HIP_TRY(srch::mutate(sp->seed, r, pool_d[cur], pool_n, B, (int32_t)n_top, dmax, sp->mutate_thr, cand, s));
      proposed += B;
    } else {
      B = sp->batch;
      HIP_TRY(srch::mutate(sp->seed, r, pool_d[cur], pool_n, sp->proposals, (int32_t)n_top, dmax, sp->mutate_thr,
                           cand, s));
      HIP_TRY(featurize(cand, sp->proposals, xp));
      RC_TRY(hesp_mlp_forward(sp->mlp, xp, sp->proposals, yp, s));
      const int64_t np2 = srch::sort_len(sp->proposals);
      HIP_TRY(srch::keys_f32(yp, sp->proposals, np2, keys, s));
      HIP_TRY(srch::sort(keys, np2, s));
      HIP_TRY(srch::key_index(keys, B, 0xFFFFFFFFull, idx, s));
      HIP_TRY(srch::gather_rows(idx, B, cand, (int32_t)n_top, sel, s));
      sim = sel;
      proposed += sp->proposals;
    }
    // exact simulation of this round's candidates
    hesp_batch hb{B, nt, dmax, nullptr, nullptr, nullptr, sim};
    hesp_outputs out{ms, st, nullptr, nullptr, nullptr, nullptr, nullptr};
    RC_TRY(hesp_simulate_batch(plan, pf, policy, &hb, &out, s));
    simulated += B;
    // incumbents: the pool's best entries of (pool, batch)
    const int new_n = (int)std::min<int64_t>(sp->pool, (int64_t)pool_n + B);
    const int64_t m2 = srch::sort_len((int64_t)pool_n + B);
    HIP_TRY(srch::keys_ms(pool_ms[cur], pool_n, ms, B, m2, keys, s));
    HIP_TRY(srch::sort(keys, m2, s));
    HIP_TRY(srch::gather_pool(keys, new_n, pool_d[cur], pool_ms[cur], pool_n, sim, ms, (int32_t)n_top,
                              pool_d[cur ^ 1], pool_ms[cur ^ 1], s));
    cur ^= 1;
    pool_n = new_n;
    // online training of the surrogate on every exact result so far (ring
    // buffer); a candidate whose simulation failed (a status other than
    // HESP_OK, e.g. a task no finite space can hold) has no makespan and is left out
    if (sur) {
      HIP_TRY(featurize(sim, B, round_x));
      HIP_TRY(srch::append_ok(st, round_x, ms, B, mlp::kInDim, rep_x, rep_ms, sp->replay, rep_pos, d_count, s));
      int64_t k = 0;
      HIP_TRY(hipMemcpyAsync(&k, d_count, 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      rep_pos = (rep_pos + k) % sp->replay;
      filled = std::min<int64_t>(sp->replay, filled + k);
      if (r == sp->warm_rounds - 1) {
        // target normalisation from the warm-up rounds' makespans
        std::vector<int64_t> h((size_t)filled);
        HIP_TRY(hipMemcpyAsync(h.data(), rep_ms, 8 * filled, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        double a = 0, b = 0;
        int64_t cnt = 0;
        for (int64_t v : h)
          if (v > 0) {
            const double l = std::log((double)v);
            a += l;
            b += l * l;
            cnt++;
          }
        if (cnt > 0) {
          mu = (float)(a / cnt);
          const double var = b / cnt - (a / cnt) * (a / cnt);
          sigma = (float)std::max(std::sqrt(std::max(var, 0.0)), 1e-3);
        }
      }
      if (r >= sp->warm_rounds - 1 && filled >= sp->train_batch) {
        RC_TRY(hesp_mlp_targets(rep_ms, filled, mu, sigma, rep_t, s));
        RC_TRY(hesp_mlp_train(sp->mlp, rep_x, rep_t, filled, sp->train_batch, sp->train_steps, sp->lr, sp->seed,
                              nullptr, s));
      }
    }
    if (trace) {
      int64_t best = -1;
      HIP_TRY(hipMemcpyAsync(&best, pool_ms[cur], 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      trace[r].wall_ms = now_ms() - t0;
      trace[r].best_makespan = best;
      trace[r].simulated = simulated;
      trace[r].proposed = proposed;
    }
  }
  HIP_TRY(hipMemcpyAsync(best_makespan, pool_ms[cur], 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(best_depth, pool_d[cur], (size_t)n_top, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (*best_makespan < 0) return fail(HESP_EINVAL, "hesp_search: no candidate was simulated successfully");
  return HESP_OK;
}

}  // extern "C"
