// hesp_mlp_api.cpp -- C ABI of the learned surrogate (declared in include/hesp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hesp.h"
#include "hesp_mlp.h"

using namespace hesp::mlp;

extern "C" int hesp_internal_fail(int code, const char* msg);   // sets the thread's last error

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

void hfree(void* p) {
  if (p) (void)hipFree(p);
}

// SplitMix64 (Steele, Lea, Flood 2014), value number idx+1 of the stream of `seed`
uint64_t mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

struct hesp_mlp {
  float* p = nullptr;       // fp32 master parameters (flat)
  float* g = nullptr;       // gradients
  float* m1 = nullptr;      // Adam first moment
  float* m2 = nullptr;      // Adam second moment
  uint16_t* wbf = nullptr;  // bf16 copy of the parameters
  uint16_t* wfr = nullptr;  // fragment-ordered bf16 copies of W1^T, W2^T, W3^T, W2, W3 (products)
  int step = 0;
  // training step workspace for `rows` rows
  int64_t rows = 0;
  TrainBufs tb{};
  void release() {
    for (void* q : {(void*)p, (void*)g, (void*)m1, (void*)m2, (void*)wbf, (void*)wfr}) hfree(q);
    release_ws();
  }
  void release_ws() {
    for (void* q : {(void*)tb.xp, (void*)tb.h1p, (void*)tb.h2p, (void*)tb.h3p, (void*)tb.d1p, (void*)tb.d2p,
                    (void*)tb.d3p, (void*)tb.dy, (void*)tb.part, (void*)tb.lossp})
      hfree(q);
    tb = TrainBufs{};
    rows = 0;
  }
  hipError_t ensure(int64_t n) {
    if (n <= rows) return hipSuccess;
    release_ws();
    hipError_t e;
    const size_t hb = (size_t)n * kHidden * sizeof(uint16_t);
    if ((e = hipMalloc(&tb.xp, (size_t)n * kInDim * sizeof(uint16_t))) || (e = hipMalloc(&tb.h1p, hb)) ||
        (e = hipMalloc(&tb.h2p, hb)) || (e = hipMalloc(&tb.h3p, hb)) || (e = hipMalloc(&tb.d1p, hb)) ||
        (e = hipMalloc(&tb.d2p, hb)) || (e = hipMalloc(&tb.d3p, hb)) ||
        (e = hipMalloc(&tb.dy, (size_t)n * sizeof(float))) ||
        (e = hipMalloc(&tb.part, (size_t)kTrainTiles * (n / 512) * kTrainPartStride * sizeof(float))) ||
        (e = hipMalloc(&tb.lossp, (size_t)(n / 16) * sizeof(float))))
      return e;
    rows = n;
    return hipSuccess;
  }
  AdamArgs adam_args(bool on, float lr) const {
    AdamArgs a{};
    a.on = on ? 1 : 0;
    a.lr = lr;
    a.b1 = 0.9f;
    a.b2 = 0.999f;
    a.eps = 1e-8f;
    a.c1 = 1.f - powf(a.b1, (float)step);
    a.c2 = 1.f - powf(a.b2, (float)step);
    a.p = p;
    a.m1 = m1;
    a.m2 = m2;
    a.wbf = wbf;
    a.wfr = wfr;
    return a;
  }
};

extern "C" {

int hesp_mlp_create(hesp_mlp** out, uint64_t seed) {
  if (!out) return fail(HESP_EINVAL, "hesp_mlp_create: null output");
  hesp_mlp* m = new (std::nothrow) hesp_mlp();
  if (!m) return fail(HESP_ENOMEM, "hesp_mlp_create: out of host memory");
  const size_t pb = kParams * sizeof(float);
  hipError_t e;
  if ((e = hipMalloc(&m->p, pb)) || (e = hipMalloc(&m->g, pb)) || (e = hipMalloc(&m->m1, pb)) ||
      (e = hipMalloc(&m->m2, pb)) || (e = hipMalloc(&m->wbf, kParams * sizeof(uint16_t))) ||
      (e = hipMalloc(&m->wfr, kFrParams * sizeof(uint16_t)))) {
    m->release();
    delete m;
    return fail(HESP_ENOMEM, "hesp_mlp_create: %s", hipGetErrorString(e));
  }
  // He-uniform weights from counter-based SplitMix64 draws, zero biases
  std::vector<float> h(kParams, 0.f);
  auto fill = [&](int64_t off, int64_t count, int fan_in, uint64_t purpose) {
    const double lim = std::sqrt(6.0 / fan_in);
    const uint64_t st = mix(seed + 0x9E3779B97F4A7C15ull * (purpose + 1));
    for (int64_t i = 0; i < count; i++) {
      const uint64_t u = mix(st + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1));
      const double r = (double)(u >> 11) * (1.0 / 9007199254740992.0);   // [0, 1)
      h[off + i] = (float)((2.0 * r - 1.0) * lim);
    }
  };
  fill(kOffW1, (int64_t)kInDim * kHidden, kInDim, 11);
  fill(kOffW2, (int64_t)kHidden * kHidden, kHidden, 12);
  fill(kOffW3, (int64_t)kHidden * kHidden, kHidden, 13);
  fill(kOffW4, kHidden, kHidden, 14);
  int rc = hesp_mlp_set_params(m, h.data(), kParams);
  if (rc) {
    m->release();
    delete m;
    return rc;
  }
  *out = m;
  return HESP_OK;
}

int hesp_mlp_destroy(hesp_mlp* m) {
  if (!m) return HESP_OK;
  m->release();
  delete m;
  return HESP_OK;
}

int64_t hesp_mlp_param_count(void) { return kParams; }

int hesp_mlp_set_params(hesp_mlp* m, const float* host, int64_t n) {
  if (!m || !host || n != kParams) return fail(HESP_EINVAL, "hesp_mlp_set_params: need %lld floats", (long long)kParams);
  HIP_TRY(hipMemcpy(m->p, host, kParams * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(m->m1, 0, kParams * sizeof(float)));
  HIP_TRY(hipMemset(m->m2, 0, kParams * sizeof(float)));
  HIP_TRY(hipMemset(m->g, 0, kParams * sizeof(float)));
  HIP_TRY(to_bf16(m->p, kParams, m->wbf, nullptr));
  HIP_TRY(frag_w(m->p, m->wfr, nullptr));
  HIP_TRY(hipDeviceSynchronize());
  m->step = 0;
  return HESP_OK;
}

int hesp_mlp_get_params(hesp_mlp* m, float* host, int64_t n) {
  if (!m || !host || n != kParams) return fail(HESP_EINVAL, "hesp_mlp_get_params: need %lld floats", (long long)kParams);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(host, m->p, kParams * sizeof(float), hipMemcpyDeviceToHost));
  return HESP_OK;
}

int hesp_mlp_get_grads(hesp_mlp* m, float* host, int64_t n) {
  if (!m || !host || n != kParams) return fail(HESP_EINVAL, "hesp_mlp_get_grads: need %lld floats", (long long)kParams);
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(host, m->g, kParams * sizeof(float), hipMemcpyDeviceToHost));
  return HESP_OK;
}

int hesp_mlp_features(const uint8_t* d_depth, int64_t n, int32_t n_top, const float* d_rate, int32_t n_rate,
                      uint16_t* d_x, void* stream) {
  if (n < 0 || n_top < 0 || n_rate < 0 || n_top + n_rate > kInDim || (n > 0 && (!d_depth || !d_x)) ||
      (n_rate > 0 && !d_rate))
    return fail(HESP_EINVAL, "hesp_mlp_features: need n_top + n_rate <= %d and device pointers", kInDim);
  if (n == 0) return HESP_OK;
  HIP_TRY(features(d_depth, n, n_top, d_rate, n_rate, d_x, (hipStream_t)stream));
  return HESP_OK;
}

int hesp_mlp_targets(const int64_t* d_makespan, int64_t n, float mu, float sigma, float* d_t, void* stream) {
  if (n < 0 || !(sigma > 0.f) || (n > 0 && (!d_makespan || !d_t))) return fail(HESP_EINVAL, "hesp_mlp_targets: bad argument");
  if (n == 0) return HESP_OK;
  HIP_TRY(targets(d_makespan, n, mu, sigma, d_t, (hipStream_t)stream));
  return HESP_OK;
}

int hesp_mlp_forward(hesp_mlp* m, const uint16_t* d_x, int64_t n, float* d_y, void* stream) {
  if (!m || n < 0 || (n > 0 && (!d_x || !d_y))) return fail(HESP_EINVAL, "hesp_mlp_forward: bad argument");
  if (n == 0) return HESP_OK;
  // one fused launch (activations never leave LDS); at most 2^31 rows per launch
  const int64_t chunk = (int64_t)1 << 31;
  for (int64_t r = 0; r < n; r += chunk)
    HIP_TRY(mlp_forward(d_x + r * kInDim, std::min(chunk, n - r), m->wfr, m->p, m->wbf + kOffW4, d_y + r,
                        (hipStream_t)stream));
  return HESP_OK;
}

int hesp_mlp_grad(hesp_mlp* m, const uint16_t* d_x, const float* d_t, int32_t batch, float* d_loss, void* stream) {
  if (!m || !d_x || !d_t || batch <= 0 || batch % 512)
    return fail(HESP_EINVAL, "hesp_mlp_grad: batch must be a positive multiple of 512");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(m->ensure(batch));
  HIP_TRY(train_rows(d_x, d_t, batch, false, 0, 0, batch, m->wfr, m->wbf, m->p, m->tb, s));
  HIP_TRY(train_wgrad(m->tb, batch, m->g, m->adam_args(false, 0.f), d_loss, s));
  return HESP_OK;
}

int hesp_mlp_adam(hesp_mlp* m, float lr, void* stream) {
  if (!m || !(lr > 0.f)) return fail(HESP_EINVAL, "hesp_mlp_adam: bad argument");
  m->step++;
  HIP_TRY(adam(m->p, m->g, m->m1, m->m2, kParams, lr, 0.9f, 0.999f, 1e-8f, m->step, m->wbf, (hipStream_t)stream));
  HIP_TRY(frag_w(m->p, m->wfr, (hipStream_t)stream));
  return HESP_OK;
}

int hesp_mlp_train(hesp_mlp* m, const uint16_t* d_x, const float* d_t, int64_t n, int32_t batch, int32_t steps,
                   float lr, uint64_t seed, float* d_loss, void* stream) {
  if (!m || !d_x || !d_t || batch <= 0 || batch % 512 || n < 1 || steps < 0 || !(lr > 0.f))
    return fail(HESP_EINVAL, "hesp_mlp_train: bad argument (batch a positive multiple of 512, n >= 1)");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(m->ensure(batch));
  for (int32_t i = 0; i < steps; i++) {
    // rows drawn with replacement (the counter is the network's Adam step
    // number); then weight gradients, and their sums with Adam fused in
    HIP_TRY(train_rows(d_x, d_t, n, true, seed, (uint64_t)m->step, batch, m->wfr, m->wbf, m->p, m->tb, s));
    m->step++;
    HIP_TRY(train_wgrad(m->tb, batch, m->g, m->adam_args(true, lr), d_loss ? d_loss + i : nullptr, s));
  }
  return HESP_OK;
}

}  // extern "C"
