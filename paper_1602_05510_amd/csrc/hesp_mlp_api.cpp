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
  uint16_t* wbt = nullptr;  // transposed bf16 copies of W1, W2, W3 (fused forward)
  int step = 0;
  int64_t rows = 0;         // activation capacity
  uint16_t *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *dza = nullptr, *dzb = nullptr;
  float *y = nullptr, *dy = nullptr, *parts = nullptr, *loss = nullptr;
  int64_t parts_cap = 0;
  uint16_t* xb = nullptr;   // sampled training batch
  float* tb = nullptr;
  int64_t sample_rows = 0;
  void release() {
    for (void* q : {(void*)p, (void*)g, (void*)m1, (void*)m2, (void*)wbf, (void*)wbt, (void*)xb, (void*)tb}) hfree(q);
    release_ws();
  }
  void release_ws() {
    for (void* q : {(void*)h1, (void*)h2, (void*)h3, (void*)dza, (void*)dzb, (void*)y, (void*)dy, (void*)parts,
                    (void*)loss})
      hfree(q);
    h1 = h2 = h3 = dza = dzb = nullptr;
    y = dy = parts = loss = nullptr;
    rows = parts_cap = 0;
  }
  hipError_t ensure(int64_t n, int64_t parts_need) {
    if (n > rows) {
      for (void* q : {(void*)h1, (void*)h2, (void*)h3, (void*)dza, (void*)dzb, (void*)y, (void*)dy}) hfree(q);
      h1 = h2 = h3 = dza = dzb = nullptr;
      y = dy = nullptr;
      rows = 0;
      hipError_t e;
      const size_t hb = (size_t)n * kHidden * sizeof(uint16_t);
      if ((e = hipMalloc(&h1, hb)) || (e = hipMalloc(&h2, hb)) || (e = hipMalloc(&h3, hb)) ||
          (e = hipMalloc(&dza, hb)) || (e = hipMalloc(&dzb, hb)) || (e = hipMalloc(&y, n * sizeof(float))) ||
          (e = hipMalloc(&dy, n * sizeof(float))))
        return e;
      rows = n;
    }
    if (parts_need > parts_cap) {
      hfree(parts);
      parts = nullptr;
      hipError_t e = hipMalloc(&parts, parts_need * sizeof(float));
      if (e) return e;
      parts_cap = parts_need;
    }
    if (!loss) {
      hipError_t e = hipMalloc(&loss, sizeof(float));
      if (e) return e;
    }
    return hipSuccess;
  }
};

namespace {

// forward pass of n rows (n <= m->rows): h1, h2, h3 and y
hipError_t forward_rows(hesp_mlp* m, const uint16_t* x, int64_t n, float* y, hipStream_t s) {
  hipError_t e;
  const uint16_t* w = m->wbf;
  if ((e = gemm(false, false, (int)n, kHidden, kInDim, 1, x, kInDim, w + kOffW1, kHidden, m->p + kOffB1, true,
                nullptr, 0, nullptr, m->h1, kHidden, s)))
    return e;
  if ((e = gemm(false, false, (int)n, kHidden, kHidden, 1, m->h1, kHidden, w + kOffW2, kHidden, m->p + kOffB2, true,
                nullptr, 0, nullptr, m->h2, kHidden, s)))
    return e;
  if ((e = gemm(false, false, (int)n, kHidden, kHidden, 1, m->h2, kHidden, w + kOffW3, kHidden, m->p + kOffB3, true,
                nullptr, 0, nullptr, m->h3, kHidden, s)))
    return e;
  return rowdot(m->h3, n, w + kOffW4, m->p + kOffB4, y, s);
}

// weight gradient dW[in][out] = act^T dz over n rows (split-K), written to g
hipError_t weight_grad(hesp_mlp* m, const uint16_t* act, int in, const uint16_t* dz, int64_t n, float* g,
                       hipStream_t s) {
  const int splits = (int)(n / 512);
  hipError_t e = gemm(true, false, in, kHidden, (int)n, splits, act, in, dz, kHidden, nullptr, false, nullptr, 0,
                      m->parts, nullptr, kHidden, s);
  if (e) return e;
  return sum_splits(m->parts, splits, (int64_t)in * kHidden, g, s);
}

hipError_t bias_grad(hesp_mlp* m, const uint16_t* a, int64_t n, const float* wcol, float* g, hipStream_t s) {
  const int slices = 64;
  hipError_t e = colsum(a, n, kHidden, wcol, slices, m->parts, s);
  if (e) return e;
  return sum_splits(m->parts, slices, kHidden, g, s);
}

}  // namespace

extern "C" {

int hesp_mlp_create(hesp_mlp** out, uint64_t seed) {
  if (!out) return fail(HESP_EINVAL, "hesp_mlp_create: null output");
  hesp_mlp* m = new (std::nothrow) hesp_mlp();
  if (!m) return fail(HESP_ENOMEM, "hesp_mlp_create: out of host memory");
  const size_t pb = kParams * sizeof(float);
  hipError_t e;
  if ((e = hipMalloc(&m->p, pb)) || (e = hipMalloc(&m->g, pb)) || (e = hipMalloc(&m->m1, pb)) ||
      (e = hipMalloc(&m->m2, pb)) || (e = hipMalloc(&m->wbf, kParams * sizeof(uint16_t))) ||
      (e = hipMalloc(&m->wbt, kTParams * sizeof(uint16_t)))) {
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
  HIP_TRY(transpose_w(m->p, m->wbt, nullptr));
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
    HIP_TRY(mlp_forward(d_x + r * kInDim, std::min(chunk, n - r), m->wbt, m->p, m->wbf + kOffW4, d_y + r,
                        (hipStream_t)stream));
  return HESP_OK;
}

int hesp_mlp_grad(hesp_mlp* m, const uint16_t* d_x, const float* d_t, int32_t batch, float* d_loss, void* stream) {
  if (!m || !d_x || !d_t || batch <= 0 || batch % 512)
    return fail(HESP_EINVAL, "hesp_mlp_grad: batch must be a positive multiple of 512");
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = batch;
  const int splits = (int)(n / 512);
  HIP_TRY(m->ensure(n, (int64_t)splits * kHidden * kHidden > 64 * kHidden ? (int64_t)splits * kHidden * kHidden
                                                                          : 64 * kHidden));
  // the loss accumulates straight into the caller's slot when one is given
  float* loss = d_loss ? d_loss : m->loss;
  HIP_TRY(zero_f32(loss, 1, s));
  HIP_TRY(forward_rows(m, d_x, n, m->y, s));
  float* g = m->g;
  const uint16_t* w = m->wbf;
  // output layer
  HIP_TRY(out_backward(m->y, d_t, n, w + kOffW4, m->h3, m->dy, m->dza, loss, s));
  HIP_TRY(bias_grad(m, m->h3, n, m->dy, g + kOffW4, s));
  HIP_TRY(sum_f32(m->dy, n, g + kOffB4, s));
  // layer 3: dz3 in dza
  HIP_TRY(weight_grad(m, m->h2, kHidden, m->dza, n, g + kOffW3, s));
  HIP_TRY(bias_grad(m, m->dza, n, nullptr, g + kOffB3, s));
  HIP_TRY(gemm(false, true, (int)n, kHidden, kHidden, 1, m->dza, kHidden, w + kOffW3, kHidden, nullptr, false, m->h2,
               kHidden, nullptr, m->dzb, kHidden, s));
  // layer 2: dz2 in dzb
  HIP_TRY(weight_grad(m, m->h1, kHidden, m->dzb, n, g + kOffW2, s));
  HIP_TRY(bias_grad(m, m->dzb, n, nullptr, g + kOffB2, s));
  HIP_TRY(gemm(false, true, (int)n, kHidden, kHidden, 1, m->dzb, kHidden, w + kOffW2, kHidden, nullptr, false, m->h1,
               kHidden, nullptr, m->dza, kHidden, s));
  // layer 1: dz1 in dza
  HIP_TRY(weight_grad(m, d_x, kInDim, m->dza, n, g + kOffW1, s));
  HIP_TRY(bias_grad(m, m->dza, n, nullptr, g + kOffB1, s));
  return HESP_OK;
}

int hesp_mlp_adam(hesp_mlp* m, float lr, void* stream) {
  if (!m || !(lr > 0.f)) return fail(HESP_EINVAL, "hesp_mlp_adam: bad argument");
  m->step++;
  HIP_TRY(adam(m->p, m->g, m->m1, m->m2, kParams, lr, 0.9f, 0.999f, 1e-8f, m->step, m->wbf, (hipStream_t)stream));
  HIP_TRY(transpose_w(m->p, m->wbt, (hipStream_t)stream));
  return HESP_OK;
}

int hesp_mlp_train(hesp_mlp* m, const uint16_t* d_x, const float* d_t, int64_t n, int32_t batch, int32_t steps,
                   float lr, uint64_t seed, float* d_loss, void* stream) {
  if (!m || !d_x || !d_t || batch <= 0 || batch % 512 || n < 1 || steps < 0 || !(lr > 0.f))
    return fail(HESP_EINVAL, "hesp_mlp_train: bad argument (batch a positive multiple of 512, n >= 1)");
  hipStream_t s = (hipStream_t)stream;
  if (m->sample_rows < batch) {
    hfree(m->xb);
    hfree(m->tb);
    m->xb = nullptr;
    m->tb = nullptr;
    m->sample_rows = 0;
    HIP_TRY(hipMalloc(&m->xb, (size_t)batch * kInDim * sizeof(uint16_t)));
    HIP_TRY(hipMalloc(&m->tb, (size_t)batch * sizeof(float)));
    m->sample_rows = batch;
  }
  for (int32_t i = 0; i < steps; i++) {
    // rows drawn with replacement; the counter is the network's Adam step number
    HIP_TRY(sample_rows(d_x, d_t, n, seed, (uint64_t)m->step, batch, m->xb, m->tb, s));
    int rc = hesp_mlp_grad(m, m->xb, m->tb, batch, d_loss ? d_loss + i : nullptr, stream);
    if (rc) return rc;
    rc = hesp_mlp_adam(m, lr, stream);
    if (rc) return rc;
  }
  return HESP_OK;
}

}  // extern "C"
