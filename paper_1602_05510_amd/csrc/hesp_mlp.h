// hesp_mlp.h -- launch-level interface of the surrogate kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hesp {
namespace mlp {

constexpr int kInDim = 32;    // input features (zero padded)
constexpr int kHidden = 256;  // width of the three hidden layers

// flat parameter layout: W1 [in][hidden], b1, W2 [hidden][hidden], b2, W3, b3, w4 [hidden], b4 [1]
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + (int64_t)kInDim * kHidden;
constexpr int64_t kOffW2 = kOffB1 + kHidden;
constexpr int64_t kOffB2 = kOffW2 + (int64_t)kHidden * kHidden;
constexpr int64_t kOffW3 = kOffB2 + kHidden;
constexpr int64_t kOffB3 = kOffW3 + (int64_t)kHidden * kHidden;
constexpr int64_t kOffW4 = kOffB3 + kHidden;
constexpr int64_t kOffB4 = kOffW4 + kHidden;
constexpr int64_t kParams = kOffB4 + 1;
// transposed bf16 copies of the weight matrices used by the fused forward pass
constexpr int64_t kOffT1 = 0;                                   // [hidden][in]
constexpr int64_t kOffT2 = kOffT1 + (int64_t)kInDim * kHidden;  // [hidden][hidden]
constexpr int64_t kOffT3 = kOffT2 + (int64_t)kHidden * kHidden;
constexpr int64_t kTParams = kOffT3 + (int64_t)kHidden * kHidden;

// whole network, any n: y[n] (fp32) from x[n][in] (bf16)
hipError_t mlp_forward(const uint16_t* x, int64_t n, const uint16_t* wt, const float* p, const uint16_t* w4, float* y,
                       hipStream_t s);
hipError_t transpose_w(const float* p, uint16_t* wt, hipStream_t s);

hipError_t gemm(bool ta, bool tb, int M, int N, int K, int splits, const uint16_t* A, int lda, const uint16_t* B,
                int ldb, const float* bias, bool relu, const uint16_t* mask, int ldm, float* out_f32,
                uint16_t* out_bf16, int ldc, hipStream_t s);
hipError_t sum_splits(const float* parts, int splits, int64_t count, float* out, hipStream_t s);
hipError_t features(const uint8_t* depth, int64_t n, int n_top, const float* rate, int n_rate, uint16_t* x,
                    hipStream_t s);
constexpr int kAggFeatures = 24;   // aggregate features before the rate features
hipError_t features_agg(const uint8_t* depth, int64_t n, int n_top, const uint8_t* info, const float* rate,
                        int n_rate, uint16_t* x, hipStream_t s);
hipError_t targets(const int64_t* ms, int64_t n, float mu, float sigma, float* t, hipStream_t s);
hipError_t rowdot(const uint16_t* h, int64_t M, const uint16_t* w, const float* b, float* y, hipStream_t s);
hipError_t out_backward(const float* y, const float* t, int64_t n, const uint16_t* w4, const uint16_t* h3, float* dy,
                        uint16_t* dz3, float* loss, hipStream_t s);
hipError_t colsum(const uint16_t* a, int64_t M, int ncol, const float* wcol, int slices, float* parts, hipStream_t s);
hipError_t sum_f32(const float* v, int64_t n, float* out, hipStream_t s);
hipError_t adam(float* w, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2, float eps,
                int step, uint16_t* wbf, hipStream_t s);
hipError_t to_bf16(const float* w, int64_t n, uint16_t* out, hipStream_t s);
hipError_t zero_f32(float* p, int64_t n, hipStream_t s);
hipError_t sample_rows(const uint16_t* x, const float* t, int64_t n, uint64_t seed, uint64_t step, int batch,
                       uint16_t* xb, float* tb, hipStream_t s);

}  // namespace mlp
}  // namespace hesp
