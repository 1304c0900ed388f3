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
// bf16 weight copies in MFMA fragment order, the operand layout of the forward
// and training products: a matrix M[row][k] (K = 32 or 256 columns) is stored
// fragment by fragment, fragment (row block rb of 16 rows, k-step ks of 32) being
// the 64 lanes x 8 values a wave loads for one 16x16x32 product, lane
// (k % 32) / 8 * 16 + row % 16 holding k .. k + 7 -- one contiguous 1 KB load.
// Matrices: W1^T [hidden][in], W2^T and W3^T [hidden][hidden] (forward products:
// rows = output features), W2 and W3 [hidden][hidden] (backward products: rows =
// input features).
constexpr int64_t kFrW1T = 0;
constexpr int64_t kFrW2T = kFrW1T + (int64_t)kInDim * kHidden;
constexpr int64_t kFrW3T = kFrW2T + (int64_t)kHidden * kHidden;
constexpr int64_t kFrW2 = kFrW3T + (int64_t)kHidden * kHidden;
constexpr int64_t kFrW3 = kFrW2 + (int64_t)kHidden * kHidden;
constexpr int64_t kFrParams = kFrW3 + (int64_t)kHidden * kHidden;
__host__ __device__ inline int64_t fr_index(int row, int k, int K) {
  return (((int64_t)(row >> 4) * (K >> 5) + (k >> 5)) * 64 + ((k & 31) >> 3) * 16 + (row & 15)) * 8 + (k & 7);
}

// whole network, any n: y[n] (fp32) from x[n][in] (bf16)
hipError_t mlp_forward(const uint16_t* x, int64_t n, const uint16_t* wt, const float* p, const uint16_t* w4, float* y,
                       hipStream_t s);
hipError_t frag_w(const float* p, uint16_t* wfr, hipStream_t s);

hipError_t features(const uint8_t* depth, int64_t n, int n_top, const float* rate, int n_rate, uint16_t* x,
                    hipStream_t s);
constexpr int kAggFeatures = 24;   // aggregate features before the rate features
hipError_t features_agg(const uint8_t* depth, int64_t n, int n_top, const uint8_t* info, const float* rate,
                        int n_rate, uint16_t* x, hipStream_t s);
hipError_t targets(const int64_t* ms, int64_t n, float mu, float sigma, float* t, hipStream_t s);
hipError_t adam(float* w, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2, float eps,
                int step, uint16_t* wbf, hipStream_t s);
hipError_t to_bf16(const float* w, int64_t n, uint16_t* out, hipStream_t s);
hipError_t zero_f32(float* p, int64_t n, hipStream_t s);

// training step buffers (device): packed inputs, activations and data gradients
// of the batch rows, dy, and the weight-gradient pass's partial sums
// (kTrainTiles x batch / 512 x kTrainPartStride floats)
struct TrainBufs {
  uint16_t *xp, *h1p, *h2p, *h3p, *d1p, *d2p, *d3p;
  float* dy;
  float* part;
  float* lossp;                // loss terms per row-pass block (at most rows / 16)
};
struct AdamArgs {
  int on;                      // 0: gradients only
  float lr, b1, b2, eps, c1, c2;
  float *p, *m1, *m2;
  uint16_t *wbf, *wfr;
};
constexpr int kTrainTiles = 36;
constexpr int64_t kTrainPartStride = 64 * 64 + 3 * 64;
// forward, output backward and hidden data gradients of `batch` rows (a multiple
// of 512): rows r of x/t, or with `sample` rows drawn as in hesp_mlp_train
hipError_t train_rows(const uint16_t* x, const float* t, int64_t n, bool sample, uint64_t seed, uint64_t step,
                      int batch, const uint16_t* wt, const uint16_t* wb, const float* p, const TrainBufs& tb,
                      hipStream_t s);
// weight and bias gradients into g; with ad.on, Adam on every parameter; the
// mean squared error of the rows into *loss (nullable)
hipError_t train_wgrad(const TrainBufs& tb, int batch, float* g, const AdamArgs& ad, float* loss, hipStream_t s);

}  // namespace mlp
}  // namespace hesp
