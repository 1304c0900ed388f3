// hesp_mlp.hip -- kernels of the learned surrogate that scores candidate
// partitionings (gfx950, bf16 MFMA with fp32 accumulation).
//
// Network: x (32 features: split depth of each top-level task, then platform
// rate features, zero padded) -> 256 -> 256 -> 256 -> 1, ReLU, mean squared
// error on a normalised log-makespan.  Weights and activations are bfloat16
// (round to nearest even) wherever they enter a product; products accumulate in
// fp32; biases, the output and the master weights (Adam) are fp32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_mlp.h"

namespace hesp {
namespace mlp {

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) uint32_t u32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) short i16x2;

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);  // NaN
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

// bf16(relu(a)) | bf16(relu(b)) << 16: the hardware conversion rounds to nearest
// even; ReLU then acts on the bf16 bit patterns as signed 16-bit integers (a
// negative value or -0 has its sign bit set and becomes +0), which equals
// rounding relu(a) and relu(b) for every finite input.
__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b) {
  const bf16x2 h = __builtin_convertvector((f32x2{a, b}), bf16x2);
  const i16x2 r = __builtin_elementwise_max(__builtin_bit_cast(i16x2, h), (i16x2{0, 0}));
  return __builtin_bit_cast(uint32_t, r);
}

// ---------------------------------------------------------------- GEMM
// C[M][N] = opA[M][K] * opB[K][N], bf16 inputs, fp32 accumulation.
//   opA[m][k] = TA ? A[k*lda + m] : A[m*lda + k]
//   opB[k][n] = TB ? B[n*ldb + k] : B[k*ldb + n]
// Epilogue: + bias[n]; ReLU; zero where mask[m*ldm + n] == 0; store fp32
// and/or bf16 at m*ldc + n.  Split-K: blockIdx.z takes K range
// [z*kc, (z+1)*kc) and writes fp32 to out_f32 + z*M*ldc.
// Tile 64x64 per 256-thread workgroup (2x2 waves of 32x32, each 2x2 MFMA
// 16x16x32 blocks); requires N % 64 == 0 and kc % 32 == 0; any M.
constexpr int TM = 64, TN = 64, TK = 32, LDS_K = TK + 8;

template <bool TA, bool TB>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int kc, const uint16_t* __restrict__ A, int lda,
                                              const uint16_t* __restrict__ B, int ldb, const float* __restrict__ bias,
                                              int relu, const uint16_t* __restrict__ mask, int ldm,
                                              float* __restrict__ out_f32, uint16_t* __restrict__ out_bf16,
                                              int ldc) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[TM][LDS_K];   // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t sB[TN][LDS_K];   // [n][k]
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
  const int kbeg = blockIdx.z * kc, kend = kbeg + kc;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = kbeg; k0 < kend; k0 += TK) {
    // stage A
    if (!TA) {
      const int r = t >> 2, kk = (t & 3) * 8;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (m0 + r < M) v = *(const u32x4*)(A + (int64_t)(m0 + r) * lda + k0 + kk);
      *(u32x4*)&sA[r][kk] = v;
    } else {
      const int k = t >> 3, mm = (t & 7) * 8;
      uint16_t v[8];
      if (m0 + mm + 7 < M) {
        const u32x4 q = *(const u32x4*)(A + (int64_t)(k0 + k) * lda + m0 + mm);
        *(u32x4*)v = q;
      } else {
        for (int j = 0; j < 8; j++) v[j] = (m0 + mm + j < M) ? A[(int64_t)(k0 + k) * lda + m0 + mm + j] : 0;
      }
      for (int j = 0; j < 8; j++) sA[mm + j][k] = v[j];
    }
    // stage B as [n][k]
    if (TB) {
      const int n = t >> 2, kk = (t & 3) * 8;
      *(u32x4*)&sB[n][kk] = *(const u32x4*)(B + (int64_t)(n0 + n) * ldb + k0 + kk);
    } else {
      const int k = t >> 3, nn = (t & 7) * 8;
      uint16_t v[8];
      *(u32x4*)v = *(const u32x4*)(B + (int64_t)(k0 + k) * ldb + n0 + nn);
      for (int j = 0; j < 8; j++) sB[nn + j][k] = v[j];
    }
    __syncthreads();
    // lane l: row/col l % 16 of a 16x16 block, k = (l / 16) * 8 .. + 8
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; i++) a[i] = *(const bf16x8*)&sA[wm * 32 + i * 16 + (l & 15)][(l >> 4) * 8];
    for (int j = 0; j < 2; j++) b[j] = *(const bf16x8*)&sB[wn * 32 + j * 16 + (l & 15)][(l >> 4) * 8];
    for (int i = 0; i < 2; i++)
      for (int j = 0; j < 2; j++) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // lane l holds rows (l / 16) * 4 + q, column l % 16 of each block
  float* outz = out_f32 ? out_f32 + (int64_t)blockIdx.z * M * ldc : nullptr;
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++)
      for (int q = 0; q < 4; q++) {
        const int m = m0 + wm * 32 + i * 16 + (l >> 4) * 4 + q;
        const int n = n0 + wn * 32 + j * 16 + (l & 15);
        if (m >= M) continue;
        float v = acc[i][j][q];
        if (bias) v += bias[n];
        if (relu) v = v > 0.f ? v : 0.f;
        if (mask && mask[(int64_t)m * ldm + n] == 0) v = 0.f;
        if (outz) outz[(int64_t)m * ldc + n] = v;
        if (out_bf16) out_bf16[(int64_t)m * ldc + n] = f2bf(v);
      }
}

// ---------------------------------------------------------------- fused forward
// The whole network for 128 rows per 512-thread workgroup.  Activations stay in
// LDS (128 x 256 bf16); weights come from L2 in a transposed bf16 copy
// (wt[n][k], k contiguous) so that each lane's weight operand is one 16-byte
// load.  Eight 16x16 blocks x two column blocks of accumulators per wave (64
// registers; 128 in all with the operand fragments and the ring of weight
// fragments), so four waves fit on each SIMD; two workgroups share a CU's LDS.
// The last layer's dot with w4 is reduced across lanes and waves through LDS.
constexpr int FM = 128, FRB = FM / 16, FWAVES = 8;
// k-steps of 32 per hidden layer; weight fragments requested this many k-steps
// ahead of their products
constexpr int FKS = kHidden / 32, FPRE = 2;

// Activation tile layout: row-major, 256 bf16 per row with no padding, the
// sixteen-byte chunks of a row permuted by an XOR with a row-dependent mask.
// The mask's bits 4..2 take eight distinct values over eight consecutive rows,
// so the sixteen-byte operand reads of a wave (16 rows x 4 chunks) spread evenly
// over the banks; its bits 2..0 are distinct over eight rows too, so the eight-
// byte epilogue stores of 16 rows meet at most two to a bank.
__device__ __forceinline__ int sh_off(int row, int col) {
  const int f = ((row & 7) << 2) | ((row >> 1) & 3);
  return row * kHidden + (((col >> 3) ^ f) << 3) + (col & 7);
}

// Products are formed transposed (A operand = weight rows, B operand =
// activation rows), so lane l of a 16x16 block holds output row (l % 16) and four
// consecutive output columns 4 (l / 16) .. + 3: one 8-byte LDS store each.
// Wave w owns all 128 rows and columns [32 w, 32 w + 32): each weight fragment
// read from L2 feeds 8 products, each activation fragment read from LDS feeds 2.
// The accumulators start from the layer's bias, so the epilogue only applies the
// ReLU, rounds to bf16 and stores.
__device__ __forceinline__ void fwd_epilogue(const f32x4 (&acc)[FRB][2], int w, int l, uint16_t* sH) {
  for (int cb = 0; cb < 2; cb++) {
    const int col = w * 32 + cb * 16 + (l >> 4) * 4;
    for (int rb = 0; rb < FRB; rb++)
      *(uint2*)&sH[sh_off(rb * 16 + (l & 15), col)] =
          make_uint2(relu_bf16x2(acc[rb][cb][0], acc[rb][cb][1]), relu_bf16x2(acc[rb][cb][2], acc[rb][cb][3]));
  }
}

// every accumulator block of the wave starts from the bias of its four columns
__device__ __forceinline__ void fwd_init(f32x4 (&acc)[FRB][2], const float* __restrict__ bias, int w, int l) {
  for (int cb = 0; cb < 2; cb++) {
    const f32x4 bv = *(const f32x4*)(bias + w * 32 + cb * 16 + (l >> 4) * 4);
    for (int rb = 0; rb < FRB; rb++) acc[rb][cb] = bv;
  }
}

__global__ void __launch_bounds__(FWAVES * 64, 4) k_mlp_fwd(const uint16_t* __restrict__ x, int64_t n,
                                                            const uint16_t* __restrict__ wt,
                                                            const float* __restrict__ p,
                                                            const uint16_t* __restrict__ w4, float* __restrict__ y) {
  __shared__ __attribute__((aligned(16))) uint16_t sH[FM * kHidden];
  __shared__ float sY[FWAVES][FM];
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * FM;
  f32x4 acc[FRB][2];
  // layer 1 (K = 32): activation operand straight from the input rows
  fwd_init(acc, p + kOffB1, w, l);
  {
    bf16x8 wf[2];
    for (int cb = 0; cb < 2; cb++)
      wf[cb] = *(const bf16x8*)(wt + kOffT1 + (int64_t)(w * 32 + cb * 16 + (l & 15)) * kInDim + (l >> 4) * 8);
    // every row block's input is requested before the first product: rows past
    // the end read the last row (n >= 1) and are then replaced by zeros, so the
    // loads carry no branch and their memory latencies overlap
    u32x4 av[FRB];
#pragma unroll
    for (int rb = 0; rb < FRB; rb++) {
      const int64_t row = r0 + rb * 16 + (l & 15);
      av[rb] = *(const u32x4*)(x + (row < n ? row : n - 1) * kInDim + (l >> 4) * 8);
    }
#pragma unroll
    for (int rb = 0; rb < FRB; rb++) {
      const bool live = r0 + rb * 16 + (l & 15) < n;
      const u32x4 v = live ? av[rb] : (u32x4{0u, 0u, 0u, 0u});
      const bf16x8 a = __builtin_bit_cast(bf16x8, v);
#pragma unroll
      for (int cb = 0; cb < 2; cb++) acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[cb], a, acc[rb][cb], 0, 0, 0);
    }
  }
  // layers 2 and 3 (K = 256): activations from LDS, weights from L2.  The 16
  // k-steps of both layers form one sequence g = 8 * layer + ks; the weight
  // fragments of step g + FPRE are requested before step g's products, into a
  // ring of FPRE + 1 register slots (the slot of step g - 1, already consumed).
  bf16x8 wq[FPRE + 1][2];
  auto wload = [&](int g) {
    const uint16_t* wl = wt + (g < FKS ? kOffT2 : kOffT3) + (int64_t)(w * 32 + (l & 15)) * kHidden + (l >> 4) * 8 +
                         (g % FKS) * 32;
#pragma unroll
    for (int cb = 0; cb < 2; cb++) wq[(g) % (FPRE + 1)][cb] = *(const bf16x8*)(wl + (int64_t)cb * 16 * kHidden);
  };
#pragma unroll
  for (int g = 0; g < FPRE; g++) wload(g);
  fwd_epilogue(acc, w, l, sH);
  __syncthreads();
#pragma unroll
  for (int g = 0; g < 2 * FKS; g++) {
    const int ks = g % FKS;
    if (ks == 0) fwd_init(acc, p + (g < FKS ? kOffB2 : kOffB3), w, l);
    if (g + FPRE < 2 * FKS) wload(g + FPRE);
    const int k0 = ks * 32;
#pragma unroll
    for (int rb = 0; rb < FRB; rb++) {
      const bf16x8 a = *(const bf16x8*)&sH[sh_off(rb * 16 + (l & 15), k0 + (l >> 4) * 8)];
#pragma unroll
      for (int cb = 0; cb < 2; cb++)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wq[g % (FPRE + 1)][cb], a, acc[rb][cb], 0, 0, 0);
    }
    if (ks == FKS - 1) {
      __syncthreads();   // every wave has read this layer's input
      if (g < FKS) {
        fwd_epilogue(acc, w, l, sH);
        __syncthreads();
      }
    }
  }
  // output: y = bf16(relu(z3 + b3)) . w4 + b4, two products per dot instruction
  float part[FRB] = {};
  for (int cb = 0; cb < 2; cb++) {
    const int col = w * 32 + cb * 16 + (l >> 4) * 4;
    const uint2 wv = *(const uint2*)(w4 + col);
    for (int rb = 0; rb < FRB; rb++) {
      part[rb] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, relu_bf16x2(acc[rb][cb][0], acc[rb][cb][1])),
                                                 __builtin_bit_cast(bf16x2, wv.x), part[rb], false);
      part[rb] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, relu_bf16x2(acc[rb][cb][2], acc[rb][cb][3])),
                                                 __builtin_bit_cast(bf16x2, wv.y), part[rb], false);
    }
  }
  for (int rb = 0; rb < FRB; rb++) {
    float v = part[rb];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (l < 16) sY[w][rb * 16 + l] = v;
  }
  __syncthreads();
  if (t < FM) {
    const int64_t row = r0 + t;
    float s = 0.f;
    for (int q = 0; q < FWAVES; q++) s += sY[q][t];
    if (row < n) y[row] = s + p[kOffB4];
  }
}

// transposed bf16 copies of W1, W2, W3 (wt[n][k] = W[k][n])
__global__ void k_transpose_w(const float* __restrict__ p, uint16_t* __restrict__ wt) {
  const int64_t total = kTParams;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t src;
    if (e < kOffT2) {
      const int64_t nn = e / kInDim, kk = e % kInDim;
      src = kOffW1 + kk * kHidden + nn;
    } else {
      const int64_t f = e < kOffT3 ? e - kOffT2 : e - kOffT3;
      const int64_t nn = f / kHidden, kk = f % kHidden;
      src = (e < kOffT3 ? kOffW2 : kOffW3) + kk * kHidden + nn;
    }
    wt[e] = f2bf(p[src]);
  }
}

// sum of `splits` fp32 slices of size count -> out (fp32)
__global__ void k_sum_splits(const float* __restrict__ parts, int splits, int64_t count, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < splits; z++) s += parts[(int64_t)z * count + i];
    out[i] = s;
  }
}

// ---------------------------------------------------------------- small kernels

// features: split depths of the candidate's top-level tasks (as numbers), then
// the platform rate features, zero padded to IN_DIM; bf16
__global__ void k_features(const uint8_t* __restrict__ depth, int64_t n, int n_top, const float* __restrict__ rate,
                           int n_rate, uint16_t* __restrict__ x) {
  const int64_t total = n * kInDim;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / kInDim;
    const int j = (int)(e % kInDim);
    float v = 0.f;
    if (j < n_top) v = (float)depth[c * n_top + j];
    else if (j < n_top + n_rate) v = rate[j - n_top];
    x[e] = f2bf(v);
  }
}

// aggregate features of large candidates, one wave per candidate: for each kind
// the fraction of its top-level tasks at each depth 0..3 (16 values), for each
// kind and each half of the k range the mean depth (8 values), then the rate
// features; info[t] = kind | (k >= nt/2) << 2 for top-level task t
__global__ void __launch_bounds__(256) k_features_agg(const uint8_t* __restrict__ depth, int64_t n, int n_top,
                                                      const uint8_t* __restrict__ info, const float* __restrict__ rate,
                                                      int n_rate, uint16_t* __restrict__ x) {
  const int l = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  float cnt[16], sum[8], num[8];
  for (int q = 0; q < 16; q++) cnt[q] = 0.f;
  for (int q = 0; q < 8; q++) sum[q] = num[q] = 0.f;
  const uint8_t* row = depth + c * n_top;
  for (int t = l; t < n_top; t += 64) {
    const int d = row[t] & 3, f = info[t];
    const int slot = (f & 3) * 4 + d, part = (f & 3) * 2 + ((f >> 2) & 1);
    // predicated updates keep the accumulators in registers
    for (int q = 0; q < 16; q++) cnt[q] += (q == slot) ? 1.f : 0.f;
    for (int q = 0; q < 8; q++) {
      sum[q] += (q == part) ? (float)d : 0.f;
      num[q] += (q == part) ? 1.f : 0.f;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    for (int q = 0; q < 16; q++) cnt[q] += __shfl_xor(cnt[q], o, 64);
    for (int q = 0; q < 8; q++) {
      sum[q] += __shfl_xor(sum[q], o, 64);
      num[q] += __shfl_xor(num[q], o, 64);
    }
  }
  if (l < kInDim) {
    float v = 0.f;
    if (l < 16) {
      float cv = 0.f, tot = 0.f;
      for (int q = 0; q < 16; q++) {
        cv = (q == l) ? cnt[q] : cv;
        tot += ((q >> 2) == (l >> 2)) ? cnt[q] : 0.f;
      }
      v = tot > 0.f ? cv / tot : 0.f;
    } else if (l < 24) {
      float sv = 0.f, nv = 0.f;
      for (int q = 0; q < 8; q++) {
        sv = (q == l - 16) ? sum[q] : sv;
        nv = (q == l - 16) ? num[q] : nv;
      }
      v = nv > 0.f ? sv / nv : 0.f;
    } else if (l < 24 + n_rate) {
      v = rate[l - 24];
    }
    x[c * kInDim + l] = f2bf(v);
  }
}

// normalised targets t = (ln(makespan) - mu) / sigma; 0 for failed candidates
__global__ void k_targets(const int64_t* __restrict__ ms, int64_t n, float mu, float sigma, float* __restrict__ t) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    t[i] = ms[i] > 0 ? (logf((float)ms[i]) - mu) / sigma : 0.f;
}

// y[m] = sum_n h[m][n] * w[n] + b (bf16 inputs, fp32 sum); one thread per row
__global__ void k_rowdot(const uint16_t* __restrict__ h, int64_t M, const uint16_t* __restrict__ w,
                         const float* __restrict__ b, float* __restrict__ y) {
  __shared__ float sw[kHidden];
  for (int i = threadIdx.x; i < kHidden; i += blockDim.x) sw[i] = bf2f(w[i]);
  __syncthreads();
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const u32x4* row = (const u32x4*)(h + m * kHidden);
  float s = 0.f;
  for (int q = 0; q < kHidden / 8; q++) {
    const u32x4 v = row[q];
    for (int e = 0; e < 4; e++) {
      s += __builtin_bit_cast(float, v[e] << 16) * sw[q * 8 + 2 * e];
      s += __builtin_bit_cast(float, v[e] & 0xFFFF0000u) * sw[q * 8 + 2 * e + 1];
    }
  }
  y[m] = s + b[0];
}

// output layer backward: dy = 2 (y - t) / n; dz3 = bf16(dy * w4 * [h3 > 0]);
// loss sums (y - t)^2 / n into loss[0].  kOutRows rows per workgroup, whose loss
// terms are summed first so that one atomic per workgroup reaches loss[0]
// (atomics on one address serialize).
constexpr int kOutRows = 16;
__global__ void k_out_backward(const float* __restrict__ y, const float* __restrict__ t, int64_t n,
                               const uint16_t* __restrict__ w4, const uint16_t* __restrict__ h3,
                               float* __restrict__ dy, uint16_t* __restrict__ dz3, float* __restrict__ loss) {
  const int64_t m0 = (int64_t)blockIdx.x * kOutRows;
  float part = 0.f;
  for (int r = 0; r < kOutRows && m0 + r < n; r++) {
    const int64_t m = m0 + r;
    const float d = y[m] - t[m];
    const float g = 2.f * d / (float)n;
    if (threadIdx.x == 0) {
      dy[m] = g;
      part += d * d / (float)n;
    }
    for (int j = threadIdx.x; j < kHidden; j += blockDim.x) {
      const uint16_t hv = h3[m * kHidden + j];
      dz3[m * kHidden + j] = hv != 0 ? f2bf(g * bf2f(w4[j])) : (uint16_t)0;
    }
  }
  if (threadIdx.x == 0) atomicAdd(loss, part);
}

// column sums: out[j] = sum_m a[m][j] (bf16) * (wcol ? wcol[m] : 1), fp32; one
// thread per (column, row slice), partial sums to parts[slice][j]
__global__ void k_colsum(const uint16_t* __restrict__ a, int64_t M, int ncol, const float* __restrict__ wcol,
                         int slices, float* __restrict__ parts) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= ncol) return;
  const int64_t rows = (M + slices - 1) / slices;
  const int64_t r0 = (int64_t)s * rows, r1 = r0 + rows < M ? r0 + rows : M;
  float acc = 0.f;
  for (int64_t m = r0; m < r1; m++) acc += bf2f(a[m * ncol + j]) * (wcol ? wcol[m] : 1.f);
  parts[(int64_t)s * ncol + j] = acc;
}

__global__ void k_sum_f32(const float* __restrict__ v, int64_t n, float* __restrict__ out) {
  __shared__ float sp[256];
  float s = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
  sp[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sp[threadIdx.x] += sp[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sp[0];
}

// Adam (Kingma and Ba, 2015) on fp32 master weights; bf16 copies refreshed
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t* __restrict__ wbf) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    const float wi = w[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    w[i] = wi;
    if (wbf) wbf[i] = f2bf(wi);
  }
}

// training batch: row r is row draw(seed, 7, step << 32 | r) mod n of (x, t)
__global__ void k_sample_rows(const uint16_t* __restrict__ x, const float* __restrict__ t, int64_t n, uint64_t seed,
                              uint64_t step, int batch, uint16_t* __restrict__ xb, float* __restrict__ tb) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= batch) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * 8ull;   // purpose 7
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = (z ^ (z >> 31)) + 0x9E3779B97F4A7C15ull * (((step << 32) | (uint64_t)r) + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  const int64_t row = (int64_t)(z % (uint64_t)n);
  const u32x4* src = (const u32x4*)(x + row * kInDim);
  u32x4* dst = (u32x4*)(xb + (int64_t)r * kInDim);
  for (int q = 0; q < kInDim / 8; q++) dst[q] = src[q];
  tb[r] = t[row];
}

__global__ void k_zero_f32(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.f;
}

__global__ void k_to_bf16(const float* __restrict__ w, int64_t n, uint16_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = f2bf(w[i]);
}

int grid1(int64_t n, int bs = 256) {
  int64_t g = (n + bs - 1) / bs;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

hipError_t gemm(bool ta, bool tb, int M, int N, int K, int splits, const uint16_t* A, int lda, const uint16_t* B,
                int ldb, const float* bias, bool relu, const uint16_t* mask, int ldm, float* out_f32,
                uint16_t* out_bf16, int ldc, hipStream_t s) {
  if (N % TN || K % (TK * splits) || M <= 0) return hipErrorInvalidValue;
  if (ta && M % 8) return hipErrorInvalidValue;
  const dim3 grid((M + TM - 1) / TM, N / TN, splits), block(256);
  const int kc = K / splits;
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<false, false>), grid, block, 0, s, M, N, kc, A, lda, B, ldb, bias, relu ? 1 : 0, mask, ldm,
                       out_f32, out_bf16, ldc);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, block, 0, s, M, N, kc, A, lda, B, ldb, bias, relu ? 1 : 0, mask, ldm,
                       out_f32, out_bf16, ldc);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, block, 0, s, M, N, kc, A, lda, B, ldb, bias, relu ? 1 : 0, mask, ldm,
                       out_f32, out_bf16, ldc);
  else
    hipLaunchKernelGGL((k_gemm<true, true>), grid, block, 0, s, M, N, kc, A, lda, B, ldb, bias, relu ? 1 : 0, mask, ldm,
                       out_f32, out_bf16, ldc);
  return hipGetLastError();
}

hipError_t mlp_forward(const uint16_t* x, int64_t n, const uint16_t* wt, const float* p, const uint16_t* w4, float* y,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((n + FM - 1) / FM)), dim3(FWAVES * 64), 0, s, x, n, wt, p, w4, y);
  return hipGetLastError();
}

hipError_t transpose_w(const float* p, uint16_t* wt, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_w, dim3(grid1(kTParams)), dim3(256), 0, s, p, wt);
  return hipGetLastError();
}

hipError_t sum_splits(const float* parts, int splits, int64_t count, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_splits, dim3(grid1(count)), dim3(256), 0, s, parts, splits, count, out);
  return hipGetLastError();
}

hipError_t features(const uint8_t* depth, int64_t n, int n_top, const float* rate, int n_rate, uint16_t* x,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3(grid1(n * kInDim)), dim3(256), 0, s, depth, n, n_top, rate, n_rate, x);
  return hipGetLastError();
}

hipError_t features_agg(const uint8_t* depth, int64_t n, int n_top, const uint8_t* info, const float* rate,
                        int n_rate, uint16_t* x, hipStream_t s) {
  hipLaunchKernelGGL(k_features_agg, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, depth, n, n_top, info, rate,
                     n_rate, x);
  return hipGetLastError();
}

hipError_t targets(const int64_t* ms, int64_t n, float mu, float sigma, float* t, hipStream_t s) {
  hipLaunchKernelGGL(k_targets, dim3(grid1(n)), dim3(256), 0, s, ms, n, mu, sigma, t);
  return hipGetLastError();
}

hipError_t rowdot(const uint16_t* h, int64_t M, const uint16_t* w, const float* b, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_rowdot, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, h, M, w, b, y);
  return hipGetLastError();
}

hipError_t out_backward(const float* y, const float* t, int64_t n, const uint16_t* w4, const uint16_t* h3, float* dy,
                        uint16_t* dz3, float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_out_backward, dim3((unsigned)((n + kOutRows - 1) / kOutRows)), dim3(256), 0, s, y, t, n, w4, h3, dy,
                     dz3, loss);
  return hipGetLastError();
}

hipError_t colsum(const uint16_t* a, int64_t M, int ncol, const float* wcol, int slices, float* parts, hipStream_t s) {
  hipLaunchKernelGGL(k_colsum, dim3((ncol + 255) / 256, slices), dim3(256), 0, s, a, M, ncol, wcol, slices, parts);
  return hipGetLastError();
}

hipError_t sum_f32(const float* v, int64_t n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_f32, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

hipError_t adam(float* w, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2, float eps,
                int step, uint16_t* wbf, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, s, w, g, m1, m2, n, lr, b1, b2, eps, c1, c2, wbf);
  return hipGetLastError();
}

hipError_t sample_rows(const uint16_t* x, const float* t, int64_t n, uint64_t seed, uint64_t step, int batch,
                       uint16_t* xb, float* tb, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_rows, dim3((batch + 255) / 256), dim3(256), 0, s, x, t, n, seed, step, batch, xb, tb);
  return hipGetLastError();
}

hipError_t zero_f32(float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f32, dim3(grid1(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t to_bf16(const float* w, int64_t n, uint16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(grid1(n)), dim3(256), 0, s, w, n, out);
  return hipGetLastError();
}

}  // namespace mlp
}  // namespace hesp
