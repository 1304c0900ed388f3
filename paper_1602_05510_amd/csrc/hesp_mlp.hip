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

// ---------------------------------------------------------------- fused forward
// The whole network for 128 rows per 512-thread workgroup.  Activations stay in
// LDS (128 x 256 bf16); weights come from L2 in the fragment-ordered bf16 copy
// of W^T (output feature rows, input features contiguous), so that each lane's
// weight operand is one 16-byte load and a wave's is one contiguous 1 KB.  Eight 16x16 blocks x two column blocks of accumulators per wave (64
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
      wf[cb] = *(const bf16x8*)(wt + kFrW1T + ((int64_t)(w * 2 + cb) * 64 + l) * 8);
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
    const uint16_t* wl = wt + (g < FKS ? kFrW2T : kFrW3T) + ((int64_t)(w * 2) * FKS + g % FKS) * 64 * 8 + l * 8;
#pragma unroll
    for (int cb = 0; cb < 2; cb++) wq[(g) % (FPRE + 1)][cb] = *(const bf16x8*)(wl + (int64_t)cb * FKS * 64 * 8);
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

// fragment-ordered bf16 copies (kFr*): W1^T, W2^T, W3^T, W2, W3
__global__ void k_frag_w(const float* __restrict__ p, uint16_t* __restrict__ wfr) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < kFrParams; e += (int64_t)gridDim.x * blockDim.x) {
    const int mat = e < kFrW2T ? 0 : (e < kFrW3T ? 1 : (e < kFrW2 ? 2 : (e < kFrW3 ? 3 : 4)));
    const int64_t base = mat == 0 ? kFrW1T : (mat == 1 ? kFrW2T : (mat == 2 ? kFrW3T : (mat == 3 ? kFrW2 : kFrW3)));
    const int K = mat == 0 ? kInDim : kHidden;
    const int64_t x = e - base, chunk = x >> 3;
    const int lane = (int)(chunk & 63), blk = (int)(chunk >> 6);
    const int row = (blk / (K >> 5)) * 16 + (lane & 15);
    const int k = (blk % (K >> 5)) * 32 + (lane >> 4) * 8 + (int)(x & 7);
    int64_t src;
    if (mat == 0) src = kOffW1 + (int64_t)k * kHidden + row;            // W1^T[n][i] = W1[i][n]
    else if (mat <= 2) src = (mat == 1 ? kOffW2 : kOffW3) + (int64_t)k * kHidden + row;
    else src = (mat == 3 ? kOffW2 : kOffW3) + (int64_t)row * kHidden + k;
    wfr[e] = f2bf(p[src]);
  }
}

// Adam (Kingma and Ba, 2015) on one fp32 master weight, as k_adam; returns the
// bf16 bits of the new weight, also stored in the bf16 copy
__device__ __forceinline__ uint16_t adam_one(const AdamArgs& a, int64_t i, float gi) {
  const float m = a.b1 * a.m1[i] + (1.f - a.b1) * gi;
  const float v = a.b2 * a.m2[i] + (1.f - a.b2) * gi * gi;
  a.m1[i] = m;
  a.m2[i] = v;
  const float wi = a.p[i] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
  a.p[i] = wi;
  const uint16_t b = f2bf(wi);
  a.wbf[i] = b;
  return b;
}

// ---------------------------------------------------------------- training step
// One gradient step is three launches.
//   k_tr_rows  (TRB rows per workgroup): forward pass with the activations kept
//              in LDS, output-layer backward, and the data gradients dz3, dz2,
//              dz1 of the hidden layers (rows are independent up to here).  The
//              inputs, activations and data gradients are also written in the
//              packed layout below, the operand layout of the next pass.
//   k_tr_wgrad (a 64 x 64 tile of a weight matrix and 512 rows per workgroup):
//              partial weight and bias gradients as MFMA products over the rows;
//   k_tr_adam  sums the partial sums of every tile in a fixed order, writes the
//              gradient and, in a training step, applies Adam and refreshes the
//              bf16 copies (so one gradient step is three launches).
// Rounding points are those of the forward pass above and of the reference:
// activations and data gradients are bf16 (round to nearest even), products
// accumulate in fp32, dy and every gradient are fp32.
// Row pass shape: RT 16-row blocks per workgroup (TRB = 16 RT rows) and NW waves,
// wave w owning CT = 16 / NW column blocks of 16, columns [16 CT w, 16 CT (w + 1)).
constexpr int TRT = 1, TNW = 16;
constexpr int TRB = 16 * TRT;

// Packed layout of a [rows][F] bf16 tensor: element (b, f) at ((b / 8) F + f) 8 + b % 8,
// so that one feature of eight consecutive rows is one 16-byte chunk.
__device__ __forceinline__ int64_t pk(int64_t b, int64_t f, int F) { return ((b >> 3) * F + f) * 8 + (b & 7); }

__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ uint32_t bf16x2_rne(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2));
}
__device__ __forceinline__ float lo_f(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__device__ __forceinline__ float hi_f(uint32_t w) { return __builtin_bit_cast(float, w & 0xFFFF0000u); }

// 4 values of rows row0 .. row0+3 of one column: into the LDS tile (row-major,
// swizzled) and into the packed global tensor (one 8-byte store; row0 % 4 == 0)
__device__ __forceinline__ void tr_put(uint32_t v01, uint32_t v23, uint16_t* sT, uint16_t* __restrict__ gp,
                                       int64_t grow0, int row0, int col) {
  sT[sh_off(row0 + 0, col)] = (uint16_t)v01;
  sT[sh_off(row0 + 1, col)] = (uint16_t)(v01 >> 16);
  sT[sh_off(row0 + 2, col)] = (uint16_t)v23;
  sT[sh_off(row0 + 3, col)] = (uint16_t)(v23 >> 16);
  *(uint2*)(gp + pk(grow0 + row0, col, kHidden)) = make_uint2(v01, v23);
}

// The weight fragments of a K = 256 product for the wave's CT column blocks
// (row blocks rb0 .. rb0 + CT - 1 of a fragment-ordered matrix), all eight
// k-steps: one contiguous 1 KB per fragment.  They do not depend on the
// activations, so each product's fragments are requested one stage ahead (a
// scheduling barrier keeps the loads where they are issued).
template <int CT>
struct WFrags {
  u32x4 f[FKS][CT];
};
template <int CT>
__device__ __forceinline__ void tr_wload(WFrags<CT>& wf, const uint16_t* __restrict__ m, int rb0, int l) {
#pragma unroll
  for (int ks = 0; ks < FKS; ks++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++) wf.f[ks][ct] = *(const u32x4*)(m + (((int64_t)(rb0 + ct) * FKS + ks) * 64 + l) * 8);
  __builtin_amdgcn_sched_barrier(0);
}

// acc[rt][ct] += rows 16 rt .. of the LDS tile sIn (K = 256) times the fragments
template <int RT, int CT>
__device__ __forceinline__ void tr_gemm(f32x4 (&acc)[RT][CT], const uint16_t* sIn, const WFrags<CT>& wf, int l) {
#pragma unroll
  for (int ks = 0; ks < FKS; ks++) {
    const int k = ks * 32 + (l >> 4) * 8;
    bf16x8 a[RT];
#pragma unroll
    for (int rt = 0; rt < RT; rt++) a[rt] = *(const bf16x8*)&sIn[sh_off(rt * 16 + (l & 15), k)];
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], as_bf(wf.f[ks][ct]), acc[rt][ct], 0, 0, 0);
  }
}

// bias of the lane's column in all four rows of every accumulator block
template <int RT, int CT>
__device__ __forceinline__ void tr_bias(f32x4 (&acc)[RT][CT], const float* __restrict__ b, int c0) {
#pragma unroll
  for (int ct = 0; ct < CT; ct++) {
    const float v = b ? b[c0 + 16 * ct] : 0.f;
#pragma unroll
    for (int rt = 0; rt < RT; rt++) acc[rt][ct] = f32x4{v, v, v, v};
  }
}

// SplitMix64 (Steele, Lea, Flood 2014): training row r of step `step` is row
// draw(seed, 7, step << 32 | r) mod n
__device__ __forceinline__ int64_t tr_row(uint64_t seed, uint64_t step, int64_t r, int64_t n) {
  auto mix = [](uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const uint64_t g = 0x9E3779B97F4A7C15ull;
  return (int64_t)(mix(mix(seed + g * 8ull) + g * (((step << 32) | (uint64_t)r) + 1)) % (uint64_t)n);
}

// sample: rows drawn as above from (x, t) of n rows; else rows blockIdx.x * TRB .. of x, t
template <int RT, int NW>
__global__ void __launch_bounds__(NW * 64) k_tr_rows(const uint16_t* __restrict__ x, const float* __restrict__ t,
                                                     int64_t n, int sample, uint64_t seed, uint64_t step, int batch,
                                                     const uint16_t* __restrict__ wt, const uint16_t* __restrict__ wb,
                                                     const float* __restrict__ p, TrainBufs tb) {
  constexpr int RB = 16 * RT, CT = 16 / NW;
  __shared__ __attribute__((aligned(16))) uint16_t sX[RB * kInDim];
  __shared__ __attribute__((aligned(16))) uint16_t sH1[RB * kHidden];
  __shared__ __attribute__((aligned(16))) uint16_t sH2[RB * kHidden];
  __shared__ __attribute__((aligned(16))) uint16_t sT3[RB * kHidden];   // dz3
  __shared__ __attribute__((aligned(16))) uint16_t sD2[RB * kHidden];   // dz2
  __shared__ float sYp[NW][RB];
  __shared__ float sDy[RB], sT[RB];
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * RB;
  const int c0 = w * 16 * CT + (l & 15);   // the lane's columns: c0 + 16 ct
  const int rb0 = w * CT;                  // their 16-row blocks of the fragment-ordered weights
  const int rq = (l >> 4) * 4;             // first of the lane's four rows in a 16-row block

  // inputs: 16 bytes per thread, and the packed copy of the rows
  for (int q = tid; q < RB * 4; q += NW * 64) {
    const int j = q >> 2, c = q & 3;
    const int64_t src = sample ? tr_row(seed, step, r0 + j, n) : r0 + j;
    *(u32x4*)&sX[j * kInDim + c * 8] = *(const u32x4*)(x + src * kInDim + c * 8);
    if (c == 0) sT[j] = t[src];
  }
  WFrags<CT> wA, wB;
  tr_wload(wA, wt + kFrW2T, rb0, l);
  __syncthreads();
  for (int q = tid; q < (RB / 8) * kInDim; q += NW * 64) {
    const int b8 = q / kInDim, f = q % kInDim;
    uint32_t v[4];
    for (int e = 0; e < 4; e++)
      v[e] = (uint32_t)sX[(b8 * 8 + 2 * e) * kInDim + f] | ((uint32_t)sX[(b8 * 8 + 2 * e + 1) * kInDim + f] << 16);
    *(u32x4*)(tb.xp + ((r0 / 8 + b8) * kInDim + f) * 8) = u32x4{v[0], v[1], v[2], v[3]};
  }

  f32x4 acc[RT][CT];
  // layer 1 (K = 32)
  tr_bias(acc, p + kOffB1, c0);
  {
    u32x4 b1[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
      b1[ct] = *(const u32x4*)(wt + kFrW1T + ((int64_t)(rb0 + ct) * 64 + l) * 8);
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
      const bf16x8 a = *(const bf16x8*)&sX[(rt * 16 + (l & 15)) * kInDim + (l >> 4) * 8];
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, as_bf(b1[ct]), acc[rt][ct], 0, 0, 0);
    }
  }
#pragma unroll
  for (int rt = 0; rt < RT; rt++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
      tr_put(relu_bf16x2(acc[rt][ct][0], acc[rt][ct][1]), relu_bf16x2(acc[rt][ct][2], acc[rt][ct][3]), sH1, tb.h1p,
             r0, rt * 16 + rq, c0 + 16 * ct);
  __syncthreads();
  // layer 2
  tr_wload(wB, wt + kFrW3T, rb0, l);
  tr_bias(acc, p + kOffB2, c0);
  tr_gemm(acc, sH1, wA, l);
#pragma unroll
  for (int rt = 0; rt < RT; rt++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
      tr_put(relu_bf16x2(acc[rt][ct][0], acc[rt][ct][1]), relu_bf16x2(acc[rt][ct][2], acc[rt][ct][3]), sH2, tb.h2p,
             r0, rt * 16 + rq, c0 + 16 * ct);
  __syncthreads();
  // layer 3: h3 stays in registers (the lane computes dz3 at the same places);
  // partial output dots over the wave's columns
  tr_wload(wA, wt + kFrW3, rb0, l);
  tr_bias(acc, p + kOffB3, c0);
  tr_gemm(acc, sH2, wB, l);
  uint32_t h3[RT][CT][2];
  float w4f[CT];
#pragma unroll
  for (int ct = 0; ct < CT; ct++) w4f[ct] = bf2f(wb[kOffW4 + c0 + 16 * ct]);
#pragma unroll
  for (int rt = 0; rt < RT; rt++) {
    float py[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      h3[rt][ct][0] = relu_bf16x2(acc[rt][ct][0], acc[rt][ct][1]);
      h3[rt][ct][1] = relu_bf16x2(acc[rt][ct][2], acc[rt][ct][3]);
      *(uint2*)(tb.h3p + pk(r0 + rt * 16 + rq, c0 + 16 * ct, kHidden)) = make_uint2(h3[rt][ct][0], h3[rt][ct][1]);
      py[0] += lo_f(h3[rt][ct][0]) * w4f[ct];
      py[1] += hi_f(h3[rt][ct][0]) * w4f[ct];
      py[2] += lo_f(h3[rt][ct][1]) * w4f[ct];
      py[3] += hi_f(h3[rt][ct][1]) * w4f[ct];
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      float v = py[q];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      if ((l & 15) == 0) sYp[w][rt * 16 + rq + q] = v;
    }
  }
  __syncthreads();
  // output, dy = 2 (y - t) / batch, loss terms (y - t)^2 / batch
  if (tid < RB) {
    float y = p[kOffB4];
    for (int q = 0; q < NW; q++) y += sYp[q][tid];
    const float d = y - sT[tid];
    const float g = 2.f * d / (float)batch;
    sDy[tid] = g;
    tb.dy[r0 + tid] = g;
    float lp = d * d / (float)batch;
    for (int o = 1; o < RB; o <<= 1) lp += __shfl_xor(lp, o, 64);
    if (tid == 0) tb.lossp[blockIdx.x] = lp;   // summed in block order by k_tr_adam
  }
  __syncthreads();
  // dz3 = bf16(dy w4) where h3 > 0
#pragma unroll
  for (int rt = 0; rt < RT; rt++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      uint16_t v[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const uint32_t hb = q & 1 ? h3[rt][ct][q >> 1] >> 16 : h3[rt][ct][q >> 1] & 0xFFFFu;
        v[q] = hb != 0 ? f2bf(sDy[rt * 16 + rq + q] * w4f[ct]) : (uint16_t)0;
      }
      tr_put(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16), sT3, tb.d3p, r0, rt * 16 + rq,
             c0 + 16 * ct);
    }
  __syncthreads();
  // dz2 = bf16(dz3 W3^T) where h2 > 0, then dz1 = bf16(dz2 W2^T) where h1 > 0
  // (W[i][n] rows are the weight fragments: output column i, k = n contiguous)
#pragma unroll
  for (int layer = 3; layer >= 2; layer--) {
    const uint16_t* sIn = layer == 3 ? sT3 : sD2;
    const uint16_t* sMask = layer == 3 ? sH2 : sH1;
    if (layer == 3) tr_wload(wB, wt + kFrW2, rb0, l);
    tr_bias(acc, nullptr, c0);
    tr_gemm(acc, sIn, layer == 3 ? wA : wB, l);
#pragma unroll
    for (int rt = 0; rt < RT; rt++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const int col = c0 + 16 * ct, row = rt * 16 + rq;
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; q++) v[q] = sMask[sh_off(row + q, col)] != 0 ? acc[rt][ct][q] : 0.f;
        const uint32_t v01 = bf16x2_rne(v[0], v[1]), v23 = bf16x2_rne(v[2], v[3]);
        if (layer == 3) {
          tr_put(v01, v23, sD2, tb.d2p, r0, row, col);
        } else {
          *(uint2*)(tb.d1p + pk(r0 + row, col, kHidden)) = make_uint2(v01, v23);
        }
      }
    if (layer == 3) __syncthreads();
  }
}

// Weight-gradient tiles: 0..3 the 32 x 64 tiles of W1 (columns 64 t ..), 4..19 the
// 64 x 64 tiles of W2 and 20..35 those of W3 (rows 64 (u / 4) .., columns 64 (u % 4) ..).
constexpr int kTrTiles = 36;
constexpr int kTrRows = 128;                    // rows of one wave's slice (four k-steps)
constexpr int kPartW = 64 * 64;                 // partial sums of one workgroup: weights,
constexpr int kPartStride = kPartW + 3 * 64;    // then bias, w4 and b4 sums (64 each)
static_assert(kTrTiles == kTrainTiles && kPartStride == kTrainPartStride, "training workspace sizes of hesp_mlp.h");

struct TileInfo {
  int layer, i0, n0, rows, F;
  bool bias, out4;
};
__device__ __forceinline__ TileInfo tile_info(int tile) {
  TileInfo t;
  t.layer = tile < 4 ? 1 : (tile < 20 ? 2 : 3);
  const int u = t.layer == 1 ? 0 : (t.layer == 2 ? tile - 4 : tile - 20);
  t.i0 = t.layer == 1 ? 0 : 64 * (u / 4);
  t.n0 = t.layer == 1 ? 64 * tile : 64 * (u % 4);
  t.rows = t.layer == 1 ? 32 : 64;
  t.F = t.layer == 1 ? kInDim : kHidden;
  t.bias = t.i0 == 0;
  t.out4 = t.layer == 3 && t.i0 == 0;
  return t;
}

// Partial sums: workgroup (tile, group g), g < G = batch / 512; its four waves sum
// the rows [(4 g + w) 128, + 128) (four k-steps, every operand requested before
// the first product) and add their sums in wave order.
__global__ void __launch_bounds__(256) k_tr_wgrad(TrainBufs tb, int G) {
  __shared__ float sAcc[4][kPartW];
  __shared__ float sVec[4][3][64];
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int tile = blockIdx.x / G, grp = blockIdx.x % G;
  const TileInfo ti = tile_info(tile);
  const int mi = ti.rows / 16;
  const uint16_t* A = ti.layer == 1 ? tb.xp : (ti.layer == 2 ? tb.h1p : tb.h2p);
  const uint16_t* B = ti.layer == 1 ? tb.d1p : (ti.layer == 2 ? tb.d2p : tb.d3p);
  const int64_t b8_0 = (int64_t)(grp * 4 + w) * (kTrRows / 8) + (l >> 4);

  constexpr int KS = kTrRows / 32;
  u32x4 fa[KS][4], fb[KS][4], fh[KS][4];
  f32x4 fd[KS][2];
#pragma unroll
  for (int ks = 0; ks < KS; ks++) {
    const int64_t b8 = b8_0 + ks * 4;
#pragma unroll
    for (int ib = 0; ib < 4; ib++)
      if (ib < mi) fa[ks][ib] = *(const u32x4*)(A + (b8 * ti.F + ti.i0 + ib * 16 + (l & 15)) * 8);
#pragma unroll
    for (int jb = 0; jb < 4; jb++) fb[ks][jb] = *(const u32x4*)(B + (b8 * kHidden + ti.n0 + jb * 16 + (l & 15)) * 8);
    if (ti.out4) {
#pragma unroll
      for (int jb = 0; jb < 4; jb++)
        fh[ks][jb] = *(const u32x4*)(tb.h3p + (b8 * kHidden + ti.n0 + jb * 16 + (l & 15)) * 8);
      fd[ks][0] = *(const f32x4*)(tb.dy + b8 * 8);
      fd[ks][1] = *(const f32x4*)(tb.dy + b8 * 8 + 4);
    }
  }
  __builtin_amdgcn_sched_barrier(0);

  f32x4 acc[4][4];
#pragma unroll
  for (int ib = 0; ib < 4; ib++)
#pragma unroll
    for (int jb = 0; jb < 4; jb++) acc[ib][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bs[4] = {0.f, 0.f, 0.f, 0.f}, ws[4] = {0.f, 0.f, 0.f, 0.f}, b4s = 0.f;
#pragma unroll
  for (int ks = 0; ks < KS; ks++) {
#pragma unroll
    for (int ib = 0; ib < 4; ib++)
      if (ib < mi)
#pragma unroll
        for (int jb = 0; jb < 4; jb++)
          acc[ib][jb] =
              __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(fa[ks][ib]), as_bf(fb[ks][jb]), acc[ib][jb], 0, 0, 0);
    if (ti.bias) {
#pragma unroll
      for (int jb = 0; jb < 4; jb++)
#pragma unroll
        for (int e = 0; e < 4; e++) bs[jb] += lo_f(fb[ks][jb][e]) + hi_f(fb[ks][jb][e]);
    }
    if (ti.out4) {
      const float d[8] = {fd[ks][0][0], fd[ks][0][1], fd[ks][0][2], fd[ks][0][3],
                          fd[ks][1][0], fd[ks][1][1], fd[ks][1][2], fd[ks][1][3]};
#pragma unroll
      for (int jb = 0; jb < 4; jb++)
#pragma unroll
        for (int e = 0; e < 4; e++) ws[jb] += lo_f(fh[ks][jb][e]) * d[2 * e] + hi_f(fh[ks][jb][e]) * d[2 * e + 1];
      if ((l & 15) == 0)
        for (int e = 0; e < 8; e++) b4s += d[e];
    }
  }

#pragma unroll
  for (int ib = 0; ib < 4; ib++)
    if (ib < mi)
#pragma unroll
      for (int jb = 0; jb < 4; jb++)
#pragma unroll
        for (int q = 0; q < 4; q++) sAcc[w][(ib * 16 + (l >> 4) * 4 + q) * 64 + jb * 16 + (l & 15)] = acc[ib][jb][q];
#pragma unroll
  for (int jb = 0; jb < 4; jb++) {
    float b = bs[jb], c = ws[jb];
    b += __shfl_xor(b, 16, 64);
    b += __shfl_xor(b, 32, 64);
    c += __shfl_xor(c, 16, 64);
    c += __shfl_xor(c, 32, 64);
    if (l < 16) {
      sVec[w][0][jb * 16 + l] = b;
      sVec[w][1][jb * 16 + l] = c;
    }
  }
  b4s += __shfl_xor(b4s, 16, 64);
  b4s += __shfl_xor(b4s, 32, 64);
  sVec[w][2][l] = l == 0 ? b4s : 0.f;
  __syncthreads();
  float* part = tb.part + ((int64_t)tile * G + grp) * kPartStride;
  const int nn = tid & 63, ib0 = (tid >> 6) * 16;   // thread: column nn, rows ib0 .. ib0 + 15
  for (int e = 0; e < 16; e++) {
    const int i = ib0 + e;
    if (i < ti.rows) {
      const int x = i * 64 + nn;
      part[x] = ((sAcc[0][x] + sAcc[1][x]) + sAcc[2][x]) + sAcc[3][x];
    }
  }
  if (tid < 3 * 64) {
    const int v = tid >> 6;
    part[kPartW + tid] = ((sVec[0][v][nn] + sVec[1][v][nn]) + sVec[2][v][nn]) + sVec[3][v][nn];
  }
}

// Sums of the G partial sums (in group order), one parameter per thread: a
// workgroup of 1024 threads takes 16 rows x 64 columns of a tile (thread: row
// t / 64, column t % 64), writes the gradient and, with ad.on, applies Adam and
// refreshes the bf16 copies (the fragment-ordered ones through LDS, one 16-byte
// store per thread).  Jobs 0..7: W1 tiles x 2 row groups; 8..135: W2, W3 tiles
// x 4.  Row group 0 of a tile also takes its bias, w4 and b4 entries; job 0 also
// sums the row pass's loss terms (in row-block order) into *loss.
constexpr int kTrJobs = 8 + 32 * 4;
__global__ void __launch_bounds__(1024) k_tr_adam(TrainBufs tb, int G, int n_rowblocks, float* __restrict__ grad,
                                                  AdamArgs ad, float* __restrict__ loss) {
  __shared__ uint16_t sW[16][64];
  const int job = blockIdx.x, tid = threadIdx.x, nn = tid & 63, e = tid >> 6;
  const int tile = job < 8 ? job / 2 : 4 + (job - 8) / 4;
  const int rg = job < 8 ? job % 2 : (job - 8) % 4;
  const TileInfo ti = tile_info(tile);
  const float* pt = tb.part + (int64_t)tile * G * kPartStride;
  auto total = [&](int x) {
    // eight partial sums requested at a time, added in group order
    float s = 0.f;
    for (int g0 = 0; g0 < G; g0 += 8) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; j++) v[j] = g0 + j < G ? pt[(int64_t)(g0 + j) * kPartStride + x] : 0.f;
#pragma unroll
      for (int j = 0; j < 8; j++) s += v[j];
    }
    return s;
  };
  const int64_t offW = ti.layer == 1 ? kOffW1 : (ti.layer == 2 ? kOffW2 : kOffW3);
  const int64_t offB = ti.layer == 1 ? kOffB1 : (ti.layer == 2 ? kOffB2 : kOffB3);
  const int i = rg * 16 + e;
  const int64_t gi = offW + (int64_t)(ti.i0 + i) * kHidden + ti.n0 + nn;
  const float gv = total(i * 64 + nn);
  grad[gi] = gv;
  if (ad.on) {
    sW[e][nn] = adam_one(ad, gi, gv);
    __syncthreads();
    const int ig = ti.i0 + rg * 16;   // first input feature (row of W) of the block
    if (tid < 128) {
      // W^T fragments: rows n, k = input feature; thread: column n0 + (tid % 64), 8 k
      const int nl = tid & 63, c = tid >> 6, n = ti.n0 + nl;
      uint32_t v[4];
      for (int q = 0; q < 4; q++) v[q] = sW[8 * c + 2 * q][nl] | (uint32_t)sW[8 * c + 2 * q + 1][nl] << 16;
      const int64_t base = ti.layer == 1 ? kFrW1T : (ti.layer == 2 ? kFrW2T : kFrW3T);
      *(u32x4*)(ad.wfr + base + fr_index(n, ig + 8 * c, ti.F)) = u32x4{v[0], v[1], v[2], v[3]};
    } else if (tid < 256 && ti.layer > 1) {
      // W fragments: rows = input features ig .. ig + 15, k = n; thread: one row, 8 n
      const int q8 = tid - 128, r = q8 & 15, c = q8 >> 4;   // c: which 8 of the 64 columns
      uint32_t v[4];
      for (int q = 0; q < 4; q++) v[q] = sW[r][8 * c + 2 * q] | (uint32_t)sW[r][8 * c + 2 * q + 1] << 16;
      const int64_t base = ti.layer == 2 ? kFrW2 : kFrW3;
      *(u32x4*)(ad.wfr + base + fr_index(ig + r, ti.n0 + 8 * c, kHidden)) = u32x4{v[0], v[1], v[2], v[3]};
    }
  }
  if (rg == 0 && tid < 64) {
    if (ti.bias) {
      const int64_t gb = offB + ti.n0 + nn;
      const float v = total(kPartW + nn);
      grad[gb] = v;
      if (ad.on) adam_one(ad, gb, v);
    }
    if (ti.out4) {
      const int64_t g4 = kOffW4 + ti.n0 + nn;
      const float v = total(kPartW + 64 + nn);
      grad[g4] = v;
      if (ad.on) adam_one(ad, g4, v);
      if (ti.n0 == 0 && nn == 0) {
        const float gb = total(kPartW + 128);
        grad[kOffB4] = gb;
        if (ad.on) adam_one(ad, kOffB4, gb);
      }
    }
  }
  if (job == 0 && tid < 64 && loss) {
    float s = 0.f;
    for (int r = tid; r < n_rowblocks; r += 64) s += tb.lossp[r];
    for (int o = 1; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
    if (tid == 0) *loss = s;
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
// the fraction of its top-level tasks at depth 0, 1, 2 and 3 or more (16
// values), for each kind and each half of the k range the mean depth (8
// values), then the rate features; info[t] = kind | (k >= nt/2) << 2 for
// top-level task t
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
    const int d = row[t], f = info[t];
    const int slot = (f & 3) * 4 + (d < 3 ? d : 3), part = (f & 3) * 2 + ((f >> 2) & 1);
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

hipError_t mlp_forward(const uint16_t* x, int64_t n, const uint16_t* wt, const float* p, const uint16_t* w4, float* y,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((n + FM - 1) / FM)), dim3(FWAVES * 64), 0, s, x, n, wt, p, w4, y);
  return hipGetLastError();
}

hipError_t frag_w(const float* p, uint16_t* wfr, hipStream_t s) {
  hipLaunchKernelGGL(k_frag_w, dim3(grid1(kFrParams)), dim3(256), 0, s, p, wfr);
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

hipError_t adam(float* w, const float* g, float* m1, float* m2, int64_t n, float lr, float b1, float b2, float eps,
                int step, uint16_t* wbf, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid1(n)), dim3(256), 0, s, w, g, m1, m2, n, lr, b1, b2, eps, c1, c2, wbf);
  return hipGetLastError();
}

hipError_t train_rows(const uint16_t* x, const float* t, int64_t n, bool sample, uint64_t seed, uint64_t step,
                      int batch, const uint16_t* wt, const uint16_t* wb, const float* p, const TrainBufs& tb,
                      hipStream_t s) {
  if (batch <= 0 || batch % 512 || n < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_tr_rows<TRT, TNW>), dim3((unsigned)(batch / TRB)), dim3(TNW * 64), 0, s, x, t, n, sample ? 1 : 0, seed,
                     step, batch, wt, wb, p, tb);
  return hipGetLastError();
}

hipError_t train_wgrad(const TrainBufs& tb, int batch, float* g, const AdamArgs& ad, float* loss, hipStream_t s) {
  if (batch <= 0 || batch % 512) return hipErrorInvalidValue;
  const int G = batch / 512;
  hipLaunchKernelGGL(k_tr_wgrad, dim3(kTrTiles * G), dim3(256), 0, s, tb, G);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tr_adam, dim3(kTrJobs), dim3(1024), 0, s, tb, G, batch / TRB, g, ad, loss);
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
