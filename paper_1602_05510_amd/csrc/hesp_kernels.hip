// hesp_kernels.hip -- candidate generation, counting and reductions (gfx950).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_core.h"
#include "hesp_device.h"
#include "hesp_internal.h"

namespace hesp {

namespace {

using namespace dev;

// ---------------------------------------------------------------- counting

__global__ void __launch_bounds__(kWave) k_count(BatchView b, int32_t* n_tasks, int64_t* n_edges) {
  const int c = blockIdx.x;
  if (c >= b.n_cand) return;
  const Cand cd = load_cand(b, c);
  if (cd.nt < 1 || cd.dmax < 0 || cd.dmax > kMaxLevel || (cd.nt << cd.dmax) > kMaxFine) {
    if (lane() == 0) {
      if (n_tasks) n_tasks[c] = 0;
      if (n_edges) n_edges[c] = 0;
    }
    return;
  }
  int64_t edges = 0, tasks = 0;
  auto depth_of = [&](int64_t t) { int d = cd.depth[t]; return d > cd.dmax ? cd.dmax : d; };
  auto first_of = [&](int64_t t) { return t << 32; };   // distinct per top-level task
  for_each_fine(cd, [&](bool valid, int64_t f, int64_t top, uint32_t cell, int d, int K, int I, int J) {
    (void)f;
    if (valid) {
      tasks++;
      edges += for_each_pred(cd.nt, depth_of, first_of, top, cell, d, K, I, J, [](int64_t) {});
    }
  });
  // wave sums
  for (int o = 32; o > 0; o >>= 1) {
    edges += __shfl_xor(edges, o, kWave);
    tasks += __shfl_xor(tasks, o, kWave);
  }
  if (lane() == 0) {
    if (n_tasks) n_tasks[c] = (int32_t)tasks;
    if (n_edges) n_edges[c] = edges;
  }
}

// ---------------------------------------------------------------- generation

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kPurposeDepth = 2, kPurposeShape = 3, kPurposeTree = 5, kPurposeDepth2 = 6;

__device__ __forceinline__ uint64_t draw(uint64_t seed, int purpose, uint64_t idx) {
  const uint64_t s = mix64(seed + kGamma * (uint64_t)(purpose + 1));
  return mix64(s + kGamma * (idx + 1));
}

// leading 21-bit chunks below thr, capped at dmax: three of the value drawn for
// idx, then (depths 4 and 5) three of a second value drawn for the same idx
__device__ __forceinline__ uint8_t depth_of_draw(uint64_t seed, uint64_t idx, uint32_t thr, int dmax) {
  int d = 0;
  for (int half = 0; half < 2 && d == 3 * half && d < dmax; half++) {
    const uint64_t u = draw(seed, half ? kPurposeDepth2 : kPurposeDepth, idx);
    for (int j = 0; j < 3 && d < dmax; j++) {
      const uint32_t ch = (uint32_t)((u >> (21 * j)) & 0x1FFFFFull);
      if (ch < thr) d++;
      else break;
    }
  }
  return (uint8_t)d;
}

__global__ void k_gen_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t n_top, int32_t dmax,
                              uint32_t thr, uint8_t* depth) {
  const int64_t total = (int64_t)n_cand * n_top;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = x / n_top, t = x % n_top;
    depth[x] = depth_of_draw(seed, ((uint64_t)(first + c) << 24) | (uint64_t)t, thr, dmax);
  }
}

// split-tree flags: flag x of candidate c is set when the leading 21 bits of the
// draw for (c << 32 | x) fall below thr
__global__ void k_gen_tree(uint64_t seed, int64_t first, int32_t n_cand, int64_t n_flags, uint32_t thr,
                           uint8_t* flags) {
  const int64_t total = (int64_t)n_cand * n_flags;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = x / n_flags, i = x % n_flags;
    const uint64_t u = draw(seed, kPurposeTree, ((uint64_t)(first + c) << 32) | (uint64_t)i);
    flags[x] = (uint32_t)(u >> 43) < thr ? 1 : 0;
  }
}

__global__ void k_gen_shape(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt_lo, int32_t nt_hi,
                            int32_t dmax_hi, int32_t* nt, int32_t* dmax, int64_t* tops) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cand) return;
  const uint64_t u = draw(seed, kPurposeShape, (uint64_t)(first + c));
  const int n = nt_lo + (int)(u % (uint64_t)(nt_hi - nt_lo + 1));
  nt[c] = n;
  dmax[c] = (int)((u >> 32) % (uint64_t)(dmax_hi + 1));
  tops[c] = tet3(n);
}

// single-workgroup exclusive scan: off[0] = 0, off[c+1] = off[c] + v[c]
__global__ void __launch_bounds__(1024) k_scan_excl(const int64_t* v, int32_t n, int64_t* off) {
  __shared__ int64_t s_part[16];
  __shared__ int64_t s_carry;
  if (threadIdx.x == 0) { s_carry = 0; off[0] = 0; }
  __syncthreads();
  const int l = lane(), wv = threadIdx.x / kWave;
  for (int base = 0; base < n; base += 1024) {
    const int i = base + threadIdx.x;
    int64_t x = i < n ? v[i] : 0;
    int64_t incl = x;
    for (int o = 1; o < kWave; o <<= 1) {
      int64_t y = __shfl_up(incl, o, kWave);
      if (l >= o) incl += y;
    }
    if (l == kWave - 1) s_part[wv] = incl;
    __syncthreads();
    int64_t pre = s_carry;
    for (int q = 0; q < wv; q++) pre += s_part[q];
    if (i < n) off[i + 1] = pre + incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t s = 0;
      for (int q = 0; q < 16; q++) s += s_part[q];
      s_carry += s;
    }
    __syncthreads();
  }
}

__global__ void k_gen_ragged_depth(uint64_t seed, int64_t first, BatchView b, uint32_t thr, uint8_t* depth) {
  const int c = blockIdx.x;
  if (c >= b.n_cand) return;
  const int nt = b.nt_arr[c], dmax = b.dmax_arr[c];
  const int64_t n_top = tet3(nt), o = b.off[c];
  for (int64_t t = threadIdx.x; t < n_top; t += blockDim.x) {
    depth[o + t] = depth_of_draw(seed, ((uint64_t)(first + c) << 24) | (uint64_t)t, thr, dmax);
  }
}

// ---------------------------------------------------------------- reductions

__global__ void __launch_bounds__(1024) k_argmin(const int64_t* v, int32_t n, int64_t* best) {
  __shared__ int64_t s_v[16];
  __shared__ int64_t s_i[16];
  int64_t bv = kInf, bi = -1;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int64_t x = v[i];
    if (x >= 0 && (x < bv || (x == bv && i < bi))) { bv = x; bi = i; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t ov = __shfl_xor(bv, o, kWave), oi = __shfl_xor(bi, o, kWave);
    if (oi >= 0 && (ov < bv || (ov == bv && (bi < 0 || oi < bi)))) { bv = ov; bi = oi; }
  }
  const int wv = threadIdx.x / kWave;
  if (lane() == 0) { s_v[wv] = bv; s_i[wv] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t rv = kInf, ri = -1;
    for (int q = 0; q < (int)(blockDim.x / kWave); q++)
      if (s_i[q] >= 0 && (s_v[q] < rv || (s_v[q] == rv && s_i[q] < ri))) { rv = s_v[q]; ri = s_i[q]; }
    best[0] = ri >= 0 ? rv : -1;
    best[1] = ri;
  }
}

__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_count(const BatchView& b, int32_t* n_tasks, int64_t* n_edges, hipStream_t s) {
  if (b.n_cand <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_count, dim3(b.n_cand), dim3(kWave), 0, s, b, n_tasks, n_edges);
  return hipGetLastError();
}

hipError_t launch_gen_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt, int32_t dmax,
                              uint32_t thr, uint8_t* depth, hipStream_t s) {
  if (n_cand <= 0) return hipSuccess;
  const int64_t total = (int64_t)n_cand * tet3(nt);
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gen_uniform, dim3((unsigned)blocks), dim3(256), 0, s, seed, first, n_cand,
                     (int32_t)tet3(nt), dmax, thr, depth);
  return hipGetLastError();
}

hipError_t launch_gen_tree(uint64_t seed, int64_t first, int32_t n_cand, int64_t n_flags, uint32_t thr,
                           uint8_t* flags, hipStream_t s) {
  if (n_cand <= 0 || n_flags <= 0) return hipSuccess;
  const int64_t total = (int64_t)n_cand * n_flags;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gen_tree, dim3((unsigned)blocks), dim3(256), 0, s, seed, first, n_cand, n_flags, thr, flags);
  return hipGetLastError();
}

hipError_t launch_gen_shape(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt_lo, int32_t nt_hi,
                            int32_t dmax_hi, int32_t* nt, int32_t* dmax, int64_t* off, hipStream_t s) {
  if (n_cand <= 0) {
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, (const int64_t*)nullptr, 0, off);
    return hipGetLastError();
  }
  // off[1..n] first holds tet(nt_c), then is scanned in place from a copy
  int64_t* tops = off + 1;
  hipLaunchKernelGGL(k_gen_shape, dim3((n_cand + 255) / 256), dim3(256), 0, s, seed, first, n_cand, nt_lo,
                     nt_hi, dmax_hi, nt, dmax, tops);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // in-place scan: each 1024-chunk reads its inputs before writing (one workgroup, ordered)
  hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, s, (const int64_t*)tops, n_cand, off);
  return hipGetLastError();
}

hipError_t launch_gen_ragged_depth(uint64_t seed, int64_t first, const BatchView& b, uint32_t thr,
                                   uint8_t* depth, hipStream_t s) {
  if (b.n_cand <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gen_ragged_depth, dim3(b.n_cand), dim3(256), 0, s, seed, first, b, thr, depth);
  return hipGetLastError();
}

hipError_t launch_argmin(const int64_t* v, int32_t n, int64_t* best, hipStream_t s) {
  hipLaunchKernelGGL(k_argmin, dim3(1), dim3(1024), 0, s, v, n, best);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, p);
  return hipGetLastError();
}

}  // namespace hesp
