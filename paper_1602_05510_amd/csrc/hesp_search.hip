// hesp_search.hip -- kernels of the partition search (gfx950): candidate
// enumeration, mutation of incumbents, ordering keys, a bitonic sort of 64-bit
// keys for top-k selection, and gathers of selected candidates.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_search.h"

namespace hesp {
namespace srch {

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr int kPurposeParent = 5, kPurposeMutate = 6;

__device__ __forceinline__ uint64_t draw(uint64_t seed, int purpose, uint64_t idx) {
  return mix64(mix64(seed + kGamma * (uint64_t)(purpose + 1)) + kGamma * (idx + 1));
}

int grid_for(int64_t n, int bs = 256) {
  int64_t g = (n + bs - 1) / bs;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// digit t (base dmax+1) of the candidate number first + c, least significant first
__global__ void k_enumerate(int64_t first, int32_t n, int32_t n_top, int32_t dmax, uint8_t* __restrict__ depth) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  uint64_t v = (uint64_t)(first + c);
  const uint64_t base = (uint64_t)dmax + 1;
  for (int t = 0; t < n_top; t++) {
    depth[c * n_top + t] = (uint8_t)(v % base);
    v /= base;
  }
}

// proposal c copies incumbent parent(c) of the pool and redraws the depth of
// each top-level task with probability thr / 2^21 (to one of the other dmax values)
__global__ void k_mutate(uint64_t seed, int64_t round, const uint8_t* __restrict__ pool, int32_t pool_n, int32_t n,
                         int32_t n_top, int32_t dmax, uint32_t thr, uint8_t* __restrict__ out) {
  const int64_t total = (int64_t)n * n_top;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / n_top;
    const int t = (int)(e - c * n_top);
    const uint64_t ci = ((uint64_t)round << 32) | (uint64_t)c;
    const int parent = (int)(draw(seed, kPurposeParent, ci) % (uint64_t)pool_n);
    const uint64_t u = mix64(draw(seed, kPurposeMutate, ci) + kGamma * (uint64_t)(t + 1));
    int d = pool[(int64_t)parent * n_top + t];
    if (dmax > 0 && (uint32_t)(u & 0x1FFFFFull) < thr) d = (d + 1 + (int)((u >> 21) % (uint64_t)dmax)) % (dmax + 1);
    out[e] = (uint8_t)d;
  }
}

constexpr uint64_t kMsCap = (1ull << 40) - 1;

__device__ __forceinline__ uint64_t ms_key(int64_t ms, uint64_t idx) {
  const uint64_t m = (ms < 0 || (uint64_t)ms > kMsCap) ? kMsCap : (uint64_t)ms;
  return (m << 24) | idx;
}

// keys of (a: na makespans, then b: nb makespans), index = position in the
// concatenation; padding up to n2 with the largest key
__global__ void k_keys_ms(const int64_t* __restrict__ a, int32_t na, const int64_t* __restrict__ b, int32_t nb,
                          int64_t n2, uint64_t* __restrict__ keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t k = ~0ull;
    if (i < na) k = ms_key(a[i], (uint64_t)i);
    else if (i < (int64_t)na + nb) k = ms_key(b[i - na], (uint64_t)i);
    keys[i] = k;
  }
}

// keys of the candidates [c0, c0 + nc) by decreasing size: (2^32-1 - tasks) << 32 | local index
__global__ void k_keys_size(const int32_t* __restrict__ n_tasks, int32_t c0, int32_t nc, int64_t n2,
                            uint64_t* __restrict__ keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t k = ~0ull;
    if (i < nc) k = ((uint64_t)(0xFFFFFFFFu - (uint32_t)n_tasks[c0 + i]) << 32) | (uint64_t)i;
    keys[i] = k;
  }
}

// keys of float scores: order-preserving bits (NaN last) above the index
__global__ void k_keys_f32(const float* __restrict__ s, int64_t n, int64_t n2, uint64_t* __restrict__ keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t k = ~0ull;
    if (i < n) {
      const float v = s[i];
      uint32_t u = __builtin_bit_cast(uint32_t, v);
      if (v != v) u = 0xFFFFFFFFu;
      else u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
      k = ((uint64_t)u << 32) | (uint64_t)i;
    }
    keys[i] = k;
  }
}

// ---- bitonic sort, ascending, n2 a power of two >= kLocal
constexpr int kLocal = 2048;   // elements per workgroup in the LDS stages

__device__ __forceinline__ void cas(uint64_t* s, int i, int l, bool up) {
  const uint64_t a = s[i], b = s[l];
  if ((a > b) == up) {
    s[i] = b;
    s[l] = a;
  }
}

// all stages with k <= kLocal
__global__ void __launch_bounds__(1024) k_sort_local(uint64_t* __restrict__ keys) {
  __shared__ uint64_t s[kLocal];
  const int64_t base = (int64_t)blockIdx.x * kLocal;
  for (int i = threadIdx.x; i < kLocal; i += 1024) s[i] = keys[base + i];
  __syncthreads();
  for (int k = 2; k <= kLocal; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int t = threadIdx.x;
      const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));   // lower element of pair t
      const bool up = (((base + i) & k) == 0);
      cas(s, i, i | j, up);
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < kLocal; i += 1024) keys[base + i] = s[i];
}

// one stage (k, j) with j >= kLocal, one thread per pair
__global__ void k_sort_step(uint64_t* __restrict__ keys, int64_t n2, int64_t k, int64_t j) {
  const int64_t pairs = n2 >> 1;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < pairs; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
    const int64_t l = i | j;
    const bool up = ((i & k) == 0);
    const uint64_t a = keys[i], b = keys[l];
    if ((a > b) == up) {
      keys[i] = b;
      keys[l] = a;
    }
  }
}

// stages j < kLocal of one k > kLocal, in LDS
__global__ void __launch_bounds__(1024) k_sort_merge(uint64_t* __restrict__ keys, int64_t k) {
  __shared__ uint64_t s[kLocal];
  const int64_t base = (int64_t)blockIdx.x * kLocal;
  for (int i = threadIdx.x; i < kLocal; i += 1024) s[i] = keys[base + i];
  __syncthreads();
  const bool up = ((base & k) == 0);
  for (int j = kLocal >> 1; j > 0; j >>= 1) {
    const int t = threadIdx.x;
    const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
    cas(s, i, i | j, up);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < kLocal; i += 1024) keys[base + i] = s[i];
}

__global__ void k_key_index(const uint64_t* __restrict__ keys, int32_t k, uint64_t mask, int32_t* __restrict__ idx) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < k) idx[r] = (int32_t)(keys[r] & mask);
}

// rows of the selected candidates: out[r] = src[idx[r]] (n_top bytes each)
__global__ void k_gather_rows(const int32_t* __restrict__ idx, int32_t k, const uint8_t* __restrict__ src,
                              int32_t n_top, uint8_t* __restrict__ out) {
  const int64_t total = (int64_t)k * n_top;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n_top;
    const int64_t t = e - r * n_top;
    out[e] = src[(int64_t)idx[r] * n_top + t];
  }
}

// new pool: the k smallest keys of (pool, batch); depths and makespans gathered
__global__ void k_gather_pool(const uint64_t* __restrict__ keys, int32_t k, const uint8_t* __restrict__ pool_d,
                              const int64_t* __restrict__ pool_ms, int32_t pool_n, const uint8_t* __restrict__ bat_d,
                              const int64_t* __restrict__ bat_ms, int32_t n_top, uint8_t* __restrict__ out_d,
                              int64_t* __restrict__ out_ms) {
  const int64_t total = (int64_t)k * n_top;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n_top;
    const int64_t t = e - r * n_top;
    const int64_t src = (int64_t)(keys[r] & 0xFFFFFFull);
    const bool from_pool = src < pool_n;
    out_d[e] = from_pool ? pool_d[src * n_top + t] : bat_d[(src - pool_n) * n_top + t];
    if (t == 0) out_ms[r] = from_pool ? pool_ms[src] : bat_ms[src - pool_n];
  }
}

// the successfully simulated rows of a round, in row order, into the replay ring
__global__ void __launch_bounds__(1024) k_append_ok(const int32_t* __restrict__ status,
                                                    const uint16_t* __restrict__ x, const int64_t* __restrict__ ms,
                                                    int64_t n, int32_t kdim, uint16_t* __restrict__ rep_x,
                                                    int64_t* __restrict__ rep_ms, int64_t ring, int64_t pos,
                                                    int64_t* __restrict__ count) {
  __shared__ int s_scan[1024];
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += 1024) {
    const int64_t r = base + threadIdx.x;
    const int ok = (r < n && status[r] == 0) ? 1 : 0;
    s_scan[threadIdx.x] = ok;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {           // inclusive scan (Hillis-Steele)
      const int v = threadIdx.x >= o ? s_scan[threadIdx.x - o] : 0;
      __syncthreads();
      s_scan[threadIdx.x] += v;
      __syncthreads();
    }
    if (ok) {
      const int64_t dst = (pos + carry + s_scan[threadIdx.x] - 1) % ring;
      for (int f = 0; f < kdim; f++) rep_x[dst * kdim + f] = x[r * kdim + f];
      rep_ms[dst] = ms[r];
    }
    carry += s_scan[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[0] = carry;
}

}  // namespace

hipError_t append_ok(const int32_t* status, const uint16_t* x, const int64_t* ms, int64_t n, int32_t kdim,
                     uint16_t* rep_x, int64_t* rep_ms, int64_t ring, int64_t pos, int64_t* count, hipStream_t s) {
  hipLaunchKernelGGL(k_append_ok, dim3(1), dim3(1024), 0, s, status, x, ms, n, kdim, rep_x, rep_ms, ring, pos, count);
  return hipGetLastError();
}

int64_t sort_len(int64_t n) {
  int64_t n2 = kLocal;
  while (n2 < n) n2 <<= 1;
  return n2;
}

hipError_t enumerate(int64_t first, int32_t n, int32_t n_top, int32_t dmax, uint8_t* depth, hipStream_t s) {
  hipLaunchKernelGGL(k_enumerate, dim3((n + 255) / 256), dim3(256), 0, s, first, n, n_top, dmax, depth);
  return hipGetLastError();
}

hipError_t mutate(uint64_t seed, int64_t round, const uint8_t* pool, int32_t pool_n, int32_t n, int32_t n_top,
                  int32_t dmax, uint32_t thr, uint8_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mutate, dim3(grid_for((int64_t)n * n_top)), dim3(256), 0, s, seed, round, pool, pool_n, n, n_top,
                     dmax, thr, out);
  return hipGetLastError();
}

hipError_t keys_ms(const int64_t* a, int32_t na, const int64_t* b, int32_t nb, int64_t n2, uint64_t* keys,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_keys_ms, dim3(grid_for(n2)), dim3(256), 0, s, a, na, b, nb, n2, keys);
  return hipGetLastError();
}

hipError_t size_order(const int32_t* n_tasks, int32_t c0, int32_t nc, uint64_t* keys, uint32_t* order, hipStream_t s) {
  const int64_t n2 = sort_len(nc);
  hipLaunchKernelGGL(k_keys_size, dim3(grid_for(n2)), dim3(256), 0, s, n_tasks, c0, nc, n2, keys);
  hipError_t e = sort(keys, n2, s);
  if (e != hipSuccess) return e;
  return key_index(keys, nc, 0xFFFFFFFFull, (int32_t*)order, s);
}

hipError_t keys_f32(const float* v, int64_t n, int64_t n2, uint64_t* keys, hipStream_t s) {
  hipLaunchKernelGGL(k_keys_f32, dim3(grid_for(n2)), dim3(256), 0, s, v, n, n2, keys);
  return hipGetLastError();
}

hipError_t sort(uint64_t* keys, int64_t n2, hipStream_t s) {
  if (n2 < kLocal || (n2 & (n2 - 1))) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)(n2 / kLocal);
  hipLaunchKernelGGL(k_sort_local, dim3(blocks), dim3(1024), 0, s, keys);
  for (int64_t k = 2 * kLocal; k <= n2; k <<= 1) {
    for (int64_t j = k >> 1; j >= kLocal; j >>= 1)
      hipLaunchKernelGGL(k_sort_step, dim3(grid_for(n2 >> 1)), dim3(256), 0, s, keys, n2, k, j);
    hipLaunchKernelGGL(k_sort_merge, dim3(blocks), dim3(1024), 0, s, keys, k);
  }
  return hipGetLastError();
}

hipError_t key_index(const uint64_t* keys, int32_t k, uint64_t mask, int32_t* idx, hipStream_t s) {
  hipLaunchKernelGGL(k_key_index, dim3((k + 255) / 256), dim3(256), 0, s, keys, k, mask, idx);
  return hipGetLastError();
}

hipError_t gather_rows(const int32_t* idx, int32_t k, const uint8_t* src, int32_t n_top, uint8_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_rows, dim3(grid_for((int64_t)k * n_top)), dim3(256), 0, s, idx, k, src, n_top, out);
  return hipGetLastError();
}

hipError_t gather_pool(const uint64_t* keys, int32_t k, const uint8_t* pool_d, const int64_t* pool_ms, int32_t pool_n,
                       const uint8_t* bat_d, const int64_t* bat_ms, int32_t n_top, uint8_t* out_d, int64_t* out_ms,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_gather_pool, dim3(grid_for((int64_t)k * n_top)), dim3(256), 0, s, keys, k, pool_d, pool_ms,
                     pool_n, bat_d, bat_ms, n_top, out_d, out_ms);
  return hipGetLastError();
}

}  // namespace srch
}  // namespace hesp
