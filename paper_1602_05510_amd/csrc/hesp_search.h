// hesp_search.h -- launch-level interface of the search kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hesp {
namespace srch {

// length of the sort buffer for n keys (a power of two, at least 2048)
int64_t sort_len(int64_t n);

hipError_t enumerate(int64_t first, int32_t n, int32_t n_top, int32_t dmax, uint8_t* depth, hipStream_t s);
hipError_t mutate(uint64_t seed, int64_t round, const uint8_t* pool, int32_t pool_n, int32_t n, int32_t n_top,
                  int32_t dmax, uint32_t thr, uint8_t* out, hipStream_t s);
// key = min(makespan, 2^40-1) << 24 | position in (a ++ b); positions < 2^24
hipError_t keys_ms(const int64_t* a, int32_t na, const int64_t* b, int32_t nb, int64_t n2, uint64_t* keys,
                   hipStream_t s);
// key = order-preserving bits of the score << 32 | position
hipError_t keys_f32(const float* v, int64_t n, int64_t n2, uint64_t* keys, hipStream_t s);
hipError_t sort(uint64_t* keys, int64_t n2, hipStream_t s);
// order[0..nc) = local indices of candidates c0 .. c0+nc-1, largest task count
// first (ties to the lower index); keys: sort_len(nc) entries of workspace
hipError_t size_order(const int32_t* n_tasks, int32_t c0, int32_t nc, uint64_t* keys, uint32_t* order, hipStream_t s);
hipError_t key_index(const uint64_t* keys, int32_t k, uint64_t mask, int32_t* idx, hipStream_t s);
hipError_t gather_rows(const int32_t* idx, int32_t k, const uint8_t* src, int32_t n_top, uint8_t* out, hipStream_t s);
// rows r < n with status[r] == 0 (features x, kdim values each, and makespan ms)
// appended to the ring buffer (rep_x, rep_ms) of `ring` rows at position pos, in
// row order; count[0] = rows appended (one workgroup)
hipError_t append_ok(const int32_t* status, const uint16_t* x, const int64_t* ms, int64_t n, int32_t kdim,
                     uint16_t* rep_x, int64_t* rep_ms, int64_t ring, int64_t pos, int64_t* count, hipStream_t s);
hipError_t gather_pool(const uint64_t* keys, int32_t k, const uint8_t* pool_d, const int64_t* pool_ms, int32_t pool_n,
                       const uint8_t* bat_d, const int64_t* bat_ms, int32_t n_top, uint8_t* out_d, int64_t* out_ms,
                       hipStream_t s);

}  // namespace srch
}  // namespace hesp
