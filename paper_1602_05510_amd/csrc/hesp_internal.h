// hesp_internal.h -- launch-level types shared by the C ABI implementation and
// the gfx950 kernels.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hesp_core.h"

namespace hesp {

constexpr int kWave = 64;
constexpr int kMaxProcs = 64;
constexpr int kMaxPtypes = 8;
constexpr int kMaxMem = 16;
constexpr int kLevels = kMaxLevel + 1;     // levels 0..5
constexpr int kXferLevels = 3;             // transfer times passed by value: up to 4^3 finest blocks
constexpr int kXferLen = 65;               // 4^3 + 1
static_assert(kXferLen == (1 << (2 * kXferLevels)) + 1, "transfer times passed by value");

// Platform tables passed by value as a kernel argument (about 1.8 KB).
struct SimTables {
  int32_t n_procs, n_ptypes, n_mem, max_level;
  int8_t proc_type[kMaxProcs];
  int8_t proc_mem[kMaxProcs];
  int64_t cost[kMaxPtypes][4][kLevels];   // task time, ns
  int64_t W[4][kLevels];                  // sum of the task time over all processors
  int64_t xfer[kXferLen];                 // transfer time by number of finest blocks (the first 65)
  const int64_t* xfer_deep;               // device copy of all 4^max_level + 1, when max_level > 3
  int32_t fcfs;                           // task order: 0 Priority-List, 1 first released first
  int32_t sel;                            // processor: 0 earliest finish, 1 earliest idle, 2 random idle,
                                          // 3 fastest idle (2, 3: tasks wait while no processor is idle)
  uint64_t seed;                          // random choices (SplitMix64)
  int32_t cache;                          // written blocks: 0 write-back, 1 write-through, 2 write-around
  int32_t bus;                            // 1: transfers contend, one at a time on each link
  int8_t link[kMaxMem];                   // link carrying the transfers into each memory space
  int32_t capped;                         // 1: some space has a finite capacity
  int64_t capacity[kMaxMem];              // blocks of side b/2^max_level; -1: unbounded
};

struct BatchView {
  int32_t n_cand, nt, dmax;                // uniform values (or maxima for a ragged batch)
  const int32_t* nt_arr;                   // nullable
  const int32_t* dmax_arr;                 // nullable
  const int64_t* off;                      // nullable: c * tet(nt)
  const uint8_t* depth;                    // split depth per top-level task, or split-tree flags
  int64_t tree_stride;                     // 0: depths; > 0: split-tree flags, this many per candidate
};

// A chunk of consecutive candidates [c0, c0 + nc) and its buffers.  The
// *_off arrays are exclusive prefix sums over the whole batch of the exact
// per-candidate sizes; a candidate's arrays start at (off[c] - off[c0]).
struct ChunkView {
  const int64_t* task_off;
  const int64_t* edge_off;
  const int64_t* vf_off;
  const int64_t* top_off;
  int32_t c0, nc;
  int64_t cap_tasks, cap_edges;            // 0 = unlimited; larger candidates get HESP_ECAPACITY
  int32_t prep_in;                          // critical-time pass: internal edges kept in LDS (1..1024)
  uint32_t* top_first;                      // tet(nt)+1 per candidate
  uint32_t* desc;                           // per task
  uint32_t* indeg;                          // per task
  uint32_t* cur;                            // per task
  uint32_t* succ;                           // per edge
  int64_t* rec;                             // 4 per task
  int64_t* fifo;                            // 3 per task
  uint32_t* ready;                          // per task
  int64_t* sortbuf;                         // 4 per task
  int64_t* vf;                              // finest blocks x memory spaces
  int64_t* use;                             // finite spaces: latest use per validity word (else null)
  uint32_t* pin;                            // finite spaces: unfinished tasks using it (else null)
  int32_t* nsrc;                            // per candidate of the chunk
  const uint32_t* order;                    // nullable: simulation order of the chunk's candidates
  const int32_t* cnt_tasks;                 // per candidate of the batch: expanded tasks
  const int64_t* cnt_edges;                 // per candidate of the batch: edges
  // region mode (region != nullptr): each candidate's arrays lie together in one
  // block of region_bytes(...) bytes at region + byte_off[c] - byte_off[c0]
  // instead of in the per-array buffers above; candidates whose block ends past
  // region_cap get HESP_ECAPACITY
  const int64_t* byte_off;
  uint8_t* region;
  int64_t region_cap;
  // fused simulation (slot_bytes > 0): the persistent kernel prepares each
  // candidate itself into slot blockIdx.x of slot_bytes bytes at region (sizes
  // from cnt_tasks / cnt_edges); candidates whose block is larger get
  // HESP_ECAPACITY
  int64_t slot_bytes;
  int32_t slot_lds;                         // 1: the slot is the workgroup's dynamic LDS (no region)
};

// largest workspace slot kept in LDS by the fused pipeline (with the event
// loop's own LDS it stays within 64 KiB per workgroup)
constexpr int64_t kLdsSlotMax = 48 << 10;

// bytes of one candidate's block in region mode: T tasks, E edges, V validity
// words, TP top-level tasks + 1 (16-byte multiple)
__host__ __device__ inline int64_t region_bytes(int64_t T, int64_t E, int64_t V, int64_t TP) {
  const int64_t b = 32 * T + 24 * T + 32 * T + 8 * V + 16 * T + 4 * E + 4 * TP;
  return (b + 15) & ~(int64_t)15;
}

struct OutView {
  int64_t* makespan;
  int32_t* status;
  int32_t* n_tasks;
  const int64_t* sched_off;
  int32_t* proc;
  int64_t* start;
  int64_t* finish;
};

hipError_t launch_count(const BatchView& b, int32_t* n_tasks, int64_t* n_edges, hipStream_t s);
// off_b (nullable): prefix sums of region_bytes per candidate; part (nullable):
// 5 x ceil(n_cand / 1024) int64 of scratch for the many-workgroup scan
hipError_t launch_layout(const BatchView& b, int32_t n_mem, const int32_t* n_tasks, const int64_t* n_edges,
                         int64_t cap_t, int64_t cap_e, int64_t* off_t, int64_t* off_e, int64_t* off_v,
                         int64_t* off_top, int64_t* off_b, hipStream_t s, int64_t* part = nullptr);
hipError_t launch_bounds(const int64_t* off_t, const int64_t* off_e, const int64_t* off_v, const int64_t* off_top,
                         int32_t n, int32_t chunk, int32_t n_chunks, int64_t* out, hipStream_t s);
hipError_t launch_prepare(const SimTables& t, const BatchView& b, const ChunkView& v, const OutView& o,
                          hipStream_t s);
// split-tree batches (b.tree_stride > 0, uniform shape): exact task and edge
// counts (scratch: one last-writer word per finest block and candidate), and
// the preparation of a chunk
hipError_t launch_count_tree(const BatchView& b, uint32_t* scratch, int32_t* n_tasks, int64_t* n_edges,
                             hipStream_t s);
hipError_t launch_prepare_tree(const SimTables& t, const BatchView& b, const ChunkView& v, const OutView& o,
                               hipStream_t s);
hipError_t launch_sim(const SimTables& t, const BatchView& b, const ChunkView& v, const OutView& o, int32_t slots,
                      int32_t group, uint32_t* counter, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* p, hipStream_t s);
// out[0] (int64, device) = the largest region_bytes of a candidate of the batch
hipError_t launch_max_region(const BatchView& b, int32_t n_mem, const int32_t* n_tasks, const int64_t* n_edges,
                             int64_t* out, hipStream_t s);
hipError_t launch_gen_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt, int32_t dmax,
                              uint32_t thr, uint8_t* depth, hipStream_t s);
hipError_t launch_gen_tree(uint64_t seed, int64_t first, int32_t n_cand, int64_t n_flags, uint32_t thr,
                           uint8_t* flags, hipStream_t s);
hipError_t launch_gen_shape(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt_lo, int32_t nt_hi,
                            int32_t dmax_hi, int32_t* nt, int32_t* dmax, int64_t* off, hipStream_t s);
hipError_t launch_gen_ragged_depth(uint64_t seed, int64_t first, const BatchView& b, uint32_t thr,
                                   uint8_t* depth, hipStream_t s);
hipError_t launch_argmin(const int64_t* v, int32_t n, int64_t* best, hipStream_t s);

}  // namespace hesp
