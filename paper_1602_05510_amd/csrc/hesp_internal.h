// hesp_internal.h -- launch-level types shared by the C ABI implementation and
// the gfx950 kernels.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hesp {

constexpr int kWave = 64;
constexpr int kMaxProcs = 64;
constexpr int kMaxPtypes = 8;
constexpr int kMaxMem = 16;
constexpr int kLevels = 4;                 // levels 0..3
constexpr int kXferLen = 65;               // 4^3 + 1

// Platform tables passed by value as a kernel argument (about 1.8 KB).
struct SimTables {
  int32_t n_procs, n_ptypes, n_mem, max_level;
  int8_t proc_type[kMaxProcs];
  int8_t proc_mem[kMaxProcs];
  int64_t cost[kMaxPtypes][4][kLevels];   // task time, ns
  int64_t W[4][kLevels];                  // sum of the task time over all processors
  int64_t xfer[kXferLen];                 // transfer time by number of finest blocks
};

struct BatchView {
  int32_t n_cand, nt, dmax;                // uniform values (or maxima for a ragged batch)
  const int32_t* nt_arr;                   // nullable
  const int32_t* dmax_arr;                 // nullable
  const int64_t* off;                      // nullable: c * tet(nt)
  const uint8_t* depth;
};

// Per-slot workspace: one slot per persistent workgroup, `stride` bytes apart.
struct Workspace {
  char* base;
  int64_t stride;
  int64_t cap_tasks, cap_edges, cap_tops, cap_vf;  // cap_vf = atoms * memory spaces
  int64_t o_top_first, o_desc, o_rec, o_indeg, o_cur, o_succ, o_fifo, o_ready, o_sort, o_vf;
};

struct OutView {
  int64_t* makespan;
  int32_t* status;
  int32_t* n_tasks;
  const int64_t* sched_off;
  int32_t* proc;
  int64_t* start;
  int64_t* finish;
};

Workspace make_workspace_layout(int64_t cap_tasks, int64_t cap_edges, int64_t cap_tops, int64_t cap_vf);

hipError_t launch_count(const BatchView& b, int32_t* n_tasks, int64_t* n_edges, hipStream_t s);
hipError_t launch_simulate(const SimTables& t, const BatchView& b, const Workspace& w, const OutView& o,
                           int32_t slots, uint32_t* counter, hipStream_t s);
hipError_t launch_gen_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt, int32_t dmax,
                              uint32_t thr, uint8_t* depth, hipStream_t s);
hipError_t launch_gen_shape(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt_lo, int32_t nt_hi,
                            int32_t dmax_hi, int32_t* nt, int32_t* dmax, int64_t* off, hipStream_t s);
hipError_t launch_gen_ragged_depth(uint64_t seed, int64_t first, const BatchView& b, uint32_t thr,
                                   uint8_t* depth, hipStream_t s);
hipError_t launch_argmin(const int64_t* v, int32_t n, int64_t* best, hipStream_t s);
hipError_t launch_max_i32_i64(const int32_t* a, const int64_t* b, int32_t n, int64_t* out2, hipStream_t s);

}  // namespace hesp
