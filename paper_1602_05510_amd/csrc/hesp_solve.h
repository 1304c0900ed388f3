// hesp_solve.h -- launch-level interface of the iterative solver's partition
// stage (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hesp {
namespace solve {

constexpr int kMaxTop = 4096;   // top-level tasks of one chain (nt <= 28)
constexpr int kMaxP = 64;       // processors (6 bits of a packed time key)
constexpr int kMaxTypes = 8;
constexpr int kLv = 6;          // split depths 0..5

struct SolveTables {
  int32_t n_procs;
  int8_t proc_type[kMaxP];
  int64_t cost[kMaxTypes][4][kLv];   // task time by processor type, kind, depth (ns)
};

struct SolveView {
  int32_t n_chains, nt, dmax, n_top;
  int32_t iter, iters, list, sampling;
  uint64_t seed;                 // chain r draws with seed + r
  uint8_t* depth;                // [n_chains][n_top] current partition
  uint8_t* best_depth;           // [n_chains][n_top]
  int64_t* best_ms;              // [n_chains]
  int64_t* trace;                // [n_chains][iters] or null
  int64_t* steps;                // [n_chains][iters][3] or null
  // schedule of the current partitions: chain r's tasks at r * stride
  int64_t stride;
  const int32_t* n_tasks;        // [n_chains]
  const int32_t* proc;
  const int64_t* start;
  const int64_t* finish;
  const int64_t* makespan;       // [n_chains]
  const int32_t* status;         // [n_chains]
  // workspace
  uint32_t* first;               // [n_chains][n_top + 1]
  uint64_t* t0key;               // [n_chains][n_top]: earliest (start, processor)
  uint64_t* fin;                 // [n_chains][n_top]: latest finish
  int32_t* par;                  // per task: latest-finishing DAG predecessor, -1 if none
  int32_t* cl;                   // per task: its cluster
  uint64_t* lastkey;             // [n_chains]: latest (finish, lowest processor)
};

// off[c] = c * stride for c = 0..count
hipError_t launch_strided(int64_t stride, int32_t count, int64_t* off, hipStream_t s);
hipError_t launch_first(const SolveView& v, hipStream_t s);
hipError_t launch_tasks(const SolveView& v, int64_t max_tasks, hipStream_t s);
hipError_t launch_part(const SolveView& v, const SolveTables& t, hipStream_t s);

// split-tree partitions: the clusters ("nodes") are the existing tasks of the
// levels below dmax, one per split flag
struct TreeSolveView {
  int32_t n_chains, nt, dmax, n_nodes;         // n_nodes = split flags per chain (<= kMaxTop)
  int32_t iter, iters, list, sampling;
  uint64_t seed;
  int64_t level_off[kLv + 1];                  // first node of each level
  uint8_t* flags;                              // [n_chains][n_nodes] current partitions
  uint8_t* best_flags;
  int64_t* best_ms;
  int64_t* trace;                              // [n_chains][iters] or null
  int64_t* steps;                              // [n_chains][iters][3]: node, 1 split / 0 merge, score
  int64_t stride;                              // tasks per chain in the schedule arrays
  const int32_t* n_tasks;
  const int32_t* proc;
  const int64_t* start;
  const int64_t* finish;
  const int64_t* makespan;
  const int32_t* status;
  // workspace
  uint32_t* lw;                                // [n_chains][finest blocks]: last writer
  uint32_t* desc;                              // per task: packed descriptor
  int32_t* par;                                // per task: latest-finishing predecessor
  uint64_t* t0key;                             // [n_chains][n_nodes]
  uint64_t* fin;                               // [n_chains][n_nodes]
  uint64_t* lastkey;                           // [n_chains]
  int32_t* lmin;                               // [n_chains]: smallest task level
};

hipError_t launch_tree_init(const TreeSolveView& v, hipStream_t s);
hipError_t launch_tree_tasks(const TreeSolveView& v, hipStream_t s);
hipError_t launch_tree_part(const TreeSolveView& v, const SolveTables& t, hipStream_t s);

}  // namespace solve
}  // namespace hesp
