/*
 * hesp.h -- C ABI of the batched HeSP scheduling-partitioning simulator for
 * AMD Instinct MI355X (gfx950).
 *
 * HeSP (Rey, Igual, Prieto-Matias, arXiv 1602.05510) takes (1) a platform of
 * memory spaces and processors tied to them and (2) a task to compute, and
 * returns (1) an equivalent set of finer-grained tasks with their dependences
 * and (2) a task-to-processor mapping, optimising performance (section 2,
 * problem statement).  This library evaluates many candidate partitionings of
 * the tiled Cholesky factorisation (Fig. 1) at once: each candidate is expanded
 * by recursive task splitting and list-scheduled by the Priority-List order and
 * the Earliest-Finish-Time processor rule with write-back caching of host data
 * in accelerator memory spaces (section 2.1, "Task and data scheduling
 * heuristics").  All times are int64 nanoseconds, so makespans are exact.
 *
 * Conventions
 *   - every function returns HESP_OK (0) or a negative status; the message of
 *     the last failing call on the calling thread is hesp_last_error();
 *   - the caller allocates every buffer it passes and keeps ownership; the
 *     library owns only the objects it creates (hesp_plan);
 *   - "d_" pointers are device pointers of the current HIP device, "host"
 *     pointers are ordinary host memory; asynchronous calls validate their
 *     arguments before enqueueing anything on `stream` (a hipStream_t, NULL =
 *     the null stream);
 *   - no C++ exception crosses this interface.
 */
#ifndef HESP_H_
#define HESP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define HESP_OK 0
#define HESP_EINVAL (-1)        /* bad argument */
#define HESP_ENOMEM (-2)        /* host or device allocation failed */
#define HESP_EHIP (-3)          /* a HIP runtime call failed */
#define HESP_ECAPACITY (-4)     /* candidate larger than the plan's workspace */
#define HESP_EUNSUPPORTED (-5)  /* policy or size outside what is implemented */

/* ---- task kinds (Fig. 1) ------------------------------------------------- */
#define HESP_CHOL 0  /* Cholesky factorisation of a diagonal block */
#define HESP_TRSM 1  /* triangular solve */
#define HESP_SYRK 2  /* symmetric rank-b update */
#define HESP_GEMM 3  /* matrix multiplication */

/* ---- limits --------------------------------------------------------------- */
#define HESP_MAX_PROCS 64   /* processors of a platform (one wavefront lane each) */
#define HESP_MAX_PTYPES 8   /* processor types */
#define HESP_MAX_MEM 16     /* memory spaces (space 0 is the host) */
#define HESP_MAX_LEVEL 3    /* split depth per task: block sides b, b/2, b/4, b/8 */
#define HESP_MAX_FINE 512   /* nt * 2^dmax, the finest tile count per dimension */

const char *hesp_last_error(void);
const char *hesp_version(void);

/* ---- cost model ------------------------------------------------------------
 * Section 2.1, "Performance and data transfer models": per processor type and
 * task kind, a task of side bl takes ceil(flops / R(bl)) ns with
 * R(bl) = Rmax * bl^2 / (bl^2 + h^2) GFLOP/s (1 GFLOP/s = 1 flop/ns) and
 * flops chol bl^3/3, trsm bl^3, syrk bl^3, gemm 2 bl^3; moving k finest
 * blocks (side b / 2^max_level, elem_bytes per element) between memory spaces
 * takes latency_ns + ceil(bytes / bw_bytes_per_ns) ns, and nothing when the
 * platform has a single shared memory space.
 */
typedef struct {
  int32_t n_ptypes;            /* 1..HESP_MAX_PTYPES */
  const int64_t *rmax_mflops;  /* host [n_ptypes][4]: peak rate per task kind, MFLOP/s, > 0 */
  const int64_t *h;            /* host [n_ptypes]: half-performance block side, >= 0 */
  int64_t b;                   /* level-0 tile side; divisible by 2^max_level */
  int32_t max_level;           /* 0..HESP_MAX_LEVEL */
  int64_t latency_ns;          /* per transfer */
  int64_t bw_bytes_per_ns;     /* = GB/s, > 0 */
  int64_t elem_bytes;          /* bytes per matrix element */
  int32_t shared_memory;       /* 1: single memory space, transfers cost 0 */
} hesp_cost_model;

/* Fills cost_ns (host [n_ptypes][4][max_level+1], level l = side b/2^l) and
 * xfer_ns (host [4^max_level + 1], index = number of finest blocks moved). */
int hesp_cost_tables(const hesp_cost_model *cm, int64_t *cost_ns, int64_t *xfer_ns);

/* ---- platform (section 2, problem input (1)) ------------------------------
 * Processor p has type proc_type[p] and works in memory space proc_mem[p];
 * space 0 is the host, where all data starts; every other space caches host
 * data (write-back).  The processor order is the EFT tie-break order (lowest
 * index wins).  All pointers are host pointers. */
typedef struct {
  int32_t n_procs;             /* 1..HESP_MAX_PROCS */
  int32_t n_ptypes;            /* 1..HESP_MAX_PTYPES */
  int32_t n_mem;               /* 1..HESP_MAX_MEM */
  int32_t max_level;           /* levels described by the tables, 0..HESP_MAX_LEVEL */
  const int32_t *proc_type;    /* [n_procs] */
  const int32_t *proc_mem;     /* [n_procs] */
  const int64_t *cost_ns;      /* [n_ptypes][4][max_level+1], >= 1 */
  const int64_t *xfer_ns;      /* [4^max_level + 1], xfer_ns[0] = 0, non-decreasing */
} hesp_platform;

/* Heuristics of section 2.1.  Only Priority-List order, EFT-P selection and
 * write-back caching are implemented; any other value gives HESP_EUNSUPPORTED. */
#define HESP_ORDER_PL 0
#define HESP_SELECT_EFT 0
#define HESP_CACHE_WB 0
typedef struct { int32_t order, select, cache; } hesp_policy;

/* ---- expansion of one candidate (host) ----------------------------------------
 * Section 2.1, "Recursive task partitioners", applied to the Fig. 1 loop nest:
 * depth[t] (host, tet(nt) = nt(nt+1)(nt+2)/6 entries in Fig. 1 order, each
 * 0..dmax) splits top-level task t depth[t] times; the result lists the fine
 * tasks (kind, level = split depth, fine loop indices K <= I <= J at that level)
 * and their successors (CSR, succ_ptr [n_tasks+1]).  Tasks are numbered
 * top-level task by top-level task, each by increasing K; every edge goes from a
 * lower to a higher number.  The edge set has the transitive closure of the
 * RaW/WaR/WaW hazards between the tasks' data blocks.
 * Two-call sizing: with tasks/succ_ptr/succ_idx NULL only n_tasks and n_edges are
 * written; otherwise the arrays must hold them. */
typedef struct { int32_t kind, level, K, I, J; } hesp_task;
int hesp_expand(int32_t nt, int32_t dmax, const uint8_t *depth, int32_t *n_tasks, int64_t *n_edges,
                hesp_task *tasks, int64_t *succ_ptr, int32_t *succ_idx);

/* ---- batches of candidates (device) -------------------------------------------
 * Candidate c has nt_c tiles per dimension, maximum split depth dmax_c and split
 * depths d_depth[mask_off_c .. mask_off_c + tet(nt_c)).  Uniform batches leave
 * d_nt / d_dmax / d_mask_off NULL and set nt / dmax (then mask_off_c = c*tet(nt)). */
typedef struct {
  int32_t n_cand;
  int32_t nt, dmax;            /* uniform shape, or the maxima over a ragged batch */
  const int32_t *d_nt;         /* [n_cand] or NULL */
  const int32_t *d_dmax;       /* [n_cand] or NULL */
  const int64_t *d_mask_off;   /* [n_cand + 1] or NULL */
  const uint8_t *d_depth;
} hesp_batch;

/* Candidate generation from counters (SplitMix64, Steele/Lea/Flood 2014): the
 * depth of top-level task t of candidate `first + c` is the number of leading
 * 21-bit chunks of the 64-bit value drawn for index ((first+c) << 24 | t) that
 * fall below split_thr (P(split) = split_thr / 2^21), capped at dmax. */
int hesp_generate_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt, int32_t dmax,
                          uint32_t split_thr, uint8_t *d_depth, void *stream);
/* Ragged shapes: nt_c = nt_lo + u mod (nt_hi-nt_lo+1), dmax_c = (u >> 32) mod (dmax_hi+1)
 * for the value u drawn for index first + c; d_mask_off gets the prefix sums of
 * tet(nt_c) (d_mask_off[0] = 0). */
int hesp_generate_ragged_shape(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt_lo,
                               int32_t nt_hi, int32_t dmax_hi, int32_t *d_nt, int32_t *d_dmax,
                               int64_t *d_mask_off, void *stream);
int hesp_generate_ragged_depth(uint64_t seed, int64_t first, const hesp_batch *batch,
                               uint32_t split_thr, uint8_t *d_depth, void *stream);

/* Expanded task and edge counts per candidate (d_n_tasks [n_cand], d_n_edges
 * [n_cand], either may be NULL). */
int hesp_count_batch(const hesp_batch *batch, int32_t *d_n_tasks, int64_t *d_n_edges, void *stream);

/* ---- plans: workspace, launch shape, capacities ------------------------------- */
typedef struct hesp_plan hesp_plan;
typedef struct {
  int32_t slots;               /* persistent single-wave workgroups; 0 = 32 per compute unit */
  int64_t max_tasks;           /* per-candidate expanded-task capacity; 0 = sized per batch */
  int64_t max_edges;           /* per-candidate edge capacity; 0 = sized per batch */
  int32_t max_nt;              /* largest nt a fixed-capacity plan must accept (0 = 64) */
} hesp_plan_opts;
int hesp_plan_create(hesp_plan **plan, const hesp_plan_opts *opts);
int hesp_plan_destroy(hesp_plan *plan);
/* device bytes currently held by the plan */
int hesp_plan_bytes(const hesp_plan *plan, int64_t *bytes);

/* ---- batched simulation ------------------------------------------------------
 * For every candidate: expansion, critical times, and the event simulation of
 * section 2.1 (ready tasks mapped in decreasing critical time as soon as they
 * are released, each to the processor with the earliest finish time counting
 * the transfers it needs; transfers issued at mapping time; write-back
 * coherence on completion).  d_makespan[c] gets the largest finish time,
 * d_status[c] HESP_OK, HESP_EINVAL (a depth above dmax_c) or HESP_ECAPACITY
 * (candidate larger than a fixed-capacity plan; makespan -1).
 * With d_sched_off non-NULL ([n_cand+1], task offsets per candidate, e.g. the
 * prefix sums of hesp_count_batch's n_tasks), the processor, start and finish
 * of every task are written at d_sched_off[c] + (task number of hesp_expand).
 * A plan with max_tasks = 0 sizes its workspace from the batch, which reads two
 * counts back to the host (one synchronisation of `stream`). */
typedef struct {
  int64_t *d_makespan;         /* [n_cand] */
  int32_t *d_status;           /* [n_cand] */
  int32_t *d_n_tasks;          /* [n_cand] expanded tasks per candidate, or NULL */
  const int64_t *d_sched_off;  /* [n_cand + 1] or NULL */
  int32_t *d_proc;             /* [d_sched_off[n_cand]] or NULL */
  int64_t *d_start;
  int64_t *d_finish;
} hesp_outputs;
int hesp_simulate_batch(hesp_plan *plan, const hesp_platform *pf, hesp_policy policy,
                        const hesp_batch *batch, const hesp_outputs *out, void *stream);

/* ---- batch reduction -------------------------------------------------------
 * Best candidate of a batch: the smallest makespan, ties to the lowest index
 * (section 2.1, "Iterative solver": the partition that best fits the platform).
 * Negative makespans (failed candidates) are ignored.  d_best gets
 * {makespan, index}, or {-1, -1} when no candidate succeeded. */
int hesp_argmin(const int64_t *d_makespan, int32_t n, int64_t *d_best, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HESP_H_ */
