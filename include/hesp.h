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
#define HESP_MAX_LEVEL 5    /* split depth per task: block sides b, b/2, ..., b/32 */
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
 * index wins).  All pointers are host pointers.
 * Finite spaces (section 2: memory spaces of finite size): capacity[m] > 0
 * bounds accelerator space m to that many blocks of side b / 2^max_level; a
 * candidate of depth dmax counts whole finest blocks of side b / 2^dmax, so it
 * holds capacity[m] / 4^(max_level - dmax) of them.  A task goes only to a
 * processor whose space can hold the finest blocks of the tasks mapped there and
 * not finished plus its own (EFT-P among those); when none can, it and the
 * tasks after it in the order wait for the next completion, and a task that no
 * space can ever hold gives HESP_ECAPACITY.  Room is made when the task is
 * mapped by dropping the least recently used other blocks of the space (use =
 * the latest mapping there of a task touching the block; ties: upper-triangle
 * tiles row by row, then row-major inside the tile); a dropped block with no
 * copy on the host is copied back first, one transfer of one finest block
 * issued at that time.  Supported with write-back caching, EFT-P, independent
 * transfers, depth batches and the unfused pipeline (else HESP_EUNSUPPORTED);
 * 64 lanes per candidate.  capacity NULL, capacity[m] <= 0 and space 0:
 * unbounded. */
typedef struct {
  int32_t n_procs;             /* 1..HESP_MAX_PROCS */
  int32_t n_ptypes;            /* 1..HESP_MAX_PTYPES */
  int32_t n_mem;               /* 1..HESP_MAX_MEM */
  int32_t max_level;           /* levels described by the tables, 0..HESP_MAX_LEVEL */
  const int32_t *proc_type;    /* [n_procs] */
  const int32_t *proc_mem;     /* [n_procs] */
  const int64_t *cost_ns;      /* [n_ptypes][4][max_level+1], >= 1 */
  const int64_t *xfer_ns;      /* [4^max_level + 1], xfer_ns[0] = 0, non-decreasing */
  const int64_t *capacity;     /* [n_mem] or NULL: blocks of side b/2^max_level per space (above) */
  const int32_t *link;         /* [n_mem] or NULL: link of the transfers into each space (hesp_policy.bus) */
} hesp_platform;

/* Heuristics of section 2.1 ("Task and data scheduling heuristics").  Tasks are
 * mapped when released (push at release).  Order of the tasks released at one
 * instant: Priority-List (decreasing critical time) or FCFS (release order; all
 * of them share the instant, so ties by scaled (K,I,J) decide); both break ties
 * by scaled (K,I,J).  Processor: EFT-P (earliest finish counting the transfers
 * the task needs) or EIT-P (earliest idle time, an idle processor counting from
 * now); ties to the lowest index.  R-P (random) and F-P (fastest: smallest task
 * time, ties to the lowest index) choose among the processors idle now (nothing
 * queued); while none is idle the remaining released tasks wait and are mapped,
 * in order, at later completions (FCFS then means earliest release first).  R-P
 * takes the u-th idle processor in index order, u = SplitMix64 value
 * draw(seed, 8, corner) mod (idle count), corner = K' << 18 | I' << 9 | J' with
 * (K', I', J') the task's first cell on the finest grid.
 * Caching (section 2: accelerator spaces as software caches of the host, space
 * 0): write-back keeps a written block only in the executing space;
 * write-through keeps it there and sends a copy to the host at the completion,
 * valid there one block transfer later; write-around keeps no accelerator copy,
 * only that host copy.  A missing block's transfer starts at the mapping time,
 * or once every missing finest block has a valid copy somewhere (write-around:
 * its host copy may still be in flight).  Other values give HESP_EUNSUPPORTED.
 * bus = 1: transfers contend (section 2: the spaces are connected by a network
 * topology): a transfer occupies the link of the space it goes into,
 * hesp_platform.link[m] (0..n_mem-1; spaces naming the same link share it;
 * NULL: one interconnect shared by every transfer), one transfer at a time per
 * link in issue order (the missing blocks of a task in their order;
 * write-through and write-around host copies queue on the host's link at the
 * completion); the EFT-P estimate sees each link's queue.  An out-of-range link
 * gives HESP_EINVAL.  bus = 0: transfers do not contend (link is ignored). */
#define HESP_ORDER_PL 0
#define HESP_ORDER_FCFS 1
#define HESP_SELECT_EFT 0
#define HESP_SELECT_EIT 1
#define HESP_SELECT_RP 2
#define HESP_SELECT_FP 3
#define HESP_CACHE_WB 0
#define HESP_CACHE_WT 1
#define HESP_CACHE_WA 2
typedef struct {
  int32_t order, select, cache;
  uint64_t seed;               /* R-P draws */
  int32_t bus;                 /* 0 or 1: transfers contend on their links */
} hesp_policy;

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
 * fall below split_thr (P(split) = split_thr / 2^21), capped at dmax; past the
 * third, the chunks of the value drawn with purpose 6 for the same index
 * continue the count (depths 4 and 5). */
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
  int32_t slots;               /* persistent single-wave workgroups of the simulation; 0 = 32 per compute unit */
  int64_t max_tasks;           /* optional per-candidate task limit (larger: HESP_ECAPACITY); 0 = none */
  int64_t max_edges;           /* optional per-candidate edge limit; 0 = none */
  int32_t chunks;              /* split every batch into at least this many chunks; the preparation of
                                  chunk i+1 then runs on a second stream while chunk i is simulated
                                  (two workspace sets); 0 or 1 = as few chunks as memory allows */
  int32_t group;               /* lanes per candidate in the event simulation: 16, 32 or 64 (>= processors);
                                  0 = chosen per batch shape by timing each size once (autotuning) */
  int32_t prep_edges;          /* critical-time pass: dependences inside one run of 64 consecutive tasks kept
                                  in LDS, 1..1024 (0 = 1024); a run with more re-reads its successor lists
                                  on every sweep (same results, slower) */
  int32_t fuse;                /* 1: fused pipeline for depth batches (64 lanes per candidate; group must be
                                  0 or 64): every wave of the persistent event loop prepares the candidates it
                                  takes into its own workspace slot, so a batch of any size and unevenness is
                                  one launch holding (resident waves x largest candidate) bytes, four
                                  waves per SIMD; about as fast as the default separate preparation launch
                                  per memory chunk on uniform batches.  2: the same with
                                  each slot in the workgroup's LDS (no device workspace at all): candidates
                                  whose workspace (104 T + 4 E + 8 V + 4 (tet(nt) + 1) bytes, T tasks, E
                                  edges, V finest blocks x memory spaces) exceeds 48 KiB get HESP_ECAPACITY */
} hesp_plan_opts;
/* A plan with max_tasks and max_edges set is a fixed-capacity plan: its
 * workspace follows from the capacities and the batch shape, so after one call
 * with a batch of a given (n_cand, nt, dmax) further calls of that shape do no
 * host synchronisation, no allocation and no autotuning (group 0: the first call
 * of a shape times 16, 32 and 64 lanes per candidate and the plan keeps the
 * choice) -- only kernel launches on `stream`, which can be captured in a HIP
 * graph and replayed (the graph keeps the batch and output pointers of the
 * captured call).  A captured group-0 call whose shape the plan has not seen
 * gives HESP_EUNSUPPORTED.  A captured
 * call runs its memory chunks one after the other on `stream` alone; a fused
 * fixed-capacity plan captures any batch as one simulation launch.  Candidates
 * above the capacities get HESP_ECAPACITY. */
int hesp_plan_create(hesp_plan **plan, const hesp_plan_opts *opts);
int hesp_plan_destroy(hesp_plan *plan);
/* device bytes currently held by the plan */
int hesp_plan_bytes(const hesp_plan *plan, int64_t *bytes);
/* Kernel timing: with `enable` set, the next hesp_simulate_batch calls record HIP
 * events around every preparation and simulation launch on their stream;
 * hesp_plan_last_ms waits for those events and returns, for the last call, the
 * summed milliseconds of the preparation launches, of the simulation launches,
 * and the number of simulation launches (ms[0], ms[1], ms[2]). */
int hesp_plan_timing(hesp_plan *plan, int32_t enable);
int hesp_plan_last_ms(hesp_plan *plan, double *ms);

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
 * counts back to the host (one synchronisation of `stream`).
 * Depths: up to HESP_MAX_LEVEL (block sides down to b/32, the deepest DAGs of
 * section 3).  A batch whose dmax (its maximum) is above 3, or a platform whose
 * max_level is, takes the unfused pipeline (else HESP_EUNSUPPORTED).  A ragged candidate above the batch's nt or dmax
 * gets HESP_EINVAL.  A platform with max_level above 3 has more transfer times
 * than the kernels take by value: the plan keeps a device copy of xfer_ns (made
 * on `stream`, after it drains, whenever the table differs from the last one);
 * a captured call needs that copy to exist already (else HESP_EUNSUPPORTED). */
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

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): hesp_simulate_batch of
 * a depth batch with no plan.  Every buffer beyond the caller's inputs and
 * outputs lies in one fixed device array of HESP_NOALLOC_BYTES bytes that the
 * library holds on each device it runs on until the process ends; the call
 * allocates nothing, reads nothing back and only enqueues kernels on `stream`.
 * Outputs and statuses are those of hesp_simulate_batch (same makespans and
 * schedules).  Limits: n_cand <= HESP_NOALLOC_MAX_CAND (else HESP_EINVAL before
 * anything is enqueued); the candidates' workspaces are laid out in candidate
 * order, region_bytes = 104 T + 4 E + 8 V + 4 (tet(nt) + 1) bytes each (T
 * tasks, E edges, V = finest blocks x memory spaces, rounded up to 16), and a
 * candidate whose workspace would end past HESP_NOALLOC_REGION bytes gets
 * HESP_ECAPACITY (makespan -1), as do all candidates after it.  group: lanes
 * per candidate (16, 32, 64, at least n_procs), 0 = the smallest that fits.
 * Platforms with max_level above 3, finite spaces, and depths above 3 in
 * 64-lane groups give HESP_EUNSUPPORTED.
 * All calls on one device share the array: calls that overlap in time on one
 * device (different streams or host threads) race and give wrong results. */
#define HESP_NOALLOC_BYTES (64 << 20)
#define HESP_NOALLOC_MAX_CAND 16384
#define HESP_NOALLOC_REGION 66189824   /* the part holding candidate workspaces */
int hesp_simulate_batch_noalloc(const hesp_platform *pf, hesp_policy policy, const hesp_batch *batch,
                                const hesp_outputs *out, int32_t group, void *stream);

/* ---- split-tree candidates ---------------------------------------------------
 * Section 2.1 ("Recursive task partitioners") applies a partition to any task,
 * so sub-tasks of one top-level task may end at different depths.  A split-tree
 * candidate holds one flag (0 or 1) per task of each uniform level-l tiling
 * (nt 2^l tiles per dimension, Fig. 1 order), levels 0 .. dmax-1 concatenated:
 * hesp_tree_flag_count(nt, dmax) = sum over l < dmax of tet(nt 2^l) bytes.  A
 * level-l task exists when all its ancestors are split; it is split itself when
 * its flag is 1 (flags of tasks that do not exist are ignored): it is replaced,
 * in place, by the blocked algorithm of its kind on the 2 x 2 sub-tiling of its
 * cell.  Flags that split every task under a top-level task to depth d give the
 * depth-d candidate of hesp_simulate_batch (same tasks, same schedule).  The
 * batch has one shape: d_flags (device) holds n_cand x flag_count bytes.
 * Schedule outputs number the tasks in program order: top-level tasks in Fig. 1
 * order, each split task replaced in place by its children in the order of the
 * Fig. 1 loop nest restricted to its 2 x 2 sub-tiling, recursively.
 * hesp_simulate_tree_batch behaves as hesp_simulate_batch (outputs, statuses,
 * fixed-capacity plans; HESP_EINVAL for a flag above 1); it also keeps a
 * last-writer table of 4 bytes per finest block and candidate in the plan.
 * hesp_count_tree_batch gives the exact task and edge counts (it allocates and
 * frees device workspace and synchronises `stream`).
 * hesp_generate_tree_uniform: flag x of candidate first + c is 1 when the
 * leading 21 bits of the SplitMix64 value draw(seed, 5, (first + c) << 32 | x)
 * fall below split_thr. */
typedef struct {
  int32_t n_cand;
  int32_t nt, dmax;
  const uint8_t *d_flags;
} hesp_tree_batch;
int64_t hesp_tree_flag_count(int32_t nt, int32_t dmax);   /* -1 for a bad shape */
int hesp_generate_tree_uniform(uint64_t seed, int64_t first, int32_t n_cand, int32_t nt, int32_t dmax,
                               uint32_t split_thr, uint8_t *d_flags, void *stream);
int hesp_count_tree_batch(const hesp_tree_batch *batch, int32_t *d_n_tasks, int64_t *d_n_edges, void *stream);
int hesp_simulate_tree_batch(hesp_plan *plan, const hesp_platform *pf, hesp_policy policy,
                             const hesp_tree_batch *batch, const hesp_outputs *out, void *stream);

/* ---- batch reduction -------------------------------------------------------
 * Best candidate of a batch: the smallest makespan, ties to the lowest index
 * (section 2.1, "Iterative solver": the partition that best fits the platform).
 * Negative makespans (failed candidates) are ignored.  d_best gets
 * {makespan, index}, or {-1, -1} when no candidate succeeded. */
int hesp_argmin(const int64_t *d_makespan, int32_t n, int64_t *d_best, void *stream);

/* ---- learned surrogate ----------------------------------------------------
 * Not part of the paper's method: a small network that predicts a candidate's
 * normalised log-makespan from its split depths and the platform's rates, so
 * that only the best-scored proposals are simulated exactly (the exact
 * simulation above decides).  Network: 32 inputs -> 256 -> 256 -> 256
 * -> 1, ReLU; weights and activations bf16 (round to nearest even) wherever they
 * enter a product, fp32 accumulation on the MFMA units, fp32 biases, fp32
 * master weights updated by Adam (Kingma and Ba 2015; beta1 0.9, beta2 0.999,
 * eps 1e-8); loss = mean squared error.  Flat parameter layout (floats):
 * W1 [32][256], b1 [256], W2 [256][256], b2, W3 [256][256], b3, w4 [256], b4 [1]. */
typedef struct hesp_mlp hesp_mlp;
int64_t hesp_mlp_param_count(void);
/* He-uniform weights from SplitMix64 draws of `seed`, zero biases */
int hesp_mlp_create(hesp_mlp **mlp, uint64_t seed);
int hesp_mlp_destroy(hesp_mlp *mlp);
/* host float arrays of hesp_mlp_param_count() entries; set resets Adam */
int hesp_mlp_set_params(hesp_mlp *mlp, const float *params, int64_t n);
int hesp_mlp_get_params(hesp_mlp *mlp, float *params, int64_t n);
int hesp_mlp_get_grads(hesp_mlp *mlp, float *grads, int64_t n);
/* d_x [n][32] bf16 bit patterns: split depths of the n_top top-level tasks,
 * then the n_rate values of d_rate, then zeros (n_top + n_rate <= 32) */
int hesp_mlp_features(const uint8_t *d_depth, int64_t n, int32_t n_top, const float *d_rate, int32_t n_rate,
                      uint16_t *d_x, void *stream);
/* d_t[i] = (ln(d_makespan[i]) - mu) / sigma */
int hesp_mlp_targets(const int64_t *d_makespan, int64_t n, float mu, float sigma, float *d_t, void *stream);
/* d_y[i] = network output for row i of d_x (any n) */
int hesp_mlp_forward(hesp_mlp *mlp, const uint16_t *d_x, int64_t n, float *d_y, void *stream);
/* gradients of the mean squared error over `batch` rows (a multiple of 512) into
 * the network's gradient buffer; d_loss (device float, nullable) gets the loss */
int hesp_mlp_grad(hesp_mlp *mlp, const uint16_t *d_x, const float *d_t, int32_t batch, float *d_loss, void *stream);
/* one Adam step with the current gradients */
int hesp_mlp_adam(hesp_mlp *mlp, float lr, void *stream);
/* `steps` (gradient, Adam) steps, each on `batch` rows (a multiple of 512) of the
 * n rows of d_x/d_t drawn with replacement: row r of step s is row
 * draw(seed, 7, s << 32 | r) mod n, s counting the network's Adam steps so far.
 * d_loss [steps] (nullable) gets each step's loss. */
int hesp_mlp_train(hesp_mlp *mlp, const uint16_t *d_x, const float *d_t, int64_t n, int32_t batch, int32_t steps,
                   float lr, uint64_t seed, float *d_loss, void *stream);
/* Rate features of a platform (host): out[4*p + kind] = log2(rmax_mflops / 131072) / 4
 * for processor type p and task kind (chol, trsm, syrk, gemm); n_out >= 4 * n_ptypes. */
int hesp_mlp_rate_features(const hesp_cost_model *cm, float *out, int32_t n_out);
/* Features of candidates with more top-level tasks than inputs: for each kind the
 * fraction of its top-level tasks at depth 0, 1, 2 and 3 or more (16 values,
 * kind-major), for
 * each kind and each half of the k range (k < nt/2, k >= nt/2) the mean depth (8
 * values), then the n_rate (<= 8) values of d_rate.  d_depth [n][tet(nt)].
 * Synchronises `stream` (a small table of the top-level tasks is uploaded). */
int hesp_mlp_features_agg(const uint8_t *d_depth, int64_t n, int32_t nt, const float *d_rate, int32_t n_rate,
                          uint16_t *d_x, void *stream);

/* ---- candidate enumeration and top-k ----------------------------------------
 * Enumeration: the depth of top-level task t of candidate c is digit t (least
 * significant first) of first + c in base dmax + 1, so the candidates
 * 0 .. (dmax+1)^tet(nt) - 1 are every partition of the instance once. */
int hesp_generate_enumerate(int64_t first, int32_t n_cand, int32_t nt, int32_t dmax, uint8_t *d_depth, void *stream);
/* Top-k: d_idx[0..k) gets the indices of the k smallest values in increasing
 * order, ties to the lower index (bitonic sort of (value, index) keys on the
 * GPU).  Makespans: negative values (failed candidates) and values >= 2^40 rank
 * last; scores: NaN ranks last.  n <= 2^24.  d_ws: caller-owned device
 * workspace of hesp_topk_workspace_bytes(n) bytes. */
int64_t hesp_topk_workspace_bytes(int64_t n);
int hesp_topk_makespan(const int64_t *d_makespan, int32_t n, int32_t k, int32_t *d_idx, void *d_ws, int64_t ws_bytes,
                       void *stream);
int hesp_topk_score(const float *d_score, int32_t n, int32_t k, int32_t *d_idx, void *d_ws, int64_t ws_bytes,
                    void *stream);

/* ---- partition search --------------------------------------------------------
 * Rounds of proposals evaluated by the exact batched simulation (the iterative
 * solver of section 2.1 keeps the partition with the best simulated makespan).
 *   RANDOM:    every round draws `batch` fresh candidates (hesp_generate_uniform).
 *   GREEDY:    after `warm_rounds` random rounds of `warm_batch` candidates, each
 *              round mutates incumbents: proposal c copies incumbent
 *              parent(c) = draw(seed, 5, round << 32 | c) mod pool_size and redraws
 *              the depth of each top-level task with probability mutate_thr / 2^21
 *              (SplitMix64 stream of draw(seed, 6, round << 32 | c)).
 *   SURROGATE: as GREEDY, but `proposals` mutations per round are scored by the
 *              network and only the `batch` best-scored are simulated; the network
 *              is trained online, each round by hesp_mlp_train (train_steps steps
 *              of train_batch rows drawn from every exact result kept in a ring of
 *              `replay` rows), with targets normalised by the warm-up rounds' log-makespans.  Features:
 *              raw depths when tet(nt) + n_rate <= 32, else the aggregate features
 *              of hesp_mlp_features_agg.
 * The incumbents are the `pool` best distinct-index results so far.  best_depth
 * (host, tet(nt) bytes) and best_makespan (host) get the best partition;
 * trace[rounds] (host, nullable) gets, after each round, the wall time since the
 * start, the best makespan, and the simulated and proposed candidate counts
 * (each round synchronises `stream`).  Device workspace is allocated per call.
 * The search takes dmax <= HESP_MAX_LEVEL (the aggregate features count depths
 * 3 to 5 in one bin).
 * The plan must not limit tasks or edges per candidate (HESP_EINVAL), so that
 * every proposal gets a makespan. */
enum { HESP_SEARCH_RANDOM = 0, HESP_SEARCH_GREEDY = 1, HESP_SEARCH_SURROGATE = 2 };
typedef struct {
  int32_t mode;
  int32_t nt, dmax;            /* instance: nt x nt tiles, split depths 0..dmax */
  int32_t rounds;
  int32_t batch;               /* exact simulations per round after the warm-up */
  int32_t warm_rounds;         /* >= 1 rounds of random candidates */
  int32_t warm_batch;
  int32_t proposals;           /* SURROGATE: proposals scored per round (>= batch) */
  int32_t pool;                /* incumbents kept */
  uint32_t split_thr;          /* random candidates, as in hesp_generate_uniform */
  uint32_t mutate_thr;         /* per-task redraw probability * 2^21 */
  uint64_t seed;
  hesp_mlp *mlp;               /* SURROGATE: the network, trained in place */
  const float *d_rate;         /* SURROGATE: platform rate features (device) */
  int32_t n_rate;
  int32_t train_steps;
  int32_t train_batch;         /* multiple of 512 */
  float lr;
  int64_t replay;              /* rows of training data kept (>= train_batch) */
} hesp_search_params;
typedef struct {
  double wall_ms;
  int64_t best_makespan;
  int64_t simulated;
  int64_t proposed;
} hesp_trace_point;
int hesp_search(hesp_plan *plan, const hesp_platform *pf, hesp_policy policy, const hesp_search_params *params,
                uint8_t *best_depth, int64_t *best_makespan, hesp_trace_point *trace, void *stream);

/* ---- iterative scheduler-partitioner (section 2.1, "Iterative solver") -------
 * n_chains independent runs, each alternating a schedule stage (the exact
 * simulation of its current partition, as hesp_simulate_batch) and a partition
 * stage that changes the split depth of one cluster (top-level task t and the
 * fine tasks it was split into).  The paper leaves the score open; this reading
 * is exact integer arithmetic on the stage's schedule:
 *   span(t) = latest finish - earliest start t0 over the cluster's tasks;
 *   ptype   = type of the processor of the cluster's earliest task (lowest
 *             processor index on ties);
 *   avail   = n_procs - (tasks with start <= t0 < finish) + 1;
 *   for every other depth d' in 0..dmax: work = sum of the task times on ptype of
 *   the cluster's tasks at depth d', width = max(1, their count >> d'),
 *   estimate = ceil(work / min(avail, width)), score = span - estimate.
 * A cluster proposes its best-scoring other depth (the smallest on ties) when
 * that score is positive (a smaller depth merges it back, a larger one splits
 * it).  Candidate clusters: ALL; CP, those with a task on the critical path (from
 * the last-finishing task, repeatedly the DAG predecessor that finished last;
 * ties to the lowest processor index); SHALLOW, those of the smallest depth
 * present.  HARD takes the largest score (smallest cluster index on ties); SOFT
 * draws u = SplitMix64 draw(seed + r, 10, iteration) mod (sum of scores) for
 * chain r and takes the first candidate, in cluster order, whose running score
 * sum exceeds u.  Without a candidate the partition stays (a fixed point).
 * d_depth [n_chains][tet(nt)] (device) holds the initial partitions and gets the
 * last ones; d_best_depth / d_best_makespan get each chain's best simulated
 * partition (earliest on ties); d_trace [n_chains][iters] (nullable) every
 * iteration's makespan; d_steps [n_chains][iters][3] (nullable) the change made
 * (cluster, new depth, score; cluster -1 when none).  A chain whose simulation
 * fails (a depth above dmax, or above a fixed-capacity plan) gets -1 in its
 * trace and keeps makespan -1 if it never succeeded.  Limits: tet(nt) <= 4096,
 * n_procs <= 64, dmax and platform max_level <= HESP_MAX_LEVEL.  Device
 * workspace is allocated per call (n_chains x tet(nt 2^dmax) tasks); the call
 * synchronises `stream` before it returns. */
#define HESP_LIST_ALL 0
#define HESP_LIST_CP 1
#define HESP_LIST_SHALLOW 2
#define HESP_SAMPLE_HARD 0
#define HESP_SAMPLE_SOFT 1
typedef struct {
  int32_t n_chains;
  int32_t nt, dmax;
  int32_t iters;
  int32_t list;                /* HESP_LIST_* */
  int32_t sampling;            /* HESP_SAMPLE_* */
  uint64_t seed;
} hesp_solve_params;
int hesp_solve(hesp_plan *plan, const hesp_platform *pf, hesp_policy policy, const hesp_solve_params *params,
               uint8_t *d_depth, uint8_t *d_best_depth, int64_t *d_best_makespan, int64_t *d_trace,
               int64_t *d_steps, void *stream);

/* The same solver on split-tree partitions (section 2.1: every task cluster,
 * nested ones included, may be merged back or repartitioned; Shallow takes the
 * tasks of minimal depth).  The clusters ("nodes") are the existing tasks of the
 * levels below dmax, node x being split flag x (hesp_tree_batch encoding):
 *   an internal node (flag 1) proposes to merge back into its own task:
 *     estimate = that task's time on the node's processor type;
 *   a leaf node (flag 0) proposes one more split: estimate = ceil(work of its
 *     2 x 2 blocked algorithm / min(avail, max(1, its task count >> 1)));
 *   span, processor type and avail from the node's tasks as above; the score is
 *   span - estimate; ALL: existing nodes; CP: those holding a task of the
 *   critical path; SHALLOW: leaf nodes at the smallest level of any task;
 *   HARD / SOFT over node order with the same draw as hesp_solve.
 * A split sets the node's flag and clears its children's (they start as
 * leaves); a merge clears the node's flag.  With dmax = 1 this is hesp_solve
 * (except SHALLOW once every cluster is split).  d_flags [n_chains][flag_count]
 * (device) holds the initial partitions and gets the last ones; d_steps gets
 * (node, 1 split / 0 merge, score), node -1 when none.  Limits: 1 <= dmax,
 * flag_count <= 4096 (nt <= 13 at dmax 2, nt <= 6 at dmax 3). */
int hesp_solve_tree(hesp_plan *plan, const hesp_platform *pf, hesp_policy policy, const hesp_solve_params *params,
                    uint8_t *d_flags, uint8_t *d_best_flags, int64_t *d_best_makespan, int64_t *d_trace,
                    int64_t *d_steps, void *stream);

/* ---- grain batches ----------------------------------------------------------
 * Section 2.1 ("Iterative solver"): a partitioned task's new tasks work on
 * blocks of size p times the original one, p in (0,1].  Here p = 1/f for any
 * integer f: top-level task t of candidate c is replaced by the blocked algorithm
 * of its kind on the f x f sub-tiling of its cell, f = fac[grain[c * tet(nt) + t]]
 * (right-looking order, fine tasks numbered top-level task by top-level task).
 * Factors that do not divide each other give blocks that overlap partially
 * (section 2.1 data DAG, Fig. 4: such an overlap gets an intersection descriptor,
 * a common child of both blocks).  Reading: every tile is cut into L x L atoms,
 * L = lcm(fac); a block of factor f is the union of its (L/f)^2 atoms, an
 * intersection is the set of atoms two blocks share, and validity, dependences
 * (the last writer of every atom a task touches) and transfers (the atoms
 * missing in the target space, one transfer per block) are kept per atom.  The
 * heuristics are those of hesp_policy, keyed by the task's first atom (K', I',
 * J') = (K, I, J) * L / f.  Power-of-two factors 1, 2, .., 2^d give exactly the
 * depth batch of dmax = d.
 * Limits: 1..HESP_GRAIN_MAX_FAC factors, each 1..HESP_GRAIN_MAX_ATOMS with
 * L <= HESP_GRAIN_MAX_ATOMS and nt * L <= HESP_MAX_FINE; n_mem <= HESP_GRAIN_MAX_MEM;
 * Priority-List or FCFS, EFT-P or EIT-P, any caching, bus = 0 and unbounded
 * spaces (else HESP_EUNSUPPORTED). */
#define HESP_GRAIN_MAX_FAC 8
#define HESP_GRAIN_MAX_ATOMS 64
#define HESP_GRAIN_MAX_MEM 8
typedef struct {
  int32_t n_cand, nt;
  int32_t n_fac;
  const int32_t *fac;          /* host [n_fac]: blocks per tile side of each grain */
  const uint8_t *grain;        /* device [n_cand][tet(nt)]: grain index (< n_fac) per top-level task */
} hesp_grain_batch;

/* Tables of the cost model of hesp_cost_tables for a grain batch: cost_ns (host
 * [n_ptypes][4][n_fac]) for tasks of side b / fac[g], and xfer_ns (host
 * [L*L + 1]) for k atoms of side b / L, both from the exact rational values
 * rounded up once (sides need not be integers; cm->max_level is ignored). */
int hesp_grain_cost_tables(const hesp_cost_model *cm, int32_t n_fac, const int32_t *fac, int64_t *cost_ns,
                           int64_t *xfer_ns);

/* Device workspace, in bytes, of hesp_simulate_grain_batch for this batch shape
 * (gb->grain and gb->n_cand are not read), n_mem memory spaces and `slots`
 * candidates in flight (one wavefront each). */
int hesp_grain_workspace(const hesp_grain_batch *gb, int32_t n_mem, int32_t slots, int64_t *bytes);

/* Simulates every candidate of a grain batch on `stream`: d_makespan [n_cand]
 * (device, -1 for a failed candidate; may be NULL with d_ws when n_cand = 0),
 * optional d_n_tasks [n_cand], d_n_edges
 * [n_cand] (expanded tasks and dependence edges) and d_status [n_cand]
 * (HESP_OK, or HESP_EINVAL for a grain index >= n_fac).  pf->cost_ns and
 * pf->xfer_ns as filled by hesp_grain_cost_tables (pf->max_level = n_fac - 1;
 * pf->capacity and pf->link unused), all task times >= 1.  d_ws holds at least
 * hesp_grain_workspace(gb, pf->n_mem, slots) bytes owned by the caller; the
 * host tables (pf, gb->fac) are read before the call returns, the device work
 * is asynchronous on `stream`, and the workspace, grain and outputs must stay
 * allocated until the stream has run it; calls sharing a workspace must not
 * overlap (the transfer table is staged at its start). */
int hesp_simulate_grain_batch(const hesp_platform *pf, hesp_policy policy, const hesp_grain_batch *gb,
                              int64_t *d_makespan, int32_t *d_n_tasks, int64_t *d_n_edges, int32_t *d_status,
                              void *d_ws, int64_t ws_bytes, int32_t slots, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HESP_H_ */
