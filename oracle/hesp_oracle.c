/*
 * hesp_oracle.c -- plain, slow, obviously-correct CPU oracle for the HeSP
 * scheduling-partitioning simulation (Rey, Igual, Prieto-Matias,
 * "HeSP: a simulation framework for solving the task scheduling-partitioning
 * problem on heterogeneous architectures", arXiv 1602.05510).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file.  It shares no code,
 * header or table with the HIP path and must never be used to produce a
 * product result.
 *
 * What it computes, step by step, in the paper's order:
 *   1. cost model (section 2.1, "Performance and data transfer models"):
 *      task time = ceil(flops / R(b)) ns with R(b) = Rmax b^2/(b^2+h^2);
 *      transfer time of k atoms = latency + ceil(bytes / bandwidth) ns;
 *   2. expansion (Fig. 1 loop nest; section 2.1 "Recursive task
 *      partitioners"): every top-level task of Fig. 1 is replaced by the
 *      blocked algorithm of its own kind on a 2^d x 2^d sub-tiling, emitted in
 *      right-looking loop order -- or, for a grain batch (partition parameter
 *      p = 1/f with any integer f, section 2.1 "Iterative solver"), on an
 *      f x f sub-tiling, so that blocks of different tasks may overlap
 *      partially (Fig. 4: intersection blocks of the data DAG);
 *   3. dependences (section 2.1, RaW/WaR/WaW): a sequential scan over the
 *      finest data atoms, last writer -> later reader/writer and
 *      readers-since-last-write -> next writer;
 *   4. critical times (section 2.1, "Priority-List"): sum of the task's time
 *      over all processors (an order-preserving multiple of the average),
 *      propagated backwards over the DAG;
 *   5. event simulation with write-back, write-through or write-around
 *      caching of host data in accelerator spaces and transfers issued when a
 *      task is scheduled (section 2.1,
 *      "Task and data scheduling heuristics"); task order Priority-List
 *      (decreasing critical time) or FCFS (order of release), processor
 *      selection EFT-P (earliest finish counting transfers), EIT-P (the
 *      processor that becomes idle first), R-P (random) or F-P (fastest) --
 *      the last two among the processors idle at that time; a task finding no
 *      idle processor waits for the next completion; optionally every transfer
 *      shares one interconnect (one at a time, in issue order);
 *   6. optionally, finite accelerator memory spaces (section 2, problem input:
 *      "finite-size memory spaces"; the spaces cache the host): a space holds
 *      at most its capacity of finest blocks, a task may go only to a processor
 *      whose space can hold the blocks of the tasks mapped there and not yet
 *      finished plus its own, and blocks are evicted least recently used first,
 *      a block with no valid host copy being copied back to the host first
 *      (readings marked "reading (capacity)" below).
 * Where the paper is silent (tie-breaks, simultaneous events, transfer issue
 * time, coherence granularity) the readings are those listed in the design
 * notes of this repository; each is marked "reading:" below.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_INF INT64_MAX

enum { OR_CHOL = 0, OR_TRSM = 1, OR_SYRK = 2, OR_GEMM = 3 };

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_ECAP = -4 };

/* ------------------------------------------------------------------------ */
/* 1. cost model                                                             */

/* flops of one task of side bl, times 3 (chol b^3/3, trsm b^3, syrk b^3, gemm 2b^3) */
static int64_t flops_times3(int type, int64_t bl)
{
    static const int64_t c[4] = {1, 3, 3, 6};
    return c[type] * bl * bl * bl;
}

static int64_t ceil_div_pos(int64_t a, int64_t b) { return a / b + (a % b != 0); }

/*
 * task time in ns = flops / R, R in flop/ns = GFLOP/s = Rmax_mflops/1000 * bl^2/(bl^2+h^2)
 *   = (flops3/3) * 1000 * (bl^2+h^2) / (Rmax_mflops * bl^2)
 * computed as one exact rational and rounded up once (reading: every task time
 * and every transfer time is rounded up on its own, everything after is exact).
 */
int oracle_task_time(int type, int64_t bl, int64_t rmax_mflops, int64_t h, int64_t *out)
{
    if (type < 0 || type > 3 || bl <= 0 || rmax_mflops <= 0 || h < 0 || !out) return OR_EINVAL;
    int64_t f3 = flops_times3(type, bl);            /* 3 * flops */
    /* num/den = (f3/3) * 1000 * (bl^2 + h^2) / (rmax * bl^2); bl^2 divides f3 */
    int64_t num = (f3 / (bl * bl)) * 1000 * (bl * bl + h * h);
    int64_t den = 3 * rmax_mflops;
    *out = ceil_div_pos(num, den);
    return OR_OK;
}

int oracle_transfer_time(int64_t n_atoms, int64_t atom_side, int64_t elem_bytes,
                         int64_t latency_ns, int64_t bw_bytes_per_ns, int shared, int64_t *out)
{
    if (!out || n_atoms < 0 || atom_side <= 0 || bw_bytes_per_ns <= 0) return OR_EINVAL;
    if (shared || n_atoms == 0) { *out = 0; return OR_OK; }
    int64_t bytes = elem_bytes * n_atoms * atom_side * atom_side;
    *out = latency_ns + ceil_div_pos(bytes, bw_bytes_per_ns);
    return OR_OK;
}

/*
 * The same two models for a block side that need not be an integer (grain
 * batches): a task on a block of side b/f, and k atoms of side b/L.
 *   time = ceil(c 1000 b (b^2 + f^2 h^2) / (3 f^3 Rmax))  (c = 1, 3, 3, 6 as above)
 *   xfer = latency + ceil(elem_bytes k b^2 / (L^2 bw))
 * Both equal the integer forms above whenever b/f and b/L are integers.
 */
static int64_t ceil_div128(__int128 a, __int128 b) { return (int64_t)(a / b + (a % b != 0)); }

static int grain_task_time(int type, int64_t b, int64_t f, int64_t rmax_mflops, int64_t h, int64_t *out)
{
    if (type < 0 || type > 3 || b <= 0 || f <= 0 || rmax_mflops <= 0 || h < 0) return OR_EINVAL;
    __int128 num = (__int128)flops_times3(type, 1) * 1000 * b * ((__int128)b * b + (__int128)f * f * h * h);
    __int128 den = (__int128)3 * f * f * f * rmax_mflops;
    *out = ceil_div128(num, den);
    return OR_OK;
}

static int grain_transfer_time(int64_t n_atoms, int64_t b, int64_t L, int64_t elem_bytes,
                               int64_t latency_ns, int64_t bw, int shared, int64_t *out)
{
    if (n_atoms < 0 || b <= 0 || L <= 0 || bw <= 0) return OR_EINVAL;
    if (shared || n_atoms == 0) { *out = 0; return OR_OK; }
    *out = latency_ns + ceil_div128((__int128)elem_bytes * n_atoms * b * b, (__int128)L * L * bw);
    return OR_OK;
}

/* Atom grid of a candidate: every tile is cut into L x L atoms, and a block of
 * grain index g (fac[g] blocks per tile side) covers (L/fac[g])^2 of them.  A
 * depth candidate has L = 2^dmax and fac[l] = 2^l; a grain batch has
 * L = lcm(fac), so the blocks of two grains are unions of common atoms and
 * their intersections (the intersection descriptors of the data DAG, Fig. 4)
 * need no node of their own. */
typedef struct { int L, n, pow2; int fac[8]; } or_grid;

static int grid_w(const or_grid *gr, int level) { return gr->L / gr->fac[level]; }

typedef struct {
    int n_procs, n_mem, n_ptypes;
    const int32_t *proc_type, *proc_mem;
    const int64_t *rmax;     /* [n_ptypes][4] MFLOP/s */
    const int64_t *h;        /* [n_ptypes] */
    int64_t b;               /* tile side at level 0 */
    int64_t latency_ns, bw, elem_bytes;
    int shared;              /* single memory space, transfers cost 0 */
    int order;               /* policy: 0 = Priority-List, 1 = FCFS */
    int select;              /* policy: 0 = EFT-P, 1 = EIT-P, 2 = R-P, 3 = F-P */
    uint64_t seed;           /* R-P draws */
    int cache;               /* policy: 0 = write-back, 1 = write-through, 2 = write-around */
    int bus;                 /* 1: transfers contend, one at a time on each link */
    const int32_t *link;     /* [n_mem] link carrying the transfers into each space, or
                                NULL: one link for every space (a shared interconnect) */
    const int64_t *capacity; /* [n_mem] bytes each accelerator space holds, or NULL;
                                <= 0 (and always for the host, space 0): unbounded */
} or_platform;

/* SplitMix64 (Steele, Lea, Flood 2014): value number idx+1 of the sequence
 * that starts at mix(seed + gamma (purpose+1)); used for the R-P choice. */
static uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t sm_draw(uint64_t seed, uint64_t purpose, uint64_t idx)
{
    const uint64_t g = 0x9E3779B97F4A7C15ull;
    return sm_mix(sm_mix(seed + g * (purpose + 1)) + g * (idx + 1));
}

/* ------------------------------------------------------------------------ */
/* 2. expansion                                                              */

typedef struct {
    int type, level, K, I, J;   /* fine loop indices at `level` (upper storage, K<=I<=J) */
    int top;                    /* index of the Fig. 1 task it comes from */
} or_task;

typedef struct { or_task *v; int n, cap; } or_tasklist;

static int tl_push(or_tasklist *l, or_task t)
{
    if (l->n == l->cap) {
        int nc = l->cap ? 2 * l->cap : 256;
        or_task *nv = (or_task *)realloc(l->v, (size_t)nc * sizeof(or_task));
        if (!nv) return OR_ENOMEM;
        l->v = nv; l->cap = nc;
    }
    l->v[l->n++] = t;
    return OR_OK;
}

static int in_range(int x, int lo, int s) { return x >= lo && x < lo + s; }

/*
 * The Fig. 1 loop nest over the fine index space, restricted to the cell of one
 * top-level task (its k, i, j ranges at granularity 2^d).  This emits exactly
 * the fine tasks whose (K,I,J) fall in the cell, in right-looking order.
 */
static int emit_cell(or_tasklist *l, int top, int d, int s, int k, int i, int j)
{
    int ks = k * s, is = i * s, js = j * s;
    for (int K = ks; K < ks + s; K++) {
        if (in_range(K, is, s) && in_range(K, js, s))
            if (tl_push(l, (or_task){OR_CHOL, d, K, K, K, top})) return OR_ENOMEM;
        if (in_range(K, is, s))
            for (int J = K + 1; J < js + s; J++)
                if (in_range(J, js, s))
                    if (tl_push(l, (or_task){OR_TRSM, d, K, K, J, top})) return OR_ENOMEM;
        for (int I = K + 1; I < is + s; I++) {
            if (!in_range(I, is, s)) continue;
            for (int J = I + 1; J < js + s; J++)
                if (in_range(J, js, s))
                    if (tl_push(l, (or_task){OR_GEMM, d, K, I, J, top})) return OR_ENOMEM;
            if (in_range(I, js, s))
                if (tl_push(l, (or_task){OR_SYRK, d, K, I, I, top})) return OR_ENOMEM;
        }
    }
    return OR_OK;
}

/* Fig. 1: top-level tasks in program order, each expanded in place on the
 * fac[depth[t]] x fac[depth[t]] sub-tiling of its cell */
static int expand(int nt, const uint8_t *depth, const or_grid *gr, or_tasklist *out)
{
    int top = 0;
    for (int k = 0; k < nt; k++) {
        if (emit_cell(out, top, depth[top], gr->fac[depth[top]], k, k, k)) return OR_ENOMEM;
        top++;
        for (int j = k + 1; j < nt; j++) {
            if (emit_cell(out, top, depth[top], gr->fac[depth[top]], k, k, j)) return OR_ENOMEM;
            top++;
        }
        for (int i = k + 1; i < nt; i++) {
            for (int j = i + 1; j < nt; j++) {
                if (emit_cell(out, top, depth[top], gr->fac[depth[top]], k, i, j)) return OR_ENOMEM;
                top++;
            }
            if (emit_cell(out, top, depth[top], gr->fac[depth[top]], k, i, i)) return OR_ENOMEM;
            top++;
        }
    }
    return OR_OK;
}

/*
 * Recursive per-task splitting (section 2.1, "Recursive task partitioners": any
 * task, fine tasks included, may be partitioned again).  split[l] holds one flag
 * per task of the uniform level-l expansion (nt * 2^l tiles, Fig. 1 order); a
 * level-l task exists when all its ancestors were split, and it is split itself
 * when its flag is set and l < dmax.  A split task is replaced, in place, by the
 * blocked algorithm of its kind on the 2 x 2 sub-tiling of its cell.
 */
typedef struct {
    int nt, dmax;
    const uint8_t *flags;     /* concatenated levels 0 .. dmax-1 */
    int64_t off[8];           /* start of level l in flags */
    int *index[8];            /* Fig. 1 position of cell (K, I, J) at level l, N_l^3 entries */
} or_tree;

static int tree_init(or_tree *t, int nt, int dmax, const uint8_t *flags)
{
    memset(t, 0, sizeof(*t));
    t->nt = nt; t->dmax = dmax; t->flags = flags;
    int64_t off = 0;
    for (int l = 0; l < dmax; l++) {
        int N = nt << l;
        t->off[l] = off;
        t->index[l] = (int *)malloc((size_t)N * N * N * sizeof(int));
        if (!t->index[l]) return OR_ENOMEM;
        int pos = 0;                       /* Fig. 1 order on N tiles */
        for (int k = 0; k < N; k++) {
            t->index[l][((size_t)k * N + k) * N + k] = pos++;
            for (int j = k + 1; j < N; j++) t->index[l][((size_t)k * N + k) * N + j] = pos++;
            for (int i = k + 1; i < N; i++) {
                for (int j = i + 1; j < N; j++) t->index[l][((size_t)k * N + i) * N + j] = pos++;
                t->index[l][((size_t)k * N + i) * N + i] = pos++;
            }
        }
        off += pos;
    }
    return OR_OK;
}

static void tree_free(or_tree *t)
{
    for (int l = 0; l < 8; l++) free(t->index[l]);
}

static int emit_tree(or_tasklist *out, const or_tree *tr, int top, int type, int l, int K, int I, int J)
{
    int N = tr->nt << l;
    if (l < tr->dmax && tr->flags[tr->off[l] + tr->index[l][((size_t)K * N + I) * N + J]]) {
        or_tasklist kids = {0, 0, 0};
        if (emit_cell(&kids, top, 1, 2, K, I, J)) { free(kids.v); return OR_ENOMEM; }
        for (int c = 0; c < kids.n; c++)
            if (emit_tree(out, tr, top, kids.v[c].type, l + 1, kids.v[c].K, kids.v[c].I, kids.v[c].J)) {
                free(kids.v);
                return OR_ENOMEM;
            }
        free(kids.v);
        return OR_OK;
    }
    return tl_push(out, (or_task){type, l, K, I, J, top});
}

static int expand_tree(int nt, int dmax, const uint8_t *flags, or_tasklist *out)
{
    or_tree tr;
    int rc = tree_init(&tr, nt, dmax, flags);
    int top = 0;
    for (int k = 0; k < nt && !rc; k++) {
        rc = emit_tree(out, &tr, top++, OR_CHOL, 0, k, k, k);
        for (int j = k + 1; j < nt && !rc; j++) rc = emit_tree(out, &tr, top++, OR_TRSM, 0, k, k, j);
        for (int i = k + 1; i < nt && !rc; i++) {
            for (int j = i + 1; j < nt && !rc; j++) rc = emit_tree(out, &tr, top++, OR_GEMM, 0, k, i, j);
            if (!rc) rc = emit_tree(out, &tr, top++, OR_SYRK, 0, k, i, i);
        }
    }
    tree_free(&tr);
    return rc;
}

/* data blocks of a fine task: (row, col, written?) at the task's level */
static int task_blocks(const or_task *t, int br[3], int bc[3], int bw[3])
{
    switch (t->type) {
    case OR_CHOL: br[0] = t->K; bc[0] = t->K; bw[0] = 1; return 1;
    case OR_TRSM: br[0] = t->K; bc[0] = t->K; bw[0] = 0;
                  br[1] = t->K; bc[1] = t->J; bw[1] = 1; return 2;
    case OR_SYRK: br[0] = t->K; bc[0] = t->I; bw[0] = 0;
                  br[1] = t->I; bc[1] = t->I; bw[1] = 1; return 2;
    default:      br[0] = t->K; bc[0] = t->I; bw[0] = 0;
                  br[1] = t->K; bc[1] = t->J; bw[1] = 0;
                  br[2] = t->I; bc[2] = t->J; bw[2] = 1; return 3;
    }
}

/* ------------------------------------------------------------------------ */
/* 3. dependences by a sequential scan over atoms                            */

typedef struct { int64_t *v; int64_t n, cap; } or_i64list;

static int il_push(or_i64list *l, int64_t x)
{
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 16;
        int64_t *nv = (int64_t *)realloc(l->v, (size_t)nc * sizeof(int64_t));
        if (!nv) return OR_ENOMEM;
        l->v = nv; l->cap = nc;
    }
    l->v[l->n++] = x;
    return OR_OK;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/*
 * Atoms: the finest blocks (side b/L).  A block (R,C) of grain l is the set
 * of atoms (R*w+u, C*w+v), 0 <= u,v < w = L/fac[l] -- the whole square, also on
 * the diagonal (reading).  Atoms are numbered row-major on the full N x N grid,
 * N = nt * L.
 */
typedef struct {
    int n;                 /* tasks */
    int64_t n_edges;
    int64_t *edge;         /* sorted unique u*n+v */
    int *succ_ptr, *succ;  /* CSR of successors */
    int *npred;
} or_dag;

static void dag_free(or_dag *g)
{
    free(g->edge); free(g->succ_ptr); free(g->succ); free(g->npred);
    memset(g, 0, sizeof(*g));
}

static int build_dag(const or_tasklist *tl, int nt, const or_grid *gr, or_dag *g)
{
    int n = tl->n, N = nt * gr->L;
    int64_t n_atoms = (int64_t)N * N;
    int64_t *last_w = (int64_t *)malloc((size_t)n_atoms * sizeof(int64_t));
    or_i64list *readers = (or_i64list *)calloc((size_t)n_atoms, sizeof(or_i64list));
    or_i64list edges = {0, 0, 0};
    int rc = OR_OK;
    memset(g, 0, sizeof(*g));
    if (!last_w || !readers) { rc = OR_ENOMEM; goto done; }
    for (int64_t a = 0; a < n_atoms; a++) last_w[a] = -1;

    for (int t = 0; t < n; t++) {
        int br[3], bc[3], bw[3];
        int nb = task_blocks(&tl->v[t], br, bc, bw);
        int w = grid_w(gr, tl->v[t].level);
        for (int bi = 0; bi < nb; bi++) {
            for (int u = 0; u < w; u++) for (int v = 0; v < w; v++) {
                int64_t a = (int64_t)(br[bi] * w + u) * N + (bc[bi] * w + v);
                if (last_w[a] >= 0 && last_w[a] != t)
                    if (il_push(&edges, last_w[a] * n + t)) { rc = OR_ENOMEM; goto done; }
                if (bw[bi]) {           /* write: WaW above, WaR from readers */
                    for (int64_t r = 0; r < readers[a].n; r++)
                        if (readers[a].v[r] != t)
                            if (il_push(&edges, readers[a].v[r] * n + t)) { rc = OR_ENOMEM; goto done; }
                    readers[a].n = 0;
                    last_w[a] = t;
                } else {                /* read: RaW above */
                    if (il_push(&readers[a], t)) { rc = OR_ENOMEM; goto done; }
                }
            }
        }
    }
    /* deduplicate */
    if (edges.n) qsort(edges.v, (size_t)edges.n, sizeof(int64_t), cmp_i64);
    int64_t m = 0;
    for (int64_t e = 0; e < edges.n; e++)
        if (e == 0 || edges.v[e] != edges.v[e - 1]) edges.v[m++] = edges.v[e];
    g->n = n; g->n_edges = m; g->edge = edges.v; edges.v = NULL;
    g->succ_ptr = (int *)calloc((size_t)n + 1, sizeof(int));
    g->succ = (int *)malloc((size_t)(m ? m : 1) * sizeof(int));
    g->npred = (int *)calloc((size_t)n ? (size_t)n : 1, sizeof(int));
    if (!g->succ_ptr || !g->succ || !g->npred) { rc = OR_ENOMEM; goto done; }
    for (int64_t e = 0; e < m; e++) {
        g->succ_ptr[g->edge[e] / n + 1]++;
        g->npred[g->edge[e] % n]++;
    }
    for (int t = 0; t < n; t++) g->succ_ptr[t + 1] += g->succ_ptr[t];
    for (int64_t e = 0; e < m; e++) g->succ[e] = (int)(g->edge[e] % n); /* sorted by u then v */
done:
    free(last_w);
    if (readers) { for (int64_t a = 0; a < n_atoms; a++) free(readers[a].v); free(readers); }
    free(edges.v);
    if (rc) dag_free(g);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* 4-5. priorities and the event simulation                                  */

/* When the transfer of a block's missing atoms into space m can start: at the
 * mapping time T, or later if some missing atom has no copy valid yet (its
 * earliest valid-from over all spaces is still ahead, as for a host copy still
 * in flight after a write-around). */
static int64_t xfer_start(const int64_t *vf, int M, int64_t N, int R, int C, int w, int m, int64_t T)
{
    int64_t go = T;
    for (int u = 0; u < w; u++) for (int v = 0; v < w; v++) {
        int64_t a = (int64_t)(R * w + u) * N + (C * w + v);
        if (vf[a * M + m] != OR_INF) continue;
        int64_t src = OR_INF;
        for (int mm = 0; mm < M; mm++) if (vf[a * M + mm] < src) src = vf[a * M + mm];
        if (src != OR_INF && src > go) go = src;
    }
    return go;
}

typedef struct {
    int nt, dmax;
    int64_t *cost;   /* [n_ptypes][4][dmax+1] */
    int64_t *xfer;   /* [4^dmax + 1] */
} or_tables;

static int make_tables(const or_platform *pf, const or_grid *gr, or_tables *tb)
{
    int L = gr->n, dmax = gr->n - 1;
    int64_t na = (int64_t)gr->L * gr->L;
    tb->cost = (int64_t *)malloc((size_t)pf->n_ptypes * 4 * L * sizeof(int64_t));
    tb->xfer = (int64_t *)malloc((size_t)(na + 1) * sizeof(int64_t));
    if (!tb->cost || !tb->xfer) return OR_ENOMEM;
    for (int pt = 0; pt < pf->n_ptypes; pt++)
        for (int ty = 0; ty < 4; ty++)
            for (int l = 0; l < L; l++)
                if (gr->pow2 ? oracle_task_time(ty, pf->b >> l, pf->rmax[pt * 4 + ty], pf->h[pt],
                                                &tb->cost[(pt * 4 + ty) * L + l])
                             : grain_task_time(ty, pf->b, gr->fac[l], pf->rmax[pt * 4 + ty], pf->h[pt],
                                               &tb->cost[(pt * 4 + ty) * L + l])) return OR_EINVAL;
    for (int64_t k = 0; k <= na; k++)
        if (gr->pow2 ? oracle_transfer_time(k, pf->b >> dmax, pf->elem_bytes, pf->latency_ns, pf->bw,
                                            pf->shared, &tb->xfer[k])
                     : grain_transfer_time(k, pf->b, gr->L, pf->elem_bytes, pf->latency_ns, pf->bw,
                                           pf->shared, &tb->xfer[k])) return OR_EINVAL;
    return OR_OK;
}

static void free_tables(or_tables *tb) { free(tb->cost); free(tb->xfer); }

/* 6. finite accelerator spaces.
 * reading (capacity): the capacity of space m counts whole finest blocks of the
 * candidate, floor(bytes / (elem_bytes (b / 2^dmax)^2)); the host is unbounded.
 * A finest block takes a place in space m while it has a copy there, valid now
 * or arriving.  Among blocks used equally recently the one with the smaller
 * number goes first: tiles of the upper triangle row by row, then row-major
 * inside a tile. */
static int64_t atom_number(int nt, int L, int row, int col)
{
    int tr = row / L, tc = col / L;
    int64_t tile = (int64_t)tr * nt - (int64_t)tr * (tr - 1) / 2 + (tc - tr);
    return tile * L * L + (int64_t)(row % L) * L + (col % L);
}

/* does finest block (row, col) belong to one of the task's blocks? */
static int task_has_atom(const or_task *t, int w, int row, int col)
{
    int br[3], bc[3], bw[3];
    int nb = task_blocks(t, br, bc, bw);
    for (int bi = 0; bi < nb; bi++)
        if (row / w == br[bi] && col / w == bc[bi]) return 1;
    return 0;
}

/* ready-set order: larger `rank` first, then smaller scaled (K,I,J).  For the
 * Priority-List order `rank` is the critical time; for FCFS it is minus the
 * release time (earlier releases first). */
typedef struct { int64_t rank; int64_t k0, k1, k2; int task; } or_hent;

static int hent_before(const or_hent *a, const or_hent *b)
{
    if (a->rank != b->rank) return a->rank > b->rank;
    if (a->k0 != b->k0) return a->k0 < b->k0;
    if (a->k1 != b->k1) return a->k1 < b->k1;
    return a->k2 < b->k2;
}

typedef struct { or_hent *v; int n; } or_heap;

static void heap_push(or_heap *h, or_hent e)
{
    int i = h->n++;
    h->v[i] = e;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (!hent_before(&h->v[i], &h->v[p])) break;
        or_hent t = h->v[i]; h->v[i] = h->v[p]; h->v[p] = t; i = p;
    }
}

static or_hent heap_pop(or_heap *h)
{
    or_hent top = h->v[0];
    h->v[0] = h->v[--h->n];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && hent_before(&h->v[l], &h->v[m])) m = l;
        if (r < h->n && hent_before(&h->v[r], &h->v[m])) m = r;
        if (m == i) break;
        or_hent t = h->v[i]; h->v[i] = h->v[m]; h->v[m] = t; i = m;
    }
    return top;
}

typedef struct {
    int64_t makespan;
    int n_tasks;
    int64_t n_edges;
} or_result;

typedef struct {
    /* optional per-task outputs, in the oracle's program order */
    int32_t max_tasks;
    int32_t *task_info;   /* [max_tasks][5] type, level, K, I, J */
    int32_t *proc;
    int64_t *start, *finish, *rank;
    int64_t max_edges;
    int32_t *edges;       /* [max_edges][2] */
} or_outputs;

/* flags of the split trees: sum over l < dmax of tet(nt 2^l) */
static int64_t tree_flag_count(int nt, int dmax)
{
    int64_t n = 0;
    for (int l = 0; l < dmax; l++) {
        int64_t N = (int64_t)nt << l;
        n += N * (N + 1) * (N + 2) / 6;
    }
    return n;
}

/* the link that carries the transfers into memory space m */
static int link_of(const or_platform *pf, int m)
{
    return pf->link ? pf->link[m] : 0;
}

/* depth: split depth per top-level task, or (tree != 0) the split flags above */
static int simulate_one(const or_platform *pf, int nt, int dmax, const uint8_t *depth, int tree,
                        const or_grid *grain, or_result *res, const or_outputs *o)
{
    or_grid grid;
    or_tasklist tl = {0, 0, 0};
    or_dag g;
    or_tables tb = {0, 0, 0, 0};
    int rc;
    int64_t *W = 0, *rank = 0, *start = 0, *finish = 0, *avail = 0, *vf = 0;
    int64_t *cap = 0, *use = 0, *lfree = 0;
    int *pin = 0;
    int *proc = 0, *left = 0, *fifo = 0, *fifo_head = 0, *fifo_tail = 0, *fifo_next = 0;
    or_heap heap = {0, 0};
    memset(&g, 0, sizeof(g));

    if (grain) {
        /* grain batch: depth[t] is the grain index of top-level task t */
        grid = *grain;
        if (nt < 1 || tree) return OR_EINVAL;
        int n_top = nt * (nt + 1) * (nt + 2) / 6;
        for (int t = 0; t < n_top; t++) if (depth[t] >= grid.n) return OR_EINVAL;
        rc = expand(nt, depth, &grid, &tl);
    } else if (nt < 1 || dmax < 0 || dmax > 6 || (pf->b >> dmax) << dmax != pf->b) {
        return OR_EINVAL;
    } else if (tree) {
        grid.L = 1 << dmax; grid.n = dmax + 1; grid.pow2 = 1;
        for (int l = 0; l <= dmax; l++) grid.fac[l] = 1 << l;
        int64_t nf = tree_flag_count(nt, dmax);
        for (int64_t x = 0; x < nf; x++) if (depth[x] > 1) return OR_EINVAL;
        rc = expand_tree(nt, dmax, depth, &tl);
    } else {
        int n_top = nt * (nt + 1) * (nt + 2) / 6;
        for (int t = 0; t < n_top; t++) if (depth[t] > dmax) return OR_EINVAL;
        grid.L = 1 << dmax; grid.n = dmax + 1; grid.pow2 = 1;
        for (int l = 0; l <= dmax; l++) grid.fac[l] = 1 << l;
        rc = expand(nt, depth, &grid, &tl);
    }
    if (rc) goto done;
    rc = build_dag(&tl, nt, &grid, &g);
    if (rc) goto done;
    rc = make_tables(pf, &grid, &tb);
    if (rc) goto done;

    int n = tl.n, P = pf->n_procs, M = pf->n_mem, L = grid.n, N = nt * grid.L;
    W = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    rank = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    start = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    finish = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    proc = (int *)malloc((size_t)n * sizeof(int));
    left = (int *)malloc((size_t)n * sizeof(int));
    fifo_next = (int *)malloc((size_t)n * sizeof(int));
    avail = (int64_t *)calloc((size_t)P, sizeof(int64_t));
    fifo_head = (int *)malloc((size_t)P * sizeof(int));
    fifo_tail = (int *)malloc((size_t)P * sizeof(int));
    vf = (int64_t *)malloc((size_t)N * N * M * sizeof(int64_t));
    heap.v = (or_hent *)malloc((size_t)n * sizeof(or_hent));
    cap = (int64_t *)malloc((size_t)M * sizeof(int64_t));
    use = (int64_t *)calloc((size_t)N * N * M, sizeof(int64_t));
    pin = (int *)calloc((size_t)N * N * M, sizeof(int));
    lfree = (int64_t *)calloc((size_t)M, sizeof(int64_t));
    if (!W || !rank || !start || !finish || !proc || !left || !fifo_next || !avail ||
        !fifo_head || !fifo_tail || !vf || !heap.v || !cap || !use || !pin || !lfree) { rc = OR_ENOMEM; goto done; }

    /* 6. capacities in finest blocks (-1: unbounded); supported with write-back
     * caching, EFT-P and independent transfers */
    int capped = 0;
    int64_t atom_bytes = grid.pow2 ? pf->elem_bytes * (pf->b >> dmax) * (pf->b >> dmax) : 0;
    for (int m = 0; m < M && !grid.pow2; m++)   /* grain batches: unbounded spaces only */
        if (m > 0 && pf->capacity && pf->capacity[m] > 0) { rc = OR_EINVAL; goto done; }
    for (int m = 0; m < M; m++) {
        cap[m] = (m > 0 && pf->capacity && pf->capacity[m] > 0) ? pf->capacity[m] / atom_bytes : -1;
        if (cap[m] >= 0) capped = 1;
    }
    if (capped && (pf->cache != 0 || pf->select != 0 || pf->bus != 0)) { rc = OR_EINVAL; goto done; }

    /* 4. critical times: sum of the task's time over all processors, then the
     * longest such path to an exit, tasks visited in reverse program order
     * (edges always point forward in program order) */
    for (int t = 0; t < n; t++) {
        int64_t s = 0;
        for (int p = 0; p < P; p++)
            s += tb.cost[(pf->proc_type[p] * 4 + tl.v[t].type) * L + tl.v[t].level];
        W[t] = s;
    }
    for (int t = n - 1; t >= 0; t--) {
        int64_t best = 0;
        for (int e = g.succ_ptr[t]; e < g.succ_ptr[t + 1]; e++)
            if (rank[g.succ[e]] > best) best = rank[g.succ[e]];
        rank[t] = W[t] + best;
    }

    /* 5. event simulation */
    for (int64_t a = 0; a < (int64_t)N * N; a++)
        for (int m = 0; m < M; m++) vf[a * M + m] = (m == 0) ? 0 : OR_INF; /* data starts on the host */
    for (int p = 0; p < P; p++) { fifo_head[p] = -1; fifo_tail[p] = -1; }
    for (int t = 0; t < n; t++) { left[t] = g.npred[t]; proc[t] = -1; }
    for (int t = 0; t < n; t++)
        if (left[t] == 0) {
            int w = grid_w(&grid, tl.v[t].level);
            heap_push(&heap, (or_hent){pf->order ? 0 : rank[t], (int64_t)tl.v[t].K * w,
                                       (int64_t)tl.v[t].I * w, (int64_t)tl.v[t].J * w, t});
        }
    /* link contention (reading of the platform's network topology): a transfer
     * occupies the link of the space it goes into, one transfer at a time per
     * link; lfree[l] is when link l is next free */
    int64_t T = 0, makespan = 0;
    int done_count = 0;
    for (;;) {
        /* (i) ready tasks are mapped now, in order; with R-P / F-P only onto
         * processors idle now (nothing queued), the others wait */
        while (heap.n) {
            int n_idle = 0, pick = -1;
            if (pf->select >= 2) {
                for (int p = 0; p < P; p++) n_idle += avail[p] <= T;
                if (n_idle == 0) break;          /* every processor busy: wait */
            }
            or_hent top = heap_pop(&heap);
            int t = top.task;
            int br[3], bc[3], bw[3];
            int nb = task_blocks(&tl.v[t], br, bc, bw);
            int w = grid_w(&grid, tl.v[t].level);
            if (pf->select == 2) {
                /* R-P: the u-th idle processor (index order), u drawn for the
                 * task's finest-grid corner (K, I, J) */
                uint64_t key = ((uint64_t)(tl.v[t].K * w) << 18) | ((uint64_t)(tl.v[t].I * w) << 9) |
                               (uint64_t)(tl.v[t].J * w);
                int u = (int)(sm_draw(pf->seed, 8, key) % (uint64_t)n_idle);
                for (int p = 0; p < P; p++)
                    if (avail[p] <= T && u-- == 0) { pick = p; break; }
            } else if (pf->select == 3) {
                /* F-P: the idle processor with the smallest task time, ties lowest */
                int64_t best_c = 0;
                for (int p = 0; p < P; p++) {
                    if (avail[p] > T) continue;
                    int64_t c = tb.cost[(pf->proc_type[p] * 4 + tl.v[t].type) * L + tl.v[t].level];
                    if (pick < 0 || c < best_c) { pick = p; best_c = c; }
                }
            }
            int best_p = -1;
            int64_t best_eft = 0, best_est = 0, best_sel = 0;
            for (int p = 0; p < P; p++) {
                if (pick >= 0 && p != pick) continue;
                int m = pf->proc_mem[p];
                if (cap[m] >= 0) {
                    /* reading (capacity): the space must hold the blocks used by the
                     * tasks mapped there and not finished (pinned) plus this task's */
                    int64_t places = 0;
                    for (int r = 0; r < N; r++) for (int c = 0; c < N; c++) {
                        int64_t a = (int64_t)r * N + c;
                        if (pin[a * M + m] > 0 || task_has_atom(&tl.v[t], w, r, c)) places++;
                    }
                    if (places > cap[m]) continue;
                }
                int64_t est = T > avail[p] ? T : avail[p];
                int64_t bus_at = lfree[link_of(pf, m)];   /* where this mapping's transfers would queue */
                for (int bi = 0; bi < nb; bi++) {
                    int64_t miss = 0, fin = INT64_MIN;
                    for (int u = 0; u < w; u++) for (int v = 0; v < w; v++) {
                        int64_t a = (int64_t)(br[bi] * w + u) * N + (bc[bi] * w + v);
                        int64_t x = vf[a * M + m];
                        if (x == OR_INF) miss++;
                        else if (x > fin) fin = x;
                    }
                    int64_t ready = fin;
                    if (miss > 0) {
                        int64_t go = xfer_start(vf, M, N, br[bi], bc[bi], w, m, T);
                        if (pf->bus && bus_at > go) go = bus_at;
                        if (pf->bus) bus_at = go + tb.xfer[miss];
                        if (go + tb.xfer[miss] > ready) ready = go + tb.xfer[miss];
                    }
                    if (ready > est) est = ready;
                }
                int64_t eft = est + tb.cost[(pf->proc_type[p] * 4 + tl.v[t].type) * L + tl.v[t].level];
                /* EFT-P: earliest finish; EIT-P: earliest time the processor is idle
                 * (reading: an idle processor counts as idle from now, so idle
                 * processors tie); ties to the lowest index */
                int64_t sel = pf->select ? (T > avail[p] ? T : avail[p]) : eft;
                if (best_p < 0 || sel < best_sel) { best_p = p; best_sel = sel; best_eft = eft; best_est = est; }
            }
            if (best_p < 0) {
                /* reading (capacity): no space can take the task now; it and the
                 * tasks after it wait for the next completion */
                heap_push(&heap, top);
                break;
            }
            /* commit: transfers of the missing atoms are issued now, at time T */
            int m = pf->proc_mem[best_p];
            if (cap[m] >= 0) {
                /* make room: evict the unpinned blocks of m that the task does not
                 * use, least recently used first; reading (capacity): a block
                 * without a host copy is first copied back to the host, one transfer
                 * per finest block, issued now */
                int64_t occ = 0, need = 0;
                for (int r = 0; r < N; r++) for (int c = 0; c < N; c++) {
                    int64_t a = (int64_t)r * N + c;
                    if (vf[a * M + m] != OR_INF) occ++;
                    else if (task_has_atom(&tl.v[t], w, r, c)) need++;
                }
                for (int64_t k = occ + need - cap[m]; k > 0; k--) {
                    int64_t va = -1, vu = 0, vn = 0;
                    for (int r = 0; r < N; r++) for (int c = 0; c < N; c++) {
                        int64_t a = (int64_t)r * N + c;
                        if (vf[a * M + m] == OR_INF || pin[a * M + m] > 0 || task_has_atom(&tl.v[t], w, r, c))
                            continue;
                        int64_t u = use[a * M + m], num = atom_number(nt, grid.L, r, c);
                        if (va < 0 || u < vu || (u == vu && num < vn)) { va = a; vu = u; vn = num; }
                    }
                    if (va < 0) { rc = OR_EINVAL; goto done; }   /* excluded by the check above */
                    if (vf[va * M + 0] == OR_INF) vf[va * M + 0] = T + tb.xfer[1];
                    vf[va * M + m] = OR_INF;
                }
            }
            for (int bi = 0; bi < nb; bi++) {
                int64_t miss = 0;
                for (int u = 0; u < w; u++) for (int v = 0; v < w; v++) {
                    int64_t a = (int64_t)(br[bi] * w + u) * N + (bc[bi] * w + v);
                    if (vf[a * M + m] == OR_INF) miss++;
                }
                if (!miss) continue;
                int64_t go = xfer_start(vf, M, N, br[bi], bc[bi], w, m, T);
                /* shared interconnect: one transfer at a time, in issue order (the
                 * blocks of one task in their order) */
                if (pf->bus && lfree[link_of(pf, m)] > go) go = lfree[link_of(pf, m)];
                if (pf->bus) lfree[link_of(pf, m)] = go + tb.xfer[miss];
                for (int u = 0; u < w; u++) for (int v = 0; v < w; v++) {
                    int64_t a = (int64_t)(br[bi] * w + u) * N + (bc[bi] * w + v);
                    if (vf[a * M + m] == OR_INF) vf[a * M + m] = go + tb.xfer[miss];
                }
            }
            /* the task's blocks in m: used now, pinned until it finishes */
            for (int bi = 0; bi < nb; bi++)
                for (int u = 0; u < w; u++) for (int v = 0; v < w; v++) {
                    int64_t a = (int64_t)(br[bi] * w + u) * N + (bc[bi] * w + v);
                    use[a * M + m] = T;
                    pin[a * M + m]++;
                }
            proc[t] = best_p; start[t] = best_est; finish[t] = best_eft;
            avail[best_p] = best_eft;
            fifo_next[t] = -1;
            if (fifo_tail[best_p] < 0) fifo_head[best_p] = t; else fifo_next[fifo_tail[best_p]] = t;
            fifo_tail[best_p] = t;
        }
        /* (ii) next event: the earliest completion at the head of a queue */
        int64_t Tn = OR_INF;
        for (int p = 0; p < P; p++)
            if (fifo_head[p] >= 0 && finish[fifo_head[p]] < Tn) Tn = finish[fifo_head[p]];
        if (Tn == OR_INF) {
            if (heap.n) { rc = OR_ECAP; goto done; }   /* nothing left to wait for */
            break;
        }
        /* (iii) all completions at Tn, before any mapping at Tn (reading) */
        for (int p = 0; p < P; p++) {
            int t = fifo_head[p];
            if (t < 0 || finish[t] != Tn) continue;
            fifo_head[p] = fifo_next[t];
            if (fifo_head[p] < 0) fifo_tail[p] = -1;
            done_count++;
            /* coherence of the written block (memory spaces as software caches of
             * the host, space 0):
             *   write-back: valid only where it was computed;
             *   write-through: valid there, and on the host once a copy issued now
             *     has arrived; nowhere else;
             *   write-around: not kept in an accelerator's space: valid on the host
             *     only, once the copy issued now has arrived.
             * reading: the copy to the host costs the transfer of the whole block */
            int br[3], bc[3], bw[3];
            int nb = task_blocks(&tl.v[t], br, bc, bw);
            int w = grid_w(&grid, tl.v[t].level), m = pf->proc_mem[p];
            for (int bi = 0; bi < nb; bi++)
                for (int u = 0; u < w; u++) for (int v = 0; v < w; v++)
                    pin[((int64_t)(br[bi] * w + u) * N + (bc[bi] * w + v)) * M + m]--;
            int64_t host_at = (m == 0) ? Tn : Tn + tb.xfer[(int64_t)w * w];
            if (pf->bus && pf->cache != 0 && m != 0) {     /* the host copy queues on the host's link */
                int64_t go = Tn > lfree[link_of(pf, 0)] ? Tn : lfree[link_of(pf, 0)];
                host_at = go + tb.xfer[(int64_t)w * w];
                lfree[link_of(pf, 0)] = host_at;
            }
            for (int bi = 0; bi < nb; bi++) {
                if (!bw[bi]) continue;
                for (int u = 0; u < w; u++) for (int v = 0; v < w; v++) {
                    int64_t a = (int64_t)(br[bi] * w + u) * N + (bc[bi] * w + v);
                    for (int mm = 0; mm < M; mm++) {
                        int64_t x = OR_INF;
                        if (pf->cache == 0) x = (mm == m) ? Tn : OR_INF;
                        else if (pf->cache == 1) x = (mm == m) ? Tn : (mm == 0 ? host_at : OR_INF);
                        else x = (mm == 0) ? host_at : OR_INF;
                        vf[a * M + mm] = x;
                    }
                }
            }
            for (int e = g.succ_ptr[t]; e < g.succ_ptr[t + 1]; e++) {
                int v = g.succ[e];
                if (--left[v] == 0) {
                    int w2 = grid_w(&grid, tl.v[v].level);
                    heap_push(&heap, (or_hent){pf->order ? -Tn : rank[v], (int64_t)tl.v[v].K * w2,
                                               (int64_t)tl.v[v].I * w2, (int64_t)tl.v[v].J * w2, v});
                }
            }
        }
        T = Tn;
        if (Tn > makespan) makespan = Tn;
    }
    if (done_count != n) { rc = OR_EINVAL; goto done; }   /* cannot happen on a DAG */

    res->makespan = makespan; res->n_tasks = n; res->n_edges = g.n_edges;
    if (o) {
        if (o->task_info || o->proc || o->start || o->finish || o->rank) {
            if (n > o->max_tasks) { rc = OR_ECAP; goto done; }
            for (int t = 0; t < n; t++) {
                if (o->task_info) {
                    o->task_info[5 * t + 0] = tl.v[t].type; o->task_info[5 * t + 1] = tl.v[t].level;
                    o->task_info[5 * t + 2] = tl.v[t].K; o->task_info[5 * t + 3] = tl.v[t].I;
                    o->task_info[5 * t + 4] = tl.v[t].J;
                }
                if (o->proc) o->proc[t] = proc[t];
                if (o->start) o->start[t] = start[t];
                if (o->finish) o->finish[t] = finish[t];
                if (o->rank) o->rank[t] = rank[t];
            }
        }
        if (o->edges) {
            if (g.n_edges > o->max_edges) { rc = OR_ECAP; goto done; }
            for (int64_t e = 0; e < g.n_edges; e++) {
                o->edges[2 * e] = (int32_t)(g.edge[e] / n);
                o->edges[2 * e + 1] = (int32_t)(g.edge[e] % n);
            }
        }
    }
    rc = OR_OK;
done:
    free(tl.v); dag_free(&g); free_tables(&tb);
    free(W); free(rank); free(start); free(finish); free(proc); free(left); free(fifo_next);
    free(avail); free(fifo_head); free(fifo_tail); free(vf); free(heap.v); free(fifo);
    free(cap); free(use); free(pin); free(lfree);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* exported entry points (plain C ABI, loaded by the tests with ctypes)      */

int oracle_simulate(int nt, int dmax, const uint8_t *depth,
                    int n_procs, const int32_t *proc_type, const int32_t *proc_mem, int n_mem,
                    int n_ptypes, const int64_t *rmax, const int64_t *h, int64_t b,
                    int64_t latency_ns, int64_t bw, int64_t elem_bytes, int shared,
                    int64_t *makespan, int32_t *n_tasks, int64_t *n_edges,
                    int32_t max_tasks, int32_t *task_info, int32_t *proc_out,
                    int64_t *start_out, int64_t *finish_out, int64_t *rank_out,
                    int64_t max_edges, int32_t *edges_out, int order, int select, uint64_t seed,
                    int cache, int tree, int bus, const int64_t *capacity, const int32_t *link)
{
    if (!depth || n_procs < 1 || !proc_type || !proc_mem || n_mem < 1 || !rmax || !h) return OR_EINVAL;
    if (order < 0 || order > 1 || select < 0 || select > 3 || cache < 0 || cache > 2 || bus < 0 || bus > 1)
        return OR_EINVAL;
    for (int p = 0; p < n_procs; p++)
        if (proc_type[p] < 0 || proc_type[p] >= n_ptypes || proc_mem[p] < 0 || proc_mem[p] >= n_mem)
            return OR_EINVAL;
    for (int m = 0; link && m < n_mem; m++)
        if (link[m] < 0 || link[m] >= n_mem) return OR_EINVAL;
    or_platform pf = {n_procs, n_mem, n_ptypes, proc_type, proc_mem, rmax, h, b,
                      latency_ns, bw, elem_bytes, shared, order, select, seed, cache, bus, link, capacity};
    or_outputs o = {max_tasks, task_info, proc_out, start_out, finish_out, rank_out, max_edges, edges_out};
    or_result r;
    int rc = simulate_one(&pf, nt, dmax, depth, tree, NULL, &r, &o);
    if (rc) return rc;
    if (makespan) *makespan = r.makespan;
    if (n_tasks) *n_tasks = r.n_tasks;
    if (n_edges) *n_edges = r.n_edges;
    return OR_OK;
}

typedef struct {
    const or_platform *pf;
    int n_cand;
    const int32_t *nt, *dmax;
    const int64_t *mask_off;
    const uint8_t *depth;
    int64_t *makespan;
    int32_t *n_tasks;
    int32_t *status;
    int tree;
    const or_grid *grain;   /* grain batch, or NULL */
    int next;
    pthread_mutex_t mu;
} or_batch_job;

static void *batch_worker(void *arg)
{
    or_batch_job *j = (or_batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        int c = j->next++;
        pthread_mutex_unlock(&j->mu);
        if (c >= j->n_cand) break;
        or_result r = {0, 0, 0};
        int rc = simulate_one(j->pf, j->nt[c], j->dmax[c], j->depth + j->mask_off[c], j->tree, j->grain, &r, NULL);
        j->makespan[c] = rc ? -1 : r.makespan;
        if (j->n_tasks) j->n_tasks[c] = rc ? 0 : r.n_tasks;
        if (j->status) j->status[c] = rc;
    }
    return NULL;
}

/* one candidate per job on a pool of n_threads POSIX threads */
int oracle_simulate_batch(int n_cand, const int32_t *nt, const int32_t *dmax,
                          const int64_t *mask_off, const uint8_t *depth,
                          int n_procs, const int32_t *proc_type, const int32_t *proc_mem, int n_mem,
                          int n_ptypes, const int64_t *rmax, const int64_t *h, int64_t b,
                          int64_t latency_ns, int64_t bw, int64_t elem_bytes, int shared,
                          int n_threads, int64_t *makespan, int32_t *n_tasks, int32_t *status,
                          int order, int select, uint64_t seed, int cache, int tree, int bus,
                          const int64_t *capacity, const int32_t *link)
{
    if (n_cand < 0 || !nt || !dmax || !mask_off || !depth || !makespan || n_threads < 1) return OR_EINVAL;
    if (order < 0 || order > 1 || select < 0 || select > 3 || cache < 0 || cache > 2 || bus < 0 || bus > 1)
        return OR_EINVAL;
    for (int m = 0; link && m < n_mem; m++)
        if (link[m] < 0 || link[m] >= n_mem) return OR_EINVAL;
    or_platform pf = {n_procs, n_mem, n_ptypes, proc_type, proc_mem, rmax, h, b,
                      latency_ns, bw, elem_bytes, shared, order, select, seed, cache, bus, link, capacity};
    or_batch_job j;
    j.pf = &pf; j.n_cand = n_cand; j.nt = nt; j.dmax = dmax; j.mask_off = mask_off; j.depth = depth;
    j.makespan = makespan; j.n_tasks = n_tasks; j.status = status; j.tree = tree; j.grain = NULL; j.next = 0;
    pthread_mutex_init(&j.mu, NULL);
    pthread_t *th = (pthread_t *)malloc((size_t)n_threads * sizeof(pthread_t));
    if (!th) return OR_ENOMEM;
    int started = 0;
    for (int i = 0; i < n_threads; i++)
        if (pthread_create(&th[i], NULL, batch_worker, &j) == 0) started++;
        else break;
    if (started == 0) batch_worker(&j);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&j.mu);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* grain batches (partition parameter p = 1/f for any integer f, section 2.1;
 * partially overlapping blocks, Fig. 4)                                     */

static int64_t gcd64(int64_t a, int64_t b) { while (b) { int64_t t = a % b; a = b; b = t; } return a; }

/* the atom grid of a factor list: L = lcm(fac), at most 64 atoms per tile side */
static int grain_grid(int n_fac, const int32_t *fac, or_grid *gr)
{
    if (n_fac < 1 || n_fac > 8 || !fac) return OR_EINVAL;
    int64_t L = 1;
    for (int g = 0; g < n_fac; g++) {
        if (fac[g] < 1 || fac[g] > 64) return OR_EINVAL;
        L = L / gcd64(L, fac[g]) * fac[g];
        if (L > 64) return OR_EINVAL;
        gr->fac[g] = fac[g];
    }
    gr->L = (int)L; gr->n = n_fac; gr->pow2 = 0;
    return OR_OK;
}

int oracle_simulate_grain(int nt, int n_fac, const int32_t *fac, const uint8_t *grain,
                          int n_procs, const int32_t *proc_type, const int32_t *proc_mem, int n_mem,
                          int n_ptypes, const int64_t *rmax, const int64_t *h, int64_t b,
                          int64_t latency_ns, int64_t bw, int64_t elem_bytes, int shared,
                          int64_t *makespan, int32_t *n_tasks, int64_t *n_edges,
                          int32_t max_tasks, int32_t *task_info, int32_t *proc_out,
                          int64_t *start_out, int64_t *finish_out, int64_t *rank_out,
                          int64_t max_edges, int32_t *edges_out, int order, int select, uint64_t seed,
                          int cache, int bus, const int32_t *link)
{
    or_grid gr;
    if (!grain || n_procs < 1 || !proc_type || !proc_mem || n_mem < 1 || !rmax || !h) return OR_EINVAL;
    if (grain_grid(n_fac, fac, &gr)) return OR_EINVAL;
    if (order < 0 || order > 1 || select < 0 || select > 3 || cache < 0 || cache > 2 || bus < 0 || bus > 1)
        return OR_EINVAL;
    for (int p = 0; p < n_procs; p++)
        if (proc_type[p] < 0 || proc_type[p] >= n_ptypes || proc_mem[p] < 0 || proc_mem[p] >= n_mem)
            return OR_EINVAL;
    for (int m = 0; link && m < n_mem; m++)
        if (link[m] < 0 || link[m] >= n_mem) return OR_EINVAL;
    or_platform pf = {n_procs, n_mem, n_ptypes, proc_type, proc_mem, rmax, h, b,
                      latency_ns, bw, elem_bytes, shared, order, select, seed, cache, bus, link, NULL};
    or_outputs o = {max_tasks, task_info, proc_out, start_out, finish_out, rank_out, max_edges, edges_out};
    or_result r;
    int rc = simulate_one(&pf, nt, 0, grain, 0, &gr, &r, &o);
    if (rc) return rc;
    if (makespan) *makespan = r.makespan;
    if (n_tasks) *n_tasks = r.n_tasks;
    if (n_edges) *n_edges = r.n_edges;
    return OR_OK;
}

/* n_cand candidates of nt tiles, grain[c * tet(nt) + t]; one candidate per job */
int oracle_simulate_grain_batch(int n_cand, int nt, int n_fac, const int32_t *fac, const uint8_t *grain,
                                int n_procs, const int32_t *proc_type, const int32_t *proc_mem, int n_mem,
                                int n_ptypes, const int64_t *rmax, const int64_t *h, int64_t b,
                                int64_t latency_ns, int64_t bw, int64_t elem_bytes, int shared,
                                int n_threads, int64_t *makespan, int32_t *n_tasks, int32_t *status,
                                int order, int select, uint64_t seed, int cache, int bus, const int32_t *link)
{
    or_grid gr;
    if (n_cand < 0 || nt < 1 || !grain || !makespan || n_threads < 1) return OR_EINVAL;
    if (grain_grid(n_fac, fac, &gr)) return OR_EINVAL;
    if (order < 0 || order > 1 || select < 0 || select > 3 || cache < 0 || cache > 2 || bus < 0 || bus > 1)
        return OR_EINVAL;
    for (int m = 0; link && m < n_mem; m++)
        if (link[m] < 0 || link[m] >= n_mem) return OR_EINVAL;
    int32_t *nts = (int32_t *)malloc((size_t)(n_cand ? n_cand : 1) * sizeof(int32_t));
    int32_t *zeros = (int32_t *)calloc((size_t)(n_cand ? n_cand : 1), sizeof(int32_t));
    int64_t *off = (int64_t *)malloc((size_t)(n_cand ? n_cand : 1) * sizeof(int64_t));
    if (!nts || !zeros || !off) { free(nts); free(zeros); free(off); return OR_ENOMEM; }
    int64_t n_top = (int64_t)nt * (nt + 1) * (nt + 2) / 6;
    for (int c = 0; c < n_cand; c++) { nts[c] = nt; off[c] = c * n_top; }
    or_platform pf = {n_procs, n_mem, n_ptypes, proc_type, proc_mem, rmax, h, b,
                      latency_ns, bw, elem_bytes, shared, order, select, seed, cache, bus, link, NULL};
    or_batch_job j;
    j.pf = &pf; j.n_cand = n_cand; j.nt = nts; j.dmax = zeros; j.mask_off = off; j.depth = grain;
    j.makespan = makespan; j.n_tasks = n_tasks; j.status = status; j.tree = 0; j.grain = &gr; j.next = 0;
    pthread_mutex_init(&j.mu, NULL);
    pthread_t *th = (pthread_t *)malloc((size_t)n_threads * sizeof(pthread_t));
    int started = 0;
    for (int i = 0; th && i < n_threads; i++)
        if (pthread_create(&th[i], NULL, batch_worker, &j) == 0) started++;
        else break;
    if (started == 0) batch_worker(&j);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    free(th); free(nts); free(zeros); free(off);
    pthread_mutex_destroy(&j.mu);
    return OR_OK;
}
