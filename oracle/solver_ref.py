"""CPU reference of HeSP's iterative scheduler-partitioner (section 2.1,
"Iterative solver"), written from the paper's description.

TEST INFRASTRUCTURE ONLY: used by the test-suite to check the library's solver;
the product path never imports it.

Every iteration is a schedule stage (an exact simulation of the current
partition, by the C oracle) followed by a partition stage that changes the
split depth of one task cluster (a top-level task of Fig. 1 and the fine tasks
it was split into).  The paper leaves the score and the partition parameter
open; the reading used here (all integer arithmetic, so that results are exact):

* span(c)   = latest finish - earliest start over the cluster's tasks;
  t0(c) the earliest start; ptype(c) the type of the processor that ran the
  task starting at t0 (lowest processor index on ties: a processor runs one
  task at a time, so the pair (start, processor) names one task).
* avail(c)  = P - (number of tasks running at t0) + 1: the processors idle when
  the cluster started, plus the one it started on ("available parallelism at its
  scheduling time").
* For every other depth d' in 0..dmax:
    work(c,d') = sum over the cluster's tasks at depth d' of their time on ptype(c);
    par(d')    = max(1, floor(tasks at depth d' / 2^d')), the tasks per step of
                 the blocked algorithm's outer loop;
    est(c,d')  = ceil(work / min(avail(c), par(d')));
    score      = span(c) - est(c,d').
  The cluster's proposal is the depth with the largest score (smallest depth on
  ties); it is a candidate when that score is positive.  A smaller depth merges
  the cluster back (p = 1 relative to the old split), a larger one splits it
  further (p < 1).
* Candidate lists: All (every cluster), CP (clusters with a task on the
  critical path, read on the task DAG with the previous step's times: from the
  last-finishing task, repeatedly the DAG predecessor that finished last, until
  a task without predecessors; ties to the lowest processor index, which is
  unique among tasks finishing together), Shallow (clusters whose depth is the
  smallest present).
* Selection: Hard, the largest score (smallest cluster index on ties); Soft,
  u = SplitMix64 draw(seed, 10, iteration) mod (sum of scores), the first
  candidate in cluster order whose running score sum exceeds u.
* No candidate: the partition is kept (a fixed point) for the remaining
  iterations.  The solver returns the best simulated partition (earliest on
  ties) and the makespan of every iteration.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

LISTS = {"all": 0, "cp": 1, "shallow": 2}
_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def _mix(z: int) -> int:
    """SplitMix64 finaliser (Steele, Lea and Flood, 2014)."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def _draw(seed: int, purpose: int, index: int) -> int:
    """Value number index+1 of the SplitMix64 sequence started at mix(seed + gamma (purpose+1))."""
    state = _mix((seed + _GAMMA * (purpose + 1)) & _M64)
    return _mix((state + _GAMMA * (index + 1)) & _M64)
SAMPLING = {"hard": 0, "soft": 1}


def tet(n: int) -> int:
    """Top-level tasks of the nt x nt tiled Cholesky loop nest (Fig. 1): n(n+1)(n+2)/6."""
    return n * (n + 1) * (n + 2) // 6


def _fine_counts(kind: int, d: int):
    """Fine tasks of each kind (chol, trsm, syrk, gemm) in a cluster of `kind` split d times."""
    s = 1 << d
    if kind == 3:
        return [0, 0, 0, s ** 3]
    if kind == 2:
        return [0, 0, s * s, s * s * (s - 1) // 2]
    if kind == 1:
        return [0, s * s, 0, s * s * (s - 1) // 2]
    return [s, s * (s - 1) // 2, s * (s - 1) // 2, s * (s - 1) * (s - 2) // 6]


def _kind_of_top(nt: int):
    kinds, cells = [], []
    for k in range(nt):
        kinds.append(0); cells.append((k, k, k))
        for j in range(k + 1, nt):
            kinds.append(1); cells.append((k, k, j))
        for i in range(k + 1, nt):
            for j in range(i + 1, nt):
                kinds.append(3); cells.append((k, i, j))
            kinds.append(2); cells.append((k, i, i))
    return kinds, {c: t for t, c in enumerate(cells)}


def candidates(n_top, depth, sched, cl, lst):
    """Clusters proposed for a change: All, CP or Shallow (see the module header);
    cl[t] is the cluster of task t."""
    start, finish, proc = sched.start.astype(np.int64), sched.finish.astype(np.int64), sched.proc
    n = len(start)
    if lst == 0:
        return list(range(n_top))
    elif lst == 2:
        dm = int(min(depth))
        cand = [c for c in range(n_top) if int(depth[c]) == dm]
    else:
        preds = [[] for _ in range(n)]
        for u, v in sched.edges:
            preds[int(v)].append(int(u))
        last = lambda xs: max(xs, key=lambda x: (int(finish[x]), -int(proc[x])))
        t = last(range(n))
        on = set()
        while True:
            on.add(int(cl[t]))
            if not preds[t]:
                break
            t = last(preds[t])
        cand = sorted(on)
    return cand


def partition_step(pf, nt, dmax, b, depth, sched, cost, it, lst, sampling, seed):
    """One partition stage: returns (cluster, new depth, score) or None."""
    kinds, index = _kind_of_top(nt)
    n_top = len(kinds)
    tasks = np.asarray(sched.tasks)
    cl = np.array([index[(int(K) >> int(l), int(I) >> int(l), int(J) >> int(l))] for (_, l, K, I, J) in tasks])
    start, finish, proc = sched.start.astype(np.int64), sched.finish.astype(np.int64), sched.proc
    P = pf.n_procs
    span, t0, pt = {}, {}, {}
    for c in range(n_top):
        idx = np.nonzero(cl == c)[0]
        first = min(idx, key=lambda t: (int(start[t]), int(proc[t])))
        t0[c] = int(start[first])
        span[c] = int(finish[idx].max()) - t0[c]
        pt[c] = int(pf.proc_type[proc[first]])
    cand = candidates(n_top, depth, sched, cl, lst)
    # proposals
    best = []
    for c in cand:
        running = int(np.sum((start <= t0[c]) & (t0[c] < finish)))
        avail = P - running + 1
        top = None
        for dn in range(dmax + 1):
            if dn == int(depth[c]):
                continue
            cnt = _fine_counts(kinds[c], dn)
            work = sum(cnt[k] * int(cost[pt[c], k, dn]) for k in range(4))
            par = max(1, sum(cnt) >> dn)
            lanes = min(avail, par)
            est = -(-work // lanes)
            score = span[c] - est
            if top is None or score > top[1]:
                top = (dn, score)
        if top is not None and top[1] > 0:
            best.append((c, top[0], top[1]))
    if not best:
        return None
    if sampling == 0:
        return max(best, key=lambda x: (x[2], -x[0]))
    total = sum(x[2] for x in best)
    u = _draw(seed, 10, it) % total
    acc = 0
    for x in best:
        acc += x[2]
        if acc > u:
            return x
    return best[-1]


def solve(pf, nt, dmax, b, iters, lst=0, sampling=0, seed=0, policy=(0, 0), depth0=None, cost=None):
    """Runs the iterative solver; returns (best depth, best makespan, makespans per iteration, steps)."""
    n_top = tet(nt)
    depth = np.zeros(n_top, np.uint8) if depth0 is None else np.array(depth0, np.uint8)
    if cost is None:
        cost = np.zeros((pf.n_ptypes, 4, dmax + 1), np.int64)
        for p in range(pf.n_ptypes):
            for k in range(4):
                for lv in range(dmax + 1):
                    cost[p, k, lv] = O.task_time(k, b >> lv, int(pf.rmax[p][k]), int(pf.h[p]))
    best_d, best_ms, trace, steps = depth.copy(), None, [], []
    fixed = False
    for it in range(iters):
        s = O.simulate(pf, nt, dmax, b, depth, detail=True, policy=policy)
        trace.append(s.makespan)
        if best_ms is None or s.makespan < best_ms:
            best_ms, best_d = s.makespan, depth.copy()
        if fixed:
            steps.append(None)
            continue
        st = partition_step(pf, nt, dmax, b, depth, s, cost, it, lst, sampling, seed)
        steps.append(st)
        if st is None:
            fixed = True
        else:
            depth[st[0]] = st[1]
    return best_d, best_ms, trace, steps


# ---------------------------------------------------------------- split-tree partitions
#
# The solver on split-tree partitions (a cluster may hold sub-clusters, section
# 2.1): the clusters are the existing tasks of the uniform level-l tilings,
# l < dmax ("nodes"; node x is split flag x of the partition).  Reading, as for
# top-level clusters:
# * span, start processor type and available parallelism of a node from the
#   tasks under it (its leaves);
# * an internal node proposes to merge back into its own task (p = 1): estimate
#   = that task's time on the node's processor type; a leaf node proposes one
#   more split (p = 1/2): estimate = ceil(work of its 2 x 2 blocked algorithm /
#   min(available, max(1, task count >> 1))); score = span - estimate;
# * All: every node; CP: nodes holding a task of the critical path; Shallow: the
#   leaf nodes at the smallest level of any task;
# * Hard / Soft over node order as before (the same draw); a split clears the
#   flags of the new children, a merge clears the node's own flag.

def _tree_nodes(nt, dmax):
    """(level, cell, kind) of every node, in flag order."""
    out = []
    for l in range(dmax):
        kinds, index = _kind_of_top(nt << l)
        cells = sorted(index, key=index.get)
        out += [(l, c, k) for c, k in zip(cells, kinds)]
    return out


def _children(cell):
    K, I, J = cell
    return [(a, b_, c) for a in (2 * K, 2 * K + 1) for b_ in (2 * I, 2 * I + 1) for c in (2 * J, 2 * J + 1)
            if a <= b_ <= c]


def partition_step_tree(pf, nt, dmax, flags, sched, cost, it, lst, sampling, seed):
    """One partition stage on a split-tree partition: (node, action, score) with
    action 1 = split, 0 = merge, or None."""
    nodes = _tree_nodes(nt, dmax)
    pos = {(l, c): x for x, (l, c, _) in enumerate(nodes)}
    exists = np.zeros(len(nodes), bool)
    for x, (l, c, _) in enumerate(nodes):
        exists[x] = l == 0 or (exists[pos[(l - 1, (c[0] >> 1, c[1] >> 1, c[2] >> 1))]] and
                               flags[pos[(l - 1, (c[0] >> 1, c[1] >> 1, c[2] >> 1))]] == 1)
    tasks = np.asarray(sched.tasks)
    start, finish, proc = sched.start.astype(np.int64), sched.finish.astype(np.int64), sched.proc
    n = len(tasks)
    # nodes holding each task: its cell shifted up to every level below dmax
    holders = []
    for (_, l, K, I, J) in tasks:
        holders.append([pos[(lv, (int(K) >> (int(l) - lv), int(I) >> (int(l) - lv), int(J) >> (int(l) - lv)))]
                        for lv in range(min(int(l), dmax - 1) + 1) if lv <= int(l)])
    under = [[] for _ in nodes]
    for t, hs in enumerate(holders):
        for x in hs:
            under[x].append(t)
    P = pf.n_procs
    # candidate list
    if lst == 1:
        preds = [[] for _ in range(n)]
        for u, v in sched.edges:
            preds[int(v)].append(int(u))
        last = lambda xs: max(xs, key=lambda y: (int(finish[y]), -int(proc[y])))
        t = last(range(n))
        on = set()
        while True:
            on.update(holders[t])
            if not preds[t]:
                break
            t = last(preds[t])
        cand = [x for x in range(len(nodes)) if exists[x] and x in on]
    elif lst == 2:
        lmin = int(tasks[:, 1].min())
        cand = [x for x in range(len(nodes)) if exists[x] and flags[x] == 0 and nodes[x][0] == lmin]
    else:
        cand = [x for x in range(len(nodes)) if exists[x]]
    best = []
    for x in cand:
        idx = under[x]
        l, cell, kind = nodes[x]
        first = min(idx, key=lambda t: (int(start[t]), int(proc[t])))
        t0 = int(start[first])
        span = int(finish[idx].max()) - t0
        pt = int(pf.proc_type[proc[first]])
        if flags[x] == 1:
            est, action = int(cost[pt, kind, l]), 0
        else:
            cnt = _fine_counts(kind, 1)
            work = sum(cnt[k] * int(cost[pt, k, l + 1]) for k in range(4))
            running = int(np.sum((start <= t0) & (t0 < finish)))
            lanes = min(P - running + 1, max(1, sum(cnt) >> 1))
            est, action = -(-work // lanes), 1
        if span - est > 0:
            best.append((x, action, span - est))
    if not best:
        return None
    if sampling == 0:
        return max(best, key=lambda y: (y[2], -y[0]))
    total = sum(y[2] for y in best)
    u = _draw(seed, 10, it) % total
    acc = 0
    for y in best:
        acc += y[2]
        if acc > u:
            return y
    return best[-1]


def apply_tree_step(nt, dmax, flags, step):
    x, action, _ = step
    nodes = _tree_nodes(nt, dmax)
    flags[x] = action
    l, cell, _ = nodes[x]
    if action == 1 and l + 1 < dmax:
        pos = {(lv, c): y for y, (lv, c, _) in enumerate(nodes)}
        for ch in _children(cell):
            flags[pos[(l + 1, ch)]] = 0


def solve_tree(pf, nt, dmax, b, iters, lst=0, sampling=0, seed=0, policy=(0, 0), flags0=None, cost=None):
    """The solver on split-tree partitions; returns (best flags, best makespan,
    makespans per iteration, steps (node, action, score) or None)."""
    nf = sum(tet(nt << l) for l in range(dmax))
    flags = np.zeros(nf, np.uint8) if flags0 is None else np.array(flags0, np.uint8)
    if cost is None:
        cost = np.zeros((pf.n_ptypes, 4, dmax + 1), np.int64)
        for p in range(pf.n_ptypes):
            for k in range(4):
                for lv in range(dmax + 1):
                    cost[p, k, lv] = O.task_time(k, b >> lv, int(pf.rmax[p][k]), int(pf.h[p]))
    best_f, best_ms, trace, steps = flags.copy(), None, [], []
    for it in range(iters):
        s = O.simulate(pf, nt, dmax, b, flags, detail=True, policy=policy, tree=True)
        trace.append(s.makespan)
        if best_ms is None or s.makespan < best_ms:
            best_ms, best_f = s.makespan, flags.copy()
        st = partition_step_tree(pf, nt, dmax, flags, s, cost, it, lst, sampling, seed)
        steps.append(st)
        if st is not None:
            apply_tree_step(nt, dmax, flags, st)
    return best_f, best_ms, trace, steps
