"""A second, independent CPU reading of the method, in pure Python (tiny cases).

Test infrastructure: used to cross-check the C oracle (two implementations of
the same reading written separately) and, with its choice hooks, to enumerate
every push-at-release schedule of a tiny DAG for brute-force optima.

Expansion here enumerates the whole fine iteration space {K <= I <= J} and
assigns every fine task to the Fig. 1 task whose cell contains it; program
order is (Fig. 1 index of the cell, K, kind order of Fig. 1 within one K).
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from typing import Dict, List, Optional, Sequence, Tuple

CHOL, TRSM, SYRK, GEMM = 0, 1, 2, 3
KIND_NAMES = ("chol", "trsm", "syrk", "gemm")
FLOP_NUM = (1, 3, 3, 6)  # flops * 3 / b^3


def fig1_tasks(nt: int) -> List[Tuple[int, int, int, int]]:
    """(kind, k, i, j) in the order the Fig. 1 loop nest issues them."""
    out = []
    for k in range(nt):
        out.append((CHOL, k, k, k))
        for j in range(k + 1, nt):
            out.append((TRSM, k, k, j))
        for i in range(k + 1, nt):
            for j in range(i + 1, nt):
                out.append((GEMM, k, i, j))
            out.append((SYRK, k, i, i))
    return out


def kind_of(K: int, I: int, J: int) -> int:
    if K == I == J:
        return CHOL
    if K == I:
        return TRSM
    if I == J:
        return SYRK
    return GEMM


# position of a kind inside one K step of Fig. 1: chol, trsm(J), then per I: gemm(J>I), syrk
def _in_step_order(kind: int, K: int, I: int, J: int) -> Tuple[int, int, int]:
    if kind == CHOL:
        return (0, 0, 0)
    if kind == TRSM:
        return (1, J, 0)
    if kind == GEMM:
        return (2, I, J)
    return (2, I, 1 << 30)  # syrk(K,I) closes the I step


def expand(nt: int, depth: Sequence[int]):
    """Fine tasks (kind, level, K, I, J, top) in program order."""
    tops = fig1_tasks(nt)
    cell_of: Dict[Tuple[int, int, int], int] = {(k, i, j): t for t, (_, k, i, j) in enumerate(tops)}
    tasks = []
    for t, (kind, k, i, j) in enumerate(tops):
        d = int(depth[t])
        s = 1 << d
        fine = []
        for K in range(k * s, k * s + s):
            for I in range(i * s, i * s + s):
                for J in range(j * s, j * s + s):
                    if K <= I <= J:
                        fine.append((kind_of(K, I, J), d, K, I, J, t))
        fine.sort(key=lambda x: (x[2],) + _in_step_order(x[0], x[2], x[3], x[4]))
        tasks.extend(fine)
        assert all(cell_of[(x[2] >> d, x[3] >> d, x[4] >> d)] == t for x in fine)
    return tasks


def expand_tree(nt: int, dmax: int, flags: Sequence[int]):
    """Fine tasks (kind, level, K, I, J, top) in program order for split-tree
    flags (one per task of each uniform level-l tiling, Fig. 1 order, levels
    concatenated): a flagged task is replaced in place by the tasks of its cell
    on the 2x2 sub-tiling, in the same K-step order, each expanded again."""
    pos = []
    base = 0
    for l in range(dmax):
        tops = fig1_tasks(nt << l)
        pos.append({(k, i, j): base + x for x, (_, k, i, j) in enumerate(tops)})
        base += len(tops)

    def rec(kind, l, K, I, J, top):
        if l < dmax and flags[pos[l][(K, I, J)]]:
            kids = [(kind_of(a, b_, c), a, b_, c)
                    for a in (2 * K, 2 * K + 1) for b_ in (2 * I, 2 * I + 1) for c in (2 * J, 2 * J + 1)
                    if a <= b_ <= c]
            kids.sort(key=lambda x: (x[1],) + _in_step_order(x[0], x[1], x[2], x[3]))
            out = []
            for (kk, a, b_, c) in kids:
                out += rec(kk, l + 1, a, b_, c, top)
            return out
        return [(kind, l, K, I, J, top)]

    tasks = []
    for t, (kind, k, i, j) in enumerate(fig1_tasks(nt)):
        tasks += rec(kind, 0, k, i, j, t)
    return tasks


def blocks(task) -> List[Tuple[int, int, bool]]:
    kind, _, K, I, J, _ = task
    if kind == CHOL:
        return [(K, K, True)]
    if kind == TRSM:
        return [(K, K, False), (K, J, True)]
    if kind == SYRK:
        return [(K, I, False), (I, I, True)]
    return [(K, I, False), (K, J, False), (I, J, True)]


def atoms(R: int, C: int, level: int, dmax: int):
    w = 1 << (dmax - level)
    return [(R * w + u, C * w + v) for u in range(w) for v in range(w)]


def edges(tasks, dmax: int):
    last_w: Dict[Tuple[int, int], int] = {}
    readers: Dict[Tuple[int, int], List[int]] = {}
    E = set()
    for t, task in enumerate(tasks):
        for (R, C, w) in blocks(task):
            for a in atoms(R, C, task[1], dmax):
                if a in last_w:
                    E.add((last_w[a], t))
                if w:
                    for r in readers.get(a, []):
                        if r != t:
                            E.add((r, t))
                    readers[a] = []
                    last_w[a] = t
                else:
                    readers.setdefault(a, []).append(t)
    return sorted(E)


def task_time(kind: int, bl: int, rmax_mflops: int, h: int) -> int:
    """ceil(flops / R(b)) in ns, exact rationals (1 GFLOP/s = 1 flop/ns)."""
    flops = Fraction(FLOP_NUM[kind] * bl ** 3, 3)
    rate = Fraction(rmax_mflops, 1000) * Fraction(bl * bl, bl * bl + h * h)
    q = flops / rate
    return -((-q.numerator) // q.denominator)


def transfer_time(n_atoms: int, atom_side: int, shared: bool, latency=10_000, bw=12, elem=8) -> int:
    if shared or n_atoms == 0:
        return 0
    q = Fraction(elem * n_atoms * atom_side * atom_side, bw)
    return latency - ((-q.numerator) // q.denominator)


INF = float("inf")


class Sim:
    """Push-at-release event simulation with optional choice hooks.

    ``choose_task(ready, sim)`` returns the next ready task to map and
    ``choose_proc(task, efts, sim)`` the processor; by default the PL order
    and EFT-P rule are used.
    """

    def __init__(self, nt, dmax, b, depth, proc_type, proc_mem, n_mem, rmax, h, shared, tree=False):
        self.tasks = expand_tree(nt, dmax, depth) if tree else expand(nt, depth)
        self.E = edges(self.tasks, dmax)
        self.nt = nt
        self.n = len(self.tasks)
        self.dmax, self.b = dmax, b
        self.P = len(proc_type)
        self.proc_type, self.proc_mem, self.n_mem = list(proc_type), list(proc_mem), n_mem
        self.shared = shared
        self.cost = [[task_time(tk[0], b >> tk[1], int(rmax[pt][tk[0]]), int(h[pt]))
                      for pt in proc_type] for tk in self.tasks]
        self.atom_side = b >> dmax
        self.succ = [[] for _ in range(self.n)]
        self.npred = [0] * self.n
        for u, v in self.E:
            self.succ[u].append(v)
            self.npred[v] += 1
        self.rank = [0] * self.n
        for t in range(self.n - 1, -1, -1):
            self.rank[t] = sum(self.cost[t]) + max([self.rank[v] for v in self.succ[t]], default=0)

    def key(self, t):
        kind, lvl, K, I, J, _ = self.tasks[t]
        sh = self.dmax - lvl
        return (-self.rank[t], K << sh, I << sh, J << sh)

    def xfer(self, k):
        return transfer_time(k, self.atom_side, self.shared)

    @staticmethod
    def go_time(miss, T, vf):
        """Transfers of the missing atoms leave once every one of them has a valid
        copy somewhere (a host copy may still be in flight)."""
        src = [min(v for v in vf[a] if v != INF) for a in miss if any(v != INF for v in vf[a])]
        return max([T] + src)

    def transfers(self, t, m, T, vf, bus):
        """Arrival time of each block of task t that space m misses (None when
        it misses nothing); bus = time the shared interconnect frees up, or None
        when transfers do not contend.  Returns (arrivals, bus after them)."""
        out = []
        for (R, C, _) in blocks(self.tasks[t]):
            at = atoms(R, C, self.tasks[t][1], self.dmax)
            miss = [a for a in at if vf[a][m] == INF]
            if not miss:
                out.append(None)
                continue
            go = self.go_time(miss, T, vf)
            if bus is not None:
                go = max(go, bus)
                bus = go + self.xfer(len(miss))
            out.append(go + self.xfer(len(miss)))
        return out, bus

    def est(self, t, p, T, avail, vf, bus=None):
        m = self.proc_mem[p]
        e = max(T, avail[p])
        arr, _ = self.transfers(t, m, T, vf, bus)
        for (R, C, _), x in zip(blocks(self.tasks[t]), arr):
            at = atoms(R, C, self.tasks[t][1], self.dmax)
            fin = [vf[a][m] for a in at if vf[a][m] != INF]
            r = max(fin) if fin else -INF
            if x is not None:
                r = max(r, x)
            e = max(e, r)
        return e

    def task_atoms(self, t):
        return [a for (R, C, _) in blocks(self.tasks[t]) for a in atoms(R, C, self.tasks[t][1], self.dmax)]

    def lru_order(self, a):
        """Tie order among equally recently used finest blocks: upper-triangle
        tiles row by row, then row-major inside the tile."""
        w = 1 << self.dmax
        tr, tc = a[0] // w, a[1] // w
        tile = sum(self.nt - r for r in range(tr)) + (tc - tr)
        return (tile, (a[0] % w) * w + a[1] % w)

    def run(self, choose_task=None, choose_proc=None, order="PL", select="EFT", seed=0, cache="WB", bus=False,
            capacity=None, links=None):
        """order: "PL" (decreasing critical time) or "FCFS" (first released first);
        select: "EFT" (earliest finish), "EIT" (processor idle first), "RP"
        (random idle processor) or "FP" (fastest idle processor); with RP / FP a
        task that finds no idle processor waits for a completion.  Ties: smaller
        scaled (K, I, J), then lower processor index.  cache: "WB" (the written
        block stays only where it was computed), "WT" (also sent to the host at
        completion) or "WA" (sent to the host, not kept by an accelerator).
        capacity: bytes per memory space (None or <= 0: unbounded; the host
        always is): a space holds at most that many whole finest blocks; a task
        goes only to a processor whose space can hold the blocks of its own and of
        the tasks mapped there and not finished; when none can, it and the tasks
        after it wait for the next completion; room is made by dropping the least
        recently used other blocks (ties by lru_order), a block with no host copy
        being copied back first (one transfer per finest block).  Returns None
        when a task can never be taken.  bus: transfers contend, one at a time
        per link; links[m] names the link of the transfers into space m (copies
        sent to the host take the host's); None: one link for all."""
        from paper_1602_05510_amd.inputs import draw
        N = 0
        vf = {}
        for t in self.tasks:
            for (R, C, _) in blocks(t):
                for a in atoms(R, C, t[1], self.dmax):
                    vf[a] = [0] + [INF] * (self.n_mem - 1)
        avail = [0] * self.P
        left = list(self.npred)
        ready = [t for t in range(self.n) if left[t] == 0]
        released = {t: 0 for t in ready}
        fifo = [[] for _ in range(self.P)]
        proc, start, finish = [None] * self.n, [None] * self.n, [None] * self.n
        T = 0
        link_free = {}                          # link -> when it is next free

        def link(m):
            return links[m] if links is not None else 0

        def free_at(m):
            return link_free.get(link(m), 0) if bus else None
        slots = [None] * self.n_mem             # finest blocks per space, None = unbounded
        if capacity is not None:
            per = 8 * self.atom_side * self.atom_side
            slots = [None if (m == 0 or capacity[m] <= 0) else capacity[m] // per for m in range(self.n_mem)]
        pins, last_use = {}, {}
        while True:
            while ready:
                idle = [q for q in range(self.P) if avail[q] <= T]
                if select in ("RP", "FP") and not idle:
                    break
                if choose_task:
                    t = choose_task(ready, self)
                elif order == "FCFS":
                    t = min(ready, key=lambda u: (released[u],) + self.key(u)[1:])
                else:
                    t = min(ready, key=self.key)
                ready.remove(t)
                ests = [self.est(t, p, T, avail, vf, free_at(self.proc_mem[p])) for p in range(self.P)]
                efts = [ests[p] + self.cost[t][p] for p in range(self.P)]
                mine = set(self.task_atoms(t))

                def fits(q):
                    m = self.proc_mem[q]
                    if slots[m] is None:
                        return True
                    held = {a for (a, mm), c in pins.items() if mm == m and c > 0}
                    return len(held | mine) <= slots[m]
                if choose_proc:
                    p = choose_proc(t, efts, self)
                elif select == "EIT":
                    p = min(range(self.P), key=lambda q: (max(T, avail[q]), q))
                elif select == "RP":
                    kind, lvl, K, I, J, _ = self.tasks[t]
                    sh = self.dmax - lvl
                    corner = ((K << sh) << 18) | ((I << sh) << 9) | (J << sh)
                    p = idle[draw(seed, 8, corner) % len(idle)]
                elif select == "FP":
                    p = min(idle, key=lambda q: (self.cost[t][q], q))
                else:
                    ok = [q for q in range(self.P) if fits(q)]
                    if not ok:
                        ready.append(t)          # waits, and so do the tasks after it
                        break
                    p = min(ok, key=lambda q: (efts[q], q))
                m = self.proc_mem[p]
                if slots[m] is not None:
                    held = [a for a in vf if vf[a][m] != INF]
                    missing = [a for a in mine if vf[a][m] == INF]
                    extra = len(held) + len(missing) - slots[m]
                    if extra > 0:
                        free = [a for a in held if pins.get((a, m), 0) == 0 and a not in mine]
                        free.sort(key=lambda a: (last_use.get((a, m), 0), self.lru_order(a)))
                        for a in free[:extra]:
                            if vf[a][0] == INF:
                                vf[a][0] = T + self.xfer(1)
                            vf[a][m] = INF
                arr, after = self.transfers(t, m, T, vf, free_at(m))
                if bus:
                    link_free[link(m)] = after
                for (R, C, _), x in zip(blocks(self.tasks[t]), arr):
                    for a in atoms(R, C, self.tasks[t][1], self.dmax):
                        if vf[a][m] == INF:
                            vf[a][m] = x
                for a in mine:
                    last_use[(a, m)] = T
                    pins[(a, m)] = pins.get((a, m), 0) + 1
                proc[t], start[t], finish[t] = p, ests[p], efts[p]
                avail[p] = efts[p]
                fifo[p].append(t)
            heads = [finish[f[0]] for f in fifo if f]
            if not heads:
                if ready:
                    return None
                break
            Tn = min(heads)
            for p in range(self.P):
                if fifo[p] and finish[fifo[p][0]] == Tn:
                    t = fifo[p].pop(0)
                    m = self.proc_mem[p]
                    for a in self.task_atoms(t):
                        pins[(a, m)] -= 1
                    for (R, C, w) in blocks(self.tasks[t]):
                        if w:
                            at = atoms(R, C, self.tasks[t][1], self.dmax)
                            home = Tn if m == 0 else Tn + self.xfer(len(at))
                            if bus and cache != "WB" and m != 0:
                                home = max(Tn, free_at(0)) + self.xfer(len(at))
                                link_free[link(0)] = home
                            for a in at:
                                copies = [INF] * self.n_mem
                                if cache == "WB" or (cache == "WT" and m != 0):
                                    copies[m] = Tn
                                if cache in ("WT", "WA"):
                                    copies[0] = home
                                vf[a] = copies
                    for v in self.succ[t]:
                        left[v] -= 1
                        if left[v] == 0:
                            ready.append(v)
                            released[v] = Tn
            T = Tn
        return max(finish), proc, start, finish


def brute_force_opt(sim: Sim, limit: int = 2_000_000) -> int:
    """Best makespan over every push-at-release schedule (task order x processor)."""
    import copy

    best = [INF]
    count = [0]

    def rec(state):
        count[0] += 1
        if count[0] > limit:
            raise RuntimeError("brute force too large")
        T, avail, vf, left, ready, fifo, finish = state
        if ready:
            for t in list(ready):
                for p in range(sim.P):
                    e = sim.est(t, p, T, avail, vf)
                    f = e + sim.cost[t][p]
                    if f >= best[0]:
                        continue
                    vf2 = {a: list(x) for a, x in vf.items()}
                    m = sim.proc_mem[p]
                    for (R, C, _) in blocks(sim.tasks[t]):
                        at = atoms(R, C, sim.tasks[t][1], sim.dmax)
                        miss = [a for a in at if vf2[a][m] == INF]
                        for a in miss:
                            vf2[a][m] = T + sim.xfer(len(miss))
                    av2 = list(avail)
                    av2[p] = f
                    fifo2 = [list(q) for q in fifo]
                    fifo2[p].append(t)
                    fin2 = dict(finish)
                    fin2[t] = f
                    r2 = [x for x in ready if x != t]
                    rec((T, av2, vf2, list(left), r2, fifo2, fin2))
            return
        heads = [finish[q[0]] for q in fifo if q]
        if not heads:
            best[0] = min(best[0], max(finish.values()))
            return
        Tn = min(heads)
        vf2 = {a: list(x) for a, x in vf.items()}
        left2 = list(left)
        fifo2 = [list(q) for q in fifo]
        r2 = []
        for p in range(sim.P):
            if fifo2[p] and finish[fifo2[p][0]] == Tn:
                t = fifo2[p].pop(0)
                m = sim.proc_mem[p]
                for (R, C, w) in blocks(sim.tasks[t]):
                    if w:
                        for a in atoms(R, C, sim.tasks[t][1], sim.dmax):
                            vf2[a] = [Tn if mm == m else INF for mm in range(sim.n_mem)]
                for v in sim.succ[t]:
                    left2[v] -= 1
                    if left2[v] == 0:
                        r2.append(v)
        rec((Tn, avail, vf2, left2, r2, fifo2, finish))

    vf0 = {}
    for t in sim.tasks:
        for (R, C, _) in blocks(t):
            for a in atoms(R, C, t[1], sim.dmax):
                vf0[a] = [0] + [INF] * (sim.n_mem - 1)
    left0 = list(sim.npred)
    rec((0, [0] * sim.P, vf0, left0, [t for t in range(sim.n) if left0[t] == 0],
         [[] for _ in range(sim.P)], {}))
    return best[0]
