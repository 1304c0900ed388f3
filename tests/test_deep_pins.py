"""DAGs of depth 4 and 5 (block sides b/16 and b/32; section 3 reports best
partitions that deep): pins of the oracle and of the seeded depth generator.

Pins: per-parent task counts in closed form (a chol split d times is the loop
nest on 2^d x 2^d tiles: tet(2^d) tasks; trsm and syrk 4^d (2^d + 1) / 2; gemm
8^d); splitting every task d times equals the unsplit loop nest on nt 2^d tiles
of side b / 2^d (same tasks, edges and schedule); the flops of every expanded
candidate sum to n^3 / 3; on one processor the makespan is the sum of the task
times; the separately written Python reading agrees on every schedule; the
generator's depths follow P(depth >= d) = p^d and are those of the one-draw rule
up to depth 3."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I
import pyoracle as PY


def _tet(n):
    return n * (n + 1) * (n + 2) // 6


def _per_parent(kind, d):
    s = 1 << d
    return [_tet(s), s * s * (s + 1) // 2, s * s * (s + 1) // 2, s ** 3][kind]


def test_per_parent_counts_depth_4_and_5():
    assert [_per_parent(k, 4) for k in range(4)] == [816, 2176, 2176, 4096]
    assert [_per_parent(k, 5) for k in range(4)] == [5984, 16896, 16896, 32768]
    pf = I.make_platform([I.ProcType("cpu", 1, 32000, 32000, 64, False)], seed=0)
    tops = PY.fig1_tasks(3)
    for d in (4, 5):
        b = 16 << d
        base = O.simulate(pf, 3, d, b, np.zeros(10, np.uint8), detail=False)
        base_n = O.simulate(pf, 3, d, b, np.zeros(10, np.uint8)).n_tasks
        assert base_n == 10 and base > 0
        for t, (kind, _, _, _) in enumerate(tops):
            dep = np.zeros(10, np.uint8)
            dep[t] = d
            s = O.simulate(pf, 3, d, b, dep)
            assert s.n_tasks - base_n + 1 == _per_parent(kind, d)
            for k, _, K, I_, J in s.tasks:
                assert K <= I_ <= J and k == PY.kind_of(K, I_, J)


@pytest.mark.parametrize("nt,d", [(1, 4), (2, 4), (1, 5)])
def test_all_split_equals_homogeneous_deep(nt, d):
    pf = I.make_platform(I.cpu_accel_types(3, 2), seed=7)
    b = 1024
    dep = np.full(_tet(nt), d, np.uint8)
    s1 = O.simulate(pf, nt, d, b, dep)
    m = nt << d
    s0 = O.simulate(pf, m, 0, b >> d, np.zeros(_tet(m), np.uint8))
    assert s1.n_tasks == _tet(m) and s1.makespan == s0.makespan
    k1 = {tuple(int(x) for x in s1.tasks[t][2:]): t for t in range(s1.n_tasks)}
    k0 = {tuple(int(x) for x in s0.tasks[t][2:]): t for t in range(s0.n_tasks)}
    assert set(k1) == set(k0)
    e1 = {(tuple(s1.tasks[u][2:]), tuple(s1.tasks[v][2:])) for u, v in s1.edges}
    e0 = {(tuple(s0.tasks[u][2:]), tuple(s0.tasks[v][2:])) for u, v in s0.edges}
    assert e1 == e0
    for key, t1 in k1.items():
        t0 = k0[key]
        assert (s1.proc[t1], s1.start[t1], s1.finish[t1]) == (s0.proc[t0], s0.start[t0], s0.finish[t0])


def test_flops_and_single_processor_sum_deep():
    pf1 = I.make_platform([I.ProcType("cpu", 1, 27000, 27000, 64, False)], seed=0)
    rng = np.random.default_rng(5)
    for nt, d in [(2, 4), (3, 4), (2, 5)]:
        b = 32 << d
        for _ in range(3):
            dep = rng.integers(0, d + 1, _tet(nt)).astype(np.uint8)
            s = O.simulate(pf1, nt, d, b, dep)
            assert sum([1, 3, 3, 6][int(k)] * (b >> int(l)) ** 3 for k, l, *_ in s.tasks) == (nt * b) ** 3
            assert s.makespan == sum(PY.task_time(int(k), b >> int(l), 27000, 64) for k, l, *_ in s.tasks)


@pytest.mark.parametrize("cache", [0, 1])
def test_python_reading_agrees_deep(cache):
    rng = np.random.default_rng(90 + cache)
    plats = [I.make_platform(I.cpu_accel_types(2, 1), seed=1), I.make_platform(I.cpu_accel_types(1, 2), seed=2)]
    for trial in range(6):
        pf = plats[trial % 2]
        nt, d = (1, 5) if trial == 5 else (2, 4)
        dep = rng.integers(0, d + 1, _tet(nt)).astype(np.uint8)
        dep[rng.integers(0, _tet(nt))] = d
        if nt == 1:
            dep[:] = rng.integers(3, 6)
        s = O.simulate(pf, nt, d, 1024, dep, policy=(0, 0, 0, cache))
        py = PY.Sim(nt, d, 1024, dep, pf.proc_type, pf.proc_mem, pf.n_mem, pf.rmax, pf.h, pf.shared_memory)
        ms, proc, start, finish = py.run(cache=["WB", "WT"][cache])
        assert ms == s.makespan, trial
        assert list(s.proc) == proc and list(s.start) == start and list(s.finish) == finish, trial


def test_generator_depths_beyond_three():
    """P(depth >= d) = p^d up to dmax, each chunk an independent 21-bit draw;
    depths up to 3 do not depend on the second draw."""
    thr = I.split_threshold(3, 5)
    p = thr / 2 ** 21
    host = I.uniform_batch(17, 2048, 8, 1024, 5, 3, 5)
    dep = host.depth.astype(np.int64)
    n = dep.size
    for d in range(1, 6):
        frac = (dep >= d).mean()
        assert abs(frac - p ** d) < 5 * np.sqrt(p ** d * (1 - p ** d) / n) + 1e-9, d
    low = I.uniform_batch(17, 2048, 8, 1024, 3, 3, 5)
    assert np.array_equal(low.depth, np.minimum(host.depth, 3))
    assert (host.depth == 5).any()
