"""Pins of the split-tree partitions (any task split again on its own; section
2.1, "Recursive task partitioners") in the CPU oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I
import pyoracle as PY


def _pf():
    return I.WORKLOADS["chol4x4_b512_d1"].platform()


@pytest.mark.parametrize("nt,dmax", [(1, 1), (2, 1), (3, 2), (4, 2), (3, 3), (2, 4), (1, 5)])
def test_uniform_trees_equal_per_cluster_depths(nt, dmax):
    """Flags that split every task under a top-level task down to its depth
    give exactly the per-cluster partition: same tasks, edges and schedule."""
    pf = _pf()
    rng = np.random.default_rng(10 * nt + dmax)
    for _ in range(4):
        dep = rng.integers(0, dmax + 1, I.tet(nt)).astype(np.uint8)
        a = O.simulate(pf, nt, dmax, 512, dep)
        b = O.simulate(pf, nt, dmax, 512, I.tree_flags_from_depth(nt, dmax, dep), tree=True)
        assert a.makespan == b.makespan and a.n_tasks == b.n_tasks and len(a.edges) == len(b.edges)
        ka = {tuple(int(x) for x in a.tasks[t]): (a.proc[t], a.start[t], a.finish[t]) for t in range(a.n_tasks)}
        kb = {tuple(int(x) for x in b.tasks[t]): (b.proc[t], b.start[t], b.finish[t]) for t in range(b.n_tasks)}
        assert ka == kb


def test_hand_derived_partial_split():
    """One 512 tile, depths 0..2: the chol is split, and of its four level-1
    tasks only the first chol again.  Tasks in program order: chol, trsm, syrk,
    chol at level 2 (the top-left 256 block), then trsm, syrk, chol at level 1.
    The level-1 trsm reads the whole top-left 256 block, last written by the
    level-2 chol(0), trsm(0,1) and chol(1); everything else is a chain, so the
    transitively reduced DAG is the chain of the seven tasks and on one CPU the
    makespan is the sum of their times."""
    flags = np.array([1, 1, 0, 0, 0], np.uint8)      # level 0: the chol; level 1: chol(0), trsm, syrk, chol(1)
    pf1 = I.make_platform([I.ProcType("cpu", 1, 32000, 32000, 64, False)], seed=0)
    s = O.simulate(pf1, 1, 2, 512, flags, tree=True)
    want = [(0, 2, 0, 0, 0), (1, 2, 0, 0, 1), (2, 2, 0, 1, 1), (0, 2, 1, 1, 1),
            (1, 1, 0, 0, 1), (2, 1, 0, 1, 1), (0, 1, 1, 1, 1)]
    assert [tuple(int(x) for x in t) for t in s.tasks] == want
    edges = {(int(u), int(v)) for u, v in s.edges}
    chain = {(t, t + 1) for t in range(6)}
    assert chain <= edges
    assert edges - chain == {(0, 4), (1, 4)}                # trsm@1 also reads atoms last written by tasks 0, 1
    times = [PY.task_time(k, 512 >> l, 32000, 64) for (k, l, *_rest) in want]
    assert s.makespan == sum(times)
    # 128: R = 32,000 * 128^2 / (128^2 + 64^2) = 25,600 MFLOP/s -> chol ceil(699,050.7 / 25.6) = 27,307,
    # trsm / syrk 2,097,152 / 25.6 = 81,920; 256: trsm / syrk 557,056, chol 185,686
    assert times == [27307, 81920, 81920, 27307, 557056, 557056, 185686]
    assert s.makespan == 1_518_252           # 2 x 27,307 + 2 x 81,920 + 2 x 557,056 + 185,686


def test_flags_below_the_last_level_are_ignored_and_values_checked():
    pf = _pf()
    # dmax = 0: no flags at all, the unsplit problem
    s0 = O.simulate(pf, 3, 0, 512, np.zeros(0, np.uint8), tree=True)
    assert s0.makespan == O.simulate(pf, 3, 0, 512, np.zeros(10, np.uint8)).makespan
    # flags of cells whose ancestors are not split have no effect
    fl = np.zeros(I.tree_flag_count(2, 2), np.uint8)
    fl[4:] = 1                                              # level-1 flags only; nothing at level 0 is split
    assert O.simulate(pf, 2, 2, 512, fl, tree=True).makespan == O.simulate(pf, 2, 2, 512, np.zeros(4, np.uint8)).makespan
    with pytest.raises(ValueError):
        O.simulate(pf, 2, 2, 512, np.full(I.tree_flag_count(2, 2), 2, np.uint8), tree=True)


def test_python_reading_agrees_on_trees():
    """The independent Python reading of the split-tree expansion gives the same
    tasks, edges and schedules on random trees."""
    rng = np.random.default_rng(55)
    plats = [I.make_platform(I.cpu_accel_types(2, 1), seed=11), I.make_platform(I.big_little_types(2, 2), seed=12)]
    for trial in range(24):
        pf = plats[trial % 2]
        nt = int(rng.integers(1, 4))
        dmax = int(rng.integers(1, 4)) if nt < 3 else int(rng.integers(1, 3))
        fl = (rng.random(I.tree_flag_count(nt, dmax)) < 0.4).astype(np.uint8)
        s = O.simulate(pf, nt, dmax, 256, fl, tree=True)
        py = PY.Sim(nt, dmax, 256, fl, pf.proc_type, pf.proc_mem, pf.n_mem, pf.rmax, pf.h, pf.shared_memory, tree=True)
        assert [tuple(t[:5]) for t in py.tasks] == [tuple(int(x) for x in r) for r in s.tasks]
        assert py.E == sorted((int(u), int(v)) for u, v in s.edges)
        ms, proc, start, finish = py.run()
        assert ms == s.makespan and list(s.proc) == proc and list(s.start) == start


def test_tree_batch_generator_marginals():
    bt = I.tree_batch(3, 64, 4, 512, 2, 1, 4)
    assert bt.depth.size == 64 * I.tree_flag_count(4, 2) and set(np.unique(bt.depth)) <= {0, 1}
    assert abs(bt.depth.mean() - 0.25) < 0.02
