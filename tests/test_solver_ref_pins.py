"""Pins of the CPU reference of the iterative scheduler-partitioner
(oracle/solver_ref.py; section 2.1, "Iterative solver", with the readings
stated in that module)."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import solver_ref as S
from paper_1602_05510_amd import inputs as I


def test_hand_derived_split_and_merge():
    """Two identical CPUs, one 512 tile, depths 0..1.
    Depth 0: one chol, 0..1,419,947; span 1,419,947; one processor busy at its
    start, so 2 - 1 + 1 = 2 available.  Depth 1: 2 chol (185,686) + trsm +
    syrk (557,056 each) = 1,485,484 of work over min(2, 4 >> 1 = 2) lanes ->
    742,742; score 1,419,947 - 742,742 = 677,205 > 0: split.  The split cluster
    is a 4-task chain, 1,485,484 long; merging back estimates 1,419,947 over
    min(2, 1) lane, score 65,537: merge.  The solver oscillates and keeps the
    unsplit partition."""
    pf = I.make_platform([I.ProcType("cpu", 2, 32000, 32000, 64, False)], seed=0)
    bd, bm, tr, steps = S.solve(pf, 1, 1, 512, 5, 0, 0)
    assert tr == [1419947, 1485484, 1419947, 1485484, 1419947]
    assert steps == [(0, 1, 677205), (0, 0, 65537), (0, 1, 677205), (0, 0, 65537), (0, 1, 677205)]
    assert list(bd) == [0] and bm == 1419947


def test_fixed_point_when_no_positive_score():
    """A CPU and an accelerator, one 512 tile: the chol runs on the accelerator
    (87,382 after a 184,763 transfer, span 87,382); split, 2 x 27,307 + 2 x
    81,920 = 218,454 over 2 lanes = 109,227 > 87,382: no candidate."""
    pf = I.make_platform([I.ProcType("cpu", 1, 32000, 32000, 64, False),
                          I.ProcType("acc", 1, 1024000, 1024000, 512, True)], seed=0)
    bd, bm, tr, steps = S.solve(pf, 1, 1, 512, 4, 0, 0)
    assert tr == [272145] * 4 and steps == [None] * 4 and bm == 272145


def test_trace_is_the_simulation_of_each_partition():
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    for lst in (0, 1, 2):
        bd, bm, tr, steps = S.solve(pf, 6, 2, 1024, 8, lst, 0)
        dep = np.zeros(I.tet(6), np.uint8)
        for it in range(8):
            assert tr[it] == O.simulate(pf, 6, 2, 1024, dep, detail=False)
            if steps[it] is not None:
                c, dn, score = steps[it]
                assert score > 0 and dep[c] != dn and 0 <= dn <= 2
                if lst == 2:
                    assert dep[c] == dep.min()          # Shallow: only the shallowest clusters
                dep[c] = dn
        assert bm == min(tr)
        assert O.simulate(pf, 6, 2, 1024, bd, detail=False) == bm


def test_soft_sampling_depends_on_the_seed_only():
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    a = S.solve(pf, 6, 2, 1024, 10, 0, 1, seed=5)
    b = S.solve(pf, 6, 2, 1024, 10, 0, 1, seed=5)
    c = S.solve(pf, 6, 2, 1024, 10, 0, 1, seed=6)
    assert a[2] == b[2] and a[3] == b[3]
    assert a[3] != c[3]


def test_splitmix64_published_sequence():
    """SplitMix64 from state 0 (gamma increments, then the finaliser) gives
    0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F: the values of
    the published generator for seed 0."""
    st = 0
    out = []
    for _ in range(3):
        st = (st + S._GAMMA) & S._M64
        out.append(S._mix(st))
    assert out == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_lanes_are_bounded_by_the_outer_loop_width():
    """Four identical CPUs: all four are available, but the split chol runs at
    most 4 tasks >> 1 = 2 per outer step, so the estimate stays 742,742 and the
    score 677,205 (four lanes would give 1,048,576)."""
    pf = I.make_platform([I.ProcType("cpu", 4, 32000, 32000, 64, False)], seed=0)
    bd, bm, tr, steps = S.solve(pf, 1, 1, 512, 2, 0, 0)
    assert steps == [(0, 1, 677205), (0, 0, 65537)]


def test_critical_path_follows_the_last_arriving_dependence():
    """nt = 3 on eight identical CPUs, nothing split.  With chol < trsm = syrk
    and gemm = 2 syrk, the (1,2) update gemm(0,1,2) (start after both trsm,
    length 2 t) outlasts chol(1) (after trsm and syrk: c + t + s + c), so the
    path from chol(2) runs syrk(1,2,2) <- trsm(1,1,2) <- gemm(0,1,2) <- trsm(0,0,1)
    (both trsm finish together; trsm(0,0,1) was mapped first, to processor 0)
    <- chol(0): Fig. 1 clusters 9, 8, 7, 3, 1, 0.  Following the earliest
    predecessor instead would pass through chol(1) (cluster 6)."""
    pf = I.make_platform([I.ProcType("cpu", 8, 32000, 32000, 64, False)], seed=0)
    dep = np.zeros(10, np.uint8)
    s = O.simulate(pf, 3, 0, 512, dep, detail=True)
    kinds, index = S._kind_of_top(3)
    cl = [index[(int(K) >> int(l), int(i) >> int(l), int(j) >> int(l))] for (_, l, K, i, j) in s.tasks]
    assert S.candidates(10, dep, s, cl, 1) == [0, 1, 3, 7, 8, 9]
    assert S.candidates(10, dep, s, cl, 0) == list(range(10))
    dep2 = dep.copy(); dep2[[0, 4]] = 1
    assert S.candidates(10, dep2, s, cl, 2) == [1, 2, 3, 5, 6, 7, 8, 9]


# ---------------------------------------------------------------- split-tree partitions

@pytest.mark.parametrize("lst", [0, 1])
@pytest.mark.parametrize("sampling", [0, 1])
def test_tree_solver_is_the_cluster_solver_at_depth_one(lst, sampling):
    """With dmax = 1 the nodes are the top-level clusters, a split is depth 1 and
    a merge depth 0: both solvers take the same steps (Shallow differs only once
    every cluster is split, so it is left out)."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    bt = I.uniform_batch(8, 3, 5, w.b, 1, 1, 2)
    for r in range(3):
        d0 = bt.candidate(r)
        a = S.solve(pf, 5, 1, w.b, 10, lst, sampling, 4 + r, depth0=d0)
        b = S.solve_tree(pf, 5, 1, w.b, 10, lst, sampling, 4 + r, flags0=I.tree_flags_from_depth(5, 1, d0))
        assert a[2] == b[2]
        assert [x if x is None else (x[0], x[1], x[2]) for x in a[3]] == b[3]


def test_tree_solver_hand_derived_merge():
    """One CPU, one 512 tile, the chol split and its first level-1 chol split
    again (seven tasks in a chain, 1,518,252 ns).  Node 0 (the whole chol) merged
    back would take 1,419,947: score 98,305; node 1 (the level-1 chol, tasks
    0..218,454) merged: 218,454 - 185,686 = 32,768; the level-1 leaves would only
    lose by splitting (one lane: trsm 4 x 81,920 + 2 x 163,840 = 655,360 >
    557,056).  Hard merges node 0; the unsplit chol is then a fixed point."""
    pf1 = I.make_platform([I.ProcType("cpu", 1, 32000, 32000, 64, False)], seed=0)
    flags = np.array([1, 1, 0, 0, 0], np.uint8)
    bf, bm, tr, steps = S.solve_tree(pf1, 1, 2, 512, 3, 0, 0, flags0=flags)
    assert tr == [1518252, 1419947, 1419947]
    assert steps == [(0, 0, 98305), None, None]
    assert list(bf) == [0, 1, 0, 0, 0] and bm == 1419947
    # Shallow: only the level-1 leaves, none of which gains
    assert S.solve_tree(pf1, 1, 2, 512, 1, 2, 0, flags0=flags)[3] == [None]


def test_tree_solver_trace_and_moves():
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    nodes = S._tree_nodes(4, 2)
    for lst in (0, 1, 2):
        bf, bm, tr, steps = S.solve_tree(pf, 4, 2, w.b, 8, lst, 1, 2)
        fl = np.zeros(I.tree_flag_count(4, 2), np.uint8)
        for it in range(8):
            assert tr[it] == O.simulate(pf, 4, 2, w.b, fl, detail=False, tree=True)
            if steps[it] is not None:
                x, action, score = steps[it]
                assert score > 0 and fl[x] != action
                S.apply_tree_step(4, 2, fl, steps[it])
        assert bm == min(tr)


def test_hard_and_soft_choice_on_a_chain():
    """nt = 2, nothing split, two identical CPUs: the four tasks form a chain.
    Scores (split to depth 1, two lanes each): chol 1,419,947 - 742,742 =
    677,205; trsm 4,259,840 - ceil(4 x 557,056 + 2 x 1,114,112) / 2) =
    2,031,616; syrk the same; chol(1) 677,205; sum 5,417,642.  Hard takes the
    trsm (tie with the syrk, lower cluster); Soft takes the first cluster whose
    running sum (677,205 / 2,708,821 / 4,740,437 / 5,417,642) exceeds
    u = draw(seed, 10, 0) mod 5,417,642."""
    pf = I.make_platform([I.ProcType("cpu", 2, 32000, 32000, 64, False)], seed=0)
    hard = S.solve(pf, 2, 1, 512, 1, 0, 0)
    assert hard[2] == [11359574] and hard[3] == [(1, 1, 2031616)]
    ends = [677205, 2708821, 4740437, 5417642]
    scores = [677205, 2031616, 2031616, 677205]
    seen = set()
    for seed in range(24):
        u = S._draw(seed, 10, 0) % 5417642
        want = next(c for c in range(4) if u < ends[c])
        got = S.solve(pf, 2, 1, 512, 1, 0, 1, seed)[3][0]
        assert got == (want, 1, scores[want]), seed
        seen.add(want)
    assert seen == {0, 1, 2, 3}


def test_tree_moves_change_the_task_count_as_stated():
    """A split replaces a leaf by its 2 x 2 blocked algorithm (4, 6 or 8 tasks,
    all leaves); a merge replaces everything under a node by one task."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    fl = I.tree_batch(12, 1, 4, w.b, 2, 1, 2).depth.copy()    # stale flags under leaves included
    nodes = S._tree_nodes(4, 2)
    bf, bm, tr, steps = S.solve_tree(pf, 4, 2, w.b, 12, 0, 1, 5, flags0=fl)
    cur = fl.copy()
    n_prev = O.simulate(pf, 4, 2, w.b, cur, tree=True).n_tasks
    kinds_fine = {0: 4, 1: 6, 2: 6, 3: 8}
    moved = 0
    for st in steps:
        if st is None:
            continue
        x, action, _ = st
        lv, cell, kind = nodes[x]
        s_before = O.simulate(pf, 4, 2, w.b, cur, tree=True)
        under = sum(1 for (_, l, K, i, j) in s_before.tasks
                    if int(l) >= lv and
                    (int(K) >> (int(l) - lv), int(i) >> (int(l) - lv), int(j) >> (int(l) - lv)) == cell)
        S.apply_tree_step(4, 2, cur, st)
        n_now = O.simulate(pf, 4, 2, w.b, cur, tree=True).n_tasks
        if action == 1:
            assert under == 1 and n_now == n_prev + kinds_fine[kind] - 1
        else:
            assert n_now == n_prev - under + 1
        n_prev = n_now
        moved += 1
    assert moved >= 6
