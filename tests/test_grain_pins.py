"""Grain batches: partition parameter p = 1/f for any integer f (section 2.1,
"Iterative solver": the new tasks depend on blocks of size p times the
original), so that blocks of two tasks split with non-divisible grains overlap
partially (section 2.1 data DAG, Fig. 4: such overlaps get an intersection
descriptor, a common child of the two blocks).

Reading: a tile is cut into L x L atoms, L = lcm of the factors in use; a block
of factor f is the union of its (L/f)^2 atoms, so an intersection descriptor is
the set of atoms the two blocks share, and validity, dependences and transfers
are tracked per atom as for power-of-two depths.

Pins (none of them re-types the oracle's arithmetic):
  * power-of-two factor lists reduce to the depth mode (itself pinned by
    hand-derived schedules): same schedule, every policy, with links;
  * one factor f for every task equals the flat loop nest on nt*f tiles of side
    b/f (a 3x3 or 6x6 tiling is the plain Fig. 1 algorithm at that tile count);
  * whole-tile tasks on an atom grid whose atom side is not an integer
    (b = 1024, L = 3) equal the unsplit depth-0 schedule;
  * the dependence edges equal a brute-force derivation in exact rational
    geometry (block rectangles cut at their own boundaries, no atom grid);
  * hand-derived predecessor sets of an intersection case
    (tests/golden/grain_examples.json);
  * one processor in one memory space: the makespan is the sum of the task
    times, each the depth-mode task time of side b/f."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I
import pyoracle as PY

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PLATS = [I.make_platform(I.cpu_accel_types(2, 1), seed=7),
         I.make_platform(I.cpu_accel_types(3, 2), seed=8),
         I.make_platform(I.cpu_accel_types(1, 3), seed=9)]
POLICIES = [(0, 0), (1, 0), (0, 1), (0, 2, 5), (0, 3), (0, 0, 0, 1), (0, 0, 0, 2), (0, 0, 0, 0, 1),
            (1, 1, 0, 1, 1)]


def _same(a, b):
    return (a.makespan == b.makespan and np.array_equal(a.tasks, b.tasks) and np.array_equal(a.proc, b.proc)
            and np.array_equal(a.start, b.start) and np.array_equal(a.finish, b.finish)
            and np.array_equal(a.rank, b.rank) and np.array_equal(a.edges, b.edges))


@pytest.mark.parametrize("trial", range(12))
def test_power_of_two_factors_are_the_depth_mode(trial):
    rng = np.random.default_rng(100 + trial)
    pf = PLATS[trial % 3]
    nt, dmax = int(rng.integers(1, 5)), int(rng.integers(0, 3))
    dep = rng.integers(0, dmax + 1, I.tet(nt)).astype(np.uint8)
    fac = [1 << l for l in range(dmax + 1)]
    pol = POLICIES[trial % len(POLICIES)]
    link = rng.integers(0, pf.n_mem, pf.n_mem).astype(np.int32) if trial % 2 else None
    a = O.simulate(pf, nt, dmax, 1024, dep, policy=pol, link=link)
    b = O.simulate_grain(pf, nt, fac, 1024, dep, policy=pol, link=link)
    assert _same(a, b)


def _flat_key(s):
    return sorted(zip(s.tasks[:, 0], s.tasks[:, 2], s.tasks[:, 3], s.tasks[:, 4],
                      s.proc, s.start, s.finish, s.rank))


@pytest.mark.parametrize("nt,f,pol", [(1, 3, (0, 0)), (2, 3, (0, 0)), (2, 3, (1, 1, 0, 1)), (1, 6, (0, 0)),
                                      (3, 3, (0, 3, 0, 2)), (2, 5, (0, 2, 11)), (2, 3, (0, 0, 0, 0, 1))])
def test_one_factor_is_the_flat_tiling(nt, f, pol):
    b = 1920                                  # divisible by 3, 5 and 6
    pf = PLATS[(nt + f) % 3]
    g = O.simulate_grain(pf, nt, [f], b, np.zeros(I.tet(nt), np.uint8), policy=pol)
    flat = O.simulate(pf, nt * f, 0, b // f, np.zeros(I.tet(nt * f), np.uint8), policy=pol)
    assert g.makespan == flat.makespan
    assert g.n_tasks == flat.n_tasks and len(g.edges) == len(flat.edges)
    assert _flat_key(g) == _flat_key(flat)


@pytest.mark.parametrize("nt", [1, 2, 3])
def test_whole_tiles_on_a_fractional_atom_grid(nt):
    pf = PLATS[nt % 3]
    a = O.simulate(pf, nt, 0, 1024, np.zeros(I.tet(nt), np.uint8))
    b = O.simulate_grain(pf, nt, [1, 3], 1024, np.zeros(I.tet(nt), np.uint8))
    assert _same(a, b)


# --- brute force in exact rational geometry ----------------------------------

def _bf_tasks(nt, fac, grain):
    out = []
    for t, (_, k, i, j) in enumerate(PY.fig1_tasks(nt)):
        f = fac[grain[t]]
        cells = [(K, Ii, J) for K in range(k * f, (k + 1) * f) for Ii in range(i * f, (i + 1) * f)
                 for J in range(j * f, (j + 1) * f) if K <= Ii <= J]
        cells.sort(key=lambda c: (c[0],) + PY._in_step_order(PY.kind_of(*c), *c))
        out += [(PY.kind_of(*c), int(grain[t]), c[0], c[1], c[2]) for c in cells]
    return out


def _bf_blocks(task, f):
    kind, _, K, Ii, J = task
    blk = {PY.CHOL: [(K, K, True)], PY.TRSM: [(K, K, False), (K, J, True)],
           PY.SYRK: [(K, Ii, False), (Ii, Ii, True)],
           PY.GEMM: [(K, Ii, False), (K, J, False), (Ii, J, True)]}[kind]
    return [((Fraction(R, f), Fraction(R + 1, f)), (Fraction(C, f), Fraction(C + 1, f)), w) for R, C, w in blk]


def _bf_edges(nt, fac, grain):
    tasks = _bf_tasks(nt, fac, grain)
    rects = [_bf_blocks(t, fac[t[1]]) for t in tasks]
    cuts = sorted({x for rs in rects for (r, c, _) in rs for x in (*r, *c)})
    last_w, readers, edges = {}, {}, set()
    for v, rs in enumerate(rects):
        for (r0, r1), (c0, c1), w in rs:
            rows = [(a, b) for a, b in zip(cuts, cuts[1:]) if r0 <= a and b <= r1]
            cols = [(a, b) for a, b in zip(cuts, cuts[1:]) if c0 <= a and b <= c1]
            for cell in ((x, y) for x in rows for y in cols):
                u = last_w.get(cell)
                if u is not None and u != v:
                    edges.add((u, v))
                if w:
                    edges.update((u2, v) for u2 in readers.get(cell, ()) if u2 != v)
                    readers[cell] = []
                    last_w[cell] = v
                else:
                    readers.setdefault(cell, []).append(v)
    return tasks, sorted(edges)


@pytest.mark.parametrize("trial", range(10))
def test_edges_equal_rational_brute_force(trial):
    rng = np.random.default_rng(700 + trial)
    nt = int(rng.integers(1, 4))
    fac = [[1, 2, 3], [1, 3], [2, 3], [1, 2, 3, 4], [1, 5, 2]][trial % 5]
    grain = rng.integers(0, len(fac), I.tet(nt)).astype(np.uint8)
    s = O.simulate_grain(PLATS[trial % 3], nt, fac, 1024, grain)
    tasks, edges = _bf_edges(nt, fac, grain)
    assert [tuple(int(x) for x in row) for row in s.tasks] == tasks
    assert sorted(map(tuple, s.edges.tolist())) == edges


def test_hand_derived_intersections():
    gold = json.load(open(os.path.join(GOLD, "grain_examples.json")))
    for case in gold["cases"]:
        s = O.simulate_grain(PLATS[0], case["nt"], case["fac"], 1024, np.array(case["grain"], np.uint8))
        assert s.n_tasks == case["n_tasks"]
        for v, preds in case["preds"].items():
            got = sorted(int(u) for u, w in s.edges.tolist() if w == int(v))
            assert got == preds, (v, got, preds)


def test_one_processor_sum_of_task_times():
    pf = I.make_platform([I.ProcType("cpu", 1, 1000, 2000, 64, False)], seed=3)
    assert pf.shared_memory
    fac, b, nt = [1, 2, 3, 4, 6], 1536, 3
    grain = np.array([4, 2, 1, 3, 0, 2, 1, 4, 3, 2], np.uint8)
    s = O.simulate_grain(pf, nt, fac, b, grain)
    want = sum(O.task_time(int(t[0]), b // fac[t[1]], int(pf.rmax[0, t[0]]), int(pf.h[0])) for t in s.tasks)
    assert s.makespan == want


def test_refusals():
    pf = PLATS[0]
    z = np.zeros(I.tet(2), np.uint8)
    for fac in ([], [0], [1, 65], [7, 11]):           # empty, zero, too fine, lcm 77 > 64
        with pytest.raises(ValueError):
            O.simulate_grain(pf, 2, fac, 1024, z)
    with pytest.raises(ValueError):
        O.simulate_grain(pf, 2, [1, 2], 1024, z + 2)   # grain index past the list


def test_grain_generator_uniform_and_seeded():
    a = I.grain_batch(5, 64, 4, 3)
    assert a.shape == (64, I.tet(4)) and a.dtype == np.uint8 and set(np.unique(a)) == {0, 1, 2}
    assert np.array_equal(a[10:20], I.grain_batch(5, 10, 4, 3, first=10))
    assert not np.array_equal(a, I.grain_batch(6, 64, 4, 3))
