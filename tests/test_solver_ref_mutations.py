"""Planted mistakes in the iterative-solver reference (oracle/solver_ref.py): each
must make at least one of its pins fail (run on the CPU, on copies of the module)."""
import importlib.util
import os
import sys

import numpy as np
import pytest

from oracle import solver_ref as S_ok
from paper_1602_05510_amd import inputs as I

SRC = S_ok.__file__

MUTANTS = {
    "avail_without_own_processor": ("        avail = P - running + 1\n", "        avail = P - running\n"),
    "estimate_rounded_down": ("            est = -(-work // lanes)\n", "            est = work // lanes\n"),
    "width_not_per_outer_step": ("            par = max(1, sum(cnt) >> dn)\n", "            par = max(1, sum(cnt))\n"),
    "ptype_of_last_task": ("        pt[c] = int(pf.proc_type[proc[first]])\n",
                           "        pt[c] = int(pf.proc_type[proc[idx[-1]]])\n"),
    "critical_path_earliest_predecessor": ("            t = last(preds[t])\n        cand = sorted(on)\n",
                                           "            t = min(preds[t], key=lambda y: (int(finish[y]), int(proc[y])))\n"
                                           "        cand = sorted(on)\n"),
    "tree_critical_path_first_predecessor": ("            t = last(preds[t])\n        cand = [x for x",
                                             "            t = preds[t][0]\n        cand = [x for x"),
    "hard_ties_to_largest_cluster": ("        return max(best, key=lambda x: (x[2], -x[0]))\n",
                                     "        return max(best, key=lambda x: (x[2], x[0]))\n"),
    "soft_scans_from_the_last": ("    acc = 0\n    for x in best:\n", "    acc = 0\n    for x in reversed(best):\n"),
    "shallow_takes_deepest": ("        dm = int(min(depth))\n", "        dm = int(max(depth))\n"),
    "tree_merge_estimate_next_level": ("            est, action = int(cost[pt, kind, l]), 0\n",
                                       "            est, action = int(cost[pt, kind, l + 1]), 0\n"),
    "tree_split_keeps_children_flags": ("            flags[pos[(l + 1, ch)]] = 0\n", "            pass\n"),
}


def _load(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/present"
    path = os.path.join(tmp_path, f"solver_{name}.py")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"solver_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _pins_pass(S):
    """The pins of tests/test_solver_ref_pins.py (hand-derived trajectories and
    choices, the depth-one equivalence of the two solvers, the critical path and
    Shallow lists, the tree moves' task counts), run on module S."""
    from oracle import oracle as O
    try:
        two = I.make_platform([I.ProcType("cpu", 2, 32000, 32000, 64, False)], seed=0)
        bd, bm, tr, steps = S.solve(two, 1, 1, 512, 5, 0, 0)
        if tr != [1419947, 1485484, 1419947, 1485484, 1419947]:
            return False
        if steps != [(0, 1, 677205), (0, 0, 65537), (0, 1, 677205), (0, 0, 65537), (0, 1, 677205)]:
            return False
        four = I.make_platform([I.ProcType("cpu", 4, 32000, 32000, 64, False)], seed=0)
        if S.solve(four, 1, 1, 512, 2, 0, 0)[3] != [(0, 1, 677205), (0, 0, 65537)]:
            return False
        acc = I.make_platform([I.ProcType("cpu", 1, 32000, 32000, 64, False),
                               I.ProcType("acc", 1, 1024000, 1024000, 512, True)], seed=0)
        if S.solve(acc, 1, 1, 512, 4, 0, 0)[2] != [272145] * 4:
            return False
        # the chain: Hard and Soft choices
        if S.solve(two, 2, 1, 512, 1, 0, 0)[3] != [(1, 1, 2031616)]:
            return False
        ends, scores = [677205, 2708821, 4740437, 5417642], [677205, 2031616, 2031616, 677205]
        for seed in range(12):
            u = S._draw(seed, 10, 0) % 5417642
            want = next(c for c in range(4) if u < ends[c])
            if S.solve(two, 2, 1, 512, 1, 0, 1, seed)[3][0] != (want, 1, scores[want]):
                return False
        # critical path and Shallow lists
        eight = I.make_platform([I.ProcType("cpu", 8, 32000, 32000, 64, False)], seed=0)
        dep = np.zeros(10, np.uint8)
        s = O.simulate(eight, 3, 0, 512, dep, detail=True)
        kinds, index = S._kind_of_top(3)
        cl = [index[(int(K) >> int(l), int(i) >> int(l), int(j) >> int(l))] for (_, l, K, i, j) in s.tasks]
        if S.candidates(10, dep, s, cl, 1) != [0, 1, 3, 7, 8, 9]:
            return False
        dep2 = dep.copy(); dep2[[0, 4]] = 1
        if S.candidates(10, dep2, s, cl, 2) != [1, 2, 3, 5, 6, 7, 8, 9]:
            return False
        # split trees: the hand-derived merge, the depth-one equivalence, task counts
        one = I.make_platform([I.ProcType("cpu", 1, 32000, 32000, 64, False)], seed=0)
        if S.solve_tree(one, 1, 2, 512, 3, 0, 0, flags0=np.array([1, 1, 0, 0, 0], np.uint8))[3] != \
                [(0, 0, 98305), None, None]:
            return False
        w = I.WORKLOADS["chol16x16_b1024_d2"]
        pf = w.platform()
        bt = I.uniform_batch(8, 2, 5, w.b, 1, 1, 2)
        for lst in (0, 1):
            for r in range(2):
                a = S.solve(pf, 5, 1, w.b, 8, lst, 1, 4 + r, depth0=bt.candidate(r))
                b = S.solve_tree(pf, 5, 1, w.b, 8, lst, 1, 4 + r,
                                 flags0=I.tree_flags_from_depth(5, 1, bt.candidate(r)))
                if a[2] != b[2]:
                    return False
        fl = I.tree_batch(12, 1, 4, w.b, 2, 1, 2).depth.copy()
        nodes = S._tree_nodes(4, 2)
        steps = S.solve_tree(pf, 4, 2, w.b, 12, 0, 1, 5, flags0=fl)[3]
        cur = fl.copy()
        n_prev = O.simulate(pf, 4, 2, w.b, cur, tree=True).n_tasks
        for st in steps:
            if st is None:
                continue
            x, action, _ = st
            lv, cell, kind = nodes[x]
            before = O.simulate(pf, 4, 2, w.b, cur, tree=True)
            under = sum(1 for (_, l, K, i, j) in before.tasks if int(l) >= lv and
                        (int(K) >> (int(l) - lv), int(i) >> (int(l) - lv), int(j) >> (int(l) - lv)) == cell)
            S.apply_tree_step(4, 2, cur, st)
            n_now = O.simulate(pf, 4, 2, w.b, cur, tree=True).n_tasks
            if action == 1 and (under != 1 or n_now != n_prev + {0: 4, 1: 6, 2: 6, 3: 8}[kind] - 1):
                return False
            if action == 0 and n_now != n_prev - under + 1:
                return False
            n_prev = n_now
    except (ValueError, KeyError, IndexError, ZeroDivisionError, StopIteration):
        return False
    return True


def test_reference_solver_passes():
    assert _pins_pass(S_ok)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    S = _load(str(tmp_path), name, old, new)
    assert not _pins_pass(S), f"planted mistake '{name}' went unnoticed"
