"""Link contention over a network topology (section 2: the platform's memory
spaces are connected according to a network topology; no model is given).

Reading: every memory space names the link that carries the transfers into it;
a link carries one transfer at a time, in issue order (the missing blocks of a
task in their order; copies sent to the host at a completion use the host's
link); the EFT-P estimate sees each link's queue.  One link for every space is
the shared interconnect.

Pins: one link for all equals the shared interconnect; link ids are labels
(renaming them changes nothing); without contention the links are ignored; a
separately written Python reading (tests/pyoracle.py) agrees on every schedule;
a hand-derived schedule (tests/golden/link_examples.json); out-of-range ids are
refused."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I
import pyoracle as PY

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KIND = {"chol": 0, "trsm": 1, "syrk": 2, "gemm": 3}
SELECT_NAMES = ["EFT", "EIT", "RP", "FP"]
CACHE_NAMES = ["WB", "WT", "WA"]
PLATS = [I.make_platform(I.cpu_accel_types(2, 1), seed=7),
         I.make_platform(I.cpu_accel_types(3, 2), seed=8),
         I.make_platform(I.cpu_accel_types(1, 3), seed=9)]


def _tet(nt):
    return nt * (nt + 1) * (nt + 2) // 6


def _case(rng, trial):
    pf = PLATS[trial % 3]
    nt, dmax = int(rng.integers(1, 5)), int(rng.integers(0, 3))
    dep = rng.integers(0, dmax + 1, _tet(nt)).astype(np.uint8)
    return pf, nt, dmax, dep


def _links(rng, n_mem):
    return rng.integers(0, n_mem, n_mem).astype(np.int32)


def _same(a, b):
    return a.makespan == b.makespan and list(a.proc) == list(b.proc) and list(a.start) == list(b.start) \
        and list(a.finish) == list(b.finish)


def test_link_worked_example():
    with open(os.path.join(GOLD, "link_examples.json")) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        pf = I.make_platform([I.ProcType(n, c, r, r, h, own) for (n, c, r, h, own) in e["platform"]["types"]],
                             seed=0)
        dep = np.array(e["depth"], np.uint8)
        s = O.simulate(pf, e["nt"], e["dmax"], e["b"], dep, policy=tuple(e["policy"]), link=e["link"])
        assert s.makespan == e["makespan"], e["name"]
        got = {tuple(int(x) for x in s.tasks[t]): (int(s.proc[t]), int(s.start[t]), int(s.finish[t]))
               for t in range(s.n_tasks)}
        for (kind, lvl, K, I_, J, p, st, fi) in e["schedule"]:
            assert got[(KIND[kind], lvl, K, I_, J)] == (p, st, fi), (e["name"], kind, K, I_, J)
        # the derivation's remark: on one shared link trsm02 goes to p0
        sh = O.simulate(pf, e["nt"], e["dmax"], e["b"], dep, policy=tuple(e["policy"]))
        t = [tuple(int(x) for x in sh.tasks[u]) for u in range(sh.n_tasks)].index((1, 0, 0, 0, 2))
        assert [int(sh.proc[t]), int(sh.start[t]), int(sh.finish[t])] == e["shared_link_trsm02"]


@pytest.mark.parametrize("cache", [0, 1, 2])
def test_one_link_for_all_is_the_shared_interconnect(cache):
    rng = np.random.default_rng(700 + cache)
    for trial in range(24):
        pf, nt, dmax, dep = _case(rng, trial)
        pol = (trial % 2, [0, 1, 3][trial % 3], 0, cache, 1)
        a = O.simulate(pf, nt, dmax, 256, dep, policy=pol)
        b = O.simulate(pf, nt, dmax, 256, dep, policy=pol, link=np.full(pf.n_mem, trial % pf.n_mem))
        assert _same(a, b), trial


def test_link_ids_are_labels():
    """Renaming the links (a permutation of the ids) changes no schedule."""
    rng = np.random.default_rng(710)
    for trial in range(30):
        pf, nt, dmax, dep = _case(rng, trial)
        lk = _links(rng, pf.n_mem)
        perm = rng.permutation(pf.n_mem).astype(np.int32)
        pol = (trial % 2, 0, 0, trial % 3, 1)
        a = O.simulate(pf, nt, dmax, 256, dep, policy=pol, link=lk)
        b = O.simulate(pf, nt, dmax, 256, dep, policy=pol, link=perm[lk])
        assert _same(a, b), trial


def test_links_without_contention_change_nothing():
    rng = np.random.default_rng(720)
    for trial in range(12):
        pf, nt, dmax, dep = _case(rng, trial)
        a = O.simulate(pf, nt, dmax, 256, dep, policy=(0, 0, 0, trial % 3, 0))
        b = O.simulate(pf, nt, dmax, 256, dep, policy=(0, 0, 0, trial % 3, 0), link=_links(rng, pf.n_mem))
        assert _same(a, b), trial


@pytest.mark.parametrize("cache", [0, 1, 2])
@pytest.mark.parametrize("policy", [(0, 0), (1, 1), (0, 3)])
def test_python_reading_agrees_on_links(policy, cache):
    rng = np.random.default_rng(730 + 10 * cache + 4 * policy[0] + policy[1])
    differs = 0
    for trial in range(16):
        pf, nt, dmax, dep = _case(rng, trial)
        lk = _links(rng, pf.n_mem)
        s = O.simulate(pf, nt, dmax, 256, dep, policy=policy + (0, cache, 1), link=lk)
        py = PY.Sim(nt, dmax, 256, dep, pf.proc_type, pf.proc_mem, pf.n_mem, pf.rmax, pf.h, pf.shared_memory)
        ms, proc, start, finish = py.run(order=["PL", "FCFS"][policy[0]], select=SELECT_NAMES[policy[1]],
                                         cache=CACHE_NAMES[cache], bus=True, links=[int(x) for x in lk])
        assert ms == s.makespan, trial
        assert list(s.proc) == proc and list(s.start) == start and list(s.finish) == finish, trial
        differs += O.simulate(pf, nt, dmax, 256, dep, policy=policy + (0, cache, 1)).makespan != ms
    assert differs >= 2, "the links must matter in some of the cases"


def test_link_ids_out_of_range_are_refused():
    pf = PLATS[1]
    dep = np.zeros(_tet(2), np.uint8)
    for bad in ([0, 1, pf.n_mem], [0, -1, 0]):
        lk = np.array(bad + [0] * (pf.n_mem - len(bad)), np.int32)[:pf.n_mem]
        with pytest.raises(ValueError):
            O.simulate(pf, 2, 0, 256, dep, policy=(0, 0, 0, 0, 1), link=lk)
