"""Finite accelerator memory spaces (section 2, problem input: memory spaces of
finite size; accelerator spaces cache the host): pins of the oracle's reading.

Reading: a space holds at most floor(capacity / block bytes) whole finest
blocks; a task goes only to a processor whose space can hold the blocks of the
tasks mapped there and not finished plus its own (EFT-P among those); room is
made by dropping the least recently used other blocks (ties: upper-triangle
tiles row by row, then row-major inside the tile), a block without a host copy
being copied back first, one transfer per finest block issued at the mapping.

Pins: capacities that can never bind give the unbounded schedules; capacities
below one block give the schedules of the platform without the accelerators;
a second implementation written separately (tests/pyoracle.py) agrees on every
schedule; hand-derived schedules (tests/golden/capacity_examples.json); and a
task no space can hold fails with the capacity status."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I
import pyoracle as PY

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KIND = {"chol": 0, "trsm": 1, "syrk": 2, "gemm": 3}


def _tet(nt):
    return nt * (nt + 1) * (nt + 2) // 6


def _block_bytes(pf, b, dmax):
    return pf.elem_bytes * (b >> dmax) ** 2


def _cap(pf, blocks, b, dmax):
    """capacity in bytes of `blocks` finest blocks in every accelerator space"""
    c = np.zeros(pf.n_mem, np.int64)
    c[1:] = blocks * _block_bytes(pf, b, dmax)
    return c


def _py(pf, nt, dmax, b, depth):
    return PY.Sim(nt, dmax, b, depth, pf.proc_type, pf.proc_mem, pf.n_mem, pf.rmax, pf.h, pf.shared_memory)


PLATS = [I.make_platform(I.cpu_accel_types(2, 1), seed=7),
         I.make_platform(I.cpu_accel_types(3, 2), seed=8),
         I.make_platform(I.cpu_accel_types(1, 2), seed=9)]


def test_capacity_that_never_binds_changes_nothing():
    """A space as large as the whole matrix never evicts: same schedules."""
    rng = np.random.default_rng(41)
    for trial in range(30):
        pf = PLATS[trial % 3]
        nt, dmax = int(rng.integers(1, 6)), int(rng.integers(0, 3))
        dep = rng.integers(0, dmax + 1, _tet(nt)).astype(np.uint8)
        n_atoms = (nt * (nt + 1) // 2) << (2 * dmax)
        for order in (0, 1):
            a = O.simulate(pf, nt, dmax, 256, dep, policy=(order, 0))
            b = O.simulate(pf, nt, dmax, 256, dep, policy=(order, 0), capacity=_cap(pf, n_atoms, 256, dmax))
            assert a.makespan == b.makespan
            assert list(a.proc) == list(b.proc) and list(a.finish) == list(b.finish)


def test_capacity_below_one_block_drops_the_accelerators():
    """A space that cannot hold one finest block never takes a task: the
    schedules are those of the same platform without its accelerators (FCFS
    order, which does not depend on the processors; Priority-List's critical
    times sum the task time over every processor, the unused ones included)."""
    rng = np.random.default_rng(42)
    for trial in range(20):
        full = PLATS[trial % 3]
        n_cpu = full.ptypes[0].count
        cpus = I.make_platform([full.ptypes[0]], seed=0, rmax=full.rmax[:1])
        nt, dmax = int(rng.integers(1, 6)), int(rng.integers(0, 3))
        dep = rng.integers(0, dmax + 1, _tet(nt)).astype(np.uint8)
        cap = np.zeros(full.n_mem, np.int64)
        cap[1:] = _block_bytes(full, 256, dmax) - 1
        a = O.simulate(full, nt, dmax, 256, dep, policy=(1, 0), capacity=cap)
        b = O.simulate(cpus, nt, dmax, 256, dep, policy=(1, 0))
        assert a.makespan == b.makespan
        assert (a.proc < n_cpu).all()
        assert list(a.proc) == list(b.proc) and list(a.start) == list(b.start)


@pytest.mark.parametrize("order", [0, 1])
def test_python_reading_agrees_on_capacity(order):
    """The separately written Python reading gives the same schedules for
    capacities around the tasks' footprints, split partitions included."""
    rng = np.random.default_rng(60 + order)
    evicted_somewhere = 0
    for trial in range(40):
        pf = PLATS[trial % 3]
        nt, dmax = int(rng.integers(2, 5)), int(rng.integers(0, 3))
        dep = rng.integers(0, dmax + 1, _tet(nt)).astype(np.uint8)
        blocks = int(rng.integers(3, 4 ** dmax * 3 + 6))
        cap = _cap(pf, blocks, 256, dmax)
        py = _py(pf, nt, dmax, 256, dep).run(order=["PL", "FCFS"][order], capacity=list(cap))
        try:
            s = O.simulate(pf, nt, dmax, 256, dep, policy=(order, 0), capacity=cap)
        except ValueError:
            assert py is None     # both: no processor can take some task
            continue
        ms, proc, start, finish = py
        assert ms == s.makespan, trial
        assert list(s.proc) == proc and list(s.start) == start and list(s.finish) == finish, trial
        n_atoms = (nt * (nt + 1) // 2) << (2 * dmax)
        u = O.simulate(pf, nt, dmax, 256, dep, policy=(order, 0))
        evicted_somewhere += blocks < n_atoms and u.makespan != s.makespan
    assert evicted_somewhere >= 5, "the cases must exercise eviction"


def test_no_space_can_hold_a_task():
    """Accelerators only, each holding fewer blocks than a task needs: the
    candidate fails (status -4, makespan -1); one more block makes it run
    (tasks that find every space full of the blocks of unfinished tasks wait)."""
    pf = I.make_platform([I.ProcType("acc", 2, 1_000_000, 1_000_000, 512, True)], seed=0)
    nt, dmax = 3, 0
    dep = np.zeros(_tet(nt), np.uint8)
    cap2 = _cap(pf, 2, 512, dmax)          # a gemm touches three blocks
    with pytest.raises(ValueError):
        O.simulate(pf, nt, dmax, 512, dep, capacity=cap2)
    assert _py(pf, nt, dmax, 512, dep).run(capacity=list(cap2)) is None
    s = O.simulate(pf, nt, dmax, 512, dep, capacity=_cap(pf, 3, 512, dmax))
    assert s.makespan > 0


def test_batch_statuses_with_capacity():
    pf = I.make_platform([I.ProcType("acc", 2, 1_000_000, 1_000_000, 512, True)], seed=0)
    host = I.uniform_batch(3, 24, 3, 512, 1, 3, 10)
    cap = _cap(pf, 8, 512, 1)              # the unsplit gemm needs 12 finest blocks
    ms, ntk, st = O.simulate_batch(pf, host, 4, capacity=cap, statuses=True)
    for c in range(host.n):
        dep = host.depth[host.mask_off[c]:host.mask_off[c + 1]]
        py = _py(pf, 3, 1, 512, dep).run(capacity=list(cap))
        if py is None:
            assert st[c] == -4 and ms[c] == -1
        else:
            assert st[c] == 0 and ms[c] == py[0]
    assert (st == -4).any() and (st == 0).any()


def test_capacity_worked_examples():
    """Hand-derived schedules with finite spaces (tests/golden/capacity_examples.json)."""
    with open(os.path.join(GOLD, "capacity_examples.json")) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        pf = I.make_platform([I.ProcType(n, c, r, r, h, own) for (n, c, r, h, own) in e["platform"]["types"]],
                             seed=0)
        cap = np.array(e["capacity_bytes"], np.int64)
        s = O.simulate(pf, e["nt"], e["dmax"], e["b"], np.array(e["depth"], np.uint8), capacity=cap)
        assert s.makespan == e["makespan"], e["name"]
        got = {tuple(int(x) for x in s.tasks[t]): (int(s.proc[t]), int(s.start[t]), int(s.finish[t]))
               for t in range(s.n_tasks)}
        for (kind, lvl, K, I_, J, p, st, fi) in e["schedule"]:
            assert got[(KIND[kind], lvl, K, I_, J)] == (p, st, fi), (e["name"], kind, K, I_, J)
