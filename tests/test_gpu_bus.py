"""GPU parity of the shared-interconnect option (every transfer one at a time,
in issue order; section 2, link contention) against the CPU oracle: makespans and
per-task schedules bit-exact, with every caching policy and heuristic class."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
NTHREADS = min(16, os.cpu_count() or 1)
HEURISTICS = [(0, 0, 0), (1, 1, 0), (0, 2, 7), (0, 3, 0)]   # (order, select, seed)


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


@pytest.fixture(scope="module")
def H(torch):
    from paper_1602_05510_amd import hesp
    return hesp


def _run(H, torch, pf_in, batch, max_level, heur, cache, sched=False, group=0, tree=False):
    pf = H.Platform.from_inputs(pf_in, batch.b, max_level)
    n = batch.n
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    kw = {}
    pol = (heur[0], heur[1], cache, heur[2], 1)
    if tree:
        H.simulate_tree_batch(H.Plan(group=group), pf, H.TreeBatch.from_host(batch), ms, st, policy=pol)
    else:
        db = H.DeviceBatch.from_host(batch)
        if sched:
            ntk, _ = H.count_batch(db)
            off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
            off[1:] = torch.cumsum(ntk.long(), 0)
            tot = int(off[-1].item())
            kw = dict(sched_off=off, proc=torch.empty(tot, dtype=torch.int32, device="cuda"),
                      start=torch.empty(tot, dtype=torch.int64, device="cuda"),
                      finish=torch.empty(tot, dtype=torch.int64, device="cuda"))
        H.simulate_batch(H.Plan(group=group), pf, db, ms, st, policy=pol, **kw)
    torch.cuda.synchronize()
    assert bool((st == 0).all().item())
    return ms.cpu().numpy(), kw


@pytest.mark.parametrize("cache", [0, 1, 2])
@pytest.mark.parametrize("heur", HEURISTICS)
def test_parity_4x4_all_candidates(H, torch, heur, cache):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = w.batch(1024)
    want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=heur + (cache, 1))
    for group in (16, 64):
        got, _ = _run(H, torch, pf, bt, w.dmax, heur, cache, group=group)
        assert np.array_equal(got, want), (heur, cache, group)


@pytest.mark.parametrize("cache", [0, 2])
def test_parity_16x16_ragged_and_trees(H, torch, cache):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    bt = w.batch(192)
    want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=(0, 0, 0, cache, 1))
    got, _ = _run(H, torch, pf, bt, w.dmax, (0, 0, 0), cache)
    assert np.array_equal(got, want)
    wr = I.WORKLOADS["ragged_bl_b512_d3"]
    pfr = wr.platform()
    br = wr.batch(3000)
    sub = br.subset([c for c in range(br.n) if br.nt[c] <= 16][:200])
    want, _ = O.simulate_batch(pfr, sub, NTHREADS, policy=(0, 0, 0, cache, 1))
    got, _ = _run(H, torch, pfr, sub, wr.dmax, (0, 0, 0), cache)
    assert np.array_equal(got, want)
    tb = I.tree_batch(41, 96, 6, w.b, 2, 1, 3)
    want, _ = O.simulate_batch(pf, tb, NTHREADS, policy=(0, 0, 0, cache, 1), tree=True)
    got, _ = _run(H, torch, pf, tb, 2, (0, 0, 0), cache, tree=True)
    assert np.array_equal(got, want)


def test_per_task_schedules(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = w.batch(24)
    _, kw = _run(H, torch, pf, bt, w.dmax, (0, 0, 0), 1, sched=True)
    off = kw["sched_off"].cpu().numpy()
    proc, start, finish = (kw[k].cpu().numpy() for k in ("proc", "start", "finish"))
    for c in range(bt.n):
        s = O.simulate(pf, w.nt, w.dmax, w.b, bt.candidate(c), policy=(0, 0, 0, 1, 1))
        tasks, _, _ = H.expand(w.nt, w.dmax, bt.candidate(c))
        want = {tuple(int(x) for x in s.tasks[t]): (int(s.proc[t]), int(s.start[t]), int(s.finish[t]))
                for t in range(s.n_tasks)}
        for t in range(len(tasks)):
            k = tuple(int(x) for x in tasks[t])
            assert want[k] == (int(proc[off[c] + t]), int(start[off[c] + t]), int(finish[off[c] + t])), (c, k)


def test_bus_worked_examples_on_gpu(H, torch):
    with open(os.path.join(GOLD, "bus_examples.json")) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        pts = [I.ProcType(n, c, r, r, h, own) for (n, c, r, h, own) in e["platform"]["types"]]
        pf = I.make_platform(pts, seed=0)
        n_top = I.tet(e["nt"])
        bt = I.Batch(e["b"], np.array([e["nt"]], np.int32), np.array([e["dmax"]], np.int32),
                     np.array([0, n_top], np.int64), np.array(e["depth"], np.uint8))
        order, select, seed, cache, _ = e["policy"]
        got, _ = _run(H, torch, pf, bt, e["dmax"], (order, select, seed), cache)
        assert int(got[0]) == e["makespan"], e["name"]
