"""GPU parity of the task orders (Priority-List, FCFS) and processor selections
(EFT-P, EIT-P, R-P, F-P) of section 2.1 against the CPU oracle: makespans and
per-task schedules bit-exact."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
KIND = {"chol": 0, "trsm": 1, "syrk": 2, "gemm": 3}
POLICIES = [(0, 0), (1, 0), (0, 1), (1, 1), (0, 2, 7), (1, 2, 7), (0, 3), (1, 3)]
NTHREADS = min(16, os.cpu_count() or 1)


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


def _run(H, torch, pf_in, batch, max_level, policy, sched=False, group=0):
    pf = H.Platform.from_inputs(pf_in, batch.b, max_level)
    db = H.DeviceBatch.from_host(batch)
    n = batch.n
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    kw = {}
    if sched:
        ntk, _ = H.count_batch(db)
        off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        off[1:] = torch.cumsum(ntk.long(), 0)
        tot = int(off[-1].item())
        kw = dict(sched_off=off, proc=torch.empty(tot, dtype=torch.int32, device="cuda"),
                  start=torch.empty(tot, dtype=torch.int64, device="cuda"),
                  finish=torch.empty(tot, dtype=torch.int64, device="cuda"))
    pol = (policy[0], policy[1], 0, policy[2] if len(policy) > 2 else 0)
    H.simulate_batch(H.Plan(group=group), pf, db, ms, st, policy=pol, **kw)
    torch.cuda.synchronize()
    assert bool((st == 0).all().item())
    return ms.cpu().numpy(), kw


@pytest.mark.parametrize("policy", POLICIES)
def test_parity_4x4_all_candidates(H, torch, policy):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = w.batch(1024)
    want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=policy)
    for group in (16, 64):
        got, _ = _run(H, torch, pf, bt, w.dmax, policy, group=group)
        assert np.array_equal(got, want), (policy, group)


@pytest.mark.parametrize("policy", POLICIES[1:])
def test_parity_16x16_and_ragged(H, torch, policy):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    bt = w.batch(192)
    want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=policy)
    got, _ = _run(H, torch, pf, bt, w.dmax, policy)
    assert np.array_equal(got, want)
    wr = I.WORKLOADS["ragged_bl_b512_d3"]
    pfr = wr.platform()
    br = wr.batch(3000)
    keep = [c for c in range(br.n) if br.nt[c] <= 16][:200]
    sub = br.subset(keep)
    want, _ = O.simulate_batch(pfr, sub, NTHREADS, policy=policy)
    got, _ = _run(H, torch, pfr, sub, wr.dmax, policy)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("policy", POLICIES[1:])
def test_per_task_schedules(H, torch, policy):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = w.batch(24)
    _, kw = _run(H, torch, pf, bt, w.dmax, policy, sched=True)
    off = kw["sched_off"].cpu().numpy()
    proc, start, finish = (kw[k].cpu().numpy() for k in ("proc", "start", "finish"))
    for c in range(bt.n):
        s = O.simulate(pf, w.nt, w.dmax, w.b, bt.candidate(c), policy=policy)
        tasks, _, _ = H.expand(w.nt, w.dmax, bt.candidate(c))
        want = {tuple(int(x) for x in s.tasks[t]): (int(s.proc[t]), int(s.start[t]), int(s.finish[t]))
                for t in range(s.n_tasks)}
        for t in range(len(tasks)):
            k = tuple(int(x) for x in tasks[t])
            assert want[k] == (int(proc[off[c] + t]), int(start[off[c] + t]), int(finish[off[c] + t])), (c, k)


def test_policy_worked_examples_on_gpu(H, torch):
    with open(os.path.join(GOLD, "policy_examples.json")) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        pts = [I.ProcType(n, c, r, r, h, own) for (n, c, r, h, own) in e["platform"]["types"]]
        pf = I.make_platform(pts, seed=0)
        n_top = I.tet(e["nt"])
        bt = I.Batch(e["b"], np.array([e["nt"]], np.int32), np.array([e["dmax"]], np.int32),
                     np.array([0, n_top], np.int64), np.array(e["depth"], np.uint8))
        got, _ = _run(H, torch, pf, bt, e["dmax"], e["policy"])
        assert int(got[0]) == e["makespan"], e["name"]


def test_random_choice_seed_changes_schedules(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = w.batch(256)
    a, _ = _run(H, torch, pf, bt, w.dmax, (0, 2, 1))
    b, _ = _run(H, torch, pf, bt, w.dmax, (0, 2, 2))
    assert not np.array_equal(a, b)
    want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=(0, 2, 2))
    assert np.array_equal(b, want)


def test_waiting_on_one_processor(H, torch):
    """One CPU: with R-P / F-P every release waits for the CPU; the makespan is the
    sum of the task times and the schedule matches the oracle task by task."""
    pf = I.make_platform([I.ProcType("cpu", 1, 30000, 30000, 64, False)], seed=0)
    bt = I.WORKLOADS["chol4x4_b512_d1"].batch(64)
    for pol in ((0, 3), (1, 3), (0, 2, 5)):
        want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=pol)
        for group in (16, 64):
            got, _ = _run(H, torch, pf, bt, 1, pol, group=group)
            assert np.array_equal(got, want), (pol, group)
