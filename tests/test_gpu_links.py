"""GPU parity of link contention over a topology (each memory space names the
link of the transfers into it; one transfer at a time per link; section 2,
network topology) against the CPU oracle: makespans and per-task schedules
bit-exact under every caching policy and heuristic class, for 16, 32 and 64
lanes per candidate, split trees, the fused pipeline, and the 20-processor,
five-space platform of the 64x64 workload."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
NTHREADS = min(16, os.cpu_count() or 1)
HEURISTICS = [(0, 0, 0), (1, 1, 0), (0, 2, 7), (1, 3, 0)]   # (order, select, seed)


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


def _run(H, torch, pf, host, heur, cache, link_bus=1, group=0, fuse=False, sched=False, tree=False):
    n = host.n
    ms = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    pol = (heur[0], heur[1], cache, heur[2], link_bus)
    kw = {}
    if tree:
        H.simulate_tree_batch(H.Plan(group=group), pf, H.TreeBatch.from_host(host), ms, st, policy=pol)
    else:
        db = H.DeviceBatch.from_host(host)
        if sched:
            cnt, _ = H.count_batch(db)
            off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
            off[1:] = torch.cumsum(cnt.long(), 0)
            tot = int(off[-1].item())
            kw = dict(sched_off=off, proc=torch.full((tot,), -1, dtype=torch.int32, device="cuda"),
                      start=torch.full((tot,), -1, dtype=torch.int64, device="cuda"),
                      finish=torch.full((tot,), -1, dtype=torch.int64, device="cuda"))
        H.simulate_batch(H.Plan(group=group, fuse=fuse), pf, db, ms, st, policy=pol, **kw)
    torch.cuda.synchronize()
    assert bool((st == 0).all().item())
    return ms.cpu().numpy(), {k: v.cpu().numpy() for k, v in kw.items()}


def _topologies(n_mem):
    """each space on its own link; the host alone and the accelerators behind one
    switch; the accelerators in pairs with the host on the first pair's link"""
    own = np.arange(n_mem, dtype=np.int32)
    switch = np.array([0] + [1] * (n_mem - 1), np.int32)
    pairs = np.array([0] + [1 + (m - 1) // 2 for m in range(1, n_mem)], np.int32)
    pairs[0] = pairs[1] if n_mem > 1 else 0
    return {"own": own, "switch": switch, "pairs": pairs}


@pytest.mark.parametrize("cache", [0, 1, 2])
@pytest.mark.parametrize("heur", HEURISTICS)
def test_parity_16x16(H, torch, heur, cache):
    """8x8 tiles of 1024, depths 0..2, on 8 CPU cores + 2 accelerators: each
    space on a link of its own, 96 candidates, 16 and 64 lanes."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    lk = _topologies(pf_in.n_mem)["own"]
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, link=lk)
    host = I.uniform_batch(w.seed, 96, 8, w.b, w.dmax, w.p_num, w.p_den, first=600 + 7 * cache)
    print(f"links: 16x16 platform, heuristic {heur}, cache {cache}", flush=True)
    want, _ = O.simulate_batch(pf_in, host, NTHREADS, policy=heur + (cache, 1), link=lk)
    shared, _ = O.simulate_batch(pf_in, host, NTHREADS, policy=heur + (cache, 1))
    assert (want != shared).sum() >= 8, "the links must matter"
    for group in (16, 64):
        got, _ = _run(H, torch, pf, host, heur, cache, group=group)
        assert np.array_equal(got, want), group


@pytest.mark.parametrize("topo", ["own", "switch", "pairs"])
def test_parity_five_spaces(H, torch, topo):
    """The 64x64 workload's platform (16 CPU cores + 4 accelerators, five
    spaces) on 16x16 tiles of 1024 at depths 0..3, write-through, 24 candidates."""
    w = I.WORKLOADS["chol64x64_b1024_d3"]
    pf_in = w.platform()
    lk = _topologies(pf_in.n_mem)[topo]
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, link=lk)
    host = I.uniform_batch(w.seed, 24, 16, w.b, w.dmax, w.p_num, w.p_den, first=40)
    print(f"links: five spaces, topology {topo} {list(lk)}", flush=True)
    want, _ = O.simulate_batch(pf_in, host, NTHREADS, policy=(0, 0, 0, 1, 1), link=lk)
    got, _ = _run(H, torch, pf, host, (0, 0, 0), 1)
    assert np.array_equal(got, want)


def test_schedules_ragged_trees_and_fused(H, torch):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    lk = _topologies(pf_in.n_mem)["switch"]
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, link=lk)
    # per-task schedules, write-around
    host = I.uniform_batch(w.seed, 8, 6, w.b, w.dmax, w.p_num, w.p_den, first=70)
    print("links: schedules", flush=True)
    _, kw = _run(H, torch, pf, host, (0, 0, 0), 2, sched=True)
    off = kw["sched_off"]
    for c in range(host.n):
        dep = host.depth[host.mask_off[c]:host.mask_off[c + 1]]
        s = O.simulate(pf_in, 6, w.dmax, w.b, dep, policy=(0, 0, 0, 2, 1), link=lk)
        tasks, _, _ = H.expand(6, w.dmax, dep)
        want = {tuple(int(x) for x in s.tasks[t]): (int(s.proc[t]), int(s.start[t]), int(s.finish[t]))
                for t in range(s.n_tasks)}
        for t in range(len(tasks)):
            k = tuple(int(x) for x in tasks[t])
            g = off[c] + t
            assert want[k] == (int(kw["proc"][g]), int(kw["start"][g]), int(kw["finish"][g])), (c, k)
    # split trees
    tb = I.tree_batch(43, 64, 6, w.b, 2, 1, 3)
    print("links: split trees", flush=True)
    want, _ = O.simulate_batch(pf_in, tb, NTHREADS, policy=(0, 0, 0, 1, 1), tree=True, link=lk)
    got, _ = _run(H, torch, pf, tb, (0, 0, 0), 1, tree=True)
    assert np.array_equal(got, want)
    # the fused pipeline
    host = I.uniform_batch(w.seed, 128, 8, w.b, w.dmax, w.p_num, w.p_den, first=800)
    print("links: fused pipeline", flush=True)
    want, _ = O.simulate_batch(pf_in, host, NTHREADS, policy=(1, 1, 0, 1, 1), link=lk)
    got, _ = _run(H, torch, pf, host, (1, 1, 0), 1, group=64, fuse=True)
    assert np.array_equal(got, want)
    # without contention the links are ignored
    got, _ = _run(H, torch, pf, host, (0, 0, 0), 0, link_bus=0)
    assert np.array_equal(got, O.simulate_batch(pf_in, host, NTHREADS)[0])


def test_link_worked_example_on_gpu(H, torch):
    with open(os.path.join(GOLD, "link_examples.json")) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        pf_in = I.make_platform([I.ProcType(n, c, r, r, h, own) for (n, c, r, h, own) in e["platform"]["types"]],
                                seed=0)
        pf = H.Platform.from_inputs(pf_in, e["b"], e["dmax"], link=e["link"])
        bt = I.Batch(e["b"], np.array([e["nt"]], np.int32), np.array([e["dmax"]], np.int32),
                     np.array([0, I.tet(e["nt"])], np.int64), np.array(e["depth"], np.uint8))
        order, select, seed, cache, bus = e["policy"]
        for group in (16, 32, 64):
            got, _ = _run(H, torch, pf, bt, (order, select, seed), cache, group=group)
            assert int(got[0]) == e["makespan"], (e["name"], group)


def test_bad_links_are_refused(H, torch):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    host = w.batch(4)
    db = H.DeviceBatch.from_host(host)
    ms = torch.empty(4, dtype=torch.int64, device="cuda")
    st = torch.empty(4, dtype=torch.int32, device="cuda")
    for bad in ([0, 1, 3], [0, -1, 0]):
        pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, link=bad)
        with pytest.raises(RuntimeError, match="link"):
            H.simulate_batch(H.Plan(), pf, db, ms, st, policy=(0, 0, 0, 0, 1))
    with pytest.raises(RuntimeError, match="link needs"):
        H.Platform.from_inputs(pf_in, w.b, w.dmax, link=[0, 1])
