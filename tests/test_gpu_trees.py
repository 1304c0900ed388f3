"""GPU parity of split-tree candidates (any task split again on its own; section
2.1, "Recursive task partitioners") against the CPU oracle through the C ABI:
makespans, counts and per-task schedules bit-exact."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu
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


def _run(H, torch, pf_in, batch, policy=(0, 0, 0), sched=False, group=0, plan=None):
    pf = H.Platform.from_inputs(pf_in, batch.b, int(batch.dmax[0]))
    tb = H.TreeBatch.from_host(batch)
    n = batch.n
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    ntk = torch.empty(n, dtype=torch.int32, device="cuda")
    kw = {}
    if sched:
        cnt, _ = H.count_tree_batch(tb)
        off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        off[1:] = torch.cumsum(cnt.long(), 0)
        tot = int(off[-1].item())
        kw = dict(sched_off=off, proc=torch.empty(tot, dtype=torch.int32, device="cuda"),
                  start=torch.empty(tot, dtype=torch.int64, device="cuda"),
                  finish=torch.empty(tot, dtype=torch.int64, device="cuda"))
    H.simulate_tree_batch(plan or H.Plan(group=group), pf, tb, ms, st, policy=policy, n_tasks=ntk, **kw)
    torch.cuda.synchronize()
    return ms.cpu().numpy(), st.cpu().numpy(), ntk.cpu().numpy(), kw


@pytest.mark.parametrize("name,nt,dmax,n", [("chol4x4_b512_d1", 4, 1, 512), ("chol4x4_b512_d1", 4, 2, 256),
                                            ("chol4x4_b512_d1", 3, 3, 96), ("chol16x16_b1024_d2", 8, 2, 96),
                                            ("chol4x4_b512_d1", 3, 4, 48), ("chol16x16_b1024_d2", 2, 5, 32)])
def test_parity_random_trees(H, torch, name, nt, dmax, n):
    w = I.WORKLOADS[name]
    pf = w.platform()
    bt = I.tree_batch(w.seed + nt, n, nt, w.b, dmax, 1, 3)
    want, ntk_want = O.simulate_batch(pf, bt, NTHREADS, tree=True)
    for group in (16, 64) if pf.n_procs <= 16 else (32, 64):
        got, st, ntk, _ = _run(H, torch, pf, bt, group=group)
        assert (st == 0).all()
        assert np.array_equal(ntk, ntk_want)
        assert np.array_equal(got, want), (name, nt, dmax, group)


def test_uniform_trees_equal_depth_candidates(H, torch):
    """Flags that split whole clusters reproduce hesp_simulate_batch's results."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax = 8, 2
    bt = I.uniform_batch(w.seed, 64, nt, w.b, dmax, 1, 3)
    flags = np.concatenate([I.tree_flags_from_depth(nt, dmax, bt.candidate(c)) for c in range(bt.n)])
    nf = I.tree_flag_count(nt, dmax)
    tb = I.Batch(w.b, bt.nt.copy(), bt.dmax.copy(), np.arange(bt.n + 1, dtype=np.int64) * nf, flags)
    got_tree, st, _, _ = _run(H, torch, pf_in, tb)
    pf = H.Platform.from_inputs(pf_in, w.b, dmax)
    db = H.DeviceBatch.from_host(bt)
    ms = torch.empty(bt.n, dtype=torch.int64, device="cuda")
    st2 = torch.empty(bt.n, dtype=torch.int32, device="cuda")
    H.simulate_batch(H.Plan(), pf, db, ms, st2)
    assert (st == 0).all() and np.array_equal(got_tree, ms.cpu().numpy())


def test_uniform_trees_equal_depth_candidates_at_depth_five(H, torch):
    """Depth-5 flags that split whole clusters reproduce hesp_simulate_batch's
    results (walk and last-writer scan on block sides down to b/32)."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax = 3, 5
    bt = I.uniform_batch(w.seed, 24, nt, w.b, dmax, 1, 2, first=70)
    assert int(bt.depth.max()) == 5
    flags = np.concatenate([I.tree_flags_from_depth(nt, dmax, bt.candidate(c)) for c in range(bt.n)])
    nf = I.tree_flag_count(nt, dmax)
    tb = I.Batch(w.b, bt.nt.copy(), bt.dmax.copy(), np.arange(bt.n + 1, dtype=np.int64) * nf, flags)
    got_tree, st, _, _ = _run(H, torch, pf_in, tb)
    want, _ = O.simulate_batch(pf_in, bt, NTHREADS)
    assert (st == 0).all() and np.array_equal(got_tree, want)


def test_generator_matches_host_draws(H, torch):
    for nt, dmax in ((4, 2), (16, 2), (3, 3), (3, 5)):
        thr = I.split_threshold(1, 3)
        tb = H.generate_tree_uniform(9, 1000, 20, nt, dmax, thr)
        host = I.tree_batch(9, 20, nt, 512, dmax, 1, 3, first=1000)
        assert np.array_equal(tb.flags.cpu().numpy()[:host.depth.size], host.depth)


def test_counts_and_per_task_schedules(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = I.tree_batch(21, 16, 4, w.b, 2, 1, 2)
    tb = H.TreeBatch.from_host(bt)
    cnt, ne = H.count_tree_batch(tb)
    _, _, _, kw = _run(H, torch, pf, bt, sched=True)
    off = kw["sched_off"].cpu().numpy()
    proc, start, finish = (kw[k].cpu().numpy() for k in ("proc", "start", "finish"))
    for c in range(bt.n):
        s = O.simulate(pf, 4, 2, w.b, bt.candidate(c), tree=True)
        assert int(cnt[c].item()) == s.n_tasks and int(ne[c].item()) == len(s.edges)
        # both number the tasks in program order (Fig. 1 order, children of a
        # split task in the loop order of its 2 x 2 sub-tiling)
        for t in range(s.n_tasks):
            assert (int(proc[off[c] + t]), int(start[off[c] + t]), int(finish[off[c] + t])) == \
                (int(s.proc[t]), int(s.start[t]), int(s.finish[t])), (c, t, tuple(int(x) for x in s.tasks[t]))


@pytest.mark.parametrize("policy", [(1, 1, 0, 0), (0, 2, 0, 5), (0, 3, 2, 0), (0, 0, 1, 0)])
def test_trees_under_other_policies(H, torch, policy):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = I.tree_batch(33, 128, 4, w.b, 2, 1, 3)
    order, select, cache, seed = policy
    want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=(order, select, seed, cache), tree=True)
    got, st, _, _ = _run(H, torch, pf, bt, policy=policy)
    assert (st == 0).all() and np.array_equal(got, want)


def test_edge_cases(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    # dmax = 0: no flags, the unsplit problem
    pf_lib = H.Platform.from_inputs(pf, w.b, 1)
    import torch as T
    ms = T.empty(1, dtype=T.int64, device="cuda")
    st = T.empty(1, dtype=T.int32, device="cuda")
    H.simulate_tree_batch(H.Plan(), pf_lib, H.TreeBatch(1, 5, 0, None), ms, st)
    assert int(st.item()) == 0
    assert int(ms.item()) == O.simulate(pf, 5, 0, w.b, np.zeros(I.tet(5), np.uint8), detail=False)
    # a flag above 1 fails its candidate only; all-split flags reach every level
    nf = I.tree_flag_count(3, 2)
    fl = np.zeros((3, nf), np.uint8)
    fl[1, 7] = 2
    fl[2, :] = 1
    bt = I.Batch(w.b, np.full(3, 3, np.int32), np.full(3, 2, np.int32), np.arange(4, dtype=np.int64) * nf,
                 fl.reshape(-1))
    got, stt, ntk, _ = _run(H, torch, pf, bt)
    assert list(stt) == [0, -1, 0] and got[1] == -1
    assert got[0] == O.simulate(pf, 3, 2, w.b, fl[0], detail=False, tree=True)
    assert got[2] == O.simulate(pf, 3, 2, w.b, np.full(I.tet(3), 2, np.uint8), detail=False)
    assert ntk[2] == I.tet(12)


def test_trees_critical_time_reread_path(H, torch):
    """Split-tree preparation shares the critical-time pass: with an LDS budget of
    one internal dependence per run the re-read path gives the same makespans."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    bt = I.tree_batch(w.seed + 3, 48, 6, w.b, 2, 1, 3)
    want, _ = O.simulate_batch(pf, bt, NTHREADS, tree=True)
    got, st, _, _ = _run(H, torch, pf, bt, plan=H.Plan(prep_edges=1))
    assert (st == 0).all() and np.array_equal(got, want)
