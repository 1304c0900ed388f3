"""DAGs of depth 4 and 5 (block sides b/16 and b/32) on the GPU against the CPU
oracle: makespans, statuses and per-task schedules bit-exact for 16, 32 and 64
lanes per candidate, uniform and uneven batches, every heuristic class, caching
policy, link contention and finite memory spaces; platforms whose transfer
table is deeper than the kernels take by value; the seeded generators; and the
combinations that are refused."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)
W = I.WORKLOADS["chol16x16_b1024_d2"]       # its platform: 8 CPU cores + 2 accelerators


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


def _run(H, torch, plan, pf, host, policy=(0, 0, 0), sched=False):
    db = H.DeviceBatch.from_host(host)
    n = host.n
    ms = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    kw = {}
    if sched:
        cnt, _ = H.count_batch(db)
        off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        off[1:] = torch.cumsum(cnt.long(), 0)
        tot = int(off[-1].item())
        kw = dict(sched_off=off, proc=torch.full((tot,), -1, dtype=torch.int32, device="cuda"),
                  start=torch.full((tot,), -1, dtype=torch.int64, device="cuda"),
                  finish=torch.full((tot,), -1, dtype=torch.int64, device="cuda"))
    H.simulate_batch(plan, pf, db, ms, st, policy=policy, **kw)
    torch.cuda.synchronize()
    return ms.cpu().numpy(), st.cpu().numpy(), {k: v.cpu().numpy() for k, v in kw.items()}


@pytest.mark.parametrize("nt,dmax", [(6, 4), (8, 4), (4, 5), (6, 5)])
def test_parity_deep(H, torch, nt, dmax):
    """96 candidates with P(split) = 1/2 per level (about 3% reach depth 5) on
    the platform's tables of dmax levels, 16, 32 and 64 lanes and the tuned choice."""
    pf_in = W.platform()
    pf = H.Platform.from_inputs(pf_in, W.b, dmax)
    host = I.uniform_batch(W.seed, 96, nt, W.b, dmax, 1, 2, first=1_000 * dmax + nt)
    assert int(host.depth.max()) == dmax
    print(f"deep: nt {nt}, dmax {dmax}, 96 candidates", flush=True)
    want, _ = O.simulate_batch(pf_in, host, NTHREADS)
    for group in (16, 32, 64, 0):
        ms, st, _ = _run(H, torch, H.Plan(group=group), pf, host)
        assert (st == 0).all(), group
        assert np.array_equal(ms, want), group


def test_schedules_deep(H, torch):
    pf_in = W.platform()
    nt, dmax = 4, 5
    pf = H.Platform.from_inputs(pf_in, W.b, dmax)
    host = I.uniform_batch(W.seed, 6, nt, W.b, dmax, 2, 3, first=77)
    print("deep: per-task schedules, dmax 5", flush=True)
    _, st, kw = _run(H, torch, H.Plan(), pf, host, sched=True)
    assert (st == 0).all()
    off = kw["sched_off"]
    for c in range(host.n):
        dep = host.depth[host.mask_off[c]:host.mask_off[c + 1]]
        s = O.simulate(pf_in, nt, dmax, W.b, dep)
        tasks, _, _ = H.expand(nt, dmax, dep)
        want = {tuple(int(x) for x in s.tasks[t]): (int(s.proc[t]), int(s.start[t]), int(s.finish[t]))
                for t in range(s.n_tasks)}
        assert len(tasks) == s.n_tasks
        for t in range(len(tasks)):
            k = tuple(int(x) for x in tasks[t])
            g = off[c] + t
            assert want[k] == (int(kw["proc"][g]), int(kw["start"][g]), int(kw["finish"][g])), (c, k)


@pytest.mark.parametrize("policy", [(1, 1, 0, 0, 0), (0, 2, 0, 7, 0), (1, 3, 0, 0, 0), (0, 0, 1, 0, 1),
                                    (0, 0, 2, 0, 0), (0, 0, 1, 0, 2)])
def test_policies_deep(H, torch, policy):
    """(order, select, cache, seed, contention): FCFS/EIT-P, R-P, FCFS/F-P,
    write-through on one interconnect, write-around, write-through with a link
    per memory space; nt 6 at depth 4."""
    pf_in = W.platform()
    nt, dmax = 6, 4
    order, select, cache, seed, bus = policy
    link = np.arange(pf_in.n_mem, dtype=np.int32) if bus == 2 else None
    pf = H.Platform.from_inputs(pf_in, W.b, dmax, link=link)
    host = I.uniform_batch(W.seed, 64, nt, W.b, dmax, 1, 2, first=500)
    print(f"deep: policy {policy}", flush=True)
    want, _ = O.simulate_batch(pf_in, host, NTHREADS, policy=(order, select, seed, cache, min(bus, 1)), link=link)
    ms, st, _ = _run(H, torch, H.Plan(), pf, host, policy=(order, select, cache, seed, min(bus, 1)))
    assert (st == 0).all()
    assert np.array_equal(ms, want)


def test_deep_tables_with_shallow_candidates(H, torch):
    """Tables of 5 levels (4^5 + 1 transfer times) for candidates of depth <= 2:
    a transfer of m blocks of side b/4 reads entry 64 m of the device copy (16, 32
    and 64 lanes), and a second platform's table replaces the copy."""
    pf_in = W.platform()
    host = I.uniform_batch(W.seed, 128, 8, W.b, 2, 3, 10, first=900)
    want, _ = O.simulate_batch(pf_in, host, NTHREADS)
    plan = H.Plan()
    pf5 = H.Platform.from_inputs(pf_in, W.b, 5)
    print("deep: 5-level tables, depth-2 candidates", flush=True)
    for group in (16, 32, 64):
        ms, st, _ = _run(H, torch, H.Plan(group=group), pf5, host)
        assert (st == 0).all() and np.array_equal(ms, want), group
    ms, _, _ = _run(H, torch, plan, pf5, host)
    assert np.array_equal(ms, want)
    other = I.make_platform(I.cpu_accel_types(8, 2), seed=W.seed + 1)
    other.bw_bytes_per_ns = 6
    ms, _, _ = _run(H, torch, plan, H.Platform.from_inputs(other, W.b, 4), host)
    assert np.array_equal(ms, O.simulate_batch(other, host, NTHREADS)[0])


def test_ragged_deep_and_generators(H, torch):
    """Uneven shapes (4..10 tiles, depth caps 0..5) drawn on the GPU equal the
    seeded host generator, and their makespans the oracle's."""
    pf_in = W.platform()
    thr = I.split_threshold(1, 2)
    db = H.generate_ragged(W.seed, 11, 160, 4, 10, 5, thr)
    host = I.ragged_batch(W.seed, 160, 4, 10, 5, W.b, 1, 2, first=11)
    torch.cuda.synchronize()
    assert np.array_equal(db.dmax_arr.cpu().numpy(), host.dmax)
    assert np.array_equal(db.depth.cpu().numpy()[:host.mask_off[-1]], host.depth)
    assert int(host.depth.max()) == 5
    du = H.generate_uniform(W.seed, 3, 64, 8, 5, thr)
    torch.cuda.synchronize()
    assert np.array_equal(du.depth.cpu().numpy(), I.uniform_batch(W.seed, 64, 8, W.b, 5, 1, 2, first=3).depth)
    pf = H.Platform.from_inputs(pf_in, W.b, 5)
    print("deep: ragged, 160 candidates", flush=True)
    n = host.n
    ms = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    H.simulate_batch(H.Plan(), pf, db, ms, st)
    torch.cuda.synchronize()
    assert bool((st == 0).all().item())
    assert np.array_equal(ms.cpu().numpy(), O.simulate_batch(pf_in, host, NTHREADS)[0])


def test_deep_refusals(H, torch):
    pf_in = W.platform()
    host = I.uniform_batch(W.seed, 8, 4, W.b, 4, 1, 2, first=5)
    db = H.DeviceBatch.from_host(host)
    ms = torch.empty(8, dtype=torch.int64, device="cuda")
    st = torch.empty(8, dtype=torch.int32, device="cuda")
    pf = H.Platform.from_inputs(pf_in, W.b, 4)
    with pytest.raises(RuntimeError, match="fused pipeline takes depths and platform levels up to 3"):
        H.simulate_batch(H.Plan(group=64, fuse=True), pf, db, ms, st)
    with pytest.raises(RuntimeError, match="at most 3 levels"):
        H.simulate_batch_noalloc(pf, db, ms, st)
    with pytest.raises(RuntimeError, match="bad problem shape"):
        H.search(H.Plan(), pf, 4, 6, H.SEARCH_RANDOM, rounds=1, batch=16, seed=1)
    with pytest.raises(Exception):
        H.generate_tree_uniform(1, 0, 4, 4, 6, 1000)       # split depth above 5
    # a ragged candidate above the batch's stated maximum depth fails alone
    rag = I.ragged_batch(W.seed, 32, 4, 6, 4, W.b, 1, 2, first=40)
    full = H.DeviceBatch.from_host(rag)
    dbr = H.DeviceBatch(full.n_cand, full.nt, 3, full.depth, full.nt_arr, full.dmax_arr, full.mask_off)
    bad = rag.dmax > 3
    assert bad.any() and (~bad).any()
    ms = torch.full((32,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((32,), 99, dtype=torch.int32, device="cuda")
    H.simulate_batch(H.Plan(), H.Platform.from_inputs(pf_in, W.b, 4), dbr, ms, st)
    torch.cuda.synchronize()
    st, ms = st.cpu().numpy(), ms.cpu().numpy()
    assert (st[bad] == H.HESP_EINVAL).all() and (ms[bad] == -1).all()
    assert (st[~bad] == 0).all()
    assert np.array_equal(ms[~bad], O.simulate_batch(pf_in, rag.subset(np.nonzero(~bad)[0]), NTHREADS)[0])


def test_graph_replay_deep(H, torch):
    """A fixed-capacity plan captured on a 5-level platform (the transfer table
    copied by an eager call first) replays equal to eager calls."""
    pf_in = W.platform()
    pf = H.Platform.from_inputs(pf_in, W.b, 5)
    thr = I.split_threshold(1, 2)
    n = 256
    batches = [H.generate_uniform(W.seed, 20_000 + r * n, n, 6, 5, thr) for r in range(3)]
    cap_t = cap_e = 0
    for b in batches:
        nt_, ne_ = H.count_batch(b)
        cap_t, cap_e = max(cap_t, int(nt_.max())), max(cap_e, int(ne_.max()))
    dep = torch.empty_like(batches[0].depth)
    dep.copy_(batches[0].depth)
    db = H.DeviceBatch(n, 6, 5, dep)
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = H.Plan(max_tasks=cap_t, max_edges=cap_e, group=16)
    print("deep: graph capture", flush=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        H.simulate_batch(plan, pf, db, ms, st)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        H.simulate_batch(plan, pf, db, ms, st)
    ms2 = torch.empty_like(ms)
    st2 = torch.empty_like(st)
    for r in (1, 2):
        dep.copy_(batches[r].depth)
        g.replay()
        torch.cuda.synchronize()
        H.simulate_batch(H.Plan(), pf, batches[r], ms2, st2)
        torch.cuda.synchronize()
        assert bool((st == 0).all().item())
        assert torch.equal(ms, ms2), r
    host = I.uniform_batch(W.seed, 32, 6, W.b, 5, 1, 2, first=20_000 + 2 * n)
    assert np.array_equal(ms[:32].cpu().numpy(), O.simulate_batch(pf_in, host, NTHREADS)[0])


@pytest.mark.parametrize("nt,dmax,blocks,n", [(4, 4, 400, 32), (4, 4, 1200, 32), (3, 5, 1500, 16)])
def test_capacity_deep(H, torch, nt, dmax, blocks, n):
    """Finite accelerator spaces holding `blocks` finest blocks (side b / 2^dmax)
    with candidates of depth 4 and 5: 64 lanes, statuses and makespans bit-exact,
    and the capacity binds."""
    pf_in = W.platform()
    cap = np.zeros(pf_in.n_mem, np.int64)
    cap[1:] = blocks * pf_in.elem_bytes * (W.b >> dmax) ** 2
    pf = H.Platform.from_inputs(pf_in, W.b, dmax, capacity_bytes=cap)
    host = I.uniform_batch(W.seed, n, nt, W.b, dmax, 1, 2, first=60 + dmax)
    print(f"deep: capacity {blocks} blocks, nt {nt}, dmax {dmax}", flush=True)
    want, _, wst = O.simulate_batch(pf_in, host, NTHREADS, capacity=cap, statuses=True)
    ms, st, _ = _run(H, torch, H.Plan(), pf, host)
    assert np.array_equal(st, wst) and (st == 0).all()
    assert np.array_equal(ms, want)
    assert (want != O.simulate_batch(pf_in, host, NTHREADS)[0]).sum() >= n // 2
