"""Finite accelerator memory spaces on the GPU against the CPU oracle:
makespans, statuses and per-task schedules bit-exact, for several capacities,
both task orders, uniform and uneven batches, and platforms where some
candidates cannot run at all.  Capacities are given to the library in blocks
of side b / 2^max_level and to the oracle in bytes (the same amount)."""
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


def _cap_bytes(pf_in, b, max_level, blocks):
    c = np.zeros(pf_in.n_mem, np.int64)
    c[1:] = blocks * pf_in.elem_bytes * (b >> max_level) ** 2
    return c


def _run(H, torch, pf, host, order=0, sched=False):
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
    H.simulate_batch(H.Plan(), pf, db, ms, st, policy=(order, 0, 0), **kw)
    torch.cuda.synchronize()
    out = [ms.cpu().numpy(), st.cpu().numpy()]
    if sched:
        out += [kw["sched_off"].cpu().numpy(), kw["proc"].cpu().numpy(), kw["start"].cpu().numpy(),
                kw["finish"].cpu().numpy()]
    return out


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("blocks", [12, 40, 160])
def test_capacity_against_oracle(H, torch, order, blocks):
    """8x8 tiles of 1024 at depths 0..2 on 8 CPU cores + 2 accelerators whose
    spaces hold `blocks` finest blocks (256 x 256); 48 candidates."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    cap = _cap_bytes(pf_in, w.b, w.dmax, blocks)
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, capacity_bytes=cap)
    host = I.uniform_batch(w.seed, 48, 8, w.b, w.dmax, w.p_num, w.p_den, first=5_000 + blocks)
    print(f"capacity: {blocks} blocks, order {order}, 48 candidates", flush=True)
    ms, st = _run(H, torch, pf, host, order)
    want, _, wst = O.simulate_batch(pf_in, host, NTHREADS, policy=(order, 0), capacity=cap, statuses=True)
    assert np.array_equal(st, wst)
    assert np.array_equal(ms, want)
    unbounded, _ = O.simulate_batch(pf_in, host, NTHREADS, policy=(order, 0))
    if blocks <= 40:
        assert (want != unbounded).sum() >= 12, "the capacity must bind"


def test_capacity_schedules_against_oracle(H, torch):
    """Per-task processors, starts and finishes of 6 candidates."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    cap = _cap_bytes(pf_in, w.b, w.dmax, 24)
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, capacity_bytes=cap)
    host = I.uniform_batch(w.seed, 6, 6, w.b, w.dmax, w.p_num, w.p_den, first=77)
    print("capacity: schedules of 6 candidates", flush=True)
    ms, st, off, proc, start, finish = _run(H, torch, pf, host, sched=True)
    assert (st == 0).all()
    for c in range(host.n):
        dep = host.depth[host.mask_off[c]:host.mask_off[c + 1]]
        s = O.simulate(pf_in, 6, w.dmax, w.b, dep, capacity=cap)
        assert s.makespan == ms[c]
        # tasks matched by (kind, level, K, I, J) through the library's expansion
        tasks, _, _ = H.expand(6, w.dmax, dep)
        key = {tuple(int(x) for x in tasks[t]): t for t in range(len(tasks))}
        assert len(key) == s.n_tasks
        for t in range(s.n_tasks):
            g = off[c] + key[tuple(int(x) for x in s.tasks[t])]
            assert (proc[g], start[g], finish[g]) == (s.proc[t], s.start[t], s.finish[t]), (c, t)


def test_capacity_ragged_against_oracle(H, torch):
    """Uneven batch (4..10 tiles of 512, depth caps 0..3) on the big.LITTLE
    workload's shapes with 2 accelerators of 48 blocks (64 x 64) each."""
    w = I.WORKLOADS["ragged_bl_b512_d3"]
    pf_in = I.make_platform(I.cpu_accel_types(4, 2), seed=w.seed)
    cap = _cap_bytes(pf_in, w.b, w.dmax, 48)
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, capacity_bytes=cap)
    host = I.ragged_batch(w.seed, 64, 4, 10, 3, w.b, w.p_num, w.p_den, first=900)
    print("capacity: ragged, 64 candidates", flush=True)
    ms, st = _run(H, torch, pf, host)
    want, _, wst = O.simulate_batch(pf_in, host, NTHREADS, capacity=cap, statuses=True)
    assert np.array_equal(st, wst)
    assert np.array_equal(ms, want)


def test_capacity_statuses_accelerators_only(H, torch):
    """Accelerators only: candidates with a task larger than a space fail with
    HESP_ECAPACITY (makespan -1), as in the oracle; the others are exact."""
    pf_in = I.make_platform([I.ProcType("acc", 2, 500_000, 2_000_000, 512, True)], seed=3)
    b, dmax = 512, 1
    cap = _cap_bytes(pf_in, b, dmax, 8)          # an unsplit gemm needs 12 finest blocks
    pf = H.Platform.from_inputs(pf_in, b, dmax, capacity_bytes=cap)
    host = I.uniform_batch(3, 64, 3, b, dmax, 3, 10, first=10)     # one gemm, split with p = 0.3
    print("capacity: accelerators only, 64 candidates", flush=True)
    ms, st = _run(H, torch, pf, host)
    want, _, wst = O.simulate_batch(pf_in, host, NTHREADS, capacity=cap, statuses=True)
    assert np.array_equal(st, np.where(wst == 0, 0, H.HESP_ECAPACITY))
    assert np.array_equal(ms, want)
    assert (st == H.HESP_ECAPACITY).any() and (st == 0).any()


def test_capacity_unsupported_combinations(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, capacity_bytes=_cap_bytes(pf_in, w.b, w.dmax, 4))
    db = H.DeviceBatch.from_host(w.batch(8))
    ms = torch.empty(8, dtype=torch.int64, device="cuda")
    st = torch.empty(8, dtype=torch.int32, device="cuda")
    for policy in [(0, 1, 0), (0, 0, 1), (0, 0, 2), (0, 2, 0), (0, 0, 0, 0, 1)]:
        with pytest.raises(RuntimeError, match="finite memory spaces"):
            H.simulate_batch(H.Plan(), pf, db, ms, st, policy=policy)
    with pytest.raises(RuntimeError, match="fused pipeline"):
        H.simulate_batch(H.Plan(group=64, fuse=True), pf, db, ms, st)
    with pytest.raises(RuntimeError, match="64 lanes"):
        H.simulate_batch(H.Plan(group=16), pf, db, ms, st)
    with pytest.raises(RuntimeError, match="finite memory spaces"):
        H.simulate_batch_noalloc(pf, db, ms, st)


def test_search_with_candidates_that_fail(H, torch):
    """Surrogate-guided search on an accelerator-only platform where most random
    partitions cannot run (a task larger than every space): the failed candidates
    neither become incumbents nor training rows; the best is a valid partition
    whose makespan the oracle reproduces."""
    pf_in = I.make_platform([I.ProcType("acc", 2, 500_000, 2_000_000, 512, True)], seed=3)
    b, dmax, nt = 512, 1, 3
    cap = _cap_bytes(pf_in, b, dmax, 8)
    pf = H.Platform.from_inputs(pf_in, b, dmax, capacity_bytes=cap)
    m = H.MLP(1)
    print("capacity: surrogate search with failing candidates", flush=True)
    best_d, best, trace = H.search(H.Plan(), pf, nt, dmax, H.SEARCH_SURROGATE, rounds=4, batch=512, seed=11,
                                   warm_batch=1024, proposals=2048, pool=16, split_thr=I.split_threshold(3, 10),
                                   mutate_thr=int(0.2 * (1 << 21)), mlp=m, train_steps=20, train_batch=512,
                                   replay=4096)
    assert best > 0 and all(t["best_makespan"] > 0 for t in trace)
    assert O.simulate(pf_in, nt, dmax, b, best_d, detail=False, capacity=cap) == best
    # plain random search gives the same kind of answer
    best_d2, best2, _ = H.search(H.Plan(), pf, nt, dmax, H.SEARCH_RANDOM, rounds=2, batch=512, seed=12,
                                 split_thr=I.split_threshold(3, 10))
    assert best2 > 0 and O.simulate(pf_in, nt, dmax, b, best_d2, detail=False, capacity=cap) == best2
