"""The fused pipeline (each wave of the 64-lane event loop prepares the
candidates it takes into its own workspace slot; one launch per batch) against
the unfused one and the CPU oracle: makespans, statuses and per-task schedules
bit-exact, under every policy class, on uniform and uneven batches, at the
capacity limit, and captured in a HIP graph."""
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


def _sim(H, torch, plan, pf, db, policy=(0, 0, 0), sched=False):
    n = db.n_cand
    ms = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    ntk = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    kw = {}
    if sched:
        cnt, _ = H.count_batch(db)
        off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        off[1:] = torch.cumsum(cnt.long(), 0)
        tot = int(off[-1].item())
        kw = dict(sched_off=off, proc=torch.full((tot,), -1, dtype=torch.int32, device="cuda"),
                  start=torch.full((tot,), -1, dtype=torch.int64, device="cuda"),
                  finish=torch.full((tot,), -1, dtype=torch.int64, device="cuda"))
    H.simulate_batch(plan, pf, db, ms, st, policy=policy, n_tasks=ntk, **kw)
    torch.cuda.synchronize()
    out = [ms.cpu().numpy(), st.cpu().numpy(), ntk.cpu().numpy()]
    if sched:
        out += [kw["proc"].cpu().numpy(), kw["start"].cpu().numpy(), kw["finish"].cpu().numpy()]
    return out


def test_fused_equals_unfused_and_oracle_16x16(H, torch):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    host = w.batch(384, first=7_000)
    db = H.DeviceBatch.from_host(host)
    print("fused: 16x16 tiles, 384 candidates, schedules", flush=True)
    fused = _sim(H, torch, H.Plan(group=64, fuse=True), pf, db, sched=True)
    for g in (64, 16):
        ref = _sim(H, torch, H.Plan(group=g), pf, db, sched=True)
        for a, b in zip(fused, ref):
            assert np.array_equal(a, b), g
    assert (fused[1] == 0).all()
    want, _ = O.simulate_batch(pf_in, host, NTHREADS)
    assert np.array_equal(fused[0], want)


@pytest.mark.parametrize("policy", [(1, 1, 0, 0, 0), (0, 2, 0, 7, 0), (1, 3, 0, 0, 0), (0, 0, 1, 0, 1),
                                    (0, 0, 2, 0, 0)])
def test_fused_policies_against_oracle(H, torch, policy):
    """(order, select, cache, seed, bus): FCFS/EIT-P, R-P, FCFS/F-P, write-through
    on a shared interconnect, write-around."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax = 8, 2
    pf = H.Platform.from_inputs(pf_in, w.b, dmax)
    host = I.uniform_batch(w.seed, 160, nt, w.b, dmax, w.p_num, w.p_den, first=31_000)
    db = H.DeviceBatch.from_host(host)
    order, select, cache, seed, bus = policy
    print(f"fused: policy {policy}", flush=True)
    got = _sim(H, torch, H.Plan(group=64, fuse=True), pf, db, policy=(order, select, cache, seed, bus))
    assert (got[1] == 0).all()
    want, _ = O.simulate_batch(pf_in, host, NTHREADS, policy=(order, select, seed, cache, bus))
    assert np.array_equal(got[0], want)


def test_fused_ragged_against_oracle(H, torch):
    w = I.WORKLOADS["ragged_bl_b512_d3"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    r = w.ragged
    host = I.ragged_batch(w.seed, 96, r["nt_lo"], 14, r["dmax_hi"], w.b, w.p_num, w.p_den, first=123)
    db = H.DeviceBatch.from_host(host)
    print("fused: ragged, 96 candidates", flush=True)
    got = _sim(H, torch, H.Plan(group=64, fuse=True), pf, db)
    assert (got[1] == 0).all()
    want, _ = O.simulate_batch(pf_in, host, NTHREADS)
    assert np.array_equal(got[0], want)
    ref = _sim(H, torch, H.Plan(group=16), pf, db)
    assert np.array_equal(got[0], ref[0])


def test_fused_statuses(H, torch):
    """A depth above dmax gives HESP_EINVAL; a fixed-capacity plan gives
    HESP_ECAPACITY to the candidates above it; the others are unaffected."""
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = H.Platform.from_inputs(w.platform(), w.b, w.dmax)
    host = w.batch(256, first=900)
    dep = host.depth.copy()
    dep[5 * 20 + 3] = 2                     # candidate 5: a depth above dmax
    db = H.DeviceBatch(256, w.nt, w.dmax, torch.from_numpy(dep).cuda())
    print("fused: statuses", flush=True)
    got = _sim(H, torch, H.Plan(group=64, fuse=True), pf, db)
    ref = _sim(H, torch, H.Plan(group=16), pf, db)
    assert got[1][5] == H.HESP_EINVAL and got[0][5] == -1
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    cnt, cne = H.count_batch(db)
    cnt = cnt.cpu().numpy()
    cap = int(np.median(cnt))
    capped = _sim(H, torch, H.Plan(group=64, max_tasks=cap, max_edges=10 ** 6, fuse=True), pf, db)
    over = cnt > cap
    over[5] = False
    ok = ~over
    ok[5] = False
    assert (capped[1][over] == H.HESP_ECAPACITY).all() and (capped[0][over] == -1).all()
    assert (capped[1][ok] == 0).all() and np.array_equal(capped[0][ok], ref[0][ok])


def test_fused_timing_reports_one_launch(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = H.Platform.from_inputs(w.platform(), w.b, w.dmax)
    db = H.generate_uniform(w.seed, 0, 2048, w.nt, w.dmax, I.split_threshold(w.p_num, w.p_den))
    plan = H.Plan(group=64, fuse=True)
    plan.timing(True)
    _sim(H, torch, plan, pf, db)
    prep_ms, sim_ms, launches = plan.last_ms()
    assert launches == 1 and sim_ms > 0.0 and prep_ms < sim_ms


def test_graph_replay_ragged_batch_one_launch(H, torch):
    """An uneven batch (8..32 tiles, depths 0..3) through a fixed-capacity plan:
    the fused pipeline needs no chunks and no read-back, so the call is captured
    once and replayed on new candidates (written into the captured buffers);
    every replay equals an eager call, and the last equals the oracle."""
    w = I.WORKLOADS["ragged_bl_b512_d3"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    r = w.ragged
    n, reps = 1536, 3
    hosts = [w.batch(n, first=50_000 + k * n) for k in range(reps + 1)]
    # the captured call reads the batch through fixed buffers (shapes, offsets,
    # depths) sized for the largest of the batches; each replay loads a new batch
    cap_t = cap_e = 0
    dbs = [H.DeviceBatch.from_host(h) for h in hosts]
    for d in dbs:
        a, b = H.count_batch(d)
        cap_t, cap_e = max(cap_t, int(a.max())), max(cap_e, int(b.max()))
    print(f"fused graph: ragged {n} candidates, capacities {cap_t} tasks {cap_e} edges", flush=True)
    dep = torch.zeros(max(int(h.mask_off[-1]) for h in hosts), dtype=torch.uint8, device="cuda")
    nt_b = torch.zeros(n, dtype=torch.int32, device="cuda")
    dm_b = torch.zeros(n, dtype=torch.int32, device="cuda")
    off_b = torch.zeros(n + 1, dtype=torch.int64, device="cuda")

    def load(k):
        h = hosts[k]
        dep[:int(h.mask_off[-1])].copy_(torch.from_numpy(np.ascontiguousarray(h.depth)))
        nt_b.copy_(torch.from_numpy(h.nt.astype(np.int32)))
        dm_b.copy_(torch.from_numpy(h.dmax.astype(np.int32)))
        off_b.copy_(torch.from_numpy(h.mask_off.astype(np.int64)))

    load(0)
    db = H.DeviceBatch(n, r["nt_hi"], r["dmax_hi"], dep, nt_b, dm_b, off_b)
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = H.Plan(max_tasks=cap_t, max_edges=cap_e, group=64, fuse=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        H.simulate_batch(plan, pf, db, ms, st)          # sizes and allocates the arena
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    plan.timing(True)
    H.simulate_batch(plan, pf, db, ms, st)
    torch.cuda.synchronize()
    assert plan.last_ms()[2] == 1, "one simulation launch for the whole uneven batch"
    plan.timing(False)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        H.simulate_batch(plan, pf, db, ms, st)
    eager_plan = H.Plan()
    ms2 = torch.empty_like(ms)
    st2 = torch.empty_like(st)
    for k in range(1, reps + 1):
        load(k)
        g.replay()
        torch.cuda.synchronize()
        H.simulate_batch(eager_plan, pf, dbs[k], ms2, st2)
        torch.cuda.synchronize()
        assert bool((st == 0).all().item()), k
        assert torch.equal(ms, ms2), k
    want, _ = O.simulate_batch(pf_in, hosts[reps], NTHREADS)
    assert np.array_equal(ms.cpu().numpy(), want)


# ------------------------------------------------------------ workspace slots in LDS

@pytest.mark.parametrize("name,n", [("chol4x4_b512_d1", 1024), ("chol16x16_b1024_d2", 0)])
def test_lds_slots_equal_unfused_and_oracle(H, torch, name, n):
    """fuse=2: each candidate's whole state in the workgroup's LDS.  The 4x4
    workload (every candidate fits) with schedules; candidates of the
    16x16 workload's platform and depth, 5 tiles (most fit)."""
    w = I.WORKLOADS[name]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    host = w.batch(n, first=3_000) if n else I.uniform_batch(w.seed, 256, 5, w.b, w.dmax, w.p_num, w.p_den, first=3)
    db = H.DeviceBatch.from_host(host)
    print(f"LDS slots: {name}, {host.n} candidates", flush=True)
    got = _sim(H, torch, H.Plan(group=64, fuse=2), pf, db, sched=True)
    ref = _sim(H, torch, H.Plan(), pf, db, sched=True)
    ok = got[1] == 0
    assert ok.sum() >= host.n // 2
    assert (got[1][~ok] == H.HESP_ECAPACITY).all() and (got[0][~ok] == -1).all()
    assert np.array_equal(got[0][ok], ref[0][ok])
    want, _ = O.simulate_batch(pf_in, host, NTHREADS)
    assert np.array_equal(got[0][ok], want[ok])
    if ok.all():
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_lds_slots_capacity_limit(H, torch):
    """Uneven batch: the candidates whose workspace exceeds the 48 KiB slot get
    HESP_ECAPACITY, exactly those (104 T + 4 E + 8 V + 4 (tet(nt) + 1) bytes,
    rounded up to 16), the others equal the oracle."""
    w = I.WORKLOADS["ragged_bl_b512_d3"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    host = I.ragged_batch(w.seed, 128, 4, 12, 3, w.b, w.p_num, w.p_den, first=4_321)
    db = H.DeviceBatch.from_host(host)
    cnt_t, cnt_e = H.count_batch(db)
    T = cnt_t.cpu().numpy().astype(np.int64)
    E = cnt_e.cpu().numpy().astype(np.int64)
    nt, dm = host.nt.astype(np.int64), host.dmax.astype(np.int64)
    V = (nt * (nt + 1) // 2) * 4 ** dm * pf_in.n_mem
    TP = nt * (nt + 1) * (nt + 2) // 6 + 1
    rb = (104 * T + 4 * E + 8 * V + 4 * TP + 15) // 16 * 16
    fits = rb <= 48 * 1024
    assert fits.any() and not fits.all(), "the case must straddle the slot"
    print("LDS slots: ragged, 128 candidates", flush=True)
    got = _sim(H, torch, H.Plan(group=64, fuse=2), pf, db)
    assert np.array_equal(got[1], np.where(fits, 0, H.HESP_ECAPACITY))
    want, _ = O.simulate_batch(pf_in, host, NTHREADS)
    assert np.array_equal(got[0][fits], want[fits]) and (got[0][~fits] == -1).all()


@pytest.mark.parametrize("policy", [(1, 1, 0, 0, 0), (0, 3, 0, 0, 0), (0, 0, 2, 0, 1)])
def test_lds_slots_policies(H, torch, policy):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    host = w.batch(256, first=77)
    db = H.DeviceBatch.from_host(host)
    order, select, cache, seed, bus = policy
    print(f"LDS slots: policy {policy}", flush=True)
    got = _sim(H, torch, H.Plan(group=64, fuse=2), pf, db, policy=(order, select, cache, seed, bus))
    assert (got[1] == 0).all()
    want, _ = O.simulate_batch(pf_in, host, NTHREADS, policy=(order, select, seed, cache, bus))
    assert np.array_equal(got[0], want)
