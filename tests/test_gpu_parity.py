"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Integers throughout: makespans, processors, start and finish times must be
bit-exact.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
KIND = {"chol": 0, "trsm": 1, "syrk": 2, "gemm": 3}
NTHREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def H(torch_cuda):
    from paper_1602_05510_amd import hesp
    return hesp


def gpu_run(H, torch, pf_in, batch, max_level, plan=None, sched=False, order=None):
    """Simulate a host batch on the GPU; returns makespan, status (and schedules)."""
    pf = H.Platform.from_inputs(pf_in, batch.b, max_level)
    if order is not None:
        batch = batch.subset(order)
    db = H.DeviceBatch.from_host(batch)
    n = batch.n
    ms = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    plan = plan or H.Plan()
    if sched:
        nt, ne = H.count_batch(db)
        off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        off[1:] = torch.cumsum(nt.to(torch.int64), 0)
        tot = int(off[-1].item())
        proc = torch.full((tot,), -1, dtype=torch.int32, device="cuda")
        start = torch.full((tot,), -1, dtype=torch.int64, device="cuda")
        fin = torch.full((tot,), -1, dtype=torch.int64, device="cuda")
        H.simulate_batch(plan, pf, db, ms, st, off, proc, start, fin)
        torch.cuda.synchronize()
        return ms.cpu().numpy(), st.cpu().numpy(), (off.cpu().numpy(), proc.cpu().numpy(), start.cpu().numpy(),
                                                     fin.cpu().numpy())
    H.simulate_batch(plan, pf, db, ms, st)
    torch.cuda.synchronize()
    return ms.cpu().numpy(), st.cpu().numpy()


def oracle_batch(pf, batch):
    ms, _ = O.simulate_batch(pf, batch, NTHREADS)
    return ms


# ------------------------------------------------------------------ generation

def test_uniform_generation_matches_inputs(H, torch_cuda):
    for name, n in [("chol4x4_b512_d1", 1024), ("chol16x16_b1024_d2", 512), ("chol64x64_b1024_d3", 8)]:
        w = I.WORKLOADS[name]
        host = w.batch(n, first=5)
        thr = I.split_threshold(w.p_num, w.p_den)
        db = H.generate_uniform(w.seed, 5, n, w.nt, w.dmax, thr)
        torch_cuda.cuda.synchronize()
        assert np.array_equal(db.depth.cpu().numpy(), host.depth), name


def test_ragged_generation_matches_inputs(H, torch_cuda):
    w = I.WORKLOADS["ragged_bl_b512_d3"]
    host = w.batch(777, first=3)
    r = w.ragged
    db = H.generate_ragged(w.seed, 3, 777, r["nt_lo"], r["nt_hi"], r["dmax_hi"],
                           I.split_threshold(w.p_num, w.p_den))
    torch_cuda.cuda.synchronize()
    assert np.array_equal(db.nt_arr.cpu().numpy(), host.nt)
    assert np.array_equal(db.dmax_arr.cpu().numpy(), host.dmax)
    assert np.array_equal(db.mask_off.cpu().numpy(), host.mask_off)
    assert np.array_equal(db.depth.cpu().numpy()[:host.mask_off[-1]], host.depth)


def test_counts_match_host_expansion(H, torch_cuda):
    for name, n in [("chol4x4_b512_d1", 64), ("chol16x16_b1024_d2", 16)]:
        w = I.WORKLOADS[name]
        bt = w.batch(n)
        db = H.DeviceBatch.from_host(bt)
        nt, ne = H.count_batch(db)
        nt, ne = nt.cpu().numpy(), ne.cpu().numpy()
        for c in range(n):
            tasks, ptr, idx = H.expand(w.nt, w.dmax, bt.candidate(c))
            assert nt[c] == len(tasks) and ne[c] == len(idx)


# ------------------------------------------------------------------ hand-derived examples

def test_worked_examples_on_gpu(H, torch_cuda):
    with open(os.path.join(GOLD, "worked_examples.json")) as f:
        ex = json.load(f)["examples"]
    for e in ex:
        pts = [I.ProcType(n, c, r, r, h, own) for (n, c, r, h, own) in e["platform"]["types"]]
        pf = I.make_platform(pts, seed=0)
        dep = np.array(e["depth"], np.uint8)
        bt = I.Batch(e["b"], np.array([e["nt"]], np.int32), np.array([e["dmax"]], np.int32),
                     np.array([0, len(dep)], np.int64), dep)
        ms, st, (off, proc, start, fin) = gpu_run(H, torch_cuda, pf, bt, e["dmax"], sched=True)
        assert st[0] == 0 and ms[0] == e["makespan"], e["name"]
        tasks, _, _ = H.expand(e["nt"], e["dmax"], dep)
        got = {tuple(int(x) for x in tasks[t]): (int(proc[t]), int(start[t]), int(fin[t])) for t in range(len(tasks))}
        for (kind, lvl, K, I_, J, p, s0, f0) in e["schedule"]:
            assert got[(KIND[kind], lvl, K, I_, J)] == (p, s0, f0), (e["name"], kind, K, I_, J)


# ------------------------------------------------------------------ makespan parity

def test_parity_chol4x4_all_candidates(H, torch_cuda):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = w.batch()
    ref = oracle_batch(pf, bt)
    for group in (0, 16, 64):
        ms, st = gpu_run(H, torch_cuda, pf, bt, w.dmax, plan=H.Plan(group=group))
        assert np.all(st == 0)
        assert np.array_equal(ms, ref), group


def test_parity_chol16x16_subset(H, torch_cuda):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    bt = w.batch(384)
    ms, st = gpu_run(H, torch_cuda, pf, bt, w.dmax)
    assert np.all(st == 0)
    assert np.array_equal(ms, oracle_batch(pf, bt))


def test_parity_ragged_big_little(H, torch_cuda):
    """The uneven big.LITTLE batch without any size filter (8..32 tiles, depths
    0..3), plus candidates drawn further on with 28..32 tiles at depth 3."""
    w = I.WORKLOADS["ragged_bl_b512_d3"]
    pf = w.platform()
    bt = w.batch(600)
    more = w.batch(3000, first=600)
    big = [c for c in range(more.n) if more.nt[c] >= 28 and more.dmax[c] == 3][:24]
    assert len(big) == 24
    bt = I.concat_batches([bt, more.subset(big)])
    assert bt.nt.max() == 32 and int(((bt.nt >= 28) & (bt.dmax == 3)).sum()) >= 24
    ms, st = gpu_run(H, torch_cuda, pf, bt, 3)
    assert np.all(st == 0)
    assert np.array_equal(ms, oracle_batch(pf, bt))


def _task_keys(tasks):
    t = np.asarray(tasks, np.int64)
    return (t[:, 0] << 40) | (t[:, 1] << 36) | (t[:, 2] << 24) | (t[:, 3] << 12) | t[:, 4]


def _check_schedule(H, w, pf, bt, c, off, proc, start, fin):
    """Per-task (processor, start, finish) of candidate c against the oracle's,
    tasks matched by (kind, level, K, I, J)."""
    s = O.simulate(pf, int(bt.nt[c]), int(bt.dmax[c]), bt.b, bt.candidate(c))
    tasks, _, _ = H.expand(int(bt.nt[c]), int(bt.dmax[c]), bt.candidate(c))
    kl, ko = _task_keys(tasks), _task_keys(s.tasks)
    assert len(kl) == len(ko) == s.n_tasks
    order_l, order_o = np.argsort(kl), np.argsort(ko)
    assert np.array_equal(kl[order_l], ko[order_o])
    g = off[c] + order_l                     # library positions, in the oracle's sorted order
    assert np.array_equal(proc[g], s.proc[order_o])
    assert np.array_equal(start[g], s.start[order_o])
    assert np.array_equal(fin[g], s.finish[order_o])
    return s.makespan


def test_parity_chol64x64_d3(H, torch_cuda):
    """The largest instance shape: 64 x 64 tiles split up to depth 3 (512 finest
    tiles per dimension, the limit of the 9-bit fine coordinates), 16 CPUs + 4
    accelerators in five memory spaces; 16 seeded candidates bit-exact and two
    of them task by task."""
    w = I.WORKLOADS["chol64x64_b1024_d3"]
    pf = w.platform()
    assert w.nt << w.dmax == 512 and pf.n_mem == 5 and pf.n_procs == 20
    bt = w.batch(16)
    ms, st, (off, proc, start, fin) = gpu_run(H, torch_cuda, pf, bt, w.dmax, sched=True)
    assert np.all(st == 0)
    assert np.array_equal(ms, oracle_batch(pf, bt))
    for c in (0, 9):
        assert ms[c] == _check_schedule(H, w, pf, bt, c, off, proc, start, fin)


def test_schedule_parity_per_task(H, torch_cuda):
    for name, n in [("chol4x4_b512_d1", 32), ("chol16x16_b1024_d2", 6)]:
        w = I.WORKLOADS[name]
        pf = w.platform()
        bt = w.batch(n, first=100)
        ms, st, (off, proc, start, fin) = gpu_run(H, torch_cuda, pf, bt, w.dmax, sched=True)
        for c in range(n):
            s = O.simulate(pf, w.nt, w.dmax, w.b, bt.candidate(c))
            tasks, _, _ = H.expand(w.nt, w.dmax, bt.candidate(c))
            key = {tuple(int(x) for x in tasks[t]): t for t in range(len(tasks))}
            assert ms[c] == s.makespan
            for t in range(s.n_tasks):
                g = off[c] + key[tuple(int(x) for x in s.tasks[t])]
                assert (proc[g], start[g], fin[g]) == (s.proc[t], s.start[t], s.finish[t])


# ------------------------------------------------------------------ edge cases

def test_edge_cases(H, torch_cuda):
    pf = I.make_platform(I.cpu_accel_types(3, 2), seed=11)
    cases = []
    rng = np.random.default_rng(5)
    for nt, dmax in [(1, 0), (1, 3), (2, 3), (3, 0), (5, 3), (8, 3), (16, 2), (9, 1)]:
        n_top = nt * (nt + 1) * (nt + 2) // 6
        for mode in ("zero", "full", "rand"):
            if mode == "zero":
                d = np.zeros(n_top, np.uint8)
            elif mode == "full":
                d = np.full(n_top, dmax, np.uint8)
            else:
                d = rng.integers(0, dmax + 1, n_top).astype(np.uint8)
            cases.append((nt, dmax, d))
    # a ragged batch holding every case at once
    nt = np.array([c[0] for c in cases], np.int32)
    dm = np.array([c[1] for c in cases], np.int32)
    off = np.zeros(len(cases) + 1, np.int64)
    off[1:] = np.cumsum([len(c[2]) for c in cases])
    bt = I.Batch(512, nt, dm, off, np.concatenate([c[2] for c in cases]))
    ms, st = gpu_run(H, torch_cuda, pf, bt, 3)
    assert np.all(st == 0)
    assert np.array_equal(ms, oracle_batch(pf, bt))


def test_bad_depth_and_capacity_status(H, torch_cuda):
    torch = torch_cuda
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = w.platform()
    bt = w.batch(8)
    bt.depth[bt.mask_off[3] + 2] = 2          # above dmax = 1
    ms, st = gpu_run(H, torch, pf, bt, 1)
    assert st[3] == H.HESP_EINVAL and ms[3] == -1
    ok = [c for c in range(8) if c != 3]
    assert np.all(st[ok] == 0)
    assert np.array_equal(ms[ok], oracle_batch(pf, bt.subset(ok)))
    # a fixed-capacity plan smaller than some candidates
    bt2 = w.batch(64)
    sizes = np.array([len(H.expand(4, 1, bt2.candidate(c))[0]) for c in range(64)])
    cap = int(np.median(sizes))
    plan = H.Plan(max_tasks=cap, max_edges=100000)
    ms2, st2 = gpu_run(H, torch, pf, bt2, 1, plan=plan)
    big = sizes > cap
    assert np.all(st2[big] == H.HESP_ECAPACITY) and np.all(ms2[big] == -1)
    assert np.all(st2[~big] == 0)
    ref = oracle_batch(pf, bt2)
    assert np.array_equal(ms2[~big], ref[~big])


def test_invariance_to_order_and_slots(H, torch_cuda):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    bt = w.batch(96, first=7)
    ref, st = gpu_run(H, torch_cuda, pf, bt, w.dmax)
    perm = np.random.default_rng(1).permutation(96)
    ms_p, _ = gpu_run(H, torch_cuda, pf, bt, w.dmax, order=perm)
    assert np.array_equal(ms_p, ref[perm])
    for slots in (1, 7, 1000):
        ms_s, _ = gpu_run(H, torch_cuda, pf, bt, w.dmax, plan=H.Plan(slots=slots))
        assert np.array_equal(ms_s, ref)
    # every lane-group size of the simulation kernel gives the same makespans
    for group in (16, 32, 64):
        ms_g, st_g = gpu_run(H, torch_cuda, pf, bt, w.dmax, plan=H.Plan(group=group))
        assert np.all(st_g == 0) and np.array_equal(ms_g, ref), group
    with pytest.raises(H.HespError):
        H.Plan(group=8)


def test_argmin(H, torch_cuda):
    torch = torch_cuda
    v = torch.tensor([5, 3, -1, 3, 9, 3], dtype=torch.int64, device="cuda")
    best = torch.zeros(2, dtype=torch.int64, device="cuda")
    H.argmin(v, best)
    assert best.cpu().tolist() == [3, 1]
    v = torch.full((5000,), 7, dtype=torch.int64, device="cuda")
    v[4321] = 2
    v[4999] = 2
    H.argmin(v, best)
    assert best.cpu().tolist() == [2, 4321]
    v = torch.full((3,), -1, dtype=torch.int64, device="cuda")
    H.argmin(v, best)
    assert best.cpu().tolist() == [-1, -1]


def test_critical_time_reread_path(H, torch_cuda):
    """The critical-time pass keeps the dependences inside each run of 64
    consecutive tasks in LDS; a plan with a small budget sends most runs through
    the path that re-reads the successor lists on every sweep: same makespans."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf = w.platform()
    bt = w.batch(64, first=11)
    ref = oracle_batch(pf, bt)
    for budget in (1, 7, 64):
        ms, st = gpu_run(H, torch_cuda, pf, bt, w.dmax, plan=H.Plan(prep_edges=budget))
        assert np.all(st == 0) and np.array_equal(ms, ref), budget
    wr = I.WORKLOADS["ragged_bl_b512_d3"]
    br = wr.batch(96, first=5)
    ms, st = gpu_run(H, torch_cuda, wr.platform(), br, 3, plan=H.Plan(prep_edges=1))
    assert np.all(st == 0) and np.array_equal(ms, oracle_batch(wr.platform(), br))
    with pytest.raises(H.HespError):
        H.Plan(prep_edges=1025)
