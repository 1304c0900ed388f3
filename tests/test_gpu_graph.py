"""Fixed-capacity plans: the simulation call captured in a HIP graph (through
torch.cuda.graph) and replayed on new candidates matches eager calls."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu


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


# three chunks: captured calls keep every chunk on the capturing stream (the
# eager two-stream pipeline is not captured)
@pytest.mark.parametrize("chunks", [1, 3])
def test_graph_replay_matches_eager(H, torch, chunks):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    thr = I.split_threshold(w.p_num, w.p_den)
    n, reps = 2048, 3
    batches = [H.generate_uniform(w.seed, 10_000 + r * n, n, w.nt, w.dmax, thr) for r in range(reps + 1)]
    cap_t = cap_e = 0
    for b in batches:
        nt_, ne_ = H.count_batch(b)
        cap_t, cap_e = max(cap_t, int(nt_.max())), max(cap_e, int(ne_.max()))
    dep = torch.empty_like(batches[0].depth)
    dep.copy_(batches[0].depth)
    db = H.DeviceBatch(n, w.nt, w.dmax, dep)
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = H.Plan(max_tasks=cap_t, max_edges=cap_e, group=16, chunks=chunks)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        H.simulate_batch(plan, pf, db, ms, st)          # sizes and allocates the workspace
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        H.simulate_batch(plan, pf, db, ms, st)
    eager_plan = H.Plan()
    ms2 = torch.empty_like(ms)
    st2 = torch.empty_like(st)
    for r in range(1, reps + 1):
        dep.copy_(batches[r].depth)
        g.replay()
        torch.cuda.synchronize()
        H.simulate_batch(eager_plan, pf, batches[r], ms2, st2)
        torch.cuda.synchronize()
        assert bool((st == 0).all().item())
        assert torch.equal(ms, ms2), r
    host = w.batch(64, first=10_000 + reps * n)
    want, _ = O.simulate_batch(pf_in, host, 8)
    assert np.array_equal(ms[:64].cpu().numpy(), want)


def test_graph_replay_with_tuned_lanes(H, torch):
    """A fixed-capacity plan with group 0: the first (eager) call of the shape
    times 16, 32 and 64 lanes per candidate and keeps the choice; the captured
    call reuses it, and the graph's replays equal eager calls and the oracle."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    thr = I.split_threshold(w.p_num, w.p_den)
    n, reps = 2048, 2
    batches = [H.generate_uniform(w.seed, 30_000 + r * n, n, w.nt, w.dmax, thr) for r in range(reps + 1)]
    cap_t = cap_e = 0
    for b in batches:
        nt_, ne_ = H.count_batch(b)
        cap_t, cap_e = max(cap_t, int(nt_.max())), max(cap_e, int(ne_.max()))
    dep = torch.empty_like(batches[0].depth)
    dep.copy_(batches[0].depth)
    db = H.DeviceBatch(n, w.nt, w.dmax, dep)
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = H.Plan(max_tasks=cap_t, max_edges=cap_e)          # group 0: tuned by the first call
    print("graph: fixed plan with tuned lanes", flush=True)
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
    for r in range(1, reps + 1):
        dep.copy_(batches[r].depth)
        g.replay()
        torch.cuda.synchronize()
        H.simulate_batch(H.Plan(), pf, batches[r], ms2, st2)
        torch.cuda.synchronize()
        assert bool((st == 0).all().item())
        assert torch.equal(ms, ms2), r
    host = w.batch(32, first=30_000 + reps * n)
    want, _ = O.simulate_batch(pf_in, host, 8)
    assert np.array_equal(ms[:32].cpu().numpy(), want)


def test_fixed_plan_capacity_status(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = H.Platform.from_inputs(w.platform(), w.b, w.dmax)
    host = w.batch(256)
    db = H.DeviceBatch.from_host(host)
    nt_, ne_ = H.count_batch(db)
    cap = int(nt_.float().median().item())
    ms = torch.empty(256, dtype=torch.int64, device="cuda")
    st = torch.empty(256, dtype=torch.int32, device="cuda")
    H.simulate_batch(H.Plan(max_tasks=cap, max_edges=10 ** 6, group=16), pf, db, ms, st)
    ref = torch.empty_like(ms)
    rst = torch.empty_like(st)
    H.simulate_batch(H.Plan(), pf, db, ref, rst)
    over = nt_ > cap
    assert bool((st[over] == H.HESP_ECAPACITY).all().item()) and bool((ms[over] == -1).all().item())
    assert bool((st[~over] == 0).all().item()) and torch.equal(ms[~over], ref[~over])


def test_chunk_pipeline_matches_single_chunk(H, torch):
    """Chunks prepared on one stream while the previous chunk is simulated on
    another (two workspace sets) give the results of a single chunk."""
    w = I.WORKLOADS["ragged_bl_b512_d3"]
    pf = H.Platform.from_inputs(w.platform(), w.b, w.dmax)
    r = w.ragged
    db = H.generate_ragged(w.seed, 0, 3000, r["nt_lo"], r["nt_hi"], r["dmax_hi"], I.split_threshold(3, 10))
    out = []
    for chunks in (1, 2, 5):
        ms = torch.empty(3000, dtype=torch.int64, device="cuda")
        st = torch.empty(3000, dtype=torch.int32, device="cuda")
        H.simulate_batch(H.Plan(chunks=chunks), pf, db, ms, st)
        torch.cuda.synchronize()
        assert bool((st == 0).all().item())
        out.append(ms)
    assert torch.equal(out[0], out[1]) and torch.equal(out[0], out[2])


def test_graph_replay_split_trees(H, torch):
    """Split-tree batches through a fixed-capacity plan: captured once, replayed
    on new flags, equal to eager calls and to the oracle."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax = 8, 2
    pf = H.Platform.from_inputs(pf_in, w.b, dmax)
    thr = I.split_threshold(w.p_num, w.p_den)
    n, reps = 1024, 3
    batches = [H.generate_tree_uniform(w.seed, 20_000 + r * n, n, nt, dmax, thr) for r in range(reps + 1)]
    cap_t = cap_e = 0
    for b in batches:
        nt_, ne_ = H.count_tree_batch(b)
        cap_t, cap_e = max(cap_t, int(nt_.max())), max(cap_e, int(ne_.max()))
    flags = torch.empty_like(batches[0].flags)
    flags.copy_(batches[0].flags)
    tb = H.TreeBatch(n, nt, dmax, flags)
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    plan = H.Plan(max_tasks=cap_t, max_edges=cap_e, group=16)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        H.simulate_tree_batch(plan, pf, tb, ms, st)     # sizes and allocates the workspace
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        H.simulate_tree_batch(plan, pf, tb, ms, st)
    eager_plan = H.Plan()
    ms2 = torch.empty_like(ms)
    st2 = torch.empty_like(st)
    for r in range(1, reps + 1):
        flags.copy_(batches[r].flags)
        g.replay()
        torch.cuda.synchronize()
        H.simulate_tree_batch(eager_plan, pf, batches[r], ms2, st2)
        torch.cuda.synchronize()
        assert bool((st == 0).all().item())
        assert torch.equal(ms, ms2), r
    host = I.tree_batch(w.seed, 48, nt, w.b, dmax, w.p_num, w.p_den, first=20_000 + reps * n)
    want, _ = O.simulate_batch(pf_in, host, 8, tree=True)
    assert np.array_equal(ms[:48].cpu().numpy(), want)
