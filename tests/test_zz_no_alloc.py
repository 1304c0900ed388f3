"""hesp_simulate_batch_noalloc (no device allocation, one fixed device array)
against hesp_simulate_batch, through the C ABI: bit-exact makespans, statuses,
task counts and schedules, on two calls in a row (the second smaller), on a
ragged batch, and at the array's capacity limit."""
import numpy as np
import pytest

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


def _run(H, torch, fn, pf, db, sched):
    n = db.n_cand
    ms = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    nt = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    extra = {}
    if sched:
        cnt, _ = H.count_batch(db)
        off = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        off[1:] = torch.cumsum(cnt.to(torch.int64), 0)
        tot = int(off[-1].item())
        extra = dict(sched_off=off, proc=torch.full((tot,), -1, dtype=torch.int32, device="cuda"),
                     start=torch.full((tot,), -1, dtype=torch.int64, device="cuda"),
                     finish=torch.full((tot,), -1, dtype=torch.int64, device="cuda"))
    fn(pf, db, ms, st, n_tasks=nt, **extra)
    torch.cuda.synchronize()
    res = [ms.cpu().numpy(), st.cpu().numpy(), nt.cpu().numpy()]
    if sched:
        res += [extra["proc"].cpu().numpy(), extra["start"].cpu().numpy(), extra["finish"].cpu().numpy()]
    return res


def _both(H, torch, pf, db, sched=False, group=0):
    plan = H.Plan()
    want = _run(H, torch, lambda p, b, m, s, **kw: H.simulate_batch(plan, p, b, m, s, **kw), pf, db, sched)
    got = _run(H, torch, lambda p, b, m, s, **kw: H.simulate_batch_noalloc(p, b, m, s, group=group, **kw), pf, db,
               sched)
    plan.close()
    return want, got


def test_noalloc_two_calls_second_smaller(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    thr = I.split_threshold(w.p_num, w.p_den)
    for n, first, sched in ((1024, 0, False), (300, 5000, True)):
        print(f"noalloc: 4x4 tiles, {n} candidates from {first}, schedules {sched}", flush=True)
        db = H.generate_uniform(w.seed, first, n, w.nt, w.dmax, thr)
        want, got = _both(H, torch, pf, db, sched)
        assert (want[1] == 0).all()
        for a, b in zip(want, got):
            assert np.array_equal(a, b)


def test_noalloc_ragged_and_wide(H, torch):
    w = I.WORKLOADS["ragged_bl_b512_d3"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, 3)
    thr = I.split_threshold(w.p_num, w.p_den)
    print("noalloc: ragged 8..12 tiles, 96 candidates", flush=True)
    db = H.generate_ragged(w.seed, 77, 96, 8, 12, 2, thr)
    want, got = _both(H, torch, pf, db, sched=True, group=32)
    assert (want[1] == 0).all()
    for a, b in zip(want, got):
        assert np.array_equal(a, b)


def test_noalloc_capacity_limit(H, torch):
    """16x16-tile candidates overflow the array: the ones that fit match, the rest
    (from the first whose workspace ends past the region) get HESP_ECAPACITY."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    n = 160
    print(f"noalloc: 16x16 tiles, {n} candidates (capacity limit)", flush=True)
    db = H.generate_uniform(w.seed, 123, n, w.nt, w.dmax, I.split_threshold(w.p_num, w.p_den))
    cnt_t, cnt_e = H.count_batch(db)
    T = cnt_t.cpu().numpy().astype(np.int64)
    E = cnt_e.cpu().numpy().astype(np.int64)
    V = (w.nt * (w.nt + 1) // 2) * 4 ** w.dmax * pf_in.n_mem
    TP = I.tet(w.nt) + 1
    rb = (104 * T + 4 * E + 8 * V + 4 * TP + 15) // 16 * 16
    fits = np.cumsum(rb) <= H.NOALLOC_REGION
    assert fits[0] and not fits[-1], "the case must straddle the limit"
    want, got = _both(H, torch, pf, db)
    assert np.array_equal(got[1], np.where(fits, 0, H.HESP_ECAPACITY))
    assert np.array_equal(got[0][fits], want[0][fits])
    assert (got[0][~fits] == -1).all()
    assert np.array_equal(got[2][fits], want[2][fits])


def test_noalloc_rejects_oversized_batch(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = H.Platform.from_inputs(w.platform(), w.b, w.dmax)
    n = H.NOALLOC_MAX_CAND + 1
    db = H.generate_uniform(w.seed, 0, n, w.nt, w.dmax, I.split_threshold(w.p_num, w.p_den))
    ms = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    with pytest.raises(H.HespError) as e:
        H.simulate_batch_noalloc(pf, db, ms, st)
    assert e.value.code == H.HESP_EINVAL
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 99).all(), "nothing may be enqueued for a rejected call"
