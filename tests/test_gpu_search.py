"""GPU tests of enumeration, top-k selection, aggregate features and the search
driver, through the C ABI, against the CPU oracle and plain numpy definitions."""
import os

import numpy as np
import pytest

from oracle import mlp_ref as R
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


def _host_batch(depth, nt, dmax, b):
    n_top = I.tet(nt)
    dep = np.ascontiguousarray(depth, np.uint8).reshape(-1)
    n = dep.size // n_top
    return I.Batch(b, np.full(n, nt, np.int32), np.full(n, dmax, np.int32),
                   np.arange(n + 1, dtype=np.int64) * n_top, dep)


@pytest.mark.parametrize("nt,dmax,first,n", [(4, 1, 123456, 5000), (2, 2, 7, 81), (3, 3, 0, 300), (2, 5, 11, 1296)])
def test_enumerate(H, torch, nt, dmax, first, n):
    db = H.generate_enumerate(first, n, nt, dmax)
    got = db.depth.cpu().numpy().reshape(n, I.tet(nt))
    want = np.zeros_like(got)
    for c in range(n):
        v = first + c
        for t in range(I.tet(nt)):
            want[c, t] = v % (dmax + 1)
            v //= dmax + 1
    assert np.array_equal(got, want)


def _order_ms(v):
    key = np.where((v < 0) | (v >= (1 << 40)), (1 << 40) - 1, v)
    return np.lexsort((np.arange(v.size), key))


@pytest.mark.parametrize("n,k", [(1, 1), (2048, 2048), (10000, 100), (70001, 7000)])
def test_topk_makespan(H, torch, n, k):
    rng = np.random.default_rng(n)
    v = rng.integers(0, 50, n).astype(np.int64) * 1000           # many ties
    v[rng.choice(n, n // 10 + 1, replace=False)] = -1             # failed candidates rank last
    idx = H.topk(torch.from_numpy(v).cuda(), k).cpu().numpy()
    assert np.array_equal(idx, _order_ms(v)[:k])


@pytest.mark.parametrize("n,k", [(3000, 3000), (100000, 1000)])
def test_topk_score(H, torch, n, k):
    rng = np.random.default_rng(n + 1)
    v = np.round(rng.normal(0, 1, n), 2).astype(np.float32)        # ties
    v[::97] = np.nan
    v[5] = -0.0
    v[6] = 0.0
    idx = H.topk(torch.from_numpy(v).cuda(), k).cpu().numpy()
    key = np.where(np.isnan(v), np.inf, v).astype(np.float64)
    # -0.0 sorts before +0.0 in the order-preserving bit mapping
    neg0 = (v == 0) & np.signbit(v)
    want = np.lexsort((np.arange(n), ~neg0, key, np.isnan(v)))
    assert np.array_equal(idx, want[:k])


def test_topk_rejects(H, torch):
    v = torch.zeros(10, dtype=torch.int64, device="cuda")
    with pytest.raises(H.HespError):
        H.topk(v, 11)


def test_features_agg(H, torch):
    rng = np.random.default_rng(3)
    nt, n = 8, 1001
    n_top = I.tet(nt)
    dep = rng.integers(0, 6, (n, n_top)).astype(np.uint8)      # depths 3..5 share one bin
    rate = rng.normal(0, 1, 8).astype(np.float32)
    x = torch.empty((n, 32), dtype=torch.int16, device="cuda")
    H.mlp_features_agg(torch.from_numpy(dep).cuda(), n, nt, torch.from_numpy(rate).cuda(), x)
    got = R.bf16_round(np.zeros(1, np.float32))  # noqa: F841 (warm the helper)
    got = (x.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    kind = np.zeros(n_top, np.int64)
    half = np.zeros(n_top, np.int64)
    t = 0
    for k in range(nt):                      # Fig. 1 order: chol, trsm row, then gemm/syrk groups
        kind[t] = 0; half[t] = 2 * k >= nt; t += 1
        for j in range(k + 1, nt):
            kind[t] = 1; half[t] = 2 * k >= nt; t += 1
        for i in range(k + 1, nt):
            for j in range(i + 1, nt):
                kind[t] = 3; half[t] = 2 * k >= nt; t += 1
            kind[t] = 2; half[t] = 2 * k >= nt; t += 1
    want = np.zeros((n, 32), np.float32)
    for kd in range(4):
        sel = kind == kd
        for d in range(4):
            want[:, kd * 4 + d] = (np.minimum(dep[:, sel], 3) == d).sum(1) / sel.sum()
        for h in range(2):
            s2 = sel & (half == h)
            want[:, 16 + kd * 2 + h] = dep[:, s2].sum(1) / s2.sum() if s2.any() else 0.0
    want[:, 24:32] = rate
    assert np.allclose(got, R.bf16_round(want), rtol=2.0 ** -8, atol=0)


def _pf(H, w):
    pf_in = w.platform()
    return pf_in, H.Platform.from_inputs(pf_in, w.b, w.dmax)


def _monotone(tr):
    b = [t["best_makespan"] for t in tr]
    return all(x >= y for x, y in zip(b, b[1:]))


def test_search_random_is_batch_min(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in, pf = _pf(H, w)
    thr = I.split_threshold(1, 2)
    plan = H.Plan()
    best, best_ms, tr = H.search(plan, pf, 4, 1, H.SEARCH_RANDOM, rounds=3, batch=300, seed=w.seed, pool=8,
                                 split_thr=thr)
    host = I.uniform_batch(w.seed, 900, 4, w.b, 1, 1, 2)
    ms, _ = O.simulate_batch(pf_in, host, NTHREADS)
    c = int(np.argmin(ms))
    assert best_ms == int(ms[c])
    assert np.array_equal(best, host.candidate(c))
    assert [t["simulated"] for t in tr] == [300, 600, 900]
    assert tr[-1]["best_makespan"] == best_ms and _monotone(tr)


@pytest.mark.parametrize("mode", ["greedy", "surrogate"])
def test_search_modes_exact(H, torch, mode):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in, pf = _pf(H, w)
    thr = I.split_threshold(1, 2)
    plan = H.Plan()
    kw = dict(rounds=6, batch=256, seed=11, warm_rounds=1, warm_batch=512, pool=16, split_thr=thr,
              mutate_thr=(1 << 21) // 10)
    if mode == "greedy":
        best, best_ms, tr = H.search(plan, pf, 4, 1, H.SEARCH_GREEDY, **kw)
        assert [t["simulated"] for t in tr] == [512 + 256 * r for r in range(6)]
    else:
        m = H.MLP(5)
        rate = torch.from_numpy(H.mlp_rate_features(pf_in.rmax)).cuda()
        best, best_ms, tr = H.search(plan, pf, 4, 1, H.SEARCH_SURROGATE, proposals=2048, mlp=m, rate=rate,
                                     train_steps=10, train_batch=512, lr=1e-3, replay=4096, **kw)
        assert [t["proposed"] for t in tr] == [512 + 2048 * r for r in range(6)]
        assert np.isfinite(m.get_params()).all()
    assert best_ms == O.simulate(pf_in, 4, 1, w.b, best, detail=False)
    assert _monotone(tr) and tr[-1]["best_makespan"] == best_ms
    # the warm-up round alone is a random search of 512 candidates
    host = I.uniform_batch(11, 512, 4, w.b, 1, 1, 2)
    ms, _ = O.simulate_batch(pf_in, host, NTHREADS)
    assert tr[0]["best_makespan"] == int(ms.min())


def test_search_surrogate_aggregate_features(H, torch):
    # 8x8 tiles: 120 top-level tasks, more than the network's inputs
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, 512, 2)
    m = H.MLP(6)
    rate = torch.from_numpy(H.mlp_rate_features(pf_in.rmax)).cuda()
    plan = H.Plan()
    best, best_ms, tr = H.search(plan, pf, 8, 2, H.SEARCH_SURROGATE, rounds=4, batch=128, seed=3, warm_rounds=1,
                                 warm_batch=512, proposals=1024, pool=8, split_thr=I.split_threshold(3, 10),
                                 mutate_thr=(1 << 21) // 20, mlp=m, rate=rate, train_steps=5, train_batch=512,
                                 lr=1e-3, replay=2048)
    assert best_ms == O.simulate(pf_in, 8, 2, 512, best, detail=False)
    assert _monotone(tr)


def test_search_at_depth_five(H, torch):
    """6x6 tiles of 1024 split up to 5 times on the 16x16 workload's platform:
    the random search's best is the minimum of the same 768 seeded candidates,
    and a surrogate-guided search (aggregate features) ends on a partition whose
    makespan the oracle reproduces."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax = 6, 5
    pf = H.Platform.from_inputs(pf_in, w.b, dmax)
    thr = I.split_threshold(1, 2)
    print("search: depth 5, random", flush=True)
    best, best_ms, tr = H.search(H.Plan(), pf, nt, dmax, H.SEARCH_RANDOM, rounds=3, batch=256, seed=31, pool=8,
                                 split_thr=thr)
    host = I.uniform_batch(31, 768, nt, w.b, dmax, 1, 2)
    assert int(host.depth.max()) == 5
    ms, _ = O.simulate_batch(pf_in, host, NTHREADS)
    c = int(np.argmin(ms))
    assert best_ms == int(ms[c]) and np.array_equal(best, host.candidate(c))
    print("search: depth 5, surrogate", flush=True)
    m = H.MLP(7)
    rate = torch.from_numpy(H.mlp_rate_features(pf_in.rmax)).cuda()
    best, best_ms, tr = H.search(H.Plan(), pf, nt, dmax, H.SEARCH_SURROGATE, rounds=3, batch=128, seed=32,
                                 warm_rounds=1, warm_batch=512, proposals=1024, pool=8, split_thr=thr,
                                 mutate_thr=(1 << 21) // 20, mlp=m, rate=rate, train_steps=5, train_batch=512,
                                 lr=1e-3, replay=2048)
    assert best_ms == O.simulate(pf_in, nt, dmax, w.b, best, detail=False)
    assert _monotone(tr)


def test_search_rejects(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    _, pf = _pf(H, w)
    with pytest.raises(H.HespError):
        H.search(H.Plan(), pf, 4, 1, H.SEARCH_GREEDY, rounds=2, batch=16, seed=1, pool=0)
    with pytest.raises(H.HespError):
        H.search(H.Plan(), pf, 4, 1, H.SEARCH_SURROGATE, rounds=2, batch=16, seed=1, pool=4)   # no network
    with pytest.raises(H.HespError):     # a capped plan could fail candidates: refused
        H.search(H.Plan(max_tasks=100, max_edges=1000, group=16), pf, 4, 1, H.SEARCH_RANDOM, rounds=2, batch=16,
                 seed=1, pool=4)


def test_exhaustive_sweep_4x4(H, torch):
    """Every one of the 2^20 partitions of the 4x4 instance, each against the
    oracle (about 73 M simulated tasks on the host cores); the best agrees too."""
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in, pf = _pf(H, w)
    n = 1 << 20
    db = H.generate_enumerate(0, n, 4, 1)
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.empty(n, dtype=torch.int32, device="cuda")
    H.simulate_batch(H.Plan(), pf, db, ms, st)
    best = torch.empty(2, dtype=torch.int64, device="cuda")
    H.argmin(ms, best)
    bm, bi = (int(x) for x in best.cpu().numpy())
    assert bool((st == 0).all().item())
    dep = db.depth.cpu().numpy().reshape(n, 20)
    # the enumeration is every depth vector once: digit t of c is depth[c][t]
    digits = (np.arange(n, dtype=np.int64)[:, None] >> np.arange(20)) & 1
    assert np.array_equal(dep, digits.astype(np.uint8))
    msh = ms.cpu().numpy()
    want, _ = O.simulate_batch(pf_in, _host_batch(dep, 4, 1, w.b), NTHREADS)
    mism = np.nonzero(msh != want)[0]
    assert mism.size == 0, f"{mism.size} of {n} partitions differ, first {mism[:8]}"
    assert bm == want.min() and bi == int(np.argmin(want))


def test_surrogate_gain_over_random_selection(H, torch):
    """What the trained network gains: on a platform it never saw, the 1% of all
    2^20 partitions it ranks best are far better than a random 1%, and contain a
    partition close to the exhaustive optimum."""
    w = I.WORKLOADS["surrogate_chol4x4"]
    thr = I.split_threshold(1, 2)
    n_pf, per = 16, 8192
    X = torch.empty((n_pf * per, 32), dtype=torch.int16, device="cuda")
    MS = torch.empty(n_pf * per, dtype=torch.int64, device="cuda")
    st = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    plan = H.Plan()
    for p in range(n_pf):
        pf_in = w.platform(p)
        pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
        db = H.generate_uniform(w.seed, p * per, per, 4, 1, thr)
        H.simulate_batch(plan, pf, db, MS[p * per:(p + 1) * per], st[:per])
        rate = torch.from_numpy(H.mlp_rate_features(pf_in.rmax)).cuda()
        H.mlp_features(db.depth, per, 20, rate, X[p * per:(p + 1) * per])
    lms = torch.log(MS.double())
    mu, sigma = float(lms.mean()), float(lms.std())
    T = torch.empty(n_pf * per, dtype=torch.float32, device="cuda")
    H.mlp_targets(MS, mu, sigma, T)
    m = H.MLP(2)
    m.train(X, T, 2048, 1500, 1e-3, seed=3)
    n = 1 << 20
    pf_in = w.platform(1000)
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    db = H.generate_enumerate(0, n, 4, 1)
    ms = torch.empty(n, dtype=torch.int64, device="cuda")
    H.simulate_batch(plan, pf, db, ms, st)
    rate = torch.from_numpy(H.mlp_rate_features(pf_in.rmax)).cuda()
    Xh = torch.empty((n, 32), dtype=torch.int16, device="cuda")
    H.mlp_features(db.depth, n, 20, rate, Xh)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    m.forward(Xh, y)
    k = n // 100
    top = ms[H.topk(y, k).long()].cpu().numpy()
    msh = ms.cpu().numpy()
    rnd = msh[np.random.default_rng(0).choice(n, k, replace=False)]
    best = msh.min()
    print("top1% best/opt", top.min() / best, "random1% best/opt", rnd.min() / best,
          "mean ratio", top.mean() / rnd.mean())
    assert top.mean() < 0.95 * rnd.mean()
    assert top.min() <= 1.02 * best
