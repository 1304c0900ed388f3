"""GPU tests of the iterative scheduler-partitioner (hesp_solve, section 2.1
"Iterative solver") through the C ABI: every chain's trajectory (makespan per
iteration, cluster changed, new depth, score), best partition and last partition
against the CPU reference oracle/solver_ref.py on the same seeded inputs."""
import numpy as np
import pytest

from oracle import solver_ref as S
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


def _run(H, torch, pf_in, nt, dmax, b, depth0, iters, lst, sampling, seed, policy=(0, 0, 0), plan=None):
    pf = H.Platform.from_inputs(pf_in, b, dmax)
    d = torch.from_numpy(np.ascontiguousarray(depth0, np.uint8)).cuda()
    best, best_ms, trace, steps = H.solve(plan or H.Plan(), pf, nt, dmax, d, iters, lst, sampling, seed,
                                          policy=policy)
    torch.cuda.synchronize()
    return (best.cpu().numpy(), best_ms.cpu().numpy(), trace.cpu().numpy(), steps.cpu().numpy(),
            d.cpu().numpy())


def _check_chain(pf_in, nt, dmax, b, depth0, iters, lst, sampling, seed, got, r, policy=(0, 0, 0)):
    best, best_ms, trace, steps, last = got
    # library policy (order, select, cache, seed) -> oracle policy (order, select, seed, cache)
    pol = (policy[0], policy[1], policy[3] if len(policy) > 3 else 0, policy[2])
    bd, bm, tr, st = S.solve(pf_in, nt, dmax, b, iters, lst, sampling, seed + r, policy=pol, depth0=depth0[r])
    assert list(trace[r]) == tr, (r, lst, sampling)
    want_steps = [(-1, -1, 0) if x is None else x for x in st]
    assert [tuple(int(v) for v in s) for s in steps[r]] == want_steps, (r, lst, sampling)
    assert int(best_ms[r]) == bm and np.array_equal(best[r], bd), (r, lst, sampling)
    dep = np.array(depth0[r], np.uint8)
    for x in st:
        if x is not None:
            dep[x[0]] = x[1]
    assert np.array_equal(last[r], dep)


def test_hand_derived_oscillation(H, torch):
    """Two identical CPUs, one 512 tile, depths 0..1: split (score 677,205) and
    merge (65,537) alternate; the unsplit partition stays the best."""
    pf_in = I.make_platform([I.ProcType("cpu", 2, 32000, 32000, 64, False)], seed=0)
    best, best_ms, trace, steps, last = _run(H, torch, pf_in, 1, 1, 512, np.zeros((1, 1)), 5, 0, 0, 0)
    assert list(trace[0]) == [1419947, 1485484, 1419947, 1485484, 1419947]
    assert [tuple(s) for s in steps[0]] == [(0, 1, 677205), (0, 0, 65537)] * 2 + [(0, 1, 677205)]
    assert int(best_ms[0]) == 1419947 and list(best[0]) == [0] and list(last[0]) == [1]


def test_fixed_point(H, torch):
    pf_in = I.make_platform([I.ProcType("cpu", 1, 32000, 32000, 64, False),
                             I.ProcType("acc", 1, 1024000, 1024000, 512, True)], seed=0)
    best, best_ms, trace, steps, last = _run(H, torch, pf_in, 1, 1, 512, np.zeros((1, 1)), 4, 0, 0, 0)
    assert list(trace[0]) == [272145] * 4
    assert [tuple(s) for s in steps[0]] == [(-1, -1, 0)] * 4


@pytest.mark.parametrize("lst", [0, 1, 2])
@pytest.mark.parametrize("sampling", [0, 1])
def test_chains_match_reference(H, torch, lst, sampling):
    """nt = 6, depths 0..2 on the heterogeneous 16-CPU + 4-accelerator platform:
    six chains from random initial partitions, twelve iterations each."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax, B, iters, seed = 6, 2, 6, 12, 1000 + 10 * lst + sampling
    bt = I.uniform_batch(seed, B, nt, w.b, dmax, 1, 3)
    depth0 = bt.depth.reshape(B, I.tet(nt))
    got = _run(H, torch, pf_in, nt, dmax, w.b, depth0, iters, lst, sampling, seed)
    for r in range(B):
        _check_chain(pf_in, nt, dmax, w.b, depth0, iters, lst, sampling, seed, got, r)


@pytest.mark.parametrize("policy", [(1, 1, 0, 0), (0, 2, 0, 77), (0, 3, 0, 0)])
def test_chains_under_other_heuristics(H, torch, policy):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax, B, iters, seed = 4, 2, 3, 8, 5
    bt = I.uniform_batch(seed, B, nt, w.b, dmax, 1, 3)
    depth0 = bt.depth.reshape(B, I.tet(nt))
    got = _run(H, torch, pf_in, nt, dmax, w.b, depth0, iters, 0, 1, seed, policy=policy)
    for r in range(B):
        _check_chain(pf_in, nt, dmax, w.b, depth0, iters, 0, 1, seed, got, r, policy=policy)


@pytest.mark.parametrize("nt,dmax,pn,pd,lst,sampling", [(3, 4, 2, 3, 0, 1), (2, 5, 3, 4, 0, 1), (3, 4, 2, 3, 1, 0)])
def test_chains_at_depth_four_and_five(H, torch, nt, dmax, pn, pd, lst, sampling):
    """Chains on tables of 4 and 5 levels, from initial partitions with tasks at
    depth 4 and 5, sixteen iterations, some steps choosing depth 4 or 5 (section
    3.2 reports best partitions of DAG depth up to 5)."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    B, iters, seed = 4, 16, 9
    bt = I.uniform_batch(78, B, nt, w.b, dmax, pn, pd)
    depth0 = bt.depth.reshape(B, I.tet(nt))
    assert (depth0 >= 4).any()
    got = _run(H, torch, pf_in, nt, dmax, w.b, depth0, iters, lst, sampling, seed)
    deep_steps = 0
    for r in range(B):
        _check_chain(pf_in, nt, dmax, w.b, depth0, iters, lst, sampling, seed, got, r)
        deep_steps += int((got[3][r][:, 1] >= 4).sum())
    assert deep_steps >= 3


def test_edge_cases(H, torch):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    # dmax = 0: no other depth, so no candidate at all
    got = _run(H, torch, pf_in, 3, 0, w.b, np.zeros((2, 10)), 3, 0, 0, 0)
    assert (got[3][:, :, 0] == -1).all() and (got[2] == got[2][:, :1]).all()
    # a chain with a depth above dmax fails (-1) without disturbing the others
    d0 = np.zeros((3, 10), np.uint8)
    d0[1, 4] = 3
    best, best_ms, trace, steps, last = _run(H, torch, pf_in, 3, 2, w.b, d0, 4, 1, 0, 0)
    assert (trace[1] == -1).all() and int(best_ms[1]) == -1 and (steps[1][:, 0] == -1).all()
    assert np.array_equal(last[1], d0[1])
    for r in (0, 2):
        _check_chain(pf_in, 3, 2, w.b, d0, 4, 1, 0, 0, (best, best_ms, trace, steps, last), r)


def test_sixteen_tiles_sampled_chains(H, torch):
    """nt = 16 (816 clusters), depths 0..2, 64 chains of 10 All/Soft iterations;
    two chains recomputed by the reference."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax, B, iters, seed = 16, 2, 64, 10, 3
    bt = I.uniform_batch(seed, B, nt, w.b, dmax, 1, 4)
    depth0 = bt.depth.reshape(B, I.tet(nt))
    got = _run(H, torch, pf_in, nt, dmax, w.b, depth0, iters, 0, 1, seed)
    for r in (0, 37):
        _check_chain(pf_in, nt, dmax, w.b, depth0, iters, 0, 1, seed, got, r)
    assert (got[1] <= got[2][:, 0]).all()


# ---------------------------------------------------------------- split-tree partitions

def _run_tree(H, torch, pf_in, nt, dmax, b, flags0, iters, lst, sampling, seed, policy=(0, 0, 0)):
    pf = H.Platform.from_inputs(pf_in, b, dmax)
    f = torch.from_numpy(np.ascontiguousarray(flags0, np.uint8)).cuda()
    best, best_ms, trace, steps = H.solve_tree(H.Plan(), pf, nt, dmax, f, iters, lst, sampling, seed, policy=policy)
    torch.cuda.synchronize()
    return (best.cpu().numpy(), best_ms.cpu().numpy(), trace.cpu().numpy(), steps.cpu().numpy(), f.cpu().numpy())


def _check_tree_chain(pf_in, nt, dmax, b, flags0, iters, lst, sampling, seed, got, r, policy=(0, 0, 0)):
    best, best_ms, trace, steps, last = got
    # library policy (order, select, cache, seed) -> oracle policy (order, select, seed, cache)
    pol = (policy[0], policy[1], policy[3] if len(policy) > 3 else 0, policy[2])
    bf, bm, tr, st = S.solve_tree(pf_in, nt, dmax, b, iters, lst, sampling, seed + r, policy=pol, flags0=flags0[r])
    assert list(trace[r]) == tr, (r, lst, sampling)
    want = [(-1, -1, 0) if x is None else x for x in st]
    assert [tuple(int(v) for v in s) for s in steps[r]] == want, (r, lst, sampling)
    assert int(best_ms[r]) == bm and np.array_equal(best[r], bf)
    fl = np.array(flags0[r], np.uint8)
    for x in st:
        if x is not None:
            S.apply_tree_step(nt, dmax, fl, x)
    assert np.array_equal(last[r], fl)


def test_tree_solver_hand_derived_merge(H, torch):
    pf_in = I.make_platform([I.ProcType("cpu", 1, 32000, 32000, 64, False)], seed=0)
    got = _run_tree(H, torch, pf_in, 1, 2, 512, np.array([[1, 1, 0, 0, 0]]), 3, 0, 0, 0)
    assert list(got[2][0]) == [1518252, 1419947, 1419947]
    assert [tuple(s) for s in got[3][0]] == [(0, 0, 98305), (-1, -1, 0), (-1, -1, 0)]


@pytest.mark.parametrize("lst", [0, 1, 2])
@pytest.mark.parametrize("sampling", [0, 1])
def test_tree_chains_match_reference(H, torch, lst, sampling):
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax, B, iters, seed = 5, 2, 5, 10, 300 + 10 * lst + sampling
    tb = I.tree_batch(seed, B, nt, w.b, dmax, 1, 3)
    flags0 = tb.depth.reshape(B, -1)
    got = _run_tree(H, torch, pf_in, nt, dmax, w.b, flags0, iters, lst, sampling, seed)
    for r in range(B):
        _check_tree_chain(pf_in, nt, dmax, w.b, flags0, iters, lst, sampling, seed, got, r)


@pytest.mark.parametrize("dmax", [4, 5])
def test_tree_chains_depth_four_and_five(H, torch, dmax):
    """One 1024 tile split up to 4 or 5 times (145 or 961 split flags), three
    chains from random split trees, ten iterations each."""
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in = w.platform()
    nt, B, iters, seed = 1, 3, 10, 5
    tb = I.tree_batch(23, B, nt, 1024, dmax, 1, 2)
    flags0 = tb.depth.reshape(B, -1)
    got = _run_tree(H, torch, pf_in, nt, dmax, 1024, flags0, iters, 0, 1, seed)
    for r in range(B):
        _check_tree_chain(pf_in, nt, dmax, 1024, flags0, iters, 0, 1, seed, got, r)


def test_tree_chains_depth_three_and_other_heuristics(H, torch):
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf_in = w.platform()
    nt, dmax, B, iters, seed = 3, 3, 4, 8, 17
    tb = I.tree_batch(seed, B, nt, w.b, dmax, 1, 2)
    flags0 = tb.depth.reshape(B, -1)
    for policy in ((0, 0, 0), (1, 1, 2, 0), (0, 3, 0, 0)):
        got = _run_tree(H, torch, pf_in, nt, dmax, w.b, flags0, iters, 0, 1, seed, policy=policy)
        for r in range(B):
            _check_tree_chain(pf_in, nt, dmax, w.b, flags0, iters, 0, 1, seed, got, r, policy=policy)


def test_tree_chains_twelve_tiles_sampled(H, torch):
    """nt = 12 (364 + 2,600 nodes), depths 0..2, 48 chains; two recomputed."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    nt, dmax, B, iters, seed = 12, 2, 48, 8, 5
    tb = I.tree_batch(seed, B, nt, w.b, dmax, 1, 4)
    flags0 = tb.depth.reshape(B, -1)
    got = _run_tree(H, torch, pf_in, nt, dmax, w.b, flags0, iters, 1, 1, seed)
    for r in (0, 29):
        _check_tree_chain(pf_in, nt, dmax, w.b, flags0, iters, 1, 1, seed, got, r)
