"""GPU parity of grain batches (partition parameter p = 1/f for any integer f,
section 2.1; partially overlapping blocks, Fig. 4) against the CPU oracle:
makespans, expanded task counts and dependence edge counts bit-exact over
factor lists with and without common divisors, several heuristics and caching
policies, a shared-memory platform, more candidates than slots, an empty
batch, a bad grain index, and sampled candidates of the 16x16-tile workload in
the benchmark's launch configuration."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)
PLATS = [I.make_platform(I.cpu_accel_types(2, 1), seed=7),
         I.make_platform(I.cpu_accel_types(3, 2), seed=8),
         I.make_platform(I.cpu_accel_types(1, 3), seed=9),
         I.make_platform(I.big_little_types(2, 2), seed=10)]


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


def _gpu(H, torch, pf, nt, fac, b, grain, pol, slots):
    n = grain.shape[0]
    g = torch.from_numpy(np.ascontiguousarray(grain)).cuda()
    ms = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    ntk = torch.zeros(n, dtype=torch.int32, device="cuda")
    ne = torch.zeros(n, dtype=torch.int64, device="cuda")
    st = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    gp = H.grain_platform(pf, b, fac)
    H.simulate_grain_batch(gp, nt, fac, g, ms, ntk, ne, st, slots=slots, policy=pol)
    torch.cuda.synchronize()
    return ms.cpu().numpy(), ntk.cpu().numpy(), ne.cpu().numpy(), st.cpu().numpy()


CASES = [  # nt, fac, platform, (order, select, cache), candidates, slots
    (3, [1, 2, 3], 0, (0, 0, 0), 200, 64),
    (4, [1, 2, 3, 4, 6], 1, (0, 0, 0), 150, 48),
    (5, [2, 3], 2, (1, 0, 1), 120, 40),
    (4, [1, 5], 1, (0, 1, 2), 100, 100),
    (3, [1, 2, 4], 0, (1, 1, 0), 100, 37),
    (2, [6], 1, (0, 0, 0), 20, 8),
    (4, [1, 2, 3], 3, (0, 0, 0), 90, 30),
    (1, [1, 2, 3, 4, 6, 8, 12, 16], 1, (0, 0, 1), 40, 16),
    (6, [1, 3, 2], 2, (0, 0, 2), 64, 64),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_parity_with_oracle(H, torch, case):
    nt, fac, pi, pol, n, slots = CASES[case]
    b = 1024
    pf = PLATS[pi]
    grain = I.grain_batch(40 + case, n, nt, len(fac))
    print(f"grain parity case {case}: nt={nt} fac={fac} pol={pol} n={n} slots={slots}", flush=True)
    ms, ntk, ne, st = _gpu(H, torch, pf, nt, fac, b, grain, pol, slots)
    assert np.all(st == 0)
    want, wn = O.simulate_grain_batch(pf, nt, fac, b, grain, n_threads=NTHREADS, policy=(pol[0], pol[1], 0, pol[2]))
    assert np.array_equal(ms, want)
    assert np.array_equal(ntk, wn)
    for c in range(0, n, max(1, n // 6)):
        s = O.simulate_grain(pf, nt, fac, b, grain[c], policy=(pol[0], pol[1], 0, pol[2]))
        assert ne[c] == len(s.edges) and ms[c] == s.makespan


def test_power_of_two_factors_match_the_depth_path(H, torch):
    pf = PLATS[1]
    w = I.uniform_batch(11, 64, 4, 1024, 2, 1, 2)
    dep = np.asarray(w.depth, np.uint8).reshape(64, -1)
    ms, _, _, st = _gpu(H, torch, pf, 4, [1, 2, 4], 1024, dep, (0, 0, 0), 64)
    want, _ = O.simulate_batch(pf, w, n_threads=NTHREADS)
    assert np.all(st == 0) and np.array_equal(ms, want)


def test_empty_batch_and_bad_grain(H, torch):
    pf = PLATS[0]
    ms, _, _, _ = _gpu(H, torch, pf, 3, [1, 2], 1024, np.zeros((0, I.tet(3)), np.uint8), (0, 0, 0), 8)
    assert ms.shape == (0,)
    grain = I.grain_batch(3, 6, 3, 2)
    grain[2, 4] = 2                                         # index past the two factors
    ms, ntk, _, st = _gpu(H, torch, pf, 3, [1, 2], 1024, grain, (0, 0, 0), 4)
    assert st[2] == -1 and ms[2] == -1 and ntk[2] == 0
    ok = [c for c in range(6) if c != 2]
    want, _ = O.simulate_grain_batch(pf, 3, [1, 2], 1024, grain[ok], n_threads=NTHREADS)
    assert np.all(st[ok] == 0) and np.array_equal(ms[ok], want)


def test_full_workload_sample(H, torch):
    w = I.GRAIN_WORKLOAD
    pf = I.make_platform(w["ptypes"], w["seed"])
    n = 512
    grain = I.grain_batch(w["seed"], n, w["nt"], len(w["fac"]))
    print(f"grain full-size sample: nt={w['nt']} fac={w['fac']} n={n}", flush=True)
    ms, ntk, ne, st = _gpu(H, torch, pf, w["nt"], list(w["fac"]), w["b"], grain, (0, 0, 0), 2048)
    assert np.all(st == 0)
    for c in (0, 1, 97, 255, 510, 511):
        s = O.simulate_grain(pf, w["nt"], list(w["fac"]), w["b"], grain[c])
        assert ms[c] == s.makespan and ntk[c] == s.n_tasks and ne[c] == len(s.edges), c
