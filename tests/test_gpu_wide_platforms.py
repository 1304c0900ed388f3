"""GPU parity on platforms wider than one 16-lane row of the wavefront (17 to 64
processors of the section 2 platform model) and at the 16-processor boundary:
makespans bit-exact against the CPU oracle under every heuristic class, the
caching policies and the shared interconnect, for each lane-group size that
holds the platform."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import inputs as I

pytestmark = pytest.mark.gpu
NTHREADS = min(16, os.cpu_count() or 1)
PLATFORMS = {"p16": (14, 2), "p17": (15, 2), "p20": (16, 4), "p40": (36, 4), "p64": (60, 4)}   # (CPUs, accelerators)
HEURISTICS = [(0, 0, 0), (1, 1, 0), (0, 2, 7), (1, 3, 0)]   # (order, select, seed)


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


def _platform(name):
    n_cpu, n_acc = PLATFORMS[name]
    return I.make_platform(I.cpu_accel_types(n_cpu, n_acc), seed=3 + n_cpu)


def _groups(pf):
    return [64] + ([32] if pf.n_procs <= 32 else []) + ([16] if pf.n_procs <= 16 else [])


def _run(H, torch, pf_in, batch, max_level, policy, group):
    pf = H.Platform.from_inputs(pf_in, batch.b, max_level)
    db = H.DeviceBatch.from_host(batch)
    ms = torch.full((batch.n,), -7, dtype=torch.int64, device="cuda")
    st = torch.full((batch.n,), 99, dtype=torch.int32, device="cuda")
    H.simulate_batch(H.Plan(group=group), pf, db, ms, st, policy=policy)
    torch.cuda.synchronize()
    assert bool((st == 0).all().item())
    return ms.cpu().numpy()


@pytest.mark.parametrize("heur", HEURISTICS)
@pytest.mark.parametrize("name", list(PLATFORMS))
def test_parity_wide_platforms(H, torch, name, heur):
    pf = _platform(name)
    assert pf.n_procs == sum(PLATFORMS[name])
    bt = I.uniform_batch(17 + pf.n_procs, 96, 6, 512, 2, 1, 3)
    want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=heur)
    for group in _groups(pf):
        got = _run(H, torch, pf, bt, 2, (heur[0], heur[1], 0, heur[2], 0), group)
        assert np.array_equal(got, want), (name, heur, group)


@pytest.mark.parametrize("cache,bus", [(1, 0), (2, 0), (0, 1), (2, 1)])
@pytest.mark.parametrize("name", ["p17", "p64"])
def test_parity_wide_platforms_memory_policies(H, torch, name, cache, bus):
    pf = _platform(name)
    bt = I.uniform_batch(29 + pf.n_procs, 64, 5, 512, 2, 1, 3)
    want, _ = O.simulate_batch(pf, bt, NTHREADS, policy=(0, 0, 0, cache, bus))
    for group in _groups(pf):
        got = _run(H, torch, pf, bt, 2, (0, 0, cache, 0, bus), group)
        assert np.array_equal(got, want), (name, cache, bus, group)
