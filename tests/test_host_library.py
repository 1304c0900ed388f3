"""CPU tests of the C ABI library: symbols, argument checks, cost tables and the
structural expansion (no GPU needed: these entry points run on the host)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_1602_05510_amd import hesp as H
from paper_1602_05510_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hesp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hesp_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = H.lib()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


def test_library_exports_match_nm():
    import subprocess
    out = subprocess.check_output(["nm", "-D", "--defined-only", H.LIB_PATH], text=True)
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for n in declared_functions():
        assert n in exported, n


def test_cost_tables_match_oracle():
    for name in ["chol4x4_b512_d1", "chol16x16_b1024_d2", "ragged_bl_b512_d3", "chol64x64_b1024_d3"]:
        w = I.WORKLOADS[name]
        pf = w.platform()
        cost, xfer = H.cost_tables(pf.rmax, pf.h, w.b, w.dmax, shared_memory=pf.shared_memory)
        for pt in range(pf.n_ptypes):
            for k in range(4):
                for l in range(w.dmax + 1):
                    assert cost[pt, k, l] == O.task_time(k, w.b >> l, int(pf.rmax[pt, k]), int(pf.h[pt]))
        for k in range(len(xfer)):
            assert xfer[k] == O.transfer_time(k, w.b >> w.dmax, pf)


def test_argument_errors():
    with pytest.raises(H.HespError) as e:
        H.expand(0, 0, np.zeros(0, np.uint8))
    assert e.value.code == H.HESP_EINVAL
    with pytest.raises(H.HespError):
        H.expand(2, 1, np.array([0, 2, 0, 0], np.uint8))      # depth above dmax
    with pytest.raises(H.HespError):
        H.expand(64, 4, np.zeros(45760, np.uint8))            # above the supported depth
    with pytest.raises(H.HespError):
        H.cost_tables(np.array([[1, 1, 1, 0]]), np.array([64]), 512, 1)  # zero rate
    with pytest.raises(H.HespError):
        H.cost_tables(np.array([[1, 1, 1, 1]]), np.array([64]), 502, 2)  # b not divisible
    assert "hesp_cost_tables" in H.lib().hesp_last_error().decode()


def _closure_contains(n, edges, queries):
    succ = [[] for _ in range(n)]
    for u, v in edges:
        succ[u].append(v)
    reach_cache = {}

    def reach(u):
        if u in reach_cache:
            return reach_cache[u]
        seen = set()
        stack = list(succ[u])
        while stack:
            x = stack.pop()
            if x not in seen:
                seen.add(x)
                stack.extend(succ[x])
        reach_cache[u] = seen
        return seen

    return all(v in reach(u) for u, v in queries)


def _compare_with_oracle(nt, dmax, depth, pf, b):
    tasks, ptr, idx = H.expand(nt, dmax, depth)
    s = O.simulate(pf, nt, dmax, b, depth)
    n = len(tasks)
    assert n == s.n_tasks
    key_lib = {tuple(int(x) for x in tasks[t]): t for t in range(n)}
    key_or = {tuple(int(x) for x in s.tasks[t]): t for t in range(n)}
    assert set(key_lib) == set(key_or)
    to_lib = np.zeros(n, np.int64)
    for k, t in key_or.items():
        to_lib[t] = key_lib[k]
    lib_edges = set()
    for u in range(n):
        for e in range(ptr[u], ptr[u + 1]):
            v = int(idx[e])
            assert v > u, "numbering must be topological"
            lib_edges.add((u, v))
    assert len(lib_edges) == ptr[n]                       # no duplicate edges
    or_edges = {(int(to_lib[u]), int(to_lib[v])) for u, v in s.edges}
    assert lib_edges <= or_edges                           # every kept edge is a real hazard
    missing = or_edges - lib_edges
    assert _closure_contains(n, lib_edges, missing)        # the dropped ones are implied
    # same critical times from both edge sets
    W = np.zeros(n, np.int64)
    for t in range(n):
        k, l = int(tasks[t][0]), int(tasks[t][1])
        W[t] = sum(O.task_time(k, b >> l, int(pf.rmax[pt, k]), int(pf.h[pt])) for pt in pf.proc_type)
    rank = np.zeros(n, np.int64)
    for t in range(n - 1, -1, -1):
        best = 0
        for e in range(ptr[t], ptr[t + 1]):
            best = max(best, rank[idx[e]])
        rank[t] = W[t] + best
    for t in range(n):
        assert rank[key_lib[tuple(int(x) for x in s.tasks[t])]] == s.rank[t]


@pytest.mark.parametrize("nt,dmax", [(1, 0), (1, 3), (2, 1), (2, 3), (3, 2), (4, 1), (4, 3), (5, 2), (6, 3), (1, 4), (2, 4), (1, 5),
                                     (2, 5)])
def test_structural_expansion_vs_atom_scan(nt, dmax):
    pf = I.make_platform(I.cpu_accel_types(2, 1), seed=3)
    rng = np.random.default_rng(100 * nt + dmax)
    n_top = nt * (nt + 1) * (nt + 2) // 6
    for trial in range(6):
        dep = rng.integers(0, dmax + 1, n_top).astype(np.uint8)
        if trial == 0:
            dep[:] = 0
        if trial == 1:
            dep[:] = dmax
        _compare_with_oracle(nt, dmax, dep, pf, 64 << dmax)


def test_structural_expansion_workload_candidates():
    for name, count in [("chol4x4_b512_d1", 8), ("chol16x16_b1024_d2", 2)]:
        w = I.WORKLOADS[name]
        pf = w.platform()
        bt = w.batch(count)
        for c in range(bt.n):
            _compare_with_oracle(w.nt, w.dmax, bt.candidate(c), pf, w.b)


def test_expand_counts_two_call():
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    bt = w.batch(3)
    for c in range(3):
        tasks, ptr, idx = H.expand(w.nt, w.dmax, bt.candidate(c))
        s = O.simulate(w.platform(), w.nt, w.dmax, w.b, bt.candidate(c), detail=False)
        assert len(tasks) > 0 and ptr[-1] == len(idx)


def test_rate_features():
    # log2(R / 2^17) / 4: R = 2^17 gives 0, R = 2^21 gives 1, R = 2^13 gives -1
    r = np.array([[1 << 17, 1 << 21, 1 << 13, 3 << 17]], np.int64)
    f = H.mlp_rate_features(r)
    assert f.dtype == np.float32 and f.shape == (4,)
    assert f[0] == 0.0 and f[1] == 1.0 and f[2] == -1.0
    assert abs(f[3] - np.log2(3) / 4) < 1e-7
    with pytest.raises(H.HespError):
        H.mlp_rate_features(np.array([[1, 2, 0, 4]], np.int64))


def test_search_argument_errors_need_no_gpu():
    # argument checks run before any device work
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = H.Platform.from_inputs(w.platform(), w.b, w.dmax)
    sp = H.SearchParams(H.SEARCH_GREEDY, 4, 1, 0, 16, 1, 16, 16, 4, 0, 0, 1, None, None, 0, 0, 512, 1e-3, 0)
    best = np.zeros(20, np.uint8)
    ms = H.i64(0)
    rc = H.lib().hesp_search(ctypes.c_void_p(1), ctypes.byref(pf.c), H.Policy(0, 0, 0), ctypes.byref(sp),
                             best.ctypes.data_as(ctypes.c_void_p), ctypes.byref(ms), None, None)
    assert rc == H.HESP_EINVAL          # rounds = 0


def test_unsupported_policies_rejected_before_device_work():
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = H.Platform.from_inputs(w.platform(), w.b, w.dmax)
    b = H.BatchC(1, 4, 1, None, None, None, None)
    out = H.OutputsC(None, None, None, None, None, None, None)
    for pol in [(2, 0, 0), (0, 4, 0), (0, 0, 3), (0, 0, -1), (1, -1, 0), (0, 0, 0, 0, 2)]:   # no such setting
        rc = H.lib().hesp_simulate_batch(ctypes.c_void_p(1), ctypes.byref(pf.c), H.Policy(*pol), ctypes.byref(b),
                                         ctypes.byref(out), None)
        assert rc == H.HESP_EUNSUPPORTED, pol


def test_solve_argument_errors_need_no_gpu():
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = H.Platform.from_inputs(w.platform(), w.b, w.dmax)
    fake = ctypes.c_void_p(1)          # never dereferenced: every check runs first
    def call(sp, plan=fake):
        return H.lib().hesp_solve(plan, ctypes.byref(pf.c), H.Policy(0, 0, 0), ctypes.byref(sp), fake, fake, fake,
                                  None, None, None)
    assert call(H.SolveParams(1, 4, 1, 4, 0, 0, 0), plan=None) == H.HESP_EINVAL
    assert call(H.SolveParams(0, 4, 1, 4, 0, 0, 0)) == H.HESP_EINVAL            # no chains
    assert call(H.SolveParams(1, 4, 1, 0, 0, 0, 0)) == H.HESP_EINVAL            # no iterations
    assert call(H.SolveParams(1, 4, 1, 4, 3, 0, 0)) == H.HESP_EINVAL            # no such list
    assert call(H.SolveParams(1, 4, 1, 4, 0, 2, 0)) == H.HESP_EINVAL            # no such sampling
    assert call(H.SolveParams(1, 4, 2, 4, 0, 0, 0)) == H.HESP_EINVAL            # dmax above the tables
    assert call(H.SolveParams(1, 2, 6, 4, 0, 0, 0)) == H.HESP_EINVAL            # dmax above 5
    assert call(H.SolveParams(1, 29, 0, 4, 0, 0, 0)) == H.HESP_EUNSUPPORTED     # tet(29) > 4096 clusters
    assert "hesp_solve" in H.lib().hesp_last_error().decode()



def test_solve_tree_argument_errors_need_no_gpu():
    w = I.WORKLOADS["chol4x4_b512_d1"]
    pf = H.Platform.from_inputs(w.platform(), w.b, 2)
    fake = ctypes.c_void_p(1)
    def call(sp, plan=fake):
        return H.lib().hesp_solve_tree(plan, ctypes.byref(pf.c), H.Policy(0, 0, 0), ctypes.byref(sp), fake, fake,
                                       fake, None, None, None)
    assert call(H.SolveParams(1, 4, 1, 4, 0, 0, 0), plan=None) == H.HESP_EINVAL
    assert call(H.SolveParams(1, 4, 0, 4, 0, 0, 0)) == H.HESP_EINVAL            # no level below dmax
    assert call(H.SolveParams(1, 1, 6, 4, 0, 0, 0)) == H.HESP_EINVAL            # dmax above 5
    assert call(H.SolveParams(1, 14, 2, 4, 0, 0, 0)) == H.HESP_EUNSUPPORTED     # 560 + 4,060 > 4,096 flags
    assert call(H.SolveParams(1, 4, 2, 4, 5, 0, 0)) == H.HESP_EINVAL            # no such list


def test_surrogate_binding_rejects_undersized_tensors():
    """The surrogate calls check every tensor's kind and length before anything
    reaches the library (a CPU-side object stands in for the device network)."""
    import torch
    m = object.__new__(H.MLP)          # no device network: nothing may be launched
    m.h = None
    x = torch.zeros((1024, 32), dtype=torch.int16)
    t = torch.zeros(1024, dtype=torch.float32)
    loss = torch.zeros(10, dtype=torch.float32)
    cases = [
        lambda: m.forward(x[:100], torch.zeros(101, dtype=torch.float32)),       # x short of rows
        lambda: m.forward(x, torch.zeros(1024, dtype=torch.float64)),            # y not float32
        lambda: m.grad(x[:511], t, 512),                                         # x short
        lambda: m.grad(x, t[:500], 512),                                         # t short
        lambda: m.grad(x, t, 512, torch.zeros(0, dtype=torch.float32)),          # no loss slot
        lambda: m.grad(x.float(), t, 512),                                       # x not bf16 bits
        lambda: m.train(x[:1000], t, 512, 10, 1e-3),                             # x short of t's rows
        lambda: m.train(x, t, 512, 11, 1e-3, loss=loss),                         # loss short of steps
        lambda: m.train(x, t.double(), 512, 10, 1e-3),                           # t not float32
        lambda: m.train(x.t(), t, 512, 10, 1e-3),                                # not contiguous
    ]
    for i, f in enumerate(cases):
        with pytest.raises(H.HespError) as e:
            f()
        assert e.value.code == H.HESP_EINVAL, i
