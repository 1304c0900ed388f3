"""Thin ctypes binding of libhesp.so (include/hesp.h), argument marshalling only.

Every step of the simulation runs in the library's HIP kernels; PyTorch is used
for device memory and streams.  Importing this module fails loudly when the
compiled library is missing.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# HESP_SANITIZE=1: the build whose host code carries the address and
# undefined-behaviour sanitizers (python -m paper_1602_05510_amd.build --sanitize)
LIB_PATH = os.path.join(PKG, "libhesp_san.so" if os.environ.get("HESP_SANITIZE") == "1" else "libhesp.so")

HESP_OK, HESP_EINVAL, HESP_ENOMEM, HESP_EHIP, HESP_ECAPACITY, HESP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
MAX_PROCS, MAX_PTYPES, MAX_MEM, MAX_LEVEL, MAX_FINE = 64, 8, 16, 5, 512

P = ctypes.c_void_p
i32, i64, u32, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64


class CostModel(ctypes.Structure):
    _fields_ = [("n_ptypes", i32), ("rmax_mflops", P), ("h", P), ("b", i64), ("max_level", i32),
                ("latency_ns", i64), ("bw_bytes_per_ns", i64), ("elem_bytes", i64), ("shared_memory", i32)]


class PlatformC(ctypes.Structure):
    _fields_ = [("n_procs", i32), ("n_ptypes", i32), ("n_mem", i32), ("max_level", i32),
                ("proc_type", P), ("proc_mem", P), ("cost_ns", P), ("xfer_ns", P), ("capacity", P), ("link", P)]


class Policy(ctypes.Structure):
    _fields_ = [("order", i32), ("select", i32), ("cache", i32), ("seed", u64), ("bus", i32)]


class Task(ctypes.Structure):
    _fields_ = [("kind", i32), ("level", i32), ("K", i32), ("I", i32), ("J", i32)]


class BatchC(ctypes.Structure):
    _fields_ = [("n_cand", i32), ("nt", i32), ("dmax", i32), ("d_nt", P), ("d_dmax", P), ("d_mask_off", P),
                ("d_depth", P)]


class TreeBatchC(ctypes.Structure):
    _fields_ = [("n_cand", i32), ("nt", i32), ("dmax", i32), ("d_flags", P)]


class GrainBatchC(ctypes.Structure):
    _fields_ = [("n_cand", i32), ("nt", i32), ("n_fac", i32), ("fac", P), ("grain", P)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("slots", i32), ("max_tasks", i64), ("max_edges", i64), ("chunks", i32), ("group", i32),
                ("prep_edges", i32), ("fuse", i32)]


class OutputsC(ctypes.Structure):
    _fields_ = [("d_makespan", P), ("d_status", P), ("d_n_tasks", P), ("d_sched_off", P), ("d_proc", P),
                ("d_start", P), ("d_finish", P)]


SEARCH_RANDOM, SEARCH_GREEDY, SEARCH_SURROGATE = 0, 1, 2
# heuristics of section 2.1: policy = (order, select, cache)
ORDER_PL, ORDER_FCFS = 0, 1
SELECT_EFT, SELECT_EIT, SELECT_RP, SELECT_FP = 0, 1, 2, 3
CACHE_WB, CACHE_WT, CACHE_WA = 0, 1, 2


class SearchParams(ctypes.Structure):
    _fields_ = [("mode", i32), ("nt", i32), ("dmax", i32), ("rounds", i32), ("batch", i32), ("warm_rounds", i32),
                ("warm_batch", i32), ("proposals", i32), ("pool", i32), ("split_thr", u32), ("mutate_thr", u32),
                ("seed", u64), ("mlp", P), ("d_rate", P), ("n_rate", i32), ("train_steps", i32),
                ("train_batch", i32), ("lr", ctypes.c_float), ("replay", i64)]


# iterative solver (section 2.1): candidate lists and final selection
LIST_ALL, LIST_CP, LIST_SHALLOW = 0, 1, 2
SAMPLE_HARD, SAMPLE_SOFT = 0, 1


class SolveParams(ctypes.Structure):
    _fields_ = [("n_chains", i32), ("nt", i32), ("dmax", i32), ("iters", i32), ("list", i32), ("sampling", i32),
                ("seed", u64)]


class TracePoint(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("best_makespan", i64), ("simulated", i64), ("proposed", i64)]


class HespError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python -m paper_1602_05510_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.hesp_last_error.restype = ctypes.c_char_p
        L.hesp_version.restype = ctypes.c_char_p
        sig = {
            "hesp_cost_tables": [ctypes.POINTER(CostModel), P, P],
            "hesp_expand": [i32, i32, P, P, P, P, P, P],
            "hesp_generate_uniform": [u64, i64, i32, i32, i32, u32, P, P],
            "hesp_generate_ragged_shape": [u64, i64, i32, i32, i32, i32, P, P, P, P],
            "hesp_generate_ragged_depth": [u64, i64, ctypes.POINTER(BatchC), u32, P, P],
            "hesp_count_batch": [ctypes.POINTER(BatchC), P, P, P],
            "hesp_plan_create": [ctypes.POINTER(P), ctypes.POINTER(PlanOpts)],
            "hesp_plan_destroy": [P],
            "hesp_plan_bytes": [P, ctypes.POINTER(i64)],
            "hesp_plan_timing": [P, i32],
            "hesp_plan_last_ms": [P, P],
            "hesp_simulate_batch": [P, ctypes.POINTER(PlatformC), Policy, ctypes.POINTER(BatchC),
                                    ctypes.POINTER(OutputsC), P],
            "hesp_simulate_batch_noalloc": [ctypes.POINTER(PlatformC), Policy, ctypes.POINTER(BatchC),
                                            ctypes.POINTER(OutputsC), i32, P],
            "hesp_argmin": [P, i32, P, P],
            "hesp_mlp_create": [ctypes.POINTER(P), u64],
            "hesp_mlp_destroy": [P],
            "hesp_mlp_set_params": [P, P, i64],
            "hesp_mlp_get_params": [P, P, i64],
            "hesp_mlp_get_grads": [P, P, i64],
            "hesp_mlp_features": [P, i64, i32, P, i32, P, P],
            "hesp_mlp_targets": [P, i64, ctypes.c_float, ctypes.c_float, P, P],
            "hesp_mlp_forward": [P, P, i64, P, P],
            "hesp_mlp_grad": [P, P, P, i32, P, P],
            "hesp_mlp_adam": [P, ctypes.c_float, P],
            "hesp_mlp_train": [P, P, P, i64, i32, i32, ctypes.c_float, u64, P, P],
            "hesp_mlp_rate_features": [ctypes.POINTER(CostModel), P, i32],
            "hesp_mlp_features_agg": [P, i64, i32, P, i32, P, P],
            "hesp_generate_enumerate": [i64, i32, i32, i32, P, P],
            "hesp_topk_makespan": [P, i32, i32, P, P, i64, P],
            "hesp_topk_score": [P, i32, i32, P, P, i64, P],
            "hesp_search": [P, ctypes.POINTER(PlatformC), Policy, ctypes.POINTER(SearchParams), P,
                            ctypes.POINTER(i64), P, P],
            "hesp_generate_tree_uniform": [u64, i64, i32, i32, i32, u32, P, P],
            "hesp_count_tree_batch": [ctypes.POINTER(TreeBatchC), P, P, P],
            "hesp_simulate_tree_batch": [P, ctypes.POINTER(PlatformC), Policy, ctypes.POINTER(TreeBatchC),
                                         ctypes.POINTER(OutputsC), P],
            "hesp_solve": [P, ctypes.POINTER(PlatformC), Policy, ctypes.POINTER(SolveParams), P, P, P, P, P, P],
            "hesp_solve_tree": [P, ctypes.POINTER(PlatformC), Policy, ctypes.POINTER(SolveParams), P, P, P, P, P, P],
            "hesp_grain_cost_tables": [ctypes.POINTER(CostModel), i32, P, P, P],
            "hesp_grain_workspace": [ctypes.POINTER(GrainBatchC), i32, i32, ctypes.POINTER(i64)],
            "hesp_simulate_grain_batch": [ctypes.POINTER(PlatformC), Policy, ctypes.POINTER(GrainBatchC), P, P, P, P,
                                          P, i64, i32, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = i32
        L.hesp_mlp_param_count.argtypes = []
        L.hesp_mlp_param_count.restype = i64
        L.hesp_tree_flag_count.argtypes = [i32, i32]
        L.hesp_tree_flag_count.restype = i64
        L.hesp_topk_workspace_bytes.argtypes = [i64]
        L.hesp_topk_workspace_bytes.restype = i64
        _lib = L
    return _lib


def _check(fn: str, rc: int):
    if rc != HESP_OK:
        raise HespError(fn, rc, lib().hesp_last_error().decode())


def _np(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(P)


def _dev(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def version() -> str:
    return lib().hesp_version().decode()


# ----------------------------------------------------------------- cost model

def cost_tables(rmax_mflops: np.ndarray, h: np.ndarray, b: int, max_level: int, latency_ns: int = 10_000,
                bw_bytes_per_ns: int = 12, elem_bytes: int = 8, shared_memory: bool = False):
    """int64 cost_ns[n_ptypes][4][max_level+1] and xfer_ns[4^max_level + 1]."""
    rmax = np.ascontiguousarray(rmax_mflops, dtype=np.int64).reshape(-1, 4)
    hh = np.ascontiguousarray(h, dtype=np.int64).reshape(-1)
    n_pt = rmax.shape[0]
    cost = np.zeros((n_pt, 4, max_level + 1), np.int64)
    xfer = np.zeros(4 ** max_level + 1, np.int64)
    cm = CostModel(n_pt, _np(rmax), _np(hh), b, max_level, latency_ns, bw_bytes_per_ns, elem_bytes,
                   int(bool(shared_memory)))
    _check("hesp_cost_tables", lib().hesp_cost_tables(ctypes.byref(cm), _np(cost), _np(xfer)))
    return cost, xfer


class Platform:
    """A platform with its cost tables (host arrays kept alive for the C structs)."""

    def __init__(self, proc_type, proc_mem, n_mem: int, cost: np.ndarray, xfer: np.ndarray, capacity=None,
                 link=None):
        """capacity: None or [n_mem] blocks of side b / 2^max_level each space
        holds (<= 0 and the host's entry: unbounded).  link: None (one
        interconnect) or [n_mem] link ids 0..n_mem-1 of the transfers into each
        space, used when the policy's bus flag is set."""
        self.proc_type = np.ascontiguousarray(proc_type, dtype=np.int32)
        self.proc_mem = np.ascontiguousarray(proc_mem, dtype=np.int32)
        self.n_mem = int(n_mem)
        self.cost = np.ascontiguousarray(cost, dtype=np.int64)
        self.xfer = np.ascontiguousarray(xfer, dtype=np.int64)
        self.max_level = self.cost.shape[2] - 1
        self.capacity = None if capacity is None else np.ascontiguousarray(capacity, dtype=np.int64)
        self.link = None if link is None else np.ascontiguousarray(link, dtype=np.int32)
        if self.link is not None and self.link.shape != (self.n_mem,):
            raise HespError("Platform", HESP_EINVAL, f"link needs {self.n_mem} entries")
        if self.capacity is not None and self.capacity.shape != (self.n_mem,):
            raise HespError("Platform", HESP_EINVAL, f"capacity needs {self.n_mem} entries")
        self.c = PlatformC(len(self.proc_type), self.cost.shape[0], self.n_mem, self.max_level,
                           _np(self.proc_type), _np(self.proc_mem), _np(self.cost), _np(self.xfer),
                           _np(self.capacity), _np(self.link))

    @classmethod
    def from_inputs(cls, pf, b: int, max_level: int, capacity_bytes=None, link=None) -> "Platform":
        """From a drawn platform of ``inputs.make_platform``; capacity_bytes
        ([n_mem] or None) becomes whole blocks of side b / 2^max_level; link as
        in the constructor."""
        cost, xfer = cost_tables(pf.rmax, pf.h, b, max_level, pf.latency_ns, pf.bw_bytes_per_ns,
                                 pf.elem_bytes, pf.shared_memory)
        cap = None
        if capacity_bytes is not None:
            blk = pf.elem_bytes * (b >> max_level) ** 2
            cap = np.array([c // blk if c > 0 else 0 for c in capacity_bytes], np.int64)
        return cls(pf.proc_type, pf.proc_mem, pf.n_mem, cost, xfer, cap, link)


# ----------------------------------------------------------------- expansion

def expand(nt: int, dmax: int, depth: np.ndarray):
    """Fine tasks (int32 [n][5]: kind, level, K, I, J) and successor CSR of one candidate."""
    dep = np.ascontiguousarray(depth, dtype=np.uint8)
    n_tasks = np.zeros(1, np.int32)
    n_edges = np.zeros(1, np.int64)
    L = lib()
    _check("hesp_expand", L.hesp_expand(nt, dmax, _np(dep), _np(n_tasks), _np(n_edges), None, None, None))
    n, m = int(n_tasks[0]), int(n_edges[0])
    tasks = np.zeros((n, 5), np.int32)
    ptr = np.zeros(n + 1, np.int64)
    idx = np.zeros(max(m, 1), np.int32)
    _check("hesp_expand", L.hesp_expand(nt, dmax, _np(dep), _np(n_tasks), _np(n_edges), _np(tasks), _np(ptr),
                                        _np(idx)))
    return tasks, ptr, idx[:m]


# ----------------------------------------------------------------- device batches

class DeviceBatch:
    """A batch of candidates in device memory (torch tensors) and its C view."""

    def __init__(self, n_cand: int, nt: int, dmax: int, depth, nt_arr=None, dmax_arr=None, mask_off=None):
        self.n_cand, self.nt, self.dmax = int(n_cand), int(nt), int(dmax)
        self.depth, self.nt_arr, self.dmax_arr, self.mask_off = depth, nt_arr, dmax_arr, mask_off
        self.c = BatchC(self.n_cand, self.nt, self.dmax, _dev(nt_arr), _dev(dmax_arr), _dev(mask_off),
                        _dev(depth))

    @classmethod
    def from_host(cls, batch, device="cuda") -> "DeviceBatch":
        import torch
        dep = torch.from_numpy(np.ascontiguousarray(batch.depth)).to(device)
        if batch.uniform:
            return cls(batch.n, int(batch.nt[0]), int(batch.dmax[0]), dep)
        return cls(batch.n, int(batch.nt.max()), int(batch.dmax.max()), dep,
                   torch.from_numpy(batch.nt.astype(np.int32)).to(device),
                   torch.from_numpy(batch.dmax.astype(np.int32)).to(device),
                   torch.from_numpy(batch.mask_off.astype(np.int64)).to(device))


def generate_uniform(seed: int, first: int, n_cand: int, nt: int, dmax: int, split_thr: int, stream=None,
                     device="cuda") -> DeviceBatch:
    import torch
    n_top = nt * (nt + 1) * (nt + 2) // 6
    dep = torch.empty(n_cand * n_top, dtype=torch.uint8, device=device)
    _check("hesp_generate_uniform", lib().hesp_generate_uniform(seed, first, n_cand, nt, dmax, split_thr,
                                                                _dev(dep), _stream(stream)))
    return DeviceBatch(n_cand, nt, dmax, dep)


def generate_ragged(seed: int, first: int, n_cand: int, nt_lo: int, nt_hi: int, dmax_hi: int, split_thr: int,
                    stream=None, device="cuda") -> DeviceBatch:
    """Ragged batch: shapes, then depths, both drawn on the GPU (one device-to-host read of the size)."""
    import torch
    nt = torch.empty(n_cand, dtype=torch.int32, device=device)
    dm = torch.empty(n_cand, dtype=torch.int32, device=device)
    off = torch.empty(n_cand + 1, dtype=torch.int64, device=device)
    st = _stream(stream)
    _check("hesp_generate_ragged_shape", lib().hesp_generate_ragged_shape(seed, first, n_cand, nt_lo, nt_hi,
                                                                          dmax_hi, _dev(nt), _dev(dm), _dev(off),
                                                                          st))
    total = int(off[-1].item())
    dep = torch.empty(max(total, 1), dtype=torch.uint8, device=device)
    b = DeviceBatch(n_cand, nt_hi, dmax_hi, dep, nt, dm, off)
    _check("hesp_generate_ragged_depth", lib().hesp_generate_ragged_depth(seed, first, ctypes.byref(b.c),
                                                                          split_thr, _dev(dep), st))
    return b


def count_batch(batch: DeviceBatch, stream=None):
    import torch
    nt = torch.empty(batch.n_cand, dtype=torch.int32, device=batch.depth.device)
    ne = torch.empty(batch.n_cand, dtype=torch.int64, device=batch.depth.device)
    _check("hesp_count_batch", lib().hesp_count_batch(ctypes.byref(batch.c), _dev(nt), _dev(ne), _stream(stream)))
    return nt, ne


class Plan:
    def __init__(self, slots: int = 0, max_tasks: int = 0, max_edges: int = 0, chunks: int = 0, group: int = 0,
                 prep_edges: int = 0, fuse: int = 0):
        """fuse: 0 separate preparation launches, 1 fused pipeline (workspace
        slots in device memory), 2 fused pipeline with each slot in LDS."""
        self.h = P()
        self.opts = PlanOpts(slots, max_tasks, max_edges, chunks, group, prep_edges, int(fuse))
        _check("hesp_plan_create", lib().hesp_plan_create(ctypes.byref(self.h), ctypes.byref(self.opts)))

    def bytes(self) -> int:
        v = i64(0)
        _check("hesp_plan_bytes", lib().hesp_plan_bytes(self.h, ctypes.byref(v)))
        return int(v.value)

    def timing(self, enable: bool = True):
        _check("hesp_plan_timing", lib().hesp_plan_timing(self.h, int(enable)))

    def last_ms(self):
        """(prepare ms, simulate ms, simulate launches) of the last simulate_batch call."""
        out = np.zeros(3, np.float64)
        _check("hesp_plan_last_ms", lib().hesp_plan_last_ms(self.h, _np(out)))
        return float(out[0]), float(out[1]), int(out[2])

    def close(self):
        if self.h:
            lib().hesp_plan_destroy(self.h)
            self.h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate_batch(plan: Plan, pf: Platform, batch: DeviceBatch, makespan, status, sched_off=None, proc=None,
                   start=None, finish=None, stream=None, policy=(0, 0, 0), n_tasks=None):
    out = OutputsC(_dev(makespan), _dev(status), _dev(n_tasks), _dev(sched_off), _dev(proc), _dev(start),
                   _dev(finish))
    _check("hesp_simulate_batch", lib().hesp_simulate_batch(plan.h, ctypes.byref(pf.c), Policy(*policy),
                                                            ctypes.byref(batch.c), ctypes.byref(out),
                                                            _stream(stream)))


NOALLOC_BYTES, NOALLOC_MAX_CAND, NOALLOC_REGION = 64 << 20, 16384, 66189824


def simulate_batch_noalloc(pf: Platform, batch: DeviceBatch, makespan, status, group: int = 0, sched_off=None,
                           proc=None, start=None, finish=None, stream=None, policy=(0, 0, 0), n_tasks=None):
    """simulate_batch without a plan: the library's fixed device array is the only workspace."""
    out = OutputsC(_dev(makespan), _dev(status), _dev(n_tasks), _dev(sched_off), _dev(proc), _dev(start),
                   _dev(finish))
    _check("hesp_simulate_batch_noalloc", lib().hesp_simulate_batch_noalloc(ctypes.byref(pf.c), Policy(*policy),
                                                                            ctypes.byref(batch.c),
                                                                            ctypes.byref(out), int(group),
                                                                            _stream(stream)))


# ----------------------------------------------------------------- grain batches

def grain_cost_tables(rmax_mflops: np.ndarray, h: np.ndarray, b: int, fac, latency_ns: int = 10_000,
                      bw_bytes_per_ns: int = 12, elem_bytes: int = 8, shared_memory: bool = False):
    """int64 cost_ns[n_ptypes][4][n_fac] (sides b / fac[g]) and xfer_ns[L*L + 1]
    (atoms of side b / L, L = lcm(fac))."""
    rmax = np.ascontiguousarray(rmax_mflops, dtype=np.int64).reshape(-1, 4)
    hh = np.ascontiguousarray(h, dtype=np.int64).reshape(-1)
    fa = np.ascontiguousarray(fac, dtype=np.int32)
    L = int(np.lcm.reduce(fa.astype(np.int64))) if len(fa) else 0
    cost = np.zeros((rmax.shape[0], 4, max(len(fa), 1)), np.int64)
    xfer = np.zeros(L * L + 1 if 0 < L <= 64 else 1, np.int64)
    cm = CostModel(rmax.shape[0], _np(rmax), _np(hh), b, 0, latency_ns, bw_bytes_per_ns, elem_bytes,
                   int(bool(shared_memory)))
    _check("hesp_grain_cost_tables", lib().hesp_grain_cost_tables(ctypes.byref(cm), len(fa), _np(fa), _np(cost),
                                                                  _np(xfer)))
    return cost, xfer


def grain_platform(pf, b: int, fac) -> Platform:
    """A Platform whose tables describe the grains of ``fac`` (from a drawn
    platform of ``inputs.make_platform``)."""
    cost, xfer = grain_cost_tables(pf.rmax, pf.h, b, fac, pf.latency_ns, pf.bw_bytes_per_ns, pf.elem_bytes,
                                   pf.shared_memory)
    return Platform(pf.proc_type, pf.proc_mem, pf.n_mem, cost, xfer)


def _grain_c(nt: int, fac: np.ndarray, grain, n_cand: int):
    return GrainBatchC(int(n_cand), int(nt), len(fac), _np(fac), _dev(grain))


def grain_workspace_bytes(nt: int, fac, n_mem: int, slots: int) -> int:
    fa = np.ascontiguousarray(fac, dtype=np.int32)
    out = i64(0)
    c = _grain_c(nt, fa, None, 0)
    _check("hesp_grain_workspace", lib().hesp_grain_workspace(ctypes.byref(c), int(n_mem), int(slots),
                                                              ctypes.byref(out)))
    return int(out.value)


def simulate_grain_batch(pf: Platform, nt: int, fac, grain, makespan, n_tasks=None, n_edges=None, status=None,
                         ws=None, slots: int = 2048, policy=(0, 0, 0), stream=None):
    """Simulate a grain batch: grain is a device uint8 tensor [n_cand][tet(nt)]
    of indices into fac; ws a device uint8 tensor of at least
    grain_workspace_bytes(nt, fac, pf.n_mem, slots) bytes (allocated here when
    None).  Returns the workspace."""
    import torch
    fa = np.ascontiguousarray(fac, dtype=np.int32)
    n_top = nt * (nt + 1) * (nt + 2) // 6
    if grain.dtype != torch.uint8 or grain.dim() != 2 or grain.shape[1] != n_top or not grain.is_contiguous():
        raise HespError("hesp_simulate_grain_batch", HESP_EINVAL, f"grain must be contiguous uint8 [n][{n_top}]")
    n_cand = int(grain.shape[0])
    for name, t, dt in (("makespan", makespan, torch.int64), ("n_tasks", n_tasks, torch.int32),
                        ("n_edges", n_edges, torch.int64), ("status", status, torch.int32)):
        if t is not None and (t.dtype != dt or not t.is_contiguous() or t.numel() < n_cand):
            raise HespError("hesp_simulate_grain_batch", HESP_EINVAL, f"{name} must be contiguous {dt} of >= {n_cand}")
    if makespan is None and n_cand:
        raise HespError("hesp_simulate_grain_batch", HESP_EINVAL, "makespan is required")
    need = grain_workspace_bytes(nt, fa, pf.n_mem, slots)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=grain.device)
    if ws.dtype != torch.uint8 or not ws.is_contiguous() or ws.numel() < need:
        raise HespError("hesp_simulate_grain_batch", HESP_EINVAL, f"ws must be contiguous uint8 of >= {need} bytes")
    c = _grain_c(nt, fa, grain, n_cand)
    _check("hesp_simulate_grain_batch",
           lib().hesp_simulate_grain_batch(ctypes.byref(pf.c), Policy(*policy), ctypes.byref(c), _dev(makespan),
                                           _dev(n_tasks), _dev(n_edges), _dev(status), _dev(ws),
                                           int(ws.numel()), int(slots), _stream(stream)))
    return ws


class TreeBatch:
    """Split-tree candidates of one shape in device memory: flags [n_cand, flag_count]."""

    def __init__(self, n_cand: int, nt: int, dmax: int, flags):
        self.n_cand, self.nt, self.dmax, self.flags = int(n_cand), int(nt), int(dmax), flags
        self.c = TreeBatchC(self.n_cand, self.nt, self.dmax, _dev(flags))

    @classmethod
    def from_host(cls, batch, device="cuda") -> "TreeBatch":
        import torch
        fl = torch.from_numpy(np.ascontiguousarray(batch.depth)).to(device)
        return cls(batch.n, int(batch.nt[0]), int(batch.dmax[0]), fl)


def tree_flag_count(nt: int, dmax: int) -> int:
    return int(lib().hesp_tree_flag_count(nt, dmax))


def generate_tree_uniform(seed: int, first: int, n_cand: int, nt: int, dmax: int, split_thr: int, stream=None,
                          device="cuda") -> TreeBatch:
    import torch
    fl = torch.empty(max(1, n_cand * tree_flag_count(nt, dmax)), dtype=torch.uint8, device=device)
    _check("hesp_generate_tree_uniform", lib().hesp_generate_tree_uniform(seed, first, n_cand, nt, dmax, split_thr,
                                                                          _dev(fl), _stream(stream)))
    return TreeBatch(n_cand, nt, dmax, fl)


def count_tree_batch(batch: TreeBatch, stream=None):
    import torch
    nt = torch.empty(max(1, batch.n_cand), dtype=torch.int32, device="cuda")
    ne = torch.empty(max(1, batch.n_cand), dtype=torch.int64, device="cuda")
    _check("hesp_count_tree_batch", lib().hesp_count_tree_batch(ctypes.byref(batch.c), _dev(nt), _dev(ne),
                                                                _stream(stream)))
    return nt[:batch.n_cand], ne[:batch.n_cand]


def simulate_tree_batch(plan: Plan, pf: Platform, batch: TreeBatch, makespan, status, sched_off=None, proc=None,
                        start=None, finish=None, stream=None, policy=(0, 0, 0), n_tasks=None):
    out = OutputsC(_dev(makespan), _dev(status), _dev(n_tasks), _dev(sched_off), _dev(proc), _dev(start),
                   _dev(finish))
    _check("hesp_simulate_tree_batch", lib().hesp_simulate_tree_batch(plan.h, ctypes.byref(pf.c), Policy(*policy),
                                                                      ctypes.byref(batch.c), ctypes.byref(out),
                                                                      _stream(stream)))


def argmin(makespan, best, stream=None):
    _check("hesp_argmin", lib().hesp_argmin(_dev(makespan), int(makespan.numel()), _dev(best), _stream(stream)))


# ----------------------------------------------------------------- learned surrogate

MLP_IN, MLP_HIDDEN = 32, 256


class MLP:
    """The surrogate network (device parameters, gradients and Adam state)."""

    def __init__(self, seed: int = 0):
        self.h = P()
        _check("hesp_mlp_create", lib().hesp_mlp_create(ctypes.byref(self.h), seed))

    @staticmethod
    def param_count() -> int:
        return int(lib().hesp_mlp_param_count())

    def set_params(self, flat: np.ndarray):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check("hesp_mlp_set_params", lib().hesp_mlp_set_params(self.h, _np(a), a.size))

    def get_params(self) -> np.ndarray:
        a = np.zeros(self.param_count(), np.float32)
        _check("hesp_mlp_get_params", lib().hesp_mlp_get_params(self.h, _np(a), a.size))
        return a

    def get_grads(self) -> np.ndarray:
        a = np.zeros(self.param_count(), np.float32)
        _check("hesp_mlp_get_grads", lib().hesp_mlp_get_grads(self.h, _np(a), a.size))
        return a

    @staticmethod
    def _need(fn: str, what: str, t, itemsize: int, is_float: bool, numel: int):
        """Raise before any launch unless tensor t is contiguous, has elements of
        the stated kind and holds at least numel of them."""
        if t is None:
            raise HespError(fn, HESP_EINVAL, f"{what} is missing")
        if not t.is_contiguous() or t.element_size() != itemsize or t.is_floating_point() != is_float:
            raise HespError(fn, HESP_EINVAL, f"{what} must be a contiguous {'float' if is_float else 'integer'} "
                                             f"tensor of {itemsize}-byte elements")
        if int(t.numel()) < numel:
            raise HespError(fn, HESP_EINVAL, f"{what} holds {int(t.numel())} elements, {numel} needed")

    def forward(self, x, y, stream=None):
        """x: uint16/int16 [n][32] bf16 bit patterns (device); y: float32 [n] (device)."""
        n = int(y.numel())
        self._need("hesp_mlp_forward", "y", y, 4, True, n)
        self._need("hesp_mlp_forward", "x", x, 2, False, n * 32)
        _check("hesp_mlp_forward", lib().hesp_mlp_forward(self.h, _dev(x), n, _dev(y), _stream(stream)))

    def grad(self, x, t, batch: int, loss=None, stream=None):
        self._need("hesp_mlp_grad", "x", x, 2, False, batch * 32)
        self._need("hesp_mlp_grad", "t", t, 4, True, batch)
        if loss is not None:
            self._need("hesp_mlp_grad", "loss", loss, 4, True, 1)
        _check("hesp_mlp_grad", lib().hesp_mlp_grad(self.h, _dev(x), _dev(t), batch, _dev(loss), _stream(stream)))

    def adam(self, lr: float, stream=None):
        _check("hesp_mlp_adam", lib().hesp_mlp_adam(self.h, lr, _stream(stream)))

    def train(self, x, t, batch: int, steps: int, lr: float, seed: int = 0, loss=None, stream=None):
        """steps Adam steps on batches drawn with replacement from the rows of (x, t)."""
        rows = int(t.numel())
        self._need("hesp_mlp_train", "t", t, 4, True, rows)
        self._need("hesp_mlp_train", "x", x, 2, False, rows * 32)
        if loss is not None:
            self._need("hesp_mlp_train", "loss", loss, 4, True, steps)
        _check("hesp_mlp_train", lib().hesp_mlp_train(self.h, _dev(x), _dev(t), int(t.numel()), batch, steps, lr,
                                                      seed, _dev(loss), _stream(stream)))

    def close(self):
        if self.h:
            lib().hesp_mlp_destroy(self.h)
            self.h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_features(depth, n: int, n_top: int, rate, x, stream=None):
    """x[n][32] (bf16 bits) from depth (uint8 [n][n_top]) and rate (float32 [n_rate]), device tensors."""
    n_rate = 0 if rate is None else int(rate.numel())
    _check("hesp_mlp_features", lib().hesp_mlp_features(_dev(depth), n, n_top, _dev(rate), n_rate, _dev(x),
                                                        _stream(stream)))


def mlp_targets(makespan, mu: float, sigma: float, t, stream=None):
    _check("hesp_mlp_targets", lib().hesp_mlp_targets(_dev(makespan), int(makespan.numel()), mu, sigma, _dev(t),
                                                      _stream(stream)))


def mlp_rate_features(rmax_mflops: np.ndarray) -> np.ndarray:
    """float32 [n_ptypes * 4] rate features of a platform's R_max table (host)."""
    rmax = np.ascontiguousarray(rmax_mflops, dtype=np.int64).reshape(-1, 4)
    h = np.zeros(rmax.shape[0], np.int64)
    cm = CostModel(rmax.shape[0], _np(rmax), _np(h), 0, 0, 0, 0, 0, 0)
    out = np.zeros(rmax.size, np.float32)
    _check("hesp_mlp_rate_features", lib().hesp_mlp_rate_features(ctypes.byref(cm), _np(out), out.size))
    return out


def mlp_features_agg(depth, n: int, nt: int, rate, x, stream=None):
    n_rate = 0 if rate is None else int(rate.numel())
    _check("hesp_mlp_features_agg", lib().hesp_mlp_features_agg(_dev(depth), n, nt, _dev(rate), n_rate, _dev(x),
                                                                _stream(stream)))


# ----------------------------------------------------------------- enumeration, top-k, search

def generate_enumerate(first: int, n_cand: int, nt: int, dmax: int, stream=None, device="cuda") -> DeviceBatch:
    import torch
    n_top = nt * (nt + 1) * (nt + 2) // 6
    dep = torch.empty(max(n_cand * n_top, 1), dtype=torch.uint8, device=device)
    _check("hesp_generate_enumerate", lib().hesp_generate_enumerate(first, n_cand, nt, dmax, _dev(dep),
                                                                    _stream(stream)))
    return DeviceBatch(n_cand, nt, dmax, dep)


def topk_workspace(n: int, device="cuda"):
    import torch
    return torch.empty(int(lib().hesp_topk_workspace_bytes(n)), dtype=torch.uint8, device=device)


def topk(values, k: int, ws=None, stream=None):
    """Indices (int32 device tensor) of the k smallest values (int64 makespans or float32 scores)."""
    import torch
    n = int(values.numel())
    if ws is None:
        ws = topk_workspace(n, values.device)
    idx = torch.empty(max(k, 1), dtype=torch.int32, device=values.device)
    fn = "hesp_topk_makespan" if values.dtype == torch.int64 else "hesp_topk_score"
    if values.dtype not in (torch.int64, torch.float32):
        raise TypeError("topk takes int64 makespans or float32 scores")
    _check(fn, getattr(lib(), fn)(_dev(values), n, k, _dev(idx), _dev(ws), int(ws.numel()), _stream(stream)))
    return idx[:k]


def search(plan: Plan, pf: Platform, nt: int, dmax: int, mode: int, rounds: int, batch: int, seed: int,
           warm_rounds: int = 1, warm_batch: int = 0, proposals: int = 0, pool: int = 64, split_thr: int = 0,
           mutate_thr: int = 0, mlp: "MLP" = None, rate=None, train_steps: int = 0, train_batch: int = 512,
           lr: float = 1e-3, replay: int = 0, stream=None, policy=(0, 0, 0)):
    """Runs hesp_search; returns (best depth (uint8 numpy), best makespan, trace as a list of dicts)."""
    sp = SearchParams(mode, nt, dmax, rounds, batch, warm_rounds, warm_batch or batch, proposals or batch, pool,
                      split_thr, mutate_thr, seed, mlp.h if mlp is not None else None, _dev(rate),
                      0 if rate is None else int(rate.numel()), train_steps, train_batch, lr, replay)
    n_top = nt * (nt + 1) * (nt + 2) // 6
    best = np.zeros(n_top, np.uint8)
    best_ms = i64(0)
    trace = (TracePoint * rounds)()
    _check("hesp_search", lib().hesp_search(plan.h, ctypes.byref(pf.c), Policy(*policy), ctypes.byref(sp), _np(best),
                                            ctypes.byref(best_ms), trace, _stream(stream)))
    tr = [{"wall_ms": t.wall_ms, "best_makespan": t.best_makespan, "simulated": t.simulated,
           "proposed": t.proposed} for t in trace]
    return best, int(best_ms.value), tr


def solve(plan: Plan, pf: Platform, nt: int, dmax: int, depth, iters: int, lst: int = LIST_ALL,
          sampling: int = SAMPLE_HARD, seed: int = 0, policy=(0, 0, 0), stream=None):
    """Runs hesp_solve on the chains whose initial partitions are the rows of
    `depth` (uint8 device tensor [n_chains, tet(nt)], updated in place to the last
    partitions); returns (best depths, best makespans, makespan per iteration,
    steps [n_chains, iters, 3] = (cluster, new depth, score))."""
    import torch
    n_top = nt * (nt + 1) * (nt + 2) // 6
    if depth.dtype != torch.uint8 or depth.dim() != 2 or depth.shape[1] != n_top or not depth.is_contiguous():
        raise ValueError("depth must be a contiguous uint8 tensor [n_chains, tet(nt)]")
    B = int(depth.shape[0])
    best = torch.empty_like(depth)
    best_ms = torch.empty(B, dtype=torch.int64, device=depth.device)
    trace = torch.empty((B, iters), dtype=torch.int64, device=depth.device)
    steps = torch.empty((B, iters, 3), dtype=torch.int64, device=depth.device)
    sp = SolveParams(B, nt, dmax, iters, lst, sampling, seed)
    _check("hesp_solve", lib().hesp_solve(plan.h, ctypes.byref(pf.c), Policy(*policy), ctypes.byref(sp), _dev(depth),
                                          _dev(best), _dev(best_ms), _dev(trace), _dev(steps), _stream(stream)))
    return best, best_ms, trace, steps


def solve_tree(plan: Plan, pf: Platform, nt: int, dmax: int, flags, iters: int, lst: int = LIST_ALL,
               sampling: int = SAMPLE_HARD, seed: int = 0, policy=(0, 0, 0), stream=None):
    """Runs hesp_solve_tree on the chains whose initial split-tree partitions are
    the rows of `flags` (uint8 device tensor [n_chains, tree_flag_count], updated in
    place); returns (best flags, best makespans, makespan per iteration, steps
    [n_chains, iters, 3] = (node, 1 split / 0 merge, score))."""
    import torch
    nf = tree_flag_count(nt, dmax)
    if flags.dtype != torch.uint8 or flags.dim() != 2 or flags.shape[1] != nf or not flags.is_contiguous():
        raise ValueError("flags must be a contiguous uint8 tensor [n_chains, tree_flag_count(nt, dmax)]")
    B = int(flags.shape[0])
    best = torch.empty_like(flags)
    best_ms = torch.empty(B, dtype=torch.int64, device=flags.device)
    trace = torch.empty((B, iters), dtype=torch.int64, device=flags.device)
    steps = torch.empty((B, iters, 3), dtype=torch.int64, device=flags.device)
    sp = SolveParams(B, nt, dmax, iters, lst, sampling, seed)
    _check("hesp_solve_tree", lib().hesp_solve_tree(plan.h, ctypes.byref(pf.c), Policy(*policy), ctypes.byref(sp),
                                                    _dev(flags), _dev(best), _dev(best_ms), _dev(trace), _dev(steps),
                                                    _stream(stream)))
    return best, best_ms, trace, steps
