"""ctypes loader for the plain-C oracle (``hesp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hesp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the same source built for the host it runs on (-march=native): the CPU baseline
# compiles it on the measuring machine itself, so it never travels between hosts
LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build (clang, so that it shares one
# sanitizer runtime with the host code of the sanitized libhesp build); loaded
# instead of LIB when HESP_SANITIZE=1 (tests/sanitized_cpu_suite.py)
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
CLANG = "/opt/rocm/llvm/bin/clang"

_libs = {}


def build(force: bool = True, native: bool = False, extra_flags=(), sanitize: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2; -march=native for the baseline
    build), or with clang and the address and undefined-behaviour sanitizers."""
    out = LIB_SAN if sanitize else (LIB_NATIVE if native else LIB)
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        flags = ["-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra"]
        if sanitize:
            cmd = [CLANG, *flags, *SAN_FLAGS]
        else:
            cmd = ["gcc", "-O2", *flags] + (["-march=native"] if native else [])
        subprocess.check_call([*cmd, *extra_flags, "-o", tmp, SRC])
        os.replace(tmp, out)
    return out


def sanitized() -> bool:
    return os.environ.get("HESP_SANITIZE") == "1"


def lib(native: bool = False):
    key = "san" if sanitized() else bool(native)
    if key not in _libs:
        path = LIB_SAN if sanitized() else (LIB_NATIVE if native else LIB)
        if not os.path.exists(path):
            build(native=native, sanitize=sanitized())
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.oracle_simulate.argtypes = [i32, i32, P, i32, P, P, i32, i32, P, P, i64, i64, i64, i64, i32,
                                      P, P, P, i32, P, P, P, P, P, i64, P, i32, i32, ctypes.c_uint64, i32, i32, i32, P, P]
        L.oracle_simulate.restype = i32
        L.oracle_simulate_batch.argtypes = [i32, P, P, P, P, i32, P, P, i32, i32, P, P, i64, i64, i64,
                                            i64, i32, i32, P, P, P, i32, i32, ctypes.c_uint64, i32, i32, i32, P, P]
        L.oracle_simulate_batch.restype = i32
        L.oracle_simulate_grain.argtypes = [i32, i32, P, P, i32, P, P, i32, i32, P, P, i64, i64, i64, i64, i32,
                                            P, P, P, i32, P, P, P, P, P, i64, P, i32, i32, ctypes.c_uint64, i32,
                                            i32, P]
        L.oracle_simulate_grain.restype = i32
        L.oracle_simulate_grain_batch.argtypes = [i32, i32, i32, P, P, i32, P, P, i32, i32, P, P, i64, i64,
                                                  i64, i64, i32, i32, P, P, P, i32, i32, ctypes.c_uint64, i32,
                                                  i32, P]
        L.oracle_simulate_grain_batch.restype = i32
        L.oracle_task_time.argtypes = [i32, i64, i64, i64, P]
        L.oracle_task_time.restype = i32
        L.oracle_transfer_time.argtypes = [i64, i64, i64, i64, i64, i32, P]
        L.oracle_transfer_time.restype = i32
        _libs[key] = L
    return _libs[key]


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def task_time(ttype: int, bl: int, rmax: int, h: int) -> int:
    out = np.zeros(1, np.int64)
    rc = lib().oracle_task_time(ttype, bl, rmax, h, _p(out))
    if rc:
        raise ValueError(f"oracle_task_time rc={rc}")
    return int(out[0])


def transfer_time(n_atoms: int, atom_side: int, pf) -> int:
    out = np.zeros(1, np.int64)
    rc = lib().oracle_transfer_time(n_atoms, atom_side, pf.elem_bytes, pf.latency_ns,
                                    pf.bw_bytes_per_ns, int(pf.shared_memory), _p(out))
    if rc:
        raise ValueError(f"oracle_transfer_time rc={rc}")
    return int(out[0])


class Schedule:
    """Oracle result for one candidate, tasks in the oracle's program order."""

    def __init__(self, makespan, tasks, proc, start, finish, rank, edges):
        self.makespan = makespan
        self.tasks = tasks      # int32 [n][5]: type, level, K, I, J
        self.proc = proc
        self.start = start
        self.finish = finish
        self.rank = rank
        self.edges = edges      # int32 [m][2]

    @property
    def n_tasks(self) -> int:
        return int(self.tasks.shape[0])


def simulate(pf, nt: int, dmax: int, b: int, depth: np.ndarray, detail: bool = True, policy=(0, 0),
             tree: bool = False, capacity=None, link=None):
    """Simulate one candidate; returns a Schedule (detail) or the makespan.

    depth: split depth per top-level task, or with tree=True the split flags of
    every level l < dmax (one per task of the uniform level-l expansion, Fig. 1
    order, levels concatenated).

    policy = (order, select[, seed[, cache[, bus]]]): order 0 = Priority-List,
    1 = FCFS; select 0 = EFT-P, 1 = EIT-P, 2 = R-P, 3 = F-P (section 2.1, "Task
    and data scheduling heuristics"); seed feeds the R-P draws; cache 0 =
    write-back, 1 = write-through, 2 = write-around; bus 1 = transfers
    contend: one at a time on each link.

    link: None (one link shared by every transfer) or the link of each memory
    space ([n_mem], ids 0..n_mem-1): with bus 1 a transfer occupies the link of
    the space it goes into (copies sent to the host occupy the host's).

    capacity: None or bytes per memory space ([n_mem]; <= 0 and the host's
    entry mean unbounded): finite accelerator spaces with least-recently-used
    eviction (write-back, EFT-P, independent transfers only)."""
    order, select, seed, cache, bus = (tuple(policy) + (0, 0, 0))[:5]
    L = lib()
    cap = None if capacity is None else np.ascontiguousarray(capacity, dtype=np.int64)
    lk = None if link is None else np.ascontiguousarray(link, dtype=np.int32)
    depth = np.ascontiguousarray(depth, dtype=np.uint8)
    ptype = np.ascontiguousarray(pf.proc_type, dtype=np.int32)
    pmem = np.ascontiguousarray(pf.proc_mem, dtype=np.int32)
    rmax = np.ascontiguousarray(pf.rmax, dtype=np.int64)
    h = np.ascontiguousarray(pf.h, dtype=np.int64)
    ms = np.zeros(1, np.int64)
    nt_out = np.zeros(1, np.int32)
    ne_out = np.zeros(1, np.int64)
    args_pf = (pf.n_procs, _p(ptype), _p(pmem), pf.n_mem, pf.n_ptypes, _p(rmax), _p(h), b,
               pf.latency_ns, pf.bw_bytes_per_ns, pf.elem_bytes, int(pf.shared_memory))
    rc = L.oracle_simulate(nt, dmax, _p(depth), *args_pf, _p(ms), _p(nt_out), _p(ne_out),
                           0, None, None, None, None, None, 0, None, order, select, seed, cache, int(tree), bus,
                           _p(cap), _p(lk))
    if rc:
        raise ValueError(f"oracle_simulate rc={rc}")
    if not detail:
        return int(ms[0])
    n, m = int(nt_out[0]), int(ne_out[0])
    tasks = np.zeros((n, 5), np.int32)
    proc = np.zeros(n, np.int32)
    start = np.zeros(n, np.int64)
    finish = np.zeros(n, np.int64)
    rank = np.zeros(n, np.int64)
    edges = np.zeros((max(m, 1), 2), np.int32)
    rc = L.oracle_simulate(nt, dmax, _p(depth), *args_pf, _p(ms), _p(nt_out), _p(ne_out),
                           n, _p(tasks), _p(proc), _p(start), _p(finish), _p(rank), m, _p(edges), order, select,
                           seed, cache, int(tree), bus, _p(cap), _p(lk))
    if rc:
        raise ValueError(f"oracle_simulate rc={rc}")
    return Schedule(int(ms[0]), tasks, proc, start, finish, rank, edges[:m])


def simulate_batch(pf, batch, n_threads: int = 1, policy=(0, 0), tree: bool = False, native: bool = False,
                   capacity=None, statuses: bool = False, link=None):
    """Makespans (int64) and expanded task counts of a whole batch (policy,
    tree, capacity and link as in simulate; with tree=True batch.depth holds split
    flags and batch.mask_off their offsets; native selects the -march=native
    build).  statuses=True returns (makespans, counts, statuses) instead of
    raising on a candidate that fails (-4: no space can hold a task)."""
    order, select, seed, cache, bus = (tuple(policy) + (0, 0, 0))[:5]
    cap = None if capacity is None else np.ascontiguousarray(capacity, dtype=np.int64)
    lk = None if link is None else np.ascontiguousarray(link, dtype=np.int32)
    L = lib(native)
    n = batch.n
    ms = np.zeros(n, np.int64)
    ntk = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    nt = np.ascontiguousarray(batch.nt, dtype=np.int32)
    dm = np.ascontiguousarray(batch.dmax, dtype=np.int32)
    off = np.ascontiguousarray(batch.mask_off, dtype=np.int64)
    dep = np.ascontiguousarray(batch.depth, dtype=np.uint8)
    ptype = np.ascontiguousarray(pf.proc_type, dtype=np.int32)
    pmem = np.ascontiguousarray(pf.proc_mem, dtype=np.int32)
    rmax = np.ascontiguousarray(pf.rmax, dtype=np.int64)
    h = np.ascontiguousarray(pf.h, dtype=np.int64)
    rc = L.oracle_simulate_batch(n, _p(nt), _p(dm), _p(off), _p(dep), pf.n_procs, _p(ptype), _p(pmem),
                                 pf.n_mem, pf.n_ptypes, _p(rmax), _p(h), batch.b, pf.latency_ns,
                                 pf.bw_bytes_per_ns, pf.elem_bytes, int(pf.shared_memory), n_threads,
                                 _p(ms), _p(ntk), _p(st), order, select, seed, cache, int(tree), bus, _p(cap),
                                 _p(lk))
    if rc:
        raise ValueError(f"oracle_simulate_batch rc={rc}")
    if statuses:
        return ms, ntk, st
    if np.any(st != 0):
        bad = int(np.nonzero(st)[0][0])
        raise ValueError(f"oracle failed on candidate {bad} rc={int(st[bad])}")
    return ms, ntk


def _pf_args(pf, b):
    ptype = np.ascontiguousarray(pf.proc_type, dtype=np.int32)
    pmem = np.ascontiguousarray(pf.proc_mem, dtype=np.int32)
    rmax = np.ascontiguousarray(pf.rmax, dtype=np.int64)
    h = np.ascontiguousarray(pf.h, dtype=np.int64)
    keep = (ptype, pmem, rmax, h)
    return keep, (pf.n_procs, _p(ptype), _p(pmem), pf.n_mem, pf.n_ptypes, _p(rmax), _p(h), b,
                  pf.latency_ns, pf.bw_bytes_per_ns, pf.elem_bytes, int(pf.shared_memory))


def simulate_grain(pf, nt: int, fac, b: int, grain: np.ndarray, detail: bool = True, policy=(0, 0), link=None):
    """One candidate of a grain batch (section 2.1: partition parameter
    p = 1/fac[g]; Fig. 4: partially overlapping blocks): top-level task t is
    split on the fac[grain[t]] x fac[grain[t]] sub-tiling of its cell.  The task
    info's level column holds the grain index.  policy and link as in simulate;
    finite capacities are not defined for grain batches."""
    order, select, seed, cache, bus = (tuple(policy) + (0, 0, 0))[:5]
    L = lib()
    fa = np.ascontiguousarray(fac, dtype=np.int32)
    gr = np.ascontiguousarray(grain, dtype=np.uint8)
    lk = None if link is None else np.ascontiguousarray(link, dtype=np.int32)
    keep, args_pf = _pf_args(pf, b)
    ms = np.zeros(1, np.int64)
    nt_out = np.zeros(1, np.int32)
    ne_out = np.zeros(1, np.int64)
    rc = L.oracle_simulate_grain(nt, len(fa), _p(fa), _p(gr), *args_pf, _p(ms), _p(nt_out), _p(ne_out),
                                 0, None, None, None, None, None, 0, None, order, select, seed, cache, bus, _p(lk))
    if rc:
        raise ValueError(f"oracle_simulate_grain rc={rc}")
    if not detail:
        return int(ms[0])
    n, m = int(nt_out[0]), int(ne_out[0])
    tasks = np.zeros((n, 5), np.int32)
    proc = np.zeros(n, np.int32)
    start = np.zeros(n, np.int64)
    finish = np.zeros(n, np.int64)
    rank = np.zeros(n, np.int64)
    edges = np.zeros((max(m, 1), 2), np.int32)
    rc = L.oracle_simulate_grain(nt, len(fa), _p(fa), _p(gr), *args_pf, _p(ms), _p(nt_out), _p(ne_out),
                                 n, _p(tasks), _p(proc), _p(start), _p(finish), _p(rank), m, _p(edges),
                                 order, select, seed, cache, bus, _p(lk))
    if rc:
        raise ValueError(f"oracle_simulate_grain rc={rc}")
    return Schedule(int(ms[0]), tasks, proc, start, finish, rank, edges[:m])


def simulate_grain_batch(pf, nt: int, fac, b: int, grain: np.ndarray, n_threads: int = 1, policy=(0, 0),
                         link=None, native: bool = False):
    """Makespans and expanded task counts of n candidates, grain [n][tet(nt)]."""
    order, select, seed, cache, bus = (tuple(policy) + (0, 0, 0))[:5]
    L = lib(native)
    fa = np.ascontiguousarray(fac, dtype=np.int32)
    gr = np.ascontiguousarray(grain, dtype=np.uint8)
    n = int(gr.shape[0])
    lk = None if link is None else np.ascontiguousarray(link, dtype=np.int32)
    keep, args_pf = _pf_args(pf, b)
    ms = np.zeros(n, np.int64)
    ntk = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    rc = L.oracle_simulate_grain_batch(n, nt, len(fa), _p(fa), _p(gr), *args_pf, n_threads, _p(ms), _p(ntk),
                                       _p(st), order, select, seed, cache, bus, _p(lk))
    if rc or np.any(st != 0):
        raise ValueError(f"oracle_simulate_grain_batch rc={rc} status={st[st != 0][:4]}")
    return ms, ntk
