"""Seeded synthetic workloads for the batched scheduling-partitioning simulator.

This module only draws random inputs.  It holds none of the method's
arithmetic (no cost model, no expansion, no scheduling): both the HIP path and
the CPU oracle consume what it produces.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used as a counter-based
generator: the value for ``(seed, purpose, index)`` is output number
``index + 1`` of a SplitMix64 sequence whose state starts at
``mix(seed + GAMMA * (purpose + 1))``.  The device side implements the same
published generator independently to build candidates on the GPU.

Workload recipes (restating the platform and candidate descriptions of the
paper's problem statement, section 2, with synthetic rate models):

* a platform is a list of processor types; every type has a processor count,
  an integer peak-rate range in MFLOP/s, the half-performance size ``h`` and
  whether each of its processors owns a memory space (accelerators) or works
  in the host space 0 (CPU cores);
* one peak rate is drawn per (processor type, task type): 4 task types
  (chol, trsm, syrk, gemm);
* a candidate partitioning is one split depth per top-level task of the tiled
  Cholesky loop nest (Fig. 1 order); the depth is the number of consecutive
  successes of a Bernoulli(p) split draw, capped at the candidate's maximum;
* a split-tree candidate holds one split flag per task of every uniform level-l
  tiling (nt * 2^l tiles per dimension, Fig. 1 order, levels 0 .. dmax-1
  concatenated); flag x of candidate c is set when the leading 21 bits of the
  draw for index (c << 32 | x) fall below the split threshold.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB

# purposes of the counter streams
P_RMAX = 1
P_DEPTH = 2
P_SHAPE = 3
P_PLATFORM = 4
P_TREE = 5
P_DEPTH2 = 6      # chunks 3..5 of a depth draw (depths 4 and 5)
P_GRAIN = 7       # grain index per top-level task of a grain batch

CHUNK_BITS = 21  # one split draw uses 21 random bits; depth <= 3 uses 63 bits


def _mix_int(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def _mix_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(MIX1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(MIX2)
        z ^= z >> np.uint64(31)
    return z


def stream_state(seed: int, purpose: int) -> int:
    return _mix_int((seed + GAMMA * (purpose + 1)) & MASK64)


def draw(seed: int, purpose: int, index: int) -> int:
    """One 64-bit value of the counter-based SplitMix64 stream."""
    return _mix_int((stream_state(seed, purpose) + GAMMA * (index + 1)) & MASK64)


def draw_np(seed: int, purpose: int, index: np.ndarray) -> np.ndarray:
    s = np.uint64(stream_state(seed, purpose))
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = s + np.uint64(GAMMA) * (idx + np.uint64(1))
    return _mix_np(z)


def split_threshold(p_num: int, p_den: int) -> int:
    """Integer threshold t with P(chunk < t) = t / 2**21 ~= p_num / p_den."""
    return (p_num << CHUNK_BITS) // p_den


def depth_from_draw(u: np.ndarray, thr: int, dmax: np.ndarray, u2=None) -> np.ndarray:
    """Number of leading 21-bit chunks below ``thr``, capped at ``dmax``: the
    three chunks of ``u``, then (depths 4 and 5) the three of ``u2``."""
    u = np.asarray(u, dtype=np.uint64)
    dmax = np.broadcast_to(np.asarray(dmax, dtype=np.int64), u.shape)
    depth = np.zeros(u.shape, dtype=np.int64)
    alive = np.ones(u.shape, dtype=bool)
    for v in ([u] if u2 is None else [u, np.asarray(u2, dtype=np.uint64)]):
        for j in range(3):
            chunk = (v >> np.uint64(CHUNK_BITS * j)) & np.uint64((1 << CHUNK_BITS) - 1)
            ok = alive & (chunk < np.uint64(thr)) & (depth < dmax)
            depth += ok
            alive &= ok
    return depth.astype(np.uint8)


def tet(n: int) -> int:
    """Number of top-level tasks of the tiled Cholesky loop nest on n x n tiles."""
    return n * (n + 1) * (n + 2) // 6


# --------------------------------------------------------------------------
# platforms

@dataclasses.dataclass(frozen=True)
class ProcType:
    name: str
    count: int
    rmax_lo: int      # MFLOP/s, inclusive
    rmax_hi: int      # MFLOP/s, inclusive
    h: int            # half-performance block size
    own_space: bool   # True: each processor owns a memory space (accelerator)


@dataclasses.dataclass
class Platform:
    ptypes: List[ProcType]
    rmax: np.ndarray          # int64 [n_ptypes][4] MFLOP/s
    h: np.ndarray             # int64 [n_ptypes]
    proc_type: np.ndarray     # int32 [n_procs]
    proc_mem: np.ndarray      # int32 [n_procs]
    n_mem: int
    shared_memory: bool       # True: single memory space, no transfers
    latency_ns: int = 10_000  # per transfer
    bw_bytes_per_ns: int = 12 # 12 GB/s
    elem_bytes: int = 8

    @property
    def n_procs(self) -> int:
        return int(self.proc_type.shape[0])

    @property
    def n_ptypes(self) -> int:
        return len(self.ptypes)


def make_platform(ptypes: Sequence[ProcType], seed: int, platform_index: int = 0,
                  rmax: Optional[np.ndarray] = None) -> Platform:
    """Draw one peak rate per (processor type, task type) and lay out processors.

    Processors are numbered type by type in the listed order; a CPU-like type
    works in memory space 0, each processor of an accelerator-like type gets a
    space of its own (1, 2, ...).
    """
    ptypes = list(ptypes)
    n_pt = len(ptypes)
    if rmax is None:
        rmax = np.zeros((n_pt, 4), dtype=np.int64)
        for pt, t in enumerate(ptypes):
            for tt in range(4):
                u = draw(seed, P_RMAX, (platform_index << 8) | (pt << 2) | tt)
                rmax[pt, tt] = t.rmax_lo + u % (t.rmax_hi - t.rmax_lo + 1)
    rmax = np.asarray(rmax, dtype=np.int64).reshape(n_pt, 4)
    proc_type, proc_mem = [], []
    next_space = 1
    for pt, t in enumerate(ptypes):
        for _ in range(t.count):
            proc_type.append(pt)
            if t.own_space:
                proc_mem.append(next_space)
                next_space += 1
            else:
                proc_mem.append(0)
    shared = next_space == 1
    return Platform(ptypes=ptypes, rmax=rmax,
                    h=np.array([t.h for t in ptypes], dtype=np.int64),
                    proc_type=np.array(proc_type, dtype=np.int32),
                    proc_mem=np.array(proc_mem, dtype=np.int32),
                    n_mem=next_space, shared_memory=shared)


CPU_CORE = dict(rmax_lo=20_000, rmax_hi=40_000, h=64, own_space=False)
ACCEL = dict(rmax_lo=500_000, rmax_hi=2_000_000, h=512, own_space=True)
BIG = dict(rmax_lo=8_000, rmax_hi=16_000, h=48, own_space=False)
LITTLE = dict(rmax_lo=1_000, rmax_hi=3_000, h=32, own_space=False)


def cpu_accel_types(n_cpu: int, n_acc: int) -> List[ProcType]:
    return [ProcType("cpu", n_cpu, **CPU_CORE), ProcType("accel", n_acc, **ACCEL)]


def big_little_types(n_big: int, n_little: int) -> List[ProcType]:
    return [ProcType("big", n_big, **BIG), ProcType("little", n_little, **LITTLE)]


# --------------------------------------------------------------------------
# candidate batches

@dataclasses.dataclass
class Batch:
    """A batch of candidate partitionings, ragged in general.

    ``depth[mask_off[c]:mask_off[c+1]]`` holds candidate c's split depth per
    top-level task (Fig. 1 order); ``nt[c]`` is its tile count per dimension
    and ``dmax[c]`` its maximum split depth.
    """
    b: int
    nt: np.ndarray        # int32 [n]
    dmax: np.ndarray      # int32 [n]
    mask_off: np.ndarray  # int64 [n+1]
    depth: np.ndarray     # uint8 [mask_off[n]]

    @property
    def n(self) -> int:
        return int(self.nt.shape[0])

    @property
    def uniform(self) -> bool:
        return bool(np.all(self.nt == self.nt[0]) and np.all(self.dmax == self.dmax[0]))

    def candidate(self, c: int) -> np.ndarray:
        return self.depth[self.mask_off[c]:self.mask_off[c + 1]]

    def subset(self, idx: Sequence[int]) -> "Batch":
        idx = np.asarray(idx, dtype=np.int64)
        parts = [self.candidate(int(c)) for c in idx]
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(p) for p in parts])
        dep = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        return Batch(self.b, self.nt[idx].copy(), self.dmax[idx].copy(), off, dep.astype(np.uint8))


def concat_batches(batches: Sequence[Batch]) -> Batch:
    """One batch holding the candidates of every batch in turn (same block side)."""
    assert batches and all(bt.b == batches[0].b for bt in batches)
    sizes = [bt.mask_off[-1] for bt in batches]
    off = np.concatenate([[0]] + [bt.mask_off[1:] + base for bt, base in
                                  zip(batches, np.cumsum([0] + sizes[:-1]))]).astype(np.int64)
    return Batch(batches[0].b, np.concatenate([bt.nt for bt in batches]).astype(np.int32),
                 np.concatenate([bt.dmax for bt in batches]).astype(np.int32), off,
                 np.concatenate([bt.depth[:bt.mask_off[-1]] for bt in batches]).astype(np.uint8))


def uniform_batch(seed: int, n_cand: int, nt: int, b: int, dmax: int, p_num: int, p_den: int,
                  first: int = 0) -> Batch:
    """n_cand candidates of one shape; depth draws use counters (candidate, task)."""
    n_top = tet(nt)
    thr = split_threshold(p_num, p_den)
    c = np.arange(first, first + n_cand, dtype=np.uint64)[:, None]
    t = np.arange(n_top, dtype=np.uint64)[None, :]
    idx = (c << np.uint64(24)) | t
    u = draw_np(seed, P_DEPTH, idx)
    u2 = draw_np(seed, P_DEPTH2, idx) if dmax > 3 else None
    depth = depth_from_draw(u, thr, dmax, u2).reshape(-1)
    off = np.arange(n_cand + 1, dtype=np.int64) * n_top
    return Batch(b, np.full(n_cand, nt, np.int32), np.full(n_cand, dmax, np.int32), off, depth)


def grain_batch(seed: int, n_cand: int, nt: int, n_fac: int, first: int = 0) -> np.ndarray:
    """Grain indices (uint8 [n_cand][tet(nt)]) drawn uniformly from 0..n_fac-1,
    one counter-based draw per (candidate, top-level task)."""
    n_top = tet(nt)
    idx = (np.arange(n_cand, dtype=np.uint64)[:, None] + np.uint64(first)) * np.uint64(n_top) \
        + np.arange(n_top, dtype=np.uint64)[None, :]
    u = draw_np(seed, P_GRAIN, idx.reshape(-1))
    return (u % np.uint64(n_fac)).astype(np.uint8).reshape(n_cand, n_top)


def tree_flag_count(nt: int, dmax: int) -> int:
    """Split flags of one split-tree candidate: one per task of each uniform
    level-l tiling, l < dmax."""
    return sum(tet(nt << l) for l in range(dmax))


def fig1_cells(n: int):
    """Cells (k, i, j) of the tasks of the loop nest of Fig. 1 on n tiles, in its order."""
    out = []
    for k in range(n):
        out.append((k, k, k))
        out += [(k, k, j) for j in range(k + 1, n)]
        for i in range(k + 1, n):
            out += [(k, i, j) for j in range(i + 1, n)]
            out.append((k, i, i))
    return out


def tree_flags_from_depth(nt: int, dmax: int, depth: np.ndarray) -> np.ndarray:
    """The split-tree encoding of a depth-per-top-level-task candidate: a level-l
    cell is flagged when its top-level task's depth exceeds l."""
    top = {c: int(d) for c, d in zip(fig1_cells(nt), depth)}
    flags = []
    for l in range(dmax):
        flags += [1 if top[(k >> l, i >> l, j >> l)] > l else 0 for (k, i, j) in fig1_cells(nt << l)]
    return np.array(flags, np.uint8)


def tree_batch(seed: int, n_cand: int, nt: int, b: int, dmax: int, p_num: int, p_den: int,
               first: int = 0) -> Batch:
    """n_cand split-tree candidates: independent Bernoulli(p) flags drawn with
    counters (candidate, flag); depth holds the flags, mask_off their offsets."""
    nf = tree_flag_count(nt, dmax)
    thr = split_threshold(p_num, p_den)
    c = np.arange(first, first + n_cand, dtype=np.uint64)[:, None]
    x = np.arange(nf, dtype=np.uint64)[None, :]
    u = draw_np(seed, P_TREE, (c << np.uint64(32)) | x)
    flags = ((u >> np.uint64(64 - CHUNK_BITS)) < np.uint64(thr)).astype(np.uint8).reshape(-1)
    off = np.arange(n_cand + 1, dtype=np.int64) * nf
    return Batch(b, np.full(n_cand, nt, np.int32), np.full(n_cand, dmax, np.int32), off, flags)


def ragged_batch(seed: int, n_cand: int, nt_lo: int, nt_hi: int, dmax_hi: int, b: int,
                 p_num: int, p_den: int, first: int = 0) -> Batch:
    """Candidates whose tile count and maximum depth are themselves drawn."""
    c = np.arange(first, first + n_cand, dtype=np.uint64)
    u = draw_np(seed, P_SHAPE, c)
    nt = (np.uint64(nt_lo) + u % np.uint64(nt_hi - nt_lo + 1)).astype(np.int32)
    dmax = ((u >> np.uint64(32)) % np.uint64(dmax_hi + 1)).astype(np.int32)
    n_top = np.array([tet(int(x)) for x in range(nt_hi + 1)], dtype=np.int64)[nt]
    off = np.zeros(n_cand + 1, dtype=np.int64)
    off[1:] = np.cumsum(n_top)
    thr = split_threshold(p_num, p_den)
    cand_of = np.repeat(c, n_top)
    t = np.arange(off[-1], dtype=np.int64) - np.repeat(off[:-1], n_top)
    idx = (cand_of << np.uint64(24)) | t.astype(np.uint64)
    uu = draw_np(seed, P_DEPTH, idx)
    uu2 = draw_np(seed, P_DEPTH2, idx) if int(dmax.max(initial=0)) > 3 else None
    depth = depth_from_draw(uu, thr, np.repeat(dmax.astype(np.int64), n_top), uu2)
    return Batch(b, nt, dmax, off, depth)


# --------------------------------------------------------------------------
# the five named workloads

@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    nt: int
    b: int
    dmax: int
    p_num: int
    p_den: int
    ptypes: List[ProcType]
    n_cand: int
    ragged: Optional[dict] = None

    def platform(self, platform_index: int = 0) -> Platform:
        return make_platform(self.ptypes, self.seed, platform_index)

    def batch(self, n_cand: Optional[int] = None, first: int = 0) -> Batch:
        n = self.n_cand if n_cand is None else n_cand
        if self.ragged:
            r = self.ragged
            return ragged_batch(self.seed, n, r["nt_lo"], r["nt_hi"], r["dmax_hi"], self.b,
                                self.p_num, self.p_den, first)
        return uniform_batch(self.seed, n, self.nt, self.b, self.dmax, self.p_num, self.p_den, first)


WORKLOADS = {
    # 4x4 tiles of 512, one optional halving per task, 4 CPU cores + 1 accelerator
    "chol4x4_b512_d1": Workload("chol4x4_b512_d1", 1, 4, 512, 1, 1, 2, cpu_accel_types(4, 1), 1024),
    # 16x16 tiles of 1024, up to two halvings (p=0.3), 8 CPU cores + 2 accelerators
    "chol16x16_b1024_d2": Workload("chol16x16_b1024_d2", 2, 16, 1024, 2, 3, 10,
                                   cpu_accel_types(8, 2), 65536),
    # ragged: 8..32 tiles of 512, per-candidate depth cap 0..3, big.LITTLE shared memory
    "ragged_bl_b512_d3": Workload("ragged_bl_b512_d3", 3, 32, 512, 3, 3, 10,
                                  big_little_types(4, 4), 262144,
                                  ragged=dict(nt_lo=8, nt_hi=32, dmax_hi=3)),
    # surrogate training set: 4x4 tiles, as the first workload, many platforms
    "surrogate_chol4x4": Workload("surrogate_chol4x4", 4, 4, 512, 1, 1, 2, cpu_accel_types(4, 1),
                                  32768),
    # search: 64x64 tiles of 1024, up to three halvings, 16 CPU cores + 4 accelerators
    "chol64x64_b1024_d3": Workload("chol64x64_b1024_d3", 5, 64, 1024, 3, 3, 10,
                                   cpu_accel_types(16, 4), 16384),
}

# grain batch on the 16x16 shape: every top-level task split with p = 1, 1/2,
# 1/3 or 1/4, drawn uniformly; platform of chol16x16_b1024_d2
GRAIN_WORKLOAD = dict(name="grain16x16_b1024_f1234", seed=2, nt=16, b=1024, fac=(1, 2, 3, 4),
                      ptypes=cpu_accel_types(8, 2), n_cand=16384)
