#!/usr/bin/env python3
"""Throughput of the batched HeSP simulator on one MI355X.

One step = the whole hot path over one batch of synthetic candidates, inputs
resident in HBM: candidate generation on the GPU from counters, expansion,
critical times and the PL/EFT-P event simulation of every candidate (one
persistent kernel), and the batch reduction to the best candidate.  Each step
draws a fresh batch (different counters).  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1602_05510_amd import inputs as I  # noqa: E402

HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_1602_05510_amd", "csrc", "hesp_sim.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# ----------------------------------------------------------------------- accounting
# Algorithmic bytes of state one simulated task touches (int64 times, 4-byte ids):
#   4 (descriptor) + 8 (critical time) + 16 (queue append and pop)
#   + 12 per successor (4 id + 8 predecessor-count read and write)
#   + 8 * M * (A_read_and_written + A_written)  (validity of every finest block of
#     the task's blocks in every memory space is read at mapping; the written
#     block is rewritten in every space at completion)
# where A counts finest blocks (atoms).  Transfers committed at mapping are data
# dependent and left out, so this is a lower bound.
_NB = {0: 1, 1: 2, 2: 2, 3: 3}


def _fine_mix(kind: int, d: int):
    """(#fine tasks, sum over them of (blocks + 1)) of a top-level task split d times."""
    s = 1 << d
    if kind == 3:
        cnt = {3: s ** 3}
    elif kind == 2:
        cnt = {2: s * s, 3: s * s * (s - 1) // 2}
    elif kind == 1:
        cnt = {1: s * s, 3: s * s * (s - 1) // 2}
    else:
        cnt = {0: s, 1: s * (s - 1) // 2, 2: s * (s - 1) // 2, 3: s * (s - 1) * (s - 2) // 6}
    return sum(cnt.values()), sum(v * (_NB[k] + 1) for k, v in cnt.items())


def algorithmic_bytes(batch, n_mem: int, n_edges_total: int) -> tuple:
    """(total bytes, total tasks) over a uniform batch."""
    nt, dmax = int(batch.nt[0]), int(batch.dmax[0])
    n_top = I.tet(nt)
    kinds = np.zeros(n_top, np.int64)
    t = 0
    for k in range(nt):
        kinds[t] = 0; t += 1
        for j in range(k + 1, nt):
            kinds[t] = 1; t += 1
        for i in range(k + 1, nt):
            for j in range(i + 1, nt):
                kinds[t] = 3; t += 1
            kinds[t] = 2; t += 1
    cnt_tab = np.zeros((4, dmax + 1), np.int64)
    atom_tab = np.zeros((4, dmax + 1), np.int64)
    for k in range(4):
        for d in range(dmax + 1):
            c, nb1 = _fine_mix(k, d)
            cnt_tab[k, d] = c
            atom_tab[k, d] = nb1 * (4 ** (dmax - d))
    dep = batch.depth.reshape(batch.n, n_top).astype(np.int64)
    tasks = int(cnt_tab[kinds[None, :], dep].sum())
    atoms = int(atom_tab[kinds[None, :], dep].sum())
    total = 28 * tasks + 12 * n_edges_total + 8 * n_mem * atoms
    return total, tasks


# ----------------------------------------------------------------------- CPU baseline

def cpu_baseline(w, pf, batch_host, gpu_makespan, budget_s: float):
    """The oracle, as it stands, on the host cores, over a bounded sample of the batch."""
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    O.build(force=False)
    cores = min(os.cpu_count() or 1, 64)
    # calibrate the sample size with a small probe
    probe = batch_host.subset(range(min(64, batch_host.n)))
    t0 = time.perf_counter()
    ms, ntk = O.simulate_batch(pf, probe, cores)
    dt = max(time.perf_counter() - t0, 1e-3)
    per_cand = dt / probe.n
    n = int(min(batch_host.n, max(probe.n, budget_s / per_cand)))
    sample = batch_host.subset(range(n))
    t0 = time.perf_counter()
    ms, ntk = O.simulate_batch(pf, sample, cores)
    dt = time.perf_counter() - t0
    exact = bool(np.array_equal(ms, gpu_makespan[:n]))
    return {"value": float(ntk.sum()) / dt, "unit": "tasks/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} candidates of the timed batch of step 0, one candidate per thread",
            "candidates_per_s": n / dt, "seconds": dt, "bit_exact_vs_gpu": exact}


# ----------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chol16x16_b1024_d2")
    ap.add_argument("--n-cand", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain 1 GiB device copy (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; the batch shards by candidate across GPUs "
                                   "but no multi-GPU path is built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_1602_05510_amd import hesp as H
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)

    w = I.WORKLOADS[args.workload]
    if w.ragged:
        raise SystemExit("bench.py times uniform workloads; the ragged one is a parity case")
    n = args.n_cand or w.n_cand
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    thr = I.split_threshold(w.p_num, w.p_den)
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()

    ms = torch.empty(n, dtype=torch.int64, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    ntk = torch.empty(n, dtype=torch.int32, device=dev)
    best = torch.empty(2, dtype=torch.int64, device=dev)

    plan = H.Plan()
    plan.timing(True)
    sim_ms = []

    def step(i: int, timed: bool):
        db = H.generate_uniform(w.seed, i * n, n, w.nt, w.dmax, thr)
        H.simulate_batch(plan, pf, db, ms, st, n_tasks=ntk)
        H.argmin(ms, best)
        if timed:
            # waits for this step's kernel events; the next step is queued after
            sim_ms.append(plan.last_ms())
        return db

    for i in range(args.warmup):
        step(1000 + i, False)
    torch.cuda.synchronize()

    tasks_total = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    task_counts = []
    for i in range(args.steps):
        step(i, True)
        task_counts.append(ntk.sum())      # device-side sum, read after the timed region
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    tasks_total = int(sum(int(x.item()) for x in task_counts))
    status_ok = bool((st == 0).all().item())
    ms_last = ms.clone()
    if not status_ok:
        raise SystemExit("simulation reported a non-OK status; the measurement is invalid")
    sim_launches = sum(x[2] for x in sim_ms)
    sim_avg_ms = float(sum(x[1] for x in sim_ms) / sim_launches)          # per k_sim launch
    prep_avg_ms = float(sum(x[0] for x in sim_ms) / sim_launches)         # per k_prepare launch
    launches_per_step = sim_launches / len(sim_ms)

    # roofline accounting for the simulation kernel (steps are statistically alike;
    # the accounting uses the batch of the last step)
    host_last = w.batch(n, first=(args.steps - 1) * n)
    db_last = H.DeviceBatch.from_host(host_last)
    _, e_last = H.count_batch(db_last)
    alg_bytes, alg_tasks = algorithmic_bytes(host_last, pf_in.n_mem, int(e_last.sum().item()))
    achieved = alg_bytes / (sim_avg_ms * launches_per_step * 1e-3) / 1e9
    traffic = None
    pmc_path = os.path.join(PROFILES, f"k_sim_{w.name}_pmc.json")
    if os.path.exists(pmc_path):
        with open(pmc_path) as f:
            pmc = json.load(f)
        if pmc.get("kernel_sha") == kernel_hash() and pmc.get("n_cand") == n:
            traffic = pmc.get("hbm_bytes_per_launch")
    traffic_note = None if traffic is not None else "no counter run on this kernel source"

    value = tasks_total / elapsed
    rec = {
        "metric": "simulated tasks/sec (bit-exact PL/EFT-P makespans)",
        "value": value,
        "unit": "tasks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": w.name, "n_cand": n, "nt": w.nt, "b": w.b, "dmax": w.dmax,
                   "split_prob": f"{w.p_num}/{w.p_den}",
                   "platform": " + ".join(f"{t.count} {t.name}" for t in w.ptypes),
                   "parallelism": "none (1 GPU)"},
        "candidates_per_s": n * args.steps / elapsed,
        "tasks_per_step": tasks_total / args.steps,
        "roofline": {"bound": "hbm", "kernel": "k_sim", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg_bytes / launches_per_step, "launch_ms": sim_avg_ms,
                     "launches_per_step": launches_per_step, "prepare_launch_ms": prep_avg_ms,
                     "kernel_sha": kernel_hash()},
    }
    if not args.no_cpu_baseline:
        host0 = w.batch(n, first=0)
        # recompute step 0's makespans for the sample comparison
        db = H.generate_uniform(w.seed, 0, n, w.nt, w.dmax, thr)
        H.simulate_batch(plan, pf, db, ms, st, n_tasks=ntk)
        torch.cuda.synchronize()
        rec["cpu_baseline"] = cpu_baseline(w, pf_in, host0, ms.cpu().numpy(), args.cpu_budget)
        rec["gpu_vs_cpu"] = value / rec["cpu_baseline"]["value"]
    if args.copy_calib:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
