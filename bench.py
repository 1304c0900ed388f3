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
import dataclasses
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
# every source the simulator kernel is compiled from: stored counters count only
# while this hash matches the one recorded with them
KERNEL_SRCS = [os.path.join(ROOT, "paper_1602_05510_amd", "csrc", f)
               for f in ("hesp_sim.hip", "hesp_sim_round.inc", "hesp_device.h", "hesp_core.h", "hesp_internal.h",
                         "hesp_tree.h")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


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

def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, pf, batch_host, gpu_makespan, budget_s: float, policy=(0, 0, 0, 0), tree: bool = False,
                 capacity=None, link=None):
    """The oracle, as it stands, built -O2 -march=native on this host, on its
    cores: the whole timed batch when it fits the time budget (else its first
    candidates), plus a single-thread rate on a smaller prefix."""
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    O.build(force=True, native=True)
    cores = min(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1), 64)
    # calibrate the sample size with a small probe
    probe = batch_host.subset(range(min(64, batch_host.n)))
    t0 = time.perf_counter()
    O.simulate_batch(pf, probe, cores, policy=policy, tree=tree, native=True, capacity=capacity, link=link)
    dt = max(time.perf_counter() - t0, 1e-3)
    per_cand = dt / probe.n
    n = int(min(batch_host.n, max(probe.n, budget_s / per_cand)))
    sample = batch_host.subset(range(n))
    t0 = time.perf_counter()
    ms, ntk = O.simulate_batch(pf, sample, cores, policy=policy, tree=tree, native=True, capacity=capacity,
                               link=link)
    dt = time.perf_counter() - t0
    exact = bool(np.array_equal(ms, gpu_makespan[:n]))
    # one thread, about a tenth of the budget
    n1 = int(min(n, max(16, 0.1 * budget_s / (per_cand * cores))))
    t0 = time.perf_counter()
    _, ntk1 = O.simulate_batch(pf, batch_host.subset(range(n1)), 1, policy=policy, tree=tree, native=True,
                               capacity=capacity, link=link)
    dt1 = time.perf_counter() - t0
    what = "the whole timed batch of step 0" if n == batch_host.n else f"the first {n} candidates of the timed batch of step 0"
    return {"value": float(ntk.sum()) / dt, "unit": "tasks/s", "cores": cores, "kind": "oracle",
            "sample": f"{what}, one candidate per thread; oracle built gcc -O2 -march=native on this host",
            "cpu_model": host_cpu_model(), "candidates": n, "candidates_per_s": n / dt, "seconds": dt,
            "bit_exact_vs_gpu": exact,
            "single_thread": {"value": float(ntk1.sum()) / dt1, "unit": "tasks/s", "candidates": n1,
                              "seconds": dt1}}


# ----------------------------------------------------------------------- surrogate

MLP_FLOPS_PER_ROW = 2 * (32 * 256 + 2 * 256 * 256 + 256)     # multiply-adds of one forward row, x2
MFMA_BF16_PEAK_TFLOPS = 2500.0


def run_surrogate(args, torch, H):
    """Train the network on exact simulations of many platforms, then score every
    partition of held-out platforms and re-simulate the best-scored 1%."""
    w = I.WORKLOADS["surrogate_chol4x4"]
    n_pf, per, n_held = args.train_platforms, w.n_cand, 4
    n_all = 1 << I.tet(w.nt)                       # 2^20 partitions of the 4x4 instance
    thr = I.split_threshold(w.p_num, w.p_den)
    dev = torch.device("cuda")
    plan = H.Plan()
    N = n_pf * per
    X = torch.empty((N, 32), dtype=torch.int16, device=dev)
    MS = torch.empty(N, dtype=torch.int64, device=dev)
    st = torch.empty(max(per, n_all), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in range(n_pf):
        pf_in = w.platform(p)
        pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
        db = H.generate_uniform(w.seed, p * per, per, w.nt, w.dmax, thr)
        H.simulate_batch(plan, pf, db, MS[p * per:(p + 1) * per], st[:per])
        if not bool((st[:per] == 0).all().item()):
            raise SystemExit("training simulation reported a non-OK status")
        rate = torch.from_numpy(H.mlp_rate_features(pf_in.rmax)).to(dev)
        H.mlp_features(db.depth, per, I.tet(w.nt), rate, X[p * per:(p + 1) * per])
    torch.cuda.synchronize()
    data_s = time.perf_counter() - t0
    lms = torch.log(MS.double())
    mu, sigma = float(lms.mean()), float(lms.std())
    T = torch.empty(N, dtype=torch.float32, device=dev)
    H.mlp_targets(MS, mu, sigma, T)
    m = H.MLP(args.mlp_seed)
    loss = torch.zeros(args.train_steps, dtype=torch.float32, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    m.train(X, T, args.train_batch, args.train_steps, args.lr, seed=args.mlp_seed, loss=loss)
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    lh = loss.cpu().numpy()
    del X, MS, T

    # held-out platforms: every partition simulated exactly (the reference for the scores) and scored
    k_top = (n_all + 99) // 100
    Xh = torch.empty((n_all, 32), dtype=torch.int16, device=dev)
    y = torch.empty(n_all, dtype=torch.float32, device=dev)
    ms = torch.empty(n_all, dtype=torch.int64, device=dev)
    ws = H.topk_workspace(n_all)
    per_pf, fwd_ms = [], []
    for q in range(n_held):
        pf_in = w.platform(n_pf + q)
        pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
        db = H.generate_enumerate(0, n_all, w.nt, w.dmax)
        H.simulate_batch(plan, pf, db, ms, st[:n_all])
        rate = torch.from_numpy(H.mlp_rate_features(pf_in.rmax)).to(dev)
        H.mlp_features(db.depth, n_all, I.tet(w.nt), rate, Xh)
        for rep in range(3):                      # first launch warms up
            e0.record()
            m.forward(Xh, y)
            e1.record()
            torch.cuda.synchronize()
            if rep:
                fwd_ms.append(e0.elapsed_time(e1))
        idx = H.topk(y, k_top, ws).long()
        # re-simulate the best-scored 1% exactly
        sub = H.DeviceBatch(k_top, w.nt, w.dmax, db.depth.view(n_all, -1)[idx].contiguous().view(-1))
        ms_top = torch.empty(k_top, dtype=torch.int64, device=dev)
        H.simulate_batch(plan, pf, sub, ms_top, st[:k_top])
        exact = ms.double()
        pred = torch.exp(y.double() * sigma + mu)
        err = (pred - exact).abs()
        best = int(ms.min())
        best_idx = int(torch.argmin(ms))
        pos = (idx == best_idx).nonzero()
        order = torch.argsort(ms)
        rnd = torch.randperm(n_all, generator=torch.Generator().manual_seed(q))[:k_top].to(dev)
        per_pf.append({
            "platform": n_pf + q,
            "mae_ns": float(err.mean()), "mae_rel": float((err / exact).mean()),
            "exhaustive_best": best,
            "top1pct_best": int(ms_top.min()),
            "top1pct_best_over_exhaustive": int(ms_top.min()) / best,
            "top1pct_resim_matches_sweep": bool(torch.equal(ms_top, ms[idx])),
            "exhaustive_best_rank_in_top1pct": int(pos[0, 0]) if pos.numel() else None,
            "top1_scored_exact_rank": int((order == int(idx[0])).nonzero()[0, 0]),
            "random1pct_best_over_exhaustive": int(ms[rnd].min()) / best,
            "top1pct_mean_over_random1pct_mean": float(ms_top.double().mean() / ms[rnd].double().mean()),
        })
    fwd = float(np.median(fwd_ms))
    tflops = MLP_FLOPS_PER_ROW * n_all / (fwd * 1e-3) / 1e12
    train_tflops = 3 * MLP_FLOPS_PER_ROW * args.train_batch * args.train_steps / (train_ms * 1e-3) / 1e12
    rec = {
        "metric": "surrogate-scored partitions/sec (bf16 MFMA forward)",
        "value": n_all / (fwd * 1e-3), "unit": "candidates/s", "n_gpus": 1, "steps": len(fwd_ms),
        "warmup": n_held, "ms_per_step": fwd, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": w.name, "train_platforms": n_pf, "pairs": N, "held_out_platforms": n_held,
                   "proposals": n_all * n_held, "top_fraction": "1%", "network": "32-256-256-256-1 ReLU",
                   "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "mfma", "kernel": "forward pass (3 bf16 GEMMs + output dot)", "achieved": tflops,
                     "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / MFMA_BF16_PEAK_TFLOPS,
                     "traffic": None, "flops_per_row": MLP_FLOPS_PER_ROW, "rows_per_launch": n_all},
        "training": {"steps": args.train_steps, "batch": args.train_batch, "lr": args.lr, "ms": train_ms,
                     "tflops": train_tflops, "loss_first": float(lh[:10].mean()), "loss_last": float(lh[-50:].mean()),
                     "data_generation_s": data_s, "target_mu": mu, "target_sigma": sigma},
        "held_out": per_pf,
        "mae_rel_mean": float(np.mean([r["mae_rel"] for r in per_pf])),
    }
    if not args.no_cpu_baseline:
        from oracle import mlp_ref as R
        p = R.unflatten(m.get_params())
        xs = Xh[:args.cpu_rows].cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        xs = xs.view(np.float32)
        t0 = time.perf_counter()
        yr, _ = R.forward(p, xs, bf16=True)
        dt = time.perf_counter() - t0
        yg = y[:args.cpu_rows].cpu().numpy()
        rec["cpu_baseline"] = {"value": args.cpu_rows / dt, "unit": "candidates/s", "cores": torch.get_num_threads(),
                               "kind": "oracle", "sample": f"first {args.cpu_rows} rows of the last held-out platform",
                               "max_abs_diff_vs_gpu": float(np.abs(yr - yg).max())}
    print(json.dumps(rec), flush=True)


# ----------------------------------------------------------------------- search

def run_search(args, torch, H):
    """Plain (random warm-up + greedy mutation) search against surrogate-guided
    search on the 64x64 instance; best makespan against wall time.  Three arms
    share one plan, warmed (workspace sized, lanes per candidate tuned) by an
    untimed round of every batch shape first: plain greedy at the full batch,
    plain greedy at the surrogate's batch (what the network adds at an equal
    simulation budget), and the surrogate-guided search."""
    w = I.WORKLOADS["chol64x64_b1024_d3"]
    nt = args.search_nt or w.nt
    print(f"search nt={nt}: library loaded", file=sys.stderr, flush=True)
    dev = torch.device("cuda")
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax)
    thr = I.split_threshold(w.p_num, w.p_den)
    mut = int(round(args.mutate * (1 << 21)))
    plan = H.Plan()
    sbatch = max(1, args.batch // args.sur_ratio)
    swarm = args.sur_warm or args.batch
    common = dict(rounds=args.rounds, seed=w.seed, warm_rounds=1, pool=args.pool, split_thr=thr, mutate_thr=mut)
    def note(msg):
        print(f"search nt={nt}: {msg}", file=sys.stderr, flush=True)

    for b in sorted({args.batch, sbatch, swarm}):
        H.search(plan, pf, nt, w.dmax, H.SEARCH_RANDOM, batch=b, warm_batch=b, rounds=1, seed=w.seed + 1000,
                 warm_rounds=1, pool=args.pool, split_thr=thr, mutate_thr=mut)
        torch.cuda.synchronize()
        note(f"warm-up round of {b} candidates done")
    plain_d, plain_best, plain_tr = H.search(plan, pf, nt, w.dmax, H.SEARCH_GREEDY, batch=args.batch,
                                             warm_batch=args.batch, **common)
    note(f"plain greedy ({args.batch} per round): best {plain_best} after {plain_tr[-1]['wall_ms']:.0f} ms")
    small_d, small_best, small_tr = H.search(plan, pf, nt, w.dmax, H.SEARCH_GREEDY, batch=sbatch, warm_batch=swarm,
                                       **common)
    note(f"plain greedy ({sbatch} per round): best {small_best} after {small_tr[-1]['wall_ms']:.0f} ms")
    m = H.MLP(args.mlp_seed)
    rate = torch.from_numpy(H.mlp_rate_features(pf_in.rmax)).to(dev)
    best_d, sur_best, sur_tr = H.search(plan, pf, nt, w.dmax, H.SEARCH_SURROGATE, batch=sbatch, warm_batch=swarm,
                                        proposals=sbatch * args.sur_proposals, mlp=m, rate=rate,
                                        train_steps=args.sur_train_steps, train_batch=512, lr=1e-3,
                                        replay=1 << 16, **common)
    note(f"surrogate-guided: best {sur_best} after {sur_tr[-1]['wall_ms']:.0f} ms")
    target = plain_best * 1.01

    def reach(tr):
        return next((t["wall_ms"] for t in tr if t["best_makespan"] <= target), None)

    r_plain, r_small, r_sur = reach(plain_tr), reach(small_tr), reach(sur_tr)
    plain_ms = plain_tr[-1]["wall_ms"]

    def ratio(a, b):
        return None if a is None or b is None else a / b

    rec = {
        "metric": "time-to-best-makespan: surrogate-guided vs plain search",
        "value": ratio(r_sur, plain_ms), "unit": "fraction of plain search wall time",
        "n_gpus": 1, "steps": args.rounds, "warmup": 0, "ms_per_step": plain_ms / args.rounds,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": w.name if nt == w.nt else f"{w.name} platform and depth, nt={nt}",
                   "nt": nt, "b": w.b, "dmax": w.dmax, "rounds": args.rounds,
                   "plain_batch": args.batch, "surrogate_batch": sbatch,
                   "surrogate_proposals": sbatch * args.sur_proposals, "pool": args.pool,
                   "mutate_prob": args.mutate, "parallelism": "none (1 GPU)"},
        "target_makespan": target,
        "ratios": {"surrogate_vs_plain_wall": ratio(r_sur, plain_ms),
                   "surrogate_vs_plain_time_to_target": ratio(r_sur, r_plain),
                   "surrogate_vs_same_batch_greedy_time_to_target": ratio(r_sur, r_small)},
        "plain": {"best_makespan": plain_best, "wall_ms": plain_ms, "reached_target_at_ms": r_plain,
                  "trace": plain_tr},
        "plain_same_batch": {"best_makespan": small_best, "wall_ms": small_tr[-1]["wall_ms"],
                             "reached_target_at_ms": r_small, "trace": small_tr},
        "surrogate": {"best_makespan": sur_best, "wall_ms": sur_tr[-1]["wall_ms"], "trace": sur_tr,
                      "reached_target_at_ms": r_sur},
    }
    if args.search_check:
        # the oracle re-simulates every arm's best partition and a seeded sample of
        # the instance's random candidates (simulated on the GPU alongside)
        from oracle import oracle as O
        bests = {"plain": (plain_d, plain_best), "plain_same_batch": (small_d, small_best),
                 "surrogate": (best_d, sur_best)}
        chk = {}
        for k, (d, v) in bests.items():
            chk[k] = int(O.simulate(pf_in, nt, w.dmax, w.b, d, detail=False)) == v
            note(f"oracle re-simulated the best of {k}: {'equal' if chk[k] else 'DIFFERENT'}")
        n_s = args.search_check
        host = I.uniform_batch(w.seed + 77, n_s, nt, w.b, w.dmax, w.p_num, w.p_den)
        ms = torch.empty(n_s, dtype=torch.int64, device=dev)
        st = torch.empty(n_s, dtype=torch.int32, device=dev)
        H.simulate_batch(plan, pf, H.DeviceBatch.from_host(host), ms, st)
        want, _ = O.simulate_batch(pf_in, host, min(16, os.cpu_count() or 1))
        chk["random_sample"] = {"candidates": n_s, "bit_exact": bool(np.array_equal(ms.cpu().numpy(), want))}
        rec["oracle_check"] = chk
    print(json.dumps(rec), flush=True)


# ----------------------------------------------------------------------- policy sweep

POLICY_NAMES = {(0, 0): "PL/EFT-P", (1, 0): "FCFS/EFT-P", (0, 1): "PL/EIT-P", (1, 1): "FCFS/EIT-P",
                (0, 2): "PL/R-P", (1, 2): "FCFS/R-P", (0, 3): "PL/F-P", (1, 3): "FCFS/F-P"}


def run_policy_sweep(args, torch, H):
    """Homogeneous tilings of one matrix (every task unsplit) under every task
    order x processor selection pair: GFLOPS = (n^3 / 3) / makespan against the
    tile count, each point checked against the oracle."""
    from oracle import oracle as O
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    pf_in = w.platform()
    n = args.sweep_n
    dev = torch.device("cuda")
    rows, exact = [], True
    plan = H.Plan()
    t_gpu = 0.0
    for nt in args.sweep_nt:
        b = n // nt
        pf = H.Platform.from_inputs(pf_in, b, 0)
        db = H.DeviceBatch(1, nt, 0, torch.zeros(I.tet(nt), dtype=torch.uint8, device=dev))
        ms = torch.empty(1, dtype=torch.int64, device=dev)
        st = torch.empty(1, dtype=torch.int32, device=dev)
        host = I.Batch(b, np.array([nt], np.int32), np.array([0], np.int32), np.array([0, I.tet(nt)], np.int64),
                       np.zeros(I.tet(nt), np.uint8))
        for (order, sel), name in POLICY_NAMES.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H.simulate_batch(plan, pf, db, ms, st, policy=(order, sel, 0, args.sweep_seed))
            torch.cuda.synchronize()
            t_gpu += time.perf_counter() - t0
            got = int(ms.item())
            want, _ = O.simulate_batch(pf_in, host, 1, policy=(order, sel, args.sweep_seed))
            exact &= got == int(want[0]) and int(st.item()) == 0
            rows.append({"nt": nt, "b": b, "policy": name, "makespan_ns": got,
                         "gflops": (n ** 3 / 3) / got})
            print(f"sweep nt={nt} {name}: {got} ns, oracle {int(want[0])}, {time.perf_counter() - t0:.2f} s",
                  file=sys.stderr, flush=True)
    best = {}
    for r in rows:
        if r["policy"] not in best or r["gflops"] > best[r["policy"]]["gflops"]:
            best[r["policy"]] = r
    rec = {"metric": "policy x tile-count sweep (homogeneous partitions)", "value": None, "unit": "GFLOPS",
           "n_gpus": 1, "steps": len(rows), "warmup": 0, "ms_per_step": 1e3 * t_gpu / len(rows),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"{w.name} platform, n={n}, unsplit tiles", "tile_counts": args.sweep_nt,
                      "seed": args.sweep_seed, "parallelism": "none (1 GPU)"},
           "bit_exact_vs_oracle": exact, "points": rows,
           "best_tile_count": {k: {"nt": v["nt"], "gflops": v["gflops"]} for k, v in best.items()}}
    print(json.dumps(rec), flush=True)


# ----------------------------------------------------------------------- iterative solver

LIST_NAMES = {0: "All", 1: "CP", 2: "Shallow"}
SAMPLING_NAMES = {0: "Hard", 1: "Soft"}


def run_solver_tree(args, torch, H):
    """The iterative solver on split-tree partitions (nodes of every level below
    dmax are clusters) on a 12x12-tile instance of the 16x16 platform, beside the
    per-cluster solver on the same instance; value = chain-iterations per second
    of All/Soft; the CPU reference is timed on one chain and its trajectory compared."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    nt, dmax, b = 12, w.dmax, w.b
    B, iters, seed = args.solve_chains, args.solve_iters, args.solve_seed
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, b, dmax)
    nf = I.tree_flag_count(nt, dmax)
    init = I.tree_batch(seed, B, nt, b, dmax, 1, 4).depth.reshape(B, nf).copy()
    init[0] = 0
    f0 = torch.from_numpy(init).cuda()
    plan = H.Plan()

    def once(lst, samp):
        f = f0.clone()
        out = H.solve_tree(plan, pf, nt, dmax, f, iters, lst, samp, seed)
        torch.cuda.synchronize()
        return out

    for _ in range(args.warmup):
        once(0, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        best, best_ms, trace, steps = once(0, 1)
    dt = time.perf_counter() - t0
    print(f"tree solver All/Soft: {B} chains x {iters} iterations, {1e3 * dt / args.steps:.1f} ms per call",
          file=sys.stderr, flush=True)
    quality = []
    for lst in (0, 1, 2):
        for samp in (0, 1):
            bf, bm, tr, st = (x.cpu().numpy() for x in once(lst, samp))
            quality.append({"list": LIST_NAMES[lst], "sampling": SAMPLING_NAMES[samp],
                            "best_makespan": int(bm.min()), "mean_best_over_initial": float(np.mean(bm / tr[:, 0])),
                            "merges": int((st[:, :, 1] == 0).sum()), "splits": int((st[:, :, 1] == 1).sum())})
    # the per-cluster solver on the same instance, chains from random depths
    d_init = I.uniform_batch(seed, B, nt, b, dmax, 1, 4).depth.reshape(B, I.tet(nt)).copy()
    d_init[0] = 0
    cluster = {}
    for lst in (0, 1):
        d = torch.from_numpy(d_init).cuda()
        _, bm, _, _ = H.solve(plan, pf, nt, dmax, d, iters, lst, 1, seed)
        cluster[LIST_NAMES[lst] + "/Soft"] = int(bm.min().item())
    tr0 = trace.cpu().numpy()
    cpu = exact = None
    if not args.no_cpu_baseline:
        from oracle import solver_ref as S
        r = min(B - 1, 3)
        t1 = time.perf_counter()
        S.solve_tree(pf_in, nt, dmax, b, 1, 0, 1, seed + r, flags0=init[r])
        one = time.perf_counter() - t1
        k = int(max(1, min(iters, args.cpu_budget / max(one, 1e-6))))
        t1 = time.perf_counter()
        _, _, want, _ = S.solve_tree(pf_in, nt, dmax, b, k, 0, 1, seed + r, flags0=init[r])
        t_cpu = time.perf_counter() - t1
        exact = list(tr0[r, :k]) == want
        cpu = {"value": k / t_cpu, "unit": "chain-iterations/s", "cores": 1, "kind": "oracle",
               "sample": f"chain {r}, {k} iterations of All/Soft on split trees"}
    rec = {"metric": "iterative solver throughput on split-tree partitions (All/Soft)",
           "value": B * iters * args.steps / dt, "unit": "chain-iterations/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"{w.name} platform, {nt}x{nt} tiles, split-tree solver", "nt": nt, "b": b,
                      "dmax": dmax, "chains": B, "iterations": iters, "nodes_per_chain": nf, "seed": seed,
                      "parallelism": "none (1 GPU)"},
           "cpu_baseline": cpu, "bit_exact_vs_oracle": exact, "quality": quality,
           "per_cluster_solver_best": cluster, "unsplit_makespan": int(tr0[0, 0])}
    print(json.dumps(rec), flush=True)


GRAIN_SRC = os.path.join(ROOT, "paper_1602_05510_amd", "csrc", "hesp_grain.hip")


def grain_kernel_hash() -> str:
    with open(GRAIN_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# fine tasks of each kind inside a top-level cell of kind `kind` split f x f
def _grain_mix(kind: int, f: int):
    if kind == 0:
        return {0: f, 1: f * (f - 1) // 2, 2: f * (f - 1) // 2, 3: f * (f - 1) * (f - 2) // 6}
    if kind in (1, 2):
        return {kind: f * f, 3: f * f * (f - 1) // 2}
    return {3: f ** 3}


def grain_algorithmic_bytes(grain, nt: int, fac, n_mem: int, n_edges: int) -> tuple:
    """Bytes of state the grain simulation must touch, by the accounting of the
    depth batches (per task 4 + 8 + 16, per edge 12, per atom of every block the
    validity in every space, the written block's twice) plus, per atom touched,
    its 4-byte last-writer entry read (and written for the written block)."""
    L = int(np.lcm.reduce(np.asarray(fac, np.int64)))
    tops = [0 if (k == i == j) else (1 if k == i else (2 if i == j else 3)) for (k, i, j) in _fig1_kij(nt)]
    per_g = {}
    for g, f in enumerate(fac):
        w2 = (L // f) ** 2
        for kind in range(4):
            t = a = aw = 0
            for fk, cnt in _grain_mix(kind, f).items():
                t += cnt
                a += cnt * _NB[fk] * w2
                aw += cnt * w2
            per_g[(kind, g)] = (t, a, aw)
    tasks = atoms = written = 0
    cnt = np.zeros((4, len(fac)), np.int64)
    for t_idx, kind in enumerate(tops):
        np.add.at(cnt[kind], grain[:, t_idx].astype(np.int64), 1)
    for (kind, g), (t, a, aw) in per_g.items():
        tasks += int(cnt[kind, g]) * t
        atoms += int(cnt[kind, g]) * a
        written += int(cnt[kind, g]) * aw
    b = tasks * 28 + n_edges * 12 + 8 * n_mem * (atoms + written) + 4 * (atoms + written)
    return b, tasks


def _fig1_kij(nt: int):
    out = []
    for k in range(nt):
        out.append((k, k, k))
        out += [(k, k, j) for j in range(k + 1, nt)]
        for i in range(k + 1, nt):
            out += [(k, i, j) for j in range(i + 1, nt)]
            out.append((k, i, i))
    return out


def run_grain(args, torch, H):
    """Grain batch (partition parameter p = 1/f per top-level task, partially
    overlapping blocks): simulated tasks per second of k_grain on the 16x16-tile
    workload, with its roofline and the oracle timed beside it."""
    w = I.GRAIN_WORKLOAD
    nt, b, fac = w["nt"], w["b"], list(w["fac"])
    n = args.n_cand or w["n_cand"]
    slots = args.slots
    pf_in = I.make_platform(w["ptypes"], w["seed"])
    pf = H.grain_platform(pf_in, b, fac)
    grains = [I.grain_batch(w["seed"], n, nt, len(fac), first=s * n) for s in range(args.warmup + args.steps)]
    dev = [torch.from_numpy(g).cuda() for g in grains]
    ms = torch.zeros(n, dtype=torch.int64, device="cuda")
    ntk = torch.zeros(n, dtype=torch.int32, device="cuda")
    ne = torch.zeros(n, dtype=torch.int64, device="cuda")
    st = torch.zeros(n, dtype=torch.int32, device="cuda")
    ws = torch.empty(H.grain_workspace_bytes(nt, fac, pf_in.n_mem, slots), dtype=torch.uint8, device="cuda")
    for s in range(args.warmup):
        H.simulate_grain_batch(pf, nt, fac, dev[s], ms, ntk, ne, st, ws=ws, slots=slots)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    tasks = 0
    t0 = time.perf_counter()
    ev0.record()
    for s in range(args.steps):
        H.simulate_grain_batch(pf, nt, fac, dev[args.warmup + s], ms, ntk, ne, st, ws=ws, slots=slots)
        if s == args.steps - 1:
            ev1.record()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kernel_ms = ev0.elapsed_time(ev1) / args.steps
    if int((st != 0).sum().item()):
        raise SystemExit("grain simulation reported a non-OK status; the measurement is invalid")
    # every step's batch has the same shape; task counts of the last one times steps
    last_tasks = int(ntk.sum().item())
    for s in range(args.steps):
        g = grains[args.warmup + s]
        tasks += grain_algorithmic_bytes(g, nt, fac, pf_in.n_mem, 0)[1]
    alg_bytes, alg_tasks = grain_algorithmic_bytes(grains[-1], nt, fac, pf_in.n_mem, int(ne.sum().item()))
    assert alg_tasks == last_tasks, (alg_tasks, last_tasks)
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = None
    pmc_path = os.path.join(PROFILES, f"k_grain_{w['name']}_pmc.json")
    if os.path.exists(pmc_path):
        with open(pmc_path) as f:
            pmc = json.load(f)
        if pmc.get("kernel_sha") == grain_kernel_hash() and pmc.get("n_cand") == n and pmc.get("slots") == slots:
            traffic = pmc.get("hbm_bytes_per_launch")
    cpu = None
    gpu_ms = ms.cpu().numpy()
    if not args.no_cpu_baseline:
        sys.path.insert(0, ROOT)
        from oracle import oracle as O
        O.build(force=True, native=True)
        cores = min(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1), 64)
        g_last = grains[-1]
        t1 = time.perf_counter()
        O.simulate_grain_batch(pf_in, nt, fac, b, g_last[:cores], n_threads=cores, native=True)
        per = max(time.perf_counter() - t1, 1e-3) / cores
        k = int(min(n, max(cores, args.cpu_budget / per)))
        t1 = time.perf_counter()
        want, wn = O.simulate_grain_batch(pf_in, nt, fac, b, g_last[:k], n_threads=cores, native=True)
        t_cpu = time.perf_counter() - t1
        cpu = {"value": float(wn.sum()) / t_cpu, "unit": "tasks/s", "cores": cores, "kind": "oracle",
               "sample": f"the first {k} candidates of the last timed batch, one candidate per thread; oracle built "
                         "gcc -O2 -march=native on this host",
               "cpu_model": host_cpu_model(), "candidates": k, "seconds": t_cpu,
               "bit_exact_vs_gpu": bool(np.array_equal(want, gpu_ms[:k]))}
    # quality beside the rate: best makespan of the last batch against the same
    # number of candidates restricted to halvings (p = 1, 1/2, 1/4: the depth batch)
    best_grain = int(ms[ms >= 0].min().item())
    pw = [1, 2, 4]
    pfw = H.grain_platform(pf_in, b, pw)
    g_pw = torch.from_numpy(I.grain_batch(w["seed"], n, nt, len(pw), first=(args.warmup + args.steps) * n)).cuda()
    ms_pw = torch.zeros(n, dtype=torch.int64, device="cuda")
    H.simulate_grain_batch(pfw, nt, pw, g_pw, ms_pw, slots=slots,
                           ws=ws if ws.numel() >= H.grain_workspace_bytes(nt, pw, pf_in.n_mem, slots) else None)
    torch.cuda.synchronize()
    quality = {"best_makespan_ns": best_grain, "best_makespan_halvings_ns": int(ms_pw[ms_pw >= 0].min().item()),
               "candidates_each": n, "halvings": pw}
    rec = {"metric": "simulated tasks per second (grain batch)", "value": tasks / dt, "unit": "tasks/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": w["name"], "nt": nt, "b": b, "factors": fac, "candidates": n, "slots": slots,
                      "tasks_per_candidate": last_tasks / n, "platform": "8 CPU cores + 2 accelerators",
                      "parallelism": "none (1 GPU)"},
           "roofline": {"bound": "hbm", "kernel": "k_grain", "achieved": achieved, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                        "algorithmic_bytes_per_launch": alg_bytes, "kernel_ms": kernel_ms,
                        "kernel_sha": grain_kernel_hash()},
           "cpu_baseline": cpu, "quality": quality}
    print(json.dumps(rec), flush=True)


def run_solver(args, torch, H):
    """The iterative scheduler-partitioner (section 2.1) on the 16x16 instance:
    many independent chains (one unsplit, the others from random initial
    partitions), each iteration an exact simulation of every
    chain plus one partition change.  value = chain-iterations per second of the
    All/Soft configuration; the other list x sampling pairs are reported for
    quality; the CPU reference is timed on one chain and its trajectory compared."""
    w = I.WORKLOADS["chol16x16_b1024_d2"]
    nt, dmax, b = w.nt, w.dmax, w.b
    B, iters, seed = args.solve_chains, args.solve_iters, args.solve_seed
    n_top = I.tet(nt)
    pf_in = w.platform()
    pf = H.Platform.from_inputs(pf_in, b, dmax)
    init = I.uniform_batch(seed, B, nt, b, dmax, 1, 4).depth.reshape(B, n_top).copy()
    init[0] = 0                     # chain 0 starts unsplit, the others from random partitions
    d0 = torch.from_numpy(init).cuda()
    plan = H.Plan()
    # uniform partitions for reference (not chains: a chain split everywhere would
    # hold every iteration back by its length)
    homog = {}
    for d in range(dmax + 1):
        ms1 = torch.empty(1, dtype=torch.int64, device="cuda")
        st1 = torch.empty(1, dtype=torch.int32, device="cuda")
        db = H.DeviceBatch(1, nt, dmax, torch.full((n_top,), d, dtype=torch.uint8, device="cuda"))
        H.simulate_batch(plan, pf, db, ms1, st1)
        homog[f"depth{d}"] = int(ms1.item())

    def once(lst, samp):
        d = d0.clone()
        out = H.solve(plan, pf, nt, dmax, d, iters, lst, samp, seed)
        torch.cuda.synchronize()
        return out

    for _ in range(args.warmup):
        once(0, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        best, best_ms, trace, steps = once(0, 1)
    dt = time.perf_counter() - t0
    value = B * iters * args.steps / dt
    print(f"solver All/Soft: {B} chains x {iters} iterations, {1e3 * dt / args.steps:.1f} ms per call",
          file=sys.stderr, flush=True)

    quality = []
    for lst in (0, 1, 2):
        for samp in (0, 1):
            bd, bm, tr, st = (x.cpu().numpy() for x in once(lst, samp))
            moved = (st[:, :, 0] >= 0).sum(axis=1)
            quality.append({"list": LIST_NAMES[lst], "sampling": SAMPLING_NAMES[samp],
                            "best_makespan": int(bm.min()), "best_chain": int(bm.argmin()),
                            "mean_best_over_initial": float(np.mean(bm / tr[:, 0])),
                            "chains_improved": int((bm < tr[:, 0]).sum()),
                            "mean_changes": float(moved.mean())})
    tr0 = trace.cpu().numpy()

    cpu = None
    exact = None
    if not args.no_cpu_baseline:
        from oracle import solver_ref as S
        r = min(B - 1, 3)
        t1 = time.perf_counter()
        S.solve(pf_in, nt, dmax, b, 1, 0, 1, seed + r, depth0=init[r])
        one = time.perf_counter() - t1
        k = int(max(1, min(iters, args.cpu_budget / max(one, 1e-6))))
        t1 = time.perf_counter()
        _, _, want, _ = S.solve(pf_in, nt, dmax, b, k, 0, 1, seed + r, depth0=init[r])
        t_cpu = time.perf_counter() - t1
        exact = list(tr0[r, :k]) == want
        cpu = {"value": k / t_cpu, "unit": "chain-iterations/s", "cores": 1, "kind": "oracle",
               "sample": f"chain {r}, {k} iterations of All/Soft (one exact simulation + partition stage each)"}

    rec = {"metric": "iterative solver throughput (All/Soft)", "value": value, "unit": "chain-iterations/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": f"{w.name} iterative solver", "nt": nt, "b": b, "dmax": dmax, "chains": B,
                      "iterations": iters, "seed": seed, "parallelism": "none (1 GPU)"},
           "cpu_baseline": cpu, "bit_exact_vs_oracle": exact,
           "homogeneous_makespans": homog, "quality": quality}
    print(json.dumps(rec), flush=True)


# ----------------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chol16x16_b1024_d2")
    ap.add_argument("--n-cand", type=int, default=0)
    ap.add_argument("--group", type=int, default=0, help="lanes per candidate (0 = autotuned)")
    ap.add_argument("--fuse", type=int, nargs="?", const=1, default=0, choices=[0, 1, 2],
                    help="fused pipeline: the 64-lane event loop prepares each candidate itself (one launch per "
                         "batch); 2: with each candidate's workspace in LDS")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=30.0)
    ap.add_argument("--train-platforms", type=int, default=64)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--train-batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--mlp-seed", type=int, default=1)
    ap.add_argument("--cpu-rows", type=int, default=65536)
    ap.add_argument("--search-nt", type=int, default=16,
                    help="tiles per dimension of the searched instance (the 64x64 one: 64)")
    ap.add_argument("--rounds", type=int, default=64)
    ap.add_argument("--search-check", type=int, default=0, metavar="N",
                    help="search: the oracle re-simulates each arm's best and N seeded random candidates")
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--mutate", type=float, default=0.004)
    ap.add_argument("--sur-ratio", type=int, default=16)
    ap.add_argument("--sur-proposals", type=int, default=16)
    ap.add_argument("--sur-warm", type=int, default=4096)
    ap.add_argument("--sur-train-steps", type=int, default=20)
    ap.add_argument("--sweep-n", type=int, default=16384)
    ap.add_argument("--sweep-nt", type=int, nargs="+", default=[2, 4, 8, 16, 32, 64])
    ap.add_argument("--sweep-seed", type=int, default=1)
    ap.add_argument("--policy", type=int, nargs=3, default=[0, 0, 0], metavar=("ORDER", "SELECT", "CACHE"),
                    help="order 0 PL / 1 FCFS, select 0 EFT-P / 1 EIT-P / 2 R-P / 3 F-P, cache 0 WB / 1 WT / 2 WA")
    ap.add_argument("--policy-seed", type=int, default=0)
    ap.add_argument("--bus", action="store_true", help="every transfer shares one interconnect")
    ap.add_argument("--links", choices=["own", "switch"], default=None,
                    help="transfers contend per link: every memory space on a link of its own, or the host "
                         "on one and the accelerators behind one switch")
    ap.add_argument("--capacity-blocks", type=int, default=0,
                    help="finite accelerator spaces: finest blocks each one holds (0: unbounded)")
    ap.add_argument("--dmax", type=int, default=None,
                    help="maximum split depth of a uniform workload (0..5; above 3: 16 or 32 lanes per candidate)")
    ap.add_argument("--tree", action="store_true",
                    help="split-tree candidates (every task split on its own) of the same shape")
    ap.add_argument("--slots", type=int, default=4096, help="grain batch: candidates in flight")
    ap.add_argument("--solve-chains", type=int, default=16384)
    ap.add_argument("--solve-iters", type=int, default=16)
    ap.add_argument("--solve-seed", type=int, default=7)
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

    if args.workload == "surrogate_chol4x4":
        return run_surrogate(args, torch, H)
    if args.workload == "chol64x64_b1024_d3":
        return run_search(args, torch, H)
    if args.workload == "policy_sweep":
        return run_policy_sweep(args, torch, H)
    if args.workload == "iterative_solver":
        return run_solver(args, torch, H)
    if args.workload == "iterative_solver_tree":
        return run_solver_tree(args, torch, H)
    if args.workload == I.GRAIN_WORKLOAD["name"]:
        return run_grain(args, torch, H)
    w = I.WORKLOADS[args.workload]
    if args.dmax is not None and args.dmax != w.dmax:
        if w.ragged:
            print(json.dumps({"error": "--dmax applies to uniform workloads"}))
            sys.exit(2)
        w = dataclasses.replace(w, dmax=args.dmax, name=f"{w.name[:w.name.rindex('_d')]}_d{args.dmax}")
    n = args.n_cand or w.n_cand
    pf_in = w.platform()
    cap_bytes = None
    if args.capacity_blocks > 0:
        # every accelerator space holds that many finest blocks (side b / 2^dmax)
        cap_bytes = np.zeros(pf_in.n_mem, np.int64)
        cap_bytes[1:] = args.capacity_blocks * pf_in.elem_bytes * (w.b >> w.dmax) ** 2
    link = None
    if args.links == "own":
        link = np.arange(pf_in.n_mem, dtype=np.int32)
    elif args.links == "switch":
        link = np.array([0] + [1] * (pf_in.n_mem - 1), np.int32)
    pf = H.Platform.from_inputs(pf_in, w.b, w.dmax, capacity_bytes=cap_bytes, link=link)
    thr = I.split_threshold(w.p_num, w.p_den)
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream()

    ms = torch.empty(n, dtype=torch.int64, device=dev)
    st = torch.empty(n, dtype=torch.int32, device=dev)
    ntk = torch.empty(n, dtype=torch.int32, device=dev)
    best = torch.empty(2, dtype=torch.int64, device=dev)

    plan = H.Plan(group=args.group, fuse=args.fuse)
    plan.timing(True)
    sim_ms = []

    def gen(i: int):
        if args.tree:
            return H.generate_tree_uniform(w.seed, i * n, n, w.nt, w.dmax, thr)
        if w.ragged:
            r = w.ragged
            return H.generate_ragged(w.seed, i * n, n, r["nt_lo"], r["nt_hi"], r["dmax_hi"], thr)
        return H.generate_uniform(w.seed, i * n, n, w.nt, w.dmax, thr)

    order, select, cache = args.policy
    bus = int(args.bus or link is not None)
    gpol = (order, select, cache, args.policy_seed, bus)

    def sim(db):
        if args.tree:
            H.simulate_tree_batch(plan, pf, db, ms, st, n_tasks=ntk, policy=gpol)
        else:
            H.simulate_batch(plan, pf, db, ms, st, n_tasks=ntk, policy=gpol)

    def step(i: int, timed: bool):
        db = gen(i)
        sim(db)
        H.argmin(ms, best)
        if timed:
            # waits for this step's kernel events; the next step is queued after
            sim_ms.append(plan.last_ms())
        return db

    for i in range(args.warmup):
        step(1000 + i, False)
        int(ntk.sum().item())          # the timed loop's own torch reduction, loaded before timing
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
    # the accounting uses the batch of the last step); uniform batches only
    achieved = traffic = alg_bytes = issue = None
    traffic_note = "split-tree batch: no algorithmic byte count" if args.tree else "ragged batch: no algorithmic byte count"
    if not w.ragged and not args.tree:
        host_last = w.batch(n, first=(args.steps - 1) * n)
        db_last = H.DeviceBatch.from_host(host_last)
        _, e_last = H.count_batch(db_last)
        alg_bytes, alg_tasks = algorithmic_bytes(host_last, pf_in.n_mem, int(e_last.sum().item()))
        achieved = alg_bytes / (sim_avg_ms * launches_per_step * 1e-3) / 1e9
        pmc_path = os.path.join(PROFILES, f"k_sim_{w.name}_pmc.json")
        if os.path.exists(pmc_path):
            with open(pmc_path) as f:
                pmc = json.load(f)
            if (pmc.get("kernel_sha") == kernel_hash() and pmc.get("n_cand") == n and tuple(args.policy) == (0, 0, 0)
                    and not bus and not args.capacity_blocks):
                traffic = pmc.get("hbm_bytes_per_launch")
        traffic_note = None if traffic is not None else "no counter run on this kernel source"
        # issue rate of the same kernel source: instructions per simulated task and
        # pipe occupancy from the SQ counter run
        sq_path = os.path.join(PROFILES, f"k_sim_{w.name}_sq.json")
        if os.path.exists(sq_path):
            with open(sq_path) as f:
                sq = json.load(f)
            if (sq.get("kernel_sha") == kernel_hash() and sq.get("n_cand") == n and tuple(args.policy) == (0, 0, 0)
                    and not bus and not args.capacity_blocks):
                issue = {k: sq[k] for k in ("valu_insts_per_task", "salu_insts_per_task", "insts_per_task",
                                            "valu_busy", "salu_busy", "wave_wait_frac", "source")}

    value = tasks_total / elapsed
    pname = (["PL", "FCFS"][order] + "/" + ["EFT-P", "EIT-P", "R-P", "F-P"][select] + "/" +
             ["WB", "WT", "WA"][cache] + ("" if not bus else ("/shared interconnect" if link is None else
                                                               f"/links {args.links} {link.tolist()}")))
    rec = {
        "metric": ("simulated tasks/sec (bit-exact PL/EFT-P makespans)" if pname == "PL/EFT-P/WB" else
                   f"simulated tasks/sec (bit-exact {pname} makespans)") + (", split-tree candidates" if args.tree else "")
                  + (f", accelerator spaces of {args.capacity_blocks} finest blocks" if args.capacity_blocks else ""),
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
        "config": {"workload": w.name + (" split trees (one Bernoulli flag per task and level)" if args.tree else ""),
                   "n_cand": n,
                   "nt": f"{w.ragged['nt_lo']}..{w.ragged['nt_hi']}" if w.ragged else w.nt, "b": w.b,
                   "dmax": f"0..{w.ragged['dmax_hi']}" if w.ragged else w.dmax,
                   "split_prob": f"{w.p_num}/{w.p_den}",
                   "platform": " + ".join(f"{t.count} {t.name}" for t in w.ptypes),
                   "policy": pname, "capacity_blocks": args.capacity_blocks or None,
                   "parallelism": "none (1 GPU)"},
        "candidates_per_s": n * args.steps / elapsed,
        "tasks_per_step": tasks_total / args.steps,
        "roofline": {"bound": "hbm", "kernel": "k_sim", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": None if achieved is None else achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "traffic_note": traffic_note,
                     "issue": issue,
                     "algorithmic_bytes_per_launch": None if alg_bytes is None else alg_bytes / launches_per_step,
                     "launch_ms": sim_avg_ms,
                     "launches_per_step": launches_per_step, "prepare_launch_ms": prep_avg_ms,
                     "kernel_sha": kernel_hash()},
    }
    if not args.no_cpu_baseline:
        if args.tree:
            host0 = I.tree_batch(w.seed, min(n, 16384), w.nt, w.b, w.dmax, w.p_num, w.p_den)
        else:
            host0 = w.batch(n, first=0)
        # recompute step 0's makespans for the sample comparison
        db = gen(0)
        sim(db)
        torch.cuda.synchronize()
        rec["cpu_baseline"] = cpu_baseline(w, pf_in, host0, ms.cpu().numpy(), args.cpu_budget,
                                           policy=(order, select, args.policy_seed, cache, bus), tree=args.tree,
                                           capacity=cap_bytes, link=link)
        rec["gpu_vs_cpu"] = value / rec["cpu_baseline"]["value"]
    if args.copy_calib:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
