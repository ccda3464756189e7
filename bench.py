#!/usr/bin/env python3
"""Benchmark of the network density-of-states hot path on one MI355X.

One step is one pass of the whole path over one synthetic graph whose edge
list is already resident in HBM:

  graph build (symmetrise / dedup / drop isolated / CSR)  -> nd_build_csr
  twin detection (hash + exact verification)              -> nd_motif_filter
  probe block + projection, M-1 Chebyshev sparse steps
  with fused fp64 global and per-node moment sums         -> nd_ldos_moments / nd_cheb_moments
  Jackson-damped histograms (global DOS, per-node PDOS)   -> nd_reconstruct

The figure of merit is G(nnz*probe*moment)/s = nnz * probes * (M-1) / step
time.  The roofline object reports the sparse step kernel (the dominant
kernel): algorithmic bytes per launch (compulsory traffic of one step: the
int32 pattern, row pointers, the degree scale, one read of X_m, one read of
X_{m-1}, one write of X_{m+1}, plus the per-node moment column when LDOS is
computed) divided by its average launch time from HIP events on the launch
stream, against the 8 TB/s HBM3E peak.

The CPU baseline times the fp64 oracle (plain numpy/scipy, one thread) on a
bounded sample, following the paper's timing protocol (the first 10 moments).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G(nnz·probe·moment)/s + HBM GB/s; probes to 1e-3 LDOS var, plain vs learned"
UNIT = "G(nnz·probe·moment)/s"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(n: int, nnz: int, k: int, ldos: bool, state_bytes: int = 4) -> int:
    """Compulsory HBM traffic of one sparse step (one kernel launch)."""
    b = 4 * nnz + 8 * (n + 1) + 4 * n + 3 * state_bytes * k * n
    if ldos:
        b += 8 * n
    return b


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload: str, k: int, ldos: bool, seed: int):
    """The oracle as it stands, timed on the first 10 moments (9 sparse
    products) of a bounded sample; returns the rate in the metric's unit."""
    import synthgraph as sg
    from oracle import graph as og, kpm, rng as orng
    if workload == "ba1m_twins":
        n, s, d = sg.barabasi_albert(1_000_000, 5, seed=seed, twin_pairs=25_000)
        sample = "same BA-1M graph and probe count, first 10 moments (9 products)"
    elif workload in ("rmat27", "rmat22"):
        n, s, d = sg.rmat(21, 8, seed=seed)
        sample = "R-MAT scale 21 ef 8 (same a,b,c,d), same probe count, first 10 moments (9 products)"
    else:
        n, s, d = sg.erdos_renyi(2000, 0.005, seed=seed)
        sample = "same ER-2000 graph and probe count, first 10 moments (9 products)"
    g = og.build_csr(n, s, d)
    H = og.normalized_adjacency(g)
    Z = orng.rademacher(g.n, k, seed)
    t0 = time.perf_counter()
    kpm.stochastic_moments(H, Z, 10, ldos=ldos)
    dt = time.perf_counter() - t0
    rate = g.nnz * k * 9 / dt / 1e9
    return {"value": rate, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": sample + "; fp64 numpy/scipy single thread, %.2f s, host CPU: %s" % (dt, cpu_model())}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ba1m_twins", choices=["ba1m_twins", "rmat27", "rmat22", "er2000"])
    ap.add_argument("--no-filter", action="store_true", help="skip twin filtering (ba1m_twins)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the hot path shards by probes, "
              "see the design notes); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": a.numel() * 4, "launches": 3}), flush=True)
        return
    import paper_1905_09758_amd as nd
    from synthgraph.workloads import WORKLOADS
    nd.require_gpu()
    W = WORKLOADS[args.workload]
    k, M = W.probes, W.moments
    use_filter = W.filter_twins and not args.no_filter
    t_gen = time.perf_counter()
    n_nodes, src, dst = W.graph(args.seed)
    t_gen = time.perf_counter() - t_gen
    src_d = torch.from_numpy(src).cuda()
    dst_d = torch.from_numpy(dst).cuda()
    del src, dst
    torch.cuda.synchronize()
    f64 = torch.float64

    out = {}

    def step(timed_kernel: bool):
        g = nd.nd_build_csr(n_nodes, src_d, dst_d)
        if "mu" not in out:
            out["mu"] = torch.empty(M, dtype=f64, device="cuda")
            out["hist"] = torch.empty(W.bins, dtype=f64, device="cuda")
            if W.ldos:
                out["ldos"] = torch.empty(g.n * M, dtype=f64, device="cuda")
                out["pdos"] = torch.empty(g.n * 50, dtype=f64, device="cuda")
        flags = nd.ND_TIME_STEPS if timed_kernel else 0
        motifs = nd.nd_motif_filter(g, args.seed) if use_filter else None
        spikes = motifs.spikes if motifs is not None else []
        if W.ldos:
            nd.nd_ldos_moments(g, motifs, k, M, args.seed, flags, out["ldos"], mu=out["mu"])
            nd.nd_reconstruct(out["ldos"], g.n, M, nd.ND_KERNEL_JACKSON, (), 50, -1.0, 1.0, out["pdos"])
            kern = nd.ND_KERNEL_JACKSON | (nd.ND_SPIKES_IN_MOMENTS if spikes else 0)
        else:
            nd.nd_cheb_moments(g, motifs, k, M, args.seed, flags, out["mu"])
            kern = nd.ND_KERNEL_JACKSON
        nd.nd_reconstruct(out["mu"], 1, M, kern, spikes, W.bins, -1.0, 1.0, out["hist"])
        return g, motifs

    for _ in range(args.warmup):
        g, motifs = step(False)
        del g, motifs
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kern_ms, kern_n = 0.0, 0
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        g, motifs = step(True)
        ms, nl = nd.nd_graph_step_timing(g)
        kern_ms += ms
        kern_n += nl
        info = (g.n, g.nnz, g.max_deg, motifs.n_classes if motifs is not None else 0)
        del g, motifs
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = ev0.elapsed_time(ev1) / args.steps
    n, nnz, max_deg, n_cls = info
    work = nnz * k * (M - 1)
    value = work / (ms_step * 1e-3) / 1e9
    avg_launch_ms = kern_ms / max(kern_n, 1)
    b_launch = algorithmic_bytes(n, nnz, k, W.ldos)
    achieved = b_launch / (avg_launch_ms * 1e-3) / 1e9
    mu = out["mu"].cpu().numpy()
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": W.describe, "n": n, "nnz": nnz, "max_deg": max_deg,
                   "probes": k, "moments": M, "twin_filter": use_filter, "twin_classes": n_cls,
                   "ldos": W.ldos, "state": "fp32 recurrence, fp64 compensated moment sums"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_cheb_step", "avg_launch_ms": round(avg_launch_ms, 5),
                     "algorithmic_bytes_per_launch": b_launch},
        "spmm_only_G_per_s": round(work / (kern_ms * 1e-3 / args.steps) / 1e9, 3) if kern_ms else None,
        "mu_head": [round(float(x), 6) for x in mu[:4]],
        "wall_s": round(wall, 3),
        "input_gen_s": round(t_gen, 2),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, k, W.ldos, args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
