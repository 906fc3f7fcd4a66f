#!/usr/bin/env python3
"""Throughput of block-partitioned triangle counting on one MI355X.

One step is one pass of the whole path over the R-MAT scale-20 edge list
(16.8 M int32 pairs already resident in HBM): clean + degree-rank + orient
(CSR build), symmetric 8 x 8 partition into blocks and block-list tasks, and
the triangle count returned to the host as a uint64.  `value` is m' (the
graph's distinct undirected edges) divided by the step time.

Prints one JSON line.  `--gpus N` with N > 1 exits: this build runs on one
GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
METRIC = "TC edges/sec at 1 MI355X (% HBM roofline); batched graphs/sec; p50/p99 latency"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_tc_block_rmat20_p8.json")
KERNEL_SOURCES = ["paper_2209_04541_amd/csrc/tc_device.hpp", "paper_2209_04541_amd/csrc/count.hip"]


def kernel_digest():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(launches_per_step):
    """HBM bytes per launch of the counting kernel from the committed
    rocprofv3 counter summary, or None when the kernel changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_digest") != kernel_digest():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(n, s, d, m):
    import oracle
    t0 = time.perf_counter()
    tri = oracle.tc(n, s, d)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "edges/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": "one full oracle pass (clean, rank, orient, merge count) over the whole "
                      "R-MAT scale-20 graph, %.1f s" % dt}, tri


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--kernel", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2209_04541_amd as P
    from paper_2209_04541_amd import gen

    torch.cuda.set_device(0)
    n, s, d = gen.rmat(args.scale, 16, gen.seed(2, 0))
    ds = torch.from_numpy(s).cuda()
    dd = torch.from_numpy(d).cuda()
    torch.cuda.synchronize()
    opts = P.options(kernel=args.kernel)

    def step():
        g = P.Graph(n, ds, dd)
        g.partition(args.p)
        c = g.count(opts)
        info = g.info()
        g.close()
        return c, info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos = []
    counts = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        c, info = step()
        counts.append(c)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps

    m = infos[0]["m"]
    W = infos[0]["probe_work"]
    kernel_ms = float(np.mean([i["t_kernel_ms"] for i in infos]))
    launches = infos[0]["kernel_launches"]
    count_ms = float(np.mean([i["t_count_ms"] for i in infos]))
    build_ms = float(np.mean([i["t_build_ms"] for i in infos]))
    part_ms = float(np.mean([i["t_partition_ms"] for i in infos]))
    # algorithmic bytes of one counting launch: every probed row A_jk[v]
    # (4 B per element, W elements), every staged row and edge list once
    # (4 B each per oriented edge) and the two row offsets of v (8 B)
    alg_bytes = 4 * W + 16 * m
    achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
    traffic = measured_traffic(launches)

    gold_tri = None
    if args.scale == 20:
        with open(os.path.join(ROOT, "tests", "golden", "workload_counts.json")) as f:
            gold_tri = json.load(f)["block"]["triangles"]

    out = {
        "metric": METRIC,
        "value": m / (ms / 1e3),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "R-MAT scale %d, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), "
                               "seed (2,0), %dx%d blocks" % (args.scale, args.p, args.p),
                   "n": n, "m_input": len(s), "m": m, "p": args.p},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "triangles": counts[0],
        "parity": (gold_tri is None or all(c == gold_tri for c in counts)),
        "count_edges_per_s": m / (count_ms / 1e3),
        "kernel_edges_per_s": m / (kernel_ms / 1e3),
        "t_build_ms": build_ms,
        "t_partition_ms": part_ms,
        "t_count_ms": count_ms,
        "t_kernel_ms": kernel_ms,
        "kernel_launches_per_step": launches,
        "algorithmic_bytes_per_launch": alg_bytes,
    }
    if not args.no_cpu_baseline:
        cb, tri = cpu_baseline(n, s, d, m)
        out["cpu_baseline"] = cb
        out["parity"] = out["parity"] and tri == counts[0]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
