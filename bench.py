#!/usr/bin/env python3
"""Throughput of block-partitioned triangle counting on one MI355X.

Default workload ("block"): one step is one pass of the whole path over the
R-MAT scale-20 edge list (16.8 M int32 pairs already resident in HBM):
clean + degree-rank + orient (CSR build), symmetric 8 x 8 partition into
blocks and block-list tasks, and the triangle count returned to the host as a
uint64.  `value` is m' (the graph's distinct undirected edges) divided by the
step time.  Other workloads (--workload plain|ooc|batch|served|support) print their
own line; they are not the default.

Prints one JSON line.  `--gpus N` with N > 1 exits: the library runs on
one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
METRIC = "TC edges/sec at 1 MI355X (% HBM roofline); batched graphs/sec; p50/p99 latency"
# device code of the counting kernel: a stored traffic measurement is used
# only while these files are unchanged
KERNEL_SOURCES = ["paper_2209_04541_amd/csrc/tc_device.hpp", "paper_2209_04541_amd/csrc/tc_kernel.hpp",
                  "paper_2209_04541_amd/csrc/wave.hpp", "paper_2209_04541_amd/csrc/count.hpp"]


# device code of the batch kernel
BATCH_SOURCES = ["paper_2209_04541_amd/csrc/batch.hip", "paper_2209_04541_amd/csrc/tc_device.hpp",
                 "paper_2209_04541_amd/csrc/wave.hpp"]

# device code of the edge-support kernel
SUPPORT_SOURCES = ["paper_2209_04541_amd/csrc/support.hip", "paper_2209_04541_amd/csrc/tc_device.hpp",
                   "paper_2209_04541_amd/csrc/wave.hpp"]


def kernel_digest(sources=KERNEL_SOURCES):
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(name, sources=KERNEL_SOURCES):
    """L2-to-fabric bytes of a step's counting launches (one launch, or all
    of a streamed step's) from the committed rocprofv3 counter summary, or
    None when the kernel changed since.  The bytes are request counts by
    size (32, 64, 128 B) times their size; they include what Infinity Cache
    answers, so they bound HBM traffic from above."""
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            t = json.load(f)
    except OSError:
        return None
    if t.get("kernel_digest") != kernel_digest(sources):
        return None
    return t.get("bytes_per_step") or t.get("bytes_per_launch")


def cpu_model():
    """The host CPU's model name and the cores this process may use."""
    name = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": name, "cores_usable": usable}


def golden(name):
    with open(os.path.join(ROOT, "tests", "golden", "workload_counts.json")) as f:
        return json.load(f).get(name)


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def base_line(args, value, unit, ms, config, dtype="int32"):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def roofline(W, m, kernel_ms, traffic_file):
    # algorithmic bytes of one counting launch: every entry of the walked
    # partial lists (4 B each, W of them: A_jk[v] per edge (u, v) of A_ij for
    # row walks, A_ik[u] for column walks), every staged list and edge list
    # once (4 B each per oriented edge) and the two row offsets of the walked
    # endpoint (8 B per oriented edge)
    alg = 4 * W + 16 * m
    achieved = alg / (kernel_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(traffic_file)}, alg


# ---------------------------------------------------------------- graph

def run_graph(args, n, s, d, p, gold_name, workload, traffic_file, opts=None, cpu_sample=None):
    import numpy as np
    import torch

    import paper_2209_04541_amd as P

    if args.host_edges:
        # edge arrays in pinned host memory: the step includes their copy
        ds = torch.from_numpy(s).pin_memory().numpy()
        dd = torch.from_numpy(d).pin_memory().numpy()
    else:
        ds = torch.from_numpy(s).cuda()
        dd = torch.from_numpy(d).cuda()
    torch.cuda.synchronize()
    opts = opts or P.options(kernel=args.kernel)

    def step():
        g = P.Graph(n, ds, dd)
        g.partition(p)
        c = g.count(opts)
        info = g.info()
        g.close()
        return c, info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos, counts, step_ms = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        c, info = step()
        step_ms.append((time.perf_counter() - a) * 1e3)
        counts.append(c)
        infos.append(info)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps

    m = infos[0]["m"]
    W = infos[0]["probe_work_col"] if infos[0]["walked_columns"] else infos[0]["probe_work"]
    launches = max(1, infos[0]["kernel_launches"])
    kernel_ms = float(np.mean([i["t_kernel_ms"] for i in infos])) / launches
    roof, alg = roofline(W, m, kernel_ms * launches, traffic_file)
    gold = golden(gold_name) if gold_name else None
    out = base_line(args, m / (ms / 1e3), "edges/s", ms, {
        "workload": workload, "n": n, "m_input": len(s), "m": m, "p": p})
    out["roofline"] = roof
    out.update({
        "triangles": counts[0],
        "parity": gold is None or all(c == gold["triangles"] for c in counts),
        "step_ms_p50": pct(step_ms, 50), "step_ms_p99": pct(step_ms, 99),
        "count_edges_per_s": m / (float(np.mean([i["t_count_ms"] for i in infos])) / 1e3),
        "kernel_edges_per_s": m / (kernel_ms * launches / 1e3),
        "t_build_ms": float(np.mean([i["t_build_ms"] for i in infos])),
        "t_partition_ms": float(np.mean([i["t_partition_ms"] for i in infos])),
        "t_count_ms": float(np.mean([i["t_count_ms"] for i in infos])),
        "t_kernel_ms_per_launch": kernel_ms,
        "kernel_launches_per_step": launches,
        "algorithmic_bytes_per_step": alg,
        "probe_work": infos[0]["probe_work"],
        "probe_work_col": infos[0]["probe_work_col"],
        "walk": "columns" if infos[0]["walked_columns"] else "rows",
        "h2d_bytes_per_step": infos[0]["h2d_bytes"],
        "block_bytes": infos[0]["block_bytes"],
    })
    out["compulsory_bytes"] = 4 * m + 8 * n  # every oriented edge and row offset read once
    if not args.no_hybrid:
        out["hybrid"] = hybrid_leg(args, n, ds, dd, p, opts, counts[0])
        out["parity"] = out["parity"] and out["hybrid"]["exact"]
    out["copy_probe_gbs"] = copy_probe_gbs()
    out["frac_of_copy_probe"] = roof["achieved"] / out["copy_probe_gbs"]
    if args.shards:
        out["shards"] = shard_leg(args, n, ds, dd, p, opts, counts[0])
        out["parity"] = out["parity"] and out["shards"]["sum_equals_count"]
    if not args.no_cpu_baseline and cpu_sample is not None:
        cb, tri = cpu_sample()
        out["cpu_baseline"] = cb
        if tri is not None:
            out["parity"] = out["parity"] and tri == counts[0]
    return out


def hybrid_leg(args, n, ds, dd, p, opts, triangles, reps=5):
    """Device-only against hybrid host + device counts (the lightest
    block-lists counted by host threads from the pinned host block store
    while the device streams the heaviest ones) on one partitioned graph.
    Each figure is the median of `reps` counts, transfers included.  An
    in-core graph's blocks are moved to the host store before its first
    hybrid count; that one-time move is reported apart."""
    import ctypes
    import numpy as np

    import paper_2209_04541_amd as P

    threads = cpu_model()["cores_usable"] or 1
    g = P.Graph(n, ds, dd)
    g.partition(p)
    exact = True

    def med(o):
        nonlocal exact
        ts, info = [], None
        for _ in range(reps):
            c = g.count(o)
            info = g.info()
            ts.append(info["t_count_ms"])
            exact = exact and c == triangles
        return float(np.median(ts)), info

    def variant(flags=0, permille=0):
        o = P.TcOptions.from_buffer_copy(opts)
        o.flags |= flags
        o.host_permille = permille
        o.host_threads = min(64, threads)
        return o

    out = {"host_threads": min(64, threads), "reps": reps}
    in_core = not (opts.flags & P.OPT_STREAM) and not opts.device_cap_bytes
    if in_core:
        out["device_in_core_ms"], _ = med(opts)
        t0 = time.perf_counter()
        g.count(variant(P.OPT_HYBRID, 0))  # moves the blocks to the host store
        out["move_to_host_store_ms"] = (time.perf_counter() - t0) * 1e3
    out["device_streamed_ms"], _ = med(variant(P.OPT_STREAM))
    ms, info = med(variant(P.OPT_HYBRID, 0))
    out["hybrid_meet"] = {"t_count_ms": ms, "host_tasks": info["host_tasks"],
                          "host_work_share": info["host_work_share"], "tasks": info["num_tasks"]}
    fixed = {}
    for pm in (10, 50, 200):
        ms, info = med(variant(P.OPT_HYBRID, pm))
        fixed[str(pm)] = {"t_count_ms": ms, "host_tasks": info["host_tasks"],
                          "host_work_share": info["host_work_share"]}
    out["hybrid_fixed_permille"] = fixed
    best_h = min([out["hybrid_meet"]["t_count_ms"]] + [v["t_count_ms"] for v in fixed.values()])
    best_d = min(out.get("device_in_core_ms", 1e30), out["device_streamed_ms"])
    out["best_hybrid_over_best_device"] = best_h / best_d
    out["exact"] = exact
    g.close()
    return out


def shard_leg(args, n, ds, dd, p, opts, triangles):
    """One device's share of the count split by task over args.shards
    devices, run on this one GPU: every shard counted once after a whole
    count has put the blocks where they live (host memory when streamed, so
    each shard's time includes copying the blocks its tasks read), then
    shard 0 timed over the bench steps."""
    import numpy as np

    import paper_2209_04541_amd as P

    S = args.shards
    g = P.Graph(n, ds, dd)
    g.partition(p)
    g.count(opts)
    of = g.task_shards(S)
    per = []
    for sh in range(S):
        c = g.count_shard(sh, S, opts)
        info = g.info()
        per.append({"triangles": c, "tasks": int((of == sh).sum()), "t_count_ms": info["t_count_ms"],
                    "t_kernel_ms": info["t_kernel_ms"], "kernel_launches": info["kernel_launches"],
                    "h2d_bytes": info["h2d_bytes"]})
    t0 = []
    for _ in range(args.steps):
        g.count_shard(0, S, opts)
        t0.append(g.info()["t_count_ms"])
    block_bytes = g.info()["block_bytes"]
    g.close()
    ts = [x["t_count_ms"] for x in per]
    return {
        "num_shards": S,
        "deal": "tasks grouped by edge block, groups dealt heaviest first to the least loaded shard",
        "shard0_t_count_ms_p50": pct(t0, 50),
        "shard0_t_count_ms_min": min(t0),
        "shard0_h2d_bytes": per[0]["h2d_bytes"],
        "block_bytes": block_bytes,
        "max_shard_t_count_ms": max(ts),
        "max_over_mean_t_count": max(ts) / float(np.mean(ts)),
        "sum_equals_count": sum(x["triangles"] for x in per) == triangles,
        "per_shard": per,
    }


def copy_probe_gbs(mib=1024, reps=5):
    """Achievable HBM bandwidth on this GPU: the best of a few device copies
    (read + write bytes over time), beside the 8 TB/s published peak."""
    import torch
    nbytes = mib << 20
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return 2 * nbytes / (best / 1e3) / 1e9


def h2d_probe_gbs(mib=1024, reps=5):
    """Achievable host-to-device rate: the best of a few copies of a pinned
    host buffer to the device."""
    import torch
    nbytes = mib << 20
    h = torch.ones(nbytes, dtype=torch.uint8).pin_memory()
    dv = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        dv.copy_(h, non_blocking=True)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del h, dv
    return nbytes / (best / 1e3) / 1e9


def oracle_full_pass(n, s, d, m, label):
    def run():
        import oracle
        t0 = time.perf_counter()
        tri = oracle.tc(n, s, d)
        dt = time.perf_counter() - t0
        out = {"value": m / dt, "unit": "edges/s", "cores": oracle.threads(), "kind": "oracle",
               "sample": "one full oracle pass (clean, rank, orient, merge count) over %s, %.1f s"
                         % (label, dt)}
        # the merge count alone on one core and on all cores (same CSR)
        _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
        threads = oracle.threads()
        for t in (threads, 1):
            oracle.set_threads(t)
            t1 = time.perf_counter()
            oracle.count_csr(n, row_off, col)
            out["count_only_edges_per_s_%dcore" % t] = m / (time.perf_counter() - t1)
        oracle.set_threads(threads)
        return out, tri
    return run


def bench_block(args):
    from paper_2209_04541_amd import gen
    n, s, d = gen.rmat(args.scale, 16, gen.seed(2, 0))
    gold = "block" if args.scale == 20 else None
    m_est = golden("block")["m"] if args.scale == 20 else len(s)
    return run_graph(args, n, s, d, args.p or 8, gold,
                     "R-MAT scale %d, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed (2,0), "
                     "%dx%d blocks" % (args.scale, args.p or 8, args.p or 8),
                     "traffic_tc_block_rmat20_p8.json",
                     cpu_sample=oracle_full_pass(n, s, d, m_est, "the whole R-MAT scale-%d graph" % args.scale))


def bench_support(args):
    """Triangles of every edge on R-MAT scale 20: per step, build the
    oriented graph from device-resident edges and write each edge's count
    into a device array."""
    import numpy as np
    import torch

    import paper_2209_04541_amd as P
    from paper_2209_04541_amd import gen

    n, s, d = gen.block_graph()
    ds = torch.from_numpy(s).cuda()
    dd = torch.from_numpy(d).cuda()
    torch.cuda.synchronize()

    def step(keep=False):
        g = P.Graph(n, ds, dd)
        out = torch.empty(g.info()["m"], dtype=torch.int32, device="cuda")
        _, tri = g.edge_support(out)
        info = g.info()
        if keep:
            return g, out, tri, info
        g.close()
        return None, None, tri, info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    infos, tris, step_ms = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        _, _, tri, info = step()
        step_ms.append((time.perf_counter() - a) * 1e3)
        tris.append(tri)
        infos.append(info)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps

    g, out, tri, info = step(keep=True)
    row_off, col, _ = g.export_csr()
    sup = out.cpu().numpy().view(np.uint32)
    # per-vertex counts from the same graph (support pass + per-vertex sums)
    tv = torch.empty(n, dtype=torch.int64, device="cuda")
    _, tri_v = g.vertex_counts(tv)
    t_vertex_ms = g.info()["t_count_ms"]
    tv_sum = int(tv.sum().item())
    # k-truss by rounds of the support pass, for a few k
    truss = {}
    for k in (4, 8, 16, 32):
        _, left, rounds = g.ktruss(k)
        inf = g.info()
        truss[str(k)] = {"edges": left, "rounds": rounds, "t_ms": inf["t_count_ms"],
                         "t_kernels_ms": inf["t_kernel_ms"]}
    c4 = g.four_cliques()  # one block (p = 1)
    inf = g.info()
    cliques = {"four_cliques": c4, "t_ms": inf["t_count_ms"], "t_kernel_ms": inf["t_kernel_ms"]}
    g.partition(8)  # block 4-lists of the 8 x 8 grid
    c4_8 = g.four_cliques()
    inf = g.info()
    cliques["p8"] = {"four_cliques": c4_8, "t_ms": inf["t_count_ms"], "t_kernel_ms": inf["t_kernel_ms"],
                     "four_lists": len(g.four_clique_lists()[0])}
    # the same 4-lists with the blocks streamed from the host store through
    # a device cache of a quarter of the store
    cap = inf["block_bytes"] // 4
    c4_s = g.four_cliques(device_cap_bytes=cap)
    inf = g.info()
    cliques["p8_streamed"] = {"four_cliques": c4_s, "device_cap_bytes": cap, "t_ms": inf["t_count_ms"],
                              "t_kernel_ms": inf["t_kernel_ms"], "h2d_bytes": inf["h2d_bytes"],
                              "launches": inf["kernel_launches"]}
    g.close()
    m = info["m"]
    T = tri
    # walked entries: for every edge (a, b), the entries of N+(a) after b
    deg = np.diff(row_off).astype(np.int64)
    walked = int((deg * (deg - 1) // 2).sum())
    kernel_ms = float(np.mean([i["t_kernel_ms"] for i in infos]))
    # algorithmic bytes: walked entries (4 B each); per edge, as an in-edge
    # its CSR position and walk length (8 B) and as a staged entry its value
    # (4 B), and the read and write of its two counter flushes (16 B); per
    # triangle one atomic on the walked edge (8 B: read and write)
    alg = 4 * walked + 28 * m + 8 * T
    achieved = alg / (kernel_ms / 1e3) / 1e9
    gold = golden("block")
    out_line = base_line(args, m / (ms / 1e3), "edges/s", ms, {
        "workload": "edge support (triangles per edge), R-MAT scale 20, edge factor 16, "
                    "(a,b,c,d)=(.57,.19,.19,.05), seed (2,0)", "n": n, "m_input": len(s), "m": m})
    out_line["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": achieved / HBM_PEAK_GBS,
                            "traffic": measured_traffic("traffic_edge_support_rmat20.json", SUPPORT_SOURCES)}
    out_line.update({
        "triangles": T,
        "parity": all(t == gold["triangles"] for t in tris) and int(sup.sum(dtype=np.uint64)) == 3 * T,
        "step_ms_p50": pct(step_ms, 50), "step_ms_p99": pct(step_ms, 99),
        "t_build_ms": float(np.mean([i["t_build_ms"] for i in infos])),
        "t_support_ms": float(np.mean([i["t_count_ms"] for i in infos])),
        "t_kernel_ms": kernel_ms,
        "kernel_edges_per_s": m / (kernel_ms / 1e3),
        "walked_entries": walked,
        "algorithmic_bytes_per_launch": alg,
        "max_support": int(sup.max()) if m else 0,
        "t_vertex_counts_ms": t_vertex_ms,
        "ktruss": truss,
        "cliques": cliques,
    })
    out_line["parity"] = out_line["parity"] and tri_v == T and tv_sum == 3 * T and c4 == c4_8 == c4_s
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        _, _, _, ro, cl = oracle.oriented_csr(n, s, d)
        t_build = time.perf_counter() - t1
        t1 = time.perf_counter()
        want = oracle.edge_support(n, ro, cl)
        dt = time.perf_counter() - t1
        out_line["cpu_baseline"] = {
            "value": m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "the oracle's per-edge counts over the whole graph, sequential (%.1f s; its build "
                      "took %.1f s on %d threads)" % (dt, t_build, oracle.threads())}
        out_line["parity"] = out_line["parity"] and bool(np.array_equal(want, sup))
    return out_line


def bench_plain(args):
    from paper_2209_04541_amd import gen
    n, s, d = gen.plain_graph()
    return run_graph(args, n, s, d, 1, "plain", "ER G(n=4096, m=32768), seed (1,0), p=1",
                     "traffic_tc_plain.json",
                     cpu_sample=oracle_full_pass(n, s, d, 32768, "the whole ER graph"))


def bench_ooc(args):
    """R-MAT scale 24, 32x32 blocks streamed from pinned host memory under an
    8 GB device cap; the step includes the host-to-device block copies."""
    import paper_2209_04541_amd as P
    from paper_2209_04541_amd import gen
    n, s, d = gen.rmat(24, 16, gen.seed(3, 0))
    cap = args.cap_mb * (1 << 20) if args.cap_mb else int(args.cap_gb * 1e9)
    cap_label = "%d MiB" % args.cap_mb if args.cap_mb else "%g GB" % args.cap_gb
    opts = P.options(kernel=args.kernel, device_cap_bytes=int(cap), stream_blocks=True)

    def cpu_sample():
        # a bounded sample: the oracle's merge count over the rows of the top
        # 1/64 of the rank range (the densest rows), scaled to edges/s by the
        # oriented edges those rows own
        import numpy as np
        import oracle
        t0 = time.perf_counter()
        keys, deg, rk, row_off, col = oracle.oriented_csr(n, s, d)
        t_build = time.perf_counter() - t0
        rows = row_off.shape[0] - 1
        lo = rows - rows // 64
        off = np.zeros(rows + 1, np.int64)
        off[lo + 1:] = row_off[lo + 1:] - row_off[lo]
        t1 = time.perf_counter()
        # rows below lo are empty in this CSR; probed rows v >= lo are intact
        oracle.count_csr(rows, off, np.ascontiguousarray(col[row_off[lo]:]))
        dt = time.perf_counter() - t1
        m_rows = int(row_off[-1] - row_off[lo])
        return {"value": m_rows / dt, "unit": "edges/s", "cores": oracle.threads(), "kind": "oracle",
                "sample": "oracle merge count over the top 1/64 of the rank range (%d oriented edges, "
                          "%.1f s; the oracle's build of the whole graph took %.1f s)"
                          % (m_rows, dt, t_build)}, None

    out = run_graph(args, n, s, d, 32, "ooc",
                    "R-MAT scale 24, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed (3,0), 32x32 "
                    "blocks in pinned host memory, %s device cap" % cap_label,
                    "traffic_tc_ooc.json", opts=opts, cpu_sample=cpu_sample)
    # block copies against what a plain pinned copy reaches (the copies
    # overlap the counting launches, so this is a lower bound of their rate)
    out["h2d_probe_gbs"] = h2d_probe_gbs()
    out["h2d_gbs_over_count"] = out["h2d_bytes_per_step"] / (out["t_count_ms"] / 1e3) / 1e9
    return out


# ---------------------------------------------------------------- batch

def bench_batch(args):
    import numpy as np
    import torch

    import paper_2209_04541_amd as P
    from paper_2209_04541_amd import gen

    G = args.graphs
    t0 = time.perf_counter()
    nv = np.empty(G, np.int32)
    parts_s, parts_d = [], []
    for g in range(G):
        n, s, d = gen.batch_graph(g)
        nv[g] = n
        parts_s.append(s)
        parts_d.append(d)
    eoff = np.zeros(G + 1, np.int64)
    eoff[1:] = np.cumsum([len(x) for x in parts_s])
    src = np.concatenate(parts_s)
    dst = np.concatenate(parts_d)
    del parts_s, parts_d
    t_gen = time.perf_counter() - t0
    ds = torch.from_numpy(src).cuda()
    dd = torch.from_numpy(dst).cuda()
    torch.cuda.synchronize()
    b = P.Batch((nv, eoff, ds, dd))
    t_build = b.times()[0]
    t_tune0 = time.perf_counter()
    counts = b.count()  # autotune + capture on first use
    t_tune = time.perf_counter() - t_tune0
    for _ in range(args.warmup):
        b.count()
    rep_ms = []
    for _ in range(args.steps):
        c2 = b.count()
        rep_ms.append(b.times()[1])
        assert np.array_equal(c2, counts)
    per_ms = []
    for _ in range(0 if args.no_per_graph else max(1, args.steps // 5)):
        c3 = b.count(per_graph=True)
        per_ms.append(b.times()[1])
        assert np.array_equal(c3, counts)
    ms = float(np.median(rep_ms))
    pg = float(np.median(per_ms)) if per_ms else float("nan")
    mtot = int(eoff[-1])
    out = base_line(args, G / (ms / 1e3), "graphs/s", ms, {
        "workload": "%d graphs, seed (4,g): even g random geometric, odd g Erdos-Renyi, n ~ U{64..8192}, "
                    "average degree ~ U{8..64}; one persistent HIP-graph launch, autotuned" % G,
        "graphs": G, "pairs": mtot, "vertices": int(nv.sum())})
    out.update({
        "per_graph_launches_ms": pg if per_ms else None,
        "per_graph_launches_graphs_per_s": G / (pg / 1e3) if per_ms else None,
        "speedup_vs_per_graph": pg / ms if per_ms else None, "batched_build_ms": t_build,
        "end_to_end_graphs_per_s": G / ((t_build + ms) / 1e3), "autotune_s": t_tune,
        "generation_s": t_gen, "triangles_total": int(counts.sum()),
    })
    # roofline of the counting launch: every walked entry (4 B), per edge of
    # an active row its staged value, its id and the walked row's two
    # offsets (16 B), per active row its id, graph id and two offsets (16 B);
    # time = one replay of the captured launch (zeroing and the 8 B-per-graph
    # copy of the counts included)
    st = b.stats()
    alg = 4 * st["walked"] + 16 * st["active_edges"] + 16 * st["active_rows"]
    achieved = alg / (ms / 1e3) / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": measured_traffic("traffic_tc_batch_10k.json", BATCH_SOURCES)}
    out.update({"algorithmic_bytes_per_launch": alg, "walked_entries": st["walked"],
                "edges": st["edges"], "active_rows": st["active_rows"]})
    # parity: every graph's count against the oracle's stored count
    gold = [int(x) for x in open(os.path.join(ROOT, "tests", "golden", "batch_counts.txt"))
            if not x.startswith("#")]
    out["parity"] = G <= len(gold) and [int(c) for c in counts] == gold[:G]
    out["parity_checked_graphs"] = G if G <= len(gold) else 0
    if not args.no_cpu_baseline:
        import oracle
        sample = list(range(0, G, max(1, G // 200)))
        t1 = time.perf_counter()
        ok = True
        for g in sample:
            n, s, d = gen.batch_graph(g)
            ok = ok and oracle.tc(n, s, d) == int(counts[g])
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": len(sample) / dt, "unit": "graphs/s", "cores": oracle.threads(),
                               "kind": "oracle", "sample": "%d of the %d graphs (every %d-th), %.1f s"
                               % (len(sample), G, max(1, G // 200), dt)}
        out["parity"] = out["parity"] and ok
    b.close()
    return out


# ---------------------------------------------------------------- served

def bench_served(args):
    """A Poisson request trace against the continuous-batching server and
    against plain sequential launches (one request at a time, build then
    count, with the grid the server would give it), on the same trace.  Requests arrive for `duration` seconds; an
    arrival that finds `max_outstanding` requests already waiting or running
    is shed (counted, not served), so an overloaded run measures capacity
    instead of an ever-growing queue.  Two traces: the configured rate, and
    `sustain_rate` (a load the sequential loop also keeps up with; 0 skips
    it).  Every served count is checked against the oracle's stored count of
    its pool graph."""
    import numpy as np
    import torch

    import paper_2209_04541_amd as P
    from paper_2209_04541_amd import gen

    torch.cuda.init()
    pool_size = args.pool
    pool = []
    print("served: generating the pool of %d graphs" % pool_size, file=sys.stderr, flush=True)
    for r in range(pool_size):
        sc, ef = gen.served_params(r)
        n, s, d = gen.served_graph(r)
        # pinned host copies so request uploads run at full link speed
        ps = torch.from_numpy(s).pin_memory().numpy()
        pd = torch.from_numpy(d).pin_memory().numpy()
        pool.append((n, ps, pd, sc, ef))
        if r % 16 == 15:
            print("served: %d pool graphs ready" % (r + 1), file=sys.stderr, flush=True)
    gold = golden("served") or {}
    K = args.max_outstanding

    def served_run(rate, duration):
        arrivals = gen.poisson_arrivals(rate, duration, gen.seed(5, 0))
        reqs = [i % pool_size for i in range(len(arrivals))]
        with P.Server(args.budget_gb << 30, borrow=True, num_streams=args.builders) as srv:
            clock0 = srv.now()
            t0 = time.perf_counter()
            outstanding = []  # (request index, ticket)
            tickets = {}
            shed = 0
            next_report = 5.0
            for i, a in enumerate(arrivals):
                now = time.perf_counter() - t0
                if now >= next_report:  # progress on stderr, a line every 5 s
                    print("served %.0f req/s: t=%.0f s, %d submitted, %d shed" % (rate, now, len(tickets), shed),
                          file=sys.stderr, flush=True)
                    next_report += 5.0
                if a > now:
                    time.sleep(a - now)
                if len(outstanding) >= K:
                    outstanding = [(j, t) for j, t in outstanding if not srv.poll(t)[0]]
                if len(outstanding) >= K:
                    shed += 1
                    continue
                n, s, d, _, _ = pool[reqs[i]]
                t = srv.submit(n, s, d)
                tickets[i] = t
                outstanding.append((i, t))
            srv.drain()
            kms, walked, edges = srv.kernel_stats()
            lat, ok, t_end = [], True, clock0
            for i, t in tickets.items():
                done, cnt, ts, td = srv.poll(t)
                lat.append((td - (clock0 + arrivals[i])) * 1e3)
                g = gold.get(str(reqs[i]))
                ok = ok and done and g is not None and cnt == g["triangles"]
                t_end = max(t_end, td)
            span = t_end - clock0
            launches = srv.launches()
        pairs = sum(len(pool[reqs[i]][1]) for i in tickets)
        return {"offered": len(arrivals), "served": len(tickets), "shed": shed, "span_s": span,
                "requests_per_s": len(tickets) / span, "input_pairs_per_s": pairs / span,
                "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "launches": launches, "exact": ok,
                "kernel_ms": kms, "walked_entries": walked, "edges_counted": edges}

    def sequential_run(rate, duration):
        arrivals = gen.poisson_arrivals(rate, duration, gen.seed(5, 0))
        reqs = [i % pool_size for i in range(len(arrivals))]
        t0 = time.perf_counter()
        queue, lat, served, shed, ok, nxt, pairs = [], [], 0, 0, True, 0, 0
        next_report = 5.0
        while nxt < len(arrivals) or queue:
            now = time.perf_counter() - t0
            if now >= next_report:
                print("sequential %.0f req/s: t=%.0f s, %d served, %d shed" % (rate, now, served, shed),
                      file=sys.stderr, flush=True)
                next_report += 5.0
            # arrivals up to now join the queue unless it is full; nothing
            # left the queue since the last request started, so its length
            # at each arrival is the length now
            while nxt < len(arrivals) and arrivals[nxt] <= now:
                if len(queue) >= K:
                    shed += 1
                else:
                    queue.append(nxt)
                nxt += 1
            if not queue:
                time.sleep(max(0.0, arrivals[nxt] - now))
                continue
            i = queue.pop(0)
            n, s, d, _, _ = pool[reqs[i]]
            with P.Graph(n, s, d) as g:
                # the grid the server gives a request of this size
                g.partition(8 if len(s) >= (1 << 18) else 1)
                c = g.count()
            lat.append((time.perf_counter() - t0 - arrivals[i]) * 1e3)
            gg = gold.get(str(reqs[i]))
            ok = ok and gg is not None and c == gg["triangles"]
            served += 1
            pairs += len(s)
        span = time.perf_counter() - t0
        return {"offered": len(arrivals), "served": served, "shed": shed, "span_s": span,
                "requests_per_s": served / span, "input_pairs_per_s": pairs / span,
                "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "exact": ok}

    main = served_run(args.rate, args.duration)
    seq = sequential_run(args.rate, args.duration)
    out = base_line(args, main["requests_per_s"], "requests/s", main["span_s"] * 1e3 / max(1, main["served"]), {
        "workload": "Poisson arrivals at %.0f req/s for %.1f s; request r: R-MAT scale ~ U{10..22}, "
                    "edge factor ~ U{8..32}, seed (5,r mod %d); %d GiB device budget, %d builders; arrivals "
                    "finding %d requests outstanding are shed" % (args.rate, args.duration, pool_size,
                                                                 args.budget_gb, args.builders, K),
        "rate": args.rate, "duration_s": args.duration, "pool": pool_size, "max_outstanding": K,
        "request_grid": "8x8 blocks from 2^18 input pairs, else one block (server and sequential alike)"})
    # a step of this line is one served request of the trace: ms_per_step is
    # the trace's span over the requests served, with no warmup
    out["steps"] = main["served"]
    out["warmup"] = 0
    out["step"] = "one served request"
    # roofline of the server's counting launches over the run: algorithmic
    # bytes (4 per walked entry, 16 per edge, as for one count) over their
    # summed device time
    if main["kernel_ms"] > 0:
        alg = 4 * main["walked_entries"] + 16 * main["edges_counted"]
        ach = alg / (main["kernel_ms"] / 1e3) / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": None}
    out.update({"p50_ms": main["p50_ms"], "p99_ms": main["p99_ms"], "server": main, "sequential": seq,
                "speedup_vs_sequential": main["requests_per_s"] / seq["requests_per_s"]})
    parity = main["exact"] and seq["exact"]
    if args.sustain_rate > 0:
        out["sustained"] = {"rate": args.sustain_rate, "duration_s": args.duration,
                            "server": served_run(args.sustain_rate, args.duration),
                            "sequential": sequential_run(args.sustain_rate, args.duration)}
        parity = parity and out["sustained"]["server"]["exact"] and out["sustained"]["sequential"]["exact"]
    out["parity"] = parity
    if not args.no_cpu_baseline:
        import oracle
        small = [i for i in range(pool_size) if pool[i][3] <= 16][:8]
        t1 = time.perf_counter()
        ok = True
        for i in small:
            n, s, d, _, _ = pool[i]
            ok = ok and oracle.tc(n, s, d) == gold[str(i)]["triangles"]
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": len(small) / dt if dt > 0 else None, "unit": "requests/s",
                               "cores": oracle.threads(), "kind": "oracle",
                               "sample": "%d pool requests of scale <= 16 counted by the oracle, %.1f s "
                                         "(larger requests take the oracle minutes each)" % (len(small), dt)}
        out["parity"] = out["parity"] and ok
    return out


def bench_bsp(args):
    """The single-block bulk-synchronous computations on the block
    workload's graph (R-MAT scale 20, edge factor 16, 8 x 8 blocks): one step
    is connected components (Shiloach-Vishkin) plus PageRank (damping 0.85,
    tolerance 1e-4, at most 20 iterations) over the partitioned graph, whose
    build and partition come before the timed region.  `value` is PageRank
    edge visits per second (m' edges per iteration over the iterations'
    time), the paper's per-iteration figure for bulk computations."""
    import numpy as np
    import torch

    import oracle
    import paper_2209_04541_amd as P
    from paper_2209_04541_amd import gen

    p = args.p or 8
    n, s, d = gen.block_graph()
    ds = torch.from_numpy(s).cuda()
    dd = torch.from_numpy(d).cuda()
    torch.cuda.synchronize()
    g = P.Graph(n, ds, dd)
    g.partition(p)
    info0 = g.info()
    m = info0["m"]

    def step():
        lab, nc, cit = g.components()
        ci = g.info()
        r, pit, err = g.pagerank()
        pi = g.info()
        return lab, nc, cit, ci, r, pit, err, pi

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    res, step_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        res.append(step())
        step_ms.append((time.perf_counter() - a) * 1e3)
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    lab, nc, cit, ci, r, pit, err, pi = res[-1]
    pr_ms = float(np.median([x[7]["t_count_ms"] for x in res]))
    pr_kernel_ms = float(np.median([x[7]["t_kernel_ms"] for x in res]))
    cc_ms = float(np.median([x[3]["t_count_ms"] for x in res]))
    cc_kernel_ms = float(np.median([x[3]["t_kernel_ms"] for x in res]))
    # algorithmic bytes of one PageRank iteration: each stored entry of every
    # block's rows and columns (2 m') reads its id (4 B) and its neighbour's
    # share (8 B); each item reads its record (12 B) and adds to one sum
    # (8 B read + 8 B write); each vertex reads its rank and two degrees and
    # writes its share and zeroed sum (32 B), then reads the sum and rank and
    # writes the new rank (24 B)
    items = info0["row_items"] + info0["col_items"]
    alg = 2 * m * 12 + items * 28 + n * 56
    per_iter_ms = pr_kernel_ms / max(1, pit)
    achieved = alg / (per_iter_ms / 1e3) / 1e9
    out = base_line(args, m * pit / (pr_ms / 1e3), "edges/s", ms, {
        "workload": "connected components + PageRank (d 0.85, tol 1e-4, <= 20 iterations) over R-MAT scale 20, "
                    "edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed (2,0), %dx%d blocks" % (p, p),
        "n": n, "m": m, "p": p}, dtype="int32+f64")
    out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    want_lab, want_nc = oracle.components(n, s, d)
    want_r, want_it, _ = oracle.pagerank(n, s, d)
    pr_ok = pit == want_it and bool(np.allclose(r, want_r, rtol=1e-10, atol=1e-15))
    cc_ok = nc == want_nc and bool(np.array_equal(lab, want_lab))
    out.update({
        "parity": pr_ok and cc_ok and all(x[1] == nc and x[5] == pit for x in res),
        "components": nc, "cc_iterations": cit, "cc_ms": cc_ms, "cc_kernel_ms": cc_kernel_ms,
        "cc_edges_per_s": m / (cc_ms / 1e3),
        "pagerank_iterations": pit, "pagerank_ms": pr_ms, "pagerank_kernel_ms": pr_kernel_ms,
        "pagerank_ms_per_iteration": pr_ms / max(1, pit), "pagerank_last_err": err,
        "pagerank_max_rel_diff_vs_oracle": float(np.max(np.abs(r - want_r) / np.maximum(want_r, 1e-300))),
        "algorithmic_bytes_per_pagerank_iteration": alg, "items": items,
        "step_ms_p50": pct(step_ms, 50), "step_ms_p99": pct(step_ms, 99),
    })
    if not args.no_cpu_baseline:
        t1 = time.perf_counter()
        _, it_cpu, _ = oracle.pagerank(n, s, d)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": m * it_cpu / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
                               "sample": "the oracle's PageRank over the whole graph, sequential, %d iterations "
                                         "including its adjacency build (%.1f s)" % (it_cpu, dt)}
    g.close()
    return out


def bench_copy(args):
    """A plain device-to-device copy of a known size: the reference that
    scales rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes."""
    import torch
    nbytes = args.copy_mib << 20
    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t = []
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        t.append(e0.elapsed_time(e1))
    ms = min(t)
    out = base_line(args, 2 * nbytes / (ms / 1e3) / 1e9, "GB/s", ms,
                    {"workload": "device copy of %d MiB (read %d MiB + write %d MiB)"
                                 % (args.copy_mib, args.copy_mib, args.copy_mib)})
    out["bytes_read_per_copy"] = nbytes
    out["bytes_written_per_copy"] = nbytes
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="block",
                    choices=["block", "plain", "ooc", "batch", "served", "support", "copy", "bsp"])
    ap.add_argument("--p", type=int, default=0)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--kernel", type=int, default=0)
    ap.add_argument("--cap-gb", type=float, default=8.0, help="device cap in GB (10^9 bytes)")
    ap.add_argument("--cap-mb", type=int, default=0, help="device cap in MiB (overrides --cap-gb)")
    ap.add_argument("--host-edges", action="store_true",
                    help="hand the edge list over in pinned host memory (its copy is then in the step)")
    ap.add_argument("--graphs", type=int, default=10000)
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--duration", type=float, default=60.0)
    ap.add_argument("--sustain-rate", type=float, default=40.0,
                    help="served: also run the trace at this rate (0 = skip)")
    ap.add_argument("--max-outstanding", type=int, default=64,
                    help="served: arrivals finding this many requests outstanding are shed")
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--budget-gb", type=int, default=64)
    ap.add_argument("--builders", type=int, default=2)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hybrid", action="store_true", help="skip the hybrid host + device comparison")
    ap.add_argument("--no-per-graph", action="store_true",
                    help="batch: skip the per-graph launches baseline (10,000 launches; for profiler runs)")
    ap.add_argument("--shards", type=int, default=0,
                    help="block and ooc workloads: also count each of this many task shards "
                         "(one device's share of a count split over that many devices)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    fn = {"block": bench_block, "plain": bench_plain, "ooc": bench_ooc, "batch": bench_batch,
          "served": bench_served, "support": bench_support, "copy": bench_copy, "bsp": bench_bsp}[args.workload]
    out = fn(args)
    if "cpu_baseline" in out:
        out["cpu_baseline"].update(cpu_model())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
