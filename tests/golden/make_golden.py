"""Writes workload_counts.json: the oracle's triangle counts and sizes for the
seeded workloads, and batch_counts.txt: the oracle's count of every graph of
the 10,000-graph batch (one line per graph, in graph order).  Calls only the
CPU oracle (and the shared input generators); run from the repository root:

    python tests/golden/make_golden.py [plain block ooc served batch]
"""
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import oracle  # noqa: E402
from paper_2209_04541_amd import gen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workload_counts.json")
BATCH_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_counts.txt")
BATCH_GRAPHS = 10000

WORKLOADS = {
    "plain": ("ER G(n=4096, m=32768), seed (1, 0)", gen.plain_graph),
    "block": ("R-MAT scale 20, edge factor 16, (.57,.19,.19,.05), seed (2, 0)", gen.block_graph),
    "ooc": ("R-MAT scale 24, edge factor 16, (.57,.19,.19,.05), seed (3, 0)", gen.ooc_graph),
}


def record(n, s, d):
    t0 = time.time()
    keys, deg, rk, row_off, col = oracle.oriented_csr(n, s, d)
    t1 = time.time()
    t = oracle.count_csr(n, row_off, col)
    t2 = time.time()
    od = np.diff(row_off)
    extra = {}
    if len(col) < 10 ** 8:  # the pair-by-pair definition is quadratic per row
        extra["probe_work_col_p1"] = oracle.probe_work_col(n, row_off, col, [0, n])
    return {
        **extra,
        "n": int(n),
        "m_input": int(len(s)),
        "m": int(len(keys)),
        "isolated": int((deg == 0).sum()),
        "max_out_degree": int(od.max()) if len(od) else 0,
        "probe_work": oracle.probe_work(n, row_off, col),
        "triangles": int(t),
        "oracle_build_s": round(t1 - t0, 2),
        "oracle_count_s": round(t2 - t1, 2),
        "oracle_threads": oracle.threads(),
    }


def _batch_one(g):
    return oracle.tc(*gen.batch_graph(g))


def batch_counts():
    """Oracle count of every batch graph, written one per line."""
    from multiprocessing import Pool
    oracle.set_threads(1)
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        counts = pool.map(_batch_one, range(BATCH_GRAPHS), chunksize=50)
    with open(BATCH_OUT, "w") as f:
        f.write("# oracle triangle count of batch graph g (seed (4, g)), line g\n")
        for c in counts:
            f.write("%d\n" % c)
    print("batch", len(counts), "graphs", sum(counts), "triangles", flush=True)


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        if name == "batch":
            batch_counts()
            continue
        if name == "served":
            # one oracle count per graph of the request pool (requests
            # r = 0 .. 63; the served trace draws its graphs from this pool)
            out = data.get("served", {})
            for r in range(64):
                sc, ef = gen.served_params(r)
                if str(r) in out and out[str(r)].get("scale") == sc:
                    continue
                n, s, d = gen.served_graph(r)
                out[str(r)] = {"scale": sc, "edge_factor": ef, "triangles": oracle.tc(n, s, d),
                               "m_input": int(len(s))}
                del s, d
                print("served", r, out[str(r)], flush=True)
                data["served"] = out
                with open(OUT, "w") as f:
                    json.dump(data, f, indent=1, sort_keys=True)
            data["served"] = out
            continue
        desc, fn = WORKLOADS[name]
        n, s, d = fn()
        rec = record(n, s, d)
        rec["workload"] = desc
        data[name] = rec
        print(name, rec, flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["plain", "block"])
