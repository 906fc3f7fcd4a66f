"""Writes workload_counts.json: the oracle's triangle counts and sizes for the
seeded workloads.  Calls only the CPU oracle (and the shared input
generators); run from the repository root:

    python tests/golden/make_golden.py [plain block ooc served]
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


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        if name == "served":
            # one oracle count per request graph of the first 64 requests
            out = {}
            for r in range(64):
                sc, ef = gen.served_params(r)
                if sc > 18:
                    continue
                n, s, d = gen.served_graph(r)
                out[str(r)] = {"scale": sc, "edge_factor": ef, "triangles": oracle.tc(n, s, d)}
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
