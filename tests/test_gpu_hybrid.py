"""GPU parity of the hybrid host + device count (heavy block-lists on the
device, light ones by the library's host kernel on host threads), of the
merged count of several graph objects, and of counts that partition from
their options.  Every per-task count is compared with the oracle's per-triple
count under the same cut vector."""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2209_04541_amd as P
from paper_2209_04541_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_tasks(g, n):
    row_off, col, _ = g.export_csr()
    B = oracle.block_counts(n, row_off, col, g.cuts())
    ijk, cnt = g.task_counts()
    for (i, j, k), c in zip(ijk, cnt):
        assert c == B[i, j, k], (i, j, k, c, B[i, j, k])
    return int(B.sum())


@pytest.mark.parametrize("permille", [0, 1, 250, 900, 1000])
def test_hybrid_per_task_counts(permille):
    n, s, d = gen.rmat(15, 16, gen.seed(97, 3))
    with P.Graph(n, s, d) as g:
        g.partition(8)
        T = g.info()["num_tasks"]
        got = g.count(hybrid=True, host_permille=permille, host_threads=4)
        info = g.info()
        say("hybrid", permille, got, "host tasks", info["host_tasks"], "of", T,
            "share", round(info["host_work_share"], 3), "launches", info["kernel_launches"])
        assert got == check_tasks(g, n)
        if permille == 1000:
            assert info["host_tasks"] == T and info["kernel_launches"] == 0
            assert abs(info["host_work_share"] - 1.0) < 1e-9
        elif permille > 0:
            assert info["host_work_share"] <= permille / 1000 + 1e-9
        assert 0 <= info["host_tasks"] <= T


@pytest.mark.parametrize("cap_frac", [0.4, 2.0])
def test_hybrid_streamed_under_cap(cap_frac):
    """Hybrid with the blocks already in the host store, under a cap that
    evicts (0.4 of the blocks) and one that holds them all."""
    n, s, d = gen.rmat(14, 16, gen.seed(97, 4))
    want = oracle.tc(n, s, d)
    with P.Graph(n, s, d) as g:
        g.partition(12)
        total = g.info()["block_bytes"]
        assert g.count(stream_blocks=True) == want
        for permille in (0, 500):
            got = g.count(hybrid=True, host_permille=permille, device_cap_bytes=int(total * cap_frac),
                          num_streams=3)
            assert got == want
            assert got == check_tasks(g, n)


def test_hybrid_degenerate_graphs():
    for (n, s, d), want in [graphs.complete(3), graphs.complete(60), graphs.wheel(40), graphs.star(9),
                            graphs.complete_bipartite(7, 9)]:
        with P.Graph(n, s, d) as g:
            g.partition(3)
            for permille in (0, 1000):
                assert g.count(hybrid=True, host_permille=permille) == want


def test_count_graphs_merged_launch():
    """pgabb_tc_count_batch: graphs with different p share one launch
    (autotuned without options); a graph whose blocks sit in the host store is
    counted on its own; per-graph task counts equal the oracle's."""
    gl = [gen.rmat(12, 8, gen.seed(96, k)) for k in range(3)] + [gen.er(700, 9000, gen.seed(96, 7)),
                                                                 graphs.complete(90)[0]]
    want = [oracle.tc(*x) for x in gl]
    objs = [P.Graph(*x) for x in gl]
    try:
        objs[0].partition(4)
        objs[1].partition(7)
        objs[3].partition(2)
        objs[4].count(stream_blocks=True)  # its blocks now live in the host store
        for rep in range(2):  # the second call finds the shape in the tuning cache
            assert P.tc_count_batch(objs) == want, rep
            for g, x in zip(objs, gl):
                assert check_tasks(g, x[0]) == oracle.tc(*x)
        assert P.tc_count_batch(objs, waves_per_block=8, rows_per_grab=3, by_rows=True) == want
        # options with p re-partition every graph first
        assert P.tc_count_batch(objs, p=5, cut_mode=P.CUT_UNIFORM) == want
        assert all(g.info()["p"] == 5 for g in objs)
        path = os.environ.get("PGABB_TUNE_CACHE")
        if path:
            with open(path) as f:
                assert "tc_graphs/" in f.read()
    finally:
        for g in objs:
            g.close()


def test_count_partitions_from_options():
    n, s, d = gen.rmat(13, 16, gen.seed(96, 9))
    want = oracle.tc(n, s, d)
    with P.Graph(n, s, d) as g:
        assert g.count(p=6) == want
        assert g.info()["p"] == 6
        assert g.count(p=6, cut_mode=P.CUT_UNIFORM) == want
        c = g.cuts()
        assert list(c) == [i * n // 6 for i in range(7)]
        g.partition(3)
        assert g.count() == want and g.info()["p"] == 3  # p = 0 keeps the partition
        assert check_tasks(g, n) == want
