"""GPU tests of the autotuners: the grid (p and cut mode) chosen per shape
class for a count of several graph objects, a grid taken from the
persisted tuning cache, and the batch's launch shape kept in that cache.
Every count is compared with the oracle, per graph and per task."""
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2209_04541_amd as P
from paper_2209_04541_amd import gen

pytestmark = pytest.mark.gpu

GRIDS = {(1, P.CUT_NNZ), (2, P.CUT_NNZ), (4, P.CUT_NNZ), (8, P.CUT_NNZ), (16, P.CUT_NNZ), (8, P.CUT_UNIFORM)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bits(x):
    return int(x).bit_length()


def check_tasks(g, n):
    row_off, col, _ = g.export_csr()
    B = oracle.block_counts(n, row_off, col, g.cuts())
    ijk, cnt = g.task_counts()
    for (i, j, k), c in zip(ijk, cnt):
        assert c == B[i, j, k], (i, j, k)
    return int(B.sum())


def grid_of(g, n):
    """(p, cut mode) of a graph's partition, the mode read from its cuts."""
    p = g.info()["p"]
    cuts = list(g.cuts())
    uniform = cuts == [i * n // p for i in range(p + 1)]
    return p, (P.CUT_UNIFORM if uniform and p > 1 else P.CUT_NNZ)


def test_grid_tuned_per_class():
    """Two shape classes (Erdos-Renyi graphs of 3,001 vertices and R-MAT
    scale-16 graphs): each class gets one grid from the candidates, the
    counts and per-task counts equal the oracle's, the choice is stored and
    a second call finds it in the cache."""
    ers = [gen.er(3001, 45000, gen.seed(980, k)) for k in range(4)]
    rms = [gen.rmat(16, 12, gen.seed(981, k)) for k in range(2)]
    gl = ers + rms
    want = [oracle.tc(*x) for x in gl]
    objs = [P.Graph(*x) for x in gl]
    try:
        got = P.tc_count_batch(objs)
        assert got == want
        t1 = objs[0].info()["t_tune_ms"]
        grids = [grid_of(g, x[0]) for g, x in zip(objs, gl)]
        say("grids", grids, "tune ms", t1)
        for g, x in zip(objs, gl):
            assert check_tasks(g, x[0]) == oracle.tc(*x)
        classes = {}
        for g, gr in zip(objs, grids):
            inf = g.info()
            classes.setdefault((bits(inf["m"]), bits(inf["max_out_degree"])), set()).add(gr)
        for cl, gs in classes.items():
            assert len(gs) == 1, cl  # one grid per class
            assert gs <= GRIDS
        path = os.environ.get("PGABB_TUNE_CACHE")
        if path:
            with open(path) as f:
                text = f.read()
            assert "tc_graphs_grid/" in text and "tc_graphs/" in text
        assert P.tc_count_batch(objs) == want
        assert [grid_of(g, x[0]) for g, x in zip(objs, gl)] == grids
        t2 = objs[0].info()["t_tune_ms"]
        say("tune ms again", t2)
        assert t2 < t1
    finally:
        for g in objs:
            g.close()


@pytest.mark.parametrize("grid", [(4, P.CUT_UNIFORM), (8, P.CUT_NNZ)])
def test_grid_from_cache_file(grid):
    """A grid with p > 1 written into the tuning cache file for the class of
    these graphs is the one the tuned count partitions with; counts and
    per-task counts equal the oracle's."""
    path = os.environ.get("PGABB_TUNE_CACHE")
    if not path:
        pytest.skip("no tuning cache file in this process")
    gl = [gen.rmat(14, 9, gen.seed(982, k)) for k in range(3)]
    want = [oracle.tc(*x) for x in gl]
    objs = [P.Graph(*x) for x in gl]
    try:
        keys = set()
        for g in objs:
            inf = g.info()
            keys.add("tc_graphs_grid/M%d/D%d" % (bits(inf["m"]), bits(inf["max_out_degree"])))
        with open(path, "a") as f:
            for k in keys:
                f.write("%s %d %d\n" % (k, grid[0], grid[1]))
        assert P.lib().pgabb_tune_cache_reload() == P.OK
        assert P.tc_count_batch(objs) == want
        for g, x in zip(objs, gl):
            assert grid_of(g, x[0]) == grid
            assert check_tasks(g, x[0]) == oracle.tc(*x)
    finally:
        for g in objs:
            g.close()


def test_batch_launch_shape_persisted():
    """The batch's autotuned launch shape is stored in the tuning cache and
    found there by the next batch of the same shape class."""
    gl = [gen.batch_graph(g) for g in range(40)]
    want = np.array([oracle.tc(*x) for x in gl], np.uint64)
    with P.Batch(gl) as b:
        assert np.array_equal(b.count(), want)
        sh = b.launch_shape()
        say("batch shape", sh)
        assert sh["kernel"] in (P.KERNEL_BITMAP, P.KERNEL_HASH)
        assert sh["waves_per_block"] in (2, 4, 8) and sh["rows_per_grab"] >= 1
        t_first = sh["t_tune_ms"]
    path = os.environ.get("PGABB_TUNE_CACHE")
    if path:
        with open(path) as f:
            assert "batch/" in f.read()
    with P.Batch(gl) as b:
        assert np.array_equal(b.count(), want)
        sh2 = b.launch_shape()
        assert (sh2["kernel"], sh2["waves_per_block"], sh2["rows_per_grab"]) == \
            (sh["kernel"], sh["waves_per_block"], sh["rows_per_grab"])
        assert sh2["t_tune_ms"] < t_first
