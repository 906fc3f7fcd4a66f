"""GPU parity of the graph path (build, partition, count) against the CPU
oracle, through the C ABI.  Counts are integers: the bar is exact equality.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import paper_2209_04541_amd as P
from paper_2209_04541_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")



def walk_bytes(info):
    """Bytes of the blocks' parts the last count's walk reads (each copied at
    least once by a streamed count of every task)."""
    return info["walk_bytes_cols"] if info["walked_columns"] else info["walk_bytes_rows"]

def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_count(n, s, d, p=1, **kw):
    with P.Graph(n, s, d) as g:
        g.partition(p, cut_mode=kw.pop("cut_mode", P.CUT_NNZ), cuts=kw.pop("cuts", None))
        return g.count(**kw) if kw else g.count()


@pytest.mark.parametrize("name,g,expected", graphs.closed_forms(), ids=lambda x: x if isinstance(x, str) else "")
def test_closed_forms(name, g, expected):
    n, s, d = g
    say("closed form", name, n, len(s))
    for p in (1, 2, 3):
        if p > max(n, 1):
            continue
        assert gpu_count(n, s, d, p) == expected, (name, p)
    n2, s2, d2 = graphs.messy(n, s, d, seed=7)
    assert gpu_count(n2, s2, d2, 2) == expected


@pytest.mark.parametrize("seed", range(12))
def test_random_small_vs_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 70))
    m = int(rng.integers(0, 4 * n * n // 3 + 1))
    s = rng.integers(0, n, size=m).astype(np.int32)
    d = rng.integers(0, n, size=m).astype(np.int32)
    want = graphs.brute_force(n, s, d)
    say("random", seed, n, m, want)
    for p in (1, 2, 5):
        if p <= n:
            assert gpu_count(n, s, d, p) == want
    assert gpu_count(n, s, d, min(4, n), cut_mode=P.CUT_UNIFORM) == want


@pytest.mark.parametrize("order_by_id", [False, True])
def test_csr_bit_identical_to_oracle(order_by_id):
    n, s, d = graphs.messy(*gen.rmat(13, 16, gen.seed(94, 0)), seed=5)
    say("csr", n, len(s), order_by_id)
    keys, deg, rk, row_off, col = oracle.oriented_csr(n, s, d, mode=1 if order_by_id else 0)
    with P.Graph(n, s, d, order_by_id=order_by_id) as g:
        r2, c2, k2 = g.export_csr()
        info = g.info()
    assert np.array_equal(r2, row_off)
    assert np.array_equal(c2, col)
    assert np.array_equal(k2, rk)
    assert info["m"] == len(keys)
    assert info["isolated"] == int((deg == 0).sum())
    assert info["max_out_degree"] == int(np.diff(row_off).max())
    assert info["probe_work"] == oracle.probe_work(n, row_off, col)


@pytest.mark.parametrize("p", [2, 3, 5, 8, 13, 33, 64])
def test_task_counts_equal_oracle_blocks(p):
    n, s, d = gen.rmat(12, 12, gen.seed(95, p))
    _, _, rk, row_off, col = oracle.oriented_csr(n, s, d)
    say("tasks", p, n, len(s))
    for mode in (P.CUT_NNZ, P.CUT_UNIFORM):
        with P.Graph(n, s, d) as g:
            g.partition(p, cut_mode=mode)
            total = g.count()
            cuts = g.cuts()
            ijk, cnt = g.task_counts()
            walk = g.info()["probe_work_col"]
        B = oracle.block_counts(n, row_off, col, cuts)
        assert walk == oracle.probe_work_col(n, row_off, col, cuts), (p, mode)
        got = np.zeros_like(B)
        for (i, j, k), c in zip(ijk, cnt):
            got[i, j, k] += c
        assert np.array_equal(got, B), (p, mode)
        assert total == int(B.sum())


def test_explicit_cuts_with_empty_stripes():
    n, s, d = gen.rmat(11, 16, gen.seed(96, 0))
    want = oracle.tc(n, s, d)
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    cuts = np.array([0, 0, 700, 700, 1500, n, n], np.int32)
    with P.Graph(n, s, d) as g:
        g.partition(len(cuts) - 1, cuts=cuts)
        assert g.count() == want
        ijk, cnt = g.task_counts()
        assert g.info()["probe_work_col"] == oracle.probe_work_col(n, row_off, col, cuts)
    B = oracle.block_counts(n, row_off, col, cuts)
    got = np.zeros_like(B)
    for (i, j, k), c in zip(ijk, cnt):
        got[i, j, k] += c
    assert np.array_equal(got, B)


@pytest.mark.parametrize("kernel", [P.KERNEL_HASH, P.KERNEL_BITMAP, P.KERNEL_SEARCH])
@pytest.mark.parametrize("waves", [2, 4, 8])
@pytest.mark.parametrize("by_rows", [False, True])
def test_forced_kernels_agree(kernel, waves, by_rows):
    n, s, d = gen.rgg(6000, 40, gen.seed(97, 0))
    want = oracle.tc(n, s, d)
    say("kernel", kernel, waves, by_rows, want)
    for p in (1, 4):
        for unroll in (1, 8):
            assert gpu_count(n, s, d, p, kernel=kernel, waves_per_block=waves, rows_per_grab=3,
                             unroll=unroll, by_rows=by_rows) == want


@pytest.mark.parametrize("by_rows", [False, True])
def test_orientations_task_counts(by_rows):
    """Row- and column-walked edge blocks find the same triangles per task."""
    n, s, d = gen.rmat(12, 16, gen.seed(95, 77))
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    with P.Graph(n, s, d) as g:
        g.partition(6)
        total = g.count(by_rows=by_rows)
        assert g.info()["walked_columns"] == (0 if by_rows else 1)
        cuts = g.cuts()
        ijk, cnt = g.task_counts()
    B = oracle.block_counts(n, row_off, col, cuts)
    got = np.zeros_like(B)
    for (i, j, k), c in zip(ijk, cnt):
        got[i, j, k] += c
    assert np.array_equal(got, B)
    assert total == int(B.sum())


def test_device_edges_torch_stream():
    import torch
    n, s, d = gen.rmat(14, 16, gen.seed(98, 0))
    want = oracle.tc(n, s, d)
    ds = torch.from_numpy(s).cuda()
    dd = torch.from_numpy(d).cuda()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        with P.Graph(n, ds, dd) as g:
            g.partition(4)
            assert g.count() == want
    torch.cuda.synchronize()


def test_device_ids_out_of_range():
    import torch
    ds = torch.tensor([0, 1, 9], dtype=torch.int32, device="cuda")
    dd = torch.tensor([1, 2, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(P.PgabbError) as ei:
        P.Graph(5, ds, dd)
    assert ei.value.status == P.EINVAL


def test_degenerate_graphs():
    z = np.zeros(0, np.int32)
    assert gpu_count(0, z, z, 1) == 0
    assert gpu_count(1, z, z, 1) == 0
    assert gpu_count(7, z, z, 3) == 0
    loops = np.arange(5, dtype=np.int32)
    assert gpu_count(5, loops, loops, 2) == 0
    assert gpu_count(2, np.array([0], np.int32), np.array([1], np.int32), 2) == 0
    tri_s = np.array([0, 1, 2, 2, 1], np.int32)
    tri_d = np.array([1, 2, 0, 0, 1], np.int32)
    assert gpu_count(3, tri_s, tri_d, 1) == 1
    assert gpu_count(3, tri_s, tri_d, 3) == 1
    # p larger than the number of non-isolated vertices, and the maximum p
    n, s, d = graphs.complete(9)[0]
    assert gpu_count(200, s, d, 64) == 84
    with P.Graph(200, s, d) as g:
        with pytest.raises(P.PgabbError):
            g.partition(65)
        with pytest.raises(P.PgabbError):
            g.partition(0)
    # count before partition means p = 1
    with P.Graph(n, s, d) as g:
        assert g.count() == 84
        assert g.info()["p"] == 1


@pytest.mark.parametrize("cap_kib", [0, 64, 256, 4096])
def test_streamed_blocks_under_caps(cap_kib):
    n, s, d = gen.rmat(14, 16, gen.seed(99, 0))
    want = oracle.tc(n, s, d)
    say("stream cap KiB", cap_kib, want)
    with P.Graph(n, s, d) as g:
        g.partition(8)
        info0 = g.info()
        try:
            got = g.count(device_cap_bytes=cap_kib * 1024, stream_blocks=True, num_streams=3)
        except P.PgabbError as e:
            # a cap below one task's three blocks is refused, never miscounted
            assert e.status == P.ENOMEM and cap_kib * 1024 < info0["block_bytes"]
            return
        info = g.info()
        assert got == want
        assert info["h2d_bytes"] >= walk_bytes(info) * 0.99
        # counting again from the host store gives the same answer
        assert g.count(device_cap_bytes=cap_kib * 1024) == want


def test_plain_workload():
    with open(os.path.join(GOLDEN, "workload_counts.json")) as f:
        gold = json.load(f)["plain"]
    n, s, d = gen.plain_graph()
    with P.Graph(n, s, d) as g:
        g.partition(1)
        assert g.count() == gold["triangles"]
        info = g.info()
    assert info["m"] == gold["m"] and info["probe_work"] == gold["probe_work"]
    assert info["probe_work_col"] == gold["probe_work_col_p1"]
    # row walks read fewer entries on this graph, so the default takes them
    assert gold["probe_work"] < gold["probe_work_col_p1"] and info["walked_columns"] == 0


@pytest.mark.parametrize("p", [1, 8])
def test_block_workload(p):
    with open(os.path.join(GOLDEN, "workload_counts.json")) as f:
        gold = json.load(f)["block"]
    n, s, d = gen.block_graph()
    say("block workload p", p)
    with P.Graph(n, s, d) as g:
        g.partition(p)
        assert g.count() == gold["triangles"]
        info = g.info()
    for k in ("m", "isolated", "max_out_degree", "probe_work"):
        assert info[k] == gold[k], k
    if p == 1:  # one stripe: the sum of squared out-degrees
        assert info["probe_work_col"] == gold["probe_work_col_p1"]
    assert info["walked_columns"] == (1 if info["probe_work_col"] <= info["probe_work"] else 0)


def test_cached_blocks_across_streams():
    """Freed blocks are reused by later graphs on other streams (the reuse
    waits for the free's event); releasing the cache between graphs changes
    nothing."""
    import torch
    n, s, d = gen.rmat(13, 16, gen.seed(98, 1))
    want = oracle.tc(n, s, d)
    streams = [torch.cuda.Stream() for _ in range(3)]
    for rep in range(6):
        with torch.cuda.stream(streams[rep % 3]):
            ds = torch.from_numpy(s).cuda()
            dd = torch.from_numpy(d).cuda()
            with P.Graph(n, ds, dd) as g:
                g.partition(1 + rep)
                assert g.count() == want, rep
        if rep == 3:
            P.release_cached_memory()
    torch.cuda.synchronize()


@pytest.mark.parametrize("n,parts", [(1100, 2), (1500, 3)])
def test_long_staged_lists_split_launch(n, parts):
    """Staged lists longer than the 1280-word region's hash table holds go to
    further launches, one per larger LDS class (rows up to 1099 entries: two
    launches; up to 1499: three).  On K_n (ranks follow ids, so row x holds
    x+1 .. n-1) the total is C(n, 3) and task (i, j, k) counts the triples
    a < b < c with a, b, c in stripes i, j, k; in core and streamed, for
    every staging kind and both walks."""
    s, d = np.triu_indices(n, 1)
    s, d = s.astype(np.int32), d.astype(np.int32)
    want = math.comb(n, 3)
    for p in (1, 3):
        with P.Graph(n, s, d) as g:
            g.partition(p)
            cuts = np.asarray(g.cuts(), dtype=np.int64)
            size = np.diff(cuts)
            B = np.zeros((p, p, p), dtype=np.int64)
            for i in range(p):
                for j in range(i, p):
                    for k in range(j, p):
                        if i == j == k:
                            B[i, j, k] = math.comb(int(size[i]), 3)
                        elif i == j:
                            B[i, j, k] = math.comb(int(size[i]), 2) * size[k]
                        elif j == k:
                            B[i, j, k] = size[i] * math.comb(int(size[j]), 2)
                        else:
                            B[i, j, k] = size[i] * size[j] * size[k]
            assert B.sum() == want
            for kernel in (P.KERNEL_AUTO, P.KERNEL_HASH, P.KERNEL_SEARCH):
                for by_rows in (False, True):
                    say("split", p, kernel, by_rows)
                    assert g.count(kernel=int(kernel), by_rows=by_rows) == want
                    ijk, cnt = g.task_counts()
                    got = np.zeros_like(B)
                    for (i, j, k), c in zip(ijk, cnt):
                        got[i, j, k] += c
                    assert np.array_equal(got, B)
                    if p == 1 and kernel != P.KERNEL_SEARCH:
                        assert g.info()["kernel_launches"] == parts
            assert g.count() == want
            info = g.info()
            assert g.count(stream_blocks=True, device_cap_bytes=info["block_bytes"] + (1 << 20)) == want
            # one window, split as the in-core launch
            assert g.info()["kernel_launches"] == info["kernel_launches"]
            assert g.info()["h2d_bytes"] >= walk_bytes(g.info())


def test_count_several_graph_objects_and_sizes():
    gl = [gen.rmat(11, 8, gen.seed(99, k)) for k in range(3)] + [gen.er(500, 3000, gen.seed(99, 9))]
    want = [oracle.tc(*x) for x in gl]
    objs = [P.Graph(*x) for x in gl]
    try:
        objs[1].partition(4)
        assert P.tc_count_batch(objs) == want  # no options: the grid is tuned too
        objs[1].partition(4)
        # options with p = 0 keep each graph's partition
        assert P.tc_count_batch(objs, kernel=int(P.KERNEL_HASH), by_rows=True) == want
        assert P.tc_count_batch([]) == []
        for g, x in zip(objs, gl):
            info = g.info()
            assert P.graph_info(g) == (info["n"], info["m"], info["p"], info["num_tasks"])
        assert P.graph_info(objs[1])[2] == 4
    finally:
        for g in objs:
            g.close()


@pytest.mark.parametrize("n,p", [(1500, 3), (0, 6)])
def test_streamed_under_small_caps(n, p):
    """Caps below the blocks' total: blocks are evicted and reloaded and the
    tasks run in the cache-locality order; counts stay exact, per task too
    (K_1500 also splits its launches by staged list length)."""
    if n:
        s, d = np.triu_indices(n, 1)
        s, d = s.astype(np.int32), d.astype(np.int32)
        want = math.comb(n, 3)
    else:
        n, s, d = gen.rmat(13, 16, gen.seed(95, 11))
        want = oracle.tc(n, s, d)
    with P.Graph(n, s, d) as g:
        g.partition(p)
        assert g.count() == want
        ijk0, cnt0 = g.task_counts()
        total = g.info()["block_bytes"]
        ran = 0
        for frac in (0.35, 0.6, 0.85):
            cap = int(total * frac)
            try:
                got = g.count(stream_blocks=True, device_cap_bytes=cap)
            except P.PgabbError as e:
                assert e.status == P.ENOMEM  # a task's three blocks exceed the cap
                continue
            ran += 1
            say("small cap", n, p, frac, got)
            assert got == want
            ijk, cnt = g.task_counts()
            assert sorted(zip(map(tuple, ijk), cnt)) == sorted(zip(map(tuple, ijk0), cnt0))
            assert g.info()["h2d_bytes"] >= walk_bytes(g.info())
        assert ran >= 1


@pytest.mark.parametrize("streams", [2, 3, 4])
def test_streamed_eviction_with_windows_in_flight(streams):
    """Caps that hold a small share of the blocks, with several compute
    streams: windows on different streams read the same blocks, so a block
    is evicted while an earlier window on another stream may still read it
    unless every stream's last reader is awaited.  Per-task counts equal the
    oracle's per-triple counts."""
    n, s, d = gen.rmat(15, 16, gen.seed(95, 21))
    with P.Graph(n, s, d) as g:
        g.partition(12)
        cuts = g.cuts()
        row_off, col, _ = g.export_csr()
        B = oracle.block_counts(n, row_off, col, cuts)
        total = g.info()["block_bytes"]
        ran = 0
        for frac in (0.25, 0.4, 0.6):
            try:
                got = g.count(stream_blocks=True, device_cap_bytes=int(total * frac), num_streams=streams)
            except P.PgabbError as e:
                assert e.status == P.ENOMEM
                continue
            ran += 1
            say("eviction", streams, frac, got, g.info()["h2d_bytes"])
            assert got == int(B.sum())
            ijk, cnt = g.task_counts()
            for (i, j, k), c in zip(ijk, cnt):
                assert c == B[i, j, k], (i, j, k)
            assert g.info()["h2d_bytes"] > walk_bytes(g.info())  # blocks were evicted and copied again
        assert ran >= 2


def test_ooc_workload_full_size():
    """R-MAT scale 24, edge factor 16 (268 M pairs), p = 32, blocks held in
    pinned host memory and streamed under an 8 GB device cap, and again under
    a 1 GiB cap that evicts blocks across four compute streams: the count
    equals the oracle's stored count."""
    with open(os.path.join(GOLDEN, "workload_counts.json")) as f:
        gold = json.load(f)["ooc"]
    import torch
    n, s, d = gen.ooc_graph()
    say("ooc generated", len(s))
    ds = torch.from_numpy(s).cuda()
    dd = torch.from_numpy(d).cuda()
    del s, d
    with P.Graph(n, ds, dd) as g:
        del ds, dd
        g.partition(32)
        say("ooc partitioned")
        got = g.count(stream_blocks=True, device_cap_bytes=8 * 10**9)
        info = g.info()
        say("ooc count", got, "h2d", info["h2d_bytes"], "ms", info["t_count_ms"])
        assert got == gold["triangles"]
        assert info["m"] == gold["m"] and info["probe_work"] == gold["probe_work"]
        got = g.count(device_cap_bytes=1 << 30, num_streams=4)
        say("ooc count at 1 GiB", got, "h2d", g.info()["h2d_bytes"])
        assert got == gold["triangles"]
