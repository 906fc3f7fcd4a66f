"""One device's share of a count split by task over several devices, through
the C ABI: the library's deal of tasks to shards against an independent
longest-processing-time deal written here from the task weights, and each
shard's counts against the oracle's per-triple counts (exact equality)."""
import heapq
import sys

import numpy as np
import pytest

import oracle
import paper_2209_04541_amd as P
from paper_2209_04541_amd import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tasks_from_csr(n, row_off, col, cuts, by_cols):
    """Block-lists (i, j, k), i <= j <= k, with three non-empty blocks,
    heaviest first by edges of the three blocks (equal weights keep the
    order of the (i, j, k) loops), and each one's estimated work: entries
    its walk reads and its items stage, a list's length taken as the mean
    over its block's non-empty rows."""
    p = len(cuts) - 1
    stripe = np.searchsorted(cuts, np.arange(n), side="right") - 1
    rows = np.repeat(np.arange(n), np.diff(row_off))
    blk = stripe[rows].astype(np.int64) * p + stripe[col]
    nnz = np.bincount(blk, minlength=p * p).reshape(p, p)
    nr = np.bincount(np.unique(blk * n + rows) // n, minlength=p * p).reshape(p, p)
    nc = np.bincount(np.unique(blk * n + col) // n, minlength=p * p).reshape(p, p)
    mean = lambda a, b: int(nnz[a, b]) / max(int(nr[a, b]), 1)

    def work(i, j, k):
        if by_cols:
            return 1 + int(int(nnz[i, j]) * mean(i, k)) + int(int(nc[i, j]) * mean(j, k))
        return 1 + int(int(nnz[i, j]) * mean(j, k)) + int(int(nr[i, j]) * mean(i, k))

    tasks = []
    for i in range(p):
        for j in range(i, p):
            for k in range(j, p):
                if nnz[i, j] and nnz[i, k] and nnz[j, k]:
                    tasks.append(((i, j, k), int(nnz[i, j] + nnz[i, k] + nnz[j, k])))
    order = sorted(range(len(tasks)), key=lambda t: -tasks[t][1])  # stable
    ijk = [tasks[t][0] for t in order]
    return ijk, [work(*x) for x in ijk]


def lpt_shards(ijk, weight, num_shards):
    """Groups of tasks sharing (i, j), heaviest group first by summed work
    (ties: earliest first task), each to the least loaded shard (ties:
    lowest index)."""
    gw, first = {}, {}
    for t, (i, j, _) in enumerate(ijk):
        gw[(i, j)] = gw.get((i, j), 0) + weight[t]
        first.setdefault((i, j), t)
    heap = [(0, s) for s in range(num_shards)]
    shard = {}
    for grp in sorted(gw, key=lambda x: (-gw[x], first[x])):
        load, s = heapq.heappop(heap)
        shard[grp] = s
        heapq.heappush(heap, (load + gw[grp], s))
    return np.array([shard[(i, j)] for i, j, _ in ijk], np.int32)


@pytest.fixture(scope="module")
def rmat14():
    n, s, d = gen.rmat(14, 16, gen.seed(97, 3))
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    return n, s, d, row_off, col, oracle.tc(n, s, d)


@pytest.mark.parametrize("p,cut_mode", [(8, P.CUT_NNZ), (5, P.CUT_UNIFORM), (1, P.CUT_NNZ),
                                        (64, P.CUT_NNZ)])
def test_deal_matches_lpt(rmat14, p, cut_mode):
    n, s, d, row_off, col, _ = rmat14
    with P.Graph(n, s, d) as g:
        g.partition(p, cut_mode=cut_mode)
        cuts = g.cuts()
        ijk, _ = g.task_counts()
        info = g.info()
        by_cols = not info["probe_work"] < info["probe_work_col"]  # the default walk
        want_ijk, weight = tasks_from_csr(n, row_off, col, cuts, by_cols)
        assert [tuple(x) for x in ijk] == want_ijk
        for S in (1, 2, 3, 8, 100):
            say("deal", p, cut_mode, S)
            got = g.task_shards(S)
            assert np.array_equal(got, lpt_shards(want_ijk, weight, S)), (p, S)


@pytest.mark.parametrize("S", [1, 3, 8])
def test_in_core_shards_sum_to_count(rmat14, S):
    n, s, d, row_off, col, want = rmat14
    with P.Graph(n, s, d) as g:
        g.partition(8)
        B = oracle.block_counts(n, row_off, col, g.cuts())
        of = g.task_shards(S)
        total = 0
        for sh in range(S):
            c = g.count_shard(sh, S)
            ijk, cnt = g.task_counts()
            say("in-core shard", S, sh, c)
            for t, (i, j, k) in enumerate(ijk):
                assert cnt[t] == (B[i, j, k] if of[t] == sh else 0), (sh, t)
            assert c == sum(int(B[i, j, k]) for t, (i, j, k) in enumerate(ijk) if of[t] == sh)
            assert g.info()["h2d_bytes"] == 0
            total += c
        assert total == want
        # a whole count afterwards reports every task again
        assert g.count() == want
        ijk, cnt = g.task_counts()
        assert all(cnt[t] == B[i, j, k] for t, (i, j, k) in enumerate(ijk))


@pytest.mark.parametrize("cap_frac", [0, 0.35])
def test_streamed_shards_copy_their_blocks(rmat14, cap_frac):
    """Blocks in host memory: a shard copies only the blocks its tasks read
    (fewer bytes than the whole store), under a cap too (with eviction)."""
    n, s, d, row_off, col, want = rmat14
    S = 4
    with P.Graph(n, s, d) as g:
        g.partition(8)
        total_bytes = g.info()["block_bytes"]
        B = oracle.block_counts(n, row_off, col, g.cuts())
        of = g.task_shards(S)
        cap = int(total_bytes * cap_frac)
        total, copied = 0, []
        for sh in range(S):
            try:
                c = g.count_shard(sh, S, stream_blocks=True, device_cap_bytes=cap)
            except P.PgabbError as e:
                assert cap and e.status == P.ENOMEM  # a task's blocks exceed the cap
                pytest.skip("cap below one task's blocks")
            ijk, cnt = g.task_counts()
            info = g.info()
            say("streamed shard", cap_frac, sh, c, info["h2d_bytes"], total_bytes)
            assert c == sum(int(B[i, j, k]) for t, (i, j, k) in enumerate(ijk) if of[t] == sh)
            assert all(cnt[t] == (B[i, j, k] if of[t] == sh else 0) for t, (i, j, k) in enumerate(ijk))
            if not cap:
                assert 0 < info["h2d_bytes"] < total_bytes
            copied.append(info["h2d_bytes"])
            total += c
        assert total == want
        inf = g.info()
        walked = inf["walk_bytes_cols"] if inf["walked_columns"] else inf["walk_bytes_rows"]
        assert sum(copied) >= walked * 0.99  # every block read by some shard
        assert g.count(device_cap_bytes=cap) == want


def test_shard_edge_cases():
    n = 40
    s, d = np.triu_indices(n, 1)
    s, d = s.astype(np.int32), d.astype(np.int32)
    want = n * (n - 1) * (n - 2) // 6
    with P.Graph(n, s, d) as g:
        with pytest.raises(P.PgabbError) as e:
            g.task_shards(2)
        assert e.value.status == P.ESTATE
        # counting a shard before partitioning partitions with p = 1
        assert g.count_shard(0, 1) == want
        g.partition(3)
        T = g.info()["num_tasks"]
        # more shards than groups of tasks: the extra shards hold nothing
        counts = [g.count_shard(sh, 64) for sh in range(64)]
        assert sum(counts) == want
        assert sum(c > 0 for c in counts) <= T
        assert len(set(g.task_shards(64))) <= T
        for bad in ((2, 2), (-1, 2), (0, 0), (0, 5000)):
            with pytest.raises(P.PgabbError) as e:
                g.count_shard(*bad)
            assert e.value.status == P.EINVAL
        with pytest.raises(P.PgabbError):
            g.task_shards(0)
        assert g.count() == want
    with P.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32)) as g:
        g.partition(2)
        assert g.count_shard(1, 2) == 0
