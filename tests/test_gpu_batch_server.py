"""GPU parity of the batched form (one persistent, graph-captured launch over
many graphs) and of the continuous-batching server, against the CPU oracle.
"""
import functools
import json
import math
import os
import sys
import time

import numpy as np
import pytest

import oracle
import paper_2209_04541_amd as P
from paper_2209_04541_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_batch(count, n_range=(64, 1500), d_range=(8, 64)):
    return [gen.batch_graph(g, n_range, d_range) for g in range(count)]


def test_batch_matches_oracle_all_shapes():
    gl = small_batch(160)
    gl += [graphs.complete(40)[0], graphs.wheel(77)[0], (0, np.zeros(0, np.int32), np.zeros(0, np.int32)),
           (5, np.zeros(0, np.int32), np.zeros(0, np.int32)), graphs.messy(*graphs.cocktail_party(9)[0])]
    want = np.array([oracle.tc(*g) for g in gl], np.uint64)
    say("batch graphs", len(gl), "triangles", int(want.sum()))
    with P.Batch(gl) as b:
        auto = b.count()  # autotuned + captured
        assert np.array_equal(auto, want)
        for kernel in (P.KERNEL_HASH, P.KERNEL_BITMAP):
            for waves in (2, 4, 8):
                for grab in (1, 5):
                    got = b.count(kernel=kernel, waves_per_block=waves, rows_per_grab=grab)
                    assert np.array_equal(got, want), (kernel, waves, grab)
        assert np.array_equal(b.count(per_graph=True), want)
        # replays of the captured launch, with eager work in between
        for rep in range(4):
            assert np.array_equal(b.count(), want), rep
            b.count(kernel=P.KERNEL_HASH, waves_per_block=2, rows_per_grab=3)


def test_batch_degenerate():
    with P.Batch([]) as b:
        assert len(b.count()) == 0
    z = np.zeros(0, np.int32)
    with P.Batch([(0, z, z), (3, z, z)]) as b:
        assert list(b.count()) == [0, 0]
    loops = np.arange(4, dtype=np.int32)
    with P.Batch([(4, loops, loops)]) as b:
        assert list(b.count()) == [0]
    with pytest.raises(P.PgabbError) as ei:
        P.Batch([(3, np.array([0, 1], np.int32), np.array([1, 3], np.int32))])
    assert ei.value.status == P.EINVAL


def test_batch_workload_sample():
    """Graphs of the 10,000-graph recipe at their real sizes (n up to 8192,
    degree up to 64), a sample of 48."""
    gl = [gen.batch_graph(g) for g in range(0, 480, 10)]
    want = np.array([oracle.tc(*g) for g in gl], np.uint64)
    with P.Batch(gl) as b:
        assert np.array_equal(b.count(), want)
        assert np.array_equal(b.count(per_graph=True), want)


def _rmat_requests(k, seed0=500):
    """k R-MAT requests of scales 10 .. 18 (r * 5 mod 9 visits every
    residue) and edge factors 8 .. 32, counted by the oracle in the test."""
    out = []
    for r in range(k):
        sc = 10 + (r * 5) % 9
        ef = 8 + (r * 5) % 25
        out.append(gen.rmat(sc, ef, gen.seed(seed0, r)))
    return out


def _served_pool():
    """Oracle counts of the served workload's request pool (written by
    tests/golden/make_golden.py from the oracle)."""
    with open(os.path.join(GOLDEN, "workload_counts.json")) as f:
        return json.load(f)["served"]


def _wait(srv, tickets, timeout=60):
    t0 = time.time()
    res = {}
    while len(res) < len(tickets):
        for t in tickets:
            if t in res:
                continue
            done, cnt, ts, td = srv.poll(t)
            if done:
                res[t] = cnt
        if time.time() - t0 > timeout:
            raise TimeoutError("server did not finish")
        time.sleep(0.001)
    return [res[t] for t in tickets]


@pytest.mark.parametrize("borrow", [False, True])
def test_server_alone_equals_mix(borrow):
    reqs = _rmat_requests(24)
    want = [oracle.tc(*g) for g in reqs]
    say("server requests", len(reqs), "borrow", borrow)
    with P.Server(8 << 30, borrow=borrow) as srv:
        alone = []
        for g in reqs[:8]:
            t = srv.submit(*g)
            alone += _wait(srv, [t])
        tickets = [srv.submit(*g) for g in reqs]
        mix = _wait(srv, tickets)
        srv.drain()
        assert srv.launches() >= 2
    assert alone == want[:8]
    assert mix == want


@functools.lru_cache(maxsize=1)
def _grid_requests():
    reqs = _rmat_requests(12, seed0=700)
    return reqs, [oracle.tc(*g) for g in reqs]


@pytest.mark.parametrize("grid", [(1, P.CUT_NNZ), (3, P.CUT_UNIFORM), (8, P.CUT_NNZ)])
def test_server_fixed_grid(grid):
    """Requests partitioned with a grid the options fix (by default requests
    of at least 2^18 pairs get 8 x 8 blocks and smaller ones one block):
    every result still equals the oracle's count."""
    p, cut = grid
    reqs, want = _grid_requests()
    say("server grid", p, "cut", cut, "requests", len(reqs))
    with P.Server(8 << 30, p=p, cut_mode=cut) as srv:
        assert _wait(srv, [srv.submit(*g) for g in reqs]) == want
        srv.drain()


def test_server_small_budget_and_rejection():
    reqs = _rmat_requests(10, seed0=600)
    want = [oracle.tc(*g) for g in reqs]
    biggest = max(len(g[1]) for g in reqs)
    budget = biggest * 40 + 64 * (1 << 20)  # admits about one request at a time
    with P.Server(budget) as srv:
        tickets = [srv.submit(*g) for g in reqs]
        assert _wait(srv, tickets) == want
        n, s, d = gen.rmat(20, 16, gen.seed(601, 0))  # 16.8 M pairs: about 0.7 GB estimated
        with pytest.raises(P.PgabbError) as ei:
            srv.submit(n, s, d)
        assert ei.value.status == P.EBUDGET
        # ids are checked when the request is built: the failure shows at poll
        bad = srv.submit(4, np.array([0], np.int32), np.array([7], np.int32))
        with pytest.raises(P.PgabbError) as ei:
            _wait(srv, [bad])
        assert ei.value.status == P.EINVAL
        # and the server keeps serving
        assert _wait(srv, [srv.submit(*reqs[0])]) == want[:1]


def test_batch_rows_longer_than_a_wave():
    """Rows with more than 64 out-neighbours fill a whole 64-lane batch of
    walked lists (the flattened walk's lane search then reaches lane 63)."""
    gl = [graphs.complete(100)[0], graphs.complete(130)[0], graphs.wheel(300)[0],
          gen.rgg(3000, 150, gen.seed(4, 99999))]
    want = np.array([oracle.tc(*g) for g in gl], np.uint64)
    with P.Batch(gl) as b:
        for kernel in (P.KERNEL_HASH, P.KERNEL_BITMAP):
            assert np.array_equal(b.count(kernel=kernel, waves_per_block=4, rows_per_grab=2), want)
        assert np.array_equal(b.count(), want)


def test_server_scales_10_to_22_alone_equals_mix():
    """The served recipe at its real sizes: one pool request per R-MAT scale
    10 .. 22 (edge factors 8 .. 32, up to 134 M pairs) plus K_1100, whose
    staged lists (up to 1099 entries) split the merged launch into two LDS
    classes.  Each result equals the oracle's count when the request runs
    alone and when all of them are submitted at once."""
    pool = _served_pool()
    by_scale = {}
    for r in sorted(pool, key=int):
        by_scale.setdefault(pool[r]["scale"], int(r))
    assert sorted(by_scale) == list(range(10, 23))
    reqs, want = [], []
    for sc in range(10, 23):
        r = by_scale[sc]
        n, s, d = gen.served_graph(r)
        assert len(s) == pool[str(r)]["m_input"]
        reqs.append((n, s, d))
        want.append(pool[str(r)]["triangles"])
        say("pool request", r, "scale", sc, "pairs", len(s))
    k_s, k_d = np.triu_indices(1100, 1)
    reqs.append((1100, k_s.astype(np.int32), k_d.astype(np.int32)))
    want.append(math.comb(1100, 3))
    with P.Server(64 << 30) as srv:
        alone = []
        for q, g in enumerate(reqs):
            say("alone", q)
            alone += _wait(srv, [srv.submit(*g)], timeout=100)
        say("mix of", len(reqs))
        tickets = [srv.submit(*g) for g in reqs]
        mix = _wait(srv, tickets, timeout=100)
        srv.drain()
    assert alone == want
    assert mix == want


def test_batch_all_10000_graphs():
    """Every graph of the 10,000-graph batch workload (even g random
    geometric, odd g Erdos-Renyi, n 64 .. 8192, degree 8 .. 64) against the
    oracle's stored count, with the autotuned, graph-captured launch."""
    want = np.array([int(x) for x in open(os.path.join(GOLDEN, "batch_counts.txt")) if not x.startswith("#")],
                    np.uint64)
    G = len(want)
    assert G == 10000
    nv = np.empty(G, np.int32)
    eoff = np.zeros(G + 1, np.int64)
    srcs, dsts = [], []
    for g in range(G):
        n, s, d = gen.batch_graph(g)
        nv[g] = n
        eoff[g + 1] = eoff[g] + len(s)
        srcs.append(s)
        dsts.append(d)
        if g % 2000 == 0:
            say("generated", g)
    src = np.concatenate(srcs)
    dst = np.concatenate(dsts)
    del srcs, dsts
    say("pairs", len(src))
    with P.Batch((nv, eoff, src, dst)) as b:
        say("built")
        got = b.count()
        say("counted")
        bad = np.nonzero(got != want)[0]
        assert len(bad) == 0, bad[:10]
        got = b.count(kernel=P.KERNEL_HASH, waves_per_block=4, rows_per_grab=4)
        assert np.array_equal(got, want)
