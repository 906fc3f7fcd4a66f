"""Randomised and invariance checks of the GPU path against brute force and
the oracle, and error paths forced from the host (an allocator hook that
fails on purpose).  Counts are integers: the bar is exact equality."""
import ctypes
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


def gpu_count(n, s, d, p=1, cuts=None, **kw):
    with P.Graph(n, s, d) as g:
        g.partition(p, cuts=cuts)
        return g.count(**kw)


def test_random_graphs_cuts_kernels_walks_streams():
    """Random graphs (loops and repeats included) x random cut vectors (empty
    stripes allowed) x staging kinds x walk orientations x in-core or
    streamed counting."""
    rng = np.random.default_rng(2024)
    kernels = [P.KERNEL_AUTO, P.KERNEL_HASH, P.KERNEL_BITMAP, P.KERNEL_SEARCH]
    for case in range(32):
        n = int(rng.integers(2, 70 if case % 2 else 500))
        m = int(rng.integers(0, 8 * n))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        want = graphs.brute_force(n, s, d) if n <= 70 else oracle.tc(n, s, d)
        p = int(rng.integers(1, min(n, 12) + 1))
        cuts = np.concatenate([[0], np.sort(rng.integers(0, n + 1, p - 1)), [n]]).astype(np.int32)
        kw = dict(kernel=int(kernels[case % 4]), by_rows=[None, True, False][case % 3],
                  waves_per_block=[2, 4, 8][case % 3], unroll=[1, 2, 4, 8][case % 4])
        if case % 5 == 0:
            kw.update(stream_blocks=True, num_streams=1 + case % 3)
        say("case", case, n, m, p, kw, want)
        assert gpu_count(n, s, d, p, cuts=cuts, **kw) == want, case


def test_relabel_shuffle_and_order_invariance():
    n, s, d = gen.rmat(12, 16, gen.seed(97, 5))
    want = oracle.tc(n, s, d)
    rng = np.random.default_rng(3)
    perm = rng.permutation(n).astype(np.int32)
    order = rng.permutation(len(s))
    for ss, dd in ((perm[s], perm[d]), (s[order], d[order]), (d, s)):
        assert gpu_count(n, ss, dd, 4) == want
    with P.Graph(n, s, d, order_by_id=True) as g:
        g.partition(3)
        assert g.count() == want


def test_batch_order_and_composition():
    gl = [gen.batch_graph(g, (64, 1200)) for g in range(40)]
    want = [oracle.tc(*g) for g in gl]
    with P.Batch(gl[::-1]) as b:
        assert list(b.count()) == want[::-1]
    with P.Batch(gl[:13]) as b:
        assert list(b.count()) == want[:13]
    with P.Batch(gl[13:] + gl[:13]) as b:
        assert list(b.count()) == want[13:] + want[:13]


def test_allocator_hook_failure_and_restore():
    """Device memory from a caller's hook (torch's caching allocator here):
    a count runs on it; failing the k-th allocation reports ENOMEM and gives
    back every block taken; removing the hook restores the library's own
    allocator."""
    import torch
    L = P.lib()
    ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
    FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
    live = {}
    state = {"calls": 0, "fail_at": None}

    def alloc(nbytes, stream, ctx):
        state["calls"] += 1
        if state["fail_at"] is not None and state["calls"] >= state["fail_at"]:
            return None
        ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device=0, stream=int(stream or 0))
        live[ptr] = nbytes
        return ptr

    def free(ptr, stream, ctx):
        live.pop(ptr)
        torch.cuda.caching_allocator_delete(ptr)

    fa, ff = ALLOC(alloc), FREE(free)
    n, s, d = gen.rmat(11, 16, gen.seed(97, 6))
    want = oracle.tc(n, s, d)
    torch.cuda.synchronize()
    assert L.pgabb_set_allocator(fa, ff, None) == P.OK
    try:
        assert gpu_count(n, s, d, 3) == want
        total = state["calls"]
        assert total > 4 and not live
        for k in sorted({1, 2, total // 3, total // 2, total - 1, total}):
            state["calls"] = 0
            state["fail_at"] = k
            with pytest.raises(P.PgabbError) as ei:
                gpu_count(n, s, d, 3)
            assert ei.value.status == P.ENOMEM, k
            assert not live, k
        state["fail_at"] = None
    finally:
        assert L.pgabb_set_allocator(None, None, None) == P.OK
        torch.cuda.synchronize()
    assert gpu_count(n, s, d, 3) == want


def test_dense_graphs_task_counts():
    """Dense random graphs (rows of hundreds of entries) under random cut
    vectors: per-task counts of row and column walks match the oracle's
    block counts, for the automatic, hash and search staging."""
    rng = np.random.default_rng(11)
    for case in range(12):
        n = int(rng.integers(150, 420))
        m = int(rng.integers(n * n // 8, n * n // 3))
        s = rng.integers(0, n, m).astype(np.int32)
        d = rng.integers(0, n, m).astype(np.int32)
        _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
        p = int(rng.integers(1, 6))
        cuts = np.concatenate([[0], np.sort(rng.integers(0, n + 1, p - 1)), [n]]).astype(np.int32)
        B = oracle.block_counts(n, row_off, col, cuts)
        kernel = int([P.KERNEL_AUTO, P.KERNEL_HASH, P.KERNEL_SEARCH][case % 3])
        for by_rows in (False, True):
            with P.Graph(n, s, d) as g:
                g.partition(p, cuts=cuts)
                total = g.count(by_rows=by_rows, kernel=kernel)
                ijk, cnt = g.task_counts()
            got = np.zeros_like(B)
            for (i, j, k), c in zip(ijk, cnt):
                got[i, j, k] += c
            say("dense case", case, n, m, p, by_rows, kernel, total)
            assert np.array_equal(got, B), (case, by_rows)
            assert total == int(B.sum())
