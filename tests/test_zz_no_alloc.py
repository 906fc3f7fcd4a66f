"""The allocation-free count (pgabb_tc_count_noalloc) against the count it
is a variant of (pgabb_tc_count_ex), through the C ABI: equal counts and
equal per-task counts on two calls in a row, the second on a smaller graph
(fewer tasks, so stale counters of the first call would show), both against
the oracle's per-triple counts; no allocation reaches the allocator hook
during the calls; sizes beyond the fixed array are refused."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_2209_04541_amd as P
from paper_2209_04541_amd import gen

pytestmark = pytest.mark.gpu

ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


class CountingHook:
    """An allocator hook that hands out torch's device memory and counts the
    allocations it sees."""

    def __init__(self):
        import torch
        self.allocs = 0
        self.live = {}

        def alloc(nbytes, stream, ctx):
            self.allocs += 1
            t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda")
            self.live[t.data_ptr()] = t
            return t.data_ptr()

        def free(ptr, stream, ctx):
            torch.cuda.synchronize()
            self.live.pop(ptr, None)

        self._a = ALLOC(alloc)
        self._f = FREE(free)

    def __enter__(self):
        assert P.lib().pgabb_set_allocator(ctypes.cast(self._a, ctypes.c_void_p),
                                           ctypes.cast(self._f, ctypes.c_void_p), None) == P.OK
        return self

    def __exit__(self, *exc):
        assert P.lib().pgabb_set_allocator(None, None, None) == P.OK


def noalloc(g, opts=None):
    c = ctypes.c_uint64()
    st = P.lib().pgabb_tc_count_noalloc(g._h, ctypes.byref(opts) if opts is not None else None, ctypes.byref(c))
    return st, int(c.value)


def per_task(g, n, cuts):
    ijk, cnt = g.task_counts()
    return sorted(zip(map(tuple, ijk), cnt.tolist()))


def oracle_tasks(n, s, d, g):
    row_off, col, _ = g.export_csr()
    B = oracle.block_counts(n, row_off, col, g.cuts())
    ijk, _ = g.task_counts()
    return sorted((tuple(t), int(B[tuple(t)])) for t in ijk)


def test_noalloc_equals_count_ex_two_calls():
    big = gen.rmat(16, 16, gen.seed(970, 0))
    small = gen.rmat(11, 8, gen.seed(970, 1))
    with P.Graph(*big) as g1, P.Graph(*small) as g2:
        g1.partition(16)
        g2.partition(5)
        want1 = g1.count()
        tasks1 = per_task(g1, big[0], g1.cuts())
        want2 = g2.count()
        tasks2 = per_task(g2, small[0], g2.cuts())
        assert tasks1 == oracle_tasks(*big, g1)
        assert tasks2 == oracle_tasks(*small, g2)
        assert want1 == oracle.tc(*big) and want2 == oracle.tc(*small)
        assert P.lib().pgabb_tc_count_noalloc_scratch_bytes() == 4 << 20
        for rep in range(2):
            with CountingHook() as hook:
                st1, c1 = noalloc(g1)
                say("noalloc big", rep, st1, c1, want1)
                t1 = per_task(g1, big[0], g1.cuts())
                st2, c2 = noalloc(g2)
                say("noalloc small", rep, st2, c2, want2)
                t2 = per_task(g2, small[0], g2.cuts())
                assert hook.allocs == 0
            assert st1 == P.OK and st2 == P.OK
            assert c1 == want1 and t1 == tasks1
            assert c2 == want2 and t2 == tasks2
        # options as the regular count takes them, one after another
        for kw in (dict(kernel=P.KERNEL_HASH), dict(by_rows=True), dict(waves_per_block=8, rows_per_grab=3),
                   dict(p=16)):
            st, c = noalloc(g1, P.options(**kw))
            assert st == P.OK and c == want1, kw
        # the allocating path does reach the hook (the hook works)
        with CountingHook() as hook:
            assert g2.count() == want2
            assert hook.allocs > 0


def test_noalloc_split_launch_and_edges():
    # K_1100: staged lists above the 1280-word class, so the launch is split
    # by staged length (the queues are cleared between the parts)
    ks, kd = np.triu_indices(1100, 1)
    with P.Graph(1100, ks.astype(np.int32), kd.astype(np.int32)) as g:
        g.partition(1)
        st, c = noalloc(g)
        assert st == P.OK and c == 1100 * 1099 * 1098 // 6
        assert g.info()["kernel_launches"] >= 2
    # an edgeless graph and an empty one
    with P.Graph(10, np.zeros(0, np.int32), np.zeros(0, np.int32)) as g:
        g.partition(2)
        assert noalloc(g) == (P.OK, 0)
    with P.Graph(0, np.zeros(0, np.int32), np.zeros(0, np.int32)) as g:
        g.partition(1)
        assert noalloc(g) == (P.OK, 0)


def test_noalloc_refusals():
    n, s, d = gen.rmat(10, 8, gen.seed(971, 0))
    with P.Graph(n, s, d) as g:
        st, c = noalloc(g)  # not partitioned
        assert st == P.ESTATE and c == P.COUNT_ERROR
        g.partition(4)
        assert noalloc(g, P.options(p=8))[0] == P.ESTATE
        assert noalloc(g, P.options(stream_blocks=True))[0] == P.EINVAL
        assert noalloc(g, P.options(hybrid=True))[0] == P.EINVAL
        assert noalloc(g, P.options(device_cap_bytes=1024))[0] == P.EINVAL
        want = g.count()
        assert noalloc(g) == (P.OK, want)
        g.count(stream_blocks=True)  # blocks now in host memory
        assert noalloc(g)[0] == P.ESTATE
    # more tasks than the 4 MiB array holds: K_300 at p = 64 has every block
    # non-empty, so all C(66, 3) = 45,760 block-lists are tasks
    ks, kd = np.triu_indices(300, 1)
    with P.Graph(300, ks.astype(np.int32), kd.astype(np.int32)) as g:
        g.partition(64)
        assert g.info()["num_tasks"] == 45760
        st, c = noalloc(g)
        assert st == P.EINVAL and b"scratch" in P.lib().pgabb_last_error()
        assert g.count() == 300 * 299 * 298 // 6
