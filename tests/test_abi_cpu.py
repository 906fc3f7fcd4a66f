"""Host-side checks of the C ABI: the library loads, exports every function
the header declares, and rejects bad arguments before any device work."""
import ctypes

import numpy as np
import pytest

import paper_2209_04541_amd as P


def test_exports_every_declared_symbol():
    L = P.lib()
    names = P.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version():
    assert "gfx950" in P.version()


def _from_edges(n, m, s, d, flags=0, out=True):
    h = ctypes.c_void_p()
    return P.lib().pgabb_graph_from_edges(n, m, s, d, flags, None, ctypes.byref(h) if out else None)


def test_argument_errors_before_device_work():
    L = P.lib()
    s = np.array([0, 1], np.int32)
    d = np.array([1, 2], np.int32)
    ps, pd = s.ctypes.data, d.ctypes.data
    assert _from_edges(3, 2, ps, pd, out=False) == P.EINVAL
    assert _from_edges(-1, 0, None, None) == P.EINVAL
    assert _from_edges(3, -1, ps, pd) == P.EINVAL
    assert _from_edges(3, 2, None, pd) == P.EINVAL
    assert _from_edges(3, 2, ps, pd, flags=0x80) == P.EINVAL
    assert _from_edges(2, 2, ps, pd) == P.EINVAL  # id 2 outside [0, 2)
    assert b"outside" in L.pgabb_last_error()
    assert L.pgabb_last_status() == P.EINVAL
    bad = np.array([0, -3], np.int32)
    assert _from_edges(5, 2, bad.ctypes.data, pd) == P.EINVAL
    assert L.pgabb_partition(None, 2) == P.EINVAL
    assert L.pgabb_partition_ex(None, 2, 0, None) == P.EINVAL
    c = ctypes.c_uint64()
    assert L.pgabb_tc_count_ex(None, None, ctypes.byref(c)) == P.EINVAL
    assert L.pgabb_tc_count(None) == P.COUNT_ERROR
    assert L.pgabb_graph_info_get(None, None) == P.EINVAL
    assert L.pgabb_graph_cuts(None, None) == P.EINVAL
    assert L.pgabb_graph_task_counts(None, None, None) == P.EINVAL
    assert L.pgabb_graph_info(None, None, None, None, None) == P.EINVAL
    sh = (ctypes.c_int32 * 4)()
    assert L.pgabb_graph_task_shards(None, 2, sh) == P.EINVAL
    assert L.pgabb_tc_count_shard(None, None, 0, 2, ctypes.byref(c)) == P.EINVAL
    assert L.pgabb_tc_edge_support(None, None, 0, None) == P.EINVAL
    assert L.pgabb_tc_vertex_counts(None, None, 0, None) == P.EINVAL
    assert L.pgabb_tc_ktruss(None, 3, None, 0, None, None) == P.EINVAL
    assert L.pgabb_count_4cliques(None, ctypes.byref(c)) == P.EINVAL
    counts = (ctypes.c_uint64 * 2)(7, 7)
    assert L.pgabb_tc_count_batch(None, -1, None, counts) == P.EINVAL
    assert L.pgabb_tc_count_batch(None, 2, None, counts) == P.EINVAL
    gs = (ctypes.c_void_p * 2)(None, None)
    assert L.pgabb_tc_count_batch(gs, 2, None, counts) == P.EINVAL
    assert list(counts) == [P.COUNT_ERROR, P.COUNT_ERROR]
    assert L.pgabb_tc_count_batch(None, 0, None, None) == P.OK
    # two distinct (never dereferenced) graph handles: the options are
    # checked before any graph is touched
    fake = (ctypes.c_void_p * 2)(0x1000, 0x2000)
    for field, value in (("p", 65), ("p", -1), ("cut_mode", 7), ("host_threads", 65),
                         ("host_permille", 1001), ("kernel", 9), ("flags", 0x400)):
        o = P.options()
        setattr(o, field, value)
        counts[0] = counts[1] = 7
        assert L.pgabb_tc_count_batch(fake, 2, ctypes.byref(o), counts) == P.EINVAL, field
        assert list(counts) == [P.COUNT_ERROR, P.COUNT_ERROR]
    dup = (ctypes.c_void_p * 2)(0x1000, 0x1000)
    assert L.pgabb_tc_count_batch(dup, 2, None, counts) == P.EINVAL
    L.pgabb_graph_destroy(None)  # NULL-safe


def test_server_calls_reject_null():
    """pgabb_server_poll(s, ticket, done, count) and pgabb_server_times."""
    L = P.lib()
    done, cnt = ctypes.c_int32(), ctypes.c_uint64()
    ts, td = ctypes.c_double(), ctypes.c_double()
    assert L.pgabb_server_poll(None, 1, ctypes.byref(done), ctypes.byref(cnt)) == P.EINVAL
    assert L.pgabb_server_times(None, 1, ctypes.byref(ts), ctypes.byref(td)) == P.EINVAL
    assert L.pgabb_server_create(0, None, None) == P.EINVAL
    assert L.pgabb_server_submit(None, 1, 0, None, None, None) == P.EINVAL
    # the requests' grid is checked when the server is created
    h = ctypes.c_void_p()
    for bad in (-1, 65):
        o = P.options(p=bad)
        assert L.pgabb_server_create(1 << 30, ctypes.byref(o), ctypes.byref(h)) == P.EINVAL
        assert not h.value


def test_options_struct_names_the_grid():
    """pgabb_tc_options carries the grid p and the cut mode (the count can
    partition on its own), and the hybrid fields."""
    names = [f for f, _ in P.TcOptions._fields_]
    assert names[:2] == ["p", "cut_mode"]
    assert {"host_threads", "host_permille", "device_cap_bytes", "num_streams"} <= set(names)
    o = P.options(p=8, cut_mode=P.CUT_UNIFORM, hybrid=True, host_permille=250)
    assert (o.p, o.cut_mode, o.host_permille) == (8, P.CUT_UNIFORM, 250)
    assert o.flags & P.OPT_HYBRID


def test_allocator_hook_argument_check():
    L = P.lib()
    ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
    fa = ALLOC(lambda b, s, c: None)
    assert L.pgabb_set_allocator(fa, None, None) == P.EINVAL
    assert L.pgabb_set_allocator(None, None, None) == P.OK


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes mirrors have the header's sizes and offsets
    (checked against a C program compiled from include/pgabb.h)."""
    import os
    import subprocess
    fields = {"pgabb_tc_options": P.TcOptions, "pgabb_graph_info_t": P.GraphInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pgabb.h"', "int main(void) {"]
    for cname, cls in fields.items():
        lines.append('printf("%%zu\\n", sizeof(%s));' % cname)
        for f, _ in cls._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(P.HERE), "include")
    subprocess.check_call(["gcc", "-I" + inc, str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = []
    for cls in fields.values():
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f, _ in cls._fields_]
    assert got == want
