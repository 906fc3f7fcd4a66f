"""Python binding of libpgabb.so, the MI355X block-partitioned triangle
counter (PGAbB's triangle-counting example: Section 3.6 for the block-list
kernel, Section 4.3 for the symmetric 2-D partition, Section 4.4 for the
scheduler).

Argument marshalling only: every step runs in the library's HIP kernels.
Edge arrays may be numpy arrays (host) or torch CUDA tensors (device); for
device tensors the current torch stream is handed to the library.  If the
library has not been built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpgabb.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pgabb.h")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EBUDGET = 0, -1, -2, -3, -4, -5
COUNT_ERROR = 2**64 - 1
EDGES_ON_DEVICE = 0x1
ORDER_BY_ID = 0x2
CUT_NNZ, CUT_UNIFORM = 0, 1
KERNEL_AUTO, KERNEL_HASH, KERNEL_BITMAP, KERNEL_SEARCH = 0, 1, 2, 3
OPT_STREAM = 0x1
OPT_ROWS = 0x8
SUPPORT_ON_DEVICE = 0x1
OPT_COLS = 0x10
OPT_HYBRID = 0x20


class PgabbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("pgabb status %d: %s" % (status, message))
        self.status = status


class TcOptions(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("cut_mode", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("num_streams", ctypes.c_int32),
                ("device_cap_bytes", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("waves_per_block", ctypes.c_int32), ("rows_per_grab", ctypes.c_int32),
                ("unroll", ctypes.c_int32), ("host_threads", ctypes.c_int32),
                ("host_permille", ctypes.c_int32)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m_input", ctypes.c_int64), ("m", ctypes.c_int64),
                ("isolated", ctypes.c_int64), ("max_out_degree", ctypes.c_int32),
                ("p", ctypes.c_int32), ("num_blocks", ctypes.c_int64),
                ("num_tasks", ctypes.c_int64), ("probe_work", ctypes.c_uint64),
                ("block_bytes", ctypes.c_uint64), ("h2d_bytes", ctypes.c_uint64),
                ("t_build_ms", ctypes.c_double), ("t_partition_ms", ctypes.c_double),
                ("t_count_ms", ctypes.c_double), ("t_kernel_ms", ctypes.c_double),
                ("kernel_launches", ctypes.c_int64), ("probe_work_col", ctypes.c_uint64),
                ("walked_columns", ctypes.c_int64), ("host_tasks", ctypes.c_int64),
                ("host_work_share", ctypes.c_double), ("row_items", ctypes.c_int64),
                ("col_items", ctypes.c_int64), ("t_tune_ms", ctypes.c_double),
                ("walk_bytes_rows", ctypes.c_uint64), ("walk_bytes_cols", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def header_functions():
    """Names of the functions declared in include/pgabb.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pgabb_[a-z0-9_]+)\s*\(", text)
    return sorted(set(n for n in names if not n.endswith("_fn")))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpgabb.so is not built: run paper_2209_04541_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_uint64)
        st = ctypes.c_int
        sig = {
            "pgabb_graph_from_edges": (st, [i32, i64, vp, vp, u32, vp, ctypes.POINTER(vp)]),
            "pgabb_partition": (st, [vp, i32]),
            "pgabb_partition_ex": (st, [vp, i32, i32, vp]),
            "pgabb_tc_count": (u64, [vp]),
            "pgabb_tc_count_ex": (st, [vp, vp, ctypes.POINTER(u64)]),
            "pgabb_tc_count_noalloc": (st, [vp, vp, ctypes.POINTER(u64)]),
            "pgabb_tc_count_noalloc_scratch_bytes": (ctypes.c_size_t, []),
            "pgabb_graph_info_get": (st, [vp, ctypes.POINTER(GraphInfo)]),
            "pgabb_graph_info": (st, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                      ctypes.POINTER(i64)]),
            "pgabb_tc_count_batch": (st, [vp, i64, vp, vp]),
            "pgabb_tune_cache_reload": (st, []),
            "pgabb_graph_export_csr": (st, [vp, vp, vp, vp]),
            "pgabb_graph_cuts": (st, [vp, vp]),
            "pgabb_graph_task_counts": (st, [vp, vp, vp]),
            "pgabb_graph_task_shards": (st, [vp, i32, vp]),
            "pgabb_tc_edge_support": (st, [vp, vp, u32, ctypes.POINTER(u64)]),
            "pgabb_tc_vertex_counts": (st, [vp, vp, u32, ctypes.POINTER(u64)]),
            "pgabb_tc_ktruss": (st, [vp, i32, vp, u32, ctypes.POINTER(i64), ctypes.POINTER(i32)]),
            "pgabb_count_4cliques": (st, [vp, ctypes.POINTER(u64)]),
            "pgabb_count_4cliques_streamed": (st, [vp, u64, ctypes.POINTER(u64)]),
            "pgabb_graph_4list_counts": (st, [vp, ctypes.POINTER(i64), vp, vp]),
            "pgabb_components": (st, [vp, vp, u32, ctypes.POINTER(i64), ctypes.POINTER(i32)]),
            "pgabb_pagerank": (st, [vp, ctypes.c_double, ctypes.c_double, i32, vp, u32, ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_double)]),
            "pgabb_tc_count_shard": (st, [vp, vp, i32, i32, ctypes.POINTER(u64)]),
            "pgabb_graph_destroy": (None, [vp]),
            "pgabb_last_status": (st, []),
            "pgabb_last_error": (ctypes.c_char_p, []),
            "pgabb_batch_create": (st, [i64, vp, vp, vp, vp, u32, vp, ctypes.POINTER(vp)]),
            "pgabb_batch_count": (st, [vp, vp, vp]),
            "pgabb_batch_times": (st, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
            "pgabb_batch_destroy": (None, [vp]),
            "pgabb_batch_launch_shape": (st, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                              ctypes.POINTER(ctypes.c_double)]),
            "pgabb_batch_stats": (st, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                       ctypes.POINTER(u64)]),
            "pgabb_server_create": (st, [u64, vp, ctypes.POINTER(vp)]),
            "pgabb_server_submit": (st, [vp, i32, i64, vp, vp, ctypes.POINTER(u64)]),
            "pgabb_server_poll": (st, [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(u64)]),
            "pgabb_server_times": (st, [vp, u64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
            "pgabb_server_drain": (st, [vp]),
            "pgabb_server_now": (ctypes.c_double, [vp]),
            "pgabb_server_stats": (st, [vp, ctypes.POINTER(u64)]),
            "pgabb_server_kernel_stats": (st, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(u64),
                                               ctypes.POINTER(u64)]),
            "pgabb_server_destroy": (None, [vp]),
            "pgabb_set_allocator": (st, [vp, vp, vp]),
            "pgabb_release_cached_memory": (st, []),
            "pgabb_version": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        msg = lib().pgabb_last_error()
        raise PgabbError(status, msg.decode() if msg else "")


def _is_torch_cuda(a):
    return type(a).__module__.startswith("torch") and getattr(a, "is_cuda", False)


def _torch_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _edges(src, dst):
    """(ptr_src, ptr_dst, m, flags, keepalive, stream) for host or device arrays."""
    if _is_torch_cuda(src) or _is_torch_cuda(dst):
        import torch
        if not (_is_torch_cuda(src) and _is_torch_cuda(dst)):
            raise ValueError("src and dst must both be device tensors or both host arrays")
        s = src.to(torch.int32).contiguous()
        d = dst.to(torch.int32).contiguous()
        if s.numel() != d.numel():
            raise ValueError("src and dst differ in length")
        return (ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()), s.numel(),
                EDGES_ON_DEVICE, (s, d), _torch_stream())
    s = np.ascontiguousarray(np.asarray(src), dtype=np.int32)
    d = np.ascontiguousarray(np.asarray(dst), dtype=np.int32)
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    stream = None
    try:
        import torch
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            stream = _torch_stream()
    except ImportError:
        pass
    return (ctypes.c_void_p(s.ctypes.data if s.size else 0), ctypes.c_void_p(d.ctypes.data if d.size else 0),
            s.size, 0, (s, d), stream)


def options(kernel=KERNEL_AUTO, num_streams=0, device_cap_bytes=0, stream_blocks=False,
            waves_per_block=0, rows_per_grab=0, unroll=0, by_rows=None, p=0, cut_mode=CUT_NNZ,
            hybrid=False, host_threads=0, host_permille=0):
    """by_rows: True walks edge blocks by rows, False by columns, None lets
    the library take the walk that reads fewer entries.  p > 0 partitions
    the graph with p (and cut_mode) before the count unless it already is.
    hybrid: light tasks on host threads (host_permille: fixed share of the
    estimated work, 0 = both sides pull from one queue until they meet)."""
    o = TcOptions()
    o.p = p
    o.cut_mode = cut_mode
    o.host_threads = host_threads
    o.host_permille = host_permille
    o.kernel = kernel
    o.num_streams = num_streams
    o.device_cap_bytes = device_cap_bytes
    o.flags = OPT_STREAM if stream_blocks else 0
    if hybrid:
        o.flags |= OPT_HYBRID
    if by_rows is not None:
        o.flags |= OPT_ROWS if by_rows else OPT_COLS
    o.waves_per_block = waves_per_block
    o.rows_per_grab = rows_per_grab
    o.unroll = unroll
    return o


class Graph:
    """A cleaned, degree-oriented graph resident on the device."""

    def __init__(self, n, src, dst, order_by_id=False, stream=None):
        ps, pd, m, flags, keep, st = _edges(src, dst)
        if order_by_id:
            flags |= ORDER_BY_ID
        if stream is not None:
            st = ctypes.c_void_p(stream)
        h = ctypes.c_void_p()
        _check(lib().pgabb_graph_from_edges(int(n), int(m), ps, pd, flags, st, ctypes.byref(h)))
        self._h = h
        self._keep = keep

    def close(self):
        if getattr(self, "_h", None):
            lib().pgabb_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def partition(self, p, cut_mode=CUT_NNZ, cuts=None):
        if cuts is not None:
            c = np.ascontiguousarray(cuts, dtype=np.int32)
            if len(c) != p + 1:
                raise ValueError("cuts must hold p + 1 values")
            _check(lib().pgabb_partition_ex(self._h, int(p), cut_mode, ctypes.c_void_p(c.ctypes.data)))
        else:
            _check(lib().pgabb_partition_ex(self._h, int(p), cut_mode, None))
        return self

    def count(self, opts=None, **kw):
        if opts is None and kw:
            opts = options(**kw)
        c = ctypes.c_uint64()
        _check(lib().pgabb_tc_count_ex(self._h, ctypes.byref(opts) if opts is not None else None,
                                       ctypes.byref(c)))
        return int(c.value)

    def count_noalloc(self, opts=None, **kw):
        """The in-core count with its scratch in the library's fixed
        per-GPU array (pgabb_tc_count_noalloc): the graph must be
        partitioned and its blocks in device memory."""
        if opts is None and kw:
            opts = options(**kw)
        c = ctypes.c_uint64()
        _check(lib().pgabb_tc_count_noalloc(self._h, ctypes.byref(opts) if opts is not None else None,
                                            ctypes.byref(c)))
        return int(c.value)

    def count_shard(self, shard, num_shards, opts=None, **kw):
        """Triangles found by the tasks dealt to `shard` of `num_shards`."""
        if opts is None and kw:
            opts = options(**kw)
        c = ctypes.c_uint64()
        _check(lib().pgabb_tc_count_shard(self._h, ctypes.byref(opts) if opts is not None else None,
                                          int(shard), int(num_shards), ctypes.byref(c)))
        return int(c.value)

    def edge_support(self, out=None):
        """Triangles containing each oriented edge (CSR order of export_csr)
        and the triangle count.  out: None (a new numpy uint32 array), a
        numpy uint32 array or a CUDA torch int32/uint32 tensor of m'
        entries (complete when the call returns)."""
        m = self.info()["m"]
        tri = ctypes.c_uint64()
        if out is None:
            out = np.empty(m, np.uint32)
        if isinstance(out, np.ndarray):
            if out.dtype != np.uint32 or out.size != m or not out.flags.c_contiguous:
                raise ValueError("out must be a contiguous uint32 array of m' entries")
            _check(lib().pgabb_tc_edge_support(self._h, ctypes.c_void_p(out.ctypes.data) if m else None, 0,
                                               ctypes.byref(tri)))
        else:
            if out.numel() != m or out.element_size() != 4 or not out.is_contiguous() or not out.is_cuda:
                raise ValueError("out must be a contiguous 4-byte CUDA tensor of m' entries")
            import torch
            torch.cuda.current_stream().synchronize()  # torch's pending writes to out come first
            _check(lib().pgabb_tc_edge_support(self._h, ctypes.c_void_p(out.data_ptr()) if m else None,
                                               SUPPORT_ON_DEVICE, ctypes.byref(tri)))
        return out, int(tri.value)

    def vertex_counts(self, out=None):
        """Triangles at each vertex by input id, and the triangle count.
        out: None (a new numpy uint64 array), a numpy uint64 array or a CUDA
        torch int64 tensor of n entries (complete when the call returns)."""
        n = self.info()["n"]
        tri = ctypes.c_uint64()
        if out is None:
            out = np.empty(n, np.uint64)
        if isinstance(out, np.ndarray):
            if out.dtype != np.uint64 or out.size != n or not out.flags.c_contiguous:
                raise ValueError("out must be a contiguous uint64 array of n entries")
            _check(lib().pgabb_tc_vertex_counts(self._h, ctypes.c_void_p(out.ctypes.data) if n else None, 0,
                                                ctypes.byref(tri)))
        else:
            if out.numel() != n or out.element_size() != 8 or not out.is_contiguous() or not out.is_cuda:
                raise ValueError("out must be a contiguous 8-byte CUDA tensor of n entries")
            import torch
            torch.cuda.current_stream().synchronize()  # torch's pending writes to out come first
            _check(lib().pgabb_tc_vertex_counts(self._h, ctypes.c_void_p(out.data_ptr()) if n else None,
                                                SUPPORT_ON_DEVICE, ctypes.byref(tri)))
        return out, int(tri.value)

    def ktruss(self, k):
        """(keep, edges, rounds): keep is a numpy uint8 mask over the oriented
        CSR positions (export_csr order), 1 for the edges of the k-truss."""
        m = self.info()["m"]
        keep = np.empty(max(m, 1), np.uint8)
        left, rounds = ctypes.c_int64(), ctypes.c_int32()
        _check(lib().pgabb_tc_ktruss(self._h, int(k), ctypes.c_void_p(keep.ctypes.data), 0, ctypes.byref(left),
                                     ctypes.byref(rounds)))
        return keep[:m], int(left.value), int(rounds.value)

    def components(self):
        """Connected components (Shiloach-Vishkin over the blocks): a numpy
        int32 array label[v] = smallest input id in v's component, the
        number of components and the iterations run."""
        n = self.info()["n"]
        label = np.empty(n, np.int32)
        nc, it = ctypes.c_int64(), ctypes.c_int32()
        _check(lib().pgabb_components(self._h, ctypes.c_void_p(label.ctypes.data) if n else None, 0,
                                      ctypes.byref(nc), ctypes.byref(it)))
        return label, int(nc.value), int(it.value)

    def pagerank(self, damping=0.85, tol=1e-4, max_iter=20):
        """PageRank over the blocks in double precision: a numpy float64
        array of ranks by input id, the iterations run and the last
        iteration's sum of absolute changes."""
        n = self.info()["n"]
        r = np.empty(n, np.float64)
        it, err = ctypes.c_int32(), ctypes.c_double()
        _check(lib().pgabb_pagerank(self._h, float(damping), float(tol), int(max_iter),
                                    ctypes.c_void_p(r.ctypes.data) if n else None, 0, ctypes.byref(it),
                                    ctypes.byref(err)))
        return r, int(it.value), float(err.value)

    def four_clique_lists(self):
        """(ijkl int32[L, 4], counts uint64[L]) of the last 4-clique count."""
        nl = ctypes.c_int64()
        _check(lib().pgabb_graph_4list_counts(self._h, ctypes.byref(nl), None, None))
        L = nl.value
        ijkl = np.empty((max(L, 1), 4), np.int32)
        cnt = np.empty(max(L, 1), np.uint64)
        _check(lib().pgabb_graph_4list_counts(self._h, None, ctypes.c_void_p(ijkl.ctypes.data),
                                              ctypes.c_void_p(cnt.ctypes.data)))
        return ijkl[:L], cnt[:L]

    def four_cliques(self, device_cap_bytes=0):
        """Sets of four pairwise adjacent vertices; with device_cap_bytes > 0
        the blocks stream from the host store through a cache of that size."""
        c = ctypes.c_uint64()
        if device_cap_bytes:
            _check(lib().pgabb_count_4cliques_streamed(self._h, ctypes.c_uint64(int(device_cap_bytes)),
                                                       ctypes.byref(c)))
        else:
            _check(lib().pgabb_count_4cliques(self._h, ctypes.byref(c)))
        return int(c.value)

    def task_shards(self, num_shards):
        """Shard of each task (order of task_counts) for num_shards devices."""
        t = self.info()["num_tasks"]
        of = np.empty(max(t, 1), np.int32)
        _check(lib().pgabb_graph_task_shards(self._h, int(num_shards), ctypes.c_void_p(of.ctypes.data)))
        return of[:t]

    def info(self):
        i = GraphInfo()
        _check(lib().pgabb_graph_info_get(self._h, ctypes.byref(i)))
        return i.as_dict()

    def export_csr(self):
        inf = self.info()
        n, m = inf["n"], inf["m"]
        row_off = np.empty(n + 1, np.int64)
        col = np.empty(max(m, 1), np.int32)
        rank = np.empty(max(n, 1), np.int32)
        _check(lib().pgabb_graph_export_csr(self._h, ctypes.c_void_p(row_off.ctypes.data),
                                            ctypes.c_void_p(col.ctypes.data),
                                            ctypes.c_void_p(rank.ctypes.data)))
        return row_off, col[:m], rank[:n]

    def cuts(self):
        p = self.info()["p"]
        c = np.empty(p + 1, np.int32)
        _check(lib().pgabb_graph_cuts(self._h, ctypes.c_void_p(c.ctypes.data)))
        return c

    def task_counts(self):
        t = self.info()["num_tasks"]
        ijk = np.empty((max(t, 1), 3), np.int32)
        cnt = np.empty(max(t, 1), np.uint64)
        _check(lib().pgabb_graph_task_counts(self._h, ctypes.c_void_p(ijk.ctypes.data),
                                             ctypes.c_void_p(cnt.ctypes.data)))
        return ijk[:t], cnt[:t]


def graph_info(g):
    """(n, m', p, tasks) of a Graph."""
    n, m, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    p = ctypes.c_int32()
    _check(lib().pgabb_graph_info(g._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(p), ctypes.byref(t)))
    return n.value, m.value, p.value, t.value


def tc_count_batch(graphs, opts=None, **kw):
    """Counts of several Graph objects in one merged launch (no options:
    autotuned launch shape)."""
    if opts is None and kw:
        opts = options(**kw)
    hs = (ctypes.c_void_p * max(len(graphs), 1))(*[g._h for g in graphs])
    out = np.zeros(max(len(graphs), 1), np.uint64)
    _check(lib().pgabb_tc_count_batch(hs, len(graphs), ctypes.byref(opts) if opts is not None else None,
                                      ctypes.c_void_p(out.ctypes.data)))
    return [int(c) for c in out[:len(graphs)]]


def tc_count(n, src, dst, p=1, **kw):
    """Build, partition and count in one call."""
    with Graph(n, src, dst) as g:
        g.partition(p)
        return g.count(**kw) if kw else g.count()


def version():
    return lib().pgabb_version().decode()


def release_cached_memory():
    """Return the library's cached free device and pinned host blocks to HIP."""
    _check(lib().pgabb_release_cached_memory())


OPT_PER_GRAPH = 0x2
SERVER_BORROW = 0x4


class Batch:
    """Many independent graphs packed into one device arena and counted by
    one persistent, graph-captured launch."""

    def __init__(self, graphs_or_arrays, stream=None):
        """graphs_or_arrays: list of (n, src, dst) host arrays, or a tuple
        (n_array, edge_off, src, dst) already packed."""
        if isinstance(graphs_or_arrays, tuple) and len(graphs_or_arrays) == 4:
            nv, eoff, src, dst = graphs_or_arrays
            nv = np.ascontiguousarray(nv, np.int32)
            eoff = np.ascontiguousarray(eoff, np.int64)
        else:
            gl = list(graphs_or_arrays)
            nv = np.array([g[0] for g in gl], np.int32)
            eoff = np.zeros(len(gl) + 1, np.int64)
            eoff[1:] = np.cumsum([len(g[1]) for g in gl])
            src = np.concatenate([np.asarray(g[1], np.int32) for g in gl]) if gl else np.zeros(0, np.int32)
            dst = np.concatenate([np.asarray(g[2], np.int32) for g in gl]) if gl else np.zeros(0, np.int32)
        ps, pd, m, flags, keep, st = _edges(src, dst)
        if m != int(eoff[-1] if len(eoff) else 0):
            raise ValueError("edge_off[-1] must equal the number of pairs")
        if stream is not None:
            st = ctypes.c_void_p(stream)
        h = ctypes.c_void_p()
        _check(lib().pgabb_batch_create(len(nv), ctypes.c_void_p(nv.ctypes.data),
                                        ctypes.c_void_p(eoff.ctypes.data), ps, pd, flags, st,
                                        ctypes.byref(h)))
        self._h = h
        self.num_graphs = len(nv)
        self._keep = (nv, eoff, keep)

    def count(self, opts=None, per_graph=False, **kw):
        if per_graph:
            opts = options(**kw)
            opts.flags |= OPT_PER_GRAPH
        elif opts is None and kw:
            opts = options(**kw)
        out = np.zeros(max(self.num_graphs, 1), np.uint64)
        _check(lib().pgabb_batch_count(self._h, ctypes.byref(opts) if opts is not None else None,
                                       ctypes.c_void_p(out.ctypes.data)))
        return out[:self.num_graphs]

    def times(self):
        b, c = ctypes.c_double(), ctypes.c_double()
        _check(lib().pgabb_batch_times(self._h, ctypes.byref(b), ctypes.byref(c)))
        return b.value, c.value

    def launch_shape(self):
        """Kernel, waves per workgroup and rows per grab of the last
        captured count, and the time its autotuning took (ms)."""
        k, w, r, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().pgabb_batch_launch_shape(self._h, ctypes.byref(k), ctypes.byref(w), ctypes.byref(r),
                                              ctypes.byref(t)))
        return {"kernel": k.value, "waves_per_block": w.value, "rows_per_grab": r.value, "t_tune_ms": t.value}

    def stats(self):
        """Sizes of the union graph: oriented edges, active rows (the
        count's work items), their edges and the entries a count walks."""
        e, r, ae, w = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64()
        _check(lib().pgabb_batch_stats(self._h, ctypes.byref(e), ctypes.byref(r), ctypes.byref(ae), ctypes.byref(w)))
        return {"edges": e.value, "active_rows": r.value, "active_edges": ae.value, "walked": w.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().pgabb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Continuous-batching triangle-count server (host threads inside the
    library; this class only forwards calls)."""

    def __init__(self, budget_bytes, borrow=False, **kw):
        o = options(**kw)
        if borrow:
            o.flags |= SERVER_BORROW
        h = ctypes.c_void_p()
        _check(lib().pgabb_server_create(int(budget_bytes), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._borrowed = {}
        self.borrow = borrow

    def submit(self, n, src, dst):
        s = np.ascontiguousarray(src, np.int32)
        d = np.ascontiguousarray(dst, np.int32)
        t = ctypes.c_uint64()
        _check(lib().pgabb_server_submit(self._h, int(n), len(s), ctypes.c_void_p(s.ctypes.data if s.size else 0),
                                         ctypes.c_void_p(d.ctypes.data if d.size else 0), ctypes.byref(t)))
        if self.borrow:
            self._borrowed[t.value] = (s, d)
        return t.value

    def poll(self, ticket):
        """(done, count, t_submit, t_done) of a request."""
        done = ctypes.c_int32()
        cnt = ctypes.c_uint64()
        st = lib().pgabb_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(cnt))
        if done.value and self.borrow:
            self._borrowed.pop(ticket, None)
        _check(st)
        ts, td = self.times(ticket) if done.value else (0.0, 0.0)
        return bool(done.value), int(cnt.value), ts, td

    def times(self, ticket):
        """(t_submit, t_done) on the server clock; t_done is 0 while it runs."""
        ts, td = ctypes.c_double(), ctypes.c_double()
        _check(lib().pgabb_server_times(self._h, ticket, ctypes.byref(ts), ctypes.byref(td)))
        return ts.value, td.value

    def drain(self):
        _check(lib().pgabb_server_drain(self._h))

    def now(self):
        return lib().pgabb_server_now(self._h)

    def launches(self):
        v = ctypes.c_uint64()
        _check(lib().pgabb_server_stats(self._h, ctypes.byref(v)))
        return v.value

    def kernel_stats(self):
        """(kernel ms, walked entries, edges) summed over the counting
        launches so far."""
        k, w, e = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().pgabb_server_kernel_stats(self._h, ctypes.byref(k), ctypes.byref(w), ctypes.byref(e)))
        return k.value, w.value, e.value

    def close(self):
        if getattr(self, "_h", None):
            lib().pgabb_server_destroy(self._h)
            self._h = None
            self._borrowed.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
