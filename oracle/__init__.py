"""CPU oracle for triangle counting -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The library under test never does, and
this package imports nothing from it: the two share no code.

``tc_oracle.c`` (plain C, gcc, optional OpenMP over rows for the final sum)
computes the triangle count of an undirected graph by its plain definition in
the oriented form the paper uses (PGAbB Section 3.6 for the problem and the
per-edge common-neighbour count over a block-list, Section 5.1 for cleaning,
Section 5.4 for degree ordering and the oriented half of the edges), and the
triangles containing each edge (edge support) and each vertex.
``bsp_oracle.c`` computes the two single-block bulk-synchronous examples
(Section 3.2): connected components by their definition (Section 3.4) and
PageRank by its iteration (Section 5.2).  This module is a thin ctypes wrapper
around both.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tc_oracle.c")
_SRC_BSP = os.path.join(_HERE, "bsp_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle_tc.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile tc_oracle.c and bsp_oracle.c with gcc into liboracle_tc.so."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu99",
                               "-ffp-contract=off", _SRC, _SRC_BSP, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.oracle_clean.restype = ctypes.c_int64
        L.oracle_clean.argtypes = [ctypes.c_int32, ctypes.c_int64, vp, vp, vp]
        L.oracle_degrees.restype = None
        L.oracle_degrees.argtypes = [ctypes.c_int32, vp, ctypes.c_int64, vp]
        L.oracle_rank.restype = None
        L.oracle_rank.argtypes = [ctypes.c_int32, vp, ctypes.c_int, vp]
        L.oracle_orient.restype = None
        L.oracle_orient.argtypes = [ctypes.c_int32, vp, ctypes.c_int64, vp, vp, vp]
        L.oracle_count.restype = ctypes.c_uint64
        L.oracle_count.argtypes = [ctypes.c_int32, vp, vp]
        L.oracle_block_counts.restype = ctypes.c_int
        L.oracle_block_counts.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp]
        L.oracle_four_clique_blocks.restype = ctypes.c_int
        L.oracle_four_clique_blocks.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp]
        L.oracle_tc.restype = ctypes.c_uint64
        L.oracle_tc.argtypes = [ctypes.c_int32, ctypes.c_int64, vp, vp, ctypes.c_int, vp]
        L.oracle_probe_work.restype = ctypes.c_uint64
        L.oracle_probe_work.argtypes = [ctypes.c_int32, vp, vp]
        L.oracle_probe_work_col.restype = ctypes.c_uint64
        L.oracle_probe_work_col.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp]
        L.oracle_edge_support.restype = None
        L.oracle_edge_support.argtypes = [ctypes.c_int32, vp, vp, vp]
        L.oracle_vertex_counts.restype = None
        L.oracle_vertex_counts.argtypes = [ctypes.c_int32, vp, vp, vp]
        L.oracle_ktruss.restype = ctypes.c_int64
        L.oracle_ktruss.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp]
        L.oracle_four_cliques.restype = ctypes.c_uint64
        L.oracle_four_cliques.argtypes = [ctypes.c_int32, vp, vp]
        L.oracle_components.restype = ctypes.c_int64
        L.oracle_components.argtypes = [ctypes.c_int32, vp, ctypes.c_int64, vp]
        L.oracle_pagerank.restype = ctypes.c_int32
        L.oracle_pagerank.argtypes = [ctypes.c_int32, vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int32, vp, vp]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_set_threads.restype = None
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _edges(src, dst):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    return src, dst


def threads() -> int:
    return int(_load().oracle_threads())


def set_threads(t: int) -> None:
    _load().oracle_set_threads(int(t))


def clean(n: int, src, dst) -> np.ndarray:
    """Sorted distinct canonical keys (min << 32 | max) as uint64."""
    src, dst = _edges(src, dst)
    keys = np.empty(max(len(src), 1), dtype=np.uint64)
    mu = _load().oracle_clean(n, len(src), _p(src), _p(dst), _p(keys))
    if mu < 0:
        raise ValueError("vertex id out of range")
    return keys[:mu].copy()


def degrees(n: int, keys: np.ndarray) -> np.ndarray:
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    deg = np.empty(max(n, 1), dtype=np.int32)
    _load().oracle_degrees(n, _p(keys), len(keys), _p(deg))
    return deg[:n]


def rank(n: int, deg: np.ndarray, mode: int = 0) -> np.ndarray:
    """mode 0: ascending (degree, id); mode 1: identity."""
    deg = np.ascontiguousarray(deg, dtype=np.int32)
    r = np.empty(max(n, 1), dtype=np.int32)
    _load().oracle_rank(n, _p(deg), mode, _p(r))
    return r[:n]


def orient(n: int, keys: np.ndarray, rnk: np.ndarray):
    """Oriented CSR (row_off int64[n+1], col int32[m']) over ranked ids."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    rnk = np.ascontiguousarray(rnk, dtype=np.int32)
    row_off = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(len(keys), 1), dtype=np.int32)
    _load().oracle_orient(n, _p(keys), len(keys), _p(rnk), _p(row_off), _p(col))
    return row_off, col[:len(keys)]


def count_csr(n: int, row_off: np.ndarray, col: np.ndarray) -> int:
    row_off = np.ascontiguousarray(row_off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if len(col) == 0:
        col = np.zeros(1, dtype=np.int32)
    return int(_load().oracle_count(n, _p(row_off), _p(col)))


def edge_support(n: int, row_off: np.ndarray, col: np.ndarray) -> np.ndarray:
    """uint32 triangles containing each oriented edge, in CSR order."""
    row_off = np.ascontiguousarray(row_off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    m = int(row_off[n]) if n > 0 else 0
    out = np.zeros(max(m, 1), dtype=np.uint32)
    if m:
        _load().oracle_edge_support(n, _p(row_off), _p(col), _p(out))
    return out[:m]


def vertex_counts(n: int, src, dst, mode: int = 0) -> np.ndarray:
    """uint64 triangles at each vertex, indexed by input id."""
    _, _, rnk, row_off, col = oriented_csr(n, src, dst, mode)
    t = np.zeros(max(n, 1), dtype=np.uint64)
    if n > 0:
        c = col if len(col) else np.zeros(1, dtype=np.int32)
        _load().oracle_vertex_counts(n, _p(row_off), _p(np.ascontiguousarray(c, dtype=np.int32)), _p(t))
    return t[:n][rnk] if n > 0 else t[:0]


def ktruss(n: int, row_off: np.ndarray, col: np.ndarray, k: int) -> np.ndarray:
    """uint8 mask over the oriented CSR positions: 1 for the edges of the
    k-truss."""
    row_off = np.ascontiguousarray(row_off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    m = int(row_off[n]) if n > 0 else 0
    keep = np.zeros(max(m, 1), dtype=np.uint8)
    if m:
        _load().oracle_ktruss(n, _p(row_off), _p(col), int(k), _p(keep))
    return keep[:m]


def four_cliques(n: int, src, dst, mode: int = 0) -> int:
    """Sets of four pairwise adjacent vertices."""
    _, _, _, row_off, col = oriented_csr(n, src, dst, mode)
    if n == 0 or len(col) == 0:
        return 0
    return int(_load().oracle_four_cliques(n, _p(row_off), _p(np.ascontiguousarray(col, dtype=np.int32))))


def four_clique_blocks(n: int, row_off: np.ndarray, col: np.ndarray, cuts) -> np.ndarray:
    """Q[i, j, k, l] = 4-cliques whose ranked vertices lie in stripes
    i <= j <= k <= l."""
    cuts = np.ascontiguousarray(cuts, dtype=np.int32)
    p = len(cuts) - 1
    row_off = np.ascontiguousarray(row_off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if len(col) == 0:
        col = np.zeros(1, dtype=np.int32)
    out = np.zeros(p ** 4, dtype=np.uint64)
    rc = _load().oracle_four_clique_blocks(n, _p(row_off), _p(col), p, _p(cuts), _p(out))
    if rc != 0:
        raise ValueError("bad cut vector")
    return out.reshape(p, p, p, p)


def probe_work(n: int, row_off: np.ndarray, col: np.ndarray) -> int:
    row_off = np.ascontiguousarray(row_off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if len(col) == 0:
        col = np.zeros(1, dtype=np.int32)
    return int(_load().oracle_probe_work(n, _p(row_off), _p(col)))


def probe_work_col(n: int, row_off: np.ndarray, col: np.ndarray, cuts) -> int:
    """W_col: over oriented edges (x, y), the out-neighbours w of x with
    stripe(w) >= stripe(y) (the entries a walk of the first endpoint's
    partial lists reads)."""
    cuts = np.ascontiguousarray(cuts, dtype=np.int32)
    row_off = np.ascontiguousarray(row_off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if len(col) == 0:
        col = np.zeros(1, dtype=np.int32)
    return int(_load().oracle_probe_work_col(n, _p(row_off), _p(col), len(cuts) - 1, _p(cuts)))


def block_counts(n: int, row_off: np.ndarray, col: np.ndarray, cuts) -> np.ndarray:
    """T[i, j, k] = triangles whose ranked vertices lie in stripes i <= j <= k."""
    cuts = np.ascontiguousarray(cuts, dtype=np.int32)
    p = len(cuts) - 1
    row_off = np.ascontiguousarray(row_off, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    if len(col) == 0:
        col = np.zeros(1, dtype=np.int32)
    out = np.zeros(p * p * p, dtype=np.uint64)
    rc = _load().oracle_block_counts(n, _p(row_off), _p(col), p, _p(cuts), _p(out))
    if rc != 0:
        raise ValueError("bad cut vector")
    return out.reshape(p, p, p)


def oriented_csr(n: int, src, dst, mode: int = 0):
    """(keys, deg, rank, row_off, col) of the cleaned, ranked, oriented graph."""
    keys = clean(n, src, dst)
    deg = degrees(n, keys)
    rnk = rank(n, deg, mode)
    row_off, col = orient(n, keys, rnk)
    return keys, deg, rnk, row_off, col


def tc(n: int, src, dst, mode: int = 0) -> int:
    """Triangle count of the undirected simple graph behind (src, dst)."""
    src, dst = _edges(src, dst)
    if n < 0:
        raise ValueError("n < 0")
    mu = ctypes.c_int64(0)
    s = src if len(src) else np.zeros(1, dtype=np.int32)
    d = dst if len(dst) else np.zeros(1, dtype=np.int32)
    t = _load().oracle_tc(n, len(src), _p(s), _p(d), mode, ctypes.byref(mu))
    if t == 2**64 - 1:
        raise ValueError("vertex id out of range")
    return int(t)


def components(n: int, src, dst):
    """(label, count): label[v] = smallest vertex id reachable from v."""
    keys = clean(n, src, dst)
    lab = np.empty(max(n, 1), dtype=np.int32)
    k = np.ascontiguousarray(keys if len(keys) else np.zeros(1, np.uint64))
    c = _load().oracle_components(n, _p(k), len(keys), _p(lab))
    if c < 0:
        raise MemoryError("oracle_components")
    return lab[:n], int(c)


def pagerank(n: int, src, dst, damping: float = 0.85, tol: float = 1e-4, max_iter: int = 20):
    """(ranks float64[n], iterations, last error) of the PageRank iteration
    on the undirected graph behind (src, dst)."""
    keys = clean(n, src, dst)
    r = np.empty(max(n, 1), dtype=np.float64)
    k = np.ascontiguousarray(keys if len(keys) else np.zeros(1, np.uint64))
    err = ctypes.c_double()
    it = _load().oracle_pagerank(n, _p(k), len(keys), float(damping), float(tol), int(max_iter), _p(r),
                                 ctypes.byref(err))
    if it < 0:
        raise MemoryError("oracle_pagerank")
    return r[:n], int(it), float(err.value)
