"""Seeded synthetic edge-list generators shared by the library's callers and
the CPU oracle's tests.

This module only draws raw (src, dst) int32 pairs; it holds none of the
triangle-counting arithmetic (no cleaning, ordering, orientation, blocking or
counting).  The heavy lifting is plain C (``gen.c``, built with gcc into
``libpgabb_gen.so``), driven by one counter-based SplitMix64 stream so every
input is reproducible from ``(config_id, index)``.

Workload recipes (the paper's 44 real graphs are not available; these stand
in for them: R-MAT for the skewed social/web/Kronecker class, the random
geometric graph for spatial high-clustering graphs, Erdos-Renyi as the
unclustered control):

* ``plain``   ER G(n=4096, m=32768), seed (1, 0)
* ``block``   R-MAT scale 20, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed (2, 0)
* ``ooc``     R-MAT scale 24, edge factor 16, same quadrants, seed (3, 0)
* ``batch``   graph g of 10,000, seed (4, g): even g random geometric, odd g
              Erdos-Renyi, n ~ U{64..8192}, average degree d ~ U{8..64}
* ``served``  request r: scale ~ U{10..22}, edge factor ~ U{8..32}, seed (5, r)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
LIB_PATH = os.path.join(_HERE, "libpgabb_gen.so")

RMAT_ABC = (0.57, 0.19, 0.19)

_lib = None


def build(force: bool = False) -> str:
    """Compile gen.c with gcc (plain C, OpenMP) into libpgabb_gen.so."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
            "-std=gnu99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.pgabb_gen_seed.restype = ctypes.c_uint64
        lib.pgabb_gen_seed.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.pgabb_gen_rmat.restype = ctypes.c_int
        lib.pgabb_gen_rmat.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       i32p, i32p]
        lib.pgabb_gen_er_num_edges.restype = ctypes.c_int64
        lib.pgabb_gen_er_num_edges.argtypes = [ctypes.c_int32, ctypes.c_int64]
        lib.pgabb_gen_er.restype = ctypes.c_int
        lib.pgabb_gen_er.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64, i32p, i32p]
        lib.pgabb_gen_rgg.restype = ctypes.c_int64
        lib.pgabb_gen_rgg.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_double,
                                      i32p, i32p, ctypes.c_int64]
        lib.pgabb_gen_uniform_int.restype = ctypes.c_int64
        lib.pgabb_gen_uniform_int.argtypes = [ctypes.c_uint64, ctypes.c_uint64,
                                              ctypes.c_int64, ctypes.c_int64]
        lib.pgabb_gen_unit.restype = ctypes.c_double
        lib.pgabb_gen_unit.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def seed(config_id: int, index: int) -> int:
    """SplitMix64 finaliser of (config_id << 32 | index)."""
    return int(_load().pgabb_gen_seed(config_id, index))


def rmat(scale: int, edge_factor: int, seed_value: int, abc=RMAT_ABC):
    """ef * 2^scale directed R-MAT samples; returns (n, src, dst)."""
    m = int(edge_factor) << int(scale)
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = _load().pgabb_gen_rmat(seed_value, scale, m, abc[0], abc[1], abc[2], _ptr(src), _ptr(dst))
    if rc != 0:
        raise ValueError("bad R-MAT parameters")
    return 1 << scale, src, dst


def er(n: int, m: int, seed_value: int):
    """Erdos-Renyi G(n, m): exactly min(m, C(n,2)) distinct non-loop pairs."""
    lib = _load()
    k = int(lib.pgabb_gen_er_num_edges(n, m))
    src = np.empty(k, dtype=np.int32)
    dst = np.empty(k, dtype=np.int32)
    if k:
        rc = lib.pgabb_gen_er(seed_value, n, m, _ptr(src), _ptr(dst))
        if rc != 0:
            raise MemoryError("ER generation failed")
    return n, src, dst


def rgg_radius(n: int, avg_degree: float) -> float:
    """Radius whose disc holds avg_degree of the other n-1 points on average
    (ignoring the square's boundary), capped at sqrt(2) (complete graph)."""
    if n < 2:
        return 0.0
    return min(math.sqrt(avg_degree / (math.pi * (n - 1))), math.sqrt(2.0))


def rgg(n: int, avg_degree: float, seed_value: int):
    """Random geometric graph in the unit square (no wrap)."""
    lib = _load()
    r = rgg_radius(n, avg_degree)
    cnt = int(lib.pgabb_gen_rgg(seed_value, n, r, None, None, 0))
    if cnt < 0:
        raise ValueError("RGG generation failed")
    src = np.empty(cnt, dtype=np.int32)
    dst = np.empty(cnt, dtype=np.int32)
    got = int(lib.pgabb_gen_rgg(seed_value, n, r, _ptr(src), _ptr(dst), cnt))
    assert got == cnt
    return n, src, dst


def uniform_int(seed_value: int, ctr: int, lo: int, hi: int) -> int:
    """Integer uniform in [lo, hi] from draw `ctr` of the stream."""
    return int(_load().pgabb_gen_uniform_int(seed_value, ctr, lo, hi))


def unit(seed_value: int, ctr: int) -> float:
    """Double uniform in [0, 1) from draw `ctr` of the stream."""
    return float(_load().pgabb_gen_unit(seed_value, ctr))


# ------------------------------------------------------------ workloads

def plain_graph():
    """ER G(n=4096, m=32768), seed (1, 0)."""
    return er(4096, 32768, seed(1, 0))


def block_graph(scale: int = 20, edge_factor: int = 16):
    """R-MAT scale 20, edge factor 16, seed (2, 0)."""
    return rmat(scale, edge_factor, seed(2, 0))


def ooc_graph(scale: int = 24, edge_factor: int = 16):
    """R-MAT scale 24, edge factor 16, seed (3, 0)."""
    return rmat(scale, edge_factor, seed(3, 0))


# Parameters of batch graph g come from a side stream so the graph's own
# stream (seed (4, g)) is used only for its edges.
_PARAM_KEY = 0x5EED5EED5EED5EED


def batch_params(g: int, n_range=(64, 8192), d_range=(8, 64)):
    """(family, n, d) of batch graph g: family 'rgg' for even g, 'er' for odd g."""
    s = seed(4, g) ^ _PARAM_KEY
    n = uniform_int(s, 0, n_range[0], n_range[1])
    d = uniform_int(s, 1, d_range[0], d_range[1])
    return ("rgg" if g % 2 == 0 else "er"), n, d


def batch_graph(g: int, n_range=(64, 8192), d_range=(8, 64)):
    """Batch graph g: random geometric (even g) or Erdos-Renyi (odd g)."""
    fam, n, d = batch_params(g, n_range, d_range)
    if fam == "rgg":
        return rgg(n, d, seed(4, g))
    m = min(int(round(n * d / 2.0)), n * (n - 1) // 2)
    return er(n, m, seed(4, g))


def served_params(r: int, scale_range=(10, 22), ef_range=(8, 32)):
    """(scale, edge_factor) of request r."""
    s = seed(5, r) ^ _PARAM_KEY
    return uniform_int(s, 0, *scale_range), uniform_int(s, 1, *ef_range)


def served_graph(r: int, scale_range=(10, 22), ef_range=(8, 32)):
    sc, ef = served_params(r, scale_range, ef_range)
    return rmat(sc, ef, seed(5, r))


def poisson_arrivals(rate_per_s: float, duration_s: float, seed_value: int):
    """Arrival times (seconds) of a Poisson process: exponential gaps
    -ln(1-U)/rate from the stream's draws."""
    out = []
    t = 0.0
    k = 0
    while True:
        t += -math.log(1.0 - unit(seed_value, k)) / rate_per_s
        k += 1
        if t >= duration_s:
            break
        out.append(t)
    return np.asarray(out, dtype=np.float64)
