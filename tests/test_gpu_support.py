"""GPU parity of the per-edge triangle counts (edge support) and the
per-vertex triangle counts against the CPU oracle, through the C ABI: exact
equality of every edge's count (in the CSR order both sides build), of every
vertex's count (by input id) and of the triangle count."""
import json
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2209_04541_amd as P
from paper_2209_04541_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(n, s, d, p=None):
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    want = oracle.edge_support(n, row_off, col)
    with P.Graph(n, s, d) as g:
        if p:
            g.partition(p)  # the support does not depend on the partition
        r, c, _ = g.export_csr()
        assert np.array_equal(r, row_off) and np.array_equal(c, col)
        got, tri = g.edge_support()
        info = g.info()
    assert np.array_equal(got, want)
    assert tri * 3 == int(want.sum(dtype=np.uint64))
    return got, tri, info


@pytest.mark.parametrize("name,g,expected", graphs.closed_forms(), ids=lambda x: x if isinstance(x, str) else "")
def test_closed_forms(name, g, expected):
    n, s, d = g
    say("support closed form", name)
    _, tri, _ = check(*graphs.messy(n, s, d, seed=3))
    assert tri == expected


@pytest.mark.parametrize("seed", range(8))
def test_random_small(seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(1, 90))
    m = int(rng.integers(0, 3 * n * n // 2 + 1))
    s = rng.integers(0, n, size=m).astype(np.int32)
    d = rng.integers(0, n, size=m).astype(np.int32)
    say("support random", seed, n, m)
    check(n, s, d, p=min(3, n))


@pytest.mark.parametrize("kind", ["rmat", "er", "rgg"])
def test_generated_graphs(kind):
    if kind == "rmat":
        n, s, d = gen.rmat(15, 16, gen.seed(61, 0))
    elif kind == "er":
        n, s, d = gen.er(20000, 300000, gen.seed(61, 1))
    else:
        n, s, d = gen.rgg(20000, 24.0, gen.seed(61, 2))
    say("support", kind, n, len(s))
    _, tri, info = check(n, s, d, p=4)
    assert tri == oracle.tc(n, s, d)
    assert info["kernel_launches"] == 1


def test_rows_longer_than_the_lds_region():
    """K_1500 plus a pendant clique: rows above 1024 entries are searched and
    counted in device memory, shorter ones in LDS."""
    n1 = 1500
    a, b = np.triu_indices(n1, 1)
    c, e = np.triu_indices(40, 1)
    s = np.concatenate([a, c + n1, [0, 5]]).astype(np.int32)
    d = np.concatenate([b, e + n1, [n1, n1 + 3]]).astype(np.int32)
    got, tri, _ = check(n1 + 40, s, d)
    assert tri == n1 * (n1 - 1) * (n1 - 2) // 6 + 40 * 39 * 38 // 6
    assert got.max() == n1 - 2


def test_device_output_and_repeat():
    import torch
    n, s, d = gen.rmat(13, 16, gen.seed(62, 0))
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    want = oracle.edge_support(n, row_off, col)
    with P.Graph(n, s, d) as g:
        out = torch.full((len(col),), 7, dtype=torch.int32, device="cuda")  # cleared by the call
        for _ in range(2):
            _, tri = g.edge_support(out)
            assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
        assert tri == oracle.count_csr(n, row_off, col)
        with pytest.raises(ValueError):
            g.edge_support(np.empty(len(col) + 1, np.uint32))
        # the count is unaffected by a support call before or after
        assert g.count() == tri


def test_empty_and_edgeless():
    for n in (0, 1, 7):
        with P.Graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32)) as g:
            got, tri = g.edge_support()
            assert got.size == 0 and tri == 0
    with P.Graph(4, np.array([0, 1], np.int32), np.array([1, 2], np.int32)) as g:
        got, tri = g.edge_support()
        assert tri == 0 and np.array_equal(got, np.zeros(2, np.uint32))


def test_block_workload_full_size():
    """R-MAT scale 20: the sum matches three times the stored count, and
    sampled edges match their common-neighbour counts computed here from
    the oracle's CSR."""
    with open(os.path.join(GOLDEN, "workload_counts.json")) as f:
        gold = json.load(f)["block"]
    n, s, d = gen.block_graph()
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    with P.Graph(n, s, d) as g:
        g.partition(8)
        got, tri = g.edge_support()
    assert tri == gold["triangles"]
    assert int(got.sum(dtype=np.uint64)) == 3 * gold["triangles"]
    m = len(col)
    U = sp.csr_matrix((np.ones(m, np.int8), col, row_off), shape=(n, n))
    A = (U + U.T).tocsr()
    rows = np.repeat(np.arange(n), np.diff(row_off))
    rng = np.random.default_rng(5)
    for e in rng.integers(0, m, size=3000):
        x, y = rows[e], col[e]
        nx_ = A.indices[A.indptr[x]:A.indptr[x + 1]]
        ny_ = A.indices[A.indptr[y]:A.indptr[y + 1]]
        assert got[e] == len(np.intersect1d(nx_, ny_, assume_unique=True)), e


# ---------------------------------------------------------------- vertex counts

def check_vertices(n, s, d):
    want = oracle.vertex_counts(n, s, d)
    with P.Graph(n, s, d) as g:
        got, tri = g.vertex_counts()
    assert np.array_equal(got, want)
    assert 3 * tri == int(want.sum())
    return got, tri


@pytest.mark.parametrize("name,g,expected", graphs.closed_forms(), ids=lambda x: x if isinstance(x, str) else "")
def test_vertex_counts_closed_forms(name, g, expected):
    n, s, d = g
    _, tri = check_vertices(*graphs.messy(n, s, d, seed=4))
    assert tri == expected


@pytest.mark.parametrize("kind", ["random", "rmat", "rgg", "k1500"])
def test_vertex_counts_graphs(kind):
    if kind == "random":
        rng = np.random.default_rng(77)
        n = 70
        s = rng.integers(0, n, 900).astype(np.int32)
        d = rng.integers(0, n, 900).astype(np.int32)
    elif kind == "rmat":
        n, s, d = gen.rmat(15, 16, gen.seed(63, 0))
    elif kind == "rgg":
        n, s, d = gen.rgg(30000, 20.0, gen.seed(63, 1))
    else:
        n = 1500
        s, d = np.triu_indices(n, 1)
        s, d = s.astype(np.int32), d.astype(np.int32)
    say("vertex counts", kind, n, len(s))
    got, _ = check_vertices(n, s, d)
    if kind == "k1500":
        assert set(got.tolist()) == {1499 * 1498 // 2}


def test_vertex_counts_device_output_and_edge_cases():
    import torch
    n, s, d = gen.rmat(12, 16, gen.seed(64, 0))
    want = oracle.vertex_counts(n, s, d)
    with P.Graph(n, s, d) as g:
        out = torch.full((n,), 5, dtype=torch.int64, device="cuda")
        _, tri = g.vertex_counts(out)
        assert np.array_equal(out.cpu().numpy().view(np.uint64), want)
        with pytest.raises(ValueError):
            g.vertex_counts(np.empty(n + 1, np.uint64))
    for n in (0, 6):
        with P.Graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32)) as g:
            got, tri = g.vertex_counts()
            assert got.size == n and tri == 0 and not got.any()


# ---------------------------------------------------------------- k-truss

def check_truss(n, s, d, k):
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    want = oracle.ktruss(n, row_off, col, k)
    with P.Graph(n, s, d) as g:
        keep, left, rounds = g.ktruss(k)
        info = g.info()
    assert np.array_equal(keep, want), k
    assert left == int(want.sum())
    assert info["kernel_launches"] == rounds
    return left, rounds


@pytest.mark.parametrize("name,g,expected", graphs.closed_forms(), ids=lambda x: x if isinstance(x, str) else "")
def test_ktruss_closed_forms(name, g, expected):
    n, s, d = graphs.messy(*g, seed=6)
    for k in (0, 2, 3, 4, 5):
        check_truss(n, s, d, k)


@pytest.mark.parametrize("kind", ["random", "rmat", "rgg"])
def test_ktruss_graphs(kind):
    if kind == "random":
        rng = np.random.default_rng(91)
        n = 80
        s = rng.integers(0, n, 1500).astype(np.int32)
        d = rng.integers(0, n, 1500).astype(np.int32)
    elif kind == "rmat":
        n, s, d = gen.rmat(14, 16, gen.seed(65, 0))
    else:
        n, s, d = gen.rgg(20000, 20.0, gen.seed(65, 1))
    for k in (3, 4, 6, 9, 14, 25):
        left, rounds = check_truss(n, s, d, k)
        say("k-truss", kind, k, left, rounds)


def test_ktruss_cliques():
    """K_300 plus a pendant K_12: the 300-truss is the large clique, the
    301-truss is empty, the 12-truss holds both cliques."""
    a, b = np.triu_indices(300, 1)
    c, e = np.triu_indices(12, 1)
    s = np.concatenate([a, c + 300, [0]]).astype(np.int32)
    d = np.concatenate([b, e + 300, [300]]).astype(np.int32)
    n = 312
    assert check_truss(n, s, d, 300)[0] == 300 * 299 // 2
    assert check_truss(n, s, d, 301)[0] == 0
    assert check_truss(n, s, d, 12)[0] == 300 * 299 // 2 + 66
    with P.Graph(5, np.zeros(0, np.int32), np.zeros(0, np.int32)) as g:
        keep, left, rounds = g.ktruss(3)
        assert keep.size == 0 and left == 0 and rounds == 0
