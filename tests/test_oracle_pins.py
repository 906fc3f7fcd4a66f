"""Pins of the CPU oracle against results fixed by mathematics or computed by
independent software: brute force on tiny graphs, closed forms, networkx,
the sparse and dense matrix identities T = sum(A o A^2) / 6, and invariances.

The oracle follows PGAbB Section 3.6 (problem and per-edge common-neighbour
count over a block-list), Section 5.1 (undirected, deduplicated inputs) and
Section 5.4 (degree ordering, oriented half of the edges).
"""
import itertools
import json
import math
import os

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st

import oracle
from paper_2209_04541_amd import gen
from tests import graphs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def nx_count(n, src, dst):
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(src, dst) if a != b)
    return sum(nx.triangles(G).values()) // 3


def sparse_identity(n, src, dst):
    """T = sum(A o (A @ A)) / 6 with scipy sparse integer matrices."""
    keep = src != dst
    s = np.concatenate([src[keep], dst[keep]]).astype(np.int64)
    d = np.concatenate([dst[keep], src[keep]]).astype(np.int64)
    A = sp.coo_matrix((np.ones(len(s), np.int64), (s, d)), shape=(n, n)).tocsr()
    A.data[:] = 1  # duplicates summed above; make it 0/1
    A.sum_duplicates()
    A.data[:] = 1
    return int((A.multiply(A @ A)).sum()) // 6


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("name,g,expected", graphs.closed_forms(), ids=lambda x: x if isinstance(x, str) else "")
def test_closed_forms(name, g, expected):
    n, s, d = g
    assert oracle.tc(n, s, d) == expected
    assert oracle.tc(n, s, d, mode=1) == expected
    n2, s2, d2 = graphs.messy(n, s, d, seed=len(name))
    assert oracle.tc(n2, s2, d2) == expected


def test_closed_form_helpers_are_right():
    # the helper graphs themselves, checked by brute force where small
    for name, (n, s, d), expected in graphs.closed_forms():
        if n <= 40:
            assert graphs.brute_force(n, s, d) == expected, name


# ------------------------------------------------------------- brute force

@settings(max_examples=60, deadline=None)
@given(st.integers(0, 40), st.floats(0.0, 1.0), st.integers(0, 2**31 - 1))
def test_brute_force_random(n, density, seed):
    rng = np.random.default_rng(seed)
    m = int(density * n * n)
    s = rng.integers(0, max(n, 1), size=m).astype(np.int32) if n else np.zeros(0, np.int32)
    d = rng.integers(0, max(n, 1), size=m).astype(np.int32) if n else np.zeros(0, np.int32)
    want = graphs.brute_force(n, s, d)
    assert oracle.tc(n, s, d) == want
    assert oracle.tc(n, s, d, mode=1) == want


# ----------------------------------------------------------- library pins

@pytest.mark.parametrize("kind", ["er", "rgg", "rmat"])
def test_networkx_and_sparse(kind):
    if kind == "er":
        n, s, d = gen.er(700, 9000, gen.seed(90, 1))
    elif kind == "rgg":
        n, s, d = gen.rgg(900, 30, gen.seed(90, 2))
    else:
        n, s, d = gen.rmat(11, 16, gen.seed(90, 3))
    t = oracle.tc(n, s, d)
    assert t == nx_count(n, s, d)
    assert t == sparse_identity(n, s, d)


def test_plain_workload_dense_identity():
    """ER G(4096, 32768): dense A @ A in float32 is exact (entries <= 4096 <
    2^24), so sum(A o A^2) / 6 is the exact count."""
    n, s, d = gen.plain_graph()
    A = np.zeros((n, n), dtype=np.float32)
    A[s, d] = 1
    A[d, s] = 1
    np.fill_diagonal(A, 0)
    A2 = A @ A
    t_dense = int(np.rint((A.astype(np.float64) * A2).sum())) // 6
    t = oracle.tc(n, s, d)
    assert t == t_dense
    assert t == nx_count(n, s, d)
    with open(os.path.join(GOLDEN, "workload_counts.json")) as f:
        gold = json.load(f)
    assert gold["plain"]["triangles"] == t


# ---------------------------------------------------------- the steps

def test_clean_degrees_rank_against_numpy():
    n, s, d = graphs.messy(*gen.rmat(10, 8, gen.seed(91, 0)), seed=3)
    keys = oracle.clean(n, s, d)
    lo = np.minimum(s, d).astype(np.uint64)
    hi = np.maximum(s, d).astype(np.uint64)
    keep = s != d
    want = np.unique((lo[keep] << np.uint64(32)) | hi[keep])
    assert np.array_equal(keys, want)
    deg = oracle.degrees(n, keys)
    ends = np.concatenate([(want >> np.uint64(32)).astype(np.int64), (want & np.uint64(0xFFFFFFFF)).astype(np.int64)])
    assert np.array_equal(deg, np.bincount(ends, minlength=n))
    rk = oracle.rank(n, deg, 0)
    order = np.lexsort((np.arange(n), deg))  # ascending degree, then id
    want_rank = np.empty(n, np.int64)
    want_rank[order] = np.arange(n)
    assert np.array_equal(rk, want_rank)
    assert np.array_equal(oracle.rank(n, deg, 1), np.arange(n))


def test_orient_properties():
    n, s, d = gen.rmat(12, 16, gen.seed(91, 1))
    keys, deg, rk, row_off, col = oracle.oriented_csr(n, s, d)
    assert row_off[0] == 0 and row_off[-1] == len(keys) == len(col)
    rows = np.repeat(np.arange(n), np.diff(row_off))
    assert np.all(col > rows)  # oriented low rank -> high rank
    for x in range(n):  # each row strictly increasing
        seg = col[row_off[x]:row_off[x + 1]]
        assert np.all(np.diff(seg) > 0)
    # same undirected edge set, in rank space
    inv = np.empty(n, np.int64)
    inv[rk] = np.arange(n)
    a, b = inv[rows], inv[col]
    got = np.sort((np.minimum(a, b).astype(np.uint64) << np.uint64(32)) | np.maximum(a, b).astype(np.uint64))
    assert np.array_equal(got, keys)
    # degree ordering bounds every out-degree by sqrt(2 m')
    assert np.diff(row_off).max() <= math.isqrt(2 * len(keys)) + 1


def _W(n, s, d):
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    return oracle.probe_work(n, row_off, col)


def test_probe_work_closed_forms():
    """W = sum over oriented edges (x, y) of |N+(y)| counts the directed
    two-step paths x -> y -> z of the oriented graph.
    K_n: ranks follow ids, so every a < b < c is one such path: C(n, 3).
    Star K_{1,k} (k >= 2): leaves rank below the hub, whose out-list is
    empty: 0.  Wheel (hub + rim of r = n - 1 >= 4): the rim ranks by id below
    the hub; rim vertex 1 has out-list {2, r, hub}, rim vertices 2 .. r - 1
    {next, hub}, r {hub}; the rim edges (v, v + 1) land on out-lists of 2
    (r - 2 times) and 1 (once), edge (1, r) on 1, the spokes on the empty
    hub: 2 (r - 2) + 2 = 2 n - 4.  Disjoint unions add."""
    for n in (1, 2, 3, 4, 7, 30):
        (nn, s, d), _ = graphs.complete(n)
        assert _W(nn, s, d) == math.comb(n, 3), n
    for k in (2, 5, 40):
        (nn, s, d), _ = graphs.star(k)
        assert _W(nn, s, d) == 0, k
    for n in (5, 6, 11, 50):
        (nn, s, d), _ = graphs.wheel(n)
        assert _W(nn, s, d) == 2 * n - 4, n
    parts = [graphs.complete(9)[0], graphs.wheel(12)[0], graphs.star(6)[0]]
    (nu, su, du), _ = graphs.disjoint_union(*[(g, 0) for g in parts])
    assert _W(nu, su, du) == math.comb(9, 3) + (2 * 12 - 4) + 0


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 40), st.floats(0.0, 1.0), st.integers(0, 2**31 - 1))
def test_probe_work_counts_two_paths(n, dens, sd):
    """Against the dense count of two-step paths: sum of (A A) over the
    oriented adjacency matrix A (built here from the oriented CSR rows)."""
    rng = np.random.default_rng(sd)
    m = int(dens * n * n)
    s = rng.integers(0, n, m).astype(np.int32)
    d = rng.integers(0, n, m).astype(np.int32)
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    A = np.zeros((n, n), np.int64)
    for x in range(n):
        A[x, col[row_off[x]:row_off[x + 1]]] = 1
    assert oracle.probe_work(n, row_off, col) == int((A @ A).sum())


def test_probe_work_against_numpy():
    n, s, d = gen.rmat(11, 8, gen.seed(91, 2))
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    od = np.diff(row_off)
    assert oracle.probe_work(n, row_off, col) == int(od[col].sum())


def test_probe_work_col_pins():
    """W_col: p = 1 gives the sum of squared out-degrees; one stripe per
    vertex gives sum d(d+1)/2 (the i-th smallest out-neighbour of x has
    d - i entries at or above it); random cuts against a numpy count."""
    n, s, d = gen.rmat(10, 8, gen.seed(91, 3))
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    od = np.diff(row_off).astype(np.int64)
    assert oracle.probe_work_col(n, row_off, col, [0, n]) == int((od * od).sum())
    assert oracle.probe_work_col(n, row_off, col, np.arange(n + 1)) == int((od * (od + 1) // 2).sum())
    rng = np.random.default_rng(5)
    for p in (2, 3, 7):
        cuts = np.concatenate([[0], np.sort(rng.integers(0, n + 1, p - 1)), [n]])
        stripe = np.minimum(np.searchsorted(cuts, np.arange(n), side="right") - 1, p - 1)
        want = 0
        for x in range(n):
            st = stripe[col[row_off[x]:row_off[x + 1]]]
            want += int((st[None, :] >= st[:, None]).sum())
        assert oracle.probe_work_col(n, row_off, col, cuts) == want, p


def _triangles_by_stripe(n, s, d, rk, cuts):
    """Enumerate triangles with networkx and bin them by the stripes of their
    ranked vertices."""
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from((int(a), int(b)) for a, b in zip(s, d) if a != b)
    p = len(cuts) - 1
    out = np.zeros((p, p, p), np.uint64)
    stripe = np.searchsorted(np.asarray(cuts), np.arange(n), side="right") - 1
    stripe = np.minimum(stripe, p - 1)
    for clique in nx.enumerate_all_cliques(G):
        if len(clique) < 3:
            continue
        if len(clique) > 3:
            break
        r = sorted(rk[v] for v in clique)
        out[stripe[r[0]], stripe[r[1]], stripe[r[2]]] += 1
    return out


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_block_counts(p):
    n, s, d = gen.rmat(9, 12, gen.seed(92, p))
    keys, deg, rk, row_off, col = oracle.oriented_csr(n, s, d)
    T = oracle.count_csr(n, row_off, col)
    rng = np.random.default_rng(p)
    inner = np.sort(rng.integers(0, n + 1, size=p - 1))
    cuts = np.concatenate([[0], inner, [n]]).astype(np.int32)
    B = oracle.block_counts(n, row_off, col, cuts)
    assert int(B.sum()) == T
    i, j, k = np.nonzero(B)
    assert np.all(i <= j) and np.all(j <= k)
    assert np.array_equal(B, _triangles_by_stripe(n, s, d, rk, cuts))


def test_block_counts_rejects_bad_cuts():
    n, s, d = graphs.complete(6)[0]
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    with pytest.raises(ValueError):
        oracle.block_counts(n, row_off, col, [0, 4, 3, 6])
    with pytest.raises(ValueError):
        oracle.block_counts(n, row_off, col, [1, 3, 6])


def test_out_of_range_ids():
    with pytest.raises(ValueError):
        oracle.tc(4, np.array([0, 4], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(ValueError):
        oracle.tc(4, np.array([-1], np.int32), np.array([1], np.int32))


def test_invariances():
    n, s, d = gen.rmat(10, 16, gen.seed(93, 0))
    t = oracle.tc(n, s, d)
    rng = np.random.default_rng(0)
    perm = rng.permutation(n).astype(np.int32)
    assert oracle.tc(n, perm[s], perm[d]) == t  # vertex relabelling
    o = rng.permutation(len(s))
    assert oracle.tc(n, d[o], s[o]) == t  # pair order and direction
    assert oracle.tc(n + 100, s, d) == t  # isolated vertices
    assert oracle.tc(n, s, d, mode=1) == t  # id order instead of degree order


def test_statistical_sanity_plain_workload():
    """ER G(4096, 32768): E[T] = C(n,3) p^3 with p = m / C(n,2), about 683."""
    n, s, d = gen.plain_graph()
    t = oracle.tc(n, s, d)
    pr = 32768 / math.comb(4096, 2)
    mean = math.comb(4096, 3) * pr ** 3
    assert abs(t - mean) < 6 * math.sqrt(mean) + 10


def test_block_workload_sparse_identity():
    """R-MAT scale 20 (the p = 8 workload): the stored oracle count equals
    sum((U[r] @ U) o U[r]) over row chunks of the degree-oriented upper
    matrix U, built here with numpy and multiplied with scipy."""
    n, s, d = gen.block_graph()
    keep = s != d
    lo = np.minimum(s, d)[keep].astype(np.int64)
    hi = np.maximum(s, d)[keep].astype(np.int64)
    k = np.unique(lo * n + hi)
    a, b = k // n, k % n
    deg = np.bincount(np.concatenate([a, b]), minlength=n)
    order = np.lexsort((np.arange(n), deg))
    rk = np.empty(n, np.int64)
    rk[order] = np.arange(n)
    r0 = np.minimum(rk[a], rk[b])
    r1 = np.maximum(rk[a], rk[b])
    U = sp.csr_matrix((np.ones(len(r0), np.int64), (r0, r1)), shape=(n, n))
    t = 0
    for r in range(0, n, 1 << 16):
        Ur = U[r:r + (1 << 16)]
        t += int((Ur @ U).multiply(Ur).sum())
    with open(os.path.join(GOLDEN, "workload_counts.json")) as f:
        gold = json.load(f)["block"]
    assert t == gold["triangles"]
    assert len(k) == gold["m"]
    assert int((deg == 0).sum()) == gold["isolated"]


# ---------------------------------------------------------------- edge support

def _support(n, s, d):
    _, _, rk, row_off, col = oracle.oriented_csr(n, s, d)
    sup = oracle.edge_support(n, row_off, col)
    a, b = graphs.support_by_pairs(n, s, d, rk, row_off, col)
    return {(int(x), int(y)): int(v) for x, y, v in zip(a, b, sup)}, row_off, col


@pytest.mark.parametrize("n,density,seed", [(9, 0.5, 1), (23, 0.3, 2), (40, 0.2, 3), (60, 0.5, 4), (1, 0, 5)])
def test_edge_support_brute_force(n, density, seed):
    rng = np.random.default_rng(seed)
    pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < density]
    n_, s, d = graphs.messy(*graphs._edges(pairs, n), seed=seed)
    got, _, _ = _support(n_, s, d)
    assert got == graphs.support_brute_force(n_, s, d)


def test_edge_support_dense_identity():
    """support({a, b}) = (A A)[a, b] for every edge: the common neighbours."""
    for n, s, d in (gen.er(300, 2500, gen.seed(41, 0)), gen.rmat(9, 16, gen.seed(41, 1)),
                    gen.rgg(400, 9.0, gen.seed(41, 2))):
        A = np.zeros((n, n), np.int64)
        m = s != d
        A[s[m], d[m]] = 1
        A[d[m], s[m]] = 1
        A2 = A @ A
        got, row_off, col = _support(n, s, d)
        assert len(got) == int(A.sum()) // 2
        assert all(A2[a, b] == v for (a, b), v in got.items())
        assert sum(got.values()) == 3 * oracle.count_csr(n, row_off, col)


def test_edge_support_closed_forms():
    (n, s, d), _ = graphs.complete(12)
    assert set(_support(n, s, d)[0].values()) == {10}
    (n, s, d), _ = graphs.complete_bipartite(4, 5)
    assert set(_support(n, s, d)[0].values()) == {0}
    (n, s, d), _ = graphs.wheel(9)  # spokes lie in 2 triangles, rim edges in 1
    assert all(v == (2 if a == 0 else 1) for (a, b), v in _support(n, s, d)[0].items())
    (n, s, d), _ = graphs.friendship(7)
    assert set(_support(n, s, d)[0].values()) == {1}
    (n, s, d), k = graphs.book(6)
    assert all(v == (k if (a, b) == (0, 1) else 1) for (a, b), v in _support(n, s, d)[0].items())
    (n, s, d), _ = graphs.complete_tripartite(2, 3, 4)  # an edge between two parts: size of the third
    part = lambda x: 0 if x < 2 else (1 if x < 5 else 2)
    size = [2, 3, 4]
    assert all(v == size[3 - part(a) - part(b)] for (a, b), v in _support(n, s, d)[0].items())


# ---------------------------------------------------------------- vertex counts

def test_vertex_counts_dense_identity_and_brute_force():
    """t(v) = (A^3)[v, v] / 2 (closed walks of length 3 through v), and a
    triple enumeration on small graphs; order by id gives the same counts."""
    for n, s, d in (gen.er(250, 2000, gen.seed(42, 0)), gen.rmat(9, 16, gen.seed(42, 1)),
                    gen.rgg(300, 10.0, gen.seed(42, 2))):
        A = np.zeros((n, n), np.int64)
        m = s != d
        A[s[m], d[m]] = 1
        A[d[m], s[m]] = 1
        want = np.diag(A @ A @ A) // 2
        got = oracle.vertex_counts(n, s, d)
        assert np.array_equal(got.astype(np.int64), want)
        assert np.array_equal(oracle.vertex_counts(n, s, d, mode=1), got)
        assert int(got.sum()) == 3 * oracle.tc(n, s, d)
    rng = np.random.default_rng(8)
    for n in (1, 7, 30):
        pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < 0.4]
        n_, s, d = graphs.messy(*graphs._edges(pairs, n), seed=n)
        t = np.zeros(n_, np.int64)
        for (a, b), v in graphs.support_brute_force(n_, s, d).items():
            t[a] += v
            t[b] += v
        assert np.array_equal(oracle.vertex_counts(n_, s, d).astype(np.int64), t // 2)


def test_vertex_counts_closed_forms():
    (n, s, d), _ = graphs.complete(9)
    assert set(oracle.vertex_counts(n, s, d).tolist()) == {math.comb(8, 2)}
    (n, s, d), _ = graphs.complete_bipartite(3, 6)
    assert set(oracle.vertex_counts(n, s, d).tolist()) == {0}
    (n, s, d), _ = graphs.wheel(10)  # hub in every rim triangle, rim vertices in 2
    assert oracle.vertex_counts(n, s, d).tolist() == [9] + [2] * 9
    (n, s, d), k = graphs.friendship(5)
    assert oracle.vertex_counts(n, s, d).tolist() == [k] + [1] * (2 * k)
    (n, s, d), k = graphs.book(4)
    assert oracle.vertex_counts(n, s, d).tolist() == [k, k] + [1] * k


# ---------------------------------------------------------------- k-truss

def _truss(n, s, d, k):
    _, _, rk, row_off, col = oracle.oriented_csr(n, s, d)
    keep = oracle.ktruss(n, row_off, col, k)
    a, b = graphs.support_by_pairs(n, s, d, rk, row_off, col)
    return {(int(x), int(y)) for x, y, f in zip(a, b, keep) if f}, len(col)


@pytest.mark.parametrize("seed", range(6))
def test_ktruss_against_whole_rounds(seed):
    """One edge at a time (the oracle) and whole rounds over the dense
    support matrix reach the same unique k-truss."""
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(10, 70))
    dens = float(rng.uniform(0.1, 0.6))
    pairs = [(x, y) for x, y in itertools.combinations(range(n), 2) if rng.random() < dens]
    n_, s, d = graphs.messy(*graphs._edges(pairs, n), seed=seed)
    for k in (2, 3, 4, 5, 7):
        got, _ = _truss(n_, s, d, k)
        assert got == graphs.ktruss_by_rounds(n_, s, d, k), k


def test_ktruss_closed_forms():
    (n, s, d), _ = graphs.complete(8)
    assert len(_truss(n, s, d, 8)[0]) == 28 and len(_truss(n, s, d, 9)[0]) == 0
    (n, s, d), _ = graphs.wheel(9)
    assert len(_truss(n, s, d, 3)[0]) == 16 and len(_truss(n, s, d, 4)[0]) == 0
    (n, s, d), _ = graphs.book(5)
    assert len(_truss(n, s, d, 3)[0]) == 11 and len(_truss(n, s, d, 4)[0]) == 0
    (n, s, d), _ = graphs.cocktail_party(3)  # octahedron: every edge in 2 triangles
    assert len(_truss(n, s, d, 4)[0]) == 12 and len(_truss(n, s, d, 5)[0]) == 0
    (n, s, d), _ = graphs.disjoint_union(graphs.complete(5), graphs.complete(4))
    got, _ = _truss(n, s, d, 5)
    assert got == {(a, b) for a, b in itertools.combinations(range(5), 2)}
    (n, s, d), _ = graphs.complete_bipartite(4, 4)
    assert len(_truss(n, s, d, 3)[0]) == 0 and len(_truss(n, s, d, 2)[0]) == 16


# ---------------------------------------------------------------- 4-cliques

def test_four_cliques_brute_force_and_networkx():
    rng = np.random.default_rng(12)
    for n, dens in ((8, 0.7), (20, 0.5), (35, 0.35), (45, 0.3)):
        pairs = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < dens]
        n_, s, d = graphs.messy(*graphs._edges(pairs, n), seed=n)
        A = np.zeros((n_, n_), bool)
        A[s, d] = A[d, s] = True
        np.fill_diagonal(A, False)
        want = sum(1 for q in itertools.combinations(range(n_), 4)
                   if all(A[x, y] for x, y in itertools.combinations(q, 2)))
        assert oracle.four_cliques(n_, s, d) == want
        assert oracle.four_cliques(n_, s, d, mode=1) == want
    n, s, d = gen.rmat(10, 16, gen.seed(43, 0))
    G = nx.Graph()
    G.add_edges_from((int(a), int(b)) for a, b in zip(s, d) if a != b)
    want = 0
    for c in nx.enumerate_all_cliques(G):  # by increasing size
        if len(c) > 4:
            break
        want += len(c) == 4
    assert oracle.four_cliques(n, s, d) == want


def test_four_cliques_closed_forms():
    (n, s, d), _ = graphs.complete(11)
    assert oracle.four_cliques(n, s, d) == math.comb(11, 4)
    (n, s, d), _ = graphs.cocktail_party(5)  # one vertex from each of 4 of the 5 pairs
    assert oracle.four_cliques(n, s, d) == 16 * math.comb(5, 4)
    (n, s, d), _ = graphs.complete_tripartite(3, 4, 5)
    assert oracle.four_cliques(n, s, d) == 0
    (n, s, d), _ = graphs.wheel(8)
    assert oracle.four_cliques(n, s, d) == 0
    (n, s, d), _ = graphs.complete(4)
    assert oracle.four_cliques(n, s, d) == 1
    (n, s, d), _ = graphs.disjoint_union(graphs.complete(6), graphs.complete(5))
    assert oracle.four_cliques(n, s, d) == math.comb(6, 4) + math.comb(5, 4)


def test_four_clique_blocks_pins():
    """Per-4-list counts: networkx's 4-cliques binned by the stripes of their
    ranked vertices, the total, the ordered support i <= j <= k <= l, and
    K_n, where the count of a stripe pattern is a product of binomials."""
    rng = np.random.default_rng(21)
    n, s, d = gen.rmat(9, 12, gen.seed(44, 0))
    _, _, rk, row_off, col = oracle.oriented_csr(n, s, d)
    G = nx.Graph()
    G.add_edges_from((int(a), int(b)) for a, b in zip(s, d) if a != b)
    cliques = [c for c in nx.enumerate_all_cliques(G) if len(c) == 4]
    total = oracle.four_cliques(n, s, d)
    assert len(cliques) == total > 0
    for p in (1, 2, 3, 5, 8):
        cuts = np.concatenate([[0], np.sort(rng.integers(0, n + 1, p - 1)), [n]]).astype(np.int32)
        Q = oracle.four_clique_blocks(n, row_off, col, cuts)
        want = np.zeros((p, p, p, p), np.uint64)
        for c in cliques:
            st = sorted(int(np.searchsorted(cuts, rk[v], side="right") - 1) for v in c)
            st = [min(x, p - 1) for x in st]
            want[tuple(st)] += 1
        assert np.array_equal(Q, want), p
        assert int(Q.sum()) == total
        idx = np.argwhere(Q > 0)
        assert all(i <= j <= k <= l for i, j, k, l in idx)
    # K_n under uniform cuts: a stripe pattern with multiplicities m_s counts
    # the product over stripes of C(size_s, m_s)
    (n, s, d), _ = graphs.complete(13)
    _, _, _, row_off, col = oracle.oriented_csr(n, s, d)
    p = 3
    cuts = np.array([0, 4, 9, 13], np.int32)
    size = np.diff(cuts)
    Q = oracle.four_clique_blocks(n, row_off, col, cuts)
    for q in itertools.combinations_with_replacement(range(p), 4):
        mult = np.bincount(q, minlength=p)
        want = 1
        for st in range(p):
            want *= math.comb(int(size[st]), int(mult[st]))
        assert int(Q[q]) == want, q
    assert int(Q.sum()) == math.comb(13, 4)
