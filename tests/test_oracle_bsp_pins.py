"""Pins of the CPU oracle's single-block bulk-synchronous computations
(connected components and PageRank, PGAbB Sections 3.2, 3.4 and 5.2)
against library routines, brute force and closed forms."""
import numpy as np
import scipy.sparse as sp
from hypothesis import given, settings, strategies as st
from scipy.sparse.csgraph import connected_components

import oracle
from paper_2209_04541_amd import gen
from tests import graphs


def _random(n, dens, sd):
    rng = np.random.default_rng(sd)
    m = int(dens * n * n)
    return n, rng.integers(0, n, m).astype(np.int32), rng.integers(0, n, m).astype(np.int32)


def _dense(n, s, d):
    A = np.zeros((n, n), np.float64)
    keep = s != d
    A[s[keep], d[keep]] = 1
    A[d[keep], s[keep]] = 1
    return A


# ------------------------------------------------------------ components

@settings(max_examples=80, deadline=None)
@given(st.integers(0, 60), st.floats(0.0, 0.08), st.integers(0, 2**31 - 1))
def test_components_against_scipy(n, dens, sd):
    n, s, d = _random(n, dens, sd)
    lab, c = oracle.components(n, s, d)
    if n == 0:
        assert c == 0 and len(lab) == 0
        return
    A = sp.coo_matrix((np.ones(len(s)), (s, d)), shape=(n, n)).tocsr()
    nc, cl = connected_components(A, directed=False)
    assert c == nc
    smallest = np.full(nc, n, np.int64)
    np.minimum.at(smallest, cl, np.arange(n))
    assert np.array_equal(lab, smallest[cl])


@settings(max_examples=40, deadline=None)
@given(st.integers(1, 25), st.floats(0.0, 0.15), st.integers(0, 2**31 - 1))
def test_components_brute_force_closure(n, dens, sd):
    """Reachability by squaring (I + A) until it stops changing."""
    n, s, d = _random(n, dens, sd)
    R = (_dense(n, s, d) + np.eye(n)) > 0
    while True:
        R2 = (R.astype(np.int64) @ R.astype(np.int64)) > 0
        if np.array_equal(R2, R):
            break
        R = R2
    want = np.array([np.nonzero(R[v])[0].min() for v in range(n)])
    assert np.array_equal(oracle.components(n, s, d)[0], want)


def test_components_closed_forms():
    (n, s, d), _ = graphs.complete(12)
    lab, c = oracle.components(n, s, d)
    assert c == 1 and not lab.any()
    (n, s, d), _ = graphs.disjoint_union(graphs.complete(5), graphs.wheel(9), graphs.star(4))
    lab, c = oracle.components(n, s, d)
    assert c == 3 and list(lab) == [0] * 5 + [5] * 9 + [14] * 5
    # isolated vertices label themselves; a path laid out from high ids down
    z = np.zeros(0, np.int32)
    assert list(oracle.components(4, z, z)[0]) == [0, 1, 2, 3]
    s = np.arange(9, 0, -1, dtype=np.int32)
    lab, c = oracle.components(10, s, s - 1)
    assert c == 1 and not lab.any()


# ------------------------------------------------------------- PageRank

def test_pagerank_regular_graphs_stay_uniform():
    """Every vertex of a regular graph passes r/deg to deg neighbours, so
    the uniform start is the fixed point: one iteration, zero change."""
    for (n, s, d), _ in (graphs.complete(9), graphs.cycle(11), graphs.hypercube(4),
                         graphs.complete_bipartite(6, 6)):
        r, it, err = oracle.pagerank(n, s, d)
        assert it == 1 and err < 1e-15
        assert np.allclose(r, 1.0 / n, rtol=0, atol=1e-15)


def test_pagerank_star_recursion():
    """Star K_{1,k}: the hub h and the k leaves l follow
    h' = (1 - d)/n + d k l and l' = (1 - d)/n + d h / k."""
    k, dmp = 7, 0.85
    (n, s, d), _ = graphs.star(k)
    for iters in (1, 2, 5, 20):
        h = l = 1.0 / n
        for _ in range(iters):
            h, l = (1 - dmp) / n + dmp * k * l, (1 - dmp) / n + dmp * h / k
        r, it, _ = oracle.pagerank(n, s, d, tol=0.0, max_iter=iters)
        assert it == iters
        assert abs(r[0] - h) < 1e-15 and np.allclose(r[1:], l, rtol=0, atol=1e-15)


@settings(max_examples=30, deadline=None)
@given(st.integers(2, 40), st.floats(0.02, 0.3), st.integers(0, 2**31 - 1))
def test_pagerank_fixed_point_solves_linear_system(n, dens, sd):
    """Iterated to convergence the ranks solve
    (I - d A D^-1) r = (1 - d)/n (D^-1 taken as 0 for isolated vertices)."""
    n, s, d = _random(n, dens, sd)
    A = _dense(n, s, d)
    deg = A.sum(axis=0)
    Dinv = np.where(deg > 0, 1.0 / np.maximum(deg, 1), 0.0)
    want = np.linalg.solve(np.eye(n) - 0.85 * A * Dinv[None, :], np.full(n, 0.15 / n))
    r, it, _ = oracle.pagerank(n, s, d, tol=0.0, max_iter=600)
    assert np.allclose(r, want, rtol=1e-9, atol=1e-14)


def test_pagerank_mass_and_stopping():
    n, s, d = gen.rmat(9, 8, gen.seed(93, 1))
    keys = oracle.clean(n, s, d)
    deg = oracle.degrees(n, keys)
    # without isolated vertices no rank leaks: the ranks sum to 1 throughout
    n2, s2, d2 = graphs.wheel(30)[0]
    for t in range(1, 6):
        r, it, _ = oracle.pagerank(n2, s2, d2, tol=0.0, max_iter=t)
        assert abs(r.sum() - 1.0) < 1e-12
    # the reported change is the L1 distance between consecutive iterates,
    # and the run stops at the first iteration whose change is below tol
    prev = oracle.pagerank(n, s, d, tol=0.0, max_iter=1)[0]
    for t in range(2, 21):
        r, it, err = oracle.pagerank(n, s, d, tol=0.0, max_iter=t)
        assert abs(err - np.abs(r - prev).sum()) < 1e-15
        prev = r
    r, it, err = oracle.pagerank(n, s, d)
    assert err < 1e-4 or it == 20
    if it > 1:
        assert oracle.pagerank(n, s, d, tol=0.0, max_iter=it - 1)[2] >= 1e-4
    # isolated vertices keep the teleport share alone
    iso = np.nonzero(deg == 0)[0]
    assert len(iso) and np.allclose(r[iso], 0.15 / n, rtol=0, atol=1e-18)
