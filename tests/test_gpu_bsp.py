"""GPU parity of the single-block bulk-synchronous computations over the
blocks (connected components by Shiloach-Vishkin, PageRank) against the CPU
oracle, through the C ABI.

Components: the labels (smallest input id per component) are unique, so
they must equal the oracle's exactly, as must the component count.
PageRank: both sides iterate in double precision; the device sums each
vertex's shares in another order (atomic additions), so each rank may differ
from the oracle's by rounding.  A sum of k shares in fp64 carries a relative
error of at most about k * 2^-53 (k up to a few thousand here: below 1e-12),
and the iteration contracts errors by the damping factor, so twenty
iterations stay well below a relative 1e-10, while any lost or doubled edge
share moves a rank by about damping / degree of it (above 1e-4 relative).
The iteration count must be the same (the seeds give stopping errors far
from the tolerance)."""
import sys

import numpy as np
import pytest

import oracle
import paper_2209_04541_amd as P
from paper_2209_04541_amd import gen
from tests import graphs

pytestmark = pytest.mark.gpu

RTOL = 1e-10
ATOL = 1e-15


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_cc(n, s, d, p=None, cut_mode=P.CUT_NNZ):
    want, wc = oracle.components(n, s, d)
    with P.Graph(n, s, d) as g:
        if p:
            g.partition(p, cut_mode=cut_mode)
        got, nc, it = g.components()
    assert nc == wc
    assert np.array_equal(got, want)
    assert it % 2 == 0 and it >= 2 or n == 0
    return it


def check_pr(n, s, d, p=None, **kw):
    want, wit, werr = oracle.pagerank(n, s, d, **kw)
    with P.Graph(n, s, d) as g:
        if p:
            g.partition(p)
        got, it, err = g.pagerank(**kw)
    assert it == wit
    np.testing.assert_allclose(got, want, rtol=RTOL, atol=ATOL)
    assert abs(err - werr) <= 1e-9 * max(1.0, abs(werr))
    return it


def _union_with_isolated(seed):
    """Several R-MAT pieces, a few cliques and paths on disjoint id ranges,
    shuffled ids and isolated vertices in between."""
    rng = np.random.default_rng(seed)
    parts = [(gen.rmat(9, 4, gen.seed(900, seed)), 0), graphs.complete(7), graphs.cycle(50), graphs.star(30),
             (gen.rmat(8, 2, gen.seed(901, seed)), 0)]
    (n, s, d), _ = graphs.disjoint_union(*parts)
    n_all = n + 200
    perm = rng.permutation(n_all).astype(np.int32)
    return n_all, perm[s], perm[d]


@pytest.mark.parametrize("p", [None, 1, 3, 8])
def test_components_small(p):
    for seed in range(3):
        n, s, d = _union_with_isolated(seed)
        say("cc union", seed, p, n, len(s))
        check_cc(n, s, d, p)
    for name, (n, s, d), _ in graphs.closed_forms():
        check_cc(n, s, d, p)


def test_components_edge_cases():
    check_cc(0, np.zeros(0, np.int32), np.zeros(0, np.int32))
    check_cc(5, np.zeros(0, np.int32), np.zeros(0, np.int32))        # no edges: every vertex alone
    check_cc(4, np.array([1, 2, 2], np.int32), np.array([1, 2, 2], np.int32))  # loops only
    # a long path in decreasing id order (hooks one step at a time)
    n = 3000
    a = np.arange(n - 1, 0, -1, dtype=np.int32)
    check_cc(n, a, a - 1, 4)
    # messy input: repeats, reversed pairs, loops
    n, s, d = gen.rmat(10, 8, gen.seed(902, 0))
    n, s, d = graphs.messy(n, s, d, seed=3)
    check_cc(n, s, d, 5)


def test_components_uniform_cuts_and_ids():
    n, s, d = gen.rmat(12, 4, gen.seed(903, 0))
    for p in (2, 7):
        check_cc(n, s, d, p, cut_mode=P.CUT_UNIFORM)


def test_components_rmat20():
    """The block workload's graph (R-MAT scale 20, edge factor 16, p = 8):
    every label against the oracle's breadth-first search."""
    n, s, d = gen.block_graph()
    it = check_cc(n, s, d, 8)
    say("cc rmat20 iterations", it)


@pytest.mark.parametrize("p", [None, 2, 8])
def test_pagerank_small(p):
    for seed in range(3):
        n, s, d = _union_with_isolated(seed)
        say("pr union", seed, p)
        check_pr(n, s, d, p)
    n, s, d = gen.rmat(12, 16, gen.seed(904, 0))
    check_pr(n, s, d, p)


def test_pagerank_options_and_edge_cases():
    n, s, d = gen.rmat(11, 8, gen.seed(905, 0))
    check_pr(n, s, d, 4, damping=0.5, tol=1e-9, max_iter=50)
    check_pr(n, s, d, 4, damping=0.85, tol=0.0, max_iter=7)    # runs to the limit
    check_pr(n, s, d, 4, damping=0.85, tol=1e-4, max_iter=0)   # no iteration: r_0
    check_pr(5, np.zeros(0, np.int32), np.zeros(0, np.int32))  # no edges: teleport share only
    with P.Graph(0, np.zeros(0, np.int32), np.zeros(0, np.int32)) as g:
        r, it, err = g.pagerank()
        assert len(r) == 0 and it == 0
    with P.Graph(n, s, d) as g:
        for bad in (dict(damping=1.5), dict(tol=-1.0), dict(max_iter=-1), dict(damping=float("nan"))):
            with pytest.raises(P.PgabbError) as ei:
                g.pagerank(**bad)
            assert ei.value.status == P.EINVAL


def test_pagerank_rmat20():
    """PageRank on the block workload's graph (R-MAT scale 20, p = 8), as
    the paper's evaluation runs it (damping 0.85, tolerance 1e-4, at most 20
    iterations)."""
    n, s, d = gen.block_graph()
    it = check_pr(n, s, d, 8)
    say("pr rmat20 iterations", it)


def test_bsp_streamed_graph_is_refused():
    n, s, d = gen.rmat(10, 8, gen.seed(906, 0))
    with P.Graph(n, s, d) as g:
        g.partition(4)
        g.count(stream_blocks=True)
        with pytest.raises(P.PgabbError) as ei:
            g.components()
        assert ei.value.status == P.ESTATE
