"""GPU parity of the 4-clique count against the CPU oracle, through the C
ABI: exact equality."""
import itertools
import math
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


def gpu_four(n, s, d):
    with P.Graph(n, s, d) as g:
        c = g.four_cliques()
        info = g.info()
    return c, info


@pytest.mark.parametrize("name,g,expected", graphs.closed_forms(), ids=lambda x: x if isinstance(x, str) else "")
def test_closed_forms(name, g, expected):
    n, s, d = graphs.messy(*g, seed=9)
    assert gpu_four(n, s, d)[0] == oracle.four_cliques(n, s, d)


def test_named_counts():
    for (g, _), want in ((graphs.complete(12), math.comb(12, 4)), (graphs.cocktail_party(6), 16 * math.comb(6, 4)),
                         (graphs.complete_tripartite(3, 4, 5), 0), (graphs.wheel(9), 0), (graphs.complete(4), 1)):
        assert gpu_four(*g)[0] == want


@pytest.mark.parametrize("seed", range(6))
def test_random_small(seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 100))
    m = int(rng.integers(0, 2 * n * n + 1))
    s = rng.integers(0, n, size=m).astype(np.int32)
    d = rng.integers(0, n, size=m).astype(np.int32)
    assert gpu_four(n, s, d)[0] == oracle.four_cliques(n, s, d)


@pytest.mark.parametrize("kind", ["rmat", "er", "rgg", "k200"])
def test_generated(kind):
    if kind == "rmat":
        n, s, d = gen.rmat(14, 16, gen.seed(66, 0))
    elif kind == "er":
        n, s, d = gen.er(20000, 400000, gen.seed(66, 1))
    elif kind == "rgg":
        n, s, d = gen.rgg(20000, 30.0, gen.seed(66, 2))
    else:
        n = 200
        s, d = np.triu_indices(n, 1)
        s, d = s.astype(np.int32), d.astype(np.int32)
    got, info = gpu_four(n, s, d)
    say("4-cliques", kind, got, info["t_kernel_ms"])
    assert got == oracle.four_cliques(n, s, d)
    assert info["kernel_launches"] == 1


def test_rows_longer_than_the_lds_region():
    """K_1100 plus a pendant K_30: rows above 1024 entries take the
    thread-per-edge path, shorter rows the staged one."""
    a, b = np.triu_indices(1100, 1)
    c, e = np.triu_indices(30, 1)
    s = np.concatenate([a, c + 1100, [0, 7]]).astype(np.int32)
    d = np.concatenate([b, e + 1100, [1100, 1101]]).astype(np.int32)
    got, info = gpu_four(1130, s, d)
    assert got == math.comb(1100, 4) + math.comb(30, 4)
    assert info["kernel_launches"] == 2


def test_empty():
    for n in (0, 3):
        assert gpu_four(n, np.zeros(0, np.int32), np.zeros(0, np.int32))[0] == 0


def check_lists(n, s, d, p, cut_mode=P.CUT_NNZ, want=None):
    """Count over a p x p partition; every 4-list's count against the
    oracle's per-stripe counts under the same cuts (or want(rank, cuts))."""
    with P.Graph(n, s, d) as g:
        g.partition(p, cut_mode=cut_mode)
        got = g.four_cliques()
        ijkl, cnt = g.four_clique_lists()
        row_off, col, rank = g.export_csr()
        cuts = g.cuts()
        Q = oracle.four_clique_blocks(n, row_off, col, cuts) if want is None else want(rank, cuts)
        info = g.info()
    assert got == int(Q.sum())
    seen = np.zeros_like(Q)
    for (i, j, k, l), c in zip(ijkl, cnt):
        assert i <= j <= k <= l
        assert c == Q[i, j, k, l], (i, j, k, l)
        seen[i, j, k, l] = 1
    # a 4-list left out (one of its six blocks empty) holds no 4-clique
    assert int(Q[seen == 0].sum()) == 0
    return got, info


@pytest.mark.parametrize("p", [1, 2, 3, 5, 8])
def test_block_lists_rmat(p):
    n, s, d = gen.rmat(13, 16, gen.seed(67, p))
    got, info = check_lists(n, s, d, p)
    say("4-lists rmat13 p", p, got, info["t_kernel_ms"])
    assert got == oracle.four_cliques(n, s, d)


@pytest.mark.parametrize("p", [2, 7])
def test_block_lists_uniform_cuts_and_closed_forms(p):
    n, s, d = gen.rgg(6000, 24.0, gen.seed(67, 20 + p))
    check_lists(n, s, d, p, cut_mode=P.CUT_UNIFORM)
    for (g, _), want in ((graphs.complete(40), math.comb(40, 4)), (graphs.cocktail_party(9), 16 * math.comb(9, 4)),
                         (graphs.complete_tripartite(5, 6, 7), 0)):
        got, _ = check_lists(*graphs.messy(*g, seed=p), p)
        assert got == want


@pytest.mark.parametrize("p", [1, 4])
def test_block_lists_long_rows(p):
    """K_1100 plus a pendant K_30: at p = 1 the rows of K_1100 exceed the
    LDS region and take the merge kernel; at p = 4 they are cut into
    stripes."""
    a, b = np.triu_indices(1100, 1)
    c, e = np.triu_indices(30, 1)
    s = np.concatenate([a, c + 1100, [0, 7]]).astype(np.int32)
    d = np.concatenate([b, e + 1100, [1100, 1101]]).astype(np.int32)

    def closed_form(rank, cuts):
        # a 4-list's count: for each clique, the product over its stripes of
        # C(members in the stripe, multiplicity) (the two pendant edges close
        # no 4-clique)
        pp = len(cuts) - 1
        st = np.searchsorted(cuts, rank, side="right") - 1
        sizes = [np.bincount(st[:1100], minlength=pp), np.bincount(st[1100:], minlength=pp)]
        Q = np.zeros((pp,) * 4, np.uint64)
        for q in itertools.combinations_with_replacement(range(pp), 4):
            mult = np.bincount(q, minlength=pp)
            Q[q] = sum(math.prod(math.comb(int(sz[t]), int(mult[t])) for t in range(pp)) for sz in sizes)
        return Q

    got, info = check_lists(1130, s, d, p, want=closed_form)
    say("4-lists K_1100 p", p, got, info["t_kernel_ms"], info["kernel_launches"])
    assert got == math.comb(1100, 4) + math.comb(30, 4)
    if p == 1:
        assert info["kernel_launches"] == 2


def test_block_lists_streamed_host_store():
    """A streamed triangle count moves the blocks to the host store; the
    4-clique count then streams them (under that count's cap) and every
    4-list's count equals the in-core one."""
    n, s, d = gen.rmat(12, 16, gen.seed(68, 0))
    with P.Graph(n, s, d) as g:
        g.partition(5)
        want = g.four_cliques()
        _, want_cnt = g.four_clique_lists()
        tri = g.count(stream_blocks=True, device_cap_bytes=g.info()["block_bytes"] // 2)
        got = g.four_cliques()
        _, cnt = g.four_clique_lists()
        info = g.info()
    assert tri == oracle.tc(n, s, d)
    assert got == want == oracle.four_cliques(n, s, d)
    assert np.array_equal(cnt, want_cnt)
    assert info["h2d_bytes"] > 0


@pytest.mark.parametrize("p", [3, 8])
def test_block_lists_streamed_caps(p):
    """Caps halved from the whole store down to the first that cannot hold
    some 4-list's six blocks (ENOMEM): every count on the way equals the
    in-core one, list by list, and smaller caps copy more."""
    n, s, d = gen.rmat(13, 16, gen.seed(69, p))
    with P.Graph(n, s, d) as g:
        g.partition(p)
        want = g.four_cliques()
        _, want_cnt = g.four_clique_lists()
        cap = g.info()["block_bytes"]
        copied = []
        for _ in range(12):
            try:
                got = g.four_cliques(device_cap_bytes=cap)
            except P.PgabbError as e:
                assert e.status == P.ENOMEM
                break
            _, cnt = g.four_clique_lists()
            assert got == want
            assert np.array_equal(cnt, want_cnt)
            copied.append(g.info()["h2d_bytes"])
            cap //= 2
        else:
            raise AssertionError("no cap was too small")
    say("4-lists streamed p", p, "bytes copied per cap", copied)
    assert len(copied) >= 2 and copied[-1] > copied[0]
    assert want == oracle.four_cliques(n, s, d)


def test_block_lists_streamed_long_rows():
    """K_1100 plus a pendant K_30 over 2 x 2 blocks, streamed under three
    quarters of the store: the merge kernel reads streamed blocks too."""
    a, b = np.triu_indices(1100, 1)
    c, e = np.triu_indices(30, 1)
    s = np.concatenate([a, c + 1100, [0, 7]]).astype(np.int32)
    d = np.concatenate([b, e + 1100, [1100, 1101]]).astype(np.int32)
    with P.Graph(1130, s, d) as g:
        g.partition(2)
        got = g.four_cliques(device_cap_bytes=g.info()["block_bytes"] * 3 // 4)
        info = g.info()
    assert got == math.comb(1100, 4) + math.comb(30, 4)
    assert info["kernel_launches"] >= 2
