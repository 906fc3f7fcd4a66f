"""GPU parity of the 4-clique count against the CPU oracle, through the C
ABI: exact equality."""
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
