"""Small named graphs with known triangle counts (closed forms), as int32
edge lists.  Test helpers only; nothing here counts triangles."""
from __future__ import annotations

import itertools
import math

import numpy as np


def _edges(pairs, n):
    if not pairs:
        return n, np.zeros(0, np.int32), np.zeros(0, np.int32)
    a = np.asarray(pairs, dtype=np.int32)
    return n, a[:, 0].copy(), a[:, 1].copy()


def complete(n):
    """K_n: C(n, 3) triangles."""
    return _edges(list(itertools.combinations(range(n), 2)), n), math.comb(n, 3)


def complete_bipartite(a, b):
    """K_{a,b}: bipartite, no triangles."""
    return _edges([(i, a + j) for i in range(a) for j in range(b)], a + b), 0


def cycle(n):
    """C_n: one triangle for n = 3, none above."""
    return _edges([(i, (i + 1) % n) for i in range(n)], n), 1 if n == 3 else 0


def wheel(n):
    """W_n = hub + cycle of n - 1 rim vertices (n >= 5): n - 1 triangles."""
    rim = n - 1
    pairs = [(0, 1 + i) for i in range(rim)] + [(1 + i, 1 + (i + 1) % rim) for i in range(rim)]
    return _edges(pairs, n), n - 1


def complete_tripartite(a, b, c):
    """K_{a,b,c}: a * b * c triangles (one vertex from each part)."""
    parts = [list(range(a)), list(range(a, a + b)), list(range(a + b, a + b + c))]
    pairs = [(x, y) for p, q in itertools.combinations(parts, 2) for x in p for y in q]
    return _edges(pairs, a + b + c), a * b * c


def cocktail_party(k):
    """K_{2,...,2} with k parts: 8 * C(k, 3) triangles."""
    n = 2 * k
    pairs = [(x, y) for x, y in itertools.combinations(range(n), 2) if x // 2 != y // 2]
    return _edges(pairs, n), 8 * math.comb(k, 3)


def friendship(k):
    """F_k: k triangles sharing one vertex."""
    pairs = []
    for t in range(k):
        a, b = 1 + 2 * t, 2 + 2 * t
        pairs += [(0, a), (0, b), (a, b)]
    return _edges(pairs, 2 * k + 1), k


def book(k):
    """B_k: k triangles sharing the edge (0, 1)."""
    pairs = [(0, 1)] + [(0, 2 + t) for t in range(k)] + [(1, 2 + t) for t in range(k)]
    return _edges(pairs, k + 2), k


def hypercube(d):
    """Q_d: bipartite, no triangles."""
    n = 1 << d
    return _edges([(v, v ^ (1 << b)) for v in range(n) for b in range(d) if v < v ^ (1 << b)], n), 0


def grid(r, c):
    """r x c grid: bipartite, no triangles."""
    pairs = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                pairs.append((v, v + 1))
            if i + 1 < r:
                pairs.append((v, v + c))
    return _edges(pairs, r * c), 0


def star(k):
    """K_{1,k}: no triangles."""
    return _edges([(0, 1 + t) for t in range(k)], k + 1), 0


def disjoint_union(*gs):
    """Disjoint union of (graph, count) pairs: counts add."""
    n = 0
    srcs, dsts, total = [], [], 0
    for (gn, s, d), c in gs:
        srcs.append(s + n)
        dsts.append(d + n)
        n += gn
        total += c
    return (n, np.concatenate(srcs).astype(np.int32), np.concatenate(dsts).astype(np.int32)), total


def closed_forms():
    """(name, (n, src, dst), expected triangles)."""
    out = []
    for n in (0, 1, 2, 3, 4, 5, 10, 33, 64, 100):
        out.append(("K%d" % n, *complete(n)))
    for a, b in ((1, 1), (3, 4), (10, 20)):
        out.append(("K%d,%d" % (a, b), *complete_bipartite(a, b)))
    for n in (3, 4, 5, 100):
        out.append(("C%d" % n, *cycle(n)))
    for n in (5, 6, 50, 513):
        out.append(("W%d" % n, *wheel(n)))
    for abc in ((1, 1, 1), (2, 3, 4), (7, 5, 9)):
        out.append(("K%d,%d,%d" % abc, *complete_tripartite(*abc)))
    for k in (3, 4, 10):
        out.append(("CP%d" % k, *cocktail_party(k)))
    for k in (1, 2, 40):
        out.append(("F%d" % k, *friendship(k)))
    for k in (1, 3, 300):
        out.append(("B%d" % k, *book(k)))
    for d in (3, 7):
        out.append(("Q%d" % d, *hypercube(d)))
    out.append(("grid", *grid(20, 30)))
    out.append(("star", *star(1000)))
    out.append(("union", *disjoint_union(complete(12), wheel(9), friendship(5), grid(4, 4))))
    return out


def messy(n, src, dst, seed=0):
    """Same graph with self-loops, repeats and reversed pairs added and the
    pair order shuffled (the cleaning must remove all of it)."""
    rng = np.random.default_rng(seed)
    s = np.asarray(src, np.int64)
    d = np.asarray(dst, np.int64)
    parts_s = [s, d, s[: len(s) // 2]]
    parts_d = [d, s, d[: len(d) // 2]]
    if n > 0:
        loops = rng.integers(0, n, size=max(1, n // 3))
        parts_s.append(loops)
        parts_d.append(loops)
    S = np.concatenate(parts_s)
    D = np.concatenate(parts_d)
    perm = rng.permutation(len(S))
    return n, S[perm].astype(np.int32), D[perm].astype(np.int32)


def brute_force(n, src, dst):
    """Triangles by checking every vertex triple against an adjacency matrix
    (n <= ~80)."""
    A = np.zeros((n, n), dtype=bool)
    for a, b in zip(src, dst):
        if a != b:
            A[a, b] = A[b, a] = True
    t = 0
    for a, b, c in itertools.combinations(range(n), 3):
        if A[a, b] and A[b, c] and A[a, c]:
            t += 1
    return t


def support_by_pairs(n, src, dst, rank, row_off, col):
    """Oracle-independent per-edge expectations are compared by vertex pair:
    map each oriented CSR edge (ranks x, y) to its input-id pair (a, b) with
    a < b."""
    inv = np.empty(n, np.int64)
    inv[np.asarray(rank, np.int64)] = np.arange(n)
    rows = np.repeat(np.arange(n), np.diff(row_off))
    a, b = inv[rows], inv[np.asarray(col, np.int64)]
    return np.minimum(a, b), np.maximum(a, b)


def support_brute_force(n, src, dst):
    """{(a, b): triangles containing edge {a, b}} by enumerating every vertex
    triple against an adjacency matrix (n <= ~80)."""
    A = np.zeros((n, n), dtype=bool)
    for a, b in zip(src, dst):
        if a != b:
            A[a, b] = A[b, a] = True
    sup = {(a, b): 0 for a, b in zip(*np.nonzero(np.triu(A)))}
    for a, b, c in itertools.combinations(range(n), 3):
        if A[a, b] and A[b, c] and A[a, c]:
            sup[(a, b)] += 1
            sup[(a, c)] += 1
            sup[(b, c)] += 1
    return sup


def ktruss_by_rounds(n, src, dst, k):
    """{(a, b)} of the k-truss by whole rounds: drop every edge whose support
    within the remaining edges, (A A)[a, b] on the dense adjacency matrix, is
    below k - 2, until a round drops none."""
    A = np.zeros((n, n), np.int64)
    for a, b in zip(src, dst):
        if a != b:
            A[a, b] = A[b, a] = 1
    while True:
        S = (A @ A) * A
        drop = (A == 1) & (S < k - 2)
        if not drop.any():
            break
        A[drop] = 0
    return {(int(a), int(b)) for a, b in zip(*np.nonzero(np.triu(A)))}
