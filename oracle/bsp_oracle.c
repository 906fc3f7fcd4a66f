/*
 * CPU ORACLE for the single-block bulk-synchronous computations --
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; it shares no code with the HIP sources.
 *
 * PGAbB Section 3.2 names a second execution mode besides the multi-block
 * pattern of triangle counting: every iteration visits every edge, one block
 * per block-list.  Its two examples are written out here by definition:
 *
 * Connected components (Section 3.4, the Shiloach-Vishkin example, which
 * computes weakly connected components).  The result has a plain
 * definition: label(v) = the smallest vertex id reachable from v in the
 * undirected graph.  (Shiloach-Vishkin hooks the larger of two roots under
 * the smaller, so each tree's root is the smallest id in it, and at the
 * fixed point every vertex points to the smallest id of its component.)
 * Evaluated by a breadth-first search from every still unlabelled vertex in
 * increasing id order: that vertex is the smallest of its component.
 *
 * PageRank (Section 5.2, bulk computations): damping d, tolerance tol,
 * iteration limit; SpMV-style iteration over the undirected graph in
 * double precision:
 *     r_0(v) = 1 / n
 *     r_{t+1}(v) = (1 - d) / n + d * sum over neighbours u of r_t(u) / deg(u)
 * stopping after iteration t + 1 when sum_v |r_{t+1}(v) - r_t(v)| < tol or
 * when the limit is reached.  Isolated vertices pass nothing on.
 *
 * Inputs: n and the cleaned canonical pair keys (min << 32 | max, sorted,
 * distinct, no loops) that oracle_clean produces.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Symmetric adjacency lists from the canonical keys: off[n + 1], adj[2 mu]. */
static int build_adj(int32_t n, const uint64_t *keys, int64_t mu, int64_t **off_out, int32_t **adj_out)
{
    int64_t *off = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *adj = malloc(sizeof(int32_t) * (size_t)(2 * mu + 1));
    int64_t *fill = malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!off || !adj || !fill) {
        free(off);
        free(adj);
        free(fill);
        return -1;
    }
    for (int64_t e = 0; e < mu; ++e) {
        off[(keys[e] >> 32) + 1]++;
        off[(keys[e] & 0xffffffffu) + 1]++;
    }
    for (int32_t v = 0; v < n; ++v) off[v + 1] += off[v];
    memcpy(fill, off, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t e = 0; e < mu; ++e) {
        int32_t a = (int32_t)(keys[e] >> 32), b = (int32_t)(keys[e] & 0xffffffffu);
        adj[fill[a]++] = b;
        adj[fill[b]++] = a;
    }
    free(fill);
    *off_out = off;
    *adj_out = adj;
    return 0;
}

/* label[v] = smallest vertex id reachable from v.  Returns the number of
 * components, or -1 on allocation failure. */
int64_t oracle_components(int32_t n, const uint64_t *keys, int64_t mu, int32_t *label)
{
    int64_t *off;
    int32_t *adj;
    if (build_adj(n, keys, mu, &off, &adj)) return -1;
    int32_t *queue = malloc(sizeof(int32_t) * ((size_t)n + 1));
    if (!queue) {
        free(off);
        free(adj);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) label[v] = -1;
    int64_t comps = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (label[s] >= 0) continue;
        ++comps;
        int64_t head = 0, tail = 0;
        label[s] = s;
        queue[tail++] = s;
        while (head < tail) {
            int32_t x = queue[head++];
            for (int64_t t = off[x]; t < off[x + 1]; ++t) {
                int32_t y = adj[t];
                if (label[y] < 0) {
                    label[y] = s;
                    queue[tail++] = y;
                }
            }
        }
    }
    free(queue);
    free(off);
    free(adj);
    return comps;
}

/* PageRank as defined above; ranks[n] receives r at the last iteration.
 * Returns the number of iterations run (>= 1 when n > 0), or -1 on
 * allocation failure.  *err_out (may be NULL) receives the last iteration's
 * sum of absolute changes. */
int32_t oracle_pagerank(int32_t n, const uint64_t *keys, int64_t mu, double d, double tol, int32_t max_iter,
                        double *ranks, double *err_out)
{
    if (n == 0) {
        if (err_out) *err_out = 0;
        return 0;
    }
    int64_t *off;
    int32_t *adj;
    if (build_adj(n, keys, mu, &off, &adj)) return -1;
    double *next = malloc(sizeof(double) * (size_t)n);
    if (!next) {
        free(off);
        free(adj);
        return -1;
    }
    for (int32_t v = 0; v < n; ++v) ranks[v] = 1.0 / n;
    int32_t it = 0;
    double err = 0;
    while (it < max_iter) {
        for (int32_t v = 0; v < n; ++v) {
            double s = 0;
            for (int64_t t = off[v]; t < off[v + 1]; ++t) {
                int32_t u = adj[t];
                s += ranks[u] / (double)(off[u + 1] - off[u]);
            }
            next[v] = (1.0 - d) / n + d * s;
        }
        err = 0;
        for (int32_t v = 0; v < n; ++v) {
            err += fabs(next[v] - ranks[v]);
            ranks[v] = next[v];
        }
        ++it;
        if (err < tol) break;
    }
    if (err_out) *err_out = err;
    free(next);
    free(off);
    free(adj);
    return it;
}
