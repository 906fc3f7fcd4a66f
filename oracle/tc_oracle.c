/*
 * CPU ORACLE for block-partitioned triangle counting -- TEST INFRASTRUCTURE.
 *
 * This file is the parity checker for the GPU library, not part of it.  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header or table with the HIP sources.
 *
 * What it computes (PGAbB, Section 3.6, "An example: triangle counting"):
 * the number of sets of three vertices of an undirected graph that are
 * pairwise adjacent.  The input is made undirected and deduplicated first
 * (Section 5.1, Dataset); self-loops are dropped as well.
 *
 * The count is the plain definition evaluated with the standard oriented
 * formulation the paper uses for TC (Section 5.4: degree-based vertex
 * ordering, and only half of the edges are needed):
 *   1. keep every undirected pair {a, b}, a != b, once;
 *   2. deg[v] = number of kept pairs containing v;
 *   3. rank vertices by ascending (deg, id) (or by id in the second mode);
 *   4. orient each pair from lower to higher rank: N+(x) = out-neighbours;
 *   5. T = sum over x, over y in N+(x), of |N+(x) & N+(y)|, by two-pointer
 *      merge of the sorted lists.
 * Each triangle with ranks r(a) < r(b) < r(c) is counted once, at edge (a, b)
 * with common neighbour c, so T is the triangle count.
 *
 * Block mode (Section 3.6, block-list composition and kernel development;
 * Section 4.3, symmetric 2-D partitioning): with cut vector
 * c_0 = 0 <= c_1 <= ... <= c_p = n applied to the ranked ids on both axes,
 * T_ijk counts the triangles whose three ranked vertices fall in stripes
 * i <= j <= k.  That is exactly what the triple (A_ij, A_ik, A_jk) finds:
 * for every edge (u, v) of block A_ij, the common out-neighbours of u and v
 * that lie in stripe k.  Here it is computed by the definition: merge the full
 * lists and bin every common neighbour by its stripe.
 *
 * Precision: all integer; counts in uint64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- helpers */

static int cmp_u64(const void *pa, const void *pb)
{
    uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return (a > b) - (a < b);
}

static int cmp_i32(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

/* Step 1: canonical undirected pairs.  keys_out must hold m entries; returns
 * the number of distinct pairs m' (written sorted, key = min << 32 | max), or
 * -1 if an id lies outside [0, n). */
int64_t oracle_clean(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     uint64_t *keys_out)
{
    int64_t k = 0;
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = src[e], b = dst[e];
        if (a < 0 || b < 0 || a >= n || b >= n) return -1;
        if (a == b) continue; /* self-loop */
        uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
        keys_out[k++] = ((uint64_t)lo << 32) | hi;
    }
    qsort(keys_out, (size_t)k, sizeof(uint64_t), cmp_u64);
    int64_t u = 0;
    for (int64_t e = 0; e < k; ++e)
        if (u == 0 || keys_out[u - 1] != keys_out[e]) keys_out[u++] = keys_out[e];
    return u;
}

/* Step 2: degree of every vertex in the simple undirected graph. */
void oracle_degrees(int32_t n, const uint64_t *keys, int64_t mu, int32_t *deg)
{
    memset(deg, 0, sizeof(int32_t) * (size_t)n);
    for (int64_t e = 0; e < mu; ++e) {
        deg[keys[e] >> 32]++;
        deg[keys[e] & 0xffffffffu]++;
    }
}

/* Step 3: rank[v] = position of v in the order.  mode 0: ascending
 * (deg, id); mode 1: ascending id (rank = id). */
static const int32_t *g_sort_deg;
static int cmp_by_deg_then_id(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    if (g_sort_deg[a] != g_sort_deg[b]) return g_sort_deg[a] < g_sort_deg[b] ? -1 : 1;
    return (a > b) - (a < b);
}

void oracle_rank(int32_t n, const int32_t *deg, int mode, int32_t *rank)
{
    if (mode == 1) {
        for (int32_t v = 0; v < n; ++v) rank[v] = v;
        return;
    }
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; ++v) order[v] = v;
    g_sort_deg = deg;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_by_deg_then_id);
    for (int32_t r = 0; r < n; ++r) rank[order[r]] = r;
    free(order);
}

/* Step 4: oriented CSR over ranked ids.  Row x (a rank) lists, in increasing
 * order, the ranks of its neighbours that have a higher rank.  row_off has
 * n + 1 entries, col has mu entries. */
void oracle_orient(int32_t n, const uint64_t *keys, int64_t mu, const int32_t *rank,
                   int64_t *row_off, int32_t *col)
{
    memset(row_off, 0, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t e = 0; e < mu; ++e) {
        int32_t ra = rank[keys[e] >> 32], rb = rank[keys[e] & 0xffffffffu];
        int32_t lo = ra < rb ? ra : rb;
        row_off[lo + 1]++;
    }
    for (int32_t x = 0; x < n; ++x) row_off[x + 1] += row_off[x];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    memcpy(fill, row_off, sizeof(int64_t) * (size_t)n);
    for (int64_t e = 0; e < mu; ++e) {
        int32_t ra = rank[keys[e] >> 32], rb = rank[keys[e] & 0xffffffffu];
        int32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        col[fill[lo]++] = hi;
    }
    free(fill);
    for (int32_t x = 0; x < n; ++x)
        qsort(col + row_off[x], (size_t)(row_off[x + 1] - row_off[x]), sizeof(int32_t), cmp_i32);
}

/* |A & B| of two increasing lists by two-pointer merge. */
static uint64_t merge_count(const int32_t *a, int64_t na, const int32_t *b, int64_t nb)
{
    uint64_t c = 0;
    int64_t i = 0, j = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else { ++c; ++i; ++j; }
    }
    return c;
}

/* Step 5: T = sum over oriented edges (x, y) of |N+(x) & N+(y)|.  Rows are
 * independent, so an OpenMP build may split them across threads (the sum of
 * integers does not depend on the order). */
uint64_t oracle_count(int32_t n, const int64_t *row_off, const int32_t *col)
{
    uint64_t total = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : total)
    for (int32_t x = 0; x < n; ++x) {
        const int32_t *nx = col + row_off[x];
        int64_t dx = row_off[x + 1] - row_off[x];
        for (int64_t t = 0; t < dx; ++t) {
            int32_t y = nx[t];
            total += merge_count(nx, dx, col + row_off[y], row_off[y + 1] - row_off[y]);
        }
    }
    return total;
}

/* Per-edge triangle counts (edge support; the per-edge quantity behind the
 * clustering coefficients of Section 1 and the peeling of k-truss named in
 * Section 3.2).  For the oriented edge at CSR position e, support[e] is the
 * number of triangles containing that edge.  Evaluated from the triangles
 * themselves: every triangle r(a) < r(b) < r(c) is found once, at edge (a, b)
 * with common out-neighbour c (the merge of step 5), and adds one to each of
 * its three edges (a, b), (a, c) and (b, c), located by their positions in
 * the merged lists.  Sequential, so the increments need no atomics. */
void oracle_edge_support(int32_t n, const int64_t *row_off, const int32_t *col, uint32_t *support)
{
    memset(support, 0, sizeof(uint32_t) * (size_t)row_off[n]);
    for (int32_t a = 0; a < n; ++a) {
        const int64_t a0 = row_off[a], da = row_off[a + 1] - a0;
        for (int64_t t = 0; t < da; ++t) {
            const int32_t b = col[a0 + t];
            const int64_t b0 = row_off[b], db = row_off[b + 1] - b0;
            int64_t i = 0, j = 0;
            while (i < da && j < db) {
                const int32_t x = col[a0 + i], y = col[b0 + j];
                if (x < y) {
                    ++i;
                } else if (y < x) {
                    ++j;
                } else {           /* c = x: triangle (a, b, c) */
                    ++support[a0 + t];  /* (a, b) */
                    ++support[a0 + i];  /* (a, c) */
                    ++support[b0 + j];  /* (b, c) */
                    ++i;
                    ++j;
                }
            }
        }
    }
}

/* Per-vertex triangle counts (the numerator of the local clustering
 * coefficient, Section 1): t[x] for rank x is the number of triangles with x
 * as a vertex.  Every triangle r(a) < r(b) < r(c), found once as in step 5,
 * adds one to each of a, b and c.  Sequential. */
void oracle_vertex_counts(int32_t n, const int64_t *row_off, const int32_t *col, uint64_t *t)
{
    memset(t, 0, sizeof(uint64_t) * (size_t)n);
    for (int32_t a = 0; a < n; ++a) {
        const int32_t *na = col + row_off[a];
        const int64_t da = row_off[a + 1] - row_off[a];
        for (int64_t s = 0; s < da; ++s) {
            const int32_t b = na[s];
            const int32_t *nb = col + row_off[b];
            const int64_t db = row_off[b + 1] - row_off[b];
            int64_t i = 0, j = 0;
            while (i < da && j < db) {
                if (na[i] < nb[j]) {
                    ++i;
                } else if (nb[j] < na[i]) {
                    ++j;
                } else {  /* c = na[i] */
                    ++t[a];
                    ++t[b];
                    ++t[na[i]];
                    ++i;
                    ++j;
                }
            }
        }
    }
}

/* k-truss (the peeling algorithm named in Section 3.2): the largest
 * subgraph in which every edge lies in at least k - 2 triangles of the
 * subgraph; it is unique.  Classic peeling, one edge at a time: start from
 * every edge's support; while some remaining edge has support below k - 2,
 * delete it, and for every vertex w still joined to both of its ends take one
 * from the supports of the edges to w (queueing those that fall below).
 * keep[e] = 1 for the oriented CSR positions left; returns their number.
 * Sequential. */
int64_t oracle_ktruss(int32_t n, const int64_t *row_off, const int32_t *col, int32_t k, uint8_t *keep)
{
    const int64_t m = row_off[n];
    if (m == 0) return 0;
    uint32_t *sup = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)m);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    uint8_t *queued = (uint8_t *)calloc((size_t)m, 1);
    /* undirected adjacency with edge positions: adj_off over vertices */
    int64_t *adj_off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * m));
    int64_t *adj_e = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * m));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int32_t x = 0; x < n; ++x)
        for (int64_t e = row_off[x]; e < row_off[x + 1]; ++e) {
            adj_off[x + 1]++;
            adj_off[col[e] + 1]++;
        }
    for (int32_t x = 0; x < n; ++x) adj_off[x + 1] += adj_off[x];
    for (int32_t x = 0; x < n; ++x) fill[x] = adj_off[x];
    /* rows in increasing x: each list receives its lower neighbours in
     * increasing order first, then its higher ones in increasing order */
    for (int32_t x = 0; x < n; ++x)
        for (int64_t e = row_off[x]; e < row_off[x + 1]; ++e) {
            const int32_t y = col[e];
            adj[fill[y]] = x; adj_e[fill[y]++] = e;
        }
    for (int32_t x = 0; x < n; ++x)
        for (int64_t e = row_off[x]; e < row_off[x + 1]; ++e) {
            adj[fill[x]] = col[e]; adj_e[fill[x]++] = e;
        }
    oracle_edge_support(n, row_off, col, sup);
    for (int64_t e = 0; e < m; ++e) keep[e] = 1;
    const uint32_t need = k > 2 ? (uint32_t)(k - 2) : 0u;
    int64_t head = 0, tail = 0;
    for (int64_t e = 0; e < m; ++e)
        if (sup[e] < need) { queue[tail++] = e; queued[e] = 1; }
    while (head < tail) {
        const int64_t e = queue[head++];
        keep[e] = 0;
        /* ends of e: its row (binary search over row_off) and column */
        int32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) / 2;
            if (row_off[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int32_t a = lo, b = col[e];
        int64_t i = adj_off[a], j = adj_off[b];
        while (i < adj_off[a + 1] && j < adj_off[b + 1]) {
            if (adj[i] < adj[j]) { ++i; continue; }
            if (adj[j] < adj[i]) { ++j; continue; }
            const int64_t ea = adj_e[i], eb = adj_e[j];
            if (keep[ea] && keep[eb]) {  /* the triangle (a, b, w) was intact */
                const int64_t two[2] = {ea, eb};
                for (int q = 0; q < 2; ++q) {
                    const int64_t f = two[q];
                    if (!queued[f]) {
                        if (--sup[f] < need) { queue[tail++] = f; queued[f] = 1; }
                    }
                }
            }
            ++i; ++j;
        }
    }
    int64_t left = 0;
    for (int64_t e = 0; e < m; ++e) left += keep[e];
    free(sup); free(queue); free(queued); free(adj_off); free(adj); free(adj_e); free(fill);
    return left;
}

/* 4-cliques (the multi-block pattern family of Section 3.2, one level past
 * triangles): sets of four pairwise adjacent vertices.  Each 4-clique with
 * ranks a < b < c < d is counted once, at the oriented edge (a, b): its
 * other two vertices c < d are both common out-neighbours of a and b, and
 * d is an out-neighbour of c.  So: for every edge (a, b), list
 * C = N+(a) & N+(b) (by merge), and count the pairs c < d of C with d in
 * N+(c) (by binary search in N+(c)).  Sequential; uint64 count. */
static int has_out(const int64_t *row_off, const int32_t *col, int32_t c, int32_t d)
{
    int64_t lo = row_off[c], hi = row_off[c + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (col[mid] < d) lo = mid + 1; else hi = mid;
    }
    return lo < row_off[c + 1] && col[lo] == d;
}

uint64_t oracle_four_cliques(int32_t n, const int64_t *row_off, const int32_t *col)
{
    int32_t maxd = 0;
    for (int32_t x = 0; x < n; ++x)
        if (row_off[x + 1] - row_off[x] > maxd) maxd = (int32_t)(row_off[x + 1] - row_off[x]);
    int32_t *common = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxd > 0 ? maxd : 1));
    uint64_t total = 0;
    for (int32_t a = 0; a < n; ++a) {
        const int32_t *na = col + row_off[a];
        const int64_t da = row_off[a + 1] - row_off[a];
        for (int64_t t = 0; t < da; ++t) {
            const int32_t b = na[t];
            const int32_t *nb = col + row_off[b];
            const int64_t db = row_off[b + 1] - row_off[b];
            int64_t i = 0, j = 0, nc = 0;
            while (i < da && j < db) {
                if (na[i] < nb[j]) ++i;
                else if (nb[j] < na[i]) ++j;
                else { common[nc++] = na[i]; ++i; ++j; }
            }
            for (int64_t x = 0; x < nc; ++x)
                for (int64_t y = x + 1; y < nc; ++y)
                    total += (uint64_t)has_out(row_off, col, common[x], common[y]);
        }
    }
    free(common);
    return total;
}

/* Number of oracle threads an OpenMP build uses (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }
#else
int oracle_threads(void) { return 1; }
void oracle_set_threads(int t) { (void)t; }
#endif

/* Stripe of ranked vertex x under cut vector cuts[0..p] (the largest s with
 * cuts[s] <= x, restricted to s < p). */
static int32_t stripe_of(int32_t x, int32_t p, const int32_t *cuts)
{
    int32_t lo = 0, hi = p - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) / 2;
        if (cuts[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Block mode: out[(i * p + j) * p + k] = T_ijk (zero unless i <= j <= k).
 * cuts must be non-decreasing with cuts[0] = 0 and cuts[p] = n.  Returns -1
 * on a bad cut vector. */
int oracle_block_counts(int32_t n, const int64_t *row_off, const int32_t *col,
                        int32_t p, const int32_t *cuts, uint64_t *out)
{
    if (p < 1 || cuts[0] != 0 || cuts[p] != n) return -1;
    for (int32_t s = 0; s < p; ++s)
        if (cuts[s] > cuts[s + 1]) return -1;
    memset(out, 0, sizeof(uint64_t) * (size_t)p * p * p);
    for (int32_t u = 0; u < n; ++u) {
        const int32_t *nu = col + row_off[u];
        int64_t du = row_off[u + 1] - row_off[u];
        int32_t si = stripe_of(u, p, cuts);
        for (int64_t t = 0; t < du; ++t) {
            int32_t v = nu[t];
            int32_t sj = stripe_of(v, p, cuts);
            const int32_t *nv = col + row_off[v];
            int64_t dv = row_off[v + 1] - row_off[v];
            int64_t a = 0, b = 0;
            while (a < du && b < dv) {
                if (nu[a] < nv[b]) ++a;
                else if (nu[a] > nv[b]) ++b;
                else {
                    int32_t sk = stripe_of(nu[a], p, cuts);
                    out[((size_t)si * p + sj) * p + sk]++;
                    ++a; ++b;
                }
            }
        }
    }
    return 0;
}

/* 4-cliques by block 4-list (PGAbB Section 3.2, the multi-block pattern
 * mode one level past triangles): out[((i * p + j) * p + k) * p + l] = the
 * 4-cliques a < b < c < d (ranks) whose vertices lie in stripes i, j, k and
 * l (so i <= j <= k <= l; zero elsewhere).  Each is found once, at its edge
 * (a, b), as in oracle_four_cliques.  cuts as in oracle_block_counts;
 * returns -1 on a bad cut vector or allocation failure. */
int oracle_four_clique_blocks(int32_t n, const int64_t *row_off, const int32_t *col,
                              int32_t p, const int32_t *cuts, uint64_t *out)
{
    if (p < 1 || cuts[0] != 0 || cuts[p] != n) return -1;
    for (int32_t s = 0; s < p; ++s)
        if (cuts[s] > cuts[s + 1]) return -1;
    memset(out, 0, sizeof(uint64_t) * (size_t)p * p * p * p);
    int32_t maxd = 0;
    for (int32_t x = 0; x < n; ++x)
        if (row_off[x + 1] - row_off[x] > maxd) maxd = (int32_t)(row_off[x + 1] - row_off[x]);
    int32_t *common = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxd > 0 ? maxd : 1));
    if (!common) return -1;
    for (int32_t a = 0; a < n; ++a) {
        const int32_t *na = col + row_off[a];
        const int64_t da = row_off[a + 1] - row_off[a];
        const int32_t si = stripe_of(a, p, cuts);
        for (int64_t t = 0; t < da; ++t) {
            const int32_t b = na[t];
            const int32_t sj = stripe_of(b, p, cuts);
            const int32_t *nb = col + row_off[b];
            const int64_t db = row_off[b + 1] - row_off[b];
            int64_t i = 0, j = 0, nc = 0;
            while (i < da && j < db) {
                if (na[i] < nb[j]) ++i;
                else if (nb[j] < na[i]) ++j;
                else { common[nc++] = na[i]; ++i; ++j; }
            }
            for (int64_t x = 0; x < nc; ++x)
                for (int64_t y = x + 1; y < nc; ++y)
                    if (has_out(row_off, col, common[x], common[y])) {
                        const int32_t sk = stripe_of(common[x], p, cuts), sl = stripe_of(common[y], p, cuts);
                        out[(((size_t)si * p + sj) * p + sk) * p + sl]++;
                    }
        }
    }
    free(common);
    return 0;
}

/* Whole pipeline: clean, degree, rank (mode), orient, count.  Returns
 * UINT64_MAX on an out-of-range id or allocation failure.  If mu_out is not
 * NULL it receives m'. */
uint64_t oracle_tc(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int mode,
                   int64_t *mu_out)
{
    if (n < 0 || m < 0) return UINT64_MAX;
    uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1));
    int32_t *deg = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *row_off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!keys || !deg || !rank || !row_off) {
        free(keys); free(deg); free(rank); free(row_off);
        return UINT64_MAX;
    }
    int64_t mu = oracle_clean(n, m, src, dst, keys);
    uint64_t t = UINT64_MAX;
    if (mu >= 0) {
        int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(mu > 0 ? mu : 1));
        if (col) {
            oracle_degrees(n, keys, mu, deg);
            oracle_rank(n, deg, mode, rank);
            oracle_orient(n, keys, mu, rank, row_off, col);
            t = oracle_count(n, row_off, col);
            free(col);
        }
        if (mu_out) *mu_out = mu;
    }
    free(keys); free(deg); free(rank); free(row_off);
    return t;
}

/* Probe work of the oriented formulation: W = sum over oriented edges (x, y)
 * of |N+(y)|, the number of list elements a merge streams from the second
 * list.  Used to state the algorithmic bytes of a count, not the count.
 * This is what a kernel reads when it walks the partial list of the second
 * endpoint (A_jk[y]) for every edge: in block form the walked lists over all
 * k >= j still cover N+(y) whole, since every out-neighbour of y ranks above
 * y. */
uint64_t oracle_probe_work(int32_t n, const int64_t *row_off, const int32_t *col)
{
    uint64_t w = 0;
    for (int32_t x = 0; x < n; ++x)
        for (int64_t t = row_off[x]; t < row_off[x + 1]; ++t) {
            int32_t y = col[t];
            w += (uint64_t)(row_off[y + 1] - row_off[y]);
        }
    return w;
}

/* Probe work when the kernel walks the first endpoint's partial lists
 * instead: for every oriented edge (x, y) of block A_ij and every k >= j,
 * the list A_ik[x] = N+(x) restricted to stripe k is read, so the work is
 * W_col = sum over oriented edges (x, y) of |{w in N+(x) : stripe(w) >=
 * stripe(y)}|, under the cut vector cuts[0..p].  For p = 1 it is the sum of
 * |N+(x)|^2.  Evaluated here by the definition, pair by pair. */
uint64_t oracle_probe_work_col(int32_t n, const int64_t *row_off, const int32_t *col,
                               int32_t p, const int32_t *cuts)
{
    uint64_t w = 0;
    for (int32_t x = 0; x < n; ++x)
        for (int64_t t = row_off[x]; t < row_off[x + 1]; ++t) {
            int32_t sy = stripe_of(col[t], p, cuts);
            for (int64_t q = row_off[x]; q < row_off[x + 1]; ++q)
                if (stripe_of(col[q], p, cuts) >= sy) ++w;
        }
    return w;
}
