/*
 * Seeded synthetic graph generators (edge lists of int32 vertex ids).
 *
 * These produce the inputs that both the triangle-count library and the
 * independent CPU oracle consume.  Nothing here cleans, orients or counts:
 * the generators only emit raw (src, dst) pairs, possibly with duplicates,
 * reciprocal pairs and self-loops, exactly as drawn.
 *
 * Random numbers come from one counter-based function, the SplitMix64
 * finaliser (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014):
 *     z = x + 0x9E3779B97F4A7C15
 *     z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
 *     z = (z ^ (z >> 27)) * 0x94D049BB133111EB
 *     return z ^ (z >> 31)
 * Draw number c of a stream keyed by k is mix(k + c * GAMMA), so any draw can
 * be recomputed independently of the others and every loop below can run in
 * parallel while staying bit-identical to a serial run.
 *
 * Families:
 *  - R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004): ef * 2^scale directed
 *    samples, each bit of (src, dst) chosen by quadrant probabilities
 *    (a, b, c, d) with no noise and no vertex permutation.
 *  - Erdos-Renyi G(n, m): exactly m distinct non-loop undirected pairs,
 *    drawn by rejection (m clamped to n(n-1)/2).
 *  - Random geometric graph: n points uniform in the unit square, an edge
 *    between every pair at Euclidean distance <= r (no torus wrap).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t x)
{
    uint64_t z = x + GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t key, uint64_t ctr) { return mix64(key + ctr * GAMMA); }

/* Seed of item `index` of configuration `config_id`. */
uint64_t pgabb_gen_seed(uint32_t config_id, uint32_t index)
{
    return mix64(((uint64_t)config_id << 32) | (uint64_t)index);
}

/* Unbiased-enough bounded integer in [0, n): high half of a 64x32 product. */
static inline uint32_t bounded(uint64_t r, uint32_t n)
{
    return (uint32_t)(((r >> 32) * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------ R-MAT */

/* Thresholds are fixed-point (2^32 scale) so the quadrant choice is integer
 * and identical everywhere.  Sample e uses words e*16 .. e*16+15 of the
 * stream; each 64-bit word supplies two 32-bit uniforms (one per level), so
 * scale <= 32 is supported. */
int pgabb_gen_rmat(uint64_t seed, int scale, int64_t num_samples,
                   double a, double b, double c, int32_t *src, int32_t *dst)
{
    if (scale < 1 || scale > 30 || num_samples < 0 || !src || !dst) return -1;
    if (a < 0 || b < 0 || c < 0 || a + b + c > 1.0) return -1;
    const uint64_t ta = (uint64_t)floor(a * 4294967296.0);
    const uint64_t tab = (uint64_t)floor((a + b) * 4294967296.0);
    const uint64_t tabc = (uint64_t)floor((a + b + c) * 4294967296.0);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < num_samples; ++e) {
        uint32_t s = 0, d = 0;
        uint64_t word = 0;
        for (int l = 0; l < scale; ++l) {
            uint32_t u;
            if ((l & 1) == 0) {
                word = draw(seed, (uint64_t)e * 16 + (uint64_t)(l >> 1));
                u = (uint32_t)word;
            } else {
                u = (uint32_t)(word >> 32);
            }
            uint32_t sb, db;
            if (u < ta) { sb = 0; db = 0; }
            else if (u < tab) { sb = 0; db = 1; }
            else if (u < tabc) { sb = 1; db = 0; }
            else { sb = 1; db = 1; }
            s = (s << 1) | sb;
            d = (d << 1) | db;
        }
        src[e] = (int32_t)s;
        dst[e] = (int32_t)d;
    }
    return 0;
}

/* -------------------------------------------------------- Erdos-Renyi G(n,m) */

/* Open-addressing set of 64-bit pair keys (key 0 is never used since the
 * stored key is (lo << 32 | hi) + 1). */
typedef struct { uint64_t *slot; uint64_t mask; } pairset;

static int pairset_insert(pairset *s, uint64_t key)
{
    uint64_t h = mix64(key) & s->mask;
    for (;;) {
        if (s->slot[h] == 0) { s->slot[h] = key; return 1; }
        if (s->slot[h] == key) return 0;
        h = (h + 1) & s->mask;
    }
}

int64_t pgabb_gen_er_num_edges(int32_t n, int64_t m)
{
    if (n < 2 || m <= 0) return 0;
    int64_t maxm = (int64_t)n * (n - 1) / 2;
    return m < maxm ? m : maxm;
}

/* Writes exactly pgabb_gen_er_num_edges(n, m) distinct pairs (u < v not
 * implied: the orientation of each pair is as drawn). */
int pgabb_gen_er(uint64_t seed, int32_t n, int64_t m, int32_t *src, int32_t *dst)
{
    if (n < 0 || m < 0 || (m > 0 && (!src || !dst))) return -1;
    int64_t target = pgabb_gen_er_num_edges(n, m);
    if (target == 0) return 0;
    uint64_t cap = 16;
    while (cap < (uint64_t)target * 2) cap <<= 1;
    pairset set = { (uint64_t *)calloc(cap, sizeof(uint64_t)), cap - 1 };
    if (!set.slot) return -2;
    int64_t have = 0;
    for (uint64_t ctr = 0; have < target; ++ctr) {
        uint64_t r = draw(seed, ctr);
        uint32_t u = bounded(r << 32, (uint32_t)n);
        uint32_t v = bounded(r, (uint32_t)n);
        if (u == v) continue;
        uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
        if (pairset_insert(&set, (((uint64_t)lo << 32) | hi) + 1)) {
            src[have] = (int32_t)u;
            dst[have] = (int32_t)v;
            ++have;
        }
    }
    free(set.slot);
    return 0;
}

/* ------------------------------------------------ random geometric graph */

/* Points: x_i, y_i = top 53 bits of draws 2i, 2i+1, scaled to [0,1).
 * Edge {i,j}, i < j, when (x_i-x_j)^2 + (y_i-y_j)^2 <= r^2.  Edges are
 * emitted with src < dst in increasing (src, dst) order.  With src == NULL
 * only the count is returned; otherwise at most `cap` edges are written. */
static void rgg_points(uint64_t seed, int32_t n, double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) {
        x[i] = (double)(draw(seed, 2 * (uint64_t)i) >> 11) * (1.0 / 9007199254740992.0);
        y[i] = (double)(draw(seed, 2 * (uint64_t)i + 1) >> 11) * (1.0 / 9007199254740992.0);
    }
}

int64_t pgabb_gen_rgg(uint64_t seed, int32_t n, double radius,
                      int32_t *src, int32_t *dst, int64_t cap)
{
    if (n < 0 || !(radius >= 0)) return -1;
    if (n < 2) return 0;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!x || !y) { free(x); free(y); return -2; }
    rgg_points(seed, n, x, y);
    /* grid of cells of side >= radius */
    int g = radius > 0 ? (int)floor(1.0 / radius) : 1;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    int32_t *cell_start = (int32_t *)calloc((size_t)g * g + 1, sizeof(int32_t));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!cell_start || !order || !cell_of) {
        free(x); free(y); free(cell_start); free(order); free(cell_of);
        return -2;
    }
    for (int32_t i = 0; i < n; ++i) {
        int cx = (int)(x[i] * g), cy = (int)(y[i] * g);
        if (cx >= g) cx = g - 1;
        if (cy >= g) cy = g - 1;
        cell_of[i] = cy * g + cx;
        cell_start[cell_of[i] + 1]++;
    }
    for (int c = 0; c < g * g; ++c) cell_start[c + 1] += cell_start[c];
    {
        int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)g * g);
        memcpy(fill, cell_start, sizeof(int32_t) * (size_t)g * g);
        for (int32_t i = 0; i < n; ++i) order[fill[cell_of[i]]++] = i;
        free(fill);
    }
    const double r2 = radius * radius;
    int64_t count = 0;
    for (int32_t i = 0; i < n; ++i) {
        int cx = cell_of[i] % g, cy = cell_of[i] / g;
        /* collect neighbours j > i from the 3x3 cell neighbourhood, then emit
         * them in increasing j so the output order is canonical */
        int32_t lo_y = cy > 0 ? cy - 1 : 0, hi_y = cy < g - 1 ? cy + 1 : g - 1;
        int32_t lo_x = cx > 0 ? cx - 1 : 0, hi_x = cx < g - 1 ? cx + 1 : g - 1;
        int64_t first = count;
        for (int32_t yy = lo_y; yy <= hi_y; ++yy)
            for (int32_t xx = lo_x; xx <= hi_x; ++xx) {
                int c = yy * g + xx;
                for (int32_t t = cell_start[c]; t < cell_start[c + 1]; ++t) {
                    int32_t j = order[t];
                    if (j <= i) continue;
                    double dx = x[i] - x[j], dy = y[i] - y[j];
                    if (dx * dx + dy * dy <= r2) {
                        if (src && count < cap) { src[count] = i; dst[count] = j; }
                        ++count;
                    }
                }
            }
        /* insertion sort of this vertex's dst values into increasing order */
        if (src) {
            int64_t last = count < cap ? count : cap;
            for (int64_t a = first + 1; a < last; ++a) {
                int32_t key = dst[a];
                int64_t b = a - 1;
                while (b >= first && dst[b] > key) { dst[b + 1] = dst[b]; --b; }
                dst[b + 1] = key;
            }
        }
    }
    free(x); free(y); free(cell_start); free(order); free(cell_of);
    return count;
}

/* ------------------------------------------------------------- scalars */

/* Integer uniform in [lo, hi] from draw `ctr` of stream `key`. */
int64_t pgabb_gen_uniform_int(uint64_t key, uint64_t ctr, int64_t lo, int64_t hi)
{
    if (hi < lo) return lo;
    uint64_t span = (uint64_t)(hi - lo) + 1;
    unsigned __int128 prod = (unsigned __int128)draw(key, ctr) * span;
    return lo + (int64_t)(uint64_t)(prod >> 64);
}

/* Double uniform in [0, 1) (53 bits) from draw `ctr` of stream `key`. */
double pgabb_gen_unit(uint64_t key, uint64_t ctr)
{
    return (double)(draw(key, ctr) >> 11) * (1.0 / 9007199254740992.0);
}
