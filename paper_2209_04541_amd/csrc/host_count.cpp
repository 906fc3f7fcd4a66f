// Host kernel K_H of the hybrid scheduler: counts one block-list from the
// block chunks held in host memory.
//
// PGAbB Section 3.6 gives one kernel body for both sides: for every edge
// (u, v) of A_ij the common entries of row u of A_ik and row v of A_jk; on
// the host it runs as a plain loop over the rows, one host thread per task
// (Section 4.4: light tasks go to CPU threads).  Both lists hold local ids of
// stripe k in increasing order, so a two-pointer merge finds the common
// entries; when one list is much shorter, its entries are looked up in the
// other by galloping binary search instead.
#include <algorithm>

#include "count.hpp"
#include "graph.hpp"

namespace pgabb {

namespace {

// |a ∩ b| for sorted lists a[0, na), b[0, nb) of distinct ids.
uint64_t intersect_sorted(const int32_t *a, int64_t na, const int32_t *b, int64_t nb) {
    if (na == 0 || nb == 0) return 0;
    if (na > nb) {
        std::swap(a, b);
        std::swap(na, nb);
    }
    uint64_t c = 0;
    if (nb > 32 * na) {
        // galloping: each entry of the short list is searched in the rest of
        // the long one, starting where the previous search ended
        const int32_t *lo = b, *end = b + nb;
        for (int64_t q = 0; q < na && lo < end; ++q) {
            lo = std::lower_bound(lo, end, a[q]);
            if (lo < end && *lo == a[q]) {
                ++c;
                ++lo;
            }
        }
        return c;
    }
    int64_t x = 0, y = 0;
    while (x < na && y < nb) {
        const int32_t u = a[x], v = b[y];
        c += u == v;
        x += u <= v;
        y += v <= u;
    }
    return c;
}

}  // namespace

uint64_t host_count_task(const pgabb_graph *g, const int32_t *arena, const Task &t) {
    const BlockInfo &ij = g->blocks[t.bij], &ik = g->blocks[t.bik], &jk = g->blocks[t.bjk];
    const int32_t *ij_rptr = arena + ij.off_rptr(), *ij_col = arena + ij.off_col();
    const int32_t *ik_rptr = arena + ik.off_rptr(), *ik_col = arena + ik.off_col();
    const int32_t *jk_rptr = arena + jk.off_rptr(), *jk_col = arena + jk.off_col();
    // A_ij and A_ik share stripe i's dense row range (same width), so row u
    // of one is row u of the other; the local column v of A_ij is row v of
    // A_jk.
    uint64_t c = 0;
    for (int32_t u = 0; u < ij.width; ++u) {
        const int32_t sb = ik_rptr[u], se = ik_rptr[u + 1];
        if (se == sb) continue;
        for (int32_t e = ij_rptr[u]; e < ij_rptr[u + 1]; ++e) {
            const int32_t v = ij_col[e];
            const int32_t wb = jk_rptr[v], we = jk_rptr[v + 1];
            c += intersect_sorted(ik_col + sb, se - sb, jk_col + wb, we - wb);
        }
    }
    return c;
}

}  // namespace pgabb
