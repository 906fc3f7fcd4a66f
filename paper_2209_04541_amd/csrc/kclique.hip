// 4-cliques (the multi-block pattern family of PGAbB Section 3.2, one
// intersection level past triangles).  Each 4-clique with ranks
// a < b < c < d is counted once, at its oriented edge (a, b): c runs over
// the common out-neighbours of a and b, and d over the entries after c that
// N+(a), N+(b) and N+(c) share.  The oriented graph is taken as one block
// (p = 1).
//
// Rows of up to kCliqueCap entries: one wave owns a row a and stages N+(a)
// in LDS.  For each b in it, the lanes look the entries of N+(b) up in the
// staged row and mark the common ones, C, in a bitmask over its positions;
// then they walk N+(c) for every c in C, flattened over the lanes, and count
// the entries that land on a marked position after c.  Longer rows: one
// thread per edge merges N+(a) (from b on) with N+(b) and, at every common
// entry c, merges the three lists from c on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>

#include "common.hpp"
#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

constexpr int kQB = 256;
constexpr int kCliqueCap = 1024;  // longest row a wave stages
constexpr int kCliqueWaves = 4;
constexpr int kCliqueSpan = 8;  // b's of a row per work item

// Work items per row: rows of 3 to kCliqueCap entries, kCliqueSpan b's each.
__global__ __launch_bounds__(kQB) void k_clique_items(const int64_t *__restrict__ row_off, int32_t n,
                                                       int64_t *__restrict__ items) {
    for (int64_t a = blockIdx.x * static_cast<int64_t>(kQB) + threadIdx.x; a < n;
         a += static_cast<int64_t>(gridDim.x) * kQB) {
        const int64_t d = row_off[a + 1] - row_off[a];
        items[a] = (d >= 3 && d <= kCliqueCap) ? (d - 2 + kCliqueSpan - 1) / kCliqueSpan : 0;
    }
}

struct CliqueLds {
    int32_t row[kCliqueCap];          // N+(a)
    int32_t mem[kCliqueCap];          // positions of C in the row
    uint32_t mask[kCliqueCap / 32];   // C as a bitmask over positions
    int64_t incl[kWave];              // inclusive prefix of the chunk's list lengths
    int64_t start[kWave];             // CSR start of each member's list
    int32_t pos[kWave];               // row position of each member
};

// First position in [lo, hi) of the staged row whose value is at least x.
__device__ __forceinline__ int32_t lds_lower_bound(const int32_t *row, int32_t lo, int32_t hi, int32_t x) {
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (row[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kCliqueWaves *kWave) void k_four_cliques_rows(const int64_t *__restrict__ row_off,
                                                                            const int32_t *__restrict__ col,
                                                                            int32_t n,
                                                                            const int64_t *__restrict__ item_pre,
                                                                            unsigned long long *__restrict__ next,
                                                                            unsigned long long *__restrict__ total) {
    __shared__ CliqueLds s_lds[kCliqueWaves];
    CliqueLds &L = s_lds[threadIdx.x / kWave];
    const int lane = lane_id();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;  // lanes under this one
    gptr<int64_t> ro = as_global(row_off);
    gptr<int32_t> cl = as_global(col);
    gptr<int64_t> ip = as_global(item_pre);
    const int64_t nitems = ip[n];
    unsigned long long cnt = 0;
    for (;;) {
        unsigned long long q0 = 0;
        if (lane == 0) q0 = atomicAdd(next, 1ull);
        q0 = shfl_t(q0, 0);
        if (q0 >= static_cast<unsigned long long>(nitems)) break;
        const int64_t q = static_cast<int64_t>(q0);
        int32_t a = 0, ahi = n - 1;  // the row holding item q: the last with item_pre <= q
        while (a < ahi) {
            const int32_t mid = (a + ahi + 1) >> 1;
            if (ip[mid] <= q) a = mid;
            else ahi = mid - 1;
        }
        const int64_t a0 = ro[a];
        const int32_t d = static_cast<int32_t>(ro[a + 1] - a0);
        const int32_t i_lo = static_cast<int32_t>(q - ip[a]) * kCliqueSpan;
        const int32_t i_hi = min(i_lo + kCliqueSpan, d - 2);
        for (int x = lane; x < d; x += kWave) L.row[x] = cl[a0 + x];
        wave_lds_sync();
        const int32_t top = L.row[d - 1];
        const int nwords = (d + 31) >> 5;
        for (int32_t i = i_lo; i < i_hi; ++i) {
            const int32_t b = L.row[i];
            const int64_t b0 = ro[b];
            const int64_t db = ro[b + 1] - b0;
            if (db < 2) continue;
            for (int w = lane; w < nwords; w += kWave) L.mask[w] = 0;
            wave_lds_sync();
            for (int64_t t = lane; t < db; t += kWave) {
                const int32_t x = cl[b0 + t];
                if (x > top) break;  // the list is sorted
                const int32_t j = lds_lower_bound(L.row, i + 1, d, x);
                if (j < d && L.row[j] == x) atomicOr(&L.mask[j >> 5], 1u << (j & 31));
            }
            wave_lds_sync();
            int32_t nc = 0;  // members of C, listed in row order
            for (int32_t j0 = i + 1; j0 < d; j0 += kWave) {
                const int32_t j = j0 + lane;
                const bool in = j < d && ((L.mask[j >> 5] >> (j & 31)) & 1u);
                const uint64_t bal = __ballot(in);
                if (in) L.mem[nc + __popcll(bal & below)] = j;
                nc += __popcll(bal);
            }
            wave_lds_sync();
            if (nc < 2) continue;
            for (int32_t m0 = 0; m0 < nc; m0 += kWave) {
                const int32_t k = m0 + lane;
                int64_t len = 0, st = 0;
                int32_t pc = 0;
                if (k < nc) {
                    pc = L.mem[k];
                    const int32_t c = L.row[pc];
                    st = ro[c];
                    len = ro[c + 1] - st;
                }
                const int64_t incl = wave_inclusive_scan(len);
                const int64_t tot = shfl_t(incl, kWave - 1);
                wave_lds_sync();  // the previous chunk's lookups are done
                L.incl[lane] = incl;
                L.start[lane] = st;
                L.pos[lane] = pc;
                wave_lds_sync();
                int lo = 0;
                for (int64_t f = 0; f < tot; f += kWave) {
                    const int64_t q = f + lane;
                    if (q >= tot) continue;
                    while (L.incl[lo] <= q) ++lo;  // lists hold q in order; q < tot = incl[63]
                    const int32_t y = cl[L.start[lo] + (q - (lo ? L.incl[lo - 1] : 0))];
                    if (y > top) continue;
                    const int32_t j2 = lds_lower_bound(L.row, L.pos[lo] + 1, d, y);
                    if (j2 < d && L.row[j2] == y && ((L.mask[j2 >> 5] >> (j2 & 31)) & 1u)) ++cnt;
                }
            }
            wave_lds_sync();  // before the next b clears the mask
        }
        wave_lds_sync();  // before the next row is staged
    }
    cnt = wave_sum(cnt);
    if (lane == 0 && cnt) atomicAdd(total, cnt);
}

__global__ __launch_bounds__(kQB) void k_four_cliques(const int64_t *__restrict__ row_off,
                                                       const int32_t *__restrict__ col, int32_t n, int64_t m,
                                                       unsigned long long *__restrict__ total) {
    gptr<int64_t> ro = as_global(row_off);
    gptr<int32_t> cl = as_global(col);
    unsigned long long cnt = 0;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kQB) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kQB) {
        int32_t lo = 0, hi = n - 1;  // row a of e: the last row whose offset is at most e
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (ro[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        if (ro[lo + 1] - ro[lo] <= kCliqueCap) continue;  // the row waves take it
        const int32_t b = cl[e];
        const int64_t ea = ro[lo + 1], eb = ro[b + 1];
        int64_t i = e + 1, j = ro[b];
        while (i < ea && j < eb) {
            const int32_t x = cl[i], y = cl[j];
            if (x < y) {
                ++i;
            } else if (y < x) {
                ++j;
            } else {  // c = x: count the entries after c common to N+(a), N+(b), N+(c)
                int64_t p = ro[x];
                const int64_t pe = ro[x + 1];
                int64_t u = i + 1, v = j + 1;
                while (p < pe && u < ea && v < eb) {
                    const int32_t X = cl[p], Y = cl[u], Z = cl[v];
                    const int32_t M = max(X, max(Y, Z));
                    if (X == M && Y == M && Z == M) {
                        ++cnt;
                        ++p;
                        ++u;
                        ++v;
                    } else {
                        p += X < M;
                        u += Y < M;
                        v += Z < M;
                    }
                }
                ++i;
                ++j;
            }
        }
    }
    cnt = wave_sum(cnt);
    if (lane_id() == 0 && cnt) atomicAdd(total, cnt);
}

}  // namespace

uint64_t four_cliques(pgabb_graph *g) {
    hipStream_t s = g->stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t m = g->m;
    uint64_t result = 0;
    g->t_kernel_ms = 0;
    g->kernel_launches = 0;
    if (m > 0) {
        DArray<unsigned long long> tot(2, s);  // count, item counter
        PGABB_HIP(hipMemsetAsync(tot.get(), 0, 2 * sizeof(unsigned long long), s));
        const unsigned grid = std::min<unsigned>(grid_for(m, kQB), 256u * 16u);
        // work items of the staged rows: kCliqueSpan b's of one row each
        DArray<int64_t> item_pre(static_cast<size_t>(g->n) + 1, s);
        k_clique_items<<<grid_for(g->n, kQB), kQB, 0, s>>>(g->row_off.get(), g->n, item_pre.get());
        PGABB_HIP(hipGetLastError());
        scan_exclusive_i64(item_pre.get(), item_pre.get(), g->n, item_pre.get() + g->n, s);
        const int rgrid = 256 * 4;
        StreamTimer tm;
        tm.start(s);
        k_four_cliques_rows<<<rgrid, kCliqueWaves * kWave, 0, s>>>(g->row_off.get(), g->col.get(), g->n,
                                                                    item_pre.get(), tot.get() + 1, tot.get());
        if (g->max_out > kCliqueCap)
            k_four_cliques<<<grid, kQB, 0, s>>>(g->row_off.get(), g->col.get(), g->n, m, tot.get());
        PGABB_HIP(hipGetLastError());
        tm.stop(s);
        Staged<unsigned long long> h(1, s);
        PGABB_HIP(hipMemcpyAsync(h.get(), tot.get(), sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        result = h[0];
        g->t_kernel_ms = tm.ms();
        g->kernel_launches = g->max_out > kCliqueCap ? 2 : 1;
    }
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return result;
}

}  // namespace pgabb
