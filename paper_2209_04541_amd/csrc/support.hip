// Triangles containing each edge (edge support): the per-edge quantity behind
// clustering coefficients (PGAbB Section 1) and the peeling of k-truss
// (Section 3.2), from the same intersections as the count (Section 3.6) with
// a different reduction.  The oriented graph is taken as one block (p = 1):
// every triangle r(a) < r(b) < r(c) is found once, as the common entry c of
// N+(a) and N+(b) for the edge (a, b), and adds one to each of its edges
// (a, b), (a, c) and (b, c).
//
// The edge is reached from its higher end: one wave owns a vertex b at a
// time, stages N+(b) in LDS with one counter per entry, and for every
// in-edge (a, b) walks the part of N+(a) after b (only c > b can lie in
// N+(b)), flattened over the lanes, 64 in-edges at a time, looking each
// walked entry up in the staged row by binary search.  This reads
// sum_a d+(a) (d+(a) - 1) / 2 entries, against sum over edges (a, b) of
// d+(b) when every N+(b) is walked from the lower end (3.6 x more on R-MAT
// scale 20).  A hit counts (b, c) in LDS (flushed once per owner), (a, b) in
// a per-in-edge LDS counter (flushed once per 64 in-edges) and (a, c), the
// walked entry, with a device atomic.  Owners are taken from the highest rank
// down: the hubs, whose in-edges are many, start first.  Rows longer than the
// LDS region are searched and counted in device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>

#include "common.hpp"
#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

constexpr int kSupWaves = 4;
constexpr int kSupCap = 1024;  // longest row staged in LDS
constexpr int kSupB = 256;
constexpr int kSupUnroll = 4;       // walked entries per lane whose loads are in flight together
constexpr int kSupFilterBits = 4096;  // hashed bitmap of the staged row

struct SupportLds {
    int32_t row[kSupCap];   // N+(b)
    uint32_t cnt[kSupCap];  // triangles found so far on edge (b, row[x])
    uint32_t filter[kSupFilterBits / 32];
    int64_t incl[kWave];    // inclusive prefix of the chunk's walk lengths
    int64_t start[kWave];   // CSR position where each walk starts
    uint32_t eab[kWave];    // CSR position of each in-edge (a, b)
    uint32_t hits[kWave];   // triangles found on each in-edge
};

__device__ __forceinline__ uint32_t filter_bit(int32_t c) {
    return (static_cast<uint32_t>(c) * 0x9E3779B1u) >> 20;  // 12 bits
}

// Row of every CSR position: the last row whose offset is at most e.
__global__ __launch_bounds__(kSupB) void k_sup_rows(const int64_t *__restrict__ row_off, int32_t n, int64_t m,
                                                     int32_t *__restrict__ rows) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kSupB) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kSupB) {
        int32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (row_off[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        rows[e] = lo;
    }
}

// Sort keys (the higher end of each edge) and values (its CSR position).
__global__ __launch_bounds__(kSupB) void k_sup_pairs(const int32_t *__restrict__ col, int64_t m,
                                                      uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kSupB) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kSupB) {
        key[e] = static_cast<uint32_t>(col[e]);
        val[e] = static_cast<uint32_t>(e);
    }
}

__global__ __launch_bounds__(kSupB) void k_sup_widen(const int32_t *__restrict__ in, int32_t n,
                                                      int64_t *__restrict__ out) {
    for (int64_t v = blockIdx.x * static_cast<int64_t>(kSupB) + threadIdx.x; v < n;
         v += static_cast<int64_t>(gridDim.x) * kSupB)
        out[v] = in[v];
}

__global__ __launch_bounds__(kSupWaves *kWave) void k_edge_support(const int64_t *__restrict__ row_off,
                                                                    const int32_t *__restrict__ col,
                                                                    const int64_t *__restrict__ in_off,
                                                                    const uint32_t *__restrict__ in_pos,
                                                                    const int32_t *__restrict__ rows, int32_t n,
                                                                    uint32_t *__restrict__ support,
                                                                    unsigned long long *__restrict__ next,
                                                                    unsigned long long *__restrict__ total) {
    __shared__ SupportLds s_lds[kSupWaves];
    SupportLds &L = s_lds[threadIdx.x / kWave];
    const int lane = lane_id();
    gptr<int64_t> ro = as_global(row_off);
    gptr<int32_t> cl = as_global(col);
    gptr<int64_t> io = as_global(in_off);
    gptr<uint32_t> ip = as_global(in_pos);
    gptr<int32_t> rw = as_global(rows);
    unsigned long long found = 0;
    for (;;) {
        unsigned long long q0 = 0;
        if (lane == 0) q0 = atomicAdd(next, 1ull);
        q0 = shfl_t(q0, 0);
        if (q0 >= static_cast<unsigned long long>(n)) break;
        const int32_t b = n - 1 - static_cast<int32_t>(q0);
        const int64_t b0 = ro[b];
        const int32_t d = static_cast<int32_t>(ro[b + 1] - b0);
        const int64_t i0 = io[b];
        const int64_t nin = io[b + 1] - i0;
        if (d == 0 || nin == 0) continue;
        const bool staged = d <= kSupCap;
        for (int x = lane; x < kSupFilterBits / 32; x += kWave) L.filter[x] = staged ? 0u : ~0u;
        wave_lds_sync();
        if (staged) {
            for (int x = lane; x < d; x += kWave) {
                const int32_t v = cl[b0 + x];
                L.row[x] = v;
                L.cnt[x] = 0;
                const uint32_t h = filter_bit(v);
                atomicOr(&L.filter[h >> 5], 1u << (h & 31));
            }
            wave_lds_sync();
        }
        auto row_at = [&](int32_t x) { return staged ? L.row[x] : cl[b0 + x]; };
        const int32_t hi_b = row_at(d - 1);  // no c above N+(b)'s last entry can match
        for (int64_t c0 = 0; c0 < nin; c0 += kWave) {
            const int64_t k = c0 + lane;
            int64_t len = 0, s0 = 0;
            uint32_t eab = 0;
            if (k < nin) {
                eab = ip[i0 + k];
                s0 = static_cast<int64_t>(eab) + 1;
                len = ro[rw[eab] + 1] - s0;
            }
            const int64_t incl = wave_inclusive_scan(len);
            const int64_t tot = shfl_t(incl, kWave - 1);
            wave_lds_sync();  // the previous chunk's flush and lookups are done
            L.incl[lane] = incl;
            L.start[lane] = s0;
            L.eab[lane] = eab;
            L.hits[lane] = 0;
            wave_lds_sync();
            // A lane's flat entries rise by 64, so the walk holding them only
            // moves forward: the first walk with incl > q (q < tot = incl[63]
            // keeps it below 64).  Hits on a lane's current walk gather in a
            // register and go to the walk's LDS counter when it moves on.
            int lo = 0, acc_lo = 0;
            uint32_t acc = 0;
            for (int64_t f = 0; f < tot; f += static_cast<int64_t>(kWave) * kSupUnroll) {
                int32_t cv[kSupUnroll];
                int64_t ev[kSupUnroll];
                int lv[kSupUnroll];
#pragma unroll
                for (int u = 0; u < kSupUnroll; ++u) {
                    const int64_t q = f + u * kWave + lane;
                    lv[u] = -1;
                    cv[u] = 0;
                    ev[u] = 0;
                    if (q < tot) {
                        while (L.incl[lo] <= q) ++lo;
                        ev[u] = L.start[lo] + (q - (lo ? L.incl[lo - 1] : 0));
                        lv[u] = lo;
                        cv[u] = cl[ev[u]];
                    }
                }
#pragma unroll
                for (int u = 0; u < kSupUnroll; ++u) {
                    const int32_t c = cv[u];
                    if (lv[u] < 0 || c > hi_b) continue;
                    const uint32_t h = filter_bit(c);
                    if (!(L.filter[h >> 5] & (1u << (h & 31)))) continue;
                    int32_t s = 0, e = d;
                    while (s < e) {
                        const int32_t mid = (s + e) >> 1;
                        if (row_at(mid) < c) s = mid + 1;
                        else e = mid;
                    }
                    if (s < d && row_at(s) == c) {
                        ++found;
                        atomicAdd(&support[ev[u]], 1u);
                        if (lv[u] != acc_lo) {
                            if (acc) atomicAdd(&L.hits[acc_lo], acc);
                            acc_lo = lv[u];
                            acc = 0;
                        }
                        ++acc;
                        if (staged) atomicAdd(&L.cnt[s], 1u);
                        else atomicAdd(&support[b0 + s], 1u);
                    }
                }
            }
            if (acc) atomicAdd(&L.hits[acc_lo], acc);
            wave_lds_sync();
            if (k < nin && L.hits[lane]) atomicAdd(&support[L.eab[lane]], L.hits[lane]);
        }
        if (staged) {
            wave_lds_sync();
            for (int x = lane; x < d; x += kWave)
                if (L.cnt[x]) atomicAdd(&support[b0 + x], L.cnt[x]);
            wave_lds_sync();  // before the next owner is staged
        }
    }
    found = wave_sum(found);
    if (lane == 0 && found) atomicAdd(total, found);
}

}  // namespace

uint64_t edge_support(pgabb_graph *g, uint32_t *out, bool out_on_device) {
    hipStream_t s = g->stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t m = g->m;
    const int32_t n = g->n;
    g->t_kernel_ms = 0;
    g->kernel_launches = 0;
    g->h2d_bytes = 0;
    uint64_t triangles = 0;
    if (m > 0) {
        PGABB_REQUIRE(m < (int64_t{1} << 32), PGABB_EINVAL, "edge support needs m' < 2^32 (m' = %lld)",
                      static_cast<long long>(m));
        DArray<uint32_t> own;
        uint32_t *sup = out;
        if (!out_on_device) {
            own.reset(static_cast<size_t>(m), s);
            sup = own.get();
        }
        // in-edges of every vertex: CSR positions sorted by the higher end
        // (stable, so ascending in the lower end), offsets from the kept
        // in-degrees
        DArray<int32_t> rows(static_cast<size_t>(m), s);
        DArray<uint32_t> key(static_cast<size_t>(m), s), key_alt(static_cast<size_t>(m), s);
        DArray<uint32_t> pos(static_cast<size_t>(m), s), pos_alt(static_cast<size_t>(m), s);
        DArray<int64_t> in_off(static_cast<size_t>(n) + 1, s);
        k_sup_rows<<<grid_for(m, kSupB), kSupB, 0, s>>>(g->row_off.get(), n, m, rows.get());
        k_sup_pairs<<<grid_for(m, kSupB), kSupB, 0, s>>>(g->col.get(), m, key.get(), pos.get());
        k_sup_widen<<<grid_for(n, kSupB), kSupB, 0, s>>>(g->indeg.get(), n, in_off.get());
        PGABB_HIP(hipGetLastError());
        scan_exclusive_i64(in_off.get(), in_off.get(), n, in_off.get() + n, s);
        const bool alt = radix_sort_u32(key.get(), key_alt.get(), pos.get(), pos_alt.get(), m, g->nb, s);
        const uint32_t *in_pos = alt ? pos_alt.get() : pos.get();
        key.release();
        key_alt.release();

        DArray<unsigned long long> ctr(2, s);  // owner counter, triangles
        PGABB_HIP(hipMemsetAsync(ctr.get(), 0, 2 * sizeof(unsigned long long), s));
        PGABB_HIP(hipMemsetAsync(sup, 0, sizeof(uint32_t) * static_cast<size_t>(m), s));
        // four workgroups of four waves fit a CU's LDS
        const int64_t want = (static_cast<int64_t>(n) + kSupWaves - 1) / kSupWaves;
        const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, 256 * 4)));
        StreamTimer tm;
        tm.start(s);
        k_edge_support<<<grid, kSupWaves * kWave, 0, s>>>(g->row_off.get(), g->col.get(), in_off.get(), in_pos,
                                                           rows.get(), n, sup, ctr.get(), ctr.get() + 1);
        PGABB_HIP(hipGetLastError());
        tm.stop(s);
        Staged<unsigned long long> h(1, s);
        PGABB_HIP(hipMemcpyAsync(h.get(), ctr.get() + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        if (!out_on_device)
            PGABB_HIP(hipMemcpyAsync(out, sup, sizeof(uint32_t) * static_cast<size_t>(m), hipMemcpyDeviceToHost,
                                     s));
        PGABB_HIP(hipStreamSynchronize(s));
        triangles = h[0];
        g->t_kernel_ms = tm.ms();
        g->kernel_launches = 1;
    }
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return triangles;
}

}  // namespace pgabb
