// Triangles containing each edge (edge support): the per-edge quantity behind
// clustering coefficients (PGAbB Section 1) and the peeling of k-truss
// (Section 3.2), from the same intersections as the count (Section 3.6) with
// a different reduction.  The oriented graph is taken as one block (p = 1):
// every triangle r(a) < r(b) < r(c) is found once, as the common entry c of
// N+(a) and N+(b) for the edge (a, b), and adds one to each of its edges
// (a, b), (a, c) and (b, c).
//
// The edge is reached from its higher end: one wave owns a vertex b at a
// time, stages N+(b) in an LDS hash table (each key with its position in the
// row, and one counter per position), and for every in-edge (a, b) walks the
// part of N+(a) after b (only c > b can lie in N+(b)), flattened over the
// lanes, 64 in-edges at a time, looking each walked entry up in the table.
// This reads sum_a d+(a) (d+(a) - 1) / 2 entries, against sum over edges
// (a, b) of d+(b) when every N+(b) is walked from the lower end (3.6 x more
// on R-MAT scale 20).  A hit counts (b, c) in LDS (flushed once per unit),
// (a, b) in a per-in-edge LDS counter (flushed once per unit) and
// (a, c), the walked entry, with a device atomic.  Work units are runs of at
// most 64 in-edges of one owner (one per lane), so an owner with many
// in-edges spreads over many waves (each stages N+(b) and flushes its own
// counters; 64 measured faster than 128 – 1024);
// units are listed from the highest rank down (the hubs, whose in-edges are
// many, start first), only for owners with both in-edges and a non-empty
// row, and dealt round-robin to eight work counters.  Rows longer than the
// LDS region are searched and counted in device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>

#include "common.hpp"
#include "graph.hpp"
#include "tc_device.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

constexpr int kSupWaves = 4;
constexpr int kSupCap = 682;      // longest row staged in LDS (table load <= 2/3)
constexpr int kSupTableLg = 10;   // at most 1024 hash slots
constexpr int kSupB = 256;
constexpr int kSupUnroll = 2;     // walk chunks in flight
constexpr int kSupUnitEdges = kWave;  // in-edges per work unit (one per lane)
constexpr int kSupQueues = 8;       // work counters, kSupQueueStride words apart
constexpr int kSupQueueStride = 32;

struct SupportLds {
    int32_t key[1 << kSupTableLg];      // hash table of N+(b): entry, or -1
    int16_t pos[1 << kSupTableLg];      // its position in the row
    uint32_t cnt[kSupCap];              // triangles found so far on edge (b, row[x])
    uint32_t hits[kWave];               // triangles found on each in-edge of the group
    int32_t own[kSupUnroll * kWave];    // list positions of the flattened walk
};

// Entries after every CSR position in its row (a thread per row): the
// length of the walk an in-edge at that position starts.
__global__ __launch_bounds__(kSupB) void k_sup_rest(const int64_t *__restrict__ row_off, int32_t n,
                                                     int32_t *__restrict__ rest) {
    for (int64_t a = blockIdx.x * static_cast<int64_t>(kSupB) + threadIdx.x; a < n;
         a += static_cast<int64_t>(gridDim.x) * kSupB) {
        const int64_t end = row_off[a + 1];
        for (int64_t e = row_off[a]; e < end; ++e) rest[e] = static_cast<int32_t>(end - e - 1);
    }
}

// The walk length of every in-edge, in in-edge order.
__global__ __launch_bounds__(kSupB) void k_sup_in_len(const uint32_t *__restrict__ in_pos,
                                                       const int32_t *__restrict__ rest, int64_t m,
                                                       int32_t *__restrict__ in_len) {
    for (int64_t k = blockIdx.x * static_cast<int64_t>(kSupB) + threadIdx.x; k < m;
         k += static_cast<int64_t>(gridDim.x) * kSupB)
        in_len[k] = rest[in_pos[k]];
}

// Work units of every owner, in processing order (rank n - 1 first): one per
// kSupUnitEdges in-edges when the owner has in-edges and a non-empty row.
__global__ __launch_bounds__(kSupB) void k_sup_unit_counts(const int64_t *__restrict__ row_off,
                                                            const int64_t *__restrict__ in_off, int32_t n,
                                                            int64_t *__restrict__ units) {
    for (int64_t r = blockIdx.x * static_cast<int64_t>(kSupB) + threadIdx.x; r < n;
         r += static_cast<int64_t>(gridDim.x) * kSupB) {
        const int64_t b = n - 1 - r;
        const int64_t d = row_off[b + 1] - row_off[b], nin = in_off[b + 1] - in_off[b];
        units[r] = (d > 0 && nin > 0) ? (nin + kSupUnitEdges - 1) / kSupUnitEdges : 0;
    }
}

// The unit list: (owner, first in-edge of the owner's unit).
__global__ __launch_bounds__(kSupB) void k_sup_unit_fill(const int64_t *__restrict__ upre, int32_t n,
                                                          int2 *__restrict__ units) {
    for (int64_t r = blockIdx.x * static_cast<int64_t>(kSupB) + threadIdx.x; r < n;
         r += static_cast<int64_t>(gridDim.x) * kSupB) {
        const int64_t u0 = upre[r], c = upre[r + 1] - u0;
        for (int64_t j = 0; j < c; ++j)
            units[u0 + j] = make_int2(static_cast<int32_t>(n - 1 - r), static_cast<int32_t>(j * kSupUnitEdges));
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

// Loads elements base + q * 64 + lane (q < U) of the flattened walk over the
// in-edge lists of the group (lane l: positions pb .. pb + len of the column
// array, at position pre of the walk), with their column positions and the
// lane whose list holds each; past total a lane gets value -1.  Lists are
// found as in walk_load: list starts scattered into `own`, then a running
// maximum over the lanes.
template <int U>
__device__ __forceinline__ void sup_walk_load(int32_t (&w)[U], uint32_t (&ev)[U], int32_t (&sl)[U], int32_t base,
                                              int32_t total, int32_t pre, int32_t len, uint32_t pb, uint32_t &carry,
                                              int32_t *own, gptr<int32_t> cl, int lane) {
    const int32_t p = pre - base;
    if (len > 0 && p >= 0 && p < U * kWave) own[p] = lane + 1;
    wave_lds_sync();
    uint32_t o[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
        o[q] = static_cast<uint32_t>(own[q * kWave + lane]);
        own[q * kWave + lane] = 0;
    }
    wave_lds_sync();
    const uint32_t rel = pb - static_cast<uint32_t>(pre);  // element e sits at position rel + e
#pragma unroll
    for (int q = 0; q < U; ++q) {
        const uint32_t s = max(wave_max_scan_dpp(o[q]), carry);
        carry = __builtin_amdgcn_readlane(s, kWave - 1);
        const int32_t e = base + q * kWave + lane;
        const bool inb = e < total;
        sl[q] = static_cast<int32_t>(s) - 1;
        ev[q] = __shfl(rel, sl[q]) + static_cast<uint32_t>(e);
        const int32_t x = cl[inb ? ev[q] : 0u];
        w[q] = inb ? x : -1;
    }
}

__global__ __launch_bounds__(kSupWaves *kWave) void k_edge_support(const int64_t *__restrict__ row_off,
                                                                    const int32_t *__restrict__ col,
                                                                    const int64_t *__restrict__ in_off,
                                                                    const uint32_t *__restrict__ in_pos,
                                                                    const int32_t *__restrict__ in_len,
                                                                    const int2 *__restrict__ units,
                                                                    const int64_t *__restrict__ nunits_dev,
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
    gptr<int32_t> il = as_global(in_len);
#pragma unroll
    for (int q = 0; q < kSupUnroll; ++q) L.own[q * kWave + lane] = 0;
    wave_lds_sync();
    const gptr<int32_t> un = as_global(reinterpret_cast<const int32_t *>(units));  // (owner, first in-edge) pairs
    const int64_t nunits = *as_global(nunits_dev);
    unsigned long long found = 0;
    const int home = static_cast<int>(blockIdx.x % kSupQueues);
    for (int qi = 0; qi < kSupQueues; ++qi) {
      const int qq = (home + qi) % kSupQueues;
      for (;;) {
        unsigned long long c0 = 0;
        if (lane == 0) c0 = atomicAdd(&next[qq * kSupQueueStride], 1ull);
        c0 = shfl_t(c0, 0);
        const int64_t u = static_cast<int64_t>(c0) * kSupQueues + qq;  // unit u sits on queue u mod 8
        if (u >= nunits) break;
        const int32_t b = un[2 * u];
        const int64_t b0 = ro[b];
        const int32_t d = static_cast<int32_t>(ro[b + 1] - b0);
        const int64_t i0 = io[b] + un[2 * u + 1];
        const int64_t nin = min(io[b + 1] - i0, static_cast<int64_t>(kSupUnitEdges));
        const bool staged = d <= kSupCap;
        // table of 2^lg >= 1.5 d slots (64 .. 2^kSupTableLg)
        int lg = 6;
        while ((1 << lg) * 2 < 3 * d && lg < kSupTableLg) ++lg;
        const uint32_t tmask = (1u << lg) - 1u;
        const int shift = 24 - lg;
        if (staged) {
            for (int x = lane; x < (1 << lg); x += kWave) L.key[x] = -1;
            wave_lds_sync();
            for (int x = lane; x < d; x += kWave) {
                const int32_t v = cl[b0 + x];
                L.cnt[x] = 0;
                uint32_t h = hash_slot(v, shift, tmask);
                while (atomicCAS(&L.key[h], -1, v) != -1) h = (h + 1) & tmask;
                L.pos[h] = static_cast<int16_t>(x);
            }
            wave_lds_sync();
        }
        const int32_t hi_b = cl[b0 + d - 1];  // no c above N+(b)'s last entry can match
        {  // the unit's in-edges, one per lane: position of (a, b) and its walk's length
            const int64_t k = lane;
            uint32_t eab = 0;
            int32_t len = 0;
            if (k < nin) {
                eab = ip[i0 + k];
                len = il[i0 + k];
            }
            const int32_t incl = wave_inclusive_scan(len);
            const int32_t pre = incl - len;
            const int32_t tot = __builtin_amdgcn_readlane(incl, kWave - 1);
            L.hits[lane] = 0;
            wave_lds_sync();
            // Hits on a lane's current walk gather in a register and go to
            // the walk's LDS counter when the lane moves to another walk.
            int32_t acc_lo = 0;
            uint32_t acc = 0;
            uint32_t carry = 0;
            int32_t w[kSupUnroll], sl[kSupUnroll];
            uint32_t ev[kSupUnroll];
            if (tot > 0) sup_walk_load<kSupUnroll>(w, ev, sl, 0, tot, pre, len, eab + 1u, carry, L.own, cl, lane);
            for (int32_t f = 0; f < tot; f += kSupUnroll * kWave) {
                int32_t wn[kSupUnroll], sn[kSupUnroll];
                uint32_t en[kSupUnroll];
                sup_walk_load<kSupUnroll>(wn, en, sn, f + kSupUnroll * kWave, tot, pre, len, eab + 1u, carry, L.own,
                                          cl, lane);
#pragma unroll
                for (int u = 0; u < kSupUnroll; ++u) {
                    const int32_t c = w[u];
                    int32_t at = -1;  // position of c in N+(b)
                    if (staged) {
                        bool go = c >= 0 && c <= hi_b;
                        uint32_t h = hash_slot(c, shift, tmask);
                        while (__ballot(go) != 0) {
                            const int32_t kv = L.key[h];
                            if (go && kv == c) at = L.pos[h];
                            go = go && kv != -1 && kv != c;
                            h = (h + 1) & tmask;
                        }
                    } else if (c >= 0 && c <= hi_b) {
                        int32_t lo = 0, hi = d;
                        while (lo < hi) {
                            const int32_t mid = (lo + hi) >> 1;
                            if (cl[b0 + mid] < c) lo = mid + 1;
                            else hi = mid;
                        }
                        if (lo < d && cl[b0 + lo] == c) at = lo;
                    }
                    if (at >= 0) {
                        ++found;
                        atomicAdd(&support[ev[u]], 1u);
                        if (sl[u] != acc_lo) {
                            if (acc) atomicAdd(&L.hits[acc_lo], acc);
                            acc_lo = sl[u];
                            acc = 0;
                        }
                        ++acc;
                        if (staged) atomicAdd(&L.cnt[at], 1u);
                        else atomicAdd(&support[b0 + at], 1u);
                    }
                    w[u] = wn[u];
                    sl[u] = sn[u];
                    ev[u] = en[u];
                }
            }
            if (acc) atomicAdd(&L.hits[acc_lo], acc);
            wave_lds_sync();
            if (k < nin && L.hits[lane]) atomicAdd(&support[eab], L.hits[lane]);
            wave_lds_sync();  // before the next unit resets the counters
        }
        if (staged) {
            wave_lds_sync();
            for (int x = lane; x < d; x += kWave)
                if (L.cnt[x]) atomicAdd(&support[b0 + x], L.cnt[x]);
            wave_lds_sync();  // before the next unit is staged
        }
      }
    }
    found = wave_sum(found);
    if (lane == 0 && found) atomicAdd(total, found);
}

}  // namespace

void in_edges(pgabb_graph *g, DArray<int64_t> &in_off, DArray<uint32_t> &in_pos) {
    hipStream_t s = g->stream;
    const int64_t m = g->m;
    const int32_t n = g->n;
    DArray<uint32_t> key(static_cast<size_t>(m), s), key_alt(static_cast<size_t>(m), s);
    DArray<uint32_t> pos(static_cast<size_t>(m), s), pos_alt(static_cast<size_t>(m), s);
    in_off.reset(static_cast<size_t>(n) + 1, s);
    k_sup_pairs<<<grid_for(m, kSupB), kSupB, 0, s>>>(g->col.get(), m, key.get(), pos.get());
    k_sup_widen<<<grid_for(n, kSupB), kSupB, 0, s>>>(g->indeg.get(), n, in_off.get());
    PGABB_HIP(hipGetLastError());
    scan_exclusive_i64(in_off.get(), in_off.get(), n, in_off.get() + n, s);
    const bool alt = radix_sort_u32(key.get(), key_alt.get(), pos.get(), pos_alt.get(), m, g->nb, s);
    in_pos = std::move(alt ? pos_alt : pos);
}

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
        DArray<int32_t> rest(static_cast<size_t>(m), s);
        k_sup_rest<<<grid_for(n, kSupB), kSupB, 0, s>>>(g->row_off.get(), n, rest.get());
        PGABB_HIP(hipGetLastError());
        DArray<int64_t> in_off;
        DArray<uint32_t> in_pos_arr;
        in_edges(g, in_off, in_pos_arr);
        const uint32_t *in_pos = in_pos_arr.get();
        DArray<int32_t> in_len(static_cast<size_t>(m), s);
        k_sup_in_len<<<grid_for(m, kSupB), kSupB, 0, s>>>(in_pos, rest.get(), m, in_len.get());
        PGABB_HIP(hipGetLastError());
        rest.release();

        // work units (at most one per owner plus one per kSupUnitEdges in-edges)
        DArray<int64_t> upre(static_cast<size_t>(n) + 1, s);
        const int64_t max_units = static_cast<int64_t>(n) + m / kSupUnitEdges + 1;
        DArray<int2> units(static_cast<size_t>(max_units), s);
        k_sup_unit_counts<<<grid_for(n, kSupB), kSupB, 0, s>>>(g->row_off.get(), in_off.get(), n, upre.get());
        PGABB_HIP(hipGetLastError());
        scan_exclusive_i64(upre.get(), upre.get(), n, upre.get() + n, s);
        k_sup_unit_fill<<<grid_for(n, kSupB), kSupB, 0, s>>>(upre.get(), n, units.get());
        PGABB_HIP(hipGetLastError());

        constexpr int kCtr = kSupQueues * kSupQueueStride + 1;  // work counters, triangles
        DArray<unsigned long long> ctr(kCtr, s);
        PGABB_HIP(hipMemsetAsync(ctr.get(), 0, kCtr * sizeof(unsigned long long), s));
        PGABB_HIP(hipMemsetAsync(sup, 0, sizeof(uint32_t) * static_cast<size_t>(m), s));
        // four workgroups of four waves fit a CU's LDS
        const int64_t want = (max_units + kSupWaves - 1) / kSupWaves;
        const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(want, 256 * 4)));
        StreamTimer tm;
        tm.start(s);
        k_edge_support<<<grid, kSupWaves * kWave, 0, s>>>(g->row_off.get(), g->col.get(), in_off.get(), in_pos,
                                                           in_len.get(), units.get(), upre.get() + n, sup, ctr.get(),
                                                           ctr.get() + kCtr - 1);
        PGABB_HIP(hipGetLastError());
        tm.stop(s);
        Staged<unsigned long long> h(1, s);
        PGABB_HIP(hipMemcpyAsync(h.get(), ctr.get() + kCtr - 1, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                 s));
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
