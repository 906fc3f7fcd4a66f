// Build phase: edge list -> cleaned, degree-ranked, oriented CSR on device.
//
// Steps (PGAbB Section 5.1: inputs made undirected and deduplicated;
// Section 5.4: degree-based vertex ordering, triangle counting needs only
// half of the edges):
//   1. pack each pair as key = min << nb | max, self-loops -> sentinel
//   2. radix sort the keys, keep the first of every run (dedupe)
//   3. deg[v] = number of distinct pairs touching v
//   4. rank = position in ascending (deg, id): a stable sort of the degrees
//      with the ids as values (ties keep id order)
//   5. relabel both ends to ranks, key = lo << nb | hi, radix sort again;
//      rows (lo) and sorted columns (hi) give the oriented CSR
#include <algorithm>

#include "common.hpp"
#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

bool radix_sort_u64_bits(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                         int64_t n, int lo_bit, int hi_bit, hipStream_t s);

namespace {

constexpr int B = 256;
constexpr uint64_t kSentinel = ~0ull;

__global__ void k_make_keys(const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
                            int64_t m, int32_t n, int nb, uint64_t *__restrict__ keys,
                            uint32_t *__restrict__ bad) {
    for (int64_t e = blockIdx.x * int64_t(B) + threadIdx.x; e < m; e += int64_t(gridDim.x) * B) {
        const int32_t a = src[e], b = dst[e];
        uint64_t key = kSentinel;
        if (a < 0 || b < 0 || a >= n || b >= n) {
            *bad = 1u;
        } else if (a != b) {
            const uint64_t lo = static_cast<uint32_t>(a < b ? a : b);
            const uint64_t hi = static_cast<uint32_t>(a < b ? b : a);
            key = (lo << nb) | hi;
        }
        keys[e] = key;
    }
}

// flag[e] = 1 for the first key of each run of equal valid keys.
__global__ void k_first_of_run(const uint64_t *__restrict__ keys, int64_t m, uint64_t valid_limit,
                               uint32_t *__restrict__ flag) {
    for (int64_t e = blockIdx.x * int64_t(B) + threadIdx.x; e < m; e += int64_t(gridDim.x) * B) {
        const uint64_t k = keys[e];
        flag[e] = (k < valid_limit && (e == 0 || keys[e - 1] != k)) ? 1u : 0u;
    }
}

__global__ void k_compact(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ flag,
                          const uint32_t *__restrict__ pos, int64_t m, uint64_t *__restrict__ out) {
    for (int64_t e = blockIdx.x * int64_t(B) + threadIdx.x; e < m; e += int64_t(gridDim.x) * B)
        if (flag[e]) out[pos[e]] = keys[e];
}

// Distinct keys are sorted by (lo, hi): the lo ends form runs, so each run
// adds its length once.  The hi ends are copied out, sorted, and counted the
// same way (scattered atomics on hub vertices would serialise).  The loop
// bound is uniform across a wave so every lane takes part in the ballots.
__global__ void k_degrees_lo(const uint64_t *__restrict__ keys, int64_t m, int nb,
                             int32_t *__restrict__ deg, uint32_t *__restrict__ his) {
    const uint64_t mask = (1ull << nb) - 1;
    const int64_t stride = int64_t(gridDim.x) * B;
    for (int64_t base = blockIdx.x * int64_t(B) + (threadIdx.x & ~63); base < m; base += stride) {
        const int64_t e = base + lane_id();
        const bool valid = e < m;
        const uint64_t k = valid ? keys[e] : 0ull;
        add_run_lengths(valid, static_cast<int64_t>(k >> nb), deg);
        if (valid) his[e] = static_cast<uint32_t>(k & mask);
    }
}

__global__ void k_degrees_hi(const uint32_t *__restrict__ his, int64_t m, int32_t *__restrict__ deg) {
    const int64_t stride = int64_t(gridDim.x) * B;
    for (int64_t base = blockIdx.x * int64_t(B) + (threadIdx.x & ~63); base < m; base += stride) {
        const int64_t e = base + lane_id();
        const bool valid = e < m;
        add_run_lengths(valid, valid ? static_cast<int64_t>(his[e]) : 0, deg);
    }
}

__global__ void k_deg_keys(const int32_t *__restrict__ deg, int32_t n, uint32_t *__restrict__ dk,
                           uint32_t *__restrict__ dv) {
    for (int64_t v = blockIdx.x * int64_t(B) + threadIdx.x; v < n; v += int64_t(gridDim.x) * B) {
        dk[v] = static_cast<uint32_t>(deg[v]);
        dv[v] = static_cast<uint32_t>(v);
    }
}

__global__ void k_invert(const uint32_t *__restrict__ perm, int32_t n, int32_t *__restrict__ rank) {
    for (int64_t r = blockIdx.x * int64_t(B) + threadIdx.x; r < n; r += int64_t(gridDim.x) * B)
        rank[perm[r]] = static_cast<int32_t>(r);
}

__global__ void k_identity(int32_t n, int32_t *__restrict__ rank) {
    for (int64_t r = blockIdx.x * int64_t(B) + threadIdx.x; r < n; r += int64_t(gridDim.x) * B)
        rank[r] = static_cast<int32_t>(r);
}

__global__ void k_orient(const uint64_t *__restrict__ ukeys, int64_t m, int nb,
                         const int32_t *__restrict__ rank, uint64_t *__restrict__ okeys) {
    const uint64_t mask = (1ull << nb) - 1;
    for (int64_t e = blockIdx.x * int64_t(B) + threadIdx.x; e < m; e += int64_t(gridDim.x) * B) {
        const uint64_t k = ukeys[e];
        const uint32_t ra = static_cast<uint32_t>(rank[k >> nb]);
        const uint32_t rb = static_cast<uint32_t>(rank[k & mask]);
        const uint64_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        okeys[e] = (lo << nb) | hi;
    }
}

__global__ void k_row_counts_and_cols(const uint64_t *__restrict__ okeys, int64_t m, int nb,
                                      int32_t *__restrict__ outdeg, int32_t *__restrict__ col) {
    const uint64_t mask = (1ull << nb) - 1;
    const int64_t stride = int64_t(gridDim.x) * B;
    for (int64_t base = blockIdx.x * int64_t(B) + (threadIdx.x & ~63); base < m; base += stride) {
        const int64_t e = base + lane_id();
        const bool valid = e < m;
        const uint64_t k = valid ? okeys[e] : 0ull;
        add_run_lengths(valid, static_cast<int64_t>(k >> nb), outdeg);
        if (valid) col[e] = static_cast<int32_t>(k & mask);
    }
}

__global__ void k_widen(const int32_t *__restrict__ in, int32_t n, int64_t *__restrict__ out) {
    for (int64_t v = blockIdx.x * int64_t(B) + threadIdx.x; v < n; v += int64_t(gridDim.x) * B)
        out[v] = in[v];
}

struct Stats {
    int32_t max_out;
    int32_t pad;
    unsigned long long isolated;
    unsigned long long probe_work;
};

// Per vertex v (rank r): indeg[r] = deg[v] - outdeg[r], the edges of v
// whose other end ranks lower; and the statistics, reduced per workgroup
// (one atomic each; launched with a small grid): the longest oriented row,
// the isolated vertices and the probe work W = sum over oriented edges
// (x, y) of outdeg[y] = sum over y of indeg[y] outdeg[y].
__global__ __launch_bounds__(B) void k_vertex_stats(const int32_t *__restrict__ deg,
                                                    const int32_t *__restrict__ rank,
                                                    const int32_t *__restrict__ outdeg, int32_t n,
                                                    int32_t *__restrict__ indeg, Stats *st) {
    __shared__ int32_t s_mx[B / 64];
    __shared__ unsigned long long s_iso[B / 64], s_w[B / 64];
    int32_t mx = 0;
    unsigned long long iso = 0, w = 0;
    for (int64_t v = blockIdx.x * int64_t(B) + threadIdx.x; v < n; v += int64_t(gridDim.x) * B) {
        const int32_t r = rank[v];
        const int32_t o = outdeg[r], i = deg[v] - o;
        indeg[r] = i;
        mx = max(mx, o);
        iso += deg[v] == 0;
        w += static_cast<unsigned long long>(i) * static_cast<unsigned long long>(o);
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) mx = max(mx, __shfl_xor(mx, d));
    iso = wave_sum(iso);
    w = wave_sum(w);
    if (lane_id() == 0) {
        s_mx[threadIdx.x >> 6] = mx;
        s_iso[threadIdx.x >> 6] = iso;
        s_w[threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < B / 64; ++q) {
            mx = max(mx, s_mx[q]);
            iso += s_iso[q];
            w += s_w[q];
        }
        atomicMax(&st->max_out, mx);
        atomicAdd(&st->isolated, iso);
        atomicAdd(&st->probe_work, w);
    }
}

unsigned cap_grid(int64_t work) {
    unsigned g = grid_for(work, B);
    return g > 65536u ? 65536u : g;
}

}  // namespace

void build_graph(pgabb_graph *g, const int32_t *src, const int32_t *dst, int64_t m) {
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    g->m_input = m;
    g->nb = std::max(1, bit_width_u64(n > 0 ? static_cast<uint64_t>(n - 1) : 0));
    const int nb = g->nb;

    g->rank.reset(static_cast<size_t>(n), s);
    g->outdeg.reset(static_cast<size_t>(n), s);
    g->indeg.reset(static_cast<size_t>(n), s);
    g->row_off.reset(static_cast<size_t>(n) + 1, s);
    if (n > 0) PGABB_HIP(hipMemsetAsync(g->outdeg.get(), 0, sizeof(int32_t) * n, s));
    PGABB_HIP(hipMemsetAsync(g->row_off.get(), 0, sizeof(int64_t) * (static_cast<size_t>(n) + 1), s));

    DArray<int32_t> deg(static_cast<size_t>(n), s);
    if (n > 0) PGABB_HIP(hipMemsetAsync(deg.get(), 0, sizeof(int32_t) * n, s));
    g->m = 0;

    if (m > 0) {
        DArray<uint64_t> keys(static_cast<size_t>(m), s), alt(static_cast<size_t>(m), s);
        // meta[0]: an endpoint lay out of range; meta[1]: distinct edges.
        // Out-of-range edges get the sentinel key, so sorting and compacting
        // them is harmless and one round trip reports both.
        DArray<uint32_t> meta(2, s);
        PGABB_HIP(hipMemsetAsync(meta.get(), 0, 2 * sizeof(uint32_t), s));
        k_make_keys<<<cap_grid(m), B, 0, s>>>(src, dst, m, n, nb, keys.get(), meta.get());
        PGABB_HIP(hipGetLastError());

        // 1-2: sort and dedupe.  Valid keys are below (n-1) << nb | (n-1) + 1;
        // the sentinel has every low 2nb bit set, so it sorts after them.
        const int kbits = 2 * nb;
        uint64_t *k0 = keys.get(), *k1 = alt.get();
        if (radix_sort_u64_bits(k0, k1, nullptr, nullptr, m, 0, kbits, s)) std::swap(k0, k1);
        const uint64_t valid_limit = (static_cast<uint64_t>(n - 1) << nb) + static_cast<uint64_t>(n);
        {
            DArray<uint32_t> flag(static_cast<size_t>(m), s), pos(static_cast<size_t>(m), s);
            k_first_of_run<<<cap_grid(m), B, 0, s>>>(k0, m, valid_limit, flag.get());
            PGABB_HIP(hipGetLastError());
            scan_exclusive_u32(flag.get(), pos.get(), m, meta.get() + 1, s);
            k_compact<<<cap_grid(m), B, 0, s>>>(k0, flag.get(), pos.get(), m, k1);
            PGABB_HIP(hipGetLastError());
            Staged<uint32_t> mh(2, s);
            PGABB_HIP(hipMemcpyAsync(mh.get(), meta.get(), mh.bytes(), hipMemcpyDeviceToHost, s));
            PGABB_HIP(hipStreamSynchronize(s));
            PGABB_REQUIRE(!mh[0], PGABB_EINVAL, "an edge endpoint lies outside [0, %d)", n);
            g->m = mh[1];
        }
        std::swap(k0, k1);  // k0: distinct keys [0, m')
        const int64_t mu = g->m;

        // 3: degrees
        if (mu > 0) {
            DArray<uint32_t> his(static_cast<size_t>(mu), s), his_alt(static_cast<size_t>(mu), s);
            k_degrees_lo<<<cap_grid(mu), B, 0, s>>>(k0, mu, nb, deg.get(), his.get());
            PGABB_HIP(hipGetLastError());
            uint32_t *hs = his.get();
            if (radix_sort_u32(his.get(), his_alt.get(), nullptr, nullptr, mu, nb, s)) hs = his_alt.get();
            k_degrees_hi<<<cap_grid(mu), B, 0, s>>>(hs, mu, deg.get());
            PGABB_HIP(hipGetLastError());
        }
        // 4: ranks
        if (g->flags & PGABB_ORDER_BY_ID) {
            k_identity<<<cap_grid(n), B, 0, s>>>(n, g->rank.get());
        } else {
            DArray<uint32_t> dk(n, s), dka(n, s), dv(n, s), dva(n, s);
            k_deg_keys<<<cap_grid(n), B, 0, s>>>(deg.get(), n, dk.get(), dv.get());
            PGABB_HIP(hipGetLastError());
            uint32_t *perm = dv.get();
            if (radix_sort_u32(dk.get(), dka.get(), dv.get(), dva.get(), n, nb, s)) perm = dva.get();
            k_invert<<<cap_grid(n), B, 0, s>>>(perm, n, g->rank.get());
        }
        PGABB_HIP(hipGetLastError());

        // 5: orient and sort by (row, col)
        if (mu > 0) {
            k_orient<<<cap_grid(mu), B, 0, s>>>(k0, mu, nb, g->rank.get(), k1);
            PGABB_HIP(hipGetLastError());
            if (radix_sort_u64_bits(k1, k0, nullptr, nullptr, mu, 0, kbits, s)) std::swap(k0, k1);
            // sorted oriented keys now in k1
            g->col.reset(static_cast<size_t>(mu), s);
            k_row_counts_and_cols<<<cap_grid(mu), B, 0, s>>>(k1, mu, nb, g->outdeg.get(), g->col.get());
            PGABB_HIP(hipGetLastError());
        }
    } else {
        k_identity<<<cap_grid(n), B, 0, s>>>(n, g->rank.get());
        PGABB_HIP(hipGetLastError());
    }
    if (g->m == 0) g->col.release();

    if (n > 0) {
        DArray<int64_t> wide(static_cast<size_t>(n), s);
        k_widen<<<cap_grid(n), B, 0, s>>>(g->outdeg.get(), n, wide.get());
        PGABB_HIP(hipGetLastError());
        scan_exclusive_i64(wide.get(), g->row_off.get(), n, g->row_off.get() + n, s);
    }

    // statistics for sizing kernels and stating algorithmic bytes
    DArray<Stats> st(1, s);
    PGABB_HIP(hipMemsetAsync(st.get(), 0, sizeof(Stats), s));
    if (n > 0) {
        k_vertex_stats<<<std::min(cap_grid(n), 1024u), B, 0, s>>>(deg.get(), g->rank.get(), g->outdeg.get(), n,
                                                                  g->indeg.get(), st.get());
    }
    PGABB_HIP(hipGetLastError());
    Staged<Stats> hs(1, s);
    PGABB_HIP(hipMemcpyAsync(hs.get(), st.get(), sizeof(Stats), hipMemcpyDeviceToHost, s));
    PGABB_HIP(hipStreamSynchronize(s));
    g->max_out = hs[0].max_out;
    g->isolated = static_cast<int64_t>(hs[0].isolated);
    g->probe_work = hs[0].probe_work;
}

}  // namespace pgabb
