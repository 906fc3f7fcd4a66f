// k-truss (the peeling algorithm named in PGAbB Section 3.2): the largest
// subgraph in which every edge lies in at least k - 2 triangles of the
// subgraph.  It is unique, so whole rounds reach it as one-edge-at-a-time
// peeling does: each round builds the graph of the edges still present,
// counts the triangles of every edge with the support pass, and keeps the
// edges with at least k - 2; rounds end when one keeps every edge.
//
// The edges of a round are rank pairs (lo, hi) in CSR order, and the
// round's graph is built with ranks as ids and id order as the vertex
// order, so its CSR lists them in that same order: the support pass's
// counts line up with the pairs without any search.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>

#include "common.hpp"
#include "graph.hpp"

namespace pgabb {

namespace {

constexpr int kKB = 256;

// Pairs (row, col) and positions of the oriented edges of the CSR.
__global__ __launch_bounds__(kKB) void k_kt_init(const int64_t *__restrict__ row_off,
                                                  const int32_t *__restrict__ col, int32_t n, int64_t m,
                                                  int32_t *__restrict__ lo_end, int32_t *__restrict__ hi_end,
                                                  uint32_t *__restrict__ pos) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kKB) {
        int32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (row_off[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        lo_end[e] = lo;
        hi_end[e] = col[e];
        pos[e] = static_cast<uint32_t>(e);
    }
}

__global__ __launch_bounds__(kKB) void k_kt_flags(const uint32_t *__restrict__ sup, int64_t m, uint32_t need,
                                                   uint32_t *__restrict__ flag) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kKB)
        flag[e] = sup[e] >= need ? 1u : 0u;
}

// Moves the kept edges to the front of the output arrays, in order.
__global__ __launch_bounds__(kKB) void k_kt_compact(const uint32_t *__restrict__ flag,
                                                     const uint32_t *__restrict__ at, int64_t m,
                                                     const int32_t *__restrict__ lo_in,
                                                     const int32_t *__restrict__ hi_in,
                                                     const uint32_t *__restrict__ pos_in,
                                                     int32_t *__restrict__ lo_out, int32_t *__restrict__ hi_out,
                                                     uint32_t *__restrict__ pos_out) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kKB) {
        if (!flag[e]) continue;
        const uint32_t q = at[e];
        lo_out[q] = lo_in[e];
        hi_out[q] = hi_in[e];
        pos_out[q] = pos_in[e];
    }
}

__global__ __launch_bounds__(kKB) void k_kt_mark(const uint32_t *__restrict__ pos, int64_t cnt,
                                                  uint8_t *__restrict__ keep) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; e < cnt;
         e += static_cast<int64_t>(gridDim.x) * kKB)
        keep[pos[e]] = 1;
}

}  // namespace

int64_t ktruss(pgabb_graph *g, int32_t k, uint8_t *keep, bool on_device, int32_t *rounds_out) {
    hipStream_t s = g->stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int32_t n = g->n;
    const int64_t m = g->m;
    int32_t rounds = 0;
    int64_t cur = m;
    double kernel_ms = 0;
    if (m > 0) {
        PGABB_REQUIRE(m < (int64_t{1} << 32), PGABB_EINVAL, "k-truss needs m' < 2^32 (m' = %lld)",
                      static_cast<long long>(m));
        const uint32_t need = k > 2 ? static_cast<uint32_t>(k - 2) : 0u;
        DArray<int32_t> lo_a(static_cast<size_t>(m), s), hi_a(static_cast<size_t>(m), s);
        DArray<int32_t> lo_b(static_cast<size_t>(m), s), hi_b(static_cast<size_t>(m), s);
        DArray<uint32_t> pos_a(static_cast<size_t>(m), s), pos_b(static_cast<size_t>(m), s);
        DArray<uint32_t> flag(static_cast<size_t>(m), s), at(static_cast<size_t>(m) + 1, s);
        k_kt_init<<<grid_for(m, kKB), kKB, 0, s>>>(g->row_off.get(), g->col.get(), n, m, lo_a.get(), hi_a.get(),
                                                   pos_a.get());
        PGABB_HIP(hipGetLastError());
        Staged<uint32_t> h_kept(1, s);
        while (cur > 0 && need > 0) {  // k <= 2: every edge stays
            ++rounds;
            pgabb_graph sub;
            sub.stream = s;
            sub.flags = PGABB_ORDER_BY_ID;
            sub.n = n;
            build_graph(&sub, lo_a.get(), hi_a.get(), cur);
            PGABB_REQUIRE(sub.m == cur, PGABB_EDEVICE, "k-truss round: %lld edges rebuilt as %lld",
                          static_cast<long long>(cur), static_cast<long long>(sub.m));
            DArray<uint32_t> sup(static_cast<size_t>(cur), s);
            edge_support(&sub, sup.get(), true);
            kernel_ms += sub.t_kernel_ms;
            k_kt_flags<<<grid_for(cur, kKB), kKB, 0, s>>>(sup.get(), cur, need, flag.get());
            scan_exclusive_u32(flag.get(), at.get(), cur, at.get() + cur, s);
            k_kt_compact<<<grid_for(cur, kKB), kKB, 0, s>>>(flag.get(), at.get(), cur, lo_a.get(), hi_a.get(),
                                                            pos_a.get(), lo_b.get(), hi_b.get(), pos_b.get());
            PGABB_HIP(hipGetLastError());
            PGABB_HIP(hipMemcpyAsync(h_kept.get(), at.get() + cur, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            PGABB_HIP(hipStreamSynchronize(s));
            const int64_t kept = h_kept[0];
            std::swap(lo_a, lo_b);
            std::swap(hi_a, hi_b);
            std::swap(pos_a, pos_b);
            if (kept == cur) break;
            cur = kept;
        }
        if (keep) {
            DArray<uint8_t> own;
            uint8_t *dst = keep;
            if (!on_device) {
                own.reset(static_cast<size_t>(m), s);
                dst = own.get();
            }
            PGABB_HIP(hipMemsetAsync(dst, 0, static_cast<size_t>(m), s));
            if (cur > 0) k_kt_mark<<<grid_for(cur, kKB), kKB, 0, s>>>(pos_a.get(), cur, dst);
            PGABB_HIP(hipGetLastError());
            if (!on_device) PGABB_HIP(hipMemcpyAsync(keep, dst, static_cast<size_t>(m), hipMemcpyDeviceToHost, s));
            PGABB_HIP(hipStreamSynchronize(s));
        }
    }
    g->t_kernel_ms = kernel_ms;
    g->kernel_launches = rounds;
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rounds_out) *rounds_out = rounds;
    return cur;
}

}  // namespace pgabb
