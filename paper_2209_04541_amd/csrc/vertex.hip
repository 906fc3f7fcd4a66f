// Triangles at each vertex (the numerator of the local clustering
// coefficient, PGAbB Section 1), from the per-edge counts: a triangle lies
// on two edges at each of its vertices, so t(v) is half the sum of the
// counts of v's edges.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>

#include "common.hpp"
#include "graph.hpp"

namespace pgabb {

namespace {

constexpr int kVB = 256;

// Adds each edge's count to both of its ends (ranks): a thread per row sums
// its row's counts for the row's own vertex and adds each count to the
// column's vertex.
__global__ __launch_bounds__(kVB) void k_vertex_sums(const int64_t *__restrict__ row_off,
                                                      const int32_t *__restrict__ col,
                                                      const uint32_t *__restrict__ sup, int32_t n,
                                                      unsigned long long *__restrict__ tv) {
    for (int64_t r = blockIdx.x * static_cast<int64_t>(kVB) + threadIdx.x; r < n;
         r += static_cast<int64_t>(gridDim.x) * kVB) {
        unsigned long long own = 0;
        for (int64_t e = row_off[r]; e < row_off[r + 1]; ++e) {
            const uint32_t c = sup[e];
            if (!c) continue;
            own += c;
            atomicAdd(&tv[col[e]], static_cast<unsigned long long>(c));
        }
        if (own) atomicAdd(&tv[r], own);
    }
}

// out[v] for input id v: half the sum at its rank.
__global__ __launch_bounds__(kVB) void k_vertex_by_id(const int32_t *__restrict__ rank,
                                                       const unsigned long long *__restrict__ tv, int32_t n,
                                                       uint64_t *__restrict__ out) {
    for (int64_t v = blockIdx.x * static_cast<int64_t>(kVB) + threadIdx.x; v < n;
         v += static_cast<int64_t>(gridDim.x) * kVB)
        out[v] = tv[rank[v]] / 2;
}

}  // namespace

uint64_t vertex_counts(pgabb_graph *g, uint64_t *out, bool out_on_device) {
    hipStream_t s = g->stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int32_t n = g->n;
    const int64_t m = g->m;
    uint64_t triangles = 0;
    if (n == 0) {
        g->t_kernel_ms = 0;
        g->kernel_launches = 0;
    } else if (m == 0) {
        g->t_kernel_ms = 0;
        g->kernel_launches = 0;
        if (out_on_device) {
            PGABB_HIP(hipMemsetAsync(out, 0, sizeof(uint64_t) * static_cast<size_t>(n), s));
            PGABB_HIP(hipStreamSynchronize(s));
        } else {
            std::memset(out, 0, sizeof(uint64_t) * static_cast<size_t>(n));
        }
    } else {
        DArray<uint32_t> sup(static_cast<size_t>(m), s);
        triangles = edge_support(g, sup.get(), true);  // kernel time and launches of the support pass
        DArray<unsigned long long> tv(static_cast<size_t>(n), s);
        PGABB_HIP(hipMemsetAsync(tv.get(), 0, sizeof(unsigned long long) * static_cast<size_t>(n), s));
        k_vertex_sums<<<grid_for(n, kVB), kVB, 0, s>>>(g->row_off.get(), g->col.get(), sup.get(), n, tv.get());
        DArray<uint64_t> own;
        uint64_t *dst = out;
        if (!out_on_device) {
            own.reset(static_cast<size_t>(n), s);
            dst = own.get();
        }
        k_vertex_by_id<<<grid_for(n, kVB), kVB, 0, s>>>(g->rank.get(), tv.get(), n, dst);
        PGABB_HIP(hipGetLastError());
        if (!out_on_device)
            PGABB_HIP(hipMemcpyAsync(out, dst, sizeof(uint64_t) * static_cast<size_t>(n), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
    }
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return triangles;
}

}  // namespace pgabb
