// 4-cliques (the multi-block pattern family of PGAbB Section 3.2, one
// intersection level past triangles).  Each 4-clique with ranks
// a < b < c < d is counted once, at its oriented edge (a, b): c runs over
// the common out-neighbours of a and b, and d over the entries after c that
// N+(a), N+(b) and N+(c) share.  One thread per edge merges N+(a) (from b
// on) with N+(b) and, at every common entry c, merges the three lists from
// c on.  The oriented graph is taken as one block (p = 1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>

#include "common.hpp"
#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

constexpr int kQB = 256;

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
        DArray<unsigned long long> tot(1, s);
        PGABB_HIP(hipMemsetAsync(tot.get(), 0, sizeof(unsigned long long), s));
        const unsigned grid = std::min<unsigned>(grid_for(m, kQB), 256u * 16u);
        StreamTimer tm;
        tm.start(s);
        k_four_cliques<<<grid, kQB, 0, s>>>(g->row_off.get(), g->col.get(), g->n, m, tot.get());
        PGABB_HIP(hipGetLastError());
        tm.stop(s);
        Staged<unsigned long long> h(1, s);
        PGABB_HIP(hipMemcpyAsync(h.get(), tot.get(), sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        result = h[0];
        g->t_kernel_ms = tm.ms();
        g->kernel_launches = 1;
    }
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return result;
}

}  // namespace pgabb
