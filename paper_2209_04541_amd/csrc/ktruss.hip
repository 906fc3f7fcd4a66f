// k-truss (the peeling algorithm named in PGAbB Section 3.2): the largest
// subgraph in which every edge lies in at least k - 2 triangles of the
// subgraph.  It is unique, so whole rounds reach it as one-edge-at-a-time
// peeling does.
//
// One support pass counts the triangles of every edge; then each round
// takes the live edges with fewer than k - 2 (the round's frontier), and for
// every triangle a frontier edge closes with two edges that are still there,
// the triangle vanishes: each of its edges outside the frontier loses one
// from its count.  A triangle with two or three frontier edges is handled
// by the frontier edge with the smallest CSR position only, so no count
// loses one twice.  Frontier edges are then dead.  The counts of the live
// edges stay the triangle counts of the live graph, so the rounds are those
// of recounting every round, at the cost of the removed edges' triangles.
//
// The triangles of a frontier edge (u, v), ranks u < v, are the common
// neighbours w of u and v in the undirected graph.  A vertex's neighbours
// are its in-edges (lower ranks, ascending) followed by its out-edges
// (higher ranks, ascending), so each list is sorted: the walk takes every
// neighbour of u (the endpoint of lower degree under degree order),
// flattened over the lanes for 64 frontier edges at a time, and finds it in
// v's list by binary search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>

#include "common.hpp"
#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

constexpr int kKB = 256;
constexpr int kPeelWaves = 4;

enum : uint8_t { kLive = 0, kDying = 1, kDead = 2 };

// Lower end (row) of every oriented edge, a thread per row.
__global__ __launch_bounds__(kKB) void k_kt_rows(const int64_t *__restrict__ row_off, int32_t n,
                                                  int32_t *__restrict__ lo_end) {
    for (int64_t a = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; a < n;
         a += static_cast<int64_t>(gridDim.x) * kKB)
        for (int64_t e = row_off[a]; e < row_off[a + 1]; ++e) lo_end[e] = static_cast<int32_t>(a);
}

// Lower end of the edge in every in-edge slot.
__global__ __launch_bounds__(kKB) void k_kt_in_nb(const uint32_t *__restrict__ in_pos,
                                                   const int32_t *__restrict__ lo_end, int64_t m,
                                                   int32_t *__restrict__ in_nb) {
    for (int64_t k = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; k < m;
         k += static_cast<int64_t>(gridDim.x) * kKB)
        in_nb[k] = lo_end[in_pos[k]];
}

__global__ __launch_bounds__(kKB) void k_kt_clear(uint8_t *__restrict__ state, int64_t m) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kKB)
        state[e] = kLive;
}

// The frontier: live edges with fewer than `need` triangles become dying
// and are appended to `front` (one counter atomic per wave).
__global__ __launch_bounds__(kKB) void k_kt_front(const uint32_t *__restrict__ sup, int64_t m, uint32_t need,
                                                   uint8_t *__restrict__ state, uint32_t *__restrict__ front,
                                                   unsigned long long *__restrict__ nfront) {
    const int lane = lane_id();
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t base = blockIdx.x * static_cast<int64_t>(kKB); base < m;
         base += static_cast<int64_t>(gridDim.x) * kKB) {
        const int64_t e = base + threadIdx.x;  // the whole wave iterates together
        bool take = false;
        if (e < m && state[e] == kLive && sup[e] < need) {
            take = true;
            state[e] = kDying;
        }
        const uint64_t mask = __ballot(take);
        if (mask == 0) continue;
        unsigned long long at = 0;
        if (lane == 0) at = atomicAdd(nfront, static_cast<unsigned long long>(__popcll(mask)));
        at = shfl_t(at, 0);
        if (take) front[at + __popcll(mask & below)] = static_cast<uint32_t>(e);
    }
}

__global__ __launch_bounds__(kKB) void k_kt_kill(const uint32_t *__restrict__ front,
                                                  const unsigned long long *__restrict__ nfront,
                                                  uint8_t *__restrict__ state) {
    const int64_t cnt = static_cast<int64_t>(*nfront);
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; i < cnt;
         i += static_cast<int64_t>(gridDim.x) * kKB)
        state[front[i]] = kDead;
}

struct PeelLds {
    int32_t pre[kWave];   // position of each lane's list in the flattened walk
    uint32_t e[kWave];    // the frontier edge (u, v)
    int32_t v[kWave];
    int32_t nin_u[kWave];   // u's in-edges
    int64_t iu0[kWave];     // u's first in-edge slot
    int64_t ou0[kWave];     // u's first out-edge position
    int64_t iv0[kWave], iv1[kWave];  // v's in-edge slots
    int64_t ov0[kWave], ov1[kWave];  // v's out-edge positions
    int32_t own[kWave];     // list starts of the current batch
};

// First index in [lo, hi) of the sorted x whose value is at least w.
template <class I>
__device__ __forceinline__ I lower_at(gptr<int32_t> x, I lo, I hi, int32_t w) {
    while (lo < hi) {
        const I mid = lo + ((hi - lo) >> 1);
        if (x[mid] < w) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One round's triangle updates: groups of 64 frontier edges, one per lane,
// from a work counter.
__global__ __launch_bounds__(kPeelWaves *kWave) void k_kt_peel(const uint32_t *__restrict__ front_,
                                                                const unsigned long long *__restrict__ nfront_,
                                                                const int64_t *__restrict__ row_off_,
                                                                const int32_t *__restrict__ col_,
                                                                const int32_t *__restrict__ lo_end_,
                                                                const int64_t *__restrict__ in_off_,
                                                                const uint32_t *__restrict__ in_pos_,
                                                                const int32_t *__restrict__ in_nb_,
                                                                const uint8_t *__restrict__ state_,
                                                                uint32_t *__restrict__ sup,
                                                                unsigned long long *__restrict__ next) {
    __shared__ PeelLds s_lds[kPeelWaves];
    PeelLds &L = s_lds[threadIdx.x / kWave];
    const int lane = lane_id();
    const gptr<uint32_t> front = as_global(front_);
    const gptr<int64_t> ro = as_global(row_off_);
    const gptr<int32_t> col = as_global(col_), lo_end = as_global(lo_end_), in_nb = as_global(in_nb_);
    const gptr<int64_t> io = as_global(in_off_);
    const gptr<uint32_t> ip = as_global(in_pos_);
    const gptr<uint8_t> state = as_global(state_);
    const int64_t cnt = static_cast<int64_t>(*as_global(nfront_));
    L.own[lane] = 0;
    wave_lds_sync();
    for (;;) {
        unsigned long long g0 = 0;
        if (lane == 0) g0 = atomicAdd(next, 1ull);
        g0 = shfl_t(g0, 0);
        const int64_t first = static_cast<int64_t>(g0) * kWave;
        if (first >= cnt) break;
        const int64_t idx = first + lane;
        int32_t len = 0;
        if (idx < cnt) {
            const uint32_t e = front[idx];
            const int32_t u = lo_end[e], v = col[e];
            const int64_t iu0 = io[u], iu1 = io[u + 1], ou0 = ro[u], ou1 = ro[u + 1];
            len = static_cast<int32_t>((iu1 - iu0) + (ou1 - ou0));
            L.e[lane] = e;
            L.v[lane] = v;
            L.nin_u[lane] = static_cast<int32_t>(iu1 - iu0);
            L.iu0[lane] = iu0;
            L.ou0[lane] = ou0;
            L.iv0[lane] = io[v];
            L.iv1[lane] = io[v + 1];
            L.ov0[lane] = ro[v];
            L.ov1[lane] = ro[v + 1];
        }
        const int32_t incl = wave_inclusive_scan(len);
        const int32_t pre = incl - len;
        const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
        L.pre[lane] = pre;
        wave_lds_sync();
        uint32_t carry = 0;
        for (int32_t base = 0; base < total; base += kWave) {
            // the lane whose list holds element base + lane: list starts
            // scattered into LDS, then a running maximum over the lanes
            const int32_t p = pre - base;
            if (len > 0 && p >= 0 && p < kWave) L.own[p] = lane + 1;
            wave_lds_sync();
            const uint32_t o = static_cast<uint32_t>(L.own[lane]);
            L.own[lane] = 0;
            wave_lds_sync();
            const uint32_t sl1 = max(wave_max_scan_dpp(o), carry);
            carry = __builtin_amdgcn_readlane(sl1, kWave - 1);
            const int32_t el = base + lane;
            if (el >= total) continue;
            const int sl = static_cast<int>(sl1) - 1;
            const int32_t t = el - L.pre[sl];  // neighbour t of u
            const uint32_t e = L.e[sl];
            const int32_t v = L.v[sl];
            int32_t w;
            uint32_t f;  // edge (u, w)
            if (t < L.nin_u[sl]) {
                const int64_t k = L.iu0[sl] + t;
                w = in_nb[k];
                f = ip[k];
            } else {
                const int64_t q = L.ou0[sl] + (t - L.nin_u[sl]);
                w = col[q];
                f = static_cast<uint32_t>(q);
            }
            if (w == v) continue;
            const uint8_t sf = state[f];
            if (sf == kDead) continue;
            uint32_t gq;  // edge (v, w), if any
            uint8_t sg;
            if (w < v) {
                const int64_t k0 = L.iv0[sl], k1 = L.iv1[sl];
                const int64_t k = lower_at<int64_t>(in_nb, k0, k1, w);
                if (k >= k1 || in_nb[k] != w) continue;
                gq = ip[k];
            } else {
                const int64_t q0 = L.ov0[sl], q1 = L.ov1[sl];
                const int64_t q = lower_at<int64_t>(col, q0, q1, w);
                if (q >= q1 || col[q] != w) continue;
                gq = static_cast<uint32_t>(q);
            }
            sg = state[gq];
            if (sg == kDead) continue;
            // the triangle vanishes; only its frontier edge of smallest
            // position updates the others
            if ((sf == kDying && f < e) || (sg == kDying && gq < e)) continue;
            if (sf == kLive) atomicSub(&sup[f], 1u);
            if (sg == kLive) atomicSub(&sup[gq], 1u);
        }
        wave_lds_sync();  // before the next group overwrites the lane records
    }
}

__global__ __launch_bounds__(kKB) void k_kt_keep(const uint8_t *__restrict__ state, int64_t m,
                                                  uint8_t *__restrict__ keep) {
    for (int64_t e = blockIdx.x * static_cast<int64_t>(kKB) + threadIdx.x; e < m;
         e += static_cast<int64_t>(gridDim.x) * kKB)
        keep[e] = state[e] == kLive ? 1 : 0;
}

}  // namespace

int64_t ktruss(pgabb_graph *g, int32_t k, uint8_t *keep, bool on_device, int32_t *rounds_out) {
    hipStream_t s = g->stream;
    const auto t0 = std::chrono::steady_clock::now();
    const int32_t n = g->n;
    const int64_t m = g->m;
    int32_t rounds = 0;
    int64_t live = m;
    double kernel_ms = 0;
    if (m > 0) {
        PGABB_REQUIRE(m < (int64_t{1} << 32), PGABB_EINVAL, "k-truss needs m' < 2^32 (m' = %lld)",
                      static_cast<long long>(m));
        const uint32_t need = k > 2 ? static_cast<uint32_t>(k - 2) : 0u;
        DArray<uint8_t> state(static_cast<size_t>(m), s);
        k_kt_clear<<<grid_for(m, kKB), kKB, 0, s>>>(state.get(), m);
        PGABB_HIP(hipGetLastError());
        if (need > 0) {  // k <= 2: every edge stays
            DArray<uint32_t> sup(static_cast<size_t>(m), s);
            edge_support(g, sup.get(), true);
            kernel_ms += g->t_kernel_ms;
            DArray<int32_t> lo_end(static_cast<size_t>(m), s), in_nb(static_cast<size_t>(m), s);
            DArray<int64_t> in_off;
            DArray<uint32_t> in_pos;
            in_edges(g, in_off, in_pos);
            k_kt_rows<<<grid_for(n, kKB), kKB, 0, s>>>(g->row_off.get(), n, lo_end.get());
            k_kt_in_nb<<<grid_for(m, kKB), kKB, 0, s>>>(in_pos.get(), lo_end.get(), m, in_nb.get());
            PGABB_HIP(hipGetLastError());
            DArray<uint32_t> front(static_cast<size_t>(m), s);
            DArray<unsigned long long> ctr(2, s);  // frontier size, group counter
            Staged<unsigned long long> h_front(1, s);
            const unsigned front_grid = std::min<unsigned>(grid_for(m, kKB), 256u * 8u);
            for (;;) {
                PGABB_HIP(hipMemsetAsync(ctr.get(), 0, 2 * sizeof(unsigned long long), s));
                k_kt_front<<<front_grid, kKB, 0, s>>>(sup.get(), m, need, state.get(), front.get(), ctr.get());
                PGABB_HIP(hipGetLastError());
                PGABB_HIP(hipMemcpyAsync(h_front.get(), ctr.get(), sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                         s));
                PGABB_HIP(hipStreamSynchronize(s));
                const int64_t nf = static_cast<int64_t>(h_front[0]);
                if (nf == 0) break;
                ++rounds;
                live -= nf;
                const int64_t groups = (nf + kWave - 1) / kWave;
                const unsigned grid = static_cast<unsigned>(
                    std::max<int64_t>(1, std::min<int64_t>((groups + kPeelWaves - 1) / kPeelWaves, 256 * 8)));
                StreamTimer tm;
                tm.start(s);
                k_kt_peel<<<grid, kPeelWaves * kWave, 0, s>>>(front.get(), ctr.get(), g->row_off.get(), g->col.get(),
                                                               lo_end.get(), in_off.get(), in_pos.get(), in_nb.get(),
                                                               state.get(), sup.get(), ctr.get() + 1);
                tm.stop(s);
                k_kt_kill<<<std::min<unsigned>(grid_for(nf, kKB), 1024u), kKB, 0, s>>>(front.get(), ctr.get(),
                                                                                    state.get());
                PGABB_HIP(hipGetLastError());
                kernel_ms += tm.ms();
            }
        }
        if (keep) {
            DArray<uint8_t> own;
            uint8_t *dst = keep;
            if (!on_device) {
                own.reset(static_cast<size_t>(m), s);
                dst = own.get();
            }
            k_kt_keep<<<grid_for(m, kKB), kKB, 0, s>>>(state.get(), m, dst);
            PGABB_HIP(hipGetLastError());
            if (!on_device) PGABB_HIP(hipMemcpyAsync(keep, dst, static_cast<size_t>(m), hipMemcpyDeviceToHost, s));
            PGABB_HIP(hipStreamSynchronize(s));
        }
    }
    g->t_kernel_ms = kernel_ms;
    g->kernel_launches = rounds;
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (rounds_out) *rounds_out = rounds;
    return live;
}

}  // namespace pgabb
