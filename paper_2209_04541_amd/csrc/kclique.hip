// 4-cliques by block 4-lists (the multi-block pattern mode of PGAbB Section
// 3.2, one intersection level past triangles).
//
// Each 4-clique with ranks a < b < c < d lies in stripes i <= j <= k <= l and
// is counted once, in the 4-list (A_ij, A_ik, A_il, A_jk, A_jl, A_kl), at its
// edge (a, b) of A_ij: c runs over C = A_ik[a] & A_jk[b] (stripe k), d over
// D = A_il[a] & A_jl[b] (stripe l), and the pair counts when (c, d) is an
// entry of A_kl.  Every pair of stripes is ordered by rank and blocks keep
// only edges from lower to higher rank, so d > c > b > a needs no test.
//
// One wave takes a work item of A_ij -- row a and a run of at most 8 of its
// entries b (a part of one of the block's own row items) -- and stages
// A_ik[a] and A_il[a] (one list when k = l) in an open-addressing hash table
// in LDS.  For each b its lanes look the entries of A_jk[b] and A_jl[b] up in
// the table and mark the ones found (C and D) by setting the stored key's top
// bit; then, for the marked keys of stripe k (C), they walk A_kl[c]
// flattened over the lanes and count the entries whose key is marked (in D),
// and finally clear the marks.  Blocks hold column ids local to their stripe,
// so when k < l the ids of stripe l enter the table shifted by the width of
// stripe k: keys of A_ik[a] lie below that width and keys of A_il[a] above
// it, and an entry of A_kl[c] (stripe l, shifted too) can only match a key
// of A_il[a].  Items whose staged rows hold more than kStageCap entries go to
// a kernel with one thread per (item, b) and plain merges.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <vector>

#include "common.hpp"
#include "graph.hpp"
#include "tc_device.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

constexpr int kQB = 256;
constexpr int kStageCap = 1024;  // entries a wave stages (both rows)
constexpr int kTableLg = 11;     // hash slots of a wave: at most 2^11
constexpr int kCliqueWaves = 4;
constexpr int kQuadUnroll = 2;   // walk chunks in flight
// A wave's work item is a run of at most kQuadSpan entries b of one of
// A_ij's row items (each row item is cut into kSplitV / kQuadSpan parts):
// rows of high-degree vertices then spread over several waves.
constexpr int kQuadSpan = 8;
constexpr int kQuadParts = kSplitV / kQuadSpan;
// A marked key has its top bit set.  Vertex ids are below 2^31 - 1, so a
// marked key is never -1, the empty slot.
constexpr int32_t kMarkBit = INT32_MIN;
constexpr int32_t kKeyBits = 0x7FFFFFFF;

// Device view of one block 4-list.
struct QuadDesc {
    BlockRef ij, ik, il, jk, jl, kl;
    int32_t slot;    // counter of the 4-list
    int32_t same;    // k == l: A_il is A_ik and A_jl is A_jk
    int32_t lshift;  // k < l: width of stripe k, added to stripe l's ids in the table; else 0
    int32_t pad;
};

// Whether a wave stages row a of A_ik (dk entries) and of A_il (dl).
__device__ __forceinline__ bool quad_staged(int32_t dk, int32_t dl, int32_t same) {
    return (same ? dk : dk + dl) <= kStageCap;
}

// The 4-list holding item q: the last t with pre[t] <= q.
__device__ __forceinline__ int32_t quad_of(gptr<int64_t> pre, int32_t nq, int64_t q) {
    int32_t lo = 0, hi = nq - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Marks the entries of the sorted list x[0, n) found in the table, each
// looked up as its id plus `add` (ids above top cannot be there).  Every
// lane of the wave calls this.
__device__ __forceinline__ void quad_mark(int32_t *H, int shift, uint32_t tmask, gptr<int32_t> x, int32_t n,
                                          int32_t top, int32_t add, int lane) {
    for (int32_t x0 = 0; x0 < n; x0 += kWave) {
        const int32_t i = x0 + lane;
        const int32_t u = i < n ? x[i] : -1;
        bool go = u >= 0 && u <= top;
        const int32_t v = u + add;
        uint32_t h = hash_slot(v, shift, tmask);
        while (__ballot(go) != 0) {
            const int32_t sv = H[h];
            if (go && sv == v) H[h] = v | kMarkBit;
            go = go && sv != -1 && (sv & kKeyBits) != v;
            h = (h + 1) & tmask;
        }
        if (__ballot(u > top) != 0) break;  // the rest of the list is above top too
    }
}

// Staged items: one wave per item from a work counter.  Counts go to the
// 4-lists' counters, one atomic per run of items of the same list a wave
// takes.
__global__ __launch_bounds__(kCliqueWaves *kWave) void k_quad_items(const QuadDesc *__restrict__ quads,
                                                                     const int64_t *__restrict__ item_pre,
                                                                     int32_t nq,
                                                                     unsigned long long *__restrict__ next,
                                                                     unsigned long long *__restrict__ counts) {
    __shared__ int32_t s_table[kCliqueWaves][1 << kTableLg];
    __shared__ int32_t s_own[kCliqueWaves][kQuadUnroll * kWave];
    int32_t *H = s_table[threadIdx.x / kWave];
    int32_t *own = s_own[threadIdx.x / kWave];
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < kQuadUnroll; ++q) own[q * kWave + lane] = 0;
    wave_lds_sync();
    const gptr<int64_t> ip = as_global(item_pre);
    const int64_t nitems = ip[nq];
    unsigned long long acc = 0;  // this lane's share of the current list's count
    int32_t acc_slot = -1;
    for (;;) {
        unsigned long long q0 = 0;
        if (lane == 0) q0 = atomicAdd(next, 1ull);
        q0 = shfl_t(q0, 0);
        if (q0 >= static_cast<unsigned long long>(nitems)) break;
        const int64_t q = static_cast<int64_t>(q0);
        const int32_t t = __builtin_amdgcn_readfirstlane(quad_of(ip, nq, q));
        const QuadDesc &Q = quads[t];
        const int64_t r = (q - ip[t]) / kQuadParts;  // row item, and its part
        const int32_t part = static_cast<int32_t>((q - ip[t]) - r * kQuadParts);
        const gptr<int32_t> it = as_global(Q.ij.items) + kItemWords * r;
        const int32_t a = it[0];
        const int32_t eb = it[1] + part * kQuadSpan, ee = min(eb + kQuadSpan, it[2]);
        if (eb >= ee) continue;
        const gptr<int32_t> ikr = as_global(Q.ik.rptr), ilr = as_global(Q.il.rptr);
        const int32_t k0 = ikr[a], dk = ikr[a + 1] - k0;
        const int32_t l0 = ilr[a], dl = ilr[a + 1] - l0;
        if (dk == 0 || dl == 0 || !quad_staged(dk, dl, Q.same)) continue;  // none, or the long kernel's
        if (t != acc_slot) {
            const unsigned long long w = wave_sum(acc);
            if (lane == 0 && w) atomicAdd(&counts[acc_slot], w);
            acc = 0;
            acc_slot = t;
        }
        const gptr<int32_t> ikc = as_global(Q.ik.col), ilc = as_global(Q.il.col);
        // table of 2^lg >= 4 x the staged entries slots (64 .. 2^kTableLg)
        const int32_t nst = Q.same ? dk : dk + dl;
        int lg = 6;
        while ((1 << lg) < 4 * nst && lg < kTableLg) ++lg;
        const int32_t T = 1 << lg;
        const uint32_t tmask = static_cast<uint32_t>(T - 1);
        const int shift = 24 - lg;
        for (int32_t s0 = lane; s0 < T; s0 += kWave) H[s0] = -1;
        wave_lds_sync();
        for (int32_t x = lane; x < nst; x += kWave) {
            const int32_t v = x < dk ? ikc[k0 + x] : ilc[l0 + x - dk] + Q.lshift;
            uint32_t h = hash_slot(v, shift, tmask);
            while (atomicCAS(&H[h], -1, v) != -1) h = (h + 1) & tmask;
        }
        wave_lds_sync();
        const int32_t topk = ikc[k0 + dk - 1], topl = ilc[l0 + dl - 1];
        const int32_t lshift = Q.lshift;
        const gptr<int32_t> ijc = as_global(Q.ij.col);
        const gptr<int32_t> jkr = as_global(Q.jk.rptr), jkc = as_global(Q.jk.col);
        const gptr<int32_t> jlr = as_global(Q.jl.rptr), jlc = as_global(Q.jl.col);
        const gptr<int32_t> klr = as_global(Q.kl.rptr), klc = as_global(Q.kl.col);
        uint32_t cnt = 0;
        for (int32_t e = eb; e < ee; ++e) {
            const int32_t b = ijc[e];
            const int32_t bk0 = jkr[b], dbk = jkr[b + 1] - bk0;
            const int32_t bl0 = jlr[b], dbl = jlr[b + 1] - bl0;
            if (dbk == 0 || dbl == 0) continue;
            quad_mark(H, shift, tmask, jkc + bk0, dbk, topk, 0, lane);  // C (and D when k = l)
            if (!Q.same) quad_mark(H, shift, tmask, jlc + bl0, dbl, topl, Q.lshift, lane);  // D
            wave_lds_sync();
            // walk A_kl[c] for the marked keys c of stripe k, 64 slots at a time
            for (int32_t s0 = 0; s0 < T; s0 += kWave) {
                const int32_t sv = H[s0 + lane];
                const bool in = sv < -1 && (sv & kKeyBits) <= topk;
                if (__ballot(in) == 0) continue;
                int32_t pb = 0, len = 0;
                if (in) {
                    const int32_t c = sv & kKeyBits;
                    pb = klr[c];
                    len = klr[c + 1] - pb;
                }
                const int32_t incl = wave_inclusive_scan(len);
                const int32_t pre = incl - len;
                const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
                if (total == 0) continue;
                uint32_t carry = 0;
                int32_t w[kQuadUnroll];
                walk_load<kQuadUnroll>(w, 0, total, pre, len, pb, carry, own, klc, lane);
                for (int32_t base = 0; base < total; base += kQuadUnroll * kWave) {
                    int32_t wn[kQuadUnroll];
                    walk_load<kQuadUnroll>(wn, base + kQuadUnroll * kWave, total, pre, len, pb, carry, own, klc,
                                           lane);
#pragma unroll
                    for (int u = 0; u < kQuadUnroll; ++u) {
                        bool go = w[u] >= 0 && w[u] <= topl;
                        const int32_t y = w[u] + lshift;  // its key in the table
                        uint32_t h = hash_slot(y, shift, tmask);
                        uint32_t hit = 0;
                        while (__ballot(go) != 0) {
                            const int32_t hv = H[h];
                            hit |= (go && hv == (y | kMarkBit)) ? 1u : 0u;
                            go = go && hv != -1 && (hv & kKeyBits) != y;
                            h = (h + 1) & tmask;
                        }
                        cnt += hit;
                        w[u] = wn[u];
                    }
                }
            }
            wave_lds_sync();  // the walk's reads are done: clear the marks
            for (int32_t s0 = lane; s0 < T; s0 += kWave) {
                const int32_t sv = H[s0];
                if (sv < -1) H[s0] = sv & kKeyBits;
            }
            wave_lds_sync();
        }
        acc += cnt;
        wave_lds_sync();  // before the next item is staged
    }
    const unsigned long long w = wave_sum(acc);
    if (lane == 0 && w) atomicAdd(&counts[acc_slot], w);
}

// First position of the sorted list x[0, n) whose value exceeds v.
__device__ __forceinline__ int32_t upper_pos(gptr<int32_t> x, int32_t n, int32_t v) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (x[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// The common entries of three sorted lists.
__device__ __forceinline__ unsigned long long three_way(gptr<int32_t> x, int32_t nx, gptr<int32_t> y, int32_t ny,
                                                        gptr<int32_t> z, int32_t nz) {
    unsigned long long c = 0;
    int32_t p = 0, u = 0, v = 0;
    while (p < nx && u < ny && v < nz) {
        const int32_t X = x[p], Y = y[u], Z = z[v];
        const int32_t M = max(X, max(Y, Z));
        if (X == M && Y == M && Z == M) {
            ++c;
            ++p;
            ++u;
            ++v;
        } else {
            p += X < M;
            u += Y < M;
            v += Z < M;
        }
    }
    return c;
}

// Items whose staged rows exceed the LDS region: one thread per (item, b).
__global__ __launch_bounds__(kQB) void k_quad_long(const QuadDesc *__restrict__ quads,
                                                    const int64_t *__restrict__ item_pre, int32_t nq,
                                                    unsigned long long *__restrict__ counts) {
    const gptr<int64_t> ip = as_global(item_pre);
    const int64_t nitems = ip[nq];
    for (int64_t g = blockIdx.x * int64_t(kQB) + threadIdx.x; g < nitems * kQuadSpan;
         g += int64_t(gridDim.x) * kQB) {
        const int64_t q = g / kQuadSpan;  // work item (a part of a row item), and its b
        const int32_t rb = static_cast<int32_t>(g - q * kQuadSpan);
        const int32_t t = quad_of(ip, nq, q);
        const QuadDesc &Q = quads[t];
        const int64_t r = (q - ip[t]) / kQuadParts;
        const int32_t part = static_cast<int32_t>((q - ip[t]) - r * kQuadParts);
        const gptr<int32_t> it = as_global(Q.ij.items) + kItemWords * r;
        const int32_t a = it[0], e = it[1] + part * kQuadSpan + rb;
        if (e >= it[2] || rb + part * kQuadSpan >= kSplitV) continue;
        const gptr<int32_t> ikr = as_global(Q.ik.rptr), ilr = as_global(Q.il.rptr);
        const int32_t k0 = ikr[a], dk = ikr[a + 1] - k0;
        const int32_t l0 = ilr[a], dl = ilr[a + 1] - l0;
        if (dk == 0 || dl == 0 || quad_staged(dk, dl, Q.same)) continue;  // the staged kernel's
        const int32_t b = as_global(Q.ij.col)[e];
        const gptr<int32_t> jkr = as_global(Q.jk.rptr), jlr = as_global(Q.jl.rptr), klr = as_global(Q.kl.rptr);
        const gptr<int32_t> ak = as_global(Q.ik.col) + k0, al = as_global(Q.il.col) + l0;
        const gptr<int32_t> bk = as_global(Q.jk.col) + jkr[b], bl = as_global(Q.jl.col) + jlr[b];
        const int32_t dbk = jkr[b + 1] - jkr[b], dbl = jlr[b + 1] - jlr[b];
        unsigned long long c = 0;
        // entries of A_ik[a] up to the first of A_jk[b] cannot be common
        int32_t x = dbk ? upper_pos(ak, dk, bk[0] - 1) : dk, y = 0;
        while (x < dk && y < dbk) {
            if (ak[x] < bk[y]) {
                ++x;
            } else if (bk[y] < ak[x]) {
                ++y;
            } else {  // c in C: entries of A_kl[c] also in A_il[a] and A_jl[b]
                const int32_t cv = ak[x];
                // with k = l, d > c: the merges of A_il[a] and A_jl[b] start
                // after c (A_kl[c] holds only entries above c)
                const int32_t ul = Q.same ? x + 1 : 0;
                const int32_t vl = Q.same ? y + 1 : 0;
                c += three_way(as_global(Q.kl.col) + klr[cv], klr[cv + 1] - klr[cv], al + ul, dl - ul, bl + vl,
                               dbl - vl);
                ++x;
                ++y;
            }
        }
        if (c) atomicAdd(&counts[Q.slot], c);
    }
}

__global__ void k_zero_u64q(unsigned long long *p, int64_t n) {
    for (int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; q < n; q += int64_t(gridDim.x) * blockDim.x)
        p[q] = 0ull;
}

}  // namespace

uint64_t four_cliques(pgabb_graph *g) {
    hipStream_t s = g->stream;
    const auto t0 = std::chrono::steady_clock::now();
    if (g->p == 0) partition_graph(g, 1, PGABB_CUT_NNZ, nullptr);
    PGABB_REQUIRE(!g->blocks_on_host, PGABB_ESTATE,
                  "the graph's blocks are held in host memory (streamed); the 4-clique count needs them in "
                  "device memory: partition the graph again");
    g->t_kernel_ms = 0;
    g->kernel_launches = 0;
    g->quads.clear();
    g->quad_counts.clear();
    const int32_t p = g->p;
    // ---- the 4-lists: i <= j <= k <= l with six non-empty blocks, heaviest
    // first (edges of the list's blocks)
    auto blk = [&](int32_t x, int32_t y) { return g->block_of[static_cast<size_t>(x) * p + y]; };
    std::vector<std::pair<int64_t, std::array<int32_t, 4>>> lists;
    for (int32_t i = 0; i < p; ++i)
        for (int32_t j = i; j < p; ++j) {
            if (blk(i, j) < 0) continue;
            for (int32_t k = j; k < p; ++k) {
                if (blk(i, k) < 0 || blk(j, k) < 0) continue;
                for (int32_t l = k; l < p; ++l) {
                    const int32_t b6[6] = {blk(i, j), blk(i, k), blk(i, l), blk(j, k), blk(j, l), blk(k, l)};
                    bool ok = true;
                    int64_t w = 0;
                    for (int32_t b : b6) {
                        ok = ok && b >= 0;
                        if (b >= 0) w += g->blocks[b].nnz;
                    }
                    if (ok) lists.push_back({w, {i, j, k, l}});
                }
            }
        }
    std::stable_sort(lists.begin(), lists.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    const int32_t NQ = static_cast<int32_t>(lists.size());
    uint64_t result = 0;
    if (NQ > 0) {
        const int32_t *arena = g->arena.get();
        auto ref = [&](int32_t b) {
            const BlockInfo &bi = g->blocks[b];
            BlockRef r;
            r.rptr = arena + bi.off_rptr();
            r.items = arena + bi.off_items();
            r.col = arena + bi.off_col();
            r.citems = arena + bi.off_citems();
            r.crow = arena + bi.off_crow();
            r.nitems = bi.nitems;
            r.ncitems = bi.ncitems;
            return r;
        };
        Staged<QuadDesc> hq(NQ, s);
        Staged<int64_t> hpre(static_cast<size_t>(NQ) + 1, s);
        hpre[0] = 0;
        for (int32_t q = 0; q < NQ; ++q) {
            const auto &L = lists[q].second;
            QuadDesc &d = hq[q];
            d.ij = ref(blk(L[0], L[1]));
            d.ik = ref(blk(L[0], L[2]));
            d.il = ref(blk(L[0], L[3]));
            d.jk = ref(blk(L[1], L[2]));
            d.jl = ref(blk(L[1], L[3]));
            d.kl = ref(blk(L[2], L[3]));
            d.slot = q;
            d.same = L[2] == L[3];
            d.lshift = d.same ? 0 : g->cuts[L[2] + 1] - g->cuts[L[2]];
            d.pad = 0;
            hpre[q + 1] = hpre[q] + static_cast<int64_t>(kQuadParts) * g->blocks[blk(L[0], L[1])].nitems;
            g->quads.push_back(L);
        }
        DArray<QuadDesc> dq(NQ, s);
        DArray<int64_t> dpre(static_cast<size_t>(NQ) + 1, s);
        DArray<unsigned long long> dcnt(static_cast<size_t>(NQ) + 1, s);  // counts, then the work counter
        PGABB_HIP(hipMemcpyAsync(dq.get(), hq.get(), hq.bytes(), hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(dpre.get(), hpre.get(), hpre.bytes(), hipMemcpyHostToDevice, s));
        k_zero_u64q<<<std::min<unsigned>(grid_for(NQ + 1, 256), 1024u), 256, 0, s>>>(dcnt.get(), NQ + 1);
        PGABB_HIP(hipGetLastError());
        const int64_t nitems = hpre[NQ];
        int32_t max_row = 0;
        for (const auto &b : g->blocks) max_row = std::max(max_row, b.max_row);
        // some row too long to stage (with p > 1, two rows of a 4-list may
        // share the table)
        const bool long_rows = (p == 1 ? max_row : 2 * max_row) > kStageCap;
        StreamTimer tm;
        tm.start(s);
        if (nitems > 0) {
            const unsigned grid =
                static_cast<unsigned>(std::min<int64_t>(256 * 4, (nitems + kCliqueWaves - 1) / kCliqueWaves));
            k_quad_items<<<grid, kCliqueWaves * kWave, 0, s>>>(dq.get(), dpre.get(), NQ, dcnt.get() + NQ, dcnt.get());
            if (long_rows)
                k_quad_long<<<std::min<unsigned>(grid_for(nitems * kQuadSpan, kQB), 256u * 16u), kQB, 0, s>>>(
                    dq.get(), dpre.get(), NQ, dcnt.get());
            PGABB_HIP(hipGetLastError());
        }
        tm.stop(s);
        Staged<unsigned long long> h(NQ, s);
        PGABB_HIP(hipMemcpyAsync(h.get(), dcnt.get(), h.bytes(), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        g->quad_counts.assign(h.get(), h.get() + NQ);
        for (int32_t q = 0; q < NQ; ++q) result += h[q];
        g->t_kernel_ms = tm.ms();
        g->kernel_launches = nitems > 0 ? (long_rows ? 2 : 1) : 0;
    }
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return result;
}

}  // namespace pgabb
