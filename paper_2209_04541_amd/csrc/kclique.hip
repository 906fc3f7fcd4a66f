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
// bit and the slot's bit in a bitmap of C or of D; then the lists A_kl[c] of
// the marked keys of stripe k (C), found from C's bitmap and gathered up to
// 64 at a time, are walked flattened over the lanes, counting the entries
// whose key is marked (in D); the bitmaps lead the clearing of the marks.
// A b with no marks costs its look-ups only.  Blocks hold column ids local
// to their stripe, so when k < l the ids of stripe l enter the table shifted
// by the width of stripe k: keys of A_ik[a] lie below that width and keys of
// A_il[a] above it, and an entry of A_kl[c] (stripe l, shifted too) can only
// match a key of A_il[a].  Items whose staged rows hold more than kStageCap
// entries go to a kernel with one thread per (item, b) and plain merges.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <list>
#include <vector>

#include "common.hpp"
#include "graph.hpp"
#include "range_pool.hpp"
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
// Work counters: the items are cut into chunks of `grab` items, chunk c
// belongs to counter c mod kQuadQueues, and a wave takes chunks from the
// counter of its workgroup's XCD (workgroups are dealt round-robin to the 8
// XCDs), moving on to the next counter when that one runs dry.  At p = 8
// most items end after a few loads (a row of A_ij with no entries in stripe
// k or l), and one counter taking one item per grab serialised the launch
// on the grabs' round trips; at p = 1 the items are heavy and large chunks
// unbalance the waves.  So the chunk is sized per launch for about
// kQuadGrabsPerWave grabs per wave, within [kQuadGrabMin, kQuadGrabMax].
constexpr int kQuadQueues = 8;
constexpr int64_t kQuadGrabsPerWave = 256;
constexpr int64_t kQuadGrabMin = 4;
constexpr int64_t kQuadGrabMax = 64;
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
// looked up as its id plus `add` (ids above top cannot be there), sets the
// marked slots' bits in `bits`, and returns how many it marked (the same on
// every lane).  Every lane of the wave calls this.
__device__ __forceinline__ int32_t quad_mark(int32_t *H, uint32_t *bits, int shift, uint32_t tmask, gptr<int32_t> x,
                                             int32_t n, int32_t top, int32_t add, int lane) {
    int32_t marked = 0;
    for (int32_t x0 = 0; x0 < n; x0 += kWave) {
        const int32_t i = x0 + lane;
        const int32_t u = i < n ? x[i] : -1;
        bool go = u >= 0 && u <= top;
        const int32_t v = u + add;
        uint32_t h = hash_slot(v, shift, tmask);
        while (__ballot(go) != 0) {
            const int32_t sv = H[h];
            const bool hit = go && sv == v;
            if (hit) {
                H[h] = v | kMarkBit;
                atomicOr(&bits[h >> 5], 1u << (h & 31));
            }
            marked += __popcll(__ballot(hit));
            go = go && sv != -1 && (sv & kKeyBits) != v;
            h = (h + 1) & tmask;
        }
        if (__ballot(u > top) != 0) break;  // the rest of the list is above top too
    }
    return marked;
}

// Staged items: one wave per item from a work counter.  Counts go to the
// 4-lists' counters, one atomic per run of items of the same list a wave
// takes.
__global__ __launch_bounds__(kCliqueWaves *kWave) void k_quad_items(const QuadDesc *__restrict__ quads,
                                                                     const int64_t *__restrict__ item_pre,
                                                                     int32_t nq,
                                                                     unsigned long long *__restrict__ next,
                                                                     int64_t grab,
                                                                     unsigned long long *__restrict__ counts) {
    __shared__ int32_t s_table[kCliqueWaves][1 << kTableLg];
    __shared__ int32_t s_own[kCliqueWaves][kQuadUnroll * kWave];
    __shared__ int32_t s_gather[kCliqueWaves][2][kWave];  // walked lists: start, length
    // slots marked in C and in D, one bit each (2^kTableLg / 32 words)
    __shared__ uint32_t s_bits[kCliqueWaves][2][(1 << kTableLg) / 32];
    int32_t *H = s_table[threadIdx.x / kWave];
    int32_t *own = s_own[threadIdx.x / kWave];
    int32_t *gpb = s_gather[threadIdx.x / kWave][0];
    int32_t *glen = s_gather[threadIdx.x / kWave][1];
    uint32_t *bits_c = s_bits[threadIdx.x / kWave][0];
    uint32_t *bits_d = s_bits[threadIdx.x / kWave][1];
    const int lane = lane_id();
#pragma unroll
    for (int q = 0; q < kQuadUnroll; ++q) own[q * kWave + lane] = 0;
    for (int q = lane; q < (1 << kTableLg) / 32; q += kWave) bits_c[q] = bits_d[q] = 0u;
    wave_lds_sync();
    const gptr<int64_t> ip = as_global(item_pre);
    const int64_t nitems = ip[nq];
    unsigned long long acc = 0;  // this lane's share of the current list's count
    int32_t acc_slot = -1;
    const int64_t nchunks = (nitems + grab - 1) / grab;
    int32_t qi = static_cast<int32_t>(blockIdx.x % kQuadQueues);
    for (int32_t dry = 0; dry < kQuadQueues;) {
        unsigned long long k = 0;
        if (lane == 0) k = atomicAdd(&next[qi], 1ull);
        k = shfl_t(k, 0);
        const int64_t c = static_cast<int64_t>(k) * kQuadQueues + qi;
        if (c >= nchunks) {  // this counter is dry: the next one
            qi = (qi + 1) % kQuadQueues;
            ++dry;
            continue;
        }
        dry = 0;
        const int64_t g0 = c * grab;
        const int64_t gend = min(g0 + grab, nitems);
        int32_t t = __builtin_amdgcn_readfirstlane(quad_of(ip, nq, g0));
        for (int64_t q = g0; q < gend; ++q) {
            while (ip[t + 1] <= q) ++t;  // the next non-empty 4-list (ip[nq] = nitems > q)
            t = __builtin_amdgcn_readfirstlane(t);
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
            if (Q.slot != acc_slot) {  // counts gather per 4-list (its slot among all the count's lists)
                const unsigned long long w = wave_sum(acc);
                if (lane == 0 && w) atomicAdd(&counts[acc_slot], w);
                acc = 0;
                acc_slot = Q.slot;
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
                const int32_t nc = quad_mark(H, bits_c, shift, tmask, jkc + bk0, dbk, topk, 0, lane);  // C (and D when k = l)
                const int32_t nd =
                    Q.same ? nc : quad_mark(H, bits_d, shift, tmask, jlc + bl0, dbl, topl, Q.lshift, lane);  // D
                if (nc + nd == 0) continue;  // nothing marked: the table is as staged
                wave_lds_sync();
                // walk A_kl[c] for the marked keys c of stripe k: the marked slots
                // are gathered, 64 slots of the table at a time, into lists of at
                // most one per lane, and each full set of 64 lists (and the last)
                // is walked as one flattened sequence; only when a pair c < d can
                // be there (C and D non-empty; two marks when they are one set)
                const bool pairs = nc > 0 && nd > 0 && (!Q.same || nc >= 2);
                auto walk_gathered = [&](int32_t ng) {
                    wave_lds_sync();  // the gathered lists are written
                    const int32_t pb = lane < ng ? gpb[lane] : 0;
                    const int32_t len = lane < ng ? glen[lane] : 0;
                    wave_lds_sync();  // read before the next lists are gathered
                    const int32_t incl = wave_inclusive_scan(len);
                    const int32_t pre = incl - len;
                    const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
                    if (total == 0) return;
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
                };
                // gather: lane q takes word q of C's bitmap (the table has at most
                // 2^kTableLg = 64 words of slots) and places its marked slots' lists
                // after those of the lanes below it; 64 lists at most per walk
                const int32_t nw = T >> 5;
                int32_t ng = 0;  // lists gathered so far (the same on every lane)
                uint32_t word = pairs && lane < nw ? bits_c[lane] : 0u;
                for (;;) {
                    const int32_t mine = __popc(word);
                    const int32_t incl = wave_inclusive_scan(mine);
                    const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
                    if (total == 0) break;
                    int32_t at = ng + incl - mine;
                    while (word != 0u && at < kWave) {
                        const int32_t slot = (lane << 5) + __builtin_ctz(word);
                        word &= word - 1u;
                        const int32_t c = H[slot] & kKeyBits;
                        const int32_t c0 = klr[c];
                        gpb[at] = c0;
                        glen[at] = klr[c + 1] - c0;
                        ++at;
                    }
                    if (ng + total <= kWave) {
                        ng += total;
                        break;
                    }
                    walk_gathered(kWave);  // full: walk these, then place the rest
                    ng = 0;
                }
                if (ng > 0) walk_gathered(ng);
                wave_lds_sync();  // the walk's reads are done: clear the marks
                if (lane < nw) {
                    uint32_t mk = bits_c[lane] | bits_d[lane];
                    while (mk != 0u) {
                        const int32_t slot = (lane << 5) + __builtin_ctz(mk);
                        mk &= mk - 1u;
                        H[slot] &= kKeyBits;
                    }
                    bits_c[lane] = 0u;
                    bits_d[lane] = 0u;
                }
                wave_lds_sync();
            }
            acc += cnt;
            wave_lds_sync();  // before the next item is staged
        }
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

namespace {

// Bytes of the row part of a block's chunk (row items, row offsets,
// columns: what the 4-clique kernels read), rounded to the pool alignment.
constexpr uint64_t kQuadAlign = 256;
uint64_t quad_chunk_bytes(const BlockInfo &b) {
    const uint64_t raw = static_cast<uint64_t>(b.walk_hi(kOrientRow) - b.walk_lo(kOrientRow)) * sizeof(int32_t);
    return (raw + kQuadAlign - 1) / kQuadAlign * kQuadAlign;
}

// Device view of a block whose row part starts at `base` (device words).
BlockRef quad_ref(const BlockInfo &bi, const int32_t *base) {
    BlockRef r;
    const int64_t lo = bi.walk_lo(kOrientRow);
    r.rptr = base + (bi.off_rptr() - lo);
    r.items = base + (bi.off_items() - lo);
    r.col = base + (bi.off_col() - lo);
    r.citems = nullptr;  // the 4-clique kernels walk rows only
    r.crow = nullptr;
    r.nitems = bi.nitems;
    r.ncitems = bi.ncitems;
    return r;
}

// Counts the 4-lists lists[first, last) (their blocks at the given device
// bases), adding to dcnt[slot]; dcnt[NQ .. NQ + kQuadQueues) are the work
// counters.
void quad_launch(pgabb_graph *g, const std::vector<std::array<int32_t, 4>> &lists, int32_t first, int32_t last,
                 const std::vector<const int32_t *> &base, unsigned long long *dcnt, int32_t NQ, double &kernel_ms,
                 int64_t &launches) {
    hipStream_t s = g->stream;
    const int32_t p = g->p;
    const int32_t W = last - first;
    auto blk = [&](int32_t x, int32_t y) { return g->block_of[static_cast<size_t>(x) * p + y]; };
    Staged<QuadDesc> hq(W, s);
    Staged<int64_t> hpre(static_cast<size_t>(W) + 1, s);
    hpre[0] = 0;
    int32_t max_row = 0;
    for (int32_t q = 0; q < W; ++q) {
        const auto &L = lists[first + q];
        QuadDesc &d = hq[q];
        const int32_t b6[6] = {blk(L[0], L[1]), blk(L[0], L[2]), blk(L[0], L[3]),
                               blk(L[1], L[2]), blk(L[1], L[3]), blk(L[2], L[3])};
        BlockRef *r6[6] = {&d.ij, &d.ik, &d.il, &d.jk, &d.jl, &d.kl};
        for (int x = 0; x < 6; ++x) {
            *r6[x] = quad_ref(g->blocks[b6[x]], base[b6[x]]);
            max_row = std::max(max_row, g->blocks[b6[x]].max_row);
        }
        d.slot = first + q;
        d.same = L[2] == L[3];
        d.lshift = d.same ? 0 : g->cuts[L[2] + 1] - g->cuts[L[2]];
        d.pad = 0;
        hpre[q + 1] = hpre[q] + static_cast<int64_t>(kQuadParts) * g->blocks[b6[0]].nitems;
    }
    const int64_t nitems = hpre[W];
    if (nitems == 0) return;
    DArray<QuadDesc> dq(W, s);
    DArray<int64_t> dpre(static_cast<size_t>(W) + 1, s);
    PGABB_HIP(hipMemcpyAsync(dq.get(), hq.get(), hq.bytes(), hipMemcpyHostToDevice, s));
    PGABB_HIP(hipMemcpyAsync(dpre.get(), hpre.get(), hpre.bytes(), hipMemcpyHostToDevice, s));
    k_zero_u64q<<<1, 64, 0, s>>>(dcnt + NQ, kQuadQueues);  // the work counters
    // some row too long to stage (with p > 1, two rows of a 4-list may
    // share the table)
    const bool long_rows = (p == 1 ? max_row : 2 * max_row) > kStageCap;
    StreamTimer tm;
    tm.start(s);
    const unsigned grid =
        static_cast<unsigned>(std::min<int64_t>(256 * 4, (nitems + kCliqueWaves - 1) / kCliqueWaves));
    int64_t grab = kQuadGrabMin;
    while (grab < kQuadGrabMax && nitems / (grab * 2) >= kQuadGrabsPerWave * grid * kCliqueWaves) grab *= 2;
    k_quad_items<<<grid, kCliqueWaves * kWave, 0, s>>>(dq.get(), dpre.get(), W, dcnt + NQ, grab, dcnt);
    if (long_rows)
        k_quad_long<<<std::min<unsigned>(grid_for(nitems * kQuadSpan, kQB), 256u * 16u), kQB, 0, s>>>(
            dq.get(), dpre.get(), W, dcnt);
    PGABB_HIP(hipGetLastError());
    tm.stop(s);
    PGABB_HIP(hipStreamSynchronize(s));  // the descriptors and the blocks may go once this returns
    kernel_ms += tm.ms();
    launches += long_rows ? 2 : 1;
}

}  // namespace

uint64_t four_cliques(pgabb_graph *g, uint64_t device_cap_bytes) {
    hipStream_t s = g->stream;
    const auto t0 = std::chrono::steady_clock::now();
    if (g->p == 0) partition_graph(g, 1, PGABB_CUT_NNZ, nullptr);
    g->t_kernel_ms = 0;
    g->kernel_launches = 0;
    g->h2d_bytes = 0;
    g->quads.clear();
    g->quad_counts.clear();
    const int32_t p = g->p;
    // ---- the 4-lists: i <= j <= k <= l with six non-empty blocks, heaviest
    // first (edges of the list's blocks)
    auto blk = [&](int32_t x, int32_t y) { return g->block_of[static_cast<size_t>(x) * p + y]; };
    std::vector<std::pair<int64_t, std::array<int32_t, 4>>> ranked;
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
                    if (ok) ranked.push_back({w, {i, j, k, l}});
                }
            }
        }
    std::stable_sort(ranked.begin(), ranked.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    const int32_t NQ = static_cast<int32_t>(ranked.size());
    for (const auto &x : ranked) g->quads.push_back(x.second);
    uint64_t result = 0;
    if (NQ > 0) {
        const int32_t nblk = static_cast<int32_t>(g->blocks.size());
        DArray<unsigned long long> dcnt(static_cast<size_t>(NQ) + kQuadQueues, s);  // counts, then the work counters
        k_zero_u64q<<<std::min<unsigned>(grid_for(NQ + kQuadQueues, 256), 1024u), 256, 0, s>>>(dcnt.get(),
                                                                                           NQ + kQuadQueues);
        PGABB_HIP(hipGetLastError());
        double kernel_ms = 0;
        int64_t launches = 0;
        const bool streamed = device_cap_bytes > 0 || g->blocks_on_host;
        if (!streamed) {
            std::vector<const int32_t *> base(nblk);
            for (int32_t b = 0; b < nblk; ++b) base[b] = g->arena.get() + g->blocks[b].walk_lo(kOrientRow);
            quad_launch(g, g->quads, 0, NQ, base, dcnt.get(), NQ, kernel_ms, launches);
        } else {
            // ---- streamed: the blocks move from the host store through a
            // cache of at most `cap` bytes.  Consecutive 4-lists form a
            // window while the union of their blocks fits the cap; the
            // window's missing blocks are copied (least recently used blocks
            // outside the window leave first; if the free ranges are too
            // fragmented the cache starts over), then the window is counted.
            if (!g->blocks_on_host) move_blocks_to_host(g);
            if (device_cap_bytes == 0) device_cap_bytes = g->host_store_cap;
            std::vector<uint64_t> bytes(nblk);
            uint64_t total = 0;
            for (int32_t b = 0; b < nblk; ++b) total += bytes[b] = quad_chunk_bytes(g->blocks[b]);
            uint64_t cap = device_cap_bytes ? std::min(device_cap_bytes, total) : total;
            cap = cap / kQuadAlign * kQuadAlign;
            auto list_blocks = [&](int32_t q, int32_t (&b6)[6]) {
                const auto &L = g->quads[q];
                const int32_t x[6] = {blk(L[0], L[1]), blk(L[0], L[2]), blk(L[0], L[3]),
                                      blk(L[1], L[2]), blk(L[1], L[3]), blk(L[2], L[3])};
                for (int y = 0; y < 6; ++y) b6[y] = x[y];
            };
            DArray<uint8_t> pool(static_cast<size_t>(cap), s);
            RangePool rp(cap);
            std::vector<uint64_t> off(nblk, UINT64_MAX);  // pool offset of resident blocks
            std::list<int32_t> lru;                       // resident blocks, least recently used first
            std::vector<std::list<int32_t>::iterator> where(nblk, lru.end());
            std::vector<int32_t> mark(nblk, -1);          // window that uses the block
            std::vector<const int32_t *> base(nblk, nullptr);
            const int32_t *host = g->host_arena.get();
            constexpr int32_t kMaxWindow = 512;  // 4-lists per launch
            int32_t q = 0, win = 0;
            while (q < NQ) {
                // the window: lists [q, e) whose blocks fit together
                std::vector<int32_t> wb;
                uint64_t need = 0;
                int32_t e = q;
                while (e < NQ && e - q < kMaxWindow) {
                    int32_t b6[6];
                    list_blocks(e, b6);
                    uint64_t add = 0;
                    std::vector<int32_t> fresh;
                    for (int32_t b : b6)
                        if (mark[b] != win && std::find(fresh.begin(), fresh.end(), b) == fresh.end()) {
                            fresh.push_back(b);
                            add += bytes[b];
                        }
                    if (need + add > cap) {
                        PGABB_REQUIRE(e > q, PGABB_ENOMEM,
                                      "device cap of %llu bytes cannot hold the %llu bytes of 4-list (%d, %d, %d, %d)",
                                      static_cast<unsigned long long>(cap), static_cast<unsigned long long>(add),
                                      g->quads[e][0], g->quads[e][1], g->quads[e][2], g->quads[e][3]);
                        break;
                    }
                    for (int32_t b : fresh) {
                        mark[b] = win;
                        wb.push_back(b);
                    }
                    need += add;
                    ++e;
                }
                // make the window's blocks resident
                for (int pass = 0; pass < 2; ++pass) {
                    bool ok = true;
                    for (int32_t b : wb) {
                        if (off[b] != UINT64_MAX) {
                            lru.splice(lru.end(), lru, where[b]);  // most recently used
                            continue;
                        }
                        uint64_t o = rp.alloc(bytes[b]);
                        while (o == UINT64_MAX) {  // evict blocks outside the window
                            auto it = lru.begin();
                            while (it != lru.end() && mark[*it] == win) ++it;
                            if (it == lru.end()) break;
                            rp.release(off[*it], bytes[*it]);
                            off[*it] = UINT64_MAX;
                            base[*it] = nullptr;
                            where[*it] = lru.end();
                            lru.erase(it);
                            o = rp.alloc(bytes[b]);
                        }
                        if (o == UINT64_MAX) {
                            ok = false;
                            break;
                        }
                        off[b] = o;
                        const BlockInfo &bi = g->blocks[b];
                        const int64_t lo = bi.walk_lo(kOrientRow);
                        const uint64_t raw = static_cast<uint64_t>(bi.walk_hi(kOrientRow) - lo) * sizeof(int32_t);
                        uint8_t *dst = pool.get() + o;
                        if (raw) PGABB_HIP(hipMemcpyAsync(dst, host + lo, raw, hipMemcpyHostToDevice, s));
                        g->h2d_bytes += raw;
                        base[b] = reinterpret_cast<const int32_t *>(dst);
                        where[b] = lru.insert(lru.end(), b);
                    }
                    if (ok) break;
                    // fragmented: drop every block and place the window from an empty cache
                    PGABB_REQUIRE(pass == 0, PGABB_EDEVICE, "4-clique block cache could not place a window");
                    for (int32_t b : lru) {
                        off[b] = UINT64_MAX;
                        base[b] = nullptr;
                        where[b] = lru.end();
                    }
                    lru.clear();
                    rp = RangePool(cap);
                }
                quad_launch(g, g->quads, q, e, base, dcnt.get(), NQ, kernel_ms, launches);
                q = e;
                ++win;
            }
        }
        Staged<unsigned long long> h(NQ, s);
        PGABB_HIP(hipMemcpyAsync(h.get(), dcnt.get(), h.bytes(), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        g->quad_counts.assign(h.get(), h.get() + NQ);
        for (int32_t x = 0; x < NQ; ++x) result += h[x];
        g->t_kernel_ms = kernel_ms;
        g->kernel_launches = launches;
    }
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return result;
}

}  // namespace pgabb
