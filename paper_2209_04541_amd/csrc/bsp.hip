// Single-block bulk-synchronous computations over the block partition
// (PGAbB Section 3.2: every iteration visits every edge, and block-lists of
// one block suffice).  Two of the paper's examples run here on the blocks
// the triangle count uses:
//
//   * connected components by Shiloach-Vishkin (Section 3.4): even
//     iterations hook -- for every edge whose endpoints point to different
//     roots, the larger root is hooked under the smaller -- and odd
//     iterations link every vertex to its tree's root by pointer jumping;
//     the iterations stop after a hooking pass that hooked nothing;
//   * PageRank (Section 5.2, an SpMV-like iteration with damping d,
//     tolerance and iteration limit), pulled through the blocks with atomic
//     additions, as the paper does on its two-dimensional layout.
//
// Work items are the blocks' own (x, b, e) records: a run of at most
// kSplitV entries of one row (or, through the stored transpose, of one
// column).  All items of all blocks form one list per launch, one item per
// lane; a lane finds its block by a binary search of the item prefix.  For
// the hooking pass the list is ordered by the stripe an item gathers from
// (the column stripe of a row item) and cut into eight contiguous ranges,
// one work queue each; workgroup b starts on queue
// b % 8, its XCD under round-robin dispatch, so each XCD's gathers fall
// mostly in one or two stripes' slice of the vertex arrays, which its L2
// holds (the two-dimensional layout's locality, per XCD).
// Vertices are ranks (the ids of the oriented graph); results come back by
// input id through the graph's rank array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

constexpr int kBB = 256;
constexpr int kBspQueues = 8;
constexpr int kBspStride = 32;  // queue counters 256 bytes apart
constexpr int kBspQueueWords = kBspQueues * kBspStride;

// Walks the work queues (queue q covers the q-th eighth of the item list): fn(item) for every item this wave takes, one item
// per lane.  Every lane of the wave must call it.
template <class F>
__device__ __forceinline__ void for_items_by_queue(int64_t total, unsigned long long *__restrict__ next, F fn) {
    const int lane = lane_id();
    const int64_t per = (total + kBspQueues - 1) / kBspQueues;
    const int home = static_cast<int>(blockIdx.x % kBspQueues);
    for (int qi = 0; qi < kBspQueues; ++qi) {
        const int q = (home + qi) % kBspQueues;
        const int64_t q0 = q * per, q1 = min(q0 + per, total);
        for (;;) {
            unsigned long long g = 0;
            if (lane == 0) g = atomicAdd(&next[q * kBspStride], static_cast<unsigned long long>(kWave));
            g = shfl_t(g, 0);
            const int64_t i0 = q0 + static_cast<int64_t>(g);
            if (i0 >= q1) break;
            const int64_t item = i0 + lane;
            if (item < q1) fn(item);
        }
    }
}

// One run of items: the row items of a block (entries in `idx` = col, item
// ids in stripe i, entries in stripe j) or its column items (idx = crow,
// item ids in stripe j, entries in stripe i).
struct BspSeg {
    const int32_t *items;
    const int32_t *idx;
    int32_t base_x;  // rank of local id 0 on the item side
    int32_t base_y;  // rank of local id 0 on the entry side
};

// Sum of v over the workgroup (kBB threads, all of which call this),
// returned to thread 0.
__device__ __forceinline__ unsigned long long block_sum(unsigned long long v) {
    __shared__ unsigned long long s_part[kBB / kWave];
    v = wave_sum(v);
    if (lane_id() == 0) s_part[threadIdx.x / kWave] = v;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kBB / kWave; ++w) t += s_part[w];
    return t;
}

// Last segment s with pre[s] <= q (pre[0] = 0 <= q < pre[nseg]).
__device__ __forceinline__ int32_t find_seg(const int64_t *__restrict__ pre, int32_t nseg, int64_t q) {
    int32_t lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBB) void k_sv_init(int32_t *__restrict__ C, int32_t n) {
    for (int64_t r = blockIdx.x * int64_t(kBB) + threadIdx.x; r < n; r += int64_t(gridDim.x) * kBB)
        C[r] = static_cast<int32_t>(r);
}

// Hooking: for every edge (u, v) with C(u) != C(v), the larger of the two
// (a root after the previous linking pass) is hooked under the smaller if it
// still is a root.  Parents only ever decrease (C(x) <= x), so the pointers
// form a forest whatever order the hooks land in.  *hooks becomes nonzero
// when a hook was made (a wave adds its hooks only while it reads zero
// there, so the word takes few atomics).
__global__ __launch_bounds__(kBB) void k_sv_hook(const BspSeg *__restrict__ segs, const int64_t *__restrict__ pre,
                                                 int32_t nseg, int32_t *__restrict__ C,
                                                 unsigned long long *__restrict__ hooks,
                                                 unsigned long long *__restrict__ next) {
    const int64_t total = pre[nseg];
    uint32_t h = 0;
    for_items_by_queue(total, next, [&](int64_t q) {
        const int32_t s = find_seg(pre, nseg, q);
        const BspSeg sg = segs[s];
        const int32_t *it = sg.items + kItemWords * (q - pre[s]);
        const int32_t u = sg.base_x + it[0];
        const int32_t b = it[1], e = it[2];
        for (int32_t t = b; t < e; ++t) {
            const int32_t v = sg.base_y + sg.idx[t];
            const int32_t cu = __atomic_load_n(&C[u], __ATOMIC_RELAXED);
            const int32_t cv = __atomic_load_n(&C[v], __ATOMIC_RELAXED);
            if (cu == cv) continue;
            const int32_t r1 = max(cu, cv), r2 = min(cu, cv);
            if (__atomic_load_n(&C[r1], __ATOMIC_RELAXED) == r1) {
                atomicMin(&C[r1], r2);
                ++h;
            }
        }
    });
    const unsigned long long sum = wave_sum(static_cast<unsigned long long>(h));
    if (lane_id() == 0 && sum && __atomic_load_n(hooks, __ATOMIC_RELAXED) == 0) atomicAdd(hooks, sum);
}

// Linking: every vertex points to the root of its tree (pointer jumping to
// the end; no hook runs meanwhile, so the roots stay fixed).
__global__ __launch_bounds__(kBB) void k_sv_link(int32_t *__restrict__ C, int32_t n) {
    for (int64_t x = blockIdx.x * int64_t(kBB) + threadIdx.x; x < n; x += int64_t(gridDim.x) * kBB) {
        int32_t y = __atomic_load_n(&C[x], __ATOMIC_RELAXED);
        for (;;) {
            const int32_t z = __atomic_load_n(&C[y], __ATOMIC_RELAXED);
            if (z == y) break;
            y = z;
        }
        __atomic_store_n(&C[x], y, __ATOMIC_RELAXED);
    }
}

// Smallest input id of each tree: minid[root] over the input ids v whose
// rank lies in the tree.  Also counts the roots (ranks x with C(x) = x; the
// loop index runs over input ids and ranks alike, both 0 .. n - 1).
__global__ __launch_bounds__(kBB) void k_sv_minid(const int32_t *__restrict__ C, const int32_t *__restrict__ rank,
                                                  int32_t n, int32_t *__restrict__ minid,
                                                  unsigned long long *__restrict__ roots) {
    uint32_t c = 0;
    const int lane = lane_id();
    const int64_t stride = int64_t(gridDim.x) * kBB;
    for (int64_t base = blockIdx.x * int64_t(kBB) + (threadIdx.x & ~(kWave - 1)); base < n; base += stride) {
        const int64_t v = base + lane;
        const bool ok = v < n;
        const int32_t root = ok ? C[rank[v]] : -1;
        // one large component holds most vertices: the lanes whose root is
        // the first lane's send one minimum, the others one atomic each
        const int32_t r0 = __builtin_amdgcn_readfirstlane(root);
        const bool same = ok && root == r0;
        int32_t mv = same ? static_cast<int32_t>(v) : INT32_MAX;
#pragma unroll
        for (int m = 1; m < kWave; m <<= 1) mv = min(mv, __shfl_xor(mv, m));
        if (lane == 0 && r0 >= 0 && mv != INT32_MAX) atomicMin(&minid[r0], mv);
        if (ok && !same) atomicMin(&minid[root], static_cast<int32_t>(v));
        c += ok && C[v] == v ? 1u : 0u;
    }
    const unsigned long long sum = block_sum(static_cast<unsigned long long>(c));
    if (threadIdx.x == 0 && sum) atomicAdd(roots, sum);  // one atomic per workgroup, at most 512
}

__global__ void k_zero_words(unsigned long long *__restrict__ p, int32_t n) {
    for (int32_t q = threadIdx.x; q < n; q += blockDim.x) p[q] = 0ull;
}

// Clears n 8-byte words with a fill kernel (no memset node: a caller may
// capture the stream).
void zero_words(unsigned long long *p, int32_t n, hipStream_t s) {
    k_zero_words<<<1, 64, 0, s>>>(p, n);
}

__global__ __launch_bounds__(kBB) void k_fill_i32(int32_t *__restrict__ p, int32_t v, int64_t n) {
    for (int64_t q = blockIdx.x * int64_t(kBB) + threadIdx.x; q < n; q += int64_t(gridDim.x) * kBB) p[q] = v;
}

__global__ __launch_bounds__(kBB) void k_sv_label(const int32_t *__restrict__ C, const int32_t *__restrict__ rank,
                                                  const int32_t *__restrict__ minid, int32_t n,
                                                  int32_t *__restrict__ label) {
    for (int64_t v = blockIdx.x * int64_t(kBB) + threadIdx.x; v < n; v += int64_t(gridDim.x) * kBB)
        label[v] = minid[C[rank[v]]];
}

// PageRank, one iteration in three launches: each vertex's share
// contrib(x) = r(x) / deg(x) (zero for isolated vertices), the pull of the
// shares over every block's rows and columns into acc, and the update
// r'(x) = (1 - d) / n + d * acc(x) with the sum of |r' - r|.
__global__ __launch_bounds__(kBB) void k_pr_prep(const double *__restrict__ r, const int32_t *__restrict__ outdeg,
                                                 const int32_t *__restrict__ indeg, int32_t n,
                                                 double *__restrict__ contrib, double *__restrict__ acc) {
    for (int64_t x = blockIdx.x * int64_t(kBB) + threadIdx.x; x < n; x += int64_t(gridDim.x) * kBB) {
        const int32_t d = outdeg[x] + indeg[x];
        contrib[x] = d ? r[x] / static_cast<double>(d) : 0.0;
        acc[x] = 0.0;
    }
}

// (PageRank walks the items in block order, grid-stride: dealt to per-XCD
// queues by gather stripe, as the hooking pass is, an iteration on R-MAT
// scale 20 took 0.81 ms against 0.72 ms.)
// The pull: each wave takes 64 consecutive items (one per lane: its target
// x and entry range) and reads their entries as one flattened run over the
// lanes -- consecutive items of a block have consecutive entry ranges, so
// the index loads are contiguous -- finding each element's item by
// scattering the items' first positions into LDS and a running maximum
// over the lanes; each element adds its source's share to its item's sum in
// LDS, and every item adds its sum to acc[x] once.
__global__ __launch_bounds__(kBB) void k_pr_pull(const BspSeg *__restrict__ segs, const int64_t *__restrict__ pre,
                                                 int32_t nseg, const double *__restrict__ contrib_,
                                                 double *__restrict__ acc) {
    __shared__ double s_sum[kBB];
    __shared__ int32_t s_own[kBB];
    const int lane = lane_id();
    double *sum = s_sum + (threadIdx.x - lane);
    int32_t *own = s_own + (threadIdx.x - lane);
    const gptr<double> contrib = as_global(contrib_);
    own[lane] = 0;
    wave_lds_sync();
    const int64_t total = pre[nseg];
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBB;
    for (int64_t q0 = blockIdx.x * int64_t(kBB) + (threadIdx.x - lane); q0 < total; q0 += stride) {
        const int64_t q = q0 + lane;
        int32_t x = 0, len = 0, by = 0;
        const int32_t *src = nullptr;  // the item's entries: src[0 .. len)
        if (q < total) {
            const int32_t s = find_seg(pre, nseg, q);
            const BspSeg sg = segs[s];
            const gptr<int32_t> it = as_global(sg.items) + kItemWords * (q - pre[s]);
            x = sg.base_x + it[0];
            const int32_t b = it[1], e = it[2];
            len = e - b;
            src = sg.idx + b;
            by = sg.base_y;
        }
        sum[lane] = 0.0;
        const int32_t incl = wave_inclusive_scan(len);
        const int32_t pre_l = incl - len;
        const int32_t tot = __builtin_amdgcn_readlane(incl, kWave - 1);
        // element el of the run is src[el - pre_l] of its item's lane
        const uint64_t rel = reinterpret_cast<uint64_t>(src) - static_cast<uint64_t>(pre_l) * sizeof(int32_t);
        const uint32_t rel_lo = static_cast<uint32_t>(rel), rel_hi = static_cast<uint32_t>(rel >> 32);
        wave_lds_sync();
        uint32_t carry = 0;
        for (int32_t base = 0; base < tot; base += kWave) {
            const int32_t p = pre_l - base;
            if (len > 0 && p >= 0 && p < kWave) own[p] = lane + 1;
            wave_lds_sync();
            const uint32_t o = static_cast<uint32_t>(own[lane]);
            own[lane] = 0;
            wave_lds_sync();
            const uint32_t sl1 = max(wave_max_scan_dpp(o), carry);
            carry = __builtin_amdgcn_readlane(sl1, kWave - 1);
            const int sl = static_cast<int>(sl1) - 1;
            const uint64_t r = (static_cast<uint64_t>(static_cast<uint32_t>(__shfl(static_cast<int>(rel_hi), sl)))
                                << 32) |
                               static_cast<uint32_t>(__shfl(static_cast<int>(rel_lo), sl));
            const int32_t yb = __shfl(by, sl);
            const int32_t el = base + lane;
            if (el < tot) {
                const gptr<int32_t> ptr = as_global(reinterpret_cast<const int32_t *>(r));
                unsafeAtomicAdd(&sum[sl], contrib[yb + ptr[el]]);
            }
        }
        wave_lds_sync();
        if (len > 0) unsafeAtomicAdd(&acc[x], sum[lane]);
        wave_lds_sync();  // before the next items reset the sums
    }
}

__global__ __launch_bounds__(kBB) void k_pr_update(double *__restrict__ r, const double *__restrict__ acc, int32_t n,
                                                   double teleport, double d, double *__restrict__ err) {
    double e = 0.0;
    for (int64_t x = blockIdx.x * int64_t(kBB) + threadIdx.x; x < n; x += int64_t(gridDim.x) * kBB) {
        const double nx = teleport + d * acc[x];
        e += fabs(nx - r[x]);
        r[x] = nx;
    }
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) e += __shfl_xor(e, m);
    // one atomic per workgroup: the launch keeps its grid small, so the
    // additions to the one address stay few
    __shared__ double s_part[kBB / kWave];
    if (lane_id() == 0) s_part[threadIdx.x / kWave] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBB / kWave; ++w) t += s_part[w];
        if (t != 0.0) unsafeAtomicAdd(err, t);
    }
}

__global__ __launch_bounds__(kBB) void k_pr_init(double *__restrict__ r, int32_t n, double v) {
    for (int64_t x = blockIdx.x * int64_t(kBB) + threadIdx.x; x < n; x += int64_t(gridDim.x) * kBB) r[x] = v;
}

__global__ __launch_bounds__(kBB) void k_pr_by_id(const double *__restrict__ r, const int32_t *__restrict__ rank,
                                                  int32_t n, double *__restrict__ out) {
    for (int64_t v = blockIdx.x * int64_t(kBB) + threadIdx.x; v < n; v += int64_t(gridDim.x) * kBB)
        out[v] = r[rank[v]];
}

// Grid of a grid-stride launch over `work` elements: enough workgroups to
// fill every CU a few times over, no more than the work needs.
unsigned bsp_grid(int64_t work) {
    const unsigned need = grid_for(work, kBB);
    return std::min(need, 256u * 16u);
}

// The item segments of the graph's blocks (rows only, or rows and columns),
// staged on the device.
struct Segs {
    DArray<BspSeg> segs;
    DArray<int64_t> pre;
    int32_t n = 0;
    int64_t total = 0;
};

void make_segs(pgabb_graph *g, bool columns_too, bool by_gather_stripe, Segs &out) {
    hipStream_t s = g->stream;
    const int32_t *arena = g->arena.get();
    // (gather stripe, segment, items), ordered by the gather stripe
    struct Entry {
        int32_t stripe;
        BspSeg seg;
        int64_t items;
    };
    std::vector<Entry> ev;
    for (const BlockInfo &bi : g->blocks) {
        if (bi.nnz == 0) continue;
        if (bi.nitems > 0)
            ev.push_back({bi.j, BspSeg{arena + bi.off_items(), arena + bi.off_col(), g->base[bi.i], g->base[bi.j]},
                          bi.nitems});
        if (columns_too && bi.ncitems > 0)
            ev.push_back({bi.i, BspSeg{arena + bi.off_citems(), arena + bi.off_crow(), g->base[bi.j], g->base[bi.i]},
                          bi.ncitems});
    }
    if (by_gather_stripe)
        std::stable_sort(ev.begin(), ev.end(), [](const Entry &a, const Entry &b) { return a.stripe < b.stripe; });
    std::vector<BspSeg> sv;
    std::vector<int64_t> pv(1, 0);
    for (const Entry &e : ev) {
        sv.push_back(e.seg);
        pv.push_back(pv.back() + e.items);
    }
    out.n = static_cast<int32_t>(sv.size());
    out.total = pv.back();
    if (out.n == 0) return;
    Staged<BspSeg> hs(sv.size(), s);
    Staged<int64_t> hp(pv.size(), s);
    std::copy(sv.begin(), sv.end(), hs.get());
    std::copy(pv.begin(), pv.end(), hp.get());
    out.segs.reset(sv.size(), s);
    out.pre.reset(pv.size(), s);
    PGABB_HIP(hipMemcpyAsync(out.segs.get(), hs.get(), hs.bytes(), hipMemcpyHostToDevice, s));
    PGABB_HIP(hipMemcpyAsync(out.pre.get(), hp.get(), hp.bytes(), hipMemcpyHostToDevice, s));
}

// The computation runs on the graph's device blocks; a graph that was never
// partitioned is partitioned with p = 1 first.
void require_blocks(pgabb_graph *g) {
    if (g->p == 0) partition_graph(g, 1, PGABB_CUT_NNZ, nullptr);
    PGABB_REQUIRE(!g->blocks_on_host, PGABB_ESTATE,
                  "the graph's blocks are held in host memory (streamed); the bulk-synchronous "
                  "computations need them in device memory: partition the graph again");
}

}  // namespace

int64_t components(pgabb_graph *g, int32_t *label, bool on_device, int32_t *iterations) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    int32_t iters = 0;
    int64_t comps = 0;
    double kernel_ms = 0;
    if (n > 0) {
        require_blocks(g);
        Segs sg;
        make_segs(g, false, true, sg);
        DArray<int32_t> C(static_cast<size_t>(n), s);
        DArray<unsigned long long> ctr(2 + kBspQueueWords, s);  // hooks, roots, work queues
        Staged<unsigned long long> hctr(2, s);
        StreamTimer tm;
        tm.start(s);
        k_sv_init<<<bsp_grid(n), kBB, 0, s>>>(C.get(), n);
        PGABB_HIP(hipGetLastError());
        tm.stop(s);
        kernel_ms += tm.ms();
        for (;;) {
            // one hooking and one linking iteration; stop after a hooking
            // pass that hooked nothing
            tm.start(s);
            zero_words(ctr.get(), 1, s);
            zero_words(ctr.get() + 2, kBspQueueWords, s);
            if (sg.total > 0)
                k_sv_hook<<<bsp_grid(sg.total), kBB, 0, s>>>(sg.segs.get(), sg.pre.get(), sg.n, C.get(), ctr.get(),
                                                             ctr.get() + 2);
            k_sv_link<<<bsp_grid(n), kBB, 0, s>>>(C.get(), n);
            PGABB_HIP(hipGetLastError());
            tm.stop(s);
            PGABB_HIP(hipMemcpyAsync(hctr.get(), ctr.get(), sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
            PGABB_HIP(hipStreamSynchronize(s));
            kernel_ms += tm.ms();
            iters += 2;
            if (hctr[0] == 0) break;
        }
        DArray<int32_t> minid(static_cast<size_t>(n), s);
        DArray<int32_t> own;
        int32_t *dst = label;
        if (!on_device) {
            own.reset(static_cast<size_t>(n), s);
            dst = own.get();
        }
        tm.start(s);
        k_fill_i32<<<bsp_grid(n), kBB, 0, s>>>(minid.get(), INT32_MAX, n);
        zero_words(ctr.get() + 1, 1, s);
        k_sv_minid<<<std::min(bsp_grid(n), 512u), kBB, 0, s>>>(C.get(), g->rank.get(), n, minid.get(), ctr.get() + 1);
        k_sv_label<<<bsp_grid(n), kBB, 0, s>>>(C.get(), g->rank.get(), minid.get(), n, dst);
        PGABB_HIP(hipGetLastError());
        tm.stop(s);
        PGABB_HIP(hipMemcpyAsync(hctr.get() + 1, ctr.get() + 1, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        if (!on_device)
            PGABB_HIP(hipMemcpyAsync(label, dst, sizeof(int32_t) * static_cast<size_t>(n), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        kernel_ms += tm.ms();
        comps = static_cast<int64_t>(hctr[1]);
    }
    if (iterations) *iterations = iters;
    g->t_kernel_ms = kernel_ms;
    g->kernel_launches = iters;
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return comps;
}

int32_t pagerank(pgabb_graph *g, double damping, double tol, int32_t max_iter, double *ranks, bool on_device,
                 double *last_err) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    int32_t iters = 0;
    double err = 0, kernel_ms = 0;
    if (n > 0) {
        require_blocks(g);
        Segs sg;
        make_segs(g, true, false, sg);
        DArray<double> r(static_cast<size_t>(n), s), contrib(static_cast<size_t>(n), s), acc(static_cast<size_t>(n), s);
        DArray<double> derr(1, s);
        Staged<double> herr(1, s);
        const double teleport = (1.0 - damping) / n;
        StreamTimer tm;
        tm.start(s);
        k_pr_init<<<bsp_grid(n), kBB, 0, s>>>(r.get(), n, 1.0 / n);
        PGABB_HIP(hipGetLastError());
        tm.stop(s);
        kernel_ms += tm.ms();
        while (iters < max_iter) {
            tm.start(s);
            k_pr_prep<<<bsp_grid(n), kBB, 0, s>>>(r.get(), g->outdeg.get(), g->indeg.get(), n, contrib.get(), acc.get());
            if (sg.total > 0)
                k_pr_pull<<<bsp_grid(sg.total), kBB, 0, s>>>(sg.segs.get(), sg.pre.get(), sg.n, contrib.get(), acc.get());
            zero_words(reinterpret_cast<unsigned long long *>(derr.get()), 1, s);  // +0.0 is all zero bits
            k_pr_update<<<std::min(bsp_grid(n), 512u), kBB, 0, s>>>(r.get(), acc.get(), n, teleport, damping,
                                                                   derr.get());
            PGABB_HIP(hipGetLastError());
            tm.stop(s);
            PGABB_HIP(hipMemcpyAsync(herr.get(), derr.get(), sizeof(double), hipMemcpyDeviceToHost, s));
            PGABB_HIP(hipStreamSynchronize(s));
            kernel_ms += tm.ms();
            ++iters;
            err = herr[0];
            if (err < tol) break;
        }
        DArray<double> own;
        double *dst = ranks;
        if (!on_device) {
            own.reset(static_cast<size_t>(n), s);
            dst = own.get();
        }
        k_pr_by_id<<<bsp_grid(n), kBB, 0, s>>>(r.get(), g->rank.get(), n, dst);
        PGABB_HIP(hipGetLastError());
        if (!on_device)
            PGABB_HIP(hipMemcpyAsync(ranks, dst, sizeof(double) * static_cast<size_t>(n), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
    }
    if (last_err) *last_err = err;
    g->t_kernel_ms = kernel_ms;
    g->kernel_launches = iters;
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return iters;
}

}  // namespace pgabb
