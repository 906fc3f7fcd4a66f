// Batched counting of many small graphs in one persistent, graph-captured
// launch.
//
// The G graphs are packed as a disjoint union: graph g owns the global
// vertex range [vbase[g], vbase[g+1]).  The build runs once over all graphs
// with the graph id in the top bits of every sort key, so one radix sort per
// step cleans, ranks (ascending (degree, id) within each graph) and orients
// every graph.  Counting is PGAbB's task-parallel execution (Section 4.4)
// applied across graphs: each row of the union with at least two
// out-neighbours is a work item; one persistent kernel drains a device work
// counter and adds every row's triangles to its graph's uint64 slot.  The
// zeroing, the kernel and the copy of the slots to pinned host memory are
// captured once into a HIP graph and replayed.
//
// The launch shape (staging structure, waves per workgroup, rows per grab)
// is picked by an autotuner that times the candidates on the batch itself
// and caches the winner by the batch's shape features.
#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>

#include "common.hpp"
#include "graph.hpp"
#include "tc_device.hpp"
#include "wave.hpp"

namespace pgabb {
bool radix_sort_u64_bits(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                         int64_t n, int lo_bit, int hi_bit, hipStream_t s);
}

struct pgabb_batch {
    hipStream_t stream = nullptr;
    int64_t G = 0;
    int nb = 1, gbits = 1;
    int64_t total_n = 0, total_m = 0, mu = 0, nactive = 0;
    int32_t max_out = 0, max_n = 0;
    uint64_t walked = 0;    // entries the count walks: sum over active rows u of sum of |N+(v)|, v in N+(u)
    int64_t m_active = 0;   // oriented edges of the active rows
    std::vector<int64_t> vbase;  // host, G + 1
    pgabb::DArray<int64_t> dvbase;
    pgabb::DArray<int32_t> rptr;      // total_n + 1
    pgabb::DArray<int32_t> col;       // mu, global ids
    pgabb::DArray<int32_t> rows;      // active rows (out-degree >= 2)
    pgabb::DArray<int32_t> row_gid;   // graph of each active row
    pgabb::DArray<int64_t> graph_row_pre;  // G + 1: active rows per graph prefix
    std::vector<int64_t> h_graph_row_pre;
    pgabb::DArray<unsigned long long> counts;  // G, then the work queues' counters
    pgabb::PinnedArray<unsigned long long> hcounts;
    // captured launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int cfg_mode = -1, cfg_waves = 0, cfg_grab = 0, cfg_words = 0;
    double t_build_ms = 0, t_count_ms = 0, t_tune_ms = 0;
    ~pgabb_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

namespace pgabb {

namespace {

constexpr int B = 256;

unsigned cap_grid(int64_t work) {
    unsigned g = grid_for(work, B);
    return g > 65536u ? 65536u : g;
}

// One workgroup per graph: key = g << 2nb | min << nb | max (loops -> sentinel).
__global__ __launch_bounds__(B) void k_batch_keys(const int32_t *__restrict__ src,
                                                  const int32_t *__restrict__ dst,
                                                  const int64_t *__restrict__ eoff,
                                                  const int32_t *__restrict__ nv, int nb,
                                                  uint64_t *__restrict__ keys,
                                                  int32_t *__restrict__ bad) {
    const int64_t g = blockIdx.x;
    const int64_t e0 = eoff[g], e1 = eoff[g + 1];
    const int32_t n = nv[g];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += B) {
        const int32_t a = src[e], b = dst[e];
        uint64_t key = ~0ull;
        if (a < 0 || b < 0 || a >= n || b >= n) {
            *bad = 1;
        } else if (a != b) {
            const uint64_t lo = static_cast<uint32_t>(a < b ? a : b);
            const uint64_t hi = static_cast<uint32_t>(a < b ? b : a);
            key = (static_cast<uint64_t>(g) << (2 * nb)) | (lo << nb) | hi;
        }
        keys[e] = key;
    }
}

__global__ void k_first_of_run_b(const uint64_t *__restrict__ keys, int64_t m, int kbits,
                                 uint32_t *__restrict__ flag) {
    for (int64_t e = blockIdx.x * int64_t(B) + threadIdx.x; e < m; e += int64_t(gridDim.x) * B) {
        const uint64_t k = keys[e];
        flag[e] = (k != ~0ull && (e == 0 || keys[e - 1] != k)) ? 1u : 0u;
    }
    (void)kbits;
}

__global__ void k_compact_b(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ flag,
                            const uint32_t *__restrict__ pos, int64_t m, uint64_t *__restrict__ out) {
    for (int64_t e = blockIdx.x * int64_t(B) + threadIdx.x; e < m; e += int64_t(gridDim.x) * B)
        if (flag[e]) out[pos[e]] = keys[e];
}

// Keys sorted by (g, lo, hi): lo ends form runs (one atomic per run), hi
// ends add one each.
__global__ void k_degrees_b(const uint64_t *__restrict__ keys, int64_t m, int nb,
                            const int64_t *__restrict__ vbase, int32_t *__restrict__ deg) {
    const uint64_t mask = (1ull << nb) - 1;
    const int64_t stride = int64_t(gridDim.x) * B;
    for (int64_t base = blockIdx.x * int64_t(B) + (threadIdx.x & ~63); base < m; base += stride) {
        const int64_t e = base + lane_id();
        const bool valid = e < m;
        const uint64_t k = valid ? keys[e] : 0ull;
        const int64_t vb = valid ? vbase[k >> (2 * nb)] : 0;
        add_run_lengths(valid, vb + static_cast<int64_t>((k >> nb) & mask), deg);
        if (valid) atomicAdd(&deg[vb + (k & mask)], 1);
    }
}

// One workgroup per graph: vertex key = g << 2nb | deg << nb | v.
__global__ __launch_bounds__(B) void k_vertex_keys_b(const int32_t *__restrict__ deg,
                                                     const int64_t *__restrict__ vbase, int nb,
                                                     uint64_t *__restrict__ vkeys) {
    const int64_t g = blockIdx.x;
    const int64_t v0 = vbase[g], v1 = vbase[g + 1];
    for (int64_t x = v0 + threadIdx.x; x < v1; x += B)
        vkeys[x] = (static_cast<uint64_t>(g) << (2 * nb)) | (static_cast<uint64_t>(deg[x]) << nb) |
                   static_cast<uint64_t>(x - v0);
}

__global__ void k_rank_b(const uint64_t *__restrict__ vkeys, int64_t total_n, int nb,
                         const int64_t *__restrict__ vbase, int32_t *__restrict__ rank) {
    const uint64_t mask = (1ull << nb) - 1;
    for (int64_t q = blockIdx.x * int64_t(B) + threadIdx.x; q < total_n; q += int64_t(gridDim.x) * B) {
        const uint64_t k = vkeys[q];
        const int64_t vb = vbase[k >> (2 * nb)];
        rank[vb + (k & mask)] = static_cast<int32_t>(q - vb);
    }
}

__global__ void k_orient_b(const uint64_t *__restrict__ ukeys, int64_t m, int nb,
                           const int64_t *__restrict__ vbase, const int32_t *__restrict__ rank,
                           uint64_t *__restrict__ okeys) {
    const uint64_t mask = (1ull << nb) - 1;
    for (int64_t e = blockIdx.x * int64_t(B) + threadIdx.x; e < m; e += int64_t(gridDim.x) * B) {
        const uint64_t k = ukeys[e];
        const uint64_t g = k >> (2 * nb);
        const int64_t vb = vbase[g];
        const uint32_t ra = static_cast<uint32_t>(rank[vb + ((k >> nb) & mask)]);
        const uint32_t rb = static_cast<uint32_t>(rank[vb + (k & mask)]);
        const uint64_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        okeys[e] = (g << (2 * nb)) | (lo << nb) | hi;
    }
}

__global__ void k_union_csr_b(const uint64_t *__restrict__ okeys, int64_t m, int nb,
                              const int64_t *__restrict__ vbase, int32_t *__restrict__ outdeg,
                              int32_t *__restrict__ col) {
    const uint64_t mask = (1ull << nb) - 1;
    const int64_t stride = int64_t(gridDim.x) * B;
    for (int64_t base = blockIdx.x * int64_t(B) + (threadIdx.x & ~63); base < m; base += stride) {
        const int64_t e = base + lane_id();
        const bool valid = e < m;
        const uint64_t k = valid ? okeys[e] : 0ull;
        const int64_t vb = valid ? vbase[k >> (2 * nb)] : 0;
        add_run_lengths(valid, vb + static_cast<int64_t>((k >> nb) & mask), outdeg);
        if (valid) col[e] = static_cast<int32_t>(vb + (k & mask));
    }
}

__global__ void k_active_flags_b(const uint32_t *__restrict__ outdeg, int64_t n,
                                 uint32_t *__restrict__ flag, int32_t *__restrict__ max_out) {
    int32_t mx = 0;
    for (int64_t x = blockIdx.x * int64_t(B) + threadIdx.x; x < n; x += int64_t(gridDim.x) * B) {
        flag[x] = outdeg[x] >= 2 ? 1u : 0u;
        mx = max(mx, static_cast<int32_t>(outdeg[x]));
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) mx = max(mx, __shfl_xor(mx, d));
    if (lane_id() == 0) atomicMax(max_out, mx);
}

// Active rows and their graphs (one workgroup per graph).
__global__ __launch_bounds__(B) void k_active_rows_b(const uint32_t *__restrict__ flag,
                                                     const uint32_t *__restrict__ pos,
                                                     const int64_t *__restrict__ vbase,
                                                     int32_t *__restrict__ rows,
                                                     int32_t *__restrict__ row_gid) {
    const int64_t g = blockIdx.x;
    for (int64_t x = vbase[g] + threadIdx.x; x < vbase[g + 1]; x += B)
        if (flag[x]) {
            rows[pos[x]] = static_cast<int32_t>(x);
            row_gid[pos[x]] = static_cast<int32_t>(g);
        }
}

// Entries a count walks (for each active row u, the lists N+(v) of its
// out-neighbours v) and the oriented edges of the active rows.
__global__ void k_walked_b(const int32_t *__restrict__ rows, int64_t nactive, const int32_t *__restrict__ rptr,
                           const int32_t *__restrict__ col, unsigned long long *__restrict__ out) {
    unsigned long long w = 0, e = 0;
    for (int64_t q = blockIdx.x * int64_t(B) + threadIdx.x; q < nactive; q += int64_t(gridDim.x) * B) {
        const int32_t u = rows[q];
        for (int32_t t = rptr[u]; t < rptr[u + 1]; ++t) {
            const int32_t v = col[t];
            w += static_cast<unsigned long long>(rptr[v + 1] - rptr[v]);
        }
        e += static_cast<unsigned long long>(rptr[u + 1] - rptr[u]);
    }
    w = wave_sum(w);
    e = wave_sum(e);
    if (lane_id() == 0) {
        if (w) atomicAdd(&out[0], w);
        if (e) atomicAdd(&out[1], e);
    }
}

__global__ void k_graph_row_pre_b(const uint32_t *__restrict__ pos, const int64_t *__restrict__ vbase,
                                  int64_t G, int64_t *__restrict__ pre) {
    for (int64_t g = blockIdx.x * int64_t(B) + threadIdx.x; g <= G; g += int64_t(gridDim.x) * B)
        pre[g] = pos[vbase[g]];
}

// Work queues of a batch launch: the active rows (grouped by graph) are cut
// into kBatchQueues contiguous ranges of equal length, each with its own
// counter; workgroup b starts on range b % kBatchQueues -- its XCD under
// the round-robin dispatch of workgroups to the 8 XCDs -- and moves on to
// the next range once its own is drained.  The waves of one XCD then walk
// the rows of a few graphs at a time, whose lists stay in that XCD's L2;
// with one counter for all, every XCD held rows of every graph in flight.
constexpr int kBatchQueues = 8;
constexpr int kBatchQueueStride = 32;  // counters 256 bytes apart
constexpr int kBatchQueueWords = kBatchQueues * kBatchQueueStride;

struct BatchArgs {
    const int32_t *rptr;
    const int32_t *col;
    const int32_t *rows;
    const int32_t *row_gid;
    const int64_t *vbase;
    int64_t first;  // items [first, last)
    int64_t last;
    int32_t grab;
    int32_t nq;     // work queues (1 or kBatchQueues)
    unsigned long long *counts;
    unsigned long long *next;  // nq counters, kBatchQueueStride apart (zero before launch)
};

template <int MODE, int LDS_WORDS, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_tc_batch(BatchArgs a) {
    __shared__ int32_t lds_all[WAVES][LDS_WORDS];
    __shared__ int32_t own_all[WAVES][2 * kWave];  // the walk's list positions (two chunks in flight)
    const int lane = lane_id();
    int32_t *lds = lds_all[threadIdx.x >> 6];
    int32_t *own = own_all[threadIdx.x >> 6];
    own[lane] = 0;
    own[kWave + lane] = 0;
    wave_lds_sync();
    if (MODE == kModeBitmap) {
        for (int q = lane; q < LDS_WORDS; q += kWave) lds[q] = 0;
        wave_lds_sync();
    }
    const int64_t per = (a.last - a.first + a.nq - 1) / a.nq;
    const int home = static_cast<int>(blockIdx.x % a.nq);
    for (int qi = 0; qi < a.nq; ++qi) {
      const int q = (home + qi) % a.nq;
      const int64_t q0 = a.first + q * per;
      const int64_t q1 = min(q0 + per, a.last);
      for (;;) {
        unsigned long long g0 = 0;
        if (lane == 0) g0 = atomicAdd(&a.next[q * kBatchQueueStride], static_cast<unsigned long long>(a.grab));
        g0 = shfl_t(g0, 0);
        const int64_t i0 = q0 + static_cast<int64_t>(g0);
        if (i0 >= q1) break;
        const int64_t i1 = min(i0 + a.grab, q1);
        const int32_t nrow = static_cast<int32_t>(i1 - i0);  // at most 64
        // the grab's row headers, lane l holding row i0 + l: graph, row,
        // bounds of N+(u), and the graph's vertex range, in two round trips
        int32_t h_gid = 0, h_u = 0, h_sb = 0, h_se = 0, h_vb = 0, h_nv = 0;
        if (lane < nrow) {
            h_gid = a.row_gid[i0 + lane];
            h_u = a.rows[i0 + lane];
        }
        if (lane < nrow) {
            h_sb = a.rptr[h_u];
            h_se = a.rptr[h_u + 1];
            const int64_t vb = a.vbase[h_gid];
            h_vb = static_cast<int32_t>(vb);
            h_nv = static_cast<int32_t>(a.vbase[h_gid + 1] - vb);
        }
        int32_t gcur = __builtin_amdgcn_readfirstlane(h_gid);
        uint32_t cnt = 0;
        // rows of at most kTinyCap entries: walked together, graph by graph
        const bool lv = lane < nrow;
        uint64_t tiny = __ballot(lv && h_se > h_sb && h_se - h_sb <= kTinyCap);
        uint64_t rest = __ballot(lv && h_se - h_sb > kTinyCap);
        while (tiny) {
            const int32_t gid = __builtin_amdgcn_readlane(h_gid, __builtin_ctzll(tiny));
            const uint64_t mg = tiny & __ballot(h_gid == gid);
            tiny &= ~mg;
            if (gid != gcur) {
                const unsigned long long s = wave_sum(static_cast<unsigned long long>(cnt));
                if (lane == 0 && s) atomicAdd(&a.counts[gcur], s);
                cnt = 0;
                gcur = gid;
            }
            cnt += tiny_items<2>(mg, h_sb, h_se, h_sb, h_se, a.col, a.col, a.rptr, a.col, own, lane);
        }
        while (rest) {
            const int l = __builtin_ctzll(rest);
            rest &= rest - 1;
            const int32_t gid = __builtin_amdgcn_readlane(h_gid, l);
            if (gid != gcur) {
                const unsigned long long s = wave_sum(static_cast<unsigned long long>(cnt));
                if (lane == 0 && s) atomicAdd(&a.counts[gcur], s);
                cnt = 0;
                gcur = gid;
            }
            const int32_t sb = __builtin_amdgcn_readlane(h_sb, l), se = __builtin_amdgcn_readlane(h_se, l);
            cnt += tc_item_core<MODE, LDS_WORDS>(a.col, sb, se, a.rptr, a.col, a.col, sb, se,
                                                 __builtin_amdgcn_readlane(h_nv, l), lds, own,
                                                 __builtin_amdgcn_readlane(h_vb, l));
        }
        const unsigned long long s = wave_sum(static_cast<unsigned long long>(cnt));
        if (lane == 0 && s) atomicAdd(&a.counts[gcur], s);
      }
    }
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(B) + threadIdx.x; i < n; i += int64_t(gridDim.x) * B) p[i] = 0;
}

template <int MODE, int LDS_WORDS, int WAVES>
void launch_batch_one(const BatchArgs &a, hipStream_t s) {
    auto kern = k_tc_batch<MODE, LDS_WORDS, WAVES>;
    int per_cu = 0;
    PGABB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WAVES * 64, 0));
    if (per_cu < 1) per_cu = 1;
    int dev = 0, cus = 0;
    PGABB_HIP(hipGetDevice(&dev));
    PGABB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t grid = static_cast<int64_t>(cus) * per_cu;
    const int64_t items = a.last - a.first;
    const int64_t blocks_needed = ((items + a.grab - 1) / a.grab + WAVES - 1) / WAVES;
    grid = std::max<int64_t>(1, std::min(grid, blocks_needed));
    kern<<<static_cast<unsigned>(grid), WAVES * 64, 0, s>>>(a);
    PGABB_HIP(hipGetLastError());
}

template <int MODE, int WAVES>
void launch_batch_words(const BatchArgs &a, int words, hipStream_t s) {
    if (words <= 320) launch_batch_one<MODE, 320, WAVES>(a, s);
    else if (words <= 640) launch_batch_one<MODE, 640, WAVES>(a, s);
    else if (words <= 1280) launch_batch_one<MODE, 1280, WAVES>(a, s);
    else launch_batch_one<MODE, 2304, WAVES>(a, s);
}

void launch_batch(const BatchArgs &a, int mode, int words, int waves, hipStream_t s) {
    if (a.last <= a.first) return;
    if (mode == kModeBitmap) {
        if (waves == 2) launch_batch_words<kModeBitmap, 2>(a, words, s);
        else if (waves == 8) launch_batch_words<kModeBitmap, 8>(a, words, s);
        else launch_batch_words<kModeBitmap, 4>(a, words, s);
    } else {
        if (waves == 2) launch_batch_words<kModeHash, 2>(a, words, s);
        else if (waves == 8) launch_batch_words<kModeHash, 8>(a, words, s);
        else launch_batch_words<kModeHash, 4>(a, words, s);
    }
}

int words_for(int mode, const pgabb_batch *b) {
    static const int kClass[] = {320, 640, 1280, 2304};
    static const int kTable[] = {256, 512, 1024, 2048};
    if (mode == kModeBitmap) {
        const int64_t w = (static_cast<int64_t>(b->max_n) + 31) / 32;
        for (int c = 0; c < 4; ++c)
            if (w <= kClass[c]) return kClass[c];
        return kClass[3];
    }
    const int64_t need = (3 * static_cast<int64_t>(b->max_out) + 1) / 2;
    for (int c = 0; c < 4; ++c)
        if (need <= kTable[c]) return kClass[c];
    return kClass[3];
}

BatchArgs batch_args(pgabb_batch *b, int grab) {
    BatchArgs a;
    a.rptr = b->rptr.get();
    a.col = b->col.get();
    a.rows = b->rows.get();
    a.row_gid = b->row_gid.get();
    a.vbase = b->dvbase.get();
    a.first = 0;
    a.last = b->nactive;
    a.grab = grab;
    a.nq = kBatchQueues;
    a.counts = b->counts.get();
    a.next = b->counts.get() + b->G;
    return a;
}

// Everything one count does, on one stream (capturable: no memset nodes).
void enqueue_count(pgabb_batch *b, int mode, int waves, int grab, hipStream_t s) {
    k_zero_u64<<<cap_grid(b->G + kBatchQueueWords), B, 0, s>>>(b->counts.get(), b->G + kBatchQueueWords);
    PGABB_HIP(hipGetLastError());
    launch_batch(batch_args(b, grab), mode, words_for(mode, b), waves, s);
    PGABB_HIP(hipMemcpyAsync(b->hcounts.get(), b->counts.get(), sizeof(unsigned long long) * b->G,
                             hipMemcpyDeviceToHost, s));
}

struct TuneVal {
    int mode, waves, grab;
};

// Shape class of a batch: bit widths of its graph count, largest graph,
// edges and longest oriented row.
std::string tune_key(const pgabb_batch *b) {
    char key[96];
    snprintf(key, sizeof key, "batch/G%d/N%d/M%d/D%d", bit_width_u64(static_cast<uint64_t>(b->G)),
             bit_width_u64(static_cast<uint64_t>(b->max_n)), bit_width_u64(static_cast<uint64_t>(b->mu)),
             bit_width_u64(static_cast<uint64_t>(b->max_out)));
    return key;
}

// The launch shape for this batch: from the persisted tuning cache, else the
// fastest of the candidates timed on the batch itself (then stored).
TuneVal autotune(pgabb_batch *b) {
    const std::string key = tune_key(b);
    {
        std::vector<int> v;
        if (tune_lookup(key, v) && v.size() == 3) return TuneVal{v[0], v[1], v[2]};
    }
    hipStream_t s = b->stream;
    StreamTimer tm;
    // fastest of `reps` timed runs after one warm run
    auto time_cfg = [&](const TuneVal &v, int reps) {
        enqueue_count(b, v.mode, v.waves, v.grab, s);
        double best_ms = 1e30;
        for (int rep = 0; rep < reps; ++rep) {
            tm.start(s);
            enqueue_count(b, v.mode, v.waves, v.grab, s);
            tm.stop(s);
            best_ms = std::min(best_ms, tm.ms());
        }
        return best_ms;
    };
    std::vector<std::pair<double, TuneVal>> timed;
    const int modes[] = {kModeBitmap, kModeHash};
    const int wavess[] = {2, 4, 8};
    const int grabs[] = {8, 16, 32};
    for (int mode : modes) {
        if (mode == kModeBitmap && (static_cast<int64_t>(b->max_n) + 31) / 32 > 2304) continue;
        for (int waves : wavess)
            for (int grab : grabs) {
                const TuneVal v{mode, waves, grab};
                timed.emplace_back(time_cfg(v, 2), v);
            }
    }
    // the leaders are often within a few per cent: time them again
    std::sort(timed.begin(), timed.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    TuneVal best = timed.front().second;
    double best_ms = 1e30;
    for (size_t q = 0; q < std::min<size_t>(3, timed.size()); ++q) {
        const double ms = std::min(timed[q].first, time_cfg(timed[q].second, 3));
        if (ms < best_ms) {
            best_ms = ms;
            best = timed[q].second;
        }
    }
    tune_store(key, {best.mode, best.waves, best.grab});
    return best;
}

void capture(pgabb_batch *b, int mode, int waves, int grab) {
    if (b->exec && b->cfg_mode == mode && b->cfg_waves == waves && b->cfg_grab == grab) return;
    if (b->exec) {
        PGABB_HIP(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
    }
    if (b->graph) {
        PGABB_HIP(hipGraphDestroy(b->graph));
        b->graph = nullptr;
    }
    hipStream_t s = b->stream;
    PGABB_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_count(b, mode, waves, grab, s);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(s, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    PGABB_HIP(hipStreamEndCapture(s, &b->graph));
    PGABB_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->cfg_mode = mode;
    b->cfg_waves = waves;
    b->cfg_grab = grab;
}

}  // namespace

void batch_build(pgabb_batch *b, const int32_t *n, const int64_t *eoff, const int32_t *src,
                 const int32_t *dst, bool on_device) {
    hipStream_t s = b->stream;
    const int64_t G = b->G;
    b->vbase.assign(G + 1, 0);
    int32_t max_n = 0;
    for (int64_t g = 0; g < G; ++g) {
        b->vbase[g + 1] = b->vbase[g] + n[g];
        max_n = std::max(max_n, n[g]);
    }
    b->max_n = max_n;
    b->total_n = b->vbase[G];
    b->total_m = G ? eoff[G] : 0;
    b->nb = std::max(1, bit_width_u64(max_n > 0 ? static_cast<uint64_t>(max_n - 1) : 0));
    b->gbits = std::max(1, bit_width_u64(static_cast<uint64_t>(G > 0 ? G - 1 : 0)));
    const int nb = b->nb;
    const int kbits = b->gbits + 2 * nb;
    PGABB_REQUIRE(kbits <= 63, PGABB_EINVAL, "batch too large to pack: %d key bits", kbits);
    PGABB_REQUIRE(b->total_n < (int64_t(1) << 31), PGABB_EINVAL, "batch holds 2^31 or more vertices");
    const int64_t m = b->total_m;

    b->dvbase.reset(G + 1, s);
    PGABB_HIP(hipMemcpyAsync(b->dvbase.get(), b->vbase.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
    b->counts.reset(G + kBatchQueueWords, s);
    b->hcounts.reset(static_cast<size_t>(std::max<int64_t>(G, 1)));
    b->rptr.reset(b->total_n + 1, s);

    DArray<int32_t> dn(G, s);
    DArray<int64_t> deoff(G + 1, s);
    if (G) {
        PGABB_HIP(hipMemcpyAsync(dn.get(), n, sizeof(int32_t) * G, hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(deoff.get(), eoff, sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
    }
    DArray<int32_t> hs, hd;
    if (m > 0 && !on_device) {
        hs.reset(m, s);
        hd.reset(m, s);
        PGABB_HIP(hipMemcpyAsync(hs.get(), src, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(hd.get(), dst, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
        src = hs.get();
        dst = hd.get();
    }

    DArray<uint32_t> outdeg(b->total_n, s);
    if (b->total_n) PGABB_HIP(hipMemsetAsync(outdeg.get(), 0, sizeof(uint32_t) * b->total_n, s));
    b->mu = 0;
    if (m > 0) {
        DArray<uint64_t> keys(m, s), alt(m, s);
        DArray<int32_t> bad(1, s);
        PGABB_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int32_t), s));
        k_batch_keys<<<static_cast<unsigned>(G), B, 0, s>>>(src, dst, deoff.get(), dn.get(), nb, keys.get(), bad.get());
        PGABB_HIP(hipGetLastError());
        int32_t bad_h = 0;
        PGABB_HIP(hipMemcpyAsync(&bad_h, bad.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        PGABB_REQUIRE(!bad_h, PGABB_EINVAL, "an edge endpoint lies outside its graph's [0, n)");
        uint64_t *k0 = keys.get(), *k1 = alt.get();
        // sentinels (~0) have every bit set, so a sort on kbits bits keeps them last
        if (radix_sort_u64_bits(k0, k1, nullptr, nullptr, m, 0, kbits, s)) std::swap(k0, k1);
        {
            DArray<uint32_t> flag(m, s), pos(m, s), total(1, s);
            k_first_of_run_b<<<cap_grid(m), B, 0, s>>>(k0, m, kbits, flag.get());
            scan_exclusive_u32(flag.get(), pos.get(), m, total.get(), s);
            k_compact_b<<<cap_grid(m), B, 0, s>>>(k0, flag.get(), pos.get(), m, k1);
            PGABB_HIP(hipGetLastError());
            uint32_t mu = 0;
            PGABB_HIP(hipMemcpyAsync(&mu, total.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            PGABB_HIP(hipStreamSynchronize(s));
            b->mu = mu;
        }
        std::swap(k0, k1);
        const int64_t mu = b->mu;
        PGABB_REQUIRE(mu < (int64_t(1) << 31), PGABB_EINVAL, "batch holds 2^31 or more edges");
        if (mu > 0) {
            DArray<int32_t> deg(b->total_n, s), rank(b->total_n, s);
            PGABB_HIP(hipMemsetAsync(deg.get(), 0, sizeof(int32_t) * b->total_n, s));
            k_degrees_b<<<cap_grid(mu), B, 0, s>>>(k0, mu, nb, b->dvbase.get(), deg.get());
            DArray<uint64_t> vk(b->total_n, s), vka(b->total_n, s);
            k_vertex_keys_b<<<static_cast<unsigned>(G), B, 0, s>>>(deg.get(), b->dvbase.get(), nb, vk.get());
            PGABB_HIP(hipGetLastError());
            uint64_t *vs = vk.get();
            if (radix_sort_u64_bits(vk.get(), vka.get(), nullptr, nullptr, b->total_n, 0, kbits, s)) vs = vka.get();
            k_rank_b<<<cap_grid(b->total_n), B, 0, s>>>(vs, b->total_n, nb, b->dvbase.get(), rank.get());
            k_orient_b<<<cap_grid(mu), B, 0, s>>>(k0, mu, nb, b->dvbase.get(), rank.get(), k1);
            PGABB_HIP(hipGetLastError());
            if (radix_sort_u64_bits(k1, k0, nullptr, nullptr, mu, 0, kbits, s)) std::swap(k0, k1);
            b->col.reset(mu, s);
            k_union_csr_b<<<cap_grid(mu), B, 0, s>>>(k1, mu, nb, b->dvbase.get(),
                                                     reinterpret_cast<int32_t *>(outdeg.get()), b->col.get());
            PGABB_HIP(hipGetLastError());
        }
    }
    // union row offsets (int32: m' < 2^31)
    if (b->total_n) {
        scan_exclusive_u32(outdeg.get(), reinterpret_cast<uint32_t *>(b->rptr.get()), b->total_n,
                           reinterpret_cast<uint32_t *>(b->rptr.get()) + b->total_n, s);
    } else {
        PGABB_HIP(hipMemsetAsync(b->rptr.get(), 0, sizeof(int32_t), s));
    }
    // active rows (out-degree >= 2) grouped by graph
    {
        DArray<uint32_t> flag(b->total_n + 1, s), pos(b->total_n + 1, s), total(1, s);
        DArray<int32_t> mx(1, s);
        PGABB_HIP(hipMemsetAsync(mx.get(), 0, sizeof(int32_t), s));
        PGABB_HIP(hipMemsetAsync(flag.get(), 0, sizeof(uint32_t) * (b->total_n + 1), s));
        if (b->total_n) k_active_flags_b<<<cap_grid(b->total_n), B, 0, s>>>(outdeg.get(), b->total_n, flag.get(), mx.get());
        scan_exclusive_u32(flag.get(), pos.get(), b->total_n + 1, total.get(), s);
        uint32_t na = 0;
        PGABB_HIP(hipMemcpyAsync(&na, total.get(), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipMemcpyAsync(&b->max_out, mx.get(), sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        b->nactive = na;
        b->rows.reset(std::max<int64_t>(na, 1), s);
        b->row_gid.reset(std::max<int64_t>(na, 1), s);
        b->graph_row_pre.reset(G + 1, s);
        if (G) {
            k_active_rows_b<<<static_cast<unsigned>(G), B, 0, s>>>(flag.get(), pos.get(), b->dvbase.get(), b->rows.get(),
                                                                   b->row_gid.get());
            k_graph_row_pre_b<<<cap_grid(G + 1), B, 0, s>>>(pos.get(), b->dvbase.get(), G, b->graph_row_pre.get());
            PGABB_HIP(hipGetLastError());
        }
        b->h_graph_row_pre.assign(G + 1, 0);
        if (G)
            PGABB_HIP(hipMemcpyAsync(b->h_graph_row_pre.data(), b->graph_row_pre.get(), sizeof(int64_t) * (G + 1),
                                     hipMemcpyDeviceToHost, s));
        DArray<unsigned long long> wk(2, s);
        k_zero_u64<<<1, B, 0, s>>>(wk.get(), 2);
        if (na) k_walked_b<<<cap_grid(na), B, 0, s>>>(b->rows.get(), na, b->rptr.get(), b->col.get(), wk.get());
        PGABB_HIP(hipGetLastError());
        unsigned long long hw[2] = {0, 0};
        PGABB_HIP(hipMemcpyAsync(hw, wk.get(), sizeof hw, hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        b->walked = hw[0];
        b->m_active = static_cast<int64_t>(hw[1]);
    }
}

// Count all graphs: autotuned + captured (opts NULL) or as given.
void batch_count(pgabb_batch *b, const pgabb_tc_options *opts, uint64_t *out) {
    hipStream_t s = b->stream;
    if (b->G == 0) return;
    StreamTimer tm;
    const bool per_graph = opts && (opts->flags & PGABB_OPT_PER_GRAPH);
    if (per_graph) {
        // plain per-graph launches, one after another on one stream
        const int mode = kModeHash;
        const int waves = 4, grab = 8;
        tm.start(s);
        k_zero_u64<<<cap_grid(b->G + kBatchQueueWords), B, 0, s>>>(b->counts.get(), b->G + kBatchQueueWords);
        DArray<unsigned long long> ctr(b->G, s);
        k_zero_u64<<<cap_grid(b->G), B, 0, s>>>(ctr.get(), b->G);
        for (int64_t g = 0; g < b->G; ++g) {
            BatchArgs a = batch_args(b, grab);
            a.first = b->h_graph_row_pre[g];
            a.last = b->h_graph_row_pre[g + 1];
            a.next = ctr.get() + g;
            a.nq = 1;
            launch_batch(a, mode, words_for(mode, b), waves, s);
        }
        PGABB_HIP(hipMemcpyAsync(b->hcounts.get(), b->counts.get(), sizeof(unsigned long long) * b->G,
                                 hipMemcpyDeviceToHost, s));
        tm.stop(s);
        b->t_count_ms = tm.ms();
    } else {
        int mode, waves, grab;
        if (opts) {
            mode = (opts->kernel == PGABB_KERNEL_HASH || opts->kernel == PGABB_KERNEL_SEARCH) ? kModeHash : kModeBitmap;
            if (mode == kModeBitmap && (static_cast<int64_t>(b->max_n) + 31) / 32 > 2304) mode = kModeHash;
            waves = opts->waves_per_block > 0 ? opts->waves_per_block : 4;
            grab = opts->rows_per_grab > 0 ? opts->rows_per_grab : 4;
        } else {
            const auto t0 = std::chrono::steady_clock::now();
            const TuneVal tv = autotune(b);
            b->t_tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            mode = tv.mode;
            waves = tv.waves;
            grab = tv.grab;
        }
        capture(b, mode, waves, grab);
        tm.start(s);
        PGABB_HIP(hipGraphLaunch(b->exec, s));
        tm.stop(s);
        b->t_count_ms = tm.ms();
    }
    PGABB_HIP(hipStreamSynchronize(s));
    for (int64_t g = 0; g < b->G; ++g) out[g] = b->hcounts[g];
}

}  // namespace pgabb

using namespace pgabb;

#define PGABB_API extern "C" __attribute__((visibility("default")))

namespace pgabb {
pgabb_status capture_status(const Error &e);
hipStream_t library_stream();
}

PGABB_API pgabb_status pgabb_batch_create(int64_t num_graphs, const int32_t *n, const int64_t *edge_off,
                                          const int32_t *src, const int32_t *dst, uint32_t flags,
                                          void *hip_stream, pgabb_batch **out) {
    if (!out) return capture_status(Error{PGABB_EINVAL, "out is NULL"});
    *out = nullptr;
    if (num_graphs < 0) return capture_status(Error{PGABB_EINVAL, "num_graphs < 0"});
    if (num_graphs > 0 && (!n || !edge_off)) return capture_status(Error{PGABB_EINVAL, "n or edge_off is NULL"});
    if (flags & ~PGABB_EDGES_ON_DEVICE) return capture_status(Error{PGABB_EINVAL, "unknown flag bits"});
    if (num_graphs > 0) {
        if (edge_off[0] != 0) return capture_status(Error{PGABB_EINVAL, "edge_off[0] must be 0"});
        for (int64_t g = 0; g < num_graphs; ++g) {
            if (n[g] < 0) return capture_status(Error{PGABB_EINVAL, "a graph has n < 0"});
            if (edge_off[g + 1] < edge_off[g]) return capture_status(Error{PGABB_EINVAL, "edge_off decreases"});
        }
        if (edge_off[num_graphs] > 0 && (!src || !dst)) return capture_status(Error{PGABB_EINVAL, "src or dst is NULL"});
        if (edge_off[num_graphs] >= (int64_t(1) << 32))
            return capture_status(Error{PGABB_EINVAL, "more than 2^32 - 1 pairs"});
    }
    pgabb_batch *b = nullptr;
    try {
        b = new pgabb_batch();
        b->G = num_graphs;
        b->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : library_stream();
        StreamTimer tm;
        tm.start(b->stream);
        batch_build(b, n, edge_off, src, dst, flags & PGABB_EDGES_ON_DEVICE);
        tm.stop(b->stream);
        b->t_build_ms = tm.ms();
        *out = b;
        return capture_status(Error{PGABB_OK, ""});
    } catch (const Error &e) {
        delete b;
        return capture_status(e);
    } catch (...) {
        delete b;
        return capture_status(Error{PGABB_EDEVICE, "unexpected internal error"});
    }
}

PGABB_API pgabb_status pgabb_batch_count(pgabb_batch *b, const pgabb_tc_options *opts, uint64_t *counts) {
    if (!b || (!counts && b->G > 0)) return capture_status(Error{PGABB_EINVAL, "NULL argument"});
    if (opts && (opts->waves_per_block < 0 || opts->rows_per_grab < 0 ||
                 (opts->waves_per_block && opts->waves_per_block != 2 && opts->waves_per_block != 4 &&
                  opts->waves_per_block != 8)))
        return capture_status(Error{PGABB_EINVAL, "bad launch shape"});
    try {
        batch_count(b, opts, counts);
        return capture_status(Error{PGABB_OK, ""});
    } catch (const Error &e) {
        return capture_status(e);
    } catch (...) {
        return capture_status(Error{PGABB_EDEVICE, "unexpected internal error"});
    }
}

PGABB_API pgabb_status pgabb_batch_times(const pgabb_batch *b, double *t_build_ms, double *t_count_ms) {
    if (!b) return capture_status(Error{PGABB_EINVAL, "batch is NULL"});
    if (t_build_ms) *t_build_ms = b->t_build_ms;
    if (t_count_ms) *t_count_ms = b->t_count_ms;
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API pgabb_status pgabb_batch_stats(const pgabb_batch *b, int64_t *edges, int64_t *active_rows,
                                         int64_t *active_edges, uint64_t *walked) {
    if (!b) return capture_status(Error{PGABB_EINVAL, "batch is NULL"});
    if (edges) *edges = b->mu;
    if (active_rows) *active_rows = b->nactive;
    if (active_edges) *active_edges = b->m_active;
    if (walked) *walked = b->walked;
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API pgabb_status pgabb_batch_launch_shape(const pgabb_batch *b, int32_t *kernel, int32_t *waves_per_block,
                                                int32_t *rows_per_grab, double *t_tune_ms) {
    if (!b) return capture_status(Error{PGABB_EINVAL, "batch is NULL"});
    if (kernel) *kernel = b->cfg_mode < 0 ? -1 : (b->cfg_mode == kModeBitmap ? PGABB_KERNEL_BITMAP : PGABB_KERNEL_HASH);
    if (waves_per_block) *waves_per_block = b->cfg_waves;
    if (rows_per_grab) *rows_per_grab = b->cfg_grab;
    if (t_tune_ms) *t_tune_ms = b->t_tune_ms;
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API void pgabb_batch_destroy(pgabb_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    delete b;
}
