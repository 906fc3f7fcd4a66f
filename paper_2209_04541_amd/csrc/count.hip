// Count phase: run every task (block-list) of a partitioned graph.
//
// In-core path: all blocks live in one device arena.  One persistent launch
// covers every task: the work items are the rows of each task's A_ij, laid
// out task after task in the heaviest-first order of the task table, and
// each wave repeatedly grabs a few consecutive items from a global counter
// (dynamic load balance over skewed rows, PGAbB Section 4.4's "heavy tasks
// first").  A wave accumulates its hits in registers and adds them to the
// task's uint64 counter when it leaves a task.
//
// Streamed path (graph blocks held in pinned host memory): see streamer.hip.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <queue>
#include <vector>

#include "common.hpp"
#include "count.hpp"
#include "graph.hpp"
#include "tc_device.hpp"
#include "tc_kernel.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

template <int MODE, int LDS_WORDS, int WAVES, int UNROLL, bool FILTER = false>
void launch_one(const CountArgs &a, hipStream_t s, int grid_override) {
    auto kern = a.orient == kOrientCol ? k_tc_tasks<MODE, LDS_WORDS, WAVES, UNROLL, kOrientCol, FILTER>
                                       : k_tc_tasks<MODE, LDS_WORDS, WAVES, UNROLL, kOrientRow, FILTER>;
    int per_cu = 0;
    PGABB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, WAVES * 64, 0));
    if (per_cu < 1) per_cu = 1;
    int dev = 0, cus = 0;
    PGABB_HIP(hipGetDevice(&dev));
    PGABB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int64_t grid = static_cast<int64_t>(cus) * per_cu;
    if (grid_override > 0) grid = grid_override;
    const int64_t units = (a.total + a.grab - 1) / a.grab;
    const int64_t blocks_needed = (units + WAVES - 1) / WAVES;
    if (grid > blocks_needed) grid = blocks_needed;
    if (grid < 1) grid = 1;
    kern<<<static_cast<unsigned>(grid), WAVES * 64, 0, s>>>(a);
    PGABB_HIP(hipGetLastError());
}

// LDS words per wave come in five classes; a hash-mode class holds a table of
// 256 .. 4096 words plus a filter (see HashLds).
template <int MODE, int WAVES, int UNROLL>
void launch_words(const CountArgs &a, int lds_words, hipStream_t s, int grid_override) {
    if (lds_words <= 320) launch_one<MODE, 320, WAVES, UNROLL>(a, s, grid_override);
    else if (lds_words <= 640) launch_one<MODE, 640, WAVES, UNROLL>(a, s, grid_override);
    else if (lds_words <= 1280) launch_one<MODE, 1280, WAVES, UNROLL>(a, s, grid_override);
    else if (lds_words <= 2304) launch_one<MODE, 2304, WAVES, UNROLL>(a, s, grid_override);
    else launch_one<MODE, 4352, WAVES, UNROLL>(a, s, grid_override);
}

template <int UNROLL>
void launch_mode(const CountArgs &a, int mode, int lds_words, int waves, hipStream_t s, int grid_override) {
    if (waves == 2) {
        if (mode == kModeBitmap) launch_words<kModeBitmap, 2, UNROLL>(a, lds_words, s, grid_override);
        else if (mode == kModeSearch) launch_one<kModeSearch, 320, 2, UNROLL>(a, s, grid_override);
        else launch_words<kModeHash, 2, UNROLL>(a, lds_words, s, grid_override);
    } else if (waves == 8) {
        if (mode == kModeBitmap) launch_words<kModeBitmap, 8, UNROLL>(a, lds_words, s, grid_override);
        else if (mode == kModeSearch) launch_one<kModeSearch, 320, 8, UNROLL>(a, s, grid_override);
        else launch_words<kModeHash, 8, UNROLL>(a, lds_words, s, grid_override);
    } else {
        if (mode == kModeBitmap) launch_words<kModeBitmap, 4, UNROLL>(a, lds_words, s, grid_override);
        else if (mode == kModeSearch) launch_one<kModeSearch, 320, 4, UNROLL>(a, s, grid_override);
        else launch_words<kModeHash, 4, UNROLL>(a, lds_words, s, grid_override);
    }
}

}  // namespace

// The hash class that keeps eight waves per SIMD.
constexpr int kSmallWords = 1280;

int choose_lds_words(int32_t mode, int32_t max_stage_len, int32_t max_width_k) {
    static const int kClass[] = {320, 640, 1280, 2304, 4352};
    static const int kTable[] = {256, 512, 1024, 2048, 4096};
    if (mode == kModeBitmap) {
        const int64_t w = (static_cast<int64_t>(max_width_k) + 31) / 32;
        for (int c = 0; c < 5; ++c)
            if (w <= kClass[c]) return kClass[c];
        return kClass[4];
    }
    if (mode == kModeHash) {
        // table of at least 1.5 x the longest staged row (load <= 2/3); at
        // least 1280 words, the most that still keeps eight waves per SIMD
        // (32 waves x 1280 words = 160 KB of LDS per CU)
        const int64_t need = (3 * static_cast<int64_t>(max_stage_len) + 1) / 2;
        for (int c = 0; c < 5; ++c)
            if (need <= kTable[c]) return std::max(kClass[c], 1280);
        return kClass[4];  // longer rows fall back to in-place search
    }
    return 320;
}

namespace {

// A launch of a split pair: the default shape (four waves, two chunks per
// batch), items filtered by staged list length.
void launch_filtered(const CountArgs &a, int mode, int lds_words, hipStream_t s, int grid_override) {
    if (mode == kModeBitmap) {
        if (lds_words <= 1280) launch_one<kModeBitmap, 1280, 4, 2, true>(a, s, grid_override);
        else if (lds_words <= 2304) launch_one<kModeBitmap, 2304, 4, 2, true>(a, s, grid_override);
        else launch_one<kModeBitmap, 4352, 4, 2, true>(a, s, grid_override);
    } else {
        if (lds_words <= 1280) launch_one<kModeHash, 1280, 4, 2, true>(a, s, grid_override);
        else if (lds_words <= 2304) launch_one<kModeHash, 2304, 4, 2, true>(a, s, grid_override);
        else launch_one<kModeHash, 4352, 4, 2, true>(a, s, grid_override);
    }
}

void launch_one(const CountArgs &a, int mode, int lds_words, int waves, hipStream_t s, int grid_override,
                int unroll) {
    // default 2: with the next batch loading while one is probed, two chunks
    // per batch keep four loads in flight per wave within 64 VGPRs (eight
    // waves per SIMD)
    switch (unroll) {
        case 1: launch_mode<1>(a, mode, lds_words, waves, s, grid_override); break;
        case 4: launch_mode<4>(a, mode, lds_words, waves, s, grid_override); break;
        case 8: launch_mode<8>(a, mode, lds_words, waves, s, grid_override); break;
        default: launch_mode<2>(a, mode, lds_words, waves, s, grid_override); break;
    }
}


}  // namespace

void launch_tc_tasks(const CountArgs &args, const LaunchKind &lk, int waves, hipStream_t s, int grid_override,
                     int unroll) {
    if (args.total <= 0) return;
    CountArgs a = args;
    a.grab = std::max(1, std::min(a.grab, kWave));  // a grab's items fit one wave's lanes
    if (lk.nparts == 1) {
        launch_one(a, lk.mode, lk.words, waves, s, grid_override, unroll);
        return;
    }
    // the parts of a split launch run at the default shape (waves and unroll
    // options apply to single launches)
    unsigned long long *const next0 = a.next;
    for (int q = 0; q < lk.nparts; ++q) {
        a.next = next0 + static_cast<size_t>(q) * kQueueWords;  // counters of their own, cleared before
        a.stage_lo = q == 0 ? 0 : lk.hi[q - 1];
        a.stage_hi = lk.hi[q];
        launch_filtered(a, lk.pmode[q], lk.pwords[q], s, grid_override);
    }
}

int default_grab(int64_t total_items, uint64_t walked) {
    // A grab should carry about 16K walked entries: light items are taken
    // many at a time, so a grab's two header round trips are shared by more
    // of them; heavy ones a few at a time, so the last grabs do not leave
    // waves idle.  (Measured on R-MAT and random geometric graphs at p = 1,
    // 8 and 32, the best grab was 16K walked entries over the mean per item,
    // within a few per cent.)  At most items / 32768, so a small launch
    // still hands about four grabs to each of the chip's 8192 wave slots; at
    // least enough for ~32K counter updates per queue: device-scope atomics
    // on one address serialise.
    // walked == 0 (work unknown): the count bound alone
    if (total_items <= 0) return 2;
    const int64_t by_atomics = (total_items + int64_t(kQueues) * 32768 - 1) / (int64_t(kQueues) * 32768);
    int64_t g = by_atomics;
    if (walked > 0) {
        const double per_item = static_cast<double>(walked) / static_cast<double>(total_items);
        const int64_t by_work = static_cast<int64_t>(16384.0 / per_item + 0.5);
        const int64_t by_spread = total_items / 32768;
        g = std::max<int64_t>(std::min<int64_t>(by_work, by_spread), by_atomics);
    }
    return static_cast<int>(std::max<int64_t>(2, std::min<int64_t>(g, 64)));
}

uint64_t walked_entries(const pgabb_graph *g, int orient) {
    return orient == kOrientCol ? g->probe_work_col : g->probe_work;
}

LaunchKind launch_kind(int32_t kernel, int32_t max_out, int32_t max_wk, int32_t min_wk) {
    LaunchKind lk;
    switch (kernel) {
        case PGABB_KERNEL_BITMAP:
            lk.mode = kModeBitmap;
            lk.words = choose_lds_words(kModeBitmap, max_out, max_wk);
            return lk;
        case PGABB_KERNEL_SEARCH:
            lk.mode = kModeSearch;
            lk.words = 320;
            return lk;
        default: break;
    }
    // Hash staging, LDS sized for tables of the longest staged list.  With
    // the automatic kernel, where a stripe's bitmap fits in that region
    // (narrow stripes: the high-degree end under nnz-balanced cuts), items
    // stage a bitmap and probe it with one read; elsewhere they hash.
    auto kind = [&](int32_t longest, int &mode, int &words) {
        words = choose_lds_words(kModeHash, longest, max_wk);
        const bool some_fit = (static_cast<int64_t>(min_wk) + 31) / 32 <= words;
        mode = (kernel != PGABB_KERNEL_HASH && some_fit) ? kModeBitmap : kModeHash;
    };
    kind(max_out, lk.mode, lk.words);
    if (lk.words > kSmallWords) {
        // one part per class from 1280 words up: lists up to a class's table
        // capacity (load <= 2/3) run with that class's region
        static const int32_t kCap[3] = {1024 * 2 / 3, 2048 * 2 / 3, INT32_MAX};
        lk.nparts = 0;
        for (int q = 0; q < 3; ++q) {
            const int32_t longest = std::min(max_out, kCap[q]);
            kind(longest, lk.pmode[q], lk.pwords[q]);
            lk.hi[q] = kCap[q];
            ++lk.nparts;
            if (max_out <= kCap[q]) break;
        }
        lk.hi[lk.nparts - 1] = INT32_MAX;
        lk.mode = lk.pmode[0];
        lk.words = lk.pwords[0];
    }
    return lk;
}

TaskDesc make_desc(const pgabb_graph *g, const int32_t *arena_base, const Task &t, int32_t slot,
                   const int64_t *chunk_dev_off) {
    auto ref = [&](int32_t b) {
        const BlockInfo &bi = g->blocks[b];
        const int32_t *c = arena_base + (chunk_dev_off ? chunk_dev_off[b] : bi.chunk_off);
        BlockRef r;
        r.rptr = c + (bi.off_rptr() - bi.chunk_off);
        r.items = c + (bi.off_items() - bi.chunk_off);
        r.col = c + (bi.off_col() - bi.chunk_off);
        r.citems = c + (bi.off_citems() - bi.chunk_off);
        r.crow = c + (bi.off_crow() - bi.chunk_off);
        r.nitems = bi.nitems;
        r.ncitems = bi.ncitems;
        return r;
    };
    TaskDesc d;
    d.ij = ref(t.bij);
    d.ik = ref(t.bik);
    d.jk = ref(t.bjk);
    d.width_k = g->cuts[t.k + 1] - g->base[t.k];
    d.slot = slot;
    return d;
}

int orient_of_option(const pgabb_tc_options &opt, const pgabb_graph *g) {
    if (opt.flags & PGABB_OPT_ROWS) return kOrientRow;
    if (opt.flags & PGABB_OPT_COLS) return kOrientCol;
    // the walk that reads fewer entries of the probed lists
    if (g && g->probe_work < g->probe_work_col) return kOrientRow;
    return kOrientCol;
}

int32_t staged_max(const pgabb_graph *g, const Task &t, int orient) {
    return g->blocks[orient == kOrientCol ? t.bjk : t.bik].max_row;
}

int64_t task_items(const pgabb_graph *g, const Task &t, int orient) {
    const BlockInfo &b = g->blocks[t.bij];
    return orient == kOrientCol ? b.ncitems : b.nitems;
}

static uint64_t count_in_core(pgabb_graph *g, const pgabb_tc_options &opt) {
    hipStream_t s = g->stream;
    const int orient = orient_of_option(opt, g);
    g->walked_columns = orient == kOrientCol;
    const int32_t T = static_cast<int32_t>(g->tasks.size());
    Staged<TaskDesc> td(T, s);
    Staged<int64_t> pre(static_cast<size_t>(T) + 1, s);
    pre[0] = 0;
    int32_t max_wk = 0, min_wk = INT32_MAX, max_st = 0;
    for (int32_t t = 0; t < T; ++t) {
        td[t] = make_desc(g, g->arena.get(), g->tasks[t], t, nullptr);
        pre[t + 1] = pre[t] + task_items(g, g->tasks[t], orient);
        max_wk = std::max(max_wk, td[t].width_k);
        min_wk = std::min(min_wk, td[t].width_k);
        max_st = std::max(max_st, staged_max(g, g->tasks[t], orient));
    }
    DArray<TaskDesc> dtd(T, s);
    DArray<int64_t> dpre(static_cast<size_t>(T) + 1, s);
    DArray<unsigned long long> dcnt(static_cast<size_t>(T) + kLaunchQueueWords, s);  // counts, then queues
    PGABB_HIP(hipMemcpyAsync(dtd.get(), td.get(), td.bytes(), hipMemcpyHostToDevice, s));
    PGABB_HIP(hipMemcpyAsync(dpre.get(), pre.get(), pre.bytes(), hipMemcpyHostToDevice, s));
    PGABB_HIP(hipMemsetAsync(dcnt.get(), 0, sizeof(unsigned long long) * (T + kLaunchQueueWords), s));

    CountArgs a;
    a.tasks = dtd.get();
    a.item_pre = dpre.get();
    a.ntasks = T;
    a.total = pre[T];
    a.counts = dcnt.get();
    a.next = dcnt.get() + T;
    // walked entries of these tasks, at the graph's mean per item
    const uint64_t walked = static_cast<uint64_t>(static_cast<double>(walked_entries(g, orient)) * g->task_share);
    a.grab = opt.rows_per_grab > 0 ? opt.rows_per_grab : default_grab(pre[T], walked);
    a.orient = orient;
    const LaunchKind lk = launch_kind(opt.kernel, max_st, max_wk, min_wk);
    const int waves = opt.waves_per_block > 0 ? opt.waves_per_block : 4;
    StreamTimer tm;
    tm.start(s);
    launch_tc_tasks(a, lk, waves, s, 0, opt.unroll);
    tm.stop(s);

    Staged<unsigned long long> hcnt(T, s);
    PGABB_HIP(hipMemcpyAsync(hcnt.get(), dcnt.get(), hcnt.bytes(), hipMemcpyDeviceToHost, s));
    PGABB_HIP(hipStreamSynchronize(s));
    g->task_counts.assign(hcnt.get(), hcnt.get() + T);
    g->t_kernel_ms = tm.ms();
    g->kernel_launches = lk.nparts;
    uint64_t total = 0;
    for (uint64_t c : g->task_counts) total += c;
    return total;
}

// The partition a count with these options runs on: the graph's own (p = 1
// if it has none), or opt.p with opt.cut_mode when they differ from it.
void ensure_partition(pgabb_graph *g, const pgabb_tc_options &opt) {
    if (opt.p > 0) {
        if (g->p != opt.p || g->cut_mode != opt.cut_mode) partition_graph(g, opt.p, opt.cut_mode, nullptr);
    } else if (g->p == 0) {
        partition_graph(g, 1, PGABB_CUT_NNZ, nullptr);
    }
}

uint64_t count_graph(pgabb_graph *g, const pgabb_tc_options &opt) {
    ensure_partition(g, opt);
    auto t0 = std::chrono::steady_clock::now();
    g->h2d_bytes = 0;
    g->t_kernel_ms = 0;
    g->kernel_launches = 0;
    g->host_tasks = 0;
    g->host_work_share = 0;
    uint64_t total = 0;
    if (!g->tasks.empty()) {
        const uint64_t block_bytes = static_cast<uint64_t>(g->arena_words) * sizeof(int32_t);
        const bool stream = g->blocks_on_host || (opt.flags & (PGABB_OPT_STREAM | PGABB_OPT_HYBRID)) ||
                            (opt.device_cap_bytes && block_bytes > opt.device_cap_bytes);
        total = stream ? count_streamed(g, opt) : count_in_core(g, opt);
    } else {
        g->task_counts.clear();
    }
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return total;
}

// Entries a task's walk reads plus those its items stage, estimated from
// block sizes (a list's length taken as its block's mean): a column walk
// reads A_ik[u] for every entry (u, v) of A_ij and stages A_jk[v] once per
// column v; a row walk reads A_jk[v] per entry and stages A_ik[u] per row.
int64_t task_work_estimate(const pgabb_graph *g, const Task &t, int orient) {
    const BlockInfo &ij = g->blocks[t.bij], &ik = g->blocks[t.bik], &jk = g->blocks[t.bjk];
    const double mean_ik = static_cast<double>(ik.nnz) / static_cast<double>(std::max(ik.nrows, 1));
    const double mean_jk = static_cast<double>(jk.nnz) / static_cast<double>(std::max(jk.nrows, 1));
    const double walk = static_cast<double>(ij.nnz) * (orient == kOrientCol ? mean_ik : mean_jk);
    const double stage = orient == kOrientCol ? static_cast<double>(ij.ncols) * mean_jk
                                              : static_cast<double>(ij.nrows) * mean_ik;
    return 1 + static_cast<int64_t>(walk) + static_cast<int64_t>(stage);
}

// Tasks are independent (Section 4.1), so a count splits over devices by
// task.  Tasks sharing their edge block A_ij form one group, so that a
// device reads each edge block it holds for all of its k; groups are dealt
// by longest processing time on the estimated work of the graph's default
// walk: heaviest first (ties: the group whose first task comes first), each
// to the least loaded shard (ties: lowest index).  The paper's task weight
// (edges of the block-list) balances edges, not work: on skewed graphs the
// walk of a task grows with the mean row length of the walked block.
std::vector<int32_t> task_shards(const pgabb_graph *g, int32_t nshards) {
    const int32_t T = static_cast<int32_t>(g->tasks.size());
    const size_t nb = g->blocks.size();
    pgabb_tc_options dflt;
    std::memset(&dflt, 0, sizeof dflt);
    const int orient = orient_of_option(dflt, g);
    std::vector<int64_t> gw(nb, 0);
    std::vector<int32_t> first(nb, -1);
    for (int32_t t = 0; t < T; ++t) {
        const Task &k = g->tasks[t];
        gw[k.bij] += task_work_estimate(g, k, orient);
        if (first[k.bij] < 0) first[k.bij] = t;
    }
    std::vector<int32_t> groups;
    for (size_t b = 0; b < nb; ++b)
        if (first[b] >= 0) groups.push_back(static_cast<int32_t>(b));
    std::sort(groups.begin(), groups.end(), [&](int32_t a, int32_t b) {
        return gw[a] != gw[b] ? gw[a] > gw[b] : first[a] < first[b];
    });
    using Load = std::pair<int64_t, int32_t>;  // (weight so far, shard)
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (int32_t s = 0; s < nshards; ++s) heap.push({0, s});
    std::vector<int32_t> group_shard(nb, -1);
    for (int32_t b : groups) {
        Load l = heap.top();
        heap.pop();
        group_shard[b] = l.second;
        l.first += gw[b];
        heap.push(l);
    }
    std::vector<int32_t> of(T);
    for (int32_t t = 0; t < T; ++t) of[t] = group_shard[g->tasks[t].bij];
    return of;
}

uint64_t count_shard(pgabb_graph *g, const pgabb_tc_options &opt, int32_t shard, int32_t nshards) {
    ensure_partition(g, opt);
    const std::vector<int32_t> of = task_shards(g, nshards);
    const int orient = orient_of_option(opt, g);
    std::vector<int32_t> idx;  // the shard's tasks, heaviest first as in the full list
    int64_t items = 0, all_items = 0;
    for (size_t t = 0; t < of.size(); ++t) {
        const int64_t it = task_items(g, g->tasks[t], orient);
        all_items += it;
        if (of[t] == shard) {
            idx.push_back(static_cast<int32_t>(t));
            items += it;
        }
    }
    std::vector<Task> all;
    all.swap(g->tasks);
    for (int32_t t : idx) g->tasks.push_back(all[t]);
    g->task_share = all_items ? static_cast<double>(items) / static_cast<double>(all_items) : 1.0;
    uint64_t total = 0;
    std::vector<uint64_t> sub;
    try {
        total = count_graph(g, opt);
        sub.swap(g->task_counts);
    } catch (...) {
        g->tasks.swap(all);
        g->task_share = 1.0;
        g->task_counts.assign(g->tasks.size(), 0);
        throw;
    }
    g->tasks.swap(all);
    g->task_share = 1.0;
    g->task_counts.assign(g->tasks.size(), 0);
    for (size_t q = 0; q < idx.size() && q < sub.size(); ++q) g->task_counts[idx[q]] = sub[q];
    return total;
}

namespace {

// The tasks of several in-core graphs as one work list.
struct MergedTasks {
    std::vector<TaskDesc> desc;
    std::vector<int64_t> pre{0};  // items per task, prefix
    int32_t max_wk = 0, min_wk = INT32_MAX, max_st = 0;
    uint64_t walked = 0;
};

MergedTasks merge_tasks(pgabb_graph *const *gs, const std::vector<int64_t> &which, int orient) {
    MergedTasks m;
    for (int64_t q : which) {
        pgabb_graph *g = gs[q];
        m.walked += walked_entries(g, orient);
        for (const Task &t : g->tasks) {
            m.desc.push_back(make_desc(g, g->arena.get(), t, static_cast<int32_t>(m.desc.size()), nullptr));
            m.pre.push_back(m.pre.back() + task_items(g, t, orient));
            m.max_wk = std::max(m.max_wk, m.desc.back().width_k);
            m.min_wk = std::min(m.min_wk, m.desc.back().width_k);
            m.max_st = std::max(m.max_st, staged_max(g, t, orient));
        }
    }
    return m;
}

// One counting launch over merged tasks, staged on stream s.  run() counts
// with a launch shape and returns the launch's device milliseconds; the
// per-task counts of the last run are read back by fetch().
class MergedLaunch {
  public:
    MergedLaunch(const MergedTasks &m, const pgabb_tc_options &opt, int orient, hipStream_t s)
        : m_(m), s_(s), T_(static_cast<int32_t>(m.desc.size())) {
        lk_ = launch_kind(opt.kernel, m.max_st, m.max_wk, m.min_wk);
        g0_ = default_grab(m.pre.back(), m.walked);
        if (T_ == 0) return;
        Staged<TaskDesc> td(T_, s);
        Staged<int64_t> pre(static_cast<size_t>(T_) + 1, s);
        std::copy(m.desc.begin(), m.desc.end(), td.get());
        std::copy(m.pre.begin(), m.pre.end(), pre.get());
        dtd_.reset(T_, s);
        dpre_.reset(static_cast<size_t>(T_) + 1, s);
        dcnt_.reset(static_cast<size_t>(T_) + kLaunchQueueWords, s);
        PGABB_HIP(hipMemcpyAsync(dtd_.get(), td.get(), td.bytes(), hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(dpre_.get(), pre.get(), pre.bytes(), hipMemcpyHostToDevice, s));
        a_.tasks = dtd_.get();
        a_.item_pre = dpre_.get();
        a_.ntasks = T_;
        a_.total = m.pre.back();
        a_.counts = dcnt_.get();
        a_.next = dcnt_.get() + T_;
        a_.orient = orient;
    }
    int32_t tasks() const { return T_; }
    int64_t items() const { return a_.total; }
    int default_grab_() const { return g0_; }
    const LaunchKind &kind() const { return lk_; }
    double run(int waves, int grab, int unroll) {
        if (T_ == 0 || a_.total == 0) return 0.0;
        PGABB_HIP(hipMemsetAsync(dcnt_.get(), 0, sizeof(unsigned long long) * (T_ + kLaunchQueueWords), s_));
        a_.grab = grab;
        tm_.start(s_);
        launch_tc_tasks(a_, lk_, waves, s_, 0, unroll);
        tm_.stop(s_);
        return tm_.ms();
    }
    std::vector<uint64_t> fetch() {
        std::vector<uint64_t> out(T_, 0);
        if (T_ == 0) return out;
        Staged<unsigned long long> h(T_, s_);
        PGABB_HIP(hipMemcpyAsync(h.get(), dcnt_.get(), h.bytes(), hipMemcpyDeviceToHost, s_));
        PGABB_HIP(hipStreamSynchronize(s_));
        std::copy(h.get(), h.get() + T_, out.begin());
        return out;
    }

  private:
    const MergedTasks &m_;
    hipStream_t s_;
    int32_t T_;
    LaunchKind lk_;
    int g0_ = 2;
    CountArgs a_{};
    DArray<TaskDesc> dtd_;
    DArray<int64_t> dpre_;
    DArray<unsigned long long> dcnt_;
    StreamTimer tm_;
};

// Shape class of a graph for the grid search: bit widths of its edges and
// of its longest oriented row.
std::string grid_class(const pgabb_graph *g) {
    char key[96];
    snprintf(key, sizeof key, "tc_graphs_grid/M%d/D%d", bit_width_u64(static_cast<uint64_t>(g->m)),
             bit_width_u64(static_cast<uint64_t>(g->max_out)));
    return key;
}

}  // namespace

// Counts of several graph objects.  Every graph whose blocks are in device
// memory joins one counting launch over all of their tasks (each task keeps
// its own counter, so each graph's per-task counts come back too); a graph
// whose blocks are streamed from the host store, or that opts ask to stream
// or count hybrid, is counted on its own.
//
// With tune (no options given), two choices are made by timing and kept in
// the persisted tuning cache:
//   1. the grid of each shape class of graphs (bit widths of m' and of the
//      longest row): p in {1, 2, 4, 8, 16} with nnz-balanced cuts, and p = 8
//      with uniform cuts, each timed as one launch over the class's graphs
//      partitioned that way;
//   2. the launch shape of the whole merged launch (waves per workgroup,
//      items per grab, chunks per load batch), keyed by graph count, tasks,
//      items, walked entries per item and longest staged list.
void count_graphs(pgabb_graph *const *gs, int64_t G, const pgabb_tc_options &opt, bool tune, uint64_t *counts) {
    const auto t_tune0 = std::chrono::steady_clock::now();
    double tune_ms = 0;
    hipStream_t s = library_stream();
    const int orient = orient_of_option(opt, nullptr);
    auto in_core = [&](pgabb_graph *g) {
        const uint64_t block_bytes = static_cast<uint64_t>(g->arena_words) * sizeof(int32_t);
        return !(g->blocks_on_host || (opt.flags & (PGABB_OPT_STREAM | PGABB_OPT_HYBRID)) ||
                 (opt.device_cap_bytes && block_bytes > opt.device_cap_bytes));
    };
    auto after_graph_streams = [&](const std::vector<int64_t> &which) {
        for (int64_t q : which) {  // launches on the library stream follow each graph's own work
            hipEvent_t ev = nullptr;
            PGABB_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            PGABB_HIP(hipEventRecord(ev, gs[q]->stream));
            PGABB_HIP(hipStreamWaitEvent(s, ev, 0));
            PGABB_HIP(hipEventDestroy(ev));
        }
    };
    if (tune) {
        // ---- 1. the grid per shape class
        std::map<std::string, std::vector<int64_t>> classes;
        for (int64_t q = 0; q < G; ++q) {
            pgabb_graph *g = gs[q];
            if (g->p == 0) partition_graph(g, 1, PGABB_CUT_NNZ, nullptr);
            if (in_core(g) && g->m > 0) classes[grid_class(g)].push_back(q);
        }
        static const int32_t kGridP[] = {1, 2, 4, 8, 16, 8};
        static const int32_t kGridCut[] = {PGABB_CUT_NNZ, PGABB_CUT_NNZ, PGABB_CUT_NNZ, PGABB_CUT_NNZ,
                                           PGABB_CUT_NNZ, PGABB_CUT_UNIFORM};
        for (auto &kv : classes) {
            std::vector<int> v;
            int32_t bp = 1, bcut = PGABB_CUT_NNZ;
            if (tune_lookup(kv.first, v) && v.size() == 2 && v[0] >= 1 && v[0] <= 64 &&
                (v[1] == PGABB_CUT_NNZ || v[1] == PGABB_CUT_UNIFORM)) {
                bp = v[0];
                bcut = v[1];
            } else {
                double best = 1e30;
                int32_t max_n = 1;
                for (int64_t q : kv.second) max_n = std::max(max_n, gs[q]->n);
                for (int c = 0; c < 6; ++c) {
                    if (kGridP[c] > max_n) continue;
                    for (int64_t q : kv.second) {
                        pgabb_graph *g = gs[q];
                        if (g->p != kGridP[c] || g->cut_mode != kGridCut[c])
                            partition_graph(g, kGridP[c], kGridCut[c], nullptr);
                    }
                    after_graph_streams(kv.second);
                    const MergedTasks mt = merge_tasks(gs, kv.second, orient);
                    MergedLaunch ml(mt, opt, orient, s);
                    const int gr = ml.default_grab_();
                    ml.run(4, gr, 2);  // warm
                    const double ms = std::min(ml.run(4, gr, 2), ml.run(4, gr, 2));
                    if (ms < best) {
                        best = ms;
                        bp = kGridP[c];
                        bcut = kGridCut[c];
                    }
                }
                tune_store(kv.first, {bp, bcut});
            }
            for (int64_t q : kv.second) {
                pgabb_graph *g = gs[q];
                if (g->p != bp || g->cut_mode != bcut) partition_graph(g, bp, bcut, nullptr);
            }
        }
    }
    std::vector<int64_t> merged;
    for (int64_t q = 0; q < G; ++q) {
        pgabb_graph *g = gs[q];
        if (!tune) ensure_partition(g, opt);
        else if (g->p == 0) partition_graph(g, 1, PGABB_CUT_NNZ, nullptr);
        if (in_core(g)) merged.push_back(q);
        else counts[q] = count_graph(g, opt);
    }
    if (merged.empty()) return;
    after_graph_streams(merged);
    for (int64_t q : merged) {
        pgabb_graph *g = gs[q];
        g->walked_columns = orient == kOrientCol;
        g->h2d_bytes = 0;
        g->host_tasks = 0;
        g->host_work_share = 0;
    }
    const MergedTasks mt = merge_tasks(gs, merged, orient);
    MergedLaunch ml(mt, opt, orient, s);
    const int g0 = ml.default_grab_();
    int waves = opt.waves_per_block > 0 ? opt.waves_per_block : 4;
    int grab = opt.rows_per_grab > 0 ? opt.rows_per_grab : g0;
    int unroll = opt.unroll;
    // ---- 2. the launch shape
    if (tune && ml.kind().nparts == 1 && ml.items() > 0) {
        const uint64_t per_item = mt.walked / static_cast<uint64_t>(ml.items());
        char key[160];
        snprintf(key, sizeof key, "tc_graphs/G%d/T%d/I%d/W%d/S%d/K%d/O%d", bit_width_u64(merged.size()),
                 bit_width_u64(ml.tasks()), bit_width_u64(ml.items()), bit_width_u64(per_item),
                 bit_width_u64(mt.max_st), ml.kind().mode, orient);
        std::vector<int> v;
        if (tune_lookup(key, v) && v.size() == 3) {
            waves = v[0];
            grab = v[1];
            unroll = v[2];
        } else {
            double best = 1e30;
            for (int w : {2, 4, 8})
                for (int gr : {std::max(1, g0 / 2), g0, std::min(64, 2 * g0)})
                    for (int un : {2, 4}) {
                        ml.run(w, gr, un);  // warm
                        const double ms = std::min(ml.run(w, gr, un), ml.run(w, gr, un));
                        if (ms < best) {
                            best = ms;
                            waves = w;
                            grab = gr;
                            unroll = un;
                        }
                    }
            tune_store(key, {waves, grab, unroll});
        }
    }
    if (tune) tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_tune0).count();
    const auto t0 = std::chrono::steady_clock::now();
    const double kernel_ms = ml.run(waves, grab, unroll);
    const std::vector<uint64_t> tc = ml.fetch();
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    size_t at = 0;
    for (int64_t q : merged) {
        pgabb_graph *g = gs[q];
        const size_t nt = g->tasks.size();
        g->task_counts.assign(tc.begin() + at, tc.begin() + at + nt);
        at += nt;
        uint64_t total = 0;
        for (uint64_t c : g->task_counts) total += c;
        counts[q] = total;
        g->t_count_ms = ms;
        g->t_kernel_ms = kernel_ms;
        g->t_tune_ms = tune_ms;
        g->kernel_launches = ml.kind().nparts;
    }
}

}  // namespace pgabb
