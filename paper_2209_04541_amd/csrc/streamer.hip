// Streamed count: blocks live in a pinned host store and move to the device
// on demand, under a byte cap.
//
// PGAbB Section 4.4: the graph is stored in host memory; the blocks of a task
// assigned to the GPU are copied with asynchronous host-to-device copies, and
// several streams let the copy of the next assignment overlap the current
// computation.  Instead of waiting for all tasks and clearing the device
// when memory runs low, this keeps a block cache: a device pool of at most
// `device_cap_bytes` managed first-fit, with least-recently-used eviction of
// blocks that no in-flight task still reads (every stream's last window that
// read a block has finished before its range is reused).
//
// Tasks are taken in the heaviest-first order and grouped into windows of a
// few tasks whose blocks are resident together.  In the hybrid mode host
// threads run the host kernel on the lightest remaining tasks, read straight
// from the host store, while the device takes windows from the heavy end
// (Section 4.4: heavy tasks to the GPU, light ones to CPU threads, all
// pulled from one task queue).  For each window the missing
// blocks are copied on a copy stream; the window's counting launch runs on
// one of several compute streams once its copies are done; windows on
// different streams overlap, and the copies of later windows overlap earlier
// launches.
//
// A graph partitioned on the device reaches its first streamed count with
// the blocks still in the device arena.  Outside the hybrid mode the count
// moves them to the host store itself, on a stream of its own: first the
// part of each block its walk reads, block by block in the order the tasks
// first use them, then the rest of the arena.  Each block's copy back waits
// only for that block's move, so the first windows start after a small part
// of the store has crossed and the moves overlap the copies back (the other
// direction of the link) and the launches.  The arena is released once the
// count ends, leaving the same host store as a move before the count.
#include <algorithm>
#include <chrono>
#include <list>
#include <map>
#include <mutex>
#include <thread>

#include "block_readers.hpp"
#include "range_pool.hpp"
#include "common.hpp"
#include "count.hpp"
#include "graph.hpp"
#include "tc_device.hpp"

namespace pgabb {

namespace {

constexpr uint64_t kAlign = 256;

// Bytes of the part of a block's chunk that a walk in `orient` reads (the
// unit of copy and of pool space), rounded up to kAlign.
uint64_t chunk_bytes(const BlockInfo &b, int orient) {
    const uint64_t raw = static_cast<uint64_t>(b.walk_hi(orient) - b.walk_lo(orient)) * sizeof(int32_t);
    return (raw + kAlign - 1) / kAlign * kAlign;
}

}  // namespace

// Moves the device arena to a pinned host store (once per partition).
void move_blocks_to_host(pgabb_graph *g) {
    if (g->blocks_on_host) return;
    hipStream_t s = g->stream;
    g->host_arena.reset(static_cast<size_t>(g->arena_words), s, true);
    if (g->arena_words)
        PGABB_HIP(hipMemcpyAsync(g->host_arena.get(), g->arena.get(), sizeof(int32_t) * g->arena_words,
                                 hipMemcpyDeviceToHost, s));
    PGABB_HIP(hipStreamSynchronize(s));
    g->arena.release();
    g->blocks_on_host = true;
}

// Order of the tasks when the blocks do not all fit under the cap: a
// simulated block cache of `cap` bytes (least recently used out first,
// never a block of the task being placed) is filled task by task, and the
// next task is always one whose blocks are missing the fewest bytes from
// it, the heaviest among equals.  Heaviest-first alone reloads blocks many
// times once the cache holds a small share of them; this order keeps the
// tasks that share blocks together.  O(T^2) on the host, with per-task
// missing bytes updated as blocks enter and leave.
std::vector<int32_t> locality_order(const pgabb_graph *g, uint64_t cap, int orient) {
    const int32_t T = static_cast<int32_t>(g->tasks.size());
    const int32_t nblk = static_cast<int32_t>(g->blocks.size());
    std::vector<std::vector<int32_t>> users(nblk);  // tasks reading each block (once each)
    std::vector<uint64_t> miss(T, 0);
    for (int32_t t = 0; t < T; ++t) {
        const Task &k = g->tasks[t];
        const int32_t bs[3] = {k.bij, k.bik, k.bjk};
        for (int q = 0; q < 3; ++q) {
            const int32_t b = bs[q];
            if ((q >= 1 && b == bs[0]) || (q == 2 && b == bs[1])) continue;  // a block listed twice
            users[b].push_back(t);
            miss[t] += chunk_bytes(g->blocks[b], orient);
        }
    }
    std::vector<char> done(T, 0), resident(nblk, 0);
    std::list<int32_t> lru;
    std::vector<std::list<int32_t>::iterator> pos(nblk);
    uint64_t used = 0;
    auto enter = [&](int32_t b) {
        resident[b] = 1;
        used += chunk_bytes(g->blocks[b], orient);
        lru.push_back(b);
        pos[b] = std::prev(lru.end());
        for (int32_t t : users[b]) miss[t] -= chunk_bytes(g->blocks[b], orient);
    };
    auto leave = [&](int32_t b) {
        resident[b] = 0;
        used -= chunk_bytes(g->blocks[b], orient);
        lru.erase(pos[b]);
        for (int32_t t : users[b]) miss[t] += chunk_bytes(g->blocks[b], orient);
    };
    std::vector<int32_t> order;
    order.reserve(T);
    for (int32_t step = 0; step < T; ++step) {
        int32_t best = -1;
        for (int32_t t = 0; t < T; ++t) {  // tasks are heaviest first: the first minimum wins
            if (done[t]) continue;
            if (best < 0 || miss[t] < miss[best]) best = t;
            if (miss[best] == 0) break;
        }
        done[best] = 1;
        order.push_back(best);
        const Task &k = g->tasks[best];
        for (int32_t b : {k.bij, k.bik, k.bjk}) {
            if (resident[b]) {
                lru.erase(pos[b]);
                lru.push_back(b);
                pos[b] = std::prev(lru.end());
                continue;
            }
            const uint64_t need = chunk_bytes(g->blocks[b], orient);
            auto it = lru.begin();
            while (used + need > cap && it != lru.end()) {
                const int32_t v = *it++;
                if (v != k.bij && v != k.bik && v != k.bjk) leave(v);
            }
            enter(b);
        }
    }
    return order;
}

uint64_t count_streamed(pgabb_graph *g, const pgabb_tc_options &opt) {
    const bool hybrid = (opt.flags & PGABB_OPT_HYBRID) != 0;
    // host threads read the store directly: it must be whole before they start
    if (hybrid) move_blocks_to_host(g);
    const bool moving = !g->blocks_on_host;  // moved below, overlapping the count
    hipStream_t s = g->stream;
    const int32_t T = static_cast<int32_t>(g->tasks.size());
    const int32_t nblk = static_cast<int32_t>(g->blocks.size());

    // bytes of the blocks these tasks read (all of them for a whole count;
    // fewer for one shard's tasks)
    // the walk decides which part of each chunk is copied
    const int orient = orient_of_option(opt, g);
    uint64_t total_bytes = 0;
    {
        std::vector<char> used(nblk, 0);
        for (const Task &t : g->tasks) used[t.bij] = used[t.bik] = used[t.bjk] = 1;
        for (int32_t b = 0; b < nblk; ++b)
            if (used[b]) total_bytes += chunk_bytes(g->blocks[b], orient);
    }
    uint64_t cap = opt.device_cap_bytes ? opt.device_cap_bytes : total_bytes;
    g->host_store_cap = opt.device_cap_bytes;
    cap = std::min(cap, total_bytes);
    cap = cap / kAlign * kAlign;
    for (const Task &t : g->tasks) {
        uint64_t need = chunk_bytes(g->blocks[t.bij], orient);
        if (t.bik != t.bij) need += chunk_bytes(g->blocks[t.bik], orient);
        if (t.bjk != t.bij && t.bjk != t.bik) need += chunk_bytes(g->blocks[t.bjk], orient);
        PGABB_REQUIRE(need <= cap, PGABB_ENOMEM,
                      "device cap of %llu bytes cannot hold the %llu bytes of task (%d, %d, %d)",
                      static_cast<unsigned long long>(cap), static_cast<unsigned long long>(need),
                      t.i, t.j, t.k);
    }

    const int nstreams = opt.num_streams > 0 ? std::min(opt.num_streams, 16) : 4;
    std::vector<hipStream_t> cs(nstreams);
    hipStream_t copy_s = nullptr;
    PGABB_HIP(hipStreamCreateWithFlags(&copy_s, hipStreamNonBlocking));
    for (auto &x : cs) PGABB_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));

    // device pool and per-run arrays
    DArray<uint8_t> pool(static_cast<size_t>(cap), s);
    DArray<TaskDesc> ddesc(static_cast<size_t>(T), s);
    DArray<int64_t> dpre(static_cast<size_t>(2 * T + 1), s);
    // counts, then kQueues work counters per window (at most T windows)
    const size_t ncnt = static_cast<size_t>(T) * (1 + kLaunchQueueWords);
    DArray<unsigned long long> dcnt(ncnt, s);
    PGABB_HIP(hipMemsetAsync(dcnt.get(), 0, sizeof(unsigned long long) * ncnt, s));
    PinnedArray<TaskDesc> hdesc;
    hdesc.reset(static_cast<size_t>(T));
    PinnedArray<int64_t> hpre;
    hpre.reset(static_cast<size_t>(2 * T + 1));
    PGABB_HIP(hipStreamSynchronize(s));

    RangePool rp(cap);
    std::vector<uint64_t> where(nblk, UINT64_MAX);   // pool offset of resident blocks
    BlockReaders readers(nblk, nstreams);            // windows per stream that read each block
    std::list<int32_t> lru;                           // resident blocks, least recent first
    std::vector<std::list<int32_t>::iterator> lru_pos(nblk);
    std::vector<hipEvent_t> done;                     // per window
    std::vector<hipEvent_t> copied;
    std::vector<hipEvent_t> kstart, kstop;            // per window launch timing

    int32_t max_wk = 0, min_wk = INT32_MAX;
    for (int32_t t = 0; t < T; ++t) {
        const int32_t wk = g->cuts[g->tasks[t].k + 1] - g->base[g->tasks[t].k];
        max_wk = std::max(max_wk, wk);
        min_wk = std::min(min_wk, wk);
    }
    int32_t max_st = 0;
    for (int32_t t = 0; t < T; ++t) max_st = std::max(max_st, staged_max(g, g->tasks[t], orient));
    const LaunchKind lk = launch_kind(opt.kernel, max_st, max_wk, min_wk);
    g->walked_columns = orient == kOrientCol;
    const int waves = opt.waves_per_block > 0 ? opt.waves_per_block : 4;
    const int grab_opt = opt.rows_per_grab;
    // A window is cut when its blocks would exceed the cap or when it would
    // copy more than about an eighth of all block bytes: the first launch
    // starts after a short copy, and later copies overlap earlier launches.
    // in the hybrid mode windows hold at most 1/32 of the tasks, so the
    // device claims work in steps small enough for the two sides to meet
    // near the balance point
    const int window_tasks = hybrid ? std::max(1, T / 32) : T;
    const uint64_t window_new_bytes = std::max<uint64_t>(64ull << 20, std::min<uint64_t>(cap / 4, total_bytes / 8));

    std::vector<int64_t> chunk_dev(nblk, 0);  // in int32 words from pool start
    // processing order of the tasks: heaviest first when every block fits
    // under the cap, else the locality order above
    std::vector<int32_t> order(T);
    for (int32_t t = 0; t < T; ++t) order[t] = t;
    if (total_bytes > cap) order = locality_order(g, cap, orient);

    // ---- the move to the host store, queued in full before the first
    // window: the walked part of every block's chunk in order of first use
    // (moved[b] marks its end), then the arena's other words
    hipStream_t move_s = nullptr;
    hipEvent_t arena_ready = nullptr;
    std::vector<hipEvent_t> moved(nblk, nullptr);
    auto end_moves = [&]() noexcept {
        if (move_s) (void)hipStreamSynchronize(move_s);
        for (auto &e : moved) {
            if (e) (void)hipEventDestroy(e);
            e = nullptr;
        }
        if (arena_ready) (void)hipEventDestroy(arena_ready);
        if (move_s) (void)hipStreamDestroy(move_s);
        move_s = nullptr;
        arena_ready = nullptr;
    };

    uint64_t h2d = 0;
    int32_t next_task = 0;  // position in `order`: the device takes [0, next_task)
    int32_t win = 0;
    int64_t pre_at = 0;

    // ---- hybrid: the host takes positions [back, T) of `order`, one task
    // at a time from the end; with a fixed share it stops at host_stop (the
    // device then stops there too).  Otherwise the cut-off is measured: a
    // host thread takes the next task only if, at the host's measured rate
    // per thread, it would finish before the device, at its measured rate,
    // finishes the work still in front of it.  Rates are estimated work
    // (walked plus staged entries) per second: the device's from its
    // completed windows, the host's from its completed tasks; until a first
    // measurement, priors of kDevicePrior and kHostPrior.
    constexpr double kDevicePrior = 2e11;  // entries/s, one MI355X in-core launch
    constexpr double kHostPrior = 2e7;     // entries/s per host thread
    std::mutex qmu;
    int32_t back = T;
    int32_t host_stop = T;
    std::vector<uint64_t> host_cnt(T, 0);
    std::vector<std::thread> host;
    double host_work = 0, all_work = 0;
    std::vector<double> est, wpre;             // estimated work by position, and its prefix
    std::vector<int32_t> win_end;              // first position after each window
    const auto t_begin = std::chrono::steady_clock::now();
    double dev_done_work = 0, dev_done_s = 0;  // under qmu: completed windows' work and time
    double host_done_work = 0, host_busy_s = 0;
    if (hybrid) {
        est.assign(T, 0);
        wpre.assign(static_cast<size_t>(T) + 1, 0);
        for (int32_t q = 0; q < T; ++q) {
            est[q] = static_cast<double>(task_work_estimate(g, g->tasks[order[q]], orient));
            all_work += est[q];
            wpre[q + 1] = wpre[q] + est[q];
        }
        if (opt.host_permille > 0) {
            const double share = all_work * opt.host_permille / 1000.0;
            double acc = 0;
            host_stop = T;
            while (host_stop > 0 && acc + est[host_stop - 1] <= share + 1e-9) acc += est[--host_stop];
        } else {
            host_stop = 0;
        }
        const int nth = opt.host_threads > 0
                            ? opt.host_threads
                            : static_cast<int>(std::max(1u, std::min(64u, std::thread::hardware_concurrency())));
        const int32_t *harena = g->host_arena.get();
        for (int h = 0; h < nth; ++h)
            host.emplace_back([&, harena] {
                for (;;) {
                    int32_t pos;
                    {
                        std::lock_guard<std::mutex> lk(qmu);
                        if (back <= std::max(next_task, host_stop)) return;
                        if (opt.host_permille == 0) {
                            const double dev_rate = dev_done_s > 0 && dev_done_work > 0
                                                        ? dev_done_work / dev_done_s : kDevicePrior;
                            const double host_rate = host_busy_s > 0 && host_done_work > 0
                                                         ? host_done_work / host_busy_s : kHostPrior;
                            const double device_left = wpre[back - 1] - wpre[next_task];
                            if (est[back - 1] / host_rate > device_left / dev_rate) return;
                        }
                        pos = --back;
                    }
                    const auto h0 = std::chrono::steady_clock::now();
                    const int32_t t = order[pos];
                    host_cnt[t] = host_count_task(g, harena, g->tasks[t]);
                    const double dt =
                        std::chrono::duration<double>(std::chrono::steady_clock::now() - h0).count();
                    std::lock_guard<std::mutex> lk(qmu);
                    host_done_work += est[pos];
                    host_busy_s += dt;
                }
            });
    }
    auto stop_host = [&]() {
        {
            std::lock_guard<std::mutex> lk(qmu);
            host_stop = T;  // host threads end after their current task
        }
        for (auto &th : host)
            if (th.joinable()) th.join();
    };

    auto touch = [&](int32_t b) {
        lru.erase(lru_pos[b]);
        lru.push_back(b);
        lru_pos[b] = std::prev(lru.end());
    };

    try {
        if (moving) {
            g->host_arena.reset(static_cast<size_t>(g->arena_words), s, true);
            PGABB_HIP(hipStreamCreateWithFlags(&move_s, hipStreamNonBlocking));
            PGABB_HIP(hipEventCreateWithFlags(&arena_ready, hipEventDisableTiming));
            PGABB_HIP(hipEventRecord(arena_ready, s));  // the arena was written on the graph's stream
            PGABB_HIP(hipStreamWaitEvent(move_s, arena_ready, 0));
            int32_t *harena = g->host_arena.get();
            const int32_t *darena = g->arena.get();
            auto move_words = [&](int64_t lo, int64_t hi) {
                if (hi > lo)
                    PGABB_HIP(hipMemcpyAsync(harena + lo, darena + lo, sizeof(int32_t) * static_cast<size_t>(hi - lo),
                                             hipMemcpyDeviceToHost, move_s));
            };
            // the part of the chunk this count's walk reads comes first
            auto move_block = [&](int32_t b) {
                if (moved[b]) return;
                move_words(g->blocks[b].walk_lo(orient), g->blocks[b].walk_hi(orient));
                PGABB_HIP(hipEventCreateWithFlags(&moved[b], hipEventDisableTiming));
                PGABB_HIP(hipEventRecord(moved[b], move_s));
            };
            for (int32_t q = 0; q < T; ++q)
                for (int32_t b : {g->tasks[order[q]].bij, g->tasks[order[q]].bik, g->tasks[order[q]].bjk})
                    move_block(b);
            for (int32_t b = 0; b < nblk; ++b) move_block(b);
            // then every word outside the walked parts
            std::vector<std::pair<int64_t, int64_t>> walked;
            for (const BlockInfo &bi : g->blocks) walked.emplace_back(bi.walk_lo(orient), bi.walk_hi(orient));
            std::sort(walked.begin(), walked.end());
            int64_t at = 0;
            for (const auto &c : walked) {
                move_words(at, c.first);
                at = std::max(at, c.second);
            }
            move_words(at, g->arena_words);
        }
        for (;;) {
            // in the hybrid mode at most one window per stream is in flight,
            // so the device claims tasks only as fast as it counts them
            if (hybrid && win >= nstreams) {
                PGABB_HIP(hipEventSynchronize(done[win - nstreams]));
                const double s_now =
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t_begin).count();
                std::lock_guard<std::mutex> lk(qmu);
                dev_done_work = wpre[win_end[win - nstreams]];
                dev_done_s = s_now;
            }
            std::unique_lock<std::mutex> qlk(qmu);
            const int32_t limit = hybrid ? (opt.host_permille > 0 ? host_stop : back) : T;
            if (next_task >= limit) break;
            // ---- form a window: tasks whose blocks fit together
            std::vector<int32_t> wtasks;  // task indices, in processing order
            const int32_t p0 = next_task;   // the window's first position in `order`
            std::vector<char> in_window(nblk, 0);
            uint64_t pinned_bytes = 0, new_bytes = 0;
            while (next_task < limit && static_cast<int>(wtasks.size()) < window_tasks) {
                const Task &t = g->tasks[order[next_task]];
                // bytes this task adds to the window (its block ids may repeat)
                uint64_t add = 0, add_new = 0;
                int32_t seen[3] = {-1, -1, -1};
                int ns = 0;
                for (int32_t b : {t.bij, t.bik, t.bjk}) {
                    bool rep = in_window[b] != 0;
                    for (int q = 0; q < ns; ++q) rep = rep || seen[q] == b;
                    if (rep) continue;
                    seen[ns++] = b;
                    add += chunk_bytes(g->blocks[b], orient);
                    if (where[b] == UINT64_MAX) add_new += chunk_bytes(g->blocks[b], orient);
                }
                if (!wtasks.empty() && (pinned_bytes + add > cap || new_bytes + add_new > window_new_bytes))
                    break;
                for (int32_t b : {t.bij, t.bik, t.bjk}) in_window[b] = 1;
                pinned_bytes += add;
                new_bytes += add_new;
                wtasks.push_back(order[next_task++]);
            }
            qlk.unlock();

            // ---- make the window's blocks resident.  If first-fit cannot place
            // a block even with every block outside the window evicted (the pool
            // is fragmented), wait for all in-flight work, empty the cache and
            // place the window again into the empty pool, where it fits.
            std::vector<int32_t> loads;
            bool placed = false;
            for (int attempt = 0; attempt < 2 && !placed; ++attempt) {
                loads.clear();
                placed = true;
                for (int32_t ti : wtasks) {
                    for (int32_t b : {g->tasks[ti].bij, g->tasks[ti].bik, g->tasks[ti].bjk}) {
                        if (where[b] != UINT64_MAX) {
                            touch(b);
                            continue;
                        }
                        const uint64_t need = chunk_bytes(g->blocks[b], orient);
                        uint64_t off = rp.alloc(need);
                        while (off == UINT64_MAX) {
                            auto it = lru.begin();
                            while (it != lru.end() && in_window[*it]) ++it;
                            if (it == lru.end()) break;
                            const int32_t v = *it;
                            readers.release(v, [&](int32_t w) { PGABB_HIP(hipEventSynchronize(done[w])); });
                            rp.release(where[v], chunk_bytes(g->blocks[v], orient));
                            where[v] = UINT64_MAX;
                            lru.erase(it);
                            off = rp.alloc(need);
                        }
                        if (off == UINT64_MAX) {
                            placed = false;
                            break;
                        }
                        where[b] = off;
                        // the chunk's start, in words from the pool's start, as if the
                        // whole chunk were there: only [walk_lo, walk_hi) is copied
                        // and read
                        chunk_dev[b] = static_cast<int64_t>(off / sizeof(int32_t)) -
                                       (g->blocks[b].walk_lo(orient) - g->blocks[b].chunk_off);
                        lru.push_back(b);
                        lru_pos[b] = std::prev(lru.end());
                        loads.push_back(b);
                    }
                    if (!placed) break;
                }
                if (!placed) {
                    for (auto x : cs) PGABB_HIP(hipStreamSynchronize(x));
                    PGABB_HIP(hipStreamSynchronize(copy_s));
                    for (int32_t v : lru) where[v] = UINT64_MAX;
                    lru.clear();
                    readers.clear();
                    rp = RangePool(cap);
                }
            }
            PGABB_REQUIRE(placed, PGABB_ENOMEM, "device cap of %llu bytes cannot hold a window",
                          static_cast<unsigned long long>(cap));
            for (int32_t b : loads) {
                const BlockInfo &bi = g->blocks[b];
                const size_t bytes = static_cast<size_t>(bi.walk_hi(orient) - bi.walk_lo(orient)) * sizeof(int32_t);
                if (moving) PGABB_HIP(hipStreamWaitEvent(copy_s, moved[b], 0));
                PGABB_HIP(hipMemcpyAsync(pool.get() + where[b], g->host_arena.get() + bi.walk_lo(orient), bytes,
                                         hipMemcpyHostToDevice, copy_s));
                h2d += bytes;
            }
            hipEvent_t ce = nullptr, de = nullptr;
            PGABB_HIP(hipEventCreateWithFlags(&ce, hipEventDisableTiming));
            PGABB_HIP(hipEventCreateWithFlags(&de, hipEventDisableTiming));
            copied.push_back(ce);
            done.push_back(de);
            PGABB_HIP(hipEventRecord(ce, copy_s));

            // ---- descriptors and launch
            // descriptors sit at the tasks' positions in `order`; each keeps its
            // task index as its counter slot
            const int32_t W = static_cast<int32_t>(wtasks.size());
            int64_t items = 0;
            hpre[pre_at] = 0;
            for (int32_t q = 0; q < W; ++q) {
                const int32_t ti = wtasks[q];
                hdesc[p0 + q] = make_desc(g, reinterpret_cast<const int32_t *>(pool.get()), g->tasks[ti], ti,
                                          chunk_dev.data());
                items += task_items(g, g->tasks[ti], orient);
                hpre[pre_at + q + 1] = items;
            }
            const int si = win % nstreams;
            hipStream_t st = cs[si];
            PGABB_HIP(hipStreamWaitEvent(st, ce, 0));
            hipEvent_t k0 = nullptr, k1 = nullptr;
            PGABB_HIP(hipEventCreate(&k0));
            PGABB_HIP(hipEventCreate(&k1));
            kstart.push_back(k0);
            kstop.push_back(k1);
            PGABB_HIP(hipMemcpyAsync(ddesc.get() + p0, hdesc.get() + p0, sizeof(TaskDesc) * W,
                                     hipMemcpyHostToDevice, st));
            PGABB_HIP(hipMemcpyAsync(dpre.get() + pre_at, hpre.get() + pre_at, sizeof(int64_t) * (W + 1),
                                     hipMemcpyHostToDevice, st));
            CountArgs a;
            a.tasks = ddesc.get() + p0;
            a.item_pre = dpre.get() + pre_at;
            a.ntasks = W;
            // from the window's item count alone: windows are heaviest-first
            // slices, whose items carry more work than the graph's mean, so
            // a grab sized from the mean would be too coarse for them
            a.grab = grab_opt > 0 ? grab_opt : default_grab(items, 0);
            a.orient = orient;
                a.total = items;
            a.counts = dcnt.get();
            a.next = dcnt.get() + T + static_cast<size_t>(win) * kLaunchQueueWords;
            PGABB_HIP(hipEventRecord(k0, st));
            launch_tc_tasks(a, lk, waves, st, 0, opt.unroll);
            PGABB_HIP(hipEventRecord(k1, st));
            PGABB_HIP(hipEventRecord(de, st));
            for (int32_t ti : wtasks)
                for (int32_t b : {g->tasks[ti].bij, g->tasks[ti].bik, g->tasks[ti].bjk}) readers.read(b, si, win);
            pre_at += W + 1;
            if (hybrid) win_end.push_back(next_task);
            ++win;
        }
        for (auto &th : host) th.join();
        for (auto x : cs) PGABB_HIP(hipStreamSynchronize(x));
        PGABB_HIP(hipStreamSynchronize(copy_s));
        if (moving) {
            PGABB_HIP(hipStreamSynchronize(move_s));
            end_moves();
            g->arena.release();
            g->blocks_on_host = true;
        }
        double kms = 0;
        for (size_t q = 0; q < kstart.size(); ++q) {
            float t = 0;
            PGABB_HIP(hipEventElapsedTime(&t, kstart[q], kstop[q]));
            kms += t;
        }
        g->t_kernel_ms = kms;
        g->task_counts.assign(T, 0);
        PGABB_HIP(hipMemcpyAsync(g->task_counts.data(), dcnt.get(), sizeof(uint64_t) * T, hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        // device tasks left their host slot at 0, host tasks their device slot
        for (int32_t t = 0; t < T; ++t) g->task_counts[t] += host_cnt[t];
        g->host_tasks = T - back;
        if (hybrid && all_work > 0) {
            for (int32_t q = back; q < T; ++q)
                host_work += static_cast<double>(task_work_estimate(g, g->tasks[order[q]], orient));
            g->host_work_share = host_work / all_work;
        }
    } catch (...) {
        stop_host();
        for (auto x : cs) (void)hipStreamSynchronize(x);
        (void)hipStreamSynchronize(copy_s);
        if (moving && !g->blocks_on_host) {  // the blocks stay in the device arena
            end_moves();
            g->host_arena.release();
        }
        for (auto e : copied) (void)hipEventDestroy(e);
        for (auto e : done) (void)hipEventDestroy(e);
        for (auto e : kstart) (void)hipEventDestroy(e);
        for (auto e : kstop) (void)hipEventDestroy(e);
        for (auto x : cs) (void)hipStreamDestroy(x);
        (void)hipStreamDestroy(copy_s);
        throw;
    }
    for (auto e : copied) (void)hipEventDestroy(e);
    for (auto e : done) (void)hipEventDestroy(e);
    for (auto e : kstart) (void)hipEventDestroy(e);
    for (auto e : kstop) (void)hipEventDestroy(e);
    for (auto x : cs) (void)hipStreamDestroy(x);
    (void)hipStreamDestroy(copy_s);
    g->h2d_bytes = h2d;
    g->kernel_launches = static_cast<int64_t>(win) * lk.nparts;
    uint64_t total = 0;
    for (uint64_t c : g->task_counts) total += c;
    return total;
}

}  // namespace pgabb
