// Request server with continuous batching.
//
// Host threads drive HIP streams:
//  - builders (options.num_streams of them, default 2, each with its own
//    stream) admit queued requests in arrival order while their estimated
//    device bytes fit the budget, and build each one (clean, rank, orient,
//    partition: options.p blocks a side, or by size, 8 for requests of at
//    least 2^18 pairs and 1 below);
//  - the counter takes every request built so far, runs all their tasks in
//    one counting launch on the count stream, returns each request's uint64
//    count, frees its device memory and wakes the builder.
// So requests that arrive while others are being counted are admitted as
// memory frees up, are built while the previous launch runs, and join the
// next launch: their device work overlaps, and each result is the same as
// when counted alone (integer sums do not depend on the batch).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "common.hpp"
#include "count.hpp"
#include "graph.hpp"
#include "tc_device.hpp"

namespace pgabb {
pgabb_status capture_status(const Error &e);
}

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    int32_t n = 0;
    int64_t m = 0;
    std::vector<int32_t> src, dst;      // owned copies
    const int32_t *bsrc = nullptr;      // borrowed arrays (PGABB_SERVER_BORROW)
    const int32_t *bdst = nullptr;
    uint64_t est = 0;
    int32_t p = 1;                      // grid of the request's partition
    double t_submit = 0, t_done = 0;
    pgabb_graph *g = nullptr;
    uint64_t count = PGABB_COUNT_ERROR;
    pgabb_status status = PGABB_OK;
    bool done = false;
};

}  // namespace

struct pgabb_server {
    uint64_t budget = 0;
    pgabb_tc_options opt{};
    std::mutex mu;
    std::condition_variable cv_build, cv_count, cv_done;
    std::deque<Request *> queue;  // submitted, not yet admitted
    std::deque<Request *> ready;  // built, waiting for a launch
    std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
    uint64_t reserved = 0;
    uint64_t next_ticket = 1;
    int64_t in_flight = 0;  // admitted, not finished
    bool stop = false;
    int builders_left = 0;  // builder threads still running
    std::vector<std::thread> builders;
    std::thread counter;
    std::vector<hipStream_t> build_streams;
    hipStream_t count_stream = nullptr;
    int device = 0;
    Clock::time_point t0 = Clock::now();
    uint64_t launches = 0;
    // counting launches' device time and the entries they walked and edges
    // they covered (for the launches' roofline)
    double kernel_ms = 0;
    uint64_t walked = 0, edges = 0;
    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace pgabb {

// Device bytes a request may hold at its peak: the build's sort buffers
// (two 8-byte keys per pair plus flags), the CSR and the blocks.
// Requests of at least this many input pairs are partitioned into 8 x 8
// blocks unless the options fix p: on R-MAT graphs of scale 18 - 22 the
// blocks' locality made the counting launch 1.8 - 2.3 times faster than one
// block, at about the same partition time; smaller requests stay one block
// (one task, the shortest partition).
constexpr int64_t kGridPairs = int64_t(1) << 18;
constexpr int32_t kGridP = 8;

int32_t request_grid(const pgabb_tc_options &opt, int32_t n, int64_t m) {
    const int32_t p = opt.p > 0 ? opt.p : (m >= kGridPairs ? kGridP : 1);
    return std::max(1, std::min(p, std::max(1, n)));
}

// Device bytes of a request while it is built and counted: its edge
// copies, sort keys and CSR (per pair) and per-vertex arrays; a grid of
// p > 1 adds the blocks' dense row offsets (about (p + 1) / 2 words per
// vertex) and their split row items.
uint64_t request_bytes(int32_t n, int64_t m, int32_t p) {
    const uint64_t per_vertex = 48 + (p > 1 ? 2 * static_cast<uint64_t>(p + 1) + 8 : 0);
    return static_cast<uint64_t>(m) * 40 + static_cast<uint64_t>(n) * per_vertex + (4ull << 20);
}

static void builder_loop(pgabb_server *s, int idx) {
    (void)hipSetDevice(s->device);
    for (;;) {
        Request *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_build.wait(lk, [&] {
                return s->stop || (!s->queue.empty() && s->reserved + s->queue.front()->est <= s->budget);
            });
            if (s->stop && s->queue.empty()) break;
            if (s->queue.empty() || s->reserved + s->queue.front()->est > s->budget) {
                if (s->stop) {
                    // cannot admit more while stopping: fail what is left
                    for (Request *q : s->queue) {
                        q->status = PGABB_ESTATE;
                        q->done = true;
                    }
                    s->queue.clear();
                    s->cv_done.notify_all();
                    break;
                }
                continue;
            }
            r = s->queue.front();
            s->queue.pop_front();
            s->reserved += r->est;
        }
        try {
            pgabb_graph *g = new pgabb_graph();
            r->g = g;
            g->n = r->n;
            g->stream = s->build_streams[idx];
            const int32_t *hs = r->bsrc ? r->bsrc : r->src.data();
            const int32_t *hd = r->bdst ? r->bdst : r->dst.data();
            if (r->m > 0) {
                DArray<int32_t> ds(static_cast<size_t>(r->m), g->stream), dd(static_cast<size_t>(r->m), g->stream);
                PGABB_HIP(hipMemcpyAsync(ds.get(), hs, sizeof(int32_t) * r->m, hipMemcpyHostToDevice, g->stream));
                PGABB_HIP(hipMemcpyAsync(dd.get(), hd, sizeof(int32_t) * r->m, hipMemcpyHostToDevice, g->stream));
                build_graph(g, ds.get(), dd.get(), r->m);
            } else {
                build_graph(g, nullptr, nullptr, 0);
            }
            partition_graph(g, r->p, s->opt.cut_mode == PGABB_CUT_UNIFORM ? PGABB_CUT_UNIFORM : PGABB_CUT_NNZ,
                            nullptr);
            PGABB_HIP(hipStreamSynchronize(g->stream));
            std::vector<int32_t>().swap(r->src);
            std::vector<int32_t>().swap(r->dst);
        } catch (const Error &e) {
            r->status = e.status;
        } catch (...) {
            r->status = PGABB_EDEVICE;
        }
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->ready.push_back(r);
        }
        s->cv_count.notify_one();
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        --s->builders_left;
    }
    s->cv_count.notify_one();
}

static void finish(pgabb_server *s, Request *r) {
    if (r->g) {
        (void)hipStreamSynchronize(r->g->stream);
        delete r->g;
        r->g = nullptr;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    r->t_done = s->now();
    r->done = true;
    s->reserved -= r->est;
    --s->in_flight;
}

static void counter_loop(pgabb_server *s) {
    (void)hipSetDevice(s->device);
    DArray<TaskDesc> dtd;
    DArray<int64_t> dpre;
    DArray<unsigned long long> dcnt;
    PinnedArray<unsigned long long> hcnt;
    StreamTimer ktimer;
    for (;;) {
        std::vector<Request *> batch;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_count.wait(lk, [&] { return !s->ready.empty() || s->builders_left == 0; });
            if (s->ready.empty() && s->builders_left == 0) break;
            batch.assign(s->ready.begin(), s->ready.end());
            s->ready.clear();
        }
        // one launch over every task of every built request in the batch
        std::vector<TaskDesc> td;
        std::vector<int64_t> pre(1, 0);
        std::vector<Request *> live;
        int32_t max_out = 0, max_wk = 0, min_wk = INT32_MAX;
        uint64_t walked = 0, edges = 0;
        for (Request *r : batch) {
            if (r->status != PGABB_OK || !r->g) {
                finish(s, r);
                continue;
            }
            const int32_t slot = static_cast<int32_t>(live.size());
            live.push_back(r);
            pgabb_graph *g = r->g;
            walked += walked_entries(g, orient_of_option(s->opt, nullptr));
            edges += static_cast<uint64_t>(g->m);
            for (const Task &t : g->tasks) {
                td.push_back(make_desc(g, g->arena.get(), t, slot, nullptr));
                pre.push_back(pre.back() + task_items(g, t, orient_of_option(s->opt, nullptr)));
                max_wk = std::max(max_wk, td.back().width_k);
                min_wk = std::min(min_wk, td.back().width_k);
                max_out = std::max(max_out, staged_max(g, t, orient_of_option(s->opt, nullptr)));
            }
        }
        if (live.empty()) {
            s->cv_build.notify_all();
            s->cv_done.notify_all();
            continue;
        }
        try {
            hipStream_t cs = s->count_stream;
            const int32_t T = static_cast<int32_t>(td.size());
            const size_t L = live.size();
            if (dcnt.size() < L + kLaunchQueueWords) {
                dcnt.reset(std::max<size_t>(2 * L + kLaunchQueueWords, 64), cs);
                hcnt.reset(dcnt.size());
            }
            if (T > 0) {
                if (dtd.size() < static_cast<size_t>(T)) dtd.reset(std::max<size_t>(2 * T, 256), cs);
                if (dpre.size() < static_cast<size_t>(T) + 1) dpre.reset(std::max<size_t>(2 * T + 2, 256), cs);
                // staged through pinned blocks so the copies do not stall the host
                Staged<TaskDesc> htd(T, cs);
                Staged<int64_t> hpre(static_cast<size_t>(T) + 1, cs);
                std::copy(td.begin(), td.end(), htd.get());
                std::copy(pre.begin(), pre.end(), hpre.get());
                PGABB_HIP(hipMemcpyAsync(dtd.get(), htd.get(), htd.bytes(), hipMemcpyHostToDevice, cs));
                PGABB_HIP(hipMemcpyAsync(dpre.get(), hpre.get(), hpre.bytes(), hipMemcpyHostToDevice, cs));
            }
            PGABB_HIP(hipMemsetAsync(dcnt.get(), 0, sizeof(unsigned long long) * (L + kLaunchQueueWords), cs));
            if (T > 0) {
                CountArgs a;
                a.tasks = dtd.get();
                a.item_pre = dpre.get();
                a.ntasks = T;
                a.grab = s->opt.rows_per_grab > 0 ? s->opt.rows_per_grab : default_grab(pre.back(), walked);
                a.orient = orient_of_option(s->opt, nullptr);
                a.total = pre.back();
                a.counts = dcnt.get();
                a.next = dcnt.get() + L;
                const LaunchKind lk = launch_kind(s->opt.kernel, max_out, max_wk, min_wk);
                ktimer.start(cs);
                launch_tc_tasks(a, lk, s->opt.waves_per_block > 0 ? s->opt.waves_per_block : 4, cs, 0,
                                s->opt.unroll);
                ktimer.stop(cs);
            }
            PGABB_HIP(hipMemcpyAsync(hcnt.get(), dcnt.get(), sizeof(unsigned long long) * L, hipMemcpyDeviceToHost, cs));
            PGABB_HIP(hipStreamSynchronize(cs));
            if (T > 0) {
                const double kms = ktimer.ms();
                std::lock_guard<std::mutex> lk(s->mu);
                s->kernel_ms += kms;
                s->walked += walked;
                s->edges += edges;
            }
            for (size_t q = 0; q < L; ++q) live[q]->count = hcnt[q];
            ++s->launches;
        } catch (const Error &e) {
            for (Request *r : live) r->status = e.status;
        } catch (...) {
            for (Request *r : live) r->status = PGABB_EDEVICE;
        }
        for (Request *r : live) finish(s, r);
        s->cv_build.notify_all();
        s->cv_done.notify_all();
    }
}

}  // namespace pgabb

using namespace pgabb;

#define PGABB_API extern "C" __attribute__((visibility("default")))

PGABB_API pgabb_status pgabb_server_create(uint64_t device_budget_bytes, const pgabb_tc_options *opts,
                                           pgabb_server **out) {
    if (!out) return capture_status(Error{PGABB_EINVAL, "out is NULL"});
    *out = nullptr;
    if (device_budget_bytes == 0) return capture_status(Error{PGABB_EINVAL, "budget is 0"});
    if (opts && (opts->p < 0 || opts->p > 64))
        return capture_status(Error{PGABB_EINVAL, "p must lie in [0, 64]"});
    pgabb_server *s = nullptr;
    try {
        s = new pgabb_server();
        s->budget = device_budget_bytes;
        if (opts) s->opt = *opts;
        PGABB_HIP(hipGetDevice(&s->device));
        const int nb = s->opt.num_streams > 0 ? std::min(s->opt.num_streams, 8) : 2;
        s->build_streams.assign(nb, nullptr);
        for (auto &bs : s->build_streams) PGABB_HIP(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
        PGABB_HIP(hipStreamCreateWithFlags(&s->count_stream, hipStreamNonBlocking));
        s->builders_left = nb;
        for (int q = 0; q < nb; ++q) s->builders.emplace_back(builder_loop, s, q);
        s->counter = std::thread(counter_loop, s);
        *out = s;
        return capture_status(Error{PGABB_OK, ""});
    } catch (const Error &e) {
        if (s) {
            for (auto bs : s->build_streams)
                if (bs) (void)hipStreamDestroy(bs);
            if (s->count_stream) (void)hipStreamDestroy(s->count_stream);
            delete s;
        }
        return capture_status(e);
    }
}

PGABB_API pgabb_status pgabb_server_submit(pgabb_server *s, int32_t n, int64_t m, const int32_t *src,
                                           const int32_t *dst, uint64_t *ticket) {
    if (!s || !ticket) return capture_status(Error{PGABB_EINVAL, "NULL argument"});
    if (n < 0 || m < 0) return capture_status(Error{PGABB_EINVAL, "n < 0 or m < 0"});
    if (m > 0 && (!src || !dst)) return capture_status(Error{PGABB_EINVAL, "src or dst is NULL"});
    // ids are checked on the device when the request is built (a host pass
    // over every pair would serialise arrivals behind it)
    const int32_t grid = request_grid(s->opt, n, m);
    const uint64_t est = request_bytes(n, m, grid);
    if (est > s->budget) return capture_status(Error{PGABB_EBUDGET, "request exceeds the device budget"});
    auto r = std::make_unique<Request>();
    r->n = n;
    r->m = m;
    r->est = est;
    r->p = grid;
    if (s->opt.flags & PGABB_SERVER_BORROW) {
        r->bsrc = src;
        r->bdst = dst;
    } else if (m > 0) {
        r->src.assign(src, src + m);
        r->dst.assign(dst, dst + m);
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return capture_status(Error{PGABB_ESTATE, "server is stopping"});
        r->ticket = s->next_ticket++;
        r->t_submit = s->now();
        *ticket = r->ticket;
        s->queue.push_back(r.get());
        ++s->in_flight;
        s->all.emplace(r->ticket, std::move(r));
    }
    s->cv_build.notify_one();
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API pgabb_status pgabb_server_poll(pgabb_server *s, uint64_t ticket, int32_t *done, uint64_t *count) {
    if (!s || !done) return capture_status(Error{PGABB_EINVAL, "NULL argument"});
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return capture_status(Error{PGABB_EINVAL, "unknown ticket"});
    Request *r = it->second.get();
    *done = r->done ? 1 : 0;
    if (count) *count = r->done ? r->count : PGABB_COUNT_ERROR;
    if (r->done && r->status != PGABB_OK)
        return capture_status(Error{r->status, "request failed"});
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API pgabb_status pgabb_server_times(pgabb_server *s, uint64_t ticket, double *t_submit, double *t_done) {
    if (!s) return capture_status(Error{PGABB_EINVAL, "server is NULL"});
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return capture_status(Error{PGABB_EINVAL, "unknown ticket"});
    Request *r = it->second.get();
    if (t_submit) *t_submit = r->t_submit;
    if (t_done) *t_done = r->done ? r->t_done : 0.0;
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API pgabb_status pgabb_server_drain(pgabb_server *s) {
    if (!s) return capture_status(Error{PGABB_EINVAL, "server is NULL"});
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->in_flight == 0; });
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API double pgabb_server_now(const pgabb_server *s) { return s ? s->now() : 0.0; }

PGABB_API pgabb_status pgabb_server_stats(const pgabb_server *s, uint64_t *launches) {
    if (!s) return capture_status(Error{PGABB_EINVAL, "server is NULL"});
    if (launches) *launches = s->launches;
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API pgabb_status pgabb_server_kernel_stats(pgabb_server *s, double *kernel_ms, uint64_t *walked,
                                                 uint64_t *edges) {
    if (!s) return capture_status(Error{PGABB_EINVAL, "server is NULL"});
    std::lock_guard<std::mutex> lk(s->mu);
    if (kernel_ms) *kernel_ms = s->kernel_ms;
    if (walked) *walked = s->walked;
    if (edges) *edges = s->edges;
    return capture_status(Error{PGABB_OK, ""});
}

PGABB_API void pgabb_server_destroy(pgabb_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_build.notify_all();
    s->cv_count.notify_all();
    for (auto &t : s->builders)
        if (t.joinable()) t.join();
    if (s->counter.joinable()) s->counter.join();
    for (auto bs : s->build_streams) (void)hipStreamDestroy(bs);
    (void)hipStreamDestroy(s->count_stream);
    delete s;
}
