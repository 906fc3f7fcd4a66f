// A count that allocates nothing, for callers that cannot allocate memory
// during the call (code under stream capture, tight serving loops, hosts
// that forbid allocation after start-up).
//
// The in-core count needs device scratch beyond the graph's own arrays: the
// task descriptors, the prefix of work items per task, one counter per task
// and the work-queue counters.  Here they live in one file-scope device
// array of kScratchBytes.  Each GPU holds its own copy of it (at its own
// address, looked up once per device with hipGetSymbolAddress) until the
// process ends.  Every call on a GPU uses that GPU's copy, so calls that
// overlap on one GPU race; the counters are cleared by a fill kernel at the
// start of each call, and the rest of the array keeps the last call's
// contents.
//
// The host side stages the descriptors in thread-local vectors that grow to
// the largest graph seen on the thread; no device or pinned memory is
// allocated, and no HIP allocation routine is called.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "count.hpp"
#include "graph.hpp"

namespace pgabb {

namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's copy of `scratch`.  In host
// code the array's name only stands for the symbol; kernels must be given
// this address.
unsigned char *scratch_on_current_device() {
    int dev = 0;
    PGABB_HIP(hipGetDevice(&dev));
    PGABB_REQUIRE(dev >= 0 && dev < kMaxDevices, PGABB_EDEVICE, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        PGABB_REQUIRE(e == hipSuccess && p, PGABB_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[dev]);
}

__global__ void k_zero_counts(unsigned long long *p, int64_t n) {
    for (int64_t q = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; q < n; q += int64_t(gridDim.x) * blockDim.x)
        p[q] = 0ull;
}

size_t round_up(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// Scratch bytes a count of T tasks needs: descriptors, item prefix, then the
// per-task and work-queue counters, each region 256-byte aligned.
size_t noalloc_need(int64_t T) {
    return round_up(sizeof(TaskDesc) * static_cast<size_t>(T)) + round_up(sizeof(int64_t) * static_cast<size_t>(T + 1)) +
           round_up(sizeof(unsigned long long) * static_cast<size_t>(T + kLaunchQueueWords));
}

uint64_t count_noalloc(pgabb_graph *g, const pgabb_tc_options &opt) {
    PGABB_REQUIRE(g->p > 0, PGABB_ESTATE, "the graph is not partitioned (partition it before this call)");
    PGABB_REQUIRE(!g->blocks_on_host, PGABB_ESTATE,
                  "the graph's blocks are held in host memory; this call counts device-resident blocks only");
    PGABB_REQUIRE(opt.p == 0 || (opt.p == g->p && opt.cut_mode == g->cut_mode), PGABB_ESTATE,
                  "options ask for another partition than the graph has (repartitioning allocates)");
    PGABB_REQUIRE(!(opt.flags & (PGABB_OPT_STREAM | PGABB_OPT_HYBRID)), PGABB_EINVAL,
                  "streamed and hybrid counts are not available without allocation");
    const uint64_t block_bytes = static_cast<uint64_t>(g->arena_words) * sizeof(int32_t);
    PGABB_REQUIRE(!opt.device_cap_bytes || block_bytes <= opt.device_cap_bytes, PGABB_EINVAL,
                  "the blocks exceed device_cap_bytes (a streamed count allocates)");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = g->stream;
    const int32_t T = static_cast<int32_t>(g->tasks.size());
    const size_t need = noalloc_need(T);
    PGABB_REQUIRE(need <= kScratchBytes, PGABB_EINVAL,
                  "%d tasks need %zu bytes of scratch; the allocation-free count holds %zu (use a smaller p)", T,
                  need, kScratchBytes);
    uint64_t total = 0;
    g->h2d_bytes = 0;
    g->host_tasks = 0;
    g->host_work_share = 0;
    g->kernel_launches = 0;
    g->t_kernel_ms = 0;
    if (T > 0) {
        unsigned char *base = scratch_on_current_device();
        TaskDesc *dtd = reinterpret_cast<TaskDesc *>(base);
        int64_t *dpre = reinterpret_cast<int64_t *>(base + round_up(sizeof(TaskDesc) * T));
        unsigned long long *dcnt = reinterpret_cast<unsigned long long *>(
            base + round_up(sizeof(TaskDesc) * T) + round_up(sizeof(int64_t) * (T + 1)));

        const int orient = orient_of_option(opt, g);
        g->walked_columns = orient == kOrientCol;
        thread_local std::vector<TaskDesc> td;
        thread_local std::vector<int64_t> pre;
        thread_local std::vector<unsigned long long> hcnt;
        td.resize(T);
        pre.assign(static_cast<size_t>(T) + 1, 0);
        int32_t max_wk = 0, min_wk = INT32_MAX, max_st = 0;
        for (int32_t t = 0; t < T; ++t) {
            td[t] = make_desc(g, g->arena.get(), g->tasks[t], t, nullptr);
            pre[t + 1] = pre[t] + task_items(g, g->tasks[t], orient);
            max_wk = std::max(max_wk, td[t].width_k);
            min_wk = std::min(min_wk, td[t].width_k);
            max_st = std::max(max_st, staged_max(g, g->tasks[t], orient));
        }
        PGABB_HIP(hipMemcpyAsync(dtd, td.data(), sizeof(TaskDesc) * T, hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(dpre, pre.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice, s));
        const int64_t ncnt = static_cast<int64_t>(T) + kLaunchQueueWords;
        k_zero_counts<<<static_cast<unsigned>(std::min<int64_t>((ncnt + 255) / 256, 1024)), 256, 0, s>>>(dcnt, ncnt);
        PGABB_HIP(hipGetLastError());

        CountArgs a;
        a.tasks = dtd;
        a.item_pre = dpre;
        a.ntasks = T;
        a.total = pre[T];
        a.counts = dcnt;
        a.next = dcnt + T;
        const uint64_t walked =
            static_cast<uint64_t>(static_cast<double>(walked_entries(g, orient)) * g->task_share);
        a.grab = opt.rows_per_grab > 0 ? opt.rows_per_grab : default_grab(pre[T], walked);
        a.orient = orient;
        const LaunchKind lk = launch_kind(opt.kernel, max_st, max_wk, min_wk);
        const int waves = opt.waves_per_block > 0 ? opt.waves_per_block : 4;
        launch_tc_tasks(a, lk, waves, s, 0, opt.unroll);

        hcnt.resize(T);
        PGABB_HIP(hipMemcpyAsync(hcnt.data(), dcnt, sizeof(unsigned long long) * T, hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        g->task_counts.assign(hcnt.begin(), hcnt.end());
        g->kernel_launches = lk.nparts;
        for (int32_t t = 0; t < T; ++t) total += hcnt[t];
    } else {
        g->task_counts.clear();
    }
    g->t_count_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return total;
}

}  // namespace pgabb
