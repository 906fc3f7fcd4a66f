// The counting kernel over the work items of a list of tasks (block-lists).
#pragma once

#include "count.hpp"
#include "graph.hpp"
#include "tc_device.hpp"
#include "wave.hpp"

namespace pgabb {

// Item g of the launch: task t = the task whose item range holds g; inside the
// task, items are taken from the end of A_ij's item list (highest ranks,
// the heaviest rows under the degree order) towards its start.  ORIENT picks
// the row items (stage A_ik[u]) or the column items (stage A_jk[v]).
//
// A wave takes up to 64 consecutive items per grab.  Lane l loads item
// g0 + l's record and the bounds of its staged list, so the headers of the
// whole grab arrive in two round trips; items whose staged list is empty
// (common when p is large) are dropped by one ballot, and the wave then
// walks the others one after another.
//
// With FILTER, only the items whose staged list length lies in
// (a.stage_lo, a.stage_hi] are counted (a launch split by list length).
template <int MODE, int LDS_WORDS, int WAVES, int UNROLL, int ORIENT, bool FILTER = false>
__global__ __launch_bounds__(WAVES * 64) void k_tc_tasks(CountArgs a) {
    __shared__ int32_t lds_all[WAVES][LDS_WORDS];
    __shared__ int32_t own_all[WAVES][UNROLL * kWave];  // the walk's list positions
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    int32_t *lds = lds_all[w];
    int32_t *own = own_all[w];
#pragma unroll
    for (int q = 0; q < UNROLL; ++q) own[q * kWave + lane] = 0;
    wave_lds_sync();
    if (MODE == kModeBitmap) {
        for (int q = lane; q < LDS_WORDS; q += kWave) lds[q] = 0;
        wave_lds_sync();
    }
    const gptr<TaskDesc> tasks = as_global(a.tasks);
    const gptr<int64_t> item_pre = as_global(a.item_pre);
    const int64_t units = (a.total + a.grab - 1) / a.grab;
    const int home = static_cast<int>(blockIdx.x % kQueues);
    for (int qi = 0; qi < kQueues; ++qi) {
        const int q = (home + qi) % kQueues;
        for (;;) {
            unsigned long long c = 0;
            if (lane == 0) c = atomicAdd(&a.next[q * kQueueStride], 1ull);
            c = shfl_t(c, 0);
            const int64_t unit = static_cast<int64_t>(c) * kQueues + q;
            if (unit >= units) break;
            const int64_t g0 = unit * a.grab;
            const int64_t g1 = min(g0 + a.grab, a.total);  // g1 - g0 <= 64
            int32_t lo = 0, hi = a.ntasks - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (item_pre[mid] <= g0) lo = mid;
                else hi = mid - 1;
            }
            const int32_t t0 = __builtin_amdgcn_readfirstlane(lo);

            // ---- per-lane item headers
            const int64_t gl = g0 + lane;
            const bool lv = gl < g1;
            int32_t tl = t0;
            for (int32_t tt = t0;; ++tt) {  // task ends inside the grab
                const int64_t end = item_pre[tt + 1];
                if (end >= g1) break;
                if (gl >= end) tl = tt + 1;
            }
            int32_t x = 0, b = 0, e = 0, sb = 0, se = 0;
            if (lv) {
                const int64_t t_begin = item_pre[tl];
                const int32_t *items = ORIENT == kOrientRow ? tasks[tl].ij.items : tasks[tl].ij.citems;
                const int64_t n = ORIENT == kOrientRow ? tasks[tl].ij.nitems : tasks[tl].ij.ncitems;
                const gptr<int32_t> r = as_global(items) + kItemWords * (n - 1 - (gl - t_begin));
                x = r[0];
                b = r[1];
                e = r[2];
                const gptr<int32_t> srp = as_global(ORIENT == kOrientRow ? tasks[tl].ik.rptr : tasks[tl].jk.rptr);
                sb = srp[x];
                se = srp[x + 1];
            }
            bool take = lv && se > sb && e > b;
            if (FILTER) take = take && se - sb > a.stage_lo && se - sb <= a.stage_hi;
            uint64_t todo = __ballot(take);

            // ---- walk the non-empty items; counts go to each item's task
            int32_t cur = -1;
            uint32_t cnt = 0;
            auto flush = [&]() {
                if (cur < 0) return;
                const unsigned long long sum = wave_sum(static_cast<unsigned long long>(cnt));
                if (lane == 0 && sum) atomicAdd(&a.counts[tasks[cur].slot], sum);
                cnt = 0;
            };
            // items with tiny staged lists: together, task by task
            uint64_t tiny = todo & __ballot(se - sb <= kTinyCap);
            todo &= ~tiny;
            while (tiny) {
                const int32_t t = __builtin_amdgcn_readlane(tl, __builtin_ctzll(tiny));
                const uint64_t mt = tiny & __ballot(tl == t);
                tiny &= ~mt;
                if (t != cur) {
                    flush();
                    cur = t;
                }
                const auto &T = tasks[t];
                if (ORIENT == kOrientRow)
                    cnt += tiny_items<UNROLL>(mt, b, e, sb, se, T.ik.col, T.ij.col, T.jk.rptr, T.jk.col, own, lane);
                else
                    cnt += tiny_items<UNROLL>(mt, b, e, sb, se, T.jk.col, T.ij.crow, T.ik.rptr, T.ik.col, own, lane);
            }
            // items with small staged lists and few walked lists: packed into
            // one LDS table, task by task, while their staged entries fit
            constexpr int kPackSlots = HashLds<LDS_WORDS>::kTableCap < 4 * HashLds<LDS_WORDS>::kFilterCap
                                           ? HashLds<LDS_WORDS>::kTableCap
                                           : 4 * HashLds<LDS_WORDS>::kFilterCap;
            uint64_t small = todo & __ballot(se - sb <= kPackS && e - b <= kPackLists);
            todo &= ~small;
            while (small) {
                const int32_t t = __builtin_amdgcn_readlane(tl, __builtin_ctzll(small));
                const uint64_t mt = small & __ballot(tl == t);
                const int32_t ns = ((mt >> lane) & 1ull) ? se - sb : 0;
                const uint64_t mp = mt & __ballot(wave_inclusive_scan(ns) <= kPackSlots / 2);
                small &= ~mp;
                if (t != cur) {
                    flush();
                    cur = t;
                }
                const auto &T = tasks[t];
                if (ORIENT == kOrientRow)
                    cnt += packed_items<UNROLL, LDS_WORDS>(mp, b, e, sb, se, T.ik.col, T.ij.col, T.jk.rptr, T.jk.col,
                                                           lds, own, lane);
                else
                    cnt += packed_items<UNROLL, LDS_WORDS>(mp, b, e, sb, se, T.jk.col, T.ij.crow, T.ik.rptr,
                                                           T.ik.col, lds, own, lane);
            }
            while (todo) {
                const int l = __builtin_ctzll(todo);
                todo &= todo - 1;
                const int32_t t = __builtin_amdgcn_readlane(tl, l);
                if (t != cur) {
                    flush();
                    cur = t;
                }
                const int32_t bl = __builtin_amdgcn_readlane(b, l);
                const int32_t el = __builtin_amdgcn_readlane(e, l);
                const int32_t sbl = __builtin_amdgcn_readlane(sb, l);
                const int32_t sel = __builtin_amdgcn_readlane(se, l);
                const auto &T = tasks[t];
                if (ORIENT == kOrientRow)
                    cnt += tc_item_core<MODE, LDS_WORDS, UNROLL>(T.ik.col, sbl, sel, T.jk.rptr, T.jk.col, T.ij.col,
                                                                 bl, el, T.width_k, lds, own);
                else
                    cnt += tc_item_core<MODE, LDS_WORDS, UNROLL>(T.jk.col, sbl, sel, T.ik.rptr, T.ik.col, T.ij.crow,
                                                                 bl, el, T.width_k, lds, own);
            }
            flush();
        }
    }
}

}  // namespace pgabb
