// Host-side interface of the counting kernels.
#pragma once

#include "graph.hpp"

namespace pgabb {

// Work queues of a counting launch: grab units are dealt round-robin to
// kQueues counters; a workgroup starts on queue blockIdx % kQueues (its XCD
// under round-robin dispatch) and moves on to the others once it is empty.
// (Measured on R-MAT scale 20 at p = 8 and scale 24 at p = 32: one
// contiguous range of units per queue, which keeps each XCD's waves on
// neighbouring items and their blocks in its own L2, made the kernel 15 %
// and 7 % slower -- the heaviest items all sit in one queue -- and runs of 4
// to 256 units per queue were within 1 % of round-robin.)
constexpr int kQueues = 8;
// Counters sit 256 bytes apart so no two share a memory channel's line.
constexpr int kQueueStride = 32;
constexpr int kQueueWords = kQueues * kQueueStride;
// Queue counters of one counting launch: one set per part of a launch split
// by staged-list length (at most 3 parts), all cleared before the launch, so
// no clearing runs between the parts.
constexpr int kMaxParts = 3;
constexpr int kLaunchQueueWords = kMaxParts * kQueueWords;

struct CountArgs {
    const TaskDesc *tasks;     // device
    const int64_t *item_pre;   // device, ntasks + 1 prefix of rows per task
    int32_t ntasks;
    int32_t grab;              // items taken per counter increment
    int64_t total;             // item_pre[ntasks]
    unsigned long long *counts;  // device, indexed by TaskDesc::slot
    unsigned long long *next;    // device, kLaunchQueueWords (zero before launch); queue q of part r at
                                 // r * kQueueWords + q * kQueueStride
    int32_t orient;              // kOrientRow or kOrientCol (which item lists)
    int32_t stage_lo = 0;        // items whose staged list has more than stage_lo
    int32_t stage_hi = INT32_MAX;  // and at most stage_hi entries
};

int choose_lds_words(int32_t mode, int32_t max_stage_len, int32_t max_width_k);
// Kernel template (staging kind) and LDS words per wave of a counting launch,
// from the kernel option, the longest staged list and the widths of stripe k
// over the launch's tasks.  When the longest staged list needs a larger
// hash table than the 1280-word region holds, the launch is split by staged
// list length into one launch per LDS class: part q takes the items whose
// staged list has more than hi[q - 1] (0 for q = 0) and at most hi[q]
// entries.  A wave region sized for a few long lists would otherwise cut
// the waves per CU for all items.
struct LaunchKind {
    int mode;    // part 0 (the only part when nparts == 1)
    int words;
    int nparts = 1;
    int32_t hi[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
    int pmode[3] = {0, 0, 0};
    int pwords[3] = {0, 0, 0};
};
LaunchKind launch_kind(int32_t kernel, int32_t max_out, int32_t max_wk, int32_t min_wk);
// Items per grab from the launch's items and the entries their walks read
// (walked = 0: from the item count alone).
int default_grab(int64_t total_items, uint64_t walked);
// Entries a walk of graph g reads in orientation `orient` (W or W_col).
uint64_t walked_entries(const pgabb_graph *g, int orient);
// kOrientRow or kOrientCol for a count of graph g (g = nullptr: a launch
// over several graphs, which walks columns unless told otherwise).
int orient_of_option(const pgabb_tc_options &opt, const pgabb_graph *g);
int64_t task_items(const pgabb_graph *g, const Task &t, int orient);
// Longest list a task stages (a row of A_jk for column walks, of A_ik for row
// walks).
int32_t staged_max(const pgabb_graph *g, const Task &t, int orient);
// One launch per part (see LaunchKind), part r on the queue counters at
// a.next + r * kQueueWords.
void launch_tc_tasks(const CountArgs &a, const LaunchKind &lk, int waves, hipStream_t s, int grid_override,
                     int unroll);
TaskDesc make_desc(const pgabb_graph *g, const int32_t *arena_base, const Task &t, int32_t slot,
                   const int64_t *chunk_dev_off);
uint64_t count_streamed(pgabb_graph *g, const pgabb_tc_options &opt);
// Entries a task's walk reads plus those its items stage, estimated from
// block sizes (each list length taken as its block's mean).
int64_t task_work_estimate(const pgabb_graph *g, const Task &t, int orient);
// Host kernel: triangles of task t from block chunks in host memory (the
// host store `arena`, laid out as the device arena).
uint64_t host_count_task(const pgabb_graph *g, const int32_t *arena, const Task &t);

}  // namespace pgabb
