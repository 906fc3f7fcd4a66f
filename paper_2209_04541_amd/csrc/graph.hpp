// The graph object: oriented CSR over degree ranks, its 2-D block partition
// and the task (block-list) table.
#pragma once

#include <memory>
#include <vector>

#include "common.hpp"

namespace pgabb {

// One block A_ij of the p x p grid, stored as a chunk of int32 words:
//   [ rptr  : width + 1   ]  dense row offsets over the stripe's row range,
//                            relative to the block's first column entry
//   [ items : 2 * nitems  ]  work items (u, c): local row u, and c, the index
//                            of a run of at most kSplitV entries of row u;
//                            increasing in (u, c)
//   [ col   : nnz         ]  local column ids (rank - base of stripe j), each
//                            row's run increasing
// Local row ids are rank - base_i, where base_i is stripe i's first rank that
// can own an edge (isolated vertices rank lowest and own none).  One chunk is
// the unit of host<->device movement.  Splitting long rows into items bounds
// the work of one item when the block plays A_ij in a task.
constexpr int32_t kSplitV = 32;

struct BlockInfo {
    int32_t i = 0, j = 0;
    int32_t width = 0;   // rows of the dense range of stripe i
    int32_t nitems = 0;  // work items (rows split into runs of kSplitV)
    int64_t nnz = 0;
    int64_t chunk_off = 0;  // int32 words from the arena start
    int64_t chunk_len = 0;  // int32 words
};

inline int64_t block_chunk_words(int32_t width, int32_t nitems, int64_t nnz) {
    return static_cast<int64_t>(width) + 1 + 2 * static_cast<int64_t>(nitems) + nnz;
}

// Device view of one block.
struct BlockRef {
    const int32_t *rptr;
    const int32_t *items;
    const int32_t *col;
    int32_t nitems;
    int32_t width;
};

// One task: the block-list (A_ij, A_ik, A_jk).
struct Task {
    int32_t i, j, k;
    int32_t bij, bik, bjk;  // indices into the block table
    int64_t weight;         // paper default estimate: edges in the block-list
};

// Device descriptor of a task as the counting kernel reads it.
struct TaskDesc {
    BlockRef ij, ik, jk;
    int32_t width_k;  // columns of stripe k
    int32_t slot;     // index of the task's counter
};

}  // namespace pgabb

struct pgabb_graph {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t flags = 0;

    int32_t n = 0;
    int64_t m_input = 0;
    int64_t m = 0;  // m'
    int nb = 1;     // bits per vertex id in packed keys
    int64_t isolated = 0;
    int32_t max_out = 0;
    uint64_t probe_work = 0;

    pgabb::DArray<int64_t> row_off;  // n + 1
    pgabb::DArray<int32_t> col;      // m'
    pgabb::DArray<int32_t> rank;     // n: rank of input id
    pgabb::DArray<int32_t> outdeg;   // n: oriented row lengths (by rank)

    // partition
    int32_t p = 0;
    std::vector<int32_t> cuts;  // p + 1
    std::vector<int32_t> base;  // p: first rank of the dense row range
    std::vector<pgabb::BlockInfo> blocks;
    std::vector<int32_t> block_of;  // p * p -> block index or -1
    int64_t arena_words = 0;
    pgabb::DArray<int32_t> arena;        // device block storage (in-core)
    pgabb::PinnedArray<int32_t> host_arena;  // host block store (streamed)
    bool blocks_on_host = false;
    std::vector<pgabb::Task> tasks;
    std::vector<uint64_t> task_counts;

    double t_build_ms = 0, t_partition_ms = 0, t_count_ms = 0, t_kernel_ms = 0;
    int64_t kernel_launches = 0;
    uint64_t h2d_bytes = 0;
};

namespace pgabb {

hipStream_t library_stream();

void build_graph(pgabb_graph *g, const int32_t *src_dev, const int32_t *dst_dev, int64_t m);
void partition_graph(pgabb_graph *g, int32_t p, int32_t cut_mode, const int32_t *cuts_host);
uint64_t count_graph(pgabb_graph *g, const pgabb_tc_options &opt);

}  // namespace pgabb
