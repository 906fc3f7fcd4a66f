// The graph object: oriented CSR over degree ranks, its 2-D block partition
// and the task (block-list) table.
#pragma once

#include <array>
#include <memory>
#include <vector>

#include "common.hpp"

namespace pgabb {

// One block A_ij of the p x p grid, stored as a chunk of int32 words holding
// the block and its transpose:
//   [ items  : 3 * nitems   ]  row work items (u, b, e): local row u and the
//                              run [b, e) of at most kSplitV of its entries,
//                              as offsets into `col`
//   [ rptr   : width + 1    ]  dense row offsets over stripe i's row range,
//                              relative to the start of `col`
//   [ col    : nnz          ]  local column ids (rank - base of stripe j)
//   [ citems : 3 * ncitems  ]  column work items (v, b, e), as above per
//                              column, offsets into `crow`
//   [ crow   : nnz          ]  local row ids of each column's entries, in
//                              column order
// Local ids are rank - base_s, where base_s is stripe s's first rank that
// can own an edge (isolated vertices rank lowest and own none).  Items bound
// the work of one wave when the block plays A_ij in a task (rows when the row
// of A_ik is staged, columns when the row of A_jk is staged).  The chunk is
// the unit of host<->device movement, and its order puts what each walk
// reads in one range: a row walk reads items, rptr and col (the edge block's
// row items and ids, the other blocks' rows); a column walk reads rptr, col,
// citems and crow.  The transpose's column offsets are needed only while
// the partition fills the chunk and are not kept.
constexpr int32_t kSplitV = 32;
constexpr int32_t kItemWords = 3;

// Which list of a block-list edge (u, v) is staged in LDS: the row u of A_ik
// (the edge block is walked by rows) or the row v of A_jk (walked by
// columns).  Both count the same common entries.
enum Orient : int { kOrientRow = 0, kOrientCol = 1 };

struct BlockInfo {
    int32_t i = 0, j = 0;
    int32_t width = 0;    // rows of the dense range of stripe i
    int32_t cwidth = 0;   // columns of the dense range of stripe j
    int32_t nitems = 0;   // row work items
    int32_t ncitems = 0;  // column work items
    int32_t max_row = 0;  // longest row of the block
    int32_t nrows = 0;    // non-empty rows
    int32_t ncols = 0;    // non-empty columns
    int64_t nnz = 0;
    int64_t chunk_off = 0;  // int32 words from the arena start
    int64_t chunk_len = 0;  // int32 words
    int64_t off_items() const { return chunk_off; }
    int64_t off_rptr() const { return off_items() + kItemWords * static_cast<int64_t>(nitems); }
    int64_t off_col() const { return off_rptr() + width + 1; }
    int64_t off_citems() const { return off_col() + nnz; }
    int64_t off_crow() const { return off_citems() + kItemWords * static_cast<int64_t>(ncitems); }
    int64_t end() const { return off_crow() + nnz; }
    // The words of the chunk a walk reads: [walk_lo, walk_hi) (kOrientRow:
    // items, rptr, col; kOrientCol: rptr, col, citems, crow).
    int64_t walk_lo(int orient) const { return orient == kOrientCol ? off_rptr() : off_items(); }
    int64_t walk_hi(int orient) const { return orient == kOrientCol ? end() : off_citems(); }
};

// Device view of one block.
struct BlockRef {
    const int32_t *rptr;
    const int32_t *items;
    const int32_t *col;
    const int32_t *citems;
    const int32_t *crow;
    int32_t nitems;
    int32_t ncitems;
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
    uint64_t probe_work = 0;      // sum over oriented edges (x, y) of |N+(y)|
    uint64_t probe_work_col = 0;  // entries column walks read under the current cuts
    int64_t walked_columns = 0;   // the last count walked columns
    double task_share = 1.0;      // work items of `tasks` over those of all
                                  // tasks (below 1 while a shard is counted)

    pgabb::DArray<int64_t> row_off;  // n + 1
    pgabb::DArray<int32_t> col;      // m'
    pgabb::DArray<int32_t> rank;     // n: rank of input id
    pgabb::DArray<int32_t> outdeg;   // n: oriented row lengths (by rank)
    pgabb::DArray<int32_t> indeg;    // n: oriented column lengths (by rank)

    // partition
    int32_t p = 0;
    int32_t cut_mode = -1;      // PGABB_CUT_* of the partition, -1 for caller cuts
    std::vector<int32_t> cuts;  // p + 1
    std::vector<int32_t> base;  // p: first rank of the dense row range
    std::vector<pgabb::BlockInfo> blocks;
    std::vector<int32_t> block_of;  // p * p -> block index or -1
    int64_t arena_words = 0;
    pgabb::DArray<int32_t> arena;        // device block storage (in-core)
    pgabb::PinnedArray<int32_t> host_arena;  // host block store (streamed)
    bool blocks_on_host = false;
    uint64_t host_store_cap = 0;  // device cap of the streamed count that moved the blocks to the host
    std::vector<pgabb::Task> tasks;
    std::vector<uint64_t> task_counts;
    std::vector<std::array<int32_t, 4>> quads;  // block 4-lists of the last 4-clique count
    std::vector<uint64_t> quad_counts;          // and their 4-cliques

    double t_build_ms = 0, t_partition_ms = 0, t_count_ms = 0, t_kernel_ms = 0;
    // events around the last partition; t_partition_ms is read from them
    // once they have passed (partitioning returns before its last kernels)
    std::unique_ptr<pgabb::StreamTimer> part_timer;
    bool part_time_pending = false;
    int64_t kernel_launches = 0;
    uint64_t h2d_bytes = 0;
    int64_t host_tasks = 0;        // tasks the host kernel counted in the last count
    double host_work_share = 0;    // their share of the tasks' estimated work
    double t_tune_ms = 0;          // tuning time of the last autotuned count of several graphs
};

namespace pgabb {

hipStream_t library_stream();

void build_graph(pgabb_graph *g, const int32_t *src_dev, const int32_t *dst_dev, int64_t m);
void partition_graph(pgabb_graph *g, int32_t p, int32_t cut_mode, const int32_t *cuts_host);
uint64_t count_graph(pgabb_graph *g, const pgabb_tc_options &opt);
// Partition g as a count with opt requires (see pgabb_tc_options.p).
void ensure_partition(pgabb_graph *g, const pgabb_tc_options &opt);
// Shard of each task when the tasks are split over nshards devices.
std::vector<int32_t> task_shards(const pgabb_graph *g, int32_t nshards);
// Triangles containing each oriented edge, into out[m'] (device or host
// memory); returns the triangle count.
uint64_t edge_support(pgabb_graph *g, uint32_t *out, bool out_on_device);
// In-edges of every vertex of the oriented graph: in_off (n + 1 offsets from
// the kept in-degrees) and in_pos (the CSR positions of the edges, grouped by
// their higher end, each group ascending in the lower end).
void in_edges(pgabb_graph *g, DArray<int64_t> &in_off, DArray<uint32_t> &in_pos);
// Triangles at each vertex, by input id, into out[n] (device or host
// memory); returns the triangle count.
uint64_t vertex_counts(pgabb_graph *g, uint64_t *out, bool out_on_device);
// Edges of the k-truss: keep[e] = 1 for the oriented CSR positions left
// (keep may be null); returns their number.
int64_t ktruss(pgabb_graph *g, int32_t k, uint8_t *keep, bool on_device, int32_t *rounds);
// Sets of four pairwise adjacent vertices.
// device_cap_bytes > 0: the blocks are streamed from the pinned host store
// (moved there first if needed) through a block cache of at most that many
// bytes; 0: in device memory, or streamed under the cap of the count that
// moved them to the host.
uint64_t four_cliques(pgabb_graph *g, uint64_t device_cap_bytes);
// Moves the device block arena to the pinned host store (once per partition).
void move_blocks_to_host(pgabb_graph *g);
// Connected components by Shiloach-Vishkin over the device blocks:
// label[v] = smallest input id of v's component; returns the number of
// components.
int64_t components(pgabb_graph *g, int32_t *label, bool on_device, int32_t *iterations);
// PageRank over the device blocks (ranks by input id); returns the
// iterations run.
int32_t pagerank(pgabb_graph *g, double damping, double tol, int32_t max_iter, double *ranks, bool on_device,
                 double *last_err);
// Counts of several graphs, in one launch where their blocks are in device
// memory (tune: launch shape from the autotuner).
void count_graphs(pgabb_graph *const *gs, int64_t G, const pgabb_tc_options &opt, bool tune, uint64_t *counts);
// The in-core count with its scratch in a fixed device array (noalloc.cpp).
uint64_t count_noalloc(pgabb_graph *g, const pgabb_tc_options &opt);
size_t noalloc_scratch_bytes();
// Count only the tasks task_shards deals to `shard`.
uint64_t count_shard(pgabb_graph *g, const pgabb_tc_options &opt, int32_t shard, int32_t nshards);

}  // namespace pgabb
