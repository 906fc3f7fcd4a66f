/*
 * pgabb.h -- C ABI of a block-partitioned triangle-counting library for
 * AMD Instinct MI355X (gfx950).
 *
 * The operation is the triangle-counting example of PGAbB (Yasar,
 * Rajamanickam, Berry, Catalyurek, "PGAbB: A Block-Based Graph Processing
 * Framework for Heterogeneous Platforms"): count the sets of three mutually
 * adjacent vertices of an undirected graph (Section 3.6).  The graph is made
 * undirected and deduplicated (Section 5.1), its vertices are ordered by
 * degree and each edge is kept once, oriented from lower to higher rank
 * (Section 5.4).  The oriented adjacency matrix is cut by one cut vector on
 * both axes into a p x p grid of blocks (symmetric rectilinear partitioning,
 * Section 4.3), and every block-list (A_ij, A_ik, A_jk), i <= j <= k, is a
 * task: for each edge (u, v) of A_ij it counts the common entries of row u of
 * A_ik and row v of A_jk (Section 3.6, block-list composition and kernel
 * development).  Tasks are weighted by their edge count and run heaviest
 * first (Section 4.1, Section 4.4).
 *
 * Conventions for every entry point:
 *  - Vertex ids are int32 in [0, n); counts are uint64.
 *  - Pointers are host pointers unless a flag or argument name says device.
 *  - Input arrays are borrowed for the duration of the call and copied; the
 *    caller keeps ownership.  Objects returned through an out-parameter are
 *    owned by the caller and released with the matching *_destroy call.
 *  - Every call returns a pgabb_status (pgabb_tc_count returns the count or
 *    PGABB_COUNT_ERROR).  On failure the reason is available from
 *    pgabb_last_error() on the same thread.  Argument errors are detected
 *    before any device work starts.
 *  - Self-loops, repeated pairs and reciprocal pairs are not errors: they
 *    are removed, as the paper's inputs were made undirected and
 *    deduplicated.  Isolated vertices are kept (n is never reduced).
 *  - Calls on one object must not overlap in time; distinct objects may be
 *    used from different threads.
 */
#ifndef PGABB_H
#define PGABB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pgabb_status {
    PGABB_OK = 0,
    PGABB_EINVAL = -1,  /* bad argument: NULL, id out of range, bad p or cuts */
    PGABB_ENOMEM = -2,  /* device or pinned host allocation failed */
    PGABB_EDEVICE = -3, /* a HIP runtime call failed */
    PGABB_ESTATE = -4,  /* call not valid in the object's current state */
    PGABB_EBUDGET = -5  /* request does not fit a server's device budget */
} pgabb_status;

/* Returned by pgabb_tc_count on failure.  No real count reaches it: a graph
 * with m' edges has at most (2 m')^{3/2} / 6 triangles, below 2^50 for any
 * m' < 2^32. */
#define PGABB_COUNT_ERROR UINT64_MAX

/* Flags of pgabb_graph_from_edges. */
#define PGABB_EDGES_ON_DEVICE 0x1u /* src/dst are device pointers */
#define PGABB_ORDER_BY_ID     0x2u /* rank vertices by id instead of degree */

/* Cut modes (pgabb_tc_options.cut_mode, pgabb_partition_ex). */
#define PGABB_CUT_NNZ     0 /* stripes hold equal shares of oriented edges */
#define PGABB_CUT_UNIFORM 1 /* stripes hold equal shares of vertex ids */

/* Intersection kernels (pgabb_tc_options.kernel). */
#define PGABB_KERNEL_AUTO   0 /* chosen per task from list lengths and widths */
#define PGABB_KERNEL_HASH   1 /* staged row in an LDS hash table */
#define PGABB_KERNEL_BITMAP 2 /* staged row in an LDS bitmap over the stripe */
#define PGABB_KERNEL_SEARCH 3 /* binary search in the staged row (no staging) */

/* Option flags. */
#define PGABB_OPT_STREAM    0x1u /* force the host block store + streamer path */
#define PGABB_OPT_PER_GRAPH 0x2u /* batch only: one plain launch per graph, in
                                    order on one stream (the baseline that the
                                    single persistent launch is measured
                                    against) */
#define PGABB_SERVER_BORROW 0x4u /* server only: submitted arrays are borrowed
                                    until the request finishes, not copied */
#define PGABB_OPT_ROWS      0x8u /* walk each edge block by rows: stage the row
                                    of A_ik, probe the rows of A_jk */
#define PGABB_OPT_COLS     0x10u /* walk each edge block by columns: stage the
                                    row of A_jk, probe the rows of A_ik.  With
                                    neither flag a graph count takes the walk
                                    that reads fewer entries (probe_work or
                                    probe_work_col of pgabb_graph_info_t, columns
                                    on a tie) and the server walks columns;
                                    both flags are EINVAL */
#define PGABB_OPT_HYBRID   0x20u /* hybrid host + device count (Section 4.4:
                                    heavy block-lists on the device, light
                                    ones on host threads; Section 3.6's host
                                    kernel).  The blocks are counted from the
                                    pinned host block store (moved there
                                    first if they are on the device): the
                                    device streams windows of the heaviest
                                    remaining tasks while host threads take
                                    the lightest remaining tasks one at a
                                    time, until the two meet (host_permille
                                    = 0), or the host takes a fixed share of
                                    the estimated work (host_permille > 0) */

typedef struct pgabb_tc_options {
    int32_t p;                 /* grid size of the count (Section 4.3): 0 = keep
                                  the graph's partition (p = 1 if it has none);
                                  1 .. 64 = partition with p and cut_mode first
                                  unless the graph already is */
    int32_t cut_mode;          /* PGABB_CUT_*, used when p > 0 */
    int32_t kernel;            /* PGABB_KERNEL_* */
    int32_t num_streams;       /* compute streams of the streamer (0 = 4) */
    uint64_t device_cap_bytes; /* 0 = no cap; otherwise block cache bound */
    uint32_t flags;            /* PGABB_OPT_* */
    int32_t waves_per_block;   /* 2, 4 or 8 waves per workgroup (0 = default) */
    int32_t rows_per_grab;     /* work items a wave takes per work-counter
                                  update, 1..64 (0 = chosen: about 16K walked
                                  entries per grab for in-core graphs and
                                  servers, from the item count when
                                  streaming) */
    int32_t unroll;            /* 64-element chunks of walked lists per load
                                  batch (the next batch loads while one is
                                  probed): 1, 2, 4 or 8 (0 = 2) */
    int32_t host_threads;      /* PGABB_OPT_HYBRID only: host threads that
                                  count the light tasks (0 = one per core,
                                  at most 64) */
    int32_t host_permille;     /* PGABB_OPT_HYBRID only: share of the tasks'
                                  estimated work, per mille, given to the
                                  host threads, lightest tasks first
                                  (0 = chosen from measured rates, see
                                  pgabb_tc_count_ex; 1000 = every task) */
} pgabb_tc_options;

typedef struct pgabb_graph pgabb_graph;

typedef struct pgabb_graph_info_t {
    int64_t n;              /* vertices (as given) */
    int64_t m_input;        /* input pairs */
    int64_t m;              /* undirected distinct non-loop edges m' */
    int64_t isolated;       /* vertices of degree 0 */
    int32_t max_out_degree; /* largest oriented row */
    int32_t p;              /* grid size (0 before partitioning) */
    int64_t num_blocks;     /* non-empty blocks */
    int64_t num_tasks;      /* block-lists with three non-empty blocks */
    uint64_t probe_work;    /* sum over oriented edges (u,v) of |N+(v)|: entries
                               read by row walks (A_jk[v] per edge of A_ij) */
    uint64_t block_bytes;   /* bytes of all block storage */
    uint64_t h2d_bytes;     /* bytes copied host->device by the last count */
    double t_build_ms;      /* device time of the last build phase */
    double t_partition_ms;  /* device time of the last partition (from its
                               first to its last device operation) */
    double t_count_ms;      /* time of the last count (incl. transfers) */
    double t_kernel_ms;     /* device time of the last count's kernels */
    int64_t kernel_launches; /* counting launches of the last count */
    uint64_t probe_work_col; /* entries read by column walks (A_ik[u] for every
                                edge (u,v) of A_ij and k >= j) under the current
                                cuts: sum over oriented edges (u,v) of
                                |{w in N+(u): stripe(w) >= stripe(v)}| */
    int64_t walked_columns;  /* 1 if the last count walked columns, 0 rows */
    int64_t host_tasks;      /* tasks the host kernel counted in the last count
                                (PGABB_OPT_HYBRID; 0 otherwise) */
    double host_work_share;  /* their share of the tasks' estimated work */
    int64_t row_items;       /* work items over all blocks' rows (runs of at
                                most 32 entries of one row of one block) */
    int64_t col_items;       /* the same over the blocks' columns */
    double t_tune_ms;        /* tuning time (grid and launch shape searches or
                                cache look-ups) of the last autotuned
                                pgabb_tc_count_batch that counted this graph */
    uint64_t walk_bytes_rows; /* bytes of the blocks' parts a row walk reads
                                 (row items, row offsets, column ids): what
                                 a streamed count walking rows copies once */
    uint64_t walk_bytes_cols; /* the same for column walks (row offsets,
                                 column ids, column items, row ids) */
} pgabb_graph_info_t;

/*
 * Build a graph from m pairs (src[e], dst[e]), 0 <= id < n.  Cleans the pairs
 * (drops self-loops, merges repeated and reciprocal pairs), ranks vertices by
 * ascending (degree, id) -- or by id with PGABB_ORDER_BY_ID -- and stores the
 * oriented graph in CSR over ranks on the device.
 *   n, m        : n >= 0, m >= 0 (m = 0 gives an edgeless graph)
 *   src, dst    : m ids each; host pointers, or device pointers with
 *                 PGABB_EDGES_ON_DEVICE (read before the call returns)
 *   hip_stream  : hipStream_t for all work on this graph (NULL = the
 *                 library's own stream)
 *   out         : receives the graph (caller-owned)
 * Errors: EINVAL (NULL pointer, n < 0, m < 0, id outside [0, n)),
 * ENOMEM, EDEVICE.
 */
pgabb_status pgabb_graph_from_edges(int32_t n, int64_t m, const int32_t *src,
                                    const int32_t *dst, uint32_t flags, void *hip_stream,
                                    pgabb_graph **out);

/*
 * Cut the oriented graph into a p x p grid with nnz-balanced cuts (stripe s
 * starts at the first row whose CSR offset reaches s * m' / p), then build
 * the blocks and the task list (PGAbB Section 4.3: symmetric rectilinear
 * partition, one cut vector for rows and columns, blocks stored as CSR with
 * local ids; Section 3.6: the block-lists (A_ij, A_ik, A_jk), i <= j <= k,
 * with three non-empty blocks; Section 4.1: tasks weighted by their edges
 * and ordered heaviest first).  1 <= p <= 64 (a narrower range than the
 * paper's, which leaves p open: a long row is split over the stripes by one
 * wave lane per stripe).  Replaces an earlier partition.
 * Errors: EINVAL (NULL, p out of range), ENOMEM, EDEVICE.
 */
pgabb_status pgabb_partition(pgabb_graph *g, int32_t p);

/*
 * As pgabb_partition with a cut mode, or with an explicit host cut vector
 * (cuts != NULL: p + 1 non-decreasing values, cuts[0] = 0, cuts[p] = n,
 * applied to ranks on both axes; empty stripes are allowed).
 */
pgabb_status pgabb_partition_ex(pgabb_graph *g, int32_t p, int32_t cut_mode,
                                const int32_t *cuts);

/*
 * Triangle count with default options: the number of sets of three mutually
 * adjacent vertices (PGAbB Section 3.6), as the sum over every task
 * (A_ij, A_ik, A_jk) and every edge (u, v) of A_ij of the common entries of
 * row u of A_ik and row v of A_jk.  Partitions with p = 1 first if the
 * graph was not partitioned.  Returns PGABB_COUNT_ERROR on failure (the
 * reason is in pgabb_last_error()).
 */
uint64_t pgabb_tc_count(pgabb_graph *g);

/* Triangle count with options (NULL = defaults); result in *count. */
pgabb_status pgabb_tc_count_ex(pgabb_graph *g, const pgabb_tc_options *opts, uint64_t *count);

/*
 * For callers that cannot allocate memory during the call (code under
 * stream capture, tight serving loops, hosts that forbid allocation after
 * start-up): the in-core count of pgabb_tc_count_ex, with its scratch (task
 * descriptors, work-item prefix, per-task and work-queue counters) in a
 * fixed device array of pgabb_tc_count_noalloc_scratch_bytes() bytes (4 MiB)
 * that each GPU the library runs on holds until the process ends.  No device
 * or pinned host memory is allocated and no HIP allocation routine is
 * called; host-side descriptors go through thread-local vectors that grow
 * to the largest graph seen on the calling thread.
 *   g     : partitioned graph whose blocks are in device memory
 *   opts  : as pgabb_tc_count_ex (NULL = defaults); p must be 0 or the
 *           graph's own, streamed and hybrid counts are refused
 *   count : receives the count (PGABB_COUNT_ERROR on failure)
 * Every call on one GPU shares that GPU's array; the counters are cleared at
 * the start of each call, the rest keeps the last call's contents, and calls
 * that overlap on one GPU (from several threads) race.  Per-task counts
 * (pgabb_graph_task_counts) are updated as by pgabb_tc_count_ex.
 * Errors: EINVAL (NULL pointer, bad options, more tasks than the array
 * holds: about 24,900 at 4 MiB, so every grid up to p = 52), ESTATE (graph not partitioned, blocks in
 * host memory, options asking for another partition), EDEVICE.
 */
pgabb_status pgabb_tc_count_noalloc(pgabb_graph *g, const pgabb_tc_options *opts, uint64_t *count);

/* Bytes of the per-GPU scratch array of pgabb_tc_count_noalloc. */
size_t pgabb_tc_count_noalloc_scratch_bytes(void);

/*
 * Count several graph objects (PGAbB Section 3.6's count, per graph; Section
 * 4.4's task-parallel execution over the tasks of all of them):
 * counts[q] for gs[q], q < num_graphs (host array of num_graphs entries).
 * Each graph is partitioned as opts says (see pgabb_tc_options.p).  The
 * tasks of every graph whose blocks are in device memory run in ONE
 * persistent counting launch on the library's stream (after each graph's
 * stream has reached the call); a graph whose blocks are in the host store,
 * or that opts ask to stream or count hybrid, is counted on its own, as by
 * pgabb_tc_count_ex.  opts == NULL selects the default options and tunes
 * (Section 6 names automatic parameter tuning as future work): first the
 * grid of each shape class of graphs (bit widths of m' and of the longest
 * oriented row) -- p of 1, 2, 4, 8 or 16 with nnz-balanced cuts, or 8 with
 * uniform cuts, each timed as one launch over the class's graphs, which
 * are then partitioned with the winner -- then the launch shape of the
 * merged launch (waves per workgroup, items per grab, chunks per load
 * batch), timed on the launch itself.  Both are searched the first time a
 * class is seen and kept in a tuning cache (in memory and in the file named
 * by PGABB_TUNE_CACHE, else $XDG_CACHE_HOME/pgabb/tune.txt or
 * $HOME/.cache/pgabb/tune.txt).  Afterwards each graph's
 * pgabb_graph_task_counts holds its own tasks' counts and
 * pgabb_graph_info_get the shared launch's times and the tuning time.  Errors: EINVAL
 * (num_graphs < 0, a NULL array or graph, a graph listed twice, bad
 * options), ENOMEM, EDEVICE; on any error every count is PGABB_COUNT_ERROR.
 * Many small graphs built together count faster as a pgabb_batch.
 */
pgabb_status pgabb_tc_count_batch(pgabb_graph *const *gs, int64_t num_graphs, const pgabb_tc_options *opts,
                                  uint64_t *counts);

/*
 * Sizes and timings of the graph.  pgabb_partition returns before its last
 * kernels have run (later calls on the graph's stream are ordered after
 * them); this call waits for them when it is the first to read the
 * partition's timing.
 */
pgabb_status pgabb_graph_info_get(const pgabb_graph *g, pgabb_graph_info_t *info);

/*
 * The main sizes alone: vertices, undirected unique edges m' (Section 5.1's
 * cleaned input), grid size p (0 before partitioning) and tasks
 * (block-lists with three non-empty blocks).  Any output may be NULL.
 */
pgabb_status pgabb_graph_info(const pgabb_graph *g, int64_t *n, int64_t *m_undirected, int32_t *p,
                              int64_t *num_tasks);

/*
 * Copy the oriented CSR to host buffers: row_off[n + 1] (int64), col[m']
 * (ranks, increasing within a row), rank[n] (rank of each input id).  Any of
 * the three may be NULL to skip it.
 */
pgabb_status pgabb_graph_export_csr(const pgabb_graph *g, int64_t *row_off, int32_t *col,
                                    int32_t *rank);

/* Copy the cut vector (p + 1 values) of the current partition. */
pgabb_status pgabb_graph_cuts(const pgabb_graph *g, int32_t *cuts);

/*
 * Per-task results of the last count: ijk[3 t .. 3 t + 2] = (i, j, k) and
 * counts[t] = triangles found by task t, for t < num_tasks, in execution
 * order.  Either pointer may be NULL.
 */
pgabb_status pgabb_graph_task_counts(const pgabb_graph *g, int32_t *ijk, uint64_t *counts);

/*
 * Shards of the tasks when a count is split over num_shards devices (PGAbB
 * Section 4.1: block-lists are independent tasks, so the count splits by
 * task).  Tasks that share their edge block A_ij form one group (a device
 * then reads each edge block it holds for all of its k); groups are dealt by
 * longest processing time: heaviest first (ties: the group whose first task
 * comes first in task order), each to the shard with the least weight so far
 * (ties: lowest index).  A group weighs the sum of its tasks' estimated
 * work under the walk a default count takes (probe_work against
 * probe_work_col, see PGABB_OPT_COLS), each list length taken as its
 * block's mean (non-empty rows and columns per block):
 *   column walk: 1 + trunc(nnz(A_ij) * mean(A_ik)) + trunc(cols(A_ij) * mean(A_jk))
 *   row walk:    1 + trunc(nnz(A_ij) * mean(A_jk)) + trunc(rows(A_ij) * mean(A_ik))
 * with mean(A) = nnz(A) / max(rows(A), 1) in double precision.
 *   num_shards : 1 .. 4096
 *   shard_of   : host array of num_tasks entries (pgabb_graph_info);
 *                shard_of[t] for task t in the order of
 *                pgabb_graph_task_counts
 * Errors: EINVAL (NULL, num_shards out of range), ESTATE (not partitioned).
 */
pgabb_status pgabb_graph_task_shards(const pgabb_graph *g, int32_t num_shards, int32_t *shard_of);

/*
 * One device's share of a count split over num_shards devices: counts only
 * the tasks pgabb_graph_task_shards deals to `shard`, as pgabb_tc_count_ex
 * does with opts (NULL = defaults; partitions with p = 1 first if the graph
 * was not partitioned).  *count receives their triangles; the counts of
 * shards 0 .. num_shards - 1 sum to the graph's triangle count.  When the
 * blocks are streamed (a device cap below their bytes, PGABB_OPT_STREAM, or
 * blocks already moved to host memory) only the blocks the shard's tasks
 * read are copied.  Afterwards pgabb_graph_task_counts reports the shard's
 * tasks' counts (0 for the other tasks) and pgabb_graph_info_get the shard
 * count's times, launches and copied bytes.
 * Errors: as pgabb_tc_count_ex; EINVAL for num_shards outside 1 .. 4096 or
 * shard outside [0, num_shards).
 */
pgabb_status pgabb_tc_count_shard(pgabb_graph *g, const pgabb_tc_options *opts, int32_t shard,
                                  int32_t num_shards, uint64_t *count);

/*
 * Triangles containing each edge (edge support; the per-edge counts behind
 * clustering coefficients, PGAbB Section 1, and k-truss peeling, Section
 * 3.2), from the intersections of Section 3.6 over the whole oriented graph
 * as one block (independent of pgabb_partition).
 *   support   : m' uint32 entries; support[e] for the oriented edge at
 *               position e of the CSR that pgabb_graph_export_csr returns
 *               (row x = rank, col[e] = the higher-ranked endpoint).  Host
 *               memory, or device memory with PGABB_SUPPORT_ON_DEVICE (the
 *               call runs on the graph's stream: finish other streams'
 *               work on it first); complete when the call returns.  May be
 *               NULL only when m' = 0.
 *   flags     : 0 or PGABB_SUPPORT_ON_DEVICE
 *   triangles : optional; the triangle count (the sum of support over
 *               three)
 * pgabb_graph_info_get then reports the call's time (t_count_ms), kernel
 * time and launches.  Errors: EINVAL (NULL graph or support, unknown
 * flags, m' >= 2^32: in-edges are indexed by 32-bit CSR positions),
 * ENOMEM, EDEVICE.
 */
#define PGABB_SUPPORT_ON_DEVICE 0x1u
pgabb_status pgabb_tc_edge_support(pgabb_graph *g, uint32_t *support, uint32_t flags, uint64_t *triangles);

/*
 * Triangles at each vertex (the numerator of the local clustering
 * coefficient 2 t(v) / (deg(v) (deg(v) - 1)), PGAbB Section 1), from the
 * per-edge counts of pgabb_tc_edge_support: t(v) is half the sum of the
 * counts of v's edges.
 *   per_vertex : n uint64 entries, indexed by input id (isolated and
 *                out-of-triangle vertices get 0).  Host memory, or device
 *                memory with PGABB_SUPPORT_ON_DEVICE (finish other streams'
 *                work on it first); complete when the call returns.  May be
 *                NULL only when n = 0.
 *   flags      : 0 or PGABB_SUPPORT_ON_DEVICE
 *   triangles  : optional; the triangle count
 * Errors: as pgabb_tc_edge_support.
 */
pgabb_status pgabb_tc_vertex_counts(pgabb_graph *g, uint64_t *per_vertex, uint32_t flags, uint64_t *triangles);

/*
 * The k-truss (the peeling algorithm named in PGAbB Section 3.2): the
 * largest subgraph in which every edge lies in at least k - 2 triangles of
 * the subgraph (unique; k <= 2 keeps every edge).  Computed by peeling in
 * rounds: one pass of pgabb_tc_edge_support counts the triangles of every
 * edge; each round removes the remaining edges with fewer than k - 2 and
 * takes the triangles they close off the counts of the other edges; the
 * rounds end when none is removed.
 *   k         : k >= 0
 *   keep      : optional; m' bytes, keep[e] = 1 for the oriented edge at CSR
 *               position e (pgabb_graph_export_csr) if it is in the k-truss,
 *               else 0.  Host memory, or device memory with
 *               PGABB_SUPPORT_ON_DEVICE; complete when the call returns.
 *   num_edges : optional; edges of the k-truss
 *   rounds    : optional; rounds that removed edges
 * pgabb_graph_info_get then reports the call's time (t_count_ms), the time
 * of the support and peeling kernels, and the rounds as launches.
 * Errors: EINVAL (NULL graph, k < 0, unknown flags, m' >= 2^32), ENOMEM,
 * EDEVICE.
 */
pgabb_status pgabb_tc_ktruss(pgabb_graph *g, int32_t k, uint8_t *keep, uint32_t flags, int64_t *num_edges,
                             int32_t *rounds);

/*
 * Number of 4-cliques (sets of four pairwise adjacent vertices; the
 * multi-block pattern family of PGAbB Section 3.2, one intersection level
 * past triangles), over the graph's partition (p = 1 first if it has
 * none): every block 4-list (A_ij, A_ik, A_il, A_jk, A_jl, A_kl),
 * i <= j <= k <= l, with six non-empty blocks is a task, heaviest first.
 * Each 4-clique a < b < c < d (ranks) is counted once, in the 4-list of its
 * stripes, at its edge (a, b) of A_ij: the pairs c in A_ik[a] & A_jk[b],
 * d in A_il[a] & A_jl[b] with (c, d) in A_kl.  Blocks in device memory are
 * read in place; blocks that a streamed count moved to the pinned host store
 * are streamed as by pgabb_count_4cliques_streamed under that count's
 * device cap (all blocks when it had none).  pgabb_graph_info_get then
 * reports the call's time, kernel time, launches and host-to-device bytes;
 * pgabb_graph_4list_counts the 4-lists and their counts.
 * Errors: EINVAL (NULL argument), ENOMEM, EDEVICE.
 */
pgabb_status pgabb_count_4cliques(pgabb_graph *g, uint64_t *count);

/*
 * The same count with the blocks streamed from the pinned host store (the
 * device arena moves there first if it is still on the device, as in a
 * streamed triangle count; Section 4.4) through a device block cache of at
 * most device_cap_bytes: consecutive 4-lists (heaviest first) form a window
 * while the union of their six blocks' row parts (row items, row offsets,
 * columns) fits the cap; each window's missing blocks are copied, least
 * recently used blocks outside the window leaving first, then the window is
 * counted.  Copies and launches of a window run in order on the graph's
 * stream.
 *   device_cap_bytes : > 0; bytes of device block cache
 * Errors: EINVAL (NULL argument, device_cap_bytes == 0), ENOMEM (the cap
 * cannot hold the six blocks of some 4-list, or allocation), EDEVICE.
 */
pgabb_status pgabb_count_4cliques_streamed(pgabb_graph *g, uint64_t device_cap_bytes, uint64_t *count);

/*
 * The block 4-lists of the last pgabb_count_4cliques on g, in processing
 * order: *num_lists (optional), ijkl[4 q .. 4 q + 3] = (i, j, k, l) and
 * counts[q] = its 4-cliques (either array may be NULL; host arrays of
 * *num_lists entries, queried first with both NULL).
 */
pgabb_status pgabb_graph_4list_counts(const pgabb_graph *g, int64_t *num_lists, int32_t *ijkl, uint64_t *counts);

/*
 * Connected components (the Shiloach-Vishkin example of PGAbB Section 3.4,
 * single-block bulk-synchronous mode of Section 3.2) over the graph's device
 * blocks: even iterations hook, for every edge whose endpoints point to
 * different roots, the larger root under the smaller; odd iterations link
 * every vertex to its root by pointer jumping; the iterations end after a
 * hooking pass that hooked nothing.  A graph that was never partitioned is
 * partitioned with p = 1 first.
 *   label          : n int32; label[v] = the smallest input id in v's
 *                    component (isolated vertices label themselves).  Host
 *                    memory, or device memory with PGABB_SUPPORT_ON_DEVICE;
 *                    complete when the call returns.  NULL allowed if n = 0.
 *   num_components : optional; components, isolated vertices included
 *   iterations     : optional; hooking plus linking iterations run (even)
 * pgabb_graph_info_get then reports the call's time (t_count_ms), its kernel
 * time and the iterations as launches.
 * Errors: EINVAL (NULL graph, NULL label with n > 0, unknown flags), ESTATE
 * (blocks held in host memory by a streamed count), ENOMEM, EDEVICE.
 */
pgabb_status pgabb_components(pgabb_graph *g, int32_t *label, uint32_t flags, int64_t *num_components,
                              int32_t *iterations);

/*
 * PageRank (PGAbB Section 5.2: SpMV-like iteration, as its evaluation runs
 * it with damping 0.85, tolerance 1e-4 and at most 20 iterations), in double
 * precision over the graph's device blocks, pulled through every block's
 * rows and stored columns with atomic additions (single-block bulk-
 * synchronous mode, Section 3.2).  With deg(x) the number of neighbours:
 *     r_0(x) = 1 / n,
 *     r_{t+1}(x) = (1 - damping) / n + damping * sum over neighbours y of
 *                  r_t(y) / deg(y);
 * isolated vertices pass nothing on.  Stops after the first iteration whose
 * sum over x of |r_{t+1}(x) - r_t(x)| is below tol, or after max_iter.
 * A graph that was never partitioned is partitioned with p = 1 first.
 *   ranks      : n doubles by input id; host memory, or device memory with
 *                PGABB_SUPPORT_ON_DEVICE; complete when the call returns.
 *                NULL allowed if n = 0.
 *   iterations : optional; iterations run
 *   last_err   : optional; the last iteration's sum of absolute changes
 * Sums run in a different order from a sequential loop (atomic additions),
 * so results agree with one to rounding, not bit for bit.
 * Errors: EINVAL (NULL graph, NULL ranks with n > 0, damping outside
 * [0, 1], tol < 0 or NaN, max_iter < 0, unknown flags), ESTATE, ENOMEM,
 * EDEVICE.
 */
pgabb_status pgabb_pagerank(pgabb_graph *g, double damping, double tol, int32_t max_iter, double *ranks,
                            uint32_t flags, int32_t *iterations, double *last_err);

/*
 * Forget the tuning choices held in memory; the tuning cache file is read
 * again when the next tuned call needs it (for a cache file edited or copied
 * in while the process runs).
 */
pgabb_status pgabb_tune_cache_reload(void);

/* Release a graph and its device and host memory.  NULL is ignored. */
void pgabb_graph_destroy(pgabb_graph *g);

/* Status and message of the last failing call on this thread. */
pgabb_status pgabb_last_status(void);
const char *pgabb_last_error(void);

/* ------------------------------------------------------------------ batch */

/*
 * Batched counting of many independent graphs in one persistent launch
 * (PGAbB's task-parallel execution, Section 4.4, applied to a set of graphs).
 * The graphs are packed into one arena as a disjoint union; each is cleaned,
 * ranked by (degree, id) within itself and oriented; one persistent kernel
 * then consumes a device work queue of rows and adds each row's triangles to
 * its graph's uint64 slot.  The launch sequence is captured once into a HIP
 * graph and replayed.
 *   num_graphs       : G >= 0
 *   n                : G vertex counts (host)
 *   edge_off         : G + 1 non-decreasing offsets into src/dst (host)
 *   src, dst         : edge_off[G] ids; host, or device with
 *                      PGABB_EDGES_ON_DEVICE
 */
typedef struct pgabb_batch pgabb_batch;

pgabb_status pgabb_batch_create(int64_t num_graphs, const int32_t *n, const int64_t *edge_off,
                                const int32_t *src, const int32_t *dst, uint32_t flags,
                                void *hip_stream, pgabb_batch **out);

/*
 * Count every graph of the batch: counts[g] for g < num_graphs (host).
 * opts == NULL selects the autotuned launch shape (searched on first use,
 * then cached by the batch's shape features); otherwise opts->kernel,
 * waves_per_block and rows_per_grab are used as given.
 */
pgabb_status pgabb_batch_count(pgabb_batch *b, const pgabb_tc_options *opts, uint64_t *counts);

/* Milliseconds of the last batch count (one replay) and of the build. */
pgabb_status pgabb_batch_times(const pgabb_batch *b, double *t_build_ms, double *t_count_ms);

/*
 * Sizes of the batch's union graph (any pointer may be NULL): oriented
 * edges m' over all graphs; active rows (out-degree >= 2, the count's work
 * items) and their edges; entries a count walks (for every active row u,
 * the out-lists of u's out-neighbours: sum over its edges (u, v) of
 * |N+(v)|).
 */
pgabb_status pgabb_batch_stats(const pgabb_batch *b, int64_t *edges, int64_t *active_rows, int64_t *active_edges,
                               uint64_t *walked);

/*
 * The launch shape of the last graph-captured count (any pointer may be
 * NULL): staging kernel (PGABB_KERNEL_BITMAP or PGABB_KERNEL_HASH; -1 before
 * the first such count), waves per workgroup, rows per grab, and the
 * milliseconds the last autotuned count spent choosing it (searching, or
 * reading the tuning cache).  The autotuner's choice is kept per shape class
 * (bit widths of graph count, largest n, m' and longest row) in the tuning
 * cache of pgabb_tc_count_batch.
 */
pgabb_status pgabb_batch_launch_shape(const pgabb_batch *b, int32_t *kernel, int32_t *waves_per_block,
                                      int32_t *rows_per_grab, double *t_tune_ms);

void pgabb_batch_destroy(pgabb_batch *b);

/* ----------------------------------------------------------------- server */

/*
 * A request server with continuous batching: requests (one graph each) are
 * admitted in arrival order while their estimated device bytes fit the
 * budget, are built by builder threads on their own streams while earlier
 * requests are being counted, and join the next counting launch as soon as
 * they are built.  Finished requests release their memory and let queued
 * ones in.
 *   device_budget_bytes : bound on the device bytes held by admitted requests
 *   opts                : counting options (NULL = defaults); num_streams is
 *                         the number of builders (0 = 2, at most 8); p is
 *                         the grid each request is partitioned with (0 =
 *                         by size: 8 for requests of at least 2^18 pairs,
 *                         else 1; at most 64, EINVAL outside [0, 64]) and
 *                         cut_mode its cuts (Section 4.3)
 */
typedef struct pgabb_server pgabb_server;

pgabb_status pgabb_server_create(uint64_t device_budget_bytes, const pgabb_tc_options *opts,
                                 pgabb_server **out);

/*
 * Queue one request; host arrays are copied before the call returns (or
 * borrowed until it finishes, with PGABB_SERVER_BORROW in the server's
 * options).  *ticket receives an id for pgabb_server_poll.  EINVAL for NULL
 * arrays or n < 0, m < 0; EBUDGET if the request can never fit the budget.
 * Ids are checked on the device when the request is built: a request with an
 * id outside [0, n) finishes with status EINVAL (pgabb_server_poll returns
 * it).
 */
pgabb_status pgabb_server_submit(pgabb_server *s, int32_t n, int64_t m, const int32_t *src,
                                 const int32_t *dst, uint64_t *ticket);

/*
 * *done = 1 and *count = triangles once the request finished, else *done = 0
 * (count may be NULL).  A finished request that failed returns its status
 * (EINVAL for an id outside [0, n), ENOMEM, EDEVICE).  EINVAL for a NULL
 * server or done, or an unknown ticket.
 */
pgabb_status pgabb_server_poll(pgabb_server *s, uint64_t ticket, int32_t *done, uint64_t *count);

/*
 * Timestamps of a request, in seconds on the server's monotonic clock
 * (pgabb_server_now): submission, and completion (0 while it runs).  Either
 * pointer may be NULL.  EINVAL for a NULL server or an unknown ticket.
 */
pgabb_status pgabb_server_times(pgabb_server *s, uint64_t ticket, double *t_submit, double *t_done);

/* Block until every submitted request has finished. */
pgabb_status pgabb_server_drain(pgabb_server *s);

/* Server clock (seconds). */
double pgabb_server_now(const pgabb_server *s);

/* Counting launches issued so far. */
pgabb_status pgabb_server_stats(const pgabb_server *s, uint64_t *launches);

/*
 * Totals over the server's counting launches so far (any pointer may be
 * NULL): their device milliseconds, the entries their walks read and the
 * oriented edges m' of the requests they counted (4 bytes per walked entry
 * plus 16 per edge are the launches' algorithmic bytes, as for a count).
 */
pgabb_status pgabb_server_kernel_stats(pgabb_server *s, double *kernel_ms, uint64_t *walked, uint64_t *edges);

void pgabb_server_destroy(pgabb_server *s);

/* ------------------------------------------------------------- allocator */

/*
 * Route the library's device allocations through caller functions (NULL,
 * NULL restores the library's caching allocator).  alloc returns NULL on
 * failure, which the library reports as ENOMEM.  Applies to allocations made
 * after the call; memory the caching allocator handed out earlier still goes
 * back to it when freed.
 *
 * The caching allocator keeps freed device blocks (and the pinned host
 * blocks it stages small copies through) for reuse by size class: up to a
 * quarter of device memory and 4 GiB of pinned memory stay cached, and a
 * failed allocation first returns every cached block to HIP.
 */
typedef void *(*pgabb_alloc_fn)(size_t bytes, void *hip_stream, void *ctx);
typedef void (*pgabb_free_fn)(void *ptr, void *hip_stream, void *ctx);
pgabb_status pgabb_set_allocator(pgabb_alloc_fn alloc, pgabb_free_fn free_fn, void *ctx);

/*
 * Return every cached free block (device memory of every device the library
 * used, and pinned host memory) to HIP, after the work that last used each
 * block has finished.  Blocks in use by live objects are not affected.
 */
pgabb_status pgabb_release_cached_memory(void);

/* Library version string. */
const char *pgabb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PGABB_H */
