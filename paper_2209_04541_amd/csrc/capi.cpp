// C ABI entry points: argument checks, error capture, object lifetime.
#include <chrono>
#include <cstring>
#include <mutex>
#include <new>

#include "common.hpp"
#include "graph.hpp"

namespace pgabb {

namespace {

thread_local pgabb_status t_status = PGABB_OK;
thread_local std::string t_message;

pgabb_status set_ok() {
    t_status = PGABB_OK;
    t_message.clear();
    return PGABB_OK;
}

pgabb_status set_err(pgabb_status st, const std::string &msg) {
    t_status = st;
    t_message = msg;
    return st;
}

}  // namespace

void fail(pgabb_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{st, buf};
}

StreamTimer::StreamTimer() {
    PGABB_HIP(hipEventCreate(&a_));
    PGABB_HIP(hipEventCreate(&b_));
}
StreamTimer::~StreamTimer() {
    if (a_) (void)hipEventDestroy(a_);
    if (b_) (void)hipEventDestroy(b_);
}
void StreamTimer::start(hipStream_t s) { PGABB_HIP(hipEventRecord(a_, s)); }
void StreamTimer::stop(hipStream_t s) { PGABB_HIP(hipEventRecord(b_, s)); }
double StreamTimer::ms() {
    PGABB_HIP(hipEventSynchronize(b_));
    float t = 0;
    PGABB_HIP(hipEventElapsedTime(&t, a_, b_));
    return t;
}

hipStream_t library_stream() {
    static hipStream_t s = [] {
        hipStream_t x = nullptr;
        PGABB_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        return x;
    }();
    return s;
}

pgabb_status capture_status(const Error &e) { return set_err(e.status, e.message); }

}  // namespace pgabb

using namespace pgabb;

#define PGABB_API extern "C" __attribute__((visibility("default")))

#define PGABB_TRY try {
#define PGABB_CATCH                                                      \
    }                                                                    \
    catch (const Error &e) {                                             \
        return set_err(e.status, e.message);                             \
    }                                                                    \
    catch (const std::bad_alloc &) {                                     \
        return set_err(PGABB_ENOMEM, "host allocation failed");          \
    }                                                                    \
    catch (...) {                                                        \
        return set_err(PGABB_EDEVICE, "unexpected internal error");      \
    }

// Largest grid: the partition kernels give each stripe of a row one lane of
// a 64-wide wavefront.
static constexpr int32_t kMaxGrid = 64;

PGABB_API pgabb_status pgabb_last_status(void) { return t_status; }
PGABB_API const char *pgabb_last_error(void) { return t_message.c_str(); }
PGABB_API const char *pgabb_version(void) { return "pgabb-mi355x 0.1 (gfx950)"; }

PGABB_API pgabb_status pgabb_set_allocator(pgabb_alloc_fn alloc, pgabb_free_fn free_fn, void *ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return set_err(PGABB_EINVAL, "alloc and free must both be set or both be NULL");
    set_allocator_hook(alloc, free_fn, alloc ? ctx : nullptr);
    return set_ok();
}

PGABB_API pgabb_status pgabb_release_cached_memory(void) {
    PGABB_TRY
    release_cached_memory();
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_graph_from_edges(int32_t n, int64_t m, const int32_t *src,
                                              const int32_t *dst, uint32_t flags, void *hip_stream,
                                              pgabb_graph **out) {
    if (!out) return set_err(PGABB_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 0) return set_err(PGABB_EINVAL, "n < 0");
    if (m < 0) return set_err(PGABB_EINVAL, "m < 0");
    if (m > 0 && (!src || !dst)) return set_err(PGABB_EINVAL, "src or dst is NULL");
    if (flags & ~(PGABB_EDGES_ON_DEVICE | PGABB_ORDER_BY_ID)) return set_err(PGABB_EINVAL, "unknown flag bits");
    if (m >= (int64_t(1) << 32)) return set_err(PGABB_EINVAL, "more than 2^32 - 1 pairs");
    // host input: check ids before any device work (a branch-free pass the
    // compiler vectorises; the offending pair is looked up only on failure)
    if (m > 0 && !(flags & PGABB_EDGES_ON_DEVICE)) {
        const uint32_t un = static_cast<uint32_t>(n);
        uint32_t bad = 0;
        for (int64_t e = 0; e < m; ++e)
            bad |= static_cast<uint32_t>(static_cast<uint32_t>(src[e]) >= un) |
                   static_cast<uint32_t>(static_cast<uint32_t>(dst[e]) >= un);
        if (bad) {
            int64_t e = 0;
            while (static_cast<uint32_t>(src[e]) < un && static_cast<uint32_t>(dst[e]) < un) ++e;
            char buf[160];
            snprintf(buf, sizeof buf, "pair %lld = (%d, %d) has an id outside [0, %d)",
                     static_cast<long long>(e), src[e], dst[e], n);
            return set_err(PGABB_EINVAL, buf);
        }
    }
    pgabb_graph *g = nullptr;
    PGABB_TRY
    g = new pgabb_graph();
    g->flags = flags;
    g->n = n;
    g->stream = hip_stream ? static_cast<hipStream_t>(hip_stream) : library_stream();
    hipStream_t s = g->stream;
    StreamTimer tm;
    tm.start(s);
    if (m > 0 && !(flags & PGABB_EDGES_ON_DEVICE)) {
        DArray<int32_t> ds(static_cast<size_t>(m), s), dd(static_cast<size_t>(m), s);
        PGABB_HIP(hipMemcpyAsync(ds.get(), src, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(dd.get(), dst, sizeof(int32_t) * m, hipMemcpyHostToDevice, s));
        build_graph(g, ds.get(), dd.get(), m);
    } else {
        build_graph(g, src, dst, m);
    }
    tm.stop(s);
    g->t_build_ms = tm.ms();
    *out = g;
    return set_ok();
    }
    catch (const Error &e) {
        delete g;
        return set_err(e.status, e.message);
    }
    catch (const std::bad_alloc &) {
        delete g;
        return set_err(PGABB_ENOMEM, "host allocation failed");
    }
    catch (...) {
        delete g;
        return set_err(PGABB_EDEVICE, "unexpected internal error");
    }
}

PGABB_API pgabb_status pgabb_partition_ex(pgabb_graph *g, int32_t p, int32_t cut_mode, const int32_t *cuts) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (p < 1 || p > kMaxGrid) return set_err(PGABB_EINVAL, "p must lie in [1, 64]");
    if (cut_mode != PGABB_CUT_NNZ && cut_mode != PGABB_CUT_UNIFORM)
        return set_err(PGABB_EINVAL, "unknown cut mode");
    if (cuts) {
        if (cuts[0] != 0 || cuts[p] != g->n) return set_err(PGABB_EINVAL, "cuts must start at 0 and end at n");
        for (int32_t s = 0; s < p; ++s)
            if (cuts[s] > cuts[s + 1]) return set_err(PGABB_EINVAL, "cuts must be non-decreasing");
    }
    PGABB_TRY
    partition_graph(g, p, cut_mode, cuts);
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_partition(pgabb_graph *g, int32_t p) {
    return pgabb_partition_ex(g, p, PGABB_CUT_NNZ, nullptr);
}

static pgabb_tc_options default_options() {
    pgabb_tc_options o;
    std::memset(&o, 0, sizeof o);
    return o;
}

// Checks the options of a count; PGABB_OK or the status already set.
static pgabb_status check_options(const pgabb_tc_options &o) {
    if (o.kernel < PGABB_KERNEL_AUTO || o.kernel > PGABB_KERNEL_SEARCH)
        return set_err(PGABB_EINVAL, "unknown kernel");
    if (o.num_streams < 0 || o.waves_per_block < 0 || o.rows_per_grab < 0)
        return set_err(PGABB_EINVAL, "negative option");
    if (o.waves_per_block && o.waves_per_block != 2 && o.waves_per_block != 4 && o.waves_per_block != 8)
        return set_err(PGABB_EINVAL, "waves_per_block must be 2, 4 or 8");
    if (o.unroll && o.unroll != 1 && o.unroll != 2 && o.unroll != 4 && o.unroll != 8)
        return set_err(PGABB_EINVAL, "unroll must be 1, 2, 4 or 8");
    if (o.p < 0 || o.p > kMaxGrid) return set_err(PGABB_EINVAL, "p must lie in [0, 64]");
    if (o.cut_mode != PGABB_CUT_NNZ && o.cut_mode != PGABB_CUT_UNIFORM) return set_err(PGABB_EINVAL, "unknown cut mode");
    if (o.host_threads < 0 || o.host_threads > 64) return set_err(PGABB_EINVAL, "host_threads must lie in [0, 64]");
    if (o.host_permille < 0 || o.host_permille > 1000) return set_err(PGABB_EINVAL, "host_permille must lie in [0, 1000]");
    if (o.flags & ~(PGABB_OPT_STREAM | PGABB_OPT_PER_GRAPH | PGABB_SERVER_BORROW | PGABB_OPT_ROWS | PGABB_OPT_COLS |
                    PGABB_OPT_HYBRID))
        return set_err(PGABB_EINVAL, "unknown option flag bits");
    if ((o.flags & PGABB_OPT_ROWS) && (o.flags & PGABB_OPT_COLS))
        return set_err(PGABB_EINVAL, "PGABB_OPT_ROWS and PGABB_OPT_COLS together");
    return PGABB_OK;
}

PGABB_API pgabb_status pgabb_tc_count_ex(pgabb_graph *g, const pgabb_tc_options *opts, uint64_t *count) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (!count) return set_err(PGABB_EINVAL, "count is NULL");
    *count = PGABB_COUNT_ERROR;
    const pgabb_tc_options o = opts ? *opts : default_options();
    const pgabb_status st = check_options(o);
    if (st != PGABB_OK) return st;
    PGABB_TRY
    *count = count_graph(g, o);
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_tc_count_noalloc(pgabb_graph *g, const pgabb_tc_options *opts, uint64_t *count) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (!count) return set_err(PGABB_EINVAL, "count is NULL");
    *count = PGABB_COUNT_ERROR;
    const pgabb_tc_options o = opts ? *opts : default_options();
    const pgabb_status st = check_options(o);
    if (st != PGABB_OK) return st;
    PGABB_TRY
    *count = count_noalloc(g, o);
    return set_ok();
    PGABB_CATCH
}

PGABB_API size_t pgabb_tc_count_noalloc_scratch_bytes(void) { return noalloc_scratch_bytes(); }

PGABB_API pgabb_status pgabb_tc_edge_support(pgabb_graph *g, uint32_t *support, uint32_t flags,
                                             uint64_t *triangles) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (!support && g->m > 0) return set_err(PGABB_EINVAL, "support is NULL");
    if (flags & ~PGABB_SUPPORT_ON_DEVICE) return set_err(PGABB_EINVAL, "unknown flag bits");
    PGABB_TRY
    const uint64_t t = edge_support(g, support, (flags & PGABB_SUPPORT_ON_DEVICE) != 0);
    if (triangles) *triangles = t;
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_tc_vertex_counts(pgabb_graph *g, uint64_t *per_vertex, uint32_t flags,
                                              uint64_t *triangles) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (!per_vertex && g->n > 0) return set_err(PGABB_EINVAL, "per_vertex is NULL");
    if (flags & ~PGABB_SUPPORT_ON_DEVICE) return set_err(PGABB_EINVAL, "unknown flag bits");
    PGABB_TRY
    const uint64_t t = vertex_counts(g, per_vertex, (flags & PGABB_SUPPORT_ON_DEVICE) != 0);
    if (triangles) *triangles = t;
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_tc_ktruss(pgabb_graph *g, int32_t k, uint8_t *keep, uint32_t flags,
                                       int64_t *num_edges, int32_t *rounds) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (k < 0) return set_err(PGABB_EINVAL, "k < 0");
    if (flags & ~PGABB_SUPPORT_ON_DEVICE) return set_err(PGABB_EINVAL, "unknown flag bits");
    PGABB_TRY
    const int64_t left = ktruss(g, k, keep, (flags & PGABB_SUPPORT_ON_DEVICE) != 0, rounds);
    if (num_edges) *num_edges = left;
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_components(pgabb_graph *g, int32_t *label, uint32_t flags, int64_t *num_components,
                                        int32_t *iterations) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (!label && g->n > 0) return set_err(PGABB_EINVAL, "label is NULL");
    if (flags & ~PGABB_SUPPORT_ON_DEVICE) return set_err(PGABB_EINVAL, "unknown flag bits");
    PGABB_TRY
    const int64_t c = components(g, label, (flags & PGABB_SUPPORT_ON_DEVICE) != 0, iterations);
    if (num_components) *num_components = c;
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_pagerank(pgabb_graph *g, double damping, double tol, int32_t max_iter, double *ranks,
                                      uint32_t flags, int32_t *iterations, double *last_err) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (!ranks && g->n > 0) return set_err(PGABB_EINVAL, "ranks is NULL");
    if (!(damping >= 0.0 && damping <= 1.0)) return set_err(PGABB_EINVAL, "damping outside [0, 1]");
    if (!(tol >= 0.0)) return set_err(PGABB_EINVAL, "tol < 0 or NaN");
    if (max_iter < 0) return set_err(PGABB_EINVAL, "max_iter < 0");
    if (flags & ~PGABB_SUPPORT_ON_DEVICE) return set_err(PGABB_EINVAL, "unknown flag bits");
    PGABB_TRY
    const int32_t it = pagerank(g, damping, tol, max_iter, ranks, (flags & PGABB_SUPPORT_ON_DEVICE) != 0, last_err);
    if (iterations) *iterations = it;
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_graph_4list_counts(const pgabb_graph *g, int64_t *num_lists, int32_t *ijkl,
                                               uint64_t *counts) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    const int64_t nq = static_cast<int64_t>(g->quads.size());
    if (num_lists) *num_lists = nq;
    for (int64_t q = 0; q < nq; ++q) {
        if (ijkl)
            for (int r = 0; r < 4; ++r) ijkl[4 * q + r] = g->quads[q][r];
        if (counts) counts[q] = g->quad_counts[q];
    }
    return set_ok();
}

PGABB_API pgabb_status pgabb_count_4cliques(pgabb_graph *g, uint64_t *count) {
    if (!g || !count) return set_err(PGABB_EINVAL, "NULL argument");
    PGABB_TRY
    *count = four_cliques(g, 0);
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_count_4cliques_streamed(pgabb_graph *g, uint64_t device_cap_bytes, uint64_t *count) {
    if (!g || !count) return set_err(PGABB_EINVAL, "NULL argument");
    if (device_cap_bytes == 0) return set_err(PGABB_EINVAL, "device_cap_bytes must be positive");
    PGABB_TRY
    *count = four_cliques(g, device_cap_bytes);
    return set_ok();
    PGABB_CATCH
}

static constexpr int32_t kMaxShards = 4096;

PGABB_API pgabb_status pgabb_graph_task_shards(const pgabb_graph *g, int32_t num_shards, int32_t *shard_of) {
    if (!g || !shard_of) return set_err(PGABB_EINVAL, "NULL argument");
    if (num_shards < 1 || num_shards > kMaxShards) return set_err(PGABB_EINVAL, "num_shards outside [1, 4096]");
    if (g->p == 0) return set_err(PGABB_ESTATE, "graph is not partitioned");
    PGABB_TRY
    const std::vector<int32_t> of = task_shards(g, num_shards);
    std::memcpy(shard_of, of.data(), sizeof(int32_t) * of.size());
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_tc_count_shard(pgabb_graph *g, const pgabb_tc_options *opts, int32_t shard,
                                            int32_t num_shards, uint64_t *count) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (!count) return set_err(PGABB_EINVAL, "count is NULL");
    *count = PGABB_COUNT_ERROR;
    if (num_shards < 1 || num_shards > kMaxShards) return set_err(PGABB_EINVAL, "num_shards outside [1, 4096]");
    if (shard < 0 || shard >= num_shards) return set_err(PGABB_EINVAL, "shard outside [0, num_shards)");
    const pgabb_tc_options o = opts ? *opts : default_options();
    const pgabb_status st = check_options(o);
    if (st != PGABB_OK) return st;
    PGABB_TRY
    *count = count_shard(g, o, shard, num_shards);
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_tc_count_batch(pgabb_graph *const *gs, int64_t num_graphs,
                                            const pgabb_tc_options *opts, uint64_t *counts) {
    if (num_graphs < 0) return set_err(PGABB_EINVAL, "num_graphs < 0");
    if (num_graphs == 0) return set_ok();
    if (!gs || !counts) return set_err(PGABB_EINVAL, "NULL argument");
    for (int64_t q = 0; q < num_graphs; ++q) counts[q] = PGABB_COUNT_ERROR;
    for (int64_t q = 0; q < num_graphs; ++q) {
        if (!gs[q]) return set_err(PGABB_EINVAL, "graph is NULL");
        for (int64_t r = 0; r < q; ++r)
            if (gs[r] == gs[q]) return set_err(PGABB_EINVAL, "a graph is listed twice");
    }
    const pgabb_tc_options o = opts ? *opts : default_options();
    const pgabb_status st = check_options(o);
    if (st != PGABB_OK) return st;
    std::vector<uint64_t> out(static_cast<size_t>(num_graphs), PGABB_COUNT_ERROR);
    PGABB_TRY
    count_graphs(gs, num_graphs, o, opts == nullptr, out.data());
    std::memcpy(counts, out.data(), sizeof(uint64_t) * out.size());
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_tune_cache_reload(void) {
    PGABB_TRY
    tune_reload();
    return set_ok();
    PGABB_CATCH
}

PGABB_API uint64_t pgabb_tc_count(pgabb_graph *g) {
    uint64_t c = PGABB_COUNT_ERROR;
    if (pgabb_tc_count_ex(g, nullptr, &c) != PGABB_OK) return PGABB_COUNT_ERROR;
    return c;
}

PGABB_API pgabb_status pgabb_graph_info_get(const pgabb_graph *g, pgabb_graph_info_t *info) {
    if (!g || !info) return set_err(PGABB_EINVAL, "NULL argument");
    if (g->part_time_pending) {
        // the last partition's device time, once its last kernels have run
        PGABB_TRY
        pgabb_graph *gm = const_cast<pgabb_graph *>(g);
        gm->t_partition_ms = gm->part_timer->ms();
        gm->part_time_pending = false;
        PGABB_CATCH
    }
    info->n = g->n;
    info->m_input = g->m_input;
    info->m = g->m;
    info->isolated = g->isolated;
    info->max_out_degree = g->max_out;
    info->p = g->p;
    info->num_blocks = static_cast<int64_t>(g->blocks.size());
    info->num_tasks = static_cast<int64_t>(g->tasks.size());
    info->probe_work = g->probe_work;
    info->block_bytes = static_cast<uint64_t>(g->arena_words) * sizeof(int32_t);
    info->h2d_bytes = g->h2d_bytes;
    info->t_build_ms = g->t_build_ms;
    info->t_partition_ms = g->t_partition_ms;
    info->t_count_ms = g->t_count_ms;
    info->t_kernel_ms = g->t_kernel_ms;
    info->kernel_launches = g->kernel_launches;
    info->probe_work_col = g->probe_work_col;
    info->walked_columns = g->walked_columns;
    info->host_tasks = g->host_tasks;
    info->host_work_share = g->host_work_share;
    info->t_tune_ms = g->t_tune_ms;
    info->row_items = 0;
    info->col_items = 0;
    info->walk_bytes_rows = 0;
    info->walk_bytes_cols = 0;
    for (const pgabb::BlockInfo &b : g->blocks) {
        info->row_items += b.nitems;
        info->col_items += b.ncitems;
        info->walk_bytes_rows += sizeof(int32_t) * static_cast<uint64_t>(b.walk_hi(pgabb::kOrientRow) -
                                                                           b.walk_lo(pgabb::kOrientRow));
        info->walk_bytes_cols += sizeof(int32_t) * static_cast<uint64_t>(b.walk_hi(pgabb::kOrientCol) -
                                                                           b.walk_lo(pgabb::kOrientCol));
    }
    return set_ok();
}

PGABB_API pgabb_status pgabb_graph_info(const pgabb_graph *g, int64_t *n, int64_t *m_undirected, int32_t *p,
                                        int64_t *num_tasks) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (m_undirected) *m_undirected = g->m;
    if (p) *p = g->p;
    if (num_tasks) *num_tasks = static_cast<int64_t>(g->tasks.size());
    return set_ok();
}

PGABB_API pgabb_status pgabb_graph_export_csr(const pgabb_graph *g, int64_t *row_off, int32_t *col, int32_t *rank) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    PGABB_TRY
    hipStream_t s = g->stream;
    if (row_off)
        PGABB_HIP(hipMemcpyAsync(row_off, g->row_off.get(), sizeof(int64_t) * (static_cast<size_t>(g->n) + 1),
                                 hipMemcpyDeviceToHost, s));
    if (col && g->m)
        PGABB_HIP(hipMemcpyAsync(col, g->col.get(), sizeof(int32_t) * g->m, hipMemcpyDeviceToHost, s));
    if (rank && g->n)
        PGABB_HIP(hipMemcpyAsync(rank, g->rank.get(), sizeof(int32_t) * g->n, hipMemcpyDeviceToHost, s));
    PGABB_HIP(hipStreamSynchronize(s));
    return set_ok();
    PGABB_CATCH
}

PGABB_API pgabb_status pgabb_graph_cuts(const pgabb_graph *g, int32_t *cuts) {
    if (!g || !cuts) return set_err(PGABB_EINVAL, "NULL argument");
    if (g->p == 0) return set_err(PGABB_ESTATE, "graph is not partitioned");
    std::memcpy(cuts, g->cuts.data(), sizeof(int32_t) * g->cuts.size());
    return set_ok();
}

PGABB_API pgabb_status pgabb_graph_task_counts(const pgabb_graph *g, int32_t *ijk, uint64_t *counts) {
    if (!g) return set_err(PGABB_EINVAL, "graph is NULL");
    if (g->p == 0) return set_err(PGABB_ESTATE, "graph is not partitioned");
    for (size_t t = 0; t < g->tasks.size(); ++t) {
        if (ijk) {
            ijk[3 * t] = g->tasks[t].i;
            ijk[3 * t + 1] = g->tasks[t].j;
            ijk[3 * t + 2] = g->tasks[t].k;
        }
        if (counts) counts[t] = t < g->task_counts.size() ? g->task_counts[t] : 0;
    }
    return set_ok();
}

PGABB_API void pgabb_graph_destroy(pgabb_graph *g) {
    if (!g) return;
    try {
        (void)hipStreamSynchronize(g->stream);
        delete g;
    } catch (...) {
    }
}
