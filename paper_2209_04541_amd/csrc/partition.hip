// Partition phase: symmetric rectilinear 2-D cut of the oriented CSR into a
// p x p grid of blocks, block storage, and the block-list (task) table.
//
// PGAbB Section 4.3 (symmetric two-dimensional partitioning: one cut vector
// for rows and columns; block ids in row-major order; per-block CSR with
// rearranged local ids) and Section 3.6 (block-lists (A_ij, A_ik, A_jk) of
// the two-dimensional triangle count).  With vertices ranked in ascending
// degree and edges oriented from lower to higher rank, only blocks with
// i <= j hold entries, and a triangle with ranks a < b < c lies in the task
// (stripe(a), stripe(b), stripe(c)), so the tasks are the triples
// i <= j <= k whose three blocks are non-empty.  Tasks are weighted by their
// edge count (the paper's default estimate) and sorted heaviest first
// (Section 4.1).
#include <algorithm>
#include <chrono>
#include <numeric>

#include "common.hpp"
#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

namespace {

constexpr int B = 256;
constexpr int kMaxP = 64;

struct CutTable {
    int32_t p;
    int32_t c[kMaxP + 1];
    int32_t base[kMaxP];
};

__device__ __forceinline__ int32_t stripe_of(int32_t x, const CutTable &ct) {
    int32_t lo = 0, hi = ct.p - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (ct.c[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// nnz-balanced cut s: first row x whose CSR offset reaches s * m' / p.
__global__ void k_nnz_cuts(const int64_t *__restrict__ row_off, int32_t n, int64_t m, int32_t p,
                           int32_t *__restrict__ cuts) {
    const int32_t s = static_cast<int32_t>(blockIdx.x * B + threadIdx.x);
    if (s > p) return;
    if (s == 0) { cuts[0] = 0; return; }
    if (s == p) { cuts[p] = n; return; }
    // smallest x in [0, n] with row_off[x] * p >= s * m
    int64_t lo = 0, hi = n;
    const int64_t target = static_cast<int64_t>(s) * m;  // < 2^38 for m' < 2^32
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (row_off[mid] * p >= target) hi = mid;
        else lo = mid + 1;
    }
    cuts[s] = static_cast<int32_t>(lo);
}

// Per block (i, j): number of entries and number of work items (each row's
// run split into pieces of at most kSplitV entries).  Each workgroup
// accumulates in LDS and flushes its non-zero counters.
__global__ __launch_bounds__(B) void k_block_sizes(const int64_t *__restrict__ row_off,
                                                   const int32_t *__restrict__ col, int32_t n,
                                                   CutTable ct,
                                                   unsigned long long *__restrict__ nnz,
                                                   unsigned int *__restrict__ rows) {
    __shared__ unsigned int s_nnz[kMaxP * kMaxP];
    __shared__ unsigned int s_rows[kMaxP * kMaxP];
    const int pp = ct.p * ct.p;
    for (int q = threadIdx.x; q < pp; q += B) {
        s_nnz[q] = 0;
        s_rows[q] = 0;
    }
    __syncthreads();
    for (int64_t x = blockIdx.x * int64_t(B) + threadIdx.x; x < n; x += int64_t(gridDim.x) * B) {
        const int64_t e0 = row_off[x], e1 = row_off[x + 1];
        if (e0 == e1) continue;
        const int32_t si = stripe_of(static_cast<int32_t>(x), ct);
        int32_t j = stripe_of(col[e0], ct);
        unsigned int run = 0;
        for (int64_t e = e0; e < e1; ++e) {
            const int32_t y = col[e];
            while (y >= ct.c[j + 1]) {
                if (run) {
                    atomicAdd(&s_nnz[si * ct.p + j], run);
                    atomicAdd(&s_rows[si * ct.p + j], (run + kSplitV - 1) / kSplitV);
                }
                run = 0;
                ++j;
            }
            ++run;
        }
        atomicAdd(&s_nnz[si * ct.p + j], run);
        atomicAdd(&s_rows[si * ct.p + j], (run + kSplitV - 1) / kSplitV);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < pp; q += B) {
        if (s_nnz[q]) {
            atomicAdd(&nnz[q], static_cast<unsigned long long>(s_nnz[q]));
            atomicAdd(&rows[q], s_rows[q]);
        }
    }
}

// Per-row entry counts of every block the row touches, written at the row's
// slot of the block's dense row range.
__global__ void k_row_slot_counts(const int64_t *__restrict__ row_off,
                                  const int32_t *__restrict__ col, int32_t n, CutTable ct,
                                  const int64_t *__restrict__ slot_base,  // p*p, -1 if no block
                                  uint32_t *__restrict__ slots) {
    for (int64_t x = blockIdx.x * int64_t(B) + threadIdx.x; x < n; x += int64_t(gridDim.x) * B) {
        const int64_t e0 = row_off[x], e1 = row_off[x + 1];
        if (e0 == e1) continue;
        const int32_t si = stripe_of(static_cast<int32_t>(x), ct);
        const int64_t lx = x - ct.base[si];
        int32_t j = stripe_of(col[e0], ct);
        uint32_t run = 0;
        for (int64_t e = e0; e < e1; ++e) {
            const int32_t y = col[e];
            while (y >= ct.c[j + 1]) {
                if (run) slots[slot_base[si * ct.p + j] + lx] = run;
                run = 0;
                ++j;
            }
            ++run;
        }
        slots[slot_base[si * ct.p + j] + lx] = run;
    }
}

// Block of slot q: the last block whose slot range starts at or before q.
__device__ __forceinline__ int32_t block_of_slot(int64_t q, const int64_t *sb, int32_t nb) {
    int32_t lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (sb[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Dense row offsets of every block from the scanned slot counts, and the
// number of work items of every row (for the item-list compaction).
__global__ __launch_bounds__(B) void k_fill_rptr(const uint32_t *__restrict__ scanned,
                                                 int64_t nslots,
                                                 const int64_t *__restrict__ slot_base_dense,
                                                 const int64_t *__restrict__ chunk_off,
                                                 const int32_t *__restrict__ width, int32_t nblk,
                                                 int32_t *__restrict__ arena,
                                                 uint32_t *__restrict__ flags) {
    extern __shared__ int64_t s_sb[];
    for (int q = threadIdx.x; q < nblk; q += B) s_sb[q] = slot_base_dense[q];
    __syncthreads();
    for (int64_t q = blockIdx.x * int64_t(B) + threadIdx.x; q < nslots; q += int64_t(gridDim.x) * B) {
        const int32_t b = block_of_slot(q, s_sb, nblk);
        const int64_t r = q - s_sb[b];
        const uint32_t v = scanned[q] - scanned[s_sb[b]];
        arena[chunk_off[b] + r] = static_cast<int32_t>(v);
        flags[q] = r < width[b] ? (scanned[q + 1] - scanned[q] + kSplitV - 1) / kSplitV : 0u;
    }
}

__global__ __launch_bounds__(B) void k_fill_items(const uint32_t *__restrict__ flags,
                                                  const uint32_t *__restrict__ pos, int64_t nslots,
                                                  const int64_t *__restrict__ slot_base_dense,
                                                  const int64_t *__restrict__ chunk_off,
                                                  const int32_t *__restrict__ width, int32_t nblk,
                                                  int32_t *__restrict__ arena) {
    extern __shared__ int64_t s_sb[];
    for (int q = threadIdx.x; q < nblk; q += B) s_sb[q] = slot_base_dense[q];
    __syncthreads();
    for (int64_t q = blockIdx.x * int64_t(B) + threadIdx.x; q < nslots; q += int64_t(gridDim.x) * B) {
        const uint32_t f = flags[q];
        if (!f) continue;
        const int32_t b = block_of_slot(q, s_sb, nblk);
        const int64_t r = q - s_sb[b];
        const uint32_t at = pos[q] - pos[s_sb[b]];
        int32_t *it = arena + chunk_off[b] + width[b] + 1 + 2 * static_cast<int64_t>(at);
        for (uint32_t c = 0; c < f; ++c) {
            it[2 * c] = static_cast<int32_t>(r);
            it[2 * c + 1] = static_cast<int32_t>(c);
        }
    }
}

// Column entries: row x's run in stripe j goes to block (stripe(x), j) at the
// row's dense offset, as local column ids.
__global__ void k_fill_cols(const int64_t *__restrict__ row_off, const int32_t *__restrict__ col,
                            int32_t n, CutTable ct, const int32_t *__restrict__ blk_index,
                            const int64_t *__restrict__ chunk_off,
                            const int32_t *__restrict__ width,
                            const int32_t *__restrict__ nitems, int32_t *__restrict__ arena) {
    for (int64_t x = blockIdx.x * int64_t(B) + threadIdx.x; x < n; x += int64_t(gridDim.x) * B) {
        const int64_t e0 = row_off[x], e1 = row_off[x + 1];
        if (e0 == e1) continue;
        const int32_t si = stripe_of(static_cast<int32_t>(x), ct);
        const int64_t lx = x - ct.base[si];
        int32_t j = -1;
        int32_t *dst = nullptr;
        int32_t cbase = 0;
        for (int64_t e = e0; e < e1; ++e) {
            const int32_t y = col[e];
            if (j < 0 || y >= ct.c[j + 1]) {
                j = stripe_of(y, ct);
                const int32_t b = blk_index[si * ct.p + j];
                const int64_t c0 = chunk_off[b];
                dst = arena + c0 + width[b] + 1 + 2 * static_cast<int64_t>(nitems[b]) + arena[c0 + lx];
                cbase = ct.base[j];
            }
            *dst++ = y - cbase;
        }
    }
}

unsigned cap_grid(int64_t work) {
    unsigned g = grid_for(work, B);
    return g > 65536u ? 65536u : g;
}

}  // namespace

void partition_graph(pgabb_graph *g, int32_t p, int32_t cut_mode, const int32_t *cuts_host) {
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    auto t0 = std::chrono::steady_clock::now();

    // ---- cut vector
    std::vector<int32_t> cuts(static_cast<size_t>(p) + 1);
    if (cuts_host) {
        std::copy(cuts_host, cuts_host + p + 1, cuts.begin());
    } else if (cut_mode == PGABB_CUT_UNIFORM) {
        for (int32_t s_ = 0; s_ <= p; ++s_)
            cuts[s_] = static_cast<int32_t>((static_cast<int64_t>(s_) * n) / p);
    } else {
        DArray<int32_t> dc(static_cast<size_t>(p) + 1, s);
        k_nnz_cuts<<<grid_for(p + 1, B), B, 0, s>>>(g->row_off.get(), n, g->m, p, dc.get());
        PGABB_HIP(hipGetLastError());
        PGABB_HIP(hipMemcpyAsync(cuts.data(), dc.get(), sizeof(int32_t) * (p + 1), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
    }

    // Ranks below `lowest` own no edge (isolated vertices rank first under the
    // degree order), so each stripe's dense row range starts at or after it.
    const int32_t lowest = (g->flags & PGABB_ORDER_BY_ID) ? 0 : static_cast<int32_t>(g->isolated);
    CutTable ct{};
    ct.p = p;
    std::vector<int32_t> base(p);
    for (int32_t i = 0; i <= p; ++i) ct.c[i] = cuts[i];
    for (int32_t i = 0; i < p; ++i) {
        base[i] = std::min(std::max(cuts[i], lowest), cuts[i + 1]);
        ct.base[i] = base[i];
    }

    // drop any previous partition
    g->arena.release();
    g->host_arena.release();
    g->blocks_on_host = false;
    g->blocks.clear();
    g->tasks.clear();
    g->task_counts.clear();
    g->block_of.assign(static_cast<size_t>(p) * p, -1);
    g->p = p;
    g->cuts = cuts;
    g->base = base;
    g->arena_words = 0;

    if (g->m > 0) {
        // ---- block sizes
        const size_t pp = static_cast<size_t>(p) * p;
        DArray<unsigned long long> dnnz(pp, s);
        DArray<unsigned int> drows(pp, s);
        PGABB_HIP(hipMemsetAsync(dnnz.get(), 0, pp * sizeof(unsigned long long), s));
        PGABB_HIP(hipMemsetAsync(drows.get(), 0, pp * sizeof(unsigned int), s));
        k_block_sizes<<<cap_grid(n), B, 0, s>>>(g->row_off.get(), g->col.get(), n, ct, dnnz.get(), drows.get());
        PGABB_HIP(hipGetLastError());
        std::vector<unsigned long long> hnnz(pp);
        std::vector<unsigned int> hrows(pp);
        PGABB_HIP(hipMemcpyAsync(hnnz.data(), dnnz.get(), pp * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipMemcpyAsync(hrows.data(), drows.get(), pp * sizeof(unsigned int), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));

        // ---- block table (row-major block order), chunk and slot layout
        std::vector<int64_t> slot_base_pp(pp, -1);
        std::vector<int64_t> slot_base_dense, chunk_off_dense;
        std::vector<int32_t> width_dense, nrows_dense;
        int64_t nslots = 0, words = 0;
        for (int32_t i = 0; i < p; ++i) {
            for (int32_t j = 0; j < p; ++j) {
                const size_t q = static_cast<size_t>(i) * p + j;
                if (!hnnz[q]) continue;
                PGABB_REQUIRE(i <= j, PGABB_EDEVICE, "entry below the diagonal in block (%d, %d)", i, j);
                BlockInfo bi;
                bi.i = i;
                bi.j = j;
                bi.width = cuts[i + 1] - base[i];
                bi.nitems = static_cast<int32_t>(hrows[q]);
                bi.nnz = static_cast<int64_t>(hnnz[q]);
                bi.chunk_off = words;
                bi.chunk_len = block_chunk_words(bi.width, bi.nitems, bi.nnz);
                words += bi.chunk_len;
                g->block_of[q] = static_cast<int32_t>(g->blocks.size());
                g->blocks.push_back(bi);
                slot_base_pp[q] = nslots;
                slot_base_dense.push_back(nslots);
                chunk_off_dense.push_back(bi.chunk_off);
                width_dense.push_back(bi.width);
                nrows_dense.push_back(bi.nitems);
                nslots += static_cast<int64_t>(bi.width) + 1;
            }
        }
        const int32_t nblk = static_cast<int32_t>(g->blocks.size());
        g->arena_words = words;
        g->arena.reset(static_cast<size_t>(words), s);

        DArray<int64_t> d_sb_pp(pp, s), d_sb(nblk, s), d_co(nblk, s);
        DArray<int32_t> d_w(nblk, s), d_nr(nblk, s), d_bidx(pp, s);
        PGABB_HIP(hipMemcpyAsync(d_sb_pp.get(), slot_base_pp.data(), pp * sizeof(int64_t), hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(d_sb.get(), slot_base_dense.data(), nblk * sizeof(int64_t), hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(d_co.get(), chunk_off_dense.data(), nblk * sizeof(int64_t), hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(d_w.get(), width_dense.data(), nblk * sizeof(int32_t), hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(d_nr.get(), nrows_dense.data(), nblk * sizeof(int32_t), hipMemcpyHostToDevice, s));
        PGABB_HIP(hipMemcpyAsync(d_bidx.get(), g->block_of.data(), pp * sizeof(int32_t), hipMemcpyHostToDevice, s));

        // ---- dense row offsets: per-row counts at their slots, one global scan
        DArray<uint32_t> slots(static_cast<size_t>(nslots) + 1, s), flags(static_cast<size_t>(nslots) + 1, s);
        PGABB_HIP(hipMemsetAsync(slots.get(), 0, (nslots + 1) * sizeof(uint32_t), s));
        k_row_slot_counts<<<cap_grid(n), B, 0, s>>>(g->row_off.get(), g->col.get(), n, ct, d_sb_pp.get(), slots.get());
        PGABB_HIP(hipGetLastError());
        scan_exclusive_u32(slots.get(), slots.get(), nslots + 1, nullptr, s);
        const size_t lds = static_cast<size_t>(nblk) * sizeof(int64_t);
        k_fill_rptr<<<cap_grid(nslots), B, lds, s>>>(slots.get(), nslots, d_sb.get(), d_co.get(), d_w.get(), nblk,
                                                     g->arena.get(), flags.get());
        PGABB_HIP(hipGetLastError());
        // ---- item lists: each row's items at the scanned item offsets
        PGABB_HIP(hipMemsetAsync(flags.get() + nslots, 0, sizeof(uint32_t), s));
        scan_exclusive_u32(flags.get(), slots.get(), nslots + 1, nullptr, s);  // reuse slots as positions
        k_fill_items<<<cap_grid(nslots), B, lds, s>>>(flags.get(), slots.get(), nslots, d_sb.get(), d_co.get(), d_w.get(),
                                                    nblk, g->arena.get());
        PGABB_HIP(hipGetLastError());
        // ---- column entries
        k_fill_cols<<<cap_grid(n), B, 0, s>>>(g->row_off.get(), g->col.get(), n, ct, d_bidx.get(), d_co.get(), d_w.get(),
                                              d_nr.get(), g->arena.get());
        PGABB_HIP(hipGetLastError());

        // ---- tasks: i <= j <= k with three non-empty blocks
        for (int32_t i = 0; i < p; ++i)
            for (int32_t j = i; j < p; ++j) {
                const int32_t bij = g->block_of[static_cast<size_t>(i) * p + j];
                if (bij < 0) continue;
                for (int32_t k = j; k < p; ++k) {
                    const int32_t bik = g->block_of[static_cast<size_t>(i) * p + k];
                    const int32_t bjk = g->block_of[static_cast<size_t>(j) * p + k];
                    if (bik < 0 || bjk < 0) continue;
                    Task t{i, j, k, bij, bik, bjk,
                           g->blocks[bij].nnz + g->blocks[bik].nnz + g->blocks[bjk].nnz};
                    g->tasks.push_back(t);
                }
            }
        std::stable_sort(g->tasks.begin(), g->tasks.end(),
                         [](const Task &a, const Task &b) { return a.weight > b.weight; });
        PGABB_HIP(hipStreamSynchronize(s));
    }
    g->task_counts.assign(g->tasks.size(), 0);
    g->t_partition_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace pgabb
