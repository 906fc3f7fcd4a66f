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

// The cut table of nnz-balanced cuts, built on the device (one workgroup):
// cut s is the first row x whose CSR offset reaches s * m' / p, and stripe
// s's dense row range starts at max(cut s, lowest) (clamped to the stripe).
__global__ __launch_bounds__(B) void k_nnz_cut_table(const int64_t *__restrict__ row_off, int32_t n,
                                                     int64_t m, int32_t p, int32_t lowest,
                                                     CutTable *__restrict__ ct) {
    __shared__ int32_t s_c[kMaxP + 1];
    for (int32_t s = threadIdx.x; s <= p; s += B) {
        int32_t c;
        if (s == 0) {
            c = 0;
        } else if (s == p) {
            c = n;
        } else {
            // smallest x in [0, n] with row_off[x] * p >= s * m
            int64_t lo = 0, hi = n;
            const int64_t target = static_cast<int64_t>(s) * m;  // < 2^38 for m' < 2^32
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (row_off[mid] * p >= target) hi = mid;
                else lo = mid + 1;
            }
            c = static_cast<int32_t>(lo);
        }
        s_c[s] = c;
        ct->c[s] = c;
    }
    __syncthreads();
    for (int32_t s = threadIdx.x; s < p; s += B) ct->base[s] = min(max(s_c[s], lowest), s_c[s + 1]);
    if (threadIdx.x == 0) ct->p = p;
}

// The row walks below give each row to one wavefront: rows of the reversed
// graph (in-edges) reach tens of thousands of entries on skewed graphs.
// Lane l of the wave handles stripe j0 + l of the row's column stripes
// [j0, j1] (p <= 64), finding the run of that stripe by binary search in the
// sorted row; per-entry work strides the row 64 entries at a time.

// First index in [lo, hi) whose column is >= c (hi when none).
__device__ __forceinline__ int64_t first_at_least(const int32_t *__restrict__ col, int64_t lo,
                                                  int64_t hi, int32_t c) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Stripe of x from cuts held in LDS (largest s < p with c[s] <= x).
__device__ __forceinline__ int32_t stripe_lds(int32_t x, const int32_t *c, int32_t p) {
    int32_t lo = 0, hi = p - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (c[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct RowRun {
    int32_t si, j;   // row stripe; this lane's column stripe
    int64_t lo, hi;  // this lane's run [lo, hi) (empty when lo == hi)
};

// Row x's run in stripe j0 + lane (a long row: more than 64 entries).
// Every lane calls it for the same x.  Each lane finds where its stripe
// starts; its run ends where the next lane's starts.  The search is first
// narrowed by 64 evenly spaced samples of the row, read in one load: lane
// j counts the samples below c[j] with one ballot per stripe of the row.
__device__ __forceinline__ RowRun row_run(const int32_t *__restrict__ col, int64_t e0, int64_t e1,
                                          int32_t x, const int32_t *c, int32_t p) {
    RowRun r;
    const int lane = lane_id();
    r.si = stripe_lds(x, c, p);
    const int32_t j0 = stripe_lds(col[e0], c, p);
    const int32_t j1 = stripe_lds(col[e1 - 1], c, p);
    r.j = j0 + lane;
    const int64_t len = e1 - e0;
    auto sample_at = [&](int q) { return e0 + ((static_cast<int64_t>(q) * len) >> 6); };
    const int32_t sv = col[sample_at(lane)];
    int below = 0;  // samples whose column is below c[r.j]
    for (int32_t k = 1; k <= j1 - j0; ++k) {
        const uint64_t m = __ballot(sv < c[j0 + k]);
        if (lane == k) below = __popcll(m);
    }
    int64_t start = e0;
    if (lane >= 1 && r.j <= j1) {
        // samples 0 .. below-1 lie below c[r.j] (sample 0 is e0, in stripe
        // j0 < r.j, so below >= 1) and sample `below` (or e1) does not
        const int64_t lo = sample_at(below - 1) + 1;
        const int64_t hi = below < 64 ? sample_at(below) : e1;
        start = first_at_least(col, lo, hi, c[r.j]);
    }
    const int64_t next = __shfl(start, lane < 63 ? lane + 1 : 63);
    r.lo = r.hi = 0;
    if (r.j <= j1) {
        r.lo = start;
        r.hi = r.j == j1 ? e1 : next;
    }
    return r;
}

// Rows are walked in two kinds of launch: short rows (at most kLongRow
// entries) a thread each, or 64 at a time per wave with their entries
// flattened over the lanes; long rows, collected into a device list first,
// by one wave each, lane l finding the run of stripe j0 + l by binary
// search.
constexpr int64_t kLongRow = 64;

// Calls f(si, j, lo, hi) for every non-empty run [lo, hi) of row x (a short
// row) in column stripe j.
template <class F>
__device__ __forceinline__ void short_row_runs(const int32_t *__restrict__ col, int64_t e0,
                                               int64_t e1, int32_t x, const int32_t *c,
                                               int32_t p, F f) {
    const int32_t si = stripe_lds(x, c, p);
    int32_t j = stripe_lds(col[e0], c, p);
    int64_t lo = e0;
    for (int64_t e = e0; e < e1; ++e) {
        const int32_t y = col[e];
        if (y >= c[j + 1]) {
            f(si, j, lo, e);
            lo = e;
            j = stripe_lds(y, c, p);
        }
    }
    f(si, j, lo, e1);
}

// The short rows, a thread each: calls g(x, e0, e1) for every non-empty row
// x of at most kLongRow entries.
template <class G>
__device__ __forceinline__ void for_short_rows(const int64_t *__restrict__ row_off, int32_t n, G g) {
    for (int64_t x = blockIdx.x * int64_t(B) + threadIdx.x; x < n; x += int64_t(gridDim.x) * B) {
        const int64_t e0 = row_off[x], e1 = row_off[x + 1];
        if (e0 == e1 || e1 - e0 > kLongRow) continue;
        g(static_cast<int32_t>(x), e0, e1);
    }
}

// Counting kernels, which act once per run, walk each short row with one
// thread (a run needs one comparison per entry); kernels that write every
// entry take the rows' entries flattened instead:
//
// The short rows (at most kLongRow entries) of all rows, 64 consecutive rows
// per wave, their entries flattened: the wave's short rows are numbered
// through by a scan of their lengths (long rows count as empty), and lane l
// takes flattened entry 64 k + l, finding its row by a search of the
// prefix sums in LDS and the start of its run (row x, column stripe j) from
// the run starts of the chunk (one ballot) or, for a run begun in an
// earlier chunk, the carried start.  Calls f(x, si, j, e, y, lo) for every
// entry e = (x, y) of a short row, lo being the first entry of its run.
// Every lane of the workgroup must call it.  Without RUNS, only x, e and y
// are meaningful (no stripes are looked up).
template <bool RUNS = true, class F>
__device__ __forceinline__ void flat_short_rows(const int64_t *__restrict__ row_off,
                                                const int32_t *__restrict__ col, int32_t n,
                                                const int32_t *c, int32_t p, F f) {
    __shared__ int32_t s_pre[B / 64][65];  // flattened start of each row, then the total
    __shared__ int64_t s_e0[B / 64][64];   // first entry of each row
    __shared__ int32_t s_si[B / 64][64];   // row stripes
    const int w = threadIdx.x >> 6, lane = lane_id();
    const uint64_t le_mask = lane == 63 ? ~0ull : ((2ull << lane) - 1);
    const int64_t stride = int64_t(gridDim.x) * B;
    for (int64_t x0 = blockIdx.x * int64_t(B) + (threadIdx.x & ~63); x0 < n; x0 += stride) {
        const int64_t x = x0 + lane;
        const int64_t e0 = x < n ? row_off[x] : 0;
        const int64_t e1 = x < n ? row_off[x + 1] : 0;
        const int32_t len = (e1 - e0 <= kLongRow) ? static_cast<int32_t>(e1 - e0) : 0;
        const int32_t incl = wave_inclusive_scan(len);
        s_pre[w][lane] = incl - len;
        if (lane == 63) s_pre[w][64] = incl;
        s_e0[w][lane] = e0;
        s_si[w][lane] = (RUNS && x < n) ? stripe_lds(static_cast<int32_t>(x), c, p) : 0;
        wave_lds_sync();
        const int32_t total = s_pre[w][64];
        int64_t carry = 0;
        for (int32_t base = 0; base < total; base += kWave) {
            const int32_t t = base + lane;
            const bool valid = t < total;
            int r = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1)
                if (s_pre[w][r + step] <= t) r += step;
            const int64_t rs = s_e0[w][r];
            const int64_t e = rs + (t - s_pre[w][r]);
            const int32_t y = valid ? col[e] : 0;
            int32_t j = 0;
            int64_t lo = 0;
            if (RUNS) {
                j = stripe_lds(y, c, p);
                const bool is_start = valid && (e == rs || col[e > rs ? e - 1 : rs] < c[j]);
                const uint64_t starts = __ballot(is_start);
                const uint64_t mine = starts & le_mask;
                // entry number of the lane's run start: runs never cross rows,
                // so the flattened distance back to the start is e - lo
                const int32_t back = mine ? lane - (63 - __clzll(mine)) : lane + 1 + static_cast<int32_t>(carry);
                lo = e - back;
                if (starts) carry = 63 - (63 - __clzll(starts));
                else carry += kWave;
            }
            if (valid) f(static_cast<int32_t>(x0 + r), s_si[w][r], j, e, y, lo);
        }
        wave_lds_sync();
    }
}

// Long rows are cut into chunks of at most kChunk entries, listed as
// (row << 32 | chunk index), so that a hub row of the reversed graph spreads
// over many waves.
constexpr int64_t kChunk = 2048;

__global__ void k_collect_long(const int64_t *__restrict__ row_off, int32_t n,
                               int64_t *__restrict__ list, unsigned int *__restrict__ count) {
    for (int64_t x = blockIdx.x * int64_t(B) + threadIdx.x; x < n; x += int64_t(gridDim.x) * B) {
        const int64_t len = row_off[x + 1] - row_off[x];
        if (len <= kLongRow) continue;
        const unsigned int nch = static_cast<unsigned int>((len + kChunk - 1) / kChunk);
        const unsigned int at = atomicAdd(count, nch);
        for (unsigned int c = 0; c < nch; ++c) list[at + c] = (x << 32) | c;
    }
}

// Capacity of the chunk list: every long row adds one chunk plus one per
// kChunk entries.
inline size_t long_list_capacity(int32_t n, int64_t m) {
    return static_cast<size_t>(n) + static_cast<size_t>(m / kChunk) + 1;
}

// The listed chunks of long rows, a wave at a time.  Calls g(x, e0, e1, c0,
// c1) with the row's entries [e0, e1) and the entries [c0, c1) this call
// owns, uniformly across the wave.
template <class G>
__device__ __forceinline__ void for_long_rows(const int64_t *__restrict__ row_off,
                                              const int64_t *__restrict__ list,
                                              const unsigned int *__restrict__ count, G g) {
    const int64_t nwaves = (int64_t(gridDim.x) * B) >> 6;
    const int64_t nl = *count;
    for (int64_t i = (blockIdx.x * int64_t(B) + threadIdx.x) >> 6; i < nl; i += nwaves) {
        const int64_t v = list[i];
        const int32_t x = static_cast<int32_t>(v >> 32);
        const int64_t e0 = row_off[x], e1 = row_off[x + 1];
        const int64_t c0 = e0 + (v & 0xffffffffll) * kChunk;
        const int64_t c1 = c0 + kChunk < e1 ? c0 + kChunk : e1;
        g(x, e0, e1, c0, c1);
    }
}

// Index of the stripe pair {a, b} among the p (p + 1) / 2 unordered pairs.
__device__ __forceinline__ int pair_index(int a, int b, int p) {
    const int lo = min(a, b), hi = max(a, b);
    return lo * (2 * p - lo + 1) / 2 + (hi - lo);
}

constexpr int kMaxPairs = kMaxP * (kMaxP + 1) / 2;

// Per block (i, j): number of entries, of non-empty rows and of work items
// (each row's run split into pieces of at most kSplitV entries).  A pass
// sees blocks on one side of the diagonal only (upper: i <= j, the oriented
// graph; else i >= j, its transpose), so each workgroup accumulates per
// unordered stripe pair in LDS and flushes its non-zero counters to the
// p x p arrays.
template <bool LONG>
__global__ __launch_bounds__(B) void k_block_sizes(const int64_t *__restrict__ row_off,
                                                   const int32_t *__restrict__ col, int32_t n,
                                                   const CutTable *__restrict__ ctp, const int64_t *__restrict__ list,
                                                   const unsigned int *__restrict__ count, bool upper,
                                                   unsigned long long *__restrict__ nnz,
                                                   unsigned int *__restrict__ items,
                                                   unsigned int *__restrict__ rows,
                                                   unsigned long long *__restrict__ walk,
                                                   unsigned int *__restrict__ maxrun) {
    __shared__ unsigned int s_nnz[kMaxPairs];
    __shared__ unsigned int s_items[kMaxPairs];
    __shared__ unsigned int s_rows[kMaxPairs];
    __shared__ unsigned int s_max[kMaxPairs];
    __shared__ int32_t s_c[kMaxP + 1];
    __shared__ unsigned long long s_walk;
    const int p = ctp->p;
    const int pp = p * p;
    const int npairs = p * (p + 1) / 2;
    for (int q = threadIdx.x; q < npairs; q += B) {
        s_nnz[q] = 0;
        s_items[q] = 0;
        s_rows[q] = 0;
        s_max[q] = 0;
    }
    for (int q = threadIdx.x; q <= p; q += B) s_c[q] = ctp->c[q];
    if (threadIdx.x == 0) s_walk = 0;
    __syncthreads();
    // Walked entries when the kernel reads A_ik[x] for every entry (x, y) of
    // A_ij and every k >= j: the run of stripe j has (hi - lo) entries, each
    // walking the (e1 - lo) entries of stripes j and above.
    unsigned long long my_walk = 0;
    int64_t row_end = 0;
    auto add = [&](int32_t si, int32_t j, int64_t lo, int64_t hi) {
        const int64_t cnt = hi - lo;
        if (cnt > 0) {
            const int t = pair_index(si, j, p);
            atomicAdd(&s_nnz[t], static_cast<unsigned int>(cnt));
            atomicAdd(&s_items[t], static_cast<unsigned int>((cnt + kSplitV - 1) / kSplitV));
            atomicAdd(&s_rows[t], 1u);
            atomicMax(&s_max[t], static_cast<unsigned int>(cnt));
            my_walk += static_cast<unsigned long long>(cnt) * static_cast<unsigned long long>(row_end - lo);
        }
    };
    if (LONG) {
        for_long_rows(row_off, list, count, [&](int32_t x, int64_t e0, int64_t e1, int64_t c0, int64_t) {
            row_end = e1;
            if (c0 != e0) return;  // per-row counts: the first chunk only
            const RowRun r = row_run(col, e0, e1, x, s_c, p);
            add(r.si, r.j, r.lo, r.hi);
        });
    } else {
        for_short_rows(row_off, n, [&](int32_t x, int64_t e0, int64_t e1) {
            row_end = e1;
            short_row_runs(col, e0, e1, x, s_c, p, add);
        });
    }
    if (walk) {
        my_walk = wave_sum(my_walk);
        if (lane_id() == 0 && my_walk) atomicAdd(&s_walk, my_walk);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < pp; q += B) {
        const int a = q / p, b = q - a * p;
        if (upper ? a > b : a < b) continue;
        const int t = pair_index(a, b, p);
        if (s_nnz[t]) {
            atomicAdd(&nnz[q], static_cast<unsigned long long>(s_nnz[t]));
            atomicAdd(&items[q], s_items[t]);
            atomicAdd(&rows[q], s_rows[t]);
            if (maxrun) atomicMax(&maxrun[q], s_max[t]);
        }
    }
    if (walk && threadIdx.x == 0 && s_walk) atomicAdd(walk, s_walk);
}

// Per-row entry counts of every block the row touches, written at the row's
// slot of the block's dense row range (slot_base indexed by (row stripe,
// column stripe)).
template <bool LONG>
__global__ __launch_bounds__(B) void k_row_slot_counts(const int64_t *__restrict__ row_off,
                                                       const int32_t *__restrict__ col, int32_t n,
                                                       const CutTable *__restrict__ ctp, const int64_t *__restrict__ list,
                                                       const unsigned int *__restrict__ count,
                                                       const int64_t *__restrict__ slot_base,
                                                       uint32_t *__restrict__ slots) {
    __shared__ int32_t s_c[kMaxP + 1];
    __shared__ int32_t s_base[kMaxP];
    const int p = ctp->p;
    for (int q = threadIdx.x; q <= p; q += B) s_c[q] = ctp->c[q];
    for (int q = threadIdx.x; q < p; q += B) s_base[q] = ctp->base[q];
    __syncthreads();
    auto put = [&](int32_t x, int32_t si, int32_t j, int64_t lo, int64_t hi) {
        if (hi > lo) slots[slot_base[si * p + j] + (x - s_base[si])] = static_cast<uint32_t>(hi - lo);
    };
    if (LONG) {
        for_long_rows(row_off, list, count, [&](int32_t x, int64_t e0, int64_t e1, int64_t c0, int64_t) {
            if (c0 != e0) return;  // per-row counts: the first chunk only
            const RowRun r = row_run(col, e0, e1, x, s_c, p);
            put(x, r.si, r.j, r.lo, r.hi);
        });
    } else {
        for_short_rows(row_off, n, [&](int32_t x, int64_t e0, int64_t e1) {
            short_row_runs(col, e0, e1, x, s_c, p,
                           [&](int32_t si, int32_t j, int64_t lo, int64_t hi) { put(x, si, j, lo, hi); });
        });
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
// number of work items of every row (for the item-list compaction).  The
// region offsets are absolute int32-word offsets in the arena.
__global__ __launch_bounds__(B) void k_fill_rptr(const uint32_t *__restrict__ scanned,
                                                 int64_t nslots,
                                                 const int64_t *__restrict__ slot_base_dense,
                                                 const int64_t *__restrict__ rptr_off,
                                                 const int32_t *__restrict__ width, int32_t nblk,
                                                 int32_t *__restrict__ rbase,
                                                 uint32_t *__restrict__ flags) {
    extern __shared__ int64_t s_sb[];
    for (int q = threadIdx.x; q < nblk; q += B) s_sb[q] = slot_base_dense[q];
    __syncthreads();
    for (int64_t q = blockIdx.x * int64_t(B) + threadIdx.x; q < nslots; q += int64_t(gridDim.x) * B) {
        const int32_t b = block_of_slot(q, s_sb, nblk);
        const int64_t r = q - s_sb[b];
        const uint32_t v = scanned[q] - scanned[s_sb[b]];
        rbase[rptr_off[b] + r] = static_cast<int32_t>(v);
        flags[q] = r < width[b] ? (scanned[q + 1] - scanned[q] + kSplitV - 1) / kSplitV : 0u;
    }
}

__global__ __launch_bounds__(B) void k_fill_items(const uint32_t *__restrict__ flags,
                                                  const uint32_t *__restrict__ pos, int64_t nslots,
                                                  const int64_t *__restrict__ slot_base_dense,
                                                  const int64_t *__restrict__ items_off,
                                                  const int64_t *__restrict__ rptr_off,
                                                  int32_t nblk, const int32_t *__restrict__ rbase,
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
        // the row's entries [start, end) (its dense offsets, written by
        // k_fill_rptr), cut into runs of at most kSplitV
        const int32_t start = rbase[rptr_off[b] + r], end = rbase[rptr_off[b] + r + 1];
        int32_t *it = arena + items_off[b] + kItemWords * static_cast<int64_t>(at);
        for (uint32_t c = 0; c < f; ++c) {
            const int32_t rb = start + static_cast<int32_t>(c) * kSplitV;
            it[kItemWords * c] = static_cast<int32_t>(r);
            it[kItemWords * c + 1] = rb;
            it[kItemWords * c + 2] = min(rb + kSplitV, end);
        }
    }
}

// Entries: row x's run in stripe j goes to the block of (stripe(x), j) at the
// row's dense offset, as local column ids.  In long launches the lane of
// stripe j first computes where entry e of its run lands (dst[j] + e), then
// the wave strides the row's entries.
template <bool LONG>
__global__ __launch_bounds__(B) void k_fill_cols(const int64_t *__restrict__ row_off,
                                                 const int32_t *__restrict__ col, int32_t n,
                                                 const CutTable *__restrict__ ctp, const int64_t *__restrict__ list,
                                                 const unsigned int *__restrict__ count,
                                                 const int32_t *__restrict__ blk_index,
                                                 const int64_t *__restrict__ rptr_off,
                                                 const int64_t *__restrict__ col_off,
                                                 const int32_t *__restrict__ rbase,
                                                 int32_t *__restrict__ arena) {
    __shared__ int32_t s_c[kMaxP + 1];
    __shared__ int32_t s_base[kMaxP];
    __shared__ int64_t s_dst[B / 64][kMaxP];
    const int p = ctp->p;
    for (int q = threadIdx.x; q <= p; q += B) s_c[q] = ctp->c[q];
    for (int q = threadIdx.x; q < p; q += B) s_base[q] = ctp->base[q];
    __syncthreads();
    const int w = threadIdx.x >> 6;
    const int lane = lane_id();
    if (!LONG) {
        flat_short_rows(row_off, col, n, s_c, p,
                        [&](int32_t x, int32_t si, int32_t j, int64_t e, int32_t y, int64_t lo) {
                            const int32_t b = blk_index[si * p + j];
                            arena[col_off[b] + rbase[rptr_off[b] + (x - s_base[si])] + (e - lo)] = y - s_base[j];
                        });
        return;
    }
    for_long_rows(row_off, list, count, [&](int32_t x, int64_t e0, int64_t e1, int64_t c0, int64_t c1) {
        const RowRun r = row_run(col, e0, e1, x, s_c, p);
        if (r.hi > r.lo) {
            const int32_t b = blk_index[r.si * p + r.j];
            s_dst[w][lane] = col_off[b] + rbase[rptr_off[b] + (x - s_base[r.si])] - r.lo;
        }
        wave_lds_sync();
        const int32_t j0 = r.j - lane;
        for (int64_t e = c0 + lane; e < c1; e += kWave) {
            const int32_t y = col[e];
            const int32_t j = stripe_lds(y, s_c, p);
            arena[s_dst[w][j - j0] + e] = y - s_base[j];
        }
        wave_lds_sync();
    });
}

// Reversed oriented graph: for every entry (x, y), the key y and the value x.
template <bool LONG>
__global__ __launch_bounds__(B) void k_rev_pairs(const int64_t *__restrict__ row_off,
                                                 const int32_t *__restrict__ col, int32_t n,
                                                 const int64_t *__restrict__ list,
                                                 const unsigned int *__restrict__ count,
                                                 uint32_t *__restrict__ ky, uint32_t *__restrict__ vx) {
    if (!LONG) {
        flat_short_rows<false>(row_off, col, n, nullptr, 0,
                               [&](int32_t x, int32_t, int32_t, int64_t e, int32_t y, int64_t) {
                                   ky[e] = static_cast<uint32_t>(y);
                                   vx[e] = static_cast<uint32_t>(x);
                               });
        return;
    }
    for_long_rows(row_off, list, count, [&](int32_t x, int64_t, int64_t, int64_t c0, int64_t c1) {
        for (int64_t e = c0 + lane_id(); e < c1; e += kWave) {
            ky[e] = static_cast<uint32_t>(col[e]);
            vx[e] = static_cast<uint32_t>(x);
        }
    });
}

__global__ void k_widen32(const int32_t *__restrict__ in, int32_t n, int64_t *__restrict__ out) {
    for (int64_t v = blockIdx.x * int64_t(B) + threadIdx.x; v < n; v += int64_t(gridDim.x) * B)
        out[v] = in[v];
}

unsigned cap_grid(int64_t work) {
    unsigned g = grid_for(work, B);
    return g > 65536u ? 65536u : g;
}

}  // namespace

void partition_graph(pgabb_graph *g, int32_t p, int32_t cut_mode, const int32_t *cuts_host) {
    hipStream_t s = g->stream;
    const int32_t n = g->n;
    if (!g->part_timer) g->part_timer = std::make_unique<StreamTimer>();
    g->part_timer->start(s);

    // ---- cut table, on the device.  Ranks below `lowest` own no edge
    // (isolated vertices rank first under the degree order), so each
    // stripe's dense row range starts at or after it.  The host reads the
    // table back with the block sizes, in one round trip.
    const int32_t lowest = (g->flags & PGABB_ORDER_BY_ID) ? 0 : static_cast<int32_t>(g->isolated);
    DArray<CutTable> dct(1, s);
    if (cuts_host || cut_mode == PGABB_CUT_UNIFORM) {
        Staged<CutTable> hct(1, s);
        CutTable &ct = hct[0];
        ct = CutTable{};
        ct.p = p;
        for (int32_t i = 0; i <= p; ++i)
            ct.c[i] = cuts_host ? cuts_host[i] : static_cast<int32_t>((static_cast<int64_t>(i) * n) / p);
        for (int32_t i = 0; i < p; ++i) ct.base[i] = std::min(std::max(ct.c[i], lowest), ct.c[i + 1]);
        PGABB_HIP(hipMemcpyAsync(dct.get(), hct.get(), sizeof(CutTable), hipMemcpyHostToDevice, s));
    } else {
        k_nnz_cut_table<<<1, B, 0, s>>>(g->row_off.get(), n, g->m, p, lowest, dct.get());
        PGABB_HIP(hipGetLastError());
    }
    const CutTable *ctp = dct.get();
    Staged<CutTable> hct(1, s);
    auto take_cuts = [&]() {
        // after the round trip: the host copy of the cut table
        std::vector<int32_t> cuts(hct[0].c, hct[0].c + p + 1), base(hct[0].base, hct[0].base + p);
        g->cuts = cuts;
        g->base = base;
    };

    // drop any previous partition
    g->arena.release();
    g->host_arena.release();
    g->blocks_on_host = false;
    g->blocks.clear();
    g->tasks.clear();
    g->task_counts.clear();
    g->block_of.assign(static_cast<size_t>(p) * p, -1);
    g->p = p;
    g->cut_mode = cuts_host ? -1 : cut_mode;
    g->arena_words = 0;
    g->probe_work_col = 0;

    if (g->m > 0) {
        const size_t pp = static_cast<size_t>(p) * p;
        const unsigned lgrid = cap_grid(n);
        constexpr unsigned kLongGrid = 1024;  // workgroups of a long-row launch

        // rows longer than kLongRow, of the forward and the reversed graph
        DArray<int64_t> long_f(long_list_capacity(n, g->m), s), long_r(long_list_capacity(n, g->m), s);
        DArray<unsigned int> nlong(2, s);
        PGABB_HIP(hipMemsetAsync(nlong.get(), 0, 2 * sizeof(unsigned int), s));
        k_collect_long<<<lgrid, B, 0, s>>>(g->row_off.get(), n, long_f.get(), nlong.get());
        PGABB_HIP(hipGetLastError());

        // ---- reversed oriented graph (in-edges, sorted by (y, x)): its blocks
        // are the transposes of the forward blocks
        // (row offsets: the scanned in-degrees from the build)
        DArray<int64_t> rev_off(static_cast<size_t>(n) + 1, s);
        DArray<uint32_t> vx(g->m, s), vx_alt(g->m, s);
        const int32_t *rev_col = nullptr;
        {
            DArray<uint32_t> ky(g->m, s), ky_alt(g->m, s);
            k_rev_pairs<false><<<lgrid, B, 0, s>>>(g->row_off.get(), g->col.get(), n, long_f.get(), nlong.get(),
                                                   ky.get(), vx.get());
            k_rev_pairs<true><<<kLongGrid, B, 0, s>>>(g->row_off.get(), g->col.get(), n, long_f.get(), nlong.get(),
                                                      ky.get(), vx.get());
            PGABB_HIP(hipGetLastError());
            // pairs come in CSR order, ascending in x within each y, so a
            // stable sort on y orders them by (y, x)
            const bool alt = radix_sort_u32(ky.get(), ky_alt.get(), vx.get(), vx_alt.get(), g->m, g->nb, s);
            rev_col = reinterpret_cast<const int32_t *>(alt ? vx_alt.get() : vx.get());
            (alt ? vx : vx_alt).release();
            DArray<int64_t> wide(static_cast<size_t>(n), s);
            k_widen32<<<lgrid, B, 0, s>>>(g->indeg.get(), n, wide.get());
            PGABB_HIP(hipGetLastError());
            scan_exclusive_i64(wide.get(), rev_off.get(), n, rev_off.get() + n, s);
        }
        k_collect_long<<<lgrid, B, 0, s>>>(rev_off.get(), n, long_r.get(), nlong.get() + 1);
        PGABB_HIP(hipGetLastError());

        // ---- block sizes, forward (entries, row items) and reversed (column items)
        // one buffer, one clear, one copy back: nnz[pp] nnz_r[pp] (u64) |
        // items[pp] items_r[pp] (u32) | walked entries of column walks (u64) |
        // longest row run per block, non-empty rows, non-empty rows of the
        // transposes (u32 each)
        const size_t nsz = 3 * pp + 1 + (3 * pp + 1) / 2;
        DArray<unsigned long long> dsz(nsz, s);
        PGABB_HIP(hipMemsetAsync(dsz.get(), 0, nsz * sizeof(unsigned long long), s));
        unsigned long long *dnnz = dsz.get(), *dnnz_r = dnnz + pp, *dwalk = dsz.get() + 3 * pp;
        unsigned int *ditems = reinterpret_cast<unsigned int *>(dnnz_r + pp), *ditems_r = ditems + pp;
        unsigned int *dmax = reinterpret_cast<unsigned int *>(dwalk + 1);
        unsigned int *drows = dmax + pp, *drows_r = drows + pp;
        k_block_sizes<false><<<lgrid, B, 0, s>>>(g->row_off.get(), g->col.get(), n, ctp, long_f.get(), nlong.get(),
                                                  true, dnnz, ditems, drows, dwalk, dmax);
        k_block_sizes<true><<<kLongGrid, B, 0, s>>>(g->row_off.get(), g->col.get(), n, ctp, long_f.get(), nlong.get(),
                                                     true, dnnz, ditems, drows, dwalk, dmax);
        k_block_sizes<false><<<lgrid, B, 0, s>>>(rev_off.get(), rev_col, n, ctp, long_r.get(), nlong.get() + 1,
                                                  false, dnnz_r, ditems_r, drows_r, nullptr, nullptr);
        k_block_sizes<true><<<kLongGrid, B, 0, s>>>(rev_off.get(), rev_col, n, ctp, long_r.get(),
                                                     nlong.get() + 1, false, dnnz_r, ditems_r, drows_r, nullptr,
                                                     nullptr);
        PGABB_HIP(hipGetLastError());
        Staged<unsigned long long> hsz(nsz, s);
        PGABB_HIP(hipMemcpyAsync(hsz.get(), dsz.get(), hsz.bytes(), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipMemcpyAsync(hct.get(), dct.get(), sizeof(CutTable), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        take_cuts();
        const std::vector<int32_t> &cuts = g->cuts, &base = g->base;
        const unsigned long long *hnnz = hsz.get();
        const unsigned int *hitems = reinterpret_cast<const unsigned int *>(hsz.get() + 2 * pp);
        const unsigned int *hitems_r = hitems + pp;
        const unsigned int *hmax = reinterpret_cast<const unsigned int *>(hsz.get() + 3 * pp + 1);
        const unsigned int *hrows = hmax + pp, *hrows_r = hrows + pp;
        g->probe_work_col = hsz[3 * pp];

        // ---- block table (row-major block order) and chunk layout
        for (int32_t i = 0; i < p; ++i) {
            for (int32_t j = 0; j < p; ++j) {
                const size_t q = static_cast<size_t>(i) * p + j;
                if (!hnnz[q]) continue;
                PGABB_REQUIRE(i <= j, PGABB_EDEVICE, "entry below the diagonal in block (%d, %d)", i, j);
                BlockInfo bi;
                bi.i = i;
                bi.j = j;
                bi.width = cuts[i + 1] - base[i];
                bi.cwidth = cuts[j + 1] - base[j];
                bi.nitems = static_cast<int32_t>(hitems[q]);
                bi.ncitems = static_cast<int32_t>(hitems_r[static_cast<size_t>(j) * p + i]);
                bi.nnz = static_cast<int64_t>(hnnz[q]);
                bi.max_row = static_cast<int32_t>(hmax[q]);
                bi.nrows = static_cast<int32_t>(hrows[q]);
                bi.ncols = static_cast<int32_t>(hrows_r[static_cast<size_t>(j) * p + i]);
                bi.chunk_off = g->arena_words;
                bi.chunk_len = bi.end() - bi.chunk_off;
                g->arena_words += bi.chunk_len;
                g->block_of[q] = static_cast<int32_t>(g->blocks.size());
                g->blocks.push_back(bi);
            }
        }
        const int32_t nblk = static_cast<int32_t>(g->blocks.size());
        g->arena.reset(static_cast<size_t>(g->arena_words), s);
        // the transposes' dense column offsets, needed only while the chunks
        // are filled
        std::vector<int64_t> coff(static_cast<size_t>(nblk) + 1, 0);
        for (int32_t b = 0; b < nblk; ++b) coff[b + 1] = coff[b] + g->blocks[b].cwidth + 1;
        DArray<int32_t> ctmp(static_cast<size_t>(std::max<int64_t>(coff[nblk], 1)), s);

        // Both passes run the same machinery: per-row run counts at dense
        // slots, one scan (row offsets), per-row item counts, one scan (item
        // lists), then the entries.  The reversed pass fills the transposes.
        // Per-block tables of each pass travel in one pinned host buffer
        // (int64 tables, then int32 tables) and one copy.
        for (int pass = 0; pass < 2; ++pass) {
            const bool rev = pass == 1;
            const int64_t *off = rev ? rev_off.get() : g->row_off.get();
            const int32_t *cl = rev ? rev_col : g->col.get();
            const int64_t *lst = rev ? long_r.get() : long_f.get();
            const unsigned int *nl = nlong.get() + (rev ? 1 : 0);
            // layout: sb_pp[pp] sb_dense[nblk] rptr_off[nblk] items_off[nblk]
            // col_off[nblk] | width[nblk] bidx[pp] (int32)
            const size_t n64 = pp + 4 * static_cast<size_t>(nblk);
            const size_t n32 = static_cast<size_t>(nblk) + pp;
            Staged<int64_t> tab(n64 + (n32 + 1) / 2, s);
            int64_t *sb_pp = tab.get(), *sb_dense = sb_pp + pp, *rptr_off = sb_dense + nblk;
            int64_t *items_off = rptr_off + nblk, *col_off = items_off + nblk;
            int32_t *width = reinterpret_cast<int32_t *>(tab.get() + n64), *bidx = width + nblk;
            std::fill(sb_pp, sb_pp + pp, int64_t(-1));
            std::fill(bidx, bidx + pp, -1);
            int64_t nslots = 0;
            for (int32_t b = 0; b < nblk; ++b) {
                const BlockInfo &bi = g->blocks[b];
                // forward: rows in stripe i, columns in stripe j; reversed: the
                // transpose, rows in stripe j, columns in stripe i
                const size_t q = rev ? static_cast<size_t>(bi.j) * p + bi.i : static_cast<size_t>(bi.i) * p + bi.j;
                sb_pp[q] = nslots;
                bidx[q] = b;
                sb_dense[b] = nslots;
                width[b] = rev ? bi.cwidth : bi.width;
                rptr_off[b] = rev ? coff[b] : bi.off_rptr();
                items_off[b] = rev ? bi.off_citems() : bi.off_items();
                col_off[b] = rev ? bi.off_crow() : bi.off_col();
                nslots += static_cast<int64_t>(width[b]) + 1;
            }
            DArray<int64_t> dtab(tab.size(), s);
            PGABB_HIP(hipMemcpyAsync(dtab.get(), tab.get(), tab.bytes(), hipMemcpyHostToDevice, s));
            const int64_t *d_sb_pp = dtab.get(), *d_sb = d_sb_pp + pp, *d_ro = d_sb + nblk, *d_io = d_ro + nblk;
            const int64_t *d_co = d_io + nblk;
            const int32_t *d_w = reinterpret_cast<const int32_t *>(dtab.get() + n64), *d_bidx = d_w + nblk;

            DArray<uint32_t> slots(static_cast<size_t>(nslots) + 1, s), flags(static_cast<size_t>(nslots) + 1, s);
            PGABB_HIP(hipMemsetAsync(slots.get(), 0, (nslots + 1) * sizeof(uint32_t), s));
            k_row_slot_counts<false><<<lgrid, B, 0, s>>>(off, cl, n, ctp, lst, nl, d_sb_pp, slots.get());
            k_row_slot_counts<true><<<kLongGrid, B, 0, s>>>(off, cl, n, ctp, lst, nl, d_sb_pp, slots.get());
            PGABB_HIP(hipGetLastError());
            scan_exclusive_u32(slots.get(), slots.get(), nslots + 1, nullptr, s);
            const size_t lds = static_cast<size_t>(nblk) * sizeof(int64_t);
            int32_t *rbase = rev ? ctmp.get() : g->arena.get();
            k_fill_rptr<<<cap_grid(nslots), B, lds, s>>>(slots.get(), nslots, d_sb, d_ro, d_w, nblk, rbase,
                                                         flags.get());
            PGABB_HIP(hipGetLastError());
            PGABB_HIP(hipMemsetAsync(flags.get() + nslots, 0, sizeof(uint32_t), s));
            scan_exclusive_u32(flags.get(), slots.get(), nslots + 1, nullptr, s);  // slots now item positions
            k_fill_items<<<cap_grid(nslots), B, lds, s>>>(flags.get(), slots.get(), nslots, d_sb, d_io, d_ro,
                                                          nblk, rbase, g->arena.get());
            PGABB_HIP(hipGetLastError());
            k_fill_cols<false><<<lgrid, B, 0, s>>>(off, cl, n, ctp, lst, nl, d_bidx, d_ro, d_co, rbase,
                                                   g->arena.get());
            k_fill_cols<true><<<kLongGrid, B, 0, s>>>(off, cl, n, ctp, lst, nl, d_bidx, d_ro, d_co, rbase,
                                                      g->arena.get());
            PGABB_HIP(hipGetLastError());
        }

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
        // no wait here: the fills run on while the caller goes on; later
        // work on the stream is ordered after them, and the scratch freed
        // above is reused only after its free's event
    } else {
        PGABB_HIP(hipMemcpyAsync(hct.get(), dct.get(), sizeof(CutTable), hipMemcpyDeviceToHost, s));
        PGABB_HIP(hipStreamSynchronize(s));
        take_cuts();
    }
    g->task_counts.assign(g->tasks.size(), 0);
    g->part_timer->stop(s);
    g->part_time_pending = true;
}

}  // namespace pgabb
