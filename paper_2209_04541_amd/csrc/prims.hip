// Device-wide primitives used by the build phase: exclusive prefix sums and
// a stable least-significant-digit radix sort.  Written for wave64: digit
// ranks inside a wave come from eight ballots (one per digit bit), so a
// 256-thread workgroup ranks 256 keys per round without per-thread
// histograms.
#include "common.hpp"
#include "wave.hpp"

namespace pgabb {

// ---------------------------------------------------------------- scans

namespace {

constexpr int SC_BLOCK = 256;
constexpr int SC_ITEMS = 8;
constexpr int SC_TILE = SC_BLOCK * SC_ITEMS;

template <class T>
__global__ __launch_bounds__(SC_BLOCK) void k_tile_sums(const T *__restrict__ in, int64_t n,
                                                        T *__restrict__ sums) {
    __shared__ T wt[SC_BLOCK / 64];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SC_TILE;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        int64_t idx = base + i * SC_BLOCK + threadIdx.x;
        if (idx < n) acc += in[idx];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) wt[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int w = 0; w < SC_BLOCK / 64; ++w) t += wt[w];
        sums[blockIdx.x] = t;
    }
}

template <class T>
__global__ __launch_bounds__(SC_BLOCK) void k_tile_scan(const T *in, T *out, int64_t n,
                                                        const T *__restrict__ tile_off,
                                                        T *total_dev) {
    __shared__ T s[SC_TILE];
    __shared__ T wt[SC_BLOCK / 64];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * SC_TILE;
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        int64_t idx = base + i * SC_BLOCK + tid;
        s[i * SC_BLOCK + tid] = idx < n ? in[idx] : T(0);
    }
    __syncthreads();
    T v[SC_ITEMS];
    T run = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        v[i] = run;
        run += s[tid * SC_ITEMS + i];
    }
    // exclusive scan of the per-thread totals across the workgroup
    T incl = wave_inclusive_scan(run);
    const int lane = tid & 63, w = tid >> 6;
    if (lane == 63) wt[w] = incl;
    __syncthreads();
    T wave_off = 0, block_total = 0;
    for (int q = 0; q < SC_BLOCK / 64; ++q) {
        if (q < w) wave_off += wt[q];
        block_total += wt[q];
    }
    T off = (tile_off ? tile_off[blockIdx.x] : T(0)) + wave_off + incl - run;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) s[tid * SC_ITEMS + i] = v[i] + off;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
        int64_t idx = base + i * SC_BLOCK + tid;
        if (idx < n) out[idx] = s[i * SC_BLOCK + tid];
    }
    if (total_dev && blockIdx.x == gridDim.x - 1 && tid == 0)
        *total_dev = (tile_off ? tile_off[blockIdx.x] : T(0)) + block_total;
}

template <class T>
void scan_exclusive(const T *in, T *out, int64_t n, T *total_dev, hipStream_t s) {
    if (n <= 0) {
        if (total_dev) PGABB_HIP(hipMemsetAsync(total_dev, 0, sizeof(T), s));
        return;
    }
    const int64_t ntiles = (n + SC_TILE - 1) / SC_TILE;
    if (ntiles == 1) {
        k_tile_scan<T><<<1, SC_BLOCK, 0, s>>>(in, out, n, nullptr, total_dev);
        PGABB_HIP(hipGetLastError());
        return;
    }
    DArray<T> sums(static_cast<size_t>(ntiles), s);
    k_tile_sums<T><<<grid_for(ntiles * SC_TILE, SC_TILE), SC_BLOCK, 0, s>>>(in, n, sums.get());
    PGABB_HIP(hipGetLastError());
    scan_exclusive<T>(sums.get(), sums.get(), ntiles, nullptr, s);
    k_tile_scan<T><<<static_cast<unsigned>(ntiles), SC_BLOCK, 0, s>>>(in, out, n, sums.get(), total_dev);
    PGABB_HIP(hipGetLastError());
}

}  // namespace

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total_dev,
                        hipStream_t s) {
    scan_exclusive<uint32_t>(in, out, n, total_dev, s);
}

void scan_exclusive_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev,
                        hipStream_t s) {
    scan_exclusive<int64_t>(in, out, n, total_dev, s);
}

// ----------------------------------------------------------- radix sort

namespace {

constexpr int RS_BLOCK = 256;
constexpr int RS_WAVES = RS_BLOCK / 64;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_BLOCK * RS_ITEMS;
constexpr int RS_BINS = 256;

// Tile layout: wave w of the workgroup owns the 1024 consecutive keys
// [base + w * 1024, base + (w + 1) * 1024) of the tile, item i of lane l
// being key base + w * 1024 + i * 64 + l.  Every load is 64 consecutive
// keys, and the wave-major order is the keys' own order, which keeps the
// scatter stable.
__device__ __forceinline__ int64_t rs_index(int64_t base, int w, int i, int lane) {
    return base + static_cast<int64_t>(w) * (RS_ITEMS * 64) + i * 64 + lane;
}

// The lanes of the wave holding the same digit d (< 256, valid lanes only):
// eight ballots, one per digit bit.
__device__ __forceinline__ uint64_t rs_peers(bool valid, uint32_t d) {
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        same &= bit ? bb : ~bb;
    }
    return same;
}

// Per-tile digit histogram, written digit-major: hist[d * ntiles + tile].
template <class K>
__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const K *__restrict__ keys, int64_t n,
                                                      int shift, uint32_t mask,
                                                      uint32_t *__restrict__ hist,
                                                      uint32_t ntiles) {
    __shared__ uint32_t h[RS_WAVES][RS_BINS];
    const int tid = threadIdx.x, w = tid >> 6;
    for (int i = tid; i < RS_WAVES * RS_BINS; i += RS_BLOCK) (&h[0][0])[i] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * RS_TILE;
#pragma unroll 4
    for (int i = 0; i < RS_ITEMS; ++i) {
        int64_t idx = base + i * RS_BLOCK + tid;
        if (idx < n) atomicAdd(&h[w][static_cast<uint32_t>(keys[idx] >> shift) & mask], 1u);
    }
    __syncthreads();
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < RS_WAVES; ++q) c += h[q][tid];
    hist[static_cast<size_t>(tid) * ntiles + blockIdx.x] = c;
}

// One workgroup per digit d: the exclusive scan of hist[d][0 .. ntiles) in
// place (keys of digit d in earlier tiles) and the digit's total in tot[d].
__global__ __launch_bounds__(RS_BLOCK) void k_rs_rowscan(uint32_t *__restrict__ hist, uint32_t ntiles,
                                                         uint32_t *__restrict__ tot) {
    constexpr int ITEMS = 8, CHUNK = RS_BLOCK * ITEMS;
    __shared__ uint32_t s[CHUNK];
    __shared__ uint32_t wt[RS_WAVES];
    uint32_t *row = hist + static_cast<size_t>(blockIdx.x) * ntiles;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < ntiles; base += CHUNK) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = base + i * RS_BLOCK + tid;
            s[i * RS_BLOCK + tid] = idx < ntiles ? row[idx] : 0u;
        }
        __syncthreads();
        uint32_t v[ITEMS], run = 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            v[i] = run;
            run += s[tid * ITEMS + i];
        }
        const uint32_t incl = wave_inclusive_scan(run);
        if (lane == 63) wt[w] = incl;
        __syncthreads();
        uint32_t off = carry, chunk_total = 0;
        for (int q = 0; q < RS_WAVES; ++q) {
            if (q < w) off += wt[q];
            chunk_total += wt[q];
        }
        off += incl - run;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) s[tid * ITEMS + i] = v[i] + off;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = base + i * RS_BLOCK + tid;
            if (idx < ntiles) row[idx] = s[i * RS_BLOCK + tid];
        }
        carry += chunk_total;
        __syncthreads();
    }
    if (tid == 0) tot[blockIdx.x] = carry;
}

// Stable scatter of one tile: each wave ranks its keys by digit with
// running per-digit counts of its own (no workgroup barrier per item), the
// tile's digit offsets follow from one scan, the tile is staged in digit
// order in LDS, and each digit run is written to its global offset
// (consecutive threads write consecutive addresses within a run).
template <class K, bool HAS_V>
__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const K *__restrict__ kin,
                                                         K *__restrict__ kout,
                                                         const uint32_t *__restrict__ vin,
                                                         uint32_t *__restrict__ vout, int64_t n,
                                                         int shift, uint32_t mask,
                                                         const uint32_t *__restrict__ hist,
                                                         const uint32_t *__restrict__ tot,
                                                         uint32_t ntiles) {
    __shared__ K sk[RS_TILE];
    __shared__ uint32_t sv[HAS_V ? RS_TILE : 1];
    __shared__ uint32_t tile_pre[RS_BINS];
    __shared__ uint32_t gofs[RS_BINS];
    __shared__ uint32_t wcnt[RS_WAVES][RS_BINS];
    __shared__ uint32_t wtot[RS_WAVES];

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * RS_TILE;
    for (int i = lane; i < RS_BINS; i += 64) wcnt[w][i] = 0;
    {
        // global offset of this tile's digit-tid keys: all keys of lower
        // digits (a scan of the digit totals) plus this digit's keys in
        // earlier tiles (the row scan)
        const uint32_t t = tid <= static_cast<int>(mask) ? tot[tid] : 0u;
        const uint32_t incl = wave_inclusive_scan(t);
        if (lane == 63) wtot[w] = incl;
        __syncthreads();
        uint32_t below = incl - t;
        for (int q = 0; q < w; ++q) below += wtot[q];
        gofs[tid] = tid <= static_cast<int>(mask)
                        ? below + hist[static_cast<size_t>(tid) * ntiles + blockIdx.x] : 0u;
        __syncthreads();
    }

    K key[RS_ITEMS];
    uint32_t val[HAS_V ? RS_ITEMS : 1];
    uint32_t pos[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t idx = rs_index(base, w, i, lane);
        key[i] = idx < n ? kin[idx] : K(0);
        if constexpr (HAS_V) val[i] = idx < n ? vin[idx] : 0u;
    }
    wave_lds_sync();

    // ---- rank inside the wave: earlier items, then lower lanes
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const bool valid = rs_index(base, w, i, lane) < n;
        const uint32_t d = valid ? (static_cast<uint32_t>(key[i] >> shift) & mask) : 0u;
        const uint64_t same = rs_peers(valid, d);
        const uint32_t below = static_cast<uint32_t>(__popcll(same & lt_mask));
        const uint32_t seen = valid ? wcnt[w][d] : 0u;  // every lane reads before the update
        wave_lds_sync();
        if (valid && below == 0) wcnt[w][d] = seen + static_cast<uint32_t>(__popcll(same));
        wave_lds_sync();
        pos[i] = seen + below;
    }
    __syncthreads();

    // ---- per digit (one per thread): the waves' counts and the tile scan
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < RS_WAVES; ++q) {
        const uint32_t x = wcnt[q][tid];
        wcnt[q][tid] = c;  // now: keys of this digit in earlier waves
        c += x;
    }
    const uint32_t incl = wave_inclusive_scan(c);
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int q = 0; q < w; ++q) off += wtot[q];
    tile_pre[tid] = off + incl - c;
    __syncthreads();

#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        if (rs_index(base, w, i, lane) < n) {
            const uint32_t d = static_cast<uint32_t>(key[i] >> shift) & mask;
            const uint32_t at = tile_pre[d] + wcnt[w][d] + pos[i];
            sk[at] = key[i];
            if constexpr (HAS_V) sv[at] = val[i];
        }
    }
    __syncthreads();

    const int count = static_cast<int>(min<int64_t>(RS_TILE, n - base));
    for (int e = tid; e < count; e += RS_BLOCK) {
        const K k = sk[e];
        const uint32_t d = static_cast<uint32_t>(k >> shift) & mask;
        const uint32_t dst = gofs[d] + (static_cast<uint32_t>(e) - tile_pre[d]);
        kout[dst] = k;
        if constexpr (HAS_V) vout[dst] = sv[e];
    }
}

template <class K>
bool radix_sort_impl(K *keys, K *keys_alt, uint32_t *vals, uint32_t *vals_alt, int64_t n,
                     int lo_bit, int hi_bit, hipStream_t s) {
    if (n <= 1 || hi_bit <= lo_bit) return false;
    PGABB_REQUIRE(n < (int64_t(1) << 32), PGABB_EINVAL, "radix sort of %lld keys exceeds 2^32",
                  static_cast<long long>(n));
    const uint32_t ntiles = static_cast<uint32_t>((n + RS_TILE - 1) / RS_TILE);
    DArray<uint32_t> hist(static_cast<size_t>(RS_BINS) * ntiles + RS_BINS, s);
    uint32_t *tot = hist.get() + static_cast<size_t>(RS_BINS) * ntiles;
    K *kc = keys, *ko = keys_alt;
    uint32_t *vc = vals, *vo = vals_alt;
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        const int width = hi_bit - shift < 8 ? hi_bit - shift : 8;
        const uint32_t mask = (1u << width) - 1u;
        k_rs_hist<K><<<ntiles, RS_BLOCK, 0, s>>>(kc, n, shift, mask, hist.get(), ntiles);
        k_rs_rowscan<<<mask + 1, RS_BLOCK, 0, s>>>(hist.get(), ntiles, tot);
        PGABB_HIP(hipGetLastError());
        if (vals)
            k_rs_scatter<K, true><<<ntiles, RS_BLOCK, 0, s>>>(kc, ko, vc, vo, n, shift, mask,
                                                               hist.get(), tot, ntiles);
        else
            k_rs_scatter<K, false><<<ntiles, RS_BLOCK, 0, s>>>(kc, ko, nullptr, nullptr, n, shift,
                                                                mask, hist.get(), tot, ntiles);
        PGABB_HIP(hipGetLastError());
        std::swap(kc, ko);
        std::swap(vc, vo);
    }
    return kc == keys_alt;
}

}  // namespace

bool radix_sort_u64(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                    int64_t n, int nbits, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, keys_alt, vals, vals_alt, n, 0, nbits, s);
}

bool radix_sort_u64_bits(uint64_t *keys, uint64_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                         int64_t n, int lo_bit, int hi_bit, hipStream_t s) {
    return radix_sort_impl<uint64_t>(keys, keys_alt, vals, vals_alt, n, lo_bit, hi_bit, s);
}

bool radix_sort_u32(uint32_t *keys, uint32_t *keys_alt, uint32_t *vals, uint32_t *vals_alt,
                    int64_t n, int nbits, hipStream_t s) {
    return radix_sort_impl<uint32_t>(keys, keys_alt, vals, vals_alt, n, 0, nbits, s);
}

}  // namespace pgabb
