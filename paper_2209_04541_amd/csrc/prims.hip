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

// Stable scatter of one tile: rank every key inside the tile by digit, stage
// the tile in digit order in LDS, then write each digit run to its global
// offset (consecutive threads write consecutive addresses within a run).
template <class K, bool HAS_V>
__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const K *__restrict__ kin,
                                                         K *__restrict__ kout,
                                                         const uint32_t *__restrict__ vin,
                                                         uint32_t *__restrict__ vout, int64_t n,
                                                         int shift, uint32_t mask,
                                                         const uint32_t *__restrict__ hist,
                                                         uint32_t ntiles) {
    __shared__ K sk[RS_TILE];
    __shared__ uint32_t sv[HAS_V ? RS_TILE : 1];
    __shared__ uint32_t run[RS_BINS];
    __shared__ uint32_t tile_pre[RS_BINS];
    __shared__ uint32_t gofs[RS_BINS];
    __shared__ uint32_t wcnt[RS_WAVES][RS_BINS];
    __shared__ uint32_t wtot[RS_WAVES];

    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * RS_TILE;

    run[tid] = 0;
#pragma unroll
    for (int q = 0; q < RS_WAVES; ++q) wcnt[q][tid] = 0;
    gofs[tid] = hist[static_cast<size_t>(tid) * ntiles + blockIdx.x];

    K key[RS_ITEMS];
    uint32_t val[HAS_V ? RS_ITEMS : 1];
    uint32_t pos[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        int64_t idx = base + i * RS_BLOCK + tid;
        key[i] = idx < n ? kin[idx] : K(0);
        if constexpr (HAS_V) val[i] = idx < n ? vin[idx] : 0u;
        pos[i] = 0;
    }
    __syncthreads();

    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const bool valid = base + i * RS_BLOCK + tid < n;
        const uint32_t d = valid ? (static_cast<uint32_t>(key[i] >> shift) & mask) : 0u;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            same &= bit ? bb : ~bb;
        }
        const uint32_t rank_w = __popcll(same & lt_mask);
        if (valid && rank_w == 0) wcnt[w][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            uint32_t before = run[d];
            for (int q = 0; q < w; ++q) before += wcnt[q][d];
            pos[i] = before + rank_w;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < RS_WAVES; ++q) {
            add += wcnt[q][tid];
            wcnt[q][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }

    // exclusive scan of the tile's digit counts (one digit per thread)
    const uint32_t c = run[tid];
    const uint32_t incl = wave_inclusive_scan(c);
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    uint32_t off = 0;
    for (int q = 0; q < w; ++q) off += wtot[q];
    tile_pre[tid] = off + incl - c;
    __syncthreads();

#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        if (base + i * RS_BLOCK + tid < n) {
            const uint32_t d = static_cast<uint32_t>(key[i] >> shift) & mask;
            const uint32_t at = tile_pre[d] + pos[i];
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
    DArray<uint32_t> hist(static_cast<size_t>(RS_BINS) * ntiles, s);
    K *kc = keys, *ko = keys_alt;
    uint32_t *vc = vals, *vo = vals_alt;
    for (int shift = lo_bit; shift < hi_bit; shift += 8) {
        const int width = hi_bit - shift < 8 ? hi_bit - shift : 8;
        const uint32_t mask = (1u << width) - 1u;
        k_rs_hist<K><<<ntiles, RS_BLOCK, 0, s>>>(kc, n, shift, mask, hist.get(), ntiles);
        PGABB_HIP(hipGetLastError());
        scan_exclusive_u32(hist.get(), hist.get(), static_cast<int64_t>(RS_BINS) * ntiles, nullptr, s);
        if (vals)
            k_rs_scatter<K, true><<<ntiles, RS_BLOCK, 0, s>>>(kc, ko, vc, vo, n, shift, mask,
                                                               hist.get(), ntiles);
        else
            k_rs_scatter<K, false><<<ntiles, RS_BLOCK, 0, s>>>(kc, ko, nullptr, nullptr, n, shift,
                                                                mask, hist.get(), ntiles);
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
