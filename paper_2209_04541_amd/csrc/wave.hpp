// Wave64 helpers (CDNA: 64 lanes per wavefront).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace pgabb {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return static_cast<int>(threadIdx.x) & (kWave - 1); }

// Shuffles of 32- and 64-bit integers built from 32-bit lane moves.
template <class T>
__device__ __forceinline__ T shfl_up_t(T v, int d) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = static_cast<uint64_t>(v);
        const uint32_t lo = __shfl_up(static_cast<uint32_t>(u), d);
        const uint32_t hi = __shfl_up(static_cast<uint32_t>(u >> 32), d);
        return static_cast<T>((static_cast<uint64_t>(hi) << 32) | lo);
    } else {
        return static_cast<T>(__shfl_up(static_cast<uint32_t>(v), d));
    }
}

template <class T>
__device__ __forceinline__ T shfl_xor_t(T v, int m) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = static_cast<uint64_t>(v);
        const uint32_t lo = __shfl_xor(static_cast<uint32_t>(u), m);
        const uint32_t hi = __shfl_xor(static_cast<uint32_t>(u >> 32), m);
        return static_cast<T>((static_cast<uint64_t>(hi) << 32) | lo);
    } else {
        return static_cast<T>(__shfl_xor(static_cast<uint32_t>(v), m));
    }
}

template <class T>
__device__ __forceinline__ T shfl_t(T v, int src) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t u = static_cast<uint64_t>(v);
        const uint32_t lo = __shfl(static_cast<uint32_t>(u), src);
        const uint32_t hi = __shfl(static_cast<uint32_t>(u >> 32), src);
        return static_cast<T>((static_cast<uint64_t>(hi) << 32) | lo);
    } else {
        return static_cast<T>(__shfl(static_cast<uint32_t>(v), src));
    }
}

// Inclusive prefix sum of 32-bit values across the 64 lanes of a wave (all
// lanes active), with DPP lane moves only (no LDS traffic): shifts by 1, 2, 4
// and 8 within each row of 16 lanes, then lane 15 of rows 0 and 2 into rows
// 1 and 3, then lane 31 into rows 2 and 3.  A lane whose shifted source lies
// outside its row adds 0.
__device__ __forceinline__ uint32_t wave_scan_dpp(uint32_t x) {
    x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0u, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0u, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Inclusive running maximum of 32-bit values across the 64 lanes of a wave
// (all lanes active), with the lane moves of wave_scan_dpp; a lane whose
// shifted source lies outside its row takes 0.
__device__ __forceinline__ uint32_t wave_max_scan_dpp(uint32_t x) {
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, false)));  // row_shr:1
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, false)));  // row_shr:2
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, false)));  // row_shr:4
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, false)));  // row_shr:8
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x142, 0xa, 0xf, false)));  // row_bcast:15
    x = max(x, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0u, x, 0x143, 0xc, 0xf, false)));  // row_bcast:31
    return x;
}

// Inclusive prefix sum across the 64 lanes of a wave (all lanes active).
template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    if constexpr (sizeof(T) == 4) {
        return static_cast<T>(wave_scan_dpp(static_cast<uint32_t>(x)));
    } else {
        const int lane = lane_id();
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const T y = shfl_up_t(x, d);
            if (lane >= d) x += y;
        }
        return x;
    }
}

// Pointers that reach a kernel through structs in memory are generic to the
// compiler, and loads through generic pointers are flat loads, which count
// against the LDS counter too: every LDS access or lane shuffle after them
// would wait for them.  Loads through these views are global loads.
template <class T>
using gptr = const __attribute__((address_space(1))) T *;

template <class T>
__device__ __forceinline__ gptr<T> as_global(const T *p) {
    return (gptr<T>)(p);
}

// Sum across the wave, returned to every lane.
template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) x += shfl_xor_t(x, m);
    return x;
}

// For the 64 consecutive elements handled by one wave, where equal keys form
// runs (the input is sorted), add each run's length to counter[key] with one
// atomic from the run's first lane.  `valid` lanes must form a prefix.
__device__ __forceinline__ void add_run_lengths(bool valid, int64_t key, int32_t *counter) {
    const int lane = lane_id();
    const uint64_t vmask = __ballot(valid);
    const int nvalid = __popcll(vmask);
    const uint32_t klo = __shfl_up(static_cast<uint32_t>(key), 1);
    const uint32_t khi = __shfl_up(static_cast<uint32_t>(static_cast<uint64_t>(key) >> 32), 1);
    const int64_t prev = static_cast<int64_t>((static_cast<uint64_t>(khi) << 32) | klo);
    const bool start = valid && (lane == 0 || prev != key);
    const uint64_t starts = __ballot(start);
    if (start) {
        const uint64_t after = lane == 63 ? 0ull : (starts & (~0ull << (lane + 1)));
        const int next = after ? __ffsll(static_cast<long long>(after)) - 1 : nvalid;
        atomicAdd(&counter[key], next - lane);
    }
}

// Order LDS accesses of the lanes of one wave: what a lane wrote before the
// call is visible to every lane of the wave after it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace pgabb
