// Device side of the block-list triangle count.
//
// PGAbB Section 3.6: for a block-list (A_ij, A_ik, A_jk) and each edge (u, v)
// of A_ij, the triangles closed inside the list are the common entries of
// row u of A_ik and row v of A_jk; the intersection may be list based or
// hash based.  Here one wavefront takes one work item of A_ij, a run of at
// most kSplitV entries v of a row u:
//   1. stage row u of A_ik (the list every probe of this row is checked
//      against) in the wave's LDS -- an open-addressing hash table, or a
//      bitmap over stripe k's columns -- or leave it in place for binary
//      search when it is too long to stage;
//   2. walk the rows A_jk[v] of all v in A_ij[u] as one flattened sequence:
//      lane l takes element base + l, so every 64-wide load is contiguous
//      within a row and no lane idles on short rows;
//   3. probe each element against the staged row and count hits in
//      registers; the caller reduces across the wave.
#pragma once

#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

enum RowMode : int { kModeHash = 0, kModeSearch = 1, kModeBitmap = 2 };

__device__ __forceinline__ uint32_t hash_slot(int32_t w, int shift) {
    return (static_cast<uint32_t>(w) * 0x9E3779B1u) >> shift;
}

// Membership of w in the sorted list a[lo, hi) by binary search.
__device__ __forceinline__ uint32_t sorted_contains(const int32_t *__restrict__ a, int32_t lo,
                                                    int32_t hi, int32_t w) {
    const int32_t end = hi;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (a[mid] < w) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && a[lo] == w) ? 1u : 0u;
}

// Triangles closed by the entries [vb, ve) of row u of ij inside the
// block-list, per lane (the sum over lanes is the item's count).  `lds` holds
// LDS_WORDS int32 words private to the wave.  Column ids of ik and jk lie in
// [wbase, wbase + width_k).  Every lane of the wave must call this with the
// same arguments.
template <int MODE, int LDS_WORDS, int UNROLL = 4>
__device__ __forceinline__ uint32_t tc_row(const BlockRef &ij, const BlockRef &ik,
                                           const BlockRef &jk, int32_t width_k, int32_t u,
                                           int32_t vb, int32_t ve, int32_t *__restrict__ lds,
                                           int32_t wbase = 0) {
    const int lane = lane_id();
    const int32_t sb = ik.rptr[u], se = ik.rptr[u + 1];
    const int32_t slen = se - sb;
    if (slen == 0 || vb >= ve) return 0u;

    // ---- stage row u of A_ik
    int mode = MODE;
    int shift = 0;
    uint32_t tmask = 0;
    int words = 0;
    if (mode == kModeBitmap) {
        words = (width_k + 31) >> 5;
        if (words > LDS_WORDS) mode = kModeHash;
    }
    if (mode == kModeHash) {
        int lg = 6;
        while ((1 << lg) < 2 * slen) ++lg;
        if ((1 << lg) > LDS_WORDS) {
            mode = kModeSearch;
        } else {
            words = 1 << lg;
            shift = 32 - lg;
            tmask = static_cast<uint32_t>(words - 1);
        }
    }
    if (mode == kModeHash) {
        for (int q = lane; q < words; q += kWave) lds[q] = -1;
        wave_lds_sync();
        for (int32_t idx = sb + lane; idx < se; idx += kWave) {
            const int32_t w = ik.col[idx];
            uint32_t h = hash_slot(w, shift);
            while (atomicCAS(&lds[h], -1, w) != -1) h = (h + 1) & tmask;
        }
        wave_lds_sync();
    } else if (mode == kModeBitmap) {
        for (int32_t idx = sb + lane; idx < se; idx += kWave) {
            const int32_t w = ik.col[idx] - wbase;
            atomicOr(reinterpret_cast<uint32_t *>(&lds[w >> 5]), 1u << (w & 31));
        }
        wave_lds_sync();
    }

    // ---- flattened walk over the rows A_jk[v], v in A_ij[u].  UNROLL
    // chunks of 64 elements are located and loaded before any is probed, so
    // each wave keeps UNROLL independent row loads in flight.
    uint32_t cnt = 0;
    for (int32_t b0 = vb; b0 < ve; b0 += kWave) {
        const int32_t idx = b0 + lane;
        int32_t pb = 0, len = 0;
        if (idx < ve) {
            const int32_t v = ij.col[idx];
            pb = jk.rptr[v];
            len = jk.rptr[v + 1] - pb;
        }
        const int32_t incl = wave_inclusive_scan(len);
        const int32_t pre = incl - len;
        const int32_t total = __shfl(incl, kWave - 1);
        for (int32_t base = 0; base < total; base += UNROLL * kWave) {
            int32_t w[UNROLL];
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) {
                w[q] = -1;
                if (base + q * kWave < total) {  // uniform across the wave
                    const int32_t e = base + q * kWave + lane;
                    // the lane holding e's row: largest l with pre_l <= e
                    int lo = 0;
#pragma unroll
                    for (int step = 32; step >= 1; step >>= 1) {
                        const int cand = lo + step;
                        if (__shfl(pre, cand) <= e) lo = cand;
                    }
                    const int32_t spre = __shfl(pre, lo);
                    const int32_t spb = __shfl(pb, lo);
                    if (e < total) w[q] = jk.col[spb + (e - spre)];
                }
            }
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) {
                const int32_t wq = w[q];
                if (wq < 0) continue;
                if (mode == kModeHash) {
                    uint32_t h = hash_slot(wq, shift);
                    for (;;) {
                        const int32_t sv = lds[h];
                        if (sv == wq) {
                            ++cnt;
                            break;
                        }
                        if (sv < 0) break;
                        h = (h + 1) & tmask;
                    }
                } else if (mode == kModeBitmap) {
                    const int32_t wl = wq - wbase;
                    cnt += (static_cast<uint32_t>(lds[wl >> 5]) >> (wl & 31)) & 1u;
                } else {
                    cnt += sorted_contains(ik.col, sb, se, wq);
                }
            }
        }
    }

    // ---- leave the LDS clean for the next row of this wave
    if (mode == kModeBitmap) {
        wave_lds_sync();
        for (int32_t idx = sb + lane; idx < se; idx += kWave) lds[(ik.col[idx] - wbase) >> 5] = 0;
        wave_lds_sync();
    } else if (mode == kModeHash) {
        wave_lds_sync();
        if (MODE == kModeBitmap) {
            // a bitmap kernel expects zeroed LDS between rows
            for (int q = lane; q < words; q += kWave) lds[q] = 0;
            wave_lds_sync();
        }
    }
    return cnt;
}

}  // namespace pgabb
