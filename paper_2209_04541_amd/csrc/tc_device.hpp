// Device side of the block-list triangle count.
//
// PGAbB Section 3.6: for a block-list (A_ij, A_ik, A_jk) and each edge (u, v)
// of A_ij, the triangles closed inside the list are the common entries of
// row u of A_ik and row v of A_jk; the intersection may be list based or
// hash based.  Here one wavefront takes one work item of A_ij: a run of at
// most kSplitV entries v of a row u (stage A_ik[u], walk the A_jk[v]), or of
// entries u of a column v (stage A_jk[v], walk the A_ik[u]):
//   1. stage the shared list in the wave's LDS -- an open-addressing hash
//      table behind a bit filter, or a bitmap over stripe k's columns -- or
//      leave it in place for binary search when it is too long to stage;
//   2. walk the other lists as one flattened sequence: lane l takes element
//      base + l, so every 64-wide load is contiguous within a list and no
//      lane idles on short lists;
//   3. probe each element against the staged list and count hits in
//      registers; the caller reduces across the wave.
#pragma once

#include "graph.hpp"
#include "wave.hpp"

namespace pgabb {

enum RowMode : int { kModeHash = 0, kModeSearch = 1, kModeBitmap = 2 };

// Hash and filter slots: Fibonacci hashing modulo 2^24.  A 24-bit multiply
// (full rate on CDNA, where 32-bit integer multiplies are quarter rate) by
// an odd constant near 0.618 * 2^24, keeping the top lg of its low 24 bits:
// slot = floor(frac(w * C / 2^24) * 2^lg).  Ids at or above 2^24 only
// collide more often (the table compares whole values).  __umul24 returns
// int here, so the product is taken as unsigned before the shift.
__device__ __forceinline__ uint32_t hash_slot(int32_t w, int shift, uint32_t mask) {
    return (static_cast<uint32_t>(__umul24(static_cast<uint32_t>(w), 0x9E3779u)) >> shift) & mask;
}

__device__ __forceinline__ uint32_t filter_slot(int32_t w, int fshift, uint32_t fmask) {
    return (static_cast<uint32_t>(__umul24(static_cast<uint32_t>(w), 0xC13FA9u)) >> fshift) & fmask;
}

// Membership of w in the sorted list a[lo, hi) by binary search.
__device__ __forceinline__ uint32_t sorted_contains(gptr<int32_t> a, int32_t lo, int32_t hi, int32_t w) {
    const int32_t end = hi;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (a[mid] < w) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && a[lo] == w) ? 1u : 0u;
}

// LDS split of a hash-mode wave region of LDS_WORDS words: a power-of-two
// table of kTableCap words and a membership filter of the rest.  The
// template sizes used are 320, 640, 1280, 2304 and 4352 words.
template <int LDS_WORDS>
struct HashLds {
    static constexpr int kTableCap = LDS_WORDS >= 4352 ? 4096
                                     : LDS_WORDS >= 2304 ? 2048
                                     : LDS_WORDS >= 1280 ? 1024
                                     : LDS_WORDS >= 640 ? 512
                                     : LDS_WORDS >= 320 ? 256 : 64;
    static constexpr int kFilterCap = LDS_WORDS - kTableCap;  // words
};

// How one item's staged list S is held, fixed before the walk.
struct Staging {
    int shift = 0, fshift = 0;  // hash and filter slot shifts (24 - lg)
    uint32_t tmask = 0;         // table size - 1
    uint32_t fmask = 0;         // filter bits - 1
    int words = 0, fwords = 0;  // table (or bitmap) and filter words
    int32_t *table = nullptr;   // hash table, after the filter
};

// Loads elements base + q * 64 + lane (q < UNROLL) of the flattened walk over
// the lists of one group of up to 64 ids (lane l: list wk_col[pb .. pb +
// len), at position pre of the walk); past the group's end a lane gets -1.
// The lane whose list holds an element is found without a search: every
// list that starts inside the batch writes its lane + 1 at its first
// position in `own` (64 * UNROLL words of the wave's LDS, zero between
// calls, and left zero), and a running maximum over the lanes fills the
// positions in between; `carry` (lane + 1 of the list holding the element
// before the batch) starts at 0 for a new group.  Walked lists are short
// next to a batch on skewed graphs (a batch often crosses several), where
// advancing one list per step cost more.  Every call issues exactly UNROLL
// loads (past the end, of element 0 of wk_col, which exists whenever a walk
// does), so the compiler can wait for one batch while the next is in
// flight.
template <int UNROLL>
__device__ __forceinline__ void walk_load(int32_t (&w)[UNROLL], int32_t base, int32_t total, int32_t pre,
                                          int32_t len, int32_t pb, uint32_t &carry, int32_t *__restrict__ own,
                                          gptr<int32_t> wk_col, int lane) {
    const int32_t p = pre - base;
    if (len > 0 && p >= 0 && p < UNROLL * kWave) own[p] = lane + 1;
    wave_lds_sync();
    uint32_t o[UNROLL];
#pragma unroll
    for (int q = 0; q < UNROLL; ++q) {
        o[q] = static_cast<uint32_t>(own[q * kWave + lane]);
        own[q * kWave + lane] = 0;
    }
    wave_lds_sync();
    const int32_t rel = pb - pre;  // element e of the walk is wk_col[rel + e] for the lane's list
#pragma unroll
    for (int q = 0; q < UNROLL; ++q) {
        const uint32_t sl = max(wave_max_scan_dpp(o[q]), carry);
        carry = __builtin_amdgcn_readlane(sl, kWave - 1);
        const int32_t e = base + q * kWave + lane;
        const bool inb = e < total;
        const int32_t off = __shfl(rel, static_cast<int>(sl) - 1);
        const int32_t x = wk_col[inb ? off + e : 0];
        w[q] = inb ? x : -1;
    }
}

// Items whose staged list has at most this many entries are walked together
// (tiny_items).
constexpr int kTinyCap = 4;

// Counts the items of the lanes in `m` (one task or graph, staged lists of
// at most kTinyCap entries; lane l: ids[b .. e) are its walked lists' ids and
// st_col[sb .. se) its staged list) in one walk instead of one after
// another.  The items' walked lists are flattened over the lanes 64 at a
// time, each list lane finding its item with the scattered lookup and taking
// the item's staged entries (held in registers, -2 padding no element
// matches); the lists' elements are then flattened over the lanes again and
// each is compared with its list's staged entries.  On hypersparse blocks an
// item walks a handful of entries, which a wave walking one item at a time
// spreads over a few of its lanes.
template <int UNROLL>
__device__ __forceinline__ uint32_t tiny_items(uint64_t m, int32_t b, int32_t e, int32_t sb, int32_t se,
                                               const int32_t *st_col_, const int32_t *ids_,
                                               const int32_t *wk_rptr_, const int32_t *wk_col_, int32_t *own,
                                               int lane) {
    const gptr<int32_t> st_col = as_global(st_col_), ids = as_global(ids_);
    const gptr<int32_t> wk_rptr = as_global(wk_rptr_), wk_col = as_global(wk_col_);
    const bool in = (m >> lane) & 1ull;
    int32_t s[kTinyCap];
#pragma unroll
    for (int t = 0; t < kTinyCap; ++t) s[t] = (in && t < se - sb) ? st_col[sb + t] : -2;
    const int32_t nl = in ? e - b : 0;  // walked lists of the lane's item
    const int32_t incl1 = wave_inclusive_scan(nl);
    const int32_t pre1 = incl1 - nl;
    const int32_t nlists = __builtin_amdgcn_readlane(incl1, kWave - 1);
    const int32_t idbase = b - pre1;  // list slot j of the item is ids[idbase + j]
    uint32_t cnt = 0;
    uint32_t carry1 = 0;
    for (int32_t j0 = 0; j0 < nlists; j0 += kWave) {
        // the item of list slot j0 + lane
        const int32_t p = pre1 - j0;
        if (nl > 0 && p >= 0 && p < kWave) own[p] = lane + 1;
        wave_lds_sync();
        const uint32_t o = static_cast<uint32_t>(own[lane]);
        own[lane] = 0;
        wave_lds_sync();
        const uint32_t il1 = max(wave_max_scan_dpp(o), carry1);
        carry1 = __builtin_amdgcn_readlane(il1, kWave - 1);
        const int il = static_cast<int>(il1) - 1;
        const int32_t j = j0 + lane;
        const int32_t ib = __shfl(idbase, il);
        int32_t ls[kTinyCap];
#pragma unroll
        for (int t = 0; t < kTinyCap; ++t) ls[t] = __shfl(s[t], il);
        int32_t pb = 0, len = 0;
        if (j < nlists) {
            const int32_t id = ids[ib + j];
            pb = wk_rptr[id];
            len = wk_rptr[id + 1] - pb;
        }
        // the elements of these lists, flattened over the lanes
        const int32_t incl = wave_inclusive_scan(len);
        const int32_t pre = incl - len;
        const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
        const int32_t rel = pb - pre;  // element x of the run is wk_col[rel + x] for the lane's list
        uint32_t carry = 0;
        for (int32_t base = 0; base < total; base += UNROLL * kWave) {
            const int32_t p2 = pre - base;
            if (len > 0 && p2 >= 0 && p2 < UNROLL * kWave) own[p2] = lane + 1;
            wave_lds_sync();
            uint32_t o2[UNROLL];
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) {
                o2[q] = static_cast<uint32_t>(own[q * kWave + lane]);
                own[q * kWave + lane] = 0;
            }
            wave_lds_sync();
            int32_t y[UNROLL], sl[UNROLL];
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) {
                const uint32_t sl1 = max(wave_max_scan_dpp(o2[q]), carry);
                carry = __builtin_amdgcn_readlane(sl1, kWave - 1);
                sl[q] = static_cast<int>(sl1) - 1;
                const int32_t x = base + q * kWave + lane;
                const bool inb = x < total;
                const int32_t off = __shfl(rel, sl[q]);
                const int32_t v = wk_col[inb ? off + x : 0];
                y[q] = inb ? v : -1;
            }
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) {
                uint32_t hit = 0;
#pragma unroll
                for (int t = 0; t < kTinyCap; ++t) hit |= y[q] == __shfl(ls[t], sl[q]) ? 1u : 0u;
                cnt += hit;
            }
        }
    }
    return cnt;
}

// Items with small staged lists and few walked lists are walked together
// too (packed_items): staged lists of at most kPackS entries, at most
// kPackLists walked lists.
constexpr int kPackS = 64;
constexpr int kPackLists = 8;

// Hash slot of value w of the pack's item il (the item enters the key, so
// equal values of different items fall apart).
__device__ __forceinline__ uint32_t pack_slot(int32_t w, int il, int shift, uint32_t mask) {
    return hash_slot(w + il * 0x3C6EF35, shift, mask);
}

// Counts the items of the lanes in `m` (one task; lane l: ids[b .. e) are
// its walked lists' ids, st_col[sb .. se) its staged list) in one walk: the
// items' staged lists go into one open-addressing table in the wave's LDS
// region, each entry with its item's lane as a tag (the table in the hash
// table words, the tags as bytes in the filter words; at most kPackSlots
// slots, load <= 1/2, so the items' staged entries must sum to at most half
// of that); the walked lists are then flattened as in tiny_items and each
// element probes the table with its list's item.  The region is left zero
// (what bitmap kernels expect; hash staging clears what it uses).
template <int UNROLL, int LDS_WORDS>
__device__ __forceinline__ uint32_t packed_items(uint64_t m, int32_t b, int32_t e, int32_t sb, int32_t se,
                                                 const int32_t *st_col_, const int32_t *ids_,
                                                 const int32_t *wk_rptr_, const int32_t *wk_col_,
                                                 int32_t *__restrict__ lds, int32_t *own, int lane) {
    constexpr int FC = HashLds<LDS_WORDS>::kFilterCap;
    constexpr int kPackSlots = HashLds<LDS_WORDS>::kTableCap < 4 * FC ? HashLds<LDS_WORDS>::kTableCap : 4 * FC;
    int32_t *table = lds + FC;
    uint8_t *tag = reinterpret_cast<uint8_t *>(lds);
    const gptr<int32_t> st_col = as_global(st_col_), ids = as_global(ids_);
    const gptr<int32_t> wk_rptr = as_global(wk_rptr_), wk_col = as_global(wk_col_);
    const bool in = (m >> lane) & 1ull;
    // ---- stage every item's list, tagged with the item's lane
    const int32_t ns = in ? se - sb : 0;
    const int32_t incls = wave_inclusive_scan(ns);
    const int32_t pres = incls - ns;
    const int32_t nsum = __builtin_amdgcn_readlane(incls, kWave - 1);
    int lg = 6;
    while ((1 << lg) < 2 * nsum && (1 << lg) < kPackSlots) ++lg;
    const uint32_t tmask = (1u << lg) - 1u;
    const int shift = 24 - lg;
    for (int q = lane; q < (1 << lg); q += kWave) table[q] = -1;
    wave_lds_sync();
    const int32_t sbase = sb - pres;  // staged entry k of the item is st_col[sbase + k]
    uint32_t carry0 = 0;
    for (int32_t k0 = 0; k0 < nsum; k0 += kWave) {
        const int32_t p = pres - k0;
        if (ns > 0 && p >= 0 && p < kWave) own[p] = lane + 1;
        wave_lds_sync();
        const uint32_t o = static_cast<uint32_t>(own[lane]);
        own[lane] = 0;
        wave_lds_sync();
        const uint32_t il1 = max(wave_max_scan_dpp(o), carry0);
        carry0 = __builtin_amdgcn_readlane(il1, kWave - 1);
        const int il = static_cast<int>(il1) - 1;
        const int32_t k = k0 + lane;
        const int32_t base_k = __shfl(sbase, il);
        if (k < nsum) {
            const int32_t v = st_col[base_k + k];
            uint32_t h = pack_slot(v, il, shift, tmask);
            while (atomicCAS(&table[h], -1, v) != -1) h = (h + 1) & tmask;
            tag[h] = static_cast<uint8_t>(il);
        }
    }
    wave_lds_sync();
    // ---- the walked lists, flattened as in tiny_items
    const int32_t nl = in ? e - b : 0;
    const int32_t incl1 = wave_inclusive_scan(nl);
    const int32_t pre1 = incl1 - nl;
    const int32_t nlists = __builtin_amdgcn_readlane(incl1, kWave - 1);
    const int32_t idbase = b - pre1;
    uint32_t cnt = 0;
    uint32_t carry1 = 0;
    for (int32_t j0 = 0; j0 < nlists; j0 += kWave) {
        const int32_t p = pre1 - j0;
        if (nl > 0 && p >= 0 && p < kWave) own[p] = lane + 1;
        wave_lds_sync();
        const uint32_t o = static_cast<uint32_t>(own[lane]);
        own[lane] = 0;
        wave_lds_sync();
        const uint32_t il1 = max(wave_max_scan_dpp(o), carry1);
        carry1 = __builtin_amdgcn_readlane(il1, kWave - 1);
        const int il = static_cast<int>(il1) - 1;  // the item of list slot j0 + lane
        const int32_t j = j0 + lane;
        const int32_t ib = __shfl(idbase, il);
        int32_t pb = 0, len = 0;
        if (j < nlists) {
            const int32_t id = ids[ib + j];
            pb = wk_rptr[id];
            len = wk_rptr[id + 1] - pb;
        }
        const int32_t incl = wave_inclusive_scan(len);
        const int32_t pre = incl - len;
        const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
        const int32_t rel = pb - pre;
        uint32_t carry = 0;
        for (int32_t base = 0; base < total; base += UNROLL * kWave) {
            const int32_t p2 = pre - base;
            if (len > 0 && p2 >= 0 && p2 < UNROLL * kWave) own[p2] = lane + 1;
            wave_lds_sync();
            uint32_t o2[UNROLL];
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) {
                o2[q] = static_cast<uint32_t>(own[q * kWave + lane]);
                own[q * kWave + lane] = 0;
            }
            wave_lds_sync();
            int32_t y[UNROLL], yi[UNROLL];
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) {
                const uint32_t sl1 = max(wave_max_scan_dpp(o2[q]), carry);
                carry = __builtin_amdgcn_readlane(sl1, kWave - 1);
                const int sl = static_cast<int>(sl1) - 1;
                const int32_t x = base + q * kWave + lane;
                const bool inb = x < total;
                const int32_t off = __shfl(rel, sl);
                yi[q] = __shfl(il, sl);  // the element's item
                const int32_t v = wk_col[inb ? off + x : 0];
                y[q] = inb ? v : -1;
            }
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) {
                bool go = y[q] >= 0;
                uint32_t h = pack_slot(y[q], yi[q], shift, tmask);
                uint32_t hit = 0;
                while (__ballot(go) != 0) {
                    const int32_t sv = table[h];
                    const bool same = go && sv == y[q] && tag[h] == static_cast<uint8_t>(yi[q]);
                    hit |= same ? 1u : 0u;
                    go = go && sv != -1 && !same;
                    h = (h + 1) & tmask;
                }
                cnt += hit;
            }
        }
    }
    // ---- leave the region zero
    wave_lds_sync();
    for (int q = lane; q < (1 << lg); q += kWave) table[q] = 0;
    for (int q = lane; q < ((1 << lg) + 3) / 4; q += kWave) lds[q] = 0;
    wave_lds_sync();
    return cnt;
}

// Adds to cnt the hits of the UNROLL elements in w (-1 = none) against S.
// Hash probes are predicated: a wave-uniform loop runs while any lane is
// still searching, with no per-lane branches.
template <int PM, int UNROLL>
__device__ __forceinline__ void probe_batch(const int32_t (&w)[UNROLL], uint32_t &cnt,
                                            const int32_t *__restrict__ lds, const Staging &sg,
                                            gptr<int32_t> st_col, int32_t sb, int32_t se,
                                            int32_t wbase) {
#pragma unroll
    for (int q = 0; q < UNROLL; ++q) {
        const int32_t wq = w[q];
        if (PM == kModeHash) {
            const uint32_t f = filter_slot(wq, sg.fshift, sg.fmask);  // in range for any wq
            const uint32_t bit = (static_cast<uint32_t>(lds[f >> 5]) >> (f & 31)) & 1u;
            bool go = (wq >= 0) & (bit != 0u);
            uint32_t h = hash_slot(wq, sg.shift, sg.tmask);
            uint32_t hit = 0;
            while (__ballot(go) != 0) {
                const int32_t sv = sg.table[h];
                hit |= (go && sv == wq) ? 1u : 0u;
                go = go && sv >= 0 && sv != wq;
                h = (h + 1) & sg.tmask;
            }
            cnt += hit;
        } else if (PM == kModeBitmap) {
            const bool ok = wq >= 0;
            const int32_t wl = ok ? wq - wbase : 0;
            const uint32_t bit = (static_cast<uint32_t>(lds[wl >> 5]) >> (wl & 31)) & 1u;
            cnt += ok ? bit : 0u;
        } else {
            if (wq >= 0) cnt += sorted_contains(st_col, sb, se, wq);
        }
    }
}

// The walk of one item once the staging kind PM is known: groups of up to 64
// walked lists; for the first group the first chunk batch is loaded before S
// is staged, and every later batch loads while the previous one is probed.
// S is staged when the first non-empty group comes (`staged` tells the
// caller whether it was), so an item whose lists are all empty stages
// nothing.
template <int PM, int UNROLL>
__device__ __forceinline__ uint32_t walk_item(Staging stg, gptr<int32_t> st_col, int32_t sb,
                                              int32_t se, gptr<int32_t> wk_rptr,
                                              gptr<int32_t> wk_col, gptr<int32_t> ids, int32_t ib,
                                              int32_t ie, int32_t g0, int32_t gn, int32_t id,
                                              int32_t *__restrict__ lds, int32_t wbase, int lane,
                                              bool &staged, int32_t *__restrict__ own) {
    uint32_t cnt = 0;
    for (;;) {  // groups of up to 64 walked lists
        int32_t pb = 0, len = 0;
        if (lane < gn) {
            pb = wk_rptr[id];
            len = wk_rptr[id + 1] - pb;
        }
        const int32_t incl = wave_inclusive_scan(len);
        const int32_t pre = incl - len;
        const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
        uint32_t carry = 0;
        int32_t w[UNROLL];
        walk_load<UNROLL>(w, 0, total, pre, len, pb, carry, own, wk_col, lane);

        if (!staged && total > 0) {
            staged = true;
            if (PM == kModeHash) {
                for (int q = lane; q < stg.words; q += kWave) stg.table[q] = -1;
                for (int q = lane; q < stg.fwords; q += kWave) lds[q] = 0;
                wave_lds_sync();
                for (int32_t idx = sb + lane; idx < se; idx += kWave) {
                    const int32_t x = st_col[idx];
                    const uint32_t f = filter_slot(x, stg.fshift, stg.fmask);
                    atomicOr(reinterpret_cast<uint32_t *>(&lds[f >> 5]), 1u << (f & 31));
                    uint32_t h = hash_slot(x, stg.shift, stg.tmask);
                    while (atomicCAS(&stg.table[h], -1, x) != -1) h = (h + 1) & stg.tmask;
                }
                wave_lds_sync();
            } else if (PM == kModeBitmap) {
                for (int32_t idx = sb + lane; idx < se; idx += kWave) {
                    const int32_t x = st_col[idx] - wbase;
                    atomicOr(reinterpret_cast<uint32_t *>(&lds[x >> 5]), 1u << (x & 31));
                }
                wave_lds_sync();
            }
        }

        for (int32_t base = 0; base < total; base += UNROLL * kWave) {
            int32_t wn[UNROLL];
            walk_load<UNROLL>(wn, base + UNROLL * kWave, total, pre, len, pb, carry, own, wk_col, lane);
            probe_batch<PM, UNROLL>(w, cnt, lds, stg, st_col, sb, se, wbase);
#pragma unroll
            for (int q = 0; q < UNROLL; ++q) w[q] = wn[q];
        }

        g0 += kWave;
        if (g0 >= ie) break;
        gn = min(ie - g0, kWave);
        id = lane < gn ? ids[g0 + lane] : 0;
    }
    return cnt;
}

// One work item of a block-list: the staged list S = st_col[sb .. se) (the
// row srow of the staging block) and the walked lists L_x = wk_col[wk_rptr[x] ..
// wk_rptr[x + 1]) for the ids x in ids[ib .. ie).  Returns, per lane, part of
// sum_x |S & L_x| (the sum over lanes is the item's count).  With the edge
// block walked by rows this is S = A_ik[u], L_v = A_jk[v] for v in A_ij[u];
// walked by columns, S = A_jk[v], L_u = A_ik[u] for u with (u, v) in A_ij.
// `lds` holds LDS_WORDS int32 words private to the wave and `own` 64 *
// UNROLL more, zero on entry and left zero (the walk's list positions).
// Column ids of both lists lie in [wbase, wbase + width_k).  Every lane of
// the wave must call this with the same arguments.
//
// Hash staging: S goes into an open-addressing table (load <= 2/3) and into
// a bit filter with about eight bits per entry; a probe reads the filter
// first, so most misses -- nine in ten probes on skewed graphs -- cost one
// LDS read.
//
// The walk issues many instructions per element, so its code keeps the
// instruction count low: the staging kind is fixed per item outside the
// element loop, hash probes are predicated, and loads go through global
// views.  It is also latency bound per item (each step's addresses come from
// the previous step's loads), so independent loads are issued together: the
// ids of the walked lists with the bounds of S, the first chunks of the walk
// before S is staged, and every later chunk before the previous one is
// probed.
template <int MODE, int LDS_WORDS, int UNROLL = 2>
__device__ __forceinline__ uint32_t tc_item_core(const int32_t *__restrict__ st_col_, int32_t sb, int32_t se,
                                                 const int32_t *__restrict__ wk_rptr_,
                                                 const int32_t *__restrict__ wk_col_,
                                                 const int32_t *__restrict__ ids_, int32_t ib, int32_t ie,
                                                 int32_t width_k, int32_t *__restrict__ lds,
                                                 int32_t *__restrict__ own, int32_t wbase = 0) {
    const int lane = lane_id();
    if (ib >= ie) return 0u;
    const gptr<int32_t> st_col = as_global(st_col_);
    const gptr<int32_t> wk_rptr = as_global(wk_rptr_), wk_col = as_global(wk_col_);
    const gptr<int32_t> ids = as_global(ids_);
    const int32_t gn = min(ie - ib, kWave);
    const int32_t id = lane < gn ? ids[ib + lane] : 0;
    const int32_t slen = se - sb;
    if (slen == 0) return 0u;

    // ---- choose how S is held
    int mode = MODE;
    Staging stg;
    if (mode == kModeBitmap) {
        stg.words = (width_k + 31) >> 5;
        if (stg.words > LDS_WORDS) mode = kModeHash;
    }
    if (mode == kModeHash) {
        constexpr int TC = HashLds<LDS_WORDS>::kTableCap;
        constexpr int FC = HashLds<LDS_WORDS>::kFilterCap;
        int lg = 6;
        while ((1 << lg) * 2 < 3 * slen) ++lg;
        if ((1 << lg) > TC || FC < 2) {
            mode = kModeSearch;
        } else {
            stg.words = 1 << lg;
            stg.shift = 24 - lg;
            stg.tmask = static_cast<uint32_t>(stg.words - 1);
            int flg = 8;  // filter bits: a power of two >= 8 * slen, >= 256
            while ((1 << flg) < 8 * slen && (1 << flg) < 32 * FC) ++flg;
            while ((1 << flg) > 32 * FC) --flg;
            stg.fwords = (1 << flg) >> 5;
            stg.fshift = 24 - flg;
            stg.fmask = static_cast<uint32_t>((1 << flg) - 1);
            stg.table = lds + FC;
        }
    }

    uint32_t cnt;
    bool staged = false;
    if (mode == kModeHash)
        cnt = walk_item<kModeHash, UNROLL>(stg, st_col, sb, se, wk_rptr, wk_col, ids, ib, ie, ib, gn, id,
                                           lds, wbase, lane, staged, own);
    else if (mode == kModeBitmap)
        cnt = walk_item<kModeBitmap, UNROLL>(stg, st_col, sb, se, wk_rptr, wk_col, ids, ib, ie, ib, gn, id,
                                             lds, wbase, lane, staged, own);
    else
        cnt = walk_item<kModeSearch, UNROLL>(stg, st_col, sb, se, wk_rptr, wk_col, ids, ib, ie, ib, gn, id,
                                             lds, wbase, lane, staged, own);

    // ---- leave the LDS clean for the next row of this wave
    if (!staged) return cnt;
    if (mode == kModeBitmap) {
        wave_lds_sync();
        for (int32_t idx = sb + lane; idx < se; idx += kWave) lds[(st_col[idx] - wbase) >> 5] = 0;
        wave_lds_sync();
    } else if (mode == kModeHash) {
        wave_lds_sync();
        if (MODE == kModeBitmap) {
            // a bitmap kernel expects zeroed LDS between rows: clear the
            // filter and table words this item used
            constexpr int FC = HashLds<LDS_WORDS>::kFilterCap;
            for (int q = lane; q < stg.fwords; q += kWave) lds[q] = 0;
            for (int q = lane; q < stg.words; q += kWave) lds[FC + q] = 0;
            wave_lds_sync();
        }
    }
    return cnt;
}

// The same with the staged list given by its row: S = st_col[st_rptr[srow]
// .. st_rptr[srow + 1]).
template <int MODE, int LDS_WORDS, int UNROLL = 2>
__device__ __forceinline__ uint32_t tc_item(const int32_t *__restrict__ st_rptr,
                                            const int32_t *__restrict__ st_col, int32_t srow,
                                            const int32_t *__restrict__ wk_rptr,
                                            const int32_t *__restrict__ wk_col,
                                            const int32_t *__restrict__ ids, int32_t ib, int32_t ie,
                                            int32_t width_k, int32_t *__restrict__ lds,
                                            int32_t *__restrict__ own, int32_t wbase = 0) {
    const gptr<int32_t> rp = as_global(st_rptr);
    return tc_item_core<MODE, LDS_WORDS, UNROLL>(st_col, rp[srow], rp[srow + 1], wk_rptr, wk_col, ids, ib, ie,
                                                 width_k, lds, own, wbase);
}

}  // namespace pgabb
