// Device code shared by the host-driven (bfs.hip) and the device-driven
// (bfs_graph.hip) single-source traversal: adjacency traits, bit helpers,
// the bottom-up level body, the long-row bottom-up body and the SPLIT output
// body. Included by one .hip file each; everything has internal linkage.
#pragma once

#include <climits>

#include "gt_internal.h"

namespace {
constexpr int TD_BLOCK = 256;
constexpr int BU_BLOCK = 256;
constexpr int BU_BLOCK_MAX = 512;  // bottom-up workgroups with the LDS-resident hub frontier
constexpr int OUT_BLOCK = 256;
constexpr int COMPACT_BLOCK = 256;

__device__ __forceinline__ void clear_set(unsigned long long* set) {
    for (int i = threadIdx.x; i < CTR_SET; i += blockDim.x) set[i] = 0;
}

// Adjacency entries of the traversed graph are int32 ids of that graph:
// caller ids (PLAIN) or core ids (SPLIT). A SPLIT discovery records its
// parent as a caller id, translated through new2old (a bottom-up hit on the
// highest-degree neighbour takes it from hint_orig instead).
template <bool SPLIT>
__device__ __forceinline__ int32_t caller_id(const int32_t* __restrict__ new2old, int32_t u) {
    return SPLIT ? new2old[u] : u;
}

// Smallest j in [a, b] with p[j] > x, given p[b] > x and p nondecreasing.
__device__ __forceinline__ int64_t first_greater(const int64_t* __restrict__ p, int64_t a, int64_t b,
                                                 int64_t x) {
    while (a < b) {
        const int64_t mid = a + ((b - a) >> 1);
        if (p[mid] > x) b = mid;
        else a = mid + 1;
    }
    return a;
}

// Byte kept per core vertex for the leaf pass: 0 = not reached, else the
// level of a leaf hanging off it (core level + 1), 255 = look the level up.
__device__ __forceinline__ uint8_t leaf_level_byte(int32_t core_level) {
    return core_level + 1 < 255 ? (uint8_t)(core_level + 1) : (uint8_t)255;
}

__device__ __forceinline__ bool bit_of(const uint64_t* __restrict__ vis, int32_t u) {
    return (vis[u >> 6] >> (u & 63)) & 1ull;
}

// Streaming accesses: data touched once per level (the dense per-vertex hint
// and degree arrays, the level and parent of a discovery) is loaded and
// stored non-temporally, so that it does not push the visited bitmap, which
// every probe of the level reads, out of L2. Top-down does the same with
// the rows of the frontier and the degrees of its discoveries.
template <class T>
__device__ __forceinline__ T ld_stream(const T* p);
template <>
__device__ __forceinline__ int32_t ld_stream<int32_t>(const int32_t* p) {
    return __builtin_nontemporal_load(p);
}

__device__ __forceinline__ void st_stream(int32_t* p, int32_t v) { __builtin_nontemporal_store(v, p); }

// Level and parent of a traversed vertex v sit at level[v * LPS] and
// parent[v * LPS]. A SPLIT traversal keeps both in one array of (level,
// parent) pairs per core vertex (parent = level + 1, LPS = 2), so that a
// discovery dirties one 8-byte slot and one cache line; a PLAIN traversal
// writes the caller's two output arrays (LPS = 1).
template <bool SPLIT>
constexpr int LPS = SPLIT ? 2 : 1;

// A discovery's level and parent as streaming stores: one 8-byte store of
// the pair (SPLIT), so that the stores of a wave cover whole lines.
template <bool SPLIT>
__device__ __forceinline__ void st_stream_lp(int32_t* level, int32_t* parent, int64_t v, int32_t l, int32_t p) {
    if (SPLIT) {
        const long long x = (long long)(uint32_t)l | ((long long)(uint32_t)p << 32);
        __builtin_nontemporal_store(x, reinterpret_cast<long long*>(level + 2 * v));
    } else {
        st_stream(&level[v], l);
        st_stream(&parent[v], p);
    }
}
// An adjacency entry loaded as streaming data: top-down reads each frontier
// row once per level.
__device__ __forceinline__ int32_t ld_id_stream(const int32_t* p) { return __builtin_nontemporal_load(p); }

// Neighbour probes of a bottom-up level (the degree-aware probe of Section
// 2.3): the highest-degree neighbour of every traversed vertex (nullptr: no
// probe) and, optionally, the second-highest with one bit per vertex telling
// whether the two cover its whole row (degree <= 2). SPLIT keeps both
// neighbours' caller ids for the parent a hit records.
struct BuHints {
    const int32_t* hint;
    const int32_t* hint_orig;
    const int32_t* hint2;      // nullptr: one probe
    const int32_t* hint2_orig;
    const uint64_t* small;
};

constexpr int BU_BATCH = 4;                       // loads in flight per lane and round trip
constexpr int BU_WINDOW = BU_BATCH * GT_WAVE;     // entries a wave reads per round trip

// First set bit at position >= a in the 256-bit mask m[0..3]; 256 if none.
__device__ __forceinline__ int first_set_from(const uint64_t m[BU_BATCH], int a) {
#pragma unroll
    for (int i = 0; i < BU_BATCH; ++i) {
        const int base = i * GT_WAVE;
        if (a < base + GT_WAVE) {
            uint64_t x = m[i];
            if (a > base) x &= ~0ull << (a - base);
            if (x) return base + __ffsll((unsigned long long)x) - 1;
        }
    }
    return BU_WINDOW;
}

// Position of the nth (0-based) set bit of x; x has more than nth set bits.
__device__ __forceinline__ int nth_set_bit(uint64_t x, int nth) {
    int pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const int c = __popcll(x & ((1ull << w) - 1));
        if (nth >= c) {
            nth -= c;
            x >>= w;
            pos += w;
        }
    }
    return pos;
}

// bitmap words a wave takes per iteration: 5 fits k_bu in 80 VGPRs without
// spilling, so that a CU holds 6 waves per SIMD, i.e. three 512-thread
// workgroups with the LDS hub frontier; 8 words (94 VGPRs) kept more loads
// in flight per wave but left room for two workgroups only
constexpr int BU_WPI = 5;

// Bottom-up level (Algorithm 1, BOTTOM-UP; Algorithm 5's 64-vertex block is
// one wavefront). A neighbour visited in the start-of-level snapshot of an
// unvisited vertex must be in the current frontier, so the snapshot stands
// in for the frontier set. A wave takes BU_WPI bitmap words (512 vertices)
// per iteration:
//  0. for every unvisited vertex: its highest-degree neighbour (dense hint
//     array, the degree-aware probe of Section 2.3), all loads of the BU_WPI
//     words issued together (a SPLIT hit takes the neighbour's caller id
//     from hint_orig, loaded for the hits only); with H2 (hh.hint2), the vertices the
//     first probe missed probe their second-highest-degree neighbour, and a
//     vertex of degree <= 2 that both probes missed has no frontier
//     neighbour: it is settled without reading its row;
//  1. the vertices the hint did not settle are packed onto the lanes, 64 per
//     round; each probes the first lane_edges entries of its row, BU_BATCH
//     independent loads per round trip;
//  2. the remaining entries of all rows still open in the round are read as
//     one flat list, BU_WINDOW entries per round trip (an entry's row is
//     found by binary search over the lanes' prefix sums); a row stops at its
//     first hit, read from the window's hit ballots; a SPLIT hit's caller
//     id is gathered from new2old;
//  3. rows longer than hub_deg that phase 1 did not settle go to bu_hub_rows.
// Each bitmap word of the next snapshot is written once. No queue of
// discoveries is built here. Hint, level and parent go through the streaming
// accesses above. Every hint probe counts as one examined entry. The
// found-degree counter sums the degrees of the vertices found in their rows
// only (a hint hit's degree is never loaded); the direction rule does not
// read it after a bottom-up level.

//
// LIST: the same, over a list of candidate vertices (the vertices still
// unvisited when the list was built, ascending) instead of over all bitmap
// words: a wave takes BU_WPI groups of 64 list entries. vis_next must then
// start as a copy of vis_cur; discoveries are OR-ed into it.
//
// LDS-resident hub frontier: the first lds_words words of the snapshot (the
// visited bits of the hubs, core ids [0, n_hub) on a hubs-first numbering,
// which take nearly every hint probe and half of all adjacency entries) are
// copied into the workgroup's LDS once, and every probe of a vertex there
// reads LDS instead of the global bitmap. The kernel then runs as a
// persistent grid, so the copy is made once per resident workgroup.
template <bool SPLIT, bool LIST = false, bool H2 = false>
__device__ __forceinline__ void bu_level(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, int64_t n,
    int64_t words, const uint64_t* __restrict__ vis_cur, uint64_t* __restrict__ vis_next,
    int32_t* __restrict__ level, int32_t* __restrict__ parent, int32_t next_level,
    int32_t* __restrict__ hub_q, unsigned long long* __restrict__ ctr,
    int lane_edges, int64_t hub_deg, const BuHints& hh, const int32_t* __restrict__ new2old,
    int64_t lds_words, const int32_t* __restrict__ list = nullptr, int64_t nlist = 0) {
    using T = int32_t;
    const int32_t* __restrict__ hint = hh.hint;
    extern __shared__ uint64_t s_vis[];
    for (int64_t i = threadIdx.x; i < lds_words; i += blockDim.x) s_vis[i] = vis_cur[i];
    __syncthreads();
    const int64_t lds_bits = lds_words * GT_WAVE;
    auto probe = [&](int32_t u) -> bool {
        return u < lds_bits ? ((s_vis[u >> 6] >> (u & 63)) & 1ull) != 0 : bit_of(vis_cur, u);
    };
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    const int64_t units = LIST ? (nlist + GT_WAVE - 1) / GT_WAVE : words;
    unsigned long long fdeg = 0, scanned = 0, examined = 0, nfound = 0;
    for (int64_t wd0 = gw * BU_WPI; wd0 < units; wd0 += nwaves * BU_WPI) {
        uint64_t vis[BU_WPI], fm[BU_WPI], pend[BU_WPI];
        bool unv[BU_WPI];
        int32_t hv[BU_WPI];
        int32_t vv[BU_WPI];
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) {
            const int64_t wd = wd0 + i;
            if (LIST) {
                const int64_t x = wd * GT_WAVE + lane;
                vv[i] = x < nlist ? list[x] : -1;
                vis[i] = 0;
            } else {
                vis[i] = wd < units ? vis_cur[wd] : ~0ull;
                vv[i] = 0;
            }
        }
        // vertex of slot i: the list entry, or lane `lane` of word wd0 + i
        auto vid = [&](int i) -> int32_t { return LIST ? vv[i] : (int32_t)((wd0 + i) * GT_WAVE + lane); };
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) {
            if (LIST) unv[i] = vv[i] >= 0 && !probe(vv[i]);
            else unv[i] = wd0 + i < units && vid(i) < n && !((vis[i] >> lane) & 1ull);
        }
        // phase 0: the highest-degree neighbour of every unvisited vertex
        // (row bounds are read only for the vertices it does not settle, in
        // phase 1, which also gives their degree)
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) hv[i] = (unv[i] && hint) ? ld_stream(&hint[vid(i)]) : -1;
        bool hf[BU_WPI], hf2[BU_WPI], open[BU_WPI];
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) {
            hf[i] = unv[i] && hv[i] >= 0 && probe(hv[i]);
            if (hv[i] >= 0) examined += 1;  // the probe reads one (copied) entry
            // with the probe on, a vertex without a hint has no neighbour
            open[i] = unv[i] && !hf[i] && (hint == nullptr || hv[i] >= 0);
        }
        int32_t h2[BU_WPI];
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) h2[i] = (H2 && open[i]) ? ld_stream(&hh.hint2[vid(i)]) : -1;
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) {
            hf2[i] = h2[i] >= 0 && probe(h2[i]);
            if (h2[i] >= 0) examined += 1;
            if (H2 && open[i] && !hf2[i]) {
                // both probes missed: a row of at most two entries is done
                const int32_t v = vid(i);
                const bool small = LIST ? bit_of(hh.small, v) : ((hh.small[wd0 + i] >> lane) & 1ull) != 0;
                if (small) open[i] = false;
            }
            if (hf2[i]) open[i] = false;
        }
        // parent of a hit: the neighbour's caller id (SPLIT: dense arrays,
        // read only where a probe hit)
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) {
            if (SPLIT && hf[i]) hv[i] = ld_stream(&hh.hint_orig[vid(i)]);
            else if (hf2[i]) hv[i] = SPLIT ? ld_stream(&hh.hint2_orig[vid(i)]) : h2[i];
        }
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) {
            const bool f = hf[i] || hf2[i];
            fm[i] = __ballot(f);
            pend[i] = __ballot(open[i]);
            if (unv[i]) scanned += 1;
            if (LIST) {
                // list entries ascend, so lanes sharing a bitmap word are
                // adjacent: OR their bits along each run of equal words and
                // let the run's last lane issue the one atomic
                const int32_t v = vid(i);
                const int32_t wv = v >= 0 ? (v >> 6) : -1;
                uint64_t x = f ? (1ull << (v & 63)) : 0ull;
#pragma unroll
                for (int o = 1; o < GT_WAVE; o <<= 1) {
                    const uint64_t y = __shfl_up(x, o, GT_WAVE);
                    const int32_t wy = __shfl_up(wv, o, GT_WAVE);
                    if (lane >= o && wy == wv) x |= y;
                }
                const int32_t wn = __shfl_down(wv, 1, GT_WAVE);
                if (x && (lane == GT_WAVE - 1 || wn != wv))
                    atomicOr((unsigned long long*)&vis_next[wv], (unsigned long long)x);
            }
            if (f) {
                const int32_t v = vid(i);
                st_stream_lp<SPLIT>(level, parent, v, next_level, hv[i]);
                nfound += 1;
            }
        }
        int cum[BU_WPI + 1];
        cum[0] = 0;
#pragma unroll
        for (int i = 0; i < BU_WPI; ++i) cum[i + 1] = cum[i] + __popcll(pend[i]);
        const int P = cum[BU_WPI];
        for (int r0 = 0; r0 < P; r0 += GT_WAVE) {
            // phase 1: lane takes the (r0 + lane)-th unsettled vertex
            const int l = r0 + lane;
            const bool act = l < P;
            int wi = 0;
#pragma unroll
            for (int i = 1; i < BU_WPI; ++i)
                if (l >= cum[i]) wi = i;
            const int j = act ? nth_set_bit(pend[wi], l - cum[wi]) : lane;
            int32_t v = LIST ? 0 : (int32_t)((wd0 + wi) * GT_WAVE + j);
            if (LIST) {
#pragma unroll
                for (int i = 0; i < BU_WPI; ++i) {
                    const int32_t tv = __shfl(vv[i], j, GT_WAVE);
                    if (i == wi) v = tv;
                }
            }
            const int64_t b = act ? off[v] : 0;
            const int64_t re = act ? off[v + 1] : 0;
            bool found = false, pending = false, hub = false;
            int32_t par = -1;
            int64_t rb = 0;
            if (act) {
                const int64_t lim = (re - b > lane_edges) ? b + lane_edges : re;
                int64_t hit_at = -1;
                for (int64_t k = b; k < lim && hit_at < 0; k += BU_BATCH) {
                    T u[BU_BATCH];
#pragma unroll
                    for (int i = 0; i < BU_BATCH; ++i) u[i] = (k + i < lim) ? col[k + i] : -1;
                    bool h[BU_BATCH];
#pragma unroll
                    for (int i = 0; i < BU_BATCH; ++i) h[i] = u[i] >= 0 && probe(u[i]);
#pragma unroll
                    for (int i = BU_BATCH - 1; i >= 0; --i)
                        if (h[i]) { hit_at = k + i; par = u[i]; }
                }
                found = hit_at >= 0;
                examined += (unsigned long long)(found ? hit_at - b + 1 : lim - b);
                rb = lim;
                if (!found && rb < re) {
                    if (re - b > hub_deg) hub = true;
                    else pending = true;
                }
            }
            // phase 2: flat list over the rows still open in this round
            uint64_t pm = __ballot(pending);
            while (pm) {
                const int32_t len = pending ? (int32_t)(re - rb) : 0;
                int32_t incl = len;
#pragma unroll
                for (int o = 1; o < GT_WAVE; o <<= 1) {
                    const int32_t y = __shfl_up(incl, o, GT_WAVE);
                    if (lane >= o) incl += y;
                }
                const int32_t excl = incl - len;
                const int32_t total = __shfl(incl, GT_WAVE - 1, GT_WAVE);
                const int32_t W = total < BU_WINDOW ? total : BU_WINDOW;
                T ent[BU_BATCH];
                uint64_t hm[BU_BATCH];
#pragma unroll
                for (int i = 0; i < BU_BATCH; ++i) {
                    const int32_t x = i * GT_WAVE + lane;
                    // owner: the last lane whose prefix start is <= x (6 fixed steps)
                    int lo = 0, hi = GT_WAVE - 1;
#pragma unroll
                    for (int st = 0; st < 6; ++st) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (__shfl(excl, mid, GT_WAVE) <= x) lo = mid;
                        else hi = mid - 1;
                    }
                    const int64_t k = __shfl(rb, lo, GT_WAVE) + (x - __shfl(excl, lo, GT_WAVE));
                    ent[i] = x < W ? col[k] : -1;
                }
#pragma unroll
                for (int i = 0; i < BU_BATCH; ++i) hm[i] = __ballot(ent[i] >= 0 && probe(ent[i]));
                int fpos = BU_WINDOW;
                if (pending && excl < W) {
                    const int32_t z = incl < W ? incl : W;
                    const int p = first_set_from(hm, excl);
                    if (p < z) {
                        fpos = p;
                        examined += (unsigned long long)(p - excl + 1);
                        found = true;
                        pending = false;
                    } else {
                        examined += (unsigned long long)(z - excl);
                        rb += z - excl;
                        if (rb >= re) pending = false;
                    }
                }
                // the parent sits in lane fpos % 64, slot fpos / 64 of the window
                const int src = fpos < BU_WINDOW ? (fpos % GT_WAVE) : lane;
                const int slot = fpos < BU_WINDOW ? (fpos / GT_WAVE) : 0;
                int32_t pv = -1;
#pragma unroll
                for (int i = 0; i < BU_BATCH; ++i) {
                    const int32_t cand = __shfl(ent[i], src, GT_WAVE);
                    if (i == slot) pv = cand;
                }
                if (fpos < BU_WINDOW) par = pv;
                pm = __ballot(pending);
            }
            if (found) {
                if (LIST) atomicOr((unsigned long long*)&vis_next[v >> 6], 1ull << (v & 63));
                st_stream_lp<SPLIT>(level, parent, v, next_level, caller_id<SPLIT>(new2old, par));
                fdeg += (unsigned long long)(re - b);
                nfound += 1;
            }
            const long long hs = wave_append(&ctr[CTR_HUBS], hub);
            if (hub) hub_q[hs] = v;
            if (!LIST) {
                // fold the round's discoveries into the words' bit masks: the
                // vertex in lane position `lane` of word i was processed by lane idx
                const int fi = found ? 1 : 0;
#pragma unroll
                for (int i = 0; i < BU_WPI; ++i) {
                    const bool mine = (pend[i] >> lane) & 1ull;
                    const int idx = cum[i] + __popcll(pend[i] & ((1ull << lane) - 1ull)) - r0;
                    const bool inr = mine && idx >= 0 && idx < GT_WAVE;
                    const int got = __shfl(fi, inr ? idx : lane, GT_WAVE);
                    fm[i] |= __ballot(inr && got);
                }
            }
        }
        if (!LIST && lane == 0) {
#pragma unroll
            for (int i = 0; i < BU_WPI; ++i)
                if (wd0 + i < units) vis_next[wd0 + i] = vis[i] | fm[i];
        }
    }
    unsigned long long* cs = ctr_slot(ctr);
    wave_add(&cs[CTR_FOUND], nfound);
    wave_add(&cs[CTR_FOUND_DEG], fdeg);
    wave_add(&cs[CTR_SCANNED], scanned);
    wave_add(&cs[CTR_EXAMINED], examined);
}

// Bottom-up for the long rows bu_level deferred: one workgroup per row,
// HUB_BLOCK * BU_BATCH entries per round trip, stopping at the first chunk
// with a hit (the lowest hit position of that chunk is the parent). Runs
// after bu_level on the same stream, so the bitmap word it ORs into is final.
constexpr int HUB_BLOCK = 256;

template <bool SPLIT>
__device__ __forceinline__ void bu_hub_rows(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, const int32_t* __restrict__ new2old,
    const uint64_t* __restrict__ vis_cur, uint64_t* __restrict__ vis_next,
    int32_t* __restrict__ level, int32_t* __restrict__ parent, int32_t next_level,
    const int32_t* __restrict__ hub_q, unsigned long long* __restrict__ ctr, int lane_edges) {
    __shared__ int s_first;
    const int tid = threadIdx.x;
    const int64_t nh = (int64_t)ctr[CTR_HUBS];
    unsigned long long* cs = ctr_slot(ctr);
    for (int64_t h = blockIdx.x; h < nh; h += gridDim.x) {
        const int32_t v = hub_q[h];
        // the first lane_edges entries were probed by k_bu already
        const int64_t b = off[v] + lane_edges, e = off[v + 1];
        int64_t hit = -1;
        for (int64_t c = b; c < e; c += (int64_t)HUB_BLOCK * BU_BATCH) {
            if (tid == 0) s_first = INT_MAX;
            __syncthreads();
            int mine = INT_MAX;
#pragma unroll
            for (int i = 0; i < BU_BATCH; ++i) {
                const int64_t kk = c + (int64_t)i * HUB_BLOCK + tid;
                if (kk < e && bit_of(vis_cur, col[kk])) {
                    const int pos = i * HUB_BLOCK + tid;
                    mine = pos < mine ? pos : mine;
                }
            }
            if (mine != INT_MAX) atomicMin(&s_first, mine);
            __syncthreads();
            const int first = s_first;
            __syncthreads();
            if (first != INT_MAX) {
                hit = c + first;
                break;
            }
        }
        if (tid == 0) {
            const unsigned long long exam = hit >= 0 ? (unsigned long long)(hit - b + 1)
                                                     : (unsigned long long)(e - b);
            atomicAdd(&cs[CTR_EXAMINED], exam);
            atomicAdd(&cs[CTR_EXAMINED_LONG], exam);
            if (hit >= 0) {
                level[(int64_t)v * LPS<SPLIT>] = next_level;
                parent[(int64_t)v * LPS<SPLIT>] = caller_id<SPLIT>(new2old, col[hit]);
                atomicOr((unsigned long long*)&vis_next[v >> 6], 1ull << (v & 63));
                atomicAdd(&cs[CTR_FOUND], 1ull);
                atomicAdd(&cs[CTR_FOUND_LONG], 1ull);
                atomicAdd(&cs[CTR_FOUND_DEG], (unsigned long long)(e - off[v]));
            }
        }
    }
}

// ------------------------------------------------------- top-down, flat --
// (used by the device-driven loop for every top-down level and by the
// host-driven loop when the frontier is a bitmap difference)
constexpr int TD_CHUNK = 4 * GT_WAVE;         // entries of one long-row chunk (4 per lane)
constexpr int TDW_BATCH = 4;                  // flat-list loads per lane and round trip
constexpr int TDW_WINDOW = TDW_BATCH * GT_WAVE;

// Top-down claims of a batch of B neighbours w[i] (-1: none) of frontier
// vertices whose caller ids are pp[i]. A neighbour is claimed when it is
// visited neither at the start of the level (va) nor since (vb) and this
// lane is the first to set its bit in vb. The bitmap words of the whole
// batch are read first, then the atomics are issued, then the discoveries
// are written, so each phase has all its memory operations in flight.
template <int B, int S>
__device__ __forceinline__ void td_claim_batch(const int32_t (&w)[B], const int32_t (&pp)[B],
                                               const uint64_t* __restrict__ va, uint64_t* vb, int32_t* lvl,
                                               int32_t* par, const int32_t* __restrict__ tdeg,
                                               int32_t next_level, bool append, unsigned long long* qtail,
                                               int32_t* qn, unsigned long long& fdeg,
                                               unsigned long long& nfound) {
    uint64_t seen[B];
#pragma unroll
    for (int i = 0; i < B; ++i) seen[i] = w[i] >= 0 ? (va[w[i] >> 6] | vb[w[i] >> 6]) : ~0ull;
    bool found[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        found[i] = false;
        const uint64_t bit = 1ull << (w[i] & 63);
        if (!(seen[i] & bit)) {
            const unsigned long long old = atomicOr((unsigned long long*)&vb[w[i] >> 6], (unsigned long long)bit);
            found[i] = !(old & bit);
        }
    }
    int32_t dg[B];
#pragma unroll
    for (int i = 0; i < B; ++i) dg[i] = found[i] ? ld_stream(&tdeg[w[i]]) : 0;
#pragma unroll
    for (int i = 0; i < B; ++i) {
        if (found[i]) {
            lvl[(int64_t)w[i] * S] = next_level;
            par[(int64_t)w[i] * S] = pp[i];
            fdeg += (unsigned long long)dg[i];
            nfound += 1;
        }
    }
    if (append) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const long long slot = wave_append(qtail, found[i]);
            if (found[i]) qn[slot] = w[i];
        }
    }
}

// One top-down level in the two-bitmap form: vis[cur] is the visited set
// with the frontier (read only during the level), vis[cur ^ 1] the visited
// set without it; claims and the frontier go into vis[cur ^ 1], which ends
// as the new visited set. The frontier is q[qi][0 .. nf) (from_q) or the
// bits of vis[cur] missing from vis[cur ^ 1]; append: discoveries are also
// appended to q[qi ^ 1]. Counters go to set (lev & 1).
struct TdLevel {
    int32_t cur, qi, next_level, lev;
    int64_t nf;
    bool from_q, append;
    int32_t* lvl;
    int32_t* par;
};

// Arrays of one traversal, as the level kernels see them.
template <bool SPLIT>
struct GArgs {
    const int64_t* off;
    const int32_t* col;
    const int32_t* new2old;   // SPLIT: caller id per core vertex (the parent recorded)
    const int32_t* tdeg;      // degree per traversed vertex
    BuHints hh;               // bottom-up neighbour probes
    uint64_t* vis[2];
    int32_t* q[2];
    int32_t* hub_q;
    unsigned long long* ctr;  // two counter sets
    int2* rows;               // top-down long rows of the level: (vertex, first chunk index)
    int64_t row_cap;
    int64_t n, words;
    int64_t td_hub_deg, bu_hub_deg;
    int32_t bu_lane_edges;
};

// Top-down level, first part: a wave per 64 frontier vertices; their short
// rows as one flat list (TDW_WINDOW entries per round trip, an entry's row
// found by binary search over the lanes' prefix sums); long rows reserved as
// chunks for td_chunks. With few frontier vertices for the grid, every row
// longer than one wave's width is cut into chunks, so a handful of frontier
// vertices still spreads over many waves.
// Expands the frontier vertex v of each lane (-1: none): long rows get a
// record for the chunk pass, short rows are read as one flat list of the
// wave (TDW_WINDOW entries per round trip, an entry's row found by binary
// search over the lanes' prefix sums) and their entries claimed.
template <bool SPLIT>
__device__ __forceinline__ void td_expand_vertices(int32_t v, int64_t hub_deg, const GArgs<SPLIT>& a,
                                                   const uint64_t* __restrict__ va, uint64_t* vb, int32_t* lvl,
                                                   int32_t* par, int32_t next_level, bool append,
                                                   unsigned long long* set, int32_t* qn, unsigned long long& fdeg,
                                                   unsigned long long& nfound, unsigned long long& examined) {
    const int lane = lane_id();
    int64_t rb = 0, re = 0;
    int32_t pid = -1;
    if (v >= 0) {
        rb = a.off[v];
        re = a.off[v + 1];
        pid = SPLIT ? a.new2old[v] : v;
    }
    const int64_t d = re - rb;
    examined += (unsigned long long)d;
    const bool longrow = d > hub_deg;
    {
        // long rows: one record per row, (vertex, index of its first
        // chunk); records and chunk ranges are reserved with one 64-bit
        // atomic (records in the high half, chunks in the low half), so
        // the chunk starts of the records increase with their index
        const int64_t nch = longrow ? (d + TD_CHUNK - 1) / TD_CHUNK : 0;
        int64_t incl = nch;
#pragma unroll
        for (int o = 1; o < GT_WAVE; o <<= 1) {
            const int64_t y = __shfl_up(incl, o, GT_WAVE);
            if (lane >= o) incl += y;
        }
        const int64_t tot = __shfl(incl, GT_WAVE - 1, GT_WAVE);
        if (tot > 0) {
            const uint64_t lm = __ballot(longrow);
            unsigned long long base = 0;
            if (lane == 0)
                base = atomicAdd(&set[CTR_TDCHUNKS],
                                 ((unsigned long long)__popcll(lm) << 32) | (unsigned long long)tot);
            base = __shfl(base, 0, GT_WAVE);
            if (longrow) {
                const int64_t r = (int64_t)(base >> 32) + lanes_below(lm);
                const int64_t c0 = (int64_t)(base & 0xFFFFFFFFull) + incl - nch;
                if (r < a.row_cap) a.rows[r] = make_int2(v, (int32_t)c0);
            }
        }
    }
    const int32_t len = (v >= 0 && !longrow) ? (int32_t)d : 0;
    int32_t incl = len;
#pragma unroll
    for (int o = 1; o < GT_WAVE; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, GT_WAVE);
        if (lane >= o) incl += y;
    }
    const int32_t excl = incl - len;
    const int32_t total = __shfl(incl, GT_WAVE - 1, GT_WAVE);
    for (int32_t b0 = 0; b0 < total; b0 += TDW_WINDOW) {
        int32_t ent[TDW_BATCH];
        int own[TDW_BATCH];
#pragma unroll
        for (int i = 0; i < TDW_BATCH; ++i) {
            const int32_t x = b0 + i * GT_WAVE + lane;
            // owner: the last lane whose prefix start is <= x
            int lo = 0, hi = GT_WAVE - 1;
#pragma unroll
            for (int st = 0; st < 6; ++st) {
                const int mid = (lo + hi + 1) >> 1;
                if (__shfl(excl, mid, GT_WAVE) <= x) lo = mid;
                else hi = mid - 1;
            }
            const int64_t k = __shfl(rb, lo, GT_WAVE) + (x - __shfl(excl, lo, GT_WAVE));
            ent[i] = x < total ? ld_id_stream(&a.col[k]) : -1;
            own[i] = lo;
        }
        int32_t w[TDW_BATCH], pp[TDW_BATCH];
#pragma unroll
        for (int i = 0; i < TDW_BATCH; ++i) {
            w[i] = ent[i];
            pp[i] = __shfl(pid, own[i], GT_WAVE);
        }
        td_claim_batch<TDW_BATCH, LPS<SPLIT>>(w, pp, va, vb, lvl, par, a.tdeg, next_level, append, &set[CTR_QTAIL], qn,
                                  fdeg, nfound);
    }
}

// Top-down level, first part: a wave takes 64 frontier vertices at a time
// (64 queue entries, or the frontier bits of 64 bitmap words packed onto the
// lanes 64 at a time) and expands them (td_expand_vertices). With few queue
// vertices for the grid, every row longer than one wave's width is cut into
// chunks, so a handful of frontier vertices still spreads over many waves.
template <bool SPLIT>
__device__ __forceinline__ void td_units(const TdLevel& c, const GArgs<SPLIT>& a) {
    const int cur = c.cur;
    const uint64_t* va = a.vis[cur];       // visited with the frontier: read only
    uint64_t* vb = a.vis[cur ^ 1];         // visited without the frontier: claims go here
    const int32_t* q = a.q[c.qi];
    int32_t* qn = a.q[c.qi ^ 1];
    const bool from_q = c.from_q, append = c.append;
    const int64_t nf = c.nf;
    const int32_t next_level = c.next_level;
    int32_t* lvl = c.lvl;
    int32_t* par = c.par;
    unsigned long long* set = a.ctr + (c.lev & 1) * CTR_SET;
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    const int64_t units = from_q ? (nf + GT_WAVE - 1) / GT_WAVE : (a.words + GT_WAVE - 1) / GT_WAVE;
    // few queue vertices for the grid: every row longer than a wave's width
    // is chunked. Long-row records are then at most the frontier size (below
    // 8 * nwaves), so this applies only when that many fit in a.rows; with
    // td_hub_deg (>= TD_CHUNK) they are at most E / TD_CHUNK, which always fit.
    const int64_t hub_deg = (from_q && units * 8 < nwaves && 8 * nwaves <= a.row_cap) ? (int64_t)GT_WAVE
                                                                                        : a.td_hub_deg;
    unsigned long long fdeg = 0, nfound = 0, examined = 0;
    for (int64_t u = gw; u < units; u += nwaves) {
        if (from_q) {
            const int64_t i = u * GT_WAVE + lane;
            int32_t v = -1;
            if (i < nf) {
                v = q[i];
                atomicOr((unsigned long long*)&vb[v >> 6], 1ull << (v & 63));
            }
            td_expand_vertices<SPLIT>(v, hub_deg, a, va, vb, lvl, par, next_level, append, set, qn, fdeg, nfound,
                                      examined);
        } else {
            // lane i holds word 64u + i; only discoveries (never in va) are
            // added to vb meanwhile, so va & ~vb is exactly the frontier
            const int64_t wd = u * GT_WAVE + lane;
            const uint64_t fw = wd < a.words ? (va[wd] & ~vb[wd]) : 0ull;
            if (fw) atomicOr((unsigned long long*)&vb[wd], (unsigned long long)fw);
            const int32_t cnt = __popcll(fw);
            int32_t incl = cnt;
#pragma unroll
            for (int o = 1; o < GT_WAVE; o <<= 1) {
                const int32_t y = __shfl_up(incl, o, GT_WAVE);
                if (lane >= o) incl += y;
            }
            const int32_t excl = incl - cnt;
            const int32_t total = __shfl(incl, GT_WAVE - 1, GT_WAVE);
            for (int32_t r0 = 0; r0 < total; r0 += GT_WAVE) {
                // lane x takes the (r0 + x)-th frontier vertex of the 64 words
                const int32_t x = r0 + lane;
                int lo = 0, hi = GT_WAVE - 1;
#pragma unroll
                for (int st = 0; st < 6; ++st) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (__shfl(excl, mid, GT_WAVE) <= x) lo = mid;
                    else hi = mid - 1;
                }
                const uint64_t ow = __shfl(fw, lo, GT_WAVE);
                const int32_t k = x - __shfl(excl, lo, GT_WAVE);
                const int32_t v = x < total ? (int32_t)((u * GT_WAVE + lo) * GT_WAVE + nth_set_bit(ow, k)) : -1;
                td_expand_vertices<SPLIT>(v, hub_deg, a, va, vb, lvl, par, next_level, append, set, qn, fdeg,
                                          nfound, examined);
            }
        }
    }
    unsigned long long* cs = ctr_slot(set);
    wave_add(&cs[CTR_FOUND], nfound);
    wave_add(&cs[CTR_FOUND_DEG], fdeg);
    wave_add(&cs[CTR_EXAMINED], examined);
}

// Top-down level, second part: the long rows' chunks of TD_CHUNK entries.
// A wave takes a contiguous range of chunk indices, finds the record of its
// first chunk by binary search over the records' first-chunk indices and
// walks forward.
template <bool SPLIT>
__device__ __forceinline__ void td_chunks(const TdLevel& c, const GArgs<SPLIT>& a) {
    constexpr int B = TD_CHUNK / GT_WAVE;
    const int cur = c.cur;
    const uint64_t* va = a.vis[cur];
    uint64_t* vb = a.vis[cur ^ 1];
    int32_t* qn = a.q[c.qi ^ 1];
    const bool append = c.append;
    const int32_t next_level = c.next_level;
    int32_t* lvl = c.lvl;
    int32_t* par = c.par;
    unsigned long long* set = a.ctr + (c.lev & 1) * CTR_SET;
    const unsigned long long packed = set[CTR_TDCHUNKS];
    int64_t nrows = (int64_t)(packed >> 32);
    nrows = nrows < a.row_cap ? nrows : a.row_cap;
    const int64_t nch = (int64_t)(packed & 0xFFFFFFFFull);
    if (nrows == 0 || nch == 0) return;
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    const int64_t per = (nch + nwaves - 1) / nwaves;
    const int64_t c0 = gw * per;
    const int64_t c1 = c0 + per < nch ? c0 + per : nch;
    unsigned long long fdeg = 0, nfound = 0;
    if (c0 < c1) {
        int64_t lo = 0, hi = nrows - 1;  // last record whose first chunk is <= c0
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if ((int64_t)a.rows[mid].y <= c0) lo = mid;
            else hi = mid - 1;
        }
        int64_t r = lo;
        int2 rec = a.rows[r];
        for (int64_t ci = c0; ci < c1; ++ci) {
            while (r + 1 < nrows && (int64_t)a.rows[r + 1].y <= ci) rec = a.rows[++r];
            const int32_t v = rec.x;
            const int64_t e = a.off[v + 1];
            const int64_t rb = a.off[v] + (ci - (int64_t)rec.y) * TD_CHUNK;
            const int32_t pid = SPLIT ? a.new2old[v] : v;
            int32_t ent[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const int64_t k = rb + i * GT_WAVE + lane;
                ent[i] = k < e ? ld_id_stream(&a.col[k]) : -1;
            }
            int32_t w[B], pp[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                w[i] = ent[i];
                pp[i] = pid;
            }
            td_claim_batch<B, LPS<SPLIT>>(w, pp, va, vb, lvl, par, a.tdeg, next_level, append, &set[CTR_QTAIL], qn, fdeg,
                              nfound);
        }
    }
    unsigned long long* cs = ctr_slot(set);
    wave_add(&cs[CTR_FOUND], nfound);
    wave_add(&cs[CTR_FOUND_DEG], fdeg);
}

// SPLIT, after the traversal: one byte per anchor k (a core vertex that
// leaves, or edge trees, hang from), 0 if anchor_core[k] was not reached,
// else its level + 1 (the level of a leaf hanging off it), 255 if that does
// not fit. Only anchors are read, so the leaf pass gathers from an array of
// n_anchor bytes (a tenth of the core on Kronecker graphs) that stays in L2.
__device__ __forceinline__ void anchor_bytes(int64_t n_anchor, const int32_t* __restrict__ anchor_core,
                                             const uint64_t* __restrict__ visit, const int2* __restrict__ lp_core,
                                             uint8_t* __restrict__ lvc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_anchor; k += stride) {
        const int32_t c = anchor_core[k];
        const bool reached = (visit[c >> 6] >> (c & 63)) & 1ull;
        lvc[k] = reached ? leaf_level_byte(lp_core[c].x) : (uint8_t)0;
    }
}

// SPLIT epilogue over caller ids v (ascending, coalesced writes):
//  v == root                -> (root, 0)
//  v == partner             -> (root, 1)   [the neighbour of a leaf root]
//  core, reached            -> (parent, core level); parents are caller ids
//  leaf, neighbour core and reached -> (neighbour, neighbour level + 1)
//  otherwise                -> (-1, -1)
// A wave covers 64 consecutive caller ids, one class group: the new id of
// a core vertex (hub or not) or a leaf is the group's first new id of that
// class plus the number of group members of the class below it. The leaf pass
// (Algorithm 7) reads the leaf list in order and gathers one byte per leaf
// (the level byte of its neighbour's anchor), so its only random reads go to
// an array of one byte per anchor. Outputs are written with streaming stores.
constexpr int OUT_ITEMS = 4;  // vertices per thread, loads issued together

__device__ __forceinline__ void split_output(
    int64_t n, const ClassGroup* __restrict__ groups, const uint64_t* __restrict__ visit,
    const uint8_t* __restrict__ lvc, const int2* __restrict__ lp_core, const int32_t* __restrict__ anchor_core,
    const int32_t* __restrict__ leaf_anchor, const int32_t* __restrict__ leaf_src_old,
    const int32_t* __restrict__ tdepth, int32_t root, int32_t partner, int32_t* __restrict__ parent_out,
    int32_t* __restrict__ level_out) {
    const int64_t step = (int64_t)OUT_BLOCK * OUT_ITEMS;
    const int lane = lane_id();
    const uint64_t below = (1ull << lane) - 1ull;
    // the wave's index in the block, as a wave-uniform value, so that the
    // class groups are read with scalar loads
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / GT_WAVE));
    const int64_t ngroups = (n + GT_WAVE - 1) / GT_WAVE;
    for (int64_t base = (int64_t)blockIdx.x * step; base < n; base += (int64_t)gridDim.x * step) {
        int64_t v[OUT_ITEMS];
        int32_t cid[OUT_ITEMS], lid[OUT_ITEMS];
        ClassGroup G[OUT_ITEMS];
#pragma unroll
        for (int i = 0; i < OUT_ITEMS; ++i) {
            const int64_t gi = (base + (int64_t)i * OUT_BLOCK) / GT_WAVE + wave;
            G[i] = gi < ngroups ? groups[gi] : ClassGroup{0ull, 0ull, 0, 0, 0, 0};
        }
#pragma unroll
        for (int i = 0; i < OUT_ITEMS; ++i) {
            v[i] = base + (int64_t)i * OUT_BLOCK + threadIdx.x;
            const uint64_t core = G[i].m0 & ~G[i].m1, leaf = G[i].m1 & ~G[i].m0, hub = G[i].m0 & G[i].m1;
            cid[i] = ((core >> lane) & 1ull)  ? G[i].core_base + __popcll(core & below)
                     : ((hub >> lane) & 1ull) ? G[i].hub_base + __popcll(hub & below)
                                              : -1;
            lid[i] = ((leaf >> lane) & 1ull) ? G[i].leaf_base + __popcll(leaf & below) : -1;
        }
        // core: own bit, level and parent; leaf: its neighbour. Every lane
        // loads both kinds, at its own index or else at the group's first
        // one (the same cache lines, always in range), so that no load
        // waits on a branch and all of them are in flight together.
        uint64_t w[OUT_ITEMS];
        int32_t lc[OUT_ITEMS], pc[OUT_ITEMS], src[OUT_ITEMS], ps[OUT_ITEMS], dp[OUT_ITEMS];
#pragma unroll
        for (int i = 0; i < OUT_ITEMS; ++i) {
            const int32_t c = cid[i] >= 0 ? cid[i] : G[i].core_base;
            const int32_t j = lid[i] >= 0 ? lid[i] : G[i].leaf_base;
            w[i] = visit[c >> 6];
            const int2 lp = lp_core[c];
            lc[i] = lp.x;
            pc[i] = lp.y;
            src[i] = leaf_anchor[j];
            ps[i] = leaf_src_old[j];
            dp[i] = tdepth ? tdepth[j] : 1;  // edge trees: hops below the core-edge vertex
        }
#pragma unroll
        for (int i = 0; i < OUT_ITEMS; ++i)
            if (lid[i] < 0) src[i] = -1;
        // leaf pass: reached iff its neighbour (its anchor src) was reached
        int32_t b[OUT_ITEMS];
#pragma unroll
        for (int i = 0; i < OUT_ITEMS; ++i) b[i] = src[i] >= 0 ? lvc[src[i]] : 0;
#pragma unroll
        for (int i = 0; i < OUT_ITEMS; ++i) {
            if (v[i] >= n) continue;
            int32_t p = -1, l = -1;
            if (cid[i] >= 0) {
                if ((w[i] >> (cid[i] & 63)) & 1ull) {
                    p = pc[i];
                    l = lc[i];
                }
            } else if (b[i] != 0) {
                p = ps[i];
                l = b[i] < 255 ? b[i] - 1 + dp[i] : lp_core[anchor_core[src[i]]].x + dp[i];
            }
            if (v[i] == root) {
                p = root;
                l = 0;
            } else if (v[i] == partner) {
                p = root;
                l = 1;
            }
            st_stream(&parent_out[v[i]], p);
            st_stream(&level_out[v[i]], l);
        }
    }
}

}  // namespace
