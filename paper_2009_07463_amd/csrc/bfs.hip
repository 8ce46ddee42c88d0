// Single-source traversal: direction-optimizing BFS (Section 2.1, Algorithm
// 1) on the traversed graph -- the whole graph for PLAIN handles, the core
// subgraph for SPLIT handles -- and, for SPLIT, the edge-tree BFS driver of
// Algorithm 9 with the leaf pass of Algorithm 7 (TEOLV).
//
// Kernels:
//  k_bfs_init      clears the visited bitmap, seeds the root, and (PLAIN)
//                  writes -1 to both outputs.
//  k_td_expand     top-down level: every adjacency entry of the frontier is
//                  one work item (edge-balanced: a prefix sum over frontier
//                  degrees maps items to rows), so hub rows are spread over
//                  the whole grid; claims by atomicOr on the bitmap word.
//  k_bu            bottom-up level: one wavefront per 64-vertex bitmap word
//                  (Algorithm 5's block = one wave); each unvisited lane scans
//                  its row until the first neighbour visited in the snapshot,
//                  long rows are finished by the whole wave; the word of the
//                  next bitmap is written once.
//  k_split_output  SPLIT epilogue in one coalesced pass over caller ids:
//                  core results translated to caller ids, the leaf pass
//                  (a leaf is reached iff its neighbour is, one level
//                  deeper), -1 for everything unreached.
#include <algorithm>
#include <climits>
#include <mutex>
#include <string>
#include <unordered_map>

#include "bfs_kernels.h"

namespace {


__global__ void k_bfs_init(uint64_t* __restrict__ visit, int64_t words, int32_t seed,
                           int32_t seed_level, int32_t seed_parent, int32_t* __restrict__ level,
                           int32_t* __restrict__ parent, int32_t* __restrict__ q0,
                           unsigned long long* __restrict__ ctr, int32_t* __restrict__ fill_level,
                           int32_t* __restrict__ fill_parent, int64_t n_fill) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t span = words > n_fill ? words : n_fill;
    for (int64_t i = tid; i < span; i += stride) {
        if (i < words)
            visit[i] = (seed >= 0 && i == (seed >> 6)) ? (1ull << (seed & 63)) : 0ull;
        if (i < n_fill) {
            const bool s = (i == seed);
            fill_level[i] = s ? seed_level : -1;
            fill_parent[i] = s ? seed_parent : -1;
        }
    }
    if (blockIdx.x == 0) {
        clear_set(ctr);
        clear_set(ctr + CTR_SET);
        if (threadIdx.x == 0 && seed >= 0) {
            q0[0] = seed;
            if (n_fill == 0) {  // SPLIT: (level, parent) pairs, LPS<true> = 2
                level[(int64_t)seed * LPS<true>] = seed_level;
                parent[(int64_t)seed * LPS<true>] = seed_parent;
            }
        }
    }
}

__global__ void k_degrees(const int64_t* __restrict__ off, int64_t n, int32_t* __restrict__ deg) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        deg[v] = (int32_t)(off[v + 1] - off[v]);
}

// Degree of the i-th frontier vertex (for the top-down prefix sum).
struct LoadFrontierDeg {
    const int32_t* q;
    const int64_t* off;
    __device__ __forceinline__ int64_t operator()(int64_t i) const {
        const int32_t u = q[i];
        return off[u + 1] - off[u];
    }
};

// Bits set in a but not in b, per 64-bit word (queue compaction).
struct LoadNewBits {
    const uint64_t* a;
    const uint64_t* b;
    __device__ __forceinline__ int64_t operator()(int64_t w) const {
        return (int64_t)__popcll(a[w] & ~b[w]);
    }
};

// Vertices (< n) whose bit is clear, per 64-bit word (unvisited list).
struct LoadUnvisited {
    const uint64_t* vis;
    int64_t n;
    __device__ __forceinline__ int64_t operator()(int64_t w) const {
        uint64_t x = ~vis[w];
        const int64_t rem = n - w * 64;
        if (rem < 64) x &= (1ull << rem) - 1ull;
        return (int64_t)__popcll(x);
    }
};

// List of the vertices (< n) whose bit is clear, ascending.
__global__ void __launch_bounds__(COMPACT_BLOCK) k_compact_unvisited(const uint64_t* __restrict__ vis, int64_t n,
                                                                     int64_t words,
                                                                     const int64_t* __restrict__ prefix,
                                                                     int32_t* __restrict__ list) {
    const int64_t stride = (int64_t)gridDim.x * COMPACT_BLOCK;
    for (int64_t w = (int64_t)blockIdx.x * COMPACT_BLOCK + threadIdx.x; w < words; w += stride) {
        uint64_t x = ~vis[w];
        const int64_t rem = n - w * 64;
        if (rem < 64) x &= (1ull << rem) - 1ull;
        int64_t pos = prefix[w];
        while (x) {
            const int j = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            list[pos++] = (int32_t)(w * 64 + j);
        }
    }
}

// Queue of the vertices whose bit is set in a and clear in b, ascending.
__global__ void __launch_bounds__(COMPACT_BLOCK) k_compact_queue(const uint64_t* __restrict__ a,
                                                                 const uint64_t* __restrict__ b,
                                                                 int64_t words,
                                                                 const int64_t* __restrict__ prefix,
                                                                 int32_t* __restrict__ q) {
    const int64_t stride = (int64_t)gridDim.x * COMPACT_BLOCK;
    for (int64_t w = (int64_t)blockIdx.x * COMPACT_BLOCK + threadIdx.x; w < words; w += stride) {
        uint64_t x = a[w] & ~b[w];
        int64_t pos = prefix[w];
        while (x) {
            const int j = __ffsll((unsigned long long)x) - 1;
            x &= x - 1;
            q[pos++] = (int32_t)(w * 64 + j);
        }
    }
}

__global__ void k_copy_words(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                             int64_t words) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += stride)
        dst[w] = src[w];
}

// Rows (prefix[r] <= e < prefix[r + 1], 0 <= r < nf) of two entries a <= b
// of the frontier's flat adjacency list, found together by one wave: lanes
// 0-31 search for a, lanes 32-63 for b, each half probing 32 evenly spaced
// rows per step (three dependent loads for frontiers of up to 32^3 vertices).
// prefix is the exclusive degree prefix sum, prefix[nf] > b.
__device__ __forceinline__ void wave_rows2(const int64_t* __restrict__ prefix, int64_t nf, int64_t a, int64_t b,
                                           int64_t* ra, int64_t* rb) {
    const int lane = lane_id();
    const int half = lane >> 5, l = lane & 31;
    const int64_t x = half ? b : a;
    int64_t lo = 0, hi = nf;  // prefix[lo] <= x < prefix[hi]
    while (__ballot(hi - lo > 1)) {
        const int64_t step = (hi - lo + 31) / 32;
        const int64_t p = lo + (int64_t)l * step;
        const bool le = p < hi && prefix[p] <= x;  // true for l = 0, then a run of lanes
        const uint32_t m = (uint32_t)(__ballot(le) >> (32 * half));
        const int64_t nlo = lo + (int64_t)(__popc(m) - 1) * step;
        hi = nlo + step < hi ? nlo + step : hi;
        lo = nlo;
    }
    *ra = __shfl(lo, 0, GT_WAVE);
    *rb = __shfl(lo, 32, GT_WAVE);
}

// Number of lanes l with v_l <= x, for v nondecreasing over the lanes: a
// binary search over the lanes' values (7 shuffles, no memory access).
__device__ __forceinline__ int lanes_le(int64_t v, int64_t x) {
    int lo = 0, hi = GT_WAVE;  // the count lies in [lo, hi]
#pragma unroll
    for (int st = 0; st < 7; ++st) {
        const int mid = (lo + hi) >> 1;
        const int64_t y = __shfl(v, mid & (GT_WAVE - 1), GT_WAVE);
        if (lo < hi) {
            if (y <= x) lo = mid + 1;
            else hi = mid;
        }
    }
    return lo;
}

// Top-down level (Algorithm 1, TOP-DOWN). Every adjacency entry of the
// frontier is one work item; a block takes spans of TD_BLOCK * items
// consecutive items, `items` (1, 2 or 4, larger for larger levels so that
// smaller ones still spread over many workgroups) per thread with all their
// loads in flight together. Wave 0
// finds the rows of the span's first and last item (wave_rows2); when the
// span covers fewer than 64 rows their boundaries sit in the lanes and every
// item finds its row by lanes_le, otherwise by a binary search over the
// span's rows. APPEND: discoveries are appended to q_next (small levels: few
// atomics on the shared tail). Otherwise only the bitmap records them and
// the next queue, if one is needed, is compacted afterwards; for SPLIT the
// degree sum of the discoveries is taken by k_frontier_deg from the bitmap
// difference (one dense pass over the core instead of a random degree load
// per discovery; over the whole graph of a PLAIN handle the pass costs more
// than the loads it saves). new2old (SPLIT) turns the frontier vertex into
// the caller id stored as parent; tdeg is the degree per vertex.
// A SPLIT level without APPEND claims with atomics whose old value it does
// not wait for: every item that saw its target clear writes the target's
// (level, parent) pair, so a target several frontier vertices reach in the
// same level gets one of their (equally valid) parents, and the level's
// discoveries are counted from the bitmap difference by k_frontier_deg.
constexpr int TD_ITEMS = 4;  // most items per thread

// Items per thread for a top-down level of mf frontier entries: 4 once
// every workgroup of a full grid has several spans of 4, fewer below.
inline int td_items(int64_t mf) {
    const int64_t full = (int64_t)TD_BLOCK * 4096;
    return mf >= 4 * TD_ITEMS * full ? 4 : mf >= 2 * full ? 2 : 1;
}

template <bool SPLIT, bool APPEND>
__global__ void __launch_bounds__(TD_BLOCK) k_td_expand(
    const int32_t* __restrict__ q, int64_t nf, const int64_t* __restrict__ prefix,
    const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int32_t* __restrict__ new2old, const int32_t* __restrict__ tdeg, uint64_t* visit,
    int32_t* __restrict__ level, int32_t* __restrict__ parent, int32_t next_level, int32_t* __restrict__ q_next,
    unsigned long long* __restrict__ ctr, unsigned long long* __restrict__ ctr_clear, int items) {
    __shared__ int64_t s_lo, s_hi;
    const int64_t X = prefix[nf];
    if (blockIdx.x == 0) clear_set(ctr_clear);
    unsigned long long fdeg = 0, nfound = 0;
    const int64_t span = (int64_t)TD_BLOCK * items;
    for (int64_t e0 = (int64_t)blockIdx.x * span; e0 < X; e0 += (int64_t)gridDim.x * span) {
        const int64_t elast = (e0 + span < X ? e0 + span : X) - 1;
        if (threadIdx.x < GT_WAVE) {
            int64_t ra, rb;
            wave_rows2(prefix, nf, e0, elast, &ra, &rb);
            if (threadIdx.x == 0) {
                s_lo = ra;
                s_hi = rb;
            }
        }
        __syncthreads();
        const int64_t lo = s_lo, hi = s_hi;
        __syncthreads();
        // narrow span: lane l holds prefix[lo + 1 + l] (the start of row lo + 1 + l)
        const bool narrow = hi - lo < GT_WAVE;
        const int64_t p_lo = prefix[lo];
        int64_t pf = INT64_MAX;
        if (narrow && lo + 1 + lane_id() <= hi) pf = prefix[lo + 1 + lane_id()];
        int64_t row[TD_ITEMS], rpos[TD_ITEMS];
#pragma unroll
        for (int j = 0; j < TD_ITEMS; ++j) {
            const int64_t e = j < items ? e0 + (int64_t)j * TD_BLOCK + threadIdx.x : X;
            if (narrow) {
                const int c = lanes_le(pf, e);
                const int64_t start = __shfl(pf, (c - 1) & (GT_WAVE - 1), GT_WAVE);
                row[j] = lo + c;
                rpos[j] = e - (c == 0 ? p_lo : start);
            } else {
                row[j] = e < X ? first_greater(prefix, lo + 1, hi + 1, e) - 1 : lo;
                rpos[j] = -1;
            }
        }
        if (!narrow) {
#pragma unroll
            for (int j = 0; j < TD_ITEMS; ++j) {
                const int64_t e = j < items ? e0 + (int64_t)j * TD_BLOCK + threadIdx.x : X;
                rpos[j] = e - prefix[row[j]];
            }
        }
        int32_t u[TD_ITEMS], w[TD_ITEMS];
#pragma unroll
        for (int j = 0; j < TD_ITEMS; ++j) u[j] = q[row[j]];
        int64_t rb[TD_ITEMS];
#pragma unroll
        for (int j = 0; j < TD_ITEMS; ++j) rb[j] = off[u[j]];
#pragma unroll
        for (int j = 0; j < TD_ITEMS; ++j) {
            const int64_t e = j < items ? e0 + (int64_t)j * TD_BLOCK + threadIdx.x : X;
            w[j] = e < X ? ld_id_stream(&col[rb[j] + rpos[j]]) : -1;
        }
        uint64_t seen[TD_ITEMS];
#pragma unroll
        for (int j = 0; j < TD_ITEMS; ++j) seen[j] = w[j] >= 0 ? visit[w[j] >> 6] : ~0ull;
        bool found[TD_ITEMS];
#pragma unroll
        for (int j = 0; j < TD_ITEMS; ++j) {
            found[j] = false;
            const uint64_t bit = 1ull << (w[j] & 63);
            if (!(seen[j] & bit)) {
                if (APPEND || !SPLIT) {
                    const uint64_t old = atomicOr((unsigned long long*)&visit[w[j] >> 6], (unsigned long long)bit);
                    found[j] = !(old & bit);
                } else {
                    (void)atomicOr((unsigned long long*)&visit[w[j] >> 6], (unsigned long long)bit);
                    found[j] = true;
                }
            }
        }
        int32_t dg[TD_ITEMS], pid[TD_ITEMS];
#pragma unroll
        for (int j = 0; j < TD_ITEMS; ++j) {
            dg[j] = ((APPEND || !SPLIT) && found[j]) ? ld_stream(&tdeg[w[j]]) : 0;
            pid[j] = (SPLIT && found[j]) ? new2old[u[j]] : u[j];
        }
#pragma unroll
        for (int j = 0; j < TD_ITEMS; ++j) {
            if (found[j]) {
                if (SPLIT) {
                    const long long x = (long long)(uint32_t)next_level | ((long long)(uint32_t)pid[j] << 32);
                    *reinterpret_cast<long long*>(level + 2 * (int64_t)w[j]) = x;
                } else {
                    level[w[j]] = next_level;
                    parent[w[j]] = pid[j];
                }
                fdeg += (unsigned long long)dg[j];
                if (APPEND || !SPLIT) nfound += 1;
            }
        }
        if (APPEND) {
#pragma unroll
            for (int j = 0; j < TD_ITEMS; ++j) {
                const long long slot = wave_append(&ctr[CTR_QTAIL], found[j]);
                if (found[j]) q_next[slot] = w[j];
            }
        }
    }
    unsigned long long* cs = ctr_slot(ctr);
    wave_add(&cs[CTR_FOUND], nfound);
    wave_add(&cs[CTR_FOUND_DEG], fdeg);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&cs[CTR_EXAMINED], (unsigned long long)X);
}

// Number and degree sum of the vertices whose bit is set in a and clear in b
// (the discoveries of a top-down level that kept its start-of-level bitmap
// in b), added to the level's CTR_FOUND and CTR_FOUND_DEG. A wave takes
// FD_WORDS bitmap words per iteration; lane l reads the degree of vertex
// 64 w + l when its bit is new, so each word's degrees are one coalesced read.
constexpr int FD_WORDS = 16;

__global__ void __launch_bounds__(256) k_frontier_deg(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                      int64_t words, const int32_t* __restrict__ tdeg,
                                                      unsigned long long* __restrict__ ctr) {
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    unsigned long long sum = 0, cnt = 0;
    for (int64_t w0 = gw * FD_WORDS; w0 < words; w0 += nwaves * FD_WORDS) {
        uint64_t x[FD_WORDS];
#pragma unroll
        for (int i = 0; i < FD_WORDS; ++i) x[i] = w0 + i < words ? (a[w0 + i] & ~b[w0 + i]) : 0ull;
#pragma unroll
        for (int i = 0; i < FD_WORDS; ++i)
            if ((x[i] >> lane) & 1ull) {
                sum += (unsigned long long)ld_stream(&tdeg[(w0 + i) * GT_WAVE + lane]);
                cnt += 1;
            }
    }
    wave_add(&ctr_slot(ctr)[CTR_FOUND_DEG], sum);
    wave_add(&ctr_slot(ctr)[CTR_FOUND], cnt);
}

// Highest-degree neighbour of every vertex (ties: first in the row), the
// A_in+ list of the degree-aware bottom-up of Section 2.3, stored densely so
// that the first bottom-up probe of 64 consecutive vertices is one coalesced
// read instead of 64 row starts; the second-highest one (hint2, -1 for a
// row of one entry) for the optional second probe; SPLIT also keeps their
// caller ids (hint_orig, hint2_orig), which a hit records as the parent. One
// wave per row; built once per handle.
template <bool SPLIT>
__global__ void k_build_hint(const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ new2old, int64_t n, int32_t* __restrict__ hint,
                             int32_t* __restrict__ hint_orig, int32_t* __restrict__ hint2,
                             int32_t* __restrict__ hint2_orig) {
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    for (int64_t v = gw; v < n; v += nwaves) {
        const int64_t b = off[v], e = off[v + 1];
        // (degree << 32) | ~position: larger = higher degree, then earlier in the row
        unsigned long long b1 = 0, b2 = 0;
        for (int64_t k = b + lane; k < e; k += GT_WAVE) {
            const int32_t u = col[k];
            const unsigned long long d = (unsigned long long)(off[u + 1] - off[u]);
            const unsigned long long key = (d << 32) | (0xFFFFFFFFull - (unsigned long long)(k - b));
            if (key > b1) {
                b2 = b1;
                b1 = key;
            } else if (key > b2) {
                b2 = key;
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {  // merge the two best of two lanes
            const unsigned long long c1 = __shfl_xor(b1, o, GT_WAVE), c2 = __shfl_xor(b2, o, GT_WAVE);
            const unsigned long long lo = b1 < c1 ? b1 : c1, hi2 = b2 > c2 ? b2 : c2;
            b1 = b1 > c1 ? b1 : c1;
            b2 = lo > hi2 ? lo : hi2;
        }
        if (lane == 0) {
            const int32_t h = (e > b) ? col[b + (int64_t)(0xFFFFFFFFull - (b1 & 0xFFFFFFFFull))] : -1;
            const int32_t h2 = (e - b > 1) ? col[b + (int64_t)(0xFFFFFFFFull - (b2 & 0xFFFFFFFFull))] : -1;
            hint[v] = h;
            hint2[v] = h2;
            if (SPLIT) {
                hint_orig[v] = h >= 0 ? new2old[h] : -1;
                hint2_orig[v] = h2 >= 0 ? new2old[h2] : -1;
            }
        }
    }
}

// One bit per vertex: its degree is at most 2, so the two hint probes cover
// its whole row.
__global__ void k_small_bits(const int64_t* __restrict__ off, int64_t n, int64_t words, uint64_t* __restrict__ small) {
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    for (int64_t w = gw; w < words; w += nwaves) {
        const int64_t v = w * GT_WAVE + lane;
        const bool sm = v < n && off[v + 1] - off[v] <= 2;
        const uint64_t m = __ballot(sm);
        if (lane == 0) small[w] = m;
    }
}

// At least 6 waves per SIMD (80 VGPRs; with BU_WPI words per iteration
// the one-probe form does not spill), so three workgroups of BU_BLOCK_MAX
// threads fit a CU.
template <bool SPLIT, bool H2>
__global__ void __launch_bounds__(BU_BLOCK_MAX, 6) k_bu(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, int64_t n,
    int64_t words, const uint64_t* __restrict__ vis_cur, uint64_t* __restrict__ vis_next,
    int32_t* __restrict__ level, int32_t* __restrict__ parent, int32_t next_level,
    int32_t* __restrict__ hub_q, unsigned long long* __restrict__ ctr,
    unsigned long long* __restrict__ ctr_clear, int lane_edges, int64_t hub_deg, BuHints hh,
    const int32_t* __restrict__ new2old, int64_t lds_words) {
    if (blockIdx.x == 0) clear_set(ctr_clear);
    bu_level<SPLIT, false, H2>(off, col, n, words, vis_cur, vis_next, level, parent, next_level, hub_q, ctr,
                               lane_edges, hub_deg, hh, new2old, lds_words);
}

// Two simpler bottom-up forms, kept to measure bu_level's wave-per-word form
// against (knob bu_form):
//  PER_WORD (bu_form 2): Algorithm 5 as a CPU thread runs it. One thread owns
//    a 64-vertex block (bitmap word), takes its unvisited bits lowest first,
//    scans each vertex's row until the first neighbour visited in the
//    snapshot, and writes the block's next word once.
//  otherwise (bu_form 3): one thread per vertex; a wave covers one word and
//    its ballot is the next word.
// Both probe the highest-degree neighbour first when the hint array is
// given (a vertex without a hint has no core neighbour), read the hubs' bits
// from LDS when lds_words > 0, and count as bu_level does (a probe is one
// examined entry; the found degree sums rows found by scanning only).
template <bool SPLIT, bool PER_WORD>
__global__ void __launch_bounds__(BU_BLOCK_MAX) k_bu_simple(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, int64_t n, int64_t words,
    const uint64_t* __restrict__ vis_cur, uint64_t* __restrict__ vis_next, int32_t* __restrict__ level,
    int32_t* __restrict__ parent, int32_t next_level, unsigned long long* __restrict__ ctr,
    unsigned long long* __restrict__ ctr_clear, const int32_t* __restrict__ hint,
    const int32_t* __restrict__ hint_orig, const int32_t* __restrict__ new2old, int64_t lds_words) {
    if (blockIdx.x == 0) clear_set(ctr_clear);
    extern __shared__ uint64_t s_vis[];
    for (int64_t i = threadIdx.x; i < lds_words; i += blockDim.x) s_vis[i] = vis_cur[i];
    __syncthreads();
    const int64_t lds_bits = lds_words * GT_WAVE;
    auto probe = [&](int32_t u) -> bool {
        return u < lds_bits ? ((s_vis[u >> 6] >> (u & 63)) & 1ull) != 0 : bit_of(vis_cur, u);
    };
    unsigned long long fdeg = 0, scanned = 0, examined = 0, nfound = 0;
    // tests unvisited vertex v; on a hit writes its level and parent
    auto visit = [&](int32_t v) -> bool {
        scanned += 1;
        if (hint) {
            const int32_t h = ld_stream(&hint[v]);
            if (h < 0) return false;
            examined += 1;
            if (probe(h)) {
                st_stream_lp<SPLIT>(level, parent, v, next_level, SPLIT ? ld_stream(&hint_orig[v]) : h);
                nfound += 1;
                return true;
            }
        }
        const int64_t b = off[v], e = off[v + 1];
        for (int64_t k = b; k < e; ++k) {
            const int32_t u = col[k];
            examined += 1;
            if (probe(u)) {
                st_stream_lp<SPLIT>(level, parent, v, next_level, caller_id<SPLIT>(new2old, u));
                fdeg += (unsigned long long)(e - b);
                nfound += 1;
                return true;
            }
        }
        return false;
    };
    if (PER_WORD) {
        const int64_t nth = (int64_t)gridDim.x * blockDim.x;
        for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += nth) {
            const uint64_t cur = vis_cur[w];
            uint64_t x = ~cur, add = 0;
            while (x) {
                const int bit = __ffsll((unsigned long long)x) - 1;
                x &= x - 1;
                const int64_t v = w * GT_WAVE + bit;
                if (v >= n) break;
                if (visit((int32_t)v)) add |= 1ull << bit;
            }
            vis_next[w] = cur | add;
        }
    } else {
        const int lane = lane_id();
        const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
        for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE; w < words; w += nwaves) {
            const uint64_t cur = vis_cur[w];
            const int64_t v = w * GT_WAVE + lane;
            const bool f = v < n && !((cur >> lane) & 1ull) && visit((int32_t)v);
            const uint64_t m = __ballot(f);
            if (lane == 0) vis_next[w] = cur | m;
        }
    }
    unsigned long long* cs = ctr_slot(ctr);
    wave_add(&cs[CTR_FOUND], nfound);
    wave_add(&cs[CTR_FOUND_DEG], fdeg);
    wave_add(&cs[CTR_SCANNED], scanned);
    wave_add(&cs[CTR_EXAMINED], examined);
}

// Top-down level whose frontier is a bitmap difference, in the flat
// two-bitmap form (TdLevel); block 0 clears the next level's counters.
template <bool SPLIT>
__global__ void __launch_bounds__(TD_BLOCK) k_td_flat(GArgs<SPLIT> a, TdLevel t, unsigned long long* ctr_clear) {
    if (blockIdx.x == 0) clear_set(ctr_clear);
    td_units<SPLIT>(t, a);
}

template <bool SPLIT>
__global__ void __launch_bounds__(TD_BLOCK) k_td_flat_rows(GArgs<SPLIT> a, TdLevel t) {
    td_chunks<SPLIT>(t, a);
}

// Bottom-up over the list of vertices still unvisited when it was built;
// vis_next starts as a copy of vis_cur.
template <bool SPLIT, bool H2>
__global__ void __launch_bounds__(BU_BLOCK_MAX) k_bu_list(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, int64_t n,
    const int32_t* __restrict__ list, int64_t nlist, const uint64_t* __restrict__ vis_cur,
    uint64_t* __restrict__ vis_next, int32_t* __restrict__ level, int32_t* __restrict__ parent, int32_t next_level,
    int32_t* __restrict__ hub_q, unsigned long long* __restrict__ ctr, unsigned long long* __restrict__ ctr_clear,
    int lane_edges, int64_t hub_deg, BuHints hh, const int32_t* __restrict__ new2old, int64_t lds_words) {
    if (blockIdx.x == 0) clear_set(ctr_clear);
    bu_level<SPLIT, true, H2>(off, col, n, 0, vis_cur, vis_next, level, parent, next_level, hub_q, ctr, lane_edges,
                              hub_deg, hh, new2old, lds_words, list, nlist);
}

template <bool SPLIT>
__global__ void __launch_bounds__(HUB_BLOCK) k_bu_hubs(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, const int32_t* __restrict__ new2old,
    const uint64_t* __restrict__ vis_cur, uint64_t* __restrict__ vis_next,
    int32_t* __restrict__ level, int32_t* __restrict__ parent, int32_t next_level,
    const int32_t* __restrict__ hub_q, unsigned long long* __restrict__ ctr, int lane_edges) {
    bu_hub_rows<SPLIT>(off, col, new2old, vis_cur, vis_next, level, parent, next_level, hub_q, ctr, lane_edges);
}

__global__ void k_anchor_bytes(int64_t n_anchor, const int32_t* __restrict__ anchor_core,
                               const uint64_t* __restrict__ visit, const int2* __restrict__ lp_core,
                               uint8_t* __restrict__ lvc) {
    anchor_bytes(n_anchor, anchor_core, visit, lp_core, lvc);
}

__global__ void __launch_bounds__(OUT_BLOCK) k_split_output(
    int64_t n, const ClassGroup* __restrict__ groups, const uint64_t* __restrict__ visit,
    const uint8_t* __restrict__ lvc, const int2* __restrict__ lp_core, const int32_t* __restrict__ anchor_core,
    const int32_t* __restrict__ leaf_anchor, const int32_t* __restrict__ leaf_src_old,
    const int32_t* __restrict__ tdepth, int32_t root, int32_t partner, int32_t* __restrict__ parent_out,
    int32_t* __restrict__ level_out) {
    split_output(n, groups, visit, lvc, lp_core, anchor_core, leaf_anchor, leaf_src_old, tdepth, root, partner,
                 parent_out, level_out);
}


// Root inside an edge tree (MH > 0): the vertices of its tree, with their
// level and parent as seen from the root, written over the output pass.
__global__ void k_tree_fix(int64_t k, const int32_t* __restrict__ fix, int32_t* __restrict__ parent_out,
                           int32_t* __restrict__ level_out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
        const int32_t v = fix[3 * i];
        level_out[v] = fix[3 * i + 1];
        parent_out[v] = fix[3 * i + 2];
    }
}

}  // namespace

// Working memory of one host-driven traversal: the handle's own buffers
// (gt_bfs), or pieces of the library's static scratch array (gt_bfs_static).
struct BfsWork {
    uint64_t* vis[2];
    int32_t* q[2];
    int64_t* prefix;
    int64_t* scan_tmp;
    int32_t* hub_q;
    int32_t* ulist;
    int2* td_rows;
    int64_t td_row_cap;
    int32_t* level;              // SPLIT: (level, parent) pairs
    uint8_t* lv8;                // SPLIT: level byte per anchor
    unsigned long long* ctr;     // two counter sets
    unsigned long long* h_ctr;   // pinned host mirror of one set (the handle's)
    hipEvent_t* ev;              // timing events, or nullptr: no timing
};

static BfsWork work_of(gt_graph* g) {
    BfsScratch& b = g->bfs;
    BfsWork w;
    w.vis[0] = b.visit[0].as<uint64_t>();
    w.vis[1] = b.visit[1].as<uint64_t>();
    w.q[0] = b.queue[0].as<int32_t>();
    w.q[1] = b.queue[1].as<int32_t>();
    w.prefix = b.prefix.as<int64_t>();
    w.scan_tmp = b.scan_tmp.as<int64_t>();
    w.hub_q = b.hub_q.as<int32_t>();
    w.ulist = b.ulist.as<int32_t>();
    w.td_rows = b.td_rows.as<int2>();
    w.td_row_cap = b.td_row_cap;
    w.level = b.level.as<int32_t>();
    w.lv8 = b.lv8.as<uint8_t>();
    w.ctr = b.ctr.as<unsigned long long>();
    w.h_ctr = b.h_ctr.as<unsigned long long>();
    w.ev = g->tune.timing ? b.ev.data() : nullptr;
    return w;
}

gt_status gt_bfs_scratch_alloc(gt_graph* g, hipStream_t s) {
    BfsScratch& b = g->bfs;
    const int64_t n = g->tn();
    b.n = n;
    b.words = (n + 63) / 64;
    for (int i = 0; i < 2; ++i) {
        GT_TRY(b.visit[i].alloc(sizeof(uint64_t) * (b.words > 0 ? b.words : 1)));
        GT_TRY(b.queue[i].alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
    }
    GT_TRY(b.prefix.alloc(sizeof(int64_t) * (n + 1)));
    GT_TRY(b.hub_q.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
    GT_TRY(b.ulist.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
    // long rows of one flat top-down level over a bitmap frontier: rows
    // longer than td_hub_deg (>= TD_CHUNK) number at most E / TD_CHUNK
    b.td_row_cap = g->tE() / TD_CHUNK + 64;
    GT_TRY(b.td_rows.alloc(sizeof(int2) * (size_t)b.td_row_cap));
    GT_TRY(b.scan_tmp.alloc(sizeof(int64_t) * scan_scratch_elems(n + 1)));
    if (g->flags & GT_BUILD_SPLIT) {
        // (level, parent) pairs of the core vertices, padded to a multiple of
        // four pairs for the 16-byte loads of the leaf-pass bytes
        GT_TRY(b.level.alloc(sizeof(int2) * (size_t)(4 * ((n + 3) / 4) + 4)));
        GT_TRY(b.lv8.alloc((size_t)(g->n_anchor > 0 ? g->n_anchor : 1)));
    }
    {
        const bool split = (g->flags & GT_BUILD_SPLIT) != 0;
        GT_TRY(b.hint.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
        GT_TRY(b.hint2.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
        GT_TRY(b.small.alloc(sizeof(uint64_t) * (b.words > 0 ? b.words : 1)));
        if (split) {
            GT_TRY(b.hint_orig.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
            GT_TRY(b.hint2_orig.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
        }
        if (n > 0) {
            if (split)
                hipLaunchKernelGGL((k_build_hint<true>), dim3(grid_for(n * GT_WAVE, 256)), dim3(256), 0, s,
                                   g->coff.as<int64_t>(), g->ccol.as<int32_t>(), g->new2old.as<int32_t>(), n,
                                   b.hint.as<int32_t>(), b.hint_orig.as<int32_t>(), b.hint2.as<int32_t>(),
                                   b.hint2_orig.as<int32_t>());
            else
                hipLaunchKernelGGL((k_build_hint<false>), dim3(grid_for(n * GT_WAVE, 256)), dim3(256), 0, s,
                                   g->off.as<int64_t>(), g->col.as<int32_t>(), (const int32_t*)nullptr, n,
                                   b.hint.as<int32_t>(), (int32_t*)nullptr, b.hint2.as<int32_t>(), (int32_t*)nullptr);
            GT_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_small_bits, dim3(grid_for(b.words * GT_WAVE, 256, 16384)), dim3(256), 0, s, g->toff(),
                               n, b.words, b.small.as<uint64_t>());
            GT_HIP(hipGetLastError());
        }
    }
    // degree of every traversed vertex (the core degree for SPLIT)
    GT_TRY(b.tdeg.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
    if (n > 0)
        hipLaunchKernelGGL(k_degrees, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, g->toff(), n,
                           b.tdeg.as<int32_t>());
    GT_HIP(hipGetLastError());
    {
        // LDS-resident hub frontier: words per workgroup and resident workgroups
        int dev = 0;
        GT_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        GT_HIP(hipGetDeviceProperties(&prop, dev));
        b.bu_lds_words_max = (int64_t)(prop.sharedMemPerBlock / sizeof(uint64_t));
        const int64_t lw = std::min<int64_t>((g->n_hub + 63) / 64, b.bu_lds_words_max);
        b.bu_resident[0] = b.bu_resident[1] = b.bu_list_resident[0] = b.bu_list_resident[1] = 0;
        if (lw > 0) {
            const bool split = (g->flags & GT_BUILD_SPLIT) != 0;
            const size_t lb = (size_t)lw * sizeof(uint64_t);
            // per kernel: the one- and two-probe forms differ in registers
            int a1 = 0, a2 = 0, l1 = 0, l2 = 0;
            if (split) {
                GT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a1, k_bu<true, false>, BU_BLOCK_MAX, lb));
                GT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a2, k_bu<true, true>, BU_BLOCK_MAX, lb));
                GT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&l1, k_bu_list<true, false>, BU_BLOCK_MAX, lb));
                GT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&l2, k_bu_list<true, true>, BU_BLOCK_MAX, lb));
            } else {
                GT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a1, k_bu<false, false>, BU_BLOCK_MAX, lb));
                GT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&a2, k_bu<false, true>, BU_BLOCK_MAX, lb));
                GT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&l1, k_bu_list<false, false>, BU_BLOCK_MAX, lb));
                GT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&l2, k_bu_list<false, true>, BU_BLOCK_MAX, lb));
            }
            b.bu_resident[0] = a1 * prop.multiProcessorCount;
            b.bu_resident[1] = a2 * prop.multiProcessorCount;
            b.bu_list_resident[0] = l1 * prop.multiProcessorCount;
            b.bu_list_resident[1] = l2 * prop.multiProcessorCount;
        }
    }
    GT_TRY(b.ctr.alloc(sizeof(unsigned long long) * 2 * CTR_SET));
    GT_TRY(b.h_ctr.alloc(sizeof(unsigned long long) * CTR_SET));
    b.ev.assign(4 * GT_MAX_LEVELS + 4, nullptr);
    for (auto& e : b.ev) GT_HIP(hipEventCreate(&e));
    return GT_OK;
}

static float ev_ms(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return -1.f;
    }
    return ms;
}

// Queue (ascending ids) of the bits set in a and clear in b.
static gt_status compact_queue(gt_graph* g, const BfsWork& w, const uint64_t* a, const uint64_t* b, int32_t* q,
                               hipStream_t s) {
    BfsScratch& sc = g->bfs;
    GT_TRY((scan_exclusive<int64_t, LoadNewBits>(LoadNewBits{a, b}, sc.words, w.prefix, w.scan_tmp, s)));
    hipLaunchKernelGGL(k_compact_queue, dim3(grid_for(sc.words, COMPACT_BLOCK, 16384)), dim3(COMPACT_BLOCK),
                       0, s, a, b, sc.words, w.prefix, q);
    GT_HIP(hipGetLastError());
    return GT_OK;
}

// Root handling (Algorithm 9): a leaf root is the parent of its only
// neighbour, which seeds the core traversal at level 1; a leaf root whose
// neighbour is a leaf (a two-vertex component) and an isolated root need no
// core traversal at all.
// Root inside an edge tree (MH > 0, Algorithm 9): walk from the root up to
// its tree's top; the core-edge vertex above it seeds the core traversal at
// the root's depth, and every other vertex of the tree gets its distance from
// the root (up to the lowest common ancestor with the root's chain, then down)
// and its parent on that path.
static void plan_tree_root(const gt_graph* g, int64_t j, RootPlan& rp) {
    const int64_t nc = g->n_core;
    const std::vector<int32_t>& par = g->h_leaf_src_old;   // tree parent, caller id
    auto tree_index = [&](int32_t caller) -> int64_t {
        if (caller < 0) return -1;
        const int64_t nv = g->h_old2new[caller];
        return (nv >= nc && nv < nc + g->n_leaf) ? nv - nc : -1;
    };
    std::unordered_map<int64_t, int32_t> pos;  // tree index on the root's chain -> hops from the root
    std::vector<int64_t> chain;
    for (int64_t x = j; x >= 0;) {
        pos.emplace(x, (int32_t)chain.size());
        chain.push_back(x);
        const int32_t p = par[(size_t)x];
        x = p >= 0 ? tree_index(p) : -1;
    }
    const int64_t top = chain.back();
    const int32_t c = g->h_leaf_src_new[(size_t)j];  // core id of the core-edge vertex, or -1
    rp.seed = (c >= 0 && c < nc) ? c : -1;
    rp.seed_level = (int32_t)chain.size();           // = the root's depth below that vertex
    rp.seed_parent = g->h_tree_old[(size_t)top];
    rp.seed_caller = rp.seed >= 0 ? par[(size_t)top] : -1;
    rp.partner = -1;
    const int64_t t = g->h_tree_of[(size_t)j];
    for (int64_t m = g->h_tree_start[(size_t)t]; m < g->h_tree_start[(size_t)t + 1]; ++m) {
        const int64_t x = g->h_tree_members[(size_t)m];
        if (x == j) continue;
        int32_t up = 0;
        int64_t y = x;
        auto it = pos.find(y);
        while (it == pos.end() && y >= 0) {  // the walk meets the chain at the top at the latest
            y = tree_index(par[(size_t)y]);
            ++up;
            it = pos.find(y);
        }
        if (it == pos.end()) continue;
        int32_t parent;
        if (up == 0) parent = g->h_tree_old[(size_t)chain[(size_t)it->second - 1]];  // on the chain: its child toward the root
        else parent = par[(size_t)x];
        rp.fix_v.push_back(g->h_tree_old[(size_t)x]);
        rp.fix_level.push_back(up + it->second);
        rp.fix_parent.push_back(parent);
    }
}

RootPlan gt_plan_root(const gt_graph* g, int32_t root) {
    RootPlan rp;
    rp.seed = root;
    rp.seed_parent = root;
    if (!(g->flags & GT_BUILD_SPLIT)) return rp;
    const int64_t nr = g->h_old2new[root];
    if (nr < g->n_core) {
        rp.seed = (int32_t)nr;
    } else if (nr < g->n_core + g->n_leaf) {
        rp.root_class = 1;
        const int64_t j = nr - g->n_core;
        if (g->mh > 0) {
            plan_tree_root(g, j, rp);
            return rp;
        }
        rp.partner = g->h_leaf_src_old[j];
        const int32_t sn = g->h_leaf_src_new[j];
        rp.seed = sn < g->n_core ? sn : -1;
        rp.seed_level = 1;
    } else {
        rp.root_class = 2;
        rp.seed = -1;
    }
    return rp;
}

// Root inside an edge tree (MH > 0): the other vertices of its tree get the
// level and parent seen from the root, after the output pass on the same
// stream. The host staging buffer is reused by the next call, which starts
// only after this one has synchronised the stream.
static gt_status apply_tree_fix(gt_graph* g, const RootPlan& rp, int32_t* parent_out, int32_t* level_out,
                                hipStream_t s) {
    const int64_t nfix = (int64_t)rp.fix_v.size();
    if (nfix == 0) return GT_OK;
    BfsScratch& b = g->bfs;
    if (nfix > b.fix_cap) {
        GT_TRY(b.fix.alloc(sizeof(int32_t) * 3 * (size_t)nfix));
        GT_TRY(b.h_fix.alloc(sizeof(int32_t) * 3 * (size_t)nfix));
        b.fix_cap = nfix;
    }
    int32_t* hf = b.h_fix.as<int32_t>();
    for (int64_t i = 0; i < nfix; ++i) {
        hf[3 * i] = rp.fix_v[(size_t)i];
        hf[3 * i + 1] = rp.fix_level[(size_t)i];
        hf[3 * i + 2] = rp.fix_parent[(size_t)i];
    }
    GT_HIP(hipMemcpyAsync(b.fix.p, hf, sizeof(int32_t) * 3 * (size_t)nfix, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_tree_fix, dim3(grid_for(nfix, 256, 4096)), dim3(256), 0, s, nfix,
                       (const int32_t*)b.fix.as<int32_t>(), parent_out, level_out);
    GT_HIP(hipGetLastError());
    return GT_OK;
}

// Launch shape of the bottom-up kernels for `units` wave iterations (groups
// of BU_WPI bitmap words or list groups). With the LDS-resident hub frontier
// (bu_lds = 1 on a hubs-first handle) a workgroup of BU_BLOCK_MAX threads
// copies the hubs' bits (up to the per-workgroup LDS limit) and the grid is
// the workgroups that fit on the device at once, each looping over many
// units; otherwise BU_BLOCK threads and up to bu_blocks workgroups.
// Neighbour probes of a bottom-up level whose frontier holds nf of the n_t
// traversed vertices, for bu_hint: 1 the highest-degree neighbour, 3 also
// the second-highest (and the small-row bits), 2 none, 4 as 3 when the
// frontier is under 1% of the vertices and as 1 otherwise (few vertices then
// have their highest-degree neighbour in it, and a degree <= 2 vertex both
// probes miss needs no row read).
static BuHints bu_hints(const BfsScratch& b, const gt_tuning& tu, int64_t nf, int64_t n_t) {
    BuHints h;
    h.hint = tu.bu_hint != 2 ? b.hint.as<int32_t>() : nullptr;
    h.hint_orig = b.hint_orig.as<int32_t>();
    const bool two = tu.bu_hint == 3 || (tu.bu_hint == 4 && nf * 100 < n_t);
    h.hint2 = two ? b.hint2.as<int32_t>() : nullptr;
    h.hint2_orig = b.hint2_orig.as<int32_t>();
    h.small = b.small.as<uint64_t>();
    return h;
}

struct BuLaunch {
    unsigned blocks, threads;
    size_t lds_bytes;
    int64_t lds_words;
};

static BuLaunch bu_launch(const gt_graph* g, int64_t units, bool list, bool h2) {
    const BfsScratch& b = g->bfs;
    const gt_tuning& tu = g->tune;
    BuLaunch l;
    l.lds_words = (tu.bu_lds == 1) ? std::min<int64_t>((g->n_hub + 63) / 64, b.bu_lds_words_max) : 0;
    if (l.lds_words > 0) {
        l.threads = BU_BLOCK_MAX;
        l.lds_bytes = (size_t)l.lds_words * sizeof(uint64_t);
        const int resident = list ? b.bu_list_resident[h2] : b.bu_resident[h2];
        l.blocks = grid_for(units, BU_BLOCK_MAX / GT_WAVE, std::max(resident, 1));
    } else {
        l.threads = BU_BLOCK;
        l.lds_bytes = 0;
        l.blocks = grid_for(units, BU_BLOCK / GT_WAVE, tu.bu_blocks);
    }
    return l;
}

template <bool SPLIT>
static gt_status bfs_run(gt_graph* g, int32_t root, int32_t* parent_out, int32_t* level_out,
                         hipStream_t s, const BfsWork& w) {
    using T = int32_t;
    BfsScratch& b = g->bfs;  // per-graph arrays (degrees, hints); working memory comes from w
    const gt_tuning& tu = g->tune;
    const bool split = SPLIT;
    const bool timing = w.ev != nullptr;
    const int64_t n_t = g->tn();
    const int64_t* off = g->toff();
    const T* col = SPLIT ? (const T*)g->ccol.p : (const T*)g->col.p;
    const int32_t* n2o = SPLIT ? g->new2old.as<int32_t>() : nullptr;
    gt_run_stats& st = g->stats;
    st.n_levels = 0;
    st.root_class = 0;
    st.ms_init = st.ms_output = st.ms_total = 0.f;

    const RootPlan rp = gt_plan_root(g, root);
    const int32_t seed = rp.seed, seed_level = rp.seed_level, partner = rp.partner, seed_parent = rp.seed_parent;
    st.root_class = rp.root_class;
    // SPLIT: the pair array (parent next to level, stride LPS<true>)
    int32_t* lvl = split ? w.level : level_out;
    int32_t* par = split ? w.level + 1 : parent_out;
    int32_t* q[2] = {w.q[0], w.q[1]};
    uint64_t* vis[2] = {w.vis[0], w.vis[1]};
    unsigned long long* ctr = w.ctr;
    unsigned long long* h = w.h_ctr;
    hipEvent_t* ev = w.ev;
    const int EV_INIT0 = 0, EV_INIT1 = 1, EV_OUT0 = 2, EV_OUT1 = 3, EV_LVL = 4;

    if (timing) GT_HIP(hipEventRecord(ev[EV_INIT0], s));
    {
        const int64_t n_fill = split ? 0 : g->n;
        const int64_t span = std::max<int64_t>(b.words, n_fill);
        hipLaunchKernelGGL(k_bfs_init, dim3(grid_for(span, 256, 16384)), dim3(256), 0, s, vis[0],
                           b.words, seed, seed_level, seed_parent, lvl, par, q[0], ctr,
                           split ? (int32_t*)nullptr : level_out,
                           split ? (int32_t*)nullptr : parent_out, n_fill);
        GT_HIP(hipGetLastError());
    }
    if (timing) GT_HIP(hipEventRecord(ev[EV_INIT1], s));

    // cur: index of the current visited bitmap. qi: queue holding the
    // frontier when need_queue is false; otherwise the frontier is the set of
    // bits in vis[cur] and not in vis[cur ^ 1] and is compacted on demand.
    int cur = 0, qi = 0, lev = 0;
    bool need_queue = false;
    int dir = GT_DIR_TOP_DOWN;  // a one-vertex frontier always starts top-down
    int64_t nf = seed >= 0 ? 1 : 0, mf = -1, mu = g->tE();
    // bottom-up over a list of the unvisited vertices once they are few
    int64_t visited = nf, nlist = -1;
    int32_t L = seed_level;
    while (nf > 0) {
        const int set = lev & 1;
        unsigned long long* c_now = ctr + set * CTR_SET;
        unsigned long long* c_next = ctr + (set ^ 1) * CTR_SET;
        const bool rec = timing && lev < GT_MAX_LEVELS;
        if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev], s));
        bool appended = false;
        int kind = GT_KERNEL_TD_EDGES;
        if (dir == GT_DIR_TOP_DOWN && need_queue && tu.td_flat == 1) {
            // frontier = bits of vis[cur] missing from vis[cur ^ 1]: flat
            // two-bitmap top-down, no queue; the new visited set ends in
            // vis[cur ^ 1] and the next frontier is again a difference
            GArgs<SPLIT> a;
            a.off = off;
            a.col = col;
            a.new2old = n2o;
            a.tdeg = b.tdeg.as<int32_t>();
            a.hh = BuHints{nullptr, nullptr, nullptr, nullptr, nullptr};
            a.vis[0] = vis[0];
            a.vis[1] = vis[1];
            a.q[0] = q[0];
            a.q[1] = q[1];
            a.hub_q = w.hub_q;
            a.ctr = ctr;
            a.rows = w.td_rows;
            a.row_cap = w.td_row_cap;
            a.n = n_t;
            a.words = b.words;
            a.td_hub_deg = tu.td_hub_deg;
            a.bu_hub_deg = tu.bu_hub_deg;
            a.bu_lane_edges = tu.bu_lane_edges;
            TdLevel tl;
            tl.cur = cur;
            tl.qi = qi;
            tl.next_level = L + 1;
            tl.lev = lev;
            tl.nf = nf;
            tl.from_q = false;
            tl.append = false;
            tl.lvl = lvl;
            tl.par = par;
            kind = GT_KERNEL_TD_FLAT;
            if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 1], s));
            hipLaunchKernelGGL((k_td_flat<SPLIT>),
                               dim3(grid_for((b.words + GT_WAVE - 1) / GT_WAVE, TD_BLOCK / GT_WAVE, tu.bu_blocks)),
                               dim3(TD_BLOCK), 0, s, a, tl, c_next);
            hipLaunchKernelGGL((k_td_flat_rows<SPLIT>), dim3(tu.bu_hub_blocks), dim3(TD_BLOCK), 0, s, a, tl);
            if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 2], s));
            GT_HIP(hipGetLastError());
            cur ^= 1;
        } else if (dir == GT_DIR_TOP_DOWN) {
            if (need_queue) {
                GT_TRY(compact_queue(g, w, vis[cur], vis[cur ^ 1], q[qi], s));
                need_queue = false;
            }
            GT_TRY((scan_exclusive<int64_t, LoadFrontierDeg>(LoadFrontierDeg{q[qi], off}, nf,
                                                             w.prefix,
                                                             w.scan_tmp, s)));
            const bool small = mf >= 0 && mf <= tu.td_small_edges;
            const int items = mf >= 0 ? td_items(mf) : 1;
            const unsigned blocks = mf >= 0 ? grid_for(mf, TD_BLOCK * items, tu.td_blocks) : 1024u;
            if (small || mf < 0) {
                if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 1], s));
                hipLaunchKernelGGL((k_td_expand<SPLIT, true>), dim3(blocks), dim3(TD_BLOCK), 0, s, q[qi],
                                   nf, w.prefix, off, col, n2o, b.tdeg.as<int32_t>(), vis[cur], lvl,
                                   par, L + 1, q[qi ^ 1], c_now, c_next, items);
                if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 2], s));
                appended = true;
            } else {
                // keep the start-of-level bitmap so the discoveries can be
                // compacted into a queue if the next level is top-down too
                hipLaunchKernelGGL(k_copy_words, dim3(grid_for(b.words, 256, 8192)), dim3(256), 0, s,
                                   vis[cur], vis[cur ^ 1], b.words);
                if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 1], s));
                hipLaunchKernelGGL((k_td_expand<SPLIT, false>), dim3(blocks), dim3(TD_BLOCK), 0, s, q[qi],
                                   nf, w.prefix, off, col, n2o, b.tdeg.as<int32_t>(), vis[cur], lvl,
                                   par, L + 1, q[qi ^ 1], c_now, c_next, items);
                if (SPLIT)
                    hipLaunchKernelGGL(k_frontier_deg,
                                       dim3(grid_for((b.words + FD_WORDS - 1) / FD_WORDS, 256 / GT_WAVE, 4096)),
                                       dim3(256), 0, s, (const uint64_t*)vis[cur], (const uint64_t*)vis[cur ^ 1],
                                       b.words, b.tdeg.as<int32_t>(), c_now);
                if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 2], s));
            }
            GT_HIP(hipGetLastError());
        } else {
            const int64_t unvisited = n_t - visited;
            const bool simple = tu.bu_form != 1;
            if (!simple && nlist < 0 && unvisited * (int64_t)tu.bu_list_div <= n_t) {
                GT_TRY((scan_exclusive<int64_t, LoadUnvisited>(LoadUnvisited{vis[cur], n_t}, b.words,
                                                               w.prefix, w.scan_tmp, s)));
                hipLaunchKernelGGL(k_compact_unvisited, dim3(grid_for(b.words, COMPACT_BLOCK, 16384)),
                                   dim3(COMPACT_BLOCK), 0, s, vis[cur], n_t, b.words, w.prefix,
                                   w.ulist);
                GT_HIP(hipGetLastError());
                nlist = unvisited;
            }
            const BuHints hh = bu_hints(b, tu, nf, n_t);
            kind = nlist >= 0 ? GT_KERNEL_BU_LIST : GT_KERNEL_BU_WORDS;
            if (simple) {
                // a thread per bitmap word (2) or per vertex (3)
                const int64_t units = tu.bu_form == 2 ? (b.words + GT_WAVE - 1) / GT_WAVE : b.words;
                const BuLaunch bl = bu_launch(g, units, false, false);
                if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 1], s));
                if (tu.bu_form == 2)
                    hipLaunchKernelGGL((k_bu_simple<SPLIT, true>), dim3(bl.blocks), dim3(bl.threads), bl.lds_bytes, s,
                                       off, col, n_t, b.words, vis[cur], vis[cur ^ 1], lvl, par, L + 1, c_now,
                                       c_next, hh.hint, hh.hint_orig, n2o, bl.lds_words);
                else
                    hipLaunchKernelGGL((k_bu_simple<SPLIT, false>), dim3(bl.blocks), dim3(bl.threads), bl.lds_bytes,
                                       s, off, col, n_t, b.words, vis[cur], vis[cur ^ 1], lvl, par, L + 1, c_now,
                                       c_next, hh.hint, hh.hint_orig, n2o, bl.lds_words);
            } else if (nlist >= 0) {
                hipLaunchKernelGGL(k_copy_words, dim3(grid_for(b.words, 256, 8192)), dim3(256), 0, s, vis[cur],
                                   vis[cur ^ 1], b.words);
                const BuLaunch bl = bu_launch(g, (nlist + GT_WAVE * BU_WPI - 1) / (GT_WAVE * BU_WPI), true, hh.hint2 != nullptr);
                if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 1], s));
                if (hh.hint2)
                    hipLaunchKernelGGL((k_bu_list<SPLIT, true>), dim3(bl.blocks), dim3(bl.threads), bl.lds_bytes, s,
                                       off, col, n_t, (const int32_t*)w.ulist, nlist, vis[cur], vis[cur ^ 1], lvl,
                                       par, L + 1, w.hub_q, c_now, c_next, tu.bu_lane_edges,
                                       (int64_t)tu.bu_hub_deg, hh, n2o, bl.lds_words);
                else
                    hipLaunchKernelGGL((k_bu_list<SPLIT, false>), dim3(bl.blocks), dim3(bl.threads), bl.lds_bytes, s,
                                       off, col, n_t, (const int32_t*)w.ulist, nlist, vis[cur], vis[cur ^ 1], lvl,
                                       par, L + 1, w.hub_q, c_now, c_next, tu.bu_lane_edges,
                                       (int64_t)tu.bu_hub_deg, hh, n2o, bl.lds_words);
            } else {
                const BuLaunch bl = bu_launch(g, (b.words + BU_WPI - 1) / BU_WPI, false, hh.hint2 != nullptr);
                if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 1], s));
                if (hh.hint2)
                    hipLaunchKernelGGL((k_bu<SPLIT, true>), dim3(bl.blocks), dim3(bl.threads), bl.lds_bytes, s, off,
                                       col, n_t, b.words, vis[cur], vis[cur ^ 1], lvl, par, L + 1, w.hub_q, c_now,
                                       c_next, tu.bu_lane_edges, (int64_t)tu.bu_hub_deg, hh, n2o, bl.lds_words);
                else
                    hipLaunchKernelGGL((k_bu<SPLIT, false>), dim3(bl.blocks), dim3(bl.threads), bl.lds_bytes, s, off,
                                       col, n_t, b.words, vis[cur], vis[cur ^ 1], lvl, par, L + 1, w.hub_q, c_now,
                                       c_next, tu.bu_lane_edges, (int64_t)tu.bu_hub_deg, hh, n2o, bl.lds_words);
            }
            GT_HIP(hipGetLastError());
            if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 2], s));
            if (!simple)
                hipLaunchKernelGGL((k_bu_hubs<SPLIT>), dim3(tu.bu_hub_blocks), dim3(HUB_BLOCK), 0, s, off, col, n2o,
                                   vis[cur], vis[cur ^ 1], lvl, par, L + 1, w.hub_q, c_now,
                                   tu.bu_lane_edges);
            GT_HIP(hipGetLastError());
            cur ^= 1;
        }
        if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 4 * lev + 3], s));
        GT_HIP(hipMemcpyAsync(h, c_now, sizeof(unsigned long long) * CTR_SET, hipMemcpyDeviceToHost, s));
        GT_HIP(hipStreamSynchronize(s));
        unsigned long long tot[CTR_N] = {};
        for (int sl = 0; sl < CTR_SLOTS; ++sl)
            for (int c = 0; c < CTR_N; ++c) tot[c] += h[sl * CTR_STRIDE + c];
        const int64_t found = (int64_t)tot[CTR_FOUND];
        const int64_t fdeg = (int64_t)tot[CTR_FOUND_DEG];
        if (lev < GT_MAX_LEVELS) {
            gt_level_stats& ls = st.level[lev];
            ls.dir = dir;
            ls.kernel = kind;
            ls.frontier = nf;
            ls.scanned = dir == GT_DIR_TOP_DOWN ? nf : (int64_t)tot[CTR_SCANNED];
            ls.examined = (int64_t)tot[CTR_EXAMINED];
            ls.examined_long = (int64_t)tot[CTR_EXAMINED_LONG];
            ls.found_long = (int64_t)tot[CTR_FOUND_LONG];
            ls.found = found;
            ls.ms = 0.f;
            ls.ms_main = 0.f;
        }
        mu -= fdeg;
        if (dir == GT_DIR_TOP_DOWN) {
            const int64_t unvisited = n_t - visited - found;
            if (fdeg > mu / tu.alpha || fdeg > (int64_t)tu.bu_gamma * unvisited) dir = GT_DIR_BOTTOM_UP;
        } else {
            if (found < nf && found <= n_t / tu.beta) dir = GT_DIR_TOP_DOWN;
        }
        if (appended) {
            qi ^= 1;
        } else {
            need_queue = true;
        }
        nf = found;
        mf = fdeg;
        visited += found;
        ++L;
        ++lev;
    }
    st.n_levels = lev;

    if (split) {
        if (timing) GT_HIP(hipEventRecord(ev[EV_OUT0], s));
        if (g->n_anchor > 0)  // level bytes are only read for leaves
            hipLaunchKernelGGL(k_anchor_bytes, dim3(grid_for(g->n_anchor, 256, 16384)), dim3(256), 0, s,
                               g->n_anchor, (const int32_t*)g->anchor_core.as<int32_t>(), (const uint64_t*)vis[cur],
                               reinterpret_cast<const int2*>(w.level), w.lv8);
        hipLaunchKernelGGL(k_split_output, dim3(grid_for((g->n + OUT_ITEMS - 1) / OUT_ITEMS, OUT_BLOCK, 1 << 20)),
                           dim3(OUT_BLOCK), 0, s, g->n, g->groups.as<ClassGroup>(), (const uint64_t*)vis[cur],
                           (const uint8_t*)w.lv8, reinterpret_cast<const int2*>(w.level),
                           (const int32_t*)g->anchor_core.as<int32_t>(), (const int32_t*)g->leaf_anchor.as<int32_t>(),
                           g->leaf_src_old.as<int32_t>(), (const int32_t*)g->tdepth.as<int32_t>(), root, partner,
                           parent_out, level_out);
        GT_HIP(hipGetLastError());
        GT_TRY(apply_tree_fix(g, rp, parent_out, level_out, s));
        if (timing) GT_HIP(hipEventRecord(ev[EV_OUT1], s));
    }
    GT_HIP(hipStreamSynchronize(s));
    if (timing) {
        st.ms_init = ev_ms(ev[EV_INIT0], ev[EV_INIT1]);
        for (int l = 0; l < lev && l < GT_MAX_LEVELS; ++l) {
            st.level[l].ms = ev_ms(ev[EV_LVL + 4 * l], ev[EV_LVL + 4 * l + 3]);
            st.level[l].ms_main = ev_ms(ev[EV_LVL + 4 * l + 1], ev[EV_LVL + 4 * l + 2]);
        }
        if (split) {
            st.ms_output = ev_ms(ev[EV_OUT0], ev[EV_OUT1]);
            st.ms_total = ev_ms(ev[EV_INIT0], ev[EV_OUT1]);
        } else {
            st.ms_total = lev > 0 ? ev_ms(ev[EV_INIT0], ev[EV_LVL + 4 * (std::min(lev, GT_MAX_LEVELS) - 1) + 3])
                                  : st.ms_init;
        }
    }
    return GT_OK;
}

extern "C" gt_status gt_bfs(gt_graph* g, int32_t root, int32_t* parent_out, int32_t* level_out,
                            void* stream) {
    if (!g || !parent_out || !level_out) return gt_fail(GT_E_INVALID, "NULL argument");
    if (root < 0 || (int64_t)root >= g->n) return gt_fail(GT_E_INVALID, "root out of range");
    std::lock_guard<std::mutex> lk(g->mu);
    if (g->tune.loop == GT_LOOP_GRAPH || g->tune.loop == GT_LOOP_DEVICE) {
        const RootPlan rp = gt_plan_root(g, root);
        GT_TRY(gt_bfs_graph(g, root, rp, parent_out, level_out, (hipStream_t)stream));
        if (rp.fix_v.empty()) return GT_OK;
        GT_TRY(apply_tree_fix(g, rp, parent_out, level_out, (hipStream_t)stream));
        GT_HIP(hipStreamSynchronize((hipStream_t)stream));
        return GT_OK;
    }
    const BfsWork w = work_of(g);
    if (g->flags & GT_BUILD_SPLIT) return bfs_run<true>(g, root, parent_out, level_out, (hipStream_t)stream, w);
    return bfs_run<false>(g, root, parent_out, level_out, (hipStream_t)stream, w);
}

// ------------------------------------------------- static working memory --
// gt_bfs_static takes the traversal's working memory from this array instead
// of the handle's buffers. The code object carries it, so each GPU the
// library is loaded on holds one copy until the process ends; the library
// never allocates or frees it. In host code `scratch` names a host-side
// stand-in: kernels are given the device address that hipGetSymbolAddress
// returns for the current device, kept per device in s_scratch_dev.
static __device__ __align__(256) unsigned char scratch[GT_BFS_STATIC_MAX_BYTES];

namespace {
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex s_scratch_mu;                                   // guards s_scratch_dev
unsigned char* s_scratch_dev[STATIC_MAX_DEVICES] = {};     // device address per device
std::mutex s_static_call_mu[STATIC_MAX_DEVICES];           // one gt_bfs_static at a time per device

// Pieces of the working memory of a host-driven traversal of n vertices and
// tE adjacency entries, carved in order at 256-byte boundaries from base
// (nullptr: sizes only). Returns the bytes used.
size_t static_layout(int64_t n, int64_t tE, int64_t n_anchor, bool split, unsigned char* base, BfsWork* w) {
    size_t at = 0;
    auto take = [&](size_t bytes) -> unsigned char* {
        unsigned char* p = base ? base + at : nullptr;
        at += (bytes + 255) & ~(size_t)255;
        return p;
    };
    const int64_t words = (n + 63) / 64;
    const int64_t n1 = n > 0 ? n : 1;
    BfsWork x{};
    x.vis[0] = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * (size_t)(words > 0 ? words : 1)));
    x.vis[1] = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * (size_t)(words > 0 ? words : 1)));
    x.q[0] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n1));
    x.q[1] = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n1));
    x.prefix = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (size_t)(n + 1)));
    x.scan_tmp = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (size_t)scan_scratch_elems(n + 1)));
    x.hub_q = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n1));
    x.ulist = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n1));
    x.td_row_cap = tE / TD_CHUNK + 64;
    x.td_rows = reinterpret_cast<int2*>(take(sizeof(int2) * (size_t)x.td_row_cap));
    x.level = nullptr;
    x.lv8 = nullptr;
    if (split) {
        x.level = reinterpret_cast<int32_t*>(take(sizeof(int2) * (size_t)(4 * ((n + 3) / 4) + 4)));
        x.lv8 = take((size_t)(n_anchor > 0 ? n_anchor : 1));
    }
    x.ctr = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * 2 * CTR_SET));
    x.h_ctr = nullptr;
    x.ev = nullptr;
    if (w) *w = x;
    return at;
}

// Device address of `scratch` on the current device, looked up once per device.
gt_status static_scratch(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lk(s_scratch_mu);
    if (!s_scratch_dev[dev]) {
        void* p = nullptr;
        GT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return gt_fail(GT_E_HIP, "hipGetSymbolAddress returned no address for the static scratch array");
        s_scratch_dev[dev] = static_cast<unsigned char*>(p);
    }
    *out = s_scratch_dev[dev];
    return GT_OK;
}
}  // namespace

extern "C" gt_status gt_bfs_static(gt_graph* g, int32_t root, int32_t* parent_out, int32_t* level_out,
                                   void* stream) {
    if (!g || !parent_out || !level_out) return gt_fail(GT_E_INVALID, "NULL argument");
    if (root < 0 || (int64_t)root >= g->n) return gt_fail(GT_E_INVALID, "root out of range");
    if (g->mh > 0)
        return gt_fail(GT_E_UNSUPPORTED, "gt_bfs_static serves PLAIN and SPLIT (MH = 0) handles, not edge trees");
    const bool split = (g->flags & GT_BUILD_SPLIT) != 0;
    const size_t need = static_layout(g->tn(), g->tE(), g->n_anchor, split, nullptr, nullptr);
    if (need > (size_t)GT_BFS_STATIC_MAX_BYTES)
        return gt_fail(GT_E_INVALID, "gt_bfs_static: this graph needs " + std::to_string(need) +
                                         " bytes of working memory; the static array holds " +
                                         std::to_string((size_t)GT_BFS_STATIC_MAX_BYTES) + " (use gt_bfs)");
    int dev = 0;
    GT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return gt_fail(GT_E_UNSUPPORTED, "device number too large");
    unsigned char* base = nullptr;
    GT_TRY(static_scratch(dev, &base));
    std::lock_guard<std::mutex> dl(s_static_call_mu[dev]);
    std::lock_guard<std::mutex> lk(g->mu);
    BfsWork w;
    (void)static_layout(g->tn(), g->tE(), g->n_anchor, split, base, &w);
    w.h_ctr = g->bfs.h_ctr.as<unsigned long long>();
    w.ev = g->tune.timing ? g->bfs.ev.data() : nullptr;
    if (split) return bfs_run<true>(g, root, parent_out, level_out, (hipStream_t)stream, w);
    return bfs_run<false>(g, root, parent_out, level_out, (hipStream_t)stream, w);
}

extern "C" gt_status gt_last_run_stats(const gt_graph* g, gt_run_stats* out) {
    if (!g || !out) return gt_fail(GT_E_INVALID, "NULL argument");
    *out = g->stats;
    return GT_OK;
}
