// Batched multi-source BFS: up to 64 traversals share one level loop, one
// bit per traversal ("slot") in a 64-bit mask per vertex of the traversed
// graph (the core for SPLIT handles). Per vertex: seen mask, frontier mask
// (double-buffered) and a 64-byte row of per-slot levels (uint8, vertex
// major). The leaf pass of Algorithm 7 and the translation to caller ids
// happen in one tiled transpose into the root-major [k][N] output.
//
// Also here: parent reconstruction from a level array, and continuous-
// batching sessions (slots admitted and retired between steps).
#include <algorithm>
#include <atomic>
#include <climits>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "gt_internal.h"

namespace {

constexpr int MS_BLOCK = 256;
constexpr int EX_TILE = 256;   // caller ids per extraction block (4 per lane)
constexpr int EX_BLOCK = 256;  // 4 waves, one per quarter of 16 slots


// Per-slot level offset: a bit first seen at step t gets level t + 1 + off.
struct SlotOffsets {
    int32_t off[64];
};

enum { MS_FOUND_V = 0, MS_FOUND_PAIRS, MS_FOUND_DEG, MS_EXAMINED };

__device__ __forceinline__ void ms_clear_set(unsigned long long* set) {
    for (int i = threadIdx.x; i < CTR_SET; i += blockDim.x) set[i] = 0;
}

// OR-reduction of a mask over the wave, folded into a shared word.
__device__ __forceinline__ void wave_or(unsigned long long* word, uint64_t m) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m |= __shfl_xor(m, o, GT_WAVE);
    if (lane_id() == 0 && m) atomicOr(word, (unsigned long long)m);
}

// 8-bit mask -> 64-bit mask with byte i = 0xFF where bit i is set.
__device__ __forceinline__ uint64_t byte_mask(uint32_t b) {
    uint64_t x = b & 0xFFu;
    x = (x | (x << 28)) & 0x0000000F0000000Full;
    x = (x | (x << 14)) & 0x0003000300030003ull;
    x = (x | (x << 7)) & 0x0101010101010101ull;
    return x * 0xFFull;
}

// Level bytes of the slots first seen this step (nx), 16 slots per 16-byte
// store: the bytes of slots seen before (s) are kept, every other byte takes
// the step's level row L (a slot's level byte is only read under its seen
// bit, so bytes of unseen slots are free).
__device__ __forceinline__ void write_levels(uint8_t* __restrict__ lv, int64_t v, uint64_t nx, uint64_t s,
                                             const uint64_t* L) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (((nx >> (16 * q)) & 0xFFFFull) == 0) continue;
        uint4* p = reinterpret_cast<uint4*>(lv + v * 64 + 16 * q);
        uint64_t w0 = L[2 * q], w1 = L[2 * q + 1];
        const uint32_t sb = (uint32_t)(s >> (16 * q)) & 0xFFFFu;
        if (sb) {
            const uint4 o = *p;
            const uint64_t k0 = byte_mask(sb), k1 = byte_mask(sb >> 8);
            w0 = (((uint64_t)o.y << 32 | o.x) & k0) | (w0 & ~k0);
            w1 = (((uint64_t)o.w << 32 | o.z) & k1) | (w1 & ~k1);
        }
        *p = make_uint4((uint32_t)w0, (uint32_t)(w0 >> 32), (uint32_t)w1, (uint32_t)(w1 >> 32));
    }
}

// 64x64 bit transpose over the wave: lane i returns the word whose bit c is
// bit i of lane c's x (six butterfly stages of half-block swaps).
__device__ __forceinline__ uint64_t wave_transpose(uint64_t x, int lane) {
    constexpr uint64_t M[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int sh = 32 >> k;
        const uint64_t y = __shfl_xor(x, sh, GT_WAVE);
        x = (lane & sh) ? ((x & ~M[k]) | ((y & ~M[k]) >> sh)) : ((x & M[k]) | ((y & M[k]) << sh));
    }
    return x;
}

__global__ void k_ms_zero(uint64_t* __restrict__ a, uint64_t* __restrict__ b, uint64_t* __restrict__ c,
                          int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (a) a[i] = 0;
        if (b) b[i] = 0;
        if (c) c[i] = 0;
    }
}

// Seeds: slot r starts at vertex seed[r] (traversed-graph id) with level
// off[r] (0, or 1 for a leaf root whose neighbour seeds the core traversal).
__global__ void k_ms_seed(int k, const int32_t* __restrict__ seed, SlotOffsets so,
                          uint64_t* __restrict__ seen, uint64_t* __restrict__ fr,
                          uint8_t* __restrict__ lv) {
    const int r = threadIdx.x;
    if (r < k && seed[r] >= 0) {
        const int64_t s = seed[r];
        atomicOr((unsigned long long*)&seen[s], 1ull << r);
        atomicOr((unsigned long long*)&fr[s], 1ull << r);
        lv[s * 64 + r] = (uint8_t)so.off[r];
    }
}

// Seeds of a session step: bits of newly admitted slots join the current
// frontier (the others keep theirs).
__global__ void k_ms_admit(int nadm, const int32_t* __restrict__ seed, const int32_t* __restrict__ slot,
                           const int32_t* __restrict__ lvl0, uint64_t* __restrict__ seen,
                           uint64_t* __restrict__ fr, uint8_t* __restrict__ lv) {
    const int i = threadIdx.x;
    if (i < nadm && seed[i] >= 0) {
        const int64_t s = seed[i];
        const int r = slot[i];
        atomicOr((unsigned long long*)&seen[s], 1ull << r);
        atomicOr((unsigned long long*)&fr[s], 1ull << r);
        lv[s * 64 + r] = (uint8_t)lvl0[i];
    }
}

// Clear retired slots' bits everywhere (sessions).
__global__ void k_ms_retire(uint64_t keep, uint64_t* __restrict__ seen, uint64_t* __restrict__ fr0,
                            uint64_t* __restrict__ fr1, uint64_t* __restrict__ fr2, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        seen[i] &= keep;
        fr0[i] &= keep;
        fr1[i] &= keep;
        fr2[i] &= keep;
    }
}

// Queue of the vertices whose frontier mask has a bit of `mask`. A block
// takes MQ_CHUNK consecutive vertices (MQ_PER_THREAD per thread, coalesced
// loads), counts its hits, reserves room with one atomic and writes them.
// The order is arbitrary: the push only ORs.
constexpr int MQ_PER_THREAD = 32;
constexpr int MQ_CHUNK = 256 * MQ_PER_THREAD;

__global__ void __launch_bounds__(256) k_ms_queue(const uint64_t* __restrict__ a, uint64_t mask, int64_t n,
                                                  int32_t* __restrict__ q, unsigned long long* __restrict__ tail) {
    __shared__ int s_cnt[4];
    __shared__ unsigned long long s_base;
    const int t = threadIdx.x, lane = lane_id(), wv = t >> 6;
    for (int64_t c0 = (int64_t)blockIdx.x * MQ_CHUNK; c0 < n; c0 += (int64_t)gridDim.x * MQ_CHUNK) {
        uint32_t fl = 0;
#pragma unroll
        for (int j = 0; j < MQ_PER_THREAD; ++j) {
            const int64_t v = c0 + j * 256 + t;
            if (v < n && (a[v] & mask) != 0) fl |= 1u << j;
        }
        const int cnt = __popc(fl);
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < GT_WAVE; o <<= 1) {
            const int y = __shfl_up(incl, o, GT_WAVE);
            if (lane >= o) incl += y;
        }
        if (lane == GT_WAVE - 1) s_cnt[wv] = incl;
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int x = s_cnt[w];
            if (w < wv) before += x;
            total += x;
        }
        if (t == 0) s_base = total ? atomicAdd(tail, (unsigned long long)total) : 0ull;
        __syncthreads();
        int64_t pos = (int64_t)s_base + before + incl - cnt;
        while (fl) {
            const int j = __ffs(fl) - 1;
            fl &= fl - 1;
            q[pos++] = (int32_t)(c0 + j * 256 + t);
        }
        __syncthreads();  // s_cnt and s_base are reused by the next chunk
    }
}

struct LoadQDeg {
    const int32_t* q;
    const int64_t* off;
    __device__ __forceinline__ int64_t operator()(int64_t i) const {
        const int32_t u = q[i];
        return off[u + 1] - off[u];
    }
};

__device__ __forceinline__ int64_t ms_first_greater(const int64_t* __restrict__ p, int64_t a, int64_t b,
                                                    int64_t x) {
    while (a < b) {
        const int64_t mid = a + ((b - a) >> 1);
        if (p[mid] > x) b = mid;
        else a = mid + 1;
    }
    return a;
}

// Push (top-down) part of a step, for the slots in `tmask`: every adjacency
// entry of a frontier vertex ORs the vertex's frontier bits (minus bits the
// neighbour has seen) into the neighbour's next mask. Edge-balanced like the
// single-source top-down.
template <bool SPLIT>
__global__ void __launch_bounds__(MS_BLOCK) k_ms_push(
    const int32_t* __restrict__ q, int64_t nf, const int64_t* __restrict__ prefix,
    const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const uint64_t* __restrict__ fr_cur, uint64_t* fr_nxt, const uint64_t* seen, uint64_t tmask) {
    __shared__ int64_t s_lo, s_hi;
    const int64_t X = prefix[nf];
    for (int64_t e0 = (int64_t)blockIdx.x * MS_BLOCK; e0 < X; e0 += (int64_t)gridDim.x * MS_BLOCK) {
        const int64_t e = e0 + threadIdx.x;
        if (threadIdx.x == 0) s_lo = ms_first_greater(prefix, 1, nf, e0) - 1;
        if (threadIdx.x == 1) {
            const int64_t elast = (e0 + MS_BLOCK < X ? e0 + MS_BLOCK : X) - 1;
            s_hi = ms_first_greater(prefix, 1, nf, elast) - 1;
        }
        __syncthreads();
        const int64_t lo = s_lo, hi = s_hi;
        __syncthreads();
        if (e < X) {
            const int64_t i = ms_first_greater(prefix, lo + 1, hi + 1, e) - 1;
            const int32_t u = q[i];
            const int32_t w = col[off[u] + (e - prefix[i])];
            const uint64_t m = fr_cur[u] & tmask & ~seen[w];
            if (m && (fr_nxt[w] & m) != m) atomicOr((unsigned long long*)&fr_nxt[w], (unsigned long long)m);
        }
    }
}

constexpr int MS_WINDOW = 4 * GT_WAVE;  // flat-list entries per wave and round trip

// End of a step (the finalize part): keep only unseen bits as the next
// frontier, mark them seen, record their levels, clear the vertex in the
// buffer that held the frontier before the current one (read by no kernel of
// this step; it becomes the next step's all-zero output buffer), and count per
// slot the new frontier's vertices and degree sum (lane r of each wave
// accumulates slot r; one atomic per slot and wave into one of SC_COPIES
// copies).
constexpr int SC_COPIES = 16;
constexpr int SC_SET = SC_COPIES * 128;  // uint64 per per-slot counter set

struct FinCounts {
    unsigned long long fv = 0, fp = 0, fd = 0, nf = 0, mf = 0;
    uint64_t any = 0;
};

// Level byte of each slot for a vertex first seen at this step (byte r % 8
// of L[r / 8]), in LDS: written by the block's first 8 threads at the start
// of the kernel (every thread calls this), read only where a level is
// written, so that it holds no registers across the pull.
__device__ __forceinline__ void step_levels(int step, const int32_t* so_off, uint64_t* L) {
    if (threadIdx.x < 8) {
        const int j = threadIdx.x;
        uint64_t x = 0;
        for (int i = 0; i < 8; ++i) x |= (uint64_t)((step + 1 + so_off[8 * j + i]) & 0xFF) << (8 * i);
        L[j] = x;
    }
    __syncthreads();
}

// Lane's vertex v (>= n: none) of the wave's 64 consecutive vertices; s: its
// seen mask at the start of the step; nb: the bits it got this step (seen
// ones included). Called by every lane of the wave.
__device__ __forceinline__ void finalize_vertex(int64_t n, int64_t v, int lane, uint64_t s, uint64_t nb,
                                                const int64_t* __restrict__ off, uint64_t* __restrict__ seen,
                                                uint64_t* __restrict__ fr_nxt, uint64_t* __restrict__ fr_old,
                                                uint8_t* __restrict__ lv, const uint64_t* L, FinCounts& fc) {
    uint64_t nx = 0;
    uint32_t d = 0;
    if (v < n) {
        nx = nb & ~s;
        if (nb) fr_nxt[v] = nx;  // a zero nb means the entry is zero already
        fr_old[v] = 0;
        if (nx) {
            seen[v] = s | nx;
            write_levels(lv, v, nx, s, L);
            d = (uint32_t)(off[v + 1] - off[v]);
            fc.fv += 1;
            fc.fp += (unsigned long long)__popcll(nx);
            fc.fd += d;
        }
    }
    if (__ballot(nx != 0) == 0) return;
    // per-slot counts: after the transpose, bit j of t says that slot `lane`
    // found the wave's vertex j; the degree sum goes bit plane by bit plane
    // of d (a ballot per plane)
    const uint64_t t = wave_transpose(nx, lane);
    fc.any |= t != 0 ? (1ull << lane) : 0ull;
    fc.nf += (unsigned long long)__popcll(t);
    uint32_t dd = d;
    for (int b = 0; __ballot(dd != 0) != 0; ++b, dd >>= 1)
        fc.mf += (unsigned long long)__popcll(t & __ballot(dd & 1u)) << b;
}

__device__ __forceinline__ void finalize_flush(const FinCounts& fc, int lane, unsigned long long* __restrict__ ctr,
                                               unsigned long long* __restrict__ sctr) {
    unsigned long long* cs = ctr_slot(ctr);
    wave_add(&cs[MS_FOUND_V], fc.fv);
    wave_add(&cs[MS_FOUND_PAIRS], fc.fp);
    wave_add(&cs[MS_FOUND_DEG], fc.fd);
    wave_or(&ctr[CTR_SHARED + 2], fc.any);
    unsigned long long* sc = sctr + (blockIdx.x % SC_COPIES) * 128;
    if (fc.nf) atomicAdd(&sc[lane], fc.nf);
    if (fc.mf) atomicAdd(&sc[64 + lane], fc.mf);
}

// Counter sets of the next step are cleared by block 0 of the step's last kernel.
__device__ __forceinline__ void clear_next_sets(unsigned long long* __restrict__ ctr_clear,
                                                unsigned long long* __restrict__ sctr_clear) {
    if (blockIdx.x == 0) {
        ms_clear_set(ctr_clear);
        for (int i = threadIdx.x; i < SC_SET; i += blockDim.x) sctr_clear[i] = 0;
    }
}

// Finalize arguments of k_ms_pull and k_ms_finalize.
struct FinArgs {
    uint64_t* fr_old;
    uint8_t* lv;
    int step;
    bool push_bits;  // fr_nxt may hold bits from this step's push
    unsigned long long* ctr_clear;
    unsigned long long* sctr;
    unsigned long long* sctr_clear;
};

// Pull (bottom-up) part of a step, for the slots in `bmask`: a vertex still
// missing some of them ORs its neighbours' frontier masks -- highest-degree
// neighbour first, then the first lane_edges entries (4 loads per round
// trip), then the rest of all still-open rows of the wave as one flat list
// (MS_WINDOW entries per round trip, a segmented OR-scan per round) -- and
// stops once every missing slot is covered. The step's finalize runs in the
// same pass, on each vertex's own entries only (the pull reads the current
// frontier, which nothing here writes), with the bits of the step's push
// read from the next mask.
template <bool SPLIT>
__device__ __forceinline__ void ms_pull_body(
    int64_t n, const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int32_t* __restrict__ hint, uint64_t bmask, uint64_t* __restrict__ seen,
    const uint64_t* __restrict__ fr_cur, uint64_t* __restrict__ fr_nxt, int lane_edges,
    unsigned long long* __restrict__ ctr, const FinArgs& fa, const int32_t* so_off) {
    using T = int32_t;
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    clear_next_sets(fa.ctr_clear, fa.sctr_clear);
    __shared__ uint64_t L[8];
    step_levels(fa.step, so_off, L);
    FinCounts fc;
    unsigned long long ex = 0;
    for (int64_t base = gw * GT_WAVE; base < n; base += nwaves * GT_WAVE) {
        const int64_t v = base + lane;
        const uint64_t sv = v < n ? seen[v] : ~0ull;
        const uint64_t miss = bmask & ~sv;
        uint64_t acc = 0;
        if (__ballot(miss != 0) != 0) {
        int64_t b = 0, e = 0;
        if (miss) {
            const T h = hint[v];
            b = off[v];
            e = off[v + 1];
            if (h >= 0) {
                acc = fr_cur[h] & miss;
                ex += 1;
            }
        }
        int64_t rb = b;
        bool open = miss && acc != miss && e > b;
        if (open) {
            const int64_t lim = (e - b > lane_edges) ? b + lane_edges : e;
            int64_t k = b;
            for (; k < lim && acc != miss; k += 4) {
                T u[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) u[i] = (k + i < lim) ? col[k + i] : 0;
                uint64_t f = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (k + i < lim) f |= fr_cur[u[i]];
                acc |= f & miss;
                ex += (unsigned long long)((lim - k) < 4 ? (lim - k) : 4);
            }
            rb = k < lim ? k : lim;
            open = acc != miss && rb < e;
        }
        while (__ballot(open)) {
            const int32_t len = open ? (int32_t)(e - rb) : 0;
            int32_t incl = len;
#pragma unroll
            for (int o = 1; o < GT_WAVE; o <<= 1) {
                const int32_t y = __shfl_up(incl, o, GT_WAVE);
                if (lane >= o) incl += y;
            }
            const int32_t excl = incl - len;
            const int32_t total = __shfl(incl, GT_WAVE - 1, GT_WAVE);
            const int32_t W = total < MS_WINDOW ? total : MS_WINDOW;
            uint64_t f[4];
            int own[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t x = i * GT_WAVE + lane;
                int lo = 0, hi = GT_WAVE - 1;
#pragma unroll
                for (int st = 0; st < 6; ++st) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (__shfl(excl, mid, GT_WAVE) <= x) lo = mid;
                    else hi = mid - 1;
                }
                const int64_t k = __shfl(rb, lo, GT_WAVE) + (x - __shfl(excl, lo, GT_WAVE));
                own[i] = x < W ? lo : GT_WAVE;
                f[i] = x < W ? fr_cur[col[k]] : 0ull;
            }
            // segmented inclusive OR-scan: owners are non-decreasing over lanes
#pragma unroll
            for (int i = 0; i < 4; ++i) {
#pragma unroll
                for (int d = 1; d < GT_WAVE; d <<= 1) {
                    const uint64_t y = __shfl_up(f[i], d, GT_WAVE);
                    const int yo = __shfl_up(own[i], d, GT_WAVE);
                    if (lane >= d && yo == own[i]) f[i] |= y;
                }
            }
            const bool has = open && excl < W;
            const int32_t z = incl < W ? incl : W;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t lo = excl - i * GT_WAVE, hi = z - i * GT_WAVE;
                const bool mine = has && hi > 0 && lo < GT_WAVE;
                const int src = mine ? ((hi < GT_WAVE ? hi : GT_WAVE) - 1) : lane;
                const uint64_t val = __shfl(f[i], src, GT_WAVE);
                if (mine) acc |= val & miss;
            }
            if (has) {
                ex += (unsigned long long)(z - excl);
                rb += z - excl;
                open = acc != miss && rb < e;
            }
        }
        }
        const uint64_t pb = (fa.push_bits && v < n) ? fr_nxt[v] : 0ull;
        finalize_vertex(n, v, lane, sv, pb | acc, off, seen, fr_nxt, fa.fr_old, fa.lv, L, fc);
    }
    wave_add(&ctr_slot(ctr)[MS_EXAMINED], ex);
    finalize_flush(fc, lane, ctr, fa.sctr);
}

template <bool SPLIT>
__global__ void __launch_bounds__(MS_BLOCK) k_ms_pull(
    int64_t n, const int64_t* __restrict__ off, const int32_t* __restrict__ col,
    const int32_t* __restrict__ hint, uint64_t bmask, uint64_t* __restrict__ seen,
    const uint64_t* __restrict__ fr_cur, uint64_t* __restrict__ fr_nxt, int lane_edges,
    unsigned long long* __restrict__ ctr, FinArgs fa, SlotOffsets so) {
    ms_pull_body<SPLIT>(n, off, col, hint, bmask, seen, fr_cur, fr_nxt, lane_edges, ctr, fa, so.off);
}

// Finalize alone, after a step without pulled slots.
__device__ __forceinline__ void ms_finalize_body(int64_t n, const int64_t* __restrict__ off,
                                                 uint64_t* __restrict__ seen, uint64_t* __restrict__ fr_nxt,
                                                 unsigned long long* __restrict__ ctr, const FinArgs& fa,
                                                 const int32_t* so_off) {
    clear_next_sets(fa.ctr_clear, fa.sctr_clear);
    const int lane = lane_id();
    __shared__ uint64_t L[8];
    step_levels(fa.step, so_off, L);
    FinCounts fc;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t base = start - lane; base < n; base += stride) {
        const int64_t v = base + lane;
        const uint64_t sv = v < n ? seen[v] : 0ull;
        const uint64_t nb = v < n ? fr_nxt[v] : 0ull;
        finalize_vertex(n, v, lane, sv, nb, off, seen, fr_nxt, fa.fr_old, fa.lv, L, fc);
    }
    finalize_flush(fc, lane, ctr, fa.sctr);
}

__global__ void __launch_bounds__(MS_BLOCK) k_ms_finalize(int64_t n, const int64_t* __restrict__ off,
                                                          uint64_t* __restrict__ seen, uint64_t* __restrict__ fr_nxt,
                                                          unsigned long long* __restrict__ ctr, FinArgs fa,
                                                          SlotOffsets so) {
    ms_finalize_body(n, off, seen, fr_nxt, ctr, fa, so.off);
}

// ------------------------------------------- device-driven batched loop --
// The same steps with every per-step parameter read from a device control
// block (MsCtl) instead of kernel arguments, so that a fixed sequence of
// steps is captured once in a HIP graph and replayed per batch:
//  - the push needs no queue and no prefix sum: a wave takes 64 consecutive
//    vertices, the rows of those in a top-down slot's frontier are read as
//    one flat list, rows longer than MS_PUSH_LONG are cut into
//    MS_PUSH_CHUNK-entry chunks that a second kernel spreads over the grid;
//  - pull and finalize are launched both and run only when their step needs
//    them (some slot pulls / none does);
//  - one wave (k_msg_ctl, lane = slot) sums the step's counters, applies each
//    slot's direction rule, rotates the frontier buffers and records the
//    step's counters in GPU-mapped host memory.
constexpr int MS_PUSH_CHUNK = 4 * GT_WAVE;
constexpr int64_t MS_PUSH_LONG = 256;  // >= MS_PUSH_CHUNK: long rows number at most E / MS_PUSH_CHUNK
constexpr int CTR_PUSHROWS = CTR_SHARED + 3;  // push long rows << 32 | their chunks

struct MsCtl {
    uint64_t active;      // slots whose frontier is not empty
    uint64_t td;          // slots in top-down (push) mode
    int32_t cur;          // frontier buffer read by the step
    int32_t step;         // steps done
    int32_t done;         // no slot active, or a level would not fit in a byte
    int32_t depth_err;
    int32_t max_extra;    // largest seed level offset + tree depth added at extraction
    int32_t pad;
    int64_t mu[64];       // unexplored edges per slot
    int64_t nf_prev[64];  // frontier size per slot at the previous step
    int32_t off[64];      // per-slot level offsets
};

// Per-call start of the control block (a kernel argument: not captured).
struct MsStart {
    uint64_t active;
    int32_t max_extra;
    int32_t pad;
    int64_t mu0;
    int32_t off[64];
};

// GPU-mapped host block: the end flag and each step's counters.
struct MsHost {
    int32_t done, depth_err, steps, pad;
    gt_level_stats level[GT_MAX_LEVELS];
};

// Arrays of the device-driven loop (fixed per handle and batch state).
struct MsGArgs {
    int64_t n;
    const int64_t* off;
    const int32_t* col;
    const int32_t* hint;
    uint64_t* seen;
    uint64_t* fr[3];
    uint8_t* lv;
    unsigned long long* ctr;   // two counter sets
    unsigned long long* sctr;  // two per-slot counter sets
    int2* rows;                // push long rows: (vertex, first chunk)
    int64_t row_cap;
    int lane_edges;
};

struct MsStep {
    const uint64_t* fr_cur;
    uint64_t* fr_nxt;
    unsigned long long* c_now;
    FinArgs fa;
};

__device__ __forceinline__ MsStep ms_step_of(const MsCtl* __restrict__ c, const MsGArgs& a) {
    const int par = c->step & 1, cur = c->cur;
    MsStep p;
    p.fr_cur = a.fr[cur];
    p.fr_nxt = a.fr[(cur + 1) % 3];
    p.c_now = a.ctr + par * CTR_SET;
    p.fa.fr_old = a.fr[(cur + 2) % 3];
    p.fa.lv = a.lv;
    p.fa.step = c->step;
    p.fa.push_bits = (c->active & c->td) != 0;
    p.fa.ctr_clear = a.ctr + (par ^ 1) * CTR_SET;
    p.fa.sctr = a.sctr + par * SC_SET;
    p.fa.sctr_clear = a.sctr + (par ^ 1) * SC_SET;
    return p;
}

__global__ void k_msg_start(MsCtl* __restrict__ c, MsStart st, MsHost* __restrict__ h) {
    const int r = threadIdx.x;
    if (r < 64) {
        c->mu[r] = st.mu0;
        c->nf_prev[r] = 1;
        c->off[r] = st.off[r];
    }
    if (r == 0) {
        c->active = st.active;
        c->td = ~0ull;
        c->cur = 0;
        c->step = 0;
        c->done = st.active == 0;
        c->depth_err = 0;
        c->max_extra = st.max_extra;
        h->done = c->done;
        h->depth_err = 0;
        h->steps = 0;
    }
}

// OR the frontier bits m of a top-down slot's vertex into its neighbour w's
// next mask, minus the bits w has seen; a plain check first, then the atomic.
__device__ __forceinline__ void push_claim(int32_t w, uint64_t m, const uint64_t* __restrict__ seen,
                                           uint64_t* fr_nxt) {
    if (w < 0 || !m) return;
    const uint64_t add = m & ~seen[w];
    if (add && (fr_nxt[w] & add) != add) atomicOr((unsigned long long*)&fr_nxt[w], (unsigned long long)add);
}

template <bool SPLIT>
__global__ void __launch_bounds__(MS_BLOCK) k_msg_push(const MsCtl* __restrict__ c, MsGArgs a) {
    if (c->done) return;
    const uint64_t tm = c->active & c->td;
    if (!tm) return;
    const MsStep p = ms_step_of(c, a);
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    for (int64_t base = gw * GT_WAVE; base < a.n; base += nwaves * GT_WAVE) {
        const int64_t v = base + lane;
        const uint64_t m = v < a.n ? (p.fr_cur[v] & tm) : 0ull;
        int64_t rb = 0, re = 0;
        if (m) {
            rb = a.off[v];
            re = a.off[v + 1];
        }
        const int64_t d = re - rb;
        const bool longrow = d > MS_PUSH_LONG;
        {
            // long rows: one record per row, (vertex, index of its first
            // chunk), reserved with one 64-bit atomic per wave (records in
            // the high half, chunks in the low half)
            const int64_t nch = longrow ? (d + MS_PUSH_CHUNK - 1) / MS_PUSH_CHUNK : 0;
            int64_t incl = nch;
#pragma unroll
            for (int o = 1; o < GT_WAVE; o <<= 1) {
                const int64_t y = __shfl_up(incl, o, GT_WAVE);
                if (lane >= o) incl += y;
            }
            const int64_t tot = __shfl(incl, GT_WAVE - 1, GT_WAVE);
            if (tot > 0) {
                const uint64_t lm = __ballot(longrow);
                unsigned long long b0 = 0;
                if (lane == 0)
                    b0 = atomicAdd(&p.c_now[CTR_PUSHROWS],
                                   ((unsigned long long)__popcll(lm) << 32) | (unsigned long long)tot);
                b0 = __shfl(b0, 0, GT_WAVE);
                if (longrow) {
                    const int64_t r = (int64_t)(b0 >> 32) + lanes_below(lm);
                    const int64_t c0 = (int64_t)(b0 & 0xFFFFFFFFull) + incl - nch;
                    if (r < a.row_cap) a.rows[r] = make_int2((int32_t)v, (int32_t)c0);
                }
            }
        }
        const int32_t len = (m && !longrow) ? (int32_t)d : 0;
        int32_t incl = len;
#pragma unroll
        for (int o = 1; o < GT_WAVE; o <<= 1) {
            const int32_t y = __shfl_up(incl, o, GT_WAVE);
            if (lane >= o) incl += y;
        }
        const int32_t excl = incl - len;
        const int32_t total = __shfl(incl, GT_WAVE - 1, GT_WAVE);
        for (int32_t b0 = 0; b0 < total; b0 += MS_WINDOW) {
            int32_t w[4];
            uint64_t mm[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int32_t x = b0 + i * GT_WAVE + lane;
                int lo = 0, hi = GT_WAVE - 1;  // owner: the last lane whose prefix start is <= x
#pragma unroll
                for (int st = 0; st < 6; ++st) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (__shfl(excl, mid, GT_WAVE) <= x) lo = mid;
                    else hi = mid - 1;
                }
                const int64_t k = __shfl(rb, lo, GT_WAVE) + (x - __shfl(excl, lo, GT_WAVE));
                mm[i] = __shfl(m, lo, GT_WAVE);
                w[i] = x < total ? a.col[k] : -1;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) push_claim(w[i], mm[i], a.seen, p.fr_nxt);
        }
    }
}

// The push's long rows, MS_PUSH_CHUNK entries per chunk: a wave takes a
// contiguous range of chunk indices, finds the record of its first chunk by
// binary search over the records' first-chunk indices and walks forward.
template <bool SPLIT>
__global__ void __launch_bounds__(MS_BLOCK) k_msg_push_chunks(const MsCtl* __restrict__ c, MsGArgs a) {
    if (c->done) return;
    const uint64_t tm = c->active & c->td;
    if (!tm) return;
    const MsStep p = ms_step_of(c, a);
    const unsigned long long packed = p.c_now[CTR_PUSHROWS];
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
    if (c0 >= c1) return;
    int64_t lo = 0, hi = nrows - 1;
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
        const int64_t rb = a.off[v] + (ci - (int64_t)rec.y) * MS_PUSH_CHUNK;
        const uint64_t m = p.fr_cur[v] & tm;
        int32_t w[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t k = rb + i * GT_WAVE + lane;
            w[i] = k < e ? a.col[k] : -1;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) push_claim(w[i], m, a.seen, p.fr_nxt);
    }
}

template <bool SPLIT>
__global__ void __launch_bounds__(MS_BLOCK) k_msg_pull(const MsCtl* __restrict__ c, MsGArgs a) {
    if (c->done) return;
    const uint64_t bm = c->active & ~c->td;
    if (!bm) return;
    const MsStep p = ms_step_of(c, a);
    ms_pull_body<SPLIT>(a.n, a.off, a.col, a.hint, bm, a.seen, p.fr_cur, p.fr_nxt, a.lane_edges, p.c_now, p.fa,
                        c->off);
}

__global__ void __launch_bounds__(MS_BLOCK) k_msg_finalize(const MsCtl* __restrict__ c, MsGArgs a) {
    if (c->done) return;
    if (c->active & ~c->td) return;  // the pull ran the finalize
    const MsStep p = ms_step_of(c, a);
    ms_finalize_body(a.n, a.off, a.seen, p.fr_nxt, p.c_now, p.fa, c->off);
}

// Between steps, one wave, lane r = slot r: the step's counts, each slot's
// direction (Beamer's rule per slot, as update_dirs on the host), the
// frontier buffers rotated, the step recorded in mapped host memory.
__global__ void __launch_bounds__(GT_WAVE) k_msg_ctl(MsCtl* c, MsGArgs a, MsHost* h, int32_t alpha, int32_t beta,
                                                      int32_t ms_alpha) {
    if (c->done) return;
    const int r = lane_id();
    const int step = c->step, par = step & 1;
    const unsigned long long* set = a.ctr + par * CTR_SET;
    const unsigned long long* sset = a.sctr + par * SC_SET;
    int64_t nf = 0, mf = 0;
    for (int cp = 0; cp < SC_COPIES; ++cp) {
        nf += (int64_t)sset[cp * 128 + r];
        mf += (int64_t)sset[cp * 128 + 64 + r];
    }
    const int64_t fp = (int64_t)wave_sum(set[r * CTR_STRIDE + MS_FOUND_PAIRS]);
    const int64_t ex = (int64_t)wave_sum(set[r * CTR_STRIDE + MS_EXAMINED]);
    const uint64_t any = set[CTR_SHARED + 2];
    const uint64_t active = c->active, td = c->td;
    bool tdr = (td >> r) & 1ull;
    bool grew = false;
    int64_t mu = c->mu[r];
    if ((active >> r) & 1ull) {
        mu -= mf;
        if (tdr) {
            if (mf > mu / alpha) tdr = false;
        } else {
            if (nf < c->nf_prev[r] && nf <= a.n / beta) tdr = true;
        }
        grew = nf > c->nf_prev[r];
        c->nf_prev[r] = nf;
        c->mu[r] = mu;
    }
    uint64_t ntd = __ballot(tdr);
    const uint64_t next = active & any;  // slots with a next step
    if ((next & ~ntd) != 0 && ms_alpha > alpha) {
        const bool join = (((next & ntd & td) >> r) & 1ull) && grew && mf > mu / ms_alpha;
        ntd &= ~__ballot(join);
    }
    if (r != 0) return;
    if (step < GT_MAX_LEVELS) {
        gt_level_stats ls;
        ls.dir = (active & ~td) ? GT_DIR_BOTTOM_UP : GT_DIR_TOP_DOWN;
        ls.kernel = ls.dir == GT_DIR_BOTTOM_UP ? GT_KERNEL_BU_WORDS : GT_KERNEL_TD_FLAT;
        ls.frontier = __popcll(active & td);
        ls.scanned = __popcll(active & ~td);
        ls.examined = ex;
        ls.found = fp;
        ls.ms = 0.f;
        ls.ms_main = 0.f;
        ls.examined_long = 0;
        ls.found_long = 0;
        h->level[step] = ls;
    }
    c->td = ntd;
    c->active = next;
    c->step = step + 1;
    c->cur = (c->cur + 1) % 3;
    int done = next == 0;
    if (!done && step + 2 + c->max_extra > 254) {  // the next step's level would not fit in a byte
        c->depth_err = 1;
        done = 1;
    }
    c->done = done;
    h->steps = step + 1;
    h->depth_err = c->depth_err;
    h->done = done;
}

// Root-major uint8 output in caller ids, one EX_TILE-vertex tile per block:
// core vertex -> its own level row; leaf -> its neighbour's row + 1 (the
// leaf pass); isolated -> unreached; by slot, the root gets 0 and the
// neighbour of a leaf root 1. Levels are only taken where the slot's seen
// bit is set. Slot r of `mask` is written to out.p[r][0..N).
struct SlotRoots {
    int32_t root[64];
    int32_t partner[64];
};
struct SlotOut {
    uint8_t* p[64];
};

// Read side: wave w of the block takes slots 16w..16w+15, lane g takes the
// four vertices 4g..4g+3 and packs, per slot, their four bytes into one
// word of the slot-major LDS tile. Write side: 16 lanes per slot row store
// its EX_TILE bytes as 16-byte pieces.
template <bool SPLIT>
__global__ void __launch_bounds__(EX_BLOCK) k_ms_extract(
    int64_t N, uint64_t mask, const int32_t* __restrict__ old2new, int64_t n_core, int64_t n_leaf,
    const int32_t* __restrict__ leaf_src_new, const int32_t* __restrict__ tdepth, const uint64_t* __restrict__ seen,
    const uint8_t* __restrict__ lv, SlotRoots sr, SlotOut out) {
    __shared__ uint32_t tile[64][EX_TILE / 4 + 4];
    const int t = threadIdx.x;
    const int qt = __builtin_amdgcn_readfirstlane(t >> 6), g = t & 63;  // wave-uniform: scalar slot fields
    const int64_t v0 = (int64_t)blockIdx.x * EX_TILE;
    uint32_t w[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t v = v0 + 4 * g + k;
        int64_t row = -1;
        uint32_t add = 0;
        if (v < N) {
            if (SPLIT) {
                const int64_t nv = old2new[v];
                if (nv < n_core) {
                    row = nv;
                } else if (nv < n_core + n_leaf) {
                    const int32_t src = leaf_src_new[nv - n_core];
                    if (src >= 0 && src < n_core) {  // a tree vertex: its core-edge vertex's row + depth
                        row = src;
                        add = tdepth ? (uint32_t)tdepth[nv - n_core] : 1u;
                    }
                }
            } else {
                row = v;
            }
        }
        uint32_t sm = 0;
        uint4 bytes = make_uint4(0, 0, 0, 0);
        if (row >= 0) {
            // the level row is loaded beside the seen word, not after it: one
            // dependent round trip less; bytes of unseen slots are masked below
            sm = (uint32_t)((seen[row] & mask) >> (16 * qt)) & 0xFFFFu;
            bytes = *reinterpret_cast<const uint4*>(lv + row * 64 + 16 * qt);
        }
        const uint32_t bw[4] = {bytes.x, bytes.y, bytes.z, bytes.w};
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = 16 * qt + i;
            uint32_t val = 255;
            if ((sm >> i) & 1u) val = (((bw[i >> 2] >> (8 * (i & 3))) & 0xFFu) + add) & 0xFFu;
            if (v == sr.root[r]) val = 0;
            else if (v == sr.partner[r]) val = 1;
            w[i] |= val << (8 * k);
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) tile[16 * qt + i][g] = w[i];
    __syncthreads();
    constexpr int PIECES = EX_TILE / 16;  // 16-byte pieces per slot row
#pragma unroll
    for (int it = 0; it < 64 * PIECES / EX_BLOCK; ++it) {
        const int idx = it * EX_BLOCK + t;
        const int r = idx / PIECES, c = idx % PIECES;
        if (!((mask >> r) & 1ull)) continue;
        const int64_t vb = v0 + 16 * c;
        if (vb >= N) continue;
        uint8_t* dst = out.p[r] + vb;
        const uint4 piece = *reinterpret_cast<const uint4*>(&tile[r][4 * c]);
        if (N - vb >= 16 && (((uintptr_t)dst) & 15) == 0) {
            *reinterpret_cast<uint4*>(dst) = piece;
        } else {
            const uint32_t pw[4] = {piece.x, piece.y, piece.z, piece.w};
            for (int i = 0; i < 16 && i < N - vb; ++i) dst[i] = (uint8_t)(pw[i >> 2] >> (8 * (i & 3)));
        }
    }
}

// Parent from levels: the first neighbour (ascending caller id) one level
// closer to the root. A lane per vertex scans the first RC_LANE entries of
// its row, 4 loads per round trip; rows still open after that are finished
// by the whole wave, 64 entries per round trip, one row after another. Rows
// are in ascending caller id on both kinds of handle; SPLIT entries are core
// ids, translated through new2old to index the caller-id level array.
constexpr int RC_LANE = 8;

template <bool SPLIT>
__device__ __forceinline__ int32_t rc_caller(const int32_t* __restrict__ new2old, int32_t u) {
    return SPLIT ? new2old[u] : u;
}

template <bool SPLIT>
__global__ void __launch_bounds__(256) k_reconstruct(int64_t N, const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ new2old,
                                                     const int32_t* __restrict__ old2new, int64_t n_core,
                                                     int64_t n_leaf, const int32_t* __restrict__ leaf_src_old,
                                                     const uint8_t* __restrict__ level, int32_t root,
                                                     int32_t partner, int32_t* __restrict__ parent) {
    using T = int32_t;
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane; base < N; base += stride) {
        const int64_t v = base + lane;
        int32_t p = -1;
        int lv = 255;
        int64_t b = 0, e = 0;
        bool open = false;
        if (v < N) {
            lv = level[v];
            if (v == root) {
                p = root;
            } else if (lv == 255 || lv == 0) {
                p = -1;
            } else if (v == partner) {
                p = root;
            } else {
                int64_t r = v;
                bool scan = true;
                if (SPLIT) {
                    const int64_t nv = old2new[v];
                    if (nv < n_core) {
                        r = nv;
                    } else {
                        scan = false;
                        if (nv < n_core + n_leaf) p = leaf_src_old[nv - n_core];
                    }
                }
                if (scan) {
                    b = off[r];
                    e = off[r + 1];
                    const int64_t lim = (e - b > RC_LANE) ? b + RC_LANE : e;
                    int64_t k = b;
                    for (; k < lim && p < 0; k += 4) {
                        T c[4];
                        int32_t u[4];
                        uint8_t l[4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) c[i] = (k + i < lim) ? col[k + i] : -1;
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            u[i] = c[i] >= 0 ? rc_caller<SPLIT>(new2old, c[i]) : 0;
                            l[i] = (k + i < lim) ? level[u[i]] : (uint8_t)255;
                        }
#pragma unroll
                        for (int i = 3; i >= 0; --i)
                            if (l[i] == lv - 1) p = u[i];  // lowest index wins
                    }
                    b = k < lim ? k : lim;
                    open = p < 0 && b < e;
                }
            }
        }
        uint64_t pend = __ballot(open);
        while (pend) {
            const int j = __ffsll((unsigned long long)pend) - 1;
            pend &= pend - 1;
            const int64_t jb = __shfl(b, j, GT_WAVE), je = __shfl(e, j, GT_WAVE);
            const int jl = __shfl(lv, j, GT_WAVE);
            int32_t found = -1;
            for (int64_t c = jb; c < je; c += GT_WAVE) {
                const int64_t kk = c + lane;
                int32_t u = -1;
                bool hit = false;
                if (kk < je) {
                    u = rc_caller<SPLIT>(new2old, col[kk]);
                    hit = level[u] == jl - 1;
                }
                const uint64_t hm = __ballot(hit);
                if (hm) {
                    found = __shfl(u, __ffsll((unsigned long long)hm) - 1, GT_WAVE);
                    break;
                }
            }
            if (lane == j) p = found;
        }
        if (v < N) parent[v] = p;
    }
}

// int32 level -> uint8 (-1 -> 255); *deep is set if a level exceeds 254.
// Four levels per thread: one 16-byte load, one 4-byte store.
__global__ void k_levels_u8(const int32_t* __restrict__ level, int64_t n, uint8_t* __restrict__ out,
                            int* __restrict__ deep) {
    const int64_t nq = (n + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride) {
        const int64_t v0 = 4 * q;
        if (v0 + 4 <= n && (((uintptr_t)(level + v0)) & 15) == 0 && (((uintptr_t)(out + v0)) & 3) == 0) {
            const int4 l = *reinterpret_cast<const int4*>(level + v0);
            const int32_t lv[4] = {l.x, l.y, l.z, l.w};
            uint32_t w = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                bad |= lv[j] > 254;
                w |= (uint32_t)(lv[j] < 0 ? 255 : (lv[j] & 0xFF)) << (8 * j);
            }
            *reinterpret_cast<uint32_t*>(out + v0) = w;
        } else {
            for (int64_t v = v0; v < n && v < v0 + 4; ++v) {
                const int32_t l = level[v];
                bad |= l > 254;
                out[v] = (uint8_t)(l < 0 ? 255 : (l & 0xFF));
            }
        }
    }
    if (bad) *deep = 1;
}

// Per-slot level overrides after an extraction (roots inside edge trees):
// fix[3i] = slot, fix[3i+1] = caller id, fix[3i+2] = level.
__global__ void k_ms_fix(int64_t k, const int32_t* __restrict__ fix, SlotOut out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride)
        out.p[fix[3 * i]][fix[3 * i + 1]] = (uint8_t)fix[3 * i + 2];
}

// Parent overrides after a reconstruction: pairs (caller id, parent).
__global__ void k_parent_fix(int64_t k, const int32_t* __restrict__ fix, int32_t* __restrict__ parent) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride)
        parent[fix[2 * i]] = fix[2 * i + 1];
}

}  // namespace

// ------------------------------------------------------------ host driver --

struct MsState {
    int64_t n = 0;
    bool ready = false;      // every buffer below is allocated for n vertices
    DevBuf seen, fr[3], lv, queue, prefix, scan_tmp, ctr, sctr, seeds, fix;  // fr: rotating frontier masks
    HostPinned h_fix;        // staging of per-slot tree overrides (k_ms_fix)
    int64_t fix_cap = 0;
    HostPinned h_ctr, h_sctr, h_seeds;
    // device-driven loop (gt_bfs_batch with ms_loop GT_LOOP_GRAPH / _DEVICE)
    DevBuf ctl, rows;        // MsCtl; push long-row records
    int64_t row_cap = 0;
    HostPinned host;         // MsHost, GPU-mapped
    void* host_dev = nullptr;
    hipStream_t cap = nullptr;
    hipGraphExec_t graph = nullptr;  // graph_levels captured steps
    gt_tuning captured{};
    MsState() = default;
    MsState(const MsState&) = delete;
    MsState& operator=(const MsState&) = delete;
    ~MsState() {
        drop_graph();
        if (cap) (void)hipStreamDestroy(cap);
    }
    void drop_graph() {
        if (graph) (void)hipGraphExecDestroy(graph);
        graph = nullptr;
    }
    void release() {
        drop_graph();
        for (DevBuf* b : {&seen, &fr[0], &fr[1], &fr[2], &lv, &queue, &prefix, &scan_tmp, &ctr, &sctr, &seeds})
            b->release();
        h_ctr.release();
        h_sctr.release();
        h_seeds.release();
        n = 0;
        ready = false;
    }
};

// Direction of each slot (Beamer's rule per traversal): top-down (push) while
// its frontier's edges are few relative to its unexplored edges, bottom-up
// (pull) in the middle, top-down again when the frontier shrinks below n/beta.
struct SlotDirs {
    uint64_t td = ~0ull;     // slots in top-down mode
    int64_t mu[64];          // unexplored edges per slot
    int64_t nf_prev[64];
    void reset_slot(int r, int64_t Et) {
        td |= 1ull << r;
        mu[r] = Et;
        nf_prev[r] = 1;
    }
};

struct gt_batch_ext {
    MsState ms;
};

static gt_status ms_alloc_all(MsState& m, int64_t n);

// The multi-source state of g, allocated on first use. A failed allocation
// releases whatever it got, so a later call starts over instead of finding a
// half-allocated state.
static gt_status ms_alloc(gt_graph* g, MsState& m) {
    if (m.n == g->tn() && m.ready) return GT_OK;
    m.ready = false;
    m.drop_graph();  // captured with the old buffers
    const gt_status st = ms_alloc_all(m, g->tn());
    if (st != GT_OK) {
        m.release();
        return st;
    }
    m.n = g->tn();
    m.ready = true;
    return GT_OK;
}

static gt_status ms_alloc_all(MsState& m, int64_t n) {
    const int64_t nn = n > 0 ? n : 1;
    GT_TRY(m.seen.alloc(sizeof(uint64_t) * nn));
    GT_TRY(m.fr[0].alloc(sizeof(uint64_t) * nn));
    GT_TRY(m.fr[1].alloc(sizeof(uint64_t) * nn));
    GT_TRY(m.fr[2].alloc(sizeof(uint64_t) * nn));
    GT_TRY(m.lv.alloc((size_t)64 * nn));
    GT_TRY(m.queue.alloc(sizeof(int32_t) * nn));
    GT_TRY(m.prefix.alloc(sizeof(int64_t) * (n + 1)));
    GT_TRY(m.scan_tmp.alloc(sizeof(int64_t) * scan_scratch_elems(n + 1)));
    GT_TRY(m.ctr.alloc(sizeof(unsigned long long) * 2 * CTR_SET));
    GT_TRY(m.sctr.alloc(sizeof(unsigned long long) * 2 * SC_SET));
    GT_TRY(m.seeds.alloc(sizeof(int32_t) * 256));
    GT_TRY(m.h_ctr.alloc(sizeof(unsigned long long) * CTR_SET));
    GT_TRY(m.h_sctr.alloc(sizeof(unsigned long long) * SC_SET));
    GT_TRY(m.h_seeds.alloc(sizeof(int32_t) * 256));
    return GT_OK;
}

// (caller id, level) written over one slot's extraction: the other vertices
// of the tree that holds a root inside an edge tree (MH > 0)
using SlotFix = std::vector<std::pair<int32_t, int32_t>>;

// Where a root's traversal starts in the traversed graph (Algorithm 9's
// root handling): seed vertex, its level, and the caller id that gets level
// 1 when the root is a leaf (-1 otherwise). MH > 0: a root inside an edge
// tree seeds its core-edge vertex at its depth, and *fix receives the other
// vertices of its tree with their levels.
static void root_seed(const gt_graph* g, int32_t root, int32_t* seed, int32_t* lvl0, int32_t* partner,
                      SlotFix* fix = nullptr) {
    *partner = -1;
    *lvl0 = 0;
    if (fix) fix->clear();
    if (!(g->flags & GT_BUILD_SPLIT)) {
        *seed = root;
        return;
    }
    const int64_t nr = g->h_old2new[root];
    if (nr < g->n_core) {
        *seed = (int32_t)nr;
    } else if (nr < g->n_core + g->n_leaf && g->mh > 0) {
        const RootPlan rp = gt_plan_root(g, root);
        *seed = rp.seed;
        *lvl0 = rp.seed_level;
        if (fix)
            for (size_t i = 0; i < rp.fix_v.size(); ++i) fix->emplace_back(rp.fix_v[i], rp.fix_level[i]);
    } else if (nr < g->n_core + g->n_leaf) {
        const int64_t j = nr - g->n_core;
        *partner = g->h_leaf_src_old[j];
        const int32_t sn = g->h_leaf_src_new[j];
        *seed = sn < g->n_core ? sn : -1;
        *lvl0 = 1;
    } else {
        *seed = -1;
    }
}

struct MsCounts {
    int64_t fv, fp, fd, ex;
    uint64_t any;
    int64_t nf[64], mf[64];
};

static gt_status ms_read(MsState& m, unsigned long long* set, unsigned long long* sset, hipStream_t s,
                         MsCounts* c) {
    unsigned long long* h = m.h_ctr.as<unsigned long long>();
    unsigned long long* hs = m.h_sctr.as<unsigned long long>();
    GT_HIP(hipMemcpyAsync(h, set, sizeof(unsigned long long) * CTR_SET, hipMemcpyDeviceToHost, s));
    GT_HIP(hipMemcpyAsync(hs, sset, sizeof(unsigned long long) * SC_SET, hipMemcpyDeviceToHost, s));
    GT_HIP(hipStreamSynchronize(s));
    unsigned long long t[4] = {0, 0, 0, 0};
    for (int sl = 0; sl < CTR_SLOTS; ++sl)
        for (int i = 0; i < 4; ++i) t[i] += h[sl * CTR_STRIDE + i];
    c->fv = (int64_t)t[MS_FOUND_V];
    c->fp = (int64_t)t[MS_FOUND_PAIRS];
    c->fd = (int64_t)t[MS_FOUND_DEG];
    c->ex = (int64_t)t[MS_EXAMINED];
    c->any = h[CTR_SHARED + 2];
    for (int r = 0; r < 64; ++r) {
        c->nf[r] = c->mf[r] = 0;
        for (int cp = 0; cp < SC_COPIES; ++cp) {
            c->nf[r] += (int64_t)hs[cp * 128 + r];
            c->mf[r] += (int64_t)hs[cp * 128 + 64 + r];
        }
    }
    return GT_OK;
}

// Update per-slot directions from one step's counts (Beamer's rule per slot).
// A top-down step costs the edges of the union of the top-down slots'
// frontiers, so when some slots pull next step anyway, a top-down slot whose
// frontier grew joins them at the lower threshold m_f > m_u / ms_alpha.
static void update_dirs(SlotDirs& sd, const MsCounts& c, uint64_t active, int64_t n_t, int alpha, int beta,
                        int ms_alpha) {
    const uint64_t td_before = sd.td;
    uint64_t grew = 0;
    for (int r = 0; r < 64; ++r) {
        if (!((active >> r) & 1ull)) continue;
        sd.mu[r] -= c.mf[r];
        const bool td = (sd.td >> r) & 1ull;
        if (td) {
            if (c.mf[r] > sd.mu[r] / alpha) sd.td &= ~(1ull << r);
        } else {
            if (c.nf[r] < sd.nf_prev[r] && c.nf[r] <= n_t / beta) sd.td |= 1ull << r;
        }
        if (c.nf[r] > sd.nf_prev[r]) grew |= 1ull << r;
        sd.nf_prev[r] = c.nf[r];
    }
    const uint64_t next = active & c.any;  // slots with a next step
    if ((next & ~sd.td) == 0 || ms_alpha <= alpha) return;
    for (int r = 0; r < 64; ++r) {
        const uint64_t bit = 1ull << r;
        if ((next & sd.td & td_before & grew & bit) && c.mf[r] > sd.mu[r] / ms_alpha) sd.td &= ~bit;
    }
}

// One level step for all active slots: push for the slots in top-down mode,
// then the pull for the others with the step's finalize in the same kernel
// (finalize alone when no slot pulls). Three frontier buffers rotate: cur
// (read), cur + 1 (next: all-zero on entry, the push ORs into it, the
// finalize keeps its unseen bits) and cur + 2 (the previous step's frontier,
// cleared here, the next step's output). On return cur is the new frontier's
// index.
template <bool SPLIT>
static gt_status ms_step(gt_graph* g, MsState& m, int& cur, uint64_t active, uint64_t tmask, int step,
                         const SlotOffsets& so, int lev, hipStream_t s, MsCounts* c, int64_t mf_est,
                         const hipEvent_t* ev = nullptr) {
    using T = int32_t;
    const int64_t n = m.n;
    const int64_t* off = g->toff();
    const T* col = SPLIT ? (const T*)g->ccol.p : (const T*)g->col.p;
    const int32_t* hint = g->bfs.hint.as<int32_t>();
    uint64_t* fr_cur = m.fr[cur].as<uint64_t>();
    uint64_t* fr_nxt = m.fr[(cur + 1) % 3].as<uint64_t>();
    uint64_t* fr_old = m.fr[(cur + 2) % 3].as<uint64_t>();  // the previous step's frontier
    unsigned long long* c_now = m.ctr.as<unsigned long long>() + (lev & 1) * CTR_SET;
    unsigned long long* c_next = m.ctr.as<unsigned long long>() + ((lev & 1) ^ 1) * CTR_SET;
    unsigned long long* s_now = m.sctr.as<unsigned long long>() + (lev & 1) * SC_SET;
    unsigned long long* s_next = m.sctr.as<unsigned long long>() + ((lev & 1) ^ 1) * SC_SET;
    const unsigned blocks = grid_for(n, MS_BLOCK, g->tune.ms_blocks);
    const uint64_t T_ = active & tmask, B_ = active & ~tmask;
    // ev (optional): step begin, pull begin, pull end, step end
    if (ev) GT_HIP(hipEventRecord(ev[0], s));
    if (T_) {
        // frontier queue of the top-down slots
        // c_now was cleared by the previous step's finalize (or at set-up)
        hipLaunchKernelGGL(k_ms_queue, dim3(grid_for(n, MQ_CHUNK, 4096)), dim3(256), 0, s, fr_cur, T_, n,
                           m.queue.as<int32_t>(), c_now + CTR_QTAIL);
        unsigned long long nq = 0;
        GT_TRY(read_scalar(c_now + CTR_QTAIL, &nq, s));
        const int64_t nfv = (int64_t)nq;
        if (nfv > 0) {
            GT_TRY((scan_exclusive<int64_t, LoadQDeg>(LoadQDeg{m.queue.as<int32_t>(), off}, nfv,
                                                      m.prefix.as<int64_t>(), m.scan_tmp.as<int64_t>(), s)));
            const unsigned pblocks = mf_est >= 0 ? grid_for(mf_est, MS_BLOCK, 16384) : 2048u;
            hipLaunchKernelGGL((k_ms_push<SPLIT>), dim3(pblocks), dim3(MS_BLOCK), 0, s, m.queue.as<int32_t>(), nfv,
                               m.prefix.as<int64_t>(), off, col, fr_cur, fr_nxt, m.seen.as<uint64_t>(), T_);
        }
    }
    const FinArgs fa{fr_old, m.lv.as<uint8_t>(), step, T_ != 0, c_next, s_now, s_next};
    if (B_) {
        // pull + finalize in one pass
        if (ev) GT_HIP(hipEventRecord(ev[1], s));
        hipLaunchKernelGGL((k_ms_pull<SPLIT>), dim3(blocks), dim3(MS_BLOCK), 0, s, n, off, col, hint, B_,
                           m.seen.as<uint64_t>(), fr_cur, fr_nxt, g->tune.bu_lane_edges, c_now, fa, so);
        if (ev) GT_HIP(hipEventRecord(ev[2], s));
    } else {
        hipLaunchKernelGGL(k_ms_finalize, dim3(blocks), dim3(MS_BLOCK), 0, s, n, off, m.seen.as<uint64_t>(), fr_nxt,
                           c_now, fa, so);
    }
    GT_HIP(hipGetLastError());
    if (ev) GT_HIP(hipEventRecord(ev[3], s));
    cur = (cur + 1) % 3;
    return ms_read(m, c_now, s_now, s, c);
}

template <bool SPLIT>
static gt_status ms_extract(gt_graph* g, MsState& m, uint64_t mask, const SlotRoots& sr, const SlotOut& so,
                            hipStream_t s, const SlotFix* fix = nullptr) {
    const int64_t N = g->n;
    hipLaunchKernelGGL((k_ms_extract<SPLIT>), dim3((unsigned)((N + EX_TILE - 1) / EX_TILE)), dim3(EX_BLOCK), 0, s,
                       N, mask, SPLIT ? g->old2new.as<int32_t>() : (const int32_t*)nullptr, g->n_core, g->n_leaf,
                       SPLIT ? g->leaf_src_new.as<int32_t>() : (const int32_t*)nullptr,
                       (const int32_t*)g->tdepth.as<int32_t>(), m.seen.as<uint64_t>(), m.lv.as<uint8_t>(), sr, so);
    GT_HIP(hipGetLastError());
    if (!fix) return GT_OK;
    int64_t k = 0;
    for (int r = 0; r < 64; ++r)
        if ((mask >> r) & 1ull) k += (int64_t)fix[r].size();
    if (k == 0) return GT_OK;
    if (k > m.fix_cap) {
        GT_TRY(m.fix.alloc(sizeof(int32_t) * 3 * (size_t)k));
        GT_TRY(m.h_fix.alloc(sizeof(int32_t) * 3 * (size_t)k));
        m.fix_cap = k;
    }
    int32_t* h = m.h_fix.as<int32_t>();
    int64_t i = 0;
    for (int r = 0; r < 64; ++r) {
        if (!((mask >> r) & 1ull)) continue;
        for (const auto& f : fix[r]) {
            if (f.second > 254) return gt_fail(GT_E_DEPTH, "a level inside the root's edge tree exceeds 254");
            h[3 * i] = r;
            h[3 * i + 1] = f.first;
            h[3 * i + 2] = f.second;
            ++i;
        }
    }
    GT_HIP(hipMemcpyAsync(m.fix.p, h, sizeof(int32_t) * 3 * (size_t)k, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ms_fix, dim3(grid_for(k, 256, 4096)), dim3(256), 0, s, k, (const int32_t*)m.fix.as<int32_t>(),
                       so);
    GT_HIP(hipGetLastError());
    return GT_OK;
}

static MsState& ms_of(gt_graph* g);

// Deepest tree vertex below its core vertex: extraction adds it to a core
// level (leaves: 1; MH > 0: up to the peeling rounds + 1).
static int tree_depth(const gt_graph* g) {
    if (!(g->flags & GT_BUILD_SPLIT) || g->n_leaf == 0) return 0;
    return g->mh > 0 ? g->tree_height + 1 : 1;
}

template <bool SPLIT>
static gt_status bfs_batch_run(gt_graph* g, const int32_t* roots, int32_t k, uint8_t* out, hipStream_t s) {
    MsState& m = ms_of(g);
    GT_TRY(ms_alloc(g, m));
    SlotOffsets so;
    SlotRoots sr;
    SlotDirs sd;
    std::memset(&so, 0, sizeof(so));
    for (int r = 0; r < 64; ++r) sr.root[r] = sr.partner[r] = -1;
    const int64_t Et = g->tE();
    int32_t* hs = m.h_seeds.as<int32_t>();
    uint64_t active = 0;
    int max_off = 0;
    std::vector<SlotFix> fix(64);
    for (int r = 0; r < k; ++r) {
        int32_t seed, l0, partner;
        root_seed(g, roots[r], &seed, &l0, &partner, &fix[(size_t)r]);
        hs[r] = seed;
        so.off[r] = l0;
        sr.root[r] = roots[r];
        sr.partner[r] = partner;
        sd.reset_slot(r, Et);
        if (seed >= 0) active |= 1ull << r;
        max_off = std::max(max_off, l0);
    }
    const int64_t n = m.n;
    hipLaunchKernelGGL(k_ms_zero, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, m.seen.as<uint64_t>(),
                       m.fr[0].as<uint64_t>(), m.fr[1].as<uint64_t>(), n);
    hipLaunchKernelGGL(k_ms_zero, dim3(8), dim3(256), 0, s, m.ctr.as<uint64_t>(), (uint64_t*)nullptr,
                       (uint64_t*)nullptr, (int64_t)(2 * CTR_SET));
    hipLaunchKernelGGL(k_ms_zero, dim3(8), dim3(256), 0, s, m.sctr.as<uint64_t>(), (uint64_t*)nullptr,
                       (uint64_t*)nullptr, (int64_t)(2 * SC_SET));
    GT_HIP(hipMemcpyAsync(m.seeds.p, hs, sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ms_seed, dim3(1), dim3(64), 0, s, k, m.seeds.as<int32_t>(), so, m.seen.as<uint64_t>(),
                       m.fr[0].as<uint64_t>(), m.lv.as<uint8_t>());
    GT_HIP(hipGetLastError());
    int cur = 0, lev = 0;
    int64_t mf = -1;
    gt_run_stats& st = g->stats;
    st.n_levels = 0;
    st.root_class = -1;  // batched run
    st.ms_init = st.ms_output = st.ms_total = 0.f;
    hipEvent_t* ev = g->bfs.ev.data();
    const bool timing = g->tune.timing != 0;
    const int tdep = tree_depth(g);
    while (active) {
        if (lev + 1 + max_off + tdep > 254) return gt_fail(GT_E_DEPTH, "batched level exceeds 254");
        MsCounts c;
        const bool rec = timing && lev < GT_MAX_LEVELS;
        const uint64_t tmask = sd.td;
        GT_TRY(ms_step<SPLIT>(g, m, cur, active, tmask, lev, so, lev, s, &c, mf, rec ? &ev[4 + 4 * lev] : nullptr));
        if (lev < GT_MAX_LEVELS) {
            gt_level_stats& ls = st.level[lev];
            ls.dir = (active & ~tmask) ? GT_DIR_BOTTOM_UP : GT_DIR_TOP_DOWN;
            ls.kernel = ls.dir == GT_DIR_BOTTOM_UP ? GT_KERNEL_BU_WORDS : GT_KERNEL_TD_EDGES;
            ls.frontier = __builtin_popcountll(active & tmask);  // slots pushed this step
            ls.scanned = __builtin_popcountll(active & ~tmask);  // slots pulled this step
            ls.examined = c.ex;
            ls.found = c.fp;
            ls.ms = 0.f;
            ls.ms_main = 0.f;
            ls.examined_long = ls.found_long = 0;
        }
        update_dirs(sd, c, active, m.n, g->tune.alpha, g->tune.beta, g->tune.ms_alpha);
        mf = c.fd;
        active &= c.any;  // a slot with an empty frontier is finished
        ++lev;
    }
    st.n_levels = lev;
    SlotOut outp;
    for (int r = 0; r < 64; ++r) outp.p[r] = r < k ? out + (int64_t)r * g->n : nullptr;
    const uint64_t kmask = k == 64 ? ~0ull : ((1ull << k) - 1ull);
    if (timing) GT_HIP(hipEventRecord(ev[2], s));
    GT_TRY(ms_extract<SPLIT>(g, m, kmask, sr, outp, s, fix.data()));
    if (timing) GT_HIP(hipEventRecord(ev[3], s));
    GT_HIP(hipStreamSynchronize(s));
    if (timing) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess) st.ms_output = ms;
        for (int l = 0; l < lev && l < GT_MAX_LEVELS; ++l) {
            if (hipEventElapsedTime(&ms, ev[4 + 4 * l], ev[4 + 4 * l + 3]) == hipSuccess) st.level[l].ms = ms;
            st.level[l].ms_main = 0.f;
            if (st.level[l].dir == GT_DIR_BOTTOM_UP &&
                hipEventElapsedTime(&ms, ev[4 + 4 * l + 1], ev[4 + 4 * l + 2]) == hipSuccess)
                st.level[l].ms_main = ms;  // the pull kernel
        }
        (void)hipGetLastError();
    }
    return GT_OK;
}

// ------------------------------------------- device-driven batched loop --

static bool ms_same_capture(const gt_tuning& a, const gt_tuning& b) {
    return a.alpha == b.alpha && a.beta == b.beta && a.ms_alpha == b.ms_alpha && a.ms_blocks == b.ms_blocks &&
           a.bu_lane_edges == b.bu_lane_edges && a.graph_levels == b.graph_levels && a.ms_loop == b.ms_loop;
}

template <bool SPLIT>
static MsGArgs ms_gargs(gt_graph* g, MsState& m) {
    MsGArgs a;
    a.n = m.n;
    a.off = g->toff();
    a.col = SPLIT ? g->ccol.as<int32_t>() : g->col.as<int32_t>();
    a.hint = g->bfs.hint.as<int32_t>();
    a.seen = m.seen.as<uint64_t>();
    for (int i = 0; i < 3; ++i) a.fr[i] = m.fr[i].as<uint64_t>();
    a.lv = m.lv.as<uint8_t>();
    a.ctr = m.ctr.as<unsigned long long>();
    a.sctr = m.sctr.as<unsigned long long>();
    a.rows = m.rows.as<int2>();
    a.row_cap = m.row_cap;
    a.lane_edges = g->tune.bu_lane_edges;
    return a;
}

// nsteps steps of the device-driven loop on stream s (launched, or captured
// when s is capturing). No argument depends on the roots or on a step.
template <bool SPLIT>
static void ms_enqueue_steps(gt_graph* g, MsState& m, int nsteps, hipStream_t s) {
    const MsGArgs a = ms_gargs<SPLIT>(g, m);
    MsCtl* c = m.ctl.as<MsCtl>();
    MsHost* h = static_cast<MsHost*>(m.host_dev);
    const gt_tuning& tu = g->tune;
    const unsigned blocks = grid_for(m.n, MS_BLOCK, tu.ms_blocks);
    for (int i = 0; i < nsteps; ++i) {
        hipLaunchKernelGGL((k_msg_push<SPLIT>), dim3(blocks), dim3(MS_BLOCK), 0, s, (const MsCtl*)c, a);
        hipLaunchKernelGGL((k_msg_push_chunks<SPLIT>), dim3(tu.ms_blocks), dim3(MS_BLOCK), 0, s, (const MsCtl*)c, a);
        hipLaunchKernelGGL((k_msg_pull<SPLIT>), dim3(blocks), dim3(MS_BLOCK), 0, s, (const MsCtl*)c, a);
        hipLaunchKernelGGL(k_msg_finalize, dim3(blocks), dim3(MS_BLOCK), 0, s, (const MsCtl*)c, a);
        hipLaunchKernelGGL(k_msg_ctl, dim3(1), dim3(GT_WAVE), 0, s, c, a, h, tu.alpha, tu.beta, tu.ms_alpha);
    }
}

template <bool SPLIT>
static gt_status ms_graph_prepare(gt_graph* g, MsState& m) {
    if (!m.ctl.p) {
        GT_TRY(m.ctl.alloc(sizeof(MsCtl)));
        GT_TRY(m.host.alloc(sizeof(MsHost), hipHostMallocMapped));
        std::memset(m.host.p, 0, sizeof(MsHost));
        GT_HIP(hipHostGetDevicePointer(&m.host_dev, m.host.p, 0));
        GT_HIP(hipStreamCreateWithFlags(&m.cap, hipStreamNonBlocking));
    }
    // push long rows (longer than MS_PUSH_LONG >= MS_PUSH_CHUNK): at most
    // E / MS_PUSH_CHUNK of them
    const int64_t cap = g->tE() / MS_PUSH_CHUNK + 64;
    if (cap > m.row_cap) {
        m.drop_graph();
        GT_TRY(m.rows.alloc(sizeof(int2) * (size_t)cap));
        m.row_cap = cap;
    }
    if (g->tune.ms_loop != GT_LOOP_GRAPH) return GT_OK;
    if (m.graph && ms_same_capture(m.captured, g->tune)) return GT_OK;
    m.drop_graph();
    GT_HIP(hipStreamBeginCapture(m.cap, hipStreamCaptureModeThreadLocal));
    ms_enqueue_steps<SPLIT>(g, m, g->tune.graph_levels, m.cap);
    const hipError_t launch_err = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t end_err = hipStreamEndCapture(m.cap, &graph);
    if (launch_err != hipSuccess || end_err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return gt_fail(GT_E_HIP, std::string("batched graph capture failed: ") +
                                     hipGetErrorString(launch_err != hipSuccess ? launch_err : end_err));
    }
    const hipError_t inst_err = hipGraphInstantiate(&m.graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (inst_err != hipSuccess) {
        m.graph = nullptr;
        return gt_fail(GT_E_HIP, std::string("batched graph instantiation failed: ") + hipGetErrorString(inst_err));
    }
    m.captured = g->tune;
    return GT_OK;
}

// gt_bfs_batch with the device-driven loop: set-up and extraction are
// ordinary launches; the steps run as graph replays (GT_LOOP_GRAPH) or as
// launches of the same kernels (GT_LOOP_DEVICE), graph_levels steps per
// host synchronisation.
template <bool SPLIT>
static gt_status bfs_batch_dev(gt_graph* g, const int32_t* roots, int32_t k, uint8_t* out, hipStream_t s) {
    MsState& m = ms_of(g);
    GT_TRY(ms_alloc(g, m));
    GT_TRY(ms_graph_prepare<SPLIT>(g, m));
    SlotOffsets so;
    SlotRoots sr;
    std::memset(&so, 0, sizeof(so));
    for (int r = 0; r < 64; ++r) sr.root[r] = sr.partner[r] = -1;
    int32_t* hs = m.h_seeds.as<int32_t>();
    uint64_t active = 0;
    int max_off = 0;
    std::vector<SlotFix> fix(64);
    for (int r = 0; r < k; ++r) {
        int32_t seed, l0, partner;
        root_seed(g, roots[r], &seed, &l0, &partner, &fix[(size_t)r]);
        hs[r] = seed;
        so.off[r] = l0;
        sr.root[r] = roots[r];
        sr.partner[r] = partner;
        if (seed >= 0) active |= 1ull << r;
        max_off = std::max(max_off, l0);
    }
    const int max_extra = max_off + tree_depth(g);
    if (active && 1 + max_extra > 254) return gt_fail(GT_E_DEPTH, "batched level exceeds 254");
    const int64_t n = m.n;
    hipLaunchKernelGGL(k_ms_zero, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, m.seen.as<uint64_t>(),
                       m.fr[0].as<uint64_t>(), m.fr[1].as<uint64_t>(), n);
    hipLaunchKernelGGL(k_ms_zero, dim3(8), dim3(256), 0, s, m.ctr.as<uint64_t>(), (uint64_t*)nullptr,
                       (uint64_t*)nullptr, (int64_t)(2 * CTR_SET));
    hipLaunchKernelGGL(k_ms_zero, dim3(8), dim3(256), 0, s, m.sctr.as<uint64_t>(), (uint64_t*)nullptr,
                       (uint64_t*)nullptr, (int64_t)(2 * SC_SET));
    GT_HIP(hipMemcpyAsync(m.seeds.p, hs, sizeof(int32_t) * k, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_ms_seed, dim3(1), dim3(64), 0, s, k, m.seeds.as<int32_t>(), so, m.seen.as<uint64_t>(),
                       m.fr[0].as<uint64_t>(), m.lv.as<uint8_t>());
    MsStart st0;
    std::memset(&st0, 0, sizeof(st0));
    st0.active = active;
    st0.max_extra = max_extra;
    st0.mu0 = g->tE();
    for (int r = 0; r < 64; ++r) st0.off[r] = so.off[r];
    MsHost* h = m.host.as<MsHost>();
    h->done = 0;
    hipLaunchKernelGGL(k_msg_start, dim3(1), dim3(64), 0, s, m.ctl.as<MsCtl>(), st0, static_cast<MsHost*>(m.host_dev));
    GT_HIP(hipGetLastError());
    const bool replay = g->tune.ms_loop == GT_LOOP_GRAPH;
    for (int64_t it = 0;; ++it) {
        if (replay) {
            GT_HIP(hipGraphLaunch(m.graph, s));
        } else {
            ms_enqueue_steps<SPLIT>(g, m, g->tune.graph_levels, s);
            GT_HIP(hipGetLastError());
        }
        GT_HIP(hipStreamSynchronize(s));
        std::atomic_thread_fence(std::memory_order_acquire);
        if (__atomic_load_n(&h->done, __ATOMIC_ACQUIRE)) break;
        // every step discovers a vertex for some slot until the last
        if (it * g->tune.graph_levels > n + 2) return gt_fail(GT_E_HIP, "device-driven batch did not end");
    }
    gt_run_stats& st = g->stats;
    st.n_levels = h->steps;
    st.root_class = -1;  // batched run
    st.ms_init = st.ms_output = st.ms_total = 0.f;
    std::memcpy(st.level, h->level, sizeof(gt_level_stats) * (size_t)std::min(h->steps, GT_MAX_LEVELS));
    if (h->depth_err) return gt_fail(GT_E_DEPTH, "batched level exceeds 254");
    SlotOut outp;
    for (int r = 0; r < 64; ++r) outp.p[r] = r < k ? out + (int64_t)r * g->n : nullptr;
    const uint64_t kmask = k == 64 ? ~0ull : ((1ull << k) - 1ull);
    hipEvent_t* ev = g->bfs.ev.data();
    const bool timing = g->tune.timing != 0;
    if (timing) GT_HIP(hipEventRecord(ev[2], s));
    GT_TRY(ms_extract<SPLIT>(g, m, kmask, sr, outp, s, fix.data()));
    if (timing) GT_HIP(hipEventRecord(ev[3], s));
    GT_HIP(hipStreamSynchronize(s));
    if (timing) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess) st.ms_output = ms;
        (void)hipGetLastError();
    }
    return GT_OK;
}

// Batch state lives beside the handle (created on first use).
static std::mutex g_ms_mu;
static std::unordered_map<const gt_graph*, MsState*> g_ms;

static MsState& ms_of(gt_graph* g) {
    std::lock_guard<std::mutex> lk(g_ms_mu);
    auto it = g_ms.find(g);
    if (it != g_ms.end()) return *it->second;
    MsState* m = new MsState();
    g_ms[g] = m;
    return *m;
}

void gt_batch_release(const gt_graph* g) {
    std::lock_guard<std::mutex> lk(g_ms_mu);
    auto it = g_ms.find(g);
    if (it != g_ms.end()) {
        delete it->second;
        g_ms.erase(it);
    }
}

extern "C" gt_status gt_bfs_batch(gt_graph* g, const int32_t* roots_host, int32_t k, uint8_t* levels_out,
                                  void* stream) {
    if (!g || !roots_host || !levels_out) return gt_fail(GT_E_INVALID, "NULL argument");
    if (k < 1 || k > 64) return gt_fail(GT_E_INVALID, "k must be in [1, 64]");
    for (int r = 0; r < k; ++r)
        if (roots_host[r] < 0 || (int64_t)roots_host[r] >= g->n) return gt_fail(GT_E_INVALID, "root out of range");
    std::lock_guard<std::mutex> lk(g->mu);
    const bool split = (g->flags & GT_BUILD_SPLIT) != 0;
    if (g->tune.ms_loop == GT_LOOP_GRAPH || g->tune.ms_loop == GT_LOOP_DEVICE)
        return split ? bfs_batch_dev<true>(g, roots_host, k, levels_out, (hipStream_t)stream)
                     : bfs_batch_dev<false>(g, roots_host, k, levels_out, (hipStream_t)stream);
    return split ? bfs_batch_run<true>(g, roots_host, k, levels_out, (hipStream_t)stream)
                 : bfs_batch_run<false>(g, roots_host, k, levels_out, (hipStream_t)stream);
}

extern "C" gt_status gt_reconstruct_parent(gt_graph* g, int32_t root, const uint8_t* level_in,
                                           int32_t* parent_out, void* stream) {
    if (!g || !level_in || !parent_out) return gt_fail(GT_E_INVALID, "NULL argument");
    if (root < 0 || (int64_t)root >= g->n) return gt_fail(GT_E_INVALID, "root out of range");
    std::lock_guard<std::mutex> lk(g->mu);
    hipStream_t s = (hipStream_t)stream;
    int32_t seed, l0, partner;
    root_seed(g, root, &seed, &l0, &partner);
    const unsigned blocks = grid_for(g->n, 256, 65536);
    if (g->flags & GT_BUILD_SPLIT) {
        hipLaunchKernelGGL((k_reconstruct<true>), dim3(blocks), dim3(256), 0, s, g->n, g->coff.as<int64_t>(),
                           g->ccol.as<int32_t>(), g->new2old.as<int32_t>(), g->old2new.as<int32_t>(), g->n_core,
                           g->n_leaf,
                           g->leaf_src_old.as<int32_t>(), level_in, root, partner, parent_out);
    } else {
        hipLaunchKernelGGL((k_reconstruct<false>), dim3(blocks), dim3(256), 0, s, g->n, g->off.as<int64_t>(),
                           g->col.as<int32_t>(), (const int32_t*)nullptr, (const int32_t*)nullptr, g->n, (int64_t)0,
                           (const int32_t*)nullptr, level_in, root, partner, parent_out);
    }
    GT_HIP(hipGetLastError());
    if (g->mh > 0 && (g->flags & GT_BUILD_SPLIT)) {
        const int64_t nr = g->h_old2new[root];
        if (nr >= g->n_core && nr < g->n_core + g->n_leaf) {
            // root inside an edge tree: parents along the root's path point
            // toward the root, and the core-edge vertex hangs from the tree top
            const RootPlan rp = gt_plan_root(g, root);
            MsState& m = ms_of(g);
            const int64_t k = (int64_t)rp.fix_v.size() + (rp.seed_caller >= 0 ? 1 : 0);
            if (k > 0) {
                if (k > m.fix_cap) {
                    GT_TRY(m.fix.alloc(sizeof(int32_t) * 3 * (size_t)k));
                    GT_TRY(m.h_fix.alloc(sizeof(int32_t) * 3 * (size_t)k));
                    m.fix_cap = k;
                }
                int32_t* h = m.h_fix.as<int32_t>();
                int64_t i = 0;
                for (size_t t = 0; t < rp.fix_v.size(); ++t, ++i) {
                    h[2 * i] = rp.fix_v[t];
                    h[2 * i + 1] = rp.fix_parent[t];
                }
                if (rp.seed_caller >= 0) {
                    h[2 * i] = rp.seed_caller;
                    h[2 * i + 1] = rp.seed_parent;
                }
                GT_HIP(hipMemcpyAsync(m.fix.p, h, sizeof(int32_t) * 2 * (size_t)k, hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_parent_fix, dim3(grid_for(k, 256, 4096)), dim3(256), 0, s, k,
                                   (const int32_t*)m.fix.as<int32_t>(), parent_out);
                GT_HIP(hipGetLastError());
                GT_HIP(hipStreamSynchronize(s));  // the staging buffer is reused by the next call
            }
        }
    }
    return GT_OK;
}

// Depth flags of gt_levels_to_u8, one per call in flight, kept per device
// for the life of the process: a call takes one from the pool and gives it
// back, so the per-query path allocates only when more calls overlap than
// ever before (hipFree would wait for the whole device).
static std::mutex g_flag_mu;
static std::unordered_map<int, std::vector<int*>> g_flag_pool;

static gt_status flag_take(int* dev_out, int** out) {
    int dev = 0;
    GT_HIP(hipGetDevice(&dev));
    *dev_out = dev;
    {
        std::lock_guard<std::mutex> lk(g_flag_mu);
        std::vector<int*>& pool = g_flag_pool[dev];
        if (!pool.empty()) {
            *out = pool.back();
            pool.pop_back();
            return GT_OK;
        }
    }
    void* p = nullptr;
    GT_TRY(gt_dev_malloc(&p, sizeof(int)));
    *out = static_cast<int*>(p);
    return GT_OK;
}

static void flag_give(int dev, int* p) {
    std::lock_guard<std::mutex> lk(g_flag_mu);
    g_flag_pool[dev].push_back(p);
}

static gt_status levels_to_u8_run(const int32_t* level_in, int64_t n, uint8_t* out, int* deep, hipStream_t s) {
    GT_TRY(fill_async<int>(deep, 1, 0, s));
    hipLaunchKernelGGL(k_levels_u8, dim3(grid_for((n + 3) / 4, 256, 16384)), dim3(256), 0, s, level_in, n, out,
                       deep);
    GT_HIP(hipGetLastError());
    int h = 0;
    GT_TRY(read_scalar(deep, &h, s));
    if (h) return gt_fail(GT_E_DEPTH, "a level exceeds 254");
    return GT_OK;
}

extern "C" gt_status gt_levels_to_u8(const int32_t* level_in, int64_t n, uint8_t* out, void* stream) {
    if (n < 0) return gt_fail(GT_E_INVALID, "n < 0");
    if (n == 0) return GT_OK;
    if (!level_in || !out) return gt_fail(GT_E_INVALID, "NULL argument");
    int dev = 0;
    int* deep = nullptr;
    GT_TRY(flag_take(&dev, &deep));
    const gt_status st = levels_to_u8_run(level_in, n, out, deep, (hipStream_t)stream);
    // the flag is free again once the call has read it back (or failed
    // before any kernel that uses it could still be running: a failed read
    // leaves the stream in error, and the flag is then not reused)
    if (st == GT_OK || st == GT_E_DEPTH) flag_give(dev, deep);
    return st;
}

// ----------------------------------------------------------- sessions ------
// A session runs the multi-source step loop over an open set of slots.
// Admitted queries join at the next step with a level offset of -step, so
// their levels count from their own start; a slot whose frontier empties is
// finished: its column is extracted into the caller's buffer and the slot's
// bits are cleared for reuse.

struct gt_session {
    gt_graph* g = nullptr;
    hipStream_t s = nullptr;
    int slots = 64;
    MsState m;
    SlotDirs sd;
    int cur = 0;
    int step = 0;
    int64_t mf = -1;
    uint64_t used = 0;     // slots holding a query
    uint64_t active = 0;   // slots whose frontier is non-empty
    SlotOffsets so{};
    SlotRoots sr{};
    uint8_t* out[64] = {};
    std::vector<SlotFix> fix = std::vector<SlotFix>(64);  // per slot: tree overrides (MH > 0)
    std::vector<int32_t> pend_seed, pend_slot, pend_l0;
    std::mutex mu;
};

extern "C" gt_status gt_session_create(gt_graph* g, int32_t slots, void* stream, gt_session** out) {
    if (!g || !out) return gt_fail(GT_E_INVALID, "NULL argument");
    if (slots < 1 || slots > 64) return gt_fail(GT_E_INVALID, "slots must be in [1, 64]");
    *out = nullptr;
    gt_session* ss = new (std::nothrow) gt_session();
    if (!ss) return gt_fail(GT_E_NOMEM, "host allocation failed");
    ss->g = g;
    ss->s = (hipStream_t)stream;
    ss->slots = slots;
    for (int r = 0; r < 64; ++r) ss->sr.root[r] = ss->sr.partner[r] = -1;
    gt_status st = ms_alloc(g, ss->m);
    if (st == GT_OK) {
        const int64_t n = ss->m.n;
        hipLaunchKernelGGL(k_ms_zero, dim3(grid_for(n, 256, 8192)), dim3(256), 0, ss->s, ss->m.seen.as<uint64_t>(),
                           ss->m.fr[0].as<uint64_t>(), ss->m.fr[1].as<uint64_t>(), n);
        hipLaunchKernelGGL(k_ms_zero, dim3(8), dim3(256), 0, ss->s, ss->m.ctr.as<uint64_t>(), (uint64_t*)nullptr,
                           (uint64_t*)nullptr, (int64_t)(2 * CTR_SET));
        hipLaunchKernelGGL(k_ms_zero, dim3(8), dim3(256), 0, ss->s, ss->m.sctr.as<uint64_t>(), (uint64_t*)nullptr,
                           (uint64_t*)nullptr, (int64_t)(2 * SC_SET));
        hipError_t e = hipStreamSynchronize(ss->s);
        if (e != hipSuccess) st = gt_fail(GT_E_HIP, hipGetErrorString(e));
    }
    if (st != GT_OK) {
        delete ss;
        return st;
    }
    *out = ss;
    return GT_OK;
}

extern "C" gt_status gt_session_admit(gt_session* ss, int32_t root, uint8_t* level_out, int32_t* slot_out) {
    if (!ss || !level_out) return gt_fail(GT_E_INVALID, "NULL argument");
    if (root < 0 || (int64_t)root >= ss->g->n) return gt_fail(GT_E_INVALID, "root out of range");
    std::lock_guard<std::mutex> lk(ss->mu);
    int r = -1;
    for (int i = 0; i < ss->slots; ++i)
        if (!((ss->used >> i) & 1ull)) {
            r = i;
            break;
        }
    if (r < 0) return gt_fail(GT_E_BUSY, "all slots are taken");
    int32_t seed, l0, partner;
    root_seed(ss->g, root, &seed, &l0, &partner, &ss->fix[(size_t)r]);
    // the query joins at the next step: its first expansion is step `step`,
    // which records level step + 1 + off, so off = l0 - step
    ss->so.off[r] = l0 - ss->step;
    ss->sr.root[r] = root;
    ss->sr.partner[r] = partner;
    ss->out[r] = level_out;
    ss->used |= 1ull << r;
    ss->sd.reset_slot(r, ss->g->tE());
    ss->pend_seed.push_back(seed);
    ss->pend_slot.push_back(r);
    ss->pend_l0.push_back(l0);
    if (slot_out) *slot_out = r;
    return GT_OK;
}

template <bool SPLIT>
static gt_status session_step_impl(gt_session* ss, uint64_t* finished) {
    gt_graph* g = ss->g;
    MsState& m = ss->m;
    hipStream_t s = ss->s;
    *finished = 0;
    // admissions join the current frontier
    const int nadm = (int)ss->pend_seed.size();
    if (nadm) {
        int32_t* hs = m.h_seeds.as<int32_t>();
        for (int i = 0; i < nadm; ++i) {
            hs[i] = ss->pend_seed[i];
            hs[64 + i] = ss->pend_slot[i];
            hs[128 + i] = ss->pend_l0[i];
            if (ss->pend_seed[i] >= 0) ss->active |= 1ull << ss->pend_slot[i];
        }
        GT_HIP(hipMemcpyAsync(m.seeds.p, hs, sizeof(int32_t) * 192, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_ms_admit, dim3(1), dim3(64), 0, s, nadm, m.seeds.as<int32_t>(), m.seeds.as<int32_t>() + 64,
                           m.seeds.as<int32_t>() + 128, m.seen.as<uint64_t>(), m.fr[ss->cur].as<uint64_t>(),
                           m.lv.as<uint8_t>());
        GT_HIP(hipGetLastError());
        ss->pend_seed.clear();
        ss->pend_slot.clear();
        ss->pend_l0.clear();
        ss->mf = -1;
    }
    uint64_t done = ss->used & ~ss->active;  // queries without a core traversal finish at once
    if (ss->active) {
        int max_level = 0;
        for (int r = 0; r < 64; ++r)
            if ((ss->active >> r) & 1ull) max_level = std::max(max_level, ss->step + 1 + ss->so.off[r]);
        if (max_level + tree_depth(g) > 254) return gt_fail(GT_E_DEPTH, "session level exceeds 254");
        // frontier size in vertices for a push step: count the non-zero masks
        MsCounts c;
        GT_TRY(ms_step<SPLIT>(g, m, ss->cur, ss->active, ss->sd.td, ss->step, ss->so, ss->step, s, &c, ss->mf));
        update_dirs(ss->sd, c, ss->active, m.n, g->tune.alpha, g->tune.beta, g->tune.ms_alpha);
        ss->mf = c.fd;
        const uint64_t still = ss->active & c.any;
        done |= ss->active & ~still;
        ss->active = still;
        ++ss->step;
    }
    if (done) {
        // extract the finished slots into their caller buffers, then free them
        SlotOut outp;
        for (int r = 0; r < 64; ++r) outp.p[r] = ((done >> r) & 1ull) ? ss->out[r] : nullptr;
        GT_TRY(ms_extract<SPLIT>(g, m, done, ss->sr, outp, s, ss->fix.data()));
        hipLaunchKernelGGL(k_ms_retire, dim3(grid_for(m.n, 256, 8192)), dim3(256), 0, s, ~done, m.seen.as<uint64_t>(),
                           m.fr[0].as<uint64_t>(), m.fr[1].as<uint64_t>(), m.fr[2].as<uint64_t>(), m.n);
        GT_HIP(hipGetLastError());
        GT_HIP(hipStreamSynchronize(s));
        ss->used &= ~done;
        for (int r = 0; r < 64; ++r)
            if ((done >> r) & 1ull) {
                ss->sr.root[r] = ss->sr.partner[r] = -1;
                ss->out[r] = nullptr;
            }
        ss->mf = -1;
    }
    *finished = done;
    return GT_OK;
}

extern "C" gt_status gt_session_step(gt_session* ss, uint64_t* finished_slots_out) {
    if (!ss || !finished_slots_out) return gt_fail(GT_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(ss->mu);
    std::lock_guard<std::mutex> lk2(ss->g->mu);
    if (ss->g->flags & GT_BUILD_SPLIT) return session_step_impl<true>(ss, finished_slots_out);
    return session_step_impl<false>(ss, finished_slots_out);
}

extern "C" gt_status gt_session_active(const gt_session* ss, int32_t* active_out) {
    if (!ss || !active_out) return gt_fail(GT_E_INVALID, "NULL argument");
    *active_out = __builtin_popcountll(ss->used);
    return GT_OK;
}

extern "C" gt_status gt_session_destroy(gt_session* ss) {
    if (!ss) return GT_OK;
    (void)hipStreamSynchronize(ss->s);
    delete ss;
    return GT_OK;
}
