// Graph construction on the device: CSR of the undirected simple graph
// (Section 5.1.1 "master data structure") and, for SPLIT handles, the
// edge-leaf view: degree classes (Algorithm 8, MH = 0), the relabelling that
// puts core vertices left and tree/isolated vertices right (Section 5.1.1),
// the core CSR and the leaf edge list with ascending leaf ids (Section 5.1.2).
#include <chrono>
#include <climits>

#include "gt_internal.h"

namespace {

// ---------------------------------------------------------------- CSR build

__global__ void k_count_degrees(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                int64_t m, int64_t n, uint32_t* __restrict__ cnt,
                                int* __restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) {
        int64_t s = src[i], d = dst[i];
        if (s < 0 || s >= n || d < 0 || d >= n) { *bad = 1; continue; }
        if (s == d) continue;
        atomicAdd(&cnt[s], 1u);
        atomicAdd(&cnt[d], 1u);
    }
}

__global__ void k_scatter(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, int64_t m,
                          const int64_t* __restrict__ off, uint32_t* __restrict__ fill,
                          int32_t* __restrict__ col) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) {
        int32_t s = src[i], d = dst[i];
        if (s == d) continue;
        col[off[s] + atomicAdd(&fill[s], 1u)] = d;
        col[off[d] + atomicAdd(&fill[d], 1u)] = s;
    }
}

// Row-length classes for the segmented sort: class c < SORT_BINS sorts rows
// of length <= 2^c in LDS; class SORT_BINS takes longer rows (bitmap sort).
constexpr int SORT_MIN_LOG = 5;   // rows of 2..32 entries share the 32-entry class
constexpr int SORT_MAX_LOG = 14;  // 16384 int32 = 64 KiB of LDS
constexpr int SORT_BINS = SORT_MAX_LOG + 2;

__device__ __forceinline__ int row_bin(int64_t len) {
    if (len <= 1) return -1;
    if (len > (1 << SORT_MAX_LOG)) return SORT_MAX_LOG + 1;
    int c = 64 - __clzll((unsigned long long)(len - 1));  // ceil(log2(len))
    return c < SORT_MIN_LOG ? SORT_MIN_LOG : c;
}

// pass 0: count rows per class; pass 1: write row ids per class.
__global__ void k_bin_rows(const int64_t* __restrict__ off, int64_t n, int pass,
                           unsigned long long* __restrict__ bin_cursor, int32_t* __restrict__ rows,
                           uint32_t* __restrict__ ucnt) {
    int64_t base = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) - lane_id();
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; base < n; base += stride) {
        int64_t v = base + lane_id();
        int b = -1;
        if (v < n) {
            int64_t len = off[v + 1] - off[v];
            b = row_bin(len);
            if (pass == 0 && b < 0) ucnt[v] = (uint32_t)len;
        }
        for (int c = SORT_MIN_LOG; c < SORT_BINS; ++c) {
            if (pass == 0) {
                uint64_t msk = __ballot(b == c);
                if (msk && lane_id() == 0) atomicAdd(&bin_cursor[c], (unsigned long long)__popcll(msk));
            } else {
                long long slot = wave_append(&bin_cursor[c], b == c);
                if (b == c) rows[slot] = (int32_t)v;
            }
        }
    }
}

// Sort RPB rows of at most SEG entries per block with a bitonic network in
// LDS, drop repeats and write the unique prefix back in place.
template <int SEG, int RPB, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_sort_rows(const int32_t* __restrict__ rows, int64_t nrows,
                                                     const int64_t* __restrict__ off,
                                                     int32_t* __restrict__ col,
                                                     uint32_t* __restrict__ ucnt) {
    constexpr int TOT = SEG * RPB;
    __shared__ int32_t buf[TOT];
    __shared__ int64_t rbeg[RPB];
    __shared__ int32_t rlen[RPB];
    __shared__ int32_t rid[RPB];
    const int tid = threadIdx.x;
    if (tid < RPB) {
        int64_t ri = (int64_t)blockIdx.x * RPB + tid;
        if (ri < nrows) {
            int32_t v = rows[ri];
            rid[tid] = v;
            rbeg[tid] = off[v];
            rlen[tid] = (int32_t)(off[v + 1] - off[v]);
        } else {
            rid[tid] = -1;
            rbeg[tid] = 0;
            rlen[tid] = 0;
        }
    }
    __syncthreads();
    for (int i = tid; i < TOT; i += BLOCK) {
        int r = i / SEG, k = i % SEG;
        buf[i] = (k < rlen[r]) ? col[rbeg[r] + k] : INT_MAX;
    }
    __syncthreads();
    for (int k = 2; k <= SEG; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < TOT; i += BLOCK) {
                int p = i ^ j;
                if (p > i) {
                    int32_t a = buf[i], b = buf[p];
                    // direction from the position inside the row's segment,
                    // so every row (not only even ones) ends ascending
                    bool up = (i & k & (SEG - 1)) == 0;
                    if ((a > b) == up) { buf[i] = b; buf[p] = a; }
                }
            }
            __syncthreads();
        }
    }
    const int wave = tid / GT_WAVE, nw = BLOCK / GT_WAVE, lane = lane_id();
    for (int r = wave; r < RPB; r += nw) {
        if (rid[r] < 0) continue;
        const int len = rlen[r];
        const int32_t* b = buf + r * SEG;
        int64_t out = rbeg[r];
        uint32_t cnt = 0;
        for (int c = 0; c < len; c += GT_WAVE) {
            int idx = c + lane;
            bool uniq = false;
            int32_t x = 0;
            if (idx < len) {
                x = b[idx];
                uniq = (idx == 0) || (x != b[idx - 1]);
            }
            uint64_t msk = __ballot(uniq);
            if (uniq) col[out + cnt + lanes_below(msk)] = x;
            cnt += (uint32_t)__popcll(msk);
        }
        if (lane == 0) ucnt[rid[r]] = cnt;
    }
}

// Rows longer than the LDS sort, in batches of rows with one bitmap over all
// vertex ids per row: mark every entry (k_huge_set), then read the set bits
// back in ascending order (k_huge_compact): sorted and without repeats by
// construction. Separate launches order the clear, mark and read phases.
constexpr int HUGE_BLOCK = 1024;
constexpr int HUGE_WPT = 4;  // bitmap words per thread per chunk

__global__ void __launch_bounds__(HUGE_BLOCK) k_huge_set(const int32_t* __restrict__ rows,
                                                         const int64_t* __restrict__ off,
                                                         const int32_t* __restrict__ col,
                                                         uint32_t* __restrict__ bitmaps,
                                                         int64_t words) {
    uint32_t* bm = bitmaps + (int64_t)blockIdx.x * words;
    const int32_t v = rows[blockIdx.x];
    const int64_t beg = off[v], len = off[v + 1] - off[v];
    for (int64_t i = threadIdx.x; i < len; i += HUGE_BLOCK) {
        uint32_t x = (uint32_t)col[beg + i];
        atomicOr(&bm[x >> 5], 1u << (x & 31));
    }
}

__global__ void __launch_bounds__(HUGE_BLOCK) k_huge_compact(const int32_t* __restrict__ rows,
                                                             const int64_t* __restrict__ off,
                                                             int32_t* __restrict__ col,
                                                             uint32_t* __restrict__ ucnt,
                                                             const uint32_t* __restrict__ bitmaps,
                                                             int64_t words) {
    __shared__ int64_t lds[HUGE_BLOCK / GT_WAVE + 1];
    const uint32_t* bm = bitmaps + (int64_t)blockIdx.x * words;
    const int tid = threadIdx.x;
    const int32_t v = rows[blockIdx.x];
    const int64_t beg = off[v];
    int64_t base = 0;
    for (int64_t w0 = 0; w0 < words; w0 += (int64_t)HUGE_BLOCK * HUGE_WPT) {
        uint32_t wv[HUGE_WPT];
        int64_t cnt = 0;
#pragma unroll
        for (int q = 0; q < HUGE_WPT; ++q) {
            int64_t w = w0 + (int64_t)tid * HUGE_WPT + q;
            wv[q] = (w < words) ? bm[w] : 0u;
            cnt += __popc(wv[q]);
        }
        int64_t tot;
        int64_t pos = base + block_exclusive_scan<int64_t>(cnt, lds, &tot);
#pragma unroll
        for (int q = 0; q < HUGE_WPT; ++q) {
            uint32_t x = wv[q];
            int64_t w = w0 + (int64_t)tid * HUGE_WPT + q;
            while (x) {
                int b = __ffs(x) - 1;
                x &= x - 1;
                col[beg + pos++] = (int32_t)(w * 32 + b);
            }
        }
        base += tot;
    }
    if (tid == 0) ucnt[v] = (uint32_t)base;
}

// Copy each row's unique prefix into the packed CSR; track the max degree.
__global__ void k_compact_rows(const int64_t* __restrict__ off_tmp, const int64_t* __restrict__ off,
                               const int32_t* __restrict__ col_tmp, int32_t* __restrict__ col,
                               int64_t n, int32_t* __restrict__ deg,
                               unsigned long long* __restrict__ max_deg) {
    const int lane = lane_id();
    int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    unsigned long long mx = 0;
    for (int64_t v0 = wave * GT_WAVE; v0 < n; v0 += nwaves * GT_WAVE) {
        // deg for 64 rows at once, then copy row by row
        int64_t v = v0 + lane;
        int64_t len = 0;
        if (v < n) {
            len = off[v + 1] - off[v];
            deg[v] = (int32_t)len;
            if ((unsigned long long)len > mx) mx = (unsigned long long)len;
        }
        int64_t last = n - v0 < GT_WAVE ? n - v0 : GT_WAVE;
        for (int64_t r = 0; r < last; ++r) {
            int64_t vr = v0 + r;
            int64_t src0 = off_tmp[vr], dst0 = off[vr], l = off[vr + 1] - dst0;
            for (int64_t k = lane; k < l; k += GT_WAVE) col[dst0 + k] = col_tmp[src0 + k];
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long y = __shfl_xor(mx, o, GT_WAVE);
        mx = y > mx ? y : mx;
    }
    if (lane == 0 && mx) atomicMax(max_deg, mx);
}

// Internal consistency check of a finished CSR: every entry is a vertex id.
__global__ void k_check_ids(const int32_t* __restrict__ col, int64_t e, int64_t n,
                            int* __restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < e; i += stride) {
        int32_t x = col[i];
        if (x < 0 || x >= n) *bad = 1;
    }
}

struct LoadU32 {
    const uint32_t* p;
    __device__ __forceinline__ int64_t operator()(int64_t i) const { return (int64_t)p[i]; }
};

// ------------------------------------------------------- edge-leaf view

// Packed class counts for one scan: bit 0..31 core (degree >= core_min),
// bit 32..63 leaf (degree 1 when core_min is 2). core_min 1 keeps the
// degree-1 vertices in the core (only isolated vertices split off).
// With a vertex-type array (MH > 0) the class comes from it instead.
enum : uint8_t { ET_CI = 0, ET_CE = 1, ET_TI = 2, ET_TL = 3, ET_VZ = 4 };  // Algorithm 8 types

__device__ __forceinline__ int vertex_kind(const int64_t* off, const uint8_t* type, int core_min, int64_t v) {
    if (type) {
        const uint8_t t = type[v];
        return t <= ET_CE ? 0 : (t <= ET_TL ? 1 : 2);
    }
    const int64_t d = off[v + 1] - off[v];
    return d >= core_min ? 0 : (d == 1 ? 1 : 2);
}

struct LoadClass {
    const int64_t* off;
    int core_min;
    const uint8_t* type;  // MH > 0: Algorithm 8 types, else nullptr
    __device__ __forceinline__ uint64_t operator()(int64_t v) const {
        const int k = vertex_kind(off, type, core_min, v);
        return k == 0 ? 1ull : (k == 1 ? (1ull << 32) : 0ull);
    }
};

__global__ void k_relabel(const int64_t* __restrict__ off, const uint64_t* __restrict__ rank,
                          int64_t n, int64_t n_core, int64_t n_leaf, int core_min,
                          const uint8_t* __restrict__ type, int32_t* __restrict__ old2new,
                          int32_t* __restrict__ new2old) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; v < n; v += stride) {
        const int kind = vertex_kind(off, type, core_min, v);
        uint64_t r = rank[v];
        int64_t lo = (int64_t)(r & 0xFFFFFFFFull), hi = (int64_t)(r >> 32);
        int64_t nv;
        if (kind == 0) {
            nv = lo;
            new2old[nv] = (int32_t)v;
        } else if (kind == 1) {
            nv = n_core + hi;
        } else {
            nv = n_core + n_leaf + (v - lo - hi);
        }
        old2new[v] = (int32_t)nv;
    }
}

// One wave per core row: count (fill == false) or write (fill == true) the
// row's core neighbours as core ids, in the row's (ascending caller-id)
// order; with the core in caller order that is ascending core id too.
template <bool FILL>
__global__ void k_core_rows(const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ old2new, const int32_t* __restrict__ new2old,
                            int64_t n_core, uint32_t* __restrict__ ccnt,
                            const int64_t* __restrict__ coff, int32_t* __restrict__ ccol) {
    const int lane = lane_id();
    int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    for (int64_t nv = wave; nv < n_core; nv += nwaves) {
        int32_t v = new2old[nv];
        int64_t b = off[v], e = off[v + 1];
        uint32_t cnt = 0;
        int64_t out = FILL ? coff[nv] : 0;
        for (int64_t k0 = b; k0 < e; k0 += GT_WAVE) {
            int64_t k = k0 + lane;
            int32_t u = -1, u2 = -1;
            bool core = false;
            if (k < e) {
                u = col[k];
                u2 = old2new[u];
                core = u2 < n_core;
            }
            uint64_t msk = __ballot(core);
            if (FILL && core) ccol[out + cnt + lanes_below(msk)] = u2;
            cnt += (uint32_t)__popcll(msk);
        }
        if (!FILL && lane == 0) ccnt[nv] = cnt;
    }
}

__global__ void k_leaf_list(const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                            const int32_t* __restrict__ old2new, int64_t n, int64_t n_core,
                            int32_t* __restrict__ leaf_src_new, int32_t* __restrict__ leaf_src_old,
                            unsigned long long* __restrict__ pairs) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long np = 0;
    for (; v < n; v += stride) {
        if (off[v + 1] - off[v] != 1 || old2new[v] < n_core) continue;
        int64_t j = old2new[v] - n_core;
        int32_t u = col[off[v]];
        int32_t un = old2new[u];
        leaf_src_new[j] = un;
        leaf_src_old[j] = u;
        if (un >= n_core) ++np;
    }
    if (np) atomicAdd(pairs, np);
}

// ------------------------------------------------ edge trees (MH > 0)
// Algorithm 8 on the device. Round 0 classifies degree 0 / 1; round h
// (1..MH) turns the CORE_INTERNAL vertices with at most one neighbour left
// into TREE_INTERNAL. A round decides on the degrees left at its start (the
// mark kernel only reads rem) and its decrements follow in a second kernel,
// as the algorithm's two degree arrays do.
__global__ void k_et_round0(const int64_t* __restrict__ off, int64_t n, uint8_t* __restrict__ type,
                            uint8_t* __restrict__ height, int32_t* __restrict__ rem) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const int64_t d = off[v + 1] - off[v];
        rem[v] = (int32_t)d;
        type[v] = d == 0 ? ET_VZ : (d == 1 ? ET_TL : ET_CI);
        height[v] = 0;
    }
}

__global__ void k_et_mark(int64_t n, int h, uint8_t* __restrict__ type, uint8_t* __restrict__ height,
                          const int32_t* __restrict__ rem, int* __restrict__ any) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool found = false;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (type[v] == ET_CI && rem[v] <= 1) {
            type[v] = ET_TI;
            height[v] = (uint8_t)h;
            found = true;
        }
    }
    if (__ballot(found) && lane_id() == 0) *any = 1;
}

// Every neighbour of a vertex classified in round h (TREE_LEAF: h = 0)
// loses one from its degree.
__global__ void k_et_decrement(const int64_t* __restrict__ off, const int32_t* __restrict__ col, int64_t n,
                               int h, const uint8_t* __restrict__ type, const uint8_t* __restrict__ height,
                               int32_t* __restrict__ rem) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint8_t t = type[v];
        if ((t == ET_TL || t == ET_TI) && height[v] == h)
            for (int64_t e = off[v]; e < off[v + 1]; ++e) atomicSub(&rem[col[e]], 1);
    }
}

// CORE_EDGE: a core vertex whose degree changed (it has a tree neighbour).
__global__ void k_et_core_edge(const int64_t* __restrict__ off, int64_t n, uint8_t* __restrict__ type,
                               const int32_t* __restrict__ rem) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (type[v] == ET_CI && rem[v] != (int32_t)(off[v + 1] - off[v])) type[v] = ET_CE;
}

__device__ __forceinline__ bool et_tree(uint8_t t) { return t == ET_TI || t == ET_TL; }

// Tree parent of every tree vertex v of height h: the one neighbour that was
// still left when v was classified -- a core vertex, or a tree vertex of a
// later round. Two tree vertices of the same round that are each other's
// last neighbour are the top of a tree without a core vertex: the smaller
// caller id is its top (no parent), the other hangs from it.
__global__ void k_et_parent(const int64_t* __restrict__ off, const int32_t* __restrict__ col, int64_t n,
                            const uint8_t* __restrict__ type, const uint8_t* __restrict__ height,
                            const int32_t* __restrict__ old2new, int64_t n_core, int32_t* __restrict__ tpar,
                            int32_t* __restrict__ told, unsigned long long* __restrict__ pairs) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long np = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const uint8_t t = type[v];
        if (!et_tree(t)) continue;
        const uint8_t h = height[v];
        int32_t p = -1;
        for (int64_t e = off[v]; e < off[v + 1]; ++e) {
            const int32_t y = col[e];
            const uint8_t ty = type[y];
            if (ty == ET_CI || ty == ET_CE || (et_tree(ty) && (height[y] > h || (height[y] == h && y < v)))) {
                p = y;
                break;
            }
        }
        const int64_t j = old2new[v] - n_core;
        tpar[j] = p;
        told[j] = (int32_t)v;
        if (t == ET_TL && p >= 0 && type[p] == ET_TL) ++np;
        if (t == ET_TL && p < 0 && off[v + 1] - off[v] == 1 && type[col[off[v]]] == ET_TL) ++np;
    }
    if (np) atomicAdd(pairs, np);
}

// Core-edge vertex, depth and tree top of the tree vertices of height h,
// run for h from the greatest height down to 0 (a parent has a greater
// height, or is a core vertex, or is the top of a tree without one).
__global__ void k_et_trees(int64_t n, int h, const uint8_t* __restrict__ type, const uint8_t* __restrict__ height,
                           const int32_t* __restrict__ old2new, int64_t n_core, const int32_t* __restrict__ tpar,
                           int32_t* __restrict__ ce, int32_t* __restrict__ depth, int32_t* __restrict__ top) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (!et_tree(type[v]) || height[v] != h) continue;
        const int64_t j = old2new[v] - n_core;
        const int32_t p = tpar[j];
        int32_t c = -1, d = 0, tp = (int32_t)j;
        if (p >= 0) {
            const int64_t np = old2new[p];
            if (np < n_core) {
                c = (int32_t)np;
                d = 1;
            } else if (height[p] == h) {  // the top of a tree without a core vertex
                d = 1;
                tp = (int32_t)(np - n_core);
            } else {
                const int64_t jp = np - n_core;
                c = ce[jp];
                d = depth[jp] + 1;
                tp = top[jp];
            }
        }
        ce[j] = c;
        depth[j] = d;
        top[j] = tp;
    }
}

// Hub-first core numbering: a capped degree histogram of the core picks the
// hub threshold; hubs then take core ids [0, n_hub) and the other core
// vertices [n_hub, n_core), each in caller-id order (a stable partition).
constexpr int HUB_HIST = 4096;

__global__ void k_core_deg_hist(const int64_t* __restrict__ off, const int32_t* __restrict__ new2old, int64_t nc,
                                unsigned long long* __restrict__ hist) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        const int32_t v = new2old[i];
        const int64_t d = off[v + 1] - off[v];
        atomicAdd(&hist[d < HUB_HIST ? d : HUB_HIST - 1], 1ull);
    }
}

struct LoadHub {
    const int64_t* off;
    const int32_t* new2old;
    int64_t min_deg;
    __device__ __forceinline__ int64_t operator()(int64_t i) const {
        const int32_t v = new2old[i];
        return (off[v + 1] - off[v]) >= min_deg ? 1 : 0;
    }
};

__global__ void k_hub_relabel(const int64_t* __restrict__ off, const int32_t* __restrict__ new2old, int64_t nc,
                              int64_t min_deg, const int64_t* __restrict__ rank, int64_t n_hub,
                              int32_t* __restrict__ new2old_out, int32_t* __restrict__ old2new) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        const int32_t v = new2old[i];
        const bool hub = (off[v + 1] - off[v]) >= min_deg;
        const int64_t nid = hub ? rank[i] : n_hub + (i - rank[i]);
        new2old_out[nid] = v;
        old2new[v] = (int32_t)nid;
    }
}

// Class groups of 64 caller ids (one wave per group): which ids are core
// vertices other than hubs and which are leaves, and the new ids of the
// first of each (within each class new ids follow caller ids).
__global__ void k_class_groups(const int32_t* __restrict__ old2new, int64_t n, int64_t n_core, int64_t n_leaf,
                               int64_t n_hub, ClassGroup* __restrict__ groups) {
    const int lane = lane_id();
    const int64_t ng = (n + GT_WAVE - 1) / GT_WAVE;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / GT_WAVE;
    for (int64_t grp = gw; grp < ng; grp += nwaves) {
        const int64_t v = grp * GT_WAVE + lane;
        const int64_t nv = v < n ? old2new[v] : INT64_MAX;
        const uint64_t cm = __ballot(nv >= n_hub && nv < n_core);
        const uint64_t lm = __ballot(nv >= n_core && nv < n_core + n_leaf);
        const uint64_t hm = __ballot(nv < n_hub);
        const int64_t cfirst = cm ? __shfl(nv, __ffsll((unsigned long long)cm) - 1, GT_WAVE) : 0;
        const int64_t lfirst = lm ? __shfl(nv, __ffsll((unsigned long long)lm) - 1, GT_WAVE) - n_core : 0;
        const int64_t hfirst = hm ? __shfl(nv, __ffsll((unsigned long long)hm) - 1, GT_WAVE) : 0;
        if (lane == 0) {
            ClassGroup G;
            G.m0 = cm | hm;
            G.m1 = lm | hm;
            G.core_base = (int32_t)cfirst;
            G.leaf_base = (int32_t)lfirst;
            G.hub_base = (int32_t)hfirst;
            G.pad = 0;
            groups[grp] = G;
        }
    }
}

}  // namespace

size_t gt_graph::device_bytes() const {
    size_t b = off.bytes + col.bytes + coff.bytes + ccol.bytes + deg.bytes + new2old.bytes +
               old2new.bytes + leaf_src_new.bytes + leaf_src_old.bytes + groups.bytes + tdepth.bytes +
               anchor_core.bytes + leaf_anchor.bytes;
    b += bfs.visit[0].bytes + bfs.visit[1].bytes + bfs.queue[0].bytes + bfs.queue[1].bytes +
         bfs.prefix.bytes + bfs.hub_q.bytes + bfs.hint.bytes + bfs.hint_orig.bytes + bfs.tdeg.bytes +
         bfs.hint2.bytes + bfs.hint2_orig.bytes + bfs.small.bytes +
         bfs.scan_tmp.bytes + bfs.ulist.bytes +
         bfs.level.bytes + bfs.lv8.bytes + bfs.ctr.bytes + bfs.gl.ctl.bytes + bfs.td_rows.bytes;
    return b;
}

// CSR of the simple undirected graph into g->off / g->col (whole graph).
static gt_status build_csr(gt_graph* g, const int32_t* src, const int32_t* dst, hipStream_t s) {
    const int64_t n = g->n, m = g->m_in;
    DevBuf cnt, bad, off_tmp, scan_tmp, col_tmp, bin_cur, rows, ucnt, maxd;
    GT_TRY(cnt.alloc(sizeof(uint32_t) * n));
    GT_TRY(bad.alloc(sizeof(int)));
    GT_TRY(off_tmp.alloc(sizeof(int64_t) * (n + 1)));
    GT_TRY(scan_tmp.alloc(sizeof(int64_t) * scan_scratch_elems(n + 1)));
    GT_TRY(fill_async<uint32_t>(cnt.as<uint32_t>(), n, 0u, s));
    GT_TRY(fill_async<int>(bad.as<int>(), 1, 0, s));
    if (m > 0) {
        hipLaunchKernelGGL(k_count_degrees, dim3(grid_for(m, 256)), dim3(256), 0, s, src, dst, m, n,
                           cnt.as<uint32_t>(), bad.as<int>());
        GT_HIP(hipGetLastError());
    }
    int h_bad = 0;
    GT_TRY(read_scalar(bad.as<int>(), &h_bad, s));
    if (h_bad) return gt_fail(GT_E_INVALID, "edge endpoint outside [0, n_vertices)");
    GT_TRY((scan_exclusive<int64_t, LoadU32>(LoadU32{cnt.as<uint32_t>()}, n, off_tmp.as<int64_t>(),
                                             scan_tmp.as<int64_t>(), s)));
    int64_t total = 0;
    GT_TRY(read_scalar(off_tmp.as<int64_t>() + n, &total, s));
    GT_TRY(col_tmp.alloc(sizeof(int32_t) * (total > 0 ? total : 1)));
    GT_TRY(fill_async<uint32_t>(cnt.as<uint32_t>(), n, 0u, s));
    if (m > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(grid_for(m, 256)), dim3(256), 0, s, src, dst, m,
                           off_tmp.as<int64_t>(), cnt.as<uint32_t>(), col_tmp.as<int32_t>());
        GT_HIP(hipGetLastError());
    }
    // bin rows by length (reuse cnt as the unique-count array)
    uint32_t* uc = cnt.as<uint32_t>();
    GT_TRY(bin_cur.alloc(sizeof(unsigned long long) * SORT_BINS));
    GT_TRY(fill_async<unsigned long long>(bin_cur.as<unsigned long long>(), SORT_BINS, 0ull, s));
    hipLaunchKernelGGL(k_bin_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, off_tmp.as<int64_t>(), n,
                       0, bin_cur.as<unsigned long long>(), (int32_t*)nullptr, uc);
    GT_HIP(hipGetLastError());
    unsigned long long h_bins[SORT_BINS];
    GT_HIP(hipMemcpyAsync(h_bins, bin_cur.p, sizeof(h_bins), hipMemcpyDeviceToHost, s));
    GT_HIP(hipStreamSynchronize(s));
    unsigned long long h_start[SORT_BINS];
    unsigned long long acc = 0;
    for (int c = 0; c < SORT_BINS; ++c) { h_start[c] = acc; acc += h_bins[c]; }
    GT_TRY(rows.alloc(sizeof(int32_t) * (acc > 0 ? acc : 1)));
    GT_HIP(hipMemcpyAsync(bin_cur.p, h_start, sizeof(h_start), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_bin_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, off_tmp.as<int64_t>(), n,
                       1, bin_cur.as<unsigned long long>(), rows.as<int32_t>(), uc);
    GT_HIP(hipGetLastError());
    int32_t* rp = rows.as<int32_t>();
    const int64_t* ot = off_tmp.as<int64_t>();
    int32_t* ct = col_tmp.as<int32_t>();
#define GT_SORT_BIN(LOG, RPB, BLK)                                                                 \
    if (h_bins[LOG]) {                                                                             \
        hipLaunchKernelGGL((k_sort_rows<(1 << LOG), RPB, BLK>),                                    \
                           dim3((unsigned)((h_bins[LOG] + RPB - 1) / RPB)), dim3(BLK), 0, s,       \
                           rp + h_start[LOG], (int64_t)h_bins[LOG], ot, ct, uc);                   \
        GT_HIP(hipGetLastError());                                                                 \
    }
    GT_SORT_BIN(5, 64, 256)
    GT_SORT_BIN(6, 32, 256)
    GT_SORT_BIN(7, 16, 256)
    GT_SORT_BIN(8, 8, 256)
    GT_SORT_BIN(9, 4, 256)
    GT_SORT_BIN(10, 2, 256)
    GT_SORT_BIN(11, 1, 256)
    GT_SORT_BIN(12, 1, 512)
    GT_SORT_BIN(13, 1, 1024)
    GT_SORT_BIN(14, 1, 1024)
#undef GT_SORT_BIN
    const int huge = SORT_MAX_LOG + 1;
    if (h_bins[huge]) {
        const int64_t words = (n + 31) / 32;
        const int64_t nh = (int64_t)h_bins[huge];
        const int64_t batch = nh < 256 ? nh : 256;
        DevBuf bms;
        GT_TRY(bms.alloc(sizeof(uint32_t) * words * batch));
        for (int64_t r0 = 0; r0 < nh; r0 += batch) {
            const int64_t nb = (nh - r0) < batch ? (nh - r0) : batch;
            const int32_t* rb = rp + h_start[huge] + r0;
            GT_TRY(fill_async<uint32_t>(bms.as<uint32_t>(), words * nb, 0u, s));
            hipLaunchKernelGGL(k_huge_set, dim3((unsigned)nb), dim3(HUGE_BLOCK), 0, s, rb, ot, ct,
                               bms.as<uint32_t>(), words);
            GT_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_huge_compact, dim3((unsigned)nb), dim3(HUGE_BLOCK), 0, s, rb, ot, ct,
                               uc, bms.as<uint32_t>(), words);
            GT_HIP(hipGetLastError());
        }
        GT_HIP(hipStreamSynchronize(s));  // bms is freed at scope exit
    }
    rows.release();
    GT_TRY(g->off.alloc(sizeof(int64_t) * (n + 1)));
    GT_TRY((scan_exclusive<int64_t, LoadU32>(LoadU32{uc}, n, g->off.as<int64_t>(),
                                             scan_tmp.as<int64_t>(), s)));
    GT_TRY(read_scalar(g->off.as<int64_t>() + n, &g->E, s));
    GT_TRY(g->col.alloc(sizeof(int32_t) * (g->E > 0 ? g->E : 1)));
    GT_TRY(maxd.alloc(sizeof(unsigned long long)));
    GT_TRY(fill_async<unsigned long long>(maxd.as<unsigned long long>(), 1, 0ull, s));
    // whole-graph degree per caller id (kept in the handle)
    GT_TRY(g->deg.alloc(sizeof(int32_t) * n));
    hipLaunchKernelGGL(k_compact_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, ot,
                       g->off.as<int64_t>(), ct, g->col.as<int32_t>(), n, g->deg.as<int32_t>(),
                       maxd.as<unsigned long long>());
    GT_HIP(hipGetLastError());
    unsigned long long h_max = 0;
    GT_TRY(read_scalar(maxd.as<unsigned long long>(), &h_max, s));
    g->max_deg = (int64_t)h_max;
    GT_TRY(fill_async<int>(bad.as<int>(), 1, 0, s));
    hipLaunchKernelGGL(k_check_ids, dim3(grid_for(g->E, 256, 16384)), dim3(256), 0, s,
                       g->col.as<int32_t>(), g->E, n, bad.as<int>());
    GT_HIP(hipGetLastError());
    GT_TRY(read_scalar(bad.as<int>(), &h_bad, s));
    if (h_bad) return gt_fail(GT_E_HIP, "internal error: CSR holds an out-of-range id");
    return GT_OK;
}

static gt_status build_split(gt_graph* g, hipStream_t s) {
    const int64_t n = g->n;
    const int64_t* off = g->off.as<int64_t>();
    const int32_t* col = g->col.as<int32_t>();
    DevBuf rank, scan_tmp, ccnt, pairs, type, height, rem, any;
    const bool et = g->mh > 0;
    const unsigned nb = grid_for(n, 256);
    if (et) {
        // Algorithm 8: degree classes, then TREE_INTERNAL rounds 1..MH
        GT_TRY(type.alloc(n));
        GT_TRY(height.alloc(n));
        GT_TRY(rem.alloc(sizeof(int32_t) * n));
        GT_TRY(any.alloc(sizeof(int)));
        hipLaunchKernelGGL(k_et_round0, dim3(nb), dim3(256), 0, s, off, n, type.as<uint8_t>(),
                           height.as<uint8_t>(), rem.as<int32_t>());
        hipLaunchKernelGGL(k_et_decrement, dim3(nb), dim3(256), 0, s, off, col, n, 0,
                           (const uint8_t*)type.as<uint8_t>(), (const uint8_t*)height.as<uint8_t>(),
                           rem.as<int32_t>());
        GT_HIP(hipGetLastError());
        int last = 0;
        for (int h = 1; h <= 254 && (g->mh == 255 || h <= g->mh); ++h) {
            GT_TRY(fill_async<int>(any.as<int>(), 1, 0, s));
            hipLaunchKernelGGL(k_et_mark, dim3(nb), dim3(256), 0, s, n, h, type.as<uint8_t>(),
                               height.as<uint8_t>(), (const int32_t*)rem.as<int32_t>(), any.as<int>());
            GT_HIP(hipGetLastError());
            int h_any = 0;
            GT_TRY(read_scalar(any.as<int>(), &h_any, s));
            if (!h_any) break;
            last = h;
            hipLaunchKernelGGL(k_et_decrement, dim3(nb), dim3(256), 0, s, off, col, n, h,
                               (const uint8_t*)type.as<uint8_t>(), (const uint8_t*)height.as<uint8_t>(),
                               rem.as<int32_t>());
            GT_HIP(hipGetLastError());
        }
        g->tree_height = last;
        hipLaunchKernelGGL(k_et_core_edge, dim3(nb), dim3(256), 0, s, off, n, type.as<uint8_t>(),
                           (const int32_t*)rem.as<int32_t>());
        GT_HIP(hipGetLastError());
        rem.release();
    }
    const uint8_t* tp = et ? type.as<uint8_t>() : nullptr;
    GT_TRY(rank.alloc(sizeof(uint64_t) * (n + 1)));
    GT_TRY(scan_tmp.alloc(sizeof(uint64_t) * scan_scratch_elems(n + 1)));
    // degree a vertex needs to stay in the traversed graph
    const int core_min = (g->flags & GT_BUILD_KEEP_ZERO) ? 0 : (g->flags & GT_BUILD_KEEP_LEAVES) ? 1 : 2;
    GT_TRY((scan_exclusive<uint64_t, LoadClass>(LoadClass{off, core_min, tp}, n, rank.as<uint64_t>(),
                                                scan_tmp.as<uint64_t>(), s)));
    uint64_t tot = 0;
    GT_TRY(read_scalar(rank.as<uint64_t>() + n, &tot, s));
    g->n_core = (int64_t)(tot & 0xFFFFFFFFull);
    g->n_leaf = (int64_t)(tot >> 32);
    g->n_zero = n - g->n_core - g->n_leaf;
    GT_TRY(g->old2new.alloc(sizeof(int32_t) * n));
    GT_TRY(g->new2old.alloc(sizeof(int32_t) * (g->n_core > 0 ? g->n_core : 1)));
    hipLaunchKernelGGL(k_relabel, dim3(grid_for(n, 256)), dim3(256), 0, s, off, rank.as<uint64_t>(),
                       n, g->n_core, g->n_leaf, core_min, tp, g->old2new.as<int32_t>(), g->new2old.as<int32_t>());
    GT_HIP(hipGetLastError());
    rank.release();
    const int64_t nc = g->n_core;
    g->n_hub = 0;
    if ((g->flags & GT_BUILD_HUBS_FIRST) && nc > 1) {
        DevBuf hist, hrank, n2o;
        GT_TRY(hist.alloc(sizeof(unsigned long long) * HUB_HIST));
        GT_TRY(fill_async<unsigned long long>(hist.as<unsigned long long>(), HUB_HIST, 0ull, s));
        hipLaunchKernelGGL(k_core_deg_hist, dim3(grid_for(nc, 256)), dim3(256), 0, s, off,
                           (const int32_t*)g->new2old.as<int32_t>(), nc, hist.as<unsigned long long>());
        GT_HIP(hipGetLastError());
        std::vector<unsigned long long> h(HUB_HIST);
        GT_HIP(hipMemcpyAsync(h.data(), hist.p, sizeof(unsigned long long) * HUB_HIST, hipMemcpyDeviceToHost, s));
        GT_HIP(hipStreamSynchronize(s));
        // smallest degree whose tail holds at most nc / 2^share of the core
        // (the top bin may exceed it)
        const int share = (int)((g->flags >> 16) & 0xFu);
        const int64_t cap = nc >> (share ? share : 4);
        int64_t min_deg = HUB_HIST - 1, tail = (int64_t)h[HUB_HIST - 1];
        for (int d = HUB_HIST - 2; d >= 2 && tail + (int64_t)h[d] <= cap; --d) {
            tail += (int64_t)h[d];
            min_deg = d;
        }
        GT_TRY(hrank.alloc(sizeof(int64_t) * (nc + 1)));
        GT_TRY((scan_exclusive<int64_t, LoadHub>(LoadHub{off, g->new2old.as<int32_t>(), min_deg}, nc,
                                                 hrank.as<int64_t>(), scan_tmp.as<int64_t>(), s)));
        int64_t n_hub = 0;
        GT_TRY(read_scalar(hrank.as<int64_t>() + nc, &n_hub, s));
        GT_TRY(n2o.alloc(sizeof(int32_t) * nc));
        hipLaunchKernelGGL(k_hub_relabel, dim3(grid_for(nc, 256)), dim3(256), 0, s, off,
                           (const int32_t*)g->new2old.as<int32_t>(), nc, min_deg, (const int64_t*)hrank.as<int64_t>(),
                           n_hub, n2o.as<int32_t>(), g->old2new.as<int32_t>());
        GT_HIP(hipGetLastError());
        GT_HIP(hipMemcpyAsync(g->new2old.p, n2o.p, sizeof(int32_t) * nc, hipMemcpyDeviceToDevice, s));
        GT_HIP(hipStreamSynchronize(s));  // n2o and hrank are freed at scope exit
        g->n_hub = n_hub;
    }
    // core CSR
    GT_TRY(ccnt.alloc(sizeof(uint32_t) * (nc > 0 ? nc : 1)));
    GT_TRY(g->coff.alloc(sizeof(int64_t) * (nc + 1)));
    if (nc > 0) {
        hipLaunchKernelGGL((k_core_rows<false>), dim3(grid_for(nc * GT_WAVE, 256)), dim3(256), 0, s, off,
                           col, g->old2new.as<int32_t>(), g->new2old.as<int32_t>(), nc,
                           ccnt.as<uint32_t>(), (const int64_t*)nullptr, (int32_t*)nullptr);
        GT_HIP(hipGetLastError());
    }
    GT_TRY((scan_exclusive<int64_t, LoadU32>(LoadU32{ccnt.as<uint32_t>()}, nc, g->coff.as<int64_t>(),
                                             scan_tmp.as<int64_t>(), s)));
    GT_TRY(read_scalar(g->coff.as<int64_t>() + nc, &g->E_core, s));
    GT_TRY(g->ccol.alloc(sizeof(int32_t) * (g->E_core > 0 ? g->E_core : 1)));
    if (nc > 0) {
        hipLaunchKernelGGL((k_core_rows<true>), dim3(grid_for(nc * GT_WAVE, 256)), dim3(256), 0, s, off,
                           col, g->old2new.as<int32_t>(), g->new2old.as<int32_t>(), nc,
                           ccnt.as<uint32_t>(), g->coff.as<int64_t>(), g->ccol.as<int32_t>());
        GT_HIP(hipGetLastError());
    }
    // leaf list (MH > 0: tree list), indexed by rank (ascending caller id)
    const int64_t nl = g->n_leaf;
    const size_t nl1 = (size_t)(nl > 0 ? nl : 1);
    GT_TRY(g->leaf_src_new.alloc(sizeof(int32_t) * nl1));
    GT_TRY(g->leaf_src_old.alloc(sizeof(int32_t) * nl1));
    GT_TRY(pairs.alloc(sizeof(unsigned long long)));
    GT_TRY(fill_async<unsigned long long>(pairs.as<unsigned long long>(), 1, 0ull, s));
    DevBuf told, ttop;
    if (!et) {
        hipLaunchKernelGGL(k_leaf_list, dim3(grid_for(n, 256)), dim3(256), 0, s, off, col,
                           g->old2new.as<int32_t>(), n, nc, g->leaf_src_new.as<int32_t>(),
                           g->leaf_src_old.as<int32_t>(), pairs.as<unsigned long long>());
        GT_HIP(hipGetLastError());
    } else {
        GT_TRY(g->tdepth.alloc(sizeof(int32_t) * nl1));
        GT_TRY(told.alloc(sizeof(int32_t) * nl1));
        GT_TRY(ttop.alloc(sizeof(int32_t) * nl1));
        hipLaunchKernelGGL(k_et_parent, dim3(nb), dim3(256), 0, s, off, col, n, (const uint8_t*)tp,
                           (const uint8_t*)height.as<uint8_t>(), (const int32_t*)g->old2new.as<int32_t>(), nc,
                           g->leaf_src_old.as<int32_t>(), told.as<int32_t>(), pairs.as<unsigned long long>());
        GT_HIP(hipGetLastError());
        for (int h = g->tree_height; h >= 0; --h) {
            hipLaunchKernelGGL(k_et_trees, dim3(nb), dim3(256), 0, s, n, h, (const uint8_t*)tp,
                               (const uint8_t*)height.as<uint8_t>(), (const int32_t*)g->old2new.as<int32_t>(), nc,
                               (const int32_t*)g->leaf_src_old.as<int32_t>(), g->leaf_src_new.as<int32_t>(),
                               g->tdepth.as<int32_t>(), ttop.as<int32_t>());
            GT_HIP(hipGetLastError());
        }
    }
    const int64_t ngroups = (n + GT_WAVE - 1) / GT_WAVE;
    GT_TRY(g->groups.alloc(sizeof(ClassGroup) * (size_t)(ngroups > 0 ? ngroups : 1)));
    hipLaunchKernelGGL(k_class_groups, dim3(grid_for(ngroups * GT_WAVE, 256, 16384)), dim3(256), 0, s,
                       g->old2new.as<int32_t>(), n, nc, nl, g->n_hub, g->groups.as<ClassGroup>());
    GT_HIP(hipGetLastError());
    unsigned long long h_pairs = 0;
    GT_TRY(read_scalar(pairs.as<unsigned long long>(), &h_pairs, s));
    g->n_leaf_pairs = (int64_t)h_pairs;
    // host mirrors for root handling
    g->h_old2new.resize(n);
    g->h_leaf_src_new.resize(nl);
    g->h_leaf_src_old.resize(nl);
    GT_HIP(hipMemcpyAsync(g->h_old2new.data(), g->old2new.p, sizeof(int32_t) * n,
                          hipMemcpyDeviceToHost, s));
    if (nl > 0) {
        GT_HIP(hipMemcpyAsync(g->h_leaf_src_new.data(), g->leaf_src_new.p, sizeof(int32_t) * nl,
                              hipMemcpyDeviceToHost, s));
        GT_HIP(hipMemcpyAsync(g->h_leaf_src_old.data(), g->leaf_src_old.p, sizeof(int32_t) * nl,
                              hipMemcpyDeviceToHost, s));
    }
    std::vector<uint8_t> h_type;
    if (et) {
        g->h_tdepth.resize(nl);
        g->h_tree_of.resize(nl);
        g->h_tree_old.resize(nl);
        h_type.resize(n);
        if (nl > 0) {
            GT_HIP(hipMemcpyAsync(g->h_tdepth.data(), g->tdepth.p, sizeof(int32_t) * nl, hipMemcpyDeviceToHost, s));
            GT_HIP(hipMemcpyAsync(g->h_tree_of.data(), ttop.p, sizeof(int32_t) * nl, hipMemcpyDeviceToHost, s));
            GT_HIP(hipMemcpyAsync(g->h_tree_old.data(), told.p, sizeof(int32_t) * nl, hipMemcpyDeviceToHost, s));
        }
        GT_HIP(hipMemcpyAsync(h_type.data(), type.p, (size_t)n, hipMemcpyDeviceToHost, s));
    }
    GT_HIP(hipStreamSynchronize(s));
    if (et) {
        g->n_ti = g->n_ce = 0;
        for (int64_t v = 0; v < n; ++v) {
            g->n_ti += h_type[v] == ET_TI;
            g->n_ce += h_type[v] == ET_CE;
        }
        // members of each tree, grouped by the tree's top (counting sort)
        g->h_tree_start.assign((size_t)nl + 1, 0);
        for (int64_t j = 0; j < nl; ++j) ++g->h_tree_start[(size_t)g->h_tree_of[j] + 1];
        for (int64_t t = 0; t < nl; ++t) g->h_tree_start[(size_t)t + 1] += g->h_tree_start[(size_t)t];
        g->h_tree_members.resize(nl);
        std::vector<int64_t> fill(g->h_tree_start.begin(), g->h_tree_start.end() - 1);
        for (int64_t j = 0; j < nl; ++j) g->h_tree_members[(size_t)fill[(size_t)g->h_tree_of[j]]++] = (int32_t)j;
    }
    // edge trees grouped by their core-edge vertex: a tree vertex's entry in
    // the leaf list names that vertex (a core id), or lies outside the core
    // for trees without one
    if (nl > 0 && nc > 0) {
        std::vector<uint32_t> per((size_t)nc, 0u);
        for (int64_t j = 0; j < nl; ++j) {
            const int32_t c = g->h_leaf_src_new[(size_t)j];
            if (c >= 0 && c < nc) ++per[(size_t)c];
        }
        int64_t mn = INT64_MAX;
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t k = per[(size_t)c];
            if (k == 0) continue;
            ++g->n_edge_trees;
            g->edge_tree_vertices += k;
            g->edge_tree_max = std::max(g->edge_tree_max, k);
            mn = std::min(mn, k);
        }
        g->edge_tree_min = g->n_edge_trees > 0 ? mn : 0;
    }
    // anchors of the leaf pass: the core vertices named by the leaf list,
    // numbered in ascending core id (both arrays hold at least one entry:
    // the output pass loads a leaf's anchor in every lane)
    GT_TRY(g->anchor_core.alloc(sizeof(int32_t)));
    GT_TRY(g->leaf_anchor.alloc(sizeof(int32_t) * nl1));
    GT_TRY(fill_async<int32_t>(g->leaf_anchor.as<int32_t>(), (int64_t)nl1, -1, s));
    if (nl > 0) {
        std::vector<int32_t> anchor_of((size_t)(nc > 0 ? nc : 1), -1);
        std::vector<int32_t> anchors, leaf_anchor((size_t)nl);
        for (int64_t j = 0; j < nl; ++j) {
            const int32_t c = g->h_leaf_src_new[(size_t)j];
            if (c >= 0 && c < nc) anchor_of[(size_t)c] = 0;
        }
        for (int64_t c = 0; c < nc; ++c)
            if (anchor_of[(size_t)c] == 0) {
                anchor_of[(size_t)c] = (int32_t)anchors.size();
                anchors.push_back((int32_t)c);
            }
        for (int64_t j = 0; j < nl; ++j) {
            const int32_t c = g->h_leaf_src_new[(size_t)j];
            leaf_anchor[(size_t)j] = (c >= 0 && c < nc) ? anchor_of[(size_t)c] : -1;
        }
        g->n_anchor = (int64_t)anchors.size();
        GT_HIP(hipStreamSynchronize(s));  // the fill above is done before the copy below
        if (!anchors.empty()) GT_TRY(g->anchor_core.alloc(sizeof(int32_t) * anchors.size()));
        if (!anchors.empty())
            GT_HIP(hipMemcpy(g->anchor_core.p, anchors.data(), sizeof(int32_t) * anchors.size(),
                             hipMemcpyHostToDevice));
        GT_HIP(hipMemcpy(g->leaf_anchor.p, leaf_anchor.data(), sizeof(int32_t) * (size_t)nl, hipMemcpyHostToDevice));
    }
    // the whole-graph CSR is not needed by the split traversal
    g->off.release();
    g->col.release();
    return GT_OK;
}

extern "C" gt_status gt_build_graph(const int32_t* src, const int32_t* dst, int64_t n_edges,
                                    int64_t n_vertices, uint32_t flags, void* stream,
                                    gt_graph** out) {
    if (!out) return gt_fail(GT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (n_vertices < 1 || n_vertices > INT32_MAX)
        return gt_fail(GT_E_INVALID, "n_vertices must be in [1, 2^31-1]");
    if (n_edges < 0) return gt_fail(GT_E_INVALID, "n_edges < 0");
    if (n_edges > 0 && (!src || !dst)) return gt_fail(GT_E_INVALID, "src/dst is NULL");
    if (flags & ~0xFFF0Fu) return gt_fail(GT_E_INVALID, "unknown flags");
    if ((flags & GT_BUILD_HUBS_FIRST) && !(flags & GT_BUILD_SPLIT))
        return gt_fail(GT_E_INVALID, "GT_BUILD_HUBS_FIRST needs GT_BUILD_SPLIT");
    if ((flags & GT_BUILD_HUB_SHARE(15)) && !(flags & GT_BUILD_HUBS_FIRST))
        return gt_fail(GT_E_INVALID, "GT_BUILD_HUB_SHARE needs GT_BUILD_HUBS_FIRST");
    if ((flags & GT_BUILD_KEEP_LEAVES) && !(flags & GT_BUILD_SPLIT))
        return gt_fail(GT_E_INVALID, "GT_BUILD_KEEP_LEAVES needs GT_BUILD_SPLIT");
    if ((flags & GT_BUILD_KEEP_ZERO) && (flags & GT_BUILD_RMZERO) != GT_BUILD_RMZERO)
        return gt_fail(GT_E_INVALID, "GT_BUILD_KEEP_ZERO needs GT_BUILD_SPLIT and GT_BUILD_KEEP_LEAVES");
    const int mh = (int)((flags >> 8) & 0xFF);
    if (mh > 0 && (!(flags & GT_BUILD_SPLIT) || (flags & GT_BUILD_KEEP_LEAVES)))
        return gt_fail(GT_E_INVALID, "GT_BUILD_MH needs GT_BUILD_SPLIT without KEEP_LEAVES");
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    gt_graph* g = new (std::nothrow) gt_graph();
    if (!g) return gt_fail(GT_E_NOMEM, "host allocation failed");
    g->flags = flags;
    g->mh = mh;
    g->n = n_vertices;
    g->m_in = n_edges;
    gt_default_tuning(&g->tune);
    gt_status st = build_csr(g, src, dst, s);
    if (st == GT_OK && (flags & GT_BUILD_SPLIT)) st = build_split(g, s);
    if (st == GT_OK) {
        if (!(flags & GT_BUILD_SPLIT)) {
            g->n_core = g->n;
            g->E_core = g->E;
        }
        st = gt_bfs_scratch_alloc(g, s);
    }
    if (st == GT_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = gt_fail(GT_E_HIP, std::string("build: ") + hipGetErrorString(e));
    }
    if (st != GT_OK) {
        delete g;
        return st;
    }
    g->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = g;
    return GT_OK;
}

extern "C" gt_status gt_graph_info_get(const gt_graph* g, gt_graph_info* o) {
    if (!g || !o) return gt_fail(GT_E_INVALID, "NULL argument");
    o->n_vertices = g->n;
    o->n_input_edges = g->m_in;
    o->n_entries = g->E;
    o->max_degree = g->max_deg;
    o->n_core = g->n_core;
    o->n_leaf = g->n_leaf;
    o->n_zero = g->n_zero;
    o->n_core_entries = g->E_core;
    o->n_leaf_pairs = g->n_leaf_pairs;
    o->device_bytes = (int64_t)g->device_bytes();
    o->build_ms = g->build_ms;
    o->flags = g->flags;
    o->tree_height = (uint32_t)g->tree_height;
    o->n_tree_internal = g->n_ti;
    o->n_core_edge = g->n_ce;
    o->n_edge_trees = g->n_edge_trees;
    o->edge_tree_vertices = g->edge_tree_vertices;
    o->edge_tree_max = g->edge_tree_max;
    o->edge_tree_min = g->edge_tree_min;
    return GT_OK;
}

extern "C" gt_status gt_graph_degrees(const gt_graph* g, int32_t* deg_out, void* stream) {
    if (!g || !deg_out) return gt_fail(GT_E_INVALID, "NULL argument");
    GT_HIP(hipMemcpyAsync(deg_out, g->deg.p, sizeof(int32_t) * g->n, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
    return GT_OK;
}
