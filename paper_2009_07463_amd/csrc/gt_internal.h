// Internal declarations of the gt library: handle layout, error plumbing,
// wavefront helpers and a device-wide exclusive scan. gfx950 (CDNA4) only:
// wavefronts are 64 lanes wide and a 64-vertex bitmap word maps to one wave.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/gt.h"

#define GT_WAVE 64

// ----------------------------------------------------------------- errors --

void gt_set_error(const std::string& msg);
gt_status gt_fail(gt_status code, const std::string& msg);

#define GT_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess)                                                          \
            return gt_fail(_e == hipErrorOutOfMemory ? GT_E_NOMEM : GT_E_HIP,          \
                           std::string(#call) + ": " + hipGetErrorString(_e));         \
    } while (0)

#define GT_TRY(expr)                          \
    do {                                      \
        gt_status _s = (expr);                \
        if (_s != GT_OK) return _s;           \
    } while (0)

// Every device allocation of the library goes through these two calls,
// which keep the process-wide count of live bytes and refuse (GT_E_NOMEM)
// an allocation that would take it past the limit of gt_set_memory_limit.
gt_status gt_dev_malloc(void** p, size_t bytes);
void gt_dev_free(void* p, size_t bytes);

// Device allocation owned by a handle or a call: freed on destruction.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) gt_dev_free(p, bytes);
        p = nullptr;
        bytes = 0;
    }
    gt_status alloc(size_t b) {
        release();
        if (b == 0) b = 16;
        GT_TRY(gt_dev_malloc(&p, b));
        bytes = b;
        return GT_OK;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// Pinned host buffer (hipHostMalloc; never hipHostRegister).
struct HostPinned {
    void* p = nullptr;
    HostPinned() = default;
    HostPinned(const HostPinned&) = delete;
    HostPinned& operator=(const HostPinned&) = delete;
    ~HostPinned() { release(); }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
    }
    gt_status alloc(size_t b, unsigned flags = hipHostMallocDefault) {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        hipError_t e = hipHostMalloc(&p, b, flags);
        if (e != hipSuccess) { p = nullptr; return gt_fail(GT_E_NOMEM, "hipHostMalloc failed"); }
        return GT_OK;
    }
    template <typename T>
    T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------- handle layout --

// Per-level counters written by the traversal kernels. Additive counters
// are spread over CTR_SLOTS slots (one 64-byte line each, slot = workgroup
// index mod CTR_SLOTS) so that no single address takes every workgroup's
// atomics; the host sums the slots. Two sets alternate so that a level
// kernel can clear the set of the following level.
enum {
    CTR_FOUND = 0,     // vertices discovered
    CTR_FOUND_DEG,     // sum of their degrees (m_f of the next frontier)
    CTR_SCANNED,       // bottom-up: unvisited vertices tested
    CTR_EXAMINED,      // adjacency entries read
    CTR_EXAMINED_LONG, // of those, read by the bottom-up long-row kernel
    CTR_FOUND_LONG,    // vertices that kernel discovered
    CTR_N
};
constexpr int CTR_SLOTS = 64;
constexpr int CTR_STRIDE = 8;                           // uint64 per slot
constexpr int CTR_SHARED = CTR_SLOTS * CTR_STRIDE;      // start of the non-distributed line
constexpr int CTR_QTAIL = CTR_SHARED + 0;               // top-down append queue tail
constexpr int CTR_HUBS = CTR_SHARED + 1;                // bottom-up rows deferred to the hub kernel
constexpr int CTR_TDCHUNKS = CTR_SHARED + 2;            // top-down long rows << 32 | their chunks (device-driven loop)
constexpr int CTR_SET = CTR_SHARED + 8;                 // uint64 per counter set

__device__ __forceinline__ unsigned long long* ctr_slot(unsigned long long* set) {
    return set + (blockIdx.x & (CTR_SLOTS - 1)) * CTR_STRIDE;
}

// Device-driven level loop (GT_LOOP_GRAPH): control block, GPU-mapped host
// block (per-call parameters in, end flag and level counters out) and the
// two captured graphs: `first` initialises and runs graph_levels levels,
// `more` runs graph_levels further levels; both end with the SPLIT output
// pass, which runs only once the traversal has ended.
struct GraphLoop {
    DevBuf ctl;                      // device control block
    HostPinned host;                 // GPU-mapped host block
    void* host_dev = nullptr;        // its device address
    hipStream_t cap = nullptr;       // private capture stream
    hipGraphExec_t first = nullptr, more = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    gt_tuning captured{};            // knobs the graphs were captured with
    bool valid = false;
    void drop_graphs() {
        if (first) (void)hipGraphExecDestroy(first);
        if (more) (void)hipGraphExecDestroy(more);
        first = more = nullptr;
        valid = false;
    }
    ~GraphLoop() {
        drop_graphs();
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

// SPLIT: classes of 64 consecutive caller ids. Each class keeps ascending
// caller-id order in the relabelling, so the new id of a vertex is its
// class's first new id in the group plus the group members of that class
// below it.
struct ClassGroup {
    uint64_t m0, m1;    // class of caller id 64g + i in bits i: (m1, m0) = 00 isolated,
                        // 01 core (not a hub), 10 leaf, 11 hub (core ids [0, n_hub))
    int32_t core_base;  // core id of the group's first non-hub core vertex
    int32_t leaf_base;  // leaf index (new id - n_core) of its first leaf
    int32_t hub_base;   // core id of its first hub
    int32_t pad;        // 32 bytes: two aligned scalar loads per group
};

struct BfsScratch {
    int64_t n = 0;              // vertices of the traversed graph
    int64_t words = 0;          // 64-bit bitmap words
    DevBuf visit[2];            // visited bitmaps (bottom-up reads one, writes the other)
    DevBuf queue[2];            // frontier queues (int32)
    DevBuf fix;                 // MH > 0, root in a tree: (vertex, level, parent) triples
    HostPinned h_fix;           // their staging buffer
    int64_t fix_cap = 0;        // triples both hold
    DevBuf qcount;              // uint64[2]: queue lengths
    DevBuf prefix;              // int64[n+1]: top-down frontier degree prefix
    DevBuf hub_q;               // int32[n]: bottom-up rows deferred to the hub kernel
    DevBuf ulist;               // int32[n]: vertices unvisited when bottom-up switched to a list
    DevBuf td_rows;             // int2: flat top-down long rows, (vertex, first chunk)
    int64_t td_row_cap = 0;
    int64_t bu_lds_words_max = 0;  // bitmap words one workgroup's LDS holds
    int bu_resident[2] = {0, 0};       // k_bu / k_bu_list workgroups resident at once with the hub
    int bu_list_resident[2] = {0, 0};  // frontier in LDS, [H2] (0: no hubs)
    DevBuf tdeg;                // int32[n]: degree of every traversed vertex
    DevBuf hint;                // int32 per vertex: its highest-degree neighbour (an id of the
                                // traversed graph), probed first by bottom-up
    DevBuf hint_orig;           // SPLIT: int32 per core vertex, that neighbour's caller id
    DevBuf hint2;               // int32 per vertex: its second-highest-degree neighbour (-1: none)
    DevBuf hint2_orig;          // SPLIT: its caller id
    DevBuf small;               // uint64[words]: bit set if the vertex has at most 2 neighbours
    DevBuf scan_tmp;            // scan partials
    DevBuf level;               // SPLIT: int2 (level, parent caller id) per core vertex
    DevBuf lv8;                 // SPLIT: uint8 per anchor (gt_graph::anchor_core) for the leaf
                                // pass: 0 not reached, else min(level + 1, 255)
    DevBuf ctr;                 // uint64[2][CTR_SET]
    HostPinned h_ctr;           // pinned mirror of one counter set
    std::vector<hipEvent_t> ev; // timing events
    GraphLoop gl;               // device-driven level loop
    BfsScratch() = default;
    BfsScratch(const BfsScratch&) = delete;
    BfsScratch& operator=(const BfsScratch&) = delete;
    ~BfsScratch() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct gt_graph {
    uint32_t flags = 0;
    int64_t n = 0;        // vertices
    int64_t m_in = 0;     // input edges
    int64_t E = 0;        // directed entries of the whole simple graph
    int64_t max_deg = 0;
    double build_ms = 0;

    // PLAIN: whole graph
    DevBuf off;           // int64[n+1]
    DevBuf col;           // int32[E]
    DevBuf deg;           // int32[n]: degree per caller id (both kinds of handle)

    // SPLIT: core + leaf list
    int64_t n_core = 0, n_leaf = 0, n_zero = 0, E_core = 0, n_leaf_pairs = 0;
    int64_t n_hub = 0;    // GT_BUILD_HUBS_FIRST: core ids [0, n_hub) are the hubs (else 0)
    DevBuf coff;          // int64[n_core+1]
    DevBuf ccol;          // int32[E_core]: core id per entry; rows in ascending caller id
    DevBuf new2old;       // int32[n_core]: caller id of core vertex
    DevBuf old2new;       // int32[n]: new id (core < n_core <= leaf < n_core+n_leaf <= isolated)
    DevBuf leaf_src_new;  // int32[n_leaf]: new id of the leaf's neighbour (MH > 0: of the
                          // core-edge vertex its tree hangs from; -1 if none)
    DevBuf leaf_src_old;  // int32[n_leaf]: caller id of the leaf's neighbour (MH > 0: of its
                          // tree parent; -1 for the top of a tree without a core vertex)
    DevBuf groups;        // ClassGroup[ceil(n / 64)]
    // anchors: the core vertices that leaves (MH > 0: edge trees) hang from,
    // ascending core id; the leaf pass reads one level byte per anchor
    int64_t n_anchor = 0;
    DevBuf anchor_core;   // int32[n_anchor]: core id of anchor k
    DevBuf leaf_anchor;   // int32[n_leaf]: anchor of leaf j's neighbour (MH > 0: of its tree's
                          // core-edge vertex); -1 if that vertex is not in the core
    std::vector<int32_t> h_old2new, h_leaf_src_new, h_leaf_src_old;  // host mirrors (root handling)

    // MH > 0 edge trees (Algorithm 8 with TREE_INTERNAL rounds); the tree
    // vertices (TREE_INTERNAL and TREE_LEAF) take the place of the leaves
    int mh = 0;                  // maximum tree height (255: unlimited)
    int tree_height = 0;         // rounds that classified a TREE_INTERNAL vertex
    int64_t n_ti = 0, n_ce = 0;  // TREE_INTERNAL and CORE_EDGE counts
    DevBuf tdepth;               // int32[n_leaf]: hops from the core-edge vertex (MH > 0)
    std::vector<int32_t> h_tdepth;                   // host mirror
    std::vector<int32_t> h_tree_of;                  // tree (index of its top vertex) of each tree vertex
    std::vector<int32_t> h_tree_old;                 // caller id of each tree vertex
    std::vector<int64_t> h_tree_start;               // members of tree t: h_tree_members[start[t]..start[t+1])
    std::vector<int32_t> h_tree_members;             // tree-vertex indices grouped by tree
    int64_t n_edge_trees = 0, edge_tree_vertices = 0, edge_tree_max = 0, edge_tree_min = 0;  // Table 3 view

    BfsScratch bfs;
    gt_run_stats stats{};
    gt_tuning tune{};
    std::mutex mu;

    // traversed graph view
    int64_t tn() const { return (flags & GT_BUILD_SPLIT) ? n_core : n; }
    int64_t tE() const { return (flags & GT_BUILD_SPLIT) ? E_core : E; }
    const int64_t* toff() const { return (flags & GT_BUILD_SPLIT) ? coff.as<int64_t>() : off.as<int64_t>(); }
    size_t device_bytes() const;
};

// Root handling of Algorithm 9 for SPLIT handles (PLAIN: the root is the seed).
struct RootPlan {
    int32_t seed = -1;        // traversed vertex the level loop starts from (-1: none)
    int32_t seed_level = 0;   // its level (1 when the root is a leaf)
    int32_t seed_parent = -1; // caller id recorded as the seed's parent
    int32_t seed_caller = -1; // MH > 0, root in a tree: caller id of the core-edge seed
    int32_t partner = -1;     // caller id of a leaf root's neighbour (MH = 0)
    int32_t root_class = 0;   // 0 core / PLAIN, 1 tree vertex, 2 isolated
    // MH > 0, root inside an edge tree: the other vertices of that tree, with
    // their level and parent as seen from the root (written after the output pass)
    std::vector<int32_t> fix_v, fix_level, fix_parent;
};
RootPlan gt_plan_root(const gt_graph* g, int32_t root);

gt_status gt_bfs_scratch_alloc(gt_graph* g, hipStream_t s);
gt_status gt_bfs_graph(gt_graph* g, int32_t root, const RootPlan& rp, int32_t* parent_out,
                       int32_t* level_out, hipStream_t s);
void gt_batch_release(const gt_graph* g);  // frees the multi-source state of g, if any
void gt_default_tuning(gt_tuning* t);

// ------------------------------------------------------- wavefront helpers --

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Number of set bits of mask in lanes below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, GT_WAVE);
    return v;
}

// Wave-aggregated append: every lane with pred gets a distinct slot of
// *counter (one atomic per wave). Returns the slot, or -1 for lanes without pred.
__device__ __forceinline__ long long wave_append(unsigned long long* counter, bool pred) {
    uint64_t m = __ballot(pred);
    if (m == 0) return -1;
    int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, GT_WAVE);
    return pred ? (long long)(base + lanes_below(m)) : -1;
}

// Wave-aggregated atomic add of a per-lane value.
__device__ __forceinline__ void wave_add(unsigned long long* counter, unsigned long long v) {
    v = wave_sum(v);
    if (lane_id() == 0 && v) atomicAdd(counter, v);
}

// ------------------------------------------------------------------- scan --
// Exclusive prefix sum of n values given by a loader functor: out[0..n],
// out[n] = total. Reduce-then-scan over tiles of SCAN_TILE values; partial
// sums are scanned recursively. All kernels are plain launches (no
// inter-block waiting).

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int64_t SCAN_TILE = (int64_t)SCAN_BLOCK * SCAN_ITEMS;

template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds, T* total) {
    // lds: at least SCAN_BLOCK / 64 + 1 entries
    const int lane = lane_id(), wave = threadIdx.x / GT_WAVE;
    T x = v;
#pragma unroll
    for (int o = 1; o < GT_WAVE; o <<= 1) {
        T y = __shfl_up(x, o, GT_WAVE);
        if (lane >= o) x += y;
    }
    if (lane == GT_WAVE - 1) lds[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        const int nw = blockDim.x / GT_WAVE;
        for (int w = 0; w < nw; ++w) { T t = lds[w]; lds[w] = run; run += t; }
        lds[nw] = run;
    }
    __syncthreads();
    T res = lds[wave] + x - v;
    *total = lds[blockDim.x / GT_WAVE];
    __syncthreads();
    return res;
}

template <typename T, typename Load>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_reduce(Load load, int64_t n, T* partial) {
    __shared__ T lds[SCAN_BLOCK / GT_WAVE + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j;
        if (i < n) s += load(i);
    }
    T tot;
    (void)block_exclusive_scan<T>(s, lds, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// offsets == nullptr: single tile. Otherwise offsets[b] is added to tile b.
template <typename T, typename Load>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_tiles(Load load, int64_t n, const T* offsets,
                                                            T* out) {
    __shared__ T lds[SCAN_BLOCK / GT_WAVE + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T vals[SCAN_ITEMS];
    T s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j;
        vals[j] = (i < n) ? load(i) : (T)0;
        s += vals[j];
    }
    T tot;
    T run = block_exclusive_scan<T>(s, lds, &tot);
    T off0 = offsets ? offsets[blockIdx.x] : (T)0;
    run += off0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j;
        if (i < n) out[i] = run;
        run += vals[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off0 + tot;
}

template <typename T>
struct LoadArray {
    const T* p;
    __device__ __forceinline__ T operator()(int64_t i) const { return p[i]; }
};

// Scratch elements needed by scan_exclusive for n values.
inline int64_t scan_scratch_elems(int64_t n) {
    int64_t total = 0;
    while (n > SCAN_TILE) {
        int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
        total += 2 * (nb + 1);
        n = nb;
    }
    return total + 2;
}

template <typename T, typename Load>
gt_status scan_exclusive(Load load, int64_t n, T* out, T* scratch, hipStream_t s) {
    if (n <= SCAN_TILE) {
        hipLaunchKernelGGL((k_scan_tiles<T, Load>), dim3(1), dim3(SCAN_BLOCK), 0, s, load, n,
                           (const T*)nullptr, out);
        GT_HIP(hipGetLastError());
        return GT_OK;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    T* partial = scratch;
    T* partial_ex = scratch + (nb + 1);
    hipLaunchKernelGGL((k_scan_reduce<T, Load>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, load,
                       n, partial);
    GT_HIP(hipGetLastError());
    GT_TRY((scan_exclusive<T, LoadArray<T>>(LoadArray<T>{partial}, nb, partial_ex,
                                             scratch + 2 * (nb + 1), s)));
    hipLaunchKernelGGL((k_scan_tiles<T, Load>), dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, s, load, n,
                       (const T*)partial_ex, out);
    GT_HIP(hipGetLastError());
    return GT_OK;
}

// ------------------------------------------------------------------- misc --

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

inline unsigned grid_for(int64_t n, int block, int64_t max_blocks = 65536) {
    int64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (unsigned)b;
}

template <typename T>
gt_status fill_async(T* p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return GT_OK;
    hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, p, n, v);
    GT_HIP(hipGetLastError());
    return GT_OK;
}

template <typename T>
gt_status read_scalar(const T* dev, T* host, hipStream_t s) {
    GT_HIP(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s));
    GT_HIP(hipStreamSynchronize(s));
    return GT_OK;
}
