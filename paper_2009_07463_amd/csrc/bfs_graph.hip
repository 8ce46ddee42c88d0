// Device-driven single-source traversal (level loop GT_LOOP_GRAPH): the
// direction-optimizing BFS of bfs.hip (Section 2.1, Algorithm 1; for SPLIT
// the driver of Algorithm 9 with the leaf pass of Algorithm 7), arranged so
// that no kernel argument depends on the root or on an earlier level, which
// lets a fixed sequence of levels be captured once in a HIP graph and be
// replayed per call. The host then synchronises once per replay instead of
// once per level.
//
//  - A device control block (GCtl) holds the next level's direction,
//    frontier source, bitmap and queue indices and counts.
//  - A level is three kernels. k_g_level runs the top-down units or the
//    bottom-up words; k_g_level_end runs the top-down long-row chunks or the
//    bottom-up long rows; k_g_ctl (one wave) sums the level's counters and
//    applies the direction rule of Beamer et al. (reference [12] of the
//    paper) for the next level. All return at once once the traversal has
//    ended. (A kernel costs about 4.5 us of launch and cache maintenance
//    whatever it does, so fewer, fused kernels matter more than in the
//    host-driven loop.)
//  - Top-down needs no prefix sum over the frontier: a wave takes 64
//    frontier vertices (64 queue entries, or the frontier bits of one bitmap
//    word), reads their short rows as one flat list, and cuts rows longer
//    than td_hub_deg into 256-entry chunks that the second kernel spreads
//    over the grid, one wave per chunk.
//
// Bitmaps: at the start of every level vis[cur] is the visited set with the
// frontier F and vis[cur^1] the visited set without F. Top-down tests
// vis[cur] (not written during the level), claims into vis[cur^1] and adds
// F to it; bottom-up reads vis[cur] and writes every word of vis[cur^1].
// Either way vis[cur^1] ends as the new visited set and vis[cur] as the new
// visited set without the new frontier, so every level swaps cur. When the
// previous level did not append its discoveries to a queue, the top-down
// frontier is the set of bits of vis[cur] missing from vis[cur^1].
#include <algorithm>
#include <atomic>
#include <cstring>

#include "bfs_kernels.h"

namespace {


struct GParams {
    int32_t root, partner, seed, seed_level, seed_parent, pad;
    int32_t* parent_out;
    int32_t* level_out;
};

// GPU-mapped host block: the host writes params before a call; the device
// writes the end flag, the number of levels and each level's counters.
struct GHost {
    GParams params;
    int32_t done, lev, pad0, pad1;
    gt_level_stats level[GT_MAX_LEVELS];
};

struct GCtl {
    int32_t dir;      // GT_DIR_* of the next level
    int32_t src;      // top-down frontier: 0 queue q[qi], 1 bits of vis[cur] not in vis[cur^1]
    int32_t append;   // a top-down level appends its discoveries to q[qi^1]
    int32_t cur;      // vis[cur]: visited set including the frontier
    int32_t qi;
    int32_t L;        // level of the frontier; discoveries get L + 1
    int32_t lev;      // levels completed
    int32_t done;
    int64_t nf, mf, mu;
    int64_t visited;  // traversed vertices reached so far
    int32_t* lvl;     // level / parent per traversed vertex
    int32_t* par;
    GParams p;
};

__global__ void k_g_setup(GHost* h, GCtl* __restrict__ c, int64_t mu0, int32_t* lvl_core,
                          int32_t* par_core) {
    if (threadIdx.x != 0) return;
    const GParams p = h->params;
    c->p = p;
    c->dir = GT_DIR_TOP_DOWN;  // a one-vertex frontier always starts top-down
    c->src = 0;
    c->append = 1;
    c->cur = 0;
    c->qi = 0;
    c->L = p.seed_level;
    c->lev = 0;
    c->done = p.seed < 0 ? 1 : 0;
    c->nf = p.seed >= 0 ? 1 : 0;
    c->visited = c->nf;
    c->mf = -1;
    c->mu = mu0;
    c->lvl = lvl_core ? lvl_core : p.level_out;
    c->par = par_core ? par_core : p.parent_out;
    h->lev = 0;
    h->done = c->done;
}

// vis[0] = {seed}, vis[1] = {} (the visited set without the frontier), both
// counter sets cleared, queue 0 = [seed]; PLAIN writes -1 to both outputs
// except the seed.
__global__ void k_g_init(const GCtl* __restrict__ c, uint64_t* __restrict__ vis0,
                         uint64_t* __restrict__ vis1, int64_t words, int32_t* __restrict__ q0,
                         unsigned long long* __restrict__ ctr, int64_t n_fill) {
    const int32_t seed = c->p.seed, sl = c->p.seed_level, sp = c->p.seed_parent;
    int32_t* fl = c->p.level_out;
    int32_t* fp = c->p.parent_out;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t span = words > n_fill ? words : n_fill;
    for (int64_t i = tid; i < span; i += stride) {
        if (i < words) {
            vis0[i] = (seed >= 0 && i == (seed >> 6)) ? (1ull << (seed & 63)) : 0ull;
            vis1[i] = 0ull;
        }
        if (i < n_fill) {
            const bool s = (i == seed);
            fl[i] = s ? sl : -1;
            fp[i] = s ? sp : -1;
        }
    }
    if (blockIdx.x == 0) {
        clear_set(ctr);
        clear_set(ctr + CTR_SET);
        if (threadIdx.x == 0 && seed >= 0) {
            q0[0] = seed;
            if (n_fill == 0) {  // SPLIT: (level, parent) pairs, LPS<true> = 2
                c->lvl[(int64_t)seed * LPS<true>] = sl;
                c->par[(int64_t)seed * LPS<true>] = sp;
            }
        }
    }
}

// Between levels (one wave): sum the level's counters, report them, choose
// the next direction (top-down -> bottom-up when the next frontier's edges
// exceed 1/alpha of the unexplored edges; back when the frontier shrinks
// below n/beta), advance the control block and clear the next level's
// counters.
__device__ __forceinline__ void level_ctl(GCtl* c, unsigned long long* ctr, GHost* h, int64_t n_t, int32_t alpha,
                                          int32_t beta, int64_t td_small, int64_t gamma) {
    const int lane = lane_id();
    const int lev = c->lev;
    unsigned long long* set = ctr + (lev & 1) * CTR_SET;
    unsigned long long s[CTR_N];
#pragma unroll
    for (int k = 0; k < CTR_N; ++k)
        s[k] = wave_sum(__hip_atomic_load(&set[lane * CTR_STRIDE + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    // the next level's set was summed two levels ago
    unsigned long long* nset = ctr + ((lev + 1) & 1) * CTR_SET;
    for (int i = lane; i < CTR_SET; i += GT_WAVE) nset[i] = 0;
    if (lane != 0) return;
    const int64_t found = (int64_t)s[CTR_FOUND], fdeg = (int64_t)s[CTR_FOUND_DEG];
    const int dir = c->dir;
    const int64_t nf = c->nf;
    if (lev < GT_MAX_LEVELS) {
        gt_level_stats ls;
        ls.dir = dir;
        ls.kernel = dir == GT_DIR_TOP_DOWN ? GT_KERNEL_TD_FLAT : GT_KERNEL_BU_WORDS;
        ls.frontier = nf;
        ls.scanned = dir == GT_DIR_TOP_DOWN ? nf : (int64_t)s[CTR_SCANNED];
        ls.examined = (int64_t)s[CTR_EXAMINED];
        ls.examined_long = (int64_t)s[CTR_EXAMINED_LONG];
        ls.found_long = (int64_t)s[CTR_FOUND_LONG];
        ls.found = found;
        ls.ms = 0.f;
        ls.ms_main = 0.f;
        h->level[lev] = ls;
    }
    const int64_t mu = c->mu - fdeg;
    int ndir = dir;
    const int64_t visited = c->visited + found;
    if (dir == GT_DIR_TOP_DOWN) {
        if (fdeg > mu / alpha || fdeg > gamma * (n_t - visited)) ndir = GT_DIR_BOTTOM_UP;
    } else {
        if (found < nf && found <= n_t / beta) ndir = GT_DIR_TOP_DOWN;
    }
    if (dir == GT_DIR_TOP_DOWN && c->append) {
        c->src = 0;
        c->qi ^= 1;
    } else {
        c->src = 1;
    }
    c->cur ^= 1;
    c->nf = found;
    c->visited = visited;
    c->mf = fdeg;
    c->mu = mu;
    c->L += 1;
    c->lev = lev + 1;
    c->dir = ndir;
    c->append = fdeg <= td_small ? 1 : 0;
    c->done = found == 0 ? 1 : 0;
    h->lev = lev + 1;
    h->done = c->done;
}

__device__ __forceinline__ TdLevel td_from(const GCtl* __restrict__ c) {
    TdLevel t;
    t.cur = c->cur;
    t.qi = c->qi;
    t.next_level = c->L + 1;
    t.lev = c->lev;
    t.nf = c->nf;
    t.from_q = c->src == 0;
    t.append = c->append != 0;
    t.lvl = c->lvl;
    t.par = c->par;
    return t;
}

// One level, first kernel: top-down units or bottom-up words.
template <bool SPLIT>
__global__ void __launch_bounds__(BU_BLOCK) k_g_level(const GCtl* __restrict__ c, GArgs<SPLIT> a) {
    if (c->done) return;
    if (c->dir == GT_DIR_TOP_DOWN) {
        td_units<SPLIT>(td_from(c), a);
    } else {
        const int cur = c->cur;
        bu_level<SPLIT>(a.off, a.col, a.n, a.words, a.vis[cur], a.vis[cur ^ 1], c->lvl, c->par, c->L + 1,
                        a.hub_q, a.ctr + (c->lev & 1) * CTR_SET, a.bu_lane_edges, a.bu_hub_deg, a.hh, a.new2old,
                        0);
    }
}

// One level, second kernel: top-down chunks or bottom-up long rows.
template <bool SPLIT>
__global__ void __launch_bounds__(HUB_BLOCK) k_g_level_end(const GCtl* __restrict__ c, GArgs<SPLIT> a) {
    if (c->done) return;
    const int cur = c->cur;
    if (c->dir == GT_DIR_TOP_DOWN) {
        td_chunks<SPLIT>(td_from(c), a);
    } else {
        bu_hub_rows<SPLIT>(a.off, a.col, a.new2old, a.vis[cur], a.vis[cur ^ 1], c->lvl, c->par, c->L + 1, a.hub_q,
                           a.ctr + (c->lev & 1) * CTR_SET, a.bu_lane_edges);
    }
}

// Between levels: one wave. (A last-workgroup-done step inside the second
// kernel would need a device-scope fence in every workgroup, which writes
// back the L2 of each XCD and costs far more than this launch.)
__global__ void __launch_bounds__(GT_WAVE) k_g_ctl(GCtl* c, unsigned long long* ctr, GHost* h, int64_t n_t,
                                                   int32_t alpha, int32_t beta, int64_t td_small, int64_t gamma) {
    if (c->done) return;
    level_ctl(c, ctr, h, n_t, alpha, beta, td_small, gamma);
}

__global__ void k_g_anchor_bytes(const GCtl* __restrict__ c, int64_t n_anchor, const int32_t* __restrict__ anchor_core,
                                 const uint64_t* vis0, const uint64_t* vis1, const int2* __restrict__ lp_core,
                                 uint8_t* __restrict__ lvc) {
    if (!c->done) return;
    anchor_bytes(n_anchor, anchor_core, c->cur ? vis1 : vis0, lp_core, lvc);
}

__global__ void __launch_bounds__(OUT_BLOCK) k_g_output(
    const GCtl* __restrict__ c, int64_t n, const ClassGroup* __restrict__ groups, const uint64_t* vis0,
    const uint64_t* vis1, const uint8_t* __restrict__ lvc, const int2* __restrict__ lp_core,
    const int32_t* __restrict__ anchor_core, const int32_t* __restrict__ leaf_anchor,
    const int32_t* __restrict__ leaf_src_old, const int32_t* __restrict__ tdepth) {
    if (!c->done) return;
    split_output(n, groups, c->cur ? vis1 : vis0, lvc, lp_core, anchor_core, leaf_anchor, leaf_src_old, tdepth,
                 c->p.root, c->p.partner, c->p.parent_out, c->p.level_out);
}


// Grid of the first level kernel: one wave per BU_WPI bitmap words, at most
// bu_blocks workgroups.
unsigned level_grid(const gt_graph* g) {
    return grid_for((g->bfs.words + BU_WPI - 1) / BU_WPI, BU_BLOCK / GT_WAVE, g->tune.bu_blocks);
}

// Knobs that change what the graphs hold.
bool same_capture(const gt_tuning& a, const gt_tuning& b) {
    return a.alpha == b.alpha && a.beta == b.beta && a.bu_lane_edges == b.bu_lane_edges &&
           a.bu_hub_deg == b.bu_hub_deg && a.bu_blocks == b.bu_blocks && a.bu_hub_blocks == b.bu_hub_blocks &&
           a.td_small_edges == b.td_small_edges && a.td_blocks == b.td_blocks && a.bu_hint == b.bu_hint &&
           a.graph_levels == b.graph_levels && a.td_hub_deg == b.td_hub_deg && a.bu_gamma == b.bu_gamma;
}

template <bool SPLIT>
void enqueue_levels(gt_graph* g, bool with_init, hipStream_t s) {
    using T = int32_t;
    BfsScratch& b = g->bfs;
    GraphLoop& gl = b.gl;
    const gt_tuning& tu = g->tune;
    const int64_t n_t = g->tn();
    const int64_t* off = g->toff();
    const T* col = SPLIT ? (const T*)g->ccol.p : (const T*)g->col.p;
    const int32_t* n2o = SPLIT ? g->new2old.as<int32_t>() : nullptr;
    GCtl* c = gl.ctl.as<GCtl>();
    GHost* h = (GHost*)gl.host_dev;
    uint64_t* v0 = b.visit[0].as<uint64_t>();
    uint64_t* v1 = b.visit[1].as<uint64_t>();
    int32_t* q0 = b.queue[0].as<int32_t>();
    int32_t* q1 = b.queue[1].as<int32_t>();
    unsigned long long* ctr = b.ctr.as<unsigned long long>();
    int32_t* lvl = SPLIT ? b.level.as<int32_t>() : nullptr;
    int32_t* par = SPLIT ? b.level.as<int32_t>() + 1 : nullptr;  // the pair array: parent next to level
    if (with_init) {
        hipLaunchKernelGGL(k_g_setup, dim3(1), dim3(64), 0, s, h, c, g->tE(), lvl, par);
        const int64_t n_fill = SPLIT ? 0 : g->n;
        const int64_t span = std::max<int64_t>(b.words, n_fill);
        hipLaunchKernelGGL(k_g_init, dim3(grid_for(span, 256, 16384)), dim3(256), 0, s, (const GCtl*)c, v0, v1,
                           b.words, q0, ctr, n_fill);
    }
    GArgs<SPLIT> a;
    a.off = off;
    a.col = col;
    a.new2old = n2o;
    a.tdeg = b.tdeg.as<int32_t>();
    a.hh.hint = tu.bu_hint != 2 ? b.hint.as<int32_t>() : nullptr;
    a.hh.hint_orig = b.hint_orig.as<int32_t>();
    a.hh.hint2 = nullptr;  // the second probe is a host-driven-loop form (bu_hint 3 and 4 act as 1 here)
    a.hh.hint2_orig = b.hint2_orig.as<int32_t>();
    a.hh.small = b.small.as<uint64_t>();
    a.vis[0] = v0;
    a.vis[1] = v1;
    a.q[0] = q0;
    a.q[1] = q1;
    a.hub_q = b.hub_q.as<int32_t>();
    a.ctr = ctr;
    a.rows = b.td_rows.as<int2>();
    a.row_cap = b.td_row_cap;
    a.n = n_t;
    a.words = b.words;
    a.td_hub_deg = tu.td_hub_deg;
    a.bu_hub_deg = tu.bu_hub_deg;
    a.bu_lane_edges = tu.bu_lane_edges;
    for (int l = 0; l < tu.graph_levels; ++l) {
        hipLaunchKernelGGL((k_g_level<SPLIT>), dim3(level_grid(g)), dim3(BU_BLOCK), 0, s, (const GCtl*)c, a);
        hipLaunchKernelGGL((k_g_level_end<SPLIT>), dim3(tu.bu_hub_blocks), dim3(HUB_BLOCK), 0, s, (const GCtl*)c,
                           a);
        hipLaunchKernelGGL(k_g_ctl, dim3(1), dim3(GT_WAVE), 0, s, c, ctr, h, n_t, tu.alpha, tu.beta,
                           (int64_t)tu.td_small_edges, (int64_t)tu.bu_gamma);
    }
    if (SPLIT) {
        if (g->n_anchor > 0)  // level bytes are only read for leaves
            hipLaunchKernelGGL(k_g_anchor_bytes, dim3(grid_for(g->n_anchor, 256, 16384)), dim3(256), 0, s,
                               (const GCtl*)c, g->n_anchor, (const int32_t*)g->anchor_core.as<int32_t>(),
                               (const uint64_t*)v0, (const uint64_t*)v1, (const int2*)lvl, b.lv8.as<uint8_t>());
        hipLaunchKernelGGL(k_g_output, dim3(grid_for((g->n + OUT_ITEMS - 1) / OUT_ITEMS, OUT_BLOCK, 1 << 20)),
                           dim3(OUT_BLOCK), 0, s, (const GCtl*)c, g->n, g->groups.as<ClassGroup>(),
                           (const uint64_t*)v0, (const uint64_t*)v1, (const uint8_t*)b.lv8.as<uint8_t>(),
                           (const int2*)lvl, (const int32_t*)g->anchor_core.as<int32_t>(),
                           (const int32_t*)g->leaf_anchor.as<int32_t>(), g->leaf_src_old.as<int32_t>(),
                           (const int32_t*)g->tdepth.as<int32_t>());
    }
}

template <bool SPLIT>
gt_status capture(gt_graph* g, bool with_init, hipGraphExec_t* out) {
    GraphLoop& gl = g->bfs.gl;
    GT_HIP(hipStreamBeginCapture(gl.cap, hipStreamCaptureModeThreadLocal));
    enqueue_levels<SPLIT>(g, with_init, gl.cap);
    const hipError_t launch_err = hipGetLastError();
    hipGraph_t graph = nullptr;
    const hipError_t end_err = hipStreamEndCapture(gl.cap, &graph);
    if (launch_err != hipSuccess || end_err != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return gt_fail(GT_E_HIP, std::string("graph capture failed: ") +
                                     hipGetErrorString(launch_err != hipSuccess ? launch_err : end_err));
    }
    const hipError_t inst_err = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    GT_HIP(inst_err);
    return GT_OK;
}

template <bool SPLIT>
gt_status prepare(gt_graph* g, bool replay) {
    GraphLoop& gl = g->bfs.gl;
    if (!gl.ctl.p) {
        GT_TRY(gl.ctl.alloc(sizeof(GCtl)));
        GT_TRY(gl.host.alloc(sizeof(GHost), hipHostMallocMapped));
        std::memset(gl.host.p, 0, sizeof(GHost));
        GT_HIP(hipHostGetDevicePointer(&gl.host_dev, gl.host.p, 0));
        GT_HIP(hipStreamCreateWithFlags(&gl.cap, hipStreamNonBlocking));
        for (auto& e : gl.ev) GT_HIP(hipEventCreate(&e));
    }
    if (gl.valid && same_capture(gl.captured, g->tune)) return GT_OK;
    gl.drop_graphs();
    gl.captured = g->tune;
    // long rows of one level: rows longer than td_hub_deg (>= TD_CHUNK) are
    // at most E/TD_CHUNK; a small queue frontier (fewer than 8 vertices per
    // wave of the grid) adds at most its own size
    const int64_t cap = g->tE() / TD_CHUNK + 8 * (int64_t)level_grid(g) * (BU_BLOCK / GT_WAVE) + 64;
    if (cap > g->bfs.td_row_cap) {
        GT_TRY(g->bfs.td_rows.alloc(sizeof(int2) * (size_t)cap));
        g->bfs.td_row_cap = cap;
    }
    if (replay) {
        GT_TRY(capture<SPLIT>(g, true, &gl.first));
        GT_TRY(capture<SPLIT>(g, false, &gl.more));
        gl.valid = true;
    }
    return GT_OK;
}

template <bool SPLIT>
gt_status run(gt_graph* g, int32_t root, const RootPlan& rp, int32_t* parent_out, int32_t* level_out,
              hipStream_t s) {
    const bool replay = g->tune.loop == GT_LOOP_GRAPH;
    GT_TRY(prepare<SPLIT>(g, replay));
    GraphLoop& gl = g->bfs.gl;
    GHost* h = gl.host.as<GHost>();
    h->params.root = root;
    h->params.partner = rp.partner;
    h->params.seed = rp.seed;
    h->params.seed_level = rp.seed_level;
    h->params.seed_parent = rp.seed_parent;
    h->params.parent_out = parent_out;
    h->params.level_out = level_out;
    h->done = 0;
    h->lev = 0;
    const bool timing = g->tune.timing != 0;
    if (timing) GT_HIP(hipEventRecord(gl.ev[0], s));
    if (replay) {
        GT_HIP(hipGraphLaunch(gl.first, s));
    } else {
        enqueue_levels<SPLIT>(g, true, s);
        GT_HIP(hipGetLastError());
    }
    if (timing) GT_HIP(hipEventRecord(gl.ev[1], s));
    for (;;) {
        GT_HIP(hipStreamSynchronize(s));
        std::atomic_thread_fence(std::memory_order_acquire);
        if (__atomic_load_n(&h->done, __ATOMIC_ACQUIRE)) break;
        // every level discovers at least one vertex until the last
        if ((int64_t)__atomic_load_n(&h->lev, __ATOMIC_ACQUIRE) > g->tn() + 1)
            return gt_fail(GT_E_HIP, "device-driven traversal did not end");
        if (replay) {
            GT_HIP(hipGraphLaunch(gl.more, s));
        } else {
            enqueue_levels<SPLIT>(g, false, s);
            GT_HIP(hipGetLastError());
        }
        if (timing) GT_HIP(hipEventRecord(gl.ev[1], s));
    }
    gt_run_stats& st = g->stats;
    st.n_levels = h->lev;
    st.root_class = rp.root_class;
    st.ms_init = st.ms_output = 0.f;
    st.ms_total = 0.f;
    const int nl = std::min<int>(st.n_levels, GT_MAX_LEVELS);
    std::memcpy(st.level, h->level, sizeof(gt_level_stats) * (size_t)nl);
    if (timing) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, gl.ev[0], gl.ev[1]) == hipSuccess) st.ms_total = ms;
        else (void)hipGetLastError();
    }
    return GT_OK;
}

}  // namespace

gt_status gt_bfs_graph(gt_graph* g, int32_t root, const RootPlan& rp, int32_t* parent_out, int32_t* level_out,
                       hipStream_t s) {
    if (g->flags & GT_BUILD_SPLIT) return run<true>(g, root, rp, parent_out, level_out, s);
    return run<false>(g, root, rp, parent_out, level_out, s);
}
