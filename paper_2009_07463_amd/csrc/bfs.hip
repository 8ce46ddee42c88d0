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

#include "gt_internal.h"

namespace {

constexpr int TD_BLOCK = 256;
constexpr int BU_BLOCK = 256;
constexpr int OUT_BLOCK = 256;

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
    if (tid == 0) {
        for (int c = 0; c < 2 * CTR_N; ++c) ctr[c] = 0;
        if (seed >= 0) {
            q0[0] = seed;
            if (n_fill == 0) {
                level[seed] = seed_level;
                parent[seed] = seed_parent;
            }
        }
    }
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

__global__ void __launch_bounds__(TD_BLOCK) k_td_expand(
    const int32_t* __restrict__ q, int64_t nf, const int64_t* __restrict__ prefix,
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, uint64_t* visit,
    int32_t* __restrict__ level, int32_t* __restrict__ parent, int32_t next_level,
    int32_t* __restrict__ q_next, unsigned long long* __restrict__ ctr,
    unsigned long long* __restrict__ ctr_clear) {
    __shared__ int64_t s_lo, s_hi;
    const int64_t X = prefix[nf];
    if (blockIdx.x == 0 && threadIdx.x < CTR_N) ctr_clear[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctr[CTR_EXAMINED] = (unsigned long long)X;
    unsigned long long fdeg = 0;
    for (int64_t e0 = (int64_t)blockIdx.x * TD_BLOCK; e0 < X; e0 += (int64_t)gridDim.x * TD_BLOCK) {
        const int64_t e = e0 + threadIdx.x;
        if (threadIdx.x == 0) s_lo = first_greater(prefix, 1, nf, e0) - 1;
        if (threadIdx.x == 1) {
            const int64_t elast = (e0 + TD_BLOCK < X ? e0 + TD_BLOCK : X) - 1;
            s_hi = first_greater(prefix, 1, nf, elast) - 1;
        }
        __syncthreads();
        const int64_t lo = s_lo, hi = s_hi;
        __syncthreads();
        bool found = false;
        int32_t w = -1;
        if (e < X) {
            const int64_t i = first_greater(prefix, lo + 1, hi + 1, e) - 1;
            const int32_t u = q[i];
            w = col[off[u] + (e - prefix[i])];
            const uint64_t bit = 1ull << (w & 63);
            uint64_t* wp = visit + (w >> 6);
            if (!(*wp & bit)) {
                const uint64_t old = atomicOr((unsigned long long*)wp, (unsigned long long)bit);
                found = !(old & bit);
            }
            if (found) {
                level[w] = next_level;
                parent[w] = u;
                fdeg += (unsigned long long)(off[w + 1] - off[w]);
            }
        }
        const long long slot = wave_append(&ctr[CTR_FOUND], found);
        if (found) q_next[slot] = w;
    }
    wave_add(&ctr[CTR_FOUND_DEG], fdeg);
}

__global__ void __launch_bounds__(BU_BLOCK) k_bu(
    const int64_t* __restrict__ off, const int32_t* __restrict__ col, int64_t n, int64_t words,
    const uint64_t* __restrict__ vis_cur, uint64_t* __restrict__ vis_next,
    int32_t* __restrict__ level, int32_t* __restrict__ parent, int32_t next_level,
    int32_t* __restrict__ q_next, unsigned long long* __restrict__ ctr,
    unsigned long long* __restrict__ ctr_clear, int lane_edges) {
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * BU_BLOCK + threadIdx.x) / GT_WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * BU_BLOCK) / GT_WAVE;
    if (blockIdx.x == 0 && threadIdx.x < CTR_N) ctr_clear[threadIdx.x] = 0;
    unsigned long long fdeg = 0, scanned = 0, examined = 0;
    for (int64_t wd = gw; wd < words; wd += nwaves) {
        const uint64_t vis = vis_cur[wd];
        const int64_t v = wd * GT_WAVE + lane;
        const bool unvis = (v < n) && !((vis >> lane) & 1ull);
        if (__ballot(unvis) == 0) {
            if (lane == 0) vis_next[wd] = vis;
            continue;
        }
        bool found = false, pending = false;
        int32_t par = -1;
        int64_t b = 0, e = 0, k = 0;
        if (unvis) {
            b = off[v];
            e = off[v + 1];
            const int64_t lim = (e - b > lane_edges) ? b + lane_edges : e;
            for (k = b; k < lim; ++k) {
                const int32_t u = col[k];
                if ((vis_cur[u >> 6] >> (u & 63)) & 1ull) {
                    found = true;
                    par = u;
                    break;
                }
            }
            examined += (unsigned long long)(found ? k - b + 1 : lim - b);
            pending = !found && lim < e;
            scanned += 1;
        }
        // rows longer than lane_edges: the whole wave scans them, one at a time
        uint64_t pm = __ballot(pending);
        while (pm) {
            const int l = __ffsll((unsigned long long)pm) - 1;
            pm &= pm - 1;
            const int64_t cb = __shfl(k, l, GT_WAVE), ce = __shfl(e, l, GT_WAVE);
            int32_t hitu = -1;
            for (int64_t c = cb; c < ce; c += GT_WAVE) {
                const int64_t kk = c + lane;
                bool hit = false;
                int32_t u = 0;
                if (kk < ce) {
                    u = col[kk];
                    hit = (vis_cur[u >> 6] >> (u & 63)) & 1ull;
                }
                const uint64_t hm = __ballot(hit);
                if (hm) {
                    const int fl = __ffsll((unsigned long long)hm) - 1;
                    hitu = __shfl(u, fl, GT_WAVE);
                    if (lane == 0) examined += (unsigned long long)(fl + 1);
                    break;
                }
                if (lane == 0) examined += (unsigned long long)(ce - c < GT_WAVE ? ce - c : GT_WAVE);
            }
            if (lane == l && hitu >= 0) {
                found = true;
                par = hitu;
            }
        }
        const uint64_t fm = __ballot(found);
        if (lane == 0) vis_next[wd] = vis | fm;
        if (found) {
            level[v] = next_level;
            parent[v] = par;
            fdeg += (unsigned long long)(e - b);
        }
        const long long slot = wave_append(&ctr[CTR_FOUND], found);
        if (found) q_next[slot] = (int32_t)v;
    }
    wave_add(&ctr[CTR_FOUND_DEG], fdeg);
    wave_add(&ctr[CTR_SCANNED], scanned);
    wave_add(&ctr[CTR_EXAMINED], examined);
}

// SPLIT epilogue over caller ids v (ascending, coalesced writes):
//  v == root                -> (root, 0)
//  v == partner             -> (root, 1)   [the neighbour of a leaf root]
//  core, visited            -> (caller id of core parent, core level)
//  leaf, neighbour core and visited -> (neighbour, neighbour level + 1)
//  otherwise                -> (-1, -1)
__global__ void __launch_bounds__(OUT_BLOCK) k_split_output(
    int64_t n, const int32_t* __restrict__ old2new, int64_t n_core, int64_t n_leaf,
    const uint64_t* __restrict__ visit, const int32_t* __restrict__ level_core,
    const int32_t* __restrict__ parent_core, const int32_t* __restrict__ new2old,
    const int32_t* __restrict__ leaf_src_new, const int32_t* __restrict__ leaf_src_old,
    int32_t root, int32_t partner, int32_t* __restrict__ parent_out,
    int32_t* __restrict__ level_out) {
    const int64_t stride = (int64_t)gridDim.x * OUT_BLOCK;
    for (int64_t v = (int64_t)blockIdx.x * OUT_BLOCK + threadIdx.x; v < n; v += stride) {
        const int64_t nv = old2new[v];
        int32_t p = -1, l = -1;
        if (v == root) {
            p = root;
            l = 0;
        } else if (v == partner) {
            p = root;
            l = 1;
        } else if (nv < n_core) {
            if ((visit[nv >> 6] >> (nv & 63)) & 1ull) {
                l = level_core[nv];
                p = new2old[parent_core[nv]];
            }
        } else if (nv < n_core + n_leaf) {
            const int64_t j = nv - n_core;
            const int32_t s = leaf_src_new[j];
            if (s < n_core && ((visit[s >> 6] >> (s & 63)) & 1ull)) {
                l = level_core[s] + 1;
                p = leaf_src_old[j];
            }
        }
        parent_out[v] = p;
        level_out[v] = l;
    }
}

}  // namespace

gt_status gt_bfs_scratch_alloc(gt_graph* g) {
    BfsScratch& b = g->bfs;
    const int64_t n = g->tn();
    b.n = n;
    b.words = (n + 63) / 64;
    for (int i = 0; i < 2; ++i) {
        GT_TRY(b.visit[i].alloc(sizeof(uint64_t) * (b.words > 0 ? b.words : 1)));
        GT_TRY(b.queue[i].alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
    }
    GT_TRY(b.prefix.alloc(sizeof(int64_t) * (n + 1)));
    GT_TRY(b.scan_tmp.alloc(sizeof(int64_t) * scan_scratch_elems(n + 1)));
    if (g->flags & GT_BUILD_SPLIT) {
        GT_TRY(b.level.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
        GT_TRY(b.parent.alloc(sizeof(int32_t) * (n > 0 ? n : 1)));
    }
    GT_TRY(b.ctr.alloc(sizeof(unsigned long long) * 2 * CTR_N));
    GT_TRY(b.h_ctr.alloc(sizeof(unsigned long long) * 2 * CTR_N));
    b.ev.assign(2 * GT_MAX_LEVELS + 4, nullptr);
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

static gt_status bfs_run(gt_graph* g, int32_t root, int32_t* parent_out, int32_t* level_out,
                         hipStream_t s) {
    BfsScratch& b = g->bfs;
    const bool split = (g->flags & GT_BUILD_SPLIT) != 0;
    const bool timing = g->tune.timing != 0;
    const int64_t n_t = g->tn();
    const int64_t* off = g->toff();
    const int32_t* col = g->tcol();
    gt_run_stats& st = g->stats;
    st.n_levels = 0;
    st.root_class = 0;
    st.ms_init = st.ms_output = st.ms_total = 0.f;

    // Root handling (Algorithm 9): a leaf root is the parent of its only
    // neighbour, which seeds the core traversal at level 1; a leaf root whose
    // neighbour is a leaf (a two-vertex component) and an isolated root need
    // no core traversal at all.
    int32_t seed = root, seed_level = 0, partner = -1;
    if (split) {
        const int64_t nr = g->h_old2new[root];
        if (nr < g->n_core) {
            seed = (int32_t)nr;
        } else if (nr < g->n_core + g->n_leaf) {
            st.root_class = 1;
            const int64_t j = nr - g->n_core;
            partner = g->h_leaf_src_old[j];
            const int32_t sn = g->h_leaf_src_new[j];
            seed = sn < g->n_core ? sn : -1;
            seed_level = 1;
        } else {
            st.root_class = 2;
            seed = -1;
        }
    }
    int32_t* lvl = split ? b.level.as<int32_t>() : level_out;
    int32_t* par = split ? b.parent.as<int32_t>() : parent_out;
    int32_t* q[2] = {b.queue[0].as<int32_t>(), b.queue[1].as<int32_t>()};
    uint64_t* vis[2] = {b.visit[0].as<uint64_t>(), b.visit[1].as<uint64_t>()};
    unsigned long long* ctr = b.ctr.as<unsigned long long>();
    unsigned long long* h = b.h_ctr.as<unsigned long long>();
    hipEvent_t* ev = b.ev.data();
    const int EV_INIT0 = 0, EV_INIT1 = 1, EV_OUT0 = 2, EV_OUT1 = 3, EV_LVL = 4;

    if (timing) GT_HIP(hipEventRecord(ev[EV_INIT0], s));
    {
        const int64_t n_fill = split ? 0 : g->n;
        const int64_t span = std::max<int64_t>(b.words, n_fill);
        hipLaunchKernelGGL(k_bfs_init, dim3(grid_for(span, 256, 16384)), dim3(256), 0, s, vis[0],
                           b.words, seed, seed_level, split ? seed : root, lvl, par, q[0], ctr,
                           split ? (int32_t*)nullptr : level_out,
                           split ? (int32_t*)nullptr : parent_out, n_fill);
        GT_HIP(hipGetLastError());
    }
    if (timing) GT_HIP(hipEventRecord(ev[EV_INIT1], s));

    const int alpha = g->tune.alpha, beta = g->tune.beta;
    int cur = 0, qi = 0, lev = 0;
    int dir = GT_DIR_TOP_DOWN;  // a one-vertex frontier always starts top-down
    int64_t nf = seed >= 0 ? 1 : 0, mf = -1, mu = g->tE();
    int32_t L = seed_level;
    while (nf > 0) {
        const int set = lev & 1;
        unsigned long long* c_now = ctr + set * CTR_N;
        unsigned long long* c_next = ctr + (set ^ 1) * CTR_N;
        const bool rec = timing && lev < GT_MAX_LEVELS;
        if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 2 * lev], s));
        if (dir == GT_DIR_TOP_DOWN) {
            GT_TRY((scan_exclusive<int64_t, LoadFrontierDeg>(LoadFrontierDeg{q[qi], off}, nf,
                                                             b.prefix.as<int64_t>(),
                                                             b.scan_tmp.as<int64_t>(), s)));
            const unsigned blocks = mf >= 0 ? grid_for(mf, TD_BLOCK, 16384) : 1024u;
            hipLaunchKernelGGL(k_td_expand, dim3(blocks), dim3(TD_BLOCK), 0, s, q[qi], nf,
                               b.prefix.as<int64_t>(), off, col, vis[cur], lvl, par, L + 1, q[qi ^ 1],
                               c_now, c_next);
            GT_HIP(hipGetLastError());
        } else {
            const int64_t waves_per_block = BU_BLOCK / GT_WAVE;
            const unsigned blocks = grid_for(b.words, (int)waves_per_block, 1 << 20);
            hipLaunchKernelGGL(k_bu, dim3(blocks), dim3(BU_BLOCK), 0, s, off, col, n_t, b.words,
                               vis[cur], vis[cur ^ 1], lvl, par, L + 1, q[qi ^ 1], c_now, c_next,
                               g->tune.bu_lane_edges);
            GT_HIP(hipGetLastError());
            cur ^= 1;
        }
        if (rec) GT_HIP(hipEventRecord(ev[EV_LVL + 2 * lev + 1], s));
        GT_HIP(hipMemcpyAsync(h, c_now, sizeof(unsigned long long) * CTR_N, hipMemcpyDeviceToHost, s));
        GT_HIP(hipStreamSynchronize(s));
        const int64_t found = (int64_t)h[CTR_FOUND];
        const int64_t fdeg = (int64_t)h[CTR_FOUND_DEG];
        if (lev < GT_MAX_LEVELS) {
            gt_level_stats& ls = st.level[lev];
            ls.dir = dir;
            ls.frontier = nf;
            ls.scanned = dir == GT_DIR_TOP_DOWN ? nf : (int64_t)h[CTR_SCANNED];
            ls.examined = (int64_t)h[CTR_EXAMINED];
            ls.found = found;
            ls.ms = 0.f;
        }
        mu -= fdeg;
        if (dir == GT_DIR_TOP_DOWN) {
            if (fdeg > mu / alpha) dir = GT_DIR_BOTTOM_UP;
        } else {
            if (found < nf && found <= n_t / beta) dir = GT_DIR_TOP_DOWN;
        }
        nf = found;
        mf = fdeg;
        qi ^= 1;
        ++L;
        ++lev;
    }
    st.n_levels = lev;

    if (split) {
        if (timing) GT_HIP(hipEventRecord(ev[EV_OUT0], s));
        hipLaunchKernelGGL(k_split_output, dim3(grid_for(g->n, OUT_BLOCK, 1 << 20)), dim3(OUT_BLOCK), 0,
                           s, g->n, g->old2new.as<int32_t>(), g->n_core, g->n_leaf, vis[cur],
                           b.level.as<int32_t>(), b.parent.as<int32_t>(), g->new2old.as<int32_t>(),
                           g->leaf_src_new.as<int32_t>(), g->leaf_src_old.as<int32_t>(), root,
                           partner, parent_out, level_out);
        GT_HIP(hipGetLastError());
        if (timing) GT_HIP(hipEventRecord(ev[EV_OUT1], s));
    }
    GT_HIP(hipStreamSynchronize(s));
    if (timing) {
        st.ms_init = ev_ms(ev[EV_INIT0], ev[EV_INIT1]);
        for (int l = 0; l < lev && l < GT_MAX_LEVELS; ++l)
            st.level[l].ms = ev_ms(ev[EV_LVL + 2 * l], ev[EV_LVL + 2 * l + 1]);
        if (split) {
            st.ms_output = ev_ms(ev[EV_OUT0], ev[EV_OUT1]);
            st.ms_total = ev_ms(ev[EV_INIT0], ev[EV_OUT1]);
        } else {
            st.ms_total = lev > 0 ? ev_ms(ev[EV_INIT0], ev[EV_LVL + 2 * std::min(lev, GT_MAX_LEVELS) - 1])
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
    return bfs_run(g, root, parent_out, level_out, (hipStream_t)stream);
}

extern "C" gt_status gt_last_run_stats(const gt_graph* g, gt_run_stats* out) {
    if (!g || !out) return gt_fail(GT_E_INVALID, "NULL argument");
    *out = g->stats;
    return GT_OK;
}
