/*
 * gt -- low-degree-split ("edge leaf view") breadth-first search on AMD
 * Instinct MI355X (gfx950). C ABI.
 *
 * The method follows C. Zhang, "A New Perspective of Graph Data and A Generic
 * and Efficient Method for Large Scale Graph Data Traversal" (arXiv
 * 2009.07463): vertices of degree 0 (VERTEX_ZERO) and degree 1 (TREE_LEAF)
 * are split off the graph (Section 4.3, Algorithm 8 with MH = 0), the
 * remaining core is relabelled so its vertices are contiguous (Section
 * 5.1.1), direction-optimizing BFS (Section 2.1, Algorithm 1) runs on the
 * core only, and one sequential pass over the leaves gives each leaf its
 * parent and level (Section 5.3, Algorithm 7 "TEOLV"; driver Algorithm 9).
 *
 * Conventions shared by every call:
 *  - Vertex ids are int32 in the caller's labelling, 0 <= id < n_vertices.
 *  - The graph is undirected; self-loops and repeated edges are ignored.
 *  - Pointers documented as "device" must point to device memory of the
 *    current HIP device (for example a torch tensor's data_ptr()); "host"
 *    pointers are ordinary CPU memory. The library never keeps a caller
 *    pointer after a call returns.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).
 *  - Every call returns a gt_status. On failure nothing has been written to
 *    caller outputs unless stated, no memory is leaked, and gt_last_error()
 *    returns a message for the calling thread.
 *  - Calls on one graph handle are serialised by the library (each handle
 *    owns one set of traversal buffers); use several handles or sessions for
 *    concurrency.
 */
#ifndef GT_H
#define GT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gt_graph gt_graph;     /* opaque, owned by the library */
typedef struct gt_session gt_session; /* opaque, owned by the library */

typedef enum {
    GT_OK = 0,
    GT_E_INVALID = -1,     /* bad argument or input (checked before any work is queued) */
    GT_E_NOMEM = -2,       /* device or host allocation failed */
    GT_E_HIP = -3,         /* a HIP runtime call failed; see gt_last_error() */
    GT_E_DEPTH = -4,       /* a batched level would not fit in uint8 (depth > 254) */
    GT_E_BUSY = -5,        /* no free slot / memory budget in a session */
    GT_E_UNSUPPORTED = -6  /* the handle was not built for this call */
} gt_status;

/* Build flags. A PLAIN handle keeps the whole graph and runs
 * direction-optimizing BFS on it; a SPLIT handle keeps the core subgraph and
 * the leaf list and runs the edge-tree BFS. GT_BUILD_RMZERO (SPLIT plus the
 * KEEP_LEAVES bit) is the ablation that removes only the isolated vertices
 * (the RmZero optimisation of the comparisons in Sections 6.2-6.4, Fig. 5):
 * degree-1 vertices stay in the core and there is no leaf pass. All return
 * identical levels. */
enum { GT_BUILD_PLAIN = 0u, GT_BUILD_SPLIT = 1u, GT_BUILD_KEEP_LEAVES = 2u, GT_BUILD_RMZERO = 3u };
/* GT_BUILD_RELABELLED (RMZERO plus the KEEP_ZERO bit): nothing is split off.
 * The whole graph goes through the SPLIT machinery -- relabelled, traversed
 * and written back in caller ids -- so with GT_BUILD_HUBS_FIRST it is plain
 * direction-optimizing BFS on the hubs-first numbering, the like-for-like
 * baseline of a hubs-first SPLIT handle. KEEP_ZERO without RMZERO is
 * GT_E_INVALID. */
enum { GT_BUILD_KEEP_ZERO = 8u, GT_BUILD_RELABELLED = 11u };
/* Maximum edge-tree height MH of a SPLIT handle (Algorithm 8; bits 8..15 of
 * the flags). 0, the default, is the edge leaf view: degree-1 vertices only.
 * h in 1..254 also moves TREE_INTERNAL vertices (peeled in rounds 1..h) into
 * the trees; 255 peels until nothing changes (the paper's MH = -1). The tree
 * vertices then take the place of the leaves everywhere (n_leaf counts them)
 * and the leaf pass becomes the edge-tree pass of Algorithm 10. */
#define GT_BUILD_MH(h) ((uint32_t)((h) & 0xFF) << 8)
#define GT_BUILD_MH_ALL GT_BUILD_MH(255)
/* SPLIT core numbering. By default the core is numbered in ascending caller
 * id. GT_BUILD_HUBS_FIRST numbers the hubs (the core vertices of highest
 * degree, about 1/16 of the core) first and the other core vertices after
 * them, each group in ascending caller id, so that the frontier masks and
 * bitmap bits of the most probed vertices share few cache lines (the layout
 * the degree-aware bottom-up of Section 2.3 favours); the output pass
 * still writes every result in caller-id order (hubs form a class of their
 * own in its 64-id groups). Results are the same. */
#define GT_BUILD_HUBS_FIRST 4u
/* With GT_BUILD_HUBS_FIRST: the hubs are the core vertices of degree at
 * least the smallest threshold that leaves at most n_core / 2^k of them
 * (k = 1..15; 0, the default, means k = 4). Without GT_BUILD_HUBS_FIRST a
 * non-zero share is rejected (GT_E_INVALID). */
#define GT_BUILD_HUB_SHARE(k) ((uint32_t)((k) & 0xF) << 16)

typedef struct {
    int64_t n_vertices;     /* N */
    int64_t n_input_edges;  /* edges in the list given to gt_build_graph */
    int64_t n_entries;      /* directed CSR entries of the simple graph (2 x edges) */
    int64_t max_degree;
    int64_t n_core;         /* vertices of degree >= 2 (the core; SPLIT only, else N;
                               RMZERO: degree >= 1; MH > 0: CORE_INTERNAL + CORE_EDGE) */
    int64_t n_leaf;         /* degree-1 vertices (TREE_LEAF; 0 for RMZERO; MH > 0: all
                               tree vertices, TREE_LEAF + TREE_INTERNAL) */
    int64_t n_zero;         /* degree-0 vertices (VERTEX_ZERO) */
    int64_t n_core_entries; /* directed entries of the core subgraph */
    int64_t n_leaf_pairs;   /* leaves whose only neighbour is also a leaf */
    int64_t device_bytes;   /* device memory held by the handle */
    double build_ms;        /* wall time of gt_build_graph */
    uint32_t flags;         /* GT_BUILD_* */
    uint32_t tree_height;   /* MH > 0: peeling rounds that found TREE_INTERNAL vertices */
    int64_t n_tree_internal;/* MH > 0: TREE_INTERNAL vertices (else 0) */
    int64_t n_core_edge;    /* MH > 0: CORE_EDGE vertices, core vertices with a tree
                               neighbour (else 0) */
    /* Edge trees grouped by their core-edge vertex (Section 4.5, Table 3):
     * the tree vertices (n_leaf of them; TREE_LEAF and, for MH > 0,
     * TREE_INTERNAL) whose path to the core ends at one core vertex count as
     * one edge tree of that vertex. Trees with no core vertex (a pair of
     * leaves, a path or star component) belong to none. SPLIT handles only,
     * else 0; min is 0 when there is no edge tree. */
    int64_t n_edge_trees;   /* core vertices with at least one tree vertex */
    int64_t edge_tree_vertices; /* tree vertices in those edge trees */
    int64_t edge_tree_max;  /* tree vertices of the largest edge tree */
    int64_t edge_tree_min;  /* tree vertices of the smallest edge tree */
} gt_graph_info;

#define GT_MAX_LEVELS 512

/* Direction of one BFS level. */
enum { GT_DIR_TOP_DOWN = 0, GT_DIR_BOTTOM_UP = 1 };

/* Kernel that ran the main part of a BFS level. */
enum {
    GT_KERNEL_TD_EDGES = 0,  /* top-down from a queue, one adjacency entry per thread */
    GT_KERNEL_TD_FLAT = 1,   /* top-down, 64 frontier vertices per wave, long rows in chunks */
    GT_KERNEL_BU_WORDS = 2,  /* bottom-up over all bitmap words */
    GT_KERNEL_BU_LIST = 3    /* bottom-up over the list of still-unvisited vertices */
};

typedef struct {
    int32_t dir;          /* GT_DIR_* */
    int32_t kernel;       /* GT_KERNEL_* */
    int64_t frontier;     /* vertices in the level's input frontier */
    int64_t scanned;      /* top-down: frontier vertices; bottom-up: unvisited vertices tested */
    int64_t examined;     /* adjacency entries read (a bottom-up probe of the
                             highest-degree neighbour counts as one) */
    int64_t found;        /* vertices discovered by the level */
    float ms;             /* device time of the level's kernels (HIP events) */
    float ms_main;        /* device time of the level's main kernel alone: the
                             top-down expand or the bottom-up word kernel
                             (gt_bfs_batch: the pull kernel, with the step's
                             finalize, of a step with pulled slots, else 0) */
    int64_t examined_long;/* bottom-up: of `examined`, entries read by the
                             long-row kernel after the main one (else 0) */
    int64_t found_long;   /* bottom-up: of `found`, vertices it discovered */
} gt_level_stats;

typedef struct {
    int32_t n_levels;     /* levels run on the (core) graph */
    int32_t root_class;   /* 0 core (or PLAIN), 1 leaf, 2 isolated */
    float ms_init;        /* output/bitmap initialisation kernel */
    float ms_output;      /* SPLIT: output + leaf pass kernel; PLAIN: 0 */
    float ms_total;       /* first to last event of the call */
    gt_level_stats level[GT_MAX_LEVELS];
} gt_run_stats;

/* Tuning knobs (see gt_get_tuning for defaults). In gt_set_tuning, a value
 * <= 0 keeps the current setting (timing: < 0 keeps it). */
typedef struct {
    int32_t alpha;            /* top-down -> bottom-up when m_f > m_u / alpha */
    int32_t beta;             /* bottom-up -> top-down when n_f < n / beta and shrinking */
    int32_t bu_lane_edges;    /* bottom-up: entries a lane scans alone before the wave helps */
    int32_t bu_hub_deg;       /* bottom-up: rows longer than this get a whole workgroup */
    int32_t bu_blocks;        /* bottom-up: workgroups (grid-stride over bitmap words) */
    int32_t bu_hub_blocks;    /* bottom-up: workgroups of the long-row kernel */
    int32_t td_small_edges;   /* top-down levels with at most this many frontier entries
                                 append discoveries to a queue; larger ones only claim
                                 bitmap bits and the queue is compacted from the bitmap */
    int32_t td_blocks;        /* top-down: maximum workgroups of the expand kernel */
    int32_t ms_blocks;        /* batched BFS: workgroups per level kernel */
    int32_t timing;           /* 1: record HIP events per level (gt_last_run_stats.ms) */
    int32_t bu_hint;          /* 1: bottom-up probes each vertex's highest-degree neighbour
                                 first, from a dense per-vertex array (degree-aware
                                 bottom-up, Section 2.3); 3: also the second-highest for the
                                 vertices the first probe missed, and a vertex of degree <= 2
                                 that both missed is settled without reading its row (host-
                                 driven loop; the device-driven loops treat 3 as 1); 4: as 3
                                 on levels whose frontier is under 1% of the traversed
                                 vertices, as 1 on the others (host-driven loop; 1 in the
                                 device-driven loops); 2: off */
    int32_t loop;             /* gt_bfs level loop: GT_LOOP_HOST, GT_LOOP_GRAPH or
                                 GT_LOOP_DEVICE */
    int32_t graph_levels;     /* GT_LOOP_GRAPH / GT_LOOP_DEVICE: levels per captured graph or
                                 per batch of launches (1 .. 64) */
    int32_t td_hub_deg;       /* GT_LOOP_GRAPH / GT_LOOP_DEVICE top-down: frontier rows longer
                                 than this (>= 256) are cut into 256-entry chunks spread over
                                 the grid */
    int32_t bu_list_div;      /* GT_LOOP_HOST bottom-up: once at most n / bu_list_div vertices
                                 are unvisited, they are listed once and later bottom-up
                                 levels test only the listed vertices (a large value: never) */
    int32_t td_flat;          /* GT_LOOP_HOST top-down after a level that left its
                                 discoveries only in the bitmap: 1 = read the frontier from
                                 the bitmap difference, 64 vertices per wave, long rows in
                                 chunks; 2 = compact it into a queue and expand edge by edge */
    int32_t ms_alpha;         /* batched BFS: in a step where some slots pull, a top-down slot
                                 whose frontier grew joins them once m_f > m_u / ms_alpha
                                 (a value <= alpha: never) */
    int32_t bu_gamma;         /* gt_bfs: top-down -> bottom-up also when the next frontier's
                                 edges exceed bu_gamma times the unvisited vertices (the
                                 probe of the highest-degree neighbour makes a bottom-up
                                 level cost about one test per unvisited vertex);
                                 2^30 (default): never. Not searched by gt_autotune: on a
                                 frontier of a few thousand vertices it picks bottom-up
                                 levels several times slower than top-down */
    int32_t ms_loop;          /* gt_bfs_batch step loop: GT_LOOP_HOST (the host reads each
                                 step's counters and picks the next step's kernels),
                                 GT_LOOP_GRAPH (default: per-slot directions decided on the
                                 device, graph_levels steps captured once in a HIP graph and
                                 replayed, one host synchronisation per replay) or
                                 GT_LOOP_DEVICE (the same kernels launched one by one) */
    int32_t bu_lds;           /* bottom-up on a hubs-first handle: 1 (default) = the hubs'
                                 visited bits (core ids [0, n_hub), up to the LDS a workgroup
                                 may hold) are copied into each workgroup's LDS and probed
                                 there, with a grid of the workgroups resident at once;
                                 2 = every probe reads the global bitmap */
    int32_t bu_form;          /* GT_LOOP_HOST bottom-up kernel: 1 (default) = a wave per
                                 64-vertex word, unsettled rows spread over the wave's lanes;
                                 2 = Algorithm 5 as written, one thread per word walking its
                                 unvisited bits; 3 = one thread per vertex. 2 and 3 exist to
                                 measure form 1 against; they take no list mode and no long-row
                                 kernel, and give the same levels. Not searched by gt_autotune */
} gt_tuning;

/* Level loop of gt_bfs.
 *  GT_LOOP_HOST   the host reads the level's counters after every level
 *                 (one stream synchronisation per level), chooses the
 *                 direction and launches the next level's kernels; per-level
 *                 device times are recorded when timing = 1.
 *  GT_LOOP_GRAPH  the direction rule runs on the device between levels and
 *                 every kernel reads its level's parameters from device
 *                 memory, so a fixed sequence of graph_levels levels is
 *                 captured once in a HIP graph and replayed per call; the
 *                 host synchronises once per replay (once per call when the
 *                 BFS depth fits). Levels and counters are the same as with
 *                 GT_LOOP_HOST; per-level device times are not recorded.
 *  GT_LOOP_DEVICE the kernels of GT_LOOP_GRAPH launched on the stream one by
 *                 one instead of replayed from a graph: the device starts on
 *                 the first kernel while the host enqueues the rest. */
enum { GT_LOOP_HOST = 1, GT_LOOP_GRAPH = 2, GT_LOOP_DEVICE = 3 };

/*
 * Build a graph handle from an undirected edge list.
 *   src, dst   device, n_edges int32 each: edge e joins src[e] and dst[e].
 *              Ids outside [0, n_vertices) make the call fail with
 *              GT_E_INVALID (detected on the device).
 *   n_vertices 1 .. 2^31 - 1. Vertices that appear in no edge are isolated.
 *   flags      GT_BUILD_PLAIN, GT_BUILD_SPLIT, GT_BUILD_RMZERO or
 *              GT_BUILD_RELABELLED; SPLIT may carry GT_BUILD_MH(h), and any
 *              of the SPLIT kinds GT_BUILD_HUBS_FIRST (KEEP_LEAVES without
 *              SPLIT, KEEP_ZERO without KEEP_LEAVES, or MH with KEEP_LEAVES
 *              or without SPLIT, is GT_E_INVALID).
 *   out        host; receives the handle.
 * The CSR build (Section 5.1.1) symmetrises, drops self-loops and repeats
 * and sorts rows. SPLIT then classifies by degree (Algorithm 8, MH = 0),
 * relabels so core vertices come first, leaves next and isolated vertices
 * last, each class in ascending caller-id order (Section 5.1.1 layout), and
 * keeps the core CSR, the relabel maps and the leaf list (Section 5.1.2).
 * Synchronous: returns after the build finished on `stream`.
 */
gt_status gt_build_graph(const int32_t* src, const int32_t* dst, int64_t n_edges,
                         int64_t n_vertices, uint32_t flags, void* stream, gt_graph** out);

/* Release a handle and all device memory it holds. NULL is allowed. */
gt_status gt_graph_destroy(gt_graph* g);

/* Sizes and counts of a handle (host struct). */
gt_status gt_graph_info_get(const gt_graph* g, gt_graph_info* out);

/* Degree of every vertex in the simple graph.
 *   deg_out  device, n_vertices int32, caller ids. Stream-ordered. */
gt_status gt_graph_degrees(const gt_graph* g, int32_t* deg_out, void* stream);

/*
 * Single-source BFS (Algorithm 1 on the whole graph for PLAIN, Algorithm 9
 * for SPLIT).
 *   root        caller id, 0 <= root < n_vertices.
 *   parent_out  device, n_vertices int32: parent[root] = root; for a reached
 *               v != root, a neighbour of v one level closer to the root;
 *               -1 if v is unreached. The choice among valid parents may
 *               differ between runs.
 *   level_out   device, n_vertices int32: hop distance from root, -1 if
 *               unreached. Deterministic.
 * Every entry of both outputs is written. Runs on `stream` and returns after
 * the outputs are complete. With the host-driven loop (GT_LOOP_HOST) the
 * call blocks on the stream once per BFS level (the direction decision reads
 * the level's counters); with GT_LOOP_GRAPH / GT_LOOP_DEVICE the direction
 * rule runs on the device and the call blocks once per graph_levels levels.
 * Every loop serves every kind of handle. For handles built with
 * GT_BUILD_MH(h > 0), a root inside an edge tree first walks its tree to the
 * core-edge vertex on the host (Algorithm 9), and the other vertices of that
 * tree are written from the walk after the traversal.
 */
gt_status gt_bfs(gt_graph* g, int32_t root, int32_t* parent_out, int32_t* level_out,
                 void* stream);

/*
 * gt_bfs without allocation, for callers that cannot allocate device memory
 * during a call (code under stream capture, tight serving loops, harnesses
 * that forbid hipMalloc). Same arguments, outputs, semantics and errors as
 * gt_bfs, with these differences:
 *  - The traversal's working memory (visited bitmaps, frontier queues, the
 *    top-down prefix sums, the core (level, parent) pairs and counters) comes
 *    from one static device array of GT_BFS_STATIC_MAX_BYTES per GPU, which
 *    the loader places with the library's code object and which lives until
 *    the process ends. The call makes no device or pinned-host allocation
 *    and frees nothing; graph-owned arrays (CSR, degrees, hints) are read as
 *    in gt_bfs.
 *  - A handle whose traversed graph (n = n_core for SPLIT, n_vertices for
 *    PLAIN; E its adjacency entries) needs more than that array holds, about
 *    32.25 * n + E / 32 bytes plus one byte per core vertex with leaves
 *    attached and alignment, is refused with GT_E_INVALID
 *    before anything is enqueued (a scale-22 Kronecker core fits; use gt_bfs
 *    for larger graphs). Handles built with GT_BUILD_MH(h > 0) are refused
 *    with GT_E_UNSUPPORTED.
 *  - It always runs the host-driven level loop (one stream sync per level),
 *    whatever the handle's `loop` knob says.
 *  - Every call on a GPU shares that GPU's array, which keeps the last call's
 *    contents; each call clears what must start empty. Calls from one
 *    process are serialised per device by the library; two calls that
 *    overlapped on one GPU would race on the array.
 */
#define GT_BFS_STATIC_MAX_BYTES (64ull << 20)
gt_status gt_bfs_static(gt_graph* g, int32_t root, int32_t* parent_out, int32_t* level_out,
                        void* stream);

/* Counters and per-level device times of the last gt_bfs or gt_bfs_batch on
 * g (host struct). For a batch (root_class = -1), one entry per step: dir =
 * GT_DIR_TOP_DOWN for a push-only step (kernel GT_KERNEL_TD_EDGES),
 * GT_DIR_BOTTOM_UP for a step with a pull over all vertices
 * (GT_KERNEL_BU_WORDS); frontier = slots pushed in the step; scanned = slots
 * pulled; examined = adjacency entries the pull read; found = (vertex, slot)
 * pairs discovered; ms_main = the pull kernel, which also runs the step's
 * finalize; ms_output = the transpose/leaf-pass kernel. */
gt_status gt_last_run_stats(const gt_graph* g, gt_run_stats* out);

/* Read / change tuning of a handle (host structs). */
gt_status gt_get_tuning(const gt_graph* g, gt_tuning* out);
gt_status gt_set_tuning(gt_graph* g, const gt_tuning* in);

/*
 * Batched multi-source BFS: k roots traversed together, one bit per root in a
 * 64-bit mask per vertex.
 *   roots_host  host, k caller ids (repeats allowed), 1 <= k <= 64.
 *   levels_out  device, k * n_vertices uint8, root-major: levels_out[r*N + v]
 *               = hop distance from roots_host[r] to v, 255 if unreached.
 * Returns GT_E_DEPTH (outputs unspecified) if some distance exceeds 254.
 * Works on PLAIN and SPLIT handles (with GT_BUILD_MH(h) too: a tree vertex
 * gets its core-edge vertex's level plus its depth, and a root inside a tree
 * gets that tree from the walk of gt_bfs). Blocks on the stream once per
 * level.
 */
gt_status gt_bfs_batch(gt_graph* g, const int32_t* roots_host, int32_t k, uint8_t* levels_out,
                       void* stream);

/*
 * Parent array from a level array (as made by gt_bfs_batch for one root).
 *   level_in    device, n_vertices uint8 (255 = unreached).
 *   parent_out  device, n_vertices int32: parent[root] = root; for a reached
 *               v, its first neighbour u in ascending id order with
 *               level[u] = level[v] - 1; -1 if unreached.
 */
gt_status gt_reconstruct_parent(gt_graph* g, int32_t root, const uint8_t* level_in,
                                int32_t* parent_out, void* stream);

/*
 * int32 levels (as gt_bfs writes them, -1 = unreached) to the uint8
 * encoding of gt_bfs_batch (255 = unreached), so that single-root answers
 * and batched ones share one format (the serving layer uses this).
 *   level_in   device, n int32.   out: device, n uint8.   n >= 0.
 * GT_E_DEPTH (out unspecified) if some level exceeds 254. Blocks on the
 * stream (it reads back that check).
 */
gt_status gt_levels_to_u8(const int32_t* level_in, int64_t n, uint8_t* out, void* stream);

/*
 * Continuous-batching session over one graph: up to `slots` (1..64) queries
 * run together in one multi-source BFS; queries admitted while others run
 * join at the next level boundary, and finished slots are refilled.
 *   gt_session_create  stream: the session's stream; out: host.
 *   gt_session_admit   root: caller id; level_out: device, n_vertices uint8,
 *                      owned by the caller and written when the query
 *                      finishes (255 = unreached); slot_out: host, may be
 *                      NULL. GT_E_BUSY if all slots are taken.
 *   gt_session_step    runs one BFS level for every active query, then
 *                      finalises finished ones; *finished_slots_out (host)
 *                      receives their slot bits. Blocks on the stream.
 *   gt_session_active  number of running queries.
 * A query's result equals gt_bfs_batch of its root alone. A session depth
 * beyond 254 levels returns GT_E_DEPTH for the affected step.
 */
gt_status gt_session_create(gt_graph* g, int32_t slots, void* stream, gt_session** out);
gt_status gt_session_admit(gt_session* s, int32_t root, uint8_t* level_out, int32_t* slot_out);
gt_status gt_session_step(gt_session* s, uint64_t* finished_slots_out);
gt_status gt_session_active(const gt_session* s, int32_t* active_out);
gt_status gt_session_destroy(gt_session* s);

/*
 * Autotuning of the knobs of g (gt_tuning) by timed trials on the device.
 * Coordinate descent from the current knobs: each knob in turn takes each
 * of its candidate values (level loop, levels per graph, alpha, beta, grid
 * sizes, long-row thresholds, ...) and a value is kept when the fastest of
 * three passes of gt_bfs over the trial roots gets more than 1% faster
 * than the best so far; GT_TUNE_BATCH then also tunes the batched BFS
 * (alpha, beta, ms_blocks, ms_alpha; two sweeps) on the fastest of three
 * gt_bfs_batch of the trial roots, so alpha and beta end up chosen for the
 * batch. Every setting returns the same levels; only the speed differs. The
 * result is applied to g (its timing setting is kept).
 *   roots_host  host, k caller ids (1 <= k <= 64): the trial workload.
 *   cache_path  host string or NULL. A text file with one line per tuned
 *               (graph signature, device): "<signature> <arch> key=value ...".
 *               The signature hashes the library version, the device's
 *               architecture name and compute-unit count, the build flags
 *               and the graph's sizes and class counts. Without
 *               GT_TUNE_FORCE a matching line is applied and no trial runs;
 *               a new result is appended.
 *   out, report host, may be NULL: the chosen knobs; how they were found.
 * Blocks until done (each trial synchronises the stream). Allocates and
 * frees its own trial outputs (8 bytes per vertex, plus k per vertex with
 * GT_TUNE_BATCH).
 */
enum { GT_TUNE_FORCE = 1u, GT_TUNE_BATCH = 2u };

typedef struct {
    uint64_t signature;     /* cache key of the graph and device */
    int32_t from_cache;     /* 1: applied from the cache, no trials */
    int32_t trials;         /* timed settings tried */
    double ms_start;        /* gt_bfs pass over the roots with the starting knobs */
    double ms_best;         /* ... with the chosen knobs */
    double ms_batch_start;  /* gt_bfs_batch of the roots (GT_TUNE_BATCH) */
    double ms_batch_best;
} gt_tune_report;

gt_status gt_autotune(gt_graph* g, const int32_t* roots_host, int32_t k, const char* cache_path,
                      uint32_t flags, void* stream, gt_tuning* out, gt_tune_report* report);

/*
 * Measurement helpers (not on the traversal path): what the device says about
 * itself, and a hand-written streaming copy whose rate is the achievable HBM
 * bandwidth the traversal kernels are compared with.
 */
typedef struct {
    char arch[64];             /* gcnArchName, e.g. "gfx950:sramecc+:xnack-" */
    char name[64];             /* marketing name */
    int32_t compute_units;
    int32_t clock_khz;         /* shader clock */
    int32_t memory_clock_khz;  /* as hipDeviceProp_t reports it */
    int32_t memory_bus_bits;
    int64_t l2_bytes;          /* L2 of one XCD as reported */
    int64_t total_bytes;       /* device memory */
    double peak_hbm_gbs;       /* 2 * memory_clock_khz * 1e3 * memory_bus_bits / 8 / 1e9
                                  (double data rate), GB/s */
} gt_device_props;

/* Properties of HIP device `device` (host struct). GT_E_INVALID for a device
 * number that does not exist. */
gt_status gt_device_props_get(int32_t device, gt_device_props* out);

/* dst[0 .. n_bytes) = src[0 .. n_bytes) with 16-byte non-temporal loads and
 * stores, grid-stride, on `stream` (not synchronised). src and dst: device,
 * 16-byte aligned, not overlapping; n_bytes a multiple of 16 (else
 * GT_E_INVALID). */
gt_status gt_stream_copy(const void* src, void* dst, int64_t n_bytes, void* stream);

/* Device memory held by the library, all handles, sessions and devices
 * together (host int64). */
gt_status gt_memory_in_use(int64_t* bytes_out);

/* Cap on gt_memory_in_use: a device allocation of the library that would
 * take it past `bytes` fails with GT_E_NOMEM as if the device were full (the
 * call that needed it returns GT_E_NOMEM, leaks nothing, and a failed
 * gt_build_graph returns no handle). 0 (the default) removes the cap.
 * Process-wide; lowering it frees nothing already held. */
gt_status gt_set_memory_limit(int64_t bytes);

/* Message for the last failing call on this thread ("" if none). */
const char* gt_last_error(void);

/* Library version string. */
const char* gt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GT_H */
