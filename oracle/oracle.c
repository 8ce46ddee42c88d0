/*
 * CPU oracle for breadth-first search on an undirected graph.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code. The GPU library never
 * calls it, and it shares no code, header or table with the GPU library.
 *
 * Everything here is plain, single-threaded and written to be checked by
 * eye against its definition:
 *
 *  - oracle_csr_count / oracle_csr_fill: the undirected simple graph of an
 *    edge list as CSR (the paper's master data structure, Section 5.1.1):
 *    every edge {s, d} with s != d gives the entries s->d and d->s; rows are
 *    sorted ascending and repeated entries dropped.
 *  - oracle_bfs: level = hop distance from the root, parent = first
 *    discoverer, by a FIFO queue. This is the result Algorithm 1
 *    (direction-optimizing BFS) and Algorithm 9 (edge-tree BFS) compute:
 *    parent[root] = root, unreached vertices get -1 (Algorithm 5 writes -1
 *    for "no parent"), and every reached vertex's parent is a neighbour one
 *    level closer to the root (the Graph500 spanning-tree rule quoted in
 *    Section 5.3).
 *  - oracle_validate: checks any (parent, level) pair against that rule.
 *  - oracle_etvca: the edge-tree vertex classification of Algorithm 8,
 *    step by step in the paper's order, for any maximum height MH.
 *
 * Parent arrays are not unique (any neighbour one level closer is a valid
 * parent), so parity of parents is checked with oracle_validate only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/*
 * off has n+1 entries. On return off[0] = 0 and off[v+1] - off[v] is the
 * number of entries row v receives before duplicates are dropped (one per
 * edge end at v, self-loops excluded). Returns off[n], or -1 if some
 * endpoint lies outside [0, n).
 */
int64_t oracle_csr_count(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         int64_t* off) {
    for (int64_t v = 0; v <= n; ++v) off[v] = 0;
    for (int64_t e = 0; e < m; ++e) {
        int64_t s = src[e], d = dst[e];
        if (s < 0 || s >= n || d < 0 || d >= n) return -1;
        if (s == d) continue;
        off[s + 1] += 1;
        off[d + 1] += 1;
    }
    for (int64_t v = 0; v < n; ++v) off[v + 1] += off[v];
    return off[n];
}

/*
 * off must come from oracle_csr_count on the same edges; col must hold
 * off[n] entries. Returns the number of directed entries E (each undirected
 * edge counted twice) with rows sorted ascending and repeats dropped, or -1
 * on error. off is rewritten to the packed rows.
 *
 * Sorting is done without comparisons, by transposing twice:
 *  1. scatter every entry r->c into row r of a scratch array (rows unsorted);
 *  2. walk the scratch rows in ascending c and append c to row r of col for
 *     every entry r found in scratch row c. Because the graph is symmetric
 *     (entry r->c exists exactly when c->r does), row r of col receives
 *     every neighbour c, in ascending order of c.
 *  3. drop repeats within each row and pack rows to the front of col.
 */
int64_t oracle_csr_fill(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        int64_t* off, int32_t* col) {
    int64_t total = off[n];
    int64_t* next = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int32_t* scratch = (int32_t*)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    if (!next || !scratch) { free(next); free(scratch); return -1; }
    /* 1: unsorted rows in scratch */
    for (int64_t v = 0; v < n; ++v) next[v] = off[v];
    for (int64_t e = 0; e < m; ++e) {
        int64_t s = src[e], d = dst[e];
        if (s == d) continue;
        scratch[next[s]++] = (int32_t)d;
        scratch[next[d]++] = (int32_t)s;
    }
    /* 2: transpose: visiting c in ascending order fills every row sorted */
    for (int64_t v = 0; v < n; ++v) next[v] = off[v];
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = off[c]; i < off[c + 1]; ++i) {
            int64_t r = scratch[i];
            col[next[r]++] = (int32_t)c;
        }
    }
    free(scratch);
    free(next);
    /* 3: drop repeats, pack */
    int64_t out = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t b = off[v], e = off[v + 1];
        off[v] = out;
        for (int64_t i = b; i < e; ++i) {
            if (i == b || col[i] != col[i - 1]) col[out++] = col[i];
        }
    }
    off[n] = out;
    return out;
}

/*
 * FIFO breadth-first search from root. parent and level have n entries.
 * Returns the number of reached vertices, or -1 on a bad root / no memory.
 */
int64_t oracle_bfs(int64_t n, const int64_t* off, const int32_t* col, int32_t root,
                   int32_t* parent, int32_t* level) {
    if (root < 0 || root >= n) return -1;
    int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!queue) return -1;
    for (int64_t v = 0; v < n; ++v) { parent[v] = -1; level[v] = -1; }
    int64_t head = 0, tail = 0;
    parent[root] = root;
    level[root] = 0;
    queue[tail++] = root;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int64_t i = off[u]; i < off[u + 1]; ++i) {
            int32_t w = col[i];
            if (level[w] == -1) {
                level[w] = level[u] + 1;
                parent[w] = u;
                queue[tail++] = w;
            }
        }
    }
    free(queue);
    return tail;
}

static int row_has(const int64_t* off, const int32_t* col, int64_t v, int32_t u) {
    int64_t lo = off[v], hi = off[v + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < u) lo = mid + 1;
        else hi = mid;
    }
    return lo < off[v + 1] && col[lo] == u;
}

/*
 * Check a BFS result (rows of col must be sorted, as oracle_csr_fill makes
 * them). Returns 0 if valid, otherwise the number of the first failed rule
 * and the offending vertex in *bad:
 *   1: parent[root] == root and level[root] == 0
 *   2: for v != root, parent[v] == -1 exactly when level[v] == -1, and no
 *      other negative values
 *   3: for reached v != root, {parent[v], v} is an edge and
 *      level[parent[v]] == level[v] - 1
 *   4: for every edge {u, w}, both ends unreached, or both reached with
 *      levels at most 1 apart
 * Rules 1, 3 and 4 together force level[v] to equal the hop distance: rule
 * 3 gives a path of length level[v], rule 4 gives level[v] <= dist by
 * induction along a shortest path.
 */
int oracle_validate(int64_t n, const int64_t* off, const int32_t* col, int32_t root,
                    const int32_t* parent, const int32_t* level, int64_t* bad) {
    *bad = -1;
    if (root < 0 || root >= n) { *bad = root; return 1; }
    if (parent[root] != root || level[root] != 0) { *bad = root; return 1; }
    for (int64_t v = 0; v < n; ++v) {
        if (v == root) continue;
        int32_t p = parent[v], l = level[v];
        if ((p == -1) != (l == -1) || p < -1 || l < -1 || p >= n) { *bad = v; return 2; }
        if (p == -1) continue;
        if (!row_has(off, col, v, p) || level[p] != l - 1) { *bad = v; return 3; }
    }
    for (int64_t u = 0; u < n; ++u) {
        for (int64_t i = off[u]; i < off[u + 1]; ++i) {
            int32_t w = col[i];
            int32_t lu = level[u], lw = level[w];
            if ((lu == -1) != (lw == -1)) { *bad = u; return 4; }
            if (lu != -1 && (lu - lw > 1 || lw - lu > 1)) { *bad = u; return 4; }
        }
    }
    return 0;
}

/* Number of vertices of degree 0, of degree 1 and of degree >= 2. */
void oracle_degree_counts(int64_t n, const int64_t* off, int64_t counts[3]) {
    counts[0] = counts[1] = counts[2] = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = off[v + 1] - off[v];
        counts[d == 0 ? 0 : (d == 1 ? 1 : 2)] += 1;
    }
}

/* Sum of degrees over reached vertices (twice the traversed edge count). */
int64_t oracle_reached_degree_sum(int64_t n, const int64_t* off, const int32_t* level) {
    int64_t s = 0;
    for (int64_t v = 0; v < n; ++v)
        if (level[v] >= 0) s += off[v + 1] - off[v];
    return s;
}

/* Vertex types of Algorithm 8. */
enum { ET_CORE_INTERNAL = 0, ET_CORE_EDGE = 1, ET_TREE_INTERNAL = 2, ET_TREE_LEAF = 3,
       ET_VERTEX_ZERO = 4 };

/*
 * Algorithm 8 (edge-tree vertex classification). height = maximum edge-tree
 * height MH (0: leaves only; -1: no limit). type has n entries. Returns 0,
 * or -1 on no memory.
 *
 * Step 1: every vertex starts CORE_INTERNAL; degree 0 -> VERTEX_ZERO,
 *         degree 1 -> TREE_LEAF, whose neighbours lose one degree.
 * Step 2: per height round, with the degrees frozen at the start of the
 *         round, each still-CORE_INTERNAL vertex of degree 0 or 1 becomes
 *         TREE_INTERNAL and its neighbours lose one degree; rounds stop when
 *         a round marks nothing or the height limit is reached.
 * Step 3: a CORE_INTERNAL vertex whose degree changed is CORE_EDGE.
 */
int oracle_etvca(int64_t n, const int64_t* off, const int32_t* col, int height, uint8_t* type) {
    int64_t* deg_pre = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* deg_new = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    if (!deg_pre || !deg_new) { free(deg_pre); free(deg_new); return -1; }
    for (int64_t v = 0; v < n; ++v) {
        type[v] = ET_CORE_INTERNAL;
        deg_pre[v] = deg_new[v] = off[v + 1] - off[v];
    }
    int flag = 0;
    for (int64_t v = 0; v < n; ++v) {
        if (deg_pre[v] == 0) {
            type[v] = ET_VERTEX_ZERO;
        } else if (deg_pre[v] == 1) {
            type[v] = ET_TREE_LEAF;
            for (int64_t i = off[v]; i < off[v + 1]; ++i) deg_new[col[i]] -= 1;
            flag = 1;
        }
    }
    int h = 1;
    while (flag == 1 && (height == -1 || h <= height)) {
        flag = 0;
        memcpy(deg_pre, deg_new, (size_t)n * sizeof(int64_t));
        for (int64_t v = 0; v < n; ++v) {
            if (type[v] == ET_CORE_INTERNAL && (deg_pre[v] == 0 || deg_pre[v] == 1)) {
                type[v] = ET_TREE_INTERNAL;
                for (int64_t i = off[v]; i < off[v + 1]; ++i) deg_new[col[i]] -= 1;
                flag = 1;
            }
        }
        h += 1;
    }
    for (int64_t v = 0; v < n; ++v) {
        if (type[v] == ET_CORE_INTERNAL && deg_new[v] != off[v + 1] - off[v])
            type[v] = ET_CORE_EDGE;
    }
    free(deg_pre);
    free(deg_new);
    return 0;
}
