/*
 * Seeded synthetic inputs: Kronecker (R-MAT) edge lists and BFS root samples.
 *
 * This module only makes inputs. It holds none of the traversal method's
 * arithmetic (no CSR, no degree classes, no BFS) and is shared by the CPU
 * oracle, the tests and the benchmark.
 *
 * Edge model (Section 6.1 of the paper: Graph500 Kronecker generator with
 * A=0.57, B=C=0.19, D=0.05, 2^scale vertices, edgefactor*2^scale edges):
 * every endpoint bit of every edge is drawn independently; one uniform
 * 32-bit draw per bit level picks the quadrant (src bit, dst bit) =
 * (0,0) with probability A, (0,1) with B, (1,0) with C and (1,1) with D,
 * using integer thresholds floor(p * 2^32). No noise is added. Labels are
 * then scrambled by a keyed bijection of [0, 2^scale) so that vertex id
 * carries no degree information.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) used as a counter-based
 * generator: draw(key, i) = mix64(key + (i + 1) * gamma), where mix64 is the
 * SplitMix64 output finaliser. Output is independent of the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GG_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t gg_draw(uint64_t key, uint64_t i) {
    return gg_mix64(key + (i + 1) * GG_GAMMA);
}

/* Distinct streams of one seed: edges, label scrambling, roots. */
static inline uint64_t gg_stream_key(uint64_t seed, uint64_t stream) {
    return gg_mix64(gg_mix64(seed ^ 0x5851F42D4C957F2DULL) + stream * GG_GAMMA);
}

uint64_t gg_random_u64(uint64_t seed, uint64_t stream, uint64_t i) {
    return gg_draw(gg_stream_key(seed, stream), i);
}

/* Keyed bijection of [0, 2^scale): rounds of odd multiply, xorshift and
 * add, each a permutation of scale-bit integers. */
typedef struct {
    uint64_t mask;
    int shift;
    uint64_t mul[4];
    uint64_t add[4];
} gg_perm;

static void gg_perm_init(gg_perm* p, int scale, uint64_t seed) {
    uint64_t key = gg_stream_key(seed, 1);
    p->mask = (scale >= 64) ? ~0ULL : ((1ULL << scale) - 1ULL);
    p->shift = (scale + 1) / 2;
    if (p->shift < 1) p->shift = 1;
    for (int r = 0; r < 4; ++r) {
        p->mul[r] = gg_draw(key, 2 * r) | 1ULL;
        p->add[r] = gg_draw(key, 2 * r + 1);
    }
}

static inline uint64_t gg_perm_apply(const gg_perm* p, uint64_t x) {
    for (int r = 0; r < 4; ++r) {
        x = (x * p->mul[r]) & p->mask;
        x ^= x >> p->shift;
        x = (x + p->add[r]) & p->mask;
    }
    return x;
}

/* Scrambled label of vertex x (exported for tests of the bijection). */
int64_t gg_scramble(int scale, uint64_t seed, int64_t x) {
    gg_perm p;
    gg_perm_init(&p, scale, seed);
    return (int64_t)gg_perm_apply(&p, (uint64_t)x);
}

/*
 * Fill src[m], dst[m] (int32) with edges [first, first + m) of the seeded
 * R-MAT stream. prob[4] = {A, B, C, D}. Returns 0, or -1 on bad arguments.
 * permute != 0 scrambles labels.
 */
int gg_kronecker_edges(int scale, int64_t first, int64_t m, const double prob[4],
                       uint64_t seed, int permute, int32_t* src, int32_t* dst) {
    if (scale < 1 || scale > 31 || m < 0 || first < 0) return -1;
    double pa = prob[0], pab = prob[0] + prob[1], pabc = prob[0] + prob[1] + prob[2];
    if (pa < 0 || pab < pa || pabc < pab || pabc > 1.0) return -1;
    const uint64_t two32 = 4294967296ULL;
    uint64_t ta = (uint64_t)(pa * (double)two32);
    uint64_t tab = (uint64_t)(pab * (double)two32);
    uint64_t tabc = (uint64_t)(pabc * (double)two32);
    const uint64_t key = gg_stream_key(seed, 0);
    const int ndraw = (scale + 1) / 2;
    gg_perm perm;
    gg_perm_init(&perm, scale, seed);

#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint64_t ge = (uint64_t)(first + e);
        uint64_t s = 0, d = 0;
        for (int j = 0; j < ndraw; ++j) {
            uint64_t r = gg_draw(key, ge * (uint64_t)ndraw + (uint64_t)j);
            for (int h = 0; h < 2; ++h) {
                int bit = 2 * j + h;
                if (bit >= scale) break;
                uint64_t u = h ? (r >> 32) : (r & 0xFFFFFFFFULL);
                /* quadrant: [0,ta) -> (0,0), [ta,tab) -> (0,1),
                 * [tab,tabc) -> (1,0), [tabc,2^32) -> (1,1); branch-free */
                uint64_t sb = (uint64_t)(u >= tab);
                uint64_t db = (uint64_t)((u >= ta) & (u < tab)) | (uint64_t)(u >= tabc);
                s |= sb << bit;
                d |= db << bit;
            }
        }
        if (permute) {
            s = gg_perm_apply(&perm, s);
            d = gg_perm_apply(&perm, d);
        }
        src[e] = (int32_t)s;
        dst[e] = (int32_t)d;
    }
    return 0;
}

/*
 * Draw k distinct roots, uniformly among vertices that touch at least one
 * edge whose endpoints differ (degree >= 1 once self-loops and duplicates
 * are dropped). Deterministic in seed. Returns the number drawn (< k only
 * if fewer such vertices exist), or -1 on bad arguments / no memory.
 */
int64_t gg_sample_roots(int64_t n, int64_t m, const int32_t* src, const int32_t* dst,
                        uint64_t seed, int64_t k, int32_t* roots) {
    if (n <= 0 || m < 0 || k < 0) return -1;
    uint8_t* touched = (uint8_t*)calloc((size_t)n, 1);
    uint8_t* taken = (uint8_t*)calloc((size_t)n, 1);
    if (!touched || !taken) { free(touched); free(taken); return -1; }
    int64_t n_touched = 0;
    for (int64_t e = 0; e < m; ++e) {
        int32_t s = src[e], d = dst[e];
        if (s == d || s < 0 || d < 0 || s >= n || d >= n) continue;
        if (!touched[s]) { touched[s] = 1; ++n_touched; }
        if (!touched[d]) { touched[d] = 1; ++n_touched; }
    }
    int64_t want = k < n_touched ? k : n_touched;
    const uint64_t key = gg_stream_key(seed, 2);
    int64_t got = 0;
    for (uint64_t t = 0; got < want; ++t) {
        uint64_t r = gg_draw(key, t);
        int64_t c = (int64_t)(((unsigned __int128)r * (unsigned __int128)(uint64_t)n) >> 64);
        if (touched[c] && !taken[c]) {
            taken[c] = 1;
            roots[got++] = (int32_t)c;
        }
    }
    free(touched);
    free(taken);
    return got;
}
