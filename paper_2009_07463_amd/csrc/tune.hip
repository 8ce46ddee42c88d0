// Autotuner: chooses the knobs of gt_tuning for one graph handle by timed
// trials on the device, and keeps the result in an optional text cache keyed
// by a signature of the graph (its sizes and class counts), the library
// version and the device (architecture name and compute-unit count).
//
// Search: coordinate descent. Starting from the handle's current knobs, each
// knob in turn is set to each of its candidate values while the others stay
// at the best found so far; a value is kept when it lowers the measured time
// by more than 2%. The measured time of a setting is the smallest of three
// passes over the trial roots (gt_bfs, one call per root, wall clock around
// the pass, after one warm-up call). Every setting returns the same levels;
// only the speed differs.
//
// Cache file: one line per tuned (graph, device) pair,
//   <signature hex> <arch> key=value ...
// The last line with a matching signature and architecture wins; new
// results are appended.
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "gt_internal.h"

namespace {

struct Knob {
    const char* name;
    int32_t gt_tuning::*field;
    std::vector<int32_t> values;
    int loops;  // bit 1 << loop: loops for which the knob matters (0: all)
};

constexpr int L_HOST = 1 << GT_LOOP_HOST;
constexpr int L_DEV = (1 << GT_LOOP_GRAPH) | (1 << GT_LOOP_DEVICE);

const std::vector<Knob>& knobs() {
    static const std::vector<Knob> k = {
        {"loop", &gt_tuning::loop, {GT_LOOP_HOST, GT_LOOP_GRAPH, GT_LOOP_DEVICE}, 0},
        {"graph_levels", &gt_tuning::graph_levels, {4, 6, 8, 10, 12}, L_DEV},
        {"alpha", &gt_tuning::alpha, {10, 14, 17, 20, 24, 30}, 0},
        {"beta", &gt_tuning::beta, {12, 24, 48}, 0},
        {"bu_blocks", &gt_tuning::bu_blocks, {2048, 4096, 8192, 16384}, 0},
        {"bu_lane_edges", &gt_tuning::bu_lane_edges, {2, 4, 8}, 0},
        {"bu_hub_deg", &gt_tuning::bu_hub_deg, {1024, 4096, 16384}, 0},
        {"bu_hub_blocks", &gt_tuning::bu_hub_blocks, {1024, 4096, 8192}, 0},
        {"td_small_edges", &gt_tuning::td_small_edges, {16384, 65536, 262144}, 0},
        {"td_blocks", &gt_tuning::td_blocks, {4096, 16384, 65536}, L_HOST},
        {"td_hub_deg", &gt_tuning::td_hub_deg, {256, 1024, 4096}, L_DEV},
        {"bu_hint", &gt_tuning::bu_hint, {1, 2, 3, 4}, 0},
        {"bu_list_div", &gt_tuning::bu_list_div, {4, 8, 16, 64, 1 << 30}, L_HOST},
        {"td_flat", &gt_tuning::td_flat, {1, 2}, L_HOST},
        {"bu_lds", &gt_tuning::bu_lds, {1, 2}, L_HOST},
    };
    return k;
}

const std::vector<Knob>& ms_knobs() {
    static const std::vector<Knob> k = {
        {"ms_loop", &gt_tuning::ms_loop, {GT_LOOP_HOST, GT_LOOP_GRAPH, GT_LOOP_DEVICE}, 0},
        {"ms_blocks", &gt_tuning::ms_blocks, {1024, 2048, 4096, 8192, 16384}, 0},
        {"ms_alpha", &gt_tuning::ms_alpha, {14, 50, 100, 300, 1000}, 0},
    };
    return k;
}

// Knobs of the batched trials: the multi-source ones (step loop, grid,
// joining rule), the direction rule (each slot follows Beamer's rule with
// alpha and beta, whose best values for 64 roots at once differ from those
// for one root at a time) and the steps per graph replay.
const std::vector<Knob>& batch_descent_knobs() {
    static const std::vector<Knob> k = [] {
        std::vector<Knob> v;
        for (const Knob& kn : knobs())
            if (kn.field == &gt_tuning::alpha || kn.field == &gt_tuning::beta) v.push_back(kn);
        for (const Knob& kn : ms_knobs()) v.push_back(kn);
        // steps per replay of the device-driven batched loop
        v.push_back(Knob{"graph_levels", &gt_tuning::graph_levels, {4, 6, 8, 10, 12}, 0});
        return v;
    }();
    return k;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

gt_status device_name(std::string* arch, int* cus) {
    int dev = 0;
    GT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    GT_HIP(hipGetDeviceProperties(&prop, dev));
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a = a.substr(0, colon);  // drop feature suffixes
    *arch = a;
    *cus = prop.multiProcessorCount;
    return GT_OK;
}

uint64_t signature(const gt_graph* g, const std::string& arch, int cus) {
    uint64_t h = 1469598103934665603ull;
    const char* ver = gt_version();
    h = fnv1a(h, ver, std::strlen(ver));
    h = fnv1a(h, arch.data(), arch.size());
    h = fnv1a(h, &cus, sizeof(cus));
    const int64_t v[] = {(int64_t)g->flags, g->n, g->E, g->max_deg, g->n_core, g->n_leaf, g->n_zero, g->E_core};
    return fnv1a(h, v, sizeof(v));
}

std::string to_line(uint64_t sig, const std::string& arch, const gt_tuning& t, bool batch) {
    std::ostringstream os;
    char hex[32];
    std::snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)sig);
    os << hex << ' ' << arch;
    for (const Knob& k : knobs()) os << ' ' << k.name << '=' << t.*(k.field);
    if (batch)
        for (const Knob& k : ms_knobs()) os << ' ' << k.name << '=' << t.*(k.field);
    return os.str();
}

// Knobs of the last matching cache line applied to *t; false if none.
bool read_cache(const char* path, uint64_t sig, const std::string& arch, gt_tuning* t) {
    std::ifstream in(path);
    if (!in) return false;
    char hex[32];
    std::snprintf(hex, sizeof(hex), "%016llx", (unsigned long long)sig);
    std::string line, hit;
    while (std::getline(in, line)) {
        std::istringstream is(line);
        std::string s, a;
        if ((is >> s >> a) && s == hex && a == arch) hit = line;
    }
    if (hit.empty()) return false;
    std::istringstream is(hit);
    std::string tok;
    is >> tok >> tok;
    gt_tuning r = *t;
    while (is >> tok) {
        const size_t eq = tok.find('=');
        if (eq == std::string::npos) continue;
        const std::string key = tok.substr(0, eq);
        const int32_t val = (int32_t)std::strtol(tok.c_str() + eq + 1, nullptr, 10);
        for (const Knob& k : knobs())
            if (key == k.name) r.*(k.field) = val;
        for (const Knob& k : ms_knobs())
            if (key == k.name) r.*(k.field) = val;
    }
    *t = r;
    return true;
}

struct Trial {
    gt_graph* g;
    const int32_t* roots;
    int32_t k;
    int32_t* parent;
    int32_t* level;
    uint8_t* batch_out;
    void* stream;
};

constexpr int TRIAL_PASSES = 3;
constexpr double KEEP_BELOW = 0.99;  // a value is kept when it is this much faster

// Smallest of TRIAL_PASSES timed passes over the trial roots, in ms.
gt_status time_bfs(const Trial& tr, const gt_tuning& t, double* ms) {
    GT_TRY(gt_set_tuning(tr.g, &t));
    GT_TRY(gt_bfs(tr.g, tr.roots[0], tr.parent, tr.level, tr.stream));
    double best = 1e300;
    for (int rep = 0; rep < TRIAL_PASSES; ++rep) {
        const auto t0 = std::chrono::steady_clock::now();
        for (int32_t i = 0; i < tr.k; ++i) GT_TRY(gt_bfs(tr.g, tr.roots[i], tr.parent, tr.level, tr.stream));
        const auto t1 = std::chrono::steady_clock::now();
        best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    *ms = best;
    return GT_OK;
}

gt_status time_batch(const Trial& tr, const gt_tuning& t, double* ms) {
    GT_TRY(gt_set_tuning(tr.g, &t));
    GT_TRY(gt_bfs_batch(tr.g, tr.roots, tr.k, tr.batch_out, tr.stream));
    double best = 1e300;
    for (int rep = 0; rep < TRIAL_PASSES; ++rep) {
        const auto t0 = std::chrono::steady_clock::now();
        GT_TRY(gt_bfs_batch(tr.g, tr.roots, tr.k, tr.batch_out, tr.stream));
        GT_HIP(hipStreamSynchronize((hipStream_t)tr.stream));
        const auto t1 = std::chrono::steady_clock::now();
        best = std::min(best, std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    *ms = best;
    return GT_OK;
}

gt_status descend(const Trial& tr, const std::vector<Knob>& ks, bool batch, gt_tuning* best, double* best_ms,
                  int* trials) {
    for (const Knob& kn : ks) {
        if (kn.loops && !(kn.loops & (1 << best->loop))) continue;
        const int32_t start = best->*(kn.field);
        for (int32_t v : kn.values) {
            if (v == start) continue;
            gt_tuning cand = *best;
            cand.*(kn.field) = v;
            double ms = 0;
            GT_TRY(batch ? time_batch(tr, cand, &ms) : time_bfs(tr, cand, &ms));
            ++*trials;
            if (ms < KEEP_BELOW * *best_ms) {
                *best = cand;
                *best_ms = ms;
            }
        }
    }
    return GT_OK;
}

gt_status autotune(gt_graph* g, const int32_t* roots, int32_t k, const char* cache_path, uint32_t flags,
                   void* stream, gt_tuning* out, gt_tune_report* rep) {
    std::string arch;
    int cus = 0;
    GT_TRY(device_name(&arch, &cus));
    const uint64_t sig = signature(g, arch, cus);
    const bool batch = (flags & GT_TUNE_BATCH) != 0;
    gt_tuning start;
    GT_TRY(gt_get_tuning(g, &start));
    const int32_t user_timing = start.timing;
    gt_tune_report r{};
    r.signature = sig;
    if (cache_path && !(flags & GT_TUNE_FORCE)) {
        gt_tuning cached = start;
        if (read_cache(cache_path, sig, arch, &cached)) {
            GT_TRY(gt_set_tuning(g, &cached));
            r.from_cache = 1;
            if (out) *out = cached;
            if (rep) *rep = r;
            return GT_OK;
        }
    }
    DevBuf parent, level, bout;
    GT_TRY(parent.alloc(sizeof(int32_t) * (size_t)g->n));
    GT_TRY(level.alloc(sizeof(int32_t) * (size_t)g->n));
    if (batch) GT_TRY(bout.alloc((size_t)g->n * (size_t)k));
    Trial tr{g, roots, k, parent.as<int32_t>(), level.as<int32_t>(), bout.as<uint8_t>(), stream};
    gt_tuning best = start;
    best.timing = 0;
    double best_ms = 0;
    gt_status st = time_bfs(tr, best, &best_ms);
    r.ms_start = best_ms;
    if (st == GT_OK) st = descend(tr, knobs(), false, &best, &best_ms, &r.trials);
    r.ms_best = best_ms;
    if (st == GT_OK && batch) {
        double bms = 0;
        st = time_batch(tr, best, &bms);
        r.ms_batch_start = bms;
        // two sweeps: alpha and ms_alpha interact (a slot's direction and
        // when growing top-down slots join the pull), so one sweep can stop
        // short of the pair that is best together
        for (int sweep = 0; sweep < 2 && st == GT_OK; ++sweep)
            st = descend(tr, batch_descent_knobs(), true, &best, &bms, &r.trials);
        r.ms_batch_best = bms;
    }
    best.timing = user_timing;
    if (st != GT_OK) {
        const std::string msg = gt_last_error();
        (void)gt_set_tuning(g, &start);
        return gt_fail(st, "autotune trial failed: " + msg);
    }
    GT_TRY(gt_set_tuning(g, &best));
    if (cache_path) {
        std::ofstream os(cache_path, std::ios::app);
        if (!os) return gt_fail(GT_E_INVALID, std::string("cannot append to tuning cache ") + cache_path);
        os << to_line(sig, arch, best, batch) << '\n';
    }
    if (out) *out = best;
    if (rep) *rep = r;
    return GT_OK;
}

}  // namespace

extern "C" gt_status gt_autotune(gt_graph* g, const int32_t* roots_host, int32_t k, const char* cache_path,
                                 uint32_t flags, void* stream, gt_tuning* out, gt_tune_report* report) {
    if (!g || !roots_host) return gt_fail(GT_E_INVALID, "NULL argument");
    if (k < 1 || k > 64) return gt_fail(GT_E_INVALID, "k must be 1 .. 64");
    if (flags & ~(uint32_t)(GT_TUNE_FORCE | GT_TUNE_BATCH)) return gt_fail(GT_E_INVALID, "unknown flags");
    for (int32_t i = 0; i < k; ++i)
        if (roots_host[i] < 0 || (int64_t)roots_host[i] >= g->n) return gt_fail(GT_E_INVALID, "root out of range");
    return autotune(g, roots_host, k, cache_path, flags, stream, out, report);
}
