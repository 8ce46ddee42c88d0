// Library-wide C entry points: errors, version, handle release, tuning.
#include <cstring>

#include "gt_internal.h"

namespace {
thread_local std::string t_last_error;
}

void gt_set_error(const std::string& msg) { t_last_error = msg; }

gt_status gt_fail(gt_status code, const std::string& msg) {
    t_last_error = msg;
    return code;
}

void gt_default_tuning(gt_tuning* t) {
    std::memset(t, 0, sizeof(*t));
    // Direction switch of Beamer et al. (reference [12] of the paper):
    // top-down -> bottom-up when the next frontier's edges exceed 1/alpha of
    // the unexplored edges; back when the frontier shrinks below n/beta.
    t->alpha = 14;
    t->beta = 24;
    t->bu_lane_edges = 4;
    t->bu_hub_deg = 4096;
    t->bu_blocks = 4096;
    t->bu_hub_blocks = 4096;
    t->td_small_edges = 65536;
    t->td_blocks = 16384;
    t->ms_blocks = 4096;
    t->ms_alpha = 50;
    t->timing = 1;
    t->bu_hint = 1;
    t->loop = GT_LOOP_HOST;
    t->graph_levels = 8;
    t->td_hub_deg = 256;
    t->bu_list_div = 16;
    t->td_flat = 1;
}

extern "C" const char* gt_last_error(void) { return t_last_error.c_str(); }

extern "C" const char* gt_version(void) { return "gt 0.1 gfx950"; }

extern "C" gt_status gt_graph_destroy(gt_graph* g) {
    if (!g) return GT_OK;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (auto& e : g->bfs.ev)
            if (e) (void)hipEventDestroy(e);
        g->bfs.ev.clear();
    }
    gt_batch_release(g);
    delete g;
    return GT_OK;
}

extern "C" gt_status gt_get_tuning(const gt_graph* g, gt_tuning* out) {
    if (!g || !out) return gt_fail(GT_E_INVALID, "NULL argument");
    *out = g->tune;
    return GT_OK;
}

extern "C" gt_status gt_set_tuning(gt_graph* g, const gt_tuning* in) {
    if (!g || !in) return gt_fail(GT_E_INVALID, "NULL argument");
    if (in->loop > GT_LOOP_DEVICE) return gt_fail(GT_E_INVALID, "loop must be GT_LOOP_HOST, _GRAPH or _DEVICE");
    if (in->graph_levels > 64) return gt_fail(GT_E_INVALID, "graph_levels must be 1 .. 64");
    if (in->td_hub_deg > 0 && in->td_hub_deg < 256) return gt_fail(GT_E_INVALID, "td_hub_deg must be >= 256");
    if (in->bu_hint > 2) return gt_fail(GT_E_INVALID, "bu_hint must be 1 or 2");
    if (in->td_flat > 2) return gt_fail(GT_E_INVALID, "td_flat must be 1 or 2");
    std::lock_guard<std::mutex> lk(g->mu);
    gt_tuning& t = g->tune;
    if (in->alpha > 0) t.alpha = in->alpha;
    if (in->beta > 0) t.beta = in->beta;
    if (in->bu_lane_edges > 0) t.bu_lane_edges = in->bu_lane_edges;
    if (in->bu_hub_deg > 0) t.bu_hub_deg = in->bu_hub_deg;
    if (in->bu_blocks > 0) t.bu_blocks = in->bu_blocks;
    if (in->bu_hub_blocks > 0) t.bu_hub_blocks = in->bu_hub_blocks;
    if (in->td_small_edges > 0) t.td_small_edges = in->td_small_edges;
    if (in->td_blocks > 0) t.td_blocks = in->td_blocks;
    if (in->ms_blocks > 0) t.ms_blocks = in->ms_blocks;
    if (in->ms_alpha > 0) t.ms_alpha = in->ms_alpha;
    if (in->timing >= 0) t.timing = in->timing;
    if (in->bu_hint > 0) t.bu_hint = in->bu_hint;
    if (in->loop > 0) t.loop = in->loop;
    if (in->graph_levels > 0) t.graph_levels = in->graph_levels;
    if (in->td_hub_deg > 0) t.td_hub_deg = in->td_hub_deg;
    if (in->bu_list_div > 0) t.bu_list_div = in->bu_list_div;
    if (in->td_flat > 0) t.td_flat = in->td_flat;
    return GT_OK;
}
