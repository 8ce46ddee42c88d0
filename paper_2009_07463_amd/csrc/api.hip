// Library-wide C entry points: errors, version, handle release, tuning.
#include <atomic>
#include <cstring>

#include "gt_internal.h"

namespace {
thread_local std::string t_last_error;

typedef int v4i __attribute__((ext_vector_type(4)));

// Streaming copy: four independent 16-byte loads in flight per thread,
// non-temporal on both sides (nothing is reused).
__global__ void __launch_bounds__(256) k_stream_copy(const v4i* __restrict__ src, v4i* __restrict__ dst,
                                                     int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const v4i a = __builtin_nontemporal_load(src + i);
        const v4i b = __builtin_nontemporal_load(src + i + stride);
        const v4i c = __builtin_nontemporal_load(src + i + 2 * stride);
        const v4i d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}
}  // namespace

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
    t->bu_gamma = 1 << 30;
    t->ms_loop = GT_LOOP_GRAPH;
    t->bu_lds = 1;
    t->bu_form = 1;
}

namespace {
std::atomic<int64_t> g_live_bytes{0};   // device bytes the library holds, all devices
std::atomic<int64_t> g_limit_bytes{0};  // 0: no limit
}  // namespace

gt_status gt_dev_malloc(void** p, size_t bytes) {
    *p = nullptr;
    const int64_t b = (int64_t)bytes;
    const int64_t lim = g_limit_bytes.load();
    const int64_t after = g_live_bytes.fetch_add(b) + b;
    if (lim > 0 && after > lim) {
        g_live_bytes.fetch_sub(b);
        return gt_fail(GT_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes would exceed the " +
                                       "library's memory limit of " + std::to_string(lim) + " bytes");
    }
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        g_live_bytes.fetch_sub(b);
        (void)hipGetLastError();
        return gt_fail(GT_E_NOMEM, "hipMalloc(" + std::to_string(bytes) + ") failed: " + hipGetErrorString(e));
    }
    return GT_OK;
}

void gt_dev_free(void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    g_live_bytes.fetch_sub((int64_t)bytes);
}

extern "C" gt_status gt_set_memory_limit(int64_t bytes) {
    if (bytes < 0) return gt_fail(GT_E_INVALID, "the limit must be >= 0");
    g_limit_bytes.store(bytes);
    return GT_OK;
}

extern "C" gt_status gt_memory_in_use(int64_t* bytes_out) {
    if (!bytes_out) return gt_fail(GT_E_INVALID, "NULL argument");
    *bytes_out = g_live_bytes.load();
    return GT_OK;
}

extern "C" const char* gt_last_error(void) { return t_last_error.c_str(); }

extern "C" gt_status gt_device_props_get(int32_t device, gt_device_props* out) {
    if (!out) return gt_fail(GT_E_INVALID, "NULL argument");
    int count = 0;
    GT_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return gt_fail(GT_E_INVALID, "no such device");
    hipDeviceProp_t p;
    GT_HIP(hipGetDeviceProperties(&p, device));
    std::memset(out, 0, sizeof(*out));
    std::strncpy(out->arch, p.gcnArchName, sizeof(out->arch) - 1);
    std::strncpy(out->name, p.name, sizeof(out->name) - 1);
    out->compute_units = p.multiProcessorCount;
    out->clock_khz = p.clockRate;
    out->memory_clock_khz = p.memoryClockRate;
    out->memory_bus_bits = p.memoryBusWidth;
    out->l2_bytes = p.l2CacheSize;
    out->total_bytes = (int64_t)p.totalGlobalMem;
    out->peak_hbm_gbs = 2.0 * (double)p.memoryClockRate * 1e3 * (double)p.memoryBusWidth / 8.0 / 1e9;
    return GT_OK;
}

extern "C" gt_status gt_stream_copy(const void* src, void* dst, int64_t n_bytes, void* stream) {
    if (n_bytes < 0 || (n_bytes & 15)) return gt_fail(GT_E_INVALID, "n_bytes must be a non-negative multiple of 16");
    if (n_bytes == 0) return GT_OK;
    if (!src || !dst) return gt_fail(GT_E_INVALID, "NULL argument");
    if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return gt_fail(GT_E_INVALID, "pointers must be 16-byte aligned");
    const int64_t n16 = n_bytes / 16;
    const unsigned blocks = grid_for((n16 + 3) / 4, 256, 8192);
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const v4i*>(src), static_cast<v4i*>(dst), n16);
    GT_HIP(hipGetLastError());
    return GT_OK;
}

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
    if (in->bu_hint > 4) return gt_fail(GT_E_INVALID, "bu_hint must be 1, 2, 3 or 4");
    if (in->td_flat > 2) return gt_fail(GT_E_INVALID, "td_flat must be 1 or 2");
    if (in->ms_loop > GT_LOOP_DEVICE) return gt_fail(GT_E_INVALID, "ms_loop must be GT_LOOP_HOST, _GRAPH or _DEVICE");
    if (in->bu_lds > 2) return gt_fail(GT_E_INVALID, "bu_lds must be 1 or 2");
    if (in->bu_form > 3) return gt_fail(GT_E_INVALID, "bu_form must be 1, 2 or 3");
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
    if (in->bu_gamma > 0) t.bu_gamma = in->bu_gamma;
    if (in->ms_loop > 0) t.ms_loop = in->ms_loop;
    if (in->bu_lds > 0) t.bu_lds = in->bu_lds;
    if (in->bu_form > 0) t.bu_form = in->bu_form;
    return GT_OK;
}
