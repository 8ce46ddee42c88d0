// Batched multi-source BFS, parent reconstruction and sessions (placeholder
// entry points until the kernels land).
#include "gt_internal.h"

extern "C" gt_status gt_bfs_batch(gt_graph*, const int32_t*, int32_t, uint8_t*, void*) {
    return gt_fail(GT_E_UNSUPPORTED, "gt_bfs_batch: not built yet");
}
extern "C" gt_status gt_reconstruct_parent(gt_graph*, int32_t, const uint8_t*, int32_t*, void*) {
    return gt_fail(GT_E_UNSUPPORTED, "gt_reconstruct_parent: not built yet");
}
extern "C" gt_status gt_session_create(gt_graph*, int32_t, void*, gt_session**) {
    return gt_fail(GT_E_UNSUPPORTED, "sessions: not built yet");
}
extern "C" gt_status gt_session_admit(gt_session*, int32_t, uint8_t*, int32_t*) {
    return gt_fail(GT_E_UNSUPPORTED, "sessions: not built yet");
}
extern "C" gt_status gt_session_step(gt_session*, uint64_t*) {
    return gt_fail(GT_E_UNSUPPORTED, "sessions: not built yet");
}
extern "C" gt_status gt_session_active(const gt_session*, int32_t*) {
    return gt_fail(GT_E_UNSUPPORTED, "sessions: not built yet");
}
extern "C" gt_status gt_session_destroy(gt_session*) { return GT_OK; }
