// Serving engine entry points (continuous batching). Implemented in a later
// revision; every call reports WF_E_STATE until then.
#include "runtime.h"

using namespace wf;

extern "C" {

wf_status wf_engine_create(int64_t, int, wf_engine** out) {
    if (out) *out = nullptr;
    return fail(WF_E_STATE, "serving engine not available in this build");
}
wf_status wf_engine_submit(wf_engine*, const wf_request*, uint64_t*) {
    return fail(WF_E_STATE, "serving engine not available in this build");
}
wf_status wf_engine_poll(wf_engine*, uint64_t*, wf_status*, int, int* n_done, int) {
    if (n_done) *n_done = 0;
    return fail(WF_E_STATE, "serving engine not available in this build");
}
wf_status wf_engine_stats(const wf_engine*, int64_t*, int64_t*, int64_t*, int64_t*) {
    return fail(WF_E_STATE, "serving engine not available in this build");
}
wf_status wf_engine_destroy(wf_engine*) { return WF_OK; }

}
