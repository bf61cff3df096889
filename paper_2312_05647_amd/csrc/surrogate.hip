// Surrogate MLP entry points (filled in with the matrix-core kernels).
#include "internal.h"

using namespace mjp;

extern "C" {
mjp_status mjp_surrogate_create(const mjp_mlp_cfg*, uint64_t, mjp_surrogate** out) {
    if (out) *out = nullptr;
    return fail(MJP_E_UNSUPPORTED, "surrogate not built yet");
}
void mjp_surrogate_destroy(mjp_surrogate*) {}
mjp_status mjp_surrogate_train(mjp_surrogate*, const float*, const float*, int32_t, const mjp_train_cfg*, float*,
                               mjp_stream_t) {
    return fail(MJP_E_UNSUPPORTED, "surrogate not built yet");
}
mjp_status mjp_surrogate_infer(const mjp_surrogate*, const float*, int32_t, float*, mjp_stream_t) {
    return fail(MJP_E_UNSUPPORTED, "surrogate not built yet");
}
int64_t mjp_surrogate_num_params(const mjp_surrogate*) { return 0; }
mjp_status mjp_surrogate_get_params(const mjp_surrogate*, float*, int64_t) {
    return fail(MJP_E_UNSUPPORTED, "surrogate not built yet");
}
mjp_status mjp_surrogate_set_params(mjp_surrogate*, const float*, int64_t) {
    return fail(MJP_E_UNSUPPORTED, "surrogate not built yet");
}
mjp_status mjp_surrogate_save(const mjp_surrogate*, const char*) {
    return fail(MJP_E_UNSUPPORTED, "surrogate not built yet");
}
mjp_status mjp_surrogate_load(const char*, mjp_surrogate** out) {
    if (out) *out = nullptr;
    return fail(MJP_E_UNSUPPORTED, "surrogate not built yet");
}


}
