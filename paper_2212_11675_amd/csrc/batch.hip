// Batched form (many systems, k right-hand sides): not yet implemented in this translation unit.
#include "gsr_internal.hpp"

using namespace gsr;

extern "C" {

gsr_status gsr_batch_setup(int32_t, const gsr_dims*, const int64_t*, const double*,
                           const int32_t*, const int32_t*, const int32_t*, int32_t,
                           const gsr_setup_opts*, void*, gsr_batch** out) {
    if (out) *out = nullptr;
    return fail(GSR_E_UNSUPPORTED, "batched solve not available");
}
gsr_status gsr_batch_destroy(gsr_batch*) { return GSR_OK; }
gsr_status gsr_batch_col_offsets(const gsr_batch*, int64_t*) {
    return fail(GSR_E_UNSUPPORTED, "batched solve not available");
}
gsr_status gsr_batch_aprod1(gsr_batch*, const double*, double*, void*) {
    return fail(GSR_E_UNSUPPORTED, "batched solve not available");
}
gsr_status gsr_batch_aprod2(gsr_batch*, const double*, double*, void*) {
    return fail(GSR_E_UNSUPPORTED, "batched solve not available");
}
gsr_status gsr_batch_solve(gsr_batch*, const double*, double*, const gsr_solve_opts*,
                           gsr_solve_info*, void*) {
    return fail(GSR_E_UNSUPPORTED, "batched solve not available");
}

}  // extern "C"
