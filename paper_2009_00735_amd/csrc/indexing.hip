// Orientation indexing (placeholder until the correlation kernels land).
#include "ar_internal.h"

extern "C" {

ar_status ar_library_create(ar_context *, const float *, int64_t, int32_t, int32_t, void *, ar_library **out)
{
    if (out) *out = nullptr;
    return ar::fail(AR_EUNSUPPORTED, "ar_library_create: not built yet");
}
ar_status ar_library_destroy(ar_library *) { return AR_OK; }
ar_status index_orientations(ar_context *, const float *, int64_t, const ar_library *, int32_t, int32_t *, float *,
                             void *)
{
    return ar::fail(AR_EUNSUPPORTED, "index_orientations: not built yet");
}
ar_status index_orientations_ex(ar_context *, const float *, int64_t, const ar_library *, int32_t, int32_t,
                                int32_t *, float *, int32_t *, void *)
{
    return ar::fail(AR_EUNSUPPORTED, "index_orientations_ex: not built yet");
}

}  // extern "C"
