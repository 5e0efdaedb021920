// Structure-factor refinement (placeholder until the kernels land).
#include "ar_internal.h"

extern "C" {

ar_status ar_sf_score_grad(ar_context *, const float *, const int64_t *, int64_t, const float *, const int32_t *,
                           const float *, int32_t, const float *, const float *, int32_t, int32_t, float *, float *,
                           void *)
{
    return ar::fail(AR_EUNSUPPORTED, "ar_sf_score_grad: not built yet");
}
ar_status ar_sf_score_f64(ar_context *, const float *, const int64_t *, int64_t, const double *, const int32_t *,
                          const float *, int32_t, const double *, const double *, int32_t, int32_t, double *, void *)
{
    return ar::fail(AR_EUNSUPPORTED, "ar_sf_score_f64: not built yet");
}
ar_status ar_sf_amplitudes(ar_context *, const float *, const int64_t *, int64_t, const float *, const int32_t *,
                           const float *, int32_t, const float *, int32_t, int32_t, float *, void *)
{
    return ar::fail(AR_EUNSUPPORTED, "ar_sf_amplitudes: not built yet");
}
ar_status ar_refine_orientations(ar_context *, const float *, const int64_t *, int64_t, float *, const int32_t *,
                                 const float *, int32_t, const float *, const float *, int32_t, int32_t, int32_t,
                                 float, float *, void *)
{
    return ar::fail(AR_EUNSUPPORTED, "ar_refine_orientations: not built yet");
}

}  // extern "C"
