// Adjoint of L = sum |a|^2 through density and force.
#include <hip/hip_runtime.h>

#include "sph_internal.hpp"

using namespace sph;

extern "C" {

sph_status sph_adjoint_ws_bytes(const sph_plan *plan, size_t *bytes)
{
    (void)plan;
    (void)bytes;
    return fail(SPH_E_UNSUPPORTED, "adjoint not built yet");
}

sph_status sph_adjoint_forward(const sph_plan *, const double *, const float *, const float *, const float *,
                               const float *, const float *, const float *, const sph_params *, float *, float *,
                               float *, float *, void *, size_t, void *)
{
    return fail(SPH_E_UNSUPPORTED, "adjoint not built yet");
}

sph_status sph_force_adjoint(const sph_plan *, const double *, const float *, const float *, const float *,
                             const float *, const float *, const float *, const float *, const float *,
                             const sph_params *, const float *, float *, float *, float *, float *, float *, void *,
                             size_t, void *)
{
    return fail(SPH_E_UNSUPPORTED, "adjoint not built yet");
}

sph_status sph_density_adjoint(const sph_plan *, const double *, const float *, const float *, const float *,
                               const float *, float *, float *, void *, size_t, void *)
{
    return fail(SPH_E_UNSUPPORTED, "adjoint not built yet");
}
}
