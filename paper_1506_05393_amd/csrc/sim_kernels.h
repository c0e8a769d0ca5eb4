// Host-side launchers shared between libmrf translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace mrf {
int launch_sim_dict(mrf_context* ctx, const Tables& t, int64_t k0, int64_t count,
                    mrf_dtype dtype, void* re, void* im, int64_t ld, double* norm, int unit_norm,
                    hipStream_t stream);
}  // namespace mrf
