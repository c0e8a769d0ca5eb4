// BF16 brute-force matching with FP32 re-scoring of the top candidates.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "match_kernels.h"

namespace mrf {
size_t bf16_workspace_bytes(const mrf_dict_view*, int32_t, int32_t, int) { return 256; }
int match_bf16(mrf_context*, const mrf_dict_view*, const void*, int32_t, int64_t, int32_t,
               const mrf_sequence*, const mrf_grid*, mrf_result_view, int64_t*, float*, void*,
               size_t, hipStream_t) {
  set_error("BF16 matching is not built yet");
  return MRF_ERR_UNSUPPORTED;
}
}  // namespace mrf
