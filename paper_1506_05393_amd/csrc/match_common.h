// Device helpers shared by the FP32 and BF16 matching kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrf {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bool beats(float s, int32_t i, float t, int32_t j) {
  return s > t || (s == t && i < j);
}

// Insert (s, e) into a list sorted best first (LDS, lanes < kk own one
// position each). Called in wave-uniform control flow.
__device__ __forceinline__ void list_insert(float* ls, int32_t* li, int kk, int lane, float s,
                                            int32_t e) {
  float cs = -1.0f;
  int32_t ci = 0x7fffffff;
  if (lane < kk) {
    cs = ls[lane];
    ci = li[lane];
  }
  const bool ahead = (lane < kk) && beats(cs, ci, s, e);
  const int p = __popcll(__ballot(ahead));  // entries that stay ahead of the new one
  if (p >= kk) return;
  const float ps = __shfl_up(cs, 1);
  const int32_t pi = __shfl_up(ci, 1);
  if (lane < kk) {
    if (lane == p) {
      ls[lane] = s;
      li[lane] = e;
    } else if (lane > p) {
      ls[lane] = ps;
      li[lane] = pi;
    }
  }
}

__device__ __forceinline__ uint32_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ uint32_t pack_bf16_pair(float lo, float hi) {
  return bf16_bits_rne(lo) | (bf16_bits_rne(hi) << 16);
}

}  // namespace mrf
