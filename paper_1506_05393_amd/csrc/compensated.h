// Compensated FP32 summation: dot products that stay in FP32 arithmetic yet
// come out as accurate as if accumulated in twice the precision (products
// and sums each rounded once; contraction is off inside these helpers).
#pragma once

#include <hip/hip_runtime.h>

namespace mrf {

// s + c += x, with the rounding error of the addition kept in c (Knuth's TwoSum).
__device__ __forceinline__ void two_sum_acc(float& s, float& c, float x) {
#pragma clang fp contract(off)
  const float t = s + x;
  const float z = t - s;
  c += (s - (t - z)) + (x - z);
  s = t;
}

// Accumulates s + a b as the unevaluated pair (s, c): the rounding error of
// the product (from an FMA) and of the sum (TwoSum) are gathered in c, the
// compensated dot product of Ogita, Rump and Oishi ("Dot2").
__device__ __forceinline__ void dot2_acc(float a, float b, float& s, float& c) {
#pragma clang fp contract(off)
  const float p = a * b;
  const float ep = fmaf(a, b, -p);
  const float t = s + p;
  const float z = t - s;
  const float es = (s - (t - z)) + (p - z);
  s = t;
  c += ep + es;
}

}  // namespace mrf
