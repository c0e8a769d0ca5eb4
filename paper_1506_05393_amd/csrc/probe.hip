// Device peak probes: what this GPU sustains for the operations the hot path
// is bound by, launched and timed like the method's kernels so that their
// fractions can be quoted against measured as well as published peaks.
//  - MFMA-only loops on register operands, one per dtype of the matching
//    GEMMs (v_mfma_f32_32x32x2_f32, v_mfma_f32_32x32x16_bf16): four
//    independent accumulators per wave, so the matrix pipe never waits for
//    a result;
//  - the BF16 loop again with operands that differ from lane to lane and
//    element to element: the chip lowers its clock under the power such
//    data draws, so this is the rate a GEMM on real data can approach;
//  - a write-only stream of 16 B stores (the dictionary generator's bound).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace mrf {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kProbeThreads = 256;
constexpr int kProbeAcc = 4;
// operand values: exact in BF16, products exact in FP32
constexpr float kProbeA = 0.5f, kProbeB = 0.25f;

__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma_f32(int64_t iters, float a, float b,
                                                                   float* __restrict__ out) {
  f32x16 acc[kProbeAcc];
#pragma unroll
  for (int i = 0; i < kProbeAcc; ++i) acc[i] = f32x16{};
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kProbeAcc; ++i)
      acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kProbeAcc; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[i][r];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma_bf16(int64_t iters, float a,
                                                                    float b,
                                                                    float* __restrict__ out) {
  bf16x8_t va, vb;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    va[k] = (__bf16)a;
    vb[k] = (__bf16)b;
  }
  f32x16 acc[kProbeAcc];
#pragma unroll
  for (int i = 0; i < kProbeAcc; ++i) acc[i] = f32x16{};
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kProbeAcc; ++i)
      acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(va, vb, acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kProbeAcc; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[i][r];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// Operand element e of fragment f in lane l: 0.375 * ((7 l + 13 f + 29 e) mod 61) - 11,
// rounded to BF16 (values in [-11, 11.5], every mantissa pattern in play).
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma_bf16_varied(int64_t iters,
                                                                           float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  bf16x8_t fr[2 * kProbeAcc];
#pragma unroll
  for (int f = 0; f < 2 * kProbeAcc; ++f)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      fr[f][e] = (__bf16)(0.375f * (float)((7 * lane + 13 * f + 29 * e) % 61) - 11.0f);
  f32x16 acc[kProbeAcc];
#pragma unroll
  for (int i = 0; i < kProbeAcc; ++i) acc[i] = f32x16{};
  for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kProbeAcc; ++i)
      acc[i] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fr[2 * i], fr[2 * i + 1], acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kProbeAcc; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[i][r];
  out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

// One 16 B store per thread, each workgroup one contiguous 4 KB piece (the
// fastest of the write-stream shapes measured: wider per-thread runs and
// grid-stride loops were slower); element i = (pattern, i, pattern, i).
__global__ __launch_bounds__(kProbeThreads) void k_probe_write(u32x4_t* __restrict__ dst,
                                                                int64_t n16, int64_t first,
                                                                uint32_t pattern) {
  const int64_t i = first + (int64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  if (i < n16) {
    const u32x4_t v = {pattern, (uint32_t)i, pattern, (uint32_t)i};
    dst[i] = v;
  }
}

}  // namespace

}  // namespace mrf

using namespace mrf;

extern "C" int mrf_probe_mfma(mrf_context* ctx, mrf_dtype dtype, int64_t iters, float* out,
                              int64_t out_len, double* flops, void* stream) {
  MRF_CHECK_ARG(ctx, "context must not be NULL");
  MRF_CHECK_ARG(dtype == MRF_F32 || dtype == MRF_BF16, "dtype must be MRF_F32 or MRF_BF16");
  MRF_CHECK_ARG(iters >= 1, "iters must be >= 1");
  MRF_CHECK_ARG(out, "out must not be NULL");
  MRF_CHECK_ARG(out_len >= kProbeThreads && out_len % kProbeThreads == 0,
                "out_len (%lld) must be a positive multiple of %d", (long long)out_len,
                kProbeThreads);
  const int64_t blocks = out_len / kProbeThreads;
  MRF_CHECK_ARG(blocks <= INT32_MAX, "out_len too large");
  hipStream_t s = (hipStream_t)stream;
  // flops per instruction: 2 * 32 * 32 * K, K = 2 (FP32) or 16 (BF16)
  const double per = dtype == MRF_F32 ? 4096.0 : 32768.0;
  const double waves = (double)blocks * (kProbeThreads / 64);
  if (flops) *flops = per * kProbeAcc * (double)iters * waves;
  if (dtype == MRF_F32) {
    ProfScope prof(ctx, "k_probe_mfma_f32", s);
    hipLaunchKernelGGL(k_probe_mfma_f32, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s, iters,
                       kProbeA, kProbeB, out);
  } else {
    ProfScope prof(ctx, "k_probe_mfma_bf16", s);
    hipLaunchKernelGGL(k_probe_mfma_bf16, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s,
                       iters, kProbeA, kProbeB, out);
  }
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}

extern "C" int mrf_probe_mfma_varied(mrf_context* ctx, int64_t iters, float* out,
                                     int64_t out_len, double* flops, void* stream) {
  MRF_CHECK_ARG(ctx, "context must not be NULL");
  MRF_CHECK_ARG(iters >= 1, "iters must be >= 1");
  MRF_CHECK_ARG(out, "out must not be NULL");
  MRF_CHECK_ARG(out_len >= kProbeThreads && out_len % kProbeThreads == 0,
                "out_len (%lld) must be a positive multiple of %d", (long long)out_len,
                kProbeThreads);
  const int64_t blocks = out_len / kProbeThreads;
  MRF_CHECK_ARG(blocks <= INT32_MAX, "out_len too large");
  hipStream_t s = (hipStream_t)stream;
  const double waves = (double)blocks * (kProbeThreads / 64);
  if (flops) *flops = 32768.0 * kProbeAcc * (double)iters * waves;
  ProfScope prof(ctx, "k_probe_mfma_bf16_varied", s);
  hipLaunchKernelGGL(k_probe_mfma_bf16_varied, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s,
                     iters, out);
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}

extern "C" int mrf_probe_write(mrf_context* ctx, void* dst, int64_t bytes, uint32_t pattern,
                               void* stream) {
  MRF_CHECK_ARG(ctx, "context must not be NULL");
  MRF_CHECK_ARG(bytes >= 0 && bytes % 16 == 0, "bytes (%lld) must be a multiple of 16",
                (long long)bytes);
  MRF_CHECK_ARG(bytes == 0 || (dst && ((uintptr_t)dst & 15) == 0),
                "dst must be a 16-byte aligned device pointer");
  if (bytes == 0) return MRF_OK;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n16 = bytes / 16;
  // launches of at most 2^30 workgroups (16 TiB) each
  const int64_t max_blocks = (int64_t)1 << 30;
  ProfScope prof(ctx, "k_probe_write", s);
  for (int64_t first = 0; first < n16; first += max_blocks * kProbeThreads) {
    int64_t blocks = (n16 - first + kProbeThreads - 1) / kProbeThreads;
    if (blocks > max_blocks) blocks = max_blocks;
    hipLaunchKernelGGL(k_probe_write, dim3((unsigned)blocks), dim3(kProbeThreads), 0, s,
                       (u32x4_t*)dst, n16, first, pattern);
  }
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}
