// K1: dictionary simulation (Appendix Eq. A2 per entry) and on-the-fly
// simulation of fingerprints at arbitrary parameter values.
//
// One thread per entry runs the readout recursion in registers (FP32 state,
// FP64 norm). Consecutive threads take consecutive entries, so every store of
// a wavefront is one contiguous 256 B (FP32 plane row) or 1 KB (BF16 4-readout
// block) segment.
#include <hip/hip_runtime.h>

#include <cmath>

#include "bloch.h"
#include "internal.h"
#include "sim_kernels.h"

namespace mrf {

struct SimArgs {
  const float2* t1;
  const float* t1ti;
  const float2* t2;
  const float4* df;
  const float* rf;
  int32_t n_tr, n1, n2, n3, n4, inversion;
  int64_t k0, count, ld;
  float* re;        // F32 planar
  float* im;
  uint4* packed;    // BF16 blocks
  double* norm;
  int32_t unit_norm;
};

__device__ __forceinline__ const float* wave_uniform(const float* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (const float*)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return bf16_rne(lo) | (bf16_rne(hi) << 16);
}

// Entry k -> per-axis indices.
__device__ __forceinline__ void unravel(int64_t k, int32_t n2, int32_t n3, int32_t n4, int32_t& i1,
                                        int32_t& i2, int32_t& i3, int32_t& i4) {
  i4 = (int32_t)(k % n4);
  k /= n4;
  i3 = (int32_t)(k % n3);
  k /= n3;
  i2 = (int32_t)(k % n2);
  i1 = (int32_t)(k / n2);
}

// mode 0: accumulate the norm only; mode 1: FP32 planar stores; mode 2: BF16
// blocks. Returns the squared norm of the simulated signal; in mode 2 *stored
// receives the squared norm of the stored (scaled, rounded) BF16 values, the
// normaliser that keeps CCs computed from the stored dictionary consistent.
template <int MODE>
__device__ __forceinline__ double run_entry(const SimArgs& a, int32_t i1, int32_t i2, int32_t i3,
                                            const float* R, int64_t e, float scale,
                                            double* stored = nullptr) {
  Spin m = initial_spin(a.inversion, a.t1ti[i1]);
  double n2 = 0.0, nb = 0.0;
  const float2* t1 = a.t1 + i1;
  const float2* t2 = a.t2 + i2;
  const float4* df = a.df + i3;
  if (MODE == 2) {
    for (int32_t j = 0; j < a.n_tr; j += 4) {
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int32_t jj = j + q;
        const float2 r1 = t1[(int64_t)jj * a.n1];
        const float2 r2 = t2[(int64_t)jj * a.n2];
        const float4 pc = df[(int64_t)jj * a.n3];
        rf_pulse(m, R + 9 * jj);
        free_evolve(m, pc.x, pc.y, r2.x, r1.x);
        n2 = fma((double)m.x, (double)m.x, n2);
        n2 = fma((double)m.y, (double)m.y, n2);
        w[q] = pack_bf16x2(m.x * scale, m.y * scale);
        const double bx = (double)__uint_as_float(w[q] << 16);
        const double by = (double)__uint_as_float(w[q] & 0xFFFF0000u);
        nb = fma(bx, bx, nb);
        nb = fma(by, by, nb);
        free_evolve(m, pc.z, pc.w, r2.y, r1.y);
      }
      a.packed[(int64_t)(j >> 2) * a.ld + e] = make_uint4(w[0], w[1], w[2], w[3]);
    }
    if (stored) *stored = nb;
  } else {
#pragma unroll 2
    for (int32_t j = 0; j < a.n_tr; ++j) {
      const float2 r1 = t1[(int64_t)j * a.n1];
      const float2 r2 = t2[(int64_t)j * a.n2];
      const float4 pc = df[(int64_t)j * a.n3];
      rf_pulse(m, R + 9 * j);
      free_evolve(m, pc.x, pc.y, r2.x, r1.x);
      n2 = fma((double)m.x, (double)m.x, n2);
      n2 = fma((double)m.y, (double)m.y, n2);
      if (MODE == 1) {
        a.re[(int64_t)j * a.ld + e] = m.x * scale;
        a.im[(int64_t)j * a.ld + e] = m.y * scale;
      }
      free_evolve(m, pc.z, pc.w, r2.y, r1.y);
    }
  }
  return n2;
}

template <int MODE>
__global__ __launch_bounds__(256) void k_sim_dict(SimArgs a) {
  const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (e >= a.count) return;
  int32_t i1, i2, i3, i4;
  unravel(a.k0 + e, a.n2, a.n3, a.n4, i1, i2, i3, i4);
  const float* R = a.rf + (int64_t)i4 * a.n_tr * 9;
  if (a.n4 == 1) R = wave_uniform(R);
  float scale = 1.0f;
  double n2 = 0.0;
  if (a.unit_norm) {
    n2 = run_entry<0>(a, i1, i2, i3, R, e, 1.0f);
    scale = n2 > 0.0 ? (float)(1.0 / sqrt(n2)) : 0.0f;
  }
  double stored = 0.0;
  double n2b = run_entry<MODE>(a, i1, i2, i3, R, e, scale, &stored);
  if (!a.unit_norm) n2 = n2b;
  if (MODE == 2) n2 = stored;  // BF16: the norm of the values actually stored
  if (a.norm) a.norm[e] = sqrt(n2);
}

// Fingerprints at arbitrary parameters: the factors are computed per readout
// in FP64 with the same functions as the tables, so on-grid parameters give
// bit-identical signals to dictionary entries.
struct SigArgs {
  const double* seq;  // [4][n_seq]: TE, TR-TE, FA, phase
  int32_t n_seq, n_tr, inversion;
  double ti;
  const double* params;  // [count][4]
  int64_t count, ld;
  float2* out;
};

__global__ __launch_bounds__(256) void k_sim_signals(SigArgs a) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i >= a.count) return;
  const double T1 = a.params[4 * i + 0], T2 = a.params[4 * i + 1];
  const double df = a.params[4 * i + 2], b1 = a.params[4 * i + 3];
  Spin m = initial_spin(a.inversion, (float)one_minus_exp(a.ti, T1));
  const double* ta = a.seq;
  const double* tb = a.seq + a.n_seq;
  const double* fa = a.seq + 2 * (int64_t)a.n_seq;
  const double* ph = a.seq + 3 * (int64_t)a.n_seq;
  for (int32_t j = 0; j < a.n_tr; ++j) {
    float R[9];
    pulse_matrix(fa[j], ph[j], b1, R);
    float cma, sa, cmb, sb;
    precession(ta[j], df, &cma, &sa);
    precession(tb[j], df, &cmb, &sb);
    rf_pulse(m, R);
    free_evolve(m, cma, sa, (float)one_minus_exp(ta[j], T2), (float)one_minus_exp(ta[j], T1));
    a.out[i * a.ld + j] = make_float2(m.x, m.y);
    free_evolve(m, cmb, sb, (float)one_minus_exp(tb[j], T2), (float)one_minus_exp(tb[j], T1));
  }
}

int launch_sim_dict(mrf_context* ctx, const Tables& t, int64_t k0, int64_t count,
                    mrf_dtype dtype, void* re, void* im, int64_t ld, double* norm, int unit_norm,
                    hipStream_t stream) {
  if (count == 0) return MRF_OK;
  SimArgs a;
  a.t1 = t.t1;
  a.t1ti = t.t1ti;
  a.t2 = t.t2;
  a.df = t.df;
  a.rf = t.rf;
  a.n_tr = t.n_tr;
  a.n1 = t.n1;
  a.n2 = t.n2;
  a.n3 = t.n3;
  a.n4 = t.n4;
  a.inversion = t.inversion;
  a.k0 = k0;
  a.count = count;
  a.ld = ld;
  a.re = (float*)re;
  a.im = (float*)im;
  a.packed = (uint4*)re;
  a.norm = norm;
  a.unit_norm = unit_norm;
  const int64_t blocks = (count + 255) / 256;
  if (blocks > INT32_MAX) {
    set_error("too many entries in one call");
    return MRF_ERR_INVALID;
  }
  ProfScope prof(ctx, "k_sim_dict", stream);
  if (dtype == MRF_F32)
    hipLaunchKernelGGL(k_sim_dict<1>, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  else
    hipLaunchKernelGGL(k_sim_dict<2>, dim3((unsigned)blocks), dim3(256), 0, stream, a);
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}

}  // namespace mrf

using namespace mrf;

extern "C" int mrf_simulate_dictionary(mrf_context* ctx, const mrf_sequence* seq,
                                       const mrf_grid* grid, int32_t n_tr, int64_t entry_begin,
                                       int64_t entry_count, mrf_dtype dtype, void* re, void* im,
                                       int64_t ld, double* norm, int32_t unit_norm,
                                       void* stream) {
  MRF_CHECK_ARG(ctx && seq, "context and sequence must not be NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  MRF_CHECK_ARG(n_tr >= 1 && n_tr <= seq->n, "n_tr %d must be in [1, %d]", n_tr, seq->n);
  MRF_CHECK_ARG(dtype == MRF_F32 || dtype == MRF_BF16, "unknown dtype %d", (int)dtype);
  const int64_t E = grid_size_checked(grid);
  MRF_CHECK_ARG(entry_begin >= 0 && entry_count >= 0 && entry_begin + entry_count <= E,
                "entry range [%lld, %lld) outside the grid of %lld entries",
                (long long)entry_begin, (long long)(entry_begin + entry_count), (long long)E);
  MRF_CHECK_ARG(ld >= entry_count, "ld (%lld) must be >= entry_count (%lld)", (long long)ld,
                (long long)entry_count);
  if (dtype == MRF_F32) {
    MRF_CHECK_ARG(entry_count == 0 || (re && im), "re and im must not be NULL");
  } else {
    MRF_CHECK_ARG(entry_count == 0 || re, "re must not be NULL");
    MRF_CHECK_ARG(im == nullptr, "im must be NULL for the packed BF16 layout");
    MRF_CHECK_ARG(n_tr % 4 == 0, "BF16 dictionaries need n_tr %% 4 == 0 (got %d)", n_tr);
    MRF_CHECK_ARG(((uintptr_t)re & 15) == 0, "BF16 dictionary must be 16-byte aligned");
  }
  const Tables* t = nullptr;
  rc = get_tables(const_cast<mrf_sequence*>(seq), grid, n_tr, (hipStream_t)stream, &t);
  if (rc) return rc;
  return launch_sim_dict(ctx, *t, entry_begin, entry_count, dtype, re, im, ld, norm, unit_norm ? 1 : 0,
                         (hipStream_t)stream);
}

extern "C" int mrf_simulate_signals(mrf_context* ctx, const mrf_sequence* seq, int32_t n_tr,
                                    const double* params, int64_t count, void* out,
                                    int64_t ld_out, void* stream) {
  MRF_CHECK_ARG(ctx && seq, "context and sequence must not be NULL");
  MRF_CHECK_ARG(n_tr >= 1 && n_tr <= seq->n, "n_tr %d must be in [1, %d]", n_tr, seq->n);
  MRF_CHECK_ARG(count >= 0, "count must be >= 0");
  MRF_CHECK_ARG(count == 0 || (params && out), "params and out must not be NULL");
  MRF_CHECK_ARG(ld_out >= n_tr, "ld_out must be >= n_tr");
  if (count == 0) return MRF_OK;
  SigArgs a;
  a.seq = seq->dev;
  a.n_seq = seq->n;
  a.n_tr = n_tr;
  a.inversion = seq->inversion;
  a.ti = seq->ti;
  a.params = params;
  a.count = count;
  a.ld = ld_out;
  a.out = (float2*)out;
  const int64_t blocks = (count + 255) / 256;
  MRF_CHECK_ARG(blocks <= INT32_MAX, "too many signals in one call");
  hipLaunchKernelGGL(k_sim_signals, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}
