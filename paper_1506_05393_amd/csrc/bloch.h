// Device step functions of the Bloch model (Appendix Eq. A2, hard-pulse RF),
// shared by every kernel that simulates an entry so that dictionary entries,
// re-scored candidates and ZOOM candidates are bit-identical.
//
// State (x, y, z) in FP32. Per readout j:
//   RF pulse     : M <- R_j M, R_j = Rz(phi_j) Rx(-B1 alpha_j) Rz(-phi_j)
//   free over TE : (x, y) <- E2 Rz(theta)(x, y), z <- E1 z + (1 - E1)
//   sample       : d_j = x + i y
//   free over TR-TE.
// The free-evolution factors are kept as (1 - E) and (cos theta - 1), which
// are exact to FP32 relative precision even when E ~ 1 and theta ~ 0, and the
// updates are written so that the fixed point z = 1 and the rotation are not
// perturbed by rounding E or cos theta to FP32.
#pragma once

#include <hip/hip_runtime.h>

namespace mrf {

struct Spin {
  float x, y, z;
};

__device__ __forceinline__ void rf_pulse(Spin& m, const float* __restrict__ R) {
  const float x = m.x, y = m.y, z = m.z;
  m.x = fmaf(R[2], z, fmaf(R[1], y, R[0] * x));
  m.y = fmaf(R[5], z, fmaf(R[4], y, R[3] * x));
  m.z = fmaf(R[8], z, fmaf(R[7], y, R[6] * x));
}

// cm1 = cos(theta) - 1, s = sin(theta), r2 = 1 - E2, r1 = 1 - E1.
__device__ __forceinline__ void free_evolve(Spin& m, float cm1, float s, float r2, float r1) {
  const float x = m.x, y = m.y;
  const float xr = fmaf(cm1, x, fmaf(-s, y, x));
  const float yr = fmaf(cm1, y, fmaf(s, x, y));
  m.x = fmaf(-r2, xr, xr);
  m.y = fmaf(-r2, yr, yr);
  m.z = fmaf(r1, 1.0f - m.z, m.z);
}

// Per-readout factors from FP64 parameters (one place, so that tables and
// on-the-fly factors round identically).
__device__ __forceinline__ double one_minus_exp(double t, double T) {
  // 1 - exp(-t/T) without cancellation; T = +inf gives 0
  return -expm1(-t / T);
}

// Precession over t ms at df Hz: (cos(theta) - 1, sin(theta)), theta = 2 pi df t / 1000.
__device__ __forceinline__ void precession(double t, double df, float* cm1, float* s) {
  const double th = 2.0 * M_PI * df / 1000.0 * t;
  const double h = sin(0.5 * th);
  *cm1 = (float)(-2.0 * h * h);
  *s = (float)sin(th);
}

// Rz(phi) Rx(-alpha) Rz(-phi), row-major, alpha = b1 * fa.
__device__ __forceinline__ void pulse_matrix(double fa_deg, double ph_deg, double b1, float* R) {
  const double al = b1 * fa_deg * (M_PI / 180.0);
  double s, c, sa, ca;
  // phase in half-turns: multiples of 180 degrees give exact 0 and +-1
  sincospi(ph_deg / 180.0, &s, &c);
  sincos(al, &sa, &ca);
  R[0] = (float)(c * c + s * s * ca);
  R[1] = (float)(c * s - s * c * ca);
  R[2] = (float)(-s * sa);
  R[3] = (float)(s * c - s * c * ca);
  R[4] = (float)(s * s + c * c * ca);
  R[5] = (float)(c * sa);
  R[6] = (float)(s * sa);
  R[7] = (float)(-c * sa);
  R[8] = (float)ca;
}

__device__ __forceinline__ Spin initial_spin(int inversion, float r1_ti) {
  Spin m{0.0f, 0.0f, inversion ? -1.0f : 1.0f};
  m.z = fmaf(r1_ti, 1.0f - m.z, m.z);
  return m;
}

}  // namespace mrf
