// Temporal smoothing of dictionary entries along the readouts (Methods,
// Experiment 4; Results, Fig. 7B): a moving Gaussian of 3 or 5 points, here
// the binomial weights (1, 2, 1) / 4 and (1, 4, 6, 4, 1) / 16. Where the
// window passes the first or last readout only the points that exist count
// and the weights are renormalised over them.
//
// The window acts on the signal as the receiver records it: sample j is
// demodulated by its RF phase (times exp(-i phi_j)) before it enters the
// window, and each output is modulated back (times exp(i phi_o)), so smoothed
// entries and fingerprints stay in the frame of the unsmoothed ones. The
// (cos, sin) pairs are exact for phases that are multiples of 90 degrees,
// where both steps only swap and negate components.
//
// Kernels that simulate an entry readout by readout smooth it with a delay
// line of five raw samples: after raw sample j is pushed, the line holds
// samples j-4 .. j and yields smoothed sample o = j - 2. The 3-point weights
// sit in the middle of the 5-point line (outer weights 0), so one delay of two
// readouts serves both lengths. Zeros fill the line before readout 0, and two
// zero pushes after the last readout yield the last two outputs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mrf {

constexpr int kSmoothLen = 5;
constexpr int kSmoothLag = 2;

// Weights and 1 / (weight sum) per output position, for one (taps, n_tr).
struct SmoothW {
  float w[kSmoothLen];  // integer weights, centred on element 2
  float full;           // 1 / sum: outputs 2 .. n_tr - 3
  float head[2];        // outputs 0 and 1 (window cut on the left)
  float tail[2];        // outputs n_tr - 2 and n_tr - 1 (cut on the right, and on the left if short)
};

// Host: the weights of `taps` (3 or 5) for sequences of n_tr readouts.
inline SmoothW smooth_weights(int taps, int32_t n_tr) {
  static const double w3[kSmoothLen] = {0.0, 1.0, 2.0, 1.0, 0.0};
  static const double w5[kSmoothLen] = {1.0, 4.0, 6.0, 4.0, 1.0};
  const double* w = taps == 5 ? w5 : w3;
  SmoothW s{};
  auto inv_den = [&](int64_t o) {  // 1 / sum of the weights of readouts inside [0, n_tr)
    double d = 0.0;
    for (int k = 0; k < kSmoothLen; ++k) {
      const int64_t r = o + k - kSmoothLag;
      if (r >= 0 && r < n_tr) d += w[k];
    }
    return d > 0.0 ? (float)(1.0 / d) : 0.0f;
  };
  double sum = 0.0;
  for (int k = 0; k < kSmoothLen; ++k) {
    s.w[k] = (float)w[k];
    sum += w[k];
  }
  s.full = (float)(1.0 / sum);
  // outputs 0 and 1 are emitted while later readouts still follow: cut on
  // the left only (for them o + 2 <= n_tr - 1 holds whenever they are
  // emitted before the end of the sequence)
  for (int o = 0; o < 2; ++o) {
    double d = 0.0;
    for (int k = 0; k < kSmoothLen; ++k)
      if (o + k - kSmoothLag >= 0) d += w[k];
    s.head[o] = (float)(1.0 / d);
  }
  s.tail[0] = inv_den((int64_t)n_tr - 2);
  s.tail[1] = inv_den((int64_t)n_tr - 1);
  return s;
}

// Device: (x + i y) times exp(-i phi), cs = (cos phi, sin phi).
__device__ __forceinline__ void smooth_demod(float2 cs, float& x, float& y) {
  const float a = x, b = y;
  x = fmaf(a, cs.x, b * cs.y);
  y = fmaf(b, cs.x, -(a * cs.y));
}

// Device: (x + i y) times exp(i phi).
__device__ __forceinline__ void smooth_remod(float2 cs, float& x, float& y) {
  const float a = x, b = y;
  x = fmaf(a, cs.x, -(b * cs.y));
  y = fmaf(a, cs.y, b * cs.x);
}

// Device: push raw sample (x, y) into the delay line.
__device__ __forceinline__ void smooth_push(float (&hx)[kSmoothLen], float (&hy)[kSmoothLen],
                                            float x, float y) {
#pragma unroll
  for (int k = 0; k + 1 < kSmoothLen; ++k) {
    hx[k] = hx[k + 1];
    hy[k] = hy[k + 1];
  }
  hx[kSmoothLen - 1] = x;
  hy[kSmoothLen - 1] = y;
}

// Device: the smoothed sample at the centre of the line, times `sc`.
__device__ __forceinline__ void smooth_out(const SmoothW& s, const float (&hx)[kSmoothLen],
                                           const float (&hy)[kSmoothLen], float sc, float& x,
                                           float& y) {
  float ax = s.w[0] * hx[0], ay = s.w[0] * hy[0];
#pragma unroll
  for (int k = 1; k < kSmoothLen; ++k) {
    ax = fmaf(s.w[k], hx[k], ax);
    ay = fmaf(s.w[k], hy[k], ay);
  }
  x = ax * sc;
  y = ay * sc;
}

}  // namespace mrf
