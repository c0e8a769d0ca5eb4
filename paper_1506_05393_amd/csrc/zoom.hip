// K6: MRF-ZOOM (Theory: MRF ZOOM; Methods: Experiment 2 zooming steps 1-5;
// Experiment 3 neighbour prior) as a persistent kernel.
//
// Each voxel is searched by a group of G lanes (8 voxels per wave for G = 8),
// pulled from an atomic queue so that voxels with uneven numbers of
// evaluations balance across the machine. A group's stage machine runs in
// group-uniform control flow; each decision's candidate entries are
// evaluated one per lane (rounds of G), simulated on the fly with the same
// step function as the dictionary kernel (bit-identical entries), with the
// correlation against the unit-norm voxel accumulated inside the readout
// loop. Each group owns a memo (entry -> CC, so every distinct entry is
// simulated once per voxel) in global memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "bloch.h"
#include "compensated.h"
#include "internal.h"
#include "smooth.h"

namespace mrf {

struct ZoomArgs {
  const float2* t1T;
  const float* t1ti;
  const float2* t2T;
  const float4* dfT;
  const float* rf;
  int32_t n_tr, inversion;
  int32_t tab_n;            // readouts per table row (>= every voxel's readout count)
  const int32_t* vox_n_tr;  // per-voxel readout counts [n_vox], or NULL (all n_tr)
  int32_t x_axis;  // every RF phase a multiple of 180 deg: pulses rotate about x
  // compact tables of symmetric TRs with x-axis pulses (all non-NULL, the
  // voxel rows 16-byte aligned and no smoothing), else half = 0
  int32_t half, tq;
  const float* h1;
  const float* h2;
  const float2* hd;
  const float2* xr;
  // readouts per LDS row holding a group's voxel scaled to unit norm (read
  // by the compact-table path), 0 = the voxel is read from global memory
  int32_t vrow;
  // otherwise (vrow == 0, compact-table path) the same scaled voxel in a
  // per-group row of vrow_g readouts in the workspace
  int32_t vrow_g;
  float2* vscaled;
  int32_t dims[4];
  const float2* vox;
  int64_t ld_vox;
  int32_t n_vox;
  const int32_t* init;       // per-axis prior centres [n_vox][4], or
  const int64_t* init_flat;  // flat grid indices [n_vox] (either may be NULL)
  // queue: n_items positions. Neighbour-prior lattice passes (lat_pass 1:
  // the voxels on every lat_stride-th row and column of each lat_w x lat_h
  // slice; 2: the others, each started at its nearest lattice voxel's result)
  int32_t n_items, lat_pass, lat_w, lat_h, lat_stride;
  int64_t* idx;
  float* cc;
  float* margin;
  float* pd_re;
  float* pd_im;
  int32_t* n_sim;
  int32_t* counter;
  int32_t memo_cap;  // slots per wave, power of two
  // [grid blocks][voxel groups][memo_cap] slots of 16 bytes: the key, then
  // the value (CC) or with distance stages both values (CC, score)
  int64_t* memo_slots;
  const mrf_zoom_schedule* sch;  // device copy (workspace)
  SmoothW sm;  // temporal smoothing of the entries (SM kernels)
  const float2* demod;  // [n_tr] (cos, sin) of the RF phases (SM kernels)
  // resident dictionary (GA kernels): entry k's readouts 2t, 2t + 1 at
  // dict[k * dict_ld4 + t], complex64 entry-major rows
  const float4* dict;
  int64_t dict_ld4;
};

// A resident entry-major dictionary, as the gathering engine reads it.
struct DictRows {
  const float4* base;
  int64_t ld4;
};

__device__ __forceinline__ int32_t round_half_away(double x) {
  return (int32_t)(x >= 0.0 ? floor(x + 0.5) : -floor(-x + 0.5));
}

// Reductions over the G lanes of a voxel's group (G divides 64; xor offsets
// below G stay inside the group).
template <int G>
__device__ __forceinline__ float grp_max(float v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, G));
  return v;
}

// (best, runner-up) of the values held by the group's lanes
template <int G>
__device__ __forceinline__ void grp_top2(float v, float& b1, float& b2) {
  float a1 = v, a2 = -INFINITY;
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) {
    const float c1 = __shfl_xor(a1, o, G), c2 = __shfl_xor(a2, o, G);
    const float n1 = fmaxf(a1, c1);
    const float n2 = fmaxf(fminf(a1, c1), fmaxf(a2, c2));
    a1 = n1;
    a2 = n2;
  }
  b1 = a1;
  b2 = a2;
}

// the group's lanes (bit l = group lane l) for which p holds
template <int G>
__device__ __forceinline__ uint64_t grp_ballot(bool p, int gbase) {
  const uint64_t m = __ballot(p);
  return G == 64 ? m : (m >> gbase) & ((1ull << (G & 63)) - 1);
}

// first group lane holding the maximum (ties: lowest lane); -1 if all are -inf
template <int G>
__device__ __forceinline__ int grp_first_max(float v, float& best, int gbase) {
  best = grp_max<G>(v);
  if (!(best > -INFINITY)) return -1;
  return __ffsll((unsigned long long)grp_ballot<G>(v == best, gbase)) - 1;
}

// Orders this wave's earlier LDS and global memory operations before its
// later ones (a block is one wave; the groups of a wave diverge, so no
// barrier can be used inside the search).
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// The fields of ZoomArgs the engine needs, copied into registers (taking the
// address of the kernel argument block would force a private-memory copy).
struct EngineParams {
  const float2* t1T;
  const float* t1ti;
  const float2* t2T;
  const float4* dfT;
  const float* rf;
  int32_t n_tr, inversion, memo_cap, x_axis;
  int32_t tab_n;  // readouts per table row (n_tr is this voxel's count, <= tab_n)
  int32_t half, tq;  // compact tables (see ZoomArgs)
  const float* h1;
  const float* h2;
  const float2* hd;
  const float2* xr;
  int32_t dims[4];
};

// DI: the engine can evaluate both objectives (CC and the distance score of
// the non-normalised fingerprint); every candidate is then simulated with the
// compensated dot product and the memo keeps both values.
template <int G, bool SM, bool GA, bool DI = false>
struct Engine {
  EngineParams pa;

  // memo key: (voxel serial << 40) | kSpecBit? | entry index (< 2^39)
  static constexpr int64_t kIndexMask = ((int64_t)1 << 40) - 1;
  static constexpr int64_t kSpecBit = (int64_t)1 << 39;
  // Look-ahead: a decision that leaves lanes of its group idle fills them
  // with entries that later decisions are likely to ask for (the next points
  // along a 1-D climb, the neighbours one more 2-D move ahead, the first
  // points of the following zoom stages at the current centre). Their values
  // go to the memo flagged kSpecBit; the first decision that reads one
  // counts it in n_sim, so n_sim still counts the entries the search
  // consulted, and no decision depends on which lane computed a value.
  // (The gathering engine reads rows instead and does not look ahead.)
  static constexpr bool kLookAhead = !GA;
  const mrf_zoom_stage* nxt;  // the stages after the running one
  int32_t n_nxt;
  const float2* vx;  // the voxel's fingerprint (global memory, read-only)
  const float2* vs;  // vx * vinv in LDS (same FP32 products), or NULL
  bool vx_scaled;    // vx already holds those products (a workspace row)
  float vinv;        // 1 / ||v||: the unit-norm voxel is vx * vinv
  double vn;         // ||v|| (FP64)
  int64_t* mkey;     // this group's memo: 16-byte slots (global memory), or
  float* mval;       // with GA separate key and value arrays (LDS)
  int32_t obj;       // objective of the stage being run (MRF_OBJ_*; DI only)
  int64_t tag;       // voxel serial << 40
  float* nbv;  // [8] neighbour values of one pruned move (LDS)
  int32_t lane;   // lane within the voxel's group of G lanes
  int32_t gbase;  // wave lane of the group's lane 0
  int32_t memo_count;
  int32_t n_sim;
  bool overflow;
  int32_t lo[4], hi[4];
  int32_t c[4];
  float cval;
  bool cknown;
  float mm;  // smallest decision margin
  // smoothing weights (SM only; the plain kernel carries no copy)
  std::conditional_t<SM, SmoothW, char> sw;
  std::conditional_t<SM, const float2*, char> dm;  // (cos, sin) of the RF phases
  std::conditional_t<GA, DictRows, char> dict;      // resident dictionary (GA)

  __device__ int64_t key(const int32_t* i) const {
    return (((int64_t)i[0] * pa.dims[1] + i[1]) * pa.dims[2] + i[2]) * pa.dims[3] + i[3];
  }
  __device__ bool in_range(const int32_t* i) const {
    for (int q = 0; q < 4; ++q)
      if (i[q] < lo[q] || i[q] > hi[q]) return false;
    return true;
  }

  // CC of this lane's entry against the voxel (Eq. 1 with a unit-norm voxel).
  // The readout loop is latency-bound unless its loads run ahead: the table
  // rows, the pulse and the voxel value of readout j + kAhead are requested
  // while readout j is computed (a ring of kAhead readouts in registers,
  // filled by a branch-free steady-state loop). Typed pointers keep the loads
  // off the generic (flat) path: tables through the global address space,
  // the voxel through LDS. With x-axis pulses (every RF phase a multiple of
  // 180 deg) only the four entries R11, R12, R21, R22 of the rotation are
  // read: R00 = 1 and the other terms are exact zeros, so the product rounds
  // as the full 3 x 3 one does.
  // six readouts ahead: on the slice each SIMD holds one wave (4096 voxels in
  // groups of 16), so nothing else hides the table reads' latency; deeper
  // rings spill more than they gain (measured 3: 11.1 ms, 6: 10.2 ms, 8: 10.6).
  // The smoothing kernel, whose delay line already fills the registers, keeps
  // three (six made it slower: 22-24 -> 27 ms).
  static constexpr int kAhead = SM ? 3 : 6;
  template <bool LANE_R, bool X_AXIS, bool COMP>
  __device__ float simulate_cc_t(const int32_t* i, float* pdr, float* pdi, double* pn2,
                                 float* psc) const {
    typedef float v2 __attribute__((ext_vector_type(2)));
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) v2 gf2;
    typedef const __attribute__((address_space(1))) v4 gf4;
    typedef const __attribute__((address_space(1))) float gf1;
    constexpr int NR = X_AXIS ? 4 : 9;  // pulse values read per readout
    const int32_t n = pa.n_tr, tn = pa.tab_n;
    gf2* p1 = (gf2*)(pa.t1T + (int64_t)i[0] * tn);
    gf2* p2 = (gf2*)(pa.t2T + (int64_t)i[1] * tn);
    gf4* pd = (gf4*)(pa.dfT + (int64_t)i[2] * tn);
    gf1* Rp = (gf1*)(pa.rf + (LANE_R ? (int64_t)i[3] * tn * 9 : 0));
    gf2* vl = (gf2*)vx;
    // the pulse values of readout j: R[0..8], or R11, R12, R21, R22
    auto ld_pulse = [&](int32_t j, float (&r)[NR]) {
      if (X_AXIS) {
        r[0] = Rp[9 * j + 4];
        r[1] = Rp[9 * j + 5];
        r[2] = Rp[9 * j + 7];
        r[3] = Rp[9 * j + 8];
      } else {
#pragma unroll
        for (int k = 0; k < NR; ++k) r[k] = Rp[9 * j + k];
      }
    };
    Spin m = initial_spin(pa.inversion, pa.t1ti[i[0]]);
    float dr = 0.0f, di = 0.0f;
    float cr = 0.0f, ci = 0.0f;  // COMP: the compensation terms of dr, di
    double n2 = 0.0;
    // SM: a delay line of five raw samples, demodulated by the RF phase;
    // readout j yields smoothed sample o = j - 2 (scale 0 while o < 0),
    // modulated back, which meets voxel value o
    float hx[kSmoothLen], hy[kSmoothLen];
#pragma unroll
    for (int k = 0; k < kSmoothLen; ++k) hx[k] = hy[k] = 0.f;
    auto vidx = [&](int32_t j) { return SM ? max(j - kSmoothLag, 0) : j; };
    auto scale_of = [&](int32_t j) -> float {
      if constexpr (SM) {
        const int32_t o = j - kSmoothLag;
        return o >= 2 ? sw.full : (o == 1 ? sw.head[1] : (o == 0 ? sw.head[0] : 0.0f));
      } else {
        return 1.0f;
      }
    };
    // the output sample's product with the voxel and its norm
    auto accumulate = [&](float sx, float sy, v2 v) {
      // v conj(d): (vr + i vi)(x - i y), v the unit-norm voxel
      const float vr = v.x * vinv, vi = v.y * vinv;
      if constexpr (COMP) {
        dot2_acc(vr, sx, dr, cr);
        dot2_acc(vi, sy, dr, cr);
        dot2_acc(vi, sx, di, ci);
        dot2_acc(-vr, sy, di, ci);
      } else {
        dr = fmaf(vr, sx, fmaf(vi, sy, dr));
        di = fmaf(vi, sx, fmaf(-vr, sy, di));
      }
      n2 = fma((double)sx, (double)sx, n2);
      n2 = fma((double)sy, (double)sy, n2);
    };
    // one readout: the pulse, free evolution over TE, the sample's product
    // with the voxel, free evolution to the end of the TR
    auto step = [&](v2 r1, v2 r2, v4 pc, v2 v, const float (&R)[NR], int32_t jr) {
      const float x = m.x, y = m.y, z = m.z;
      if (X_AXIS) {
        m.y = fmaf(R[1], z, R[0] * y);
        m.z = fmaf(R[3], z, R[2] * y);
      } else {
        m.x = fmaf(R[2], z, fmaf(R[1], y, R[0] * x));
        m.y = fmaf(R[5], z, fmaf(R[4], y, R[3] * x));
        m.z = fmaf(R[8], z, fmaf(R[7], y, R[6] * x));
      }
      free_evolve(m, pc.x, pc.y, r2.x, r1.x);
      float sx = m.x, sy = m.y;
      if constexpr (SM) {
        smooth_demod(dm[jr], sx, sy);
        smooth_push(hx, hy, sx, sy);
        smooth_out(sw, hx, hy, scale_of(jr), sx, sy);
        smooth_remod(dm[max(jr - kSmoothLag, 0)], sx, sy);
      }
      accumulate(sx, sy, v);
      free_evolve(m, pc.z, pc.w, r2.y, r1.y);
    };
    int32_t j = 0;
    if (n >= 2 * kAhead) {
      v2 q1[kAhead], q2[kAhead], qv[kAhead];
      v4 qd[kAhead];
      float qr[kAhead][NR];
#pragma unroll
      for (int q = 0; q < kAhead; ++q) {
        q1[q] = p1[q];
        q2[q] = p2[q];
        qd[q] = pd[q];
        qv[q] = vl[vidx(q)];
        ld_pulse(q, qr[q]);
      }
      // the ring holds readouts j .. j + kAhead - 1, and j + kAhead <= n
      for (; j + 2 * kAhead <= n; j += kAhead) {
#pragma unroll
        for (int q = 0; q < kAhead; ++q) {
          const v2 r1 = q1[q], r2 = q2[q], v = qv[q];
          const v4 pc = qd[q];
          float R[NR];
#pragma unroll
          for (int k = 0; k < NR; ++k) R[k] = qr[q][k];
          const int32_t jn = j + q + kAhead;
          q1[q] = p1[jn];
          q2[q] = p2[jn];
          qd[q] = pd[jn];
          qv[q] = vl[vidx(jn)];
          ld_pulse(jn, qr[q]);
          step(r1, r2, pc, v, R, j + q);
        }
      }
#pragma unroll
      for (int q = 0; q < kAhead; ++q)
        step(q1[q], q2[q], qd[q], qv[q], qr[q], j + q);
      j += kAhead;
    }
    for (; j < n; ++j) {
      float R[NR];
      ld_pulse(j, R);
      const v2 r1 = p1[j], r2 = p2[j], v = vl[vidx(j)];
      const v4 pc = pd[j];
      step(r1, r2, pc, v, R, j);
    }
    if constexpr (SM) {
      // the last two outputs: zeros pushed after the last readout
#pragma unroll
      for (int t = 0; t < kSmoothLag; ++t) {
        const int32_t o = n - kSmoothLag + t;
        float sx, sy;
        smooth_push(hx, hy, 0.f, 0.f);
        smooth_out(sw, hx, hy, sw.tail[t], sx, sy);
        if (o >= 0) {
          smooth_remod(dm[o], sx, sy);
          accumulate(sx, sy, vl[o]);
        }
      }
    }
    return finish<COMP>(dr, di, cr, ci, n2, pdr, pdi, pn2, psc);
  }
  // CC (and with COMP the distance score) from the dot-product sums and the
  // entry's squared norm; the optional outputs take the sums
  template <bool COMP>
  __device__ float finish(float dr, float di, float cr, float ci, double n2, float* pdr,
                          float* pdi, double* pn2, float* psc) const {
    if constexpr (COMP) {
      // the pairs as FP64 values; |<v, d>| = |<v * vinv, d>| / vinv, and
      // the distance score -||v - exp(i phi) d||^2 / ||v||^2 (best phase)
      // = -(1 + ||d||^2 / ||v||^2 - 2 |<v, d>| / ||v||^2)
      const double sr = (double)dr + (double)cr, si = (double)di + (double)ci;
      const double dabs = sqrt(sr * sr + si * si);
      if (pdr) *pdr = (float)sr;
      if (pdi) *pdi = (float)si;
      if (pn2) *pn2 = n2;
      if (psc) {
        const double vv = vn * vn;
        *psc = vn > 0.0 ? (float)(-(1.0 + n2 / vv - 2.0 * (dabs / (double)vinv) / vv))
                        : (float)(-n2);
      }
      if (!(n2 > 0.0)) return 0.0f;
      return (float)(dabs / sqrt(n2));
    } else {
      (void)cr;
      (void)ci;
      (void)psc;
      if (pdr) *pdr = dr;
      if (pdi) *pdi = di;
      if (pn2) *pn2 = n2;
      if (!(n2 > 0.0)) return 0.0f;
      return (float)(sqrt((double)dr * dr + (double)di * di) / sqrt(n2));
    }
  }

  // simulate_cc_t for symmetric TRs with x-axis pulses, from the compact
  // tables: both halves of a TR apply the same factors, so one 16-byte load
  // brings four readouts of 1-E1 or 1-E2, or two of the precession, and the
  // pulses of four readouts are one scalar load when every lane uses B1 = 1
  // (LANE_R: the B1 axis picks the row, one vector load per readout). The
  // arithmetic is that of simulate_cc_t, operation for operation, so the
  // values are the same. The loads run kAq quads (four readouts) ahead.
  static constexpr int kAq = 4;
  // VM: where the voxel comes from: 0 vx (scaled here), 1 vx holding the
  // scaled products (workspace row), 2 the LDS copy vs
  template <bool LANE_R, bool COMP, int VM>
  __device__ float simulate_half(const int32_t* i, float* pdr, float* pdi, double* pn2,
                                 float* psc) const {
    typedef float v2 __attribute__((ext_vector_type(2)));
    typedef float v4 __attribute__((ext_vector_type(4)));
    typedef const __attribute__((address_space(1))) v4 gf4;
    typedef const __attribute__((address_space(1))) float gf1;
    typedef const __attribute__((address_space(1))) v2 gf2;
    typedef const __attribute__((address_space(4))) v4 cf4;
    typedef const __attribute__((address_space(3))) v4 lf4;
    typedef const __attribute__((address_space(3))) v2 lf2;
    constexpr bool VS = VM == 2, SCALED = VM != 0;
    const int32_t n = pa.n_tr, tq = pa.tq;
    gf1* p1 = (gf1*)(pa.h1 + (int64_t)i[0] * tq);
    gf1* p2 = (gf1*)(pa.h2 + (int64_t)i[1] * tq);
    gf2* pd = (gf2*)(pa.hd + (int64_t)i[2] * tq);
    gf4* q1 = (gf4*)p1;
    gf4* q2 = (gf4*)p2;
    gf4* qd = (gf4*)pd;
    gf4* qv = (gf4*)vx;
    // pulses: (R11, R12) per readout, R21 = -R12 and R22 = R11
    gf4* rl = (gf4*)(pa.xr + (LANE_R ? (int64_t)i[3] * tq : 0));
    cf4* ru = (cf4*)pa.xr;
    gf2* r1l = (gf2*)(pa.xr + (LANE_R ? (int64_t)i[3] * tq : 0));
    Spin m = initial_spin(pa.inversion, pa.t1ti[i[0]]);
    float dr = 0.0f, di = 0.0f, cr = 0.0f, ci = 0.0f;
    double n2 = 0.0;
    auto step = [&](float r1, float r2, float cm1, float sn, float vxr, float vxi, float c,
                    float sp) {
      {
        // the x-axis rotation (as simulate_cc_t: R21 y is -(R12 y) exactly)
        const float y = m.y, z = m.z;
        m.y = fmaf(sp, z, c * y);
        m.z = fmaf(c, z, -sp * y);
      }
      free_evolve(m, cm1, sn, r2, r1);
      const float sx = m.x, sy = m.y;
      // the LDS or workspace copy already holds these products
      const float vr = SCALED ? vxr : vxr * vinv, vi = SCALED ? vxi : vxi * vinv;
      if constexpr (COMP) {
        dot2_acc(vr, sx, dr, cr);
        dot2_acc(vi, sy, dr, cr);
        dot2_acc(vi, sx, di, ci);
        dot2_acc(-vr, sy, di, ci);
      } else {
        dr = fmaf(vr, sx, fmaf(vi, sy, dr));
        di = fmaf(vi, sx, fmaf(-vr, sy, di));
      }
      n2 = fma((double)sx, (double)sx, n2);
      n2 = fma((double)sy, (double)sy, n2);
      free_evolve(m, cm1, sn, r2, r1);
    };
    // one quad: readouts 4k .. 4k + 3
    struct Quad {
      v4 a, b, d0, d1, v0, v1;
      v4 r[LANE_R ? 2 : 1];
    };
    auto load = [&](int32_t k, Quad& u) {
      u.a = q1[k];
      u.b = q2[k];
      u.d0 = qd[2 * k];
      u.d1 = qd[2 * k + 1];
      if constexpr (VS) {
        u.v0 = ((lf4*)vs)[2 * k];
        u.v1 = ((lf4*)vs)[2 * k + 1];
      } else {
        u.v0 = qv[2 * k];
        u.v1 = qv[2 * k + 1];
      }
      if constexpr (LANE_R) {
        u.r[0] = rl[2 * k];
        u.r[1] = rl[2 * k + 1];
      }
    };
    auto run = [&](int32_t k, const Quad& u) {
      // k is the same on every lane that runs the loop: the pulses are
      // scalar loads
      const int32_t ks = __builtin_amdgcn_readfirstlane(k);
      const v4 P0 = LANE_R ? u.r[0] : ru[2 * ks];
      const v4 P1 = LANE_R ? u.r[1] : ru[2 * ks + 1];
      step(u.a.x, u.b.x, u.d0.x, u.d0.y, u.v0.x, u.v0.y, P0.x, P0.y);
      step(u.a.y, u.b.y, u.d0.z, u.d0.w, u.v0.z, u.v0.w, P0.z, P0.w);
      step(u.a.z, u.b.z, u.d1.x, u.d1.y, u.v1.x, u.v1.y, P1.x, P1.y);
      step(u.a.w, u.b.w, u.d1.z, u.d1.w, u.v1.z, u.v1.w, P1.z, P1.w);
    };
    const int32_t nq = n >> 2;
    int32_t k = 0;
    if (nq >= 2 * kAq) {
      Quad ring[kAq];
#pragma unroll
      for (int t = 0; t < kAq; ++t) load(t, ring[t]);
      // the ring holds quads k .. k + kAq - 1, and k + kAq < nq
      for (; k + 2 * kAq <= nq; k += kAq) {
#pragma unroll
        for (int t = 0; t < kAq; ++t) {
          run(k + t, ring[t]);
          load(k + t + kAq, ring[t]);
        }
      }
#pragma unroll
      for (int t = 0; t < kAq; ++t) run(k + t, ring[t]);
      k += kAq;
    }
    for (; k < nq; ++k) {
      Quad u;
      load(k, u);
      run(k, u);
    }
    gf2* vv = (gf2*)vx;
    for (int32_t j = 4 * nq; j < n; ++j) {
      const v2 c = pd[j];
      v2 v;
      if constexpr (VS) {
        v = ((lf2*)vs)[j];
      } else {
        v = vv[j];
      }
      const v2 P = r1l[j];
      step(p1[j], p2[j], c.x, c.y, v.x, v.y, P.x, P.y);
    }
    return finish<COMP>(dr, di, cr, ci, n2, pdr, pdi, pn2, psc);
  }

  // GA: CC of up to kGather resident entries against the voxel, read by the
  // whole group: lane l takes readout pairs l, l + G, ... of every entry's
  // row (each load instruction covers G x 16 contiguous bytes of a row) and
  // of the voxel (shared by the entries), then the partial sums are reduced
  // over the group. Entries at or beyond `cnt` are skipped. Every lane
  // returns every result.
  static constexpr int kGather = 8;
  __device__ void gather_cc(const int64_t (&ks)[kGather], int cnt, float (&cv)[kGather],
                            float* pdr = nullptr, float* pdi = nullptr,
                            double* pn2 = nullptr) const {
    float dr[kGather], di[kGather];
    double n2[kGather];
#pragma unroll
    for (int e = 0; e < kGather; ++e) {
      dr[e] = di[e] = 0.0f;
      n2[e] = 0.0;
    }
    if constexpr (GA) {
      typedef float v4 __attribute__((ext_vector_type(4)));
      typedef float v2 __attribute__((ext_vector_type(2)));
      typedef const __attribute__((address_space(1))) v4 gf4;
      typedef const __attribute__((address_space(1))) v2 gf2;
      const int32_t n = pa.n_tr, nq = (n + 1) >> 1;
      gf4* row[kGather];
#pragma unroll
      for (int e = 0; e < kGather; ++e) row[e] = (gf4*)(dict.base + ks[e] * dict.ld4);
      gf2* vl = (gf2*)vx;
#pragma unroll 2
      for (int32_t t = lane; t < nq; t += G) {
        v4 d[kGather];
#pragma unroll
        for (int e = 0; e < kGather; ++e)
          if (e < cnt) d[e] = row[e][t];
        const v2 v0 = vl[2 * t];
        const bool pair = 2 * t + 1 < n;  // an odd readout count: the row's padding
        v2 v1 = {0.0f, 0.0f};
        if (pair) v1 = vl[2 * t + 1];
        const float vr0 = v0.x * vinv, vi0 = v0.y * vinv;
        const float vr1 = v1.x * vinv, vi1 = v1.y * vinv;
#pragma unroll
        for (int e = 0; e < kGather; ++e) {
          if (e < cnt) {
            v4 x = d[e];
            if (!pair) {
              x.z = 0.0f;
              x.w = 0.0f;
            }
            dr[e] = fmaf(vr0, x.x, fmaf(vi0, x.y, dr[e]));
            di[e] = fmaf(vi0, x.x, fmaf(-vr0, x.y, di[e]));
            dr[e] = fmaf(vr1, x.z, fmaf(vi1, x.w, dr[e]));
            di[e] = fmaf(vi1, x.z, fmaf(-vr1, x.w, di[e]));
            n2[e] = fma((double)x.x, (double)x.x, n2[e]);
            n2[e] = fma((double)x.y, (double)x.y, n2[e]);
            n2[e] = fma((double)x.z, (double)x.z, n2[e]);
            n2[e] = fma((double)x.w, (double)x.w, n2[e]);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < kGather; ++e) {
        if (e < cnt) {
          for (int o = G / 2; o > 0; o >>= 1) {
            dr[e] += __shfl_xor(dr[e], o, G);
            di[e] += __shfl_xor(di[e], o, G);
            n2[e] += __shfl_xor(n2[e], o, G);
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < kGather; ++e)
      cv[e] = n2[e] > 0.0
                  ? (float)(sqrt((double)dr[e] * dr[e] + (double)di[e] * di[e]) / sqrt(n2[e]))
                  : 0.0f;
    if (pdr) *pdr = dr[0];
    if (pdi) *pdi = di[0];
    if (pn2) *pn2 = n2[0];
  }

  // DI kernels simulate every candidate with the compensated dot product
  // (psc receives the distance score)
  __device__ float simulate_cc(const int32_t* i, float* pdr = nullptr, float* pdi = nullptr,
                               double* pn2 = nullptr, float* psc = nullptr) const {
    if constexpr (!SM) {
      if (pa.half) {
        if constexpr (G >= 16) {
          if (vs)
            return pa.dims[3] > 1 ? simulate_half<true, DI, 2>(i, pdr, pdi, pn2, psc)
                                  : simulate_half<false, DI, 2>(i, pdr, pdi, pn2, psc);
        }
        if (vx_scaled)
          return pa.dims[3] > 1 ? simulate_half<true, DI, 1>(i, pdr, pdi, pn2, psc)
                                : simulate_half<false, DI, 1>(i, pdr, pdi, pn2, psc);
        return pa.dims[3] > 1 ? simulate_half<true, DI, 0>(i, pdr, pdi, pn2, psc)
                              : simulate_half<false, DI, 0>(i, pdr, pdi, pn2, psc);
      }
    }
    if (pa.dims[3] > 1)
      return pa.x_axis ? simulate_cc_t<true, true, DI>(i, pdr, pdi, pn2, psc)
                       : simulate_cc_t<true, false, DI>(i, pdr, pdi, pn2, psc);
    return pa.x_axis ? simulate_cc_t<false, true, DI>(i, pdr, pdi, pn2, psc)
                     : simulate_cc_t<false, false, DI>(i, pdr, pdi, pn2, psc);
  }

  // Memo: this group's private open-addressing table in global memory. A
  // slot is 16 bytes, the key (voxel serial << 40 | entry index) and then
  // the value(s), so a probe and its value share a cache line; slots of
  // earlier voxels count as empty, so the table is never cleared between
  // voxels. Loads and stores are device-coherent (they bypass the
  // non-coherent L1).
  __device__ uint32_t memo_home(int64_t k) const {
    return (uint32_t)(((uint64_t)k * 0x9E3779B97F4A7C15ull) >> 40) & (uint32_t)(pa.memo_cap - 1);
  }
  __device__ int64_t* slot_key(uint32_t s) const { return GA ? mkey + s : mkey + 2 * (int64_t)s; }
  __device__ float* slot_val(uint32_t s) const {
    return GA ? mval + s : (float*)(mkey + 2 * (int64_t)s + 1);
  }
  // GA: the memo lives in LDS (one voxel group per wave), so a probe or a
  // store costs an LDS access instead of an L2 round trip.
  __device__ int64_t memo_ld_key(uint32_t s) const {
    if constexpr (GA) return mkey[s];
    return __hip_atomic_load(slot_key(s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // DI: both values of a slot are one 64-bit word (CC low, score high)
  __device__ float2 memo_ld_pair(uint32_t s) const {
    const uint64_t w = __hip_atomic_load((uint64_t*)slot_val(s), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return make_float2(__uint_as_float((uint32_t)w), __uint_as_float((uint32_t)(w >> 32)));
  }
  __device__ float memo_ld_val(uint32_t s) const {
    if constexpr (GA) return mval[s];
    if constexpr (DI) {
      const float2 p = memo_ld_pair(s);
      return obj == MRF_OBJ_DIST ? p.y : p.x;
    }
    return __hip_atomic_load(slot_val(s), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // rewrites a slot's key (its value stays): clears the look-ahead flag
  __device__ void memo_st_key(uint32_t s, int64_t kv) const {
    if constexpr (GA) {
      mkey[s] = kv;
    } else {
      __hip_atomic_store(slot_key(s), kv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __device__ void memo_st(uint32_t s, int64_t kv, float v, float v2 = 0.0f) const {
    if constexpr (GA) {
      mval[s] = v;
      mkey[s] = kv;
    } else {
      if constexpr (DI) {
        const uint64_t w = (uint64_t)__float_as_uint(v) | ((uint64_t)__float_as_uint(v2) << 32);
        __hip_atomic_store((uint64_t*)slot_val(s), w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        (void)v2;
        __hip_atomic_store(slot_val(s), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __hip_atomic_store(slot_key(s), kv, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }

  // Wave-level evaluation: every lane with `valid` asks for the value at i.
  // When the group simulates in this call, every lane of it that asks for
  // nothing new (no point, or a memo hit) takes a look-ahead point instead:
  // the free lane of rank r (counted from the group's lane 0) takes
  // more(r, q) when that returns true. Look-ahead entries go to the memo
  // only (never twice for one entry); each lane returns its own point's value.
  struct NoMore {
    __device__ bool operator()(int, int32_t*) const { return false; }
  };
  __device__ float eval(bool valid, const int32_t* i) { return eval(valid, i, NoMore()); }
  template <class More>
  __device__ float eval(bool valid, const int32_t* i, More&& more) {
    float val = -INFINITY;
    float nv = 0.0f, nv2 = 0.0f;  // a simulated entry's value(s), for the memo
    bool need = false, spec = false;
    bool first_read = false;  // a decision's first read of a look-ahead entry
    int64_t k = -1;
    int32_t pt[4] = {0, 0, 0, 0};
    const int32_t cap = pa.memo_cap;
    // probe the memo for k: the slot of a hit, -1 on a miss
    auto probe = [&](int64_t kk, int64_t& mk_out) -> int32_t {
      const int64_t tagged = tag | kk;
      uint32_t s = memo_home(kk);
      for (int32_t n = 0; n < cap; ++n) {
        const int64_t mk = memo_ld_key(s);
        if ((mk & ~kSpecBit) == tagged) {
          mk_out = mk;
          return (int32_t)s;
        }
        if ((mk & ~kIndexMask) != tag) break;  // empty for this voxel
        s = (s + 1) & (cap - 1);
      }
      return -1;
    };
    if (valid && in_range(i)) {
      k = key(i);
      for (int q = 0; q < 4; ++q) pt[q] = i[q];
      int64_t mk = 0;
      const int32_t s = probe(k, mk);
      need = s < 0;
      if (!need) {
        val = memo_ld_val((uint32_t)s);
        if (kLookAhead && (mk & kSpecBit)) {
          first_read = true;
          memo_st_key((uint32_t)s, tag | k);
        }
      }
    }
    uint64_t mspec = 0;
    if constexpr (kLookAhead) {
      if (grp_ballot<G>(need, gbase) != 0) {
        const uint64_t fm = grp_ballot<G>(!need, gbase);
        if (!need) {
          const int r = __popcll(fm & ((1ull << lane) - 1));
          int32_t q[4];
          if (more(r, q) && in_range(q)) {
            const int64_t kq = key(q);
            int64_t mk = 0;
            if (probe(kq, mk) < 0) {
              need = true;
              spec = true;
              k = kq;
              for (int a = 0; a < 4; ++a) pt[a] = q[a];
            }
          }
        }
        // one evaluation per entry: a look-ahead lane gives way to a lane
        // that asks for the same entry, and to a lower look-ahead lane
        bool drop = false;
        for (int o = 0; o < G; ++o) {
          const int64_t ko = __shfl(k, o, G);
          const int no = __shfl((int)need | ((int)spec << 1), o, G);
          if (spec && (no & 1) && ko == k && o != lane && (!(no & 2) || o < lane)) drop = true;
        }
        if (drop) need = spec = false;
        mspec = grp_ballot<G>(need && spec, gbase);
      }
    }
    if constexpr (GA) {
      // the group reads the needed entries together, kGather at a time
      uint64_t nm = grp_ballot<G>(need, gbase);
      while (nm) {
        int64_t ks[kGather];
        int srcs[kGather];
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < kGather; ++e) {
          srcs[e] = -1;
          if (nm) {
            srcs[e] = __ffsll((unsigned long long)nm) - 1;
            nm &= nm - 1;
            cnt = e + 1;
          }
          // unused slots repeat the first entry (a valid row, never read)
          ks[e] = __shfl(k, srcs[e] >= 0 ? srcs[e] : srcs[0], G);
        }
        float cv[kGather];
        gather_cc(ks, cnt, cv);
#pragma unroll
        for (int e = 0; e < kGather; ++e)
          if (lane == srcs[e]) val = nv = cv[e];
      }
    } else {
      if (need) {
        if constexpr (DI) {
          float sc = 0.0f;
          nv = simulate_cc(pt, nullptr, nullptr, nullptr, &sc);
          nv2 = sc;
          if (!spec) val = obj == MRF_OBJ_DIST ? sc : nv;
        } else {
          nv = simulate_cc(pt);
          if (!spec) val = nv;
        }
      }
    }
    uint64_t m = grp_ballot<G>(need, gbase);
    n_sim += __popcll(m & ~mspec) + __popcll(grp_ballot<G>(first_read, gbase));
    while (m) {
      const int src = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      const bool sp = (mspec >> src) & 1;
      const int64_t ks = __shfl(k, src, G);
      const float vv = __shfl(nv, src, G);
      const float v2 = DI ? __shfl(nv2, src, G) : 0.0f;
      // look-ahead entries keep to half the slots, so the entries that
      // decisions ask for still find room
      if (memo_count * 4 < cap * 3 && (!sp || memo_count * 2 < cap)) {
        if (lane == 0) {
          uint32_t s = memo_home(ks);
          while ((memo_ld_key(s) & ~kIndexMask) == tag) s = (s + 1) & (cap - 1);
          memo_st(s, tag | ks | (sp ? kSpecBit : 0), vv, v2);
        }
        ++memo_count;
      } else if (!sp) {
        overflow = true;
      }
    }
    wave_fence();  // the memo stores complete before later loads
    return val;
  }

  __device__ void need_centre() {
    if (!cknown) {
      const float v = eval(lane == 0, c);
      cval = __shfl(v, 0, G);
      cknown = true;
    }
  }

  __device__ void log_top2(float v, bool include_centre) {
    float b1, b2;
    grp_top2<G>(v, b1, b2);
    const int nf = __popcll(grp_ballot<G>(v > -INFINITY, gbase));
    if (include_centre) {
      const float c1 = cval;
      const float n1 = fmaxf(b1, c1);
      const float n2 = fmaxf(fminf(b1, c1), b2);
      b1 = n1;
      b2 = n2;
    }
    if (nf + (include_centre ? 1 : 0) >= 2) mm = fminf(mm, b1 - b2);
  }
  __device__ void log_pair(float x, float y) {
    if (x > -INFINITY && y > -INFINITY) mm = fminf(mm, fabsf(x - y));
  }

  // ---- stages --------------------------------------------------------------
  __device__ void scan_stride(int ax, int s) {
    s = s > 0 ? s : 1;
    const int32_t count = (hi[ax] - lo[ax]) / s + 1;
    float best = -INFINITY, r1 = -INFINITY, r2 = -INFINITY;
    int32_t bp = c[ax];
    int nf = 0;
    for (int32_t base = 0; base < count; base += G) {
      const int32_t q = base + lane;
      int32_t p[4] = {c[0], c[1], c[2], c[3]};
      p[ax] = lo[ax] + q * s;
      const float v = eval(q < count, p);
      float rb;
      const int src = grp_first_max<G>(v, rb, gbase);
      if (src >= 0 && rb > best) {  // earlier rounds hold lower indices: keep them on ties
        best = rb;
        bp = __shfl(p[ax], src, G);
      }
      float t1, t2;
      grp_top2<G>(v, t1, t2);
      const float n1 = fmaxf(r1, t1), n2 = fmaxf(fminf(r1, t1), fmaxf(r2, t2));
      r1 = n1;
      r2 = n2;
      nf += __popcll(grp_ballot<G>(v > -INFINITY, gbase));
    }
    if (nf >= 2) mm = fminf(mm, r1 - r2);
    if (best > -INFINITY) {
      c[ax] = bp;
      cval = best;
      cknown = true;
    }
  }

  // points given by a per-lane generator, in increasing index order; the
  // centre is kept on ties, then the lowest index wins
  template <typename Gen>
  __device__ void scan_points(int ax, int32_t count, Gen gen) {
    need_centre();
    float best = cval, r1 = cval, r2 = -INFINITY;
    int32_t bp = c[ax];
    int nf = 1;
    for (int32_t base = 0; base < count; base += G) {
      const int32_t q = base + lane;
      int32_t p[4] = {c[0], c[1], c[2], c[3]};
      p[ax] = q < count ? gen(q) : c[ax];
      const float v = eval(q < count, p);
      float rb;
      const int src = grp_first_max<G>(v, rb, gbase);
      if (src >= 0 && rb > best) {
        best = rb;
        bp = __shfl(p[ax], src, G);
      }
      float t1, t2;
      grp_top2<G>(v, t1, t2);
      const float n1 = fmaxf(r1, t1), n2 = fmaxf(fminf(r1, t1), fmaxf(r2, t2));
      r1 = n1;
      r2 = n2;
      nf += __popcll(grp_ballot<G>(v > -INFINITY, gbase));
    }
    if (nf >= 2) mm = fminf(mm, r1 - r2);
    c[ax] = bp;
    cval = best;
  }

  __device__ void scan_window(int ax, int s, int w) {
    s = s > 0 ? s : 1;
    const int32_t M = w / s;
    const int32_t cc0 = c[ax];
    // m in [m_lo, m_hi] \ {0} with lo <= c + m s <= hi
    int32_t m_lo = -M, m_hi = M;
    while (m_lo < 0 && cc0 + m_lo * s < lo[ax]) ++m_lo;
    while (m_hi > 0 && cc0 + m_hi * s > hi[ax]) --m_hi;
    const bool has0 = m_lo <= 0 && m_hi >= 0;
    const int32_t count = (m_hi - m_lo + 1) - (has0 ? 1 : 0);
    scan_points(ax, count, [&](int32_t q) {
      int32_t m = m_lo + q;
      if (has0 && m >= 0) m += 1;
      return cc0 + m * s;
    });
  }

  __device__ void scan_hops(int ax, double h) {
    h = h >= 1.0 ? h : 1.0;
    const int32_t cc0 = c[ax];
    int32_t nneg = 0, npos = 0;
    while (cc0 + round_half_away(-(double)(nneg + 1) * h) >= lo[ax]) ++nneg;
    while (cc0 + round_half_away((double)(npos + 1) * h) <= hi[ax]) ++npos;
    scan_points(ax, nneg + npos, [&](int32_t q) {
      if (q < nneg) return cc0 + round_half_away(-(double)(nneg - q) * h);
      return cc0 + round_half_away((double)(q - nneg + 1) * h);
    });
  }

  // ---- look-ahead points ---------------------------------------------------
  // The first decision of a zoom stage taken from the centre asks for
  // c -/+ s (1-D) or the 8 neighbours (2-D); a scan is not looked into.
  __device__ static int first_count(const mrf_zoom_stage& st) {
    return st.kind == MRF_ZOOM1 ? 2 : (st.kind == MRF_ZOOM2 ? 8 : 0);
  }
  __device__ void first_point(const mrf_zoom_stage& st, int q, int32_t* p) const {
    for (int a = 0; a < 4; ++a) p[a] = c[a];
    const int s0 = st.step0 > 0 ? st.step0 : 1;
    if (st.kind == MRF_ZOOM1) {
      p[st.axis0] += q == 0 ? -s0 : s0;
    } else {
      const int s1 = st.step1 > 0 ? st.step1 : 1;
      p[st.axis0] += nb_d0(q) * s0;
      p[st.axis1] += nb_d1(q) * s1;
    }
  }
  // points of the first decisions of the next two stages, up to a scan
  __device__ int ahead_count() const {
    int n = 0;
    for (int t = 0; t < n_nxt && t < 2; ++t) {
      const int m = first_count(nxt[t]);
      if (m == 0) break;
      n += m;
    }
    return n;
  }
  __device__ void ahead_point(int r, int32_t* p) const {
    for (int t = 0; t < n_nxt && t < 2; ++t) {
      const int m = first_count(nxt[t]);
      if (r < m) {
        first_point(nxt[t], r, p);
        return;
      }
      r -= m;
    }
  }
  // look-ahead point r of a 1-D zoom decision at c (step s on axis ax; dir
  // = the direction of the stage's last move, 0 before any): the next point
  // of the climb (both ways before a move), the next stages' first points,
  // then further along the climb
  __device__ void zoom1_ahead(int r, int ax, int s, int dir, int32_t* p) const {
    for (int a = 0; a < 4; ++a) p[a] = c[a];
    const int n0 = dir == 0 ? 2 : 1;
    if (r < n0) {
      p[ax] += (dir == 0 ? (r == 0 ? 2 : -2) : 2 * dir) * s;
      return;
    }
    r -= n0;
    const int na = ahead_count();
    if (r < na) {
      ahead_point(r, p);
      return;
    }
    r -= na;
    if (dir == 0) {
      const int m = 3 + r / 2;
      p[ax] += ((r & 1) ? -m : m) * s;
    } else {
      p[ax] += (3 + r) * dir * s;
    }
  }
  // look-ahead point r of a 2-D zoom decision at c: the points that become
  // neighbours after one more move along the last direction d (3 after a
  // move along an axis, 5 after a diagonal one; none before a move), then
  // the next stages' first points; false past them
  __device__ bool zoom2_ahead(int r, int a0, int a1, int s0, int s1, int d, int32_t* p) const {
    for (int a = 0; a < 4; ++a) p[a] = c[a];
    if (d >= 0) {
      for (int w = 0; w < 8; ++w) {
        const int e0 = nb_d0(d) + nb_d0(w), e1 = nb_d1(d) + nb_d1(w);
        if (e0 != 2 && e0 != -2 && e1 != 2 && e1 != -2) continue;
        if (r == 0) {
          p[a0] += e0 * s0;
          p[a1] += e1 * s1;
          return true;
        }
        --r;
      }
    }
    if (r < ahead_count()) {
      ahead_point(r, p);
      return true;
    }
    return false;
  }

  __device__ void move_to(const int32_t* p, float v) {
    for (int q = 0; q < 4; ++q) c[q] = p[q];
    cval = v;
  }

  __device__ void zoom1(int ax, int s, bool pruned) {
    s = s > 0 ? s : 1;
    need_centre();
    int dir = 0;
    for (int guard = 0; guard < (1 << 20); ++guard) {
      int32_t L[4] = {c[0], c[1], c[2], c[3]}, R[4] = {c[0], c[1], c[2], c[3]};
      L[ax] -= s;
      R[ax] += s;
      if (pruned) {
        // R first; L is the first look-ahead point
        const float vr = __shfl(eval(lane == 0, R,
                                     [&](int r, int32_t* q) {
                                       if (r == 0) {
                                         for (int a = 0; a < 4; ++a) q[a] = L[a];
                                       } else {
                                         zoom1_ahead(r - 1, ax, s, dir, q);
                                       }
                                       return true;
                                     }),
                                0, G);
        log_pair(vr, cval);
        if (vr > cval) {
          move_to(R, vr);
          dir = 1;
          continue;
        }
        const float vl = __shfl(eval(lane == 0, L), 0, G);
        log_pair(vl, cval);
        if (vl > cval) {
          move_to(L, vl);
          dir = -1;
          continue;
        }
        break;
      }
      int32_t P[4];
      for (int a = 0; a < 4; ++a) P[a] = lane == 0 ? L[a] : R[a];
      const float v = eval(lane < 2, P, [&](int r, int32_t* q) {
        zoom1_ahead(r, ax, s, dir, q);
        return true;
      });
      log_top2(lane < 2 ? v : -INFINITY, true);
      const float vl = __shfl(v, 0, G), vr = __shfl(v, 1, G);
      const bool right = vr > vl;
      const float bv = right ? vr : vl;
      if (bv > cval) {
        move_to(right ? R : L, bv);
        dir = right ? 1 : -1;
      } else {
        break;
      }
    }
  }

  // offsets of neighbour w in the order L, R, D, U, LD, LU, RD, RU
  __device__ static int nb_d0(int w) { return (w == 0 || w == 4 || w == 5) ? -1 : ((w == 1 || w >= 6) ? 1 : 0); }
  __device__ static int nb_d1(int w) { return (w == 2 || w == 4 || w == 6) ? -1 : ((w == 3 || w == 5 || w == 7) ? 1 : 0); }
  __device__ void neighbour(int w, int a0, int a1, int s0, int s1, int32_t* p) const {
    for (int q = 0; q < 4; ++q) p[q] = c[q] + (q == a0 ? nb_d0(w) * s0 : 0) + (q == a1 ? nb_d1(w) * s1 : 0);
  }

  // evaluate the neighbours in `mask` (bit w = neighbour w), one per lane;
  // the look-ahead takes the move's other neighbours first, then the
  // points of zoom2_ahead (d: the last move's direction, -1 before any)
  __device__ void eval_nb(uint32_t mask, int a0, int a1, int s0, int s1, int d) {
    int32_t p[4];
    neighbour(lane & 7, a0, a1, s0, s1, p);
    const bool mine = lane < 8 && ((mask >> lane) & 1u);
    const float v = eval(mine, p, [&](int r, int32_t* q) {
      for (int w = 0; w < 8; ++w) {
        if ((mask >> w) & 1u) continue;
        if (r == 0) {
          neighbour(w, a0, a1, s0, s1, q);
          return true;
        }
        --r;
      }
      return zoom2_ahead(r, a0, a1, s0, s1, d, q);
    });
    if (mine) nbv[lane] = v;
    wave_fence();
  }

  __device__ void zoom2(int a0, int a1, int s0, int s1, bool pruned) {
    s0 = s0 > 0 ? s0 : 1;
    s1 = s1 > 0 ? s1 : 1;
    need_centre();
    enum { NL = 0, NR, ND, NU, NLD, NLU, NRD, NRU };
    int d = -1;  // the last move's direction
    for (int guard = 0; guard < (1 << 20); ++guard) {
      if (!pruned) {
        int32_t p[4];
        neighbour(lane & 7, a0, a1, s0, s1, p);
        const float v = eval(lane < 8, p, [&](int r, int32_t* q) {
          return zoom2_ahead(r, a0, a1, s0, s1, d, q);
        });
        log_top2(lane < 8 ? v : -INFINITY, true);
        float bv;
        const int src = grp_first_max<G>(lane < 8 ? v : -INFINITY, bv, gbase);
        if (src >= 0 && bv > cval) {
          int32_t q[4];
          neighbour(src, a0, a1, s0, s1, q);
          move_to(q, bv);
          d = src;
        } else {
          break;
        }
        continue;
      }
      // evaluation-saving rules (Theory section)
      float* v = nbv;
      if (lane < 8) v[lane] = -INFINITY;
      wave_fence();
      const float C = cval;
      eval_nb((1u << NL) | (1u << ND), a0, a1, s0, s1, d);
      log_pair(v[NL], C);
      log_pair(v[ND], C);
      const bool upL = v[NL] > C, upD = v[ND] > C;
      int target = -1;
      uint32_t cand = 0;
      if (upL && upD) {
        cand = (1u << NL) | (1u << ND);
        eval_nb(1u << NLD, a0, a1, s0, s1, d);
        log_pair(v[NLD], C);
        if (v[NLD] > C) target = NLD;
      } else if (!upL && !upD) {
        eval_nb((1u << NR) | (1u << NU), a0, a1, s0, s1, d);
        log_pair(v[NR], C);
        log_pair(v[NU], C);
        const bool upR = v[NR] > C, upU = v[NU] > C;
        if (!upR && !upU) break;
        if (upR && upU) {
          cand = (1u << NR) | (1u << NU);
          eval_nb(1u << NRU, a0, a1, s0, s1, d);
          log_pair(v[NRU], C);
          if (v[NRU] > C) target = NRU;
        } else {
          target = upR ? NR : NU;
        }
      } else if (upL) {
        cand = 1u << NL;
        eval_nb(1u << NU, a0, a1, s0, s1, d);
        log_pair(v[NU], C);
        if (v[NU] > C) {
          cand |= 1u << NU;
          eval_nb(1u << NLU, a0, a1, s0, s1, d);
          log_pair(v[NLU], C);
          if (v[NLU] > C) target = NLU;
        } else {
          target = NL;
        }
      } else {
        cand = 1u << ND;
        eval_nb(1u << NR, a0, a1, s0, s1, d);
        log_pair(v[NR], C);
        if (v[NR] > C) {
          cand |= 1u << NR;
          eval_nb(1u << NRD, a0, a1, s0, s1, d);
          log_pair(v[NRD], C);
          if (v[NRD] > C) target = NRD;
        } else {
          target = ND;
        }
      }
      if (target < 0) {
        float bv = -INFINITY;
        for (int w = 0; w < 8; ++w)
          if (((cand >> w) & 1u) && v[w] > bv) {
            bv = v[w];
            target = w;
          }
        if (target < 0 || !(bv > C)) break;
      }
      int32_t q[4];
      neighbour(target, a0, a1, s0, s1, q);
      move_to(q, v[target]);
      d = target;
    }
  }

  __device__ void run_stage(const mrf_zoom_stage& st, bool pruned) {
    if constexpr (DI) {
      const int32_t o = st.objective == MRF_OBJ_DIST ? MRF_OBJ_DIST : MRF_OBJ_CC;
      if (o != obj) {
        // the centre's value under this stage's objective (a memo hit)
        obj = o;
        cknown = false;
      }
    }
    switch (st.kind) {
      case MRF_SCAN_STRIDE: scan_stride(st.axis0, st.step0); break;
      case MRF_SCAN_WINDOW: scan_window(st.axis0, st.step0, st.window); break;
      case MRF_SCAN_HOPS: scan_hops(st.axis0, st.hop); break;
      case MRF_ZOOM1: zoom1(st.axis0, st.step0, pruned); break;
      case MRF_ZOOM2: zoom2(st.axis0, st.axis1, st.step0, st.step1, pruned); break;
      default: break;
    }
  }
};

// Resets the work counter and stores the schedule (passed by value, so it is
// captured at launch) where the search kernel reads it.
__global__ void k_zoom_init(int32_t* counter, mrf_zoom_schedule sch, mrf_zoom_schedule* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *counter = 0;
    *dst = sch;
  }
}

// LDS bytes per voxel group: the per-start results and the neighbour values
// of one pruned move.
__host__ __device__ inline size_t zoom_group_lds() {
  return MRF_ZOOM_MAX_STARTS * (sizeof(int64_t) + sizeof(float)) + 8 * sizeof(float);
}

// Offset of the voxel rows (16-byte aligned) after the groups' LDS.
__host__ __device__ inline size_t zoom_vrow_offset(int ng) {
  return ((size_t)ng * zoom_group_lds() + 15) & ~(size_t)15;
}

// The gathering engine's memo: slots per wave, in LDS (a slice voxel visits
// ~150 entries; past 3/4 of the slots values are no longer kept and n_sim
// is reported negative, as with the global memo).
constexpr int32_t kGatherMemo = 1024;
__host__ __device__ inline size_t zoom_gather_memo_lds() {
  return (size_t)kGatherMemo * (sizeof(int64_t) + sizeof(float));
}

// One wave per block, 64 / G voxels per wave: each group of G lanes runs its
// own voxel's stage machine and pulls its own voxels from the queue, so the
// lanes that a decision leaves idle in one group work for the others.
// Groups of 8 lanes serve large voxel counts (many waves per SIMD): the
// kernel is then held to 256 VGPRs so that two waves share a SIMD and hide
// each other's load latency (measured on a 256 x 256 four-parameter slice:
// 518 -> 455 ms; at 128 VGPRs the spills cost 4x). Larger groups run one
// wave per SIMD and keep the whole register file.
template <int G, bool SM, bool GA, bool DI>
__global__ __launch_bounds__(64, (G <= 8 ? 2 : 1)) void k_zoom(ZoomArgs a) {
  constexpr int NG = 64 / G;
  extern __shared__ __align__(16) unsigned char sm[];
  const int lane = threadIdx.x;
  const int grp = lane / G, glane = lane % G, gbase = grp * G;
  unsigned char* gsm = sm + (size_t)grp * zoom_group_lds();
  int64_t* fin_k = (int64_t*)gsm;                                                  // [MAX_STARTS]
  float* fin_v = (float*)(fin_k + MRF_ZOOM_MAX_STARTS);                             // [MAX_STARTS]
  float* nbv = fin_v + MRF_ZOOM_MAX_STARTS;                                        // [8]
  const mrf_zoom_schedule* __restrict__ S = a.sch;
  // this group's memo; serial 0 marks never-used slots
  int64_t* mkey;
  float* mval;
  int32_t memo_cap;
  if constexpr (GA) {
    // one group per wave: the memo follows the group's LDS (8-byte aligned)
    static_assert(G == 64 || !GA, "the gathering engine runs one voxel group per wave");
    mkey = (int64_t*)(sm + ((NG * zoom_group_lds() + 7) & ~(size_t)7));
    mval = (float*)(mkey + kGatherMemo);
    memo_cap = kGatherMemo;
    for (int32_t i = lane; i < kGatherMemo; i += 64) mkey[i] = 0;
  } else {
    // 16-byte slots: two int64 words each (key, then the value words)
    mkey = a.memo_slots + ((int64_t)blockIdx.x * NG + grp) * a.memo_cap * 2;
    mval = nullptr;
    memo_cap = a.memo_cap;
    for (int32_t i = lane; i < NG * a.memo_cap; i += 64)
      __hip_atomic_store(a.memo_slots + ((int64_t)blockIdx.x * NG * a.memo_cap + i) * 2,
                         (int64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  int64_t serial = 0;

  const int32_t W = a.lat_w, H = a.lat_h, L = a.lat_stride;
  const int32_t lw = a.lat_pass ? (W + L - 1) / L : 0, lh = a.lat_pass ? (H + L - 1) / L : 0;
  for (;;) {
    int p = 0;
    if (glane == 0) p = atomicAdd(a.counter, 1);
    p = __shfl(p, 0, G);
    if (p >= a.n_items) break;
    // queue position -> voxel (slice-major raster order for the lattice passes)
    int v = p;
    int32_t prior_v = -1;
    if (a.lat_pass == 1) {
      const int32_t s = p / (lw * lh), r = p % (lw * lh);
      v = (s * H + (r / lw) * L) * W + (r % lw) * L;
    } else if (a.lat_pass == 2) {
      const int32_t x = v % W, y = (v / W) % H, s = v / (W * H);
      if (x % L == 0 && y % L == 0) continue;  // a lattice voxel: done in the first pass
      // nearest lattice voxel in Chebyshev distance, ties to the lower raster
      // index: D = the larger of the per-axis distances to the nearest lattice
      // line; every lattice voxel within D on both axes is a nearest one, and
      // the lowest raster index among them takes the lowest row, then column
      const int32_t qx = x / L, qy = y / L;
      const int32_t dx = min(x - qx * L, (qx + 1) * L < W ? (qx + 1) * L - x : L);
      const int32_t dy = min(y - qy * L, (qy + 1) * L < H ? (qy + 1) * L - y : L);
      const int32_t D = max(dx, dy);
      const int32_t px = (max(x - D, 0) + L - 1) / L * L;
      const int32_t py = (max(y - D, 0) + L - 1) / L * L;
      prior_v = (s * H + py) * W + px;
    }

    // the voxel's norm (FP64); the search reads the voxel scaled by 1 / norm.
    // Summed in an order that does not depend on the group size (so neither
    // does any result): group lane l < 8 adds readouts l, l + 8, ... in
    // turn, the eight partial sums are added pairwise, and lane 0's total is
    // broadcast to the group.
    const float2* src = a.vox + (int64_t)v * a.ld_vox;
    // this voxel's readouts: a batch may mix readout counts (prefixes of the
    // same sequence, whose tables are prefixes of the longest one's)
    // (clamped to the tables' [1, n_tr], so no table row is read past its end)
    const int32_t n = a.vox_n_tr ? min(max(a.vox_n_tr[v], 1), a.n_tr) : a.n_tr;
    double s2 = 0.0;
    if (glane < 8) {
      for (int32_t j = glane; j < n; j += 8) {
        const float2 x = src[j];
        s2 = fma((double)x.x, (double)x.x, s2);
        s2 = fma((double)x.y, (double)x.y, s2);
      }
    }
    for (int o = 4; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, G);
    s2 = __shfl(s2, 0, G);
    const double nv = sqrt(s2);
    const float inv = nv > 0.0 ? (float)(1.0 / nv) : 0.0f;
    ++serial;
    // the scaled voxel in the group's LDS row (the earlier voxel's reads
    // ended before the fence that closed its iteration)
    // (or in its workspace row: the group's lanes share the CU's L1, so the
    // workgroup fence makes the row visible to them)
    float2* vsh = nullptr;
    float2* vgl = nullptr;
    if (a.half && a.vrow) {
      vsh = (float2*)(sm + zoom_vrow_offset(NG) + (size_t)grp * a.vrow * sizeof(float2));
    } else if (a.half && a.vscaled) {
      vgl = a.vscaled + ((int64_t)blockIdx.x * NG + grp) * a.vrow_g;
    }
    if (float2* dst = vsh ? vsh : vgl) {
      for (int32_t j = glane; j < n; j += G) {
        const float2 x = src[j];
        dst[j] = make_float2(x.x * inv, x.y * inv);
      }
      wave_fence();
    }

    Engine<G, SM, GA, DI> e;
    e.pa.t1T = a.t1T;
    e.pa.t1ti = a.t1ti;
    e.pa.t2T = a.t2T;
    e.pa.dfT = a.dfT;
    e.pa.rf = a.rf;
    e.pa.n_tr = n;
    e.pa.tab_n = a.tab_n;
    e.pa.inversion = a.inversion;
    e.pa.x_axis = a.x_axis;
    e.pa.half = a.half;
    e.pa.tq = a.tq;
    e.pa.h1 = a.h1;
    e.pa.h2 = a.h2;
    e.pa.hd = a.hd;
    e.pa.xr = a.xr;
    if constexpr (SM) {
      e.sw = a.sm;
      e.dm = a.demod;
    }
    if constexpr (GA) e.dict = DictRows{a.dict, a.dict_ld4};
    e.pa.memo_cap = memo_cap;
    for (int q = 0; q < 4; ++q) e.pa.dims[q] = a.dims[q];

    e.vx = vgl ? vgl : src;
    e.vs = vsh;
    e.vx_scaled = vgl != nullptr;
    e.vinv = inv;
    e.vn = nv;
    e.obj = MRF_OBJ_CC;
    e.nxt = S->stages;
    e.n_nxt = 0;
    e.mkey = mkey;
    e.mval = mval;
    e.tag = serial << 40;
    e.nbv = nbv;
    e.lane = glane;
    e.gbase = gbase;
    e.memo_count = 0;
    e.n_sim = 0;
    e.overflow = false;
    e.mm = INFINITY;
    const bool has_init = a.init || a.init_flat || prior_v >= 0;
    int32_t ini[4] = {0, 0, 0, 0};
    if (a.init) {
      for (int q = 0; q < 4; ++q) ini[q] = a.init[4 * (int64_t)v + q];
    } else if (a.init_flat || prior_v >= 0) {
      // the first pass wrote the lattice voxel's result before this launch
      int64_t k = prior_v >= 0 ? a.idx[prior_v] : a.init_flat[v];
      if (k < 0) k = 0;  // a search that returned no entry: start at the grid origin
      for (int q = 3; q >= 0; --q) {
        ini[q] = (int32_t)(k % a.dims[q]);
        k /= a.dims[q];
      }
    }
    const int32_t* init = has_init ? ini : nullptr;
    for (int q = 0; q < 4; ++q) {
      e.lo[q] = 0;
      e.hi[q] = a.dims[q] - 1;
      if (init && S->prior_half[q] >= 0) {
        e.lo[q] = max(0, init[q] - S->prior_half[q]);
        e.hi[q] = min(a.dims[q] - 1, init[q] + S->prior_half[q]);
      }
    }
    const int n_starts = init ? 1 : S->n_starts;
    float bv = -INFINITY;
    int64_t bk = INT64_MAX;
    int32_t bi[4] = {0, 0, 0, 0};
    for (int st = 0; st < n_starts; ++st) {
      const int32_t* s0 = init ? init : S->starts[st];
      for (int q = 0; q < 4; ++q) e.c[q] = min(max(s0[q], e.lo[q]), e.hi[q]);
      e.cknown = false;
      e.obj = MRF_OBJ_CC;
      for (int i = 0; i < S->n_stages; ++i) {
        e.nxt = S->stages + i + 1;
        e.n_nxt = S->n_stages - i - 1;
        e.run_stage(S->stages[i], S->pruned != 0);
      }
      for (int r = 0; r < S->outer_max && S->n_outer > 0; ++r) {
        const int32_t b0 = e.c[0], b1 = e.c[1], b2 = e.c[2], b3 = e.c[3];
        for (int i = 0; i < S->n_outer; ++i) {
          e.nxt = S->outer + i + 1;
          e.n_nxt = S->n_outer - i - 1;
          e.run_stage(S->outer[i], S->pruned != 0);
        }
        if (b0 == e.c[0] && b1 == e.c[1] && b2 == e.c[2] && b3 == e.c[3]) break;
      }
      e.need_centre();
      const int64_t k = e.key(e.c);
      if (glane == 0) {
        fin_v[st] = e.cval;
        fin_k[st] = k;
      }
      if (e.cval > bv || (e.cval == bv && k < bk)) {
        bv = e.cval;
        bk = k;
        for (int q = 0; q < 4; ++q) bi[q] = e.c[q];
      }
    }
    wave_fence();
    for (int st = 0; st < n_starts; ++st)
      if (fin_k[st] != bk) e.log_pair(bv, fin_v[st]);

    // proton density of the found entry: <v, d> / ||d||^2 (and, for DI, its
    // CC: the search's last values may be distance scores)
    float dr = 0.0f, di = 0.0f;
    double n2 = 0.0;
    float cc_best = bv;
    if constexpr (GA) {
      if (a.pd_re || a.pd_im) {
        constexpr int KG = Engine<G, SM, GA, DI>::kGather;
        int64_t ks[KG];
        for (int q = 0; q < KG; ++q) ks[q] = bk;
        float cv[KG];
        e.gather_cc(ks, 1, cv, &dr, &di, &n2);
      }
    } else {
      if (glane == 0 && (DI || a.pd_re || a.pd_im)) {
        const float c1 = e.simulate_cc(bi, &dr, &di, &n2);
        if (DI) cc_best = c1;
      }
    }
    if (glane == 0) {
      a.idx[v] = bk;
      if (a.cc) a.cc[v] = cc_best;
      if (a.margin) a.margin[v] = e.mm;
      if (a.n_sim) a.n_sim[v] = e.overflow ? -e.n_sim : e.n_sim;
      if (a.pd_re) a.pd_re[v] = n2 > 0.0 ? (float)(nv * (double)dr / n2) : 0.0f;
      if (a.pd_im) a.pd_im[v] = n2 > 0.0 ? (float)(nv * (double)di / n2) : 0.0f;
    }
    wave_fence();
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <bool SM, bool GA, bool DI = false>
static void launch_zoom_groups(int group, int blocks, size_t lds, hipStream_t st,
                               const ZoomArgs& a) {
  if constexpr (GA) {
    (void)group;  // whole-wave groups (zoom_plan)
    hipLaunchKernelGGL((k_zoom<64, SM, GA, DI>), dim3(blocks), dim3(64), lds, st, a);
  } else {
    if (group == 8)
      hipLaunchKernelGGL((k_zoom<8, SM, GA, DI>), dim3(blocks), dim3(64), lds, st, a);
    else if (group == 16)
      hipLaunchKernelGGL((k_zoom<16, SM, GA, DI>), dim3(blocks), dim3(64), lds, st, a);
    else if (group == 32)
      hipLaunchKernelGGL((k_zoom<32, SM, GA, DI>), dim3(blocks), dim3(64), lds, st, a);
    else
      hipLaunchKernelGGL((k_zoom<64, SM, GA, DI>), dim3(blocks), dim3(64), lds, st, a);
  }
}

static int32_t h_round_half_away(double x) {
  return (int32_t)(x >= 0.0 ? std::floor(x + 0.5) : -std::floor(-x + 0.5));
}

static int32_t h_idx_step(double r, const mrf_axis& ax) {
  if (ax.n < 2) return 1;
  const double d = (ax.v[ax.n - 1] - ax.v[0]) / (double)(ax.n - 1);
  return std::max(1, h_round_half_away(r / d));
}

static int32_t h_nearest(const mrf_axis& ax, double v) {
  int32_t b = 0;
  for (int32_t i = 1; i < ax.n; ++i)
    if (std::fabs(ax.v[i] - v) < std::fabs(ax.v[b] - v)) b = i;
  return b;
}

static mrf_zoom_stage stage(int32_t kind, int32_t a0, int32_t a1, int32_t s0, int32_t s1,
                            int32_t w, double hop) {
  mrf_zoom_stage s;
  s.kind = kind;
  s.axis0 = a0;
  s.axis1 = a1;
  s.step0 = s0;
  s.step1 = s1;
  s.window = w;
  s.hop = hop;
  s.objective = MRF_OBJ_CC;
  return s;
}

// Launch plan: LDS per wave, persistent grid size and workspace layout
// (work counter | schedule copy | memo keys | memo values).
struct ZoomPlan {
  size_t lds;
  int blocks;
  int group;  // lanes per voxel
  int32_t cap;
  int32_t vrow;    // readouts per LDS voxel row (0: none)
  int32_t vrow_g;  // readouts per workspace voxel row (0: none)
  size_t off_sched, off_slots, off_vrow, total;
};

// Lanes per voxel: the smallest group (most voxels per wave) that still
// gives every SIMD a wave. A 2-D move evaluates up to 8 neighbours at once,
// so groups of 8 leave the fewest lanes idle once there are enough voxels
// (measured on the four-parameter volume: 8 lanes 825 ms, 16 lanes 1035 ms,
// 64 lanes 2233 ms per 256 x 256 slice; on a 64 x 64 slice 16 lanes, one
// wave per SIMD, beat 8 lanes, half a wave per SIMD).
constexpr int kZoomGroups[] = {8, 16, 32, 64};

static ZoomPlan zoom_plan(int n_cu, int32_t n_vox, int32_t n_tr, int64_t grid_entries,
                          bool gather = false) {
  ZoomPlan p;
  // memo slots per voxel group: fine 4-parameter grids make long unit-step walks
  p.cap = grid_entries > ((int64_t)1 << 26) ? 32768 : 4096;
  p.group = 64;
  // gathering: whole waves per voxel (each row read 1 KB per instruction)
  for (int g : kZoomGroups)
    if (!gather && ((int64_t)n_vox + 64 / g - 1) / (64 / g) >= 4 * (int64_t)n_cu) {
      p.group = g;
      break;
    }
  const int ng = 64 / p.group;
  p.lds = (size_t)ng * zoom_group_lds() + 16;
  if (gather) p.lds = ((p.lds + 7) & ~(size_t)7) + zoom_gather_memo_lds();
  // groups of 16 lanes and more (one wave per SIMD, four per CU) keep their
  // voxel in LDS when four waves' rows fit a CU's 160 KB
  p.vrow = 0;
  if (!gather && p.group >= 16 && n_tr > 0) {
    const int32_t vr = (n_tr + 3) / 4 * 4;
    const size_t with = zoom_vrow_offset(ng) + (size_t)ng * vr * sizeof(float2) + 16;
    if (4 * with <= 160 * 1024) {
      p.vrow = vr;
      p.lds = with;
    }
  }
  // persistent blocks: no more than can be resident (one wave per SIMD, two
  // for 8-lane groups), since a block that starts late finds the queue empty
  const int resident = gather ? 16 : (p.group <= 8 ? 8 : 4);
  const int per_cu = std::max(1, std::min(resident, (int)((160 * 1024) / p.lds)));
  const int64_t waves_needed = ((int64_t)n_vox + ng - 1) / ng;
  p.blocks = (int)std::max<int64_t>(1, std::min<int64_t>(waves_needed, (int64_t)n_cu * per_cu));
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t slots = (size_t)p.blocks * ng * p.cap;
  p.off_sched = 256;
  p.off_slots = al(p.off_sched + sizeof(mrf_zoom_schedule));
  // scaled voxel rows in the workspace when they are not in LDS
  p.vrow_g = (!gather && p.vrow == 0 && n_tr > 0) ? (n_tr + 3) / 4 * 4 : 0;
  p.off_vrow = al(p.off_slots + 16 * slots);
  p.total = al(p.off_vrow + sizeof(float2) * (size_t)p.blocks * ng * p.vrow_g);
  return p;
}

}  // namespace mrf

using namespace mrf;

extern "C" int mrf_zoom_schedule_paper(const mrf_grid* g, const mrf_sequence* seq,
                                       mrf_zoom_schedule* o) {
  int rc = check_grid(g);
  if (rc) return rc;
  MRF_CHECK_ARG(seq && o, "NULL argument");
  *o = mrf_zoom_schedule();
  const double omega = seq->omega_hz;  // 1000 / min TR
  const mrf_axis &T1 = g->t1_ms, &T2 = g->t2_ms, &DF = g->df_hz;
  const double ddf = DF.n > 1 ? (DF.v[DF.n - 1] - DF.v[0]) / (double)(DF.n - 1) : 1.0;
  int k = 0;
  // step 1: df at the starting T1/T2 (scan, narrow window, +-k omega hops)
  o->stages[k++] = stage(MRF_SCAN_STRIDE, 2, 0, h_idx_step(60.0, DF), 0, 0, 0.0);
  o->stages[k++] = stage(MRF_SCAN_WINDOW, 2, 0, h_idx_step(3.0, DF), 0, h_idx_step(75.0, DF), 0.0);
  const double hop = omega / ddf;
  o->stages[k++] = stage(MRF_SCAN_HOPS, 2, 0, 0, 0, 0, hop < 1.0 ? 1.0 : hop);
  // step 2: 2-D zoom at 200 then 100 ms
  o->stages[k++] = stage(MRF_ZOOM2, 0, 1, h_idx_step(200.0, T1), h_idx_step(200.0, T2), 0, 0.0);
  o->stages[k++] = stage(MRF_ZOOM2, 0, 1, h_idx_step(100.0, T1), h_idx_step(100.0, T2), 0, 0.0);
  // step 3: unit-step df scan over +-omega/2
  o->stages[k++] = stage(MRF_SCAN_WINDOW, 2, 0, 1, 0, h_idx_step(0.5 * omega, DF), 0.0);
  // step 4: interleaved 1-D zooms
  o->stages[k++] = stage(MRF_ZOOM1, 0, 0, h_idx_step(100.0, T1), 0, 0, 0.0);
  o->stages[k++] = stage(MRF_ZOOM1, 1, 0, h_idx_step(100.0, T2), 0, 0, 0.0);
  const double fine[3] = {50.0, 20.0, 10.0};
  for (double r : fine) o->stages[k++] = stage(MRF_ZOOM1, 0, 0, h_idx_step(r, T1), 0, 0, 0.0);
  for (double r : fine) o->stages[k++] = stage(MRF_ZOOM1, 1, 0, h_idx_step(r, T2), 0, 0, 0.0);
  if (g->b1.n > 1) {
    const double b1s[5] = {0.1, 0.05, 0.02, 0.01, 0.005};
    for (double r : b1s) o->stages[k++] = stage(MRF_ZOOM1, 3, 0, h_idx_step(r, g->b1), 0, 0, 0.0);
  }
  // step 5: final 2-D zoom at the finest resolution
  o->stages[k++] = stage(MRF_ZOOM2, 0, 1, 1, 1, 0, 0.0);
  o->n_stages = k;
  if (g->b1.n > 1) {
    o->outer[0] = stage(MRF_ZOOM2, 0, 1, 1, 1, 0, 0.0);
    o->outer[1] = stage(MRF_ZOOM1, 3, 0, 1, 0, 0, 0.0);
    o->outer[2] = stage(MRF_SCAN_WINDOW, 2, 0, 1, 0, h_idx_step(0.5 * omega, DF), 0.0);
    o->n_outer = 3;
    o->outer_max = 3;
  }
  o->n_starts = 1;
  o->starts[0][0] = h_nearest(T1, 1000.0);
  o->starts[0][1] = h_nearest(T2, 500.0);
  o->starts[0][2] = 0;
  o->starts[0][3] = g->b1.n > 1 ? h_nearest(g->b1, 1.0) : 0;
  o->pruned = 0;
  for (int a = 0; a < 4; ++a) o->prior_half[a] = -1;
  return MRF_OK;
}

extern "C" int mrf_zoom_schedule_prior(const mrf_grid* g, const double* half,
                                       mrf_zoom_schedule* o) {
  int rc = check_grid(g);
  if (rc) return rc;
  MRF_CHECK_ARG(o, "NULL argument");
  // Experiment 3: T1p +- 3000 ms, T2p +- 800 ms, dfp +- 150 Hz (B1 +- 0.3)
  static const double kPaper[4] = {3000.0, 800.0, 150.0, 0.3};
  const double* h = half ? half : kPaper;
  const mrf_axis* ax[4] = {&g->t1_ms, &g->t2_ms, &g->df_hz, &g->b1};
  int32_t out[4];
  for (int a = 0; a < 4; ++a) {
    MRF_CHECK_ARG(!std::isnan(h[a]), "half width %d is NaN", a);
    // an axis of one value (or none) is searched whole; so is a negative width
    out[a] = (ax[a]->n < 2 || h[a] < 0.0) ? -1 : h_idx_step(h[a], *ax[a]);
  }
  for (int a = 0; a < 4; ++a) o->prior_half[a] = out[a];
  return MRF_OK;
}

extern "C" int mrf_zoom_schedule_multistart(const mrf_grid* g, const mrf_sequence* seq,
                                            int32_t n_t1, int32_t n_t2, int32_t outer_max,
                                            mrf_zoom_schedule* o) {
  int rc = mrf_zoom_schedule_paper(g, seq, o);
  if (rc) return rc;
  MRF_CHECK_ARG(n_t1 >= 1 && n_t2 >= 1 && n_t1 * n_t2 <= MRF_ZOOM_MAX_STARTS,
                "need 1 <= n_t1 * n_t2 <= %d starts", MRF_ZOOM_MAX_STARTS);
  MRF_CHECK_ARG(outer_max >= 0 && outer_max <= 64, "outer_max must be in [0, 64]");
  // starts: an n_t1 x n_t2 lattice of grid indices spanning each axis from
  // its first to its last value (a single start sits at the middle)
  auto lattice = [](int32_t k, int32_t n, int32_t q) {
    if (k == 1) return (n - 1) / 2;
    return h_round_half_away((double)q * (double)(n - 1) / (double)(k - 1));
  };
  const int32_t b1 = o->starts[0][3];
  o->n_starts = n_t1 * n_t2;
  for (int32_t a = 0; a < n_t1; ++a)
    for (int32_t b = 0; b < n_t2; ++b) {
      int32_t* st = o->starts[a * n_t2 + b];
      st[0] = lattice(n_t1, g->t1_ms.n, a);
      st[1] = lattice(n_t2, g->t2_ms.n, b);
      st[2] = 0;
      st[3] = b1;
    }
  // outer rounds: the df window and fine df scans of step 1 and step 3,
  // then 2-D zooms from 100 ms down to the unit step (and the unit B1 zoom)
  const mrf_axis &T1 = g->t1_ms, &T2 = g->t2_ms;
  int k = 0;
  o->outer[k++] = o->stages[1];
  o->outer[k++] = o->stages[5];
  const double rs[4] = {100.0, 50.0, 20.0, 10.0};
  for (double r : rs)
    o->outer[k++] = stage(MRF_ZOOM2, 0, 1, h_idx_step(r, T1), h_idx_step(r, T2), 0, 0.0);
  o->outer[k++] = stage(MRF_ZOOM2, 0, 1, 1, 1, 0, 0.0);
  if (g->b1.n > 1) o->outer[k++] = stage(MRF_ZOOM1, 3, 0, 1, 0, 0, 0.0);
  o->n_outer = k;
  o->outer_max = outer_max;
  return MRF_OK;
}

extern "C" int mrf_zoom_schedule_finest_objective(mrf_zoom_schedule* o, int32_t objective) {
  MRF_CHECK_ARG(o, "NULL argument");
  MRF_CHECK_ARG(objective == MRF_OBJ_CC || objective == MRF_OBJ_DIST,
                "objective must be MRF_OBJ_CC or MRF_OBJ_DIST");
  MRF_CHECK_ARG(o->n_stages >= 0 && o->n_stages <= MRF_ZOOM_MAX_STAGES &&
                    o->n_outer >= 0 && o->n_outer <= MRF_ZOOM_MAX_STAGES,
                "bad stage counts");
  auto finest = [](const mrf_zoom_stage& st) {
    switch (st.kind) {
      case MRF_ZOOM2: return st.step0 <= 1 && st.step1 <= 1;
      case MRF_ZOOM1:
      case MRF_SCAN_WINDOW:
      case MRF_SCAN_STRIDE: return st.step0 <= 1;
      default: return false;
    }
  };
  for (int i = 0; i < o->n_stages; ++i)
    if (finest(o->stages[i])) o->stages[i].objective = objective;
  for (int i = 0; i < o->n_outer; ++i)
    if (finest(o->outer[i])) o->outer[i].objective = objective;
  return MRF_OK;
}

extern "C" int mrf_zoom_schedule_local(const mrf_grid* g, int32_t outer_max,
                                       mrf_zoom_schedule* o) {
  int rc = check_grid(g);
  if (rc) return rc;
  MRF_CHECK_ARG(o, "NULL argument");
  MRF_CHECK_ARG(outer_max >= 0 && outer_max <= 64, "outer_max must be in [0, 64]");
  *o = mrf_zoom_schedule();
  int k = 0;
  o->stages[k++] = stage(MRF_ZOOM2, 0, 1, 1, 1, 0, 0.0);
  o->stages[k++] = stage(MRF_ZOOM1, 2, 0, 1, 0, 0, 0.0);
  if (g->b1.n > 1) o->stages[k++] = stage(MRF_ZOOM1, 3, 0, 1, 0, 0, 0.0);
  o->n_stages = k;
  for (int i = 0; i < k; ++i) o->outer[i] = o->stages[i];
  o->n_outer = k;
  o->outer_max = outer_max;
  o->n_starts = 1;
  o->starts[0][0] = g->t1_ms.n / 2;
  o->starts[0][1] = g->t2_ms.n / 2;
  o->starts[0][2] = g->df_hz.n / 2;
  o->starts[0][3] = g->b1.n > 1 ? g->b1.n / 2 : 0;
  o->pruned = 0;
  for (int a = 0; a < 4; ++a) o->prior_half[a] = -1;
  return MRF_OK;
}

static int check_schedule(const mrf_zoom_schedule* s, const int32_t* dims) {
  MRF_CHECK_ARG(s != nullptr, "schedule is NULL");
  MRF_CHECK_ARG(s->n_stages >= 0 && s->n_stages <= MRF_ZOOM_MAX_STAGES, "bad n_stages");
  MRF_CHECK_ARG(s->n_outer >= 0 && s->n_outer <= MRF_ZOOM_MAX_STAGES, "bad n_outer");
  MRF_CHECK_ARG(s->outer_max >= 0 && s->outer_max <= 64, "outer_max must be in [0, 64]");
  MRF_CHECK_ARG(s->n_starts >= 1 && s->n_starts <= MRF_ZOOM_MAX_STARTS, "bad n_starts");
  for (int l = 0; l < 2; ++l) {
    const mrf_zoom_stage* st = l ? s->outer : s->stages;
    const int n = l ? s->n_outer : s->n_stages;
    for (int i = 0; i < n; ++i) {
      MRF_CHECK_ARG(st[i].kind >= MRF_SCAN_STRIDE && st[i].kind <= MRF_ZOOM2,
                    "stage %d: unknown kind %d", i, st[i].kind);
      MRF_CHECK_ARG(st[i].axis0 >= 0 && st[i].axis0 < 4 && st[i].axis1 >= 0 && st[i].axis1 < 4,
                    "stage %d: axis out of range", i);
      MRF_CHECK_ARG(st[i].kind != MRF_ZOOM2 || st[i].axis0 != st[i].axis1,
                    "stage %d: a 2-D zoom needs two different axes", i);
      MRF_CHECK_ARG(st[i].window >= 0 && std::isfinite(st[i].hop), "stage %d: bad window/hop", i);
      MRF_CHECK_ARG(st[i].objective == MRF_OBJ_CC || st[i].objective == MRF_OBJ_DIST,
                    "stage %d: unknown objective %d", i, st[i].objective);
    }
  }
  for (int i = 0; i < s->n_starts; ++i)
    for (int a = 0; a < 4; ++a)
      MRF_CHECK_ARG(s->starts[i][a] >= 0 && s->starts[i][a] < dims[a],
                    "start %d: index %d out of range on axis %d", i, s->starts[i][a], a);
  return MRF_OK;
}

extern "C" int mrf_zoom_workspace(mrf_context* ctx, const mrf_grid* grid, int32_t n_vox,
                                  int32_t n_tr, size_t* bytes) {
  MRF_CHECK_ARG(ctx && bytes, "NULL argument");
  int rc = check_grid(grid);
  if (rc) return rc;
  MRF_CHECK_ARG(n_vox >= 0 && n_tr >= 1, "bad sizes");
  // enough for the simulating and the gathering engine
  const int64_t E = grid_size_checked(grid);
  *bytes = std::max(zoom_plan(ctx->n_cu, n_vox, n_tr, E).total,
                    zoom_plan(ctx->n_cu, n_vox, n_tr, E, true).total);
  return MRF_OK;
}

// dict == NULL: candidates are simulated (seq required); otherwise they are
// read from the resident entry-major dictionary (seq unused).
static int zoom_search(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid,
                       const mrf_zoom_schedule* sched, const void* vox, int32_t n_vox,
                       int64_t ld_vox, int32_t n_tr, const int32_t* init_idx,
                       const int64_t* init_flat, mrf_result_view out, void* workspace,
                       size_t ws_bytes, void* stream, const int32_t* lattice = nullptr,
                       const mrf_dict_view* dict = nullptr, const int32_t* vox_n_tr = nullptr) {
  MRF_CHECK_ARG(ctx && (seq || dict), "context and sequence (or dictionary) must not be NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  const int32_t dims[4] = {grid->t1_ms.n, grid->t2_ms.n, grid->df_hz.n,
                           grid->b1.n > 0 ? grid->b1.n : 1};
  rc = check_schedule(sched, dims);
  if (rc) return rc;
  if (dict) {
    MRF_CHECK_ARG(dict->dtype == MRF_F32_ROWS,
                  "the resident dictionary must be MRF_F32_ROWS (entry-major rows)");
    MRF_CHECK_ARG(dict->entry_base == 0 && dict->n_entries == grid_size_checked(grid),
                  "the resident dictionary must hold the whole grid (entries 0..%lld)",
                  (long long)grid_size_checked(grid) - 1);
    MRF_CHECK_ARG(n_tr >= 1 && n_tr <= dict->n_tr, "n_tr %d must be in [1, %d]", n_tr,
                  dict->n_tr);
    MRF_CHECK_ARG(dict->ld >= dict->n_tr && dict->ld % 2 == 0, "dictionary ld must be even and >= n_tr");
    MRF_CHECK_ARG(dict->re && ((uintptr_t)dict->re & 15) == 0,
                  "dictionary rows must be a 16-byte aligned device pointer");
  } else {
    MRF_CHECK_ARG(n_tr >= 1 && n_tr <= seq->n, "n_tr %d must be in [1, %d]", n_tr, seq->n);
  }
  MRF_CHECK_ARG(n_vox >= 0, "n_vox must be >= 0");
  if (n_vox == 0) return MRF_OK;
  MRF_CHECK_ARG(vox != nullptr && out.idx != nullptr, "vox and out.idx must not be NULL");
  MRF_CHECK_ARG(ld_vox >= n_tr, "ld_vox must be >= n_tr");
  bool dist = false;  // any stage scored by the distance objective
  for (int i = 0; i < sched->n_stages; ++i) dist |= sched->stages[i].objective == MRF_OBJ_DIST;
  for (int i = 0; i < sched->n_outer; ++i) dist |= sched->outer[i].objective == MRF_OBJ_DIST;
  MRF_CHECK_ARG(!vox_n_tr || dict || !seq->smooth,
                "per-voxel readout counts need a sequence without smoothing");
  if (dist && (dict || seq->smooth)) {
    set_error("distance-objective stages need the simulating search without smoothing");
    return MRF_ERR_UNSUPPORTED;
  }
  const ZoomPlan plan = zoom_plan(ctx->n_cu, n_vox, n_tr, grid_size_checked(grid), dict != nullptr);
  MRF_CHECK_ARG(workspace != nullptr && ws_bytes >= plan.total,
                "workspace too small (%zu < %zu bytes)", ws_bytes, plan.total);
  hipStream_t st = (hipStream_t)stream;
  static const Tables no_tables;
  const Tables* t = &no_tables;
  TablesRef tref;  // held until the launches are enqueued
  if (!dict) {
    rc = get_tables(const_cast<mrf_sequence*>(seq), grid, n_tr, st, &tref);
    if (rc) return rc;
    t = tref.get();
  }

  ZoomArgs a;
  a.t1T = t->t1T;
  a.t1ti = t->t1ti;
  a.t2T = t->t2T;
  a.dfT = t->dfT;
  a.rf = t->rf;
  a.n_tr = n_tr;
  a.tab_n = n_tr;  // the tables (or rows) hold n_tr readouts; voxels may use prefixes
  a.vox_n_tr = vox_n_tr;
  a.inversion = t->inversion;
  a.x_axis = t->x_axis_pulses;
  a.tq = t->tq;
  a.h1 = t->h1;
  a.h2 = t->h2;
  a.hd = t->hd;
  a.xr = t->xr;
  a.vrow = plan.vrow;
  a.vrow_g = plan.vrow_g;
  a.vscaled = plan.vrow_g ? (float2*)((char*)workspace + plan.off_vrow) : nullptr;
  a.half = (!dict && !t->smooth && t->h1 && t->h2 && t->hd && t->xr &&
            (uintptr_t)vox % 16 == 0 && ld_vox % 2 == 0)
               ? 1
               : 0;
  a.sm = smooth_weights(t->smooth ? t->smooth : 3, n_tr);
  a.demod = t->demod;
  a.dict = dict ? (const float4*)dict->re : nullptr;
  a.dict_ld4 = dict ? dict->ld / 2 : 0;
  for (int q = 0; q < 4; ++q) a.dims[q] = dims[q];
  a.vox = (const float2*)vox;
  a.ld_vox = ld_vox;
  a.n_vox = n_vox;
  a.init = init_idx;
  a.init_flat = init_flat;
  a.n_items = n_vox;
  a.lat_pass = 0;
  a.lat_w = lattice ? lattice[0] : 1;
  a.lat_h = lattice ? lattice[1] : 1;
  a.lat_stride = lattice ? lattice[3] : 1;
  a.idx = out.idx;
  a.cc = out.cc;
  a.margin = out.margin;
  a.pd_re = out.pd_re;
  a.pd_im = out.pd_im;
  a.n_sim = out.n_sim;
  char* ws = (char*)workspace;
  a.counter = (int32_t*)ws;
  a.memo_cap = plan.cap;
  a.memo_slots = (int64_t*)(ws + plan.off_slots);
  mrf_zoom_schedule* dsch = (mrf_zoom_schedule*)(ws + plan.off_sched);
  a.sch = dsch;
  const int blocks = plan.blocks;
  const size_t lds = plan.lds;
  hipLaunchKernelGGL(k_zoom_init, dim3(1), dim3(64), 0, st, a.counter, *sched, dsch);
  MRF_HIP(hipGetLastError());
  auto launch = [&]() {
    ProfScope prof(ctx, "k_zoom", st);
    if (dict)
      launch_zoom_groups<false, true>(plan.group, blocks, lds, st, a);
    else if (t->smooth)
      launch_zoom_groups<true, false>(plan.group, blocks, lds, st, a);
    else if (dist)
      launch_zoom_groups<false, false, true>(plan.group, blocks, lds, st, a);
    else
      launch_zoom_groups<false, false>(plan.group, blocks, lds, st, a);
  };
  if (!lattice) {
    launch();
  } else {
    // pass 1: the lattice voxels, no prior
    const int32_t L = lattice[3];
    a.lat_pass = 1;
    a.n_items = lattice[2] * ((lattice[0] + L - 1) / L) * ((lattice[1] + L - 1) / L);
    launch();
    MRF_HIP(hipGetLastError());
    // pass 2: every other voxel from its nearest lattice voxel's result
    hipLaunchKernelGGL(k_zoom_init, dim3(1), dim3(64), 0, st, a.counter, *sched, dsch);
    MRF_HIP(hipGetLastError());
    a.lat_pass = 2;
    a.n_items = n_vox;
    launch();
  }
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}

extern "C" int mrf_zoom_search(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid,
                               const mrf_zoom_schedule* sched, const void* vox, int32_t n_vox,
                               int64_t ld_vox, int32_t n_tr, const int32_t* init_idx,
                               mrf_result_view out, void* workspace, size_t ws_bytes,
                               void* stream) {
  return zoom_search(ctx, seq, grid, sched, vox, n_vox, ld_vox, n_tr, init_idx, nullptr, out,
                     workspace, ws_bytes, stream);
}

extern "C" int mrf_zoom_search_ragged(mrf_context* ctx, const mrf_sequence* seq,
                                      const mrf_grid* grid, const mrf_zoom_schedule* sched,
                                      const void* vox, int32_t n_vox, int64_t ld_vox,
                                      int32_t n_tr_max, const int32_t* vox_n_tr,
                                      mrf_result_view out, void* workspace, size_t ws_bytes,
                                      void* stream) {
  MRF_CHECK_ARG(vox_n_tr != nullptr || n_vox == 0, "vox_n_tr must not be NULL");
  return zoom_search(ctx, seq, grid, sched, vox, n_vox, ld_vox, n_tr_max, nullptr, nullptr, out,
                     workspace, ws_bytes, stream, nullptr, nullptr, vox_n_tr);
}

extern "C" int mrf_zoom_search_dict(mrf_context* ctx, const mrf_dict_view* dict,
                                    const mrf_grid* grid, const mrf_zoom_schedule* sched,
                                    const void* vox, int32_t n_vox, int64_t ld_vox, int32_t n_tr,
                                    const int32_t* init_idx, mrf_result_view out,
                                    void* workspace, size_t ws_bytes, void* stream) {
  MRF_CHECK_ARG(dict != nullptr, "dict must not be NULL");
  return zoom_search(ctx, nullptr, grid, sched, vox, n_vox, ld_vox, n_tr, init_idx, nullptr, out,
                     workspace, ws_bytes, stream, nullptr, dict);
}

extern "C" int mrf_zoom_search_from(mrf_context* ctx, const mrf_sequence* seq,
                                    const mrf_grid* grid, const mrf_zoom_schedule* sched,
                                    const void* vox, int32_t n_vox, int64_t ld_vox, int32_t n_tr,
                                    const int64_t* start_idx, mrf_result_view out,
                                    void* workspace, size_t ws_bytes, void* stream) {
  MRF_CHECK_ARG(start_idx != nullptr || n_vox == 0, "start_idx must not be NULL");
  return zoom_search(ctx, seq, grid, sched, vox, n_vox, ld_vox, n_tr, nullptr, start_idx, out,
                     workspace, ws_bytes, stream);
}

extern "C" int mrf_zoom_search_lattice(mrf_context* ctx, const mrf_sequence* seq,
                                       const mrf_grid* grid, const mrf_zoom_schedule* sched,
                                       const void* vox, int32_t width, int32_t height,
                                       int32_t n_slices, int64_t ld_vox, int32_t n_tr,
                                       int32_t stride, mrf_result_view out, void* workspace,
                                       size_t ws_bytes, void* stream) {
  MRF_CHECK_ARG(width >= 1 && height >= 1 && n_slices >= 1, "volume sizes must be >= 1");
  MRF_CHECK_ARG(stride >= 1 && stride <= 64, "stride must be in [1, 64]");
  const int64_t n = (int64_t)width * height * n_slices;
  MRF_CHECK_ARG(n <= INT32_MAX, "too many voxels in one call");
  const int32_t lat[4] = {width, height, n_slices, stride};
  return zoom_search(ctx, seq, grid, sched, vox, (int32_t)n, ld_vox, n_tr, nullptr, nullptr, out,
                     workspace, ws_bytes, stream, lat);
}
