// K1: dictionary simulation (Appendix Eq. A2 per entry) and on-the-fly
// simulation of fingerprints at arbitrary parameter values.
//
// One thread runs the readout recursion of two entries in registers (FP32
// state, FP32 partial sums of |m|^2 over four readouts added into FP64). A
// block of 512 threads owns 1024 consecutive entries: thread t takes entries
// t and t + 512, so every store instruction of a wavefront writes one
// contiguous 256 B (FP32 plane row) or 1 KB (BF16 four-readout block) run.
// (512-thread blocks share each staged df chunk among twice the entries of
// 256-thread ones and measure a few percent faster.)
//
// The kernel is bound by its HBM writes. Three things keep it there:
//  - stores are non-temporal buffer stores: the write stream does not evict
//    the step tables from L2, and a per-row buffer range drops the ragged tail
//    without branches;
//  - the df table (the widest, 16 B per entry and readout) is staged through
//    LDS eight readouts at a time, prefetched into registers one chunk ahead;
//  - table rows, pulse matrices and store rows are addressed from scalar
//    registers, so the per-readout vector work is the Bloch update itself.
#include <hip/hip_runtime.h>

#include <cmath>

#include "bloch.h"
#include "compensated.h"
#include "internal.h"
#include "sim_kernels.h"
#include "smooth.h"

namespace mrf {

namespace {

constexpr int kThreads = 512;
constexpr int kQ = 2;                              // entries per thread
constexpr int kBlockEntries = kThreads * kQ;
constexpr int kChunk = 8;                          // readouts per staged df chunk
constexpr int kChunkRows = 16;                     // MODE 4: one 128-byte line per entry
constexpr int kLdsMaxN3 = 128;                     // longest df axis staged through LDS
// readouts per chunk: MODE 4 stages 16 outputs per entry (a full line of its row)
template <int MODE>
constexpr int chunk_of() { return MODE == 4 ? kChunkRows : kChunk; }
constexpr int kRsrcWord3 = 0x00020000;             // raw 32-bit buffer format

// pulse kinds: general 3x3 or x-axis rotation, one matrix per wavefront
// (no B1 axis: read through the scalar cache) or one per lane (B1 axis)
enum PulseKind { kGeneralUniform = 0, kXAxisUniform = 1, kGeneralLane = 2, kXAxisLane = 3 };

typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, int32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, kRsrcWord3);
}

__device__ __forceinline__ float2 load2(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

__device__ __forceinline__ float4 load4(rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

constexpr int kNonTemporal = 2;  // buffer cache-policy bit: streaming store

__device__ __forceinline__ void store1(float v, rsrc_t r, uint32_t voff) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, 0, kNonTemporal);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store4(const uint32_t w[4], rsrc_t r, uint32_t voff) {
  const u32x4 v = {w[0], w[1], w[2], w[3]};
  __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, 0, kNonTemporal);
}

// LDS writes visible to the block; s_barrier without the full fence of
// __syncthreads, which would also wait for every outstanding HBM store.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Round-to-nearest-even to BF16, two values per instruction (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  const f32x2_t v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
}

// Entry k -> per-axis indices (B1 fastest, then df, T2, T1).
__device__ __forceinline__ void unravel(int64_t k, int32_t n2, int32_t n3, int32_t n4, int32_t& i1,
                                        int32_t& i2, int32_t& i3, int32_t& i4) {
  i4 = (int32_t)(k % n4);
  k /= n4;
  i3 = (int32_t)(k % n3);
  k /= n3;
  i2 = (int32_t)(k % n2);
  i1 = (int32_t)(k / n2);
}

// x-axis pulse: with R00 = 1 and R01 = R02 = R10 = R20 = 0 exactly, the
// general product rounds to the same values (the zero terms add exact zeros).
template <int PK>
__device__ __forceinline__ void pulse(Spin& m, const float* __restrict__ R) {
  if (PK == kXAxisUniform || PK == kXAxisLane) {
    const float y = m.y, z = m.z;
    m.y = fmaf(R[5], z, R[4] * y);
    m.z = fmaf(R[8], z, R[7] * y);
  } else {
    rf_pulse(m, R);
  }
}

}  // namespace

struct SimArgs {
  int32_t n_tr, n1, n2, n3, n4, inversion, unit_norm;
  int32_t t1_bytes, t2_bytes, df_bytes;  // table extents (buffer ranges)
  int64_t k0, count, ld;
  float* re;        // F32 planar
  float* im;
  uint4* packed;    // BF16 blocks
  double* norm;
  double* norm_b;   // MODE 5: the norm of the stored BF16 values
  float* cc;        // CC map output (MODE 3)
  SmoothW sm;       // temporal smoothing weights (SM kernels)
  const float2* demod;  // [n_tr] (cos, sin) of the RF phases (SM kernels)
};

struct EntryState {
  uint32_t o1[kQ], o2[kQ], i3[kQ];  // byte offsets into the t1/t2 rows, df column
  const float* rq[kQ];              // per-lane pulse matrices (B1 axis)
  float r1ti[kQ];
};

// CC-map accumulators (MODE 3): <v, d> per entry, FP32 partial sums of four
// readouts added with compensation (TwoSum: the sum and its rounding error,
// both FP32), and ||v||^2, a norm, whose partials are added into FP64 as the
// entry norms are.
struct Dots {
  float re[kQ], re_c[kQ], im[kQ], im_c[kQ];
  double vn2;
};

// One pass over all readouts for the thread's kQ entries. MODE 0 accumulates
// the norm only, MODE 1 stores FP32 planes, MODE 4 stores FP32 entry-major
// rows (two readouts per 16-byte store), MODE 2 stores BF16 blocks and
// also accumulates the norm of the stored (scaled, rounded) values into nb,
// MODE 5 stores both the FP32 planes and the BF16 blocks (and both norms),
// MODE 3 stores nothing and accumulates v conj(d) against the fingerprint
// `vox` (one value per readout, the same for every thread) into dt.
// SM: the entry is smoothed over the readouts (a five-sample delay line per
// entry, in the frame demodulated by the RF phase; output o = j - 2 leaves
// the line while raw sample j enters it, and two zero pushes after the last
// readout give the last two outputs).
template <int MODE, int PK, bool DF_LDS, bool SCALED, bool SM>
__device__ __forceinline__ void sim_pass(const SimArgs& a, const EntryState& st,
                                         const float* __restrict__ rftab, rsrc_t r1s, rsrc_t r2s,
                                         rsrc_t rds, float4* sdf, int64_t blk0, int32_t nrec,
                                         const float (&scale)[kQ], double (&n2)[kQ],
                                         double (&nb)[kQ], const float2* __restrict__ vox,
                                         Dots& dt) {
  constexpr int CH = chunk_of<MODE>();
  constexpr int kPrefetch = CH * kLdsMaxN3 / kThreads;  // float4 per thread per chunk
  const uint32_t tid = threadIdx.x;
  const int32_t n_tr = a.n_tr, n3 = a.n3;
  const int32_t per = CH * n3;  // staged float4 per chunk
  Spin m[kQ];
  float hx[kQ][kSmoothLen], hy[kQ][kSmoothLen];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    m[q] = initial_spin(a.inversion, st.r1ti[q]);
    n2[q] = 0.0;
    nb[q] = 0.0;
    dt.re[q] = dt.im[q] = dt.re_c[q] = dt.im_c[q] = 0.0f;
#pragma unroll
    for (int k = 0; k < kSmoothLen; ++k) hx[q][k] = hy[q][k] = 0.f;
  }
  dt.vn2 = 0.0;
  // FP32 partial sums over (up to) four outputs, added into FP64
  float part[kQ], partb[kQ], pre[kQ], pim[kQ], pv = 0.f;
  uint32_t w[kQ][4];  // one BF16 block of four outputs
  // MODE 4: 16 outputs of each entry, stored as one 128-byte burst of its row
  f32x4_t w16[kQ][kChunkRows / 2];
  bool live[kQ];      // MODE 4: the entry exists (tail lanes recompute the last one)
#pragma unroll
  for (int q = 0; q < kQ; ++q) live[q] = blk0 + tid + kThreads * q < a.count;
#pragma unroll
  for (int q = 0; q < kQ; ++q) part[q] = partb[q] = pre[q] = pim[q] = 0.f;
  auto flush = [&]() {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      n2[q] += (double)part[q];
      nb[q] += (double)partb[q];
      part[q] = partb[q] = 0.f;
      if (MODE == 3) {
        two_sum_acc(dt.re[q], dt.re_c[q], pre[q]);
        two_sum_acc(dt.im[q], dt.im_c[q], pim[q]);
        pre[q] = pim[q] = 0.f;
      }
    }
    if (MODE == 3) {
      dt.vn2 += (double)pv;
      pv = 0.f;
    }
  };
  // MODE 4: outputs [o0, o0 + count) of the staging buffer to the entry's row
  auto store_rows = [&](int q, int32_t o0, int32_t count) {
    float2* row = (float2*)a.re + (blk0 + tid + kThreads * q) * a.ld + o0;
#pragma unroll
    for (int p = 0; p < kChunkRows / 2; ++p) {
      if (!live[q]) break;
      if (2 * p + 1 < count) {
        *(f32x4_t*)(row + 2 * p) = w16[q][p];
      } else if (2 * p < count) {
        *(f32x2_t*)(row + 2 * p) = f32x2_t{w16[q][p].x, w16[q][p].y};
      }
    }
  };
  // output sample o of entry q (ol = o & (CH - 1), a compile-time constant in
  // the readout loop): norm, store or fingerprint product
  auto emit = [&](int q, int ol, int32_t o, float sx, float sy, float2 vo) {
    part[q] = fmaf(sx, sx, part[q]);
    part[q] = fmaf(sy, sy, part[q]);
    const float ox = SCALED ? sx * scale[q] : sx;
    const float oy = SCALED ? sy * scale[q] : sy;
    if (MODE == 4 && ol < 0) {
      // the two outputs after the last readout (smoothing): stored directly
      float2* row = (float2*)a.re + (blk0 + tid + kThreads * q) * a.ld;
      if (live[q]) *(f32x2_t*)(row + o) = f32x2_t{ox, oy};
    } else if (MODE == 4) {
      // staged at position ol (known at compile time); a full group of 16
      // goes out as one burst
#pragma unroll
      for (int p = 0; p < kChunkRows / 2; ++p) {
        if (p == (ol >> 1)) {
          if (ol & 1) {
            w16[q][p].z = ox;
            w16[q][p].w = oy;
          } else {
            w16[q][p].x = ox;
            w16[q][p].y = oy;
          }
        }
      }
      if (ol == kChunkRows - 1) store_rows(q, o - (kChunkRows - 1), kChunkRows);
    }
    if (MODE == 1 || MODE == 5) {
      // (nrec counts 4-byte records per plane row)
      const int32_t rec = MODE == 5 ? nrec / 4 : nrec;
      const rsrc_t wr = make_rsrc(a.re + (int64_t)o * a.ld + blk0, rec);
      const rsrc_t wi = make_rsrc(a.im + (int64_t)o * a.ld + blk0, rec);
      store1(ox, wr, 4u * (tid + kThreads * q));
      store1(oy, wi, 4u * (tid + kThreads * q));
    }
    if (MODE == 2 || MODE == 5) {
      const uint32_t v = pack_bf16x2(ox, oy);
      w[q][ol & 3] = v;
      // |stored value|^2: BF16 products are exact in FP32 (v_dot2_f32_bf16)
      const bf16x2_t b = __builtin_bit_cast(bf16x2_t, v);
      partb[q] = __builtin_amdgcn_fdot2_f32_bf16(b, b, partb[q], false);
      if ((ol & 3) == 3) {
        const rsrc_t wr = make_rsrc(a.packed + (int64_t)(o >> 2) * a.ld + blk0, nrec);
        store4(w[q], wr, 16u * (tid + kThreads * q));
      }
    }
    if (MODE == 3) {
      pre[q] = fmaf(vo.x, ox, fmaf(vo.y, oy, pre[q]));
      pim[q] = fmaf(vo.y, ox, fmaf(-vo.x, oy, pim[q]));
    }
  };
  float4 pf[kPrefetch];
  if (DF_LDS) {
#pragma unroll
    for (int p = 0; p < kPrefetch; ++p) pf[p] = load4(rds, 16u * (tid + kThreads * p), 0);
#pragma unroll
    for (int p = 0; p < kPrefetch; ++p)
      if ((int32_t)(tid + kThreads * p) < per) sdf[tid + kThreads * p] = pf[p];
    lds_barrier();
  }
  const int32_t nch = (n_tr + CH - 1) / CH;
  for (int32_t c = 0; c < nch; ++c) {
    const int32_t j0 = c * CH;
    const float4* sd = sdf + (c & 1) * per;
    if (DF_LDS && c + 1 < nch) {
      // rows j0+8.. of the step-major table are contiguous. The whole offset
      // goes in the vector operand, which the buffer range check covers:
      // reads past the table end return zero and are never used.
      const uint32_t row = (uint32_t)(j0 + CH) * (uint32_t)n3 * 16u;
#pragma unroll
      for (int p = 0; p < kPrefetch; ++p)
        pf[p] = load4(rds, row + 16u * (tid + kThreads * p), 0);
    }
#pragma unroll
    for (int jj = 0; jj < CH; ++jj) {
      const int32_t j = j0 + jj;
      if (j < n_tr) {
        // the output of this readout (j0 is a multiple of CH, so o & (CH - 1)
        // is known at compile time)
        const int32_t o = SM ? j - kSmoothLag : j;
        const int ol = SM ? ((jj - kSmoothLag) & (CH - 1)) : (jj & (CH - 1));
        const bool out = !SM || o >= 0;
        float sc = 1.f;
        float2 dmj = make_float2(1.f, 0.f), dmo = make_float2(1.f, 0.f);
        if (SM) {
          sc = o >= 2 ? a.sm.full : (o == 1 ? a.sm.head[1] : a.sm.head[0]);
          dmj = a.demod[j];
          dmo = a.demod[o >= 0 ? o : 0];
        }
        float2 vo = make_float2(0.f, 0.f);
        if (MODE == 3 && out) {
          vo = vox[o];
          pv = fmaf(vo.x, vo.x, fmaf(vo.y, vo.y, pv));
        }
#pragma unroll
        for (int q = 0; q < kQ; ++q) {
          const float2 r1 = load2(r1s, st.o1[q], (uint32_t)j * a.n1 * 8u);
          const float2 r2 = load2(r2s, st.o2[q], (uint32_t)j * a.n2 * 8u);
          const float4 pc = DF_LDS ? sd[jj * n3 + st.i3[q]]
                                   : load4(rds, 16u * st.i3[q], (uint32_t)j * n3 * 16u);
          if (PK == kGeneralUniform || PK == kXAxisUniform)
            pulse<PK>(m[q], rftab + 9 * j);
          else
            pulse<PK>(m[q], st.rq[q] + 9 * j);
          free_evolve(m[q], pc.x, pc.y, r2.x, r1.x);
          float sx = m[q].x, sy = m[q].y;
          if (SM) {
            smooth_demod(dmj, sx, sy);
            smooth_push(hx[q], hy[q], sx, sy);
            smooth_out(a.sm, hx[q], hy[q], sc, sx, sy);
            smooth_remod(dmo, sx, sy);
          }
          if (out) emit(q, ol, o, sx, sy, vo);
          free_evolve(m[q], pc.z, pc.w, r2.y, r1.y);
        }
      }
      if ((jj & 3) == 3) flush();
    }
    if (DF_LDS) {
      if (c + 1 < nch) {
        float4* nx = sdf + ((c + 1) & 1) * per;
#pragma unroll
        for (int p = 0; p < kPrefetch; ++p)
          if ((int32_t)(tid + kThreads * p) < per) nx[tid + kThreads * p] = pf[p];
      }
      lds_barrier();
    }
  }
  if (SM) {
    // the last two outputs (BF16 entries have n_tr % 4 == 0: they fill
    // positions 2 and 3 of the last block; MODE 4 stores them directly)
#pragma unroll
    for (int t = 0; t < kSmoothLag; ++t) {
      const int32_t o = n_tr - kSmoothLag + t;
      float2 vo = make_float2(0.f, 0.f);
      if (MODE == 3 && o >= 0) {
        vo = vox[o];
        pv = fmaf(vo.x, vo.x, fmaf(vo.y, vo.y, pv));
      }
      const float2 dmo = a.demod[o >= 0 ? o : 0];
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        float sx, sy;
        smooth_push(hx[q], hy[q], 0.f, 0.f);
        smooth_out(a.sm, hx[q], hy[q], a.sm.tail[t], sx, sy);
        smooth_remod(dmo, sx, sy);
        if (o >= 0) emit(q, MODE == 4 ? -1 : 2 + t, o, sx, sy, vo);
      }
    }
    flush();
  }
  if (MODE == 4) {
    // the staged outputs after the last full group of 16 (with smoothing the
    // readout loop stages outputs up to n_tr - 3)
    const int32_t end = SM ? max(n_tr - kSmoothLag, 0) : n_tr;
    const int32_t r = end & (kChunkRows - 1);
    if (r) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) store_rows(q, end - r, r);
    }
  }
}

template <int MODE, int PK, bool DF_LDS, bool SM>
__global__ __launch_bounds__(kThreads) void k_sim_dict(SimArgs a, const float2* __restrict__ t1tab,
                                                       const float2* __restrict__ t2tab,
                                                       const float4* __restrict__ dftab,
                                                       const float* __restrict__ rftab,
                                                       const float* __restrict__ t1ti,
                                                       const float2* __restrict__ vox) {
  extern __shared__ float4 sdf[];
  const uint32_t tid = threadIdx.x;
  const int64_t blk0 = (int64_t)blockIdx.x * kBlockEntries;
  const int64_t rem = a.count - blk0;
  const int32_t nb_entries = (int32_t)(rem < kBlockEntries ? rem : kBlockEntries);
  // buffer range in bytes of one store row: 16 per entry for BF16 blocks
  // (MODE 5: FP32 plane rows use a quarter of it), 4 for FP32 planes
  const int32_t nrec = nb_entries * ((MODE == 2 || MODE == 5) ? 16 : 4);
  EntryState st;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    int64_t e = blk0 + tid + kThreads * q;
    if (e >= a.count) e = a.count - 1;  // tail lanes recompute the last entry, never store it
    int32_t i1, i2, i3, i4;
    unravel(a.k0 + e, a.n2, a.n3, a.n4, i1, i2, i3, i4);
    st.o1[q] = 8u * (uint32_t)i1;
    st.o2[q] = 8u * (uint32_t)i2;
    st.i3[q] = (uint32_t)i3;
    st.rq[q] = rftab + (int64_t)i4 * a.n_tr * 9;
    st.r1ti[q] = t1ti[i1];
  }
  const rsrc_t r1s = make_rsrc(t1tab, a.t1_bytes);
  const rsrc_t r2s = make_rsrc(t2tab, a.t2_bytes);
  const rsrc_t rds = make_rsrc(dftab, a.df_bytes);
  float scale[kQ];
  double n2[kQ], nb[kQ];
  Dots dt;
  if (MODE != 3 && a.unit_norm) {
    // two passes: the norm first, then the entries divided by it
#pragma unroll
    for (int q = 0; q < kQ; ++q) scale[q] = 1.0f;
    sim_pass<0, PK, DF_LDS, false, SM>(a, st, rftab, r1s, r2s, rds, sdf, blk0, nrec, scale, n2, nb,
                                   vox, dt);
#pragma unroll
    for (int q = 0; q < kQ; ++q) scale[q] = n2[q] > 0.0 ? (float)(1.0 / sqrt(n2[q])) : 0.0f;
    double n2b[kQ];
    sim_pass<MODE, PK, DF_LDS, true, SM>(a, st, rftab, r1s, r2s, rds, sdf, blk0, nrec, scale, n2b, nb,
                                     vox, dt);
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) scale[q] = 1.0f;
    sim_pass<MODE, PK, DF_LDS, false, SM>(a, st, rftab, r1s, r2s, rds, sdf, blk0, nrec, scale, n2, nb,
                                      vox, dt);
  }
  if (MODE == 3) {
    // CC = |<v, d>| / (||v|| ||d||) (Eq. 1), 0 when either norm is 0
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int64_t e = blk0 + tid + kThreads * q;
      // |<v, d>|^2 in FP32 from the compensated sums; the norms in FP64
      const float re = dt.re[q] + dt.re_c[q], im = dt.im[q] + dt.im_c[q];
      const float num = fmaf(re, re, im * im);
      const double den = n2[q] * dt.vn2;
      if (e < a.count) a.cc[e] = den > 0.0 ? (float)sqrt((double)num / den) : 0.0f;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int64_t e = blk0 + tid + kThreads * q;
      // BF16: the norm of the values actually stored
      if (e < a.count && a.norm) a.norm[e] = sqrt(MODE == 2 ? nb[q] : n2[q]);
      if (MODE == 5 && e < a.count && a.norm_b) a.norm_b[e] = sqrt(nb[q]);
    }
  }
}

template <int MODE, int PK, bool SM>
static void launch_sim_smooth(const SimArgs& a, const Tables& t, bool df_lds, int64_t blocks,
                              hipStream_t stream, const float2* vox) {
  const dim3 g((unsigned)blocks), b(kThreads);
  const size_t lds = df_lds ? 2 * sizeof(float4) * chunk_of<MODE>() * (size_t)a.n3 : 0;
  if (df_lds)
    hipLaunchKernelGGL((k_sim_dict<MODE, PK, true, SM>), g, b, lds, stream, a, t.t1, t.t2, t.df,
                       t.rf, t.t1ti, vox);
  else
    hipLaunchKernelGGL((k_sim_dict<MODE, PK, false, SM>), g, b, 0, stream, a, t.t1, t.t2, t.df,
                       t.rf, t.t1ti, vox);
}

template <int MODE, int PK>
static void launch_sim_variant(const SimArgs& a, const Tables& t, bool df_lds, int64_t blocks,
                               hipStream_t stream, const float2* vox) {
  if (t.smooth)
    launch_sim_smooth<MODE, PK, true>(a, t, df_lds, blocks, stream, vox);
  else
    launch_sim_smooth<MODE, PK, false>(a, t, df_lds, blocks, stream, vox);
}

template <int MODE>
static void launch_sim_mode(SimArgs a, const Tables& t, int64_t blocks, hipStream_t stream,
                            const float2* vox = nullptr) {
  const bool df_lds = a.n3 <= kLdsMaxN3;
  if (t.smooth) {
    a.sm = smooth_weights(t.smooth, a.n_tr);
    a.demod = t.demod;
  }
  const bool lane = a.n4 > 1;
  if (!lane && t.x_axis_pulses)
    launch_sim_variant<MODE, kXAxisUniform>(a, t, df_lds, blocks, stream, vox);
  else if (!lane)
    launch_sim_variant<MODE, kGeneralUniform>(a, t, df_lds, blocks, stream, vox);
  else if (t.x_axis_pulses)
    launch_sim_variant<MODE, kXAxisLane>(a, t, df_lds, blocks, stream, vox);
  else
    launch_sim_variant<MODE, kGeneralLane>(a, t, df_lds, blocks, stream, vox);
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

// Temporal smoothing of complex64 signals (fingerprints, Experiment 4): one
// wave per signal walks its readouts 64 at a time, holding the previous,
// current and next 64 raw values in registers and taking the window from
// neighbouring lanes; every load of a chunk precedes the stores that
// overwrite it, so in == out (same row stride) is safe. Same weights, order
// of operations and end scales as the dictionary's delay line.
struct SmoothArgs {
  const float2* in;
  float2* out;
  int64_t ld_in, ld_out, n_sig;
  int32_t n_tr;
  SmoothW sm;
  const float2* demod;  // [n_tr] (cos, sin) of the RF phases, or NULL (zero phases)
};

__global__ __launch_bounds__(256) void k_smooth_signals(SmoothArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.n_sig) return;  // the whole wave (row is uniform over it)
  const float2* x = a.in + row * a.ld_in;
  float2* y = a.out + row * a.ld_out;
  const int32_t n = a.n_tr;
  // raw sample j demodulated by its RF phase
  auto load = [&](int32_t j) {
    float2 v = make_float2(0.f, 0.f);
    if (j < n) {
      v = x[j];
      if (a.demod) smooth_demod(a.demod[j], v.x, v.y);
    }
    return v;
  };
  float2 prev = make_float2(0.f, 0.f);
  float2 cur = load(lane);
  for (int32_t j0 = 0; j0 < n; j0 += 64) {
    const int32_t jn = j0 + 64 + lane;
    const float2 nxt = load(jn);
    float hx[kSmoothLen], hy[kSmoothLen];
#pragma unroll
    for (int k = 0; k < kSmoothLen; ++k) {
      const int l = lane + k - kSmoothLag;  // lane of raw sample j + k - 2 in its chunk
      const int src = l & 63;
      const float px = __shfl(prev.x, src), py = __shfl(prev.y, src);
      const float cx = __shfl(cur.x, src), cy = __shfl(cur.y, src);
      const float nx = __shfl(nxt.x, src), ny = __shfl(nxt.y, src);
      hx[k] = l < 0 ? px : (l >= 64 ? nx : cx);
      hy[k] = l < 0 ? py : (l >= 64 ? ny : cy);
    }
    const int32_t j = j0 + lane;
    const float sc = j == n - 1   ? a.sm.tail[1]
                     : j == n - 2 ? a.sm.tail[0]
                     : j == 0     ? a.sm.head[0]
                     : j == 1     ? a.sm.head[1]
                                  : a.sm.full;
    float ox, oy;
    smooth_out(a.sm, hx, hy, sc, ox, oy);
    if (j < n) {
      if (a.demod) smooth_remod(a.demod[j], ox, oy);
      y[j] = make_float2(ox, oy);
    }
    prev = cur;
    cur = nxt;
  }
}

// Launch arguments shared by the dictionary and CC-map launches.
static int sim_args(const Tables& t, int64_t k0, int64_t count, SimArgs* out, int64_t* blocks) {
  // the step tables are addressed through 32-bit buffer ranges
  const int64_t nt = t.n_tr;
  const int64_t b1 = 8 * nt * t.n1, b2 = 8 * nt * t.n2, b3 = 16 * nt * t.n3;
  if (b1 > INT32_MAX || b2 > INT32_MAX || b3 > INT32_MAX) {
    set_error("grid axis too long: a step table of n_tr x axis length exceeds 2 GiB");
    return MRF_ERR_INVALID;
  }
  SimArgs a{};
  a.n_tr = t.n_tr;
  a.n1 = t.n1;
  a.n2 = t.n2;
  a.n3 = t.n3;
  a.n4 = t.n4;
  a.inversion = t.inversion;
  a.t1_bytes = (int32_t)b1;
  a.t2_bytes = (int32_t)b2;
  a.df_bytes = (int32_t)b3;
  a.k0 = k0;
  a.count = count;
  *blocks = (count + kBlockEntries - 1) / kBlockEntries;
  if (*blocks > INT32_MAX) {
    set_error("too many entries in one call");
    return MRF_ERR_INVALID;
  }
  *out = a;
  return MRF_OK;
}

int launch_sim_dict(mrf_context* ctx, const Tables& t, int64_t k0, int64_t count,
                    mrf_dtype dtype, void* re, void* im, int64_t ld, double* norm, int unit_norm,
                    hipStream_t stream) {
  if (count == 0) return MRF_OK;
  SimArgs a;
  int64_t blocks = 0;
  int rc = sim_args(t, k0, count, &a, &blocks);
  if (rc) return rc;
  a.unit_norm = unit_norm;
  a.ld = ld;
  a.re = (float*)re;
  a.im = (float*)im;
  a.packed = (uint4*)re;
  a.norm = norm;
  ProfScope prof(ctx, "k_sim_dict", stream);
  if (dtype == MRF_F32)
    launch_sim_mode<1>(a, t, blocks, stream);
  else if (dtype == MRF_F32_ROWS)
    launch_sim_mode<4>(a, t, blocks, stream);
  else
    launch_sim_mode<2>(a, t, blocks, stream);
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}

// The FP32 planar and raw BF16 dictionaries of one entry range from one
// recursion pass (MODE 5).
static int launch_sim_pair(mrf_context* ctx, const Tables& t, int64_t k0, int64_t count,
                           float* re, float* im, void* packed, int64_t ld, double* norm,
                           double* norm_b, hipStream_t stream) {
  if (count == 0) return MRF_OK;
  SimArgs a;
  int64_t blocks = 0;
  int rc = sim_args(t, k0, count, &a, &blocks);
  if (rc) return rc;
  a.unit_norm = 0;
  a.ld = ld;
  a.re = re;
  a.im = im;
  a.packed = (uint4*)packed;
  a.norm = norm;
  a.norm_b = norm_b;
  ProfScope prof(ctx, "k_sim_dict", stream);
  launch_sim_mode<5>(a, t, blocks, stream);
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}

// CC map of one fingerprint (Experiment 1): the dictionary recursion of every
// entry, with the CC of Eq. 1 accumulated on the fly; nothing else is stored.
static int launch_cc_map(mrf_context* ctx, const Tables& t, int64_t k0, int64_t count,
                         const float2* vox, float* cc, hipStream_t stream) {
  if (count == 0) return MRF_OK;
  SimArgs a;
  int64_t blocks = 0;
  int rc = sim_args(t, k0, count, &a, &blocks);
  if (rc) return rc;
  a.cc = cc;
  ProfScope prof(ctx, "k_cc_map", stream);
  launch_sim_mode<3>(a, t, blocks, stream, vox);
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
  MRF_CHECK_ARG(dtype == MRF_F32 || dtype == MRF_BF16 || dtype == MRF_F32_ROWS,
                "unknown dtype %d", (int)dtype);
  const int64_t E = grid_size_checked(grid);
  MRF_CHECK_ARG(entry_begin >= 0 && entry_count >= 0 && entry_begin + entry_count <= E,
                "entry range [%lld, %lld) outside the grid of %lld entries",
                (long long)entry_begin, (long long)(entry_begin + entry_count), (long long)E);
  if (dtype == MRF_F32_ROWS) {
    MRF_CHECK_ARG(ld >= n_tr && ld % 2 == 0, "entry-major rows need an even ld >= n_tr (got %lld)",
                  (long long)ld);
    MRF_CHECK_ARG(entry_count == 0 || re, "re must not be NULL");
    MRF_CHECK_ARG(im == nullptr, "im must be NULL for entry-major rows");
    MRF_CHECK_ARG(((uintptr_t)re & 15) == 0, "entry-major rows must be 16-byte aligned");
  } else {
    MRF_CHECK_ARG(ld >= entry_count, "ld (%lld) must be >= entry_count (%lld)", (long long)ld,
                  (long long)entry_count);
  }
  if (dtype == MRF_F32) {
    MRF_CHECK_ARG(entry_count == 0 || (re && im), "re and im must not be NULL");
  } else if (dtype == MRF_BF16) {
    MRF_CHECK_ARG(entry_count == 0 || re, "re must not be NULL");
    MRF_CHECK_ARG(im == nullptr, "im must be NULL for the packed BF16 layout");
    MRF_CHECK_ARG(n_tr % 4 == 0, "BF16 dictionaries need n_tr %% 4 == 0 (got %d)", n_tr);
    MRF_CHECK_ARG(((uintptr_t)re & 15) == 0, "BF16 dictionary must be 16-byte aligned");
  }
  TablesRef tref;  // held until the launches are enqueued
  rc = get_tables(const_cast<mrf_sequence*>(seq), grid, n_tr, (hipStream_t)stream, &tref);
  const Tables* t = tref.get();
  if (rc) return rc;
  return launch_sim_dict(ctx, *t, entry_begin, entry_count, dtype, re, im, ld, norm, unit_norm ? 1 : 0,
                         (hipStream_t)stream);
}

extern "C" int mrf_simulate_dictionary_pair(mrf_context* ctx, const mrf_sequence* seq,
                                            const mrf_grid* grid, int32_t n_tr,
                                            int64_t entry_begin, int64_t entry_count, float* re,
                                            float* im, void* packed, int64_t ld, double* norm,
                                            double* norm_bf16, void* stream) {
  MRF_CHECK_ARG(ctx && seq, "context and sequence must not be NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  MRF_CHECK_ARG(n_tr >= 1 && n_tr <= seq->n, "n_tr %d must be in [1, %d]", n_tr, seq->n);
  MRF_CHECK_ARG(n_tr % 4 == 0, "BF16 dictionaries need n_tr %% 4 == 0 (got %d)", n_tr);
  const int64_t E = grid_size_checked(grid);
  MRF_CHECK_ARG(entry_begin >= 0 && entry_count >= 0 && entry_begin + entry_count <= E,
                "entry range [%lld, %lld) outside the grid of %lld entries",
                (long long)entry_begin, (long long)(entry_begin + entry_count), (long long)E);
  MRF_CHECK_ARG(ld >= entry_count, "ld (%lld) must be >= entry_count (%lld)", (long long)ld,
                (long long)entry_count);
  MRF_CHECK_ARG(entry_count == 0 || (re && im && packed), "re, im and packed must not be NULL");
  MRF_CHECK_ARG(((uintptr_t)packed & 15) == 0, "BF16 dictionary must be 16-byte aligned");
  TablesRef tref;  // held until the launch is enqueued
  rc = get_tables(const_cast<mrf_sequence*>(seq), grid, n_tr, (hipStream_t)stream, &tref);
  const Tables* t = tref.get();
  if (rc) return rc;
  return launch_sim_pair(ctx, *t, entry_begin, entry_count, re, im, packed, ld, norm, norm_bf16,
                         (hipStream_t)stream);
}

extern "C" int mrf_cc_map(mrf_context* ctx, const mrf_sequence* seq, const mrf_grid* grid,
                          int32_t n_tr, const void* vox, int32_t n_vox, int64_t ld_vox,
                          int64_t entry_begin, int64_t entry_count, float* cc, int64_t ld_cc,
                          void* stream) {
  MRF_CHECK_ARG(ctx && seq, "context and sequence must not be NULL");
  int rc = check_grid(grid);
  if (rc) return rc;
  MRF_CHECK_ARG(n_tr >= 1 && n_tr <= seq->n, "n_tr %d must be in [1, %d]", n_tr, seq->n);
  MRF_CHECK_ARG(n_vox >= 0, "n_vox must be >= 0");
  MRF_CHECK_ARG(ld_vox >= n_tr, "ld_vox (%lld) must be >= n_tr (%d)", (long long)ld_vox, n_tr);
  const int64_t E = grid_size_checked(grid);
  MRF_CHECK_ARG(entry_begin >= 0 && entry_count >= 0 && entry_begin + entry_count <= E,
                "entry range [%lld, %lld) outside the grid of %lld entries",
                (long long)entry_begin, (long long)(entry_begin + entry_count), (long long)E);
  MRF_CHECK_ARG(ld_cc >= entry_count, "ld_cc (%lld) must be >= entry_count (%lld)",
                (long long)ld_cc, (long long)entry_count);
  if (n_vox == 0 || entry_count == 0) return MRF_OK;
  MRF_CHECK_ARG(vox && cc, "vox and cc must not be NULL");
  MRF_CHECK_ARG(((uintptr_t)vox & 7) == 0, "vox must be 8-byte aligned (complex64)");
  TablesRef tref;  // held until the launches are enqueued
  rc = get_tables(const_cast<mrf_sequence*>(seq), grid, n_tr, (hipStream_t)stream, &tref);
  const Tables* t = tref.get();
  if (rc) return rc;
  for (int32_t v = 0; v < n_vox; ++v) {
    rc = launch_cc_map(ctx, *t, entry_begin, entry_count, (const float2*)vox + (int64_t)v * ld_vox,
                       cc + (int64_t)v * ld_cc, (hipStream_t)stream);
    if (rc) return rc;
  }
  return MRF_OK;
}

extern "C" int mrf_smooth_signals(mrf_context* ctx, const mrf_sequence* seq, const void* in,
                                  int64_t ld_in, void* out, int64_t ld_out, int64_t n_sig,
                                  int32_t n_tr, int32_t taps, void* stream) {
  MRF_CHECK_ARG(ctx, "context must not be NULL");
  MRF_CHECK_ARG(!seq || n_tr <= seq->n, "n_tr (%d) exceeds the sequence length (%d)", n_tr,
                seq ? seq->n : 0);
  MRF_CHECK_ARG(taps == 0 || taps == 1 || taps == 3 || taps == 5,
                "taps must be 0, 1, 3 or 5 (got %d)", taps);
  MRF_CHECK_ARG(n_sig >= 0 && n_tr >= 0, "n_sig and n_tr must be >= 0");
  MRF_CHECK_ARG(ld_in >= n_tr && ld_out >= n_tr, "row strides must be >= n_tr");
  if (n_sig == 0 || n_tr == 0) return MRF_OK;
  MRF_CHECK_ARG(in && out, "in and out must not be NULL");
  MRF_CHECK_ARG(((uintptr_t)in & 7) == 0 && ((uintptr_t)out & 7) == 0,
                "signals must be 8-byte aligned (complex64)");
  const uintptr_t ib = (uintptr_t)in, ob = (uintptr_t)out;
  const uintptr_t ie = ib + 8 * (uintptr_t)((n_sig - 1) * ld_in + n_tr);
  const uintptr_t oe = ob + 8 * (uintptr_t)((n_sig - 1) * ld_out + n_tr);
  MRF_CHECK_ARG((ib == ob && ld_in == ld_out) || ie <= ob || oe <= ib,
                "in and out must be the same rows or not overlap");
  hipStream_t s = (hipStream_t)stream;
  if (taps <= 1) {
    if (ib != ob)
      MRF_HIP(hipMemcpy2DAsync(out, 8 * (size_t)ld_out, in, 8 * (size_t)ld_in, 8 * (size_t)n_tr,
                               (size_t)n_sig, hipMemcpyDeviceToDevice, s));
    return MRF_OK;
  }
  const int64_t blocks = (n_sig + 3) / 4;
  MRF_CHECK_ARG(blocks <= INT32_MAX, "too many signals in one call");
  SmoothArgs a;
  a.in = (const float2*)in;
  a.out = (float2*)out;
  a.ld_in = ld_in;
  a.ld_out = ld_out;
  a.n_sig = n_sig;
  a.n_tr = n_tr;
  a.sm = smooth_weights(taps, n_tr);
  a.demod = seq ? seq->demod : nullptr;
  ProfScope prof(ctx, "k_smooth_signals", s);
  hipLaunchKernelGGL(k_smooth_signals, dim3((unsigned)blocks), dim3(256), 0, s, a);
  MRF_HIP(hipGetLastError());
  return MRF_OK;
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
