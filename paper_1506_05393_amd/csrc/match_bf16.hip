// BF16 brute-force matching with FP32 re-scoring of the top candidates.
//
// Same complex-as-real GEMM as the FP32 path (Theory Eq. 1), on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation. The BF16 dictionary is
// stored in blocks of 4 readouts, [j/4][entry][Re d_j, Im d_j x 4], which is
// exactly one lane's 8-element operand of the instruction; the voxel operand
// is packed the same way: row 2v holds (Re v, Im v) pairs, row 2v+1 holds
// (Im v, -Re v), so C[2v][k] = Re s_vk and C[2v+1][k] = Im s_vk.
// The top-k of every voxel (k <= 8) is then re-simulated in FP32 with the
// dictionary kernel's step function and re-scored exactly (K5).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "bloch.h"
#include "internal.h"
#include "match_common.h"
#include "match_kernels.h"
#include "compensated.h"
#include "smooth.h"

namespace mrf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Workgroup tile 256 x 256: 8 waves in 2 x 4, each 128 x 64 = 4 x 2 blocks
// of 32 x 32 (128 accumulators, so two waves share each SIMD and one issues
// MFMAs while the other waits; measured 5% faster than 4 waves of 128 x 128
// at one wave per SIMD). One instruction covers K = 16 = 2 blocks of 4
// readouts (lanes 0-31: block 2s, lanes 32-63: block 2s + 1).
constexpr int BBM = 256;
constexpr int BBN = 256;
constexpr int BKB = 4;        // 4-readout blocks per pipeline stage (16 readouts, K = 32)
constexpr int NSTAGE = 4;     // LDS ring of stages; loads run NSTAGE-1 stages ahead (3: 1.6% slower)
constexpr int BKK_MAX = 8;    // candidate list length in the epilogue
constexpr int NW = 8;         // waves per workgroup: 2 (rows) x 4 (columns)
constexpr int WCN = 4;        // column waves
constexpr int TNB = 2;        // 32-column blocks per wave (64 columns)
constexpr int LPS = 4;        // global->LDS loads per wave per stage

struct MatchB16Args {
  const uint4* A;       // [nblk_pad][m_pad] 16-byte blocks
  const uint4* B;       // [nblk][ld]
  const double* norm;   // [n_entries] or NULL
  int32_t nblk, nblk_pad, m_pad, n_vox_pad;
  int64_t ld, n_entries;
  int32_t n_row_tiles, n_chunks, n_col_tiles, kk;
  int32_t grp_rows, grp_chunks;  // workgroups resident on one XCD: grp_rows x grp_chunks
  float* part_s;        // [n_chunks][2][n_vox_pad][kk]
  int32_t* part_i;
  uint32_t* sync;       // [n_groups][8] tile arrival counters (zeroed by k_pack_bf16)
};

typedef __attribute__((address_space(3))) void* lds_ptr;
typedef const __attribute__((address_space(1))) void* glb_ptr;

// One wavefront moves 64 x 16 B from global memory straight into LDS: lane l
// reads `src` (its own address) and the data lands at dst + 16 l.
__device__ __forceinline__ void load_to_lds(const uint4* src, uint4* dst) {
  __builtin_amdgcn_global_load_lds((glb_ptr)src, (lds_ptr)dst, 16, 0, 0);
}

// Issue the loads of one stage (BKB blocks of A rows and B columns): wave w
// moves 64-row (64-column) chunk w & 3 of blocks (w >> 2) and (w >> 2) + 2.
__device__ __forceinline__ void issue_stage(const MatchB16Args& a, uint4* As, uint4* Bs, int st,
                                            int c, int row0, int64_t col0, int wave, int lane) {
  const int ch = wave & 3;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int i = (wave >> 2) + 2 * h;
    const int blk = c * BKB + i;
    load_to_lds(a.A + (int64_t)blk * a.m_pad + row0 + ch * 64 + lane,
                As + (st * BKB + i) * BBM + ch * 64);
    const int bb = blk < a.nblk ? blk : a.nblk - 1;
    int64_t col = col0 + ch * 64 + lane;
    col = col < a.ld ? col : a.ld - 1;
    load_to_lds(a.B + (int64_t)bb * a.ld + col, Bs + (st * BKB + i) * BBN + ch * 64);
  }
}

// Visiting order of a workgroup's nt column tiles: every TS-th tile first
// (raising the top-k thresholds early, so the rest inserts few candidates),
// then the others in order. Returns the tile offset of the k-th visit.
constexpr int TS = 16;
constexpr int kMaxLate = 32;  // consecutive timed-out alignment waits before a workgroup stops aligning
__device__ __forceinline__ int tile_at(int k, int nt) {
  const int n1 = (nt + TS - 1) / TS;
  if (k < n1) return k * TS;
  const int m = k - n1;
  return m + m / (TS - 1) + 1;
}

// The entry norms of this lane's 4 tile columns (1 when the dictionary has
// unit-norm entries; columns past the last entry read entry 0, masked later).
__device__ __forceinline__ void load_norms(const MatchB16Args& a, int64_t col0, int wc, int lane,
                                           double (&nrm)[TNB]) {
#pragma unroll
  for (int bn = 0; bn < TNB; ++bn) {
    const int64_t e = col0 + wc * 64 + bn * 32 + (lane & 31);
    nrm[bn] = a.norm ? a.norm[e < a.n_entries ? e : 0] : 1.0;
  }
}

// The A and B fragments of MFMA group s (0 or 1) of ring slot st for this lane.
__device__ __forceinline__ void read_frags(const uint4* As, const uint4* Bs, int st, int s, int wr,
                                           int wc, int lane, bf16x8 (&fa)[4], bf16x8 (&fb)[TNB]) {
  const bf16x8* as =
      (const bf16x8*)(As + (st * BKB + 2 * s + (lane >> 5)) * BBM + wr * 128 + (lane & 31));
  const bf16x8* bs =
      (const bf16x8*)(Bs + (st * BKB + 2 * s + (lane >> 5)) * BBN + wc * 64 + (lane & 31));
#pragma unroll
  for (int i = 0; i < 4; ++i) fa[i] = as[32 * i];
#pragma unroll
  for (int j = 0; j < TNB; ++j) fb[j] = bs[32 * j];
}

__device__ __forceinline__ void mfma_group(floatx16 (&acc)[4][TNB], const bf16x8 (&fa)[4],
                                           const bf16x8 (&fb)[TNB]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TNB; ++j)
      acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
}

__global__ __launch_bounds__(512) void k_match_bf16(MatchB16Args a) {
  // Workgroups are dealt to the 8 XCDs in turn (w & 7), and each XCD starts
  // its slots in order, one workgroup per CU. The slots that run together on
  // an XCD form a grp_rows x grp_chunks block: every voxel tile is then read
  // into that XCD's L2 once for grp_chunks workgroups, and every dictionary
  // tile once for grp_rows (rather than all row tiles against one chunk,
  // which re-reads the whole voxel operand for every dictionary tile).
  const int w = blockIdx.x;
  const int xcd = w & 7;
  const int slot = w >> 3;
  const int per = a.grp_rows * a.grp_chunks;
  const int within = slot % per;
  const int rt = (slot / per) * a.grp_rows + within % a.grp_rows;
  const int chunk = xcd + 8 * (within / a.grp_rows);
  if (rt >= a.n_row_tiles || chunk >= a.n_chunks) return;
  // Tile-phase alignment of the workgroups resident together on this XCD:
  // each one counts its finished tiles into ctr and, before its next tile,
  // waits (bounded) until every peer has finished as many. In step, the 8
  // readers of a dictionary tile and the 4 readers of a voxel tile fetch each
  // stage within a few microseconds of each other and the later ones hit in
  // L2 (L2 hit rate 0.80 against 0.26 unaligned). Timing only: results do
  // not depend on it.
  const int grp = slot / per;
  uint32_t* ctr = a.sync + grp * 8 + xcd;
  const int rows_valid = min(a.grp_rows, a.n_row_tiles - grp * a.grp_rows);
  int n_late = 0;  // consecutive timed-out waits (lane 0 of wave 0 only)

  extern __shared__ __align__(16) unsigned char smem[];
  uint4* As = (uint4*)smem;                  // [NSTAGE][BKB][BBM]
  uint4* Bs = As + NSTAGE * BKB * BBM;       // [NSTAGE][BKB][BBN]
  float* Ls = (float*)(Bs + NSTAGE * BKB * BBN);  // [NW waves][64 voxels][BKK_MAX]
  int32_t* Li = (int32_t*)(Ls + NW * 64 * BKK_MAX);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int kk = a.kk;
  const int row0 = rt * BBM;
  float* myLs = Ls + wave * 64 * BKK_MAX;
  int32_t* myLi = Li + wave * 64 * BKK_MAX;
  for (int i = lane; i < 64 * BKK_MAX; i += 64) {
    myLs[i] = -1.0f;
    myLi[i] = 0x7fffffff;
  }

  const int ct_begin = (int)((int64_t)chunk * a.n_col_tiles / a.n_chunks);
  const int ct_end = (int)((int64_t)(chunk + 1) * a.n_col_tiles / a.n_chunks);
  const int n_kc = a.nblk_pad / BKB;

  // Tile pipeline: the entry norms and the first NSTAGE stages of a tile are
  // requested before the previous tile's epilogue runs, so their latency is
  // hidden behind it. Loads complete in issue order, so the norm loads (issued
  // first) have landed whenever a stage wait below is satisfied.
  double nrm[TNB];
  if (ct_begin < ct_end) {
    load_norms(a, (int64_t)ct_begin * BBN, wc, lane, nrm);
    for (int p = 0; p < NSTAGE; ++p)
      if (p < n_kc) issue_stage(a, As, Bs, p, p, row0, (int64_t)ct_begin * BBN, wave, lane);
  }
  const int n_ct = ct_end - ct_begin;
  for (int ct = ct_begin; ct < ct_end; ++ct) {
    const int64_t col0 = (int64_t)(ct_begin + tile_at(ct - ct_begin, n_ct)) * BBN;
    floatx16 acc[4][TNB];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < TNB; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

    // stage 0 landed for this wave (stages 1-3 may still be in flight), then
    // for everyone (wait and barrier in one asm statement: no LDS read can be
    // moved above it)
    static_assert(NSTAGE == 4 && LPS == 4, "the waits below count LPS loads per stage");
    if (n_kc >= 4)
      asm volatile("s_waitcnt vmcnt(12)\n\ts_barrier" ::: "memory");
    else if (n_kc == 3)
      asm volatile("s_waitcnt vmcnt(8)\n\ts_barrier" ::: "memory");
    else if (n_kc == 2)
      asm volatile("s_waitcnt vmcnt(4)\n\ts_barrier" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");

    // Each stage is two MFMA groups (K = 16 each). The fragments of the next
    // group are read from LDS while the current group's 16 MFMAs run. Between
    // the groups every wave has finished reading the stage's ring slot and
    // stage c + 1 has landed (one barrier); after the second group the slot
    // is refilled with stage c + NSTAGE. In the last stage the next-group
    // reads fetch a slot that is never used.
    bf16x8 fa0[4], fb0[TNB], fa1[4], fb1[TNB];
    read_frags(As, Bs, 0, 0, wr, wc, lane, fa0, fb0);
    for (int c = 0; c < n_kc; ++c) {
      const int st = c % NSTAGE;
      read_frags(As, Bs, st, 1, wr, wc, lane, fa1, fb1);
      mfma_group(acc, fa0, fb0);
#pragma unroll
      for (int g = 0; g < 4 + TNB; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // 1 MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // 1 LDS read
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 4 * TNB - 4 - TNB, 0);
      // this wave's reads of slot st are done and stage c + 1 landed, then
      // everyone's
      const int ahead = min(n_kc - 2 - c, NSTAGE - 2);
      if (ahead >= 2)
        asm volatile("s_waitcnt lgkmcnt(0) vmcnt(8)\n\ts_barrier" ::: "memory");
      else if (ahead == 1)
        asm volatile("s_waitcnt lgkmcnt(0) vmcnt(4)\n\ts_barrier" ::: "memory");
      else
        asm volatile("s_waitcnt lgkmcnt(0) vmcnt(0)\n\ts_barrier" ::: "memory");
      read_frags(As, Bs, (c + 1) % NSTAGE, 0, wr, wc, lane, fa0, fb0);
      mfma_group(acc, fa1, fb1);
#pragma unroll
      for (int g = 0; g < 4 + TNB; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 4 * TNB - 4 - TNB, 0);
      if (c + NSTAGE < n_kc) issue_stage(a, As, Bs, st, c + NSTAGE, row0, col0, wave, lane);
    }

    // every wave is past its last reads of the ring: the next tile's norms and
    // first stages go out now and land during this epilogue
    float inv[TNB];
    int32_t ecol[TNB];
#pragma unroll
    for (int bn = 0; bn < TNB; ++bn) {
      const int64_t e = col0 + wc * 64 + bn * 32 + (lane & 31);
      ecol[bn] = (int32_t)e;
      inv[bn] = e < a.n_entries ? (nrm[bn] > 0.0 ? (float)(1.0 / (nrm[bn] * nrm[bn])) : 0.0f)
                                : -1.0f;
    }
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (ct + 1 < ct_end) {
      const int64_t col1 = (int64_t)(ct_begin + tile_at(ct + 1 - ct_begin, n_ct)) * BBN;
      load_norms(a, col1, wc, lane, nrm);
      for (int p = 0; p < NSTAGE; ++p)
        if (p < n_kc) issue_stage(a, As, Bs, p, p, row0, col1, wave, lane);
      if (tid == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    // ---- epilogue (as in the FP32 kernel) ----
    // one row block (4 x 32 x 32 accumulators) at a time: a rolled loop with a
    // switch keeps only 64 accumulator values live in VGPRs
#pragma unroll 1
    for (int bm = 0; bm < 4; ++bm) {
      floatx16 blk[TNB];
      switch (bm) {
        case 0: blk[0] = acc[0][0]; blk[1] = acc[0][1]; break;
        case 1: blk[0] = acc[1][0]; blk[1] = acc[1][1]; break;
        case 2: blk[0] = acc[2][0]; blk[1] = acc[2][1]; break;
        default: blk[0] = acc[3][0]; blk[1] = acc[3][1]; break;
      }
      // thresholds (the current k-th best of each voxel of this block), read
      // once; an insertion below can only raise a threshold, so a value read
      // here lets through a superset of the candidates, which list_insert
      // filters exactly
      float thr[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int vme = bm * 16 + 4 * (q >> 1) + 2 * (lane >> 5) + (q & 1);
        thr[q] = myLs[vme * BKK_MAX + kk - 1];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int r = 4 * (q >> 1) + 2 * (q & 1);
        float sc[TNB];
#pragma unroll
        for (int bn = 0; bn < TNB; ++bn) {
          const float re = blk[bn][r], im = blk[bn][r + 1];
          sc[bn] = inv[bn] < 0.0f ? -1.0f : (re * re + im * im) * inv[bn];
        }
        const float mx = fmaxf(sc[0], sc[1]);
        if (__ballot(mx > thr[q]) == 0) continue;  // common case
        const int vme = bm * 16 + 4 * (q >> 1) + 2 * (lane >> 5) + (q & 1);
#pragma unroll
        for (int bn = 0; bn < TNB; ++bn) {
          uint64_t m = __ballot(sc[bn] > myLs[vme * BKK_MAX + kk - 1]);
          while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const float sv = __shfl(sc[bn], src);
            const int32_t e = __shfl(ecol[bn], src);
            const int vl = bm * 16 + 4 * (q >> 1) + 2 * (src >> 5) + (q & 1);
            list_insert(myLs + vl * BKK_MAX, myLi + vl * BKK_MAX, kk, lane, sv, e);
          }
        }
      }
    }
    if (ct + 1 < ct_end) {
      if (tid == 0) {
        // arrivals after this tile: every participant adds one per tile it
        // ends with another tile still to do
        const int i1 = ct - ct_begin + 1;
        uint32_t target = 0;
        for (int j = 0; j < a.grp_chunks; ++j) {
          const int c2 = xcd + 8 * j;
          if (c2 >= a.n_chunks) break;
          const int nt = (int)((int64_t)(c2 + 1) * a.n_col_tiles / a.n_chunks) -
                         (int)((int64_t)c2 * a.n_col_tiles / a.n_chunks);
          target += (uint32_t)rows_valid * (uint32_t)max(min(nt - 1, i1), 0);
        }
        // bounded wait (50 us of the 100 MHz real-time counter): peers that
        // are not resident (other kernels hold the CUs) only cost time, and
        // after kMaxLate timeouts in a row this workgroup stops aligning.
        // Runs of up to 12 are normal in the first tiles of a round, whose
        // list insertions (8 per voxel in the first tile) make workgroups
        // uneven; an instrumented run saw 4-41 waits over 20 us per workgroup
        // over its 1542 tiles.
        const uint64_t t0 = wall_clock64();
        bool late = false;
        while (n_late < kMaxLate &&
               __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
          if (wall_clock64() - t0 > 5000) {
            late = true;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
        n_late = late ? n_late + 1 : (n_late < kMaxLate ? 0 : n_late);
      }
      __syncthreads();
    }
  }

  for (int i = lane; i < 64 * kk; i += 64) {
    const int vl = i / kk, p = i % kk;
    const int v = (row0 + wr * 128) / 2 + vl;
    if (v < a.n_vox_pad) {
      const int64_t o = (((int64_t)chunk * WCN + wc) * a.n_vox_pad + v) * kk + p;
      a.part_s[o] = myLs[vl * BKK_MAX + p];
      a.part_i[o] = myLi[vl * BKK_MAX + p];
    }
  }
}

// K2 (BF16): unit-norm voxel (FP64 norm), packed in 4-readout blocks.
__global__ __launch_bounds__(64) void k_pack_bf16(const float2* __restrict__ vox, int64_t ld_vox,
                                                  int32_t n_vox, int32_t n_tr, int32_t nblk_pad,
                                                  int32_t m_pad, uint4* __restrict__ A,
                                                  double* __restrict__ vnorm, uint32_t* sync,
                                                  int32_t n_sync) {
  const int v = blockIdx.x;
  const int lane = threadIdx.x;
  if (v == 0)
    for (int i = lane; i < n_sync; i += 64) sync[i] = 0;
  double s2 = 0.0;
  if (v < n_vox) {
    for (int j = lane; j < n_tr; j += 64) {
      const float2 x = vox[(int64_t)v * ld_vox + j];
      s2 = fma((double)x.x, (double)x.x, s2);
      s2 = fma((double)x.y, (double)x.y, s2);
    }
  }
  for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o);
  const double nv = sqrt(s2);
  const float inv = nv > 0.0 ? (float)(1.0 / nv) : 0.0f;
  if (lane == 0 && v < n_vox) vnorm[v] = nv;
  for (int b = lane; b < nblk_pad; b += 64) {
    uint32_t re_row[4], im_row[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = 4 * b + q;
      float2 x = make_float2(0.f, 0.f);
      if (v < n_vox && j < n_tr) x = vox[(int64_t)v * ld_vox + j];
      const float xr = x.x * inv, xi = x.y * inv;
      re_row[q] = pack_bf16_pair(xr, xi);
      im_row[q] = pack_bf16_pair(xi, -xr);
    }
    A[(int64_t)b * m_pad + 2 * v] = make_uint4(re_row[0], re_row[1], re_row[2], re_row[3]);
    A[(int64_t)b * m_pad + 2 * v + 1] = make_uint4(im_row[0], im_row[1], im_row[2], im_row[3]);
  }
}

// K5: re-simulate each voxel's BF16 candidates in FP32 (same step function
// and tables as the dictionary) and re-score them exactly; one lane per
// (voxel, candidate), 8 lanes per voxel. SM: the candidates are smoothed as
// the dictionary is (the same delay line, weights and order of operations).
struct RescoreArgs {
  SmoothW sm;
  const float2* demod;  // [n_tr] (cos, sin) of the RF phases (SM)
  const float2* t1T;
  const float* t1ti;
  const float2* t2T;
  const float4* dfT;
  const float* rf;
  int32_t n_tr, inversion, n2, n3, n4;
  const float2* vox;
  int64_t ld_vox;
  int32_t n_vox, kk, top_k;
  const double* vnorm;
  const float* best_s;  // [n_vox][kk] BF16 estimates (CC^2)
  const int32_t* best_i;
  int64_t entry_base;
  int64_t* idx;
  float* cc;
  float* margin;
  float* pd_re;
  float* pd_im;
  int64_t* topk_idx;
  float* topk_cc;
};

template <bool SM>
__global__ __launch_bounds__(64) void k_rescore(RescoreArgs a) {
  const int lane = threadIdx.x;
  const int v = blockIdx.x * 8 + (lane >> 3);
  const int q = lane & 7;
  const bool active = v < a.n_vox && q < a.kk;
  int32_t e = 0x7fffffff;
  if (active) e = a.best_i[(int64_t)v * a.kk + q];
  // <v, d> in FP32 with compensated (TwoSum) accumulation: the sum carries
  // about one FP32 ulp of error instead of growing with sqrt(n_tr); the entry
  // norm accumulates in FP64.
  float sr = 0.f, cr = 0.f, si = 0.f, ci = 0.f;
  double n2 = 0.0;
  const bool sim = active && e != 0x7fffffff;
  if (sim) {
    const int64_t k = a.entry_base + e;
    int64_t t = k;
    const int32_t i4 = (int32_t)(t % a.n4);
    t /= a.n4;
    const int32_t i3 = (int32_t)(t % a.n3);
    t /= a.n3;
    const int32_t i2 = (int32_t)(t % a.n2);
    const int32_t i1 = (int32_t)(t / a.n2);
    const int32_t n = a.n_tr;
    const float2* p1 = a.t1T + (int64_t)i1 * n;
    const float2* p2 = a.t2T + (int64_t)i2 * n;
    const float4* pd = a.dfT + (int64_t)i3 * n;
    const float* R = a.rf + (int64_t)i4 * n * 9;
    const float2* x = a.vox + (int64_t)v * a.ld_vox;
    Spin m = initial_spin(a.inversion, a.t1ti[i1]);
    // output sample o (= j, or j - 2 behind the smoothing delay line)
    auto acc = [&](int32_t o, float dx, float dy) {
      const float2 s = x[o];
      // v conj(d)
      two_sum_acc(sr, cr, fmaf(s.x, dx, s.y * dy));
      two_sum_acc(si, ci, fmaf(s.y, dx, -(s.x * dy)));
      n2 = fma((double)dx, (double)dx, n2);
      n2 = fma((double)dy, (double)dy, n2);
    };
    float hx[kSmoothLen], hy[kSmoothLen];
#pragma unroll
    for (int k = 0; k < kSmoothLen; ++k) hx[k] = hy[k] = 0.f;
    for (int32_t j = 0; j < n; ++j) {
      const float2 r1 = p1[j];
      const float2 r2 = p2[j];
      const float4 pc = pd[j];
      rf_pulse(m, R + 9 * j);
      free_evolve(m, pc.x, pc.y, r2.x, r1.x);
      if (SM) {
        const int32_t o = j - kSmoothLag;
        const float sc = o >= 2 ? a.sm.full : (o == 1 ? a.sm.head[1] : a.sm.head[0]);
        float dx = m.x, dy = m.y;
        smooth_demod(a.demod[j], dx, dy);
        smooth_push(hx, hy, dx, dy);
        smooth_out(a.sm, hx, hy, sc, dx, dy);
        if (o >= 0) {
          smooth_remod(a.demod[o], dx, dy);
          acc(o, dx, dy);
        }
      } else {
        acc(j, m.x, m.y);
      }
      free_evolve(m, pc.z, pc.w, r2.y, r1.y);
    }
    if (SM) {
#pragma unroll
      for (int t = 0; t < kSmoothLag; ++t) {
        const int32_t o = n - kSmoothLag + t;
        float dx, dy;
        smooth_push(hx, hy, 0.f, 0.f);
        smooth_out(a.sm, hx, hy, a.sm.tail[t], dx, dy);
        if (o >= 0) {
          smooth_remod(a.demod[o], dx, dy);
          acc(o, dx, dy);
        }
      }
    }
  }
  const double dr = (double)sr + (double)cr, di = (double)si + (double)ci;
  float c = -1.0f;
  if (sim) {
    const double nv = a.vnorm[v];
    c = (n2 > 0.0 && nv > 0.0) ? (float)(sqrt(dr * dr + di * di) / (sqrt(n2) * nv)) : 0.0f;
  }
  // best and runner-up among the 8 lanes of this voxel (ties: lower index)
  float bc = c;
  int32_t be = sim ? e : 0x7fffffff;
  int bl = q;
  for (int o = 4; o > 0; o >>= 1) {
    const float oc = __shfl_xor(bc, o, 8);
    const int32_t oe = __shfl_xor(be, o, 8);
    const int ol = __shfl_xor(bl, o, 8);
    if (beats(oc, oe, bc, be)) {
      bc = oc;
      be = oe;
      bl = ol;
    }
  }
  float sc = (q == bl) ? -1.0f : c;  // runner-up: best of the others
  for (int o = 4; o > 0; o >>= 1) sc = fmaxf(sc, __shfl_xor(sc, o, 8));
  const double bdr = __shfl(dr, (lane & ~7) + bl);
  const double bdi = __shfl(di, (lane & ~7) + bl);
  const double bn2 = __shfl(n2, (lane & ~7) + bl);
  if (v < a.n_vox && q == 0) {
    a.idx[v] = be == 0x7fffffff ? -1 : a.entry_base + be;
    if (a.cc) a.cc[v] = fmaxf(bc, 0.0f);
    if (a.margin) a.margin[v] = sc < 0.0f ? INFINITY : bc - sc;
    if (a.pd_re) a.pd_re[v] = bn2 > 0.0 ? (float)(bdr / bn2) : 0.0f;
    if (a.pd_im) a.pd_im[v] = bn2 > 0.0 ? (float)(bdi / bn2) : 0.0f;
  }
  if (v < a.n_vox && q < a.top_k) {
    const float s = a.best_s[(int64_t)v * a.kk + q];
    if (a.topk_idx) a.topk_idx[(int64_t)v * a.top_k + q] = e == 0x7fffffff ? -1 : a.entry_base + e;
    if (a.topk_cc) a.topk_cc[(int64_t)v * a.top_k + q] = sqrtf(fmaxf(s, 0.0f));
  }
}

// ---------------------------------------------------------------------------
static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct PlanB {
  int32_t nblk, nblk_pad, m_pad, n_vox_pad, n_row_tiles, n_col_tiles, n_chunks, kk;
  int32_t grp_rows, grp_chunks, n_wg;
  size_t off_A, off_vn, off_ps, off_pi, off_bs, off_bi, off_sync, total;
  int32_t n_sync;
};

static PlanB plan_bf16(const mrf_dict_view* d, int32_t n_vox, int32_t top_k, int n_cu) {
  PlanB p;
  p.kk = std::max(top_k, 2);
  p.nblk = d->n_tr / 4;
  p.nblk_pad = (p.nblk + BKB - 1) / BKB * BKB;
  p.m_pad = std::max((2 * n_vox + BBM - 1) / BBM * BBM, BBM);
  p.n_vox_pad = p.m_pad / 2;
  p.n_row_tiles = p.m_pad / BBM;
  p.n_col_tiles = (int32_t)((d->n_entries + BBN - 1) / BBN);
  // one workgroup per CU (the LDS ring takes most of it), n_cu / 8 per XCD:
  // up to 8 row tiles x the rest in chunks resident together on an XCD
  const int per_xcd = std::max(n_cu / 8, 1);
  p.grp_rows = std::min(p.n_row_tiles, 8);
  p.grp_chunks = std::max(per_xcd / p.grp_rows, 1);
  p.grp_chunks = std::min(p.grp_chunks, std::max((p.n_col_tiles + 7) / 8, 1));
  p.n_chunks = 8 * p.grp_chunks;
  const int n_groups = (p.n_row_tiles + p.grp_rows - 1) / p.grp_rows;
  p.n_wg = 8 * n_groups * p.grp_rows * p.grp_chunks;
  size_t o = 0;
  p.off_A = o;
  o = al(o + sizeof(uint4) * (size_t)p.nblk_pad * p.m_pad);
  p.off_vn = o;
  o = al(o + sizeof(double) * (size_t)p.n_vox_pad);
  const size_t np = (size_t)p.n_chunks * WCN * p.n_vox_pad * p.kk;
  p.off_ps = o;
  o = al(o + sizeof(float) * np);
  p.off_pi = o;
  o = al(o + sizeof(int32_t) * np);
  p.off_bs = o;
  o = al(o + sizeof(float) * (size_t)p.n_vox_pad * p.kk);
  p.off_bi = o;
  o = al(o + sizeof(int32_t) * (size_t)p.n_vox_pad * p.kk);
  p.n_sync = 8 * n_groups;
  p.off_sync = o;
  o = al(o + sizeof(uint32_t) * (size_t)p.n_sync);
  p.total = o;
  return p;
}

size_t bf16_workspace_bytes(const mrf_dict_view* d, int32_t n_vox, int32_t top_k, int n_cu) {
  return plan_bf16(d, n_vox, top_k, n_cu).total;
}

int match_bf16(mrf_context* ctx, const mrf_dict_view* d, const void* vox, int32_t n_vox,
               int64_t ld_vox, int32_t top_k, const mrf_sequence* seq, const mrf_grid* grid,
               mrf_result_view out, int64_t* topk_idx, float* topk_cc, void* workspace,
               size_t ws_bytes, hipStream_t st) {
  MRF_CHECK_ARG(seq != nullptr && grid != nullptr,
                "a BF16 dictionary needs seq and grid (candidates are re-simulated in FP32)");
  int rc = check_grid(grid);
  if (rc) return rc;
  MRF_CHECK_ARG(top_k >= 2 && top_k <= BKK_MAX, "BF16 matching needs top_k in [2, %d]", BKK_MAX);
  MRF_CHECK_ARG(d->n_tr <= seq->n, "dictionary n_tr exceeds the sequence length");
  MRF_CHECK_ARG(d->entry_base + d->n_entries <= grid_size_checked(grid),
                "dictionary entries exceed the grid");
  const PlanB p = plan_bf16(d, n_vox, top_k, ctx->n_cu);
  MRF_CHECK_ARG(ws_bytes >= p.total, "workspace too small (%zu < %zu bytes)", ws_bytes, p.total);
  TablesRef tref;  // held until the launches are enqueued
  rc = get_tables(const_cast<mrf_sequence*>(seq), grid, d->n_tr, st, &tref);
  const Tables* t = tref.get();
  if (rc) return rc;
  char* ws = (char*)workspace;
  uint4* A = (uint4*)(ws + p.off_A);
  double* vn = (double*)(ws + p.off_vn);
  float* ps = (float*)(ws + p.off_ps);
  int32_t* pi = (int32_t*)(ws + p.off_pi);
  float* bs = (float*)(ws + p.off_bs);
  int32_t* bi = (int32_t*)(ws + p.off_bi);
  {
    ProfScope prof(ctx, "k_pack_bf16", st);
    hipLaunchKernelGGL(k_pack_bf16, dim3(p.n_vox_pad), dim3(64), 0, st, (const float2*)vox,
                       ld_vox, n_vox, d->n_tr, p.nblk_pad, p.m_pad, A, vn,
                       (uint32_t*)(ws + p.off_sync), p.n_sync);
  }
  MRF_HIP(hipGetLastError());
  MatchB16Args a;
  a.A = A;
  a.B = (const uint4*)d->re;
  a.norm = d->norm;
  a.nblk = p.nblk;
  a.nblk_pad = p.nblk_pad;
  a.m_pad = p.m_pad;
  a.n_vox_pad = p.n_vox_pad;
  a.ld = d->ld;
  a.n_entries = d->n_entries;
  a.n_row_tiles = p.n_row_tiles;
  a.n_chunks = p.n_chunks;
  a.n_col_tiles = p.n_col_tiles;
  a.kk = p.kk;
  a.grp_rows = p.grp_rows;
  a.grp_chunks = p.grp_chunks;
  a.part_s = ps;
  a.part_i = pi;
  a.sync = (uint32_t*)(ws + p.off_sync);
  // 128 KB of ring + 32 KB of candidate lists: the whole 160 KB of a CU
  const size_t lds = sizeof(uint4) * NSTAGE * BKB * (BBM + BBN) +
                     (sizeof(float) + sizeof(int32_t)) * NW * 64 * BKK_MAX;
  static_assert(sizeof(uint4) * NSTAGE * BKB * (BBM + BBN) +
                        (sizeof(float) + sizeof(int32_t)) * NW * 64 * BKK_MAX <=
                    160 * 1024,
                "LDS budget of one CU");
  static bool attr = false;
  if (!attr) {
    MRF_HIP(hipFuncSetAttribute((const void*)k_match_bf16,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    attr = true;
  }
  {
    ProfScope prof(ctx, "k_match_bf16", st);
    hipLaunchKernelGGL(k_match_bf16, dim3(p.n_wg), dim3(64 * NW), lds, st, a);
  }
  MRF_HIP(hipGetLastError());
  MergeArgs m;
  m.part_s = ps;
  m.part_i = pi;
  m.n_lists = p.n_chunks * WCN;
  m.n_vox = n_vox;
  m.n_vox_pad = p.n_vox_pad;
  m.kk = p.kk;
  m.top_k = top_k;
  m.entry_base = d->entry_base;
  m.best_s = bs;
  m.best_i = bi;
  m.idx = nullptr;  // final outputs come from the re-scoring
  m.cc = nullptr;
  m.margin = nullptr;
  m.topk_idx = nullptr;
  m.topk_cc = nullptr;
  rc = launch_merge(ctx, m, st);
  if (rc) return rc;
  RescoreArgs r;
  r.t1T = t->t1T;
  r.t1ti = t->t1ti;
  r.t2T = t->t2T;
  r.dfT = t->dfT;
  r.rf = t->rf;
  r.n_tr = d->n_tr;
  r.inversion = t->inversion;
  r.n2 = t->n2;
  r.n3 = t->n3;
  r.n4 = t->n4;
  r.vox = (const float2*)vox;
  r.ld_vox = ld_vox;
  r.n_vox = n_vox;
  r.kk = p.kk;
  r.top_k = top_k;
  r.vnorm = vn;
  r.best_s = bs;
  r.best_i = bi;
  r.entry_base = d->entry_base;
  r.idx = out.idx;
  r.cc = out.cc;
  r.margin = out.margin;
  r.pd_re = out.pd_re;
  r.pd_im = out.pd_im;
  r.topk_idx = topk_idx;
  r.topk_cc = topk_cc;
  r.sm = smooth_weights(t->smooth ? t->smooth : 3, d->n_tr);
  r.demod = t->demod;
  {
    ProfScope prof(ctx, "k_rescore", st);
    if (t->smooth)
      hipLaunchKernelGGL(k_rescore<true>, dim3((n_vox + 7) / 8), dim3(64), 0, st, r);
    else
      hipLaunchKernelGGL(k_rescore<false>, dim3((n_vox + 7) / 8), dim3(64), 0, st, r);
  }
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}

}  // namespace mrf
