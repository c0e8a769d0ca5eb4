// Brute-force matching (Theory Eq. 1, exhaustive search): K2 voxel packing,
// K3 complex GEMM on MFMA with a fused per-voxel top-k epilogue, K4 merge.
//
// The complex inner products s_vk = sum_j vhat_j conj(d_kj) are formed from
// three real GEMMs over the readouts (see K3 below), and
// CC_vk^2 = |s_vk|^2 / ||d_k||^2. The score matrix is never written: every
// workgroup keeps the running top-k of its voxels over its share of the
// entries and writes only those lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "compensated.h"
#include "internal.h"
#include "match_common.h"
#include "match_kernels.h"

namespace mrf {

// Tile geometry of the FP32 GEMM (workgroup of 256 threads = 4 waves).
constexpr int BN = 128;      // entries per tile
// readouts per LDS chunk: 72 KB of LDS, two workgroups per CU. With 8
// readouts (44 KB, three workgroups per CU) the chunk's barrier and refill
// took a larger share: 3.15 s instead of 2.85 s on the slice.
constexpr int KC = 16;
constexpr int NLD = KC / 4;  // float4 of B each thread moves per chunk
// Candidate lists kept in the epilogue: up to 16 in the default kernel (72 KB
// of LDS, two workgroups per CU); longer lists (up to 64, the boundary's
// limit) take a kernel instance with 64-entry lists (120 KB, one per CU).
constexpr int KK_SHORT = 16;
constexpr int KK_MAX = 64;
constexpr int kWgPerCu = 2;  // resident workgroups per CU (LDS allows two)

// ---------------------------------------------------------------------------
// K3, three-product form. With T1 = sum vr dr, T2 = sum vi di and
// T3 = sum (vr + vi)(dr - di) (v the unit voxel, d the entry, sums over the
// readouts), Re s = T1 + T2 and Im s = T3 - T1 + T2: three real GEMMs with
// K = n_tr instead of one with M = 2 V and K = 2 n_tr, so 6 V N E matrix
// flops instead of 8 V N E. A holds three planes [vr | vi | vr + vi] of the
// voxels, B stays the dictionary's two planes; dr - di is formed from the
// two B fragments in registers. Tile: 64 voxels x 128 entries, four waves
// 2 x 2, each 32 voxels x 64 entries = two 32 x 32 blocks per product;
// v_mfma_f32_32x32x2_f32 takes two readouts of one plane per instruction
// (lanes 0-31 readout 2p, lanes 32-63 readout 2p + 1). Against the
// two-rows-per-voxel form (M = 2 V, K = 2 n_tr, 8 V N E flops) this measured
// 3.14 s instead of 3.38 s on the 64 x 64 slice with 8-readout chunks (the
// thresholds of the top-k filter read from the lists in LDS keep the extra
// accumulators within three waves per SIMD without spills), 2.85 s with
// 16-readout chunks at two waves per SIMD.
// ---------------------------------------------------------------------------
constexpr int BV3 = 64;                      // voxels per tile
constexpr int NLA3 = 3 * KC * BV3 / 4 / 256;  // float4 of A every thread moves per chunk
constexpr int NLA3_REM = 3 * KC * BV3 / 4 - NLA3 * 256;  // and the threads moving one more

struct Match3Args {
  const float* A;       // [3][n_tr_pad][v_pad]
  const float* Bre;     // [n_tr][ld]
  const float* Bim;
  const double* norm;   // [n_entries] or NULL
  int32_t n_tr, n_tr_pad, v_pad;
  int64_t ld, n_entries;
  int32_t n_row_tiles, n_chunks, n_col_tiles, kk;
  float* part_s;        // [n_chunks][2][v_pad][kk]
  int32_t* part_i;
};

typedef __attribute__((address_space(3))) void* lds_ptr3;
typedef const __attribute__((address_space(1))) void* glb_ptr3;

// Chunk c's voxel planes ([g][s][c4], 16 float4 per row) and dictionary
// planes ([g][s][c4], 32 float4 per row) moved straight into LDS buffer `buf`
// with global_load_lds_dwordx4: each wave's 64 lanes fill one contiguous 1 KB
// piece. No registers stage the chunk, so the loads go out at the start of the
// previous chunk's MFMAs and land while they run. (With loads into registers
// and ds_write the compiler sank the loads to the end of the MFMA block to
// save registers and waited for them at once: every chunk paid a full
// global-load round trip; this form measured 7% faster, 2616-2622 against
// 2821-2830 ms on the slice.) Readouts past n_tr are clamped to a stored row
// (they meet zero voxel rows), columns past ld to the last float4 (masked in
// the epilogue).
__device__ __forceinline__ void issue_chunk3(const Match3Args& a, float* As, float* Bs, int buf,
                                             int c, int vox0, int64_t col0, int tid) {
  static_assert(NLA3_REM == 0, "the voxel planes move in whole rounds of 256 float4");
  const int s0 = c * KC;
  const int wave = tid >> 6;
  float* as = As + buf * 3 * KC * BV3;
  float* bs = Bs + buf * 2 * KC * BN;
#pragma unroll
  for (int i = 0; i < NLA3; ++i) {
    const int idx = i * 256 + tid;
    const int g = idx / (KC * 16);
    const int s = (idx / 16) % KC;
    const int c4 = idx & 15;
    const float* src = a.A + ((int64_t)g * a.n_tr_pad + s0 + s) * a.v_pad + vox0 + 4 * c4;
    __builtin_amdgcn_global_load_lds((glb_ptr3)src, (lds_ptr3)(as + 4 * (i * 256 + wave * 64)),
                                     16, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < NLD; ++i) {
    const int idx = i * 256 + tid;
    const int g = idx / (KC * 32);
    const int s = (idx / 32) % KC;
    const int c4 = idx & 31;
    int64_t col = col0 + 4 * c4;
    col = col + 4 <= a.ld ? col : a.ld - 4;
    const int row = s0 + s < a.n_tr ? s0 + s : a.n_tr - 1;
    const float* bp = g ? a.Bim : a.Bre;
    __builtin_amdgcn_global_load_lds((glb_ptr3)(bp + (int64_t)row * a.ld + col),
                                     (lds_ptr3)(bs + 4 * (i * 256 + wave * 64)), 16, 0, 0);
  }
}

template <int KL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_match_f32_3m(
    Match3Args a) {
  // XCD-aware mapping: consecutive workgroup ids go to different XCDs
  // (round robin over 8), so the row tiles of one column chunk are grouped on
  // one XCD and share its L2 for the dictionary tiles.
  const int w = blockIdx.x;
  const int xcd = w & 7;
  const int slot = w >> 3;
  const int rt = slot % a.n_row_tiles;
  const int chunk = xcd + 8 * (slot / a.n_row_tiles);
  if (chunk >= a.n_chunks) return;

  extern __shared__ __align__(16) unsigned char smem[];
  float* As = (float*)smem;                    // [2 buf][3 g][KC][BV3]
  float* Bs = As + 2 * 3 * KC * BV3;           // [2 buf][2 g][KC][BN]
  float* Ls = Bs + 2 * 2 * KC * BN;            // [4 waves][32 voxels][KL]
  int32_t* Li = (int32_t*)(Ls + 4 * 32 * KL);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int h = lane >> 5;
  const int kk = a.kk;
  const int vox0 = rt * BV3;

  float* myLs = Ls + wave * 32 * KL;
  int32_t* myLi = Li + wave * 32 * KL;
  for (int i = lane; i < 32 * KL; i += 64) {
    myLs[i] = -1.0f;
    myLi[i] = 0x7fffffff;
  }
  __syncthreads();  // the lists' initial values before the first threshold read

  const int ct_begin = (int)((int64_t)chunk * a.n_col_tiles / a.n_chunks);
  const int ct_end = (int)((int64_t)(chunk + 1) * a.n_col_tiles / a.n_chunks);
  const int n_kc = a.n_tr_pad / KC;

  for (int ct = ct_begin; ct < ct_end; ++ct) {
    const int64_t col0 = (int64_t)ct * BN;
    floatx16 t1[2], t2[2], t3[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) t1[j][r] = t2[j][r] = t3[j][r] = 0.0f;

    issue_chunk3(a, As, Bs, 0, 0, vox0, col0, tid);
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    for (int c = 0; c < n_kc; ++c) {
      const int buf = c & 1;
      if (c + 1 < n_kc) issue_chunk3(a, As, Bs, buf ^ 1, c + 1, vox0, col0, tid);
      const float* as = As + buf * 3 * KC * BV3 + h * BV3 + wr * 32 + (lane & 31);
      const float* bs = Bs + buf * 2 * KC * BN + h * BN + wc * 64 + (lane & 31);
#pragma unroll
      for (int p = 0; p < KC / 2; ++p) {
        const int s = 2 * p;
        const float a1 = as[s * BV3], a2 = as[(KC + s) * BV3], a3 = as[(2 * KC + s) * BV3];
        const float r0 = bs[s * BN], r1 = bs[s * BN + 32];
        const float i0 = bs[(KC + s) * BN], i1 = bs[(KC + s) * BN + 32];
        t1[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, r0, t1[0], 0, 0, 0);
        t1[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, r1, t1[1], 0, 0, 0);
        t2[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, i0, t2[0], 0, 0, 0);
        t2[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a2, i1, t2[1], 0, 0, 0);
        t3[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a3, r0 - i0, t3[0], 0, 0, 0);
        t3[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a3, r1 - i1, t3[1], 0, 0, 0);
      }
      // chunk c + 1 landed for this wave, then for everyone (and every wave
      // is past its reads of buffer buf, which chunk c + 2 refills)
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    }

    // ---- epilogue: scores of this tile, threshold filter, list insertion ----
    float inv[2];
    int32_t ecol[2];
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) {
      const int64_t e = col0 + wc * 64 + bn * 32 + (lane & 31);
      ecol[bn] = (int32_t)e;
      if (e < a.n_entries) {
        double n = a.norm ? a.norm[e] : 1.0;
        inv[bn] = n > 0.0 ? (float)(1.0 / (n * n)) : 0.0f;
      } else {
        inv[bn] = -1.0f;  // marks a padding column
      }
    }
#pragma unroll
    for (int bn = 0; bn < 2; ++bn) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        // output row 8 (r / 4) + 4 h + r % 4 of the block = voxel slot
        const float re = t1[bn][r] + t2[bn][r];
        const float im = t3[bn][r] - t1[bn][r] + t2[bn][r];
        const float sc = inv[bn] < 0.0f ? -1.0f : (re * re + im * im) * inv[bn];
        // this lane's voxel: the k-th best so far (read from its list)
        const float thr = myLs[(8 * (r >> 2) + 4 * h + (r & 3)) * KL + kk - 1];
        const bool cand = sc > thr;
        uint64_t m = __ballot(cand);
        while (m) {
          const int src = __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          const float sv = __shfl(sc, src);
          const int32_t e = __shfl(ecol[bn], src);
          const int vl = 8 * (r >> 2) + 4 * (src >> 5) + (r & 3);
          list_insert(myLs + vl * KL, myLi + vl * KL, kk, lane, sv, e);
        }
      }
    }
  }

  // write this wave's lists: partial[chunk][wc][voxel][kk]
  for (int i = lane; i < 32 * kk; i += 64) {
    const int vl = i / kk, p = i % kk;
    const int v = vox0 + wr * 32 + vl;
    if (v < a.v_pad) {
      const int64_t o = (((int64_t)chunk * 2 + wc) * a.v_pad + v) * kk + p;
      a.part_s[o] = myLs[vl * KL + p];
      a.part_i[o] = myLi[vl * KL + p];
    }
  }
}

// K2 for the three-product form: A = [vr | vi | vr + vi] of the unit voxels,
// time-major, zero past n_tr and past n_vox. One wave per voxel.
__global__ __launch_bounds__(64) void k_pack_f32_3m(const float2* __restrict__ vox,
                                                    int64_t ld_vox, int32_t n_vox, int32_t n_tr,
                                                    int32_t n_tr_pad, int32_t v_pad,
                                                    float* __restrict__ A,
                                                    double* __restrict__ vnorm) {
  const int v = blockIdx.x;
  const int lane = threadIdx.x;
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
  const int64_t plane = (int64_t)n_tr_pad * v_pad;
  for (int j = lane; j < n_tr_pad; j += 64) {
    float2 x = make_float2(0.f, 0.f);
    if (v < n_vox && j < n_tr) x = vox[(int64_t)v * ld_vox + j];
    const float xr = x.x * inv, xi = x.y * inv;
    float* col = A + (int64_t)j * v_pad + v;
    col[0] = xr;
    col[plane] = xi;
    col[2 * plane] = xr + xi;
  }
}

// ---------------------------------------------------------------------------
// K4: merge the partial lists of every chunk into the final top-k per voxel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_merge(MergeArgs a) {
  const int v = blockIdx.x * 64 + threadIdx.x;
  if (v >= a.n_vox) return;
  float ls[KK_SHORT];
  int32_t li[KK_SHORT];
  for (int p = 0; p < KK_SHORT; ++p) {
    ls[p] = -1.0f;
    li[p] = 0x7fffffff;
  }
  for (int l = 0; l < a.n_lists; ++l) {
    const int64_t o = ((int64_t)l * a.n_vox_pad + v) * a.kk;
    for (int p = 0; p < a.kk; ++p) {
      float s = a.part_s[o + p];
      int32_t e = a.part_i[o + p];
      if (e == 0x7fffffff) break;
      if (!beats(s, e, ls[a.kk - 1], li[a.kk - 1])) break;  // lists are sorted
      int q = a.kk - 1;
      while (q > 0 && beats(s, e, ls[q - 1], li[q - 1])) {
        ls[q] = ls[q - 1];
        li[q] = li[q - 1];
        --q;
      }
      ls[q] = s;
      li[q] = e;
    }
  }
  for (int p = 0; p < a.kk; ++p) {
    a.best_s[(int64_t)v * a.kk + p] = ls[p];
    a.best_i[(int64_t)v * a.kk + p] = li[p];
  }
  const float c1 = sqrtf(fmaxf(ls[0], 0.0f));
  if (a.idx) a.idx[v] = li[0] == 0x7fffffff ? -1 : a.entry_base + li[0];
  if (a.cc) a.cc[v] = c1;
  if (a.margin) a.margin[v] = li[1] == 0x7fffffff ? INFINITY : c1 - sqrtf(fmaxf(ls[1], 0.0f));
  for (int p = 0; p < a.top_k; ++p) {
    if (a.topk_idx)
      a.topk_idx[(int64_t)v * a.top_k + p] = li[p] == 0x7fffffff ? -1 : a.entry_base + li[p];
    if (a.topk_cc) a.topk_cc[(int64_t)v * a.top_k + p] = sqrtf(fmaxf(ls[p], 0.0f));
  }
}

// K4 for lists longer than 16: one wave per voxel, lane p holding entry p of
// the running list. Each chunk's sorted list is read by the wave at once and
// its entries are inserted in order with the wave-parallel shift of
// list_insert, stopping at the first one that cannot enter. The result, the
// best kk by (score desc, index asc), is the same as k_merge's.
__global__ __launch_bounds__(64) void k_merge_wave(MergeArgs a) {
  const int v = blockIdx.x;
  const int lane = threadIdx.x;
  if (v >= a.n_vox) return;
  const int kk = a.kk;
  float cs = -1.0f;
  int32_t ci = 0x7fffffff;
  for (int l = 0; l < a.n_lists; ++l) {
    const int64_t o = ((int64_t)l * a.n_vox_pad + v) * kk;
    float s = -1.0f;
    int32_t e = 0x7fffffff;
    if (lane < kk) {
      s = a.part_s[o + lane];
      e = a.part_i[o + lane];
    }
    for (int p = 0; p < kk; ++p) {
      const float sp = __shfl(s, p);
      const int32_t ep = __shfl(e, p);
      if (ep == 0x7fffffff) break;
      const float ls_last = __shfl(cs, kk - 1);
      const int32_t li_last = __shfl(ci, kk - 1);
      if (!beats(sp, ep, ls_last, li_last)) break;  // the chunk's list is sorted
      const bool ahead = lane < kk && beats(cs, ci, sp, ep);
      const int q = __popcll(__ballot(ahead));
      const float ps = __shfl_up(cs, 1);
      const int32_t pi = __shfl_up(ci, 1);
      if (lane < kk) {
        if (lane == q) {
          cs = sp;
          ci = ep;
        } else if (lane > q) {
          cs = ps;
          ci = pi;
        }
      }
    }
  }
  if (lane < kk) {
    a.best_s[(int64_t)v * kk + lane] = cs;
    a.best_i[(int64_t)v * kk + lane] = ci;
  }
  const float s0 = __shfl(cs, 0), s1 = __shfl(cs, 1);
  const int32_t i0 = __shfl(ci, 0), i1 = __shfl(ci, 1);
  if (lane == 0) {
    const float c1 = sqrtf(fmaxf(s0, 0.0f));
    if (a.idx) a.idx[v] = i0 == 0x7fffffff ? -1 : a.entry_base + i0;
    if (a.cc) a.cc[v] = c1;
    if (a.margin) a.margin[v] = i1 == 0x7fffffff ? INFINITY : c1 - sqrtf(fmaxf(s1, 0.0f));
  }
  if (lane < a.top_k) {
    if (a.topk_idx)
      a.topk_idx[(int64_t)v * a.top_k + lane] = ci == 0x7fffffff ? -1 : a.entry_base + ci;
    if (a.topk_cc) a.topk_cc[(int64_t)v * a.top_k + lane] = sqrtf(fmaxf(cs, 0.0f));
  }
}

// PD = <v, d> / ||d||^2 of the best entry (Theory: PD from the signal scale).
// One wave per voxel; FP32 planar dictionary. The product is accumulated in
// FP32 with compensation (Dot2) and the lanes' pairs are added with TwoSum;
// only the entry's norm is accumulated in FP64.
__global__ __launch_bounds__(64) void k_pd_f32(const float2* __restrict__ vox, int64_t ld_vox,
                                               int32_t n_vox, int32_t n_tr, const float* Bre,
                                               const float* Bim, int64_t ld,
                                               const int32_t* best_i, int32_t kk,
                                               const double* norm, float* pd_re, float* pd_im) {
  const int v = blockIdx.x;
  const int lane = threadIdx.x;
  if (v >= n_vox) return;
  const int32_t e = best_i[(int64_t)v * kk];
  float sr = 0.0f, cr = 0.0f, si = 0.0f, ci = 0.0f;
  double n2 = 0.0;
  if (e != 0x7fffffff) {
    for (int j = lane; j < n_tr; j += 64) {
      const float2 x = vox[(int64_t)v * ld_vox + j];
      const float dr = Bre[(int64_t)j * ld + e], di = Bim[(int64_t)j * ld + e];
      dot2_acc(x.x, dr, sr, cr);
      dot2_acc(x.y, di, sr, cr);
      dot2_acc(x.y, dr, si, ci);
      dot2_acc(-x.x, di, si, ci);
      n2 = fma((double)dr, (double)dr, n2);
      n2 = fma((double)di, (double)di, n2);
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    // the partner's pair as it was before this step's addition
    const float osr = __shfl_xor(sr, o), ocr = __shfl_xor(cr, o);
    const float osi = __shfl_xor(si, o), oci = __shfl_xor(ci, o);
    two_sum_acc(sr, cr, osr);
    cr += ocr;
    two_sum_acc(si, ci, osi);
    ci += oci;
    n2 += __shfl_xor(n2, o);
  }
  if (lane == 0) {
    // n_tr may be a prefix of the stored entries: use the prefix norm
    (void)norm;
    const float d2 = (float)n2;
    if (pd_re) pd_re[v] = d2 > 0.0f ? (sr + cr) / d2 : 0.0f;
    if (pd_im) pd_im[v] = d2 > 0.0f ? (si + ci) / d2 : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int launch_merge(mrf_context* ctx, const MergeArgs& m, hipStream_t st) {
  {
    ProfScope prof(ctx, "k_merge", st);
    if (m.kk <= KK_SHORT)
      hipLaunchKernelGGL(k_merge, dim3((m.n_vox + 63) / 64), dim3(64), 0, st, m);
    else
      hipLaunchKernelGGL(k_merge_wave, dim3(m.n_vox), dim3(64), 0, st, m);
  }
  MRF_HIP(hipGetLastError());
  return MRF_OK;
}

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }


struct Plan {
  int32_t n_tr_pad, n_vox_pad, n_row_tiles, n_col_tiles, n_chunks, kk;
  size_t off_A, off_vn, off_ps, off_pi, off_bs, off_bi, total;
};

static Plan make_plan(const mrf_dict_view* d, int32_t n_vox, int32_t top_k, int n_cu) {
  Plan p;
  p.kk = std::max(top_k, 2);
  p.n_tr_pad = (d->n_tr + KC - 1) / KC * KC;
  p.n_vox_pad = std::max((n_vox + BV3 - 1) / BV3 * BV3, BV3);
  p.n_row_tiles = p.n_vox_pad / BV3;
  p.n_col_tiles = (int32_t)((d->n_entries + BN - 1) / BN);
  // enough chunks for two rounds of the three resident workgroups per CU, a
  // multiple of 8 (XCDs)
  int want = (2 * kWgPerCu * n_cu + p.n_row_tiles - 1) / p.n_row_tiles;
  want = std::min(want, std::max(p.n_col_tiles, 1));
  p.n_chunks = std::max(8, (want + 7) / 8 * 8);
  size_t o = 0;
  p.off_A = o;
  o = al(o + sizeof(float) * 3 * (size_t)p.n_tr_pad * p.n_vox_pad);
  p.off_vn = o;
  o = al(o + sizeof(double) * (size_t)p.n_vox_pad);
  const size_t np = (size_t)p.n_chunks * 2 * p.n_vox_pad * p.kk;
  p.off_ps = o;
  o = al(o + sizeof(float) * np);
  p.off_pi = o;
  o = al(o + sizeof(int32_t) * np);
  p.off_bs = o;
  o = al(o + sizeof(float) * (size_t)p.n_vox_pad * p.kk);
  p.off_bi = o;
  o = al(o + sizeof(int32_t) * (size_t)p.n_vox_pad * p.kk);
  p.total = o;
  return p;
}

static int check_view(const mrf_dict_view* d) {
  MRF_CHECK_ARG(d != nullptr, "dictionary view is NULL");
  MRF_CHECK_ARG(d->dtype == MRF_F32 || d->dtype == MRF_BF16, "unknown dictionary dtype");
  MRF_CHECK_ARG(d->n_tr >= 1, "dictionary n_tr must be >= 1");
  MRF_CHECK_ARG(d->n_entries >= 1 && d->n_entries <= 0x7ffffffe,
                "dictionary n_entries (%lld) out of range", (long long)d->n_entries);
  MRF_CHECK_ARG(d->ld >= d->n_entries, "dictionary ld must be >= n_entries");
  MRF_CHECK_ARG(d->ld % 4 == 0, "dictionary ld must be a multiple of 4");
  MRF_CHECK_ARG(d->re != nullptr, "dictionary re is NULL");
  MRF_CHECK_ARG(((uintptr_t)d->re & 15) == 0, "dictionary re must be 16-byte aligned");
  if (d->dtype == MRF_F32) {
    MRF_CHECK_ARG(d->im != nullptr, "dictionary im is NULL");
    MRF_CHECK_ARG(((uintptr_t)d->im & 15) == 0, "dictionary im must be 16-byte aligned");
  } else {
    MRF_CHECK_ARG(d->im == nullptr, "im must be NULL for a packed BF16 dictionary");
    MRF_CHECK_ARG(d->n_tr % 4 == 0, "BF16 dictionary n_tr must be a multiple of 4");
  }
  MRF_CHECK_ARG(d->entry_base >= 0, "entry_base must be >= 0");
  return MRF_OK;
}

}  // namespace mrf

using namespace mrf;

extern "C" int mrf_match_workspace(mrf_context* ctx, const mrf_dict_view* d, int32_t n_vox,
                                   int32_t top_k, size_t* bytes) {
  MRF_CHECK_ARG(ctx && bytes, "NULL argument");
  int rc = check_view(d);
  if (rc) return rc;
  MRF_CHECK_ARG(n_vox >= 0, "n_vox must be >= 0");
  MRF_CHECK_ARG(top_k >= 1 && top_k <= KK_MAX, "top_k must be in [1, %d]", KK_MAX);
  if (d->dtype == MRF_BF16) {
    *bytes = bf16_workspace_bytes(d, n_vox, top_k, ctx->n_cu);
    return MRF_OK;
  }
  *bytes = make_plan(d, n_vox, top_k, ctx->n_cu).total;
  return MRF_OK;
}

namespace mrf {

size_t match_f32_workspace_bytes(const mrf_dict_view* d, int32_t n_vox, int32_t top_k, int n_cu) {
  return make_plan(d, n_vox, top_k, n_cu).total;
}

// FP32 brute force (K2 packing, K3 GEMM with the fused top-k, K4 merge, PD of
// the best entry) with the caller's workspace. The arguments have been
// checked by the entry point (view, sizes, pointers). `profile` = false keeps
// the launches free of event creation (the allocation-free entry point).
int match_f32_run(mrf_context* ctx, const mrf_dict_view* d, const void* vox, int32_t n_vox,
                  int64_t ld_vox, int32_t top_k, mrf_result_view out, int64_t* topk_idx,
                  float* topk_cc, void* workspace, size_t ws_bytes, hipStream_t st,
                  bool profile) {
  const Plan p = make_plan(d, n_vox, top_k, ctx->n_cu);
  MRF_CHECK_ARG(ws_bytes >= p.total, "workspace too small (%zu < %zu bytes)", ws_bytes, p.total);
  char* ws = (char*)workspace;
  float* A = (float*)(ws + p.off_A);
  double* vn = (double*)(ws + p.off_vn);
  float* ps = (float*)(ws + p.off_ps);
  int32_t* pi = (int32_t*)(ws + p.off_pi);
  float* bs = (float*)(ws + p.off_bs);
  int32_t* bi = (int32_t*)(ws + p.off_bi);
  mrf_context* pctx = profile ? ctx : nullptr;

  {
    ProfScope prof(pctx, "k_pack_f32", st);
    hipLaunchKernelGGL(k_pack_f32_3m, dim3(p.n_vox_pad), dim3(64), 0, st, (const float2*)vox,
                       ld_vox, n_vox, d->n_tr, p.n_tr_pad, p.n_vox_pad, A, vn);
  }
  MRF_HIP(hipGetLastError());
  Match3Args a;
  a.A = A;
  a.Bre = (const float*)d->re;
  a.Bim = (const float*)d->im;
  a.norm = d->norm;
  a.n_tr = d->n_tr;
  a.n_tr_pad = p.n_tr_pad;
  a.v_pad = p.n_vox_pad;
  a.ld = d->ld;
  a.n_entries = d->n_entries;
  a.n_row_tiles = p.n_row_tiles;
  a.n_chunks = p.n_chunks;
  a.n_col_tiles = p.n_col_tiles;
  a.kk = p.kk;
  a.part_s = ps;
  a.part_i = pi;
  const int grid_wg = p.n_row_tiles * p.n_chunks;
  const bool longl = p.kk > KK_SHORT;
  const size_t lds = sizeof(float) * (2 * 3 * KC * BV3 + 2 * 2 * KC * BN) +
                     (sizeof(float) + sizeof(int32_t)) * 4 * 32 * (longl ? KK_MAX : KK_SHORT);
  const void* kfn = longl ? (const void*)k_match_f32_3m<KK_MAX> : (const void*)k_match_f32_3m<KK_SHORT>;
  static std::once_flag attr_once[2];
  hipError_t attr_rc = hipSuccess;
  std::call_once(attr_once[longl ? 1 : 0], [&]() {
    attr_rc = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  });
  MRF_HIP(attr_rc);
  {
    ProfScope prof(pctx, "k_match_f32", st);
    if (longl)
      hipLaunchKernelGGL(k_match_f32_3m<KK_MAX>, dim3(grid_wg), dim3(256), lds, st, a);
    else
      hipLaunchKernelGGL(k_match_f32_3m<KK_SHORT>, dim3(grid_wg), dim3(256), lds, st, a);
  }
  MRF_HIP(hipGetLastError());

  MergeArgs m;
  m.part_s = ps;
  m.part_i = pi;
  m.n_lists = p.n_chunks * 2;
  m.n_vox = n_vox;
  m.n_vox_pad = p.n_vox_pad;
  m.kk = p.kk;
  m.top_k = top_k;
  m.entry_base = d->entry_base;
  m.best_s = bs;
  m.best_i = bi;
  m.idx = out.idx;
  m.cc = out.cc;
  m.margin = out.margin;
  m.topk_idx = topk_idx;
  m.topk_cc = topk_cc;
  int rc = launch_merge(pctx, m, st);
  if (rc) return rc;
  if (out.pd_re || out.pd_im) {
    hipLaunchKernelGGL(k_pd_f32, dim3(n_vox), dim3(64), 0, st, (const float2*)vox, ld_vox, n_vox,
                       d->n_tr, (const float*)d->re, (const float*)d->im, d->ld, bi, p.kk,
                       d->norm, out.pd_re, out.pd_im);
    MRF_HIP(hipGetLastError());
  }
  return MRF_OK;
}

int match_f32_scratch(mrf_context* ctx, const mrf_dict_view* d, const void* vox, int32_t n_vox,
                      int64_t ld_vox, int32_t top_k, mrf_result_view out, int64_t* topk_idx,
                      float* topk_cc, void* scratch, size_t scratch_bytes, hipStream_t st) {
  MRF_CHECK_ARG(ctx != nullptr, "context is NULL");
  int rc = check_view(d);
  if (rc) return rc;
  MRF_CHECK_ARG(d->dtype == MRF_F32,
                "the allocation-free brute force takes FP32 dictionaries only (BF16 "
                "re-scoring builds step tables on first use)");
  MRF_CHECK_ARG(n_vox >= 0, "n_vox must be >= 0");
  MRF_CHECK_ARG(top_k >= 1 && top_k <= KK_MAX, "top_k must be in [1, %d]", KK_MAX);
  if (n_vox == 0) return MRF_OK;
  MRF_CHECK_ARG(vox != nullptr, "vox is NULL");
  MRF_CHECK_ARG(ld_vox >= d->n_tr, "ld_vox (%lld) must be >= n_tr (%d)", (long long)ld_vox, d->n_tr);
  MRF_CHECK_ARG(out.idx != nullptr, "out.idx is NULL");
  MRF_CHECK_ARG(scratch != nullptr, "no static scratch on device %d", ctx->device);
  const size_t need = match_f32_workspace_bytes(d, n_vox, top_k, ctx->n_cu);
  MRF_CHECK_ARG(need <= scratch_bytes,
                "%d voxels x %d readouts (top_k %d) need %zu bytes of scratch, the static "
                "scratch holds %zu: match fewer voxels per call", n_vox, d->n_tr, top_k, need,
                scratch_bytes);
  return match_f32_run(ctx, d, vox, n_vox, ld_vox, top_k, out, topk_idx, topk_cc, scratch,
                       scratch_bytes, st, false);
}

}  // namespace mrf

extern "C" int mrf_match_bruteforce(mrf_context* ctx, const mrf_dict_view* d, const void* vox,
                                    int32_t n_vox, int64_t ld_vox, int32_t top_k,
                                    const mrf_sequence* seq, const mrf_grid* grid,
                                    mrf_result_view out, int64_t* topk_idx, float* topk_cc,
                                    void* workspace, size_t ws_bytes, void* stream) {
  MRF_CHECK_ARG(ctx != nullptr, "context is NULL");
  int rc = check_view(d);
  if (rc) return rc;
  MRF_CHECK_ARG(n_vox >= 0, "n_vox must be >= 0");
  MRF_CHECK_ARG(top_k >= 1 && top_k <= KK_MAX, "top_k must be in [1, %d]", KK_MAX);
  if (n_vox == 0) return MRF_OK;
  MRF_CHECK_ARG(vox != nullptr, "vox is NULL");
  MRF_CHECK_ARG(ld_vox >= d->n_tr, "ld_vox (%lld) must be >= n_tr (%d)", (long long)ld_vox, d->n_tr);
  MRF_CHECK_ARG(out.idx != nullptr, "out.idx is NULL");
  MRF_CHECK_ARG(workspace != nullptr, "workspace is NULL");
  hipStream_t st = (hipStream_t)stream;
  if (d->dtype == MRF_BF16) {
    return match_bf16(ctx, d, vox, n_vox, ld_vox, top_k, seq, grid, out, topk_idx, topk_cc,
                      workspace, ws_bytes, st);
  }
  return match_f32_run(ctx, d, vox, n_vox, ld_vox, top_k, out, topk_idx, topk_cc, workspace,
                       ws_bytes, st, true);
}
