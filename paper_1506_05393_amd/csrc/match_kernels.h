// Declarations shared by the FP32 and BF16 matching translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace mrf {
size_t bf16_workspace_bytes(const mrf_dict_view* d, int32_t n_vox, int32_t top_k, int n_cu);
int match_bf16(mrf_context* ctx, const mrf_dict_view* d, const void* vox, int32_t n_vox,
               int64_t ld_vox, int32_t top_k, const mrf_sequence* seq, const mrf_grid* grid,
               mrf_result_view out, int64_t* topk_idx, float* topk_cc, void* workspace,
               size_t ws_bytes, hipStream_t stream);

// Merge of per-chunk candidate lists [n_lists][n_vox_pad][kk] into the final
// per-voxel list (best_s/best_i [n_vox][kk]) and the FP32 outputs.
struct MergeArgs {
  const float* part_s;
  const int32_t* part_i;
  int32_t n_lists, n_vox, n_vox_pad, kk, top_k;
  int64_t entry_base;
  float* best_s;
  int32_t* best_i;
  int64_t* idx;
  float* cc;
  float* margin;
  int64_t* topk_idx;
  float* topk_cc;
};
int launch_merge(mrf_context* ctx, const MergeArgs& m, hipStream_t st);
}  // namespace mrf

namespace mrf {
// FP32 brute force on a caller-provided buffer (the pieces of
// mrf_match_bruteforce's FP32 path). match_f32_run expects checked
// arguments; match_f32_scratch checks them itself (FP32 views only) and
// refuses a buffer smaller than the plan needs.
size_t match_f32_workspace_bytes(const mrf_dict_view* d, int32_t n_vox, int32_t top_k, int n_cu);
int match_f32_run(mrf_context* ctx, const mrf_dict_view* d, const void* vox, int32_t n_vox,
                  int64_t ld_vox, int32_t top_k, mrf_result_view out, int64_t* topk_idx,
                  float* topk_cc, void* workspace, size_t ws_bytes, hipStream_t st,
                  bool profile);
int match_f32_scratch(mrf_context* ctx, const mrf_dict_view* d, const void* vox, int32_t n_vox,
                      int64_t ld_vox, int32_t top_k, mrf_result_view out, int64_t* topk_idx,
                      float* topk_cc, void* scratch, size_t scratch_bytes, hipStream_t st);
}  // namespace mrf
