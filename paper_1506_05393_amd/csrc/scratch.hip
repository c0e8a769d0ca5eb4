// Allocation-free FP32 brute force: the workspace of mrf_match_bruteforce's
// FP32 path (packed voxel operand, per-chunk candidate lists, merged lists)
// lives in a static device array instead of a caller or library allocation.
//
// The array's name is a host-side stand-in in host code: the device address
// of each GPU's copy is looked up once per device with hipGetSymbolAddress
// (at context creation, with the device current) and only that address is
// handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"
#include "match_kernels.h"

namespace mrf {
// 64 MiB: a 64 x 64 slice (4096 voxels) at N = 1000 with top_k <= 8 fits
// (50.7 MB at top_k = 1).
constexpr size_t kScratchBytes = (size_t)64 << 20;
}  // namespace mrf

// one copy per GPU, held until the process ends
static __device__ __align__(256) unsigned char scratch[mrf::kScratchBytes];

namespace mrf {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// Looks up this device's copy of the array (the device must be current).
int scratch_setup(int device) {
  MRF_CHECK_ARG(device >= 0 && device < kMaxDevices, "device %d beyond the scratch table",
                device);
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return MRF_OK;
  void* p = nullptr;
  MRF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  MRF_CHECK_ARG(p != nullptr, "no device address for the static scratch on device %d", device);
  g_ptr[device] = p;
  return MRF_OK;
}

static void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace mrf

extern "C" size_t mrf_static_scratch_bytes(void) { return mrf::kScratchBytes; }

extern "C" int mrf_match_bruteforce_noalloc(mrf_context* ctx, const mrf_dict_view* dict,
                                            const void* vox, int32_t n_vox, int64_t ld_vox,
                                            int32_t top_k, mrf_result_view out,
                                            int64_t* topk_idx, float* topk_cc, void* stream) {
  MRF_CHECK_ARG(ctx != nullptr, "context is NULL");
  return mrf::match_f32_scratch(ctx, dict, vox, n_vox, ld_vox, top_k, out, topk_idx, topk_cc,
                                mrf::scratch_ptr(ctx->device), mrf::kScratchBytes,
                                (hipStream_t)stream);
}
