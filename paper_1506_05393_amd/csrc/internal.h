// Internal definitions shared by the libmrf translation units (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/libmrf.h"
#include "table_cache.h"

namespace mrf {

void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

#define MRF_CHECK_ARG(cond, ...)      \
  do {                                \
    if (!(cond)) {                    \
      ::mrf::set_error(__VA_ARGS__);  \
      return MRF_ERR_INVALID;         \
    }                                 \
  } while (0)

#define MRF_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::mrf::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),  \
                       __FILE__, __LINE__);                                    \
      return MRF_ERR_DEVICE;                                                   \
    }                                                                          \
  } while (0)

// Device tables of one (sequence, grid, n_tr): per-readout factors, FP64
// computed and rounded to FP32 once (layouts step-major, see tables.hip).
struct Tables {
  uint64_t key = 0;
  int32_t n_tr = 0, n1 = 0, n2 = 0, n3 = 0, n4 = 0;  // n4 >= 1
  int32_t inversion = 1;
  // every RF phase of the first n_tr readouts is a multiple of 180 degrees, so
  // each pulse is a rotation about the x axis (pulse_matrix then gives exact
  // zeros off that axis and R00 = 1)
  int32_t x_axis_pulses = 0;
  // dictionary entries smoothed over 3 or 5 readouts (0: none), from the sequence
  int32_t smooth = 0;
  const float2* demod = nullptr;  // [n_tr] (cos, sin) of the RF phases (the sequence's)
  float2* t1 = nullptr;   // [n_tr][n1]  (1-E1 over TE, 1-E1 over TR-TE)
  float* t1ti = nullptr;  // [n1]        (1-E1 over TI)
  float2* t2 = nullptr;   // [n_tr][n2]  (1-E2 over TE, 1-E2 over TR-TE)
  float4* df = nullptr;   // [n_tr][n3]  (cos-1, sin over TE, cos-1, sin over TR-TE)
  float* rf = nullptr;    // [n4][n_tr][9] pulse rotation matrix
  // entry-major copies (one row per axis value) for kernels whose lanes walk
  // different entries through the readouts (ZOOM, re-scoring)
  float2* t1T = nullptr;  // [n1][n_tr]
  float2* t2T = nullptr;  // [n2][n_tr]
  float4* dfT = nullptr;  // [n3][n_tr]
  // TE = TR - TE at every readout (TE = TR / 2, as in bSSFP): both halves of
  // each TR share their factors, kept once in compact entry-major rows of tq
  // readouts (n_tr rounded up to a multiple of 4, so a 16-byte load covers
  // four readouts of h1 / h2 and two of hd); NULL otherwise
  int32_t symmetric = 0;
  int32_t tq = 0;
  float* h1 = nullptr;   // [n1][tq]  1-E1 over TE
  float* h2 = nullptr;   // [n2][tq]  1-E2 over TE
  float2* hd = nullptr;  // [n3][tq]  (cos-1, sin) over TE
  // x-axis pulses (x_axis_pulses): a rotation about x, whose only entries
  // that are not exact 0 or 1 are R11 = R22 and R12 = -R21 (pulse_matrix
  // rounds them so); (R11, R12) per readout, NULL otherwise
  float2* xr = nullptr;  // [n4][tq]
  void* block = nullptr;  // one allocation holding all of the above
};
// A held reference to built tables (see get_tables).
using TablesRef = std::shared_ptr<const Tables>;

}  // namespace mrf

struct mrf_context {
  int device = 0;
  int n_cu = 0;
  int warp = 64;
  // kernel timing (mrf_profile_*)
  bool prof_on = false;
  std::mutex prof_mu;
  struct ProfRec {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof;
};

namespace mrf {
// Brackets one kernel launch with events on `stream` when profiling is on.
class ProfScope {
 public:
  ProfScope(mrf_context* ctx, const char* name, hipStream_t stream);
  ~ProfScope();

 private:
  mrf_context* ctx_;
  const char* name_;
  hipStream_t stream_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};
}  // namespace mrf

struct mrf_sequence {
  mrf_context* ctx = nullptr;
  int32_t n = 0;
  std::vector<double> fa, ph, tr, te;
  int32_t inversion = 1;
  double ti = 0.0;
  int32_t smooth = 0;     // temporal smoothing of dictionary entries: 0, 3 or 5 readouts
  double omega_hz = 0.0;  // 1000 / min TR: CC pseudo-period in df (Property II)
  double* dev = nullptr;  // device FP64 [4][n]: TE, TR-TE, flip angle, RF phase
  float2* demod = nullptr;  // device [n] (cos, sin) of the RF phase (inside dev's allocation)
  // the tables of the last four (grid contents, n_tr) keys
  mrf::LruCache<std::pair<uint64_t, int32_t>, mrf::Tables> cache{4};
};

namespace mrf {
// Validate a grid (axis lengths, strictly increasing, finite where required).
int check_grid(const mrf_grid* g);
// Tables of (seq, grid, n_tr), built (on `stream`) on first use and cached.
// *out holds a reference: keep it while the tables are in use (an entry
// evicted meanwhile by another thread's lookups is freed when released).
int get_tables(mrf_sequence* seq, const mrf_grid* g, int32_t n_tr, hipStream_t stream,
               TablesRef* out);
int64_t grid_size_checked(const mrf_grid* g);
// Looks up the device address of this device's static scratch (scratch.hip);
// called once per device with the device current.
int scratch_setup(int device);
}  // namespace mrf
