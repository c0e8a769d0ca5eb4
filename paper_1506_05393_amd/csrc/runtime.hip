// libmrf runtime: errors, context, sequences, grids and the per-(sequence,
// grid) step tables (Appendix Eq. A2 factors, built by the K0 kernel).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

#include "bloch.h"
#include "internal.h"

namespace mrf {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

int64_t grid_size_checked(const mrf_grid* g) {
  return (int64_t)g->t1_ms.n * g->t2_ms.n * g->df_hz.n * (g->b1.n > 0 ? g->b1.n : 1);
}

static int check_axis(const mrf_axis& a, const char* name, bool allow_empty, bool positive) {
  if (a.n < 0 || (!allow_empty && a.n < 1)) {
    set_error("grid axis %s has invalid length %d", name, a.n);
    return MRF_ERR_INVALID;
  }
  if (a.n > 0 && !a.v) {
    set_error("grid axis %s has a NULL value list", name);
    return MRF_ERR_INVALID;
  }
  for (int32_t i = 0; i < a.n; ++i) {
    double v = a.v[i];
    if (std::isnan(v) || (positive && !(v > 0.0)) || (!positive && !std::isfinite(v))) {
      set_error("grid axis %s value %d (%g) is out of range", name, i, v);
      return MRF_ERR_INVALID;
    }
    if (i > 0 && !(v > a.v[i - 1])) {
      set_error("grid axis %s must be strictly increasing (index %d)", name, i);
      return MRF_ERR_INVALID;
    }
  }
  return MRF_OK;
}

int check_grid(const mrf_grid* g) {
  if (!g) {
    set_error("grid is NULL");
    return MRF_ERR_INVALID;
  }
  int rc;
  if ((rc = check_axis(g->t1_ms, "t1", false, true))) return rc;
  if ((rc = check_axis(g->t2_ms, "t2", false, true))) return rc;
  if ((rc = check_axis(g->df_hz, "df", false, false))) return rc;
  if ((rc = check_axis(g->b1, "b1", true, false))) return rc;
  // (ZOOM's memo keys hold an entry index in 39 bits)
  if (grid_size_checked(g) > ((int64_t)1 << 39)) {
    set_error("grid too large (more than 2^39 entries)");
    return MRF_ERR_INVALID;
  }
  return MRF_OK;
}

// ---------------------------------------------------------------------------
// K0: step tables. One thread per table element; every factor is evaluated
// in FP64 and rounded to FP32 once.
//   t1[j][i] = (1 - exp(-TE_j/T1_i), 1 - exp(-(TR_j-TE_j)/T1_i))
//   t2[j][i] likewise for T2
//   df[j][i] = (cos a - 1, sin a, cos b - 1, sin b), a = 2 pi df_i TE_j/1000,
//              b = 2 pi df_i (TR_j-TE_j)/1000
//   rf[b][j] = Rz(phi_j) Rx(-B1_b alpha_j) Rz(-phi_j), row-major 3x3
// ---------------------------------------------------------------------------
struct K0Args {
  const double* ta;    // [n_tr] TE
  const double* tb;    // [n_tr] TR - TE
  const double* fa;    // [n_tr] deg
  const double* ph;    // [n_tr] deg
  const double* ax1;   // [n1]
  const double* ax2;   // [n2]
  const double* ax3;   // [n3]
  const double* ax4;   // [n4] (B1 values; 1.0 when the axis is empty)
  double ti;
  int32_t n_tr, n1, n2, n3, n4;
  float2* t1;
  float* t1ti;
  float2* t2;
  float4* df;
  float* rf;
  float2* t1T;
  float2* t2T;
  float4* dfT;
  int32_t tq;  // compact row length (when any of h1, h2, hd, xr is set)
  float* h1;
  float* h2;
  float2* hd;
  float2* xr;
};

__global__ void k_step_tables(K0Args a) {
  const int64_t n_t1 = (int64_t)a.n_tr * a.n1;
  const int64_t n_t2 = (int64_t)a.n_tr * a.n2;
  const int64_t n_df = (int64_t)a.n_tr * a.n3;
  const int64_t n_rf = (int64_t)a.n_tr * a.n4;
  const int64_t total = n_t1 + a.n1 + n_t2 + n_df + n_rf;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t u = t;
    if (u < n_t1) {
      int j = (int)(u / a.n1), i = (int)(u % a.n1);
      const float2 f = make_float2((float)one_minus_exp(a.ta[j], a.ax1[i]),
                                   (float)one_minus_exp(a.tb[j], a.ax1[i]));
      a.t1[u] = f;
      a.t1T[(int64_t)i * a.n_tr + j] = f;
      if (a.h1) a.h1[(int64_t)i * a.tq + j] = f.x;
      continue;
    }
    u -= n_t1;
    if (u < a.n1) {
      a.t1ti[u] = (float)one_minus_exp(a.ti, a.ax1[u]);
      continue;
    }
    u -= a.n1;
    if (u < n_t2) {
      int j = (int)(u / a.n2), i = (int)(u % a.n2);
      const float2 f = make_float2((float)one_minus_exp(a.ta[j], a.ax2[i]),
                                   (float)one_minus_exp(a.tb[j], a.ax2[i]));
      a.t2[u] = f;
      a.t2T[(int64_t)i * a.n_tr + j] = f;
      if (a.h2) a.h2[(int64_t)i * a.tq + j] = f.x;
      continue;
    }
    u -= n_t2;
    if (u < n_df) {
      int j = (int)(u / a.n3), i = (int)(u % a.n3);
      float4 f;
      precession(a.ta[j], a.ax3[i], &f.x, &f.y);
      precession(a.tb[j], a.ax3[i], &f.z, &f.w);
      a.df[u] = f;
      a.dfT[(int64_t)i * a.n_tr + j] = f;
      if (a.hd) a.hd[(int64_t)i * a.tq + j] = make_float2(f.x, f.y);
      continue;
    }
    u -= n_df;
    {
      int b = (int)(u / a.n_tr), j = (int)(u % a.n_tr);
      float* R = a.rf + ((int64_t)b * a.n_tr + j) * 9;
      pulse_matrix(a.fa[j], a.ph[j], a.ax4[b], R);
      if (a.xr) a.xr[(int64_t)b * a.tq + j] = make_float2(R[4], R[5]);
    }
  }
}

static uint64_t fnv(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

static uint64_t grid_key(const mrf_grid* g, int32_t n_tr) {
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, &n_tr, sizeof n_tr);
  const mrf_axis* ax[4] = {&g->t1_ms, &g->t2_ms, &g->df_hz, &g->b1};
  for (auto* a : ax) {
    h = fnv(h, &a->n, sizeof a->n);
    if (a->n > 0) h = fnv(h, a->v, sizeof(double) * (size_t)a->n);
  }
  return h;
}

// Owner of one built table block: frees the device memory with the last
// reference.
static std::shared_ptr<Tables> own_tables(const Tables& t) {
  return std::shared_ptr<Tables>(new Tables(t), [](Tables* p) {
    if (p->block) (void)hipFree(p->block);
    delete p;
  });
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Builds the tables of (seq, g, n_tr) on `stream` and waits for them.
static int build_tables(mrf_sequence* seq, const mrf_grid* g, int32_t n_tr, uint64_t key,
                        hipStream_t stream, std::shared_ptr<Tables>* out) {
  Tables t;
  t.key = key;
  t.n_tr = n_tr;
  t.n1 = g->t1_ms.n;
  t.n2 = g->t2_ms.n;
  t.n3 = g->df_hz.n;
  t.n4 = g->b1.n > 0 ? g->b1.n : 1;
  t.inversion = seq->inversion;
  t.smooth = seq->smooth;
  t.demod = seq->demod;
  t.x_axis_pulses = 1;
  for (int32_t j = 0; j < n_tr; ++j)
    if (std::fmod(seq->ph[j], 180.0) != 0.0) t.x_axis_pulses = 0;
  const size_t nt = (size_t)(n_tr > 0 ? n_tr : 1);
  size_t o_t1 = 0;
  size_t o_ti = align256(o_t1 + sizeof(float2) * nt * t.n1);
  size_t o_t2 = align256(o_ti + sizeof(float) * t.n1);
  size_t o_df = align256(o_t2 + sizeof(float2) * nt * t.n2);
  size_t o_rf = align256(o_df + sizeof(float4) * nt * t.n3);
  size_t o_t1T = align256(o_rf + sizeof(float) * 9 * nt * t.n4);
  size_t o_t2T = align256(o_t1T + sizeof(float2) * nt * t.n1);
  size_t o_dfT = align256(o_t2T + sizeof(float2) * nt * t.n2);
  // compact tables: symmetric TRs (TE exactly equal to TR - TE in FP64, so
  // both halves' FP32 factors are the same numbers) and x-axis pulses
  t.symmetric = n_tr > 0;
  for (int32_t j = 0; j < n_tr; ++j)
    if (seq->te[j] != seq->tr[j] - seq->te[j]) t.symmetric = 0;
  t.tq = (int32_t)((nt + 3) / 4 * 4);
  const size_t tq = (size_t)t.tq;
  size_t o_h1 = align256(o_dfT + sizeof(float4) * nt * t.n3);
  size_t o_h2 = align256(o_h1 + (t.symmetric ? sizeof(float) * tq * t.n1 : 0));
  size_t o_hd = align256(o_h2 + (t.symmetric ? sizeof(float) * tq * t.n2 : 0));
  size_t o_xr = align256(o_hd + (t.symmetric ? sizeof(float2) * tq * t.n3 : 0));
  size_t o_in = align256(o_xr + (t.x_axis_pulses ? sizeof(float2) * tq * t.n4 : 0));
  // staged FP64 inputs: ta, tb, fa, ph, ax1..ax4
  const size_t n_in = 4 * nt + t.n1 + t.n2 + t.n3 + t.n4;
  size_t total = o_in + sizeof(double) * n_in;
  if (hipMalloc(&t.block, total) != hipSuccess) {
    set_error("out of device memory for step tables (%zu bytes)", total);
    return MRF_ERR_OOM;
  }
  char* base = (char*)t.block;
  t.t1 = (float2*)(base + o_t1);
  t.t1ti = (float*)(base + o_ti);
  t.t2 = (float2*)(base + o_t2);
  t.df = (float4*)(base + o_df);
  t.rf = (float*)(base + o_rf);
  t.t1T = (float2*)(base + o_t1T);
  t.t2T = (float2*)(base + o_t2T);
  t.dfT = (float4*)(base + o_dfT);
  if (t.symmetric) {
    t.h1 = (float*)(base + o_h1);
    t.h2 = (float*)(base + o_h2);
    t.hd = (float2*)(base + o_hd);
  }
  if (t.x_axis_pulses) t.xr = (float2*)(base + o_xr);
  std::vector<double> in(n_in);
  double* p = in.data();
  for (int32_t j = 0; j < n_tr; ++j) {
    p[j] = seq->te[j];
    p[nt + j] = seq->tr[j] - seq->te[j];
    p[2 * nt + j] = seq->fa[j];
    p[3 * nt + j] = seq->ph[j];
  }
  double* q = p + 4 * nt;
  for (int32_t i = 0; i < t.n1; ++i) *q++ = g->t1_ms.v[i];
  for (int32_t i = 0; i < t.n2; ++i) *q++ = g->t2_ms.v[i];
  for (int32_t i = 0; i < t.n3; ++i) *q++ = g->df_hz.v[i];
  for (int32_t i = 0; i < t.n4; ++i) *q++ = g->b1.n > 0 ? g->b1.v[i] : 1.0;
  double* din = (double*)(base + o_in);
  hipError_t e = hipMemcpyAsync(din, in.data(), sizeof(double) * n_in, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) {
    K0Args a;
    a.ta = din;
    a.tb = din + nt;
    a.fa = din + 2 * nt;
    a.ph = din + 3 * nt;
    a.ax1 = din + 4 * nt;
    a.ax2 = a.ax1 + t.n1;
    a.ax3 = a.ax2 + t.n2;
    a.ax4 = a.ax3 + t.n3;
    a.ti = seq->ti;
    a.n_tr = n_tr;
    a.n1 = t.n1;
    a.n2 = t.n2;
    a.n3 = t.n3;
    a.n4 = t.n4;
    a.t1 = t.t1;
    a.t1ti = t.t1ti;
    a.t2 = t.t2;
    a.df = t.df;
    a.rf = t.rf;
    a.t1T = t.t1T;
    a.t2T = t.t2T;
    a.dfT = t.dfT;
    a.tq = t.tq;
    a.h1 = t.h1;
    a.h2 = t.h2;
    a.hd = t.hd;
    a.xr = t.xr;
    int64_t work = (int64_t)nt * (t.n1 + t.n2 + t.n3 + t.n4) + t.n1;
    int blocks = (int)std::min<int64_t>((work + 255) / 256, 4096);
    hipLaunchKernelGGL(k_step_tables, dim3(blocks), dim3(256), 0, stream, a);
    e = hipGetLastError();
  }
  // the host staging buffer must outlive the copy
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  std::shared_ptr<Tables> owned = own_tables(t);
  if (e != hipSuccess) {
    set_error("building step tables failed: %s", hipGetErrorString(e));
    return MRF_ERR_DEVICE;  // `owned` frees the block
  }
  *out = std::move(owned);
  return MRF_OK;
}

int get_tables(mrf_sequence* seq, const mrf_grid* g, int32_t n_tr, hipStream_t stream,
               TablesRef* out) {
  const uint64_t key = grid_key(g, n_tr);
  return seq->cache.get(std::make_pair(key, n_tr),
                        [&](std::shared_ptr<Tables>* made) {
                          return build_tables(seq, g, n_tr, key, stream, made);
                        },
                        out);
}

ProfScope::ProfScope(mrf_context* ctx, const char* name, hipStream_t stream)
    : ctx_(ctx), name_(name), stream_(stream) {
  if (!ctx_ || !ctx_->prof_on) return;
  if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess) {
    a_ = b_ = nullptr;
    return;
  }
  (void)hipEventRecord(a_, stream_);
}

ProfScope::~ProfScope() {
  if (!a_ || !b_) return;
  (void)hipEventRecord(b_, stream_);
  std::lock_guard<std::mutex> lock(ctx_->prof_mu);
  ctx_->prof.push_back({name_, a_, b_});
}

}  // namespace mrf

using namespace mrf;

extern "C" {

int mrf_profile_enable(mrf_context* ctx, int32_t enable) {
  MRF_CHECK_ARG(ctx != nullptr, "context is NULL");
  ctx->prof_on = enable != 0;
  return MRF_OK;
}

int mrf_profile_read(mrf_context* ctx, const char* kernel, int32_t reset, double* total_ms,
                     int64_t* launches) {
  MRF_CHECK_ARG(ctx && kernel, "NULL argument");
  std::lock_guard<std::mutex> lock(ctx->prof_mu);
  double ms = 0.0;
  int64_t n = 0;
  for (auto& r : ctx->prof) {
    if (r.name != kernel) continue;
    MRF_HIP(hipEventSynchronize(r.b));
    float t = 0.0f;
    MRF_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    ++n;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (reset) {
    std::vector<mrf_context::ProfRec> keep;
    for (auto& r : ctx->prof) {
      if (r.name == kernel) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
      } else {
        keep.push_back(r);
      }
    }
    ctx->prof.swap(keep);
  }
  return MRF_OK;
}

const char* mrf_status_str(int s) {
  switch (s) {
    case MRF_OK: return "ok";
    case MRF_ERR_INVALID: return "invalid argument";
    case MRF_ERR_OOM: return "out of memory";
    case MRF_ERR_DEVICE: return "device error";
    case MRF_ERR_NOT_READY: return "not ready";
    case MRF_ERR_REJECTED: return "rejected";
    case MRF_ERR_UNSUPPORTED: return "unsupported";
    case MRF_ERR_CANCELLED: return "cancelled";
    default: return "unknown status";
  }
}

const char* mrf_last_error(void) { return g_err; }

const char* mrf_version(void) { return "libmrf 0.1 (gfx950)"; }

int mrf_context_create(int device, mrf_context** out) {
  MRF_CHECK_ARG(out != nullptr, "out is NULL");
  *out = nullptr;
  int n = 0;
  MRF_HIP(hipGetDeviceCount(&n));
  MRF_CHECK_ARG(device >= 0 && device < n, "device %d out of range (%d devices)", device, n);
  MRF_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  MRF_HIP(hipGetDeviceProperties(&prop, device));
  int rc = scratch_setup(device);
  if (rc) return rc;
  mrf_context* c = new (std::nothrow) mrf_context();
  if (!c) {
    set_error("out of host memory");
    return MRF_ERR_OOM;
  }
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  c->warp = prop.warpSize;
  *out = c;
  return MRF_OK;
}

int mrf_context_destroy(mrf_context* ctx) {
  if (!ctx) return MRF_OK;
  for (auto& r : ctx->prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  delete ctx;
  return MRF_OK;
}

int mrf_sequence_create(mrf_context* ctx, const mrf_sequence_desc* d, mrf_sequence** out) {
  MRF_CHECK_ARG(ctx && d && out, "NULL argument");
  *out = nullptr;
  MRF_CHECK_ARG(d->n >= 1, "sequence length %d must be >= 1", d->n);
  MRF_CHECK_ARG(d->fa_deg && d->phase_deg && d->tr_ms && d->te_ms, "sequence arrays must not be NULL");
  MRF_CHECK_ARG(d->ti_ms >= 0.0 && std::isfinite(d->ti_ms), "ti_ms must be finite and >= 0");
  MRF_CHECK_ARG(d->smooth == 0 || d->smooth == 1 || d->smooth == 3 || d->smooth == 5,
                "smooth must be 0, 1, 3 or 5 (got %d)", d->smooth);
  double trmin = INFINITY;
  for (int32_t j = 0; j < d->n; ++j) {
    MRF_CHECK_ARG(std::isfinite(d->fa_deg[j]) && std::isfinite(d->phase_deg[j]),
                  "readout %d: flip angle and phase must be finite", j);
    MRF_CHECK_ARG(d->te_ms[j] > 0.0 && d->te_ms[j] < d->tr_ms[j] && std::isfinite(d->tr_ms[j]),
                  "readout %d: need 0 < te (%g) < tr (%g)", j, d->te_ms[j], d->tr_ms[j]);
    trmin = std::min(trmin, d->tr_ms[j]);
  }
  mrf_sequence* s = new (std::nothrow) mrf_sequence();
  if (!s) {
    set_error("out of host memory");
    return MRF_ERR_OOM;
  }
  s->ctx = ctx;
  s->n = d->n;
  s->fa.assign(d->fa_deg, d->fa_deg + d->n);
  s->ph.assign(d->phase_deg, d->phase_deg + d->n);
  s->tr.assign(d->tr_ms, d->tr_ms + d->n);
  s->te.assign(d->te_ms, d->te_ms + d->n);
  s->inversion = d->inversion ? 1 : 0;
  s->ti = d->ti_ms;
  s->smooth = d->smooth > 1 ? d->smooth : 0;
  s->omega_hz = 1000.0 / trmin;
  {
    std::vector<double> h(4 * (size_t)d->n);
    for (int32_t j = 0; j < d->n; ++j) {
      h[j] = d->te_ms[j];
      h[d->n + j] = d->tr_ms[j] - d->te_ms[j];
      h[2 * (size_t)d->n + j] = d->fa_deg[j];
      h[3 * (size_t)d->n + j] = d->phase_deg[j];
    }
    // (cos, sin) of each RF phase in FP32, exact for multiples of 90 degrees:
    // the frame that temporal smoothing demodulates into
    std::vector<float2> cs(d->n);
    for (int32_t j = 0; j < d->n; ++j) {
      const double p = d->phase_deg[j];
      if (std::fmod(p, 90.0) == 0.0) {
        const int q = (int)(((long long)(p / 90.0) % 4 + 4) % 4);
        static const float qc[4] = {1.0f, 0.0f, -1.0f, 0.0f}, qs[4] = {0.0f, 1.0f, 0.0f, -1.0f};
        cs[j] = make_float2(qc[q], qs[q]);
      } else {
        const double a = p * (M_PI / 180.0);
        cs[j] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
    }
    const size_t bytes = sizeof(double) * h.size() + sizeof(float2) * cs.size();
    if (hipMalloc(&s->dev, bytes) != hipSuccess) {
      delete s;
      set_error("out of device memory for the sequence");
      return MRF_ERR_OOM;
    }
    s->demod = (float2*)(s->dev + h.size());
    hipError_t e = hipMemcpy(s->dev, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(s->demod, cs.data(), sizeof(float2) * cs.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(s->dev);
      delete s;
      set_error("uploading the sequence failed: %s", hipGetErrorString(e));
      return MRF_ERR_DEVICE;
    }
  }
  *out = s;
  return MRF_OK;
}

int mrf_sequence_destroy(mrf_sequence* s) {
  if (!s) return MRF_OK;
  s->cache.clear();  // tables still held by a running call are freed by that call
  if (s->dev) (void)hipFree(s->dev);
  delete s;
  return MRF_OK;
}

int64_t mrf_grid_size(const mrf_grid* g) {
  if (check_grid(g) != MRF_OK) return -1;
  return grid_size_checked(g);
}

}  // extern "C"
