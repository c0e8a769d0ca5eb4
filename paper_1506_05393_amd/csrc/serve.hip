// Serving: resident dictionaries, first-in first-out admission by HBM
// footprint, continuous batching of brute-force and MRF-ZOOM requests over
// several device streams. One scheduler thread makes every device call; the
// submit/poll/cancel entry points only touch host state under the mutex.
//
// Memory: slot dictionaries are allocated at registration; every batch takes
// one contiguous block (gathered voxels, result arrays, search workspace)
// from a device arena sized to the budget left beside the dictionaries.
// Admission reserves each request's own batch footprint; a batch of several
// requests never needs more than the sum of their reservations (checked when
// the batch is formed), so the arena's use never exceeds the reservations,
// which never exceed the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace mrf {
namespace {

constexpr size_t kAlign = 256;
constexpr int32_t kDefaultMaxBatchVox = 65536;
constexpr int32_t kTopKF32 = 2;   // the margin needs the runner-up
constexpr int32_t kTopKBF16 = 8;  // candidates re-scored in FP32

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Norms of a stored prefix of n_tr readouts, with the dictionary kernel's
// arithmetic: FP32 partial sums over groups of four readouts (from readout
// 0), each added into FP64. A prefix norm therefore equals bit for bit the
// norm that a dictionary simulated with n_tr readouts receives.
__global__ __launch_bounds__(256) void k_prefix_norm_f32(const float* __restrict__ re,
                                                         const float* __restrict__ im, int64_t ld,
                                                         int64_t n, int32_t n_tr,
                                                         double* __restrict__ norm) {
  const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  for (int32_t j0 = 0; j0 < n_tr; j0 += 4) {
    float part = 0.f;
    for (int32_t j = j0; j < j0 + 4 && j < n_tr; ++j) {
      const float x = re[(int64_t)j * ld + e], y = im[(int64_t)j * ld + e];
      part = fmaf(x, x, part);
      part = fmaf(y, y, part);
    }
    acc += (double)part;
  }
  norm[e] = sqrt(acc);
}

__global__ __launch_bounds__(256) void k_prefix_norm_bf16(const uint4* __restrict__ packed,
                                                          int64_t ld, int64_t n, int32_t n_blk,
                                                          double* __restrict__ norm) {
  const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (e >= n) return;
  double acc = 0.0;
  for (int32_t b = 0; b < n_blk; ++b) {
    const uint4 w = packed[(int64_t)b * ld + e];
    float part = 0.f;
    part = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w.x),
                                           __builtin_bit_cast(bf16x2_t, w.x), part, false);
    part = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w.y),
                                           __builtin_bit_cast(bf16x2_t, w.y), part, false);
    part = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w.z),
                                           __builtin_bit_cast(bf16x2_t, w.z), part, false);
    part = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, w.w),
                                           __builtin_bit_cast(bf16x2_t, w.w), part, false);
    acc += (double)part;
  }
  norm[e] = sqrt(acc);
}

// Per-voxel readout counts of a ZOOM batch: n values from one request.
__global__ __launch_bounds__(256) void k_fill_i32(int32_t* __restrict__ dst, int64_t n,
                                                  int32_t value) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i < n) dst[i] = value;
}

// First-fit allocator over [0, cap) with coalescing; offsets only (the
// device base is added by the caller, or absent on the fake device).
class Arena {
 public:
  void init(size_t cap) {
    cap_ = cap;
    free_.clear();
    if (cap) free_[0] = cap;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, o = it->first + bytes;
      free_.erase(it);
      if (rest) free_[o] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t peak() const { return peak_; }
  size_t capacity() const { return cap_; }

 private:
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Slot {
  const mrf_sequence* seq = nullptr;
  std::vector<double> axis[4];
  mrf_grid grid{};
  mrf_dtype dtype = MRF_F32;
  int32_t n_tr_max = 0;
  int64_t n_entries = 0, ld = 0;
  void* re = nullptr;  // F32 real plane or BF16 packed blocks
  void* im = nullptr;
  std::map<int32_t, double*> norms;  // readout count -> device norms
  mrf_zoom_schedule sched{};
  mrf_zoom_schedule local{};  // unit-step refinement of BF16 brute-force results
  size_t resident = 0;
};

struct Req {
  uint64_t ticket = 0;
  mrf_request r{};
  int32_t state = MRF_REQ_QUEUED;
  bool admitted = false;
  double t_submit = -1, t_start = -1, t_done = -1;
  size_t footprint = 0;
  std::string err;
};

// Byte layout of one batch's block.
struct Layout {
  int64_t ld_stage = 0;
  size_t stage = 0, idx = 0, cc = 0, margin = 0, pd_re = 0, pd_im = 0, n_sim = 0, vn = 0, ws = 0;
  size_t start = 0;  // refinement: the re-scored entries it starts from
  size_t ws_bytes = 0, total = 0;
};

struct Batch {
  int32_t slot = 0, mode = 0, n_tr = 0;
  int64_t n_vox = 0;
  std::vector<Req*> reqs;
  Layout L;
  size_t off = 0;
  double t_ready = 0;  // fake device: completion time
  bool failed = false;
  std::string err;
};

}  // namespace
}  // namespace mrf

using namespace mrf;

struct mrf_server {
  mrf_context* ctx = nullptr;
  mrf_server_config cfg{};
  bool fake = false;
  std::vector<std::unique_ptr<Slot>> slots;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  char* arena_base = nullptr;
  Arena arena;
  bool arena_ready = false;

  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> pending;   // submitted, not yet admitted (FIFO)
  std::deque<Req*> admitted;  // admitted, waiting for a stream (FIFO)
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::vector<std::unique_ptr<Batch>> running;  // one per stream
  uint64_t next_ticket = 1;
  size_t resident = 0, reserved = 0;
  int32_t inflight = 0;
  mrf_server_stats st{};
  bool stop = false;
  std::thread th;
  std::chrono::steady_clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace mrf {
namespace {

mrf_dict_view slot_view(const Slot& s, int32_t n_tr) {
  mrf_dict_view v{};
  v.dtype = s.dtype;
  v.n_tr = n_tr;
  v.n_entries = s.n_entries;
  v.ld = s.ld;
  v.re = s.re;
  v.im = s.dtype == MRF_F32 ? s.im : nullptr;
  auto it = s.norms.find(n_tr);
  v.norm = it == s.norms.end() ? nullptr : it->second;
  v.entry_base = 0;
  return v;
}

int batch_layout(mrf_server* srv, const Slot& s, int32_t mode, int32_t n_tr, int64_t n_vox,
                 Layout* L) {
  L->ld_stage = (n_tr + 63) / 64 * 64;
  size_t o = 0;
  L->stage = o;
  o += align_up((size_t)n_vox * (size_t)L->ld_stage * 8);
  L->idx = o;
  o += align_up((size_t)n_vox * 8);
  size_t* f4[] = {&L->cc, &L->margin, &L->pd_re, &L->pd_im, &L->n_sim, &L->vn};
  for (size_t* p : f4) {
    *p = o;
    o += align_up((size_t)n_vox * 4);
  }
  L->start = o;
  o += align_up((size_t)n_vox * 8);
  size_t ws = 0;
  if (srv->fake) {
    ws = 4096 + (size_t)n_vox * 64;
  } else if (mode == MRF_SERVE_BRUTE) {
    const mrf_dict_view v = slot_view(s, n_tr);
    int rc = mrf_match_workspace(srv->ctx, &v, (int32_t)n_vox,
                                 s.dtype == MRF_BF16 ? kTopKBF16 : kTopKF32, &ws);
    if (rc) return rc;
    if (srv->cfg.refine_bf16 && s.dtype == MRF_BF16) {
      size_t wz = 0;
      rc = mrf_zoom_workspace(srv->ctx, &s.grid, (int32_t)n_vox, n_tr, &wz);
      if (rc) return rc;
      ws = std::max(ws, wz);
    }
  } else {
    const int rc = mrf_zoom_workspace(srv->ctx, &s.grid, (int32_t)n_vox, n_tr, &ws);
    if (rc) return rc;
  }
  L->ws = o;
  L->ws_bytes = ws;
  o += align_up(ws);
  L->total = o;
  return MRF_OK;
}

// Enqueue one batch on stream `si`. On failure the batch is marked failed;
// whatever was enqueued still completes before the block is reused.
void launch_batch(mrf_server* srv, Batch* b, int si) {
  if (srv->fake) {
    b->t_ready = srv->now_ms() + srv->cfg.fake_ns_per_byte * (double)b->L.total * 1e-6;
    for (Req* r : b->reqs)
      if (r->ticket == srv->cfg.fake_fail_ticket) {
        b->failed = true;
        b->err = "injected device failure (fake device)";
      }
    return;
  }
  const Slot& s = *srv->slots[b->slot];
  hipStream_t st = srv->streams[si];
  char* base = srv->arena_base + b->off;
  const Layout& L = b->L;
  char* stage = base + L.stage;
  auto fail = [&](const char* what, const char* msg) {
    b->failed = true;
    b->err = std::string(what) + ": " + msg;
  };
  // gather: each request's voxels, its own readout count, rows of the batch's
  // longest count; ZOOM batches also get every voxel's readout count
  int64_t v0 = 0;
  for (Req* r : b->reqs) {
    const hipError_t e = hipMemcpy2DAsync(stage + (size_t)v0 * L.ld_stage * 8, (size_t)L.ld_stage * 8,
                                          r->r.vox, (size_t)r->r.ld_vox * 8, (size_t)r->r.n_tr * 8,
                                          (size_t)r->r.n_vox, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
      fail("gathering voxels", hipGetErrorString(e));
      break;
    }
    if (b->mode == MRF_SERVE_ZOOM) {
      hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((r->r.n_vox + 255) / 256)), dim3(256), 0, st,
                         (int32_t*)(base + L.vn) + v0, (int64_t)r->r.n_vox, r->r.n_tr);
      const hipError_t e2 = hipGetLastError();
      if (e2 != hipSuccess) {
        fail("gathering voxels", hipGetErrorString(e2));
        break;
      }
    }
    v0 += r->r.n_vox;
  }
  mrf_result_view o{};
  o.idx = (int64_t*)(base + L.idx);
  o.cc = (float*)(base + L.cc);
  o.margin = (float*)(base + L.margin);
  o.pd_re = (float*)(base + L.pd_re);
  o.pd_im = (float*)(base + L.pd_im);
  const bool refined = b->mode == MRF_SERVE_BRUTE && srv->cfg.refine_bf16 && s.dtype == MRF_BF16;
  o.n_sim = b->mode == MRF_SERVE_ZOOM || refined ? (int32_t*)(base + L.n_sim) : nullptr;
  if (!b->failed) {
    int rc = MRF_OK;
    if (b->mode == MRF_SERVE_BRUTE) {
      // one GEMM per readout count (the requests are ordered by count), on
      // consecutive voxel ranges of the stage, sharing the workspace in turn
      int64_t c0 = 0;
      size_t i = 0;
      while (rc == MRF_OK && i < b->reqs.size()) {
        const int32_t n_tr = b->reqs[i]->r.n_tr;
        int64_t nv = 0;
        for (; i < b->reqs.size() && b->reqs[i]->r.n_tr == n_tr; ++i) nv += b->reqs[i]->r.n_vox;
        const mrf_dict_view v = slot_view(s, n_tr);
        mrf_result_view oc = o;
        oc.idx += c0;
        oc.cc += c0;
        oc.margin += c0;
        oc.pd_re += c0;
        oc.pd_im += c0;
        rc = mrf_match_bruteforce(srv->ctx, &v, stage + (size_t)c0 * L.ld_stage * 8, (int32_t)nv,
                                  L.ld_stage, s.dtype == MRF_BF16 ? kTopKBF16 : kTopKF32, s.seq,
                                  &s.grid, oc, nullptr, nullptr, base + L.ws, L.ws_bytes, st);
        if (rc == MRF_OK && srv->cfg.refine_bf16 && s.dtype == MRF_BF16) {
          // unit-step FP32 refinement from the re-scored entries
          int64_t* start = (int64_t*)(base + L.start) + c0;
          const hipError_t e = hipMemcpyAsync(start, oc.idx, (size_t)nv * 8,
                                              hipMemcpyDeviceToDevice, st);
          if (e != hipSuccess) {
            fail("refinement", hipGetErrorString(e));
            break;
          }
          oc.n_sim = (int32_t*)(base + L.n_sim) + c0;
          rc = mrf_zoom_search_from(srv->ctx, s.seq, &s.grid, &s.local,
                                    stage + (size_t)c0 * L.ld_stage * 8, (int32_t)nv, L.ld_stage,
                                    n_tr, start, oc, base + L.ws, L.ws_bytes, st);
        }
        c0 += nv;
      }
    } else {
      rc = mrf_zoom_search_ragged(srv->ctx, s.seq, &s.grid, &s.sched, stage, (int32_t)b->n_vox,
                                  L.ld_stage, b->n_tr, (const int32_t*)(base + L.vn), o,
                                  base + L.ws, L.ws_bytes, st);
    }
    if (rc) fail("search", mrf_last_error());
  }
  if (!b->failed) {
    v0 = 0;
    for (Req* r : b->reqs) {
      const size_t n = (size_t)r->r.n_vox;
      const mrf_result_view& d = r->r.out;
      struct {
        void* dst;
        const void* src;
        size_t bytes;
      } cp[] = {{d.idx, o.idx + v0, n * 8},     {d.cc, o.cc + v0, n * 4},
                {d.margin, o.margin + v0, n * 4}, {d.pd_re, o.pd_re + v0, n * 4},
                {d.pd_im, o.pd_im + v0, n * 4},
                {o.n_sim ? d.n_sim : nullptr, o.n_sim ? o.n_sim + v0 : nullptr, n * 4}};
      for (auto& c : cp) {
        if (!c.dst || !c.src) continue;
        const hipError_t e = hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) {
          fail("scattering results", hipGetErrorString(e));
          break;
        }
      }
      if (b->failed) break;
      v0 += r->r.n_vox;
    }
  }
  const hipError_t e = hipEventRecord(srv->events[si], st);
  if (e != hipSuccess) {
    fail("recording completion", hipGetErrorString(e));
    (void)hipStreamSynchronize(st);  // nothing may still use the block
  }
}

// 1 = finished (check b->failed), 0 = still running.
int query_batch(mrf_server* srv, Batch* b, int si) {
  if (srv->fake) return srv->now_ms() >= b->t_ready ? 1 : 0;
  const hipError_t e = hipEventQuery(srv->events[si]);
  if (e == hipErrorNotReady) return 0;
  if (e != hipSuccess && !b->failed) {
    b->failed = true;
    b->err = std::string("device error: ") + hipGetErrorString(e);
  }
  return 1;
}

void finish_batch(mrf_server* srv, Batch* b) {
  const double t = srv->now_ms();
  for (Req* r : b->reqs) {
    r->t_done = t;
    r->state = b->failed ? MRF_REQ_FAILED : MRF_REQ_DONE;
    if (b->failed) {
      r->err = b->err;
      srv->st.failed++;
    } else {
      srv->st.done++;
    }
    srv->reserved -= r->footprint;
    srv->inflight--;
  }
  srv->arena.release(b->off, b->L.total);
}

void admit(mrf_server* srv) {
  const size_t avail = srv->cfg.hbm_budget_bytes - srv->resident;
  while (!srv->pending.empty()) {
    Req* r = srv->pending.front();
    if (r->state == MRF_REQ_CANCELLED) {
      srv->pending.pop_front();
      continue;
    }
    if (srv->inflight >= srv->cfg.max_inflight || srv->reserved + r->footprint > avail) break;
    srv->pending.pop_front();
    r->admitted = true;
    srv->st.admitted++;
    srv->reserved += r->footprint;
    srv->inflight++;
    srv->st.peak_reserved_bytes = std::max(srv->st.peak_reserved_bytes, srv->reserved);
    srv->st.peak_inflight = std::max(srv->st.peak_inflight, srv->inflight);
    srv->admitted.push_back(r);
  }
}

// Form and launch batches on idle streams. Keys (slot, mode) are taken in
// the order of their oldest admitted request; a key's batch holds that
// request and every later admitted request of the same key, whatever its
// readout count, until max_batch_vox or the reservations stop it (then it is
// full); its buffers are laid out for its longest count. With a batching
// window a key's batch waits until its oldest request is that old, unless it
// is full or the server drains; *wake receives the earliest such deadline.
void launch_ready(mrf_server* srv, double* wake) {
  const int64_t max_vox = srv->cfg.max_batch_vox > 0 ? srv->cfg.max_batch_vox : kDefaultMaxBatchVox;
  const double window = srv->cfg.batch_window_ms;
  for (size_t si = 0; si < srv->running.size(); ++si) {
    while (!srv->admitted.empty() && srv->admitted.front()->state == MRF_REQ_CANCELLED)
      srv->admitted.pop_front();
    if (srv->running[si] || srv->admitted.empty()) continue;
    std::unique_ptr<Batch> b;
    Layout L;
    std::vector<std::pair<int32_t, int32_t>> seen;
    for (Req* head : srv->admitted) {
      if (head->state == MRF_REQ_CANCELLED) continue;
      const std::pair<int32_t, int32_t> key(head->r.slot, head->r.mode);
      if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
      seen.push_back(key);
      auto c = std::make_unique<Batch>();
      c->slot = key.first;
      c->mode = key.second;
      c->n_tr = 0;
      const Slot& s = *srv->slots[c->slot];
      size_t reserved_sum = 0;
      bool full = false;
      Layout Lc;
      for (Req* r : srv->admitted) {
        if (r->state == MRF_REQ_CANCELLED) continue;
        if (r->r.slot != c->slot || r->r.mode != c->mode) continue;
        if (!c->reqs.empty() && c->n_vox + r->r.n_vox > max_vox) {
          full = true;
          break;
        }
        const int32_t n_tr = std::max(c->n_tr, r->r.n_tr);
        Layout L2;
        if (batch_layout(srv, s, c->mode, n_tr, c->n_vox + r->r.n_vox, &L2)) {
          full = true;
          break;
        }
        if (!c->reqs.empty() && L2.total > reserved_sum + r->footprint) {
          full = true;
          break;
        }
        c->reqs.push_back(r);
        c->n_vox += r->r.n_vox;
        c->n_tr = n_tr;
        reserved_sum += r->footprint;
        Lc = L2;
      }
      if (c->reqs.empty()) continue;
      const double due = head->t_submit + window;
      if (window > 0.0 && !full && !srv->stop && srv->now_ms() < due) {
        *wake = std::min(*wake, due);
        continue;
      }
      b = std::move(c);
      L = Lc;
      break;
    }
    if (!b) return;  // nothing ready for any idle stream
    // brute force runs one GEMM per readout count: order the requests by count
    if (b->mode == MRF_SERVE_BRUTE)
      std::stable_sort(b->reqs.begin(), b->reqs.end(),
                       [](const Req* x, const Req* y) { return x->r.n_tr < y->r.n_tr; });
    if (!srv->arena.alloc(L.total, &b->off)) return;  // fragmented: wait for a completion
    b->L = L;
    for (Req* r : b->reqs) {
      srv->admitted.erase(std::find(srv->admitted.begin(), srv->admitted.end(), r));
      r->state = MRF_REQ_RUNNING;
      r->t_start = srv->now_ms();
    }
    srv->st.batches++;
    srv->st.max_batch_requests = std::max<int64_t>(srv->st.max_batch_requests, (int64_t)b->reqs.size());
    const int mi = b->mode == MRF_SERVE_ZOOM ? 1 : 0;
    srv->st.mode_batches[mi]++;
    srv->st.mode_requests[mi] += (int64_t)b->reqs.size();
    for (Req* r : b->reqs)
      if (r->r.n_tr != b->reqs.front()->r.n_tr) {
        srv->st.mixed_length_batches[mi]++;
        break;
      }
    launch_batch(srv, b.get(), (int)si);
    srv->running[si] = std::move(b);
  }
}

void scheduler(mrf_server* srv) {
  if (!srv->fake) (void)hipSetDevice(srv->ctx->device);
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    bool busy = false;
    for (size_t si = 0; si < srv->running.size(); ++si) {
      Batch* b = srv->running[si].get();
      if (!b) continue;
      if (query_batch(srv, b, (int)si)) {
        finish_batch(srv, b);
        srv->running[si].reset();
      } else {
        busy = true;
      }
    }
    admit(srv);
    double wake = INFINITY;  // a batching window's next deadline (ms)
    launch_ready(srv, &wake);
    for (auto& b : srv->running) busy = busy || (bool)b;
    if (srv->stop && !busy && srv->pending.empty() && srv->admitted.empty()) break;
    if (busy) {
      srv->cv.wait_for(lk, std::chrono::microseconds(100));
    } else if (wake < INFINITY) {
      const double d = std::max(wake - srv->now_ms(), 0.0);
      srv->cv.wait_for(lk, std::chrono::microseconds((int64_t)(d * 1000.0) + 50));
    } else {
      srv->cv.wait(lk);
    }
  }
}

int check_request(mrf_server* srv, const mrf_request* q) {
  MRF_CHECK_ARG(q, "request is NULL");
  MRF_CHECK_ARG(q->slot >= 0 && q->slot < (int32_t)srv->slots.size(), "unknown slot %d", q->slot);
  const Slot& s = *srv->slots[q->slot];
  MRF_CHECK_ARG(q->mode == MRF_SERVE_BRUTE || q->mode == MRF_SERVE_ZOOM, "unknown mode %d", q->mode);
  MRF_CHECK_ARG(q->n_tr >= 1 && q->n_tr <= s.n_tr_max, "n_tr %d must be in [1, %d]", q->n_tr,
                s.n_tr_max);
  if (q->mode == MRF_SERVE_BRUTE)
    MRF_CHECK_ARG(s.norms.count(q->n_tr), "n_tr %d is not a registered length of slot %d",
                  q->n_tr, q->slot);
  MRF_CHECK_ARG(q->n_vox >= 0, "n_vox must be >= 0");
  if (q->n_vox > 0) {
    MRF_CHECK_ARG(q->vox && q->out.idx, "vox and out.idx must not be NULL");
    MRF_CHECK_ARG(q->ld_vox >= q->n_tr, "ld_vox (%lld) must be >= n_tr (%d)",
                  (long long)q->ld_vox, q->n_tr);
  }
  return MRF_OK;
}

void free_slot(mrf_server* srv, Slot& s) {
  if (srv->fake) return;
  if (s.re) (void)hipFree(s.re);
  if (s.im) (void)hipFree(s.im);
  for (auto& kv : s.norms) (void)hipFree(kv.second);
  s.re = s.im = nullptr;
  s.norms.clear();
}

}  // namespace
}  // namespace mrf

extern "C" int mrf_server_create(mrf_context* ctx, const mrf_server_config* cfg, mrf_server** out) {
  MRF_CHECK_ARG(cfg && out, "cfg and out must not be NULL");
  MRF_CHECK_ARG(cfg->fake_device || ctx, "context must not be NULL");
  MRF_CHECK_ARG(cfg->max_inflight >= 1, "max_inflight must be >= 1");
  MRF_CHECK_ARG(cfg->n_streams >= 1 && cfg->n_streams <= 16, "n_streams must be in [1, 16]");
  MRF_CHECK_ARG(cfg->max_batch_vox >= 0, "max_batch_vox must be >= 0");
  MRF_CHECK_ARG(cfg->batch_window_ms >= 0.0, "batch_window_ms must be >= 0");
  MRF_CHECK_ARG(!cfg->fake_device || cfg->fake_ns_per_byte >= 0, "fake_ns_per_byte must be >= 0");
  auto srv = std::make_unique<mrf_server>();
  srv->ctx = ctx;
  srv->cfg = *cfg;
  srv->fake = cfg->fake_device != 0;
  srv->t0 = std::chrono::steady_clock::now();
  srv->st.budget_bytes = cfg->hbm_budget_bytes;
  srv->running.resize(cfg->n_streams);
  if (!srv->fake) {
    MRF_HIP(hipSetDevice(ctx->device));
    for (int i = 0; i < cfg->n_streams; ++i) {
      hipStream_t s;
      hipEvent_t e;
      MRF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      srv->streams.push_back(s);
      MRF_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      srv->events.push_back(e);
    }
  }
  srv->th = std::thread(scheduler, srv.get());
  *out = srv.release();
  return MRF_OK;
}

extern "C" int mrf_server_register(mrf_server* srv, const mrf_sequence* seq, const mrf_grid* grid,
                                   mrf_dtype dtype, const int32_t* n_tr, int32_t n_lengths,
                                   int32_t* slot) {
  MRF_CHECK_ARG(srv && slot && n_tr && n_lengths >= 1, "server, n_tr, slot must be given");
  MRF_CHECK_ARG(srv->fake || seq, "sequence must not be NULL");
  // a slot serves shorter readout counts from prefixes of one resident
  // dictionary; a smoothed entry's prefix is not the smoothed prefix
  MRF_CHECK_ARG(!seq || seq->smooth == 0,
                "sequences with temporal smoothing cannot be served (prefix dictionaries)");
  MRF_CHECK_ARG(dtype == MRF_F32 || dtype == MRF_BF16, "unknown dtype %d", (int)dtype);
  int rc = check_grid(grid);
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    MRF_CHECK_ARG(!srv->arena_ready, "slots must be registered before the first request");
  }
  auto s = std::make_unique<Slot>();
  int32_t n_max = 0;
  for (int32_t i = 0; i < n_lengths; ++i) {
    MRF_CHECK_ARG(n_tr[i] >= 1 && (!seq || n_tr[i] <= seq->n), "readout count %d out of range",
                  n_tr[i]);
    MRF_CHECK_ARG(dtype != MRF_BF16 || n_tr[i] % 4 == 0,
                  "BF16 slots need readout counts that are multiples of 4 (got %d)", n_tr[i]);
    n_max = std::max(n_max, n_tr[i]);
  }
  s->seq = seq;
  s->dtype = dtype;
  s->n_tr_max = n_max;
  const mrf_axis* ax[4] = {&grid->t1_ms, &grid->t2_ms, &grid->df_hz, &grid->b1};
  mrf_axis* dst[4] = {&s->grid.t1_ms, &s->grid.t2_ms, &s->grid.df_hz, &s->grid.b1};
  for (int i = 0; i < 4; ++i) {
    s->axis[i].assign(ax[i]->v, ax[i]->v + ax[i]->n);
    dst[i]->n = ax[i]->n;
    dst[i]->v = s->axis[i].data();
  }
  s->n_entries = grid_size_checked(&s->grid);
  s->ld = (s->n_entries + 255) / 256 * 256;
  std::vector<int32_t> lengths(n_tr, n_tr + n_lengths);
  std::sort(lengths.begin(), lengths.end());
  lengths.erase(std::unique(lengths.begin(), lengths.end()), lengths.end());
  const size_t dict_bytes = dtype == MRF_F32 ? 2 * (size_t)n_max * s->ld * 4
                                             : (size_t)(n_max / 4) * s->ld * 16;
  const size_t norm_bytes = (size_t)s->n_entries * 8;
  s->resident = dict_bytes + lengths.size() * norm_bytes;
  if (srv->resident + s->resident > srv->cfg.hbm_budget_bytes) {
    set_error("slot needs %zu resident bytes; %zu of the %zu byte budget are left", s->resident,
              srv->cfg.hbm_budget_bytes - srv->resident, srv->cfg.hbm_budget_bytes);
    return MRF_ERR_REJECTED;
  }
  if (!srv->fake) {
    MRF_HIP(hipSetDevice(srv->ctx->device));
    hipStream_t st = srv->streams[0];
    auto bail = [&](int code) {
      free_slot(srv, *s);
      return code;
    };
    if (dtype == MRF_F32) {
      if (hipMalloc(&s->re, dict_bytes / 2) != hipSuccess ||
          hipMalloc(&s->im, dict_bytes / 2) != hipSuccess) {
        set_error("out of device memory for a %zu byte dictionary", dict_bytes);
        return bail(MRF_ERR_OOM);
      }
    } else if (hipMalloc(&s->re, dict_bytes) != hipSuccess) {
      set_error("out of device memory for a %zu byte dictionary", dict_bytes);
      return bail(MRF_ERR_OOM);
    }
    for (int32_t n : lengths) {
      double* p = nullptr;
      if (hipMalloc(&p, norm_bytes) != hipSuccess) {
        set_error("out of device memory for norms");
        return bail(MRF_ERR_OOM);
      }
      s->norms[n] = p;
    }
    rc = mrf_simulate_dictionary(srv->ctx, seq, &s->grid, n_max, 0, s->n_entries, dtype, s->re,
                                 s->im, s->ld, s->norms[n_max], 0, st);
    if (rc) return bail(rc);
    const unsigned blocks = (unsigned)((s->n_entries + 255) / 256);
    for (int32_t n : lengths) {
      if (n == n_max) continue;
      if (dtype == MRF_F32)
        hipLaunchKernelGGL(k_prefix_norm_f32, dim3(blocks), dim3(256), 0, st, (const float*)s->re,
                           (const float*)s->im, s->ld, s->n_entries, n, s->norms[n]);
      else
        hipLaunchKernelGGL(k_prefix_norm_bf16, dim3(blocks), dim3(256), 0, st, (const uint4*)s->re,
                           s->ld, s->n_entries, n / 4, s->norms[n]);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      set_error("building the slot dictionary failed");
      return bail(MRF_ERR_DEVICE);
    }
    rc = mrf_zoom_schedule_paper(&s->grid, seq, &s->sched);
    if (rc) return bail(rc);
    rc = mrf_zoom_schedule_local(&s->grid, 8, &s->local);
    if (rc) return bail(rc);
  } else {
    for (int32_t n : lengths) s->norms[n] = nullptr;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->resident += s->resident;
  srv->st.resident_bytes = srv->resident;
  *slot = (int32_t)srv->slots.size();
  srv->slots.push_back(std::move(s));
  return MRF_OK;
}

extern "C" int mrf_serve_submit(mrf_server* srv, const mrf_request* req, uint64_t* ticket) {
  MRF_CHECK_ARG(srv && ticket, "server and ticket must not be NULL");
  int rc = check_request(srv, req);
  if (rc) return rc;
  auto r = std::make_unique<Req>();
  r->r = *req;
  if (req->n_vox > 0) {
    // reserved at the slot's longest readout count: a batch's buffers are laid
    // out for its longest count, so any mix of counts fits the reservations
    const Slot& s = *srv->slots[req->slot];
    Layout L;
    rc = batch_layout(srv, s, req->mode, s.n_tr_max, req->n_vox, &L);
    if (rc) return rc;
    r->footprint = L.total;
  }
  std::lock_guard<std::mutex> lk(srv->mu);
  if (!srv->arena_ready) {
    // the arena takes what the budget leaves beside the registered slots
    const size_t cap = srv->cfg.hbm_budget_bytes - srv->resident;
    if (!srv->fake && cap > 0) {
      if (hipSetDevice(srv->ctx->device) != hipSuccess ||
          hipMalloc((void**)&srv->arena_base, cap) != hipSuccess) {
        srv->arena_base = nullptr;
        set_error("out of device memory for the %zu byte request arena", cap);
        return MRF_ERR_OOM;
      }
    }
    srv->arena.init(cap);
    srv->arena_ready = true;
  }
  if (r->footprint > srv->cfg.hbm_budget_bytes - srv->resident) {
    srv->st.rejected++;
    set_error("request needs %zu bytes; the budget leaves %zu beside the resident dictionaries",
              r->footprint, srv->cfg.hbm_budget_bytes - srv->resident);
    return MRF_ERR_REJECTED;
  }
  r->ticket = srv->next_ticket++;
  r->t_submit = srv->now_ms();
  srv->st.submitted++;
  Req* p = r.get();
  if (req->n_vox == 0) {
    p->state = MRF_REQ_DONE;
    p->t_start = p->t_done = p->t_submit;
    srv->st.done++;
  } else {
    srv->pending.push_back(p);
  }
  *ticket = p->ticket;
  srv->reqs.emplace(p->ticket, std::move(r));
  srv->cv.notify_all();
  return MRF_OK;
}

extern "C" int mrf_serve_poll(mrf_server* srv, uint64_t ticket, int32_t* state, double* t_submit_ms,
                              double* t_start_ms, double* t_done_ms) {
  MRF_CHECK_ARG(srv && state, "server and state must not be NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  MRF_CHECK_ARG(it != srv->reqs.end(), "unknown ticket %llu", (unsigned long long)ticket);
  const Req& r = *it->second;
  *state = r.state;
  if (t_submit_ms) *t_submit_ms = r.t_submit;
  if (t_start_ms) *t_start_ms = r.t_start;
  if (t_done_ms) *t_done_ms = r.t_done;
  if (r.state == MRF_REQ_FAILED) set_error("%s", r.err.c_str());
  return MRF_OK;
}

extern "C" int mrf_serve_cancel(mrf_server* srv, uint64_t ticket) {
  MRF_CHECK_ARG(srv, "server must not be NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  MRF_CHECK_ARG(it != srv->reqs.end(), "unknown ticket %llu", (unsigned long long)ticket);
  Req& r = *it->second;
  if (r.state == MRF_REQ_RUNNING) {
    set_error("request %llu is running", (unsigned long long)ticket);
    return MRF_ERR_NOT_READY;
  }
  if (r.state != MRF_REQ_QUEUED) return MRF_OK;
  r.state = MRF_REQ_CANCELLED;
  r.t_done = srv->now_ms();
  srv->st.cancelled++;
  if (r.admitted) {  // release its reservation; the queues skip cancelled entries
    srv->reserved -= r.footprint;
    srv->inflight--;
  }
  srv->cv.notify_all();
  return MRF_OK;
}

extern "C" int mrf_server_stats_read(mrf_server* srv, mrf_server_stats* out) {
  MRF_CHECK_ARG(srv && out, "server and out must not be NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = srv->st;
  out->resident_bytes = srv->resident;
  out->reserved_bytes = srv->reserved;
  out->arena_peak_bytes = srv->arena.peak();
  return MRF_OK;
}

extern "C" int mrf_server_destroy(mrf_server* srv) {
  if (!srv) return MRF_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  if (srv->th.joinable()) srv->th.join();
  if (!srv->fake) {
    (void)hipSetDevice(srv->ctx->device);
    for (auto& s : srv->slots) free_slot(srv, *s);
    if (srv->arena_base) (void)hipFree(srv->arena_base);
    for (hipEvent_t e : srv->events) (void)hipEventDestroy(e);
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
  }
  delete srv;
  return MRF_OK;
}
