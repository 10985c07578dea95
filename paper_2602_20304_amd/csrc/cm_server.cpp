// Serving loop: continuous batching of collision requests over resident
// geometry.
//
// A scheduler thread admits pending requests in arrival order while their
// device footprint fits in the HBM budget, their pinned result buffers fit in
// the host budget and a stream slot is free; every admitted request gets its
// own stream, device workspace (stream-ordered allocation) and device error
// word, so requests that arrive while others run are admitted as soon as
// memory and a slot free up, and their kernels overlap on the GPU.  Results
// (and gradients for backward requests) are copied to pinned host blocks
// taken at admission from a server-wide pool (reused after
// cm_server_release) and owned by the server until then.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "cm_context.h"
#include "cm_kernels.h"

using namespace cm;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Last error message of a failing server call, per calling thread.
thread_local std::string t_server_error;

cm_status srv_fail(cm_status s, const std::string& msg) {
  t_server_error = msg;
  return s;
}

struct Request {
  uint64_t ticket = 0;
  // host copies
  std::vector<int32_t> body_offsets, body_geom;
  std::vector<float> pose, cot_point, cot_normal, cot_dist, cot_weight;
  cm_params params{};
  bool want_bwd = false, want_geom = false;
  int32_t n_scenes = 0, n_bodies = 0, capacity = 0;
  int64_t pool = 0, n_geoms = 0;   // vertex pool and geometry count the gradients are laid out for
  int64_t tape_pool = 0;           // index-pool entries of a backward request's adjoint tape
  uint64_t footprint = 0, host_bytes = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  enum State { PENDING, RUNNING, DONE, FAILED } state = PENDING;
  cm_status status = CM_OK;
  int slot = -1;
  void* dev = nullptr;             // device workspace (one stream-ordered allocation, carved)
  // one pinned host block, carved: error word, n_pairs, offsets, pairs,
  // outputs (point 3, normal 3, dist, weight; each [cap*K]), gradients
  char* host = nullptr;
  size_t host_cap = 0;
  uint32_t* h_err = nullptr;
  int32_t* h_n_pairs = nullptr;
  int32_t* h_offsets = nullptr;
  int32_t* h_pairs = nullptr;
  float* h_out = nullptr;
  float* h_gpose = nullptr;
  float* h_gtau = nullptr;
  float* h_gvert = nullptr;
  float* h_gpar = nullptr;
  hipEvent_t done_ev = nullptr;
};

struct Carve {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += sizeof(T) * std::max<size_t>(n, 1);
    return p;
  }
};

// Pinned host bytes of one request's results (the same carving as launch_request).
size_t host_bytes(const Request& r) {
  const size_t cap = size_t(std::max(r.capacity, 1));
  const int K = r.params.K;
  Carve c{nullptr};
  c.take<uint32_t>(1);
  c.take<int32_t>(1);
  c.take<int32_t>(r.n_scenes + 1);
  c.take<int32_t>(2 * cap);
  c.take<float>(8 * cap * K);
  if (r.want_bwd) {
    c.take<float>(6 * size_t(r.n_bodies));
    c.take<float>(1);
    if (r.want_geom) {
      c.take<float>(3 * size_t(r.pool));
      c.take<float>(4 * size_t(r.n_geoms));
    }
  }
  return c.off + 256;
}

}  // namespace

struct cm_server {
  cm_context* ctx = nullptr;
  uint64_t budget = 0, host_budget = 0;
  uint64_t in_flight = 0;     // device bytes of running requests
  uint64_t host_in_use = 0;   // pinned bytes held by admitted, unreleased requests
  uint64_t host_pooled = 0;   // pinned bytes of released blocks kept for reuse
  std::multimap<size_t, char*> host_pool;   // released pinned blocks by size
  int n_slots = 1;
  std::vector<hipStream_t> streams;
  std::vector<int> slot_busy;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  std::deque<uint64_t> pending;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  std::atomic<bool> stop{false};
  uint64_t next_ticket = 1;
  int n_running = 0;
};

namespace {

// A pinned block of at least `need` bytes for a request being admitted
// (caller holds srv->mu): the smallest pooled block that fits, else a new
// one after freeing pooled blocks until the host budget allows it.  Returns
// false when the budget cannot take it now (the request waits).
bool take_host_block(cm_server* srv, Request& r) {
  const size_t need = r.host_bytes;
  auto it = srv->host_pool.lower_bound(need);
  if (it != srv->host_pool.end() && it->first <= 2 * need) {
    r.host = it->second;
    r.host_cap = it->first;
    srv->host_pooled -= it->first;
    srv->host_pool.erase(it);
    srv->host_in_use += r.host_cap;
    return true;
  }
  while (srv->host_in_use + srv->host_pooled + need > srv->host_budget && !srv->host_pool.empty()) {
    auto big = std::prev(srv->host_pool.end());
    (void)hipHostFree(big->second);
    srv->host_pooled -= big->first;
    srv->host_pool.erase(big);
  }
  if (srv->host_in_use + need > srv->host_budget) return false;
  void* p = nullptr;
  if (hipHostMalloc(&p, need) != hipSuccess) return false;
  r.host = static_cast<char*>(p);
  r.host_cap = need;
  srv->host_in_use += need;
  return true;
}

void give_host_block(cm_server* srv, Request& r) {
  if (!r.host) return;
  srv->host_in_use -= r.host_cap;
  srv->host_pool.emplace(r.host_cap, r.host);
  srv->host_pooled += r.host_cap;
  r.host = nullptr;
}

// Persistent grid of one request: the whole GPU at the kernel's occupancy
// (requests on other streams take over CUs as this grid's workgroups
// retire), but no more workgroups than candidate pairs.
long long request_grid(const cm_context* ctx, int occupancy, size_t cap) {
  return std::max<long long>(1, std::min<long long>((long long)occupancy * ctx->num_cus, (long long)cap));
}

// Device bytes one request needs (inputs, outputs, scratch, gradients).
uint64_t footprint(const Request& r, long long grid, long long stride) {
  const int K = r.params.K;
  const uint64_t cap = uint64_t(std::max(r.capacity, 1));
  uint64_t b = 0;
  b += 4ull * (r.n_scenes + 1) * 2 + 4ull * r.n_bodies + 28ull * r.n_bodies;      // offsets, geom ids, poses
  b += 8ull + 8ull * cap + 32ull * cap * K;                                        // error, n_pairs, pairs, outputs
  b += 4ull * (r.n_scenes / 1024 + 2);                                             // scan tiles
  b += 4ull * uint64_t(grid) * uint64_t(stride);                                   // per-workgroup scratch
  b += 512;                                                                       // work-queue counters
  if (r.want_bwd) {
    b += 32ull * cap * K + 24ull * r.n_bodies + 4ull;                              // cotangents, g_pose, g_tau
    if (r.want_geom) b += 12ull * uint64_t(r.pool) + 16ull * uint64_t(r.n_geoms);   // g_vertices, g_params
    b += 256ull + uint64_t(tape_records_bytes(int64_t(cap), K)) + 4ull * uint64_t(r.tape_pool);   // adjoint tape
  }
  return b + 64 * 256;
}

// Index-pool entries of a served backward request's adjoint tape: what every
// pair's window could fill, at most 4,096 entries a pair on average and the
// pool limit of the direct backward (a pair whose window no longer fits is
// recomputed whole by the adjoint, so the bound costs time, not results).
int64_t served_tape_pool(const cm_context* ctx, size_t cap) {
  const int64_t per_pair = std::min<int64_t>(2LL * ctx->maxV + 2LL * ctx->maxE * ctx->maxE, 4096);
  return std::max<int64_t>(2, std::min<int64_t>(int64_t(cap) * per_pair, 1LL << 28));
}

void launch_request(cm_server* srv, Request& r) {
  cm_context* ctx = srv->ctx;
  hipStream_t st = srv->streams[r.slot];
  ParamsDev pd;
  if (resolve_params(ctx, &r.params, &pd) != CM_OK) { r.status = CM_ERR_INVALID_ARG; return; }
  const int K = pd.K;
  const size_t cap = size_t(std::max(r.capacity, 1));
  Carve h{r.host};
  r.h_err = h.take<uint32_t>(1);
  r.h_n_pairs = h.take<int32_t>(1);
  r.h_offsets = h.take<int32_t>(r.n_scenes + 1);
  r.h_pairs = h.take<int32_t>(2 * cap);
  r.h_out = h.take<float>(8 * cap * K);
  if (r.want_bwd) {
    r.h_gpose = h.take<float>(6 * size_t(r.n_bodies));
    r.h_gtau = h.take<float>(1);
    if (r.want_geom) {
      r.h_gvert = h.take<float>(3 * size_t(r.pool));
      r.h_gpar = h.take<float>(4 * size_t(r.n_geoms));
    }
  }
  FwdLaunch f;
  f.tb = ctx_tables(ctx);
  f.maxV = std::max(ctx->maxV, 1); f.maxE = std::max(ctx->maxE, 1); f.maxF = std::max(ctx->maxF, 1);
  f.block = 256; f.kmax = kmax_for(K); f.order = nullptr; f.range = nullptr;
  // workgroups take pairs from a work queue (traced witnesses keep the
  // static order); the hint selects the work-queue kernel's occupancy
  const bool dyn = pd.refine == 0;
  f.queue = dyn ? reinterpret_cast<int*>(1) : nullptr;
  // grid already folded into the footprint: recompute the same value
  f.prm = pd;
  const int occ = fwd_place_edges(f);
  f.queue = nullptr;
  f.grid = int(request_grid(ctx, occ, cap));
  f.scratch_stride = fwd_scratch_floats(f.maxV, f.maxE);
  if (hipMallocAsync(&r.dev, size_t(r.footprint), st) != hipSuccess) { r.status = CM_ERR_OOM; return; }
  Carve c{static_cast<char*>(r.dev)};
  uint32_t* d_err = c.take<uint32_t>(1);
  int32_t* d_bo = c.take<int32_t>(r.n_scenes + 1);
  int32_t* d_bg = c.take<int32_t>(r.n_bodies);
  float* d_pose = c.take<float>(7 * size_t(r.n_bodies));
  int32_t* d_np = c.take<int32_t>(1);
  int32_t* d_off = c.take<int32_t>(r.n_scenes + 1);
  int32_t* d_pairs = c.take<int32_t>(2 * cap);
  float* d_out = c.take<float>(8 * cap * K);
  int32_t* d_tiles = c.take<int32_t>(r.n_scenes / 1024 + 2);
  float* d_scr = c.take<float>(size_t(f.grid) * size_t(f.scratch_stride));
  int* d_fq = c.take<int>(64);   // forward work-queue counter
  int* d_bq = c.take<int>(64);   // adjoint work-queue counter
  TapeDev tv;
  if (r.want_bwd) {
    // the forward records the adjoint's tape (s_[k], SoftSort row sums, each
    // pair's window) beside its outputs; the adjoint reads it back
    const long long tb = 256 + tape_records_bytes((long long)cap, K) + 4LL * r.tape_pool;
    char* d_tape = c.take<char>(size_t(tb));
    tape_layout(d_tape, tb, (long long)cap, K, &tv);
  }
  f.err = d_err;
  (void)hipMemsetAsync(d_err, 0, sizeof(uint32_t), st);
  (void)hipMemcpyAsync(d_bo, r.body_offsets.data(), 4 * r.body_offsets.size(), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(d_bg, r.body_geom.data(), 4 * r.body_geom.size(), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(d_pose, r.pose.data(), 4 * r.pose.size(), hipMemcpyHostToDevice, st);
  BatchDev bd{r.n_scenes, r.n_bodies, 0, d_bo, d_bg, d_pose, nullptr, nullptr};
  OutDev od{int32_t(cap), d_np, d_off, d_pairs, d_out, d_out + 3 * cap * K, d_out + 6 * cap * K, d_out + 7 * cap * K};
  f.bt = bd; f.out = od; f.scratch = d_scr;
  if (dyn) f.queue = d_fq;
  if (r.want_bwd) f.tape = tv;
  if (launch_broadphase(f.tb, bd, pd.margin, od, d_tiles, d_err, st) != hipSuccess ||
      (dyn && launch_counter_reset(d_fq, st) != hipSuccess) ||
      (r.want_bwd && launch_tape_reset(tv, st) != hipSuccess) ||
      launch_collide_fwd(f, st) != hipSuccess) {
    r.status = CM_ERR_DEVICE;
    return;
  }
  if (r.want_bwd) {
    // cotangents: each given one is copied, the others are zero
    float* d_cp = c.take<float>(3 * cap * K);
    float* d_cn = c.take<float>(3 * cap * K);
    float* d_cd = c.take<float>(cap * K);
    float* d_cw = c.take<float>(cap * K);
    float* d_gpose = c.take<float>(6 * size_t(r.n_bodies));
    float* d_gtau = c.take<float>(1);
    float* d_gvert = r.want_geom ? c.take<float>(3 * size_t(r.pool)) : nullptr;
    float* d_gpar = r.want_geom ? c.take<float>(4 * size_t(r.n_geoms)) : nullptr;
    auto put = [&](float* d, const std::vector<float>& v, size_t n) {
      (void)hipMemsetAsync(d, 0, 4 * n, st);
      if (!v.empty()) (void)hipMemcpyAsync(d, v.data(), 4 * std::min(v.size(), n), hipMemcpyHostToDevice, st);
    };
    put(d_cp, r.cot_point, 3 * cap * K);
    put(d_cn, r.cot_normal, 3 * cap * K);
    put(d_cd, r.cot_dist, cap * K);
    put(d_cw, r.cot_weight, cap * K);
    (void)hipMemsetAsync(d_gpose, 0, 24 * size_t(r.n_bodies), st);
    (void)hipMemsetAsync(d_gtau, 0, 4, st);
    if (r.want_geom) {
      (void)hipMemsetAsync(d_gvert, 0, 12 * size_t(r.pool), st);
      (void)hipMemsetAsync(d_gpar, 0, 16 * size_t(r.n_geoms), st);
    }
    BwdLaunch b;
    b.f = f;
    b.f.queue = d_bq;      // the adjoint's own work queue
    b.f.tape = tv;
    b.f.tape.pool_used = nullptr;
    b.cot = CotDev{d_cp, d_cn, d_cd, d_cw};
    b.gr = GradDev{d_gpose, d_gvert, d_gpar, d_gtau, (long long)r.pool};
    b.f.grid = int(std::min<long long>(request_grid(ctx, bwd_place(b), cap), f.grid));   // fits the forward's scratch
    if (launch_counter_reset(d_bq, st) != hipSuccess || launch_collide_bwd(b, st) != hipSuccess) {
      r.status = CM_ERR_DEVICE;
      return;
    }
    (void)hipMemcpyAsync(r.h_gpose, d_gpose, 24 * size_t(r.n_bodies), hipMemcpyDeviceToHost, st);
    (void)hipMemcpyAsync(r.h_gtau, d_gtau, 4, hipMemcpyDeviceToHost, st);
    if (r.want_geom) {
      (void)hipMemcpyAsync(r.h_gvert, d_gvert, 12 * size_t(r.pool), hipMemcpyDeviceToHost, st);
      (void)hipMemcpyAsync(r.h_gpar, d_gpar, 16 * size_t(r.n_geoms), hipMemcpyDeviceToHost, st);
    }
  }
  (void)hipMemcpyAsync(r.h_err, d_err, 4, hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(r.h_n_pairs, d_np, 4, hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(r.h_offsets, d_off, 4 * size_t(r.n_scenes + 1), hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(r.h_pairs, d_pairs, 8 * cap, hipMemcpyDeviceToHost, st);
  (void)hipMemcpyAsync(r.h_out, d_out, 32 * cap * K, hipMemcpyDeviceToHost, st);
  (void)hipFreeAsync(r.dev, st);
  r.dev = nullptr;
  (void)hipEventCreateWithFlags(&r.done_ev, hipEventDisableTiming);
  (void)hipEventRecord(r.done_ev, st);
}

// Status of a completed request from its device error word.
cm_status status_of(const Request& r) {
  const uint32_t e = *r.h_err;
  if (e & ERR_BAD_GEOM) return CM_ERR_NOT_FOUND;
  if (e & ERR_NO_ADJOINT) return CM_ERR_INVALID_ARG;
  if (e) return CM_ERR_DEVICE;
  return *r.h_n_pairs > r.capacity ? CM_ERR_CAPACITY : CM_OK;
}

void worker_loop(cm_server* srv) {
  hipSetDevice(srv->ctx->device);
  while (!srv->stop.load()) {
    std::vector<Request*> to_launch;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      // admit in arrival order while device memory, host memory and a slot are free
      while (!srv->pending.empty()) {
        Request& r = *srv->reqs[srv->pending.front()];
        const auto it = std::find(srv->slot_busy.begin(), srv->slot_busy.end(), 0);
        if (it == srv->slot_busy.end() || srv->in_flight + r.footprint > srv->budget) break;
        if (!take_host_block(srv, r)) break;
        r.slot = int(it - srv->slot_busy.begin());
        *it = 1;
        srv->in_flight += r.footprint;
        r.state = Request::RUNNING;
        r.t_start = now_s();
        srv->n_running++;
        srv->pending.pop_front();
        to_launch.push_back(&r);
      }
    }
    for (Request* r : to_launch) launch_request(srv, *r);
    // retire finished requests
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      for (auto& kv : srv->reqs) {
        Request& r = *kv.second;
        if (r.state != Request::RUNNING) continue;
        bool done = false;
        if (r.status != CM_OK) {
          if (r.slot >= 0) (void)hipStreamSynchronize(srv->streams[r.slot]);
          if (r.dev) { (void)hipFree(r.dev); r.dev = nullptr; }
          done = true;
        } else if (r.done_ev && hipEventQuery(r.done_ev) == hipSuccess) {
          r.status = status_of(r);
          done = true;
        }
        if (done) {
          r.t_done = now_s();
          r.state = (r.status == CM_OK || r.status == CM_ERR_CAPACITY) ? Request::DONE : Request::FAILED;
          srv->in_flight -= r.footprint;
          srv->slot_busy[r.slot] = 0;
          srv->n_running--;
          if (r.done_ev) { (void)hipEventDestroy(r.done_ev); r.done_ev = nullptr; }
          srv->cv.notify_all();
        }
      }
      if (srv->pending.empty() && srv->n_running == 0)
        srv->cv.wait_for(lk, std::chrono::milliseconds(2));
    }
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
}

}  // namespace

extern "C" {

const char* cm_server_last_error(void) { return t_server_error.c_str(); }

cm_status cm_server_create(cm_context* ctx, uint64_t hbm_budget_bytes, int32_t n_streams, cm_server** out) {
  if (!ctx || !out || n_streams < 1 || n_streams > 32 || hbm_budget_bytes == 0)
    return srv_fail(CM_ERR_INVALID_ARG, "null context or output, n_streams outside 1..32, or a zero budget");
  hipSetDevice(ctx->device);
  cm_server* srv = new cm_server();
  srv->ctx = ctx;
  srv->budget = hbm_budget_bytes;
  srv->host_budget = 8ull << 30;
  srv->n_slots = n_streams;
  srv->streams.resize(n_streams);
  srv->slot_busy.assign(n_streams, 0);
  for (auto& s : srv->streams) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto& t : srv->streams)
        if (t) (void)hipStreamDestroy(t);
      delete srv;
      return srv_fail(CM_ERR_DEVICE, "server stream creation failed");
    }
  }
  ctx->servers++;
  srv->worker = std::thread(worker_loop, srv);
  *out = srv;
  return CM_OK;
}

cm_status cm_server_set_host_budget(cm_server* srv, uint64_t host_budget_bytes) {
  if (!srv || host_budget_bytes == 0) return srv_fail(CM_ERR_INVALID_ARG, "null server or a zero budget");
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->host_budget = host_budget_bytes;
  srv->cv.notify_all();
  return CM_OK;
}

cm_status cm_server_submit(cm_server* srv, const cm_request* q, uint64_t* ticket) {
  if (!srv || !q || !ticket) return srv_fail(CM_ERR_INVALID_ARG, "null server, request or ticket");
  if (q->n_scenes < 0 || q->n_bodies < 0 || (q->n_scenes > 0 && (!q->body_offsets || !q->body_geom || !q->pose)))
    return srv_fail(CM_ERR_INVALID_ARG, "negative sizes or missing batch arrays");
  if (q->params.K < 1 || q->params.K > CM_MAX_K || !(q->params.tau > 0.f) ||
      (q->params.flags & ~(CM_FLAG_NO_EE | CM_FLAG_ONE_SIDED_VS | CM_FLAG_SAFEGUARD)))
    return srv_fail(CM_ERR_INVALID_ARG, "K outside 1..32, tau <= 0 or unknown flags");
  const bool presel = q->params.presel_vertices != 0 || q->params.presel_edges != 0;
  if (presel && (q->params.presel_vertices < 1 || q->params.presel_vertices > CM_MAX_PRESEL ||
                 q->params.presel_edges < 1 || q->params.presel_edges > CM_MAX_PRESEL))
    return srv_fail(CM_ERR_INVALID_ARG, "presel_vertices / presel_edges must both be in 1..64 (or both 0)");
  if ((q->params.flags & CM_FLAG_SAFEGUARD) && !presel)
    return srv_fail(CM_ERR_INVALID_ARG, "CM_FLAG_SAFEGUARD needs pre-selection");
  if (q->params.refine_steps < 0 || q->params.refine_steps > CM_MAX_REFINE ||
      (q->params.refine_steps > 0 && q->params.K > 16))
    return srv_fail(CM_ERR_INVALID_ARG, "refine_steps outside 0..8, or with K > 16");
  auto r = std::make_unique<Request>();
  r->n_scenes = q->n_scenes;
  r->n_bodies = q->n_bodies;
  if (q->n_scenes > 0) {
    r->body_offsets.assign(q->body_offsets, q->body_offsets + q->n_scenes + 1);
    r->body_geom.assign(q->body_geom, q->body_geom + q->n_bodies);
    r->pose.assign(q->pose, q->pose + 7 * size_t(q->n_bodies));
  } else {
    r->body_offsets.assign(1, 0);
  }
  const cm_context* ctx = srv->ctx;
  const int32_t G = int32_t(ctx->h.recs.size());
  for (int32_t g : r->body_geom)
    if (g < 0 || g >= G || ctx->h.recs[g].type < 0)
      return srv_fail(CM_ERR_NOT_FOUND, "body_geom names no live geometry: " + std::to_string(g));
  if (r->body_offsets[0] != 0) return srv_fail(CM_ERR_INVALID_ARG, "body_offsets[0] must be 0");
  long long ncand = 0;
  for (int s = 0; s < q->n_scenes; ++s) {
    const long long nb = r->body_offsets[s + 1] - r->body_offsets[s];
    if (nb < 0 || r->body_offsets[s + 1] > q->n_bodies)
      return srv_fail(CM_ERR_INVALID_ARG, "body_offsets must be non-decreasing and at most n_bodies");
    ncand += nb * (nb - 1) / 2;
  }
  r->capacity = q->capacity > 0 ? q->capacity : int32_t(std::min<long long>(ncand, 1LL << 30));
  r->params = q->params;
  r->want_bwd = q->want_backward != 0;
  r->want_geom = r->want_bwd && q->want_geometry_grads != 0;
  r->pool = int64_t(ctx->h.vx.size());
  r->n_geoms = G;
  const int K = q->params.K;
  const size_t cap = size_t(std::max(r->capacity, 1));
  if (r->want_bwd) {
    if (q->cot_point) r->cot_point.assign(q->cot_point, q->cot_point + 3 * cap * K);
    if (q->cot_normal) r->cot_normal.assign(q->cot_normal, q->cot_normal + 3 * cap * K);
    if (q->cot_dist) r->cot_dist.assign(q->cot_dist, q->cot_dist + cap * K);
    if (q->cot_weight) r->cot_weight.assign(q->cot_weight, q->cot_weight + cap * K);
  }
  // footprint with the grid this request will use
  FwdLaunch f{};
  f.tb = ctx_tables(ctx);
  f.maxV = std::max(ctx->maxV, 1); f.maxE = std::max(ctx->maxE, 1); f.maxF = std::max(ctx->maxF, 1);
  f.block = 256; f.kmax = kmax_for(K);
  f.queue = q->params.refine_steps == 0 ? reinterpret_cast<int*>(1) : nullptr;   // work-queue kernel's occupancy
  f.prm.presel_v = presel ? q->params.presel_vertices : 0;   // selects the kernel whose occupancy applies
  f.prm.presel_e = presel ? q->params.presel_edges : 0;
  f.prm.sq = ctx->has_sq ? 1 : 0;
  f.prm.refine = q->params.refine_steps;
  const long long grid = request_grid(ctx, fwd_place_edges(f), cap);
  if (r->want_bwd) r->tape_pool = served_tape_pool(ctx, cap);
  r->footprint = footprint(*r, grid, fwd_scratch_floats(f.maxV, f.maxE));
  r->host_bytes = host_bytes(*r);
  if (r->footprint > srv->budget)
    return srv_fail(CM_ERR_REJECTED, "request needs " + std::to_string(r->footprint) +
                                         " B of device memory, beyond the server's budget");
  if (r->host_bytes > srv->host_budget)
    return srv_fail(CM_ERR_REJECTED, "request needs " + std::to_string(r->host_bytes) +
                                         " B of pinned result memory, beyond the server's budget");
  r->t_submit = now_s();
  std::lock_guard<std::mutex> lk(srv->mu);
  r->ticket = srv->next_ticket++;
  *ticket = r->ticket;
  srv->pending.push_back(r->ticket);
  srv->reqs[r->ticket] = std::move(r);
  srv->cv.notify_all();
  return CM_OK;
}

cm_status cm_server_poll(cm_server* srv, uint64_t ticket, cm_result* out) {
  if (!srv || !out) return srv_fail(CM_ERR_INVALID_ARG, "null server or result");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return srv_fail(CM_ERR_NOT_FOUND, "no such ticket");
  Request& r = *it->second;
  if (r.state == Request::PENDING || r.state == Request::RUNNING) return CM_ERR_NOT_READY;
  std::memset(out, 0, sizeof(*out));
  out->status = r.status;
  out->t_submit = r.t_submit;
  out->t_start = r.t_start;
  out->t_done = r.t_done;
  out->footprint_bytes = r.footprint;
  out->capacity = r.capacity;
  out->vertex_pool = int32_t(r.pool);
  out->n_geometries = int32_t(r.n_geoms);
  if (!r.host || !r.h_out) return r.status;   // failed before its results were laid out
  const size_t cap = size_t(std::max(r.capacity, 1));
  const int K = r.params.K;
  out->n_pairs = *r.h_n_pairs;
  out->pair_offsets = r.h_offsets;
  out->pairs = r.h_pairs;
  out->point = r.h_out;
  out->normal = r.h_out + 3 * cap * K;
  out->dist = r.h_out + 6 * cap * K;
  out->weight = r.h_out + 7 * cap * K;
  out->g_pose = r.h_gpose;
  out->g_tau = r.h_gtau;
  out->g_vertices = r.h_gvert;
  out->g_params = r.h_gpar;
  return r.status;
}

cm_status cm_server_release(cm_server* srv, uint64_t ticket) {
  if (!srv) return srv_fail(CM_ERR_INVALID_ARG, "null server");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return srv_fail(CM_ERR_NOT_FOUND, "no such ticket");
  Request& r = *it->second;
  if (r.state == Request::PENDING || r.state == Request::RUNNING) return CM_ERR_NOT_READY;
  give_host_block(srv, r);
  srv->reqs.erase(it);
  srv->cv.notify_all();
  return CM_OK;
}

cm_status cm_server_stats(cm_server* srv, uint64_t* in_flight_bytes, int32_t* n_pending, int32_t* n_running) {
  if (!srv) return srv_fail(CM_ERR_INVALID_ARG, "null server");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (in_flight_bytes) *in_flight_bytes = srv->in_flight;
  if (n_pending) *n_pending = int32_t(srv->pending.size());
  if (n_running) *n_running = srv->n_running;
  return CM_OK;
}

cm_status cm_server_destroy(cm_server* srv) {
  if (!srv) return srv_fail(CM_ERR_INVALID_ARG, "null server");
  {
    // drain: wait for every admitted or pending request to finish
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv.wait(lk, [&] { return srv->pending.empty() && srv->n_running == 0; });
  }
  srv->stop.store(true);
  srv->cv.notify_all();
  if (srv->worker.joinable()) srv->worker.join();
  for (auto& s : srv->streams) (void)hipStreamDestroy(s);
  srv->ctx->servers--;
  for (auto& kv : srv->reqs)
    if (kv.second->host) (void)hipHostFree(kv.second->host);
  for (auto& kv : srv->host_pool) (void)hipHostFree(kv.second);
  delete srv;
  return CM_OK;
}

}  // extern "C"
