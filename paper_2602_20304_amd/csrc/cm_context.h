// The library context: geometry store (host mirror + device tables) and the
// workspace the kernels use.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cm_internal.h"

struct CmPools {
  std::vector<cm::GeomRec> recs;
  std::vector<double> vx, vy, vz;
  std::vector<int32_t> e0, e1;
  std::vector<double> fnx, fny, fnz, fo;
  std::vector<int32_t> f0, f1, f2;
};

template <typename T>
struct CmDevPtr;

struct CmDevPools {
  cm::GeomRec* recs = nullptr;
  double *vx = nullptr, *vy = nullptr, *vz = nullptr;
  int32_t *e0 = nullptr, *e1 = nullptr;
  double *fnx = nullptr, *fny = nullptr, *fnz = nullptr, *fo = nullptr;
  int32_t *f0 = nullptr, *f1 = nullptr, *f2 = nullptr;
};

struct CmDevCaps {
  size_t recs = 0, vx = 0, vy = 0, vz = 0, e0 = 0, e1 = 0, fnx = 0, fny = 0, fnz = 0, fo = 0, f0 = 0, f1 = 0, f2 = 0;
};

// Block sizes the fused path's autotuner may time per size class.
constexpr int kTuneBlocks = 3;
constexpr int kTuneBlock[kTuneBlocks] = {256, 128, 64};

struct cm_context {
  int device = 0;
  int num_cus = 1;
  std::string arch;           // device architecture name (autotune cache key)
  CmPools h;
  CmDevPools d;
  CmDevCaps dcap;
  int maxV = 0, maxE = 0, maxF = 0;
  bool has_sq = false;   // some geometry is a superquadric union
  unsigned* d_err = nullptr;
  int* d_tile_sums = nullptr;
  size_t tile_cap = 0;
  float* d_scratch = nullptr;
  size_t scratch_cap = 0;
  // the allocation-free forward's workspace on this device (static array)
  void* noalloc_scratch = nullptr;
  std::string noalloc_error;
  void* d_work = nullptr;      // fused path: queue counter, order, keys
  size_t work_cap = 0;
  int* d_fwd_queue = nullptr;  // the plain forward's work-queue counter
  size_t fwd_queue_cap = 0;
  void* d_bwd = nullptr;       // backward workspace: pool and work-queue counters, the adjoint's tape (records, index pool)
  size_t bwd_cap = 0;
  // fused path: size-class plan (per K), tuned block sizes, captured graphs
  int geom_version = 0;
  int servers = 0;             // live servers (geometry is frozen while > 0)
  int plan_K = -1, plan_version = -1;
  bool plan_tuned = false;
  int plan_scale = -1;         // batch-size bucket the block sizes were tuned for
  int cls_maxE[3] = {0, 0, 0}, cls_maxV[3] = {0, 0, 0}, cls_maxF[3] = {0, 0, 0}, cls_block[3] = {256, 256, 256};
  int cls_bound[2] = {96, 300};
  float cls_tuned_ms[3][kTuneBlocks] = {};   // autotune sample timings (kTuneBlock order), 0 = not timed
  int cls_tune_n[3] = {0, 0, 0};   // sample sizes
  int cls_cached[3] = {0, 0, 0};   // choice taken from the cache file
  void* d_fused = nullptr;
  size_t fused_cap = 0;
  hipStream_t cap_stream = nullptr;
  struct GraphEntry {
    uint64_t key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
    graphs.clear();
  }
  std::string last_error;
  // cross-stream ordering of calls that use the workspace above
  hipStream_t last_stream = nullptr;
  hipEvent_t order_ev = nullptr;
  bool order_pending = false;
  // opt-in event timing (cm_set_kernel_timing)
  struct Timer {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double ms = 0.0;
    long long launches = 0;
  };
  bool timing = false;
  Timer timers[CM_N_TIMERS];
  std::vector<hipEvent_t> spare_events;

  void release_all() {
    auto F = [](void* p) { if (p) hipFree(p); };
    F(d.recs); F(d.vx); F(d.vy); F(d.vz); F(d.e0); F(d.e1); F(d.fnx); F(d.fny); F(d.fnz); F(d.fo);
    F(d.f0); F(d.f1); F(d.f2);
    F(d_err); F(d_tile_sums); F(d_scratch); F(d_work); F(d_bwd); F(d_fwd_queue); F(d_fused);
    drop_graphs();
    for (auto& t : timers) {
      for (auto& pr : t.pending) { (void)hipEventDestroy(pr.first); (void)hipEventDestroy(pr.second); }
      t.pending.clear();
    }
    for (auto ev : spare_events) (void)hipEventDestroy(ev);
    if (order_ev) (void)hipEventDestroy(order_ev);
    order_ev = nullptr;
    spare_events.clear();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    d = CmDevPools();
  }
};

cm_status cm_fail(cm_context* ctx, cm_status s, const std::string& msg);
cm_status cm_hip(cm_context* ctx, hipError_t e, const char* what);
hipError_t ensure_bytes(void** p, size_t* cap, size_t need);
hipError_t ctx_ensure(cm_context* ctx, void** p, size_t* cap, size_t need);
cm::Tables ctx_tables(const cm_context* ctx);
cm_status resolve_params(cm_context* ctx, const cm_params* prm, cm::ParamsDev* pd);
// Calls that use the context's workspace are ordered across streams: before
// queuing work on `st`, ctx_order makes st wait for the previous such call
// when that one went to another stream; ctx_mark records the point after the
// new call's work.  Neither acts on a stream under capture (a captured
// sequence stays on one stream).
cm_status ctx_order(cm_context* ctx, hipStream_t st);
void ctx_mark(cm_context* ctx, hipStream_t st);
cm_status resolve_batch(cm_context* ctx, const cm_batch* b, cm::BatchDev* bd);
cm_status resolve_out(cm_context* ctx, const cm_manifold* o, cm::OutDev* od);
cm_status ctx_broadphase(cm_context* ctx, const cm::BatchDev& bd, const cm::ParamsDev& pd, const cm::OutDev& od,
                         hipStream_t st);
int kmax_for(int K);
// Timing brackets: begin returns the start event (or null when timing is off)
// and end records the stop event and queues the pair for cm_kernel_time.
hipEvent_t timer_begin(cm_context* ctx, hipStream_t st);
void timer_end(cm_context* ctx, int timer, hipEvent_t start, hipStream_t st);
