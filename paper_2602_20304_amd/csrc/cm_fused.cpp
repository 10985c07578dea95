// Fused batched forward: size classes with their own LDS sizing and tuned
// block size, cost-ordered dynamic work queues, and the whole sequence
// (broadphase, classification, one persistent launch per class) captured in
// a hipGraph that is replayed for later calls on the same buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "cm_context.h"
#include "cm_kernels.h"

using namespace cm;

namespace {

// Per-class LDS maxima from the context's geometries: a pair is in class c
// when the larger edge count of its bodies is within the class bound.
void build_plan(cm_context* ctx, int K) {
  if (ctx->plan_K == K && ctx->plan_version == ctx->geom_version) return;
  for (int c = 0; c < kNumClasses; ++c) { ctx->cls_maxE[c] = ctx->cls_maxV[c] = ctx->cls_maxF[c] = 0; }
  for (const GeomRec& r : ctx->h.recs) {
    for (int c = 0; c < kNumClasses; ++c) {
      const int bound = c < 2 ? ctx->cls_bound[c] : 1 << 30;
      if (r.ne <= bound) {
        ctx->cls_maxE[c] = std::max(ctx->cls_maxE[c], r.ne);
        ctx->cls_maxV[c] = std::max(ctx->cls_maxV[c], r.nv);
        ctx->cls_maxF[c] = std::max(ctx->cls_maxF[c], r.nf);
      }
    }
  }
  for (int c = 0; c < kNumClasses; ++c) {
    ctx->cls_maxE[c] = std::max(ctx->cls_maxE[c], 1);
    ctx->cls_maxV[c] = std::max(ctx->cls_maxV[c], 1);
    ctx->cls_maxF[c] = std::max(ctx->cls_maxF[c], 1);
    ctx->cls_block[c] = 256;
  }
  ctx->plan_K = K;
  ctx->plan_version = ctx->geom_version;
  ctx->plan_tuned = false;
  ctx->drop_graphs();
}

FwdLaunch class_launch(cm_context* ctx, const BatchDev& bd, const ParamsDev& pd, const OutDev& od, int c, int block,
                       const FusedWork& w) {
  FwdLaunch f;
  f.tb = ctx_tables(ctx);
  f.bt = bd; f.prm = pd; f.out = od;
  f.maxV = ctx->cls_maxV[c]; f.maxE = ctx->cls_maxE[c]; f.maxF = ctx->cls_maxF[c];
  f.block = (pd.presel_v > 0 || pd.sq) ? 256 : block;   // those kernels are built for 256-thread blocks
  f.kmax = kmax_for(pd.K);
  f.order = w.order;
  f.range = w.ranges + 2 * c;
  f.queue = w.queues + c;
  f.err = ctx->d_err;
  f.grid = std::max(1, fwd_occupancy(f) * ctx->num_cus);
  f.scratch_stride = fwd_scratch_floats(f.maxV, f.maxE);
  return f;
}

uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ULL + (h << 6) + (h >> 2);
  return h;
}

}  // namespace

extern "C" cm_status cm_collide_fused(cm_context* ctx, const cm_batch* batch, const cm_params* prm, cm_manifold* out,
                                      void* stream) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  ParamsDev pd; BatchDev bd; OutDev od;
  cm_status s;
  if ((s = resolve_params(ctx, prm, &pd)) != CM_OK) return s;
  if (pd.refine > 0) return cm_fail(ctx, CM_ERR_INVALID_ARG, "the fused path does not support witness sphere tracing");
  if ((s = resolve_batch(ctx, batch, &bd)) != CM_OK) return s;
  if ((s = resolve_out(ctx, out, &od)) != CM_OK) return s;
  hipSetDevice(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = ctx_order(ctx, st)) != CM_OK) return s;
  build_plan(ctx, pd.K);

  // work buffers: counts, ranges, queues, order[cap], keys[cap]
  const size_t head = 4 * (kNumClasses * kNumBuckets + 2 * kNumClasses + kNumClasses + 16);
  const size_t need = head + 8 * size_t(std::max(od.capacity, 1));
  hipError_t e = ctx_ensure(ctx, &ctx->d_fused, &ctx->fused_cap, need);
  if (e != hipSuccess) return cm_hip(ctx, e, "fused work buffers");
  int* base = static_cast<int*>(ctx->d_fused);
  FusedWork w;
  w.counts = base;
  w.ranges = w.counts + kNumClasses * kNumBuckets;
  w.queues = w.ranges + 2 * kNumClasses;
  w.order = reinterpret_cast<int*>(reinterpret_cast<char*>(ctx->d_fused) + head);
  w.keys = w.order + std::max(od.capacity, 1);

  FwdLaunch fl[kNumClasses];
  auto plan_scratch = [&]() -> cm_status {
    size_t sneed = 0;
    for (int c = 0; c < kNumClasses; ++c) {
      fl[c] = class_launch(ctx, bd, pd, od, c, ctx->cls_block[c], w);
      sneed = std::max(sneed, size_t(fl[c].grid) * size_t(fl[c].scratch_stride) * sizeof(float));
    }
    hipError_t e2 = ctx_ensure(ctx, reinterpret_cast<void**>(&ctx->d_scratch), &ctx->scratch_cap, sneed);
    if (e2 != hipSuccess) return cm_hip(ctx, e2, "fused scratch");
    for (int c = 0; c < kNumClasses; ++c) fl[c].scratch = ctx->d_scratch;
    return CM_OK;
  };
  const int cmax[2] = {ctx->cls_bound[0], ctx->cls_bound[1]};
  auto record = [&](hipStream_t s2) -> hipError_t {
    hipError_t e2 = launch_broadphase(ctx_tables(ctx), bd, pd.margin, od, ctx->d_tile_sums, ctx->d_err, s2);
    if (e2 != hipSuccess) return e2;
    if (od.capacity == 0) return hipSuccess;
    if ((e2 = launch_fused_prepare(ctx_tables(ctx), bd, od, cmax, w, s2)) != hipSuccess) return e2;
    for (int c = 0; c < kNumClasses; ++c)
      if ((e2 = launch_collide_fwd(fl[c], s2)) != hipSuccess) return e2;
    return hipSuccess;
  };
  const size_t tiles = size_t(bd.n_scenes) / 1024 + 2;
  e = ctx_ensure(ctx, reinterpret_cast<void**>(&ctx->d_tile_sums), &ctx->tile_cap, tiles * sizeof(int));
  if (e != hipSuccess) return cm_hip(ctx, e, "tile sums");

  // autotune the block size of each class once per plan, on this batch
  // (full-method calls on the basic primitives only: pre-selection and the
  // extended primitives always run 256-thread blocks)
  if (!ctx->plan_tuned && od.capacity > 0 && pd.presel_v == 0 && !pd.sq) {
    ctx->cls_block[0] = ctx->cls_block[1] = ctx->cls_block[2] = 256;
    if ((s = plan_scratch()) != CM_OK) return s;
    if ((e = record(st)) != hipSuccess) return cm_hip(ctx, e, "fused warm-up");
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    for (int c = 0; c < kNumClasses; ++c) {
      float best = 1e30f;
      int best_block = 256;
      for (int blk : {256, 128}) {
        ctx->cls_block[c] = blk;
        if ((s = plan_scratch()) != CM_OK) return s;
        (void)hipMemsetAsync(w.queues + c, 0, sizeof(int), st);
        (void)hipEventRecord(e0, st);
        if ((e = launch_collide_fwd(fl[c], st)) != hipSuccess) return cm_hip(ctx, e, "autotune launch");
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; best_block = blk; }
      }
      ctx->cls_block[c] = best_block;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->plan_tuned = true;
  }
  if ((s = plan_scratch()) != CM_OK) return s;

  uint64_t key = 0x51ed270b27a3cc1dULL;
  const uint64_t parts[] = {uint64_t(uintptr_t(bd.body_offsets)), uint64_t(uintptr_t(bd.body_geom)),
                            uint64_t(uintptr_t(bd.pose)), uint64_t(uintptr_t(bd.cand_offsets)),
                            uint64_t(uintptr_t(bd.cand_pairs)), uint64_t(bd.n_scenes), uint64_t(bd.n_bodies),
                            uint64_t(bd.n_cand), uint64_t(uintptr_t(od.n_pairs)), uint64_t(uintptr_t(od.pairs)),
                            uint64_t(uintptr_t(od.point)), uint64_t(uintptr_t(od.normal)),
                            uint64_t(uintptr_t(od.dist)), uint64_t(uintptr_t(od.weight)),
                            uint64_t(uintptr_t(od.pair_offsets)), uint64_t(od.capacity), uint64_t(pd.K), uint64_t(pd.flags),
                            uint64_t(pd.presel_v), uint64_t(pd.presel_e)};
  for (uint64_t v : parts) key = mix(key, v);
  double dv[4] = {pd.tau, pd.lam, pd.eps_n, double(pd.margin)};
  for (double d : dv) { uint64_t b; std::memcpy(&b, &d, 8); key = mix(key, b); }
  for (auto& g : ctx->graphs)
    if (g.key == key) {
      hipEvent_t t0 = timer_begin(ctx, st);
      if ((s = cm_hip(ctx, hipGraphLaunch(g.exec, st), "graph replay")) != CM_OK) return s;
      timer_end(ctx, CM_TIMER_FUSED, t0, st);
      ctx_mark(ctx, st);
      return CM_OK;
    }

  if (!ctx->cap_stream && (e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    return cm_hip(ctx, e, "capture stream");
  if ((e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return cm_hip(ctx, e, "begin capture");
  hipError_t er = record(ctx->cap_stream);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(ctx->cap_stream, &graph);
  if (er != hipSuccess) { if (graph) (void)hipGraphDestroy(graph); return cm_hip(ctx, er, "capture"); }
  if (e != hipSuccess) return cm_hip(ctx, e, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return cm_hip(ctx, e, "graph instantiate");
  if (ctx->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  ctx->graphs.push_back({key, exec});
  hipEvent_t t0 = timer_begin(ctx, st);
  if ((s = cm_hip(ctx, hipGraphLaunch(exec, st), "graph launch")) != CM_OK) return s;
  timer_end(ctx, CM_TIMER_FUSED, t0, st);
  ctx_mark(ctx, st);
  return CM_OK;
}
