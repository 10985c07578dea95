// Fused batched forward: size classes with their own LDS sizing and tuned
// block size, cost-ordered dynamic work queues, and the whole sequence
// (broadphase, classification, one persistent launch per class) captured in
// a hipGraph that is replayed for later calls on the same buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include <sys/stat.h>

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
  f.grid = std::max(1, fwd_place_edges(f) * ctx->num_cus);
  f.scratch_stride = fwd_scratch_floats(f.maxV, f.maxE);
  return f;
}

// Persistent autotune cache: one "key block" line per tuned (device, size
// class) configuration, in the file named by CM_TUNE_CACHE (default
// $HOME/.cache/cm_fused_tune.txt; none without HOME).  Read on first use and
// whenever that name changes, appended to after each tuning; an unreadable
// or unwritable file only disables the cache.
std::mutex g_tune_mu;
bool g_tune_loaded = false;
std::string g_tune_loaded_path;
std::map<std::string, int> g_tune;

std::string tune_path() {
  if (const char* p = std::getenv("CM_TUNE_CACHE")) return p;
  if (const char* h = std::getenv("HOME")) return std::string(h) + "/.cache/cm_fused_tune.txt";
  return std::string();
}

std::string tune_key(const cm_context* ctx, int c, int kmax, int scale) {
  std::ostringstream k;
  k << ctx->arch << ":cu" << ctx->num_cus << ":E" << ctx->cls_maxE[c] << ":V" << ctx->cls_maxV[c] << ":F"
    << ctx->cls_maxF[c] << ":k" << kmax << ":n" << scale;
  return k.str();
}

// Batch-size bucket of a tuning: floor(log2(candidate pairs)) / 2, one bucket
// per factor of 4 (a block size that wins on a few thousand pairs need not
// win on millions).
int tune_scale(int capacity) {
  int l = 0;
  while ((2LL << l) <= (long long)capacity) ++l;
  return l / 2;
}

int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const std::string p = tune_path();
  if (!g_tune_loaded || p != g_tune_loaded_path) {   // (re)read when the file name changes
    g_tune_loaded = true;
    g_tune_loaded_path = p;
    g_tune.clear();
    std::ifstream in(p);
    std::string k;
    int b;
    while (in >> k >> b)   // only block sizes the tuner can choose
      if (std::find(kTuneBlock, kTuneBlock + kTuneBlocks, b) != kTuneBlock + kTuneBlocks) g_tune[k] = b;
  }
  auto it = g_tune.find(key);
  return it == g_tune.end() ? 0 : it->second;
}

void tune_store(const std::string& key, int block) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = block;
  const std::string p = tune_path();
  if (p.empty()) return;
  const size_t slash = p.find_last_of('/');
  if (slash != std::string::npos && slash > 0) (void)::mkdir(p.substr(0, slash).c_str(), 0755);
  std::ofstream out(p, std::ios::app);
  if (out) out << key << " " << block << "\n";
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
  TapeDev tv;   // the adjoint's tape, recorded by the class kernels when given
  if (od.tape && od.capacity > 0 && !tape_layout(od.tape, od.tape_bytes, od.capacity, pd.K, &tv))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "the tape is smaller than cm_tape_bytes gives for this capacity and K");
  hipSetDevice(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = ctx_order(ctx, st)) != CM_OK) return s;
  build_plan(ctx, pd.K);

  // work buffers: counts, ranges, queues, order[cap], keys[cap]
  const size_t head = 4 * (kNumClasses * kNumBuckets + 2 * kNumClasses + kNumClasses + 16);
  // order[cap], keys[cap], then the autotune sample (cap pairs + range + queue)
  const size_t need = head + 12 * size_t(std::max(od.capacity, 1)) + 64;
  hipError_t e = ctx_ensure(ctx, &ctx->d_fused, &ctx->fused_cap, need);
  if (e != hipSuccess) return cm_hip(ctx, e, "fused work buffers");
  int* base = static_cast<int*>(ctx->d_fused);
  FusedWork w;
  w.counts = base;
  w.ranges = w.counts + kNumClasses * kNumBuckets;
  w.queues = w.ranges + 2 * kNumClasses;
  w.order = reinterpret_cast<int*>(reinterpret_cast<char*>(ctx->d_fused) + head);
  w.keys = w.order + std::max(od.capacity, 1);
  w.sample = w.keys + std::max(od.capacity, 1);

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
    if (tv.base && (e2 = launch_tape_reset(tv, s2)) != hipSuccess) return e2;
    for (int c = 0; c < kNumClasses; ++c) {
      FwdLaunch f = fl[c];
      f.tape = tv;
      if ((e2 = launch_collide_fwd(f, s2)) != hipSuccess) return e2;
    }
    return hipSuccess;
  };
  const size_t tiles = size_t(bd.n_scenes) / 1024 + 2;
  e = ctx_ensure(ctx, reinterpret_cast<void**>(&ctx->d_tile_sums), &ctx->tile_cap, tiles * sizeof(int));
  if (e != hipSuccess) return cm_hip(ctx, e, "tile sums");

  // Autotune the block size of each size class once per plan: cached
  // choices first; otherwise, after this batch's broadphase and
  // classification, every candidate block size runs on the same evenly
  // strided sample of the class's cost order (about 1/16 of the class, at
  // least 4 pairs per workgroup of the larger grid) and the fastest is kept
  // (full-method calls on the basic primitives only: pre-selection and the
  // extended primitives always run 256-thread blocks).
  const int scale = tune_scale(od.capacity);
  if ((!ctx->plan_tuned || ctx->plan_scale != scale) && od.capacity > 0 && pd.presel_v == 0 && !pd.sq) {
    const int kmax = kmax_for(pd.K);
    bool all_cached = true;
    for (int c = 0; c < kNumClasses; ++c) {
      const int b = tune_lookup(tune_key(ctx, c, kmax, scale));
      ctx->cls_cached[c] = b;
      ctx->cls_block[c] = b ? b : 256;
      all_cached &= b != 0;
    }
    if (!all_cached) {
      if ((s = plan_scratch()) != CM_OK) return s;
      if ((e = launch_broadphase(ctx_tables(ctx), bd, pd.margin, od, ctx->d_tile_sums, ctx->d_err, st)) != hipSuccess ||
          (e = launch_fused_prepare(ctx_tables(ctx), bd, od, cmax, w, st)) != hipSuccess)
        return cm_hip(ctx, e, "autotune classification");
      int ranges[2 * kNumClasses];
      if ((e = hipMemcpyAsync(ranges, w.ranges, sizeof(ranges), hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (e = hipStreamSynchronize(st)) != hipSuccess)
        return cm_hip(ctx, e, "autotune ranges");
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        return cm_hip(ctx, e, "autotune events");
      for (int c = 0; c < kNumClasses && s == CM_OK; ++c) {
        const int count = ranges[2 * c + 1];
        ctx->cls_tune_n[c] = 0;
        for (int bi = 0; bi < kTuneBlocks; ++bi) ctx->cls_tuned_ms[c][bi] = 0.f;
        if (ctx->cls_cached[c] || count <= 0) continue;
        float best = 1e30f;
        int best_block = 256;
        // candidates that keep at least 2 waves per SIMD (256 always)
        bool try_b[kTuneBlocks];
        int max_grid = 1;
        for (int bi = 0; bi < kTuneBlocks; ++bi) {
          const FwdLaunch t = class_launch(ctx, bd, pd, od, c, kTuneBlock[bi], w);
          try_b[bi] = bi == 0 || (t.grid / std::max(ctx->num_cus, 1)) * (kTuneBlock[bi] / 64) >= 8;
          if (try_b[bi]) max_grid = std::max(max_grid, t.grid);
        }
        {
          // the same strided sample for every candidate: about 1/16 of the
          // class, at least 4 pairs per workgroup of the largest grid
          const int n = std::min(count, std::max(count / 16, 4 * max_grid));
          ctx->cls_tune_n[c] = n;
          if ((e = launch_fused_sample(w, c, n, w.sample, w.sample + n + 1, st)) != hipSuccess) {
            s = cm_hip(ctx, e, "autotune sample");
            break;
          }
        }
        for (int bi = 0; bi < kTuneBlocks; ++bi) {
          if (!try_b[bi]) continue;
          ctx->cls_block[c] = kTuneBlock[bi];
          if ((s = plan_scratch()) != CM_OK) break;
          FwdLaunch t = fl[c];
          const int n = ctx->cls_tune_n[c];
          t.order = w.sample;
          t.range = w.sample + n + 1;
          t.queue = w.sample + n + 3;
          (void)hipMemsetAsync(t.queue, 0, sizeof(int), st);
          (void)hipEventRecord(e0, st);
          if ((e = launch_collide_fwd(t, st)) != hipSuccess) { s = cm_hip(ctx, e, "autotune launch"); break; }
          (void)hipEventRecord(e1, st);
          (void)hipEventSynchronize(e1);
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          ctx->cls_tuned_ms[c][bi] = ms;
          if (ms < best) { best = ms; best_block = kTuneBlock[bi]; }
        }
        ctx->cls_block[c] = best_block;
        if (s == CM_OK) tune_store(tune_key(ctx, c, kmax, scale), best_block);
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (s != CM_OK) return s;
    }
    ctx->plan_tuned = true;
    ctx->plan_scale = scale;
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
                            uint64_t(pd.presel_v), uint64_t(pd.presel_e), uint64_t(uintptr_t(od.tape)),
                            uint64_t(od.tape_bytes)};
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

// The fused path's current plan: per size class its largest edge count, the
// block size in use, the autotune sample size and the sample timings at
// blocks 256 and 128 (0 when not timed), and whether the choice came from
// the cache file.
extern "C" cm_status cm_fused_tuning(cm_context* ctx, int32_t* class_max_edges, int32_t* class_blocks,
                                     int32_t* sample_pairs, float* sample_ms, int32_t* from_cache) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  for (int c = 0; c < kNumClasses; ++c) {
    if (class_max_edges) class_max_edges[c] = ctx->cls_maxE[c];
    if (class_blocks) class_blocks[c] = ctx->cls_block[c];
    if (sample_pairs) sample_pairs[c] = ctx->cls_tune_n[c];
    if (sample_ms)
      for (int bi = 0; bi < kTuneBlocks; ++bi) sample_ms[kTuneBlocks * c + bi] = ctx->cls_tuned_ms[c][bi];
    if (from_cache) from_cache[c] = ctx->cls_cached[c] != 0;
  }
  return CM_OK;
}
