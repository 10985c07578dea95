// C ABI implementation: context, geometry store, forward entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "cm_context.h"
#include "cm_kernels.h"

using namespace cm;

namespace {

const char* kStatusStr[] = {"ok", "invalid argument", "out of memory", "device error", "not ready",
                            "rejected", "not found", "capacity exceeded", "degenerate geometry"};

}  // namespace

cm_status cm_fail(cm_context* ctx, cm_status s, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return s;
}

cm_status cm_hip(cm_context* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return CM_OK;
  return cm_fail(ctx, e == hipErrorOutOfMemory ? CM_ERR_OOM : CM_ERR_DEVICE,
                 std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
static hipError_t dev_upload(T** dptr, size_t* cap, const std::vector<T>& h) {
  const size_t need = std::max<size_t>(h.size(), 1);
  if (*cap < need) {
    if (*dptr) (void)hipFree(*dptr);
    *dptr = nullptr;
    size_t c = std::max(need, *cap * 2);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dptr), c * sizeof(T));
    if (e != hipSuccess) { *cap = 0; return e; }
    *cap = c;
  }
  if (!h.empty()) return hipMemcpy(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  return hipSuccess;
}

hipError_t ensure_bytes(void** p, size_t* cap, size_t need) {
  if (*cap >= need && *p) return hipSuccess;
  if (*p) { (void)hipFree(*p); *p = nullptr; *cap = 0; }
  need = std::max<size_t>(need, 256);
  hipError_t e = hipMalloc(p, need);
  if (e == hipSuccess) *cap = need;
  return e;
}

// Grow a context workspace buffer; captured graphs hold workspace pointers,
// so any reallocation drops them.
hipError_t ctx_ensure(cm_context* ctx, void** p, size_t* cap, size_t need) {
  if (*cap >= need && *p) return hipSuccess;
  ctx->drop_graphs();
  return ensure_bytes(p, cap, need);
}

cm_status ctx_upload_tables(cm_context* ctx) {
  hipError_t e;
#define UP(field) \
  if ((e = dev_upload(&ctx->d.field, &ctx->dcap.field, ctx->h.field)) != hipSuccess) return cm_hip(ctx, e, "upload " #field);
  UP(recs) UP(vx) UP(vy) UP(vz) UP(e0) UP(e1) UP(fnx) UP(fny) UP(fnz) UP(fo) UP(f0) UP(f1) UP(f2)
#undef UP
  return CM_OK;
}

Tables ctx_tables(const cm_context* ctx) {
  Tables t;
  t.geoms = ctx->d.recs;
  t.n_geoms = int32_t(ctx->h.recs.size());
  t.vx = ctx->d.vx; t.vy = ctx->d.vy; t.vz = ctx->d.vz;
  t.e0 = ctx->d.e0; t.e1 = ctx->d.e1;
  t.fnx = ctx->d.fnx; t.fny = ctx->d.fny; t.fnz = ctx->d.fnz; t.fo = ctx->d.fo;
  t.f0 = ctx->d.f0; t.f1 = ctx->d.f1; t.f2 = ctx->d.f2;
  return t;
}

extern "C" {

const char* cm_status_str(cm_status s) {
  const int i = -int(s);
  if (i < 0 || i >= int(sizeof(kStatusStr) / sizeof(kStatusStr[0]))) return "unknown status";
  return kStatusStr[i];
}

const char* cm_last_error(cm_context* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

cm_status cm_context_create(int device, cm_context** out) {
  if (!out) return CM_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return CM_ERR_DEVICE;
  if (device < 0 || device >= n) return CM_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return CM_ERR_DEVICE;
  cm_context* ctx = new cm_context();
  ctx->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ctx; return CM_ERR_DEVICE; }
  ctx->num_cus = prop.multiProcessorCount;
  ctx->arch = prop.gcnArchName;
  if (hipMalloc(&ctx->d_err, sizeof(unsigned)) != hipSuccess || hipMemset(ctx->d_err, 0, sizeof(unsigned)) != hipSuccess) {
    delete ctx;
    return CM_ERR_OOM;
  }
  // device address of the allocation-free forward's static workspace (a
  // failure only disables cm_collide_noalloc, which then reports it)
  const hipError_t se = noalloc_scratch(device, &ctx->noalloc_scratch);
  if (se != hipSuccess || !ctx->noalloc_scratch) {
    ctx->noalloc_scratch = nullptr;
    ctx->noalloc_error = std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(se);
    (void)hipGetLastError();
  }
  *out = ctx;
  return CM_OK;
}

cm_status cm_context_destroy(cm_context* ctx) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  ctx->release_all();
  delete ctx;
  return CM_OK;
}

cm_status cm_check_errors(cm_context* ctx, void* stream) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  hipSetDevice(ctx->device);
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return cm_hip(ctx, e, "stream synchronize");
  unsigned bits = 0;
  if ((e = hipMemcpy(&bits, ctx->d_err, sizeof(unsigned), hipMemcpyDeviceToHost)) != hipSuccess)
    return cm_hip(ctx, e, "read error word");
  if (bits) hipMemset(ctx->d_err, 0, sizeof(unsigned));
  if (bits & ERR_BAD_GEOM) return cm_fail(ctx, CM_ERR_NOT_FOUND, "batch references an invalid body or geometry id");
  if (bits & ERR_CAPACITY) return cm_fail(ctx, CM_ERR_CAPACITY, "more kept pairs than the output capacity");
  if (bits & ERR_NO_ADJOINT)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "the adjoint of superquadric unions is not built (those pairs were skipped)");
  if (bits) return cm_fail(ctx, CM_ERR_DEVICE, "device error bits set");
  return CM_OK;
}

cm_status cm_geometry_create(cm_context* ctx, int32_t n, const int32_t* types, const float* params,
                             const int64_t* pt_offsets, const float* points, int32_t* out_ids) {
  if (!ctx || n < 0 || (n > 0 && (!types || !params || !out_ids))) return CM_ERR_INVALID_ARG;
  if (n == 0) return CM_OK;
  if (ctx->servers > 0) return cm_fail(ctx, CM_ERR_INVALID_ARG, "geometry is frozen while a server is running");
  for (int i = 0; i < n; ++i) {
    if (types[i] < CM_SPHERE || types[i] > CM_OPC)
      return cm_fail(ctx, CM_ERR_INVALID_ARG, "unknown geometry type");
    if ((types[i] == CM_POLYTOPE || types[i] == CM_SQ_UNION || types[i] == CM_OPC) && (!pt_offsets || !points))
      return cm_fail(ctx, CM_ERR_INVALID_ARG, "polytopes, superquadric unions and point clouds need points");
  }
  std::vector<HostMesh> meshes(n);
  std::vector<std::string> errs(n);
  std::atomic<int> bad{-1};
  const int nt = std::max(1, std::min<int>(16, int(std::thread::hardware_concurrency())));
  auto work = [&](int t) {
    for (int i = t; i < n; i += nt) {
      const float* pts = nullptr;
      int64_t np = 0;
      if (types[i] == CM_POLYTOPE || types[i] == CM_SQ_UNION || types[i] == CM_OPC) {
        np = pt_offsets[i + 1] - pt_offsets[i];
        pts = points + 3 * pt_offsets[i];
      }
      if (!build_mesh(types[i], params + 4 * i, pts, np, &meshes[i], &errs[i])) {
        int exp = -1;
        bad.compare_exchange_strong(exp, i);
      }
    }
  };
  if (n >= 64 && nt > 1) {
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t) th.emplace_back(work, t);
    for (auto& x : th) x.join();
  } else {
    for (int i = 0; i < n; ++i) {
      const float* pts = nullptr;
      int64_t np = 0;
      if (types[i] == CM_POLYTOPE || types[i] == CM_SQ_UNION || types[i] == CM_OPC) { np = pt_offsets[i + 1] - pt_offsets[i]; pts = points + 3 * pt_offsets[i]; }
      if (!build_mesh(types[i], params + 4 * i, pts, np, &meshes[i], &errs[i])) { bad = i; break; }
    }
  }
  if (bad >= 0) return cm_fail(ctx, CM_ERR_GEOMETRY, "geometry " + std::to_string(int(bad)) + ": " + errs[bad]);
  hipSetDevice(ctx->device);
  auto& h = ctx->h;
  for (int i = 0; i < n; ++i) {
    const HostMesh& m = meshes[i];
    GeomRec r;
    std::memset(&r, 0, sizeof(r));
    r.type = m.type;
    r.nv = int32_t(m.v.size() / 3);
    r.ne = int32_t(m.e.size() / 2);
    r.nf = int32_t(m.f.size() / 3);
    r.v_off = int32_t(h.vx.size());
    r.e_off = int32_t(h.e0.size());
    r.f_off = int32_t(h.fnx.size());
    for (int k = 0; k < 4; ++k) r.p[k] = m.p[k];
    r.bound_r = m.bound_r;
    for (int v = 0; v < r.nv; ++v) { h.vx.push_back(m.vd[3 * v]); h.vy.push_back(m.vd[3 * v + 1]); h.vz.push_back(m.vd[3 * v + 2]); }
    for (int e = 0; e < r.ne; ++e) { h.e0.push_back(m.e[2 * e]); h.e1.push_back(m.e[2 * e + 1]); }
    for (int f = 0; f < r.nf; ++f) {
      h.fnx.push_back(m.pd[4 * f]); h.fny.push_back(m.pd[4 * f + 1]);
      h.fnz.push_back(m.pd[4 * f + 2]); h.fo.push_back(m.pd[4 * f + 3]);
      h.f0.push_back(m.f[3 * f]); h.f1.push_back(m.f[3 * f + 1]); h.f2.push_back(m.f[3 * f + 2]);
    }
    ctx->maxV = std::max(ctx->maxV, r.nv);
    ctx->maxE = std::max(ctx->maxE, r.ne);
    ctx->maxF = std::max(ctx->maxF, r.nf);
    if (r.type == CM_SQ_UNION || r.type == CM_OPC) ctx->has_sq = true;   // extended primitives
    out_ids[i] = int32_t(h.recs.size());
    h.recs.push_back(r);
  }
  ctx->geom_version++;
  ctx->drop_graphs();
  return ctx_upload_tables(ctx);
}

// Destroy geometries: their records keep their ids with a negative type (a
// batch that references them is flagged CM_ERR_NOT_FOUND), the vertex / edge
// / plane pools are repacked without them (vertex offsets of the remaining
// geometries change), the context maxima are recomputed and the device
// tables re-uploaded.  All ids are checked before anything changes.
cm_status cm_geometry_destroy(cm_context* ctx, const int32_t* ids, int32_t n) {
  if (!ctx || n < 0 || (n > 0 && !ids)) return CM_ERR_INVALID_ARG;
  if (n == 0) return CM_OK;
  if (ctx->servers > 0) return cm_fail(ctx, CM_ERR_INVALID_ARG, "geometry is frozen while a server is running");
  auto& h = ctx->h;
  std::vector<char> kill(h.recs.size(), 0);
  for (int i = 0; i < n; ++i) {
    const int32_t id = ids[i];
    if (id < 0 || id >= int32_t(h.recs.size()) || h.recs[id].type < 0)
      return cm_fail(ctx, CM_ERR_NOT_FOUND, "no such geometry: " + std::to_string(id));
    kill[id] = 1;
  }
  hipSetDevice(ctx->device);
  // the tables may still be read by queued work
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return cm_hip(ctx, e, "synchronize before destroy");
  CmPools np;
  np.recs = h.recs;
  ctx->maxV = ctx->maxE = ctx->maxF = 0;
  ctx->has_sq = false;
  for (size_t g = 0; g < h.recs.size(); ++g) {
    GeomRec& r = np.recs[g];
    if (kill[g] || r.type < 0) {
      std::memset(&r, 0, sizeof(r));
      r.type = -1;
      continue;
    }
    const GeomRec& o = h.recs[g];
    r.v_off = int32_t(np.vx.size());
    r.e_off = int32_t(np.e0.size());
    r.f_off = int32_t(np.fnx.size());
    np.vx.insert(np.vx.end(), h.vx.begin() + o.v_off, h.vx.begin() + o.v_off + o.nv);
    np.vy.insert(np.vy.end(), h.vy.begin() + o.v_off, h.vy.begin() + o.v_off + o.nv);
    np.vz.insert(np.vz.end(), h.vz.begin() + o.v_off, h.vz.begin() + o.v_off + o.nv);
    np.e0.insert(np.e0.end(), h.e0.begin() + o.e_off, h.e0.begin() + o.e_off + o.ne);
    np.e1.insert(np.e1.end(), h.e1.begin() + o.e_off, h.e1.begin() + o.e_off + o.ne);
    np.fnx.insert(np.fnx.end(), h.fnx.begin() + o.f_off, h.fnx.begin() + o.f_off + o.nf);
    np.fny.insert(np.fny.end(), h.fny.begin() + o.f_off, h.fny.begin() + o.f_off + o.nf);
    np.fnz.insert(np.fnz.end(), h.fnz.begin() + o.f_off, h.fnz.begin() + o.f_off + o.nf);
    np.fo.insert(np.fo.end(), h.fo.begin() + o.f_off, h.fo.begin() + o.f_off + o.nf);
    np.f0.insert(np.f0.end(), h.f0.begin() + o.f_off, h.f0.begin() + o.f_off + o.nf);
    np.f1.insert(np.f1.end(), h.f1.begin() + o.f_off, h.f1.begin() + o.f_off + o.nf);
    np.f2.insert(np.f2.end(), h.f2.begin() + o.f_off, h.f2.begin() + o.f_off + o.nf);
    ctx->maxV = std::max(ctx->maxV, r.nv);
    ctx->maxE = std::max(ctx->maxE, r.ne);
    ctx->maxF = std::max(ctx->maxF, r.nf);
    if (r.type == CM_SQ_UNION || r.type == CM_OPC) ctx->has_sq = true;
  }
  h = std::move(np);
  ctx->geom_version++;
  ctx->drop_graphs();
  return ctx_upload_tables(ctx);
}

cm_status cm_geometry_info(cm_context* ctx, int32_t id, cm_geometry_info_t* out) {
  if (!ctx || !out) return CM_ERR_INVALID_ARG;
  if (id < 0 || id >= int32_t(ctx->h.recs.size()) || ctx->h.recs[id].type < 0)
    return cm_fail(ctx, CM_ERR_NOT_FOUND, "no such geometry");
  const GeomRec& r = ctx->h.recs[id];
  // a superquadric union keeps its primitives in the plane pool: no faces
  out->type = r.type; out->n_vertices = r.nv; out->n_edges = r.ne;
  out->n_faces = (r.type == CM_SQ_UNION || r.type == CM_OPC) ? 0 : r.nf;
  out->vertex_offset = r.v_off; out->bound_radius = r.bound_r;
  return CM_OK;
}

cm_status cm_geometry_mesh(cm_context* ctx, int32_t id, float* vertices, int32_t* edges, int32_t* faces) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  if (id < 0 || id >= int32_t(ctx->h.recs.size()) || ctx->h.recs[id].type < 0)
    return cm_fail(ctx, CM_ERR_NOT_FOUND, "no such geometry");
  const GeomRec& r = ctx->h.recs[id];
  const auto& h = ctx->h;
  if (vertices) for (int v = 0; v < r.nv; ++v) {
    vertices[3 * v] = float(h.vx[r.v_off + v]);
    vertices[3 * v + 1] = float(h.vy[r.v_off + v]);
    vertices[3 * v + 2] = float(h.vz[r.v_off + v]);
  }
  if (edges) for (int e = 0; e < r.ne; ++e) { edges[2 * e] = h.e0[r.e_off + e]; edges[2 * e + 1] = h.e1[r.e_off + e]; }
  if (faces && r.type != CM_SQ_UNION && r.type != CM_OPC) for (int f = 0; f < r.nf; ++f) {
    faces[3 * f] = h.f0[r.f_off + f]; faces[3 * f + 1] = h.f1[r.f_off + f]; faces[3 * f + 2] = h.f2[r.f_off + f];
  }
  return CM_OK;
}

int32_t cm_geometry_count(cm_context* ctx) { return ctx ? int32_t(ctx->h.recs.size()) : -1; }
int32_t cm_vertex_pool_size(cm_context* ctx) { return ctx ? int32_t(ctx->h.vx.size()) : -1; }

}  // extern "C"

// ---------------------------------------------------------------- forward helpers

cm_status resolve_params(cm_context* ctx, const cm_params* prm, ParamsDev* pd) {
  if (!prm) return cm_fail(ctx, CM_ERR_INVALID_ARG, "null params");
  if (!(prm->tau > 0.f) || !std::isfinite(prm->tau)) return cm_fail(ctx, CM_ERR_INVALID_ARG, "tau must be > 0");
  if (prm->K < 1 || prm->K > CM_MAX_K) return cm_fail(ctx, CM_ERR_INVALID_ARG, "K must be in 1..32");
  if (prm->flags & ~(CM_FLAG_NO_EE | CM_FLAG_ONE_SIDED_VS | CM_FLAG_SAFEGUARD))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "unknown flags");
  if (prm->refine_steps < 0 || prm->refine_steps > CM_MAX_REFINE)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "refine_steps must be in 0..8");
  if (prm->refine_steps > 0 && prm->K > 16)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "witness sphere tracing needs K <= 16");
  const bool presel = prm->presel_vertices != 0 || prm->presel_edges != 0;
  if (presel && (prm->presel_vertices < 1 || prm->presel_vertices > CM_MAX_PRESEL || prm->presel_edges < 1 ||
                 prm->presel_edges > CM_MAX_PRESEL))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "presel_vertices / presel_edges must both be in 1..64 (or both 0)");
  if ((prm->flags & CM_FLAG_SAFEGUARD) && !presel)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "CM_FLAG_SAFEGUARD needs pre-selection");
  pd->tau = double(prm->tau);
  pd->inv_tau = 1.0 / pd->tau;
  pd->c_log2 = kLog2e / pd->tau;
  pd->tl = pd->tau * kLn2;
  pd->lam = prm->lambda_reg < 0.f ? 0.01 : double(prm->lambda_reg);
  if (!(pd->lam > 0.0)) return cm_fail(ctx, CM_ERR_INVALID_ARG, "lambda_reg must be > 0");
  pd->eps_n = prm->eps_n < 0.f ? pd->tau * pd->tau : double(prm->eps_n);
  if (!(pd->eps_n > 0.0)) return cm_fail(ctx, CM_ERR_INVALID_ARG, "eps_n must be > 0");
  pd->margin = prm->cull_margin < 0.f ? 10.0f * prm->tau : prm->cull_margin;
  pd->eps_tied = prm->eps_n < 0.f ? 1 : 0;
  pd->K = prm->K;
  pd->flags = prm->flags;
  pd->presel_v = presel ? prm->presel_vertices : 0;
  pd->presel_e = presel ? prm->presel_edges : 0;
  pd->sq = ctx->has_sq ? 1 : 0;
  pd->refine = prm->refine_steps;
  return CM_OK;
}

cm_status resolve_batch(cm_context* ctx, const cm_batch* b, BatchDev* bd) {
  if (!b) return cm_fail(ctx, CM_ERR_INVALID_ARG, "null batch");
  if (b->n_scenes < 0 || b->n_bodies < 0) return cm_fail(ctx, CM_ERR_INVALID_ARG, "negative sizes");
  if (b->n_scenes > 0 && (!b->body_offsets || !b->body_geom || !b->pose))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "batch arrays missing");
  if ((b->cand_offsets == nullptr) != (b->cand_pairs == nullptr) && b->n_cand > 0)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "cand_offsets and cand_pairs go together");
  if (b->cand_offsets && b->n_cand < 0) return cm_fail(ctx, CM_ERR_INVALID_ARG, "negative n_cand");
  if (ctx->h.recs.empty()) return cm_fail(ctx, CM_ERR_INVALID_ARG, "no geometry created");
  bd->n_scenes = b->n_scenes; bd->n_bodies = b->n_bodies; bd->n_cand = b->n_cand;
  bd->body_offsets = b->body_offsets; bd->body_geom = b->body_geom; bd->pose = b->pose;
  bd->cand_offsets = b->cand_offsets; bd->cand_pairs = b->cand_offsets ? b->cand_pairs : nullptr;
  return CM_OK;
}

cm_status resolve_out(cm_context* ctx, const cm_manifold* o, OutDev* od) {
  if (!o || !o->n_pairs || !o->pair_offsets || o->capacity < 0)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "bad manifold outputs");
  if (o->capacity > 0 && (!o->pairs || !o->point || !o->normal || !o->dist || !o->weight))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "manifold output arrays missing");
  if (o->tape && (reinterpret_cast<uintptr_t>(o->tape) & 15))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "the tape must be 16-byte aligned");
  od->capacity = o->capacity; od->n_pairs = o->n_pairs; od->pair_offsets = o->pair_offsets; od->pairs = o->pairs;
  od->point = o->point; od->normal = o->normal; od->dist = o->dist; od->weight = o->weight;
  od->tape = static_cast<char*>(o->tape);
  od->tape_bytes = o->tape ? o->tape_bytes : 0;
  return CM_OK;
}

int kmax_for(int K) { return K <= 8 ? 8 : (K <= 16 ? 16 : 32); }

static bool capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

cm_status ctx_order(cm_context* ctx, hipStream_t st) {
  if (!ctx->order_pending || st == ctx->last_stream || capturing(st)) return CM_OK;
  return cm_hip(ctx, hipStreamWaitEvent(st, ctx->order_ev, 0), "cross-stream ordering");
}

void ctx_mark(cm_context* ctx, hipStream_t st) {
  if (capturing(st)) return;
  if (!ctx->order_ev && hipEventCreateWithFlags(&ctx->order_ev, hipEventDisableTiming) != hipSuccess) {
    ctx->order_ev = nullptr;
    return;
  }
  if (hipEventRecord(ctx->order_ev, st) == hipSuccess) {
    ctx->last_stream = st;
    ctx->order_pending = true;
  }
}

cm_status ctx_broadphase(cm_context* ctx, const BatchDev& bd, const ParamsDev& pd, const OutDev& od, hipStream_t st) {
  const Tables tb = ctx_tables(ctx);
  const size_t tiles = size_t(bd.n_scenes) / 1024 + 2;
  hipError_t e = ctx_ensure(ctx, reinterpret_cast<void**>(&ctx->d_tile_sums), &ctx->tile_cap, tiles * sizeof(int));
  if (e != hipSuccess) return cm_hip(ctx, e, "tile sums");
  return cm_hip(ctx, launch_broadphase(tb, bd, pd.margin, od, ctx->d_tile_sums, ctx->d_err, st), "broadphase launch");
}

cm_status ctx_prepare_fwd(cm_context* ctx, const BatchDev& bd, const ParamsDev& pd, const OutDev& od, int block,
                          bool dynamic, FwdLaunch* f) {
  f->tb = ctx_tables(ctx);
  f->bt = bd; f->prm = pd; f->out = od;
  f->maxV = std::max(ctx->maxV, 1); f->maxE = std::max(ctx->maxE, 1); f->maxF = std::max(ctx->maxF, 1);
  f->block = block;
  f->kmax = kmax_for(pd.K);
  f->order = nullptr; f->range = nullptr; f->queue = dynamic ? reinterpret_cast<int*>(1) : nullptr;   // dispatch hint
  // (dynamic: the caller gives the launch a work-queue counter; the grid and
  // occupancy are those of the work-queue instantiation)
  const int lds = fwd_lds_bytes(f->maxV, f->maxE, f->maxF, block, f->kmax, pd.presel_v > 0);
  if (lds > 160 * 1024)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "the context's largest geometry needs " + std::to_string(lds) +
                                                " B of LDS for this forward (160 KiB per workgroup)");
  f->err = ctx->d_err;
  const int occ = fwd_place_edges(*f);
  f->queue = nullptr;
  f->grid = std::max(1, occ * ctx->num_cus);
  if (od.capacity > 0 && f->grid > od.capacity) f->grid = std::max(1, od.capacity);
  f->scratch_stride = fwd_scratch_floats(f->maxV, f->maxE);
  const size_t need = size_t(f->grid) * size_t(f->scratch_stride) * sizeof(float);
  hipError_t e = ctx_ensure(ctx, reinterpret_cast<void**>(&ctx->d_scratch), &ctx->scratch_cap, need);
  if (e != hipSuccess) return cm_hip(ctx, e, "forward scratch");
  f->scratch = ctx->d_scratch;
  return CM_OK;
}

extern "C" cm_status cm_collide(cm_context* ctx, const cm_batch* batch, const cm_params* prm, cm_manifold* out,
                                void* stream) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  ParamsDev pd; BatchDev bd; OutDev od;
  cm_status s;
  if ((s = resolve_params(ctx, prm, &pd)) != CM_OK) return s;
  if ((s = resolve_batch(ctx, batch, &bd)) != CM_OK) return s;
  if ((s = resolve_out(ctx, out, &od)) != CM_OK) return s;
  hipSetDevice(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = ctx_order(ctx, st)) != CM_OK) return s;
  FwdLaunch f;
  // workgroups take pairs from a work queue (an atomic counter) so that
  // uneven pair costs do not leave a tail; traced witnesses keep the
  // static order
  const bool dyn = pd.refine == 0;
  if (od.capacity > 0 && (s = ctx_prepare_fwd(ctx, bd, pd, od, 256, dyn, &f)) != CM_OK) return s;
  if (od.tape && od.capacity > 0 && !tape_layout(od.tape, od.tape_bytes, od.capacity, pd.K, &f.tape))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "the tape is smaller than cm_tape_bytes gives for this capacity and K");
  if (od.capacity > 0 && dyn) {
    hipError_t e = ctx_ensure(ctx, reinterpret_cast<void**>(&ctx->d_fwd_queue), &ctx->fwd_queue_cap, 256);
    if (e != hipSuccess) return cm_hip(ctx, e, "forward work queue");
    f.queue = ctx->d_fwd_queue;
  }
  hipEvent_t t0 = timer_begin(ctx, st);
  if ((s = ctx_broadphase(ctx, bd, pd, od, st)) != CM_OK) return s;
  timer_end(ctx, CM_TIMER_BROADPHASE, t0, st);
  if (od.capacity > 0) {
    if (f.tape.base && (s = cm_hip(ctx, launch_tape_reset(f.tape, st), "tape reset")) != CM_OK) return s;
    if (f.queue && (s = cm_hip(ctx, launch_counter_reset(f.queue, st), "work queue reset")) != CM_OK) return s;
    t0 = timer_begin(ctx, st);
    if ((s = cm_hip(ctx, launch_collide_fwd(f, st), "collide launch")) != CM_OK) return s;
    timer_end(ctx, CM_TIMER_FORWARD, t0, st);
  }
  ctx_mark(ctx, st);
  return CM_OK;
}

// The forward of cm_collide with every workspace in the static device array
// (no allocation): tile sums at the array's start, then one scratch slot per
// workgroup of the pair kernel, whose grid is cut to the slots that fit.  All
// checks run before the first launch.
extern "C" cm_status cm_collide_noalloc(cm_context* ctx, const cm_batch* batch, const cm_params* prm,
                                        cm_manifold* out, void* stream) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  ParamsDev pd; BatchDev bd; OutDev od;
  cm_status s;
  if ((s = resolve_params(ctx, prm, &pd)) != CM_OK) return s;
  if ((s = resolve_batch(ctx, batch, &bd)) != CM_OK) return s;
  if ((s = resolve_out(ctx, out, &od)) != CM_OK) return s;
  if (!ctx->noalloc_scratch) return cm_fail(ctx, CM_ERR_DEVICE, ctx->noalloc_error);
  if (od.tape) return cm_fail(ctx, CM_ERR_INVALID_ARG, "the allocation-free forward records no tape");
  const size_t cap = CM_NOALLOC_SCRATCH_BYTES;
  const size_t tiles = size_t(bd.n_scenes) / 1024 + 2;
  const size_t tile_bytes = (tiles * sizeof(int) + 255) & ~size_t(255);
  if (tile_bytes > cap)
    return cm_fail(ctx, CM_ERR_CAPACITY, "the broadphase tile sums of " + std::to_string(bd.n_scenes) +
                                             " scenes need " + std::to_string(tile_bytes) + " B, beyond the " +
                                             std::to_string(cap) + " B static workspace");
  char* base = static_cast<char*>(ctx->noalloc_scratch);
  hipSetDevice(ctx->device);
  FwdLaunch f;
  f.tb = ctx_tables(ctx);
  f.bt = bd; f.prm = pd; f.out = od;
  f.maxV = std::max(ctx->maxV, 1); f.maxE = std::max(ctx->maxE, 1); f.maxF = std::max(ctx->maxF, 1);
  f.block = 256;
  f.kmax = kmax_for(pd.K);
  f.order = nullptr; f.range = nullptr; f.queue = nullptr; f.err = ctx->d_err;
  f.scratch_stride = fwd_scratch_floats(f.maxV, f.maxE);
  f.scratch = reinterpret_cast<float*>(base + tile_bytes);
  f.grid = 1;
  if (od.capacity > 0) {
    const int lds = fwd_lds_bytes(f.maxV, f.maxE, f.maxF, f.block, f.kmax, pd.presel_v > 0);
    if (lds > 160 * 1024)
      return cm_fail(ctx, CM_ERR_INVALID_ARG, "the context's largest geometry needs " + std::to_string(lds) +
                                                  " B of LDS for this forward (160 KiB per workgroup)");
    const size_t slot = size_t(f.scratch_stride) * sizeof(float);
    const size_t slots = (cap - tile_bytes) / slot;
    if (slots < 1)
      return cm_fail(ctx, CM_ERR_CAPACITY, "one workgroup of this forward needs " + std::to_string(slot) +
                                               " B of scratch (largest geometry: " + std::to_string(ctx->maxE) +
                                               " edges), beyond the " + std::to_string(cap - tile_bytes) +
                                               " B left in the static workspace");
    const int occ = fwd_place_edges(f);
    f.grid = int(std::min<size_t>(size_t(std::max(1, occ * ctx->num_cus)), slots));
    f.grid = std::max(1, std::min(f.grid, od.capacity));
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = cm_hip(ctx, launch_broadphase(f.tb, bd, pd.margin, od, reinterpret_cast<int*>(base), ctx->d_err, st),
                  "broadphase launch")) != CM_OK)
    return s;
  if (od.capacity == 0) return CM_OK;
  return cm_hip(ctx, launch_collide_fwd(f, st), "collide launch");
}

extern "C" cm_status cm_ee_witness(cm_context* ctx, const float* edges, int64_t n, float tau, float lambda_reg,
                                   int32_t mode, float* out, void* stream) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  if (n < 0) return cm_fail(ctx, CM_ERR_INVALID_ARG, "negative query count");
  if (mode != CM_EE_SMOOTH && mode != CM_EE_HARD) return cm_fail(ctx, CM_ERR_INVALID_ARG, "unknown mode");
  if (mode == CM_EE_SMOOTH && (!(tau > 0.f) || !std::isfinite(tau)))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "tau must be > 0");
  if (n == 0) return CM_OK;
  if (!edges || !out) return cm_fail(ctx, CM_ERR_INVALID_ARG, "null buffer");
  const uintptr_t e0 = reinterpret_cast<uintptr_t>(edges), e1 = e0 + 12 * 4 * uint64_t(n);
  const uintptr_t o0 = reinterpret_cast<uintptr_t>(out), o1 = o0 + 9 * 4 * uint64_t(n);
  if (e0 < o1 && o0 < e1) return cm_fail(ctx, CM_ERR_INVALID_ARG, "edges and out overlap");
  ParamsDev pd{};
  const double t = mode == CM_EE_SMOOTH ? double(tau) : 1.0;
  pd.tau = t;
  pd.inv_tau = 1.0 / t;
  pd.c_log2 = kLog2e / t;
  pd.tl = t * kLn2;
  pd.lam = lambda_reg < 0.f ? 0.01 : double(lambda_reg);
  if (!(pd.lam > 0.0) || !std::isfinite(pd.lam)) return cm_fail(ctx, CM_ERR_INVALID_ARG, "lambda_reg must be > 0");
  hipSetDevice(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t t0 = timer_begin(ctx, st);
  cm_status s = cm_hip(ctx, launch_ee_witness(edges, n, pd, mode == CM_EE_HARD, out, st), "ee witness launch");
  if (s != CM_OK) return s;
  timer_end(ctx, CM_TIMER_EE_WITNESS, t0, st);
  return CM_OK;
}

hipEvent_t timer_begin(cm_context* ctx, hipStream_t st) {
  if (!ctx->timing) return nullptr;
  hipEvent_t ev = nullptr;
  if (!ctx->spare_events.empty()) {
    ev = ctx->spare_events.back();
    ctx->spare_events.pop_back();
  } else if (hipEventCreate(&ev) != hipSuccess) {
    return nullptr;
  }
  if (hipEventRecord(ev, st) != hipSuccess) {
    ctx->spare_events.push_back(ev);
    return nullptr;
  }
  return ev;
}

void timer_end(cm_context* ctx, int timer, hipEvent_t start, hipStream_t st) {
  if (!start) return;
  hipEvent_t ev = timer_begin(ctx, st);
  if (!ev) {
    ctx->spare_events.push_back(start);
    return;
  }
  ctx->timers[timer].pending.push_back({start, ev});
}

extern "C" cm_status cm_set_kernel_timing(cm_context* ctx, int32_t enable) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  hipSetDevice(ctx->device);
  for (auto& t : ctx->timers) {
    for (auto& pr : t.pending) {
      (void)hipEventSynchronize(pr.second);
      ctx->spare_events.push_back(pr.first);
      ctx->spare_events.push_back(pr.second);
    }
    t.pending.clear();
    t.ms = 0.0;
    t.launches = 0;
  }
  ctx->timing = enable != 0;
  return CM_OK;
}

extern "C" cm_status cm_kernel_time(cm_context* ctx, int32_t timer, double* total_ms, int64_t* launches) {
  if (!ctx || timer < 0 || timer >= CM_N_TIMERS) return CM_ERR_INVALID_ARG;
  hipSetDevice(ctx->device);
  auto& t = ctx->timers[timer];
  for (auto& pr : t.pending) {
    hipError_t e = hipEventSynchronize(pr.second);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
    if (e != hipSuccess) return cm_hip(ctx, e, "kernel timing");
    t.ms += ms;
    t.launches += 1;
    ctx->spare_events.push_back(pr.first);
    ctx->spare_events.push_back(pr.second);
  }
  t.pending.clear();
  if (total_ms) *total_ms = t.ms;
  if (launches) *launches = t.launches;
  return CM_OK;
}

// Entries of the adjoint tape's index pool (4 B each): CM_ADJOINT_TAPE
// (0 turns the tape off: the adjoint recomputes the whole forward per pair),
// default 2^28.
static long long tape_pool_entries() {
  const char* v = std::getenv("CM_ADJOINT_TAPE");
  if (!v || !*v) return 1LL << 28;
  const long long n = std::atoll(v);
  return n <= 0 ? 0 : std::min(n, (1LL << 31) - 1);
}

// The pool the backward records into on its own: no more entries than every
// pair of the capacity could fill with its candidates' indices.
static long long tape_default_pool(const cm_context* ctx, long long capacity) {
  const long long most = capacity * (2LL * ctx->maxV + 2LL * ctx->maxE * ctx->maxE);
  return std::min(tape_pool_entries(), std::max(most, 1LL));
}

extern "C" cm_status cm_tape_bytes(cm_context* ctx, int32_t capacity, int32_t K, int64_t pool_entries, int64_t* bytes) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  if (!bytes || capacity < 0 || K < 1 || K > CM_MAX_K)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "null result, negative capacity or K outside 1..32");
  long long pool = pool_entries > 0 ? (long long)pool_entries : tape_default_pool(ctx, capacity);
  pool = std::max(pool, 2LL);
  *bytes = 256 + tape_records_bytes(capacity, K) + 4 * pool;
  return CM_OK;
}

extern "C" cm_status cm_collide_backward(cm_context* ctx, const cm_batch* batch, const cm_params* prm,
                                         const cm_manifold* fwd, const cm_cotangent* cot, cm_grads* out,
                                         void* stream) {
  if (!ctx) return CM_ERR_INVALID_ARG;
  ParamsDev pd; BatchDev bd; OutDev od;
  cm_status s;
  if ((s = resolve_params(ctx, prm, &pd)) != CM_OK) return s;
  if ((s = resolve_batch(ctx, batch, &bd)) != CM_OK) return s;
  if ((s = resolve_out(ctx, fwd, &od)) != CM_OK) return s;
  if (!cot || !out) return cm_fail(ctx, CM_ERR_INVALID_ARG, "null cotangent or gradient struct");
  if ((pd.presel_v > 0 || pd.refine > 0) && (ctx->maxV > 4096 || ctx->maxE > 4096))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "the pre-selection and sphere-tracing adjoints need at most 4096 vertices and edges per body");
  hipSetDevice(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((s = ctx_order(ctx, st)) != CM_OK) return s;
  const long long pool = (long long)ctx->h.vx.size();
  const long long G = (long long)ctx->h.recs.size();
  hipError_t e;
  if (out->g_pose && (e = hipMemsetAsync(out->g_pose, 0, sizeof(float) * 6 * size_t(bd.n_bodies), st)) != hipSuccess)
    return cm_hip(ctx, e, "zero g_pose");
  if (out->g_vertices && (e = hipMemsetAsync(out->g_vertices, 0, sizeof(float) * 3 * size_t(pool), st)) != hipSuccess)
    return cm_hip(ctx, e, "zero g_vertices");
  if (out->g_params && (e = hipMemsetAsync(out->g_params, 0, sizeof(float) * 4 * size_t(G), st)) != hipSuccess)
    return cm_hip(ctx, e, "zero g_params");
  if (out->g_tau && (e = hipMemsetAsync(out->g_tau, 0, sizeof(float), st)) != hipSuccess)
    return cm_hip(ctx, e, "zero g_tau");
  if (od.capacity == 0) {
    ctx_mark(ctx, st);
    return CM_OK;
  }
  BwdLaunch b;
  b.f.tb = ctx_tables(ctx);
  b.f.bt = bd; b.f.prm = pd; b.f.out = od;
  b.f.maxV = std::max(ctx->maxV, 1); b.f.maxE = std::max(ctx->maxE, 1); b.f.maxF = std::max(ctx->maxF, 1);
  b.f.block = 256;
  b.f.kmax = kmax_for(pd.K);
  b.f.order = nullptr; b.f.range = nullptr; b.f.queue = nullptr; b.f.err = ctx->d_err;
  b.cot = CotDev{cot->g_point, cot->g_normal, cot->g_dist, cot->g_weight};
  b.gr = GradDev{out->g_pose, out->g_vertices, out->g_params, out->g_tau, pool};
  const int lds = bwd_lds_bytes(b.f.maxV, b.f.maxE, b.f.maxF, 256, pd.presel_v > 0);
  if (lds > 160 * 1024)
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "the context's largest geometry needs " + std::to_string(lds) +
                                                " B of LDS for this adjoint (160 KiB per workgroup)");
  int occ = bwd_place(b);
  // When LDS holds one 256-thread workgroup per CU (one wave per SIMD), a
  // 512-thread one brings two waves per SIMD to the same LDS (the full
  // method on the basic primitives has that variant)
  if (pd.presel_v == 0 && !pd.sq && pd.refine == 0 &&
      bwd_lds_bytes(b.f.maxV, b.f.maxE, b.f.maxF, 512, false) <= 160 * 1024) {
    BwdLaunch b5 = b;
    b5.f.block = 512;
    b5.f.hi_occ = 0;
    b5.f.edges_out = 0;
    const int occ5 = bwd_occupancy(b5);
    if (occ5 * 8 > occ * 4) { b = b5; occ = occ5; }
  }
  b.f.grid = std::max(1, occ * ctx->num_cus);
  if (b.f.grid > od.capacity) b.f.grid = std::max(1, od.capacity);
  b.f.scratch_stride = fwd_scratch_floats(b.f.maxV, b.f.maxE);
  // The adjoint's tape: the forward kernel (at its own occupancy) records per
  // kept pair s_[k], the SoftSort row sums and the candidates within the
  // adjoint's window, so the adjoint kernel skips the forward's candidate
  // pass; a pair whose list no longer fits the pool is recomputed whole.
  // A tape recorded by the caller's forward is used as it is; without one
  // the forward kernel records it here, into the context's workspace.
  TapeDev tv;
  if (od.tape && !tape_layout(od.tape, od.tape_bytes, od.capacity, pd.K, &tv))
    return cm_fail(ctx, CM_ERR_INVALID_ARG, "the tape is smaller than cm_tape_bytes gives for this capacity and K");
  const long long pool_cap = od.tape ? 0 : tape_default_pool(ctx, od.capacity);
  FwdLaunch f1;
  const bool dyn1 = pd.refine == 0;   // the tape forward takes pairs from a work queue too
  if (pool_cap > 0 && (s = ctx_prepare_fwd(ctx, bd, pd, od, 256, dyn1, &f1)) != CM_OK) return s;
  if (pool_cap > 0 && dyn1) {
    if ((e = ctx_ensure(ctx, reinterpret_cast<void**>(&ctx->d_fwd_queue), &ctx->fwd_queue_cap, 256)) != hipSuccess)
      return cm_hip(ctx, e, "forward work queue");
    if ((e = launch_counter_reset(ctx->d_fwd_queue, st)) != hipSuccess) return cm_hip(ctx, e, "work queue reset");
    f1.queue = ctx->d_fwd_queue;
  }
  const size_t need = size_t(b.f.grid) * size_t(b.f.scratch_stride) * sizeof(float);
  if ((e = ctx_ensure(ctx, reinterpret_cast<void**>(&ctx->d_scratch), &ctx->scratch_cap, need)) != hipSuccess)
    return cm_hip(ctx, e, "backward scratch");
  b.f.scratch = ctx->d_scratch;
  // The workspace's first 256 B hold the tape's pool counter (byte 0) and
  // the adjoint's work-queue counter (byte 128); the recorded tape follows.
  const long long bytes = 256 + (pool_cap > 0 ? tape_records_bytes(od.capacity, pd.K) + 4 * pool_cap : 0);
  if ((e = ctx_ensure(ctx, &ctx->d_bwd, &ctx->bwd_cap, size_t(bytes))) != hipSuccess)
    return cm_hip(ctx, e, "adjoint workspace");
  int* queue = reinterpret_cast<int*>(static_cast<char*>(ctx->d_bwd) + 128);
  if ((e = launch_counter_reset(queue, st)) != hipSuccess) return cm_hip(ctx, e, "work queue reset");
  b.f.queue = queue;
  if (pool_cap > 0) {
    tape_layout(static_cast<char*>(ctx->d_bwd), bytes, od.capacity, pd.K, &tv);
    if ((e = launch_tape_reset(tv, st)) != hipSuccess) return cm_hip(ctx, e, "tape reset");
    f1.scratch = ctx->d_scratch;   // the ensures above may have moved it
    f1.tape = tv;
    f1.tape.skip_out = 1;
  }
  b.f.tape = tv;
  b.f.tape.pool_used = nullptr;
  hipEvent_t t0 = timer_begin(ctx, st);
  if (pool_cap > 0 && (s = cm_hip(ctx, launch_collide_fwd(f1, st), "adjoint tape launch")) != CM_OK) return s;
  if ((s = cm_hip(ctx, launch_collide_bwd(b, st), "backward launch")) != CM_OK) return s;
  timer_end(ctx, CM_TIMER_BACKWARD, t0, st);
  ctx_mark(ctx, st);
  return CM_OK;
}
