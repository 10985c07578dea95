// Host-visible launch interface of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "cm_internal.h"

namespace cm {

// Per-pair record the forward kernel leaves for the adjoint (the adjoint's
// tape), tape_stride(K) bytes per kept pair: int32 count of the candidates
// within the adjoint's window, int32 form (0: none recorded, the pool was
// full; 1: their indices, int32, in three ascending runs: vertex-SDF
// candidates, edge-edge witnesses 1, witnesses 2; 2: a mask of one bit per
// candidate, 64-bit words), int64 offset of that list or mask in the pool
// (4-byte entries), then the K top scores s_[k] and the K x 9 SoftSort row
// sums (float64).  Each pair takes the smaller form, carved from the pool by
// one atomic.
struct TapeDev {
  char* base = nullptr;     // null: no tape
  int* pool = nullptr;      // window indices of every recorded pair
  unsigned long long* pool_used = nullptr;   // entries carved so far (zeroed before the forward)
  long long pool_cap = 0;   // entries the pool holds
  int skip_out = 0;         // 1: the forward kernel writes the tape only, no manifold outputs
};
__host__ __device__ inline long long tape_stride(int K) { return 16LL + 80LL * K; }

struct FwdLaunch {
  Tables tb;
  BatchDev bt;
  ParamsDev prm;
  OutDev out;
  float* scratch;              // per-workgroup slots of scratch_stride floats
  long long scratch_stride;
  int maxV, maxE, maxF;        // LDS sizing (context-wide maxima)
  int edges_out = 0;           // 1: the edge arrays live in the scratch slot (fwd_place_edges)
  int hi_occ = 0;              // 1: the kernel's higher-occupancy variant (fwd_place_edges, bwd_place)
  TapeDev tape;                // optional adjoint tape written by the forward kernel
  const int* order;            // optional pair order (cost-sorted), or null
  const int* range;            // optional device int2 {start, count} into order, or null
  int* queue;                  // dynamic work-queue counter (zeroed), or null for static round robin
  unsigned* err;
  int grid, block, kmax;
};

// Scratch floats per workgroup: per edge pair the unsigned distance and the
// QP solution (al1, al2, ln con) in float64, then the float32 candidate
// scores and the int32 list of filtered candidates (both nvs + 2 nee long),
// then room for both bodies' edge arrays (float64, used when they do not fit
// in LDS), then per edge the float64 value-query shift of the other body
// along its segment (A's edges, then B's; see PairEngine::cull), then a copy
// of the candidate pass's group face masks (for the queries of filtered
// candidates, after the LDS that holds them has been reused).
__host__ __device__ inline long long scratch_edges_offset(int maxV, int maxE) {
  return 8LL * maxE * maxE + 2 * (2LL * maxE * maxE + 2LL * maxV) + 128;
}
__host__ __device__ inline long long scratch_shift_offset(int maxV, int maxE) {
  return scratch_edges_offset(maxV, maxE) + 24LL * maxE;
}
constexpr int kFaceMaskBytes = 72;   // a face mask: 8 words and a count
__host__ __device__ inline long long scratch_mask_offset(int maxV, int maxE) {
  return scratch_shift_offset(maxV, maxE) + 4LL * maxE;
}
__host__ __device__ inline long long fwd_scratch_floats(int maxV, int maxE) {
  return scratch_mask_offset(maxV, maxE) + 4LL * ((maxE + 7) / 8) * kFaceMaskBytes / 4;
}

struct CotDev {
  const float* gp;   // [3][cap*K]
  const float* gn;   // [3][cap*K]
  const float* gd;   // [cap*K]
  const float* gw;   // [cap*K]
};

struct GradDev {
  float* g_pose;       // [6][n_bodies]
  float* g_vertices;   // [3][pool]
  float* g_params;     // [4][n_geoms]
  float* g_tau;        // [1]
  long long pool;
};

struct BwdLaunch {
  FwdLaunch f;
  CotDev cot;
  GradDev gr;
};

int fwd_lds_bytes(int maxV, int maxE, int maxF, int block, int kmax, bool presel = false, bool edges_out = false);
int bwd_lds_bytes(int maxV, int maxE, int maxF, int block, bool presel = false, bool edges_out = false);
int bwd_occupancy(const BwdLaunch& b);
// Chooses the adjoint's edge placement (LDS or scratch slot) and register
// budget (b.f.edges_out, b.f.hi_occ) for the most waves per SIMD; returns
// the workgroups per CU of the choice.
int bwd_place(BwdLaunch& b);
hipError_t launch_collide_bwd(const BwdLaunch& b, hipStream_t st);
int fwd_occupancy(const FwdLaunch& f);
// Zeroes the tape's pool counter (a kernel, so it can sit in a captured graph).
hipError_t launch_tape_reset(const TapeDev& t, hipStream_t st);
// Zeroes a work-queue counter (a kernel, likewise).
hipError_t launch_counter_reset(int* counter, hipStream_t st);
// Byte layout of a caller-owned tape of `bytes` for `capacity` pairs at K:
// counter (256 B), records, pool.  Returns false when it is too small.
inline long long tape_records_bytes(long long capacity, int K) { return (capacity * tape_stride(K) + 255) & ~255LL; }
inline bool tape_layout(char* base, long long bytes, long long capacity, int K, TapeDev* t) {
  const long long hdr = tape_records_bytes(capacity, K);
  if (!base || bytes < 256 + hdr + 8) return false;
  t->pool_used = reinterpret_cast<unsigned long long*>(base);
  t->base = base + 256;
  t->pool = reinterpret_cast<int*>(base + 256 + hdr);
  t->pool_cap = (bytes - 256 - hdr) / 4;
  t->skip_out = 0;
  return true;
}
// Sets f.edges_out when keeping the edge arrays in the scratch slot lets more
// workgroups share a CU than keeping them in LDS (LDS-limited launches);
// returns the workgroups per CU of the chosen placement.
int fwd_place_edges(FwdLaunch& f);
hipError_t launch_broadphase(const Tables& tb, const BatchDev& bt, float margin, const OutDev& out, int* tile_sums,
                             unsigned* err, hipStream_t st);
hipError_t launch_collide_fwd(const FwdLaunch& f, hipStream_t st);

// Device address of the allocation-free entry point's static workspace
// (CM_NOALLOC_SCRATCH_BYTES) on `device`, looked up on the first call for that
// device and cached; later calls return the cached address and status.
hipError_t noalloc_scratch(int device, void** out);

// batched E-E witness points of independent edge pairs: edges [12][n],
// out [9][n] (float32 rows of stride n); hard = no smoothing
hipError_t launch_ee_witness(const float* edges, long long n, const ParamsDev& prm, bool hard, float* out,
                             hipStream_t st);

// fused path: size classes and cost order
constexpr int kNumClasses = 3;
constexpr int kNumBuckets = 48;
struct FusedWork {
  int* counts;    // [kNumClasses * kNumBuckets] histogram, then scatter cursors
  int* ranges;    // [kNumClasses][2] {start, count}
  int* queues;    // [kNumClasses] work-queue counters
  int* order;     // [capacity] pair indices, class-major, cost-descending
  int* keys;      // [capacity]
  int* sample;    // [capacity + 4] autotune sample order, then its range {0, n} and queue counter
};
hipError_t launch_fused_prepare(const Tables& tb, const BatchDev& bt, const OutDev& out, const int* class_maxE,
                                const FusedWork& w, hipStream_t st);
// autotuning sample: n pairs evenly strided over class c's cost order into
// sample[], with the device range {0, min(n, count)} in sample_range[2]
hipError_t launch_fused_sample(const FusedWork& w, int c, int n, int* sample, int* sample_range, hipStream_t st);

}  // namespace cm
