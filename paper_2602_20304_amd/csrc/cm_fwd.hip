// gfx950 kernels of the forward path: broadphase + per-scene compaction, and
// the per-pair contact manifold (vertex-SDF, all-pairs edge-edge, SoftSort
// K-manifold).
#include <hip/hip_runtime.h>

#include "cm_kernels.h"
#include "cm_pair.cuh"

namespace cm {

// ============================================================ broadphase
// Keep (a, b) iff d2 <= r*r, d2 = (dx*dx + dy*dy) + dz*dz, r = (Ra + Rb) + margin,
// every operation rounded to float32 with no contraction.
__device__ __attribute__((noinline)) bool bp_keep(const float* __restrict__ pose, int nb, int a, int b, float Ra,
                                                  float Rb, float margin) {
#pragma clang fp contract(off)
  const float dx = pose[4 * nb + b] - pose[4 * nb + a];
  const float dy = pose[5 * nb + b] - pose[5 * nb + a];
  const float dz = pose[6 * nb + b] - pose[6 * nb + a];
  const float d2 = (dx * dx + dy * dy) + dz * dz;
  const float r = (Ra + Rb) + margin;
  return d2 <= r * r;
}

__device__ __forceinline__ bool body_radius(const Tables& tb, const BatchDev& bt, int body, float& R,
                                            unsigned* err) {
  if (body < 0 || body >= bt.n_bodies) { atomicOr(err, ERR_BAD_GEOM); return false; }
  const int g = bt.body_geom[body];
  // a destroyed geometry keeps its id with a negative type
  if (g < 0 || g >= tb.n_geoms || tb.geoms[g].type < 0) { atomicOr(err, ERR_BAD_GEOM); return false; }
  R = tb.geoms[g].bound_r;
  return true;
}

// Visit every candidate pair of scene s in order, calling f(a, b, kept).
template <typename F>
__device__ __forceinline__ void scene_pairs(const Tables& tb, const BatchDev& bt, float margin, int s, unsigned* err,
                                            F&& f) {
  if (bt.cand_offsets) {
    const int c0 = bt.cand_offsets[s], c1 = bt.cand_offsets[s + 1];
    for (int c = c0; c < c1; ++c) {
      const int a = bt.cand_pairs[c], b = bt.cand_pairs[bt.n_cand + c];
      float Ra, Rb;
      if (!body_radius(tb, bt, a, Ra, err) || !body_radius(tb, bt, b, Rb, err)) continue;
      if (bp_keep(bt.pose, bt.n_bodies, a, b, Ra, Rb, margin)) f(a, b);
    }
  } else {
    const int b0 = bt.body_offsets[s], b1 = bt.body_offsets[s + 1];
    for (int a = b0; a < b1; ++a) {
      float Ra;
      if (!body_radius(tb, bt, a, Ra, err)) continue;
      for (int b = a + 1; b < b1; ++b) {
        float Rb;
        if (!body_radius(tb, bt, b, Rb, err)) continue;
        if (bp_keep(bt.pose, bt.n_bodies, a, b, Ra, Rb, margin)) f(a, b);
      }
    }
  }
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

// Per-scene kept counts + tile-local inclusive scan.  offsets[s+1] receives
// the tile-local inclusive sum, tile_sums[tile] the tile total.
__global__ __launch_bounds__(kScanThreads) void bp_count_scan(Tables tb, BatchDev bt, float margin,
                                                              int* __restrict__ offsets, int* __restrict__ tile_sums,
                                                              unsigned* err) {
  __shared__ int part[kScanThreads];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int acc = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int s = base + i;
    int c = 0;
    if (s < bt.n_scenes) scene_pairs(tb, bt, margin, s, err, [&](int, int) { ++c; });
    acc += c;
    v[i] = acc;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 1; o < kScanThreads; o <<= 1) {
    const int x = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += x;
    __syncthreads();
  }
  const int excl = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < bt.n_scenes) offsets[base + i + 1] = v[i] + excl;
  if (threadIdx.x == kScanThreads - 1) tile_sums[blockIdx.x] = part[kScanThreads - 1];
}

// Exclusive scan of tile sums (single block, loops for many tiles).
__global__ __launch_bounds__(1024) void scan_tiles(int* __restrict__ tile_sums, int n_tiles) {
  __shared__ int part[1024];
  int carry = 0;
  for (int base = 0; base < n_tiles; base += 1024) {
    const int i = base + threadIdx.x;
    const int x = i < n_tiles ? tile_sums[i] : 0;
    part[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int y = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += y;
      __syncthreads();
    }
    if (i < n_tiles) tile_sums[i] = carry + part[threadIdx.x] - x;
    const int tot = part[1023];
    __syncthreads();
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanThreads) void add_tile_offsets(int* __restrict__ offsets,
                                                                 const int* __restrict__ tile_sums, int n_scenes,
                                                                 int* __restrict__ n_pairs, int capacity,
                                                                 unsigned* err) {
  const int i = blockIdx.x * kScanThreads + threadIdx.x;
  if (i < n_scenes) offsets[i + 1] += tile_sums[i / kScanTile];
  if (i == 0) offsets[0] = 0;
  if (i == n_scenes - 1 || (n_scenes == 0 && i == 0)) {
    const int tot = n_scenes > 0 ? offsets[n_scenes] : 0;
    *n_pairs = tot;
    if (tot > capacity) atomicOr(err, ERR_CAPACITY);
  }
}

// Write the kept pairs of each scene at its offset (scene-major, candidate order).
__global__ __launch_bounds__(256) void bp_emit(Tables tb, BatchDev bt, float margin, const int* __restrict__ offsets,
                                               int* __restrict__ pairs, int capacity, unsigned* err) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= bt.n_scenes) return;
  int o = offsets[s];
  scene_pairs(tb, bt, margin, s, err, [&](int a, int b) {
    if (o < capacity) { pairs[o] = a; pairs[capacity + o] = b; }
    ++o;
  });
}

// ============================================================ per-pair manifold

// Occupancy target: 4 waves per SIMD (<= 128 VGPRs, the rest spilled to
// private memory) for K <= 8, where the per-lane top-K list is short; 2
// otherwise.  At K <= 8 the extra waves hide more of the float64 latency
// than the spills cost (hulls of 64 points: 709 ms at 3 waves, 623 at 4).
// At K = 16 the largest uneven pairs fill a CU's LDS with two workgroups,
// so a tighter register budget only adds spills (4 waves: 7.64 -> 7.81 s
// for that class).
// WAVES > 0 overrides the target (the work-queue kernel of the full method has
// a 5-wave variant at K 8 and a 4-wave one at K 16, chosen where LDS leaves
// room for the extra workgroups).
template <int BLOCK, int KMAX, bool DYN, bool PRESEL = false, bool SQ = false, bool REFINE = false, int WAVES = 0>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(WAVES > 0 ? WAVES : ((KMAX <= 8 && !SQ && !REFINE) ? 4 : 2))))
void collide_fwd(Tables tb, BatchDev bt, ParamsDev prm, OutDev out,
                                                     float* __restrict__ scratch, long long scratch_stride, int maxV,
                                                     int maxE, int maxF, const int* __restrict__ order,
                                                     const int* __restrict__ range, int* __restrict__ queue,
                                                     unsigned* err, int edges_out, TapeDev tape) {
  extern __shared__ float4 smem4[];
  __shared__ PairShared ps;
  PairEngine<BLOCK, KMAX, true, PRESEL, SQ, REFINE> P(ps, reinterpret_cast<char*>(smem4), tb, bt, prm,
                                          scratch + (long long)blockIdx.x * scratch_stride, maxV, maxE, maxF,
                                          PRESEL ? presel_lds_bytes(maxV, maxE) : 0, edges_out != 0);
  const int tid = threadIdx.x;
  const int K = prm.K;
  // items: all kept pairs, or the [start, start + count) slice of `order`
  // given by `range` (one size class of the fused path)
  const int n_pairs = range ? range[1] : min(*out.n_pairs, out.capacity);
  const int* ord = range ? order + range[0] : order;

  int item = DYN ? 0 : blockIdx.x;
  while (true) {
    if (DYN) {
      if (tid == 0) ps.next = atomicAdd(queue, 1);
      __syncthreads();
      item = ps.next;
    }
    if (item >= n_pairs) break;
    const int pi = ord ? ord[item] : item;
    if (P.setup(out.pairs[pi], out.pairs[out.capacity + pi], err)) {
      P.stage();
      if (PRESEL) P.select();
      P.cull();
      double tk[KMAX];
      P.scores(tk);
      P.topk(tk);
      P.softsort();
      if (tape.base) {
        // the adjoint's tape: s_[k], the row sums, the candidates within its window
        char* rec = tape.base + (long long)pi * tape_stride(K);
        double* td = reinterpret_cast<double*>(rec + 16);
        for (int i = tid; i < 10 * K; i += BLOCK) td[i] = i < K ? P.sTop[i] : P.sAcc[i - K];
        const int tot = P.window(kAdjointTaus);
        // the smaller form: indices (tot entries) or a mask (2 entries per 64 candidates)
        const long long mask_n = 2LL * ((P.ps.ncand + 63) >> 6);
        const bool as_mask = mask_n < (long long)tot;
        const long long need = as_mask ? mask_n : (long long)tot;
        if (tid == 0) {
          // a mask starts on an 8-byte boundary: one spare entry
          const unsigned long long o = atomicAdd(tape.pool_used, (unsigned long long)(need + (as_mask ? 1 : 0)));
          const unsigned long long start = as_mask ? (o + 1ull) & ~1ull : o;
          const bool fits = start + (unsigned long long)need <= (unsigned long long)tape.pool_cap;
          ps.tape_off = fits ? (long long)start : -1;
          reinterpret_cast<int*>(rec)[0] = tot;
          reinterpret_cast<int*>(rec)[1] = fits ? (as_mask ? 2 : 1) : 0;
          reinterpret_cast<long long*>(rec)[1] = fits ? (long long)start : 0;
        }
        __syncthreads();
        const long long start = ps.tape_off;
        if (start >= 0) {
          if (as_mask) P.window_mask(kAdjointTaus, reinterpret_cast<unsigned long long*>(tape.pool + start));
          else P.write_window_runs(tot, tape.pool + start);
        }
      }
      // outputs: divide by row sums, rotate to world
      for (int kk = tid; !tape.skip_out && kk < K; kk += BLOCK) {
        const double* a = P.sAcc + 9 * kk;
        // a row with no candidate (fewer candidates than K) is all zeros
        const bool live = a[0] > 0.0;
        const double inv = live ? 1.0 / a[0] : 0.0;
        const double px = a[1] * inv, py = a[2] * inv, pz = a[3] * inv;
        const double nx = a[4] * inv, ny = a[5] * inv, nz = a[6] * inv;
        const double* R = ps.RA;
        const double tx = live ? ps.tA[0] : 0.0, ty = live ? ps.tA[1] : 0.0, tz = live ? ps.tA[2] : 0.0;
        const long long o = (long long)pi * K + kk;
        const long long CK = (long long)out.capacity * K;
        out.point[o] = float(R[0] * px + R[1] * py + R[2] * pz + tx);
        out.point[CK + o] = float(R[3] * px + R[4] * py + R[5] * pz + ty);
        out.point[2 * CK + o] = float(R[6] * px + R[7] * py + R[8] * pz + tz);
        out.normal[o] = float(R[0] * nx + R[1] * ny + R[2] * nz);
        out.normal[CK + o] = float(R[3] * nx + R[4] * ny + R[5] * nz);
        out.normal[2 * CK + o] = float(R[6] * nx + R[7] * ny + R[8] * nz);
        out.dist[o] = float(a[7] * inv);
        out.weight[o] = float(a[8] * inv);
      }
    }
    __syncthreads();
    if (!DYN) item += gridDim.x;
  }
}

// ============================================================ launchers

__global__ void tape_reset(unsigned long long* counter) {
  if (threadIdx.x == 0) *counter = 0ull;
}

__global__ void counter_reset(int* counter) {
  if (threadIdx.x == 0) *counter = 0;
}

hipError_t launch_counter_reset(int* counter, hipStream_t st) {
  hipLaunchKernelGGL(counter_reset, dim3(1), dim3(64), 0, st, counter);
  return hipGetLastError();
}

hipError_t launch_tape_reset(const TapeDev& t, hipStream_t st) {
  hipLaunchKernelGGL(tape_reset, dim3(1), dim3(64), 0, st, t.pool_used);
  return hipGetLastError();
}

int fwd_lds_bytes(int maxV, int maxE, int maxF, int block, int kmax, bool presel, bool edges_out) {
  (void)kmax;
  const int extra = presel ? presel_lds_bytes(maxV, maxE) : 0;
  return lds_layout(maxE, maxF, block, extra, edges_out).bytes + extra;
}

hipError_t launch_broadphase(const Tables& tb, const BatchDev& bt, float margin, const OutDev& out, int* tile_sums,
                             unsigned* err, hipStream_t st) {
  const int S = bt.n_scenes;
  const int n_tiles = (S + kScanTile - 1) / kScanTile;
  if (S > 0) {
    hipLaunchKernelGGL(bp_count_scan, dim3(n_tiles), dim3(kScanThreads), 0, st, tb, bt, margin, out.pair_offsets,
                       tile_sums, err);
    hipLaunchKernelGGL(scan_tiles, dim3(1), dim3(1024), 0, st, tile_sums, n_tiles);
  }
  hipLaunchKernelGGL(add_tile_offsets, dim3(S > 0 ? (S + kScanThreads - 1) / kScanThreads : 1), dim3(kScanThreads), 0,
                     st, out.pair_offsets, tile_sums, S, out.n_pairs, out.capacity, err);
  if (S > 0)
    hipLaunchKernelGGL(bp_emit, dim3((S + 255) / 256), dim3(256), 0, st, tb, bt, margin, out.pair_offsets, out.pairs,
                       out.capacity, err);
  return hipGetLastError();
}

template <int BLOCK, int KMAX, bool DYN, bool PRESEL = false, bool SQ = false, bool REFINE = false, int WAVES = 0>
static hipError_t launch_fwd_t(const FwdLaunch& f, hipStream_t st) {
  auto kern = collide_fwd<BLOCK, KMAX, DYN, PRESEL, SQ, REFINE, WAVES>;
  const int lds = fwd_lds_bytes(f.maxV, f.maxE, f.maxF, BLOCK, KMAX, PRESEL, f.edges_out != 0);
  hipLaunchKernelGGL(kern, dim3(f.grid), dim3(BLOCK), lds, st, f.tb, f.bt, f.prm, f.out, f.scratch,
                     f.scratch_stride, f.maxV, f.maxE, f.maxF, f.order, f.range, f.queue, f.err, f.edges_out,
                     f.tape);
  return hipGetLastError();
}

template <int BLOCK, int KMAX, bool DYN, bool PRESEL = false, bool SQ = false, bool REFINE = false, int WAVES = 0>
static int occ_t(int maxV, int maxE, int maxF, bool edges_out) {
  int nb = 0;
  const int lds = fwd_lds_bytes(maxV, maxE, maxF, BLOCK, KMAX, PRESEL, edges_out);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, collide_fwd<BLOCK, KMAX, DYN, PRESEL, SQ, REFINE, WAVES>, BLOCK,
                                                   lds) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

#define CM_FWD_DISPATCH(FN, ...)                                                       \
  switch (f.block) {                                                                   \
    case 128:                                                                          \
      if (f.kmax == 8) return FN<128, 8, DYNV>(__VA_ARGS__);                           \
      if (f.kmax == 16) return FN<128, 16, DYNV>(__VA_ARGS__);                         \
      return FN<128, 32, DYNV>(__VA_ARGS__);                                           \
    default:                                                                           \
      if (f.kmax == 8) return FN<256, 8, DYNV>(__VA_ARGS__);                           \
      if (f.kmax == 16) return FN<256, 16, DYNV>(__VA_ARGS__);                         \
      return FN<256, 32, DYNV>(__VA_ARGS__);                                           \
  }

// Pre-selection and contexts that hold superquadric unions run in their own
// instantiations (block 256, static order).
// Sphere-traced witnesses: block 256, static order, K <= 16 (the paper's
// manifolds are small; each refined candidate costs several SDF queries).
template <bool PRESEL, bool SQ>
static hipError_t launch_refine(const FwdLaunch& f, hipStream_t st) {
  if (f.kmax == 8) return launch_fwd_t<256, 8, false, PRESEL, SQ, true>(f, st);
  return launch_fwd_t<256, 16, false, PRESEL, SQ, true>(f, st);
}
template <bool PRESEL, bool SQ>
static int occ_refine(const FwdLaunch& f) {
  if (f.kmax == 8) return occ_t<256, 8, false, PRESEL, SQ, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
  return occ_t<256, 16, false, PRESEL, SQ, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
}

// The extended primitives (superquadric unions, point clouds): block 256.
template <bool DYN, bool PRESEL>
static hipError_t launch_sq_k(const FwdLaunch& f, hipStream_t st) {
  if (f.kmax == 8) return launch_fwd_t<256, 8, DYN, PRESEL, true>(f, st);
  if (f.kmax == 16) return launch_fwd_t<256, 16, DYN, PRESEL, true>(f, st);
  return launch_fwd_t<256, 32, DYN, PRESEL, true>(f, st);
}
template <bool DYN, bool PRESEL>
static int occ_sq_k(const FwdLaunch& f) {
  if (f.kmax == 8) return occ_t<256, 8, DYN, PRESEL, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
  if (f.kmax == 16) return occ_t<256, 16, DYN, PRESEL, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
  return occ_t<256, 32, DYN, PRESEL, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
}

hipError_t launch_collide_fwd(const FwdLaunch& f, hipStream_t st) {
  if (f.prm.refine > 0) {
    if (f.queue || f.block != 256 || f.kmax > 16 || f.maxV > 4096 || f.maxE > 4096) return hipErrorInvalidValue;
    const bool ps = f.prm.presel_v > 0;
    if (f.prm.sq) return ps ? launch_refine<true, true>(f, st) : launch_refine<false, true>(f, st);
    return ps ? launch_refine<true, false>(f, st) : launch_refine<false, false>(f, st);
  }
  if (f.prm.sq) {   // static order (cm_collide) or the fused path's work queue
    if (f.block != 256 || f.maxV > 4096 || f.maxE > 4096) return hipErrorInvalidValue;
    const bool ps = f.prm.presel_v > 0;
    if (f.queue) return ps ? launch_sq_k<true, true>(f, st) : launch_sq_k<true, false>(f, st);
    return ps ? launch_sq_k<false, true>(f, st) : launch_sq_k<false, false>(f, st);
  }
  if (f.prm.presel_v > 0) {
    // the selection tracks taken items in a 64-bit mask per lane: <= 4096 per
    // set; static order (cm_collide) or the fused path's work queue
    if (f.block != 256 || f.maxV > 4096 || f.maxE > 4096) return hipErrorInvalidValue;
    if (f.queue) {
      if (f.kmax == 8) return launch_fwd_t<256, 8, true, true>(f, st);
      if (f.kmax == 16) return launch_fwd_t<256, 16, true, true>(f, st);
      return launch_fwd_t<256, 32, true, true>(f, st);
    }
    if (f.kmax == 8) return launch_fwd_t<256, 8, false, true>(f, st);
    if (f.kmax == 16) return launch_fwd_t<256, 16, false, true>(f, st);
    return launch_fwd_t<256, 32, false, true>(f, st);
  }
  if (f.queue) {
    constexpr bool DYNV = true;
    if (f.hi_occ && f.block == 256 && f.kmax == 8) return launch_fwd_t<256, 8, true, false, false, false, 5>(f, st);
    if (f.hi_occ && f.block == 256 && f.kmax == 16) return launch_fwd_t<256, 16, true, false, false, false, 4>(f, st);
    if (f.block == 64) {   // single-wave workgroups: the fused path's small pairs
      if (f.kmax == 8) return launch_fwd_t<64, 8, true>(f, st);
      if (f.kmax == 16) return launch_fwd_t<64, 16, true>(f, st);
      return launch_fwd_t<64, 32, true>(f, st);
    }
    CM_FWD_DISPATCH(launch_fwd_t, f, st)
  } else {
    constexpr bool DYNV = false;
    CM_FWD_DISPATCH(launch_fwd_t, f, st)
  }
}

int fwd_occupancy(const FwdLaunch& f) {
  if (f.prm.refine > 0) {
    const bool ps = f.prm.presel_v > 0;
    if (f.prm.sq) return ps ? occ_refine<true, true>(f) : occ_refine<false, true>(f);
    return ps ? occ_refine<true, false>(f) : occ_refine<false, false>(f);
  }
  if (f.prm.sq) {
    const bool ps = f.prm.presel_v > 0;
    if (f.queue) return ps ? occ_sq_k<true, true>(f) : occ_sq_k<true, false>(f);
    return ps ? occ_sq_k<false, true>(f) : occ_sq_k<false, false>(f);
  }
  if (f.prm.presel_v > 0) {
    if (f.queue) {
      if (f.kmax == 8) return occ_t<256, 8, true, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
      if (f.kmax == 16) return occ_t<256, 16, true, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
      return occ_t<256, 32, true, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
    }
    if (f.kmax == 8) return occ_t<256, 8, false, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
    if (f.kmax == 16) return occ_t<256, 16, false, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
    return occ_t<256, 32, false, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
  }
  if (f.queue) {
    constexpr bool DYNV = true;
    if (f.block == 64) {
      if (f.kmax == 8) return occ_t<64, 8, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
      if (f.kmax == 16) return occ_t<64, 16, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
      return occ_t<64, 32, true>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
    }
    if (f.hi_occ && f.block == 256 && f.kmax == 8)
      return occ_t<256, 8, true, false, false, false, 5>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
    if (f.hi_occ && f.block == 256 && f.kmax == 16)
      return occ_t<256, 16, true, false, false, false, 4>(f.maxV, f.maxE, f.maxF, f.edges_out != 0);
    CM_FWD_DISPATCH(occ_t, f.maxV, f.maxE, f.maxF, f.edges_out != 0)
  } else {
    constexpr bool DYNV = false;
    CM_FWD_DISPATCH(occ_t, f.maxV, f.maxE, f.maxF, f.edges_out != 0)
  }
}

int fwd_place_edges(FwdLaunch& f) {
  f.hi_occ = 0;
  f.edges_out = 0;
  const int in = fwd_occupancy(f);
  f.edges_out = 1;
  const int out = fwd_occupancy(f);
  f.edges_out = out > in ? 1 : 0;
  const int best = out > in ? out : in;
  // the full method's work-queue kernel in 256-thread blocks: take the
  // higher-occupancy variant where it fits more workgroups per CU than the
  // default; at K 8 (5 waves) for polytopes of at least 128 edges only
  // (hulls of 64 points, 186 edges: 623 -> 613 ms; the mixed scenes, at most
  // 90 edges, lost 99 -> 110 ms), at K 16 (4 waves) whatever the size (the
  // uneven workload's middle class: 698 -> 480 ms; its largest class, two
  // workgroups per CU either way, keeps the default)
  if (f.queue && f.block == 256 && ((f.kmax == 8 && f.maxE >= 128) || f.kmax == 16) && f.prm.presel_v == 0 &&
      !f.prm.sq && f.prm.refine == 0) {
    const int edges_out = f.edges_out;
    f.hi_occ = 1;
    f.edges_out = 0;
    const int in5 = fwd_occupancy(f);
    f.edges_out = 1;
    const int out5 = fwd_occupancy(f);
    const int best5 = out5 > in5 ? out5 : in5;
    if (best5 > best) {
      f.edges_out = out5 > in5 ? 1 : 0;
      return best5;
    }
    f.hi_occ = 0;
    f.edges_out = edges_out;
  }
  return best;
}

}  // namespace cm
