// Fused batched path, device side: classify kept pairs into size classes,
// order them by estimated cost (largest first within each class) with a
// counting sort, and prepare the per-class work queues.  Launched inside a
// captured hipGraph together with the broadphase and the per-class
// persistent forward kernels, so nothing here may use hipMemset.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cm_kernels.h"

namespace cm {

__global__ void fused_zero(int* __restrict__ counts, int* __restrict__ queues) {
  const int i = threadIdx.x;
  if (i < kNumClasses * kNumBuckets) counts[i] = 0;
  if (i < kNumClasses) queues[i] = 0;
}

// Per-pair cost (VALU slots, rough): E-E pairs dominate, each costing a QP plus
// four SDF queries whose price grows with the polytope face counts.
__device__ __forceinline__ float pair_cost(const GeomRec& A, const GeomRec& B) {
  const float fa = A.type == CM_POLYTOPE ? float(A.nf) * 14.f : 60.f;
  const float fb = B.type == CM_POLYTOPE ? float(B.nf) * 14.f : 60.f;
  return float(A.ne) * float(B.ne) * (400.f + 2.f * (fa + fb)) + float(A.nv) * fb + float(B.nv) * fa;
}

// Wave-aggregated claim of one slot per lane at counter[key]: one atomic per
// distinct key held by the wave's active lanes (leader = lowest pending
// lane); each lane gets the counter's old value plus its rank among the
// lanes holding the same key.  The loop runs once per distinct key and its
// condition is wave-uniform (a ballot).
__device__ __forceinline__ int wave_claim(int* __restrict__ counter, int key) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(1);
  int slot = 0;
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const int lk = __shfl(key, leader);
    const unsigned long long same = __ballot(key == lk);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counter[lk], __popcll(same));
    base = __shfl(base, leader);
    if (key == lk) slot = base + __popcll(same & ((1ull << lane) - 1ull));
    pending &= ~same;
  }
  return slot;
}

__global__ void fused_classify(Tables tb, BatchDev bt, OutDev out, int cmax0, int cmax1, int* __restrict__ counts,
                               int* __restrict__ keys) {
  const int n = min(*out.n_pairs, out.capacity);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int a = out.pairs[i], b = out.pairs[out.capacity + i];
    const int ga = bt.body_geom[a], gb = bt.body_geom[b];
    int key = -1;
    if (ga >= 0 && ga < tb.n_geoms && gb >= 0 && gb < tb.n_geoms && tb.geoms[ga].type >= 0 && tb.geoms[gb].type >= 0) {
      const GeomRec A = tb.geoms[ga], B = tb.geoms[gb];
      const int e = max(A.ne, B.ne);
      const int c = e <= cmax0 ? 0 : (e <= cmax1 ? 1 : 2);
      const float cost = pair_cost(A, B);
      int bucket = int(log2f(fmaxf(cost, 1.f)));
      bucket = min(max(bucket, 0), kNumBuckets - 1);
      key = c * kNumBuckets + (kNumBuckets - 1 - bucket);   // costly first
    } else {
      key = kNumBuckets - 1;                                 // invalid: class 0, cheapest; flagged by the kernel
    }
    (void)wave_claim(counts, key);
    keys[i] = key;
  }
}

// Exclusive scan of the (class, bucket) histogram into scatter cursors and
// per-class {start, count} ranges.  One small block.
__global__ void fused_scan(int* __restrict__ counts, int* __restrict__ ranges) {
  if (threadIdx.x != 0) return;
  int run = 0;
  for (int c = 0; c < kNumClasses; ++c) {
    const int start = run;
    for (int b = 0; b < kNumBuckets; ++b) {
      const int k = c * kNumBuckets + b;
      const int v = counts[k];
      counts[k] = run;
      run += v;
    }
    ranges[2 * c] = start;
    ranges[2 * c + 1] = run - start;
  }
}

__global__ void fused_scatter(OutDev out, const int* __restrict__ keys, int* __restrict__ cursors,
                              int* __restrict__ order) {
  const int n = min(*out.n_pairs, out.capacity);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int pos = wave_claim(cursors, keys[i]);
    order[pos] = i;
  }
}

// Evenly strided sample of size class c's cost order (autotuning): sample[i]
// = order[start + i * count / m] for i < m = min(n, count), and the sample's
// {0, m} range for the class kernel.
__global__ void fused_sample(const int* __restrict__ order, const int* __restrict__ ranges, int c, int n,
                             int* __restrict__ sample, int* __restrict__ sample_range) {
  const int start = ranges[2 * c], count = ranges[2 * c + 1];
  const int m = min(n, count);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    sample[i] = order[start + int((long long)i * count / m)];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sample_range[0] = 0;
    sample_range[1] = m;
  }
}

hipError_t launch_fused_sample(const FusedWork& w, int c, int n, int* sample, int* sample_range, hipStream_t st) {
  const int grid = std::max(1, std::min(1024, (n + 255) / 256));
  hipLaunchKernelGGL(fused_sample, dim3(grid), dim3(256), 0, st, w.order, w.ranges, c, n, sample, sample_range);
  return hipGetLastError();
}

hipError_t launch_fused_prepare(const Tables& tb, const BatchDev& bt, const OutDev& out, const int* class_maxE,
                                const FusedWork& w, hipStream_t st) {
  hipLaunchKernelGGL(fused_zero, dim3(1), dim3(256), 0, st, w.counts, w.queues);
  const int grid = std::max(1, std::min(2048, (out.capacity + 255) / 256));
  hipLaunchKernelGGL(fused_classify, dim3(grid), dim3(256), 0, st, tb, bt, out, class_maxE[0], class_maxE[1], w.counts,
                     w.keys);
  hipLaunchKernelGGL(fused_scan, dim3(1), dim3(64), 0, st, w.counts, w.ranges);
  hipLaunchKernelGGL(fused_scatter, dim3(grid), dim3(256), 0, st, out, w.keys, w.counts, w.order);
  return hipGetLastError();
}

}  // namespace cm
