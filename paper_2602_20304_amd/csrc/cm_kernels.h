// Host-visible launch interface of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "cm_internal.h"

namespace cm {

struct FwdLaunch {
  Tables tb;
  BatchDev bt;
  ParamsDev prm;
  OutDev out;
  float* scratch;              // per-workgroup slots of scratch_stride floats
  long long scratch_stride;
  int maxV, maxE, maxF;        // LDS sizing (context-wide maxima)
  const int* order;            // optional pair order (cost-sorted), or null
  int* queue;                  // dynamic work-queue counter (zeroed), or null for static round robin
  unsigned* err;
  int grid, block, kmax;
};

// Scratch floats per workgroup: unsigned-distance matrix + candidate scores.
inline long long fwd_scratch_floats(int maxV, int maxE) {
  return 2LL * maxE * maxE + 2LL * maxE * maxE + 2LL * maxV + 64;   // f64 D + f32 scores
}

int fwd_lds_bytes(int maxV, int maxE, int maxF, int block, int kmax);
int fwd_occupancy(const FwdLaunch& f);
hipError_t launch_broadphase(const Tables& tb, const BatchDev& bt, float margin, const OutDev& out, int* tile_sums,
                             unsigned* err, hipStream_t st);
hipError_t launch_collide_fwd(const FwdLaunch& f, hipStream_t st);

}  // namespace cm
