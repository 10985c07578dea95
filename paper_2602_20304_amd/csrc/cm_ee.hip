// Batched edge-edge witness points of independent edge pairs: the E-E
// routine of Sec. IV-D-2 (regularised QP, analytic active set) and IV-D-3
// (witness points) on its own, in the shape of the witness-point speed
// experiment of Sec. V (Fig. 6).  Each query is one pair of edges; the
// smoothed solver is the one the pair kernels use, and the unsmoothed variant
// (Ours-NS) takes the same active set with hard decisions.
//
// Streaming layout: 12 float32 input rows and 9 float32 output rows, each of
// stride n, so every row is read or written by consecutive lanes; one query
// per thread, loads and stores marked nontemporal (nothing is reused).
// Measured on MI355X at 10^7 queries, this shape moves data as fast as a
// plain kernel with the same 12-in / 9-out rows and no arithmetic; wider
// per-thread vectors (2 or 4 queries) were slower.
#include "cm_device.cuh"
#include "cm_kernels.h"

namespace cm {
namespace {

constexpr int kEEBlock = 256;

// Exact minimiser of the regularised QP over [0,1]^2 (no smoothing): the
// unconstrained minimiser when it is in the box, else the best of the four
// box-edge minimisers (each clamped to [0, 1]), lower edge index on ties.
__device__ __forceinline__ EEQP ee_qp_hard(const D3& a0, const D3& t1, const D3& b0, const D3& t2, double lam) {
  const D3 b = d3(a0.x - b0.x, a0.y - b0.y, a0.z - b0.z);
  const double Q11 = dot(t1, t1) + lam, Q22 = dot(t2, t2) + lam;
  const double Q12 = -dot(t1, t2);
  const double hl = 0.5 * lam;
  const double c1 = dot(b, t1) - hl;
  const double c2 = -dot(b, t2) - hl;
  const double det = Q11 * Q22 - Q12 * Q12;
  const double idet = rcp64(det);
  const double au1 = (Q12 * c2 - c1 * Q22) * idet;
  const double au2 = (Q12 * c1 - c2 * Q11) * idet;
  double al1 = au1, al2 = au2, con = 1.0;
  if (!(au1 >= 0.0 && au1 <= 1.0 && au2 >= 0.0 && au2 <= 1.0)) {
    const double i11 = rcp64(Q11), i22 = rcp64(Q22);
    const double x[4] = {1.0, 0.0, fmin(fmax(-(Q12 + c1) * i11, 0.0), 1.0), fmin(fmax(-c1 * i11, 0.0), 1.0)};
    const double y[4] = {fmin(fmax(-(Q12 + c2) * i22, 0.0), 1.0), fmin(fmax(-c2 * i22, 0.0), 1.0), 1.0, 0.0};
    double best = INFINITY;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      // objective 1/2 al^T Q al + c^T al
      const double J = 0.5 * (Q11 * x[j] * x[j] + 2.0 * Q12 * x[j] * y[j] + Q22 * y[j] * y[j]) + c1 * x[j] + c2 * y[j];
      if (J < best) { best = J; al1 = x[j]; al2 = y[j]; }
    }
    con = 0.0;
  }
  EEQP r = ee_from_alpha(a0, t1, b0, t2, al1, al2, con > 0.0 ? 0.0 : -INFINITY);
  r.con = con;
  return r;
}

template <bool HARD>
__device__ __forceinline__ void ee_one(const float (&v)[12], double lam, const Temp& T, float (&o)[9]) {
  const D3 a0 = d3(v[0], v[1], v[2]);
  const D3 t1 = d3(double(v[3]) - double(v[0]), double(v[4]) - double(v[1]), double(v[5]) - double(v[2]));
  const D3 b0 = d3(v[6], v[7], v[8]);
  const D3 t2 = d3(double(v[9]) - double(v[6]), double(v[10]) - double(v[7]), double(v[11]) - double(v[8]));
  const EEQP q = HARD ? ee_qp_hard(a0, t1, b0, t2, lam) : ee_qp(a0, t1, b0, t2, lam, T);
  o[0] = float(q.al1);
  o[1] = float(q.al2);
  o[2] = float(q.con);
  o[3] = float(a0.x + q.al1 * t1.x);
  o[4] = float(a0.y + q.al1 * t1.y);
  o[5] = float(a0.z + q.al1 * t1.z);
  o[6] = float(b0.x + q.al2 * t2.x);
  o[7] = float(b0.y + q.al2 * t2.y);
  o[8] = float(b0.z + q.al2 * t2.z);
}

template <bool HARD>
__global__ __launch_bounds__(kEEBlock) void ee_witness_kernel(const float* __restrict__ ed, long long n, ParamsDev prm,
                                                              float* __restrict__ out) {
  const long long i = static_cast<long long>(blockIdx.x) * kEEBlock + threadIdx.x;
  if (i >= n) return;
  const Temp T = make_temp(prm);
  float v[12], o[9];
#pragma unroll
  for (int r = 0; r < 12; ++r) v[r] = __builtin_nontemporal_load(ed + r * n + i);
  ee_one<HARD>(v, prm.lam, T, o);
#pragma unroll
  for (int r = 0; r < 9; ++r) __builtin_nontemporal_store(o[r], out + r * n + i);
}

}  // namespace

hipError_t launch_ee_witness(const float* edges, long long n, const ParamsDev& prm, bool hard, float* out,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + kEEBlock - 1) / kEEBlock;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(blocks)), block(kEEBlock);
  if (hard) hipLaunchKernelGGL(ee_witness_kernel<true>, grid, block, 0, st, edges, n, prm, out);
  else hipLaunchKernelGGL(ee_witness_kernel<false>, grid, block, 0, st, edges, n, prm, out);
  return hipGetLastError();
}

}  // namespace cm
