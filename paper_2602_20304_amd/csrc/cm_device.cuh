// Device-side math shared by the gfx950 forward and adjoint kernels:
// smooth operators (Sec. III), SDF primitives (Sec. IV-B), the E-E witness
// QP (Sec. IV-D) and wave-level reductions.
//
// Precision model.  The soft operators amplify rounding error by 1/tau, so
// geometric algebra (transforms, plane distances, the QP, witness points,
// distances, scores) runs in float64: on gfx950 a v_fma_f64 issues at the
// same rate as an unpacked v_fma_f32.  Exponentials and logarithms use the
// float32 hardware units (v_exp_f32 / v_log_f32) on float64-prepared
// arguments; their results only enter through terms that are scaled by tau
// or bounded, which keeps every output within ~1e-6 of the FP64 definition.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cm_internal.h"

namespace cm {

// Candidates scoring more than 30 tau below the K-th largest score are left
// out of the SoftSort sums: each has weight below exp(-30) ~ 9.4e-14 against
// a row sum >= 1, so even 10^5 of them move a row's weighted mean by less
// than 1e-8 of the spread of its fields, far below float32 resolution.
constexpr double kFilterTaus = 30.0;
// The adjoint skips candidates whose largest SoftSort weight is below
// exp(-18) ~ 1.5e-8 relative: their share of any gradient is far below the
// float32 outputs' and the gradient tolerance's resolution.
constexpr double kAdjointTaus = 18.0;

struct Temp {
  double tau, inv_tau, c, tl;   // c = log2(e) / tau, tl = tau * ln 2
};

// The constants come precomputed in the kernel arguments, so they stay in
// scalar registers.
__device__ __forceinline__ Temp make_temp(const ParamsDev& prm) {
  Temp T;
  T.tau = prm.tau;
  T.inv_tau = prm.inv_tau;
  T.c = prm.c_log2;
  T.tl = prm.tl;
  return T;
}

// Wave-uniform copies (v_readfirstlane): values every lane holds equal, so
// the compiler can keep them in scalar registers.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uni(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// float32 hardware transcendentals
__device__ __forceinline__ float ex2f(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float lg2f(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// exp(-a / tau) for a >= 0 given in float64 (result float32)
__device__ __forceinline__ float expn(double a, const Temp& T) { return ex2f(float(-a * T.c)); }

// 1/x in float64 for finite x with |x| well inside the normal range:
// v_rcp_f64 (about 26 correct bits) plus two Newton steps.  Used where the
// operand is bounded away from zero by construction (Q11, Q22, det Q >= lambda
// terms, sums >= 1, sqrt(|d|^2 + eps)).
__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// 1/sqrt(x) in float64 for x well inside the normal range (as rcp64):
// v_rsq_f64 plus two Newton steps r <- r (3/2 - x r^2 / 2), eight VALU
// operations where sqrt and a division take about 28.
__device__ __forceinline__ double rsq64(double x) {
  double r = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  r = fma(r, fma(-h * r, r, 0.5), r);
  r = fma(r, fma(-h * r, r, 0.5), r);
  return r;
}
// sqrt(x) and 1/sqrt(x) for x >= 0 through rsq64; x at or below 2^-700 (a
// length below 1e-105) gives 0 for both.
__device__ __forceinline__ void sqrt_rsq64(double x, double& s, double& r) {
  const bool pos = x > 0x1p-700;
  const double y = rsq64(pos ? x : 1.0);
  r = pos ? y : 0.0;
  s = pos ? x * y : 0.0;
}

// a * b + c as one v_fma_f64 whose addend c is a wave-uniform constant in
// scalar registers.  Written with fma(), the compiler picks the tied form
// v_fmac_f64 (addend = destination) and first copies the coefficient into
// a vector register: two VALU operations per Horner step instead of one.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}

// exp(x) for x <= 700 in float64, branch free: Cody-Waite reduction
// x = n ln2 + r, |r| <= ln2 / 2, then a degree-7 polynomial of e^r with
// p(0) = 1 whose other coefficients were fitted by a Remez exchange on the
// relative error over that interval (max 2.3e-10), scaled by 2^n.  Inputs
// below -745 are clamped, so the result underflows to zero there.
__device__ __forceinline__ double exp64n(double x) {
  x = fmax(x, -745.0);
  const double n = rint(x * kLog2e);
  double r = fma(-n, 6.93147180369123816490e-01, x);   // ln2 high part
  r = fma(-n, 1.90821492927058770002e-10, r);          // ln2 low part
  double p = 1.7378911869613724e-04;
  p = fma3(p, r, 1.3941038928452576e-03);
  p = fma3(p, r, 8.3385787951517860e-03);
  p = fma3(p, r, 4.1666353940642690e-02);
  p = fma3(p, r, 1.6666635163904225e-01);
  p = fma3(p, r, 5.0000000468041280e-01);
  p = fma3(p, r, 1.0000000046987592e+00);
  p = fma3(p, r, 1.0);
  return ldexp(p, int(n));
}

// 2^a for a <= 1000 in float64, branch free: a = n + r with r = a - n
// exact, then the polynomial of exp64n at r ln 2 (|r ln 2| <= 0.35; max
// relative error 2.3e-10).  Inputs below -1075 are clamped (the result
// underflows to zero).
__device__ __forceinline__ double exp2_64(double a) {
  a = fmax(a, -1075.0);
  const double n = rint(a);
  const double t = (a - n) * kLn2;
  double p = 1.7378911869613724e-04;
  p = fma3(p, t, 1.3941038928452576e-03);
  p = fma3(p, t, 8.3385787951517860e-03);
  p = fma3(p, t, 4.1666353940642690e-02);
  p = fma3(p, t, 1.6666635163904225e-01);
  p = fma3(p, t, 5.0000000468041280e-01);
  p = fma3(p, t, 1.0000000046987592e+00);
  p = fma3(p, t, 1.0);
  return ldexp(p, int(n));
}
// sigma(u / tau) in float64
__device__ __forceinline__ double sig64(double u, const Temp& T) {
  const double e = exp64n(-fabs(u) * T.inv_tau);
  const double r = rcp64(1.0 + e);
  return u >= 0.0 ? r : e * r;
}
// tanh(u / tau) in float64
__device__ __forceinline__ double tanh64(double u, const Temp& T) {
  const double e = exp64n(-2.0 * fabs(u) * T.inv_tau);
  return copysign((1.0 - e) * rcp64(1.0 + e), u);
}

// tau * softplus(x / tau) = max(x, 0) + tau ln(1 + exp(-|x| / tau))
__device__ __forceinline__ double softplus_t(double x, const Temp& T) {
  const float e = expn(fabs(x), T);
  return fmax(x, 0.0) + T.tl * double(lg2f(1.f + e));
}
__device__ __forceinline__ double clip01(double x, const Temp& T) {
  return softplus_t(x, T) - softplus_t(x - 1.0, T);
}
// ln sigma(u / tau)
__device__ __forceinline__ double lsig(double u, const Temp& T) {
  const float e = expn(fabs(u), T);
  return fmin(u, 0.0) * T.inv_tau - kLn2 * double(lg2f(1.f + e));
}
// sigma(u / tau) and ln sigma(u / tau)
__device__ __forceinline__ void sig_lsig(double u, const Temp& T, double& s, double& ls) {
  const float e = expn(fabs(u), T);
  const float r = frcp(1.f + e);
  s = double(u >= 0.0 ? r : e * r);
  ls = fmin(u, 0.0) * T.inv_tau - kLn2 * double(lg2f(1.f + e));
}
// tanh(u / tau)
__device__ __forceinline__ double tanh_t(double u, const Temp& T) {
  const float e = expn(2.0 * fabs(u), T);
  return copysign(double((1.f - e) * frcp(1.f + e)), u);
}

__device__ __forceinline__ double sgn1(double x) { return x >= 0.0 ? 1.0 : -1.0; }

struct D3 {
  double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ __forceinline__ double dot(const D3& a, const D3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// ----------------------------------------------------------------- SDFs
// Body-frame SDF of an analytic primitive and its gradient.
__device__ __forceinline__ void sdf_analytic(int type, const float* p, const D3& l, double& phi, D3& g) {
  if (type == CM_SPHERE) {
    double n, inv;
    sqrt_rsq64(dot(l, l), n, inv);
    phi = n - double(p[0]);
    g = d3(l.x * inv, l.y * inv, l.z * inv);
  } else if (type == CM_CAPSULE) {
    const double h = p[1];
    const double zc = fmin(fmax(l.z, -h), h);
    const D3 y = d3(l.x, l.y, l.z - zc);
    double n, inv;
    sqrt_rsq64(dot(y, y), n, inv);
    phi = n - double(p[0]);
    g = d3(y.x * inv, y.y * inv, y.z * inv);
  } else {  // rounded box: outer half-extents p[0..2], rounding p[3]
    const double rr = p[3];
    const double qx = fabs(l.x) - (double(p[0]) - rr), qy = fabs(l.y) - (double(p[1]) - rr),
                 qz = fabs(l.z) - (double(p[2]) - rr);
    const double mx = fmax(qx, 0.0), my = fmax(qy, 0.0), mz = fmax(qz, 0.0);
    const double s = mx * mx + my * my + mz * mz;
    if (s > 0x1p-700) {
      double n, inv;
      sqrt_rsq64(s, n, inv);
      phi = n - rr;
      g = d3(sgn1(l.x) * mx * inv, sgn1(l.y) * my * inv, sgn1(l.z) * mz * inv);
    } else {
      const double qm = fmax(qx, fmax(qy, qz));
      phi = qm - rr;
      const int j = (qx >= qy && qx >= qz) ? 0 : (qy >= qz ? 1 : 2);
      g = d3(j == 0 ? sgn1(l.x) : 0.0, j == 1 ? sgn1(l.y) : 0.0, j == 2 ? sgn1(l.z) : 0.0);
    }
  }
}

// SDF query kinds.  kValue: phi only.  kFull: phi and gradient at a
// general point.  kSurfGrad: gradient only, at a point on the body's own
// boundary (a witness point on one of its edges).
enum SdfMode { kValue = 0, kFull = 1, kSurfGrad = 2 };

// tau-LSE over body-frame planes, staged in LDS pre-scaled by c = log2(e)/tau:
// pd[f] = c (n.xyz, o).  With y_f = n_f . x - o_f and y'_f = c y_f,
// phi = LSE_tau(y) = tau ln 2 (m' + log2 sum_f 2^(y'_f - m')), m' = max y'_f,
// and the gradient is the softmax-weighted sum of the normals (the scale c
// cancels in the normalised weights).  The value sums float32 powers of two
// (its error is tau times their relative error).  The gradient enters the
// clashing indicator divided by tau, so its weights are float64; a plane
// whose weight is below 2^-36 (~e^-25) relative to the largest for every lane
// of the wave is skipped (< 2e-11 per plane).  At a point on the polytope's
// own boundary the largest plane value is 0 (convexity), so kSurfGrad shifts
// by 0 and needs no max pass and no value sum; a smoothed witness can sit
// past an edge's end by at most ~0.28 tau times the edge length, which keeps
// every shifted exponent below ~0.4.
template <int MODE>
__device__ __forceinline__ void sdf_poly(const double4* __restrict__ pd, int nf, const D3& x, const Temp& T,
                                         double& phi, D3& g) {
  double m = 0.0;
  if (MODE != kSurfGrad) {
    m = -1e300;
#pragma unroll 2
    for (int f = 0; f < nf; ++f) {
      const double4 q = pd[f];
      m = fmax(m, fma(q.x, x.x, fma(q.y, x.y, fma(q.z, x.z, -q.w))));
    }
  }
  float s = 0.f;
  double S = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll 2
  for (int f = 0; f < nf; ++f) {
    const double4 q = pd[f];
    const double a = fma(q.x, x.x, fma(q.y, x.y, fma(q.z, x.z, -q.w))) - m;
    if (MODE != kSurfGrad) s += ex2f(float(a));
    if (MODE != kValue) {
      const bool sig = a > -36.0;
      if (__any(sig)) {
        const double e = sig ? exp2_64(a) : 0.0;
        S += e;
        ax = fma(e, q.x, ax); ay = fma(e, q.y, ay); az = fma(e, q.z, az);
      }
    }
  }
  if (MODE != kSurfGrad) phi = T.tl * (m + double(lg2f(s)));
  if (MODE != kValue) {
    const double inv = S > 0.0 ? T.tl * rcp64(S) : 0.0;
    g = d3(ax * inv, ay * inv, az * inv);
  }
}

// A body as seen in the pair frame (the frame of body A).
struct BodyView {
  int type, nv, ne, nf;
  float p[4];
  double R[9];   // body frame -> pair frame rotation (row-major); unused for A
  double t[3];   // body origin in the pair frame; unused for A
  const double4* planes;  // LDS, body frame (polytopes): c (n.xyz, o), c = log2(e) / tau
};

// Load a body view that every lane of the workgroup shares from LDS into
// wave-uniform registers.
__device__ __forceinline__ BodyView load_uniform(const BodyView& src, bool with_pose) {
  BodyView v;
  v.type = uni(src.type); v.nv = uni(src.nv); v.ne = uni(src.ne); v.nf = uni(src.nf);
#pragma unroll
  for (int i = 0; i < 4; ++i) v.p[i] = uni(src.p[i]);
  if (with_pose) {
#pragma unroll
    for (int i = 0; i < 9; ++i) v.R[i] = uni(src.R[i]);
#pragma unroll
    for (int i = 0; i < 3; ++i) v.t[i] = uni(src.t[i]);
  }
  v.planes = nullptr;
  return v;
}

// Polytopes of up to 64 * kMaxMaskWords faces are culled.
constexpr int kMaxMaskWords = 8;
// No shift given for a masked value query: it runs its max pass.
constexpr double kNoShift = 1e300;
// A subset of a polytope's faces, in LDS: the first n words (bit f of word
// f / 64), shared by every active lane of a wave; n = 0 means all faces.
struct FaceMask {
  unsigned long long w[kMaxMaskWords];
  int n;
};

__device__ __forceinline__ unsigned long long uni64(unsigned long long v) {
  const int lo = __builtin_amdgcn_readfirstlane(int(v & 0xffffffffull));
  const int hi = __builtin_amdgcn_readfirstlane(int(v >> 32));
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Word w of a face mask, limited to the polytope's nf faces, made
// wave-uniform (scalar registers).
__device__ __forceinline__ unsigned long long mask_word(const FaceMask& mk, int w, int nf) {
  const int rem = nf - 64 * w;
  const unsigned long long valid = rem >= 64 ? ~0ull : (rem > 0 ? (1ull << rem) - 1ull : 0ull);
  return uni64(mk.w[w]) & valid;
}

// body(f) for each face f of a mask that every lane of the wave shares, in
// increasing order (a wave-uniform walk over its set bits), or for every one
// of the nf faces when mk is null or empty.
template <typename F>
__device__ __forceinline__ void for_faces(const FaceMask* mk, int nf, F&& body) {
  const int nw = mk ? __builtin_amdgcn_readfirstlane(mk->n) : 0;
  if (nw == 0) {
    for (int f = 0; f < nf; ++f) body(f);
    return;
  }
  for (int w = 0; w < nw; ++w) {
    unsigned long long bits = mask_word(*mk, w, nf);
    while (bits) {
      const int b = __builtin_ctzll(bits);
      bits &= bits - 1ull;
      body(64 * w + b);
    }
  }
}

// Orders a wave's LDS accesses before and after it (the wave's LDS
// operations complete in issue order; this keeps the compiler from moving
// them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sdf_poly restricted to the faces of a mask that every active lane of the
// wave shares: a wave-uniform walk over its set bits in increasing face order,
// two faces per step with both LDS loads issued before either is used (a
// one-face step exposes the load latency).  shift (kValue): the lane's
// shift of the float32 sum when it has one (a lower bound of the largest
// plane value within 100 of it, so the sum stays in range); the max pass
// runs only when a lane of the wave has none.
template <int MODE>
__device__ __forceinline__ void sdf_poly_masked(const double4* __restrict__ pd, int nf, const FaceMask& mk,
                                                const D3& x, const Temp& T, double& phi, D3& g,
                                                double shift = kNoShift) {
  const int nw = mk.n;
  double m = 0.0;
  const bool shifted = MODE == kValue && shift < kNoShift;
  if (MODE != kSurfGrad && !__all(shifted)) {
    m = -1e300;
    for (int w = 0; w < nw; ++w) {
      const double4* pw = pd + 64 * w;
      unsigned long long bits = mask_word(mk, w, nf);
      while (bits) {
        const int b0 = __builtin_ctzll(bits);
        bits &= bits - 1ull;
        if (bits) {
          const int b1 = __builtin_ctzll(bits);
          bits &= bits - 1ull;
          const double4 q0 = pw[b0], q1 = pw[b1];
          const double y0 = fma(q0.x, x.x, fma(q0.y, x.y, fma(q0.z, x.z, -q0.w)));
          const double y1 = fma(q1.x, x.x, fma(q1.y, x.y, fma(q1.z, x.z, -q1.w)));
          m = fmax(m, fmax(y0, y1));
        } else {
          const double4 q0 = pw[b0];
          m = fmax(m, fma(q0.x, x.x, fma(q0.y, x.y, fma(q0.z, x.z, -q0.w))));
        }
      }
    }
  }
  if (shifted) m = shift;
  float s = 0.f;
  double S = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
  for (int w = 0; w < nw; ++w) {
    const double4* pw = pd + 64 * w;
    unsigned long long bits = mask_word(mk, w, nf);
    while (bits) {
      const int b0 = __builtin_ctzll(bits);
      bits &= bits - 1ull;
      // a second face, or the first again with zero weight
      const bool two = bits != 0ull;
      const int b1 = two ? __builtin_ctzll(bits) : b0;
      if (two) bits &= bits - 1ull;
      const double4 q0 = pw[b0], q1 = pw[b1];
      const double a0 = fma(q0.x, x.x, fma(q0.y, x.y, fma(q0.z, x.z, -q0.w))) - m;
      const double a1 = fma(q1.x, x.x, fma(q1.y, x.y, fma(q1.z, x.z, -q1.w))) - m;
      // sums in face order, as in sdf_poly (the padding face adds exact
      // zeros), so culled and full evaluations round alike
      if (MODE != kSurfGrad) {
        const float e0 = ex2f(float(a0));
        const float e1 = two ? ex2f(float(a1)) : 0.f;
        s += e0;
        s += e1;
      }
      if (MODE != kValue) {
        const bool sig0 = a0 > -36.0, sig1 = two && a1 > -36.0;
        if (__any(sig0 || sig1)) {
          const double e0 = sig0 ? exp2_64(a0) : 0.0;
          const double e1 = sig1 ? exp2_64(a1) : 0.0;
          S += e0;
          ax = fma(e0, q0.x, ax); ay = fma(e0, q0.y, ay); az = fma(e0, q0.z, az);
          S += e1;
          ax = fma(e1, q1.x, ax); ay = fma(e1, q1.y, ay); az = fma(e1, q1.z, az);
        }
      }
    }
  }
  if (MODE != kSurfGrad) {
    // a shifted sum can reach 2^100: its exponent goes in exactly, so that
    // the float32 logarithm only sees the mantissa
    int E = 0;
    const float sm = shifted ? frexpf(s, &E) : s;
    phi = T.tl * ((m + double(E)) + double(lg2f(sm)));
  }
  if (MODE != kValue) {
    const double inv = S > 0.0 ? T.tl * rcp64(S) : 0.0;
    g = d3(ax * inv, ay * inv, az * inv);
  }
}

// log2(s) for a normal s > 0 in float64: s = f 2^e with f in [1/sqrt 2,
// sqrt 2), then log2 f = (2 / ln 2) atanh(y), y = (f - 1) / (f + 1), |y| <=
// 0.172, by the odd series through y^15 (next term below 4e-14 relative).
__device__ __forceinline__ double log2_64(double s) {
  int e;
  double f = frexp(s, &e);
  if (f < 0.70710678118654752) { f *= 2.0; e -= 1; }
  const double y = (f - 1.0) / (f + 1.0), y2 = y * y;
  double p = 1.0 / 15.0;
  p = fma(p, y2, 1.0 / 13.0);
  p = fma(p, y2, 1.0 / 11.0);
  p = fma(p, y2, 1.0 / 9.0);
  p = fma(p, y2, 1.0 / 7.0);
  p = fma(p, y2, 1.0 / 5.0);
  p = fma(p, y2, 1.0 / 3.0);
  p = fma(p, y2, 1.0);
  return double(e) + 2.0 * kLog2e * y * p;
}

// Smooth union of superquadrics (Sec. IV-B, SQ primitives and smooth
// union) at body-frame point l.  Each primitive is 5 staged double4: the
// rows of its rotation transposed with its translation in .w (so the
// primitive-frame point is y = R^T (l - t)), then (1/a, 1/b, 1/c, eps1) and
// (1/eps2, eps2/eps1, 1/eps1, eps2).  With s = y / (a, b, c) the
// inside-outside function is f = ((s_x^2)^(1/eps2) + (s_y^2)^(1/eps2))^(eps2/eps1)
// + (s_z^2)^(1/eps1) and phi_i = |y| (1 - f^(-eps1/2)); the union is
// -LSE_tau(-phi_i), accumulated online (running minimum, rescaled sums).
// Powers use the float64 exp2_64 / log2_64 above (the values feed weights
// divided by tau).
// GRAD: also the union gradient, sum_i pi_i grad phi_i, or with NDIR the V-S
// normal direction sum_i pi_i grad f_i (normals of superquadrics come from
// grad f), pi = softmax(-phi_i / tau).
// (s^2)^p for the superquadric powers, 0 at s = 0
__device__ __forceinline__ double sqpow(double s, double p) {
  const double s2 = s * s;
  return s2 > 0.0 ? exp2_64(p * log2_64(s2)) : 0.0;
}

template <bool GRAD, bool NDIR>
__device__ __forceinline__ void sdf_squnion(const double4* __restrict__ sq, int nslots, const D3& l, const Temp& T,
                                            double& phi, D3& g) {
  const int M = nslots / 5;
  double mn = 0.0, S = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
  for (int i = 0; i < M; ++i) {
    const double4 r0 = sq[5 * i], r1 = sq[5 * i + 1], r2 = sq[5 * i + 2], s3 = sq[5 * i + 3], s4 = sq[5 * i + 4];
    const double dx = l.x - r0.w, dy = l.y - r1.w, dz = l.z - r2.w;
    const double yx = fma(r0.x, dx, fma(r0.y, dy, r0.z * dz));
    const double yy = fma(r1.x, dx, fma(r1.y, dy, r1.z * dz));
    const double yz = fma(r2.x, dx, fma(r2.y, dy, r2.z * dz));
    const double sx = yx * s3.x, sy = yy * s3.y, sz = yz * s3.z;
    const double e1 = s3.w, ie2 = s4.x, r21 = s4.y, ie1 = s4.z;
    // (s^2)^p = 2^(p log2 s^2), 0 at s = 0 (the branch-free exp2_64 /
    // log2_64 of this file: relative error ~1e-9, far inside what the
    // weights' division by tau can amplify to a visible difference)
    const double Ax = sqpow(sx, ie2), Ay = sqpow(sy, ie2), Cz = sqpow(sz, ie1);
    const double u = Ax + Ay;
    const double U = u > 0.0 ? exp2_64(r21 * log2_64(u)) : 0.0;
    const double f = U + Cz;
    const double r = sqrt(fma(yx, yx, fma(yy, yy, yz * yz)));
    const double q = exp2_64(-0.5 * e1 * log2_64(f));
    const double ph = r * (1.0 - q);
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (GRAD) {
      // d/ds (s^2)^p = 2 p (s^2)^p / s (0 at s = 0: 2p > 1 for exponents <= 1.9)
      const double du = u > 0.0 ? r21 * U / u : 0.0;
      const double gx = sx != 0.0 ? du * 2.0 * ie2 * Ax / sx * s3.x : 0.0;
      const double gy = sy != 0.0 ? du * 2.0 * ie2 * Ay / sy * s3.y : 0.0;
      const double gz = sz != 0.0 ? 2.0 * ie1 * Cz / sz * s3.z : 0.0;
      double hx = gx, hy = gy, hz = gz;
      if (!NDIR) {
        // grad phi_i = (1 - q) y / |y| + |y| (eps1 / 2) (q / f) grad f
        const double a = r > 0.0 ? (1.0 - q) / r : 0.0, b = r * 0.5 * e1 * q / f;
        hx = fma(a, yx, b * gx); hy = fma(a, yy, b * gy); hz = fma(a, yz, b * gz);
      }
      // back to the body frame: R (h) = sum_k h_k (row k of R^T)
      vx = fma(hx, r0.x, fma(hy, r1.x, hz * r2.x));
      vy = fma(hx, r0.y, fma(hy, r1.y, hz * r2.y));
      vz = fma(hx, r0.z, fma(hy, r1.z, hz * r2.z));
    }
    if (i == 0) {
      mn = ph; S = 1.0; ax = vx; ay = vy; az = vz;
    } else if (ph < mn) {
      const double sc = exp64n(-(mn - ph) * T.inv_tau);
      S = fma(S, sc, 1.0); ax = fma(ax, sc, vx); ay = fma(ay, sc, vy); az = fma(az, sc, vz);
      mn = ph;
    } else {
      const double w = exp64n(-(ph - mn) * T.inv_tau);
      S += w; ax = fma(w, vx, ax); ay = fma(w, vy, ay); az = fma(w, vz, az);
    }
  }
  phi = mn - T.tau * kLn2 * log2_64(S);
  if (GRAD) {
    const double iS = 1.0 / S;
    g = d3(ax * iS, ay * iS, az * iS);
  }
}

// Oriented point cloud (Sec. IV-B, OPC primitives) at body-frame point l:
// phi = sum_j B_j h_j / sum_j B_j with h_j = n_j . (l - p_j) and the Gaussian
// basis B_j = exp(-|l - p_j|^2 / (2 sigma_j^2)), weights taken relative to
// their maximum (two passes).  Each point is 2 staged double4: (p, 1 / (2
// sigma^2)) and (unit n, 1 / sigma^2).  GRAD: grad phi by the quotient rule,
// (sum_j B_j (n_j + g_j (h_j - phi))) / sum_j B_j with g_j = -(l - p_j) / sigma^2.
template <bool GRAD>
__device__ __forceinline__ void sdf_opc(const double4* __restrict__ pc, int nslots, const D3& l, double& phi, D3& g) {
  const int N = nslots / 2;
  double m = -INFINITY;
  for (int j = 0; j < N; ++j) {
    const double4 a = pc[2 * j];
    const double dx = l.x - a.x, dy = l.y - a.y, dz = l.z - a.z;
    m = fmax(m, -fma(dx, dx, fma(dy, dy, dz * dz)) * a.w);
  }
  double S = 0.0, A = 0.0, nx = 0.0, ny = 0.0, nz = 0.0, hx = 0.0, hy = 0.0, hz = 0.0, qx = 0.0, qy = 0.0, qz = 0.0;
  for (int j = 0; j < N; ++j) {
    const double4 a = pc[2 * j], b = pc[2 * j + 1];
    const double dx = l.x - a.x, dy = l.y - a.y, dz = l.z - a.z;
    const double w = exp64n(-fma(dx, dx, fma(dy, dy, dz * dz)) * a.w - m);
    const double h = fma(b.x, dx, fma(b.y, dy, b.z * dz));
    S += w;
    A = fma(w, h, A);
    if (GRAD) {
      nx = fma(w, b.x, nx); ny = fma(w, b.y, ny); nz = fma(w, b.z, nz);
      const double wq = -w * b.w;   // w * g_j / (l - p_j)
      qx = fma(wq, dx, qx); qy = fma(wq, dy, qy); qz = fma(wq, dz, qz);
      hx = fma(wq * h, dx, hx); hy = fma(wq * h, dy, hy); hz = fma(wq * h, dz, hz);
    }
  }
  const double iS = 1.0 / S;
  phi = A * iS;
  if (GRAD) g = d3((nx + hx - phi * qx) * iS, (ny + hy - phi * qy) * iS, (nz + hz - phi * qz) * iS);
}

// SDF value of a body at a pair-frame point with a float64 LSE for
// polytopes (float64 weights and logarithm): the pre-selection metrics, whose
// differences are divided by tau in the selection weights.  IDENT: the body
// is A.
template <bool IDENT, bool SQ = false>
__device__ __forceinline__ double sdf_value64(const BodyView& B, const D3& x, const Temp& T) {
  D3 l = x;
  if (!IDENT) {
    const double dx = x.x - B.t[0], dy = x.y - B.t[1], dz = x.z - B.t[2];
    l = d3(B.R[0] * dx + B.R[3] * dy + B.R[6] * dz, B.R[1] * dx + B.R[4] * dy + B.R[7] * dz,
           B.R[2] * dx + B.R[5] * dy + B.R[8] * dz);
  }
  if (SQ && B.type == CM_SQ_UNION) {
    double phi;
    D3 g;
    sdf_squnion<false, false>(B.planes, B.nf, l, T, phi, g);
    return phi;
  }
  if (SQ && B.type == CM_OPC) {
    double phi;
    D3 g;
    sdf_opc<false>(B.planes, B.nf, l, phi, g);
    return phi;
  }
  if (B.type != CM_POLYTOPE) {
    double phi;
    D3 g;
    sdf_analytic(B.type, B.p, l, phi, g);
    return phi;
  }
  double m = -1e300;
  for (int f = 0; f < B.nf; ++f) {
    const double4 q = B.planes[f];
    m = fmax(m, fma(q.x, l.x, fma(q.y, l.y, fma(q.z, l.z, -q.w))));
  }
  double S = 0.0;
  for (int f = 0; f < B.nf; ++f) {
    const double4 q = B.planes[f];
    S += exp2_64(fma(q.x, l.x, fma(q.y, l.y, fma(q.z, l.z, -q.w))) - m);
  }
  return T.tl * (m + log2_64(S));
}

// SDF of a body at a pair-frame point; gradient returned in the pair frame.
// MODE: SdfMode (kValue leaves g untouched, kSurfGrad leaves phi untouched
// for polytopes).  IDENT: the body is A, whose frame is the pair frame.
// mk: face subset for polytopes, shared by every active lane of the wave
// (null or mk->n == 0: all faces).  NDIR: for superquadric unions return the
// V-S normal direction (from grad f) instead of grad phi.  SQ: the extended
// primitives (superquadric unions, oriented point clouds) are handled, in
// the kernels built for contexts that hold them only (their loops would
// raise every call site's register pressure).
template <int MODE, bool IDENT, bool NDIR = false, bool SQ = false>
__device__ __forceinline__ void sdf_body(const BodyView& B, const D3& x, const Temp& T, double& phi, D3& g,
                                         const FaceMask* mk = nullptr, double shift = kNoShift) {
  D3 l = x;
  if (!IDENT) {
    const double dx = x.x - B.t[0], dy = x.y - B.t[1], dz = x.z - B.t[2];
    l = d3(B.R[0] * dx + B.R[3] * dy + B.R[6] * dz, B.R[1] * dx + B.R[4] * dy + B.R[7] * dz,
           B.R[2] * dx + B.R[5] * dy + B.R[8] * dz);
  }
  D3 lg;
  if (B.type == CM_POLYTOPE) {
    if (mk && mk->n > 0) sdf_poly_masked<MODE>(B.planes, B.nf, *mk, l, T, phi, lg, shift);
    else sdf_poly<MODE>(B.planes, B.nf, l, T, phi, lg);
  } else if (SQ && B.type == CM_SQ_UNION) {
    sdf_squnion<MODE != kValue, NDIR>(B.planes, B.nf, l, T, phi, lg);
  } else if (SQ && B.type == CM_OPC) {
    sdf_opc<MODE != kValue>(B.planes, B.nf, l, phi, lg);
  } else {
    sdf_analytic(B.type, B.p, l, phi, lg);
  }
  if (MODE != kValue) {
    if (IDENT) g = lg;
    else g = d3(B.R[0] * lg.x + B.R[1] * lg.y + B.R[2] * lg.z, B.R[3] * lg.x + B.R[4] * lg.y + B.R[5] * lg.z,
                B.R[6] * lg.x + B.R[7] * lg.y + B.R[8] * lg.z);
  }
}

// ----------------------------------------------------------------- E-E QP
// Edge e of a body in LDS (pair frame, structure of arrays of doubles):
// p0 = (x0, y0, z0), t = (tx, ty, tz).
struct EdgeSoA {
  double* x0; double* y0; double* z0; double* tx; double* ty; double* tz;
  __device__ __forceinline__ void get(int e, D3& p0, D3& t) const {
    p0 = d3(x0[e], y0[e], z0[e]);
    t = d3(tx[e], ty[e], tz[e]);
  }
};

struct EEQP {
  double al1, al2, log_con;
  D3 de;      // Delta e = e1 - e2
  double con; // the inside-box indicator itself (set by ee_qp only)
};

// The QP result from its solution: Delta e = (a0 - b0) + al1 t1 - al2 t2.
__device__ __forceinline__ EEQP ee_from_alpha(const D3& a0, const D3& t1, const D3& b0, const D3& t2, double al1,
                                              double al2, double log_con) {
  const D3 b = d3(a0.x - b0.x, a0.y - b0.y, a0.z - b0.z);
  EEQP r;
  r.al1 = al1;
  r.al2 = al2;
  r.log_con = log_con;
  r.de = d3(b.x + al1 * t1.x - al2 * t2.x, b.y + al1 * t1.y - al2 * t2.y, b.z + al1 * t1.z - al2 * t2.z);
  return r;
}

// Smoothed analytic active-set solution of the regularised E-E QP
// (Sec. IV-D-2): unconstrained minimiser -Q^{-1} c, four soft-clipped
// box-edge minimisers blended by a soft argmin of their objective values,
// soft inside-box indicator, blend.  Objective values are evaluated in the
// residual form 1/2 |b + A al|^2 + lambda/2 |al - 1/2|^2, which differs from
// 1/2 al^T Q al + c^T al by a constant (the soft argmin is shift invariant).
__device__ __forceinline__ EEQP ee_qp(const D3& a0, const D3& t1, const D3& b0, const D3& t2, double lam,
                                      const Temp& T) {
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
  const double i11 = rcp64(Q11), i22 = rcp64(Q22);
  const double xa = clip01(-(Q12 + c2) * i22, T);   // on al1 = 1
  const double xb = clip01(-c2 * i22, T);           // on al1 = 0
  const double xc = clip01(-(Q12 + c1) * i11, T);   // on al2 = 1
  const double xd = clip01(-c1 * i11, T);           // on al2 = 0
  auto cost = [&](double a1, double a2) {
    const double rx = b.x + a1 * t1.x - a2 * t2.x;
    const double ry = b.y + a1 * t1.y - a2 * t2.y;
    const double rz = b.z + a1 * t1.z - a2 * t2.z;
    const double u = a1 - 0.5, v = a2 - 0.5;
    return 0.5 * ((rx * rx + ry * ry + rz * rz) + lam * (u * u + v * v));
  };
  const double j0 = cost(1.0, xa), j1 = cost(0.0, xb), j2 = cost(xc, 1.0), j3 = cost(xd, 0.0);
  const double jm = fmin(fmin(j0, j1), fmin(j2, j3));
  // soft argmin weights and the inside-box indicator move the witness
  // points directly, so they use float64 exponentials
  const double w0 = exp64n(-(j0 - jm) * T.inv_tau), w1 = exp64n(-(j1 - jm) * T.inv_tau);
  const double w2 = exp64n(-(j2 - jm) * T.inv_tau), w3 = exp64n(-(j3 - jm) * T.inv_tau);
  const double iw = rcp64((w0 + w1) + (w2 + w3));
  const double ac1 = (w0 + w2 * xc + w3 * xd) * iw;
  const double ac2 = (w0 * xa + w1 * xb + w2) * iw;
  // the product of the four logistic factors sigma(x / tau) of the box test,
  // each m / (1 + e) with e = exp(-|x| / tau) and m = 1 (x >= 0) or e, over
  // one reciprocal
  double num = 1.0, den = 1.0;
  auto factor = [&](double x) {
    const double e = exp64n(-fabs(x) * T.inv_tau);
    num *= x >= 0.0 ? 1.0 : e;
    den *= 1.0 + e;
  };
  factor(au1);
  factor(1.0 - au1);
  factor(au2);
  factor(1.0 - au2);
  const double con = num * rcp64(den);
  const double log_con = (lsig(au1, T) + lsig(1.0 - au1, T)) + (lsig(au2, T) + lsig(1.0 - au2, T));
  EEQP r = ee_from_alpha(a0, t1, b0, t2, con * au1 + (1.0 - con) * ac1, con * au2 + (1.0 - con) * ac2, log_con);
  r.con = con;
  return r;
}

// ----------------------------------------------------------------- candidates
struct Cand {
  double s;     // score -d + tau ln w
  double d;     // signed distance
  double lw;    // ln w
  D3 p;         // point (pair frame)
  D3 n;         // pair normal A -> B (pair frame)
};

// Both E-E witness candidates of edge pair (k, l) (Sec. IV-D-3 and the
// activity indicator): sign via soft sign of the opposing SDF gradient,
// penetration via the opposing SDF value, clashing via both gradients,
// nearest neighbour via the row / column LSE of the unsigned distances.
// q is the edge pair's QP solution (ee_qp).  m1 / m2: null (all faces), or
// the face masks (A's faces, B's faces) for the queries at e1 / e2, shared by
// every active lane of the wave.  OWN_FULL: the edges are soft pre-selected
// averages, which need not lie on their own bodies' surfaces, so the
// own-body queries are full ones; safeguard then multiplies both activities
// by sigma(-phi_A(e1)/tau) sigma(-phi_B(e2)/tau).  REFINE: each witness is
// first traced onto its own body's smoothed surface (Supp., sphere tracing):
// along the fixed unit direction of grad phi at the QP witness, x <- x -
// phi(x) n, `steps` times; points, distances, normals and the sign /
// penetration / clashing tests use the traced points, the nearest-neighbour
// term keeps the QP distance, and every query visits all faces (a moved
// point is outside what the segment's face masks bound).
template <bool OWN_FULL = false, bool SQ = false, bool REFINE = false>
__device__ __forceinline__ void ee_candidates(const D3& a0, const D3& t1, const D3& b0, const D3& t2, const EEQP& q,
                                              double row_lse, double col_lse, const BodyView& A, const BodyView& B,
                                              double eps_n, const Temp& T, const FaceMask* m1, const FaceMask* m2,
                                              Cand& c1, Cand& c2, bool safeguard = false, int steps = 0,
                                              double sh1 = kNoShift, double sh2 = kNoShift) {
  D3 e1 = d3(a0.x + q.al1 * t1.x, a0.y + q.al1 * t1.y, a0.z + q.al1 * t1.z);
  D3 e2 = d3(b0.x + q.al2 * t2.x, b0.y + q.al2 * t2.y, b0.z + q.al2 * t2.z);
  double dqp, idum;   // dqp: the nearest-neighbour term's distance
  sqrt_rsq64(dot(q.de, q.de), dqp, idum);
  D3 de = q.de;
  if (REFINE) {
    m1 = nullptr;
    m2 = nullptr;
    double ph;
    D3 g, dg;
    sdf_body<kFull, true, false, SQ>(A, e1, T, ph, g);
    double in = rcp64(sqrt(dot(g, g)));
    const D3 n1 = d3(g.x * in, g.y * in, g.z * in);
    for (int s = 0; s < steps; ++s) {
      if (s > 0) sdf_body<kValue, true, false, SQ>(A, e1, T, ph, dg);
      e1 = d3(e1.x - ph * n1.x, e1.y - ph * n1.y, e1.z - ph * n1.z);
    }
    sdf_body<kFull, false, false, SQ>(B, e2, T, ph, g);
    in = rcp64(sqrt(dot(g, g)));
    const D3 n2 = d3(g.x * in, g.y * in, g.z * in);
    for (int s = 0; s < steps; ++s) {
      if (s > 0) sdf_body<kValue, false, false, SQ>(B, e2, T, ph, dg);
      e2 = d3(e2.x - ph * n2.x, e2.y - ph * n2.y, e2.z - ph * n2.z);
    }
    de = d3(e1.x - e2.x, e1.y - e2.y, e1.z - e2.z);
  }
  const double dsq = dot(de, de);
  const double dbar = REFINE ? sqrt(dsq) : dqp;
  const double in = rsq64(dsq + eps_n);
  const D3 nb = d3(de.x * in, de.y * in, de.z * in);
  double phiB1, phiA2, dum;
  D3 gA, gB, dg;
  double phiA1 = 0.0, phiB2 = 0.0;
  sdf_body<kValue, false, false, SQ>(B, e1, T, phiB1, dg, m1 ? m1 + 1 : nullptr, sh1);
  if (OWN_FULL || REFINE) sdf_body<kFull, true, false, SQ>(A, e1, T, phiA1, gA, m1);
  else sdf_body<kSurfGrad, true, false, SQ>(A, e1, T, dum, gA, m1);                   // e1 lies on an edge of A
  sdf_body<kValue, true, false, SQ>(A, e2, T, phiA2, dg, m2, sh2);
  if (OWN_FULL || REFINE) sdf_body<kFull, false, false, SQ>(B, e2, T, phiB2, gB, m2 ? m2 + 1 : nullptr);
  else sdf_body<kSurfGrad, false, false, SQ>(B, e2, T, dum, gB, m2 ? m2 + 1 : nullptr);   // e2 lies on an edge of B
  const double gam1 = tanh64(dot(gB, nb), T);
  const double gam2 = tanh64(-dot(gA, nb), T);
  double base = q.log_con + lsig(-dot(gA, gB), T);
  if (OWN_FULL && safeguard) base += lsig(-phiA1, T) + lsig(-phiB2, T);
  const double lp1 = base + lsig(-phiB1, T);
  const double lp2 = base + lsig(-phiA2, T);
  c1.d = gam1 * dbar;
  c2.d = gam2 * dbar;
  c1.lw = lp1 + (row_lse - dqp) * T.inv_tau;
  c2.lw = lp2 + (col_lse - dqp) * T.inv_tau;
  c1.s = -c1.d + T.tau * lp1 + (row_lse - dqp);
  c2.s = -c2.d + T.tau * lp2 + (col_lse - dqp);
  c1.p = e1;
  c2.p = e2;
  // witness 1: nu = -gam1 n_bar; witness 2: nu = gam2 (-n_bar)
  c1.n = d3(-gam1 * nb.x, -gam1 * nb.y, -gam1 * nb.z);
  c2.n = d3(-gam2 * nb.x, -gam2 * nb.y, -gam2 * nb.z);
}

// V-S candidate (Sec. IV-C): vertex v (pair frame) of one body against the
// SDF of the other; sgn = -1 for A's vertices (the normal of B pushes A),
// +1 for B's vertices.  OTHER_IS_A: the SDF is A's (identity frame).
template <bool OTHER_IS_A, bool SQ = false>
__device__ __forceinline__ void vs_candidate(const D3& v, const BodyView& other, double sgn, const Temp& T,
                                             Cand& c) {
  double phi;
  D3 g;
  sdf_body<kFull, OTHER_IS_A, true, SQ>(other, v, T, phi, g);
  const double in = sgn * rsq64(T.tau + dot(g, g));
  c.p = v;
  c.n = d3(g.x * in, g.y * in, g.z * in);
  c.d = phi;
  c.lw = lsig(-phi, T);
  c.s = -phi + T.tau * c.lw;
}

// ----------------------------------------------------------------- waves
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// merge (min m, sum s of exp(-(x - m)/tau)) pairs across a wave
__device__ __forceinline__ void wave_lse_merge(double& m, float& s, const Temp& T) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double m2 = __shfl_xor(m, o, 64);
    const float s2 = __shfl_xor(s, o, 64);
    const double M = fmin(m, m2);
    const float a = (m == M) ? s : s * expn(m - M, T);
    const float b = (m2 == M) ? s2 : s2 * expn(m2 - M, T);
    m = M; s = a + b;
  }
}
// online update of (m, s) with a new value x: one exp, branch free
__device__ __forceinline__ void lse_push(double& m, float& s, double x, const Temp& T) {
  const float e = expn(fabs(x - m), T);
  const bool lower = x < m;
  s = lower ? fmaf(s, e, 1.f) : s + e;
  m = lower ? x : m;
}

// quaternion (w, x, y, z), not necessarily unit -> rotation matrix (row-major)
__device__ __forceinline__ void quat_to_R(double w, double x, double y, double z, double* R) {
  const double in = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  w *= in; x *= in; y *= in; z *= in;
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}

}  // namespace cm
