// Reverse-mode derivatives of the per-candidate computations (the gradient
// the paper obtains by automatic differentiation of the routine).  Each
// function recomputes its forward intermediates from the inputs, then walks
// the operations backwards.  Derivative conventions at kinks: |x|' = sign(x)
// with sign(0) = 0 for the SoftSort distance, clamp' = 1 inside / 0 outside,
// the rounded-box interior face is the lowest index of the maximum.
#pragma once
#include "cm_device.cuh"

namespace cm {

__device__ __forceinline__ D3 add(const D3& a, const D3& b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ D3 sub(const D3& a, const D3& b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ D3 scl(const D3& a, double s) { return d3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ D3 axpy(double s, const D3& a, const D3& b) { return d3(fma(s, a.x, b.x), fma(s, a.y, b.y), fma(s, a.z, b.z)); }
__device__ __forceinline__ D3 cross(const D3& a, const D3& b) {
  return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ D3 rot(const double* R, const D3& v) {
  return d3(R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z, R[6] * v.x + R[7] * v.y + R[8] * v.z);
}
__device__ __forceinline__ D3 rotT(const double* R, const D3& v) {
  return d3(R[0] * v.x + R[3] * v.y + R[6] * v.z, R[1] * v.x + R[4] * v.y + R[7] * v.z, R[2] * v.x + R[5] * v.y + R[8] * v.z);
}

// d/du and d/dtau of ln sigma(u / tau)
__device__ __forceinline__ void lsig_d(double u, const Temp& T, double& du, double& dtau) {
  const double om = sig64(-u, T);           // 1 - sigma(u / tau)
  du = om * T.inv_tau;
  dtau = -u * om * T.inv_tau * T.inv_tau;
}

// A staged face plane (scaled by log2(e) / tau) back in length units.
__device__ __forceinline__ double4 unscaled(const double4& q, const Temp& T) {
  return make_double4(q.x * T.tl, q.y * T.tl, q.z * T.tl, q.w * T.tl);
}

// Wave sum of a float into lane 63 (all 64 lanes must participate), with
// DPP moves only (no LDS permutes): pairs and quads (quad_perm), the two
// halves of each row of 16 lanes (row_half_mirror, row_mirror), then the row
// broadcasts: lane 15 of rows 0 / 2 into rows 1 / 3, lane 31 into rows 2, 3.
// The other lanes end with partial sums.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float x) {
  return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROWS, 0xf, false));
}
__device__ __forceinline__ float wave_sum_last(float v) {
  v = dpp_add<0xb1, 0xf>(v);    // quad_perm [1, 0, 3, 2]
  v = dpp_add<0x4e, 0xf>(v);    // quad_perm [2, 3, 0, 1]
  v = dpp_add<0x141, 0xf>(v);   // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);   // row_mirror
  v = dpp_add<0x142, 0xa>(v);   // row_bcast:15 into rows 1, 3
  v = dpp_add<0x143, 0xc>(v);   // row_bcast:31 into rows 2, 3
  return v;
}

// ---- forward-mode derivatives for superquadric unions
// A float64 value with its derivatives along four inputs (the query point's
// x, y, z and tau).  Evaluating the union with it yields the Jacobian of
// (phi, gradient) in one pass, Hessian terms included.
struct Dual4 {
  double v, d[4];
};
__device__ __forceinline__ Dual4 dconst(double v) { return Dual4{v, {0.0, 0.0, 0.0, 0.0}}; }
__device__ __forceinline__ Dual4 dvar(double v, int k) {
  Dual4 r = dconst(v);
  r.d[k] = 1.0;
  return r;
}
__device__ __forceinline__ Dual4 operator+(const Dual4& a, const Dual4& b) {
  return Dual4{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2], a.d[3] + b.d[3]}};
}
__device__ __forceinline__ Dual4 operator-(const Dual4& a, const Dual4& b) {
  return Dual4{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2], a.d[3] - b.d[3]}};
}
__device__ __forceinline__ Dual4 operator*(const Dual4& a, const Dual4& b) {
  Dual4 r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
__device__ __forceinline__ Dual4 operator*(double s, const Dual4& a) {
  return Dual4{s * a.v, {s * a.d[0], s * a.d[1], s * a.d[2], s * a.d[3]}};
}
__device__ __forceinline__ Dual4 operator/(const Dual4& a, const Dual4& b) {
  const double ib = 1.0 / b.v, q = a.v * ib;
  Dual4 r;
  r.v = q;
#pragma unroll
  for (int k = 0; k < 4; ++k) r.d[k] = (a.d[k] - q * b.d[k]) * ib;
  return r;
}
// f(a) with f(a.v) = fv and f'(a.v) = fd
__device__ __forceinline__ Dual4 dchain(const Dual4& a, double fv, double fd) {
  return Dual4{fv, {fd * a.d[0], fd * a.d[1], fd * a.d[2], fd * a.d[3]}};
}
__device__ __forceinline__ Dual4 dsqrt(const Dual4& a) {
  const double s = sqrt(a.v);
  return dchain(a, s, s > 0.0 ? 0.5 / s : 0.0);
}
__device__ __forceinline__ Dual4 dexp2(const Dual4& a) {
  const double e = exp2(a.v);
  return dchain(a, e, e * kLn2);
}
__device__ __forceinline__ Dual4 dlog2(const Dual4& a) { return dchain(a, log2(a.v), 1.0 / (a.v * kLn2)); }
__device__ __forceinline__ Dual4 dexp(const Dual4& a) {
  const double e = exp(a.v);
  return dchain(a, e, e);
}

// The superquadric union of sdf_squnion (same records, same definitions)
// over Dual4 inputs: phi and either grad phi or (ndir) the V-S normal
// direction sum_i pi_i grad f_i, each with its derivatives.  Powers (s^2)^p
// are taken as 2^(p log2 s^2) where s != 0 and as 0 at s = 0, where their
// derivatives (2p > 1) vanish too.
__device__ __forceinline__ void sq_union_dual(const double4* __restrict__ sq, int nslots, const Dual4& lx,
                                              const Dual4& ly, const Dual4& lz, const Dual4& tau, bool ndir,
                                              Dual4& phi, Dual4& gx, Dual4& gy, Dual4& gz) {
  const int M = nslots / 5;
  const Dual4 itau = dconst(1.0) / tau;
  Dual4 mn = dconst(0.0), S = dconst(0.0), ax = dconst(0.0), ay = dconst(0.0), az = dconst(0.0);
  auto ppow = [](const Dual4& s, double p) {   // (s^2)^p
    if (s.v == 0.0) return dconst(0.0);
    return dexp2(p * dlog2(s * s));
  };
  for (int i = 0; i < M; ++i) {
    const double4 r0 = sq[5 * i], r1 = sq[5 * i + 1], r2 = sq[5 * i + 2], s3 = sq[5 * i + 3], s4 = sq[5 * i + 4];
    const Dual4 dx = lx - dconst(r0.w), dy = ly - dconst(r1.w), dz = lz - dconst(r2.w);
    const Dual4 yx = r0.x * dx + r0.y * dy + r0.z * dz;
    const Dual4 yy = r1.x * dx + r1.y * dy + r1.z * dz;
    const Dual4 yz = r2.x * dx + r2.y * dy + r2.z * dz;
    const Dual4 sx = s3.x * yx, sy = s3.y * yy, sz = s3.z * yz;
    const double e1 = s3.w, ie2 = s4.x, r21 = s4.y, ie1 = s4.z;
    const Dual4 Ax = ppow(sx, ie2), Ay = ppow(sy, ie2), Cz = ppow(sz, ie1);
    const Dual4 u = Ax + Ay;
    const Dual4 U = u.v > 0.0 ? dexp2(r21 * dlog2(u)) : dconst(0.0);
    const Dual4 f = U + Cz;
    const Dual4 r = dsqrt(yx * yx + yy * yy + yz * yz);
    const Dual4 q = dexp2((-0.5 * e1) * dlog2(f));
    const Dual4 ph = r * (dconst(1.0) - q);
    // grad f in the primitive frame: d/ds (s^2)^p = 2 p (s^2)^p / s
    const Dual4 du = u.v > 0.0 ? r21 * (U / u) : dconst(0.0);
    const Dual4 gfx = sx.v != 0.0 ? (2.0 * ie2 * s3.x) * (du * (Ax / sx)) : dconst(0.0);
    const Dual4 gfy = sy.v != 0.0 ? (2.0 * ie2 * s3.y) * (du * (Ay / sy)) : dconst(0.0);
    const Dual4 gfz = sz.v != 0.0 ? (2.0 * ie1 * s3.z) * (Cz / sz) : dconst(0.0);
    Dual4 hx = gfx, hy = gfy, hz = gfz;
    if (!ndir) {
      const Dual4 a = r.v > 0.0 ? (dconst(1.0) - q) / r : dconst(0.0);
      const Dual4 b = (0.5 * e1) * (r * q / f);
      hx = a * yx + b * gfx; hy = a * yy + b * gfy; hz = a * yz + b * gfz;
    }
    const Dual4 vx = r0.x * hx + r1.x * hy + r2.x * hz;
    const Dual4 vy = r0.y * hx + r1.y * hy + r2.y * hz;
    const Dual4 vz = r0.z * hx + r1.z * hy + r2.z * hz;
    if (i == 0) {
      mn = ph; S = dconst(1.0); ax = vx; ay = vy; az = vz;
    } else if (ph.v < mn.v) {
      const Dual4 sc = dexp((ph - mn) * itau);
      S = S * sc + dconst(1.0); ax = ax * sc + vx; ay = ay * sc + vy; az = az * sc + vz;
      mn = ph;
    } else {
      const Dual4 w = dexp((mn - ph) * itau);
      S = S + w; ax = ax + w * vx; ay = ay + w * vy; az = az + w * vz;
    }
  }
  phi = mn - kLn2 * (tau * dlog2(S));
  gx = ax / S; gy = ay / S; gz = az / S;
}

// The oriented point cloud of sdf_opc over Dual4 inputs: phi and grad phi
// with their derivatives (no tau dependence).
__device__ __forceinline__ void opc_dual(const double4* __restrict__ pc, int nslots, const Dual4& lx, const Dual4& ly,
                                         const Dual4& lz, Dual4& phi, Dual4& gx, Dual4& gy, Dual4& gz) {
  const int N = nslots / 2;
  double m = -INFINITY;
  for (int j = 0; j < N; ++j) {
    const double4 a = pc[2 * j];
    const double dx = lx.v - a.x, dy = ly.v - a.y, dz = lz.v - a.z;
    m = fmax(m, -(dx * dx + dy * dy + dz * dz) * a.w);
  }
  Dual4 S = dconst(0.0), A = dconst(0.0), nx = dconst(0.0), ny = dconst(0.0), nz = dconst(0.0);
  Dual4 hx = dconst(0.0), hy = dconst(0.0), hz = dconst(0.0), qx = dconst(0.0), qy = dconst(0.0), qz = dconst(0.0);
  for (int j = 0; j < N; ++j) {
    const double4 a = pc[2 * j], b = pc[2 * j + 1];
    const Dual4 dx = lx - dconst(a.x), dy = ly - dconst(a.y), dz = lz - dconst(a.z);
    const Dual4 w = dexp((-a.w) * (dx * dx + dy * dy + dz * dz) - dconst(m));
    const Dual4 h = b.x * dx + b.y * dy + b.z * dz;
    S = S + w;
    A = A + w * h;
    nx = nx + b.x * w; ny = ny + b.y * w; nz = nz + b.z * w;
    const Dual4 wq = (-b.w) * w;
    qx = qx + wq * dx; qy = qy + wq * dy; qz = qz + wq * dz;
    hx = hx + (wq * h) * dx; hy = hy + (wq * h) * dy; hz = hz + (wq * h) * dz;
  }
  phi = A / S;
  gx = (nx + hx - phi * qx) / S;
  gy = (ny + hy - phi * qy) / S;
  gz = (nz + hz - phi * qz) / S;
}

// Gradient sinks of one body during the adjoint of a pair (LDS, float atomics).
struct BodySink {
  float* plane;    // [4][maxF] adjoints of (n.xyz, o) in the body frame, or null
  float* param;    // [4] adjoints of the analytic parameters
  int maxF;
};

// Adjoint of the body-frame SDF query (phi, g) at l given (phi_bar, g_bar).
// Returns l_bar; accumulates parameter / plane adjoints and tau_bar.
// WAVE: all 64 lanes execute this call together (plane adjoints are summed
// across the wave, into lane 63, before one atomic per plane).
// SQ: superquadric unions are handled (kernels built for contexts holding
// them); ndir: the gradient output g_bar refers to is their V-S normal
// direction.  Their record adjoints are not accumulated (no geometry
// gradient for them); point and tau adjoints are.
template <bool WAVE, bool SQ = false>
__device__ __forceinline__ D3 sdf_local_bwd(int type, const float* p, const double4* __restrict__ pl, int nf, const D3& l,
                                            double phib, const D3& gb, const Temp& T, const BodySink& sink,
                                            double& taub, D3& g_out, bool ndir = false, bool surf = false,
                                            const FaceMask* mk = nullptr) {
  if (SQ && (type == CM_SQ_UNION || type == CM_OPC)) {
    Dual4 ph, gx, gy, gz;
    if (type == CM_SQ_UNION)
      sq_union_dual(pl, nf, dvar(l.x, 0), dvar(l.y, 1), dvar(l.z, 2), dvar(T.tau, 3), ndir, ph, gx, gy, gz);
    else
      opc_dual(pl, nf, dvar(l.x, 0), dvar(l.y, 1), dvar(l.z, 2), ph, gx, gy, gz);
    g_out = d3(gx.v, gy.v, gz.v);
    double o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) o[k] = phib * ph.d[k] + gb.x * gx.d[k] + gb.y * gy.d[k] + gb.z * gz.d[k];
    taub += o[3];
    return d3(o[0], o[1], o[2]);
  }
  if (type == CM_SPHERE) {
    double n, inv;
    sqrt_rsq64(dot(l, l), n, inv);
    const D3 g = scl(l, inv);
    g_out = g;
    const double gg = dot(g, gb);
    atomicAdd(&sink.param[0], float(-phib));
    return add(scl(g, phib), scl(sub(gb, scl(g, gg)), inv));
  }
  if (type == CM_CAPSULE) {
    const double h = p[1];
    const double zc = fmin(fmax(l.z, -h), h);
    const D3 y = d3(l.x, l.y, l.z - zc);
    double n, inv;
    sqrt_rsq64(dot(y, y), n, inv);
    const D3 g = scl(y, inv);
    g_out = g;
    const D3 yb = add(scl(g, phib), scl(sub(gb, scl(g, dot(g, gb))), inv));
    const bool above = l.z > h, below = l.z < -h;
    atomicAdd(&sink.param[0], float(-phib));
    atomicAdd(&sink.param[1], float(above ? -yb.z : (below ? yb.z : 0.0)));
    return d3(yb.x, yb.y, (above || below) ? yb.z : 0.0);
  }
  if (type == CM_BOX) {
    const double rr = p[3];
    const double q[3] = {fabs(l.x) - (double(p[0]) - rr), fabs(l.y) - (double(p[1]) - rr), fabs(l.z) - (double(p[2]) - rr)};
    const double sg[3] = {sgn1(l.x), sgn1(l.y), sgn1(l.z)};
    const double m[3] = {fmax(q[0], 0.0), fmax(q[1], 0.0), fmax(q[2], 0.0)};
    const double s = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    const double gbv[3] = {gb.x, gb.y, gb.z};
    double qb[3] = {0.0, 0.0, 0.0};
    double rhob = -phib;
    if (s > 0x1p-700) {
      double n, inv;
      sqrt_rsq64(s, n, inv);
      g_out = d3(sg[0] * m[0] * inv, sg[1] * m[1] * inv, sg[2] * m[2] * inv);
      // phi = |m| - rho ; g_i = sg_i m_i / |m|
      double sgb = 0.0;
      for (int i = 0; i < 3; ++i) sgb += sg[i] * gbv[i] * m[i];
      for (int i = 0; i < 3; ++i) {
        const double mb = phib * m[i] * inv + sg[i] * gbv[i] * inv - m[i] * sgb * inv * inv * inv;
        qb[i] = q[i] > 0.0 ? mb : 0.0;
      }
    } else {
      const int j = (q[0] >= q[1] && q[0] >= q[2]) ? 0 : (q[1] >= q[2] ? 1 : 2);
      g_out = d3(j == 0 ? sg[0] : 0.0, j == 1 ? sg[1] : 0.0, j == 2 ? sg[2] : 0.0);
      qb[j] = phib;
    }
    // q_i = |l_i| - (h_i - rho)
    for (int i = 0; i < 3; ++i) {
      atomicAdd(&sink.param[i], float(-qb[i]));
      rhob += qb[i];
    }
    atomicAdd(&sink.param[3], float(rhob));
    return d3(sg[0] * qb[0], sg[1] * qb[1], sg[2] * qb[2]);
  }
  // polytope: phi = tau LSE(y / tau), y_f = n_f . l - o_f, g = sum_f pi_f n_f.
  // surf (wave-uniform): every lane's point lies on the body's own boundary
  // (an E-E witness on its own edge), where the largest plane value is 0 up
  // to the smoothed witness's overshoot (as the forward's surface-gradient
  // query): the shift is 0 and the max pass is skipped.  mk: the faces to
  // visit, shared by every lane of the wave (null: all), as in the forward's
  // masked queries.
  double m = surf ? 0.0 : -1e300;
  if (!surf) {
    for_faces(mk, nf, [&](int f) __attribute__((always_inline)) {
      const double4 q = unscaled(pl[f], T);
      m = fmax(m, fma(q.x, l.x, fma(q.y, l.y, fma(q.z, l.z, -q.w))));
    });
  }
  double S = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, py = 0.0;
  for_faces(mk, nf, [&](int f) __attribute__((always_inline)) {
    const double4 q = unscaled(pl[f], T);
    const double yv = fma(q.x, l.x, fma(q.y, l.y, fma(q.z, l.z, -q.w)));
    const double a = (yv - m) * T.c;
    if (!__any(a > -40.0)) return;   // below 2^-40 on every lane, as the adjoint pass below
    const double e = double(ex2f(float(a)));
    S += e; gx = fma(e, q.x, gx); gy = fma(e, q.y, gy); gz = fma(e, q.z, gz);
    py = fma(e, yv, py);
  });
  const double iS = S > 0.0 ? rcp64(S) : 0.0;   // S >= 1 (the largest plane's term is about 1)
  const D3 g = d3(gx * iS, gy * iS, gz * iS);
  g_out = g;
  const double gbg = dot(gb, g);
  if (phib != 0.0) taub += phib * ((m + T.tau * log(S)) - py * iS) * T.inv_tau;
  D3 lb = d3(0.0, 0.0, 0.0);
  double tz = 0.0;
  for_faces(mk, nf, [&](int f) __attribute__((always_inline)) {
    const double4 q = unscaled(pl[f], T);
    const double yv = fma(q.x, l.x, fma(q.y, l.y, fma(q.z, l.z, -q.w)));
    const double a = (yv - m) * T.c;
    // a face whose softmax weight is below 2^-40 for every lane of the wave
    // (or every active lane) adds nothing the float32 sums could hold: skipped
    // together (wave-uniform, so the wave sums below stay whole-wave)
    if (!__any(a > -40.0)) return;
    const double pi = double(ex2f(float(a))) * iS;
    const double zb = pi * (gb.x * q.x + gb.y * q.y + gb.z * q.z - gbg);   // softmax adjoint of g
    const double yb = phib * pi + zb * T.inv_tau;
    tz += zb * yv;
    lb = d3(fma(yb, double(q.x), lb.x), fma(yb, double(q.y), lb.y), fma(yb, double(q.z), lb.z));
    if (sink.plane) {
      float v0 = float(yb * l.x + pi * gb.x), v1 = float(yb * l.y + pi * gb.y), v2 = float(yb * l.z + pi * gb.z),
            v3 = float(-yb);
      if (WAVE) {
        v0 = wave_sum_last(v0); v1 = wave_sum_last(v1); v2 = wave_sum_last(v2); v3 = wave_sum_last(v3);
        if ((threadIdx.x & 63) == 63) {
          atomicAdd(&sink.plane[f], v0); atomicAdd(&sink.plane[sink.maxF + f], v1);
          atomicAdd(&sink.plane[2 * sink.maxF + f], v2); atomicAdd(&sink.plane[3 * sink.maxF + f], v3);
        }
      } else {
        atomicAdd(&sink.plane[f], v0); atomicAdd(&sink.plane[sink.maxF + f], v1);
        atomicAdd(&sink.plane[2 * sink.maxF + f], v2); atomicAdd(&sink.plane[3 * sink.maxF + f], v3);
      }
    }
  });
  taub -= tz * T.inv_tau * T.inv_tau;
  return lb;
}

// Twist adjoint of body B's placement in the pair frame: rho and omega parts.
struct Twist {
  double r[3], w[3];
};

// Adjoint of an SDF query of body V at pair-frame point x.  IDENT: the body
// is A (pair frame).  For body B the query moves with B: its placement twist
// receives rho -= x_bar, omega += g x g_bar - x x x_bar.
template <bool WAVE, bool IDENT, bool SQ = false>
__device__ __forceinline__ D3 sdf_body_bwd(const BodyView& V, const D3& x, double phib, const D3& gb, const Temp& T,
                                           const BodySink& sink, double& taub, Twist& tw, bool ndir = false,
                                           bool surf = false, const FaceMask* mk = nullptr) {
  if (IDENT) {
    D3 g;
    return sdf_local_bwd<WAVE, SQ>(V.type, V.p, V.planes, V.nf, x, phib, gb, T, sink, taub, g, ndir, surf, mk);
  }
  const D3 l = rotT(V.R, sub(x, d3(V.t[0], V.t[1], V.t[2])));
  const D3 gbl = rotT(V.R, gb);
  D3 gl;
  const D3 lb = sdf_local_bwd<WAVE, SQ>(V.type, V.p, V.planes, V.nf, l, phib, gbl, T, sink, taub, gl, ndir, surf, mk);
  const D3 xb = rot(V.R, lb);
  const D3 g = rot(V.R, gl);
  const D3 c1 = cross(g, gb), c2 = cross(x, xb);
  tw.r[0] -= xb.x; tw.r[1] -= xb.y; tw.r[2] -= xb.z;
  tw.w[0] += c1.x - c2.x; tw.w[1] += c1.y - c2.y; tw.w[2] += c1.z - c2.z;
  return xb;
}

// ---- witness sphere tracing (Supp., refinement of the witness points)
// Forward: (phi_0, g) = the full query at the QP witness w, n = g / |g|,
// x_0 = w, x_{s+1} = x_s - phi(x_s) n for s < steps (phi(x_0) = phi_0).  The
// step values phi_s are kept for the reverse; x_s is rebuilt from them.
struct Trace {
  D3 w, n;                    // start point, unit direction (0 on lanes that do not trace)
  double ig;                  // 1 / |grad phi(w)|
  double ph[CM_MAX_REFINE];   // phi(x_s)
};

__device__ __forceinline__ void trace_none(const D3& x, Trace& tr) {
  tr.w = x;
  tr.n = d3(0.0, 0.0, 0.0);
  tr.ig = 0.0;
  for (int s = 0; s < CM_MAX_REFINE; ++s) tr.ph[s] = 0.0;
}

// The same operations, in the same order, as the forward's tracing; returns x_steps.
template <bool IDENT, bool SQ>
__device__ __forceinline__ D3 trace_fwd(const BodyView& V, const D3& w, const Temp& T, int steps, Trace& tr) {
  double ph;
  D3 g, dg;
  sdf_body<kFull, IDENT, false, SQ>(V, w, T, ph, g);
  const double in = rcp64(sqrt(dot(g, g)));
  tr.w = w;
  tr.ig = in;
  tr.n = d3(g.x * in, g.y * in, g.z * in);
  for (int s = 0; s < CM_MAX_REFINE; ++s) tr.ph[s] = 0.0;
  D3 x = w;
  for (int s = 0; s < steps; ++s) {
    if (s > 0) sdf_body<kValue, IDENT, false, SQ>(V, x, T, ph, dg);
    tr.ph[s] = ph;
    x = d3(x.x - ph * tr.n.x, x.y - ph * tr.n.y, x.z - ph * tr.n.z);
  }
  return x;
}

// Reverse of trace_fwd: given the adjoint xb of x_steps returns that of w.
// x_{s+1} = x_s - phi_s n gives x_s_bar += grad phi(x_s) (-n . x_{s+1}_bar)
// and n_bar -= phi_s x_{s+1}_bar; at s = 0 the query at w also carries the
// direction's gradient adjoint (n_bar - n (n . n_bar)) / |g|.  Every lane of
// the wave calls this together (wave-summed plane adjoints); a lane that does
// not trace passes xb = 0 and trace_none's record.
template <bool IDENT, bool SQ>
__device__ __forceinline__ D3 trace_bwd(const BodyView& V, const Trace& tr, D3 xb, const Temp& T, int steps,
                                        const BodySink& sink, double& taub, Twist& tw) {
  const D3 zero = d3(0.0, 0.0, 0.0);
  double c = 0.0;
  for (int s = 0; s < steps; ++s) c += tr.ph[s];
  D3 nb = zero;
  for (int s = steps - 1; s >= 1; --s) {
    c -= tr.ph[s];   // x_s = w - (phi_0 + ... + phi_{s-1}) n
    const D3 x = d3(tr.w.x - c * tr.n.x, tr.w.y - c * tr.n.y, tr.w.z - c * tr.n.z);
    nb = axpy(-tr.ph[s], xb, nb);
    xb = add(xb, sdf_body_bwd<true, IDENT, SQ>(V, x, -dot(tr.n, xb), zero, T, sink, taub, tw));
  }
  nb = axpy(-tr.ph[0], xb, nb);
  const D3 gb = scl(sub(nb, scl(tr.n, dot(tr.n, nb))), tr.ig);
  return add(xb, sdf_body_bwd<true, IDENT, SQ>(V, tr.w, -dot(tr.n, xb), gb, T, sink, taub, tw));
}

// Adjoint of the smoothed E-E QP (recomputes the forward).  Given adjoints of
// (al1, al2, log_con) accumulates adjoints of the edge data a0, t1, b0, t2 and tau.
__device__ __forceinline__ void ee_qp_bwd(const D3& a0, const D3& t1, const D3& b0, const D3& t2, double lam,
                                          const Temp& T, double al1b, double al2b, double lcb, D3& a0b, D3& t1b,
                                          D3& b0b, D3& t2b, double& taub) {
  // ---- forward
  const D3 b = sub(a0, b0);
  const double Q11 = dot(t1, t1) + lam, Q22 = dot(t2, t2) + lam, Q12 = -dot(t1, t2);
  const double hl = 0.5 * lam;
  const double c1 = dot(b, t1) - hl, c2 = -dot(b, t2) - hl;
  const double det = Q11 * Q22 - Q12 * Q12, idet = rcp64(det);   // as the forward QP
  const double au1 = (Q12 * c2 - c1 * Q22) * idet, au2 = (Q12 * c1 - c2 * Q11) * idet;
  const double i11 = rcp64(Q11), i22 = rcp64(Q22);
  const double xi[4] = {-(Q12 + c2) * i22, -c2 * i22, -(Q12 + c1) * i11, -c1 * i11};
  double x[4];
  for (int i = 0; i < 4; ++i) x[i] = clip01(xi[i], T);
  const double A1[4] = {1.0, 0.0, x[2], x[3]}, A2[4] = {x[0], x[1], 1.0, 0.0};
  D3 r[4];
  double j[4];
  for (int i = 0; i < 4; ++i) {
    r[i] = d3(b.x + A1[i] * t1.x - A2[i] * t2.x, b.y + A1[i] * t1.y - A2[i] * t2.y, b.z + A1[i] * t1.z - A2[i] * t2.z);
    const double u = A1[i] - 0.5, v = A2[i] - 0.5;
    j[i] = 0.5 * (dot(r[i], r[i]) + lam * (u * u + v * v));
  }
  const double jm = fmin(fmin(j[0], j[1]), fmin(j[2], j[3]));
  double w[4], ws = 0.0;
  for (int i = 0; i < 4; ++i) { w[i] = exp64n(-(j[i] - jm) * T.inv_tau); ws += w[i]; }
  double pi[4];
  for (int i = 0; i < 4; ++i) pi[i] = w[i] / ws;
  const double ac1 = pi[0] + pi[2] * x[2] + pi[3] * x[3];
  const double ac2 = pi[0] * x[0] + pi[1] * x[1] + pi[2];
  const double u[4] = {au1, 1.0 - au1, au2, 1.0 - au2};
  double Sg[4];
  for (int i = 0; i < 4; ++i) Sg[i] = sig64(u[i], T);
  const double con = (Sg[0] * Sg[1]) * (Sg[2] * Sg[3]);
  // ---- reverse
  const double conb = al1b * (au1 - ac1) + al2b * (au2 - ac2);
  double au1b = al1b * con, au2b = al2b * con;
  const double ac1b = al1b * (1.0 - con), ac2b = al2b * (1.0 - con);
  const double W = conb * con + lcb;
  au1b += W * ((1.0 - Sg[0]) - (1.0 - Sg[1])) * T.inv_tau;
  au2b += W * ((1.0 - Sg[2]) - (1.0 - Sg[3])) * T.inv_tau;
  taub -= W * (u[0] * (1.0 - Sg[0]) + u[1] * (1.0 - Sg[1]) + u[2] * (1.0 - Sg[2]) + u[3] * (1.0 - Sg[3])) *
          T.inv_tau * T.inv_tau;
  const double pib[4] = {ac1b + ac2b * x[0], ac2b * x[1], ac1b * x[2] + ac2b, ac1b * x[3]};
  double xb[4] = {ac2b * pi[0], ac2b * pi[1], ac1b * pi[2], ac1b * pi[3]};
  double ps = 0.0;
  for (int i = 0; i < 4; ++i) ps += pi[i] * pib[i];
  D3 bb = d3(0.0, 0.0, 0.0);
  for (int i = 0; i < 4; ++i) {
    const double zb = pi[i] * (pib[i] - ps);
    const double jb = -zb * T.inv_tau;
    taub += zb * (j[i] - jm) * T.inv_tau * T.inv_tau;
    bb = axpy(jb, r[i], bb);
    t1b = axpy(jb * A1[i], r[i], t1b);
    t2b = axpy(-jb * A2[i], r[i], t2b);
    if (i < 2) xb[i] += jb * (-dot(r[i], t2) + lam * (A2[i] - 0.5));
    else xb[i] += jb * (dot(r[i], t1) + lam * (A1[i] - 0.5));
  }
  double Q11b = 0.0, Q22b = 0.0, Q12b = 0.0, c1b = 0.0, c2b = 0.0;
  for (int i = 0; i < 4; ++i) {
    const double a = xi[i], s0 = sig64(a, T), s1 = sig64(a - 1.0, T);
    const double xib = xb[i] * (s0 - s1);
    taub += xb[i] * ((softplus_t(a, T) - a * s0) - (softplus_t(a - 1.0, T) - (a - 1.0) * s1)) * T.inv_tau;
    if (i == 0) { Q12b -= xib * i22; c2b -= xib * i22; Q22b -= xib * xi[0] * i22; }
    else if (i == 1) { c2b -= xib * i22; Q22b -= xib * xi[1] * i22; }
    else if (i == 2) { Q12b -= xib * i11; c1b -= xib * i11; Q11b -= xib * xi[2] * i11; }
    else { c1b -= xib * i11; Q11b -= xib * xi[3] * i11; }
  }
  const double N1b = au1b * idet, N2b = au2b * idet;
  const double detb = -(au1b * au1 + au2b * au2) * idet;
  Q12b += N1b * c2 + N2b * c1;
  c2b += N1b * Q12 - N2b * Q11;
  c1b += -N1b * Q22 + N2b * Q12;
  Q22b -= N1b * c1;
  Q11b -= N2b * c2;
  Q11b += detb * Q22;
  Q22b += detb * Q11;
  Q12b -= 2.0 * detb * Q12;
  t1b = axpy(2.0 * Q11b, t1, t1b);
  t2b = axpy(2.0 * Q22b, t2, t2b);
  t1b = axpy(-Q12b, t2, t1b);
  t2b = axpy(-Q12b, t1, t2b);
  bb = axpy(c1b, t1, bb);
  t1b = axpy(c1b, b, t1b);
  bb = axpy(-c2b, t2, bb);
  t2b = axpy(-c2b, b, t2b);
  a0b = add(a0b, bb);
  b0b = sub(b0b, bb);
}

}  // namespace cm
