// Host-side geometry construction: analytic-body meshes, convex hulls of
// polytope point sets, face planes and bounding radii (Sec. IV-A: every
// surface carries a mesh (V, E) and an SDF; Sec. IV-B: a convex polyhedron
// is the set of its face planes (n_f, p_f)).
//
// Compiled with -ffp-contract=off so the float32 bounding radius follows the
// documented operation order exactly.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_set>
#include <utility>

#include "cm_internal.h"

namespace cm {
namespace {

struct Face {
  int a, b, c;
  double n[3];
  double d;
  bool alive;
};

inline void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
inline void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

Face make_face(const std::vector<double>& P, int a, int b, int c) {
  Face f;
  f.a = a; f.b = b; f.c = c; f.alive = true;
  double u[3], v[3];
  sub3(&P[3 * b], &P[3 * a], u);
  sub3(&P[3 * c], &P[3 * a], v);
  cross3(u, v, f.n);
  double l = std::sqrt(dot3(f.n, f.n));
  if (l > 0) { f.n[0] /= l; f.n[1] /= l; f.n[2] /= l; }
  f.d = dot3(f.n, &P[3 * a]);
  return f;
}

inline uint64_t ekey(int a, int b) { return (uint64_t(uint32_t(a)) << 32) | uint32_t(b); }

void ring(double lat_deg, double out[8][3]) {
  const double la = lat_deg * M_PI / 180.0;
  for (int j = 0; j < 8; ++j) {
    const double th = 2.0 * M_PI * j / 8.0;
    out[j][0] = std::cos(la) * std::cos(th);
    out[j][1] = std::cos(la) * std::sin(th);
    out[j][2] = std::sin(la);
  }
}

// ---- superquadric unions (Sec. IV-B, SQ primitives and smooth union)
// Record of one primitive: a, b, c, eps1, eps2, tx, ty, tz, qw, qx, qy, qz.
struct SqPrim {
  double ax[3], e1, e2, t[3], R[9];   // R: primitive frame -> body frame (row-major)
};

inline double spow(double v, double e) { return std::copysign(std::pow(std::fabs(v), e), v); }

// inside-outside function of primitive P at body-frame point x
double sq_f(const SqPrim& P, const double* x) {
  const double d[3] = {x[0] - P.t[0], x[1] - P.t[1], x[2] - P.t[2]};
  double y[3];
  for (int k = 0; k < 3; ++k) y[k] = P.R[k] * d[0] + P.R[3 + k] * d[1] + P.R[6 + k] * d[2];   // R^T d
  const double sx = y[0] / P.ax[0], sy = y[1] / P.ax[1], sz = y[2] / P.ax[2];
  const double u = std::pow(sx * sx, 1.0 / P.e2) + std::pow(sy * sy, 1.0 / P.e2);
  return std::pow(u, P.e2 / P.e1) + std::pow(sz * sz, 1.0 / P.e1);
}

// Per-primitive parametric grid: south pole, rings at -60 / -30 / 0 / 30 /
// 60 degrees of 6 longitudes, north pole (32 vertices); edges: pole spokes,
// ring edges, meridians and one diagonal per quad between rings (90 edges).
constexpr int kSqLon = 6, kSqRings = 5, kSqLocalV = 2 + kSqLon * kSqRings;
const double kSqRingDeg[kSqRings] = {-60.0, -30.0, 0.0, 30.0, 60.0};

void sq_local_edges(std::vector<int>* E) {
  auto ring = [](int r, int j) { return 1 + r * kSqLon + (j % kSqLon); };
  const int north = 1 + kSqRings * kSqLon;
  for (int j = 0; j < kSqLon; ++j) { E->push_back(0); E->push_back(ring(0, j)); }
  for (int r = 0; r < kSqRings; ++r)
    for (int j = 0; j < kSqLon; ++j) { E->push_back(ring(r, j)); E->push_back(ring(r, j + 1)); }
  for (int r = 0; r + 1 < kSqRings; ++r) {
    for (int j = 0; j < kSqLon; ++j) { E->push_back(ring(r, j)); E->push_back(ring(r + 1, j)); }
    for (int j = 0; j < kSqLon; ++j) { E->push_back(ring(r, j)); E->push_back(ring(r + 1, j + 1)); }
  }
  for (int j = 0; j < kSqLon; ++j) { E->push_back(ring(kSqRings - 1, j)); E->push_back(north); }
}

// body-frame position of local sample k of primitive P
void sq_sample(const SqPrim& P, int k, double* out) {
  double c[3];
  if (k == 0 || k == kSqLocalV - 1) {
    c[0] = 0.0; c[1] = 0.0; c[2] = (k == 0 ? -1.0 : 1.0) * P.ax[2];
  } else {
    const int r = (k - 1) / kSqLon, j = (k - 1) % kSqLon;
    const double eta = kSqRingDeg[r] * (M_PI / 180.0), om = 2.0 * M_PI * j / kSqLon;
    const double ce = spow(std::cos(eta), P.e1), se = spow(std::sin(eta), P.e1);
    c[0] = P.ax[0] * ce * spow(std::cos(om), P.e2);
    c[1] = P.ax[1] * ce * spow(std::sin(om), P.e2);
    c[2] = P.ax[2] * se;
  }
  for (int i = 0; i < 3; ++i) out[i] = P.R[3 * i] * c[0] + P.R[3 * i + 1] * c[1] + P.R[3 * i + 2] * c[2] + P.t[i];
}

constexpr int kOpcKnn = 4;   // mesh edges of an oriented point cloud: k-nearest-neighbour graph

}  // namespace

bool convex_hull(const float* pts, int64_t n, std::vector<int32_t>* vid, std::vector<int32_t>* tris,
                 std::vector<int32_t>* edges, std::string* err) {
  if (n < 4) { *err = "polytope needs at least 4 points"; return false; }
  std::vector<double> P(3 * n);
  double scale = 0;
  for (int64_t i = 0; i < 3 * n; ++i) {
    P[i] = double(pts[i]);
    if (!std::isfinite(P[i])) { *err = "non-finite polytope point"; return false; }
    scale = std::max(scale, std::fabs(P[i]));
  }
  if (scale == 0) { *err = "degenerate polytope"; return false; }
  const double eps = 1e-10 * scale;

  // initial tetrahedron from extreme points
  int i0 = 0;
  for (int i = 1; i < n; ++i) if (P[3 * i] < P[3 * i0]) i0 = i;
  int i1 = -1; double best = -1;
  for (int i = 0; i < n; ++i) {
    double d[3]; sub3(&P[3 * i], &P[3 * i0], d);
    double v = dot3(d, d);
    if (v > best) { best = v; i1 = i; }
  }
  if (best <= eps * eps) { *err = "degenerate polytope (coincident points)"; return false; }
  int i2 = -1; best = -1;
  double e01[3]; sub3(&P[3 * i1], &P[3 * i0], e01);
  for (int i = 0; i < n; ++i) {
    double d[3], c[3]; sub3(&P[3 * i], &P[3 * i0], d); cross3(e01, d, c);
    double v = dot3(c, c);
    if (v > best) { best = v; i2 = i; }
  }
  if (best <= eps * eps * dot3(e01, e01)) { *err = "degenerate polytope (collinear points)"; return false; }
  Face base = make_face(P, i0, i1, i2);
  int i3 = -1; best = -1;
  for (int i = 0; i < n; ++i) {
    double v = std::fabs(dot3(base.n, &P[3 * i]) - base.d);
    if (v > best) { best = v; i3 = i; }
  }
  if (best <= eps) { *err = "degenerate polytope (coplanar points)"; return false; }

  std::vector<Face> F;
  const int tet[4][3] = {{i0, i1, i2}, {i0, i1, i3}, {i0, i2, i3}, {i1, i2, i3}};
  double cen[3] = {0, 0, 0};
  for (int q : {i0, i1, i2, i3}) for (int k = 0; k < 3; ++k) cen[k] += 0.25 * P[3 * q + k];
  for (auto& t : tet) {
    Face f = make_face(P, t[0], t[1], t[2]);
    if (dot3(f.n, cen) - f.d > 0) f = make_face(P, t[0], t[2], t[1]);
    F.push_back(f);
  }

  std::vector<int> visible;
  std::unordered_set<uint64_t> vis_edges;
  std::vector<std::pair<int, int>> horizon;
  for (int p = 0; p < n; ++p) {
    if (p == i0 || p == i1 || p == i2 || p == i3) continue;
    const double* x = &P[3 * p];
    visible.clear();
    for (int fi = 0; fi < int(F.size()); ++fi)
      if (F[fi].alive && dot3(F[fi].n, x) - F[fi].d > eps) visible.push_back(fi);
    if (visible.empty()) continue;  // interior point
    vis_edges.clear();
    for (int fi : visible) {
      const Face& f = F[fi];
      vis_edges.insert(ekey(f.a, f.b)); vis_edges.insert(ekey(f.b, f.c)); vis_edges.insert(ekey(f.c, f.a));
    }
    horizon.clear();
    for (int fi : visible) {
      const Face& f = F[fi];
      const int es[3][2] = {{f.a, f.b}, {f.b, f.c}, {f.c, f.a}};
      for (auto& e : es)
        if (!vis_edges.count(ekey(e[1], e[0]))) horizon.push_back({e[0], e[1]});
    }
    for (int fi : visible) F[fi].alive = false;
    for (auto& e : horizon) F.push_back(make_face(P, e.first, e.second, p));
    if (F.size() > 8 * size_t(n) + 64) {  // compact dead faces
      std::vector<Face> G;
      for (auto& f : F) if (f.alive) G.push_back(f);
      F.swap(G);
    }
  }

  std::vector<int32_t> remap(n, -1);
  std::vector<int32_t> used;
  for (auto& f : F) if (f.alive) { remap[f.a] = 1; remap[f.b] = 1; remap[f.c] = 1; }
  vid->clear();
  for (int i = 0; i < n; ++i) if (remap[i] == 1) { remap[i] = int32_t(vid->size()); vid->push_back(i); }
  tris->clear();
  std::vector<std::pair<int, int>> es;
  for (auto& f : F) {
    if (!f.alive) continue;
    int a = remap[f.a], b = remap[f.b], c = remap[f.c];
    tris->push_back(a); tris->push_back(b); tris->push_back(c);
    es.push_back({std::min(a, b), std::max(a, b)});
    es.push_back({std::min(b, c), std::max(b, c)});
    es.push_back({std::min(c, a), std::max(c, a)});
  }
  std::sort(es.begin(), es.end());
  es.erase(std::unique(es.begin(), es.end()), es.end());
  edges->clear();
  for (auto& e : es) { edges->push_back(e.first); edges->push_back(e.second); }
  const int64_t V = vid->size(), E = es.size(), Fn = tris->size() / 3;
  if (V - E + Fn != 2) { *err = "hull construction failed (Euler characteristic)"; return false; }
  return true;
}

// Reorder a polytope's edges so that each run of 8 consecutive edges is
// spatially compact: recursive median splits of the edge midpoints along the
// axis of largest extent, with the first part of every split a multiple of 8.
// The pair kernels give one wave an 8 x 8 tile of (edge of A, edge of B)
// pairs and skip, for the whole wave, the faces that are far from all 8
// edges of each side; compact runs keep those unions small.
static void order_edges_spatially(const std::vector<double>& vd, std::vector<int32_t>* edges) {
  const int ne = int(edges->size() / 2);
  if (ne <= 8) return;
  std::vector<double> mid(3 * size_t(ne));
  for (int e = 0; e < ne; ++e)
    for (int k = 0; k < 3; ++k)
      mid[3 * e + k] = 0.5 * (vd[3 * (*edges)[2 * e] + k] + vd[3 * (*edges)[2 * e + 1] + k]);
  std::vector<int> ids(ne);
  for (int e = 0; e < ne; ++e) ids[e] = e;
  std::vector<int> out;
  out.reserve(ne);
  std::vector<std::pair<int, int>> stack = {{0, ne}};   // [lo, hi) ranges of ids, processed in order
  while (!stack.empty()) {
    const auto [lo, hi] = stack.back();
    stack.pop_back();
    if (hi - lo <= 8) {
      out.insert(out.end(), ids.begin() + lo, ids.begin() + hi);
      continue;
    }
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int i = lo; i < hi; ++i)
      for (int k = 0; k < 3; ++k) {
        mn[k] = std::min(mn[k], mid[3 * ids[i] + k]);
        mx[k] = std::max(mx[k], mid[3 * ids[i] + k]);
      }
    int ax = 0;
    for (int k = 1; k < 3; ++k) if (mx[k] - mn[k] > mx[ax] - mn[ax]) ax = k;
    std::stable_sort(ids.begin() + lo, ids.begin() + hi, [&](int a, int b) {
      return mid[3 * a + ax] < mid[3 * b + ax];
    });
    const int half = std::min(hi - lo, ((hi - lo + 1) / 2 + 7) / 8 * 8);
    stack.push_back({lo + half, hi});   // second part after the first
    stack.push_back({lo, lo + half});
  }
  std::vector<int32_t> re(edges->size());
  for (int i = 0; i < ne; ++i) {
    re[2 * i] = (*edges)[2 * out[i]];
    re[2 * i + 1] = (*edges)[2 * out[i] + 1];
  }
  edges->swap(re);
}

bool build_mesh(int32_t type, const float* params, const float* pts, int64_t n_pts, HostMesh* out,
                std::string* err) {
  HostMesh& m = *out;
  m = HostMesh();
  m.type = type;
  for (int k = 0; k < 4; ++k) m.p[k] = params ? params[k] : 0.f;
  // analytic mesh vertices are functions of the float32 parameters, kept in
  // float64 so that the kernels see the same mesh as the definition
  auto push_v = [&](double x, double y, double z) {
    m.v.push_back(float(x)); m.v.push_back(float(y)); m.v.push_back(float(z));
    m.vd.push_back(x); m.vd.push_back(y); m.vd.push_back(z);
  };
  auto push_e = [&](int a, int b) { m.e.push_back(a); m.e.push_back(b); };
  if (type == CM_SPHERE || type == CM_CAPSULE) {
    const double r = m.p[0], h = (type == CM_CAPSULE) ? double(m.p[1]) : 0.0;
    if (!(r > 0) || !(h >= 0)) { *err = "sphere/capsule needs r > 0, half_len >= 0"; return false; }
    double rl[8][3], r0[8][3], rh[8][3];
    ring(-45, rl); ring(0, r0); ring(45, rh);
    if (type == CM_SPHERE) {
      // south pole, rings at -45 / 0 / +45 degrees, north pole: 26 V, 56 E
      push_v(0, 0, -r);
      for (auto& d : rl) push_v(r * d[0], r * d[1], r * d[2]);
      for (auto& d : r0) push_v(r * d[0], r * d[1], r * d[2]);
      for (auto& d : rh) push_v(r * d[0], r * d[1], r * d[2]);
      push_v(0, 0, r);
      for (int j = 0; j < 8; ++j) push_e(0, 1 + j);
      for (int rr : {1, 9, 17}) for (int j = 0; j < 8; ++j) push_e(rr + j, rr + (j + 1) % 8);
      for (int j = 0; j < 8; ++j) push_e(1 + j, 9 + j);
      for (int j = 0; j < 8; ++j) push_e(9 + j, 17 + j);
      for (int j = 0; j < 8; ++j) push_e(17 + j, 25);
    } else {
      // lower hemisphere (centre -h) and upper hemisphere (centre +h): 34 V, 72 E
      push_v(0, 0, -r - h);
      for (auto& d : rl) push_v(r * d[0], r * d[1], r * d[2] - h);
      for (auto& d : r0) push_v(r * d[0], r * d[1], r * d[2] - h);
      for (auto& d : r0) push_v(r * d[0], r * d[1], r * d[2] + h);
      for (auto& d : rh) push_v(r * d[0], r * d[1], r * d[2] + h);
      push_v(0, 0, r + h);
      for (int j = 0; j < 8; ++j) push_e(0, 1 + j);
      for (int rr : {1, 9, 17, 25}) for (int j = 0; j < 8; ++j) push_e(rr + j, rr + (j + 1) % 8);
      for (int j = 0; j < 8; ++j) push_e(1 + j, 9 + j);
      for (int j = 0; j < 8; ++j) push_e(9 + j, 17 + j);
      for (int j = 0; j < 8; ++j) push_e(17 + j, 25 + j);
      for (int j = 0; j < 8; ++j) push_e(25 + j, 33);
    }
    m.bound_r = (type == CM_SPHERE) ? m.p[0] : (m.p[1] + m.p[0]);
    return true;
  }
  if (type == CM_BOX) {
    if (!(m.p[0] > 0 && m.p[1] > 0 && m.p[2] > 0) || !(m.p[3] >= 0) ||
        m.p[3] > std::min(m.p[0], std::min(m.p[1], m.p[2]))) {
      *err = "box needs half-extents > 0 and 0 <= rounding <= min half-extent";
      return false;
    }
    for (int i = 0; i < 8; ++i)
      push_v((i & 1) ? m.p[0] : -m.p[0], (i & 2) ? m.p[1] : -m.p[1], (i & 4) ? m.p[2] : -m.p[2]);
    for (int bit : {1, 2, 4}) for (int i = 0; i < 8; ++i) if (!(i & bit)) push_e(i, i | bit);
    const float hx = m.p[0], hy = m.p[1], hz = m.p[2];
    m.bound_r = std::sqrt((hx * hx + hy * hy) + hz * hz);
    return true;
  }
  if (type == CM_POLYTOPE) {
    std::vector<int32_t> vid, tris, edges;
    if (!convex_hull(pts, n_pts, &vid, &tris, &edges, err)) return false;
    for (int32_t i : vid)
      for (int k = 0; k < 3; ++k) {
        m.v.push_back(pts[3 * i + k]);
        m.vd.push_back(double(pts[3 * i + k]));
      }
    order_edges_spatially(m.vd, &edges);
    m.e = edges;
    m.f = tris;
    const size_t nf = tris.size() / 3;
    for (size_t t = 0; t < nf; ++t) {
      double a[3], b[3], c[3];
      for (int k = 0; k < 3; ++k) {
        a[k] = m.v[3 * tris[3 * t] + k]; b[k] = m.v[3 * tris[3 * t + 1] + k]; c[k] = m.v[3 * tris[3 * t + 2] + k];
      }
      double u[3], v[3], nn[3];
      sub3(b, a, u); sub3(c, a, v); cross3(u, v, nn);
      double l = std::sqrt(dot3(nn, nn));
      for (int k = 0; k < 3; ++k) nn[k] /= l;
      const double o = dot3(nn, a);
      m.planes.push_back(float(nn[0])); m.planes.push_back(float(nn[1])); m.planes.push_back(float(nn[2]));
      m.planes.push_back(float(o));
      m.pd.push_back(nn[0]); m.pd.push_back(nn[1]); m.pd.push_back(nn[2]); m.pd.push_back(o);
    }
    float mx = 0.f;
    for (int64_t i = 0; i < n_pts; ++i) {
      const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
      const float q = (x * x + y * y) + z * z;
      mx = std::max(mx, q);
    }
    m.bound_r = std::sqrt(mx);
    return true;
  }
  if (type == CM_SQ_UNION) {
    if (n_pts % 4 != 0 || n_pts < 4 || n_pts / 4 > CM_MAX_SQ) {
      *err = "superquadric union needs 1.." + std::to_string(CM_MAX_SQ) + " primitives of 4 xyz rows";
      return false;
    }
    const int M = int(n_pts / 4);
    std::vector<SqPrim> P(M);
    float bound = 0.f;
    for (int i = 0; i < M; ++i) {
      const float* r = pts + 12 * i;
      for (int k = 0; k < 12; ++k)
        if (!std::isfinite(r[k])) { *err = "non-finite superquadric record"; return false; }
      SqPrim& q = P[i];
      for (int k = 0; k < 3; ++k) { q.ax[k] = r[k]; q.t[k] = r[5 + k]; }
      q.e1 = r[3]; q.e2 = r[4];
      if (!(q.ax[0] > 0 && q.ax[1] > 0 && q.ax[2] > 0) || !(q.e1 >= 0.1 && q.e1 <= 1.9) ||
          !(q.e2 >= 0.1 && q.e2 <= 1.9)) {
        *err = "superquadric needs semi-axes > 0 and exponents in [0.1, 1.9]";
        return false;
      }
      double w = r[8], x = r[9], y = r[10], z = r[11];
      const double n = std::sqrt(w * w + x * x + y * y + z * z);
      if (!(n > 0)) { *err = "superquadric quaternion is zero"; return false; }
      w /= n; x /= n; y /= n; z /= n;
      const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                           2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                           2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
      std::memcpy(q.R, R, sizeof(R));
      // float32 bound: |t| + |(a, b, c)| (the primitive lies in its box)
      const float tn = std::sqrt((r[5] * r[5] + r[6] * r[6]) + r[7] * r[7]);
      const float an = std::sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
      bound = std::max(bound, tn + an);
    }
    // mesh: every primitive's grid minus vertices strictly inside another
    // primitive (f_j < 1) and the edges that touch them
    std::vector<int> le;
    sq_local_edges(&le);
    std::vector<int> index(size_t(M) * kSqLocalV, -1);
    for (int i = 0; i < M; ++i)
      for (int k = 0; k < kSqLocalV; ++k) {
        double x[3];
        sq_sample(P[i], k, x);
        bool inside = false;
        for (int j = 0; j < M && !inside; ++j) inside = (j != i) && sq_f(P[j], x) < 1.0;
        if (inside) continue;
        index[size_t(i) * kSqLocalV + k] = int(m.vd.size() / 3);
        push_v(x[0], x[1], x[2]);
      }
    if (m.vd.empty()) { *err = "superquadric union mesh is empty"; return false; }
    for (int i = 0; i < M; ++i)
      for (size_t e = 0; e < le.size(); e += 2) {
        const int a = index[size_t(i) * kSqLocalV + le[e]], b = index[size_t(i) * kSqLocalV + le[e + 1]];
        if (a >= 0 && b >= 0) push_e(a, b);
      }
    // device records: 5 float64 quadruples per primitive in the plane pool:
    // the rows of R^T with t in .w, then (1/a, 1/b, 1/c, eps1) and
    // (1/eps2, eps2/eps1, 1/eps1, eps2); face ids are unused zeros
    for (int i = 0; i < M; ++i) {
      const SqPrim& q = P[i];
      const double slot[20] = {q.R[0], q.R[3], q.R[6], q.t[0], q.R[1], q.R[4], q.R[7], q.t[1],
                               q.R[2], q.R[5], q.R[8], q.t[2], 1.0 / q.ax[0], 1.0 / q.ax[1], 1.0 / q.ax[2], q.e1,
                               1.0 / q.e2, q.e2 / q.e1, 1.0 / q.e1, q.e2};
      for (int k = 0; k < 20; ++k) { m.pd.push_back(slot[k]); m.planes.push_back(float(slot[k])); }
      for (int k = 0; k < 15; ++k) m.f.push_back(0);
    }
    m.bound_r = bound;
    return true;
  }
  if (type == CM_OPC) {
    if (n_pts % 3 != 0 || n_pts < 3 || n_pts / 3 > CM_MAX_OPC) {
      *err = "oriented point cloud needs 1.." + std::to_string(CM_MAX_OPC) + " points of 3 xyz rows";
      return false;
    }
    const int N = int(n_pts / 3);
    float mx = 0.f, smax = 0.f;
    for (int j = 0; j < N; ++j) {
      const float* r = pts + 9 * j;
      for (int k = 0; k < 7; ++k)
        if (!std::isfinite(r[k])) { *err = "non-finite oriented point"; return false; }
      const double nn = std::sqrt(double(r[3]) * r[3] + double(r[4]) * r[4] + double(r[5]) * r[5]);
      if (!(r[6] > 0.f) || !(nn > 0)) { *err = "oriented point needs sigma > 0 and a nonzero normal"; return false; }
      push_v(r[0], r[1], r[2]);
      mx = std::max(mx, (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
      smax = std::max(smax, r[6]);
      const double sg = r[6];
      // device records: (p, 1 / (2 sigma^2)) and (unit n, 1 / sigma^2); face ids unused
      const double slot[8] = {double(r[0]), double(r[1]), double(r[2]), 1.0 / (2.0 * sg * sg),
                              r[3] / nn, r[4] / nn, r[5] / nn, 1.0 / (sg * sg)};
      for (int k = 0; k < 8; ++k) { m.pd.push_back(slot[k]); m.planes.push_back(float(slot[k])); }
      for (int k = 0; k < 6; ++k) m.f.push_back(0);
    }
    // mesh edges: the undirected k-nearest-neighbour graph (ties by index)
    const std::vector<double>& P = m.vd;
    std::vector<std::pair<int, int>> es;
    std::vector<std::pair<double, int>> d2(N);
    const int k = std::min(kOpcKnn, N - 1);
    for (int i = 0; i < N; ++i) {
      for (int j = 0; j < N; ++j) {
        const double dx = P[3 * j] - P[3 * i], dy = P[3 * j + 1] - P[3 * i + 1], dz = P[3 * j + 2] - P[3 * i + 2];
        d2[j] = {j == i ? HUGE_VAL : (dx * dx + dy * dy) + dz * dz, j};
      }
      std::partial_sort(d2.begin(), d2.begin() + k, d2.end());
      for (int q = 0; q < k; ++q) {
        const int j = d2[q].second;
        es.push_back({std::min(i, j), std::max(i, j)});
      }
    }
    std::sort(es.begin(), es.end());
    es.erase(std::unique(es.begin(), es.end()), es.end());
    for (auto& e : es) push_e(e.first, e.second);
    m.bound_r = std::sqrt(mx) + smax;
    return true;
  }
  *err = "unknown geometry type";
  return false;
}

}  // namespace cm
