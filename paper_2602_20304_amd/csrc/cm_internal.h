// Internal structures shared by the host runtime and the gfx950 kernels.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/cm.h"

namespace cm {

// One geometry record in device memory (64 bytes).  Offsets index the
// context's vertex / edge / face pools; all coordinates are in the body frame.
struct GeomRec {
  int32_t type, nv, ne, nf;
  int32_t v_off, e_off, f_off, pad0;
  float p[4];        // sphere (r) | capsule (r, h) | box (hx, hy, hz, rounding)
  float bound_r;     // float32 bounding radius about the body origin
  float pad1[3];
};

// Device pointers of the geometry tables (structure-of-arrays pools).
struct Tables {
  const GeomRec* geoms;
  int32_t n_geoms;
  const double* vx; const double* vy; const double* vz;    // vertex pool (float64)
  const int32_t* e0; const int32_t* e1;                    // edge pool (local vertex ids)
  const double* fnx; const double* fny; const double* fnz; const double* fo;   // plane pool (float64)
  const int32_t* f0; const int32_t* f1; const int32_t* f2; // face vertex ids (local)
};

struct BatchDev {
  int32_t n_scenes, n_bodies, n_cand;
  const int32_t* body_offsets;
  const int32_t* body_geom;
  const float* pose;
  const int32_t* cand_offsets;
  const int32_t* cand_pairs;
};

constexpr double kLog2e = 1.4426950408889634;
constexpr double kLn2 = 0.6931471805599453;

struct ParamsDev {
  double tau, lam, eps_n;   // tau is the float32 input widened; defaults resolved in float64
  double inv_tau;           // 1 / tau
  double c_log2;            // log2(e) / tau
  double tl;                // tau ln 2
  float margin;             // broadphase margin (float32 predicate)
  int32_t K;
  int32_t eps_tied;         // eps_n = tau^2 (its tau dependence enters the adjoint)
  uint32_t flags;           // CM_FLAG_*
  int32_t presel_v, presel_e;   // soft top-K pre-selection sizes (0: off)
  int32_t sq;                   // the context holds superquadric unions (selects the kernels built for them)
  int32_t refine;               // sphere-tracing steps of the E-E witnesses (0: off)
};

struct OutDev {
  int32_t capacity;
  int32_t* n_pairs;
  int32_t* pair_offsets;
  int32_t* pairs;
  float* point; float* normal; float* dist; float* weight;
  char* tape;                   // the adjoint's tape (caller-owned), or null
  long long tape_bytes;
};

// Device error bits (sticky until cm_check_errors).
enum : uint32_t { ERR_BAD_GEOM = 1u, ERR_CAPACITY = 2u, ERR_K = 4u, ERR_NO_ADJOINT = 8u };

// Host-side mesh of one geometry, built by geometry.cpp.
struct HostMesh {
  int32_t type = 0;
  float p[4] = {0, 0, 0, 0};
  std::vector<float> v;       // 3 * nv (float32 copy for the mesh query API)
  std::vector<double> vd;     // 3 * nv vertices in float64 (what the kernels use)
  std::vector<int32_t> e;     // 2 * ne
  std::vector<int32_t> f;     // 3 * nf (polytopes)
  std::vector<float> planes;  // 4 * nf (n, o), float32 copy
  std::vector<double> pd;     // 4 * nf (n, o) in float64 (what the kernels use)
  float bound_r = 0.f;
};

// Build the mesh of one descriptor; returns false (with a message) for
// degenerate input.
bool build_mesh(int32_t type, const float* params, const float* pts, int64_t n_pts, HostMesh* out,
                std::string* err);

// Convex hull of points (double precision incremental construction).
// Returns hull vertex ids (ascending input order), outward triangles
// (indices into that vertex list) and unique edges (i < j).
bool convex_hull(const float* pts, int64_t n, std::vector<int32_t>* vid, std::vector<int32_t>* tris,
                 std::vector<int32_t>* edges, std::string* err);

}  // namespace cm
