// Test-only shim: exposes the library's host geometry builder through a C
// function so the CPU test suite can check it without a GPU.
#include <cstring>
#include <string>

#include "cm_internal.h"

extern "C" int shim_build_mesh(int type, const float* params, const float* pts, long n_pts, float* v, int* nv,
                               int* e, int* ne, int* f, int* nf, float* planes, float* bound, char* err) {
  cm::HostMesh m;
  std::string msg;
  if (!cm::build_mesh(type, params, pts, n_pts, &m, &msg)) {
    std::strncpy(err, msg.c_str(), 255);
    return 0;
  }
  *nv = int(m.v.size() / 3); *ne = int(m.e.size() / 2); *nf = int(m.f.size() / 3);
  std::memcpy(v, m.v.data(), m.v.size() * sizeof(float));
  std::memcpy(e, m.e.data(), m.e.size() * sizeof(int));
  if (!m.f.empty()) std::memcpy(f, m.f.data(), m.f.size() * sizeof(int));
  if (!m.planes.empty()) std::memcpy(planes, m.planes.data(), m.planes.size() * sizeof(float));
  *bound = m.bound_r;
  return 1;
}
