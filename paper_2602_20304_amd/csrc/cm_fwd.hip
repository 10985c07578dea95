// gfx950 kernels of the forward path: broadphase + per-scene compaction, and
// the per-pair contact manifold (vertex-SDF, all-pairs edge-edge, SoftSort
// K-manifold).
#include <hip/hip_runtime.h>

#include "cm_device.cuh"
#include "cm_kernels.h"

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
  if (g < 0 || g >= tb.n_geoms) { atomicOr(err, ERR_BAD_GEOM); return false; }
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

struct PairShared {
  BodyView A, B;
  double RA[9], tA[3];   // pair frame -> world
  int ga, gb, valid;
  int nvs, nee, ncand;
  int next;              // dynamic work-queue item
};

template <int KM>
__device__ __forceinline__ void tk_insert(double (&tk)[KM], double x) {
  if (x > tk[KM - 1]) {
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      const double hi = fmax(tk[i], x);
      x = fmin(tk[i], x);
      tk[i] = hi;
    }
  }
}

// Pass-3 record of a candidate near the top-K scores.
struct Rec {
  double s, d;
  float px, py, pz, nx, ny, nz, w, pad;
};

// LDS carve-out for one pair (byte offsets).
struct LdsLayout {
  int eA, eB, pA, pB, row, col, red, top, rec, cnt, bytes;
};

__host__ __device__ inline LdsLayout lds_layout(int maxV, int maxE, int maxF, int block, int kmax) {
  (void)maxV; (void)kmax;
  LdsLayout L;
  int o = 0;
  L.eA = o; o += 6 * 8 * maxE;
  L.eB = o; o += 6 * 8 * maxE;
  L.row = o; o += 8 * maxE;
  L.col = o; o += 8 * maxE;
  L.red = o; o += 2 * 8 * block;       // LSE partials / reductions
  L.top = o; o += 8 * (32 + 16);       // top-K values + scratch
  L.rec = o; o += int(sizeof(Rec)) * block;
  L.pA = o; o += 16 * maxF;
  L.pB = o; o += 16 * maxF;
  L.cnt = o; o += 64;
  L.bytes = (o + 15) & ~15;
  return L;
}

__device__ __forceinline__ EdgeSoA edge_soa(char* base, int maxE) {
  double* d = reinterpret_cast<double*>(base);
  return EdgeSoA{d, d + maxE, d + 2 * maxE, d + 3 * maxE, d + 4 * maxE, d + 5 * maxE};
}

// vertex v of a geometry (body frame, float) -> pair frame (double)
__device__ __forceinline__ D3 load_vertex(const Tables& tb, const GeomRec& G, int v, const BodyView& B) {
  const int i = G.v_off + v;
  const D3 l = d3(tb.vx[i], tb.vy[i], tb.vz[i]);
  if (B.ident) return l;
  return d3(B.R[0] * l.x + B.R[1] * l.y + B.R[2] * l.z + B.t[0], B.R[3] * l.x + B.R[4] * l.y + B.R[5] * l.z + B.t[1],
            B.R[6] * l.x + B.R[7] * l.y + B.R[8] * l.z + B.t[2]);
}

template <int BLOCK, int KMAX, bool DYN>
__global__ __launch_bounds__(BLOCK) void collide_fwd(Tables tb, BatchDev bt, ParamsDev prm, OutDev out,
                                                     float* __restrict__ scratch, long long scratch_stride, int maxV,
                                                     int maxE, int maxF, const int* __restrict__ order,
                                                     int* __restrict__ queue, unsigned* err) {
  extern __shared__ float4 smem4[];
  char* smem = reinterpret_cast<char*>(smem4);
  __shared__ PairShared ps;
  const LdsLayout L = lds_layout(maxV, maxE, maxF, BLOCK, KMAX);
  const EdgeSoA EA = edge_soa(smem + L.eA, maxE);
  const EdgeSoA EB = edge_soa(smem + L.eB, maxE);
  float4* sPA = reinterpret_cast<float4*>(smem + L.pA);
  float4* sPB = reinterpret_cast<float4*>(smem + L.pB);
  double* sRow = reinterpret_cast<double*>(smem + L.row);
  double* sCol = reinterpret_cast<double*>(smem + L.col);
  double* sRed = reinterpret_cast<double*>(smem + L.red);
  double* sTop = reinterpret_cast<double*>(smem + L.top);
  Rec* sRec = reinterpret_cast<Rec*>(smem + L.rec);
  int* sCnt = reinterpret_cast<int*>(smem + L.cnt);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = BLOCK / 64;
  const Temp T = make_temp(prm.tau);
  const double lam = prm.lam, eps_n = prm.eps_n;
  const int K = prm.K;
  const int n_pairs = min(*out.n_pairs, out.capacity);
  double* Dbuf = reinterpret_cast<double*>(scratch + (long long)blockIdx.x * scratch_stride);
  float* Sbuf = reinterpret_cast<float*>(Dbuf + (long long)maxE * maxE);

  int item = DYN ? 0 : blockIdx.x;
  while (true) {
    if (DYN) {
      if (tid == 0) ps.next = atomicAdd(queue, 1);
      __syncthreads();
      item = ps.next;
    }
    if (item >= n_pairs) break;
    const int pi = order ? order[item] : item;

    // ---------------------------------------------------- setup (pose ingest)
    if (tid == 0) {
      const int a = out.pairs[pi], b = out.pairs[out.capacity + pi];
      const int ga = bt.body_geom[a], gb = bt.body_geom[b];
      ps.valid = (ga >= 0 && ga < tb.n_geoms && gb >= 0 && gb < tb.n_geoms);
      if (!ps.valid) {
        atomicOr(err, ERR_BAD_GEOM);
      } else {
        const GeomRec GA = tb.geoms[ga], GB = tb.geoms[gb];
        ps.ga = ga; ps.gb = gb;
        const int nb = bt.n_bodies;
        double RA[9], RB[9];
        quat_to_R(bt.pose[a], bt.pose[nb + a], bt.pose[2 * nb + a], bt.pose[3 * nb + a], RA);
        quat_to_R(bt.pose[b], bt.pose[nb + b], bt.pose[2 * nb + b], bt.pose[3 * nb + b], RB);
        const double tA[3] = {bt.pose[4 * nb + a], bt.pose[5 * nb + a], bt.pose[6 * nb + a]};
        const double dt[3] = {double(bt.pose[4 * nb + b]) - tA[0], double(bt.pose[5 * nb + b]) - tA[1],
                              double(bt.pose[6 * nb + b]) - tA[2]};
        for (int i = 0; i < 9; ++i) ps.RA[i] = RA[i];
        for (int i = 0; i < 3; ++i) ps.tA[i] = tA[i];
        // B in the pair frame: Rr = RA^T RB, tr = RA^T (tB - tA)
        for (int i = 0; i < 3; ++i) {
          for (int j = 0; j < 3; ++j)
            ps.B.R[3 * i + j] = RA[i] * RB[j] + RA[3 + i] * RB[3 + j] + RA[6 + i] * RB[6 + j];
          ps.B.t[i] = RA[i] * dt[0] + RA[3 + i] * dt[1] + RA[6 + i] * dt[2];
        }
        for (int i = 0; i < 9; ++i) ps.A.R[i] = (i % 4 == 0) ? 1.0 : 0.0;
        for (int i = 0; i < 3; ++i) ps.A.t[i] = 0.0;
        ps.A.ident = true; ps.B.ident = false;
        ps.A.type = GA.type; ps.A.nv = GA.nv; ps.A.ne = GA.ne; ps.A.nf = GA.nf;
        ps.B.type = GB.type; ps.B.nv = GB.nv; ps.B.ne = GB.ne; ps.B.nf = GB.nf;
        for (int i = 0; i < 4; ++i) { ps.A.p[i] = GA.p[i]; ps.B.p[i] = GB.p[i]; }
        ps.nvs = GA.nv + GB.nv;
        ps.nee = GA.ne * GB.ne;
        ps.ncand = ps.nvs + 2 * ps.nee;
        if (GA.nv > maxV || GB.nv > maxV || GA.ne > maxE || GB.ne > maxE || GA.nf > maxF || GB.nf > maxF) {
          ps.valid = 0;
          atomicOr(err, ERR_BAD_GEOM);
        }
      }
    }
    __syncthreads();
    if (!ps.valid) {
      if (!DYN) item += gridDim.x;
      __syncthreads();
      continue;
    }
    BodyView A = ps.A, B = ps.B;
    A.planes = sPA; B.planes = sPB;
    const GeomRec& GA = tb.geoms[ps.ga];
    const GeomRec& GB = tb.geoms[ps.gb];
    const int nvA = A.nv, neA = A.ne, neB = B.ne, nfA = A.nf, nfB = B.nf;

    // ---------------------------------------------------- stage edges (pair frame, f64) and planes (body frames)
    for (int i = tid; i < neA + neB; i += BLOCK) {
      const bool isA = i < neA;
      const int e = isA ? i : i - neA;
      const GeomRec& G = isA ? GA : GB;
      const BodyView& V = isA ? A : B;
      const D3 p0 = load_vertex(tb, G, tb.e0[G.e_off + e], V);
      const D3 p1 = load_vertex(tb, G, tb.e1[G.e_off + e], V);
      const EdgeSoA& E = isA ? EA : EB;
      E.x0[e] = p0.x; E.y0[e] = p0.y; E.z0[e] = p0.z;
      E.tx[e] = p1.x - p0.x; E.ty[e] = p1.y - p0.y; E.tz[e] = p1.z - p0.z;
    }
    for (int i = tid; i < nfA + nfB; i += BLOCK) {
      const bool isA = i < nfA;
      const int f = isA ? GA.f_off + i : GB.f_off + (i - nfA);
      (isA ? sPA : sPB)[isA ? i : i - nfA] = make_float4(tb.fnx[f], tb.fny[f], tb.fnz[f], tb.fo[f]);
    }
    __syncthreads();

    double tk[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) tk[i] = -INFINITY;

    // ---------------------------------------------------- V-S candidates (Sec. IV-C), both ways
    for (int i = tid; i < ps.nvs; i += BLOCK) {
      Cand c;
      if (i < nvA) vs_candidate(load_vertex(tb, GA, i, A), B, -1.0, T, c);
      else vs_candidate(load_vertex(tb, GB, i - nvA, B), A, 1.0, T, c);
      Sbuf[i] = float(c.s);
      tk_insert<KMAX>(tk, c.s);
    }

    // ---------------------------------------------------- E-E pass 1: unsigned distances D
    {
      const int nee = ps.nee;
      int k = tid / neB, l = tid - (tid / neB) * neB;
      const int sk = BLOCK / neB, sl = BLOCK - sk * neB;
      for (int idx = tid; idx < nee; idx += BLOCK) {
        D3 a0, t1, b0, t2;
        EA.get(k, a0, t1);
        EB.get(l, b0, t2);
        Dbuf[idx] = ee_dist(a0, t1, b0, t2, lam, T);
        k += sk; l += sl;
        if (l >= neB) { l -= neB; ++k; }
      }
    }
    __syncthreads();
    // row LSE over l (one wave per row, coalesced)
    for (int k = wave; k < neA; k += NW) {
      double m = INFINITY;
      float s = 0.f;
      for (int l = lane; l < neB; l += 64) lse_push(m, s, Dbuf[k * neB + l], T);
      wave_lse_merge(m, s, T);
      if (lane == 0) sRow[k] = m - T.tl * double(lg2f(s));
    }
    // column LSE over k (threads over columns, k split in chunks, coalesced)
    {
      const int nch = neB >= BLOCK ? 1 : BLOCK / neB;
      for (int lb = 0; lb < neB; lb += BLOCK) {
        const int l = lb + (tid % (neB >= BLOCK ? BLOCK : neB));
        const int ch = neB >= BLOCK ? 0 : tid / neB;
        double m = INFINITY;
        float s = 0.f;
        if (ch < nch && l < neB) {
          const int k0 = (ch * neA) / nch, k1 = ((ch + 1) * neA) / nch;
          for (int k = k0; k < k1; ++k) lse_push(m, s, Dbuf[k * neB + l], T);
        }
        sRed[tid] = m;
        sRed[BLOCK + tid] = double(s);
        __syncthreads();
        if (ch == 0 && l < neB) {
          double M = sRed[tid];
          float S = float(sRed[BLOCK + tid]);
          for (int c = 1; c < nch; ++c) {
            const double m2 = sRed[c * neB + tid];
            const float s2 = float(sRed[BLOCK + c * neB + tid]);
            const double Mn = fmin(M, m2);
            const float a = (M == Mn) ? S : S * expn(M - Mn, T);
            const float b = (m2 == Mn) ? s2 : s2 * expn(m2 - Mn, T);
            M = Mn; S = a + b;
          }
          sCol[l] = M - T.tl * double(lg2f(S));
        }
        __syncthreads();
      }
    }
    __syncthreads();

    // ---------------------------------------------------- E-E pass 2: candidates, scores, top-K
    {
      const int nee = ps.nee, nvs = ps.nvs;
      int k = tid / neB, l = tid - (tid / neB) * neB;
      const int sk = BLOCK / neB, sl = BLOCK - sk * neB;
      for (int idx = tid; idx < nee; idx += BLOCK) {
        D3 a0, t1, b0, t2;
        EA.get(k, a0, t1);
        EB.get(l, b0, t2);
        Cand c1, c2;
        ee_candidates(a0, t1, b0, t2, sRow[k], sCol[l], A, B, lam, eps_n, T, c1, c2);
        Sbuf[nvs + 2 * idx] = float(c1.s);
        Sbuf[nvs + 2 * idx + 1] = float(c2.s);
        tk_insert<KMAX>(tk, c1.s);
        tk_insert<KMAX>(tk, c2.s);
        k += sk; l += sl;
        if (l >= neB) { l -= neB; ++k; }
      }
    }

    // ---------------------------------------------------- block top-K merge (values, with multiplicity)
    for (int r = 0; r < K; ++r) {
      const double h = tk[0];
      const double wm = wave_max(h);
      const unsigned long long ball = __ballot(h == wm);
      if (lane == 0) {
        sRed[wave] = wm;
        sRed[NW + wave] = double(wave * 64 + (int)__ffsll((long long)ball) - 1);
      }
      __syncthreads();
      double bm = sRed[0];
      int win = int(sRed[NW]);
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        const double v = sRed[w];
        if (v > bm) { bm = v; win = int(sRed[NW + w]); }
      }
      if (tid == win) {
#pragma unroll
        for (int i = 0; i < KMAX - 1; ++i) tk[i] = tk[i + 1];
        tk[KMAX - 1] = -INFINITY;
      }
      if (tid == 0) sTop[r] = bm;
      __syncthreads();
    }

    // ---------------------------------------------------- pass 3: SoftSort accumulation
    // Rows: Gamma_ki = exp(-|s_[k] - s_i| / tau) / sum_j (...); only candidates
    // within 40 tau of s_[K] can contribute at float32 resolution.
    const float thr = float(sTop[K - 1] - kFilterTaus * T.tau) - 1e-6f * fabsf(float(sTop[K - 1]));
    const int nacc = 9 * K;
    constexpr int NSLOT = (9 * CM_MAX_K + BLOCK - 1) / BLOCK;
    double acc[NSLOT];   // thread owns (k, field) slots tid, tid + BLOCK, ...
#pragma unroll
    for (int i = 0; i < NSLOT; ++i) acc[i] = 0.0;
    const int ncand = ps.ncand, nvs = ps.nvs;
    for (int base = 0; base < ncand; base += BLOCK) {
      const int idx = base + tid;
      const bool pass = idx < ncand && Sbuf[idx] >= thr;
      const unsigned long long ball = __ballot(pass);
      const int below = __popcll(ball & ((1ull << lane) - 1ull));
      if (lane == 0) sCnt[wave] = __popcll(ball);
      __syncthreads();
      int off = 0, tot = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int c = sCnt[w];
        off += (w < wave) ? c : 0;
        tot += c;
      }
      if (tot == 0) {
        __syncthreads();
        continue;
      }
      if (pass) {
        Cand c;
        if (idx < nvs) {
          if (idx < nvA) vs_candidate(load_vertex(tb, GA, idx, A), B, -1.0, T, c);
          else vs_candidate(load_vertex(tb, GB, idx - nvA, B), A, 1.0, T, c);
        } else {
          const int e = idx - nvs;
          const int ee = e >> 1;
          const int k = ee / neB, l = ee - k * neB;
          D3 a0, t1, b0, t2;
          EA.get(k, a0, t1);
          EB.get(l, b0, t2);
          Cand c1, c2;
          ee_candidates(a0, t1, b0, t2, sRow[k], sCol[l], A, B, lam, eps_n, T, c1, c2);
          c = (e & 1) ? c2 : c1;
        }
        Rec& rr = sRec[off + below];
        rr.s = c.s; rr.d = c.d;
        rr.px = float(c.p.x); rr.py = float(c.p.y); rr.pz = float(c.p.z);
        rr.nx = float(c.n.x); rr.ny = float(c.n.y); rr.nz = float(c.n.z);
        rr.w = ex2f(float(c.lw * kLog2e));
      }
      __syncthreads();
#pragma unroll
      for (int slot = 0; slot < NSLOT; ++slot) {
        const int j = tid + slot * BLOCK;
        if (j < nacc) {
          const int kk = j / 9, f = j - kk * 9;
          const double sk = sTop[kk];
          double a = 0.0;
          for (int r = 0; r < tot; ++r) {
            const Rec& rr = sRec[r];
            const double e = double(expn(fabs(sk - rr.s), T));
            double v;
            switch (f) {
              case 0: v = 1.0; break;
              case 1: v = rr.px; break;
              case 2: v = rr.py; break;
              case 3: v = rr.pz; break;
              case 4: v = rr.nx; break;
              case 5: v = rr.ny; break;
              case 6: v = rr.nz; break;
              case 7: v = rr.d; break;
              default: v = rr.w; break;
            }
            a = fma(e, v, a);
          }
          acc[slot] += a;
        }
      }
      __syncthreads();
    }
    // outputs: divide by row sums, rotate to world
    {
      double* sAcc = reinterpret_cast<double*>(sRec);   // reuse: [9K]
#pragma unroll
      for (int slot = 0; slot < NSLOT; ++slot) {
        const int j = tid + slot * BLOCK;
        if (j < nacc) sAcc[j] = acc[slot];
      }
      __syncthreads();
      for (int kk = tid; kk < K; kk += BLOCK) {
        const double* a = sAcc + 9 * kk;
        const double inv = 1.0 / a[0];
        const double px = a[1] * inv, py = a[2] * inv, pz = a[3] * inv;
        const double nx = a[4] * inv, ny = a[5] * inv, nz = a[6] * inv;
        const double* R = ps.RA;
        const long long o = (long long)pi * K + kk;
        const long long CK = (long long)out.capacity * K;
        out.point[o] = float(R[0] * px + R[1] * py + R[2] * pz + ps.tA[0]);
        out.point[CK + o] = float(R[3] * px + R[4] * py + R[5] * pz + ps.tA[1]);
        out.point[2 * CK + o] = float(R[6] * px + R[7] * py + R[8] * pz + ps.tA[2]);
        out.normal[o] = float(R[0] * nx + R[1] * ny + R[2] * nz);
        out.normal[CK + o] = float(R[3] * nx + R[4] * ny + R[5] * nz);
        out.normal[2 * CK + o] = float(R[6] * nx + R[7] * ny + R[8] * nz);
        out.dist[o] = float(a[7] * inv);
        out.weight[o] = float(a[8] * inv);
      }
      __syncthreads();
    }
    if (!DYN) item += gridDim.x;
  }
}

// ============================================================ launchers

int fwd_lds_bytes(int maxV, int maxE, int maxF, int block, int kmax) {
  return lds_layout(maxV, maxE, maxF, block, kmax).bytes;
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

template <int BLOCK, int KMAX, bool DYN>
static hipError_t launch_fwd_t(const FwdLaunch& f, hipStream_t st) {
  auto kern = collide_fwd<BLOCK, KMAX, DYN>;
  const int lds = fwd_lds_bytes(f.maxV, f.maxE, f.maxF, BLOCK, KMAX);
  hipLaunchKernelGGL(kern, dim3(f.grid), dim3(BLOCK), lds, st, f.tb, f.bt, f.prm, f.out, f.scratch,
                     f.scratch_stride, f.maxV, f.maxE, f.maxF, f.order, f.queue, f.err);
  return hipGetLastError();
}

template <int BLOCK, int KMAX, bool DYN>
static int occ_t(int maxV, int maxE, int maxF) {
  int nb = 0;
  const int lds = fwd_lds_bytes(maxV, maxE, maxF, BLOCK, KMAX);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, collide_fwd<BLOCK, KMAX, DYN>, BLOCK, lds) != hipSuccess)
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

hipError_t launch_collide_fwd(const FwdLaunch& f, hipStream_t st) {
  if (f.queue) {
    constexpr bool DYNV = true;
    CM_FWD_DISPATCH(launch_fwd_t, f, st)
  } else {
    constexpr bool DYNV = false;
    CM_FWD_DISPATCH(launch_fwd_t, f, st)
  }
}

int fwd_occupancy(const FwdLaunch& f) {
  if (f.queue) {
    constexpr bool DYNV = true;
    CM_FWD_DISPATCH(occ_t, f.maxV, f.maxE, f.maxF)
  } else {
    constexpr bool DYNV = false;
    CM_FWD_DISPATCH(occ_t, f.maxV, f.maxE, f.maxF)
  }
}

}  // namespace cm
