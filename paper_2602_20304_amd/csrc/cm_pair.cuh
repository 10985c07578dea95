// Per-pair forward engine shared by the forward and adjoint kernels.
//
// One workgroup owns one body pair at a time.  Phases (all in the frame of
// body A):
//   setup    pose ingest: R_A, t_A, and body B's pose relative to A
//   stage    edges of both bodies (FP64 SoA) and face planes (body frames,
//            scaled by log2(e) / tau) in LDS
//   scores   V-S candidates both ways (Sec. IV-C); E-E distance pass with the
//            row / column LSE of the unsigned-distance matrix (nearest-neighbour
//            indicators, Sec. IV-D); E-E candidate pass (witness QP, SDF queries,
//            sign, penetration, clashing, activity, score); per-lane top-K
//   topk     block merge of the per-lane top-K score lists (with multiplicity)
//   softsort SoftSort rows over the candidates within 30 tau of s_[K]
#pragma once
#include "cm_device.cuh"
#include "cm_kernels.h"

namespace cm {

struct PairShared {
  BodyView A, B;
  double RA[9], tA[3];   // pair frame -> world
  int ga, gb, valid, a, b;
  int nvs, nee, ncand;
  int next;              // dynamic work-queue item
  long long tape_off;    // pool offset of this pair's tape window (-1: the pool is full)
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

// Record of a candidate near the top-K scores.
struct Rec {
  double s, d;
  float px, py, pz, nx, ny, nz, w;
  int idx;
};

struct LdsLayout {
  int eA, eB, row, col, red, top, rec, acc, pA, pB, cnt, g1, g2, bytes;
  bool edges_lds;   // false: the edge arrays live in the workgroup's scratch slot
};

// Dynamic LDS a workgroup may use on gfx950 (160 KB per CU), leaving room for
// the kernels' static shared variables.
constexpr int kLdsBudget = 160 * 1024 - 1024;
// Virtual threads of the column LSE's chunking (the same in every block size).
constexpr int kColSlots = 256;
static_assert(sizeof(FaceMask) == kFaceMaskBytes, "the scratch copy of the group masks is sized for this");

// 64-bit words of a face mask (0: culling off): the fewest powers of two
// covering maxF faces, up to kMaxMaskWords (512 faces); larger polytopes
// are not culled.
__host__ __device__ inline int mask_words(int maxF) {
  int w = 1;
  while (64 * w < maxF && w < kMaxMaskWords) w <<= 1;
  return 64 * w >= maxF ? w : 0;
}

// extra: LDS bytes the calling kernel needs beyond the engine.  When the
// whole does not fit kLdsBudget, or when edges_out is set (the launch found
// that it fits more workgroups per CU that way), both bodies' edge arrays
// (96 B per edge) live in the workgroup's scratch slot instead.
__host__ __device__ inline LdsLayout lds_layout(int maxE, int maxF, int block, int extra = 0, bool edges_out = false) {
  LdsLayout L;
  int o = 0;
  const int edge_bytes = 2 * 6 * 8 * maxE;
  // the face masks (cull to pass 2) and the SoftSort records (after pass 2)
  // are never live together: they share one region.  Masks of the groups of
  // 8 consecutive edges: per group of A's and of B's edges, the union over
  // the group's segments (faces of A, faces of B).
  const int group_bytes = mask_words(maxF) > 0 ? 2 * ((maxE + 7) / 8) * 2 * int(sizeof(FaceMask)) : 0;
  const int rec_bytes = int(sizeof(Rec)) * block;
  const int shared_bytes = ((rec_bytes > group_bytes ? rec_bytes : group_bytes) + 7) & ~7;
  const int red_n = block > kColSlots ? block : kColSlots;   // reduction slots: 2 x 8 B each
  L.edges_lds = !edges_out;
  if (L.edges_lds) {
    // size with the edges in LDS (same sequence as below)
    int t = edge_bytes + 16 * maxE + 16 * red_n + 8 * 64 + shared_bytes + 8 * 9 * CM_MAX_K + 64 * maxF + 64;
    if (((t + 15) & ~15) + extra > kLdsBudget) L.edges_lds = false;
  }
  L.eA = L.eB = -1;
  if (L.edges_lds) {
    L.eA = o; o += 6 * 8 * maxE;
    L.eB = o; o += 6 * 8 * maxE;
  }
  L.row = o; o += 8 * maxE;
  L.col = o; o += 8 * maxE;
  L.red = o; o += 2 * 8 * red_n;
  L.top = o; o += 8 * 64;
  L.rec = o;
  L.g1 = o;                      // [group of A's edges][A's faces, B's faces]
  L.g2 = o + group_bytes / 2;    // [group of B's edges][A's faces, B's faces]
  o += shared_bytes;
  L.acc = o; o += 8 * 9 * CM_MAX_K;
  L.pA = o; o += 32 * maxF;    // double4 planes (n.xyz, o)
  L.pB = o; o += 32 * maxF;
  L.cnt = o; o += 64;
  L.bytes = (o + 15) & ~15;
  return L;
}

// LDS bytes of the pre-selection arrays (PRESEL engines): the metrics of
// every vertex and edge of both bodies, the selected values x_[k] of the four
// sets, the soft vertices [2][K][3] and soft edge endpoints [2][K][6].
__host__ __device__ inline int presel_lds_bytes(int maxV, int maxE) {
  return 8 * (2 * maxV + 2 * maxE) + 8 * 4 * CM_MAX_PRESEL + 8 * 2 * CM_MAX_PRESEL * 3 + 8 * 2 * CM_MAX_PRESEL * 6;
}

// CULL: the candidate pass visits edge pairs in 8 x 8 tiles whose witness
// queries use the per-segment face masks (the forward kernel and the
// adjoint's recompute of it, so both take the same path); without it the
// edge pairs go row-major and every face is visited.  PRESEL: soft top-K
// pre-selection (select()) replaces the bodies' vertices and edges by the
// selected soft ones before the candidate passes.
template <int BLOCK, int KMAX, bool CULL, bool PRESEL = false, bool SQ = false, bool REFINE = false>
struct PairEngine {
  static constexpr int NW = BLOCK / 64;

  PairShared& ps;
  const Tables& tb;
  const BatchDev& bt;
  EdgeSoA EA, EB;
  double4* sPA;
  double4* sPB;
  double* sRow;
  double* sCol;
  double* sRed;
  double* sTop;
  Rec* sRec;
  double* sAcc;   // [9K] unnormalised SoftSort sums (1, p, nu, d, w) per row
  int* sCnt;
  FaceMask* sG1;             // [ceil(maxE / 8)][2] face masks of groups of 8 edges of A, see cull()
  FaceMask* sG2;             // [ceil(maxE / 8)][2] the same for B's edges
  double* gShift;            // scratch [2][maxE]: per edge of A the shift of B's value queries on it, then
                             // per edge of B that of A's (kNoShift: none), see cull()
  FaceMask* gMask;           // scratch copy of sG1 ([ceil(maxE / 8)][2]) then sG2, made by cull()
  int MW;
  double* Dbuf;   // [maxE^2] unsigned distance of edge pair (k, l) at k * neB + l
  double* Al1;    // [maxE^2] QP solution al1, al2 and ln con of the same edge pair
  double* Al2;
  double* Lcon;
  float* Sbuf;    // [nvs + 2 nee] candidate scores (float32, filter only)
  int* List;      // [nvs + 2 nee + 64] compacted indices of filtered candidates
  double* sMet;     // PRESEL: metrics [maxV] A's vertices, [maxV] B's, [maxE] A's edges, [maxE] B's
  double* sSel;     // PRESEL: [4][CM_MAX_PRESEL] selected values of the four sets
  double* sSoft;    // PRESEL: soft vertices [2][CM_MAX_PRESEL][3], then soft edges [2][CM_MAX_PRESEL][6]
  int kv, ke;       // PRESEL: requested K_V, K_E
  int refine;       // REFINE: sphere-tracing steps of the E-E witnesses
  Temp T;
  double lam, eps_n;
  unsigned flags;   // CM_FLAG_*
  int K, maxV, maxE, maxF;
  int tid, lane, wave;
  BodyView A, B;
  const GeomRec* GA;
  const GeomRec* GB;

  __device__ __forceinline__ PairEngine(PairShared& ps_, char* smem, const Tables& tb_, const BatchDev& bt_, const ParamsDev& prm,
                        float* slot, int maxV_, int maxE_, int maxF_, int lds_extra = 0, bool edges_out = false)
      : ps(ps_), tb(tb_), bt(bt_) {
    const LdsLayout L = lds_layout(maxE_, maxF_, BLOCK, lds_extra, edges_out);
    double* e = L.edges_lds ? reinterpret_cast<double*>(smem + L.eA)
                            : reinterpret_cast<double*>(slot + scratch_edges_offset(maxV_, maxE_));
    EA = EdgeSoA{e, e + maxE_, e + 2 * maxE_, e + 3 * maxE_, e + 4 * maxE_, e + 5 * maxE_};
    e = L.edges_lds ? reinterpret_cast<double*>(smem + L.eB) : e + 6 * maxE_;
    EB = EdgeSoA{e, e + maxE_, e + 2 * maxE_, e + 3 * maxE_, e + 4 * maxE_, e + 5 * maxE_};
    sPA = reinterpret_cast<double4*>(smem + L.pA);
    sPB = reinterpret_cast<double4*>(smem + L.pB);
    sRow = reinterpret_cast<double*>(smem + L.row);
    sCol = reinterpret_cast<double*>(smem + L.col);
    sRed = reinterpret_cast<double*>(smem + L.red);
    sTop = reinterpret_cast<double*>(smem + L.top);
    sRec = reinterpret_cast<Rec*>(smem + L.rec);
    sAcc = reinterpret_cast<double*>(smem + L.acc);
    sCnt = reinterpret_cast<int*>(smem + L.cnt);
    sG1 = reinterpret_cast<FaceMask*>(smem + L.g1);
    sG2 = reinterpret_cast<FaceMask*>(smem + L.g2);
    sMet = reinterpret_cast<double*>(smem + L.bytes);
    sSel = sMet + 2 * maxV_ + 2 * maxE_;
    sSoft = sSel + 4 * CM_MAX_PRESEL;
    kv = prm.presel_v;
    ke = prm.presel_e;
    refine = prm.refine;
    MW = CULL ? mask_words(maxF_) : 0;
    const long long mm = (long long)maxE_ * maxE_;
    Dbuf = reinterpret_cast<double*>(slot);
    Al1 = Dbuf + mm;
    Al2 = Al1 + mm;
    Lcon = Al2 + mm;
    Sbuf = reinterpret_cast<float*>(Lcon + mm);
    List = reinterpret_cast<int*>(Sbuf + 2 * mm + 2LL * maxV_);
    gShift = reinterpret_cast<double*>(slot + scratch_shift_offset(maxV_, maxE_));
    gMask = reinterpret_cast<FaceMask*>(slot + scratch_mask_offset(maxV_, maxE_));
    T = make_temp(prm);
    lam = prm.lam;
    flags = prm.flags;
    eps_n = prm.eps_n;
    K = prm.K;
    maxV = maxV_; maxE = maxE_; maxF = maxF_;
    tid = threadIdx.x; lane = tid & 63; wave = tid >> 6;
  }

  // ------------------------------------------------------------ setup
  // Thread 0 reads the pair and both poses; returns false (uniformly) for
  // an invalid pair.
  __device__ __forceinline__ bool setup(int a, int b, unsigned* err) {
    if (tid == 0) {
      ps.a = a; ps.b = b;
      const int ga = bt.body_geom[a], gb = bt.body_geom[b];
      ps.valid = (ga >= 0 && ga < tb.n_geoms && gb >= 0 && gb < tb.n_geoms);
      if (!ps.valid) {
        atomicOr(err, ERR_BAD_GEOM);
      } else {
        const GeomRec G1 = tb.geoms[ga], G2 = tb.geoms[gb];
        ps.ga = ga; ps.gb = gb;
        if (G1.type < 0 || G2.type < 0) {   // destroyed geometry
          ps.valid = 0;
          atomicOr(err, ERR_BAD_GEOM);
        }
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
        ps.A.type = G1.type; ps.A.nv = G1.nv; ps.A.ne = G1.ne; ps.A.nf = G1.nf;
        ps.B.type = G2.type; ps.B.nv = G2.nv; ps.B.ne = G2.ne; ps.B.nf = G2.nf;
        for (int i = 0; i < 4; ++i) { ps.A.p[i] = G1.p[i]; ps.B.p[i] = G2.p[i]; }
        ps.nvs = G1.nv + ((flags & CM_FLAG_ONE_SIDED_VS) ? 0 : G2.nv);
        ps.nee = (flags & CM_FLAG_NO_EE) ? 0 : G1.ne * G2.ne;
        ps.ncand = ps.nvs + 2 * ps.nee;
        if (ps.valid && (G1.nv > maxV || G2.nv > maxV || G1.ne > maxE || G2.ne > maxE || G1.nf > maxF || G2.nf > maxF)) {
          ps.valid = 0;
          atomicOr(err, ERR_BAD_GEOM);
        }
      }
    }
    __syncthreads();
    if (!ps.valid) return false;
    A = load_uniform(ps.A, false);
    B = load_uniform(ps.B, true);
    A.planes = sPA; B.planes = sPB;
    GA = &tb.geoms[ps.ga];
    GB = &tb.geoms[ps.gb];
    return true;
  }

  // vertex v of a geometry (body frame, float) -> pair frame (double);
  // IDENT: the body is A (its frame is the pair frame)
  template <bool IDENT>
  __device__ __forceinline__ D3 vertex(const GeomRec& G, int v, const BodyView& V) const {
    const int i = G.v_off + v;
    const D3 l = d3(tb.vx[i], tb.vy[i], tb.vz[i]);
    if (IDENT) return l;
    return d3(V.R[0] * l.x + V.R[1] * l.y + V.R[2] * l.z + V.t[0], V.R[3] * l.x + V.R[4] * l.y + V.R[5] * l.z + V.t[1],
              V.R[6] * l.x + V.R[7] * l.y + V.R[8] * l.z + V.t[2]);
  }

  // ------------------------------------------------------------ stage
  __device__ __forceinline__ void stage() {
    const int neA = A.ne, neB = B.ne, nfA = A.nf, nfB = B.nf;
    for (int i = tid; i < neA + neB; i += BLOCK) {
      const bool isA = i < neA;
      const int e = isA ? i : i - neA;
      const GeomRec& G = isA ? *GA : *GB;
      const int i0 = tb.e0[G.e_off + e], i1 = tb.e1[G.e_off + e];
      const D3 p0 = isA ? vertex<true>(G, i0, A) : vertex<false>(G, i0, B);
      const D3 p1 = isA ? vertex<true>(G, i1, A) : vertex<false>(G, i1, B);
      // select the destination pointers by value (a reference select would
      // force the engine object into scratch memory)
      double* x0 = isA ? EA.x0 : EB.x0;
      double* y0 = isA ? EA.y0 : EB.y0;
      double* z0 = isA ? EA.z0 : EB.z0;
      double* tx = isA ? EA.tx : EB.tx;
      double* ty = isA ? EA.ty : EB.ty;
      double* tz = isA ? EA.tz : EB.tz;
      x0[e] = p0.x; y0[e] = p0.y; z0[e] = p0.z;
      tx[e] = p1.x - p0.x; ty[e] = p1.y - p0.y; tz[e] = p1.z - p0.z;
    }
    for (int i = tid; i < nfA + nfB; i += BLOCK) {
      const bool isA = i < nfA;
      const int f = isA ? GA->f_off + i : GB->f_off + (i - nfA);
      const int j = isA ? i : i - nfA;
      // planes pre-scaled by c = log2(e) / tau (the polytope SDF works in
      // binary-exponent units)
      // (superquadric-union and point-cloud records are staged as they are)
      const int ty = isA ? A.type : B.type;
      const double c = (ty == CM_SQ_UNION || ty == CM_OPC) ? 1.0 : T.c;
      (isA ? sPA : sPB)[j] = make_double4(c * tb.fnx[f], c * tb.fny[f], c * tb.fnz[f], c * tb.fo[f]);
    }
    __syncthreads();
  }

  // ------------------------------------------------------------ pre-selection
  // Soft top-K pre-selection (PRESEL): every vertex gets the other body's SDF
  // at it as penetration metric (float64 LSE: the selection weights divide
  // metric differences by tau), every edge the mean of its corners'; for
  // each of the four sets (A's vertices, B's, A's edges, B's) the K largest
  // values x_[k] of x = -metric are found (a wave per set), and each soft
  // vertex / edge k is the average of the set's positions with SoftSort
  // weights exp(-|x_[k] - x_i| / tau) (one thread per selected item; float64
  // exponentials, as the weights move geometry).  The soft edges then replace
  // the staged edges and the counts shrink to the selection sizes.
  // sel_idx (optional, [4][CM_MAX_PRESEL]): receives the index within its set
  // of the item whose value is x_[k] (the adjoint routes x_[k]'s gradient there).
  __device__ __forceinline__ void select(int* sel_idx = nullptr) {
    const int nvA = A.nv, nvB = B.nv, neA = A.ne, neB = B.ne;
    double* mVA = sMet;
    double* mVB = sMet + maxV;
    double* mEA = sMet + 2 * maxV;
    double* mEB = mEA + maxE;
    for (int i = tid; i < nvA + nvB; i += BLOCK) {
      if (i < nvA) mVA[i] = sdf_value64<false, SQ>(B, vertex<true>(*GA, i, A), T);
      else mVB[i - nvA] = sdf_value64<true, SQ>(A, vertex<false>(*GB, i - nvA, B), T);
    }
    __syncthreads();
    for (int i = tid; i < neA + neB; i += BLOCK) {
      const bool onA = i < neA;
      const int e = onA ? i : i - neA;
      const GeomRec* G = onA ? GA : GB;
      const double* mv = onA ? mVA : mVB;
      double* me = onA ? mEA : mEB;
      me[e] = 0.5 * (mv[tb.e0[G->e_off + e]] + mv[tb.e1[G->e_off + e]]);
    }
    __syncthreads();
    const int Kva = min(kv, nvA), Kvb = min(kv, nvB), Kea = min(ke, neA), Keb = min(ke, neB);
    // hard top-K of -metric per set: K rounds of a wave-wide maximum; the
    // lowest lane holding it removes its item (bit j of `taken`: item lane + 64 j)
    for (int set = wave; set < 4; set += NW) {
      const double* m = set == 0 ? mVA : set == 1 ? mVB : set == 2 ? mEA : mEB;
      const int D = set == 0 ? nvA : set == 1 ? nvB : set == 2 ? neA : neB;
      const int Ks = set == 0 ? Kva : set == 1 ? Kvb : set == 2 ? Kea : Keb;
      unsigned long long taken = 0ull;
      for (int r = 0; r < Ks; ++r) {
        double best = -INFINITY;
        int bj = -1;
        for (int j = 0; lane + 64 * j < D; ++j) {
          const double x = -m[lane + 64 * j];
          if (!((taken >> j) & 1ull) && x > best) { best = x; bj = j; }
        }
        const double wm = wave_max(best);
        const unsigned long long ball = __ballot(bj >= 0 && best == wm);
        if (lane == __ffsll((long long)ball) - 1) {
          taken |= 1ull << bj;
          if (sel_idx) sel_idx[set * CM_MAX_PRESEL + r] = lane + 64 * bj;
        }
        if (lane == 0) sSel[set * CM_MAX_PRESEL + r] = wm;
      }
    }
    __syncthreads();
    // soft items: thread t < Kva + Kvb + Kea + Keb builds one
    double* softE = sSoft + 2 * CM_MAX_PRESEL * 3;
    if (tid < Kva + Kvb + Kea + Keb) {
      int set = 0, k = tid;
      if (k >= Kva) { k -= Kva; set = 1;
        if (k >= Kvb) { k -= Kvb; set = 2;
          if (k >= Kea) { k -= Kea; set = 3; } } }
      const double* m = set == 0 ? mVA : set == 1 ? mVB : set == 2 ? mEA : mEB;
      const int D = set == 0 ? nvA : set == 1 ? nvB : set == 2 ? neA : neB;
      const double xk = sSel[set * CM_MAX_PRESEL + k];
      double sw = 0.0, a[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int i = 0; i < D; ++i) {
        const double w = exp64n(-fabs(xk + m[i]) * T.inv_tau);   // x_i = -m[i]
        sw += w;
        if (set < 2) {
          const D3 v = set == 0 ? vertex<true>(*GA, i, A) : vertex<false>(*GB, i, B);
          a[0] = fma(w, v.x, a[0]); a[1] = fma(w, v.y, a[1]); a[2] = fma(w, v.z, a[2]);
        } else {
          D3 p0, t;
          if (set == 2) EA.get(i, p0, t);
          else EB.get(i, p0, t);
          a[0] = fma(w, p0.x, a[0]); a[1] = fma(w, p0.y, a[1]); a[2] = fma(w, p0.z, a[2]);
          a[3] = fma(w, p0.x + t.x, a[3]); a[4] = fma(w, p0.y + t.y, a[4]); a[5] = fma(w, p0.z + t.z, a[5]);
        }
      }
      const double inv = 1.0 / sw;   // sw >= 1: the row's own maximum has weight 1
      if (set < 2) {
        double* o = sSoft + 3 * (set * CM_MAX_PRESEL + k);
        o[0] = a[0] * inv; o[1] = a[1] * inv; o[2] = a[2] * inv;
      } else {
        double* o = softE + 6 * ((set - 2) * CM_MAX_PRESEL + k);
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = a[c] * inv;
      }
    }
    __syncthreads();
    // the soft edges replace the staged ones; counts shrink
    for (int i = tid; i < Kea + Keb; i += BLOCK) {
      const bool onA = i < Kea;
      const int k = onA ? i : i - Kea;
      const double* o = softE + 6 * ((onA ? 0 : CM_MAX_PRESEL) + k);
      double* x0 = onA ? EA.x0 : EB.x0;
      double* y0 = onA ? EA.y0 : EB.y0;
      double* z0 = onA ? EA.z0 : EB.z0;
      double* tx = onA ? EA.tx : EB.tx;
      double* ty = onA ? EA.ty : EB.ty;
      double* tz = onA ? EA.tz : EB.tz;
      x0[k] = o[0]; y0[k] = o[1]; z0[k] = o[2];
      tx[k] = o[3] - o[0]; ty[k] = o[4] - o[1]; tz[k] = o[5] - o[2];
    }
    A.nv = Kva; A.ne = Kea;
    B.nv = Kvb; B.ne = Keb;
    if (tid == 0) {
      ps.A.nv = Kva; ps.A.ne = Kea;
      ps.B.nv = Kvb; ps.B.ne = Keb;
      ps.nvs = Kva + ((flags & CM_FLAG_ONE_SIDED_VS) ? 0 : Kvb);
      ps.nee = (flags & CM_FLAG_NO_EE) ? 0 : Kea * Keb;
      ps.ncand = ps.nvs + 2 * ps.nee;
    }
    __syncthreads();
  }

  // ------------------------------------------------------------ cull
  // Per edge segment of A and of B (extended to the witness range of the
  // smoothed QP, alpha in [-0.3 tau, 1 + 0.3 tau]): the faces of each
  // polytope whose plane can come within 38 binary orders (scaled units) of
  // the largest plane value at some point of the segment.  Plane values are
  // linear along the segment, so face g is dropped when
  // max(y'_g(p0), y'_g(p1)) < max_f min(y'_f(p0), y'_f(p1)) - 38, which
  // bounds its term in the LSE and in the gradient softmax below 2^-38.
  // Witness 1 lies on an edge of A, witness 2 on an edge of B.  The
  // candidate pass needs the union over each group of 8 consecutive edges
  // (the rows and columns of its tiles): each edge's thread ORs its
  // segment's words into its group's masks (LDS atomics), so no per-edge
  // mask is stored.
  __device__ __forceinline__ void cull() {
    if (!CULL || MW == 0 || ps.nee == 0) return;
    const double ext = 0.3 * T.tau;
    const int neA = A.ne;
    const int ngA = (neA + 7) >> 3, ngB = (B.ne + 7) >> 3;
    for (int i = tid; i < 2 * (ngA + ngB); i += BLOCK) {
      FaceMask& m = i < 2 * ngA ? sG1[i] : sG2[i - 2 * ngA];
      for (int w = 0; w < MW; ++w) m.w[w] = 0ull;
      m.n = MW;
    }
    __syncthreads();
    for (int i = tid; i < neA + B.ne; i += BLOCK) {
      const bool onA = i < neA;
      const int k = onA ? i : i - neA;
      D3 a0, t1;
      if (onA) EA.get(k, a0, t1);
      else EB.get(k, a0, t1);
      const D3 p0 = d3(a0.x - ext * t1.x, a0.y - ext * t1.y, a0.z - ext * t1.z);
      const D3 p1 = d3(a0.x + (1.0 + ext) * t1.x, a0.y + (1.0 + ext) * t1.y, a0.z + (1.0 + ext) * t1.z);
      FaceMask* grp = (onA ? sG1 : sG2) + 2 * (k >> 3);
      const double sA = seg_mask_or(A, false, p0, p1, grp[0].w);
      const double sB = seg_mask_or(B, true, p0, p1, grp[1].w);
      gShift[i] = onA ? sB : sA;   // the other body's (the own body's queries are surface ones)
    }
    __syncthreads();
    // a copy for the filtered candidates' queries (records overwrite sG1 / sG2)
    if (!union_masks()) return;
    const int gw = int(sizeof(FaceMask) / 8), nA = 2 * ngA, nB = 2 * ngB, gB0 = 2 * ((maxE + 7) >> 3);
    for (int i = tid; i < (nA + nB) * gw; i += BLOCK) {
      const int m = i / gw, w = i - m * gw;
      const unsigned long long* src = reinterpret_cast<const unsigned long long*>(m < nA ? sG1 + m : sG2 + (m - nA));
      reinterpret_cast<unsigned long long*>(m < nA ? gMask + m : gMask + gB0 + (m - nA))[w] = src[w];
    }
  }
  // The union of the group masks of a wave's candidates idx (lanes with act)
  // into U[0..3]: A's and B's faces near witness 1, A's and B's near witness
  // 2 (LDS, this wave's), for queries that all the wave's lanes share;
  // returns U, or null when a lane holds a vertex candidate (or none is
  // active, or union_masks() is false).  Every lane of the wave calls it.
  // For pairs whose polytopes have at most 64 faces the walks save less
  // than the union costs (measured on hulls of 32 points); a property of the
  // pair, so that every launch shape decides alike.
  __device__ __forceinline__ bool union_masks() const { return MW > 0 && (A.nf > 64 || B.nf > 64); }
  __device__ __forceinline__ const FaceMask* wave_union(bool act, int idx, FaceMask* U) const {
    if (!union_masks() || ps.nee == 0) return nullptr;
    const bool eecand = act && idx >= ps.nvs;
    if (__ballot(act && !eecand) != 0ull || __ballot(eecand) == 0ull) return nullptr;
    if (lane < 4 * MW) U[lane / MW].w[lane - (lane / MW) * MW] = 0ull;
    if (lane < 4) U[lane].n = MW;
    wave_lds_sync();
    if (eecand) {
      const int ee_i = (idx - ps.nvs) >> 1;
      const int k = ee_i / B.ne, l = ee_i - k * B.ne;
      const FaceMask* g1 = gMask + 2 * (k >> 3);
      const FaceMask* g2 = gMask + 2 * ((maxE + 7) >> 3) + 2 * (l >> 3);
      for (int w = 0; w < MW; ++w) {
        const unsigned long long a0 = g1[0].w[w], a1 = g1[1].w[w], a2 = g2[0].w[w], a3 = g2[1].w[w];
        if (a0) atomicOr(&U[0].w[w], a0);
        if (a1) atomicOr(&U[1].w[w], a1);
        if (a2) atomicOr(&U[2].w[w], a2);
        if (a3) atomicOr(&U[3].w[w], a3);
      }
    }
    wave_lds_sync();
    return U;
  }
  // OR the faces of V near segment [p0w, p1w] (pair frame) into out[MW];
  // returns a shift for V's value queries at points of the segment, or
  // kNoShift.  With y_f the scaled plane values, L = max_f min(y_f(p0),
  // y_f(p1)) and U = max_f max(y_f(p0), y_f(p1)), every point x of the
  // segment has L <= max_f y_f(x) <= U (y_f is affine along it), and the
  // face attaining L is in the mask; so L shifts the masked float32 sum of
  // 2^(y_f - L) into [1, nf 2^(U - L)] and replaces the max pass when
  // U - L <= 100.
  __device__ __forceinline__ double seg_mask_or(const BodyView& V, bool moved, const D3& p0w, const D3& p1w,
                                                unsigned long long* out) const {
    if (V.type != CM_POLYTOPE) {
      for (int w = 0; w < MW; ++w) atomicOr(out + w, ~0ull);
      return kNoShift;
    }
    D3 p0 = p0w, p1 = p1w;
    if (moved) {
      p0 = d3(V.R[0] * (p0w.x - V.t[0]) + V.R[3] * (p0w.y - V.t[1]) + V.R[6] * (p0w.z - V.t[2]),
              V.R[1] * (p0w.x - V.t[0]) + V.R[4] * (p0w.y - V.t[1]) + V.R[7] * (p0w.z - V.t[2]),
              V.R[2] * (p0w.x - V.t[0]) + V.R[5] * (p0w.y - V.t[1]) + V.R[8] * (p0w.z - V.t[2]));
      p1 = d3(V.R[0] * (p1w.x - V.t[0]) + V.R[3] * (p1w.y - V.t[1]) + V.R[6] * (p1w.z - V.t[2]),
              V.R[1] * (p1w.x - V.t[0]) + V.R[4] * (p1w.y - V.t[1]) + V.R[7] * (p1w.z - V.t[2]),
              V.R[2] * (p1w.x - V.t[0]) + V.R[5] * (p1w.y - V.t[1]) + V.R[8] * (p1w.z - V.t[2]));
    }
    double L = -1e300;
    for (int f = 0; f < V.nf; ++f) {
      const double4 q = V.planes[f];
      const double y0 = fma(q.x, p0.x, fma(q.y, p0.y, fma(q.z, p0.z, -q.w)));
      const double y1 = fma(q.x, p1.x, fma(q.y, p1.y, fma(q.z, p1.z, -q.w)));
      L = fmax(L, fmin(y0, y1));
    }
    unsigned long long m = 0ull;
    double U = -1e300;
    for (int f = 0; f < V.nf; ++f) {
      const double4 q = V.planes[f];
      const double y0 = fma(q.x, p0.x, fma(q.y, p0.y, fma(q.z, p0.z, -q.w)));
      const double y1 = fma(q.x, p1.x, fma(q.y, p1.y, fma(q.z, p1.z, -q.w)));
      U = fmax(U, fmax(y0, y1));
      if (fmax(y0, y1) >= L - 38.0) m |= 1ull << (f & 63);
      if ((f & 63) == 63 || f == V.nf - 1) {
        if (m) atomicOr(out + (f >> 6), m);
        m = 0ull;
      }
    }
    return U - L <= 100.0 ? L : kNoShift;
  }

  // ------------------------------------------------------------ candidates
  // soft vertex i of the selection (A's first, then B's), pair frame
  __device__ __forceinline__ D3 soft_vertex(int i) const {
    const double* v = sSoft + 3 * (i < A.nv ? i : CM_MAX_PRESEL + (i - A.nv));
    return d3(v[0], v[1], v[2]);
  }
  __device__ __forceinline__ void vs(int i, Cand& c) const {
    if (PRESEL) {
      if (i < A.nv) vs_candidate<false, SQ>(soft_vertex(i), B, -1.0, T, c);
      else vs_candidate<true, SQ>(soft_vertex(i), A, 1.0, T, c);
      return;
    }
    if (i < A.nv) vs_candidate<false, SQ>(vertex<true>(*GA, i, A), B, -1.0, T, c);
    else vs_candidate<true, SQ>(vertex<false>(*GB, i - A.nv, B), A, 1.0, T, c);
  }
  // both candidates of edge pair (k, l) from the QP solution stored by the
  // distance pass.  m1 / m2: the face masks of the groups holding edge k of
  // A / edge l of B, shared by every active lane of the wave (a pass-2
  // tile), or null (every face: recomputes of filtered candidates, whose
  // lanes hold unrelated edge pairs; the two differ by less than 2^-38
  // relative).
  __device__ __forceinline__ void ee(int k, int l, Cand& c1, Cand& c2, const FaceMask* m1 = nullptr,
                                     const FaceMask* m2 = nullptr, double sh1 = kNoShift,
                                     double sh2 = kNoShift) const {
    D3 a0, t1, b0, t2;
    EA.get(k, a0, t1);
    EB.get(l, b0, t2);
    const int i = k * B.ne + l;
    const EEQP q = ee_from_alpha(a0, t1, b0, t2, Al1[i], Al2[i], Lcon[i]);
    ee_candidates<PRESEL, SQ, REFINE>(a0, t1, b0, t2, q, sRow[k], sCol[l], A, B, eps_n, T, m1, m2, c1, c2,
                                      PRESEL && (flags & CM_FLAG_SAFEGUARD), refine, sh1, sh2);
  }
  // candidate idx in the fixed order: A's vertices, B's vertices, E-E (k, l)
  // row-major with witness 1 before witness 2
  // U: the wave's union masks (wave_union) for an E-E candidate, or null.
  __device__ __forceinline__ void candidate(int idx, Cand& c, const FaceMask* U = nullptr) const {
    if (idx < ps.nvs) {
      vs(idx, c);
    } else {
      const int e = idx - ps.nvs;
      const int ee_i = e >> 1;
      const int k = ee_i / B.ne, l = ee_i - k * B.ne;
      Cand c1, c2;
      ee(k, l, c1, c2, U, U ? U + 2 : nullptr, U ? gShift[k] : kNoShift, U ? gShift[A.ne + l] : kNoShift);
      c = (e & 1) ? c2 : c1;
    }
  }

  // ------------------------------------------------------------ scores
  // E-E pass 1: the unsigned distance D and QP solution of every edge pair,
  // then the row and column LSE of D (ends with a barrier).
  __device__ __forceinline__ void pass1() {
    const int neA = A.ne, neB = B.ne, nee = ps.nee;
    {
      int k = tid / neB, l = tid - (tid / neB) * neB;
      const int sk = BLOCK / neB, sl = BLOCK - sk * neB;
      for (int idx = tid; idx < nee; idx += BLOCK) {
        D3 a0, t1, b0, t2;
        EA.get(k, a0, t1);
        EB.get(l, b0, t2);
        const EEQP q = ee_qp(a0, t1, b0, t2, lam, T);
        double dq, idum;
        sqrt_rsq64(dot(q.de, q.de), dq, idum);   // as the candidates' nearest-neighbour distance
        Dbuf[idx] = dq;
        Al1[idx] = q.al1;
        Al2[idx] = q.al2;
        Lcon[idx] = q.log_con;
        k += sk; l += sl;
        if (l >= neB) { l -= neB; ++k; }
      }
    }
    __syncthreads();
    if (nee == 0) return;   // vertex-SDF candidates only (CM_FLAG_NO_EE)
    // row LSE over l (one wave per row, coalesced)
    for (int k = wave; k < neA; k += NW) {
      double m = INFINITY;
      float s = 0.f;
      for (int l = lane; l < neB; l += 64) lse_push(m, s, Dbuf[k * neB + l], T);
      wave_lse_merge(m, s, T);
      if (lane == 0) sRow[k] = m - T.tl * double(lg2f(s));
    }
    // column LSE over k (threads over columns, k split in chunks, coalesced).
    // The chunking is that of kColSlots virtual threads whatever the block
    // size (a thread takes slots tid, tid + BLOCK, ...), so the float32 sums
    // associate alike in every instantiation: columns of width >= kColSlots
    // run whole, narrower ones in kColSlots / neB chunks of rows merged in
    // chunk order.
    if (neB >= kColSlots) {
      for (int l = tid; l < neB; l += BLOCK) {
        double m = INFINITY;
        float s = 0.f;
        for (int k = 0; k < neA; ++k) lse_push(m, s, Dbuf[k * neB + l], T);
        sCol[l] = m - T.tl * double(lg2f(s));
      }
    } else {
      const int nch = kColSlots / neB;
      for (int v = tid; v < kColSlots; v += BLOCK) {
        const int l = v % neB, ch = v / neB;
        double m = INFINITY;
        float s = 0.f;
        if (ch < nch) {
          const int k0 = (ch * neA) / nch, k1 = ((ch + 1) * neA) / nch;
          for (int k = k0; k < k1; ++k) lse_push(m, s, Dbuf[k * neB + l], T);
        }
        sRed[v] = m;
        sRed[kColSlots + v] = double(s);
      }
      __syncthreads();
      for (int l = tid; l < neB; l += BLOCK) {
        double M = sRed[l];
        float S = float(sRed[kColSlots + l]);
        for (int c = 1; c < nch; ++c) {
          const double m2 = sRed[c * neB + l];
          const float s2 = float(sRed[kColSlots + c * neB + l]);
          const double Mn = fmin(M, m2);
          const float a = (M == Mn) ? S : S * expn(M - Mn, T);
          const float bb = (m2 == Mn) ? s2 : s2 * expn(m2 - Mn, T);
          M = Mn; S = a + bb;
        }
        sCol[l] = M - T.tl * double(lg2f(S));
      }
    }
    __syncthreads();
  }

  // Scores of every candidate into Sbuf and the per-lane top-K lists.
  __device__ __forceinline__ void scores(double (&tk)[KMAX]) {
    const int neA = A.ne, neB = B.ne, nee = ps.nee, nvs = ps.nvs;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) tk[i] = -INFINITY;
    // V-S candidates (Sec. IV-C), both ways
    for (int i = tid; i < nvs; i += BLOCK) {
      Cand c;
      vs(i, c);
      Sbuf[i] = float(c.s);
      tk_insert<KMAX>(tk, c.s);
    }
    pass1();
    if (nee == 0) return;
    // E-E pass 2: candidates, scores, top-K.  The forward kernel gives each
    // wave 8 x 8 tiles of edge pairs (lane = 8 kk + ll), whose witness
    // queries share the tile's face masks (polytope edges are stored in
    // spatially compact runs of 8); the adjoint's recompute goes row-major
    // over the block.  One inlined form of the candidate code per kernel
    // keeps register pressure down.
    if (CULL) {
      const int ntl = (neB + 7) >> 3, ntiles = ((neA + 7) >> 3) * ntl;
      const int kk = lane >> 3, ll = lane & 7;
      for (int t = wave; t < ntiles; t += NW) {
        const int k0 = (t / ntl) * 8, l0 = (t - (t / ntl) * ntl) * 8;
        // the tile's group masks: [A's faces, B's faces] near its rows / columns
        const FaceMask* m1 = MW > 0 ? sG1 + 2 * (k0 >> 3) : nullptr;
        const FaceMask* m2 = MW > 0 ? sG2 + 2 * (l0 >> 3) : nullptr;
        const int k = k0 + kk, l = l0 + ll;
        if (k < neA && l < neB) {
          const int idx = k * neB + l;
          Cand c1, c2;
          // the value queries' shifts along the lane's segments (cull)
          const double sh1 = MW > 0 ? gShift[k] : kNoShift, sh2 = MW > 0 ? gShift[neA + l] : kNoShift;
          ee(k, l, c1, c2, m1, m2, sh1, sh2);
          Sbuf[nvs + 2 * idx] = float(c1.s);
          Sbuf[nvs + 2 * idx + 1] = float(c2.s);
          tk_insert<KMAX>(tk, c1.s);
          tk_insert<KMAX>(tk, c2.s);
        }
      }
    } else {
      int k = tid / neB, l = tid - (tid / neB) * neB;
      const int sk = BLOCK / neB, sl = BLOCK - sk * neB;
      for (int idx = tid; idx < nee; idx += BLOCK) {
        Cand c1, c2;
        ee(k, l, c1, c2);
        Sbuf[nvs + 2 * idx] = float(c1.s);
        Sbuf[nvs + 2 * idx + 1] = float(c2.s);
        tk_insert<KMAX>(tk, c1.s);
        tk_insert<KMAX>(tk, c2.s);
        k += sk; l += sl;
        if (l >= neB) { l -= neB; ++k; }
      }
    }
  }

  // ------------------------------------------------------------ top-K
  // Block merge of per-lane sorted lists: K rounds of block max; the lowest
  // thread holding the maximum pops it.  sTop[0..K) = s_[1] >= ... >= s_[K].
  __device__ __forceinline__ void topk(double (&tk)[KMAX]) {
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
  }

  // ------------------------------------------------------------ filtered iteration
  // The window test of candidate idx: its stored score within `taus` tau of
  // s_[K] (thr from window_thr), or its bit in a recorded mask.
  __device__ __forceinline__ float window_thr(double taus) const {
    return float(sTop[K - 1] - taus * T.tau) - 1e-6f * fabsf(float(sTop[K - 1]));
  }
  // Compacts the candidates in the window into List: each wave its
  // contiguous share of the candidates (ballot prefix sums, candidate order
  // kept); returns their count (after a barrier; the wave counts stay in
  // sCnt for list_at).  mask: the window as recorded by the forward (one bit
  // per candidate, device memory) instead of the stored scores.
  __device__ __forceinline__ int window(double taus, const unsigned long long* __restrict__ mask = nullptr) {
    const float thr = window_thr(taus);
    const int ncand = ps.ncand;
    const int seg = (ncand + NW - 1) / NW;
    const int lo = min(ncand, wave * seg), hi = min(ncand, lo + seg);
    int n = 0;
    for (int b = lo; b < hi; b += 64) {
      const int idx = b + lane;
      const bool pass = idx < hi && (mask ? ((mask[idx >> 6] >> (idx & 63)) & 1ull) != 0ull : Sbuf[idx] >= thr);
      const unsigned long long ball = __ballot(pass);
      if (pass) List[lo + n + __popcll(ball & ((1ull << lane) - 1ull))] = idx;
      n += __popcll(ball);
    }
    if (lane == 0) sCnt[wave] = n;
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) tot += sCnt[w];
    return tot;
  }
  // Writes the window as a bit mask (bit idx & 63 of word idx >> 6), one
  // ballot per 64 candidates.
  __device__ __forceinline__ void window_mask(double taus, unsigned long long* __restrict__ mask) const {
    const float thr = window_thr(taus);
    const int ncand = ps.ncand;
    for (int b = wave * 64; b < ncand; b += BLOCK) {
      const int idx = b + lane;
      const unsigned long long ball = __ballot(idx < ncand && Sbuf[idx] >= thr);
      if (lane == 0) mask[b >> 6] = ball;
    }
  }
  // Writes the window compacted by window() (tot candidates) to dst in three
  // runs, each in candidate order: the vertex-SDF candidates, the edge-edge
  // witnesses 1, the witnesses 2.  Waves of the adjoint that take one run
  // then need one penetration query adjoint instead of both.  Uses sRed.
  __device__ __forceinline__ void write_window_runs(int tot, int* __restrict__ dst) {
    int* cnt = reinterpret_cast<int*>(sRed);   // [3][NW] per-wave counts of a chunk
    int* run = cnt + 3 * NW;                   // [3] run sizes
    const int nvs = ps.nvs;
    auto cls_of = [&](int idx) __attribute__((always_inline)) { return idx < nvs ? 0 : (((idx - nvs) & 1) ? 2 : 1); };
    if (tid < 3) run[tid] = 0;
    __syncthreads();
    for (int base = 0; base < tot; base += BLOCK) {
      const int p = base + tid;
      const int c = p < tot ? cls_of(list_at(p)) : 3;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const unsigned long long b = __ballot(c == k);
        if (lane == 0 && b) atomicAdd(&run[k], __popcll(b));
      }
    }
    __syncthreads();
    int off[3] = {0, run[0], run[0] + run[1]};
    __syncthreads();
    for (int base = 0; base < tot; base += BLOCK) {
      const int p = base + tid;
      const int idx = p < tot ? list_at(p) : 0;
      const int c = p < tot ? cls_of(idx) : 3;
      unsigned long long b[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) b[k] = __ballot(c == k);
      if (lane == 0)
        for (int k = 0; k < 3; ++k) cnt[k * NW + wave] = __popcll(b[k]);
      __syncthreads();
      if (c < 3) {
        int before = 0;
        for (int w = 0; w < wave; ++w) before += cnt[c * NW + w];
        dst[off[c] + before + __popcll(b[c] & ((1ull << lane) - 1ull))] = idx;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k)
        for (int w = 0; w < NW; ++w) off[k] += cnt[k * NW + w];
      __syncthreads();
    }
  }
  // Candidate index at position p (< window's count) of the compacted list.
  __device__ __forceinline__ int list_at(int p) const {
    // the wave region holding list position p: the last wave whose start is
    // <= p (empty regions share the next region's start)
    int reg = 0, off = 0, acc = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      if (p >= acc) { reg = w; off = acc; }
      acc += sCnt[w];
    }
    const int seg = (ps.ncand + NW - 1) / NW;
    return List[min(ps.ncand, reg * seg) + (p - off)];
  }
  // Candidate idx evaluated into this thread's record.
  __device__ __forceinline__ void record(int idx, const FaceMask* U = nullptr) {
    Cand c;
    candidate(idx, c, U);
    Rec& rr = sRec[tid];
    rr.s = c.s; rr.d = c.d;
    rr.px = float(c.p.x); rr.py = float(c.p.y); rr.pz = float(c.p.z);
    rr.nx = float(c.n.x); rr.ny = float(c.n.y); rr.nz = float(c.n.z);
    rr.w = ex2f(float(c.lw * kLog2e));
    rr.idx = idx;
  }
  // Visit the candidates whose stored score is within `taus` tau of s_[K]:
  // the compacted list is evaluated densely in chunks of BLOCK, one
  // candidate record per thread in sRec, and body(n) runs with all threads
  // after a barrier for each chunk of n records.  The forward may have
  // recorded the same window: ntape >= 0 indices at lst, or else a mask
  // (device memory); otherwise the stored scores are scanned.  full = false:
  // only the records' candidate indices are written (a body that evaluates
  // the candidates itself).
  // um: LDS for 4 face masks per wave, through which the records of a wave
  // of E-E candidates query (wave_union; the values differ from the
  // all-faces ones by less than 2^-38 relative), or null.
  template <typename F>
  __device__ __forceinline__ void for_window(const int* __restrict__ lst, int ntape,
                                             const unsigned long long* __restrict__ mask, F&& body, double taus,
                                             bool full = true, FaceMask* um = nullptr) {
    const int tot = ntape >= 0 ? ntape : window(taus, mask);
    if (ntape < 0 && tot == 0) __syncthreads();   // sCnt is rewritten by the next call
    for (int base = 0; base < tot; base += BLOCK) {
      const int p = base + tid;
      int idx = 0;
      if (p < tot) {
        idx = ntape >= 0 ? lst[p] : list_at(p);
        if (idx < 0 || idx >= ps.ncand) idx = 0;   // a recorded list holds valid indices; never read past the pair
      }
      const FaceMask* U = (full && um != nullptr) ? wave_union(p < tot, idx, um + 4 * wave) : nullptr;
      if (p < tot) {
        if (full) record(idx, U);
        else sRec[tid].idx = idx;
      }
      __syncthreads();
      body(min(BLOCK, tot - base));
      __syncthreads();
    }
  }
  template <typename F>
  __device__ __forceinline__ void for_filtered(F&& body, double taus = kFilterTaus, FaceMask* um = nullptr) {
    for_window(nullptr, -1, nullptr, body, taus, true, um);
  }

  // ------------------------------------------------------------ SoftSort
  // sAcc[9k + f] = sum_i exp(-|s_[k] - s_i| / tau) * field_f(i), field 0 = 1.
  // G consecutive lanes own row k (G = BLOCK / K rounded down to a power of
  // two, at most 64, so a row's lanes sit in one wave); lane j of the group
  // takes records j, j + G, ... and the exponential once for all nine fields.
  // The G partial sums of a row meet in a shuffle tree at the end.
  __device__ __forceinline__ void softsort() {
    int G = 64;
    while (G * K > BLOCK) G >>= 1;
    const int kk = tid / G, j0 = tid - kk * G;
    const bool act = kk < K;
    const double sk = act ? sTop[kk] : 0.0;
    double a[9];
#pragma unroll
    for (int f = 0; f < 9; ++f) a[f] = 0.0;
    // the per-wave union masks of the records live in the reduction slots,
    // which nothing else uses here (topk is done)
    for_filtered([&](int tot) {
      if (!act) return;
      for (int r = j0; r < tot; r += G) {
        const Rec& rr = sRec[r];
        const double e = double(expn(fabs(sk - rr.s), T));
        a[0] += e;
        a[1] = fma(e, double(rr.px), a[1]);
        a[2] = fma(e, double(rr.py), a[2]);
        a[3] = fma(e, double(rr.pz), a[3]);
        a[4] = fma(e, double(rr.nx), a[4]);
        a[5] = fma(e, double(rr.ny), a[5]);
        a[6] = fma(e, double(rr.nz), a[6]);
        a[7] = fma(e, rr.d, a[7]);
        a[8] = fma(e, double(rr.w), a[8]);
      }
    }, kFilterTaus, CULL ? reinterpret_cast<FaceMask*>(sRed) : nullptr);
    for (int off = G >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int f = 0; f < 9; ++f) a[f] += __shfl_xor(a[f], off);
    }
    if (act && j0 == 0) {
#pragma unroll
      for (int f = 0; f < 9; ++f) sAcc[9 * kk + f] = a[f];
    }
    __syncthreads();
  }
};

}  // namespace cm
