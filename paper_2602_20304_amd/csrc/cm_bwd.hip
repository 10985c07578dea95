// gfx950 adjoint of the contact manifold: vector-Jacobian product of the
// K-contact manifold with respect to body poses (left tangent twists),
// polytope hull vertices, analytic geometry parameters and tau.
//
// One workgroup per kept pair.  The forward phases are recomputed with the
// shared engine (no E x E state was stored by the forward), then:
//   A1  SoftSort adjoint, part 1: adjoints of the K top scores s_[k] and the
//       candidate j_k that attains each of them
//   A2  per-candidate adjoint for every candidate within 18 tau of s_[K]
//       (all others have SoftSort weight below exp(-18)): score / weight /
//       field adjoints -> indicators -> SDF queries -> witness QP -> edges
//   N   nearest-neighbour adjoint: row / column LSE adjoints flow back into
//       every unsigned distance D_kl of the touched rows and columns
//   S   (pre-selection only) SoftSort-selection adjoint: the soft vertices'
//       and soft edges' adjoints flow to the mesh vertices through the
//       normalised weights, and to the penetration metrics through the
//       weights' dependence on x_i and x_[k]; the metrics' adjoints then run
//       through the SDF queries that produced them
//   G   face-plane adjoints -> hull vertices, mesh vertices -> parameters,
//       B's placement twist and the output transform -> world pose twists
#include <hip/hip_runtime.h>

#include "cm_adjoint.cuh"
#include "cm_kernels.h"
#include "cm_pair.cuh"

namespace cm {

struct BwdLds {
  int vA, vB, plA, plB, prm, rbar, cbar, cot, F, top, best, bt, tw, um, sv, se, si, mb, sk, bytes;
};

// presel: the selection adjoint's arrays follow (soft vertex adjoints
// [2][CM_MAX_PRESEL][3], soft edge endpoint adjoints [2][CM_MAX_PRESEL][6],
// selected indices [4][CM_MAX_PRESEL], metric adjoints of both bodies'
// vertices [2][maxV], weight sums and <adjoint, soft item> per item [2][4][CM_MAX_PRESEL]).
__host__ __device__ inline BwdLds bwd_layout(int base, int maxV, int maxE, int maxF, int block, bool presel) {
  BwdLds L;
  int o = base;
  L.vA = o; o += 4 * 3 * maxV;
  L.vB = o; o += 4 * 3 * maxV;
  L.plA = o; o += 4 * 4 * maxF;
  L.plB = o; o += 4 * 4 * maxF;
  L.prm = o; o += 4 * 8;
  L.rbar = o; o += 4 * maxE;
  L.cbar = o; o += 4 * maxE;
  o = (o + 7) & ~7;
  L.cot = o; o += 8 * 8 * CM_MAX_K;    // pair-frame cotangents per row: p(3) nu(3) d w
  L.F = o; o += 8 * 10 * CM_MAX_K;     // normalised row outputs (8) + Z + Gbar
  L.top = o; o += 8 * CM_MAX_K;        // adjoint of s_[k]
  L.best = o; o += 4 * (CM_MAX_K + block);
  o = (o + 7) & ~7;
  L.bt = o; o += 8 * block;            // A1: each slice's own term of its nearest candidate
  L.tw = o; o += 8 * 8;                // output twist terms
  L.um = o; o += 4 * (block / 64) * int(sizeof(FaceMask));   // A2: per wave, the union face masks of its 4 query slots
  L.sv = L.se = L.si = L.mb = L.sk = o;
  if (presel) {
    L.sv = o; o += 4 * 2 * CM_MAX_PRESEL * 3;
    L.se = o; o += 4 * 2 * CM_MAX_PRESEL * 6;
    L.si = o; o += 4 * 4 * CM_MAX_PRESEL;
    L.mb = o; o += 4 * 2 * maxV;
    o = (o + 7) & ~7;
    L.sk = o; o += 8 * 2 * 4 * CM_MAX_PRESEL;
  }
  L.bytes = (o + 15) & ~15;
  return L;
}

// LDS the adjoint needs beyond the engine (an upper bound for any base),
// including the engine's pre-selection arrays when presel.
__host__ __device__ inline int bwd_extra_bytes(int maxV, int maxE, int maxF, int block, bool presel) {
  return bwd_layout(0, maxV, maxE, maxF, block, presel).bytes + 32 + (presel ? presel_lds_bytes(maxV, maxE) : 0);
}

struct Six {
  double c[6];
};

struct BwdArgs {
  CotDev cot;
  GradDev gr;
};

// Two waves per SIMD (256 registers a lane, some spilled to private memory)
// for the kernels without the extended primitives, whose dual-number
// queries would spill several times more; those take one.
// WAVES > 0 overrides the target: the full method's 256-thread kernel has a
// 3-wave variant, taken where LDS (edge arrays in the scratch slot) leaves
// room for a third workgroup per CU.
template <int BLOCK, int KMAX, bool PRESEL, bool SQ, bool REFINE = false, int WAVES = 0>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WAVES > 0 ? WAVES : (SQ ? 1 : 2))))
void collide_bwd(Tables tb, BatchDev bt, ParamsDev prm, OutDev fwd, BwdArgs ga, float* __restrict__ scratch,
                 long long scratch_stride, int maxV, int maxE, int maxF, unsigned* err, TapeDev tape,
                 int* __restrict__ queue, int edges_out) {
  extern __shared__ float4 smem4[];
  char* smem = reinterpret_cast<char*>(smem4);
  __shared__ PairShared ps;
  const int extra = bwd_extra_bytes(maxV, maxE, maxF, BLOCK, PRESEL);
  PairEngine<BLOCK, KMAX, true, PRESEL, SQ, REFINE> P(ps, smem, tb, bt, prm, scratch + (long long)blockIdx.x * scratch_stride,
                                                  maxV, maxE, maxF, extra, edges_out != 0);
  // the engine's pre-selection arrays sit right after its own layout
  const BwdLds L = bwd_layout(lds_layout(maxE, maxF, BLOCK, extra, edges_out != 0).bytes +
                                  (PRESEL ? presel_lds_bytes(maxV, maxE) : 0),
                              maxV, maxE, maxF, BLOCK, PRESEL);
  float* vA3 = reinterpret_cast<float*>(smem + L.vA);
  float* vB3 = reinterpret_cast<float*>(smem + L.vB);
  float* plA = reinterpret_cast<float*>(smem + L.plA);
  float* plB = reinterpret_cast<float*>(smem + L.plB);
  float* prA = reinterpret_cast<float*>(smem + L.prm);
  float* prB = prA + 4;
  float* rbar = reinterpret_cast<float*>(smem + L.rbar);
  float* cbar = reinterpret_cast<float*>(smem + L.cbar);
  double* cotL = reinterpret_cast<double*>(smem + L.cot);
  double* Fk = reinterpret_cast<double*>(smem + L.F);
  double* topb = reinterpret_cast<double*>(smem + L.top);
  int* bestI = reinterpret_cast<int*>(smem + L.best);
  double* btl = reinterpret_cast<double*>(smem + L.bt);
  double* twOut = reinterpret_cast<double*>(smem + L.tw);
  FaceMask* umask = reinterpret_cast<FaceMask*>(smem + L.um);
  float* svb = reinterpret_cast<float*>(smem + L.sv);   // PRESEL: soft vertex adjoints
  float* seb = reinterpret_cast<float*>(smem + L.se);   // PRESEL: soft edge endpoint adjoints
  int* selI = reinterpret_cast<int*>(smem + L.si);
  float* mbar = reinterpret_cast<float*>(smem + L.mb);  // PRESEL: metric adjoints, A's vertices then B's
  double* sK = reinterpret_cast<double*>(smem + L.sk);
  const bool safeguard = PRESEL && (prm.flags & CM_FLAG_SAFEGUARD);
  // Face masks for the window's E-E queries: each wave of E-E candidates
  // queries through the union of its candidates' group masks (the candidate
  // pass's, kept by cull in the scratch slot), for the pairs the engine's
  // union_masks() takes.  Witnesses lie on their edges, so not with
  // pre-selection (soft edges), tracing (moved points) or the extended
  // primitives.
  const bool use_masks_k = !PRESEL && !REFINE && !SQ;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = BLOCK / 64;
  const int K = prm.K;
  const Temp& T = P.T;
  const int n_pairs = min(*fwd.n_pairs, fwd.capacity);
  const long long CK = (long long)fwd.capacity * K;

  // pairs from a work queue (an atomic counter, zeroed by the launch) when
  // given, so workgroups that drew cheap pairs take more; else round-robin
  for (int it = 0;; ++it) {
    int pi = blockIdx.x + it * gridDim.x;
    if (queue) {
      if (tid == 0) ps.next = atomicAdd(queue, 1);
      __syncthreads();
      pi = ps.next;
    }
    if (pi >= n_pairs) break;
    if (!P.setup(fwd.pairs[pi], fwd.pairs[fwd.capacity + pi], err)) {
      __syncthreads();
      continue;
    }
    const BodyView& A = P.A;
    const BodyView& B = P.B;
    const bool use_masks = use_masks_k && P.union_masks();   // this pair's (uniform)
    FaceMask* const um = use_masks ? umask : nullptr;
    if (!SQ && (A.type >= CM_SQ_UNION || B.type >= CM_SQ_UNION)) {   // not built for these: flagged, skipped
      if (tid == 0) atomicOr(err, ERR_NO_ADJOINT);
      __syncthreads();
      continue;
    }
    // mesh counts (pre-selection shrinks A.nv ... to the selection sizes)
    const int nvA_m = A.nv, nvB_m = B.nv, nfA = A.nf, nfB = B.nf;
    for (int i = tid; i < 3 * maxV; i += BLOCK) { vA3[i] = 0.f; vB3[i] = 0.f; }
    if (PRESEL) {
      for (int i = tid; i < 2 * CM_MAX_PRESEL * 9; i += BLOCK) (i < 6 * CM_MAX_PRESEL ? svb[i] : seb[i - 6 * CM_MAX_PRESEL]) = 0.f;
      for (int i = tid; i < 2 * maxV; i += BLOCK) mbar[i] = 0.f;
    }
    for (int i = tid; i < 4 * maxF; i += BLOCK) { plA[i] = 0.f; plB[i] = 0.f; }
    for (int i = tid; i < maxE; i += BLOCK) { rbar[i] = 0.f; cbar[i] = 0.f; }
    if (tid < 8) prA[tid] = 0.f;
    // face-plane adjoints only feed the hull-vertex gradient: without it
    // they are not accumulated
    const bool want_planes = ga.gr.g_vertices != nullptr;
    const BodySink sinkA{(want_planes && A.type == CM_POLYTOPE) ? plA : nullptr, prA, maxF};
    const BodySink sinkB{(want_planes && B.type == CM_POLYTOPE) ? plB : nullptr, prB, maxF};

    // ------------------------------------------------ recompute the forward
    P.stage();
    if (PRESEL) P.select(selI);
    // candidate-space counts (the selection sizes under pre-selection)
    const int nvA = A.nv, neB = B.ne;
    const int steps = REFINE ? min(max(P.refine, 1), CM_MAX_REFINE) : 0;   // sphere-tracing steps
    // The forward's tape for this pair, when recorded whole: s_[k], the
    // SoftSort row sums and the candidates within the adjoint's window.  Then
    // only the distance pass is recomputed (the candidates' records need the
    // QP solutions and row / column LSE); otherwise the whole forward is.
    int ntape = -1;
    const int* tlist = nullptr;
    const unsigned long long* tmask = nullptr;
    const double* tdat = nullptr;
    if (tape.base) {
      const char* rec = tape.base + (long long)pi * tape_stride(K);
      const int c = reinterpret_cast<const int*>(rec)[0], form = reinterpret_cast<const int*>(rec)[1];
      const long long off = reinterpret_cast<const long long*>(rec)[1];
      const long long mask_n = 2LL * ((ps.ncand + 63) >> 6);
      if (c >= 0 && c <= ps.ncand && off >= 0) {
        if (form == 1 && off + c <= tape.pool_cap) {
          ntape = c;
          tlist = tape.pool + off;
        } else if (form == 2 && (off & 1) == 0 && off + mask_n <= tape.pool_cap) {
          tmask = reinterpret_cast<const unsigned long long*>(tape.pool + off);
        }
      }
      if (tlist || tmask) tdat = reinterpret_cast<const double*>(rec + 16);
    }
    if (tdat) {
      if (use_masks) P.cull();   // the group masks (and their scratch copy) for the window's queries
      P.pass1();
      for (int i = tid; i < 10 * K; i += BLOCK) {
        if (i < K) P.sTop[i] = tdat[i];
        else P.sAcc[i - K] = tdat[i];
      }
      __syncthreads();
    } else {
      P.cull();
      double tk[KMAX];
      P.scores(tk);
      P.topk(tk);
      P.softsort();
    }
    // A1 and A2 visit the window as three runs (vertex candidates, witnesses
    // 1, witnesses 2): a recorded list already is; a recorded mask, or the
    // scores just recomputed, are compacted once here and written in runs
    // over the stored scores, which nothing reads after this
    if (!tlist) {
      const int tot = P.window(kAdjointTaus, tmask);
      int* runs = reinterpret_cast<int*>(P.Sbuf);
      P.write_window_runs(tot, runs);
      tlist = runs;
      ntape = tot;
      tmask = nullptr;
    }

    // ------------------------------------------------ cotangents in the pair frame
    if (tid < K) {
      const int k = tid;
      const long long o = (long long)pi * K + k;
      const double* R = ps.RA;
      const D3 gP = ga.cot.gp ? d3(ga.cot.gp[o], ga.cot.gp[CK + o], ga.cot.gp[2 * CK + o]) : d3(0, 0, 0);
      const D3 gN = ga.cot.gn ? d3(ga.cot.gn[o], ga.cot.gn[CK + o], ga.cot.gn[2 * CK + o]) : d3(0, 0, 0);
      const D3 pb = rotT(R, gP), nb = rotT(R, gN);
      double* c = cotL + 8 * k;
      c[0] = pb.x; c[1] = pb.y; c[2] = pb.z; c[3] = nb.x; c[4] = nb.y; c[5] = nb.z;
      c[6] = ga.cot.gd ? double(ga.cot.gd[o]) : 0.0;
      c[7] = ga.cot.gw ? double(ga.cot.gw[o]) : 0.0;
      const double* a = P.sAcc + 9 * k;
      double* F = Fk + 10 * k;
      const double iz = a[0] > 0.0 ? 1.0 / a[0] : 0.0;   // empty row: no candidate
      double gbar = 0.0;
      for (int f = 0; f < 8; ++f) { F[f] = a[f + 1] * iz; gbar += c[f] * F[f]; }
      F[8] = a[0];
      F[9] = gbar;
    }
    __syncthreads();
    if (tid == 0) {
      // world twist of A from the output transform P_k = R_A p_k + t_A, N_k = R_A nu_k
      double r[3] = {0, 0, 0}, w[3] = {0, 0, 0};
      const double* R = ps.RA;
      for (int k = 0; k < K; ++k) {
        const long long o = (long long)pi * K + k;
        const double* F = Fk + 10 * k;
        if (!(F[8] > 0.0)) continue;   // empty row: a constant output
        const D3 Pw = add(rot(R, d3(F[0], F[1], F[2])), d3(ps.tA[0], ps.tA[1], ps.tA[2]));
        const D3 Nw = rot(R, d3(F[3], F[4], F[5]));
        const D3 gP = ga.cot.gp ? d3(ga.cot.gp[o], ga.cot.gp[CK + o], ga.cot.gp[2 * CK + o]) : d3(0, 0, 0);
        const D3 gN = ga.cot.gn ? d3(ga.cot.gn[o], ga.cot.gn[CK + o], ga.cot.gn[2 * CK + o]) : d3(0, 0, 0);
        const D3 c1 = cross(Pw, gP), c2 = cross(Nw, gN);
        r[0] += gP.x; r[1] += gP.y; r[2] += gP.z;
        w[0] += c1.x + c2.x; w[1] += c1.y + c2.y; w[2] += c1.z + c2.z;
      }
      for (int i = 0; i < 3; ++i) { twOut[i] = r[i]; twOut[3 + i] = w[i]; }
    }

    double taub = 0.0;
    Twist tw = {{0, 0, 0}, {0, 0, 0}};

    // ------------------------------------------------ A1: adjoints of s_[k]
    {
      const int kk = tid % K, nsl = BLOCK / K, sl = tid / K;
      const bool act = sl < nsl;
      double sbp = 0.0, best = INFINITY, bterm = 0.0;
      int bidx = 0x7fffffff;
      P.for_window(tlist, ntape, tmask, [&](int tot) {
        if (!act) return;
        const double* F = Fk + 10 * kk;
        const double* c = cotL + 8 * kk;
        const double sk = P.sTop[kk];
        for (int r = sl; r < tot; r += nsl) {
          const Rec& R = P.sRec[r];
          const double dl = sk - R.s;
          if (!(F[8] > 0.0)) continue;   // empty row
          const double G = double(expn(fabs(dl), T)) / F[8];
          const double fv[8] = {R.px, R.py, R.pz, R.nx, R.ny, R.nz, R.d, R.w};
          double gi = 0.0;
          for (int f = 0; f < 8; ++f) gi += c[f] * fv[f];
          const double ab = G * (gi - F[9]);
          const double sg = dl > 0.0 ? 1.0 : (dl < 0.0 ? -1.0 : 0.0);
          const double term = -ab * sg * T.inv_tau;
          sbp += term;
          taub += ab * fabs(dl) * T.inv_tau * T.inv_tau;
          if (fabs(dl) < best || (fabs(dl) == best && R.idx < bidx)) { best = fabs(dl); bidx = R.idx; bterm = term; }
        }
      }, kAdjointTaus, true, um);
      P.sRed[tid] = act ? sbp : 0.0;
      P.sRed[BLOCK + tid] = act ? best : INFINITY;
      bestI[CM_MAX_K + tid] = act ? bidx : 0x7fffffff;
      btl[tid] = act ? bterm : 0.0;
      __syncthreads();
      if (tid < K) {
        double s = 0.0, b = INFINITY, bt = 0.0;
        int bi = 0x7fffffff;
        for (int q = 0; q < nsl; ++q) {
          const int t = q * K + tid;
          s += P.sRed[t];
          const double v = P.sRed[BLOCK + t];
          const int vi = bestI[CM_MAX_K + t];
          if (v < b || (v == b && vi < bi)) { b = v; bi = vi; bt = btl[t]; }
        }
        // s_[k] is the score of the candidate attaining it, whose own term
        // |s_[k] - s_j| has derivative 0 there (|x|' = 0 at 0): left out here
        // and in A2, so both sides agree however its score is recomputed
        topb[tid] = s - bt;
        bestI[tid] = bi;
      }
      __syncthreads();
    }

    // endpoint adjoints of edge pair (k, l): to the mesh vertices, or to the
    // soft edges under pre-selection
    auto edge_adj = [&](int k, int l, const D3& va0, const D3& va1, const D3& vb0, const D3& vb1) __attribute__((always_inline)) {
      if (PRESEL) {
        float* a = seb + 6 * k;
        float* b = seb + 6 * (CM_MAX_PRESEL + l);
        atomicAdd(&a[0], float(va0.x)); atomicAdd(&a[1], float(va0.y)); atomicAdd(&a[2], float(va0.z));
        atomicAdd(&a[3], float(va1.x)); atomicAdd(&a[4], float(va1.y)); atomicAdd(&a[5], float(va1.z));
        atomicAdd(&b[0], float(vb0.x)); atomicAdd(&b[1], float(vb0.y)); atomicAdd(&b[2], float(vb0.z));
        atomicAdd(&b[3], float(vb1.x)); atomicAdd(&b[4], float(vb1.y)); atomicAdd(&b[5], float(vb1.z));
        return;
      }
      const int ia0 = tb.e0[P.GA->e_off + k], ia1 = tb.e1[P.GA->e_off + k];
      const int ib0 = tb.e0[P.GB->e_off + l], ib1 = tb.e1[P.GB->e_off + l];
      atomicAdd(&vA3[ia0], float(va0.x)); atomicAdd(&vA3[maxV + ia0], float(va0.y)); atomicAdd(&vA3[2 * maxV + ia0], float(va0.z));
      atomicAdd(&vA3[ia1], float(va1.x)); atomicAdd(&vA3[maxV + ia1], float(va1.y)); atomicAdd(&vA3[2 * maxV + ia1], float(va1.z));
      atomicAdd(&vB3[ib0], float(vb0.x)); atomicAdd(&vB3[maxV + ib0], float(vb0.y)); atomicAdd(&vB3[2 * maxV + ib0], float(vb0.z));
      atomicAdd(&vB3[ib1], float(vb1.x)); atomicAdd(&vB3[maxV + ib1], float(vb1.y)); atomicAdd(&vB3[2 * maxV + ib1], float(vb1.z));
    };

    // ------------------------------------------------ A2: per-candidate adjoints
    P.for_window(tlist, ntape, tmask, [&](int tot) {
      if (wave * 64 >= tot) return;        // whole wave idle (uniform)
      const bool live = tid < tot;
      // the candidate's record as A1 evaluated it (the same scores, so that
      // ties and the attaining candidates' signs agree with A1's)
      const Rec R = P.sRec[live ? tid : 0];
      double sb = 0.0;
      double fb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (live) {
        const double fv[8] = {R.px, R.py, R.pz, R.nx, R.ny, R.nz, R.d, R.w};
        for (int k = 0; k < K; ++k) {
          const double* F = Fk + 10 * k;
          const double* c = cotL + 8 * k;
          const double dl = P.sTop[k] - R.s;
          if (!(F[8] > 0.0)) continue;   // empty row
          const double G = double(expn(fabs(dl), T)) / F[8];
          double gi = 0.0;
          for (int f = 0; f < 8; ++f) { gi += c[f] * fv[f]; fb[f] += G * c[f]; }
          const double ab = G * (gi - F[9]);
          if (bestI[k] == R.idx) sb += topb[k];   // the attaining candidate: its own term is 0 (A1)
          else sb += ab * (dl > 0.0 ? 1.0 : (dl < 0.0 ? -1.0 : 0.0)) * T.inv_tau;
        }
      }
      const int idx = R.idx;
      const bool is_vs = idx < ps.nvs;
      // a wave of E-E candidates queries through the union masks the
      // records were evaluated with (for_window): slot 0 A's faces near e1,
      // 1 B's near e1, 2 A's near e2, 3 B's near e2 (wave-uniform)
      const bool masked = use_masks && __ballot(live && is_vs) == 0ull;
      const FaceMask* U = umask + 4 * wave;
      const FaceMask* U0 = masked ? U : nullptr;
      const FaceMask* U1 = masked ? U + 1 : nullptr;
      const FaceMask* U2 = masked ? U + 2 : nullptr;
      const FaceMask* U3 = masked ? U + 3 : nullptr;
      // ---- stage 1: forward values and the seeds of four SDF query slots
      // slot 0: A at X0 (gradient adjoint), slot 1: B at X1, slot 2: A at X2, slot 3: B at X3
      D3 X[4];
      double phib[4] = {0, 0, 0, 0};
      D3 gbar[4] = {d3(0, 0, 0), d3(0, 0, 0), d3(0, 0, 0), d3(0, 0, 0)};
      D3 a0, t1, b0, t2, de, pb = d3(fb[0], fb[1], fb[2]), nbb = d3(0, 0, 0);
      double al1 = 0, al2 = 0, dbar = 0, rho = 0, dbarb = 0, lcb = 0;
      int k = 0, l = 0, wit = 0;
      // REFINE: both witnesses' traces, the QP distance vector and its adjoint
      Trace trA, trB;
      D3 dqe = d3(0, 0, 0);
      double dqp = 0, dqpb = 0;
      if (is_vs) {
        const bool ofA = idx < nvA;
        const D3 x = PRESEL ? P.soft_vertex(idx)
                            : (ofA ? P.template vertex<true>(*P.GA, idx, A) : P.template vertex<false>(*P.GB, idx - nvA, B));
        const double sgn = ofA ? -1.0 : 1.0;
        double phi;
        D3 g;
        if (ofA) sdf_body<kFull, false, true, SQ>(B, x, T, phi, g);
        else sdf_body<kFull, true, true, SQ>(A, x, T, phi, g);
        const double in = rsq64(T.tau + dot(g, g));
        const double lw = lsig(-phi, T), w = exp(lw);
        const double dtot = fb[6] - sb, lwb = T.tau * sb + w * fb[7];
        taub += sb * lw;
        const D3 nub = d3(fb[3], fb[4], fb[5]);
        const double gn = dot(g, nub);
        const D3 gb = scl(sub(scl(nub, in), scl(g, gn * in * in * in)), sgn);
        taub -= sgn * gn * in * in * in * 0.5;
        double du, dt;
        lsig_d(-phi, T, du, dt);
        const double phb = dtot - lwb * du;
        taub += lwb * dt;
        for (int s = 0; s < 4; ++s) X[s] = x;
        const int s = ofA ? 1 : 0;
        phib[s] = phb;
        gbar[s] = gb;
        if (REFINE) { trace_none(x, trA); trace_none(x, trB); }
      } else {
        const int e = idx - ps.nvs;
        const int ee_i = e >> 1;
        wit = e & 1;
        k = ee_i / neB; l = ee_i - k * neB;
        P.EA.get(k, a0, t1);
        P.EB.get(l, b0, t2);
        // the QP solution the distance pass stored for this edge pair
        const EEQP q = ee_from_alpha(a0, t1, b0, t2, P.Al1[ee_i], P.Al2[ee_i], P.Lcon[ee_i]);
        al1 = q.al1; al2 = q.al2; de = q.de;
        D3 e1 = axpy(al1, t1, a0), e2 = axpy(al2, t2, b0);
        if (REFINE) {   // each witness traced onto its own body
          dqe = q.de;
          dqp = sqrt(dot(q.de, q.de));
          e1 = trace_fwd<true, SQ>(A, e1, T, steps, trA);
          e2 = trace_fwd<false, SQ>(B, e2, T, steps, trB);
          de = sub(e1, e2);
        }
        const double dsq = dot(de, de);
        double idum;
        sqrt_rsq64(dsq, dbar, idum);
        const double dnn = REFINE ? dqp : dbar;   // the nearest-neighbour term's distance
        rho = rsq64(dsq + P.eps_n);
        const D3 nb = scl(de, rho);
        double phiB1, phiA2, dum, phiA1 = 0.0, phiB2 = 0.0;
        D3 gA, gB, dg;
        sdf_body<kValue, false, false, SQ>(B, e1, T, phiB1, dg, U1);
        sdf_body<kValue, true, false, SQ>(A, e2, T, phiA2, dg, U2);
        if (PRESEL || REFINE) {   // soft edges / traced points need not lie on the edges: full queries
          sdf_body<kFull, true, false, SQ>(A, e1, T, phiA1, gA);
          sdf_body<kFull, false, false, SQ>(B, e2, T, phiB2, gB);
        } else {
          sdf_body<kSurfGrad, true, false, SQ>(A, e1, T, dum, gA, U0);
          sdf_body<kSurfGrad, false, false, SQ>(B, e2, T, dum, gB, U3);
        }
        const double u1 = dot(gB, nb), u2 = -dot(gA, nb), ucl = -dot(gA, gB);
        const double gam1 = tanh64(u1, T), gam2 = tanh64(u2, T);
        const double gam = wit ? gam2 : gam1;
        const double lcl = lsig(ucl, T);
        const double lp = wit ? lsig(-phiA2, T) : lsig(-phiB1, T);
        const double lse = wit ? P.sCol[l] : P.sRow[k];
        const double lsg = safeguard ? lsig(-phiA1, T) + lsig(-phiB2, T) : 0.0;
        const double lw = q.log_con + lcl + lp + lsg + (lse - dnn) * T.inv_tau;
        const double w = exp(lw);
        const double dtot = fb[6] - sb, lwb = T.tau * sb + w * fb[7];
        taub += sb * lw;
        const D3 nub = d3(fb[3], fb[4], fb[5]);
        const double gamb = dtot * dbar - dot(nub, nb);   // d = gam dbar, nu = -gam n_bar
        dbarb = dtot * gam;
        nbb = scl(nub, -gam);
        lcb = lwb;
        double du, dt;
        lsig_d(ucl, T, du, dt);
        const double uclb = lwb * du;
        taub += lwb * dt;
        D3 gAb = scl(gB, -uclb), gBb = scl(gA, -uclb);
        lsig_d(wit ? -phiA2 : -phiB1, T, du, dt);
        const double phb = -lwb * du;
        taub += lwb * dt;
        if (safeguard) {   // inside indicators of the soft witnesses on their own bodies
          lsig_d(-phiA1, T, du, dt);
          phib[0] = -lwb * du;
          taub += lwb * dt;
          lsig_d(-phiB2, T, du, dt);
          phib[3] = -lwb * du;
          taub += lwb * dt;
        }
        if (live) atomicAdd(wit ? &cbar[l] : &rbar[k], float(lwb * T.inv_tau));
        (REFINE ? dqpb : dbarb) -= lwb * T.inv_tau;
        taub -= lwb * (lse - dnn) * T.inv_tau * T.inv_tau;
        if (!wit) {
          const double ub = gamb * (1.0 - gam1 * gam1) * T.inv_tau;
          taub -= ub * u1 * T.inv_tau;
          gBb = axpy(ub, nb, gBb);
          nbb = axpy(ub, gB, nbb);
        } else {
          const double ub = gamb * (1.0 - gam2 * gam2) * T.inv_tau;
          taub -= ub * u2 * T.inv_tau;
          gAb = axpy(-ub, nb, gAb);
          nbb = axpy(-ub, gA, nbb);
        }
        X[0] = e1; X[1] = e1; X[2] = e2; X[3] = e2;
        gbar[0] = gAb;
        if (!wit) phib[1] = phb; else phib[2] = phb;
        gbar[3] = gBb;
      }
      // ---- stage 2: SDF adjoints, every lane of the wave together
      // (a V-S slot's gradient adjoint refers to the V-S normal direction);
      // a slot whose adjoints are zero on every lane of the wave contributes
      // nothing and is skipped (a wave-uniform test)
      auto used = [](double ph, const D3& g) {
        return __ballot(ph != 0.0 || g.x != 0.0 || g.y != 0.0 || g.z != 0.0) != 0ull;
      };
      const D3 zero = d3(0, 0, 0);
      // slots 0 and 3 of E-E candidates query a witness on its own body's
      // edge (not so for soft pre-selected edges or traced points)
      const bool surf = !PRESEL && !REFINE && __ballot(live && is_vs) == 0ull;
      const D3 xb0 = used(phib[0], gbar[0]) ? sdf_body_bwd<true, true, SQ>(A, X[0], phib[0], gbar[0], T, sinkA, taub, tw, is_vs, surf, U0) : zero;
      const D3 xb1 = used(phib[1], gbar[1]) ? sdf_body_bwd<true, false, SQ>(B, X[1], phib[1], gbar[1], T, sinkB, taub, tw, is_vs, false, U1) : zero;
      const D3 xb2 = used(phib[2], gbar[2]) ? sdf_body_bwd<true, true, SQ>(A, X[2], phib[2], gbar[2], T, sinkA, taub, tw, false, false, U2) : zero;
      const D3 xb3 = used(phib[3], gbar[3]) ? sdf_body_bwd<true, false, SQ>(B, X[3], phib[3], gbar[3], T, sinkB, taub, tw, false, surf, U3) : zero;
      // E-E: adjoints of the two witness points (zero on idle lanes, whose
      // seeds are all zero)
      D3 e1b = zero, e2b = zero;
      if (!is_vs) {
        const double dn = dot(de, nbb);
        D3 deb = sub(scl(nbb, rho), scl(de, rho * rho * rho * dn));
        if (prm.eps_tied && live) taub += -0.5 * rho * rho * rho * dn * 2.0 * T.tau;
        if (dbar > 0.0) deb = axpy(dbarb / dbar, de, deb);
        e1b = add(add(xb0, xb1), deb);
        e2b = sub(add(xb2, xb3), deb);
        if (!wit) e1b = add(e1b, pb); else e2b = add(e2b, pb);
      }
      // ---- stage 2b (REFINE): back through both traces to the QP witnesses,
      // every lane of the wave together (V-S and idle lanes carry zero)
      if (REFINE && __ballot(!is_vs) != 0ull) {
        e1b = trace_bwd<true, SQ>(A, trA, e1b, T, steps, sinkA, taub, tw);
        e2b = trace_bwd<false, SQ>(B, trB, e2b, T, steps, sinkB, taub, tw);
        if (dqp > 0.0) {   // the nearest-neighbour term's QP distance
          const D3 dq = scl(dqe, dqpb / dqp);
          e1b = add(e1b, dq);
          e2b = sub(e2b, dq);
        }
      }
      if (!live) return;
      // ---- stage 3: back to vertices / edges
      if (is_vs) {
        const bool ofA = idx < nvA;
        const D3 xb = add(pb, ofA ? xb1 : xb0);
        const int i = ofA ? idx : idx - nvA;
        if (PRESEL) {
          float* V = svb + 3 * ((ofA ? 0 : CM_MAX_PRESEL) + i);
          atomicAdd(&V[0], float(xb.x)); atomicAdd(&V[1], float(xb.y)); atomicAdd(&V[2], float(xb.z));
        } else {
          float* V = ofA ? vA3 : vB3;
          atomicAdd(&V[i], float(xb.x));
          atomicAdd(&V[maxV + i], float(xb.y));
          atomicAdd(&V[2 * maxV + i], float(xb.z));
        }
      } else {
        // e1b / e2b: adjoints of the QP witnesses a0 + al1 t1, b0 + al2 t2
        D3 a0b = e1b, t1b = scl(e1b, al1), b0b = e2b, t2b = scl(e2b, al2);
        ee_qp_bwd(a0, t1, b0, t2, P.lam, T, dot(e1b, t1), dot(e2b, t2), lcb, a0b, t1b, b0b, t2b, taub);
        edge_adj(k, l, sub(a0b, t1b), t1b, sub(b0b, t2b), t2b);
      }
    }, kAdjointTaus, true, um);
    __syncthreads();

    // ------------------------------------------------ N: nearest-neighbour LSE adjoint
    {
      const int nee = ps.nee;
      for (int idx = tid; idx < nee; idx += BLOCK) {
        const int k = idx / neB, l = idx - k * neB;
        const double rb = rbar[k], cb = cbar[l];
        if (rb == 0.0 && cb == 0.0) continue;
        // the row / column softmax weights from the stored distance; an
        // entry whose weights are both below e^-28 (7e-13) is skipped before
        // any QP work
        const double D = P.Dbuf[idx];
        const double zr = (P.sRow[k] - D) * T.inv_tau, zc = (P.sCol[l] - D) * T.inv_tau;
        const bool sr = rb != 0.0 && zr > -28.0, sc = cb != 0.0 && zc > -28.0;
        if (!sr && !sc) continue;
        const double pr = sr ? exp64n(zr) : 0.0, pc = sc ? exp64n(zc) : 0.0;
        const double Db = rb * pr + cb * pc;
        taub += (rb * pr * (P.sRow[k] - D) + cb * pc * (P.sCol[l] - D)) * T.inv_tau;
        if (Db == 0.0 || !(D > 0.0)) continue;
        D3 a0, t1, b0, t2;
        P.EA.get(k, a0, t1);
        P.EB.get(l, b0, t2);
        const EEQP q = ee_from_alpha(a0, t1, b0, t2, P.Al1[idx], P.Al2[idx], P.Lcon[idx]);
        const D3 deb = scl(q.de, Db / D);
        D3 a0b = deb, t1b = scl(deb, q.al1), b0b = scl(deb, -1.0), t2b = scl(deb, -q.al2);
        ee_qp_bwd(a0, t1, b0, t2, P.lam, T, dot(deb, t1), -dot(deb, t2), 0.0, a0b, t1b, b0b, t2b, taub);
        edge_adj(k, l, sub(a0b, t1b), t1b, sub(b0b, t2b), t2b);
      }
    }
    __syncthreads();

    // ------------------------------------------------ S: selection adjoint
    // Soft item k of a set is sum_i (w_ki / S_k) p_i with w_ki =
    // exp(-|x_[k] - x_i| / tau), x_i = -metric_i, S_k = sum_i w_ki, and
    // x_[k] = x_{j_k} for the item j_k the hard top-K picked.  With g_k the
    // item's adjoint and c_ki = (w_ki / S_k) g_k . (p_i - soft_k):
    //   p_i      += (w_ki / S_k) g_k
    //   x_i      += c_ki sign(x_[k] - x_i) / tau
    //   x_{j_k}  -= sum_i c_ki sign(x_[k] - x_i) / tau
    //   tau      += c_ki |x_[k] - x_i| / tau^2
    // and metric_bar = -x_bar; an edge's metric is the mean of its corners'.
    if (PRESEL) {
      const int Kva = P.A.nv, Kvb = P.B.nv, Kea = P.A.ne, Keb = P.B.ne;
      const int neA_m = P.GA->ne, neB_m = P.GB->ne;
      const double* mVA = P.sMet;
      const double* mEA = P.sMet + 2 * maxV;
      // sets: 0 A's vertices, 1 B's, 2 A's edges, 3 B's (selects, not arrays:
      // a runtime index into a private array would live in scratch memory)
      auto nsel = [&](int set) __attribute__((always_inline)) { return set == 0 ? Kva : set == 1 ? Kvb : set == 2 ? Kea : Keb; };
      auto nall = [&](int set) __attribute__((always_inline)) { return set == 0 ? nvA_m : set == 1 ? nvB_m : set == 2 ? neA_m : neB_m; };
      // position of element i of a set: a vertex (c[3..5] = 0) or an edge's
      // two corners (values, not array references: a referenced array stays
      // in scratch memory)
      auto pos = [&](int set, int i) __attribute__((always_inline)) -> Six {
        Six p;
        int c0 = i, c1 = -1;
        if (set >= 2) {
          const GeomRec& G = set == 2 ? *P.GA : *P.GB;
          c0 = tb.e0[G.e_off + i];
          c1 = tb.e1[G.e_off + i];
        }
        const bool onA = (set & 1) == 0;
        const D3 v0 = onA ? P.template vertex<true>(*P.GA, c0, A) : P.template vertex<false>(*P.GB, c0, B);
        D3 v1 = d3(0, 0, 0);
        if (c1 >= 0) v1 = onA ? P.template vertex<true>(*P.GA, c1, A) : P.template vertex<false>(*P.GB, c1, B);
        p.c[0] = v0.x; p.c[1] = v0.y; p.c[2] = v0.z; p.c[3] = v1.x; p.c[4] = v1.y; p.c[5] = v1.z;
        return p;
      };
      auto metric = [&](int set, int i) __attribute__((always_inline)) { return set < 2 ? mVA[set * maxV + i] : mEA[(set - 2) * maxE + i]; };
      // adjoint (g) or value (!g) of soft item k (a vertex: entries 3..5 are 0)
      auto item = [&](int set, int k, bool adj) __attribute__((always_inline)) -> Six {
        Six r;
        const bool vert = set < 2;
        const float* ga = vert ? svb + 3 * (set * CM_MAX_PRESEL + k) : seb + 6 * ((set - 2) * CM_MAX_PRESEL + k);
        const double* sv = vert ? P.sSoft + 3 * (set * CM_MAX_PRESEL + k)
                                : P.sSoft + 2 * CM_MAX_PRESEL * 3 + 6 * ((set - 2) * CM_MAX_PRESEL + k);
#pragma unroll
        for (int c = 0; c < 6; ++c) r.c[c] = (c < 3 || !vert) ? (adj ? double(ga[c]) : sv[c]) : 0.0;
        return r;
      };
      // metric adjoint of element i of a set onto the vertex metrics
      auto add_metric = [&](int set, int i, double xb) __attribute__((always_inline)) {
        if (set < 2) {
          atomicAdd(&mbar[set * maxV + i], float(-xb));
        } else {
          const GeomRec& G = set == 2 ? *P.GA : *P.GB;
          float* mb = mbar + (set - 2) * maxV;
          atomicAdd(&mb[tb.e0[G.e_off + i]], float(-0.5 * xb));
          atomicAdd(&mb[tb.e1[G.e_off + i]], float(-0.5 * xb));
        }
      };
      // S1: one thread per soft item: S_k, g_k . soft_k, and the x_[k] / tau terms
      if (tid < Kva + Kvb + Kea + Keb) {
        int set = 0, k = tid;
        if (k >= Kva) { k -= Kva; set = 1;
          if (k >= Kvb) { k -= Kvb; set = 2;
            if (k >= Kea) { k -= Kea; set = 3; } } }
        const int D = nall(set);
        const double xk = P.sSel[set * CM_MAX_PRESEL + k];
        const Six g = item(set, k, true), sv = item(set, k, false);
        double Sk = 0.0, gs = 0.0;
        for (int i = 0; i < D; ++i) Sk += exp64n(-fabs(xk + metric(set, i)) * T.inv_tau);
#pragma unroll
        for (int c = 0; c < 6; ++c) gs = fma(g.c[c], sv.c[c], gs);
        const double iS = 1.0 / Sk;
        double xkb = 0.0, tb_ = 0.0;
        for (int i = 0; i < D; ++i) {
          const double dl = xk + metric(set, i);
          const double wn = exp64n(-fabs(dl) * T.inv_tau) * iS;
          const Six p = pos(set, i);
          double gp = 0.0;
#pragma unroll
          for (int c = 0; c < 6; ++c) gp = fma(g.c[c], p.c[c], gp);
          const double cki = wn * (gp - gs);
          xkb -= cki * (dl > 0.0 ? 1.0 : (dl < 0.0 ? -1.0 : 0.0)) * T.inv_tau;
          tb_ += cki * fabs(dl) * T.inv_tau * T.inv_tau;
        }
        taub += tb_;
        sK[set * CM_MAX_PRESEL + k] = iS;
        sK[4 * CM_MAX_PRESEL + set * CM_MAX_PRESEL + k] = gs;
        add_metric(set, selI[set * CM_MAX_PRESEL + k], xkb);
      }
      __syncthreads();
      // S2: one thread per set element: position and x_i adjoints
      const int nElem = nvA_m + nvB_m + neA_m + neB_m;
      for (int t = tid; t < nElem; t += BLOCK) {
        int set = 0, i = t;
        if (i >= nvA_m) { i -= nvA_m; set = 1;
          if (i >= nvB_m) { i -= nvB_m; set = 2;
            if (i >= neA_m) { i -= neA_m; set = 3; } } }
        const int Ks = nsel(set);
        const double xi = -metric(set, i);
        const Six p = pos(set, i);
        double pb[6] = {0, 0, 0, 0, 0, 0}, xib = 0.0;
        for (int k = 0; k < Ks; ++k) {
          const double dl = P.sSel[set * CM_MAX_PRESEL + k] - xi;
          const double wn = exp64n(-fabs(dl) * T.inv_tau) * sK[set * CM_MAX_PRESEL + k];
          const Six g = item(set, k, true);
          double gp = 0.0;
#pragma unroll
          for (int c = 0; c < 6; ++c) { gp = fma(g.c[c], p.c[c], gp); pb[c] = fma(wn, g.c[c], pb[c]); }
          const double cki = wn * (gp - sK[4 * CM_MAX_PRESEL + set * CM_MAX_PRESEL + k]);
          xib += cki * (dl > 0.0 ? 1.0 : (dl < 0.0 ? -1.0 : 0.0)) * T.inv_tau;
        }
        add_metric(set, i, xib);
        const bool onA = (set & 1) == 0;
        float* V = onA ? vA3 : vB3;
        int c0 = i, c1 = -1;
        if (set >= 2) {
          const GeomRec& G = onA ? *P.GA : *P.GB;
          c0 = tb.e0[G.e_off + i];
          c1 = tb.e1[G.e_off + i];
        }
        atomicAdd(&V[c0], float(pb[0])); atomicAdd(&V[maxV + c0], float(pb[1])); atomicAdd(&V[2 * maxV + c0], float(pb[2]));
        if (c1 >= 0) {
          atomicAdd(&V[c1], float(pb[3])); atomicAdd(&V[maxV + c1], float(pb[4])); atomicAdd(&V[2 * maxV + c1], float(pb[5]));
        }
      }
      __syncthreads();
      // S3: the metrics are SDF queries of the other body at every mesh
      // vertex; whole waves per block of 64 vertices (the plane adjoints are
      // summed across the wave)
      for (int base = wave * 64; base < nvA_m; base += BLOCK) {
        const int v = base + lane;
        const bool live = v < nvA_m;
        const D3 x = P.template vertex<true>(*P.GA, live ? v : 0, A);
        const D3 xb = sdf_body_bwd<true, false, SQ>(B, x, live ? double(mbar[v]) : 0.0, d3(0, 0, 0), T, sinkB, taub, tw);
        if (live) { atomicAdd(&vA3[v], float(xb.x)); atomicAdd(&vA3[maxV + v], float(xb.y)); atomicAdd(&vA3[2 * maxV + v], float(xb.z)); }
      }
      for (int base = wave * 64; base < nvB_m; base += BLOCK) {
        const int v = base + lane;
        const bool live = v < nvB_m;
        const D3 x = P.template vertex<false>(*P.GB, live ? v : 0, B);
        const D3 xb = sdf_body_bwd<true, true, SQ>(A, x, live ? double(mbar[maxV + v]) : 0.0, d3(0, 0, 0), T, sinkA, taub, tw);
        if (live) { atomicAdd(&vB3[v], float(xb.x)); atomicAdd(&vB3[maxV + v], float(xb.y)); atomicAdd(&vB3[2 * maxV + v], float(xb.z)); }
      }
      __syncthreads();
    }

    // ------------------------------------------------ G: geometry and pose gradients
    // face planes -> hull vertices (body frames)
    for (int i = tid; want_planes && i < nfA + nfB; i += BLOCK) {
      const bool isA = i < nfA;
      const int f = isA ? i : i - nfA;
      const GeomRec& G = isA ? *P.GA : *P.GB;
      if (G.type != CM_POLYTOPE) continue;   // superquadric records are not face planes
      const float* pl = isA ? plA : plB;
      const int iv[3] = {tb.f0[G.f_off + f], tb.f1[G.f_off + f], tb.f2[G.f_off + f]};
      D3 v[3];
      for (int j = 0; j < 3; ++j) v[j] = d3(tb.vx[G.v_off + iv[j]], tb.vy[G.v_off + iv[j]], tb.vz[G.v_off + iv[j]]);
      const D3 ea = sub(v[1], v[0]), eb = sub(v[2], v[0]);
      const D3 u = cross(ea, eb);
      const double iu = 1.0 / sqrt(dot(u, u));
      const D3 n = scl(u, iu);
      const double ob = pl[3 * maxF + f];
      const D3 nb = add(d3(pl[f], pl[maxF + f], pl[2 * maxF + f]), scl(v[0], ob));
      const D3 ub = scl(sub(nb, scl(n, dot(n, nb))), iu);
      const D3 eab = cross(eb, ub), ebb = cross(ub, ea);
      const D3 g0 = sub(scl(n, ob), add(eab, ebb));
      const D3 gv[3] = {g0, eab, ebb};
      if (ga.gr.g_vertices) {
        for (int j = 0; j < 3; ++j) {
          const long long o = G.v_off + iv[j];
          atomicAdd(&ga.gr.g_vertices[o], float(gv[j].x));
          atomicAdd(&ga.gr.g_vertices[ga.gr.pool + o], float(gv[j].y));
          atomicAdd(&ga.gr.g_vertices[2LL * ga.gr.pool + o], float(gv[j].z));
        }
      }
    }
    // mesh vertices -> hull vertices / analytic parameters, and B's placement twist
    for (int i = tid; i < nvA_m + nvB_m; i += BLOCK) {
      const bool isA = i < nvA_m;
      const int v = isA ? i : i - nvA_m;
      const GeomRec& G = isA ? *P.GA : *P.GB;
      const float* V = isA ? vA3 : vB3;
      D3 gb = d3(V[v], V[maxV + v], V[2 * maxV + v]);   // pair frame
      const D3 lv = d3(tb.vx[G.v_off + v], tb.vy[G.v_off + v], tb.vz[G.v_off + v]);
      if (!isA) {
        const D3 x = P.template vertex<false>(G, v, B);
        const D3 c = cross(x, gb);
        tw.r[0] += gb.x; tw.r[1] += gb.y; tw.r[2] += gb.z;
        tw.w[0] += c.x; tw.w[1] += c.y; tw.w[2] += c.z;
        gb = rotT(B.R, gb);
      }
      if (G.type == CM_POLYTOPE) {
        if (ga.gr.g_vertices) {
          const long long o = G.v_off + v;
          atomicAdd(&ga.gr.g_vertices[o], float(gb.x));
          atomicAdd(&ga.gr.g_vertices[ga.gr.pool + o], float(gb.y));
          atomicAdd(&ga.gr.g_vertices[2LL * ga.gr.pool + o], float(gb.z));
        }
      } else if (G.type < CM_SQ_UNION) {   // no record gradient for superquadric unions / point clouds
        float* pr = isA ? prA : prB;
        if (G.type == CM_SPHERE) {
          atomicAdd(&pr[0], float(dot(lv, gb) / double(G.p[0])));
        } else if (G.type == CM_CAPSULE) {
          const double s = v < 17 ? -1.0 : 1.0;
          const D3 u = scl(d3(lv.x, lv.y, lv.z - s * double(G.p[1])), 1.0 / double(G.p[0]));
          atomicAdd(&pr[0], float(dot(u, gb)));
          atomicAdd(&pr[1], float(s * gb.z));
        } else {
          atomicAdd(&pr[0], float((v & 1 ? 1.0 : -1.0) * gb.x));
          atomicAdd(&pr[1], float((v & 2 ? 1.0 : -1.0) * gb.y));
          atomicAdd(&pr[2], float((v & 4 ? 1.0 : -1.0) * gb.z));
        }
      }
    }
    // block reduction of tau_bar and B's twist
    {
      double vals[7] = {taub, tw.r[0], tw.r[1], tw.r[2], tw.w[0], tw.w[1], tw.w[2]};
      for (int j = 0; j < 7; ++j) {
        double v = vals[j];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        vals[j] = v;
      }
      __syncthreads();
      if (lane == 0)
        for (int j = 0; j < 7; ++j) P.sRed[j * NW + wave] = vals[j];
      __syncthreads();
      if (tid == 0) {
        double s[7];
        for (int j = 0; j < 7; ++j) {
          s[j] = 0.0;
          for (int w = 0; w < NW; ++w) s[j] += P.sRed[j * NW + w];
        }
        if (ga.gr.g_tau) atomicAdd(ga.gr.g_tau, float(s[0]));
        // eta (pair frame, B relative to A) -> world twists
        const double* R = ps.RA;
        const D3 rB = rot(R, d3(s[1], s[2], s[3]));
        const D3 wB = add(rot(R, d3(s[4], s[5], s[6])), cross(d3(ps.tA[0], ps.tA[1], ps.tA[2]), rB));
        if (ga.gr.g_pose) {
          const int a = ps.a, b = ps.b, nb = bt.n_bodies;
          const double gb6[6] = {rB.x, rB.y, rB.z, wB.x, wB.y, wB.z};
          for (int c = 0; c < 6; ++c) {
            atomicAdd(&ga.gr.g_pose[c * nb + b], float(gb6[c]));
            atomicAdd(&ga.gr.g_pose[c * nb + a], float(twOut[c] - gb6[c]));
          }
        }
      }
    }
    __syncthreads();
    if (ga.gr.g_params && tid < 8) {
      const bool isA = tid < 4;
      const GeomRec& G = isA ? *P.GA : *P.GB;
      const int gid = isA ? ps.ga : ps.gb;
      if (G.type < CM_POLYTOPE)
        atomicAdd(&ga.gr.g_params[(tid & 3) * (long long)tb.n_geoms + gid], prA[tid]);
    }
    __syncthreads();
  }
}

int bwd_lds_bytes(int maxV, int maxE, int maxF, int block, bool presel, bool edges_out) {
  const int extra = bwd_extra_bytes(maxV, maxE, maxF, block, presel);
  const int pre = presel ? presel_lds_bytes(maxV, maxE) : 0;
  return bwd_layout(lds_layout(maxE, maxF, block, extra, edges_out).bytes + pre, maxV, maxE, maxF, block, presel).bytes;
}

template <int BLOCK, int KMAX, bool PRESEL, bool SQ, bool REFINE = false, int WAVES = 0>
static hipError_t launch_bwd_t(const BwdLaunch& b, hipStream_t st) {
  const int lds = bwd_lds_bytes(b.f.maxV, b.f.maxE, b.f.maxF, BLOCK, PRESEL, b.f.edges_out != 0);
  BwdArgs ga{b.cot, b.gr};
  hipLaunchKernelGGL((collide_bwd<BLOCK, KMAX, PRESEL, SQ, REFINE, WAVES>), dim3(b.f.grid), dim3(BLOCK), lds, st, b.f.tb,
                     b.f.bt, b.f.prm, b.f.out, ga, b.f.scratch, b.f.scratch_stride, b.f.maxV, b.f.maxE, b.f.maxF,
                     b.f.err, b.f.tape, b.f.queue, b.f.edges_out);
  return hipGetLastError();
}

template <int BLOCK, int KMAX, bool PRESEL, bool SQ, bool REFINE = false, int WAVES = 0>
static int bwd_occ_t(const BwdLaunch& b) {
  int nb = 0;
  const int lds = bwd_lds_bytes(b.f.maxV, b.f.maxE, b.f.maxF, BLOCK, PRESEL, b.f.edges_out != 0);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, collide_bwd<BLOCK, KMAX, PRESEL, SQ, REFINE, WAVES>, BLOCK,
                                                   lds) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <bool PRESEL, bool SQ>
static hipError_t launch_bwd_k(const BwdLaunch& b, hipStream_t st) {
  if (!PRESEL && !SQ && b.f.hi_occ) {   // the 3-wave variant (K <= 16)
    if (b.f.kmax == 8) return launch_bwd_t<256, 8, false, false, false, 3>(b, st);
    if (b.f.kmax == 16) return launch_bwd_t<256, 16, false, false, false, 3>(b, st);
  }
  if (b.f.kmax == 8) return launch_bwd_t<256, 8, PRESEL, SQ>(b, st);
  if (b.f.kmax == 16) return launch_bwd_t<256, 16, PRESEL, SQ>(b, st);
  return launch_bwd_t<256, 32, PRESEL, SQ>(b, st);
}

template <bool PRESEL, bool SQ>
static int bwd_occ_k(const BwdLaunch& b) {
  if (!PRESEL && !SQ && b.f.hi_occ) {
    if (b.f.kmax == 8) return bwd_occ_t<256, 8, false, false, false, 3>(b);
    if (b.f.kmax == 16) return bwd_occ_t<256, 16, false, false, false, 3>(b);
  }
  if (b.f.kmax == 8) return bwd_occ_t<256, 8, PRESEL, SQ>(b);
  if (b.f.kmax == 16) return bwd_occ_t<256, 16, PRESEL, SQ>(b);
  return bwd_occ_t<256, 32, PRESEL, SQ>(b);
}

// Sphere-traced witnesses (K <= 16, as in the forward).
template <bool PRESEL, bool SQ>
static hipError_t launch_bwd_refine(const BwdLaunch& b, hipStream_t st) {
  if (b.f.kmax == 8) return launch_bwd_t<256, 8, PRESEL, SQ, true>(b, st);
  return launch_bwd_t<256, 16, PRESEL, SQ, true>(b, st);
}

template <bool PRESEL, bool SQ>
static int bwd_occ_refine(const BwdLaunch& b) {
  if (b.f.kmax == 8) return bwd_occ_t<256, 8, PRESEL, SQ, true>(b);
  return bwd_occ_t<256, 16, PRESEL, SQ, true>(b);
}

// Pre-selection and contexts that hold superquadric unions run in their own
// instantiations (the selection tracks taken items in a 64-bit mask per
// lane: <= 4096 per set).
hipError_t launch_collide_bwd(const BwdLaunch& b, hipStream_t st) {
  const bool ps = b.f.prm.presel_v > 0, sq = b.f.prm.sq != 0;
  if (b.f.block == 512) {   // the full method on the basic primitives only
    if (ps || sq || b.f.prm.refine > 0) return hipErrorInvalidValue;
    if (b.f.kmax == 8) return launch_bwd_t<512, 8, false, false>(b, st);
    if (b.f.kmax == 16) return launch_bwd_t<512, 16, false, false>(b, st);
    return launch_bwd_t<512, 32, false, false>(b, st);
  }
  if ((ps || sq || b.f.prm.refine > 0) && (b.f.maxV > 4096 || b.f.maxE > 4096)) return hipErrorInvalidValue;
  if (b.f.prm.refine > 0) {
    if (b.f.kmax > 16) return hipErrorInvalidValue;
    if (sq) return ps ? launch_bwd_refine<true, true>(b, st) : launch_bwd_refine<false, true>(b, st);
    return ps ? launch_bwd_refine<true, false>(b, st) : launch_bwd_refine<false, false>(b, st);
  }
  if (sq) return ps ? launch_bwd_k<true, true>(b, st) : launch_bwd_k<false, true>(b, st);
  return ps ? launch_bwd_k<true, false>(b, st) : launch_bwd_k<false, false>(b, st);
}

int bwd_place(BwdLaunch& b) {
  b.f.hi_occ = 0;
  b.f.edges_out = 0;
  const int base = bwd_occupancy(b);
  // the full method at K <= 16 in 256-thread blocks: the edge arrays in the
  // scratch slot and the 3-wave register budget, where that fits more
  // workgroups per CU
  if (b.f.block == 256 && b.f.kmax <= 16 && b.f.prm.presel_v == 0 && !b.f.prm.sq && b.f.prm.refine == 0) {
    b.f.hi_occ = 1;
    b.f.edges_out = 1;
    const int hi = bwd_occupancy(b);
    if (hi > base) return hi;
    b.f.hi_occ = 0;
    b.f.edges_out = 0;
  }
  return base;
}

int bwd_occupancy(const BwdLaunch& b) {
  const bool ps = b.f.prm.presel_v > 0, sq = b.f.prm.sq != 0;
  if (b.f.block == 512) {
    if (ps || sq || b.f.prm.refine > 0) return 1;
    if (b.f.kmax == 8) return bwd_occ_t<512, 8, false, false>(b);
    if (b.f.kmax == 16) return bwd_occ_t<512, 16, false, false>(b);
    return bwd_occ_t<512, 32, false, false>(b);
  }
  if (b.f.prm.refine > 0) {
    if (sq) return ps ? bwd_occ_refine<true, true>(b) : bwd_occ_refine<false, true>(b);
    return ps ? bwd_occ_refine<true, false>(b) : bwd_occ_refine<false, false>(b);
  }
  if (sq) return ps ? bwd_occ_k<true, true>(b) : bwd_occ_k<false, true>(b);
  return ps ? bwd_occ_k<true, false>(b) : bwd_occ_k<false, false>(b);
}

}  // namespace cm
