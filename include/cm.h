/*
 * cm.h -- C ABI of the MI355X (gfx950) contact-manifold library.
 *
 * Computes, for every colliding pair of rigid bodies in a batch of scenes, the
 * smooth contact manifold of "Smoothly Differentiable and Efficiently
 * Vectorizable Contact Manifold Generation" (arXiv 2602.20304):
 *   - vertex-SDF contacts, both ways (Sec. IV-C; SDF primitives Sec. IV-B),
 *   - edge-edge contacts for all edge pairs: smoothed analytic active-set
 *     witness QP with L2 regularisation, soft sign, penetration,
 *     nearest-neighbour, clashing and activity indicators (Sec. IV-D),
 *   - a fixed-size manifold of K contacts per pair, obtained by SoftSort
 *     (Sec. III, soft top-K) over all candidates with scores
 *     s = -d + tau * log(w).
 * Inputs: geometries, poses and the smoothing factor tau (problem statement,
 * Sec. IV-A).  Outputs per kept pair: K contact points, pair normals (from
 * body A towards body B), signed distances and activity weights.
 *
 * Conventions
 *   - Every function returns cm_status (CM_OK = 0, negative = error).  No C++
 *     exception crosses the ABI.  cm_last_error() gives a message for the last
 *     failing call on a context.
 *   - "device" pointers are HIP device memory on the context's device; "host"
 *     pointers are ordinary CPU memory.  The caller owns every pointer it
 *     passes; device buffers must stay valid until the work queued on the
 *     given stream has completed.  The context owns the geometry tables and
 *     its workspace.
 *   - Streams are passed as void* holding a hipStream_t (NULL = default
 *     stream).  Work is queued asynchronously; argument errors are reported
 *     synchronously, device-side data errors (an out-of-range geometry id,
 *     more kept pairs than the output capacity) are recorded in a device
 *     error word that cm_check_errors() reads (it synchronises the stream).
 *   - A context is not thread-safe; the server functions are.  Calls on one
 *     context that use its workspace (cm_collide, cm_collide_fused,
 *     cm_collide_backward) may go to different streams: a call on another
 *     stream than the previous such call first makes its stream wait for that
 *     call's work (an event), so they serialise rather than corrupt each
 *     other's scratch.  Under stream capture no such wait is inserted: keep
 *     a captured sequence on one stream.  cm_collide_noalloc uses the
 *     device-wide static workspace instead (see there).
 *   - Layouts are structure-of-arrays.  Poses: float [7][n_bodies] with rows
 *     (qw, qx, qy, qz, tx, ty, tz); the quaternion need not be normalised.
 *   - Geometry type ids / params:
 *       CM_SPHERE   (r)            mesh: 26 vertices, 56 edges on the sphere
 *       CM_CAPSULE  (r, half_len)  core segment on local z; mesh 34 V / 72 E
 *       CM_BOX      (hx, hy, hz, rounding)  outer half-extents; mesh 8 V / 12 E
 *       CM_POLYTOPE convex hull of the given points; SDF = tau-LSE over the
 *                   face planes (convex-polyhedron primitive, Sec. IV-B)
 *       CM_SQ_UNION smooth union -LSE_tau(-phi_i) of 1..CM_MAX_SQ superquadric
 *                   primitives (Sec. IV-B, SQ primitives and smooth union),
 *                   phi_i = |y| (1 - f_i(y)^(-eps1/2)) at the primitive-frame
 *                   point y; V-S normals from the union's softmax mix of
 *                   grad f_i.  Given as 4 xyz rows per primitive in the point
 *                   array: (a, b, c), (eps1, eps2, tx), (ty, tz, qw),
 *                   (qx, qy, qz) -- semi-axes > 0, exponents in [0.1, 1.9],
 *                   the primitive's pose in the body frame.  Mesh: per
 *                   primitive a parametric grid of 32 V / 90 E (poles, rings
 *                   at -60..60 degrees of 6 longitudes, one diagonal per
 *                   quad) minus the vertices strictly inside another
 *                   primitive.  cm_collide_backward differentiates through
 *                   them (pose twists and tau; their records take no
 *                   gradient and their g_params entries stay 0); for
 *                   exponents above 1 the normal field's derivative is
 *                   unbounded on a primitive's axis planes, where mesh edges
 *                   lie, so gradients there are ill-conditioned.
 *                   Contexts that hold them run every forward (plain and
 *                   fused) in 256-thread blocks.
 *       CM_OPC      oriented point cloud (Sec. IV-B, OPC primitives):
 *                   phi = sum_j B_j n_j . (x - p_j) / sum_j B_j with the
 *                   Gaussian basis B_j = exp(-|x - p_j|^2 / (2 sigma_j^2));
 *                   1..CM_MAX_OPC points given as 3 xyz rows each in the
 *                   point array: position, normal (normalised here),
 *                   (sigma > 0, 0, 0).  Mesh: the points as vertices and the
 *                   edges of their 4-nearest-neighbour graph.  Like
 *                   superquadric unions: run by the kernels built for
 *                   contexts holding either, no record gradient.
 */
#ifndef CM_H
#define CM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CM_OK = 0,
  CM_ERR_INVALID_ARG = -1,
  CM_ERR_OOM = -2,
  CM_ERR_DEVICE = -3,
  CM_ERR_NOT_READY = -4,
  CM_ERR_REJECTED = -5,
  CM_ERR_NOT_FOUND = -6,
  CM_ERR_CAPACITY = -7,
  CM_ERR_GEOMETRY = -8
} cm_status;

enum { CM_SPHERE = 0, CM_CAPSULE = 1, CM_BOX = 2, CM_POLYTOPE = 3, CM_SQ_UNION = 4, CM_OPC = 5 };
#define CM_MAX_SQ 32
#define CM_MAX_OPC 512

/* Largest K the kernels support. */
#define CM_MAX_K 32

typedef struct cm_context cm_context;
typedef struct cm_server cm_server;

/* Method parameters (Sec. III / IV).  tau is the single smoothing factor used
 * by every soft operator; lambda_reg is the L2 regularisation weight of the
 * E-E QP (Sec. IV-D-2); eps_n is the epsilon of the unsigned E-E normal
 * Delta e / sqrt(|Delta e|^2 + eps_n) (Sec. IV-D-3); cull_margin is the
 * broadphase margin.  Negative values select the defaults: lambda_reg 0.01,
 * eps_n tau^2, cull_margin 10 * tau (computed in float32). */
typedef struct {
  float tau;
  float lambda_reg;
  float eps_n;
  float cull_margin;
  int32_t K;          /* contacts per pair, 1..CM_MAX_K */
  uint32_t flags;     /* CM_FLAG_* below, 0 = the full method */
  int32_t presel_vertices;  /* soft top-K pre-selection: K_V, K_E per body, */
  int32_t presel_edges;     /* 1..CM_MAX_PRESEL each; both 0 = off (below)  */
  int32_t refine_steps;     /* witness sphere tracing: 0 = off, 1..CM_MAX_REFINE (below) */
} cm_params;

/* Witness sphere tracing (supplementary material, refinement of the witness
 * points by sphere tracing).  With refine_steps > 0 each E-E witness is moved
 * onto its own body's smoothed surface: along the fixed unit direction of
 * grad phi at the QP witness, x <- x - phi(x) n, refine_steps times; the
 * contact point, distance, normal and the sign / penetration / clashing tests
 * use the moved points, the nearest-neighbour ranking keeps the QP
 * distances.  cm_collide, cm_collide_backward and served requests (forward
 * and backward) take it with K <= 16 and at most 4096 vertices and edges per
 * body; cm_collide_fused returns CM_ERR_INVALID_ARG for it.  The adjoint
 * reverses every step: x_s_bar gains grad phi(x_s) (-n . x_{s+1}_bar), the
 * direction gains -phi(x_s) x_{s+1}_bar, and the direction's adjoint reaches
 * the QP witness through the Hessian of phi there. */
#define CM_MAX_REFINE 8

/* Simplifications the paper evaluates for speed (supplementary material,
 * possible simplifications): CM_FLAG_NO_EE drops the edge-edge candidates
 * (vertex-SDF contacts only); CM_FLAG_ONE_SIDED_VS keeps only A's vertices
 * against B's SDF.  Candidate order is unchanged otherwise. */
#define CM_FLAG_NO_EE 1u
#define CM_FLAG_ONE_SIDED_VS 2u

/* Soft top-K pre-selection (Sec. IV-A overview; supplementary material on
 * picking the top-K numbers and on safeguarding).  With presel_vertices and
 * presel_edges > 0, every vertex of a pair gets the other body's SDF at it as
 * penetration metric and every edge the mean of its corners' metrics; SoftSort
 * rows over -metric select min(K_V, |V|) vertices and min(K_E, |E|) edges per
 * body as weighted averages, and the candidates are built from those only
 * (V-S over the selected vertices, E-E over the selected edge pairs).
 * CM_FLAG_SAFEGUARD additionally scales every E-E activity by the soft
 * indicators that both witness points lie inside their own bodies.
 * cm_collide, cm_collide_fused, cm_collide_backward (whose gradient also
 * runs through the selection weights into every vertex's metric) and served
 * requests take it.  Bodies of at
 * most 4096 vertices and edges (else CM_ERR_INVALID_ARG or CM_ERR_DEVICE). */
#define CM_MAX_PRESEL 64
#define CM_FLAG_SAFEGUARD 4u

/* A batch of scenes.  Bodies of scene s are body_offsets[s] .. [s+1]-1.
 * Candidate pairs: all i < j within each scene when cand_offsets is NULL,
 * otherwise cand_pairs[0][c], cand_pairs[1][c] (global body ids) for the
 * candidates cand_offsets[s] .. [s+1]-1 of scene s.  All arrays device. */
typedef struct {
  int32_t n_scenes;
  int32_t n_bodies;
  const int32_t* body_offsets;   /* [n_scenes + 1] */
  const int32_t* body_geom;      /* [n_bodies] geometry id per body */
  const float* pose;             /* [7][n_bodies] */
  const int32_t* cand_offsets;   /* [n_scenes + 1] or NULL */
  const int32_t* cand_pairs;     /* [2][n_cand] or NULL */
  int32_t n_cand;
} cm_batch;

/* Caller-owned output buffers (device).  Pair p, contact k lives at index
 * p * K + k of each SoA row; point / normal are [3][capacity * K]. */
typedef struct {
  int32_t capacity;      /* rows available for kept pairs */
  int32_t* n_pairs;      /* [1]  number of kept pairs (may exceed capacity) */
  int32_t* pair_offsets; /* [n_scenes + 1] exclusive scan of kept pairs per scene */
  int32_t* pairs;        /* [2][capacity] body ids (A, B) of each kept pair */
  float* point;          /* [3][capacity * K] world-frame contact points */
  float* normal;         /* [3][capacity * K] pair normals, A -> B */
  float* dist;           /* [capacity * K] signed distances */
  float* weight;         /* [capacity * K] activity weights in [0, 1] */
  void* tape;            /* optional (NULL = none): the adjoint's tape, cm_tape_bytes bytes, 16-byte aligned */
  int64_t tape_bytes;    /* size of `tape` */
} cm_manifold;

/* Cotangents of the manifold outputs (device, same layout as cm_manifold;
 * any may be NULL = zero). */
typedef struct {
  const float* g_point;
  const float* g_normal;
  const float* g_dist;
  const float* g_weight;
} cm_cotangent;

/* Gradient outputs (device).  Every buffer is overwritten (not accumulated).
 * g_pose:     [6][n_bodies] left-tangent gradient (rho, omega) of each body:
 *             T' = Exp(xi) T, so a world point moves by rho + omega x p.
 * g_vertices: [3][n_vertices_total] per geometry vertex (context vertex pool;
 *             cm_geometry_info gives each geometry's offset).  For polytopes
 *             these are the hull vertices in ascending input-point order.
 * g_params:   [4][n_geometries] per analytic-geometry parameter.
 * g_tau:      [1] derivative with respect to tau.
 * Gradients with respect to geometry are summed over every use. */
typedef struct {
  float* g_pose;
  float* g_vertices;
  float* g_params;
  float* g_tau;
} cm_grads;

typedef struct {
  int32_t type;
  int32_t n_vertices, n_edges, n_faces;
  int32_t vertex_offset;   /* into the context vertex pool */
  float bound_radius;      /* float32 bounding radius about the body origin */
} cm_geometry_info_t;

/* ---------------------------------------------------------------- context */
cm_status cm_context_create(int device, cm_context** out);
cm_status cm_context_destroy(cm_context* ctx);
const char* cm_status_str(cm_status s);
const char* cm_last_error(cm_context* ctx);
/* Synchronise `stream` and report device-side errors recorded since the last
 * check (CM_ERR_CAPACITY, CM_ERR_NOT_FOUND), then clear them. */
cm_status cm_check_errors(cm_context* ctx, void* stream);

/* ---------------------------------------------------------------- geometry
 * Create n geometries (Sec. IV-A: every surface has a mesh and an SDF).
 * types[n], params[n*4] (host); POLYTOPE point sets are points[3*k] for
 * k in pt_offsets[i] .. pt_offsets[i+1]-1 (host, float xyz).  The library
 * builds the meshes (convex hull for polytopes: vertices, edges, outward
 * triangle planes), bounding radii and device tables.  out_ids[n] receives
 * the new ids.  Fails with CM_ERR_GEOMETRY for degenerate point sets. */
cm_status cm_geometry_create(cm_context* ctx, int32_t n, const int32_t* types, const float* params,
                             const int64_t* pt_offsets, const float* points, int32_t* out_ids);
cm_status cm_geometry_info(cm_context* ctx, int32_t id, cm_geometry_info_t* out);
/* Host copy of a geometry's mesh: vertices[3*nv] (xyz), edges[2*ne], faces[3*nf]
 * (any may be NULL). */
cm_status cm_geometry_mesh(cm_context* ctx, int32_t id, float* vertices, int32_t* edges, int32_t* faces);
int32_t cm_geometry_count(cm_context* ctx);
int32_t cm_vertex_pool_size(cm_context* ctx);
/* Destroy n geometries (host ids[n]).  Every id must name a live geometry of
 * this context (else CM_ERR_NOT_FOUND and nothing changes); geometry is
 * frozen while a server runs (CM_ERR_INVALID_ARG).  The call waits for the
 * device to finish queued work, then repacks the vertex / edge / plane
 * tables without the destroyed geometries: the other geometries keep their
 * ids but their vertex_offset (cm_geometry_info) may change, and
 * cm_vertex_pool_size shrinks.  Destroyed ids are not reused; a batch that
 * still references one is flagged like an out-of-range id (CM_ERR_NOT_FOUND
 * from cm_check_errors), and cm_geometry_info / cm_geometry_mesh return
 * CM_ERR_NOT_FOUND for it.  cm_geometry_count keeps counting ids. */
cm_status cm_geometry_destroy(cm_context* ctx, const int32_t* ids, int32_t n);

/* ---------------------------------------------------------------- forward
 * Broadphase (keep a candidate pair iff its float32 bounding spheres overlap
 * within cull_margin), per-scene compaction, then the contact manifold of
 * every kept pair (Sec. IV-C, IV-D, soft top-K of Sec. III).  The plain
 * kernel: one workgroup per pair; workgroups take pairs in batch order from a
 * work queue (static round-robin with traced witnesses, refine_steps > 0). */
cm_status cm_collide(cm_context* ctx, const cm_batch* batch, const cm_params* prm, cm_manifold* out,
                     void* stream);

/* Same results (bit for bit) through the fused batched path: pairs are
 * ordered by cost into size classes and pulled from device work queues by
 * persistent grids whose block sizes are autotuned (below); the whole
 * sequence is captured once per (batch shape, parameters) in a hipGraph and
 * replayed.  Takes pre-selection and the extended primitives; returns
 * CM_ERR_INVALID_ARG for refine_steps > 0. */
cm_status cm_collide_fused(cm_context* ctx, const cm_batch* batch, const cm_params* prm, cm_manifold* out,
                           void* stream);
/* The fused path's autotuner: pairs fall in 3 size classes by the larger edge
 * count of their bodies (<= 96, <= 300, above), each with its own LDS sizing
 * and persistent grid.  Once per (geometry set, K, batch-size bucket: one
 * per factor of 4 in candidate pairs) the first cm_collide_fused call
 * classifies its batch, times each class's kernel at
 * 256-, 128- and 64-thread blocks (those that keep at least 2 waves per
 * SIMD; 256 always) on the same evenly strided sample of the class's cost
 * order (about 1/16 of its pairs) and keeps the fastest; the
 * choice is stored in the text file named by CM_TUNE_CACHE (default
 * $HOME/.cache/cm_fused_tune.txt), keyed by device architecture, CU count
 * the class's largest vertex / edge / face counts, K and the batch-size
 * bucket, and read back by later processes instead of timing.  cm_fused_tuning reports the current
 * plan: per class (arrays of 3, any may be NULL) the largest edge count, the
 * block size, the sample size, the sample timings in ms at 256, 128 and 64
 * ([3][3], 0 when not timed) and whether the choice came from the cache.
 * Results do not depend on the block size. */
cm_status cm_fused_tuning(cm_context* ctx, int32_t* class_max_edges, int32_t* class_blocks, int32_t* sample_pairs,
                          float* sample_ms, int32_t* from_cache);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, hosts that forbid hipMalloc): the same
 * forward as cm_collide (same kernels, same arguments, bit-identical
 * results), with every workspace -- the broadphase scan's tile sums and the
 * per-workgroup scratch slots of the pair kernel -- taken from one static
 * device array of CM_NOALLOC_SCRATCH_BYTES compiled into the library instead
 * of the context's growable workspace.  It calls no hipMalloc / hipFree and
 * records no timing events.  The array's device address is looked up once
 * per device in cm_context_create; if that lookup failed, this call returns
 * CM_ERR_DEVICE.  The pair kernel's grid shrinks to the number of
 * workgroup slots that fit (fewer than cm_collide launches for large meshes,
 * hence slower); a batch whose tile sums plus one slot exceed the array
 * returns CM_ERR_CAPACITY with the sizes in cm_last_error.  Nothing in the
 * array needs to start at zero.  Every call on one device shares that
 * device's single array: calls that overlap in time on one device (several
 * streams, contexts or threads) race and corrupt each other's results, so
 * order them on one stream. */
#define CM_NOALLOC_SCRATCH_BYTES (64u << 20)
cm_status cm_collide_noalloc(cm_context* ctx, const cm_batch* batch, const cm_params* prm, cm_manifold* out,
                             void* stream);

/* ---------------------------------------------------------------- backward
 * Vector-Jacobian product of the manifold (the gradient the paper obtains by
 * automatic differentiation and times in Sec. V): recomputes every per-pair
 * intermediate from the inputs and the kept-pair list in `fwd` (no E x E
 * state is stored by the forward), then reverses the SoftSort, the
 * activity/score terms, the nearest-neighbour softmaxes, the SDF queries,
 * the witness QP and the rigid transforms (with refine_steps > 0 also the
 * sphere-tracing steps, above).  Broadphase decisions and hull topology are
 * held fixed.  It runs as two launches on `stream`: the forward kernel
 * records, per kept pair, s_[k], the SoftSort row sums and the candidates
 * within the adjoint's window (the adjoint's tape: a context workspace of
 * capacity x (16 + 80 K) bytes plus a pool holding each pair's window as
 * candidate indices or, when smaller, one bit per candidate), then the
 * adjoint kernel recomputes only the distance pass and reverses the rest.
 * The pool holds 2^28 four-byte entries (1 GiB) by default, fewer when the
 * context's meshes cannot fill them; the environment variable
 * CM_ADJOINT_TAPE sets that count, and 0 turns the tape off (the adjoint
 * then recomputes the whole forward per pair, as it also does for pairs
 * whose windows no longer fit).  Both ways give the same gradients up to
 * the order of float32 atomic additions. */
cm_status cm_collide_backward(cm_context* ctx, const cm_batch* batch, const cm_params* prm,
                              const cm_manifold* fwd, const cm_cotangent* cot, cm_grads* out, void* stream);

/* The adjoint's tape recorded by the forward (device memory the caller owns,
 * as for the other outputs).  When a manifold's `tape` is non-NULL,
 * cm_collide and cm_collide_fused also record into it, per kept pair, s_[k],
 * the SoftSort row sums and the adjoint's window, and cm_collide_backward
 * given that manifold reverses from it instead of running the recording
 * forward itself (one launch instead of two).  The tape belongs to the
 * forward call that recorded it: the batch contents (poses, geometry) and
 * parameters must be unchanged when the backward uses it, or the gradients
 * are wrong (the kernels still stay within their buffers).  cm_tape_bytes
 * gives the size for `capacity` pairs at K with pool_entries four-byte pool
 * entries (<= 0: the pool cm_collide_backward would use on its own for this
 * context, see above); pairs whose windows do not fit the pool are
 * recomputed whole by the backward.  A tape smaller than cm_tape_bytes(...,
 * 2, ...) or not 16-byte aligned: CM_ERR_INVALID_ARG.  cm_collide_noalloc
 * does not record one (CM_ERR_INVALID_ARG for a non-NULL tape).
 * Layout (for callers that inspect the windows): bytes [0, 256) hold the
 * pool's fill counter (uint64 at 0); kept pair p's record starts at byte
 * 256 + p (16 + 80 K): int32 count of its window's candidates, int32 form
 * (0: not recorded, the pool was full; 1: int32 candidate indices in three
 * runs, each ascending: the vertex-SDF candidates, the edge-edge witnesses 1,
 * the witnesses 2; 2: one bit per candidate, bit i & 63 of uint64 word
 * i >> 6), int64 offset
 * of that list or mask in the pool in 4-byte entries, float64 s_[1..K], then
 * the float64 SoftSort row sums [K][9]; the pool starts at byte 256 +
 * (capacity (16 + 80 K) rounded up to a multiple of 256).  Candidate indices
 * follow the order A's vertices, B's vertices, then edge pairs (k, l)
 * row-major with witness 1 before witness 2. */
cm_status cm_tape_bytes(cm_context* ctx, int32_t capacity, int32_t K, int64_t pool_entries, int64_t* bytes);

/* ---------------------------------------------------------------- E-E witness points
 * The edge-edge witness routine on its own, over n independent edge pairs:
 * the regularised QP of Sec. IV-D-2 solved by the analytic active set, and
 * the witness points of Sec. IV-D-3, as in the witness-point speed
 * experiment of Sec. V (Fig. 6).  Edge 1 runs a0 -> a1, edge 2 b0 -> b1.
 *   edges  device float32 [12][n], rows a0.x a0.y a0.z a1.x a1.y a1.z
 *          b0.x b0.y b0.z b1.x b1.y b1.z, row stride n (read only)
 *   out    device float32 [9][n], rows alpha1, alpha2, con, e1.x e1.y e1.z,
 *          e2.x e2.y e2.z, row stride n; con is the indicator that the
 *          unconstrained minimiser lies in [0,1]^2 (soft, or 0/1 with
 *          CM_EE_HARD); e1 - e2 gives the unsigned distance and normal
 *   tau        temperature of the smoothed solver (> 0; unused with CM_EE_HARD)
 *   lambda_reg regulariser (< 0: 0.01; otherwise > 0)
 *   mode       CM_EE_SMOOTH (the method) or CM_EE_HARD (no smoothing: the
 *              exact minimiser over the box, the paper's Ours-NS)
 * Computes in float64.  Both buffers stay the caller's; they must not
 * overlap.  n = 0 does nothing; n < 0, a null buffer with n > 0 or an unknown
 * mode returns CM_ERR_INVALID_ARG.  Asynchronous on stream. */
#define CM_EE_SMOOTH 0
#define CM_EE_HARD 1
cm_status cm_ee_witness(cm_context* ctx, const float* edges, int64_t n, float tau, float lambda_reg, int32_t mode,
                        float* out, void* stream);

/* ---------------------------------------------------------------- serving
 * A continuous-batching request loop over resident geometry (the serving
 * form; no passage of the paper: it serves the method of Sec. IV to many
 * callers).  A scheduler thread admits requests in arrival order while (a)
 * their device footprint (inputs, outputs, per-workgroup scratch, gradients)
 * fits in hbm_budget_bytes beside the running ones, (b) their pinned host
 * result block fits in the host budget (8 GiB unless set with
 * cm_server_set_host_budget) beside the results not yet released, and (c)
 * one of n_streams stream slots is free;
 * admitted requests run concurrently, one stream each, with their own
 * device workspace and device error word.  submit copies the request (host
 * arrays) and returns a ticket; a request that could never fit either budget
 * is rejected at submit with CM_ERR_REJECTED.  poll returns CM_ERR_NOT_READY
 * until the request completed, then fills the result, whose host arrays the
 * server owns until cm_server_release (released blocks are reused, so
 * release results promptly: unreleased results hold host budget and can keep
 * later requests waiting).  A completed request's status: CM_OK,
 * CM_ERR_CAPACITY (more kept pairs than capacity; the first capacity pairs
 * are valid), CM_ERR_NOT_FOUND (a destroyed geometry), CM_ERR_OOM or
 * CM_ERR_DEVICE.  The geometry of the context is frozen while a server
 * exists.  submit / poll / release / stats are thread-safe; a failing
 * server call leaves its message in cm_server_last_error() of the calling
 * thread (the context's cm_last_error is not used by the server). */
typedef struct {
  int32_t n_scenes;
  int32_t n_bodies;
  const int32_t* body_offsets;   /* host [n_scenes + 1], body_offsets[0] = 0, non-decreasing */
  const int32_t* body_geom;      /* host [n_bodies] live geometry ids */
  const float* pose;             /* host [7][n_bodies] */
  cm_params params;
  int32_t want_backward;         /* also the vector-Jacobian product of L = <cot, outputs> */
  const float* cot_point;        /* host [3][capacity*K] or NULL = 0 (backward only) */
  const float* cot_normal;       /* host [3][capacity*K] or NULL */
  const float* cot_dist;         /* host [capacity*K] or NULL */
  const float* cot_weight;       /* host [capacity*K] or NULL */
  int32_t want_geometry_grads;   /* backward: also g_vertices and g_params */
  int32_t capacity;              /* output pair capacity (<= 0: all candidate pairs) */
} cm_request;

typedef struct {
  cm_status status;
  int32_t n_pairs;
  int32_t capacity;              /* row stride of the manifold arrays below */
  const int32_t* pair_offsets;   /* host [n_scenes + 1] */
  const int32_t* pairs;          /* host [2][capacity] */
  const float* point;            /* host [3][capacity*K] */
  const float* normal;
  const float* dist;
  const float* weight;
  const float* g_pose;           /* host [6][n_bodies] (backward) */
  const float* g_tau;            /* host [1] (backward) */
  const float* g_vertices;       /* host [3][vertex_pool] (backward with want_geometry_grads) */
  const float* g_params;         /* host [4][n_geometries] (same) */
  int32_t vertex_pool;           /* row stride of g_vertices (the pool size at submit) */
  int32_t n_geometries;          /* row stride of g_params */
  double t_submit, t_start, t_done;   /* seconds, server clock */
  uint64_t footprint_bytes;      /* device bytes the request was admitted with */
} cm_result;

/* ---------------------------------------------------------------- timing
 * Opt-in kernel timing for measurement.  While enabled, every cm_collide /
 * cm_collide_fused / cm_collide_backward / cm_ee_witness call records a pair of HIP events on
 * the caller's stream around each timed unit: CM_TIMER_BROADPHASE (broadphase
 * and compaction), CM_TIMER_FORWARD (the forward pair kernel),
 * CM_TIMER_BACKWARD (the adjoint kernel), CM_TIMER_FUSED (one replay of the
 * fused graph), CM_TIMER_EE_WITNESS (one cm_ee_witness launch).  cm_kernel_time waits for the recorded events and returns the
 * summed milliseconds and the number of timed launches since timing was
 * enabled.  Enabling resets the sums.  Not for use under stream capture. */
enum {
  CM_TIMER_BROADPHASE = 0,
  CM_TIMER_FORWARD = 1,
  CM_TIMER_BACKWARD = 2,
  CM_TIMER_FUSED = 3,
  CM_TIMER_EE_WITNESS = 4,
  CM_N_TIMERS = 5
};
cm_status cm_set_kernel_timing(cm_context* ctx, int32_t enable);
cm_status cm_kernel_time(cm_context* ctx, int32_t timer, double* total_ms, int64_t* launches);

cm_status cm_server_create(cm_context* ctx, uint64_t hbm_budget_bytes, int32_t n_streams, cm_server** out);
cm_status cm_server_set_host_budget(cm_server* srv, uint64_t host_budget_bytes);
cm_status cm_server_submit(cm_server* srv, const cm_request* req, uint64_t* ticket);
cm_status cm_server_poll(cm_server* srv, uint64_t ticket, cm_result* out);
cm_status cm_server_release(cm_server* srv, uint64_t ticket);
cm_status cm_server_stats(cm_server* srv, uint64_t* in_flight_bytes, int32_t* n_pending, int32_t* n_running);
cm_status cm_server_destroy(cm_server* srv);
const char* cm_server_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CM_H */
