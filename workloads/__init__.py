"""Seeded synthetic scene generators shared by the tests, the oracle and bench.py.

This module holds NO arithmetic of the contact-manifold method: it only draws
random scene descriptions (geometry descriptors, poses, candidate pair lists,
cotangents) and rounds them once to float32.  Both the FP64 oracle and the HIP
library consume exactly these float32 values.

Geometry type ids and parameter slots (shared vocabulary of the boundary):
  SPHERE   = 0 : params = (r, 0, 0, 0)
  CAPSULE  = 1 : params = (r, half_length, 0, 0), core segment along local z
  BOX      = 2 : params = (hx, hy, hz, rounding)   outer half-extents
  POLYTOPE = 3 : params unused; ``points`` holds the hull input points (local)
  SQ_UNION = 4 : params unused; ``points`` holds 4 xyz rows per superquadric
                 primitive: (a, b, c), (eps1, eps2, tx), (ty, tz, qw),
                 (qx, qy, qz) -- semi-axes, shape exponents and the
                 primitive's pose in the body frame

Poses are quaternion + translation, stored structure-of-arrays as a float32
array ``pose[7, n_bodies]`` with rows (qw, qx, qy, qz, tx, ty, tz).

The five workload families follow the synthetic configurations of the build
plan: a small cube-cube batch, a mixed 8-body batch, a polytope batch for the
adjoint, an uneven batch with penetration forcing, and a serving request mix.
Rotations are uniform (normalised 4-D Gaussians), points "uniform on an
ellipsoid" are sphere-uniform directions scaled by the semi-axes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SPHERE, CAPSULE, BOX, POLYTOPE, SQ_UNION, OPC = 0, 1, 2, 3, 4, 5
BOX_ROUNDING = 0.02


@dataclass
class GeomSet:
    """A set of geometry descriptors (float32, host)."""
    types: np.ndarray                 # int32 [G]
    params: np.ndarray                # float32 [G, 4]
    pt_off: np.ndarray                # int64 [G+1] offsets into points
    points: np.ndarray                # float32 [P, 3]

    @property
    def n(self) -> int:
        return int(self.types.shape[0])

    def points_of(self, g: int) -> np.ndarray:
        return self.points[self.pt_off[g]:self.pt_off[g + 1]]

    def subset(self, ids) -> "GeomSet":
        ids = np.asarray(ids, dtype=np.int64)
        pts = [self.points_of(int(g)) for g in ids]
        cnt = np.array([p.shape[0] for p in pts], dtype=np.int64)
        off = np.zeros(len(ids) + 1, dtype=np.int64)
        off[1:] = np.cumsum(cnt)
        allp = np.concatenate(pts, axis=0) if len(pts) and off[-1] > 0 else np.zeros((0, 3), np.float32)
        return GeomSet(self.types[ids].copy(), self.params[ids].copy(), off, allp.astype(np.float32))


@dataclass
class Batch:
    """A batch of scenes: bodies (geometry id + pose) and candidate pairs."""
    geoms: GeomSet
    body_offsets: np.ndarray          # int32 [S+1]
    body_geom: np.ndarray             # int32 [nb]   geometry id per body
    pose: np.ndarray                  # float32 [7, nb]
    tau: float
    K: int
    cand_offsets: Optional[np.ndarray] = None   # int32 [S+1] or None = all i<j
    cand_pairs: Optional[np.ndarray] = None     # int32 [2, nc] global body ids
    name: str = ""
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        # tau crosses the boundary as float32: keep the float32 value on both sides
        self.tau = float(np.float32(self.tau))

    @property
    def n_scenes(self) -> int:
        return int(self.body_offsets.shape[0] - 1)

    @property
    def n_bodies(self) -> int:
        return int(self.body_geom.shape[0])

    def candidate_pairs(self):
        """All candidate pairs in scene-major order as (scene, a, b) arrays."""
        if self.cand_pairs is not None:
            sc = np.repeat(np.arange(self.n_scenes, dtype=np.int32),
                           np.diff(self.cand_offsets).astype(np.int64))
            return sc, self.cand_pairs[0].copy(), self.cand_pairs[1].copy()
        scs, As, Bs = [], [], []
        bo = self.body_offsets
        nbs = np.diff(bo)
        for nb in np.unique(nbs):
            sel = np.nonzero(nbs == nb)[0]
            ii, jj = np.triu_indices(int(nb), k=1)
            s_rep = np.repeat(sel, len(ii))
            base = np.repeat(bo[sel], len(ii))
            scs.append(s_rep)
            As.append(base + np.tile(ii, len(sel)))
            Bs.append(base + np.tile(jj, len(sel)))
        if not scs:
            z = np.zeros(0, np.int32)
            return z, z, z
        sc = np.concatenate(scs); a = np.concatenate(As); b = np.concatenate(Bs)
        order = np.lexsort((b, a, sc))
        return sc[order].astype(np.int32), a[order].astype(np.int32), b[order].astype(np.int32)


# ----------------------------------------------------------------------------- draws

def _rng(cfg: int, seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[cfg * 1_000_003 + seed, stream]))


def uniform_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1.0
    return q


def ellipsoid_points(rng: np.random.Generator, n: int, semi_axes) -> np.ndarray:
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * np.asarray(semi_axes, dtype=np.float64)[None, :]


def _pose_array(q: np.ndarray, t: np.ndarray) -> np.ndarray:
    return np.concatenate([q.T, t.T], axis=0).astype(np.float32)


def _geomset(types, params, point_lists) -> GeomSet:
    types = np.asarray(types, dtype=np.int32)
    params = np.asarray(params, dtype=np.float32).reshape(-1, 4)
    cnt = np.array([0 if p is None else len(p) for p in point_lists], dtype=np.int64)
    off = np.zeros(len(point_lists) + 1, dtype=np.int64)
    off[1:] = np.cumsum(cnt)
    pts = [p for p in point_lists if p is not None and len(p)]
    allp = np.concatenate(pts, axis=0).astype(np.float32) if pts else np.zeros((0, 3), np.float32)
    return GeomSet(types, params, off, allp)


def _analytic_params(rng, kind: int) -> np.ndarray:
    if kind == SPHERE:
        return np.array([rng.uniform(0.1, 0.5), 0, 0, 0])
    if kind == CAPSULE:
        return np.array([rng.uniform(0.05, 0.2), rng.uniform(0.1, 0.5), 0, 0])
    h = rng.uniform(0.1, 0.5, size=3)
    return np.array([h[0], h[1], h[2], BOX_ROUNDING])


# ----------------------------------------------------------------------------- configs

def cube_pairs(n_scenes: int = 4096, seed: int = 0, tau: float = 0.01, K: int = 8,
               box_rounding: float = BOX_ROUNDING) -> Batch:
    """Small plain-forward batch: one pair of unit cubes per scene.

    Body A sits at the identity; body B has translation U[-1.1, 1.1]^3 and a
    uniform rotation.  Both bodies share geometry id 0 (half-extents 0.5).
    """
    rng = _rng(1, seed)
    geoms = _geomset([BOX], [[0.5, 0.5, 0.5, box_rounding]], [None])
    S = n_scenes
    q = np.zeros((2 * S, 4)); q[:, 0] = 1.0
    t = np.zeros((2 * S, 3))
    q[1::2] = uniform_quats(rng, S)
    t[1::2] = rng.uniform(-1.1, 1.1, size=(S, 3))
    return Batch(geoms=geoms,
                 body_offsets=(2 * np.arange(S + 1)).astype(np.int32),
                 body_geom=np.zeros(2 * S, np.int32),
                 pose=_pose_array(q, t), tau=tau, K=K, name="cube_pairs")


MIXED_SLOTS = (SPHERE, SPHERE, CAPSULE, CAPSULE, BOX, BOX, POLYTOPE, POLYTOPE)


def mixed_scenes(n_scenes: int = 65536, seed: int = 0, tau: float = 0.005, K: int = 8,
                 poly_points: int = 32) -> Batch:
    """Plain-forward batched workload: 8 bodies of mixed types per scene.

    Slots: 2 spheres, 2 capsules, 2 boxes, 2 polytopes (hull of 32 points on an
    ellipsoid with semi-axes U[0.2, 0.5]).  Centres U[-1, 1]^3, uniform
    rotations, all 28 pairs are candidates.
    """
    rng = _rng(2, seed)
    S = n_scenes
    nb = 8 * S
    kinds = np.tile(np.array(MIXED_SLOTS, dtype=np.int32), S)
    params = np.zeros((nb, 4))
    pts = [None] * nb
    r_s = rng.uniform(0.1, 0.5, size=(S, 2))
    r_c = rng.uniform(0.05, 0.2, size=(S, 2))
    h_c = rng.uniform(0.1, 0.5, size=(S, 2))
    h_b = rng.uniform(0.1, 0.5, size=(S, 2, 3))
    ax = rng.uniform(0.2, 0.5, size=(S, 2, 3))
    dirs = rng.standard_normal((S, 2, poly_points, 3))
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    base = 8 * np.arange(S)
    params[base + 0, 0] = r_s[:, 0]; params[base + 1, 0] = r_s[:, 1]
    params[base + 2, 0] = r_c[:, 0]; params[base + 2, 1] = h_c[:, 0]
    params[base + 3, 0] = r_c[:, 1]; params[base + 3, 1] = h_c[:, 1]
    params[base + 4, :3] = h_b[:, 0]; params[base + 4, 3] = BOX_ROUNDING
    params[base + 5, :3] = h_b[:, 1]; params[base + 5, 3] = BOX_ROUNDING
    polys = dirs * ax[:, :, None, :]
    # points of polytope bodies are contiguous: slot 6 then slot 7 of each scene
    cnt = np.zeros(nb, dtype=np.int64)
    cnt[base + 6] = poly_points; cnt[base + 7] = poly_points
    off = np.zeros(nb + 1, dtype=np.int64); off[1:] = np.cumsum(cnt)
    allp = polys.reshape(-1, 3).astype(np.float32)
    geoms = GeomSet(kinds, params.astype(np.float32), off, allp)
    q = uniform_quats(rng, nb)
    t = rng.uniform(-1.0, 1.0, size=(nb, 3))
    return Batch(geoms=geoms,
                 body_offsets=(8 * np.arange(S + 1)).astype(np.int32),
                 body_geom=np.arange(nb, dtype=np.int32),
                 pose=_pose_array(q, t), tau=tau, K=K, name="mixed_scenes")


def polytope_scenes(n_scenes: int = 16384, seed: int = 0, tau: float = 0.01, K: int = 8,
                    n_points: int = 64, bodies: int = 4, centre_box: float = 0.5) -> Batch:
    """Differentiation workload: 4 convex polytopes per scene.

    Each polytope is the hull of 64 points on the unit sphere scaled per axis
    by U[0.3, 0.6].  Centres U[-0.5, 0.5]^3 so most of the 6 pairs collide.
    """
    rng = _rng(3, seed)
    S = n_scenes
    nb = bodies * S
    ax = rng.uniform(0.3, 0.6, size=(nb, 3))
    dirs = rng.standard_normal((nb, n_points, 3))
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    pts = (dirs * ax[:, None, :]).reshape(-1, 3).astype(np.float32)
    off = (n_points * np.arange(nb + 1)).astype(np.int64)
    geoms = GeomSet(np.full(nb, POLYTOPE, np.int32), np.zeros((nb, 4), np.float32), off, pts)
    q = uniform_quats(rng, nb)
    t = rng.uniform(-centre_box, centre_box, size=(nb, 3))
    return Batch(geoms=geoms,
                 body_offsets=(bodies * np.arange(S + 1)).astype(np.int32),
                 body_geom=np.arange(nb, dtype=np.int32),
                 pose=_pose_array(q, t), tau=tau, K=K, name="polytope_scenes")


def _quat_to_R(q: np.ndarray) -> np.ndarray:
    # rotation matrices for placing bodies (generator-side only)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z); R[..., 0, 1] = 2 * (x * y - w * z); R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z); R[..., 1, 1] = 1 - 2 * (x * x + z * z); R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y); R[..., 2, 1] = 2 * (y * z + w * x); R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _support(kind: int, params: np.ndarray, pts: Optional[np.ndarray], R: np.ndarray, u: np.ndarray) -> float:
    """Support value max_{x in body} u.x (body at the origin, rotation R).

    Used only to place bodies so that their support intervals overlap by a
    chosen depth.  Analytic bodies use their exact surfaces.
    """
    ul = R.T @ u
    if kind == SPHERE:
        return float(params[0])
    if kind == CAPSULE:
        return float(params[0] + params[1] * abs(ul[2]))
    if kind == BOX:
        rr = params[3]
        return float(np.sum((params[:3] - rr) * np.abs(ul)) + rr)
    return float(np.max(pts.astype(np.float64) @ ul))


def uneven_scenes(n_scenes: int = 100_000, seed: int = 0, tau: float = 0.01, K: int = 16,
                  mean_pairs: float = 12.0, max_pairs: int = 64, v_min: int = 8, v_max: int = 256,
                  analytic_frac: float = 0.2, pen_frac: float = 0.3, pen_max: float = 0.05) -> Batch:
    """Uneven batching workload.

    Pairs per scene ~ Geometric(mean 12) clipped to [1, 64]; each scene holds
    that many disjoint body pairs listed explicitly as candidates.  80% of
    bodies are polytopes with log-uniform vertex counts in [8, 256] (points on
    random ellipsoids), 20% analytic.  30% of pairs are placed so that the
    support intervals along a random direction overlap by U[0, 0.05].
    """
    rng = _rng(4, seed)
    S = n_scenes
    p_geo = 1.0 / mean_pairs
    P = np.clip(rng.geometric(p_geo, size=S), 1, max_pairs).astype(np.int64)
    n_pairs = int(P.sum())
    nb = 2 * n_pairs
    is_poly = rng.uniform(size=nb) >= analytic_frac
    akind = rng.integers(0, 3, size=nb)
    kinds = np.where(is_poly, POLYTOPE, akind).astype(np.int32)
    nv = np.round(np.exp(rng.uniform(np.log(v_min), np.log(v_max), size=nb))).astype(np.int64)
    nv = np.where(is_poly, nv, 0)
    params = np.zeros((nb, 4))
    r_s = rng.uniform(0.1, 0.5, size=nb)
    r_c = rng.uniform(0.05, 0.2, size=nb)
    h_c = rng.uniform(0.1, 0.5, size=nb)
    h_b = rng.uniform(0.1, 0.5, size=(nb, 3))
    params[kinds == SPHERE, 0] = r_s[kinds == SPHERE]
    params[kinds == CAPSULE, 0] = r_c[kinds == CAPSULE]
    params[kinds == CAPSULE, 1] = h_c[kinds == CAPSULE]
    params[kinds == BOX, :3] = h_b[kinds == BOX]
    params[kinds == BOX, 3] = BOX_ROUNDING
    ax = rng.uniform(0.2, 0.5, size=(nb, 3))
    off = np.zeros(nb + 1, dtype=np.int64); off[1:] = np.cumsum(nv)
    dirs = rng.standard_normal((int(off[-1]), 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    owner = np.repeat(np.arange(nb), nv)
    pts = (dirs * ax[owner]).astype(np.float32)
    params = params.astype(np.float32)
    q = uniform_quats(rng, nb)
    t = rng.uniform(-1.0, 1.0, size=(nb, 3))
    # penetration forcing on a Bernoulli(0.3) subset of pairs
    force = rng.uniform(size=n_pairs) < pen_frac
    u_dirs = rng.standard_normal((n_pairs, 3))
    u_dirs /= np.linalg.norm(u_dirs, axis=1, keepdims=True)
    depth = rng.uniform(0.0, pen_max, size=n_pairs)
    qf = q.astype(np.float32).astype(np.float64)
    Rs = _quat_to_R(qf)
    for i in np.nonzero(force)[0]:
        a, b = 2 * i, 2 * i + 1
        u = u_dirs[i]
        ha = _support(kinds[a], params[a], pts[off[a]:off[a + 1]], Rs[a], u)
        hb = _support(kinds[b], params[b], pts[off[b]:off[b + 1]], Rs[b], -u)
        t[b] = t[a] + u * (ha + hb - depth[i])
    geoms = GeomSet(kinds, params, off, pts)
    body_offsets = np.zeros(S + 1, dtype=np.int64); body_offsets[1:] = np.cumsum(2 * P)
    cand_offsets = np.zeros(S + 1, dtype=np.int64); cand_offsets[1:] = np.cumsum(P)
    cand = np.stack([2 * np.arange(n_pairs), 2 * np.arange(n_pairs) + 1]).astype(np.int32)
    return Batch(geoms=geoms, body_offsets=body_offsets.astype(np.int32),
                 body_geom=np.arange(nb, dtype=np.int32), pose=_pose_array(q, t),
                 tau=tau, K=K, cand_offsets=cand_offsets.astype(np.int32), cand_pairs=cand,
                 name="uneven_scenes", meta={"forced": force})


def polytope_pool(n_geoms: int = 256, seed: int = 0, n_points: int = 64) -> GeomSet:
    """Resident pool of polytopes shaped like the differentiation workload."""
    rng = _rng(5, seed, 1)
    ax = rng.uniform(0.3, 0.6, size=(n_geoms, 3))
    dirs = rng.standard_normal((n_geoms, n_points, 3))
    dirs /= np.linalg.norm(dirs, axis=-1, keepdims=True)
    pts = (dirs * ax[:, None, :]).reshape(-1, 3).astype(np.float32)
    off = (n_points * np.arange(n_geoms + 1)).astype(np.int64)
    return GeomSet(np.full(n_geoms, POLYTOPE, np.int32), np.zeros((n_geoms, 4), np.float32), off, pts)


@dataclass
class Request:
    """One serving request: a scene batch over resident pool geometries."""
    arrival_s: float
    n_env: int
    body_offsets: np.ndarray
    body_geom: np.ndarray             # ids into the resident pool
    pose: np.ndarray
    want_bwd: bool
    seed: int


def serving_requests(n_requests: int = 2000, seed: int = 0, rate_hz: float = 10.0,
                     env_min: int = 1024, env_max: int = 65536, bodies_min: int = 2,
                     bodies_max: int = 16, pool_size: int = 256) -> list:
    """Poisson request stream over a resident polytope pool.

    Each request: n_env ~ log-uniform[1k, 64k] environments, 2..16 bodies per
    environment drawn from the pool, centres U[-1, 1]^3, uniform rotations,
    forward or forward+backward with probability 1/2.
    """
    rng = _rng(5, seed)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    arr = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n_requests):
        r2 = _rng(5, seed, 100 + i)
        n_env = int(np.round(np.exp(r2.uniform(np.log(env_min), np.log(env_max)))))
        nbe = r2.integers(bodies_min, bodies_max + 1, size=n_env)
        bo = np.zeros(n_env + 1, np.int64); bo[1:] = np.cumsum(nbe)
        nb = int(bo[-1])
        geo = r2.integers(0, pool_size, size=nb).astype(np.int32)
        q = uniform_quats(r2, nb)
        t = r2.uniform(-1.0, 1.0, size=(nb, 3))
        reqs.append(Request(float(arr[i]), n_env, bo.astype(np.int32), geo, _pose_array(q, t),
                            bool(r2.uniform() < 0.5), 100 + i))
    return reqs


def cotangents(n_pairs: int, K: int, seed: int = 0):
    """Random FP32 cotangents (a_k, b_k) for L = sum a_k w_k d_k + sum b_k . nu_k.

    Returns a[n_pairs*K] and b[3, n_pairs*K] (float32).
    """
    rng = _rng(6, seed)
    a = rng.standard_normal(n_pairs * K).astype(np.float32)
    b = rng.standard_normal((3, n_pairs * K)).astype(np.float32)
    return a, b


def edge_pairs(n: int, seed: int = 0) -> np.ndarray:
    """n edge pairs with endpoints uniform in the unit cube, float32 [n, 4, 3]
    (rows a0, a1, b0, b1): the queries of the witness-point speed experiment
    (Sec. V, Fig. 6)."""
    rng = _rng(7, seed)
    return rng.random((n, 4, 3), dtype=np.float32)


def subset_scenes(batch: Batch, scenes) -> Batch:
    """Batch restricted to the given scenes (geometry set kept whole)."""
    scenes = np.asarray(scenes, dtype=np.int64)
    bo = batch.body_offsets.astype(np.int64)
    bodies = np.concatenate([np.arange(bo[s], bo[s + 1]) for s in scenes]) if len(scenes) else np.zeros(0, np.int64)
    nbs = bo[scenes + 1] - bo[scenes]
    new_bo = np.zeros(len(scenes) + 1, np.int64); new_bo[1:] = np.cumsum(nbs)
    out = Batch(geoms=batch.geoms, body_offsets=new_bo.astype(np.int32),
                body_geom=batch.body_geom[bodies].copy(), pose=batch.pose[:, bodies].copy(),
                tau=batch.tau, K=batch.K, name=batch.name + "[subset]")
    if batch.cand_pairs is not None:
        remap = -np.ones(batch.n_bodies, np.int64)
        remap[bodies] = np.arange(len(bodies))
        co = batch.cand_offsets.astype(np.int64)
        sel = np.concatenate([np.arange(co[s], co[s + 1]) for s in scenes]) if len(scenes) else np.zeros(0, np.int64)
        ncs = co[scenes + 1] - co[scenes]
        new_co = np.zeros(len(scenes) + 1, np.int64); new_co[1:] = np.cumsum(ncs)
        out.cand_offsets = new_co.astype(np.int32)
        out.cand_pairs = remap[batch.cand_pairs[:, sel]].astype(np.int32)
    return out


# ----------------------------------------------------------------------------- superquadric unions

def sq_union_records(rng: np.random.Generator, n_prims: int = 18, spread=(0.4, 0.3, 0.55),
                     axes=(0.07, 0.16), eps=(0.3, 1.5)) -> np.ndarray:
    """One body as a union of superquadrics, packed 4 xyz rows per primitive.

    A stand-in for a decomposed articulated mesh: a torso primitive at the
    origin (semi-axes about 2x the others) and n_prims - 1 primitives whose
    centres are uniform in an ellipsoid of semi-axes ``spread``, semi-axes
    U[axes], exponents U[eps], uniform orientations.
    """
    M = int(n_prims)
    ax = rng.uniform(axes[0], axes[1], size=(M, 3))
    ax[0] *= 2.0
    e = rng.uniform(eps[0], eps[1], size=(M, 2))
    d = rng.standard_normal((M, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    t = d * rng.uniform(0.0, 1.0, size=(M, 1)) ** (1.0 / 3.0) * np.asarray(spread)[None, :]
    t[0] = 0.0
    q = uniform_quats(rng, M)
    rec = np.concatenate([ax, e, t, q], axis=1)           # a b c e1 e2 tx ty tz qw qx qy qz
    return rec.reshape(M * 4, 3).astype(np.float32)


def sq_scenes(n_scenes: int = 4096, seed: int = 0, tau: float = 0.01, K: int = 8, n_prims: int = 18,
              n_geoms: int = 8, bodies: int = 2, eps=(0.3, 1.5)) -> Batch:
    """Superquadric-union bodies (the paper's default primitive family):
    ``bodies`` per scene drawn from a pool of ``n_geoms`` unions of
    ``n_prims`` primitives (exponents U[eps]), centres uniform in a
    1.2-wide cube so that most pairs touch or overlap, uniform rotations."""
    rng = _rng(6, seed)
    recs = [sq_union_records(rng, n_prims, eps=eps) for _ in range(n_geoms)]
    gs = _geomset([SQ_UNION] * n_geoms, np.zeros((n_geoms, 4)), recs)
    nb = n_scenes * bodies
    body_geom = rng.integers(0, n_geoms, size=nb).astype(np.int32)
    t = rng.uniform(-0.6, 0.6, size=(nb, 3))
    q = uniform_quats(rng, nb)
    offs = (np.arange(n_scenes + 1) * bodies).astype(np.int32)
    return Batch(gs, offs, body_geom, _pose_array(q, t), tau, K, name="sq_scenes")


# ----------------------------------------------------------------------------- oriented point clouds

def opc_torus_records(rng: np.random.Generator, nu: int = 16, nv: int = 8) -> np.ndarray:
    """A torus (a non-convex surface) as an oriented point cloud: major radius
    U[0.25, 0.35], minor U[0.08, 0.14], nu x nv grid samples with their exact
    normals and bandwidth sigma = 0.5 x the minor-circle spacing; 3 xyz rows
    per point (position, normal, (sigma, 0, 0))."""
    R, r = rng.uniform(0.25, 0.35), rng.uniform(0.08, 0.14)
    u = 2 * np.pi * (np.arange(nu) + rng.uniform()) / nu
    v = 2 * np.pi * (np.arange(nv) + rng.uniform()) / nv
    U, V = np.meshgrid(u, v, indexing="ij")
    U, V = U.reshape(-1), V.reshape(-1)
    p = np.stack([(R + r * np.cos(V)) * np.cos(U), (R + r * np.cos(V)) * np.sin(U), r * np.sin(V)], axis=1)
    n = np.stack([np.cos(V) * np.cos(U), np.cos(V) * np.sin(U), np.sin(V)], axis=1)
    sg = np.full((len(p), 1), 0.5 * 2 * np.pi * r / nv)
    rec = np.concatenate([p, n, sg, np.zeros((len(p), 2))], axis=1)
    return rec.reshape(-1, 3).astype(np.float32)


def opc_scenes(n_scenes: int = 1024, seed: int = 0, tau: float = 0.01, K: int = 8, n_geoms: int = 4,
               nu: int = 16, nv: int = 8, with_analytic: bool = True) -> Batch:
    """Pairs of oriented-point-cloud tori (and, with_analytic, a sphere or
    rounded box as a third body) with centres U[-0.35, 0.35]^3 so that the
    tori interlock or touch, uniform rotations."""
    rng = _rng(8, seed)
    recs = [opc_torus_records(rng, nu, nv) for _ in range(n_geoms)]
    types = [OPC] * n_geoms + ([SPHERE, BOX] if with_analytic else [])
    params = [[0] * 4] * n_geoms + ([[0.12, 0, 0, 0], [0.1, 0.08, 0.12, BOX_ROUNDING]] if with_analytic else [])
    gs = _geomset(types, params, recs + ([None, None] if with_analytic else []))
    per = 3 if with_analytic else 2
    nb = n_scenes * per
    cols = [rng.integers(0, n_geoms, n_scenes), rng.integers(0, n_geoms, n_scenes)]
    if with_analytic:
        cols.append(rng.integers(n_geoms, n_geoms + 2, n_scenes))
    body_geom = np.stack(cols, axis=1).reshape(-1).astype(np.int32)
    t = rng.uniform(-0.35, 0.35, size=(nb, 3))
    q = uniform_quats(rng, nb)
    return Batch(gs, (np.arange(n_scenes + 1) * per).astype(np.int32), body_geom, _pose_array(q, t), tau, K,
                 name="opc_scenes")
