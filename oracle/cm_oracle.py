"""FP64 CPU oracle for smooth contact-manifold generation.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module; only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU
baseline leg use it.  It shares no code with the HIP library.

It is a plain, slow, obviously-correct transcription of the method of
"Smoothly Differentiable and Efficiently Vectorizable Contact Manifold
Generation" (arXiv 2602.20304) in float64 PyTorch CPU ops, one body pair at a
time.  Gradients come from PyTorch autograd of this forward (the analytic
gradient of exactly this function).

Sections of the paper followed (cited per function below):
  * Sec. III           smooth operators (sigmoid comparison, tanh sign,
                       softplus, softclip, soft argmin, LSE, SoftSort top-K)
  * Sec. IV-A          problem statement: poses in, K x (p, d, n) out
  * Sec. IV-B          SDF primitives (convex polyhedron = LSE over planes)
  * Sec. IV-C          vertex-SDF contacts
  * Sec. IV-D          E-E witness QP with L2 regularisation, analytic active
                       set, sign assignment, penetration / nearest-neighbour /
                       clashing indicators, activity indicator
  * Supp. C            smooth operator and E-E routine pseudo-code (used as a
                       description of what is computed, not transcribed)

Readings where the paper is silent or garbled:
  R1  unconstrained minimiser is -Q^{-1} c (the text drops the sign)
  R2  edge minimiser on alpha1 = 1 is -(Q12 + c2)/Q22 (text has a sign slip)
  R3  the cost of the (alpha1, 0) edge point is J evaluated there (the
      supplementary pseudo-code multiplies c1 by the wrong variable)
  R4  the second witness uses the reversed unsigned normal (-n_bar) for its
      sign test ("vice-versa"), so separated bodies give d1 = d2 = +d_bar
  R5  every soft temperature is tau; lambda = 0.01 absolute; eps_n = tau^2
  R6  V-S activity w = sigma(-d/tau) (the penetration test applied to vertices)
  R7  the fixed-size K manifold: score s = -d + tau log w, hard top-K values
      of s, SoftSort rows softmax(-|s_[k] - s_i| / tau) over all candidates
  R8  output normals use the pair convention (pointing from body A to body B)
  R9  analytic-body meshes: box = 8 corners / 12 edges; sphere = 26 vertices
      (poles + 3 latitude rings of 8) / 56 edges; capsule = 34 vertices / 72
      edges; all vertices on the exact surface
  R10 rounded box: outer half-extents h, rounding radius rho (exact SDF)
  R17 soft top-K pre-selection (Sec. IV-A overview, Supp. "picking the top-K
      numbers" and "safeguarding"): vertex metric = SDF of the other body at
      the vertex, edge metric = mean of its two corners' metrics; the same K_V
      and K_E for both bodies, clamped to each body's counts; the selection
      SoftSort uses tau and ranks -metric (deepest first); the optional
      safeguard multiplies both witnesses' activities by
      sigma(-phi_A(e1)/tau) sigma(-phi_B(e2)/tau)
  R11 V-S output normal grad(phi)/sqrt(tau + |grad(phi)|^2); sign and clash
      tests use the raw SDF gradient
  R12 broadphase (not in the paper): keep a pair iff its bounding spheres
      overlap within a margin (default 10 tau), defined in float32
  R18 superquadric unions (Sec. IV-B, SQ primitives and smooth union): a
      body is the smooth union -LSE_tau(-phi_i) of M superquadrics; each
      phi_i = |y| (1 - f(y)^(-eps1/2)) at its primitive-frame point y (the
      radial distance; the printed division by |x| would not be a length);
      E-E sign / clash tests use grad phi of the union, V-S normals the
      union's softmax mix of grad f_i (the footnote on SQ normals), normalised
      as in R11; mesh = per primitive a parametric grid (poles, rings at
      -60 / -30 / 0 / 30 / 60 deg of 6 longitudes, quads split by one
      diagonal: 32 vertices, 90 edges), minus
      the vertices strictly inside another primitive (f_j < 1) and their edges;
      a power of a coordinate that is exactly 0 has derivative 0 (its true
      derivative is infinite for exponents above 1, a kink like R13's)
  R19 witness sphere tracing (Supp., refinement of the witness points): each
      witness is moved along the fixed unit direction n = grad phi / |grad phi|
      of its own body's SDF at the QP witness (e1 on A, e2 on B) by
      x <- x - phi(x) n, a fixed number of steps; points, distances,
      normals and the sign, penetration and clashing tests then use the moved
      points, while the nearest-neighbour ranking keeps the QP distances
  R20 oriented point clouds (Sec. IV-B, OPC primitives): the radial basis is
      B_j(x - p_j; sigma_j) = exp(-|x - p_j|^2 / (2 sigma_j^2)) (the paper
      names the interpolant, not its kernel); normals are unit-normalised;
      the body's mesh is the point set with the edges of its 4-nearest-
      neighbour graph (ties by index); bound = max |p_j| + max sigma_j
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch
from scipy.spatial import ConvexHull

DT = torch.float64
SPHERE, CAPSULE, BOX, POLYTOPE, SQ_UNION, OPC = 0, 1, 2, 3, 4, 5
OPC_KNN = 4
LAMBDA_DEFAULT = 0.01


def _t(x, requires_grad=False):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=DT).clone().requires_grad_(requires_grad)


# ============================================================== Sec. III operators
# Each operator is its plain definition; logaddexp / logsumexp / softmax are the
# library routines for log(e^a + e^b), log sum exp and normalised exponentials.

def sigmoid(z):
    """Soft comparison [z > 0] ~ sigma(z) (Sec. III)."""
    return torch.sigmoid(z)


def log_sigmoid(z):
    """log sigma(z) = -log(1 + e^{-z})."""
    return -torch.logaddexp(torch.zeros_like(z), -z)


def softplus_t(x, tau):
    """s_+(x) = tau log(1 + exp(x / tau)) (Sec. III)."""
    return tau * torch.logaddexp(torch.zeros_like(x), x / tau)


def clip_s(x, lo, hi, tau):
    """Soft clip: lo + s_+(x - lo) - s_+(x - hi) (Sec. III)."""
    return lo + softplus_t(x - lo, tau) - softplus_t(x - hi, tau)


def within_s(x, lo, hi, tau):
    """Soft [lo <= x <= hi] as a product of two soft comparisons (Supp. C)."""
    return sigmoid((x - lo) / tau) * sigmoid((hi - x) / tau)


def log_within_s(x, lo, hi, tau):
    return log_sigmoid((x - lo) / tau) + log_sigmoid((hi - x) / tau)


def argmin_s(c, tau, dim=-1):
    """Soft argmin: softmax(-c / tau) (Sec. III)."""
    return torch.softmax(-c / tau, dim=dim)


def lse_t(y, tau, dim=-1):
    """LSE(y) = tau log sum exp(y / tau) (Sec. III)."""
    return tau * torch.logsumexp(y / tau, dim=dim)


def sign_s(x, tau):
    """Soft sign tanh(x / tau) (Sec. III)."""
    return torch.tanh(x / tau)


# ============================================================== geometry (Sec. IV-A/B)

def _ring_dirs(lat_deg: float):
    la = math.radians(lat_deg)
    return [(math.cos(la) * math.cos(2 * math.pi * j / 8), math.cos(la) * math.sin(2 * math.pi * j / 8),
             math.sin(la)) for j in range(8)]


def sphere_mesh_topology():
    """Reading R9: sphere mesh = south pole, rings at -45, 0, +45 deg, north pole.

    Returns unit directions [26, 3] and edges [56, 2].
    """
    dirs = [(0.0, 0.0, -1.0)] + _ring_dirs(-45) + _ring_dirs(0) + _ring_dirs(45) + [(0.0, 0.0, 1.0)]
    E = []
    rings = [1, 9, 17]
    for j in range(8):
        E.append((0, 1 + j))
    for r in rings:
        for j in range(8):
            E.append((r + j, r + (j + 1) % 8))
    for r0, r1 in ((1, 9), (9, 17)):
        for j in range(8):
            E.append((r0 + j, r1 + j))
    for j in range(8):
        E.append((17 + j, 25))
    return np.array(dirs), np.array(E, dtype=np.int64)


def capsule_mesh_topology():
    """Reading R9: capsule mesh = two hemispheres (pole, 45-deg ring, equator ring).

    Returns unit directions [34, 3], hemisphere side (+1 upper / -1 lower)
    [34] and edges [72, 2].  Vertex = r * dir + side * h * z.
    """
    dirs = [(0.0, 0.0, -1.0)] + _ring_dirs(-45) + _ring_dirs(0) + _ring_dirs(0) + _ring_dirs(45) + [(0.0, 0.0, 1.0)]
    side = [-1.0] * 17 + [1.0] * 17
    E = []
    for j in range(8):
        E.append((0, 1 + j))
    for r in (1, 9, 17, 25):
        for j in range(8):
            E.append((r + j, r + (j + 1) % 8))
    for r0, r1 in ((1, 9), (9, 17), (17, 25)):
        for j in range(8):
            E.append((r0 + j, r1 + j))
    for j in range(8):
        E.append((25 + j, 33))
    return np.array(dirs), np.array(side), np.array(E, dtype=np.int64)


def box_mesh_topology():
    """Reading R9: 8 corners (bit b of the index selects +h along axis b), 12 edges."""
    signs = np.array([[1.0 if (i >> a) & 1 else -1.0 for a in range(3)] for i in range(8)])
    E = [(i, i | bit) for bit in (1, 2, 4) for i in range(8) if not i & bit]
    return signs, np.array(E, dtype=np.int64)


def hull_topology(points: np.ndarray):
    """Convex hull of the polytope points (Qhull via scipy, a library step).

    Returns (vertex ids into points, sorted ascending), triangles [F, 3] as
    indices into that vertex list oriented counter-clockwise seen from
    outside, and unique edges [E, 2] (i < j).
    """
    P = np.asarray(points, dtype=np.float64)
    hull = ConvexHull(P)
    vid = np.array(sorted(hull.vertices.tolist()), dtype=np.int64)
    remap = -np.ones(len(P), dtype=np.int64)
    remap[vid] = np.arange(len(vid))
    tris = []
    for simp, eq in zip(hull.simplices, hull.equations):
        a, b, c = P[simp[0]], P[simp[1]], P[simp[2]]
        n = np.cross(b - a, c - a)
        if np.dot(n, eq[:3]) < 0:
            simp = simp[[0, 2, 1]]
        tris.append(remap[simp])
    tris = np.array(tris, dtype=np.int64)
    es = set()
    for t in tris:
        for i, j in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            es.add((min(i, j), max(i, j)))
    edges = np.array(sorted(es), dtype=np.int64)
    return vid, tris, edges


SQ_LON = 6
SQ_RINGS_DEG = (-60.0, -30.0, 0.0, 30.0, 60.0)


def sq_local_topology():
    """Reading R18: parametric samples (eta, omega) of one superquadric's mesh
    and its edges.  Local vertex 0 is the south pole, then the rings (6 each,
    omega = 2 pi j / 6), then the north pole; edges: pole spokes, ring edges,
    meridians between rings and one diagonal per quad (32 vertices, 90 edges).
    Poles are flagged with eta = +-pi/2 and placed exactly at (0, 0, +-c)."""
    samples = [(-math.pi / 2, 0.0)]
    for deg in SQ_RINGS_DEG:
        for j in range(SQ_LON):
            samples.append((math.radians(deg), 2 * math.pi * j / SQ_LON))
    samples.append((math.pi / 2, 0.0))
    nr = len(SQ_RINGS_DEG)
    ring = lambda r, j: 1 + r * SQ_LON + (j % SQ_LON)
    north = 1 + nr * SQ_LON
    E = [(0, ring(0, j)) for j in range(SQ_LON)]
    for r in range(nr):
        E += [(ring(r, j), ring(r, j + 1)) for j in range(SQ_LON)]
    for r in range(nr - 1):
        E += [(ring(r, j), ring(r + 1, j)) for j in range(SQ_LON)]
        E += [(ring(r, j), ring(r + 1, j + 1)) for j in range(SQ_LON)]
    E += [(ring(nr - 1, j), north) for j in range(SQ_LON)]
    return samples, np.array(E, dtype=np.int64)


def _spow(v, e):
    """sign(v) |v|^e (the superquadric's signed power), 0 at v = 0 with
    derivative 0 there (reading R18's convention for zero coordinates)."""
    nz = v != 0
    vs = torch.where(nz, v, torch.ones_like(v))
    return torch.where(nz, torch.sign(vs) * torch.abs(vs) ** e, torch.zeros_like(v))


def _ppow(v, p):
    """(v^2)^p, 0 at v = 0 with derivative 0 there (R18)."""
    nz = v != 0
    vs = torch.where(nz, v, torch.ones_like(v))
    return torch.where(nz, (vs * vs) ** p, torch.zeros_like(v))


def sq_unpack(rec):
    """Superquadric records [M, 12] -> axes [M, 3], eps1 [M], eps2 [M],
    rotation primitive -> body [M, 3, 3], translation [M, 3].  Record layout:
    a, b, c, eps1, eps2, tx, ty, tz, qw, qx, qy, qz (unit-normalised here)."""
    ax, e1, e2, t = rec[:, 0:3], rec[:, 3], rec[:, 4], rec[:, 5:8]
    q = rec[:, 8:12]
    q = q / torch.sqrt((q * q).sum(-1, keepdim=True))
    R = torch.stack([quat_to_R(q[i]) for i in range(q.shape[0])])
    return ax, e1, e2, R, t


def sq_inside_outside(y, ax, e1, e2):
    """Inside-outside function f and its gradient at primitive-frame points y
    [..., M, 3] (Sec. IV-B, SQ primitives): with scaled coordinates
    s = y / (a, b, c), f = ((s_x^2)^(1/eps2) + (s_y^2)^(1/eps2))^(eps2/eps1)
    + (s_z^2)^(1/eps1).  Powers of a zero coordinate are 0 and so are their
    derivatives there (R18), so autograd stays finite on the axis planes."""
    s = y / ax
    A = _ppow(s[..., 0], 1.0 / e2)
    B = _ppow(s[..., 1], 1.0 / e2)
    C = _ppow(s[..., 2], 1.0 / e1)
    u = A + B
    upos = u > 0
    us = torch.where(upos, u, torch.ones_like(u))
    f = torch.where(upos, us ** (e2 / e1), torch.zeros_like(u)) + C
    # d/ds (s^2)^p = 2 p sign(s) |s|^(2p - 1)
    dA = 2.0 / e2 * _spow(s[..., 0], 2.0 / e2 - 1.0)
    dB = 2.0 / e2 * _spow(s[..., 1], 2.0 / e2 - 1.0)
    dC = 2.0 / e1 * _spow(s[..., 2], 2.0 / e1 - 1.0)
    du = torch.where(upos, (e2 / e1) * us ** (e2 / e1 - 1.0), torch.zeros_like(u))
    g = torch.stack([du * dA / ax[..., 0], du * dB / ax[..., 1], dC / ax[..., 2]], dim=-1)
    return f, g


def sq_union_sdf(rec, x, tau):
    """Smooth union of superquadrics at body-frame points x [..., 3]
    (Sec. IV-B; reading R18).  Returns phi, grad phi and the V-S normal
    direction sum_i pi_i grad f_i, pi = softmax(-phi_i / tau)."""
    ax, e1, e2, R, t = sq_unpack(rec)
    y = ((x[..., None, :] - t)[..., None, :] @ R).squeeze(-2)        # y_i = R_i^T (x - t_i)
    f, gf = sq_inside_outside(y, ax, e1, e2)
    r = torch.sqrt((y * y).sum(-1))
    q = f ** (-e1 / 2.0)
    phi_i = r * (1.0 - q)
    gphi = (1.0 - q)[..., None] * y / r[..., None] + (r * (e1 / 2.0) * q / f)[..., None] * gf
    phi = -lse_t(-phi_i, tau, dim=-1)
    pi = torch.softmax(-phi_i / tau, dim=-1)
    to_body = lambda v: (R @ v[..., None]).squeeze(-1)                   # R_i v_i
    grad = (pi[..., None] * to_body(gphi)).sum(-2)
    ndir = (pi[..., None] * to_body(gf)).sum(-2)
    return phi, grad, ndir


def sq_union_mesh(rec_np):
    """Mesh of a superquadric union (reading R18): per primitive the
    parametric grid of sq_local_topology, minus vertices strictly inside
    another primitive and the edges touching them.  Returns the kept
    (primitive, local sample) list and edges [E, 2] over the kept vertices."""
    rec = torch.as_tensor(np.asarray(rec_np, dtype=np.float64))
    M = rec.shape[0]
    samples, le = sq_local_topology()
    pts = sq_points(rec, [(i, k) for i in range(M) for k in range(len(samples))]).numpy()
    ax, e1, e2, R, t = sq_unpack(rec)
    n = len(samples)
    keep = []
    for i in range(M):
        for k in range(n):
            x = torch.as_tensor(pts[i * n + k])
            y = ((x - t)[:, None, :] @ R).squeeze(-2)
            f, _ = sq_inside_outside(y, ax, e1, e2)
            inside = [(j != i) and bool(f[j] < 1.0) for j in range(M)]
            if not any(inside):
                keep.append((i, k))
    index = {v: j for j, v in enumerate(keep)}
    E = []
    for i in range(M):
        for a, b in le:
            if (i, a) in index and (i, b) in index:
                E.append((index[(i, a)], index[(i, b)]))
    return keep, np.array(E, dtype=np.int64).reshape(-1, 2)


def sq_points(rec, which):
    """Body-frame positions of parametric samples (primitive, local index):
    (a C(eta)^eps1 C(omega)^eps2, b C(eta)^eps1 S(omega)^eps2, c S(eta)^eps1)
    with signed powers, rotated and translated by the primitive's pose."""
    samples, _ = sq_local_topology()
    ax, e1, e2, R, t = sq_unpack(rec)
    out = []
    for i, k in which:
        eta, om = samples[k]
        if abs(eta) == math.pi / 2:
            c = torch.stack([ax[i, 0] * 0.0, ax[i, 1] * 0.0, ax[i, 2] * (1.0 if eta > 0 else -1.0)])
        else:
            ce, se = torch.tensor(math.cos(eta), dtype=DT), torch.tensor(math.sin(eta), dtype=DT)
            co, so = torch.tensor(math.cos(om), dtype=DT), torch.tensor(math.sin(om), dtype=DT)
            c = torch.stack([ax[i, 0] * _spow(ce, e1[i]) * _spow(co, e2[i]),
                             ax[i, 1] * _spow(ce, e1[i]) * _spow(so, e2[i]),
                             ax[i, 2] * _spow(se, e1[i])])
        out.append(R[i] @ c + t[i])
    return torch.stack(out)


def opc_unpack(rec):
    """Oriented point records [N, 9] (p, n, sigma, 0, 0) -> p [N, 3], unit
    n [N, 3], sigma [N]."""
    p, n, sg = rec[:, 0:3], rec[:, 3:6], rec[:, 6]
    return p, n / torch.sqrt((n * n).sum(-1, keepdim=True)), sg


def opc_sdf(rec, x):
    """Radial-basis SDF of an oriented point cloud at body-frame points x
    [..., 3] (Sec. IV-B, OPC primitives; reading R20):
    phi = sum_j B_j n_j . (x - p_j) / sum_j B_j with Gaussian B_j, and its
    gradient by the quotient rule."""
    p, n, sg = opc_unpack(rec)
    d = x[..., None, :] - p                                   # [..., N, 3]
    h = (d * n).sum(-1)                                       # n_j . (x - p_j)
    lb = -(d * d).sum(-1) / (2.0 * sg * sg)                   # log B_j
    w = torch.softmax(lb, dim=-1)                             # B_j / sum B
    phi = (w * h).sum(-1)
    dlb = -d / (sg * sg)[:, None]                             # grad log B_j
    grad = (w[..., None] * (n + dlb * (h - phi[..., None])[..., None])).sum(-2)
    return phi, grad


def opc_knn_edges(p_np, k=OPC_KNN):
    """Edges of the k-nearest-neighbour graph of the points (R20): i -- j
    when j is among the k nearest of i (squared distances, ties by the lower
    index), undirected, unique, sorted."""
    P = np.asarray(p_np, dtype=np.float64)
    es = set()
    for i in range(len(P)):
        d2 = ((P - P[i]) ** 2).sum(-1)
        d2[i] = np.inf
        order = sorted(range(len(P)), key=lambda j: (d2[j], j))[:min(k, len(P) - 1)]
        for j in order:
            es.add((min(i, j), max(i, j)))
    return np.array(sorted(es), dtype=np.int64).reshape(-1, 2)


@dataclass
class OGeom:
    """Oracle geometry: type, differentiable parameters and mesh topology.

    ``params`` (analytic) or ``points`` (polytope, hull vertices only) are
    float64 leaf tensors; the mesh vertices and face planes are functions of
    them, so autograd reaches the geometry parameters.
    """
    kind: int
    params: Optional[torch.Tensor] = None   # [4]
    points: Optional[torch.Tensor] = None   # [V, 3] hull vertices (polytope)
    vertex_ids: Optional[np.ndarray] = None # input point index of each hull vertex
    edges: Optional[np.ndarray] = None      # [E, 2]
    tris: Optional[np.ndarray] = None       # [F, 3]
    _aux: Optional[np.ndarray] = None
    sq: Optional[torch.Tensor] = None       # [M, 12] superquadric records (SQ_UNION)
    opc: Optional[torch.Tensor] = None      # [N, 9] oriented point records (OPC)

    def vertices(self) -> torch.Tensor:
        """Mesh vertices in the body frame (Sec. IV-A: every surface has a mesh)."""
        if self.kind == POLYTOPE:
            return self.points
        if self.kind == SQ_UNION:
            return sq_points(self.sq, self._aux)
        if self.kind == OPC:
            return self.opc[:, 0:3]
        p = self.params
        if self.kind == SPHERE:
            return p[0] * _t(self._aux)
        if self.kind == CAPSULE:
            dirs, side = self._aux
            return p[0] * _t(dirs) + p[1] * _t(side)[:, None] * _t([0.0, 0.0, 1.0])[None, :]
        if self.kind == BOX:
            return _t(self._aux) * p[:3][None, :]
        raise ValueError(self.kind)

    def planes(self):
        """Outward unit face normals n_f and offsets o_f = n_f . v (Sec. IV-B, CP)."""
        V = self.points
        t = torch.as_tensor(self.tris)
        v0, v1, v2 = V[t[:, 0]], V[t[:, 1]], V[t[:, 2]]
        n = torch.linalg.cross(v1 - v0, v2 - v0)
        n = n / torch.sqrt((n * n).sum(-1, keepdim=True))
        o = (n * v0).sum(-1)
        return n, o


def make_geom(kind: int, params=None, points=None, requires_grad=False) -> OGeom:
    if kind == OPC:
        rec = np.asarray(points, dtype=np.float64).reshape(-1, 9)
        return OGeom(kind, params=_t(np.zeros(4)), edges=opc_knn_edges(rec[:, 0:3]), opc=_t(rec, requires_grad))
    if kind == SQ_UNION:
        rec = np.asarray(points, dtype=np.float64).reshape(-1, 12)
        keep, edges = sq_union_mesh(rec)
        return OGeom(kind, params=_t(np.zeros(4)), edges=edges, _aux=keep, sq=_t(rec, requires_grad))
    if kind == POLYTOPE:
        vid, tris, edges = hull_topology(points)
        pts = _t(np.asarray(points, dtype=np.float64)[vid], requires_grad)
        return OGeom(kind, points=pts, vertex_ids=vid, edges=edges, tris=tris)
    prm = _t(np.asarray(params, dtype=np.float64)[:4], requires_grad)
    if kind == SPHERE:
        dirs, edges = sphere_mesh_topology()
        return OGeom(kind, params=prm, edges=edges, _aux=dirs)
    if kind == CAPSULE:
        dirs, side, edges = capsule_mesh_topology()
        return OGeom(kind, params=prm, edges=edges, _aux=(dirs, side))
    if kind == BOX:
        signs, edges = box_mesh_topology()
        return OGeom(kind, params=prm, edges=edges, _aux=signs)
    raise ValueError(kind)


def geom_from_set(gs, g: int, requires_grad=False) -> OGeom:
    return make_geom(int(gs.types[g]), params=gs.params[g], points=gs.points_of(g), requires_grad=requires_grad)


def _sgn(x):
    return torch.where(x >= 0, torch.ones_like(x), -torch.ones_like(x))


def sdf_local(G: OGeom, x: torch.Tensor, tau, planes=None, chunk: int = 1 << 22, with_ndir=False):
    """Smooth SDF phi and its gradient at body-frame points x [..., 3]
    (and with_ndir: the V-S normal direction, the gradient itself except for
    superquadric unions, reading R18).

    sphere  |x| - r
    capsule |x - clamp(x_z, -h, h) z| - r
    box     rounded box with outer half-extents h and rounding rho (R10)
    polytope LSE_tau over face planes n_f . x - o_f (Sec. IV-B, CP primitive);
             gradient = softmax-weighted sum of face normals.
    """
    if G.kind == SQ_UNION:
        phi, g, nd = sq_union_sdf(G.sq, x, tau)
        return (phi, g, nd) if with_ndir else (phi, g)
    if G.kind == OPC:
        phi, g = opc_sdf(G.opc, x)
        return (phi, g, g) if with_ndir else (phi, g)
    if with_ndir:
        phi, g = sdf_local(G, x, tau, planes, chunk)
        return phi, g, g
    if G.kind == SPHERE:
        nrm = torch.sqrt((x * x).sum(-1))
        return nrm - G.params[0], x / nrm[..., None]
    if G.kind == CAPSULE:
        r, h = G.params[0], G.params[1]
        zc = torch.minimum(torch.maximum(x[..., 2], -h), h)
        y = torch.stack([x[..., 0], x[..., 1], x[..., 2] - zc], dim=-1)
        nrm = torch.sqrt((y * y).sum(-1))
        return nrm - r, y / nrm[..., None]
    if G.kind == BOX:
        h, rho = G.params[:3], G.params[3]
        q = torch.abs(x) - (h - rho)
        qp = torch.clamp(q, min=0.0)
        s = (qp * qp).sum(-1)
        outside = (q > 0).any(-1)
        n_out = torch.sqrt(torch.where(outside, s, torch.ones_like(s)))
        qmax, jmax = q.max(-1)
        phi = torch.where(outside, n_out, torch.zeros_like(s)) + torch.clamp(qmax, max=0.0) - rho
        g_out = _sgn(x) * qp / n_out[..., None]
        g_in = _sgn(x) * torch.nn.functional.one_hot(jmax, 3).to(DT)
        g = torch.where(outside[..., None], g_out, g_in)
        return phi, g
    if G.kind == POLYTOPE:
        n, o = planes if planes is not None else G.planes()
        shp = x.shape[:-1]
        xf = x.reshape(-1, 3)
        F = n.shape[0]
        step = max(1, chunk // max(F, 1))
        phis, grads = [], []
        for i in range(0, xf.shape[0], step):
            y = xf[i:i + step] @ n.T - o[None, :]
            phis.append(lse_t(y, tau, dim=-1))
            grads.append(torch.softmax(y / tau, dim=-1) @ n)
        if not phis:
            return xf.new_zeros(shp), xf.new_zeros(shp + (3,))
        return torch.cat(phis).reshape(shp), torch.cat(grads).reshape(shp + (3,))
    raise ValueError(G.kind)


# ============================================================== poses (Sec. IV-A)

def quat_to_R(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of a (w, x, y, z) quaternion after normalisation."""
    q = q / torch.sqrt((q * q).sum())
    w, x, y, z = q[0], q[1], q[2], q[3]
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)]),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)]),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]),
    ])


def hat(w):
    z = torch.zeros((), dtype=DT)
    return torch.stack([torch.stack([z, -w[2], w[1]]), torch.stack([w[2], z, -w[0]]),
                        torch.stack([-w[1], w[0], z])])


def so3_exp(w):
    th = torch.sqrt((w * w).sum())
    if float(th) < 1e-12:
        return torch.eye(3, dtype=DT) + hat(w)
    K = hat(w / th)
    return torch.eye(3, dtype=DT) + torch.sin(th) * K + (1 - torch.cos(th)) * (K @ K)


def se3_exp(xi):
    """Exp of a twist (rho, omega) -> (R, t) with t = V(omega) rho."""
    rho, w = xi[:3], xi[3:]
    th = torch.sqrt((w * w).sum())
    R = so3_exp(w)
    if float(th) < 1e-12:
        V = torch.eye(3, dtype=DT) + 0.5 * hat(w)
    else:
        K = hat(w / th)
        V = torch.eye(3, dtype=DT) + (1 - torch.cos(th)) / th * K + (th - torch.sin(th)) / th * (K @ K)
    return R, V @ rho


def pose_Rt(pose7, xi=None, exact=False):
    """(R, t) of a pose given as (qw, qx, qy, qz, tx, ty, tz).

    With a twist xi = (rho, omega) the pose is left-perturbed, T' = Exp(xi) T.
    ``exact=False`` uses the first-order form (I + [omega]x) which has the same
    derivative at xi = 0 (used with autograd); ``exact=True`` uses Exp (used
    for finite differences).
    """
    p = torch.as_tensor(np.asarray(pose7, dtype=np.float64), dtype=DT)
    R = quat_to_R(p[:4])
    t = p[4:7]
    if xi is None:
        return R, t
    if exact:
        Rx, tx = se3_exp(xi)
        return Rx @ R, Rx @ t + tx
    W = hat(xi[3:])
    return R + W @ R, t + xi[:3] + W @ t


# ============================================================== one body pair

def sdf_world(G: OGeom, R, t, X, tau, planes=None, with_ndir=False):
    """phi_G and grad phi_G (world frame) at world points X [..., 3] (and
    with_ndir: the V-S normal direction, reading R18)."""
    xl = (X - t) @ R
    if with_ndir:
        phi, gl, nl = sdf_local(G, xl, tau, planes, with_ndir=True)
        return phi, gl @ R.T, nl @ R.T
    phi, gl = sdf_local(G, xl, tau, planes)
    return phi, gl @ R.T


def _dot(u, v):
    return (u * v).sum(-1)


def ee_qp(a0, a1, b0, b1, tau, lam=LAMBDA_DEFAULT):
    """Smoothed analytic active-set solution of the regularised E-E QP (Sec. IV-D-2).

    Edges e1(al1) = a0 + al1 (a1 - a0), e2(al2) = b0 + al2 (b1 - b0); objective
    |e1 - e2|^2 + lam [(al1 - 1/2)^2 + (al2 - 1/2)^2], written (up to a constant
    and a factor 2) as J(al) = 1/2 al^T Q al + c^T al with A = [t1, -t2],
    b = a0 - b0, Q = A^T A + lam I, c = A^T b - lam/2 (1, 1).
    Steps: (i) unconstrained minimiser, (ii) the four soft-clipped box-edge
    minimisers blended by a soft argmin of their costs, (iii) soft indicator
    that the unconstrained minimiser is inside [0,1]^2, (iv) blend.
    Broadcasts over leading dimensions.
    """
    t1 = a1 - a0
    t2 = b1 - b0
    bv = a0 - b0
    Q11 = _dot(t1, t1) + lam
    Q12 = -_dot(t1, t2)
    Q22 = _dot(t2, t2) + lam
    c1 = _dot(bv, t1) - 0.5 * lam
    c2 = -_dot(bv, t2) - 0.5 * lam
    Q11, Q12, Q22, c1, c2 = torch.broadcast_tensors(Q11, Q12, Q22, c1, c2)

    def J(x1, x2):
        q11, q12, q22, k1, k2 = (v[..., None] for v in (Q11, Q12, Q22, c1, c2))
        return 0.5 * (q11 * x1 * x1 + 2.0 * q12 * x1 * x2 + q22 * x2 * x2) + k1 * x1 + k2 * x2

    # (i) unconstrained minimiser al_u = -Q^{-1} c   (reading R1)
    det = Q11 * Q22 - Q12 * Q12
    au1 = (-c1 * Q22 + Q12 * c2) / det
    au2 = (-c2 * Q11 + Q12 * c1) / det
    # (ii) minimisers along the four box edges, soft-clipped (reading R2)
    one, zero = torch.ones_like(Q12), torch.zeros_like(Q12)
    x_a = clip_s(-(Q12 + c2) / Q22, 0.0, 1.0, tau)     # on al1 = 1
    x_b = clip_s(-c2 / Q22, 0.0, 1.0, tau)             # on al1 = 0
    x_c = clip_s(-(Q12 + c1) / Q11, 0.0, 1.0, tau)     # on al2 = 1
    x_d = clip_s(-c1 / Q11, 0.0, 1.0, tau)             # on al2 = 0
    cand1 = torch.stack([one, zero, x_c, x_d], dim=-1)
    cand2 = torch.stack([x_a, x_b, one, zero], dim=-1)
    costs = J(cand1, cand2)                              # (reading R3)
    pi = argmin_s(costs, tau, dim=-1)
    ac1 = (pi * cand1).sum(-1)
    ac2 = (pi * cand2).sum(-1)
    # (iii) soft indicator that al_u is inside the box; (iv) blend
    con = within_s(au1, 0.0, 1.0, tau) * within_s(au2, 0.0, 1.0, tau)
    log_con = log_within_s(au1, 0.0, 1.0, tau) + log_within_s(au2, 0.0, 1.0, tau)
    al1 = con * au1 + (1.0 - con) * ac1
    al2 = con * au2 + (1.0 - con) * ac2
    return dict(al1=al1, al2=al2, au1=au1, au2=au2, con=con, log_con=log_con, costs=costs)


def ee_qp_hard(a0, a1, b0, b1, lam=LAMBDA_DEFAULT):
    """The E-E QP without smoothing (Ours-NS of the witness-point experiment, Sec. V, Fig. 6).

    With lam > 0 the objective is strictly convex, so its minimiser over the
    box [0,1]^2 is unique: the unconstrained minimiser when it lies in the
    box, otherwise the best of the minimisers along the four box edges (each a
    one-dimensional convex quadratic, minimised by clamping its stationary
    point to [0, 1]).  Ties go to the lower edge index (order: al1 = 1,
    al1 = 0, al2 = 1, al2 = 0).  Returns al1, al2 and con (1 inside, 0 not).
    """
    t1 = a1 - a0
    t2 = b1 - b0
    bv = a0 - b0
    Q11 = _dot(t1, t1) + lam
    Q12 = -_dot(t1, t2)
    Q22 = _dot(t2, t2) + lam
    c1 = _dot(bv, t1) - 0.5 * lam
    c2 = -_dot(bv, t2) - 0.5 * lam
    Q11, Q12, Q22, c1, c2 = torch.broadcast_tensors(Q11, Q12, Q22, c1, c2)
    det = Q11 * Q22 - Q12 * Q12
    au1 = (-c1 * Q22 + Q12 * c2) / det
    au2 = (-c2 * Q11 + Q12 * c1) / det
    inside = (au1 >= 0) & (au1 <= 1) & (au2 >= 0) & (au2 <= 1)
    one, zero = torch.ones_like(Q12), torch.zeros_like(Q12)
    cand1 = torch.stack([one, zero, torch.clamp(-(Q12 + c1) / Q11, 0.0, 1.0),
                         torch.clamp(-c1 / Q11, 0.0, 1.0)], dim=-1)
    cand2 = torch.stack([torch.clamp(-(Q12 + c2) / Q22, 0.0, 1.0), torch.clamp(-c2 / Q22, 0.0, 1.0),
                         one, zero], dim=-1)
    x1, x2 = cand1, cand2
    q11, q12, q22, k1, k2 = (v[..., None] for v in (Q11, Q12, Q22, c1, c2))
    costs = 0.5 * (q11 * x1 * x1 + 2.0 * q12 * x1 * x2 + q22 * x2 * x2) + k1 * x1 + k2 * x2
    best = torch.argmin(costs, dim=-1, keepdim=True)    # first index of the minimum
    b1_ = torch.gather(cand1, -1, best)[..., 0]
    b2_ = torch.gather(cand2, -1, best)[..., 0]
    al1 = torch.where(inside, au1, b1_)
    al2 = torch.where(inside, au2, b2_)
    return dict(al1=al1, al2=al2, con=inside.to(al1.dtype), costs=costs)


def ee_witness_batch(edges, tau, lam=LAMBDA_DEFAULT, hard=False):
    """Witness points of independent edge pairs (Sec. IV-D-2, IV-D-3): the
    shape of the paper's witness-point vectorisation experiment (Sec. V, Fig. 6).

    edges: [n, 4, 3] rows a0, a1, b0, b1.  Returns float64 numpy arrays al1,
    al2, con [n] and e1, e2 [n, 3].
    """
    e = torch.as_tensor(np.asarray(edges, dtype=np.float64))
    a0, a1, b0, b1 = e[:, 0], e[:, 1], e[:, 2], e[:, 3]
    with torch.no_grad():
        q = ee_qp_hard(a0, a1, b0, b1, lam) if hard else ee_qp(a0, a1, b0, b1, tau, lam)
        e1, e2, _, _ = ee_witness(a0, a1, b0, b1, q["al1"], q["al2"], 1.0)
    return dict(al1=q["al1"].numpy(), al2=q["al2"].numpy(), con=q["con"].numpy(), e1=e1.numpy(), e2=e2.numpy())


def ee_witness(a0, a1, b0, b1, al1, al2, eps_n):
    """Witness points, unsigned distance and unsigned normal (Sec. IV-D-3).

    e_b = edge_b(al_b); de = e1 - e2; d_bar = |de|; n_bar = de / sqrt(|de|^2 + eps).
    """
    e1 = a0 + al1[..., None] * (a1 - a0)
    e2 = b0 + al2[..., None] * (b1 - b0)
    de = e1 - e2
    dsq = _dot(de, de)
    return e1, e2, torch.sqrt(dsq), de / torch.sqrt(dsq + eps_n)[..., None]


def ee_sign(gA_e1, gB_e2, nbar, tau):
    """Soft signs of the two witnesses (Sec. IV-D-3, reading R4).

    gamma1 = softsign(grad phi_B(e2) . n_bar), gamma2 = softsign(grad phi_A(e1) . (-n_bar)).
    """
    return sign_s(_dot(gB_e2, nbar), tau), sign_s(_dot(gA_e1, -nbar), tau)


def vs_normal(g, tau):
    """V-S normal grad(phi) / sqrt(tau + |grad(phi)|^2) (Sec. IV-B, reading R11)."""
    return g / torch.sqrt(tau + _dot(g, g))[..., None]


def nn_log_indicators(dbar, tau):
    """log of the nearest-neighbour soft indicators (eq. nn_check).

    Row-wise soft argmin over l of -D[k, :] / tau and column-wise over k.
    """
    return torch.log_softmax(-dbar / tau, dim=1), torch.log_softmax(-dbar / tau, dim=0)


def soft_topk(x, K: int, tau):
    """SoftSort soft top-K (Sec. III): Gamma [K, D] with rows
    softmax_i(-|x_[k] - x_i| / tau), x_[k] the k-th largest entry of x."""
    top = torch.topk(x, K, sorted=True).values
    return torch.softmax(-torch.abs(top[:, None] - x[None, :]) / tau, dim=1)


def preselect(GA, RA, tA, GB, RB, tB, tau, KV: int, KE: int, planesA=None, planesB=None):
    """Soft top-K pre-selection of vertices and edges (Sec. IV-A overview;
    Supp. on picking the top-K numbers and on safeguarding; reading R17).

    Every vertex gets the SDF of the other body at it as its penetration
    metric, every edge the mean of its corners' metrics; the K_V deepest
    vertices and K_E deepest edges of each body are selected by SoftSort
    rows over -metric, and the selected points are the Gamma-weighted
    averages of the vertex positions (of the edge endpoints).  Returns world
    arrays: soft vertices of A [KV_A, 3] and B, soft edge endpoints of A
    (a0 [KE_A, 3], a1) and of B (b0, b1).
    """
    vA = GA.vertices() @ RA.T + tA
    vB = GB.vertices() @ RB.T + tB
    mA, _ = sdf_world(GB, RB, tB, vA, tau, planesB)
    mB, _ = sdf_world(GA, RA, tA, vB, tau, planesA)
    eA, eB = GA.edges, GB.edges
    meA = 0.5 * (mA[eA[:, 0]] + mA[eA[:, 1]])
    meB = 0.5 * (mB[eB[:, 0]] + mB[eB[:, 1]])
    GvA = soft_topk(-mA, min(KV, vA.shape[0]), tau)
    GvB = soft_topk(-mB, min(KV, vB.shape[0]), tau)
    GeA = soft_topk(-meA, min(KE, eA.shape[0]), tau)
    GeB = soft_topk(-meB, min(KE, eB.shape[0]), tau)
    return (GvA @ vA, GvB @ vB, GeA @ vA[eA[:, 0]], GeA @ vA[eA[:, 1]], GeB @ vB[eB[:, 0]], GeB @ vB[eB[:, 1]])


def sphere_trace(G, R, t, x, tau, planes, steps: int):
    """Refinement of witness points onto the smoothed surface of the body
    they belong to (Supp., sphere tracing; reading R19): along the fixed unit
    direction n of grad phi at the start, x <- x - phi(x) n, `steps` times.
    For a metric SDF one step lands on the surface."""
    _, g = sdf_world(G, R, t, x, tau, planes)
    n = g / torch.sqrt(_dot(g, g))[..., None]
    for _ in range(steps):
        phi, _ = sdf_world(G, R, t, x, tau, planes)
        x = x - phi[..., None] * n
    return x


def pair_candidates(GA: OGeom, RA, tA, GB: OGeom, RB, tB, tau, lam=LAMBDA_DEFAULT, eps_n=None, no_ee=False,
                    one_sided_vs=False, presel=None, safeguard=False, refine=0):
    """All contact candidates of one body pair (A, B) in world coordinates.

    Returns dict of p [C,3], nu [C,3] (pair convention, A -> B), d [C],
    logw [C] with the candidate order: A's vertices, B's vertices, then E-E
    pairs (k, l) row-major with witness 1 before witness 2.  no_ee drops the
    E-E candidates and one_sided_vs B's vertices (the paper's simplifications,
    supplementary material).  presel = (K_V, K_E): the candidates are built
    from the soft pre-selected vertices and edges instead (preselect), and
    safeguard scales the E-E activities by the inside indicators (R17).
    """
    if eps_n is None:
        eps_n = tau * tau
    planesA = GA.planes() if GA.kind == POLYTOPE else None
    planesB = GB.planes() if GB.kind == POLYTOPE else None
    vA = GA.vertices() @ RA.T + tA
    vB = GB.vertices() @ RB.T + tB
    eA, eB = GA.edges, GB.edges
    a0, a1 = vA[eA[:, 0]][:, None, :], vA[eA[:, 1]][:, None, :]
    b0, b1 = vB[eB[:, 0]][None, :, :], vB[eB[:, 1]][None, :, :]
    if presel is not None:
        vA, vB, sa0, sa1, sb0, sb1 = preselect(GA, RA, tA, GB, RB, tB, tau, presel[0], presel[1], planesA, planesB)
        a0, a1, b0, b1 = sa0[:, None, :], sa1[:, None, :], sb0[None, :, :], sb1[None, :, :]

    # ---- vertex-SDF contacts (Sec. IV-C; normals R11; weights R6)
    phiB_v, _, gB_v = sdf_world(GB, RB, tB, vA, tau, planesB, with_ndir=True)
    phiA_v, _, gA_v = sdf_world(GA, RA, tA, vB, tau, planesA, with_ndir=True)
    vs_p = torch.cat([vA, vB])
    vs_nu = torch.cat([-vs_normal(gB_v, tau), vs_normal(gA_v, tau)])   # pair convention (R8)
    vs_d = torch.cat([phiB_v, phiA_v])
    vs_logw = log_sigmoid(-vs_d / tau)

    # ---- edge-edge contacts over all |E_A| x |E_B| edge pairs (Sec. IV-D)
    qp = ee_qp(a0, a1, b0, b1, tau, lam)
    e1, e2, dbar, nbar = ee_witness(a0, a1, b0, b1, qp["al1"], qp["al2"], eps_n)
    dbar_nn = dbar
    if refine:
        # witnesses traced onto their own bodies' smoothed surfaces (R19)
        e1 = sphere_trace(GA, RA, tA, e1, tau, planesA, refine)
        e2 = sphere_trace(GB, RB, tB, e2, tau, planesB, refine)
        de = e1 - e2
        dsq = _dot(de, de)
        dbar = torch.sqrt(dsq)
        nbar = de / torch.sqrt(dsq + eps_n)[..., None]

    # SDF queries at the witness points
    phiB_e1, _ = sdf_world(GB, RB, tB, e1, tau, planesB)
    _, gA_e1 = sdf_world(GA, RA, tA, e1, tau, planesA)
    phiA_e2, _ = sdf_world(GA, RA, tA, e2, tau, planesA)
    _, gB_e2 = sdf_world(GB, RB, tB, e2, tau, planesB)

    gam1, gam2 = ee_sign(gA_e1, gB_e2, nbar, tau)
    d1, d2 = gam1 * dbar, gam2 * dbar
    n1 = gam1[..., None] * nbar           # pushes A away from B
    n2 = gam2[..., None] * (-nbar)        # pushes B away from A
    # penetration (eq. sdf_check), clashing, nearest neighbours (eq. nn_check)
    log_pen1 = log_sigmoid(-phiB_e1 / tau)
    log_pen2 = log_sigmoid(-phiA_e2 / tau)
    log_cl = log_sigmoid(-_dot(gA_e1, gB_e2) / tau)
    log_nn1, log_nn2 = nn_log_indicators(dbar_nn, tau)
    # activity indicator Gamma_b = con * pen_b * nn_b * cl, in the log domain
    logG1 = qp["log_con"] + log_pen1 + log_nn1 + log_cl
    logG2 = qp["log_con"] + log_pen2 + log_nn2 + log_cl
    if safeguard:
        # both averaged edges must lie inside their own bodies (R17)
        phiA_e1, _ = sdf_world(GA, RA, tA, e1, tau, planesA)
        phiB_e2, _ = sdf_world(GB, RB, tB, e2, tau, planesB)
        log_sg = log_sigmoid(-phiA_e1 / tau) + log_sigmoid(-phiB_e2 / tau)
        logG1 = logG1 + log_sg
        logG2 = logG2 + log_sg

    ee_p = torch.stack([e1, e2], dim=2).reshape(-1, 3)
    ee_nu = torch.stack([-n1, n2], dim=2).reshape(-1, 3)   # pair convention (R8)
    ee_d = torch.stack([d1, d2], dim=2).reshape(-1)
    ee_logw = torch.stack([logG1, logG2], dim=2).reshape(-1)
    nA = vA.shape[0]
    if one_sided_vs:
        vs_p, vs_nu, vs_d, vs_logw = vs_p[:nA], vs_nu[:nA], vs_d[:nA], vs_logw[:nA]
    if no_ee:
        ee_p, ee_nu, ee_d, ee_logw = ee_p[:0], ee_nu[:0], ee_d[:0], ee_logw[:0]
    out = dict(p=torch.cat([vs_p, ee_p]), nu=torch.cat([vs_nu, ee_nu]),
               d=torch.cat([vs_d, ee_d]), logw=torch.cat([vs_logw, ee_logw]))
    out["extra"] = dict(qp=qp, dbar=dbar, e1=e1, e2=e2, gam1=gam1, gam2=gam2, log_pen1=log_pen1,
                        log_pen2=log_pen2, log_cl=log_cl, log_nn1=log_nn1, log_nn2=log_nn2,
                        n_vs=vs_d.shape[0])
    return out


def manifold(c, tau, K: int):
    """Fixed-size K-contact manifold from candidates (reading R7, SoftSort Sec. III).

    s_i = -d_i + tau log w_i; s_[1] >= ... >= s_[K] the K largest scores;
    Gamma_ki = softmax_i(-|s_[k] - s_i| / tau); outputs are Gamma @ (p, nu, d, w).
    With fewer than K candidates the remaining rows are empty: zero point,
    normal, distance and weight (reading R15).
    """
    s = -c["d"] + tau * c["logw"]
    n = s.shape[0]
    k = min(K, n)
    top = torch.topk(s, k, sorted=True).values
    G = torch.softmax(-torch.abs(top[:, None] - s[None, :]) / tau, dim=1)
    w = torch.exp(c["logw"])
    out = dict(p=G @ c["p"], nu=G @ c["nu"], d=G @ c["d"], w=G @ w, s_top=top)
    if k < K:
        pad = K - k
        for key in ("p", "nu"):
            out[key] = torch.cat([out[key], out[key].new_zeros(pad, 3)])
        for key in ("d", "w"):
            out[key] = torch.cat([out[key], out[key].new_zeros(pad)])
        out["s_top"] = torch.cat([top, top.new_full((pad,), -float("inf"))])
    return out


def collide_pair(GA, poseA, GB, poseB, tau, K, lam=LAMBDA_DEFAULT, eps_n=None, xiA=None, xiB=None,
                 exact_exp=False, no_ee=False, one_sided_vs=False, presel=None, safeguard=False, refine=0):
    """Contact manifold g_{A,B} of one pair (Sec. IV-A): K x (p, nu, d, w)."""
    RA, tA = pose_Rt(poseA, xiA, exact_exp)
    RB, tB = pose_Rt(poseB, xiB, exact_exp)
    c = pair_candidates(GA, RA, tA, GB, RB, tB, tau, lam, eps_n, no_ee=no_ee, one_sided_vs=one_sided_vs,
                        presel=presel, safeguard=safeguard, refine=refine)
    return manifold(c, tau, K)


# ============================================================== broadphase (R12, float32)

def bound_radius_f32(kind: int, params, points) -> np.float32:
    """Bounding radius about the body origin, in float32 arithmetic.

    sphere r; capsule h + r; box sqrt((hx^2 + hy^2) + hz^2);
    polytope sqrt(max_v ((x^2 + y^2) + z^2)); superquadric union
    max_i sqrt((tx^2 + ty^2) + tz^2) + sqrt((a^2 + b^2) + c^2) (each
    superquadric lies in its (a, b, c) box).
    """
    f = np.float32
    p = np.asarray(params, dtype=np.float32)
    if kind == OPC:
        r = np.asarray(points, dtype=np.float32).reshape(-1, 9)
        n2 = (r[:, 0] * r[:, 0] + r[:, 1] * r[:, 1]) + r[:, 2] * r[:, 2]
        return np.float32(np.sqrt(n2.max(), dtype=np.float32) + r[:, 6].max())
    if kind == SQ_UNION:
        r = np.asarray(points, dtype=np.float32).reshape(-1, 12)
        tn = np.sqrt((r[:, 5] * r[:, 5] + r[:, 6] * r[:, 6]) + r[:, 7] * r[:, 7], dtype=np.float32)
        an = np.sqrt((r[:, 0] * r[:, 0] + r[:, 1] * r[:, 1]) + r[:, 2] * r[:, 2], dtype=np.float32)
        return np.float32((tn + an).max())
    if kind == SPHERE:
        return f(p[0])
    if kind == CAPSULE:
        return f(p[1]) + f(p[0])
    if kind == BOX:
        return np.sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2], dtype=np.float32)
    P = np.asarray(points, dtype=np.float32)
    n2 = (P[:, 0] * P[:, 0] + P[:, 1] * P[:, 1]) + P[:, 2] * P[:, 2]
    return np.sqrt(n2.max(), dtype=np.float32)


def default_margin_f32(tau) -> np.float32:
    return np.float32(10.0) * np.float32(tau)


def broadphase(batch, margin=None):
    """Kept pairs and per-scene offsets (R12).

    Keep (a, b) iff d2 <= r*r with dx = tb_x - ta_x etc.,
    d2 = (dx*dx + dy*dy) + dz*dz and r = (R_a + R_b) + margin, every operation
    rounded to float32.  Scene-major order; all i<j pairs per scene unless an
    explicit candidate list is given (kept in its order).
    Returns pairs int32 [2, n] and offsets int32 [S+1].
    """
    f = np.float32
    m = default_margin_f32(batch.tau) if margin is None or margin < 0 else f(margin)
    gs = batch.geoms
    Rg = np.array([bound_radius_f32(int(gs.types[g]), gs.params[g], gs.points_of(g)) for g in range(gs.n)],
                  dtype=np.float32)
    sc, a, b = batch.candidate_pairs()
    Rb = Rg[batch.body_geom]
    T = batch.pose[4:7].astype(np.float32)
    dx = T[0, b] - T[0, a]
    dy = T[1, b] - T[1, a]
    dz = T[2, b] - T[2, a]
    d2 = (dx * dx + dy * dy) + dz * dz
    r = (Rb[a] + Rb[b]) + m
    keep = d2 <= r * r
    cnt = np.bincount(sc[keep], minlength=batch.n_scenes) if len(sc) else np.zeros(batch.n_scenes, np.int64)
    off = np.zeros(batch.n_scenes + 1, dtype=np.int64)
    off[1:] = np.cumsum(cnt)
    pairs = np.stack([a[keep], b[keep]]).astype(np.int32)
    return pairs, off.astype(np.int32)


# ============================================================== batch helpers

class GeomCache:
    def __init__(self, gs, requires_grad=False):
        self.gs = gs
        self.rg = requires_grad
        self.cache = {}

    def __getitem__(self, g):
        g = int(g)
        if g not in self.cache:
            self.cache[g] = geom_from_set(self.gs, g, self.rg)
        return self.cache[g]


def collide_batch(batch, pair_list=None, lam=LAMBDA_DEFAULT, eps_n=None, margin=None, cache=None, no_ee=False,
                  one_sided_vs=False, presel=None, safeguard=False, refine=0):
    """Forward manifold for the kept pairs of a batch (or a given pair subset).

    Returns (pairs [2,n], offsets [S+1], outputs dict of numpy float64 arrays
    p [n,K,3], nu [n,K,3], d [n,K], w [n,K]).
    """
    if pair_list is None:
        pairs, offsets = broadphase(batch, margin)
    else:
        pairs, offsets = np.asarray(pair_list, dtype=np.int32), None
    cache = cache or GeomCache(batch.geoms)
    n, K = pairs.shape[1], batch.K
    out = dict(p=np.zeros((n, K, 3)), nu=np.zeros((n, K, 3)), d=np.zeros((n, K)), w=np.zeros((n, K)))
    with torch.no_grad():
        for i in range(n):
            a, b = int(pairs[0, i]), int(pairs[1, i])
            GA, GB = cache[batch.body_geom[a]], cache[batch.body_geom[b]]
            m = collide_pair(GA, batch.pose[:, a], GB, batch.pose[:, b], batch.tau, K, lam, eps_n,
                             no_ee=no_ee, one_sided_vs=one_sided_vs, presel=presel, safeguard=safeguard,
                             refine=refine)
            for k in ("p", "nu", "d", "w"):
                out[k][i] = m[k].numpy()
    return pairs, offsets, out


def pair_grad(GA, poseA, GB, poseB, tau, K, cot, lam=LAMBDA_DEFAULT, eps_n=None, no_ee=False, one_sided_vs=False,
              presel=None, safeguard=False, refine=0):
    """Gradient of L = <cot, outputs> for one pair by autograd of the forward
    (with presel, also through the SoftSort selection weights and metrics).

    cot: dict with any of p [K,3], nu [K,3], d [K], w [K] (numpy).
    Returns dict: xiA [6], xiB [6] (left tangents (rho, omega)), geomA, geomB
    (params [4] or hull-vertex points [V,3]), tau, and the forward values.
    GA / GB must have been built with requires_grad=True (they may be the same
    object when a geometry is shared).
    """
    xiA = torch.zeros(6, dtype=DT, requires_grad=True)
    xiB = torch.zeros(6, dtype=DT, requires_grad=True)
    tau_t = torch.tensor(float(tau), dtype=DT, requires_grad=True)
    m = collide_pair(GA, poseA, GB, poseB, tau_t, K, lam, eps_n, xiA, xiB, no_ee=no_ee, one_sided_vs=one_sided_vs,
                     presel=presel, safeguard=safeguard, refine=refine)
    L = torch.zeros((), dtype=DT)
    for k, v in cot.items():
        L = L + (m[k] * torch.as_tensor(np.asarray(v, dtype=np.float64))).sum()
    leaves = [xiA, xiB, tau_t]
    ga = GA.points if GA.kind == POLYTOPE else GA.params
    gb = GB.points if GB.kind == POLYTOPE else GB.params
    geo = [x for x in ([ga] if gb is ga else [ga, gb]) if x.requires_grad]
    grads = torch.autograd.grad(L, leaves + geo, allow_unused=True)
    z = lambda g, ref: torch.zeros_like(ref) if g is None else g
    out = dict(xiA=z(grads[0], xiA).numpy(), xiB=z(grads[1], xiB).numpy(), tau=float(z(grads[2], tau_t)),
               L=float(L.detach()), fwd={k: v.detach().numpy() for k, v in m.items()})
    gmap = {id(x): z(g, x).detach().numpy() for x, g in zip(geo, grads[3:])}
    out["geomA"] = gmap.get(id(ga), np.zeros(tuple(ga.shape)))
    out["geomB"] = gmap.get(id(gb), np.zeros(tuple(gb.shape)))
    return out


def pose_tangent_to_world(xi):
    """Split a (rho, omega) tangent gradient into its two 3-vectors."""
    xi = np.asarray(xi)
    return xi[:3], xi[3:]
