"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with a
closed form, a limit, an invariant, a brute-force search or an independent
library routine.  The pytest wrappers live in ``test_oracle_pins.py``; the
mutation test plants plausible mistakes in the oracle and checks that at least
one pin catches each.  Pins reference oracle functions through the module so
that a monkeypatched oracle is what they exercise.
"""
from __future__ import annotations

import math

import numpy as np
import torch
from scipy.spatial import Delaunay
from scipy.spatial.transform import Rotation

from oracle import cm_oracle as O
import workloads as W

DT = torch.float64


def T(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=DT)


# ----------------------------------------------------------------------------- operators

def pin_operator_identities():
    """sigma(z)+sigma(-z)=1; s+(x)-s+(-x)=x; clip_s(x)+clip_s(1-x)=1; bounds of LSE."""
    rng = np.random.default_rng(1)
    x = T(rng.uniform(-3, 3, 200))
    for tau in (0.5, 0.05, 0.003):
        assert torch.allclose(O.sigmoid(x / tau) + O.sigmoid(-x / tau), torch.ones_like(x), atol=1e-14)
        assert torch.allclose(O.softplus_t(x, tau) - O.softplus_t(-x, tau), x, atol=1e-12)
        assert torch.allclose(O.clip_s(x, 0.0, 1.0, tau) + O.clip_s(1 - x, 0.0, 1.0, tau), torch.ones_like(x),
                              atol=1e-12)
        y = T(rng.normal(size=(30, 17)))
        L = O.lse_t(y, tau, dim=-1)
        mx = y.max(-1).values
        assert bool((L >= mx - 1e-12).all()) and bool((L <= mx + tau * math.log(17) + 1e-12).all())
        p = O.argmin_s(y, tau, dim=-1)
        assert torch.allclose(p.sum(-1), torch.ones(30, dtype=DT), atol=1e-13)
        z = x[torch.abs(x / tau) < 30] / tau
        assert torch.allclose(O.log_sigmoid(z), torch.log(torch.sigmoid(z)), atol=1e-12, rtol=1e-12)
        assert torch.allclose(O.sign_s(x, tau), 2 * torch.sigmoid(2 * x / tau) - 1, atol=1e-13)


def pin_operator_limits():
    """tau -> 0: clip_s -> clamp, within_s -> indicator, argmin_s -> one-hot, LSE -> max."""
    rng = np.random.default_rng(2)
    x = T(rng.uniform(-2, 3, 500))
    x = x[(torch.abs(x) > 1e-3) & (torch.abs(x - 1) > 1e-3)]
    tau = 1e-7
    assert torch.allclose(O.clip_s(x, 0.0, 1.0, tau), torch.clamp(x, 0.0, 1.0), atol=1e-6)
    ind = ((x >= 0) & (x <= 1)).to(DT)
    assert torch.allclose(O.within_s(x, 0.0, 1.0, tau), ind, atol=1e-9)
    y = T(rng.normal(size=(40, 9)))
    p = O.argmin_s(y, tau, dim=-1)
    assert torch.equal(p.argmax(-1), y.argmin(-1)) and bool((p.max(-1).values > 1 - 1e-9).all())
    assert torch.allclose(O.lse_t(y, tau, -1), y.max(-1).values, atol=1e-6)
    assert torch.allclose(O.sign_s(x, tau), torch.sign(x), atol=1e-9)


# ----------------------------------------------------------------------------- geometry

def _sphere_surface(n):
    rng = np.random.default_rng(3)
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _brute_dist(X, S):
    """min over surface samples of |x - s| (chunked)."""
    out = np.empty(len(X))
    for i in range(0, len(X), 64):
        D = np.linalg.norm(X[i:i + 64, None, :] - S[None, :, :], axis=-1)
        out[i:i + 64] = D.min(1)
    return out


def _rounded_box_surface(h, rho, n_side=90):
    """Dense samples of a rounded box surface: the Minkowski sum of the inner
    box (h - rho) and a ball of radius rho, generated as inner-box surface
    points pushed out along unit directions that keep them on the outer shell."""
    b = np.asarray(h) - rho
    rng = np.random.default_rng(4)
    U = rng.normal(size=(n_side ** 2 * 6, 3))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    # support point of the inner box in direction u, plus rho * u
    S = np.sign(U) * b[None, :] + rho * U
    # flat faces: also sample the face interiors directly
    faces = []
    g = np.linspace(-1, 1, n_side)
    A, B = np.meshgrid(g, g)
    A, B = A.ravel(), B.ravel()
    for ax in range(3):
        o = [a for a in range(3) if a != ax]
        for sg in (-1, 1):
            P = np.zeros((len(A), 3))
            P[:, ax] = sg * (b[ax] + rho)
            P[:, o[0]] = A * b[o[0]]
            P[:, o[1]] = B * b[o[1]]
            faces.append(P)
    # edges (quarter-cylinder parts): for each edge sample the outward arc
    edges = []
    t = np.linspace(-1, 1, n_side)
    ang = np.linspace(0, np.pi / 2, n_side)
    for ax in range(3):
        o = [a for a in range(3) if a != ax]
        for s0 in (-1, 1):
            for s1 in (-1, 1):
                TT, AA = np.meshgrid(t, ang)
                P = np.zeros((TT.size, 3))
                P[:, ax] = TT.ravel() * b[ax]
                P[:, o[0]] = s0 * (b[o[0]] + rho * np.cos(AA.ravel()))
                P[:, o[1]] = s1 * (b[o[1]] + rho * np.sin(AA.ravel()))
                edges.append(P)
    return np.concatenate([S] + faces + edges)


def _inside_rounded_box(X, h, rho):
    b = np.asarray(h) - rho
    return np.linalg.norm(X - np.clip(X, -b, b), axis=1) < rho


def pin_analytic_sdf_brute_force():
    """sphere / capsule / rounded-box SDF vs distance to dense surface samples."""
    rng = np.random.default_rng(5)
    X = rng.uniform(-0.9, 0.9, size=(300, 3))
    # sphere r = 0.4
    S = 0.4 * _sphere_surface(60000)
    G = O.make_geom(O.SPHERE, params=[0.4, 0, 0, 0])
    phi, _ = O.sdf_local(G, T(X), 0.01)
    ref = _brute_dist(X, S) * np.where(np.linalg.norm(X, axis=1) < 0.4, -1, 1)
    assert np.max(np.abs(phi.numpy() - ref)) < 6e-3
    # capsule r = 0.2, h = 0.3: sphere-swept segment
    r, h = 0.2, 0.3
    U = _sphere_surface(30000)
    zs = rng.uniform(-h, h, size=30000)
    ang = rng.uniform(0, 2 * np.pi, 30000)
    cyl = np.stack([r * np.cos(ang), r * np.sin(ang), zs], 1)
    caps = r * U + np.where(U[:, 2:3] > 0, 1, -1) * np.array([0, 0, h])
    S = np.concatenate([cyl, caps])
    G = O.make_geom(O.CAPSULE, params=[r, h, 0, 0])
    phi, _ = O.sdf_local(G, T(X), 0.01)
    seg = np.stack([np.zeros(len(X)), np.zeros(len(X)), np.clip(X[:, 2], -h, h)], 1)
    inside = np.linalg.norm(X - seg, axis=1) < r
    ref = _brute_dist(X, S) * np.where(inside, -1, 1)
    assert np.max(np.abs(phi.numpy() - ref)) < 6e-3
    # rounded box
    hb, rho = np.array([0.5, 0.3, 0.2]), 0.05
    S = _rounded_box_surface(hb, rho)
    G = O.make_geom(O.BOX, params=[hb[0], hb[1], hb[2], rho])
    phi, _ = O.sdf_local(G, T(X), 0.01)
    ref = _brute_dist(X, S) * np.where(_inside_rounded_box(X, hb, rho), -1, 1)
    assert np.max(np.abs(phi.numpy() - ref)) < 8e-3


def pin_sdf_gradients_fd():
    """Analytic SDF gradients vs central differences of the SDF value."""
    rng = np.random.default_rng(6)
    X = T(rng.uniform(-0.8, 0.8, size=(50, 3)))
    pts = W.ellipsoid_points(np.random.default_rng(7), 20, [0.4, 0.3, 0.5])
    geoms = [O.make_geom(O.SPHERE, params=[0.4, 0, 0, 0]), O.make_geom(O.CAPSULE, params=[0.2, 0.3, 0, 0]),
             O.make_geom(O.BOX, params=[0.5, 0.3, 0.2, 0.05]), O.make_geom(O.POLYTOPE, points=pts)]
    h = 1e-6
    with torch.no_grad():
        for G in geoms:
            _, g = O.sdf_local(G, X, 0.05)
            for j in range(3):
                e = torch.zeros(3, dtype=DT); e[j] = h
                fd = (O.sdf_local(G, X + e, 0.05)[0] - O.sdf_local(G, X - e, 0.05)[0]) / (2 * h)
                assert torch.allclose(g[:, j], fd, atol=2e-6), (G.kind, j)


def pin_polytope_inside_delaunay():
    """tau -> 0 polytope SDF: sign agrees with scipy Delaunay point location, and
    inside points have |phi| = distance to the nearest face (brute force)."""
    rng = np.random.default_rng(8)
    pts = W.ellipsoid_points(rng, 40, [0.5, 0.3, 0.4])
    G = O.make_geom(O.POLYTOPE, points=pts)
    X = rng.uniform(-0.6, 0.6, size=(2000, 3))
    with torch.no_grad():
        phi, _ = O.sdf_local(G, T(X), 1e-8)
    phi = phi.numpy()
    inside = Delaunay(pts).find_simplex(X) >= 0
    far = np.abs(phi) > 1e-4
    assert np.all((phi[far] < 0) == inside[far])
    # inside: -phi equals distance to the closest triangle (sampled barycentric grid)
    P = pts[G.vertex_ids]
    tri = P[G.tris]
    a = np.linspace(0, 1, 60)
    A, B = np.meshgrid(a, a)
    m = (A + B) <= 1
    bary = np.stack([1 - A[m] - B[m], A[m], B[m]], 1)
    S = np.einsum("sk,fkd->fsd", bary, tri).reshape(-1, 3)
    Xin = X[inside & far][:100]
    d_in = _brute_dist(Xin, S)
    phi_in = phi[inside & far][:100]
    assert np.max(np.abs(-phi_in - d_in)) < 5e-3


def pin_hull_counts():
    """Hull of points on an ellipsoid: every point is a vertex, Euler V-E+F=2,
    E = 3V-6, F = 2V-4, every face plane has all points on its inner side."""
    rng = np.random.default_rng(9)
    for n in (8, 32, 64, 100):
        pts = W.ellipsoid_points(rng, n, [0.3, 0.45, 0.5]).astype(np.float32)
        vid, tris, edges = O.hull_topology(pts)
        V, E, F = len(vid), len(edges), len(tris)
        assert V == n and E == 3 * V - 6 and F == 2 * V - 4 and V - E + F == 2
        G = O.make_geom(O.POLYTOPE, points=pts)
        n_, o_ = G.planes()
        dist = pts.astype(np.float64) @ n_.detach().numpy().T - o_.detach().numpy()[None, :]
        assert dist.max() < 1e-7
        assert np.allclose(np.linalg.norm(n_.detach().numpy(), axis=1), 1.0)


def pin_analytic_meshes():
    """Sphere / capsule vertices lie on the exact surface; box corners at +-h;
    edge counts 56 / 72 / 12; no duplicate edges; every vertex has degree >= 3."""
    G = O.make_geom(O.SPHERE, params=[0.3, 0, 0, 0])
    V = G.vertices()
    with torch.no_grad():
        assert V.shape == (26, 3) and G.edges.shape == (56, 2)
        assert torch.allclose(O.sdf_local(G, V, 0.01)[0], torch.zeros(26, dtype=DT), atol=1e-14)
        G = O.make_geom(O.CAPSULE, params=[0.1, 0.25, 0, 0])
        V = G.vertices()
        assert V.shape == (34, 3) and G.edges.shape == (72, 2)
        assert torch.allclose(O.sdf_local(G, V, 0.01)[0], torch.zeros(34, dtype=DT), atol=1e-14)
        G = O.make_geom(O.BOX, params=[0.5, 0.2, 0.1, 0.02])
        V = G.vertices()
        assert V.shape == (8, 3) and G.edges.shape == (12, 2)
        assert torch.allclose(torch.abs(V), T([0.5, 0.2, 0.1]).expand(8, 3))
    for G in (O.make_geom(O.SPHERE, params=[0.3, 0, 0, 0]), O.make_geom(O.CAPSULE, params=[0.1, 0.25, 0, 0]),
              O.make_geom(O.BOX, params=[0.5, 0.2, 0.1, 0.02])):
        e = {tuple(sorted(x)) for x in G.edges.tolist()}
        assert len(e) == len(G.edges)
        deg = np.bincount(G.edges.ravel())
        assert deg.min() >= 3
        # box edges are axis aligned and of length 2h
        if G.kind == O.BOX:
            with torch.no_grad():
                V = G.vertices().numpy()
            L = np.linalg.norm(V[G.edges[:, 0]] - V[G.edges[:, 1]], axis=1)
            assert sorted(np.round(L, 9).tolist()) == sorted([1.0] * 4 + [0.4] * 4 + [0.2] * 4)


def pin_quaternion_rotation():
    """quat_to_R equals scipy's rotation matrix (scalar-last convention there)."""
    rng = np.random.default_rng(10)
    for _ in range(20):
        q = rng.normal(size=4)
        R = O.quat_to_R(T(q)).numpy()
        Rs = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        assert np.allclose(R, Rs, atol=1e-14)


# ----------------------------------------------------------------------------- E-E QP

def _seg_closest_brute(a0, a1, b0, b1, lam=0.0, n=401, levels=4):
    """argmin over [0,1]^2 of |e1 - e2|^2 + lam((x-.5)^2 + (y-.5)^2) by grid
    search with successive local refinement."""
    lo1, hi1, lo2, hi2 = 0.0, 1.0, 0.0, 1.0
    best = None
    for _ in range(levels):
        x = np.linspace(lo1, hi1, n)
        y = np.linspace(lo2, hi2, n)
        X, Y = np.meshgrid(x, y, indexing="ij")
        E1 = a0[None, None] + X[..., None] * (a1 - a0)[None, None]
        E2 = b0[None, None] + Y[..., None] * (b1 - b0)[None, None]
        f = ((E1 - E2) ** 2).sum(-1) + lam * ((X - 0.5) ** 2 + (Y - 0.5) ** 2)
        i, j = np.unravel_index(np.argmin(f), f.shape)
        best = (x[i], y[j], f[i, j])
        w1, w2 = (hi1 - lo1) * 4 / n, (hi2 - lo2) * 4 / n
        lo1, hi1 = max(0.0, x[i] - w1), min(1.0, x[i] + w1)
        lo2, hi2 = max(0.0, y[j] - w2), min(1.0, y[j] + w2)
    return best


def _rand_edges(rng, n):
    return [tuple(rng.uniform(0, 1, size=(4, 3))) for _ in range(n)]


def pin_qp_hard_limit_segments():
    """tau -> 0 and lambda -> 0: witness distance = textbook segment-segment
    distance (brute force); witness parameters match when the minimum is unique."""
    rng = np.random.default_rng(11)
    for a0, a1, b0, b1 in _rand_edges(rng, 25):
        x, y, f = _seg_closest_brute(a0, a1, b0, b1)
        with torch.no_grad():
            qp = O.ee_qp(T(a0), T(a1), T(b0), T(b1), 1e-9, 1e-12)
            e1, e2, dbar, _ = O.ee_witness(T(a0), T(a1), T(b0), T(b1), qp["al1"], qp["al2"], 1e-18)
        assert abs(float(dbar) - math.sqrt(f)) < 1e-6
        assert abs(float(qp["al1"]) - x) < 1e-4 and abs(float(qp["al2"]) - y) < 1e-4


def pin_qp_regularised_limit():
    """tau -> 0 with lambda > 0: the exact minimiser of the regularised box QP."""
    rng = np.random.default_rng(12)
    for lam in (0.01, 0.3):
        for a0, a1, b0, b1 in _rand_edges(rng, 20):
            x, y, f = _seg_closest_brute(a0, a1, b0, b1, lam)
            with torch.no_grad():
                qp = O.ee_qp(T(a0), T(a1), T(b0), T(b1), 1e-9, lam)
            assert abs(float(qp["al1"]) - x) < 1e-4 and abs(float(qp["al2"]) - y) < 1e-4, (lam, x, y)


def pin_qp_no_smoothing():
    """Ours-NS: the exact minimiser of the regularised box QP, against grid
    search and scipy's bounded quasi-Newton solver; it is the tau -> 0 limit
    of the smoothed routine; the batched witness form agrees pair by pair."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(13)
    for lam in (0.01, 0.3):
        E = np.array(_rand_edges(rng, 20))
        for a0, a1, b0, b1 in E:
            x, y, f = _seg_closest_brute(a0, a1, b0, b1, lam)
            with torch.no_grad():
                q = O.ee_qp_hard(T(a0), T(a1), T(b0), T(b1), lam)
                qs = O.ee_qp(T(a0), T(a1), T(b0), T(b1), 1e-9, lam)
            fun = lambda z: float(((a0 + z[0] * (a1 - a0) - b0 - z[1] * (b1 - b0)) ** 2).sum()
                                  + lam * ((z[0] - 0.5) ** 2 + (z[1] - 0.5) ** 2))
            r = minimize(fun, [0.5, 0.5], method="L-BFGS-B", bounds=[(0, 1), (0, 1)], options=dict(ftol=1e-15, gtol=1e-12))
            got = np.array([float(q["al1"]), float(q["al2"])])
            assert np.abs(got - [x, y]).max() < 1e-4, (lam, got, x, y)
            assert np.abs(got - r.x).max() < 1e-5, (lam, got, r.x)
            assert fun(got) <= r.fun + 1e-12
            assert abs(float(qs["al1"]) - got[0]) < 1e-6 and abs(float(qs["al2"]) - got[1]) < 1e-6
            inside = 0 < r.x[0] < 1 and 0 < r.x[1] < 1
            assert float(q["con"]) == (1.0 if inside else 0.0) or min(r.x.min(), 1 - r.x.max()) < 1e-6
        wb = O.ee_witness_batch(E, 0.05, lam, hard=True)
        ws = O.ee_witness_batch(E, 0.05, lam)
        for i, (a0, a1, b0, b1) in enumerate(E):
            with torch.no_grad():
                q = O.ee_qp_hard(T(a0), T(a1), T(b0), T(b1), lam)
                qs = O.ee_qp(T(a0), T(a1), T(b0), T(b1), 0.05, lam)
            assert wb["al1"][i] == float(q["al1"]) and wb["al2"][i] == float(q["al2"])
            assert np.allclose(wb["e1"][i], a0 + wb["al1"][i] * (a1 - a0), atol=1e-15)
            assert np.allclose(wb["e2"][i], b0 + wb["al2"][i] * (b1 - b0), atol=1e-15)
            assert abs(ws["al1"][i] - float(qs["al1"])) < 1e-15 and abs(ws["con"][i] - float(qs["con"])) < 1e-15


def pin_qp_edge_swap_symmetry():
    """Swapping the two edges swaps (al1, al2) and leaves d_bar unchanged."""
    rng = np.random.default_rng(13)
    E = np.array(_rand_edges(rng, 200))
    a0, a1, b0, b1 = (T(E[:, i]) for i in range(4))
    with torch.no_grad():
        for tau in (0.1, 0.01):
            q = O.ee_qp(a0, a1, b0, b1, tau, 0.01)
            r = O.ee_qp(b0, b1, a0, a1, tau, 0.01)
            assert torch.allclose(q["al1"], r["al2"], atol=1e-12) and torch.allclose(q["al2"], r["al1"], atol=1e-12)
            assert torch.allclose(q["con"], r["con"], atol=1e-12)


def _rotating_edge_trace(tau, lam, n=2001):
    th = torch.linspace(0.0, math.pi, n, dtype=DT)
    u = torch.stack([torch.sin(th), torch.cos(th), torch.zeros_like(th)], 1)
    a0, a1 = -u, u
    b0 = T([-3.0, -1.2, 0.0]).expand(n, 3)
    b1 = T([3.0, -1.2, 0.0]).expand(n, 3)
    with torch.no_grad():
        qp = O.ee_qp(a0, a1, b0, b1, tau, lam)
        e1, _, _, _ = O.ee_witness(a0, a1, b0, b1, qp["al1"], qp["al2"], tau * tau)
    return e1


def pin_rotating_edge_continuity():
    """Didactic rotating-edge experiment (Sec. IV-D, Fig. 3 setup): the unsmoothed
    witness point on the rotating edge jumps at the parallel configuration,
    the regularised + smoothed one moves continuously."""
    jump_hard = (_rotating_edge_trace(1e-9, 1e-12).diff(dim=0).norm(dim=1)).max()
    jump_soft = (_rotating_edge_trace(0.1, 0.5).diff(dim=0).norm(dim=1)).max()
    assert float(jump_hard) > 1.0
    assert float(jump_soft) < 0.02


# ----------------------------------------------------------------------------- pair level

def _pose(q, t):
    return np.concatenate([np.asarray(q, float), np.asarray(t, float)])


def _cand(GA, pA, GB, pB, tau, lam=0.01):
    RA, tA = O.pose_Rt(pA)
    RB, tB = O.pose_Rt(pB)
    with torch.no_grad():
        return O.pair_candidates(GA, RA, tA, GB, RB, tB, tau, lam)


def pin_crossing_edges_sign():
    """Hand-built: cube A above cube B (B turned 45 deg about z).  For the
    crossing bottom/top edge pairs: separated by gap g -> d1 = d2 = +g and
    pair normals -z; interpenetrating by delta -> d1 = d2 = -delta, normals -z;
    clash indicator ~ 1 for these pairs."""
    GA = O.make_geom(O.BOX, params=[0.5, 0.5, 0.5, 1e-6])
    GB = O.make_geom(O.BOX, params=[0.5, 0.5, 0.5, 1e-6])
    qB = [math.cos(math.pi / 8), 0, 0, math.sin(math.pi / 8)]
    for gap in (0.05, -0.03):
        c = _cand(GA, _pose([1, 0, 0, 0], [0, 0, 1.0 + gap]), GB, _pose(qB, [0, 0, 0]), 1e-4, 1e-10)
        ex = c["extra"]
        e1, e2 = ex["e1"].numpy(), ex["e2"].numpy()
        # crossing pairs: both witnesses at the two faces' heights, at the same xy
        zA, zB = 0.5 + gap, 0.5
        sel = (np.abs(e1[..., 2] - zA) < 1e-6) & (np.abs(e2[..., 2] - zB) < 1e-6) & \
              (np.linalg.norm(e1[..., :2] - e2[..., :2], axis=-1) < 1e-4)
        assert sel.sum() == 8, sel.sum()
        d1 = (ex["gam1"] * ex["dbar"]).numpy()[sel]
        d2 = (ex["gam2"] * ex["dbar"]).numpy()[sel]
        assert np.allclose(d1, gap, atol=1e-5) and np.allclose(d2, gap, atol=1e-5)
        nv = c["nu"].numpy()[ex["n_vs"]:].reshape(12, 12, 2, 3)[sel]
        assert np.allclose(nv, np.array([0, 0, -1.0]), atol=1e-3)
        assert np.all(np.exp(ex["log_cl"].numpy()[sel]) > 0.99)


def pin_vs_weights_point_in_polytope():
    """tau -> 0: V-S weights are the hard point-in-body test (Delaunay)."""
    rng = np.random.default_rng(14)
    pa = W.ellipsoid_points(rng, 30, [0.5, 0.4, 0.45])
    pb = W.ellipsoid_points(rng, 30, [0.35, 0.5, 0.3])
    GA, GB = O.make_geom(O.POLYTOPE, points=pa), O.make_geom(O.POLYTOPE, points=pb)
    qA, qB = W.uniform_quats(rng, 2)
    poseA, poseB = _pose(qA, [0.1, 0, 0]), _pose(qB, [0.35, 0.2, -0.1])
    c = _cand(GA, poseA, GB, poseB, 1e-8)
    nA = len(GA.vertex_ids)
    w = np.exp(c["logw"].numpy()[:c["extra"]["n_vs"]])
    d = c["d"].numpy()[:c["extra"]["n_vs"]]
    RA, tA = (x.numpy() for x in O.pose_Rt(poseA))
    RB, tB = (x.numpy() for x in O.pose_Rt(poseB))
    vA = pa[GA.vertex_ids] @ RA.T + tA
    vB = pb[GB.vertex_ids] @ RB.T + tB
    inB = Delaunay(pb).find_simplex((vA - tB) @ RB) >= 0
    inA = Delaunay(pa).find_simplex((vB - tA) @ RA) >= 0
    inside = np.concatenate([inB, inA])
    far = np.abs(d) > 1e-4
    assert far.sum() > 40 and inside[far].any() and (~inside[far]).any()
    assert np.all(np.abs(w[far] - inside[far]) < 1e-9)


def pin_vs_normal_sphere():
    """A vertex of A near a sphere B: candidate normal = -(outward unit normal of
    B)/sqrt(1 + tau) and d = |x - c| - r (closed form)."""
    GA = O.make_geom(O.BOX, params=[0.2, 0.2, 0.2, 0.01])
    GB = O.make_geom(O.SPHERE, params=[0.3, 0, 0, 0])
    tau = 0.02
    c = _cand(GA, _pose([1, 0, 0, 0], [0.0, 0.0, 0.0]), GB, _pose([1, 0, 0, 0], [0.25, 0.3, 0.35]), tau)
    with torch.no_grad():
        V = GA.vertices().numpy()
    u = V - np.array([0.25, 0.3, 0.35])
    dist = np.linalg.norm(u, axis=1)
    assert np.allclose(c["d"].numpy()[:8], dist - 0.3, atol=1e-14)
    assert np.allclose(c["nu"].numpy()[:8], -(u / dist[:, None]) / math.sqrt(1 + tau), atol=1e-14)


def pin_nn_rows_columns():
    """Nearest-neighbour indicators: rows of nn1 and columns of nn2 sum to 1;
    tau -> 0 gives the hard arg-min along each row / column."""
    rng = np.random.default_rng(15)
    D = T(rng.uniform(0, 1, size=(7, 11)))
    l1, l2 = O.nn_log_indicators(D, 0.05)
    assert torch.allclose(torch.exp(l1).sum(1), torch.ones(7, dtype=DT), atol=1e-13)
    assert torch.allclose(torch.exp(l2).sum(0), torch.ones(11, dtype=DT), atol=1e-13)
    l1, l2 = O.nn_log_indicators(D, 1e-7)
    assert torch.equal(torch.exp(l1).argmax(1), D.argmin(1))
    assert torch.equal(torch.exp(l2).argmax(0), D.argmin(0))


def _hard_face_gradient(eq, x, tie=1e-9, margin=1e-4):
    """tau -> 0 gradient of a polytope's smoothed SDF at x from scipy's hull
    facets: the mean outward normal of the facets whose planes attain the
    largest value at x (a point on an edge or vertex ties its facets).  Also
    returns that largest plane value and whether another facet lies within
    `margin` of it without tying (a kink the limit cannot resolve)."""
    v = eq[:, :3] @ x + eq[:, 3]
    m = v.max()
    tied = v >= m - tie
    kink = bool(((v < m - tie) & (v > m - margin)).any())
    return eq[tied, :3].mean(0), m, kink


def _activity_hard_limit(seed, lam, tau=1e-7, margin=1e-4):
    """One polytope pair: the oracle's E-E activities exp(log Gamma_b) beside
    the product of independent hard indicators, and per-sample validity (every
    factor at least `margin` from its kink)."""
    from scipy.optimize import lsq_linear
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(700 + seed)
    GA = O.make_geom(O.POLYTOPE, points=W.ellipsoid_points(rng, 14, rng.uniform(0.25, 0.45, 3)))
    GB = O.make_geom(O.POLYTOPE, points=W.ellipsoid_points(rng, 13, rng.uniform(0.25, 0.45, 3)))
    qA, qB = W.uniform_quats(rng, 2)
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    pA, pB = _pose(qA, [0, 0, 0]), _pose(qB, (0.2 + 0.1 * (seed % 5)) * u)
    RA, tA = O.pose_Rt(pA)
    RB, tB = O.pose_Rt(pB)
    with torch.no_grad():
        c = O.pair_candidates(GA, RA, tA, GB, RB, tB, tau, lam)
        PA = (GA.vertices() @ RA.T + tA).numpy()
        PB = (GB.vertices() @ RB.T + tB).numpy()
    EA, EB = np.asarray(GA.edges), np.asarray(GB.edges)
    nA, nB = len(EA), len(EB)
    ex = c["extra"]
    act = np.exp(c["logw"].numpy()[ex["n_vs"]:].reshape(nA, nB, 2))
    eqA, eqB = ConvexHull(PA).equations, ConvexHull(PB).equations
    dlA, dlB = Delaunay(PA), Delaunay(PB)
    # hard witnesses: the regularised box QP solved by bounded-variable least
    # squares (|M a - y|^2 = |e1 - e2|^2 + lam |a - 1/2|^2); the unconstrained
    # minimiser by ordinary least squares
    sl = math.sqrt(lam)
    con = np.zeros((nA, nB))
    side = np.zeros((nA, nB), int)
    ok = np.ones((nA, nB), bool)
    e1 = np.zeros((nA, nB, 3))
    e2 = np.zeros((nA, nB, 3))
    for k in range(nA):
        a0, a1 = PA[EA[k, 0]], PA[EA[k, 1]]
        for l in range(nB):
            b0, b1 = PB[EB[l, 0]], PB[EB[l, 1]]
            M = np.zeros((5, 2))
            M[:3, 0], M[:3, 1], M[3, 0], M[4, 1] = a1 - a0, b0 - b1, sl, sl
            y = np.concatenate([b0 - a0, [0.5 * sl, 0.5 * sl]])
            au = np.linalg.lstsq(M, y, rcond=None)[0]
            al = np.clip(lsq_linear(M, y, bounds=(0.0, 1.0), method="bvls", tol=1e-14).x, 0.0, 1.0)
            e1[k, l], e2[k, l] = a0 + al[0] * (a1 - a0), b0 + al[1] * (b1 - b0)
            con[k, l] = float(np.all((au > 0) & (au < 1)))
            side[k, l] = -1 if (au < 0).any() else (1 if (au > 1).any() else 0)
            ok[k, l] = np.minimum(np.abs(au), np.abs(au - 1)).min() >= margin
    # a near tie of box-edge costs leaves the smoothed witness between two
    # points even at tau = 1e-7; those samples (rare) are not limits
    moved = (np.linalg.norm(ex["e1"].numpy() - e1, axis=-1) + np.linalg.norm(ex["e2"].numpy() - e2, axis=-1)) > 1e-6
    assert moved.mean() < 0.03, moved.mean()
    ok &= ~moved
    # nearest neighbours: hard arg-min of each row (witness 1) / column (witness 2)
    D = np.linalg.norm(e1 - e2, axis=-1)

    def nn_hard(Dm):
        idx = Dm.argmin(1)
        gap = Dm - Dm.min(1, keepdims=True)
        second = np.sort(Dm, axis=1)[:, 1] - Dm.min(1)
        hard = np.zeros_like(Dm)
        hard[np.arange(len(Dm)), idx] = 1.0
        valid = (gap >= margin) | ((hard == 1.0) & (second[:, None] >= margin))
        return hard, valid
    nn1, okn1 = nn_hard(D)
    nn2, okn2 = (m.T for m in nn_hard(D.T))
    pen1, pen2, cl = (np.zeros((nA, nB)) for _ in range(3))
    okp1, okp2, okc = (np.ones((nA, nB), bool) for _ in range(3))
    for k in range(nA):
        for l in range(nB):
            x1, x2 = e1[k, l], e2[k, l]
            gA, _, kinkA = _hard_face_gradient(eqA, x1)
            gB, _, kinkB = _hard_face_gradient(eqB, x2)
            mB1 = _hard_face_gradient(eqB, x1)[1]
            mA2 = _hard_face_gradient(eqA, x2)[1]
            pen1[k, l], okp1[k, l] = float(dlB.find_simplex(x1) >= 0), abs(mB1) > margin
            pen2[k, l], okp2[k, l] = float(dlA.find_simplex(x2) >= 0), abs(mA2) > margin
            dot = gA @ gB
            cl[k, l], okc[k, l] = float(dot < 0), abs(dot) > margin and not (kinkA or kinkB)
    return dict(act=act, con=con, side=side, pen1=pen1, pen2=pen2, nn1=nn1, nn2=nn2, cl=cl,
                v1=ok & okn1 & okp1 & okc, v2=ok & okn2 & okp2 & okc, qp=ex["qp"])


def pin_ee_activity_hard_limit():
    """E-E activity Gamma_b = con * pen_b * nn_b * cl (Sec. IV-D-3) as tau -> 0
    (1e-7, samples at least 1e-4 from every kink), factor by factor against
    independent hard tests on pairs of 14- and 13-point hulls: con against
    the unconstrained least-squares minimiser of the regularised QP lying
    inside the box, pen_b against scipy's Delaunay location of the witness
    (found by bounded-variable least squares) in the other hull, nn_b against
    the arg-min along each row (witness 1) / column (witness 2) of the
    witness distances, cl against the sign of the dot product of the two
    hulls' facet normals at the witnesses.  The seeded pairs must include, for
    every factor, samples where it alone is zero, and samples where the
    row and column indicators differ, so that dropping or exchanging a
    factor changes some activity from 1 to 0 or back.  A weak regulariser
    (lam = 1e-3) makes box-edge minimisers common.  Also exp(log con) = con
    at finite tau."""
    cover = dict(con=0, pen=0, nn=0, cl=0, all=0, swap=0, below=0, above=0)
    for seed in range(20):
        r = _activity_hard_limit(seed, 1e-3)
        G1 = r["con"] * r["pen1"] * r["nn1"] * r["cl"]
        G2 = r["con"] * r["pen2"] * r["nn2"] * r["cl"]
        assert r["v1"].mean() > 0.8 and r["v2"].mean() > 0.8
        assert np.abs(r["act"][..., 0] - G1)[r["v1"]].max() < 1e-6, seed
        assert np.abs(r["act"][..., 1] - G2)[r["v2"]].max() < 1e-6, seed
        f = dict(con=r["con"], pen=r["pen1"], nn=r["nn1"], cl=r["cl"])
        for name in f:
            rest = np.prod([f[o] for o in f if o != name], axis=0)
            cover[name] += int(((f[name] == 0) & (rest == 1) & r["v1"]).sum())
        cover["all"] += int(((G1 == 1) & r["v1"]).sum())
        both = r["v1"] & r["v2"] & (r["con"] * r["cl"] == 1) & (r["nn1"] != r["nn2"])
        cover["swap"] += int((both & ((r["pen1"] == 1) | (r["pen2"] == 1))).sum())
        rest = r["pen1"] * r["nn1"] * r["cl"]
        cover["below"] += int(((r["side"] == -1) & (rest == 1) & r["v1"]).sum())
        cover["above"] += int(((r["side"] == 1) & (rest == 1) & r["v1"]).sum())
    assert min(cover.values()) >= 2, cover
    # log con is the log of con (at finite tau, both sides of the box)
    rng = np.random.default_rng(31)
    E = np.array(_rand_edges(rng, 300)) * 2.0 - 0.5
    with torch.no_grad():
        for tau in (0.3, 0.05):
            q = O.ee_qp(*(T(E[:, i]) for i in range(4)), tau, 0.01)
            assert torch.allclose(torch.exp(q["log_con"]), q["con"], rtol=1e-12, atol=1e-300)
            assert bool((q["au1"] < -0.5).any() and (q["au1"] > 1.5).any())


def _rand_cands(rng, C=60):
    return dict(p=T(rng.normal(size=(C, 3))), nu=T(rng.normal(size=(C, 3))), d=T(rng.normal(0, 0.1, C)),
                logw=T(-np.abs(rng.normal(0, 3, C))))


def pin_manifold_properties():
    """SoftSort manifold: rows sum to 1 (constant fields pass through),
    invariance to candidate order, w_k in [0, 1], and the tau -> 0 limit picks
    the K deepest active candidates in order."""
    rng = np.random.default_rng(16)
    c = _rand_cands(rng)
    K = 6
    m = O.manifold(c, 0.05, K)
    cc = dict(c); cc["d"] = torch.full_like(c["d"], 0.7); cc["p"] = T(np.tile([1.0, -2.0, 3.0], (60, 1)))
    mc = O.manifold(cc, 0.05, K)
    assert torch.allclose(mc["d"], torch.full((K,), 0.7, dtype=DT), atol=1e-13)
    assert torch.allclose(mc["p"], T(np.tile([1.0, -2.0, 3.0], (K, 1))), atol=1e-12)
    perm = torch.as_tensor(rng.permutation(60))
    mp = O.manifold({k: v[perm] for k, v in c.items()}, 0.05, K)
    for k in ("p", "nu", "d", "w"):
        assert torch.allclose(m[k], mp[k], atol=1e-12)
    assert bool((m["w"] >= 0).all()) and bool((m["w"] <= 1).all())
    # tau -> 0: only active (w = 1) candidates, deepest (most negative d) first
    act = rng.uniform(size=60) < 0.4
    c2 = dict(c); c2["logw"] = T(np.where(act, 0.0, -1e6))
    m2 = O.manifold(c2, 1e-7, K)
    ref = np.sort(c["d"].numpy()[act])[:K]
    assert np.allclose(m2["d"].numpy(), ref, atol=1e-6)
    assert np.allclose(m2["w"].numpy(), 1.0, atol=1e-6)


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _pair_case(kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "poly":
        GA = O.make_geom(O.POLYTOPE, points=W.ellipsoid_points(rng, 14, [0.45, 0.35, 0.4]))
        GB = O.make_geom(O.POLYTOPE, points=W.ellipsoid_points(rng, 12, [0.3, 0.45, 0.35]))
    elif kind == "capbox":
        GA = O.make_geom(O.CAPSULE, params=[0.15, 0.3, 0, 0])
        GB = O.make_geom(O.BOX, params=[0.3, 0.25, 0.2, 0.02])
    else:
        GA = O.make_geom(O.SPHERE, params=[0.35, 0, 0, 0])
        GB = O.make_geom(O.POLYTOPE, points=W.ellipsoid_points(rng, 12, [0.3, 0.45, 0.35]))
    qA, qB = W.uniform_quats(rng, 2)
    return GA, _pose(qA, rng.uniform(-0.2, 0.2, 3)), GB, _pose(qB, rng.uniform(-0.2, 0.2, 3) + [0.35, 0.1, 0])


def pin_rigid_motion_invariance():
    """Moving both bodies by one rigid motion moves p, rotates nu and leaves d, w."""
    rng = np.random.default_rng(17)
    for kind, seed in (("poly", 1), ("capbox", 2), ("sphpoly", 3)):
        GA, pA, GB, pB = _pair_case(kind, seed)
        qg = W.uniform_quats(rng, 1)[0]
        tg = rng.uniform(-1, 1, 3)
        Rg = O.quat_to_R(T(qg)).numpy()
        move = lambda p: _pose(_quat_mul(qg, p[:4]), Rg @ p[4:] + tg)
        with torch.no_grad():
            m = O.collide_pair(GA, pA, GB, pB, 0.02, 8)
            mm = O.collide_pair(GA, move(pA), GB, move(pB), 0.02, 8)
        assert np.allclose(mm["p"].numpy(), m["p"].numpy() @ Rg.T + tg, atol=1e-9)
        assert np.allclose(mm["nu"].numpy(), m["nu"].numpy() @ Rg.T, atol=1e-9)
        assert np.allclose(mm["d"].numpy(), m["d"].numpy(), atol=1e-9)
        assert np.allclose(mm["w"].numpy(), m["w"].numpy(), atol=1e-9)


def pin_pair_swap_antisymmetry():
    """collide(B, A) = collide(A, B) with nu negated and p, d, w unchanged."""
    for kind, seed in (("poly", 4), ("capbox", 5), ("sphpoly", 6)):
        GA, pA, GB, pB = _pair_case(kind, seed)
        with torch.no_grad():
            m = O.collide_pair(GA, pA, GB, pB, 0.02, 8)
            s = O.collide_pair(GB, pB, GA, pA, 0.02, 8)
        assert np.allclose(s["nu"].numpy(), -m["nu"].numpy(), atol=1e-9)
        for k in ("p", "d", "w"):
            assert np.allclose(s[k].numpy(), m[k].numpy(), atol=1e-9)


def pin_simplification_flags():
    """Ours-NE / Ours-NE-S (supplementary material): a polytope A against a
    sphere B.  One-sided V-S candidates are exactly A's hull points in world
    coordinates with the closed-form sphere distance |v - c| - r; without E-E
    the candidate list is both bodies' vertices; K beyond the candidate count
    leaves empty rows and does not change the others; dropping E-E keeps the
    pair-swap antisymmetry."""
    rng = np.random.default_rng(41)
    pts = W.ellipsoid_points(rng, 14, [0.45, 0.35, 0.4])
    GA = O.make_geom(O.POLYTOPE, points=pts)
    r = 0.3
    GB = O.make_geom(O.SPHERE, params=[r, 0, 0, 0])
    qA, qB = W.uniform_quats(rng, 2)
    pA, pB = _pose(qA, [0.0, 0.0, 0.0]), _pose(qB, [0.55, 0.1, -0.05])
    tau = 0.02
    RA, tA = O.pose_Rt(pA)
    RB, tB = O.pose_Rt(pB)
    with torch.no_grad():
        full = O.pair_candidates(GA, RA, tA, GB, RB, tB, tau)
        ne = O.pair_candidates(GA, RA, tA, GB, RB, tB, tau, no_ee=True)
        nes = O.pair_candidates(GA, RA, tA, GB, RB, tB, tau, no_ee=True, one_sided_vs=True)
    hull = np.unique(np.asarray(GA.edges).reshape(-1))
    nA, nB = len(hull), GB.vertices().shape[0]
    assert nes["d"].shape[0] == nA and ne["d"].shape[0] == nA + nB
    assert full["d"].shape[0] == nA + nB + 2 * GA.edges.shape[0] * GB.edges.shape[0]
    Rq = O.quat_to_R(T(qA)).numpy()
    vw = np.asarray(GA.vertices(), float) @ Rq.T
    assert np.allclose(nes["p"].numpy(), vw, atol=1e-12)
    # the hull points of the mesh are the input points that are hull vertices
    assert all(np.abs(pts.astype(float) - v).max(axis=1).min() < 1e-6 for v in np.asarray(GA.vertices(), float))
    c = np.asarray(pB[4:], float)
    d_ref = np.linalg.norm(vw - c, axis=1) - r
    assert np.allclose(nes["d"].numpy(), d_ref, atol=1e-12)
    for k in ("p", "nu", "d", "logw"):
        assert torch.equal(ne[k], full[k][:nA + nB])
    K = nA + 5
    m_full = O.manifold(nes, tau, nA)
    m_pad = O.manifold(nes, tau, K)
    for k in ("p", "nu", "d", "w"):
        assert torch.allclose(m_pad[k][:nA], m_full[k], atol=1e-14)
        assert bool((m_pad[k][nA:] == 0).all())
    with torch.no_grad():
        m = O.collide_pair(GA, pA, GB, pB, tau, 6, no_ee=True)
        s = O.collide_pair(GB, pB, GA, pA, tau, 6, no_ee=True)
    assert np.allclose(s["nu"].numpy(), -m["nu"].numpy(), atol=1e-9)
    for k in ("p", "d", "w"):
        assert np.allclose(s[k].numpy(), m[k].numpy(), atol=1e-9)


def pin_soft_topk():
    """SoftSort selection rows: stochastic, invariant to reordering the
    inputs (columns move with them), one-hot on the sorted top-K as tau -> 0,
    Gamma x -> the K largest values in order."""
    rng = np.random.default_rng(51)
    x = T(rng.normal(size=40))
    G = O.soft_topk(x, 7, 0.3)
    assert torch.allclose(G.sum(1), torch.ones(7, dtype=DT), atol=1e-14)
    perm = torch.as_tensor(rng.permutation(40))
    Gp = O.soft_topk(x[perm], 7, 0.3)
    assert torch.allclose(Gp, G[:, perm], atol=1e-14)
    G0 = O.soft_topk(x, 7, 1e-6)
    order = np.argsort(-x.numpy())[:7]
    assert np.allclose(G0.numpy(), np.eye(40)[order], atol=1e-12)
    assert np.allclose((G0 @ x).numpy(), np.sort(x.numpy())[::-1][:7], atol=1e-12)


def pin_preselect_against_sphere():
    """Pre-selection of a polytope's vertices and edges against a sphere: the
    metrics are the closed-form distance |v - c| - r, so as tau -> 0 the soft
    vertices are the K_V vertices nearest the sphere's surface (deepest first)
    and the soft edges those with the smallest mean corner metric."""
    rng = np.random.default_rng(52)
    GA = O.make_geom(O.POLYTOPE, points=W.ellipsoid_points(rng, 20, [0.45, 0.35, 0.4]))
    GB = O.make_geom(O.SPHERE, params=[0.3, 0, 0, 0])
    qA, qB = W.uniform_quats(rng, 2)
    pA, pB = _pose(qA, [0.0, 0.0, 0.0]), _pose(qB, [0.5, 0.1, -0.05])
    tau = 1e-7
    RA, tA = O.pose_Rt(pA)
    RB, tB = O.pose_Rt(pB)
    with torch.no_grad():
        sVA, sVB, a0, a1, b0, b1 = O.preselect(GA, RA, tA, GB, RB, tB, tau, 5, 6)
    vw = np.asarray(GA.vertices(), float) @ O.quat_to_R(T(qA)).numpy().T
    m = np.linalg.norm(vw - np.asarray(pB[4:], float), axis=1) - 0.3
    order = np.argsort(m)
    assert np.allclose(sVA.numpy(), vw[order[:5]], atol=1e-9)
    E = np.asarray(GA.edges)
    me = 0.5 * (m[E[:, 0]] + m[E[:, 1]])
    eo = np.argsort(me)[:6]
    assert np.allclose(a0.numpy(), vw[E[eo, 0]], atol=1e-9) and np.allclose(a1.numpy(), vw[E[eo, 1]], atol=1e-9)
    assert sVB.shape == (5, 3) and b0.shape == (6, 3)


def pin_preselect_everything_limit():
    """Selecting every vertex and edge with sharp SoftSort rows gives back the
    full method: the same candidates in another order, hence the same
    manifold (the manifold does not depend on candidate order)."""
    for kind, seed in (("poly", 53), ("capbox", 54)):
        GA, pA, GB, pB = _pair_case(kind, seed)
        tau = 1e-5
        nv = max(GA.vertices().shape[0], GB.vertices().shape[0])
        ne = max(GA.edges.shape[0], GB.edges.shape[0])
        with torch.no_grad():
            full = O.collide_pair(GA, pA, GB, pB, tau, 6)
            sel = O.collide_pair(GA, pA, GB, pB, tau, 6, presel=(nv, ne))
        for k in ("p", "nu", "d", "w"):
            assert np.allclose(sel[k].numpy(), full[k].numpy(), atol=1e-8), (kind, k)


def pin_preselect_safeguard():
    """Safeguard: edges taken from the bodies' own meshes have witnesses on
    their own surfaces, where the smoothed SDF is >= 0, so both inside
    indicators are <= 1/2 and every E-E log-activity drops by >= 2 ln 2;
    vertex candidates are untouched."""
    GA, pA, GB, pB = _pair_case("poly", 55)
    tau = 1e-4   # sharp selection: the soft edges are mesh edges
    RA, tA = O.pose_Rt(pA)
    RB, tB = O.pose_Rt(pB)
    with torch.no_grad():
        c0 = O.pair_candidates(GA, RA, tA, GB, RB, tB, tau, presel=(4, 5))
        c1 = O.pair_candidates(GA, RA, tA, GB, RB, tB, tau, presel=(4, 5), safeguard=True)
    nvs = c0["extra"]["n_vs"]
    assert torch.equal(c0["logw"][:nvs], c1["logw"][:nvs])
    drop = (c1["logw"][nvs:] - c0["logw"][nvs:]).numpy()
    assert drop.shape[0] == 2 * 5 * 5 and np.all(drop <= -2 * math.log(2) + 1e-6), drop.max()


# ----------------------------------------------------------------------------- gradients

def _loss_fd(GA, pA, GB, pB, tau, K, cot, xiA, xiB):
    with torch.no_grad():
        m = O.collide_pair(GA, pA, GB, pB, tau, K, xiA=T(xiA), xiB=T(xiB), exact_exp=True)
        return sum(float((m[k] * T(v)).sum()) for k, v in cot.items())


def _cot(rng, K):
    return dict(p=rng.normal(size=(K, 3)), nu=rng.normal(size=(K, 3)), d=rng.normal(size=K), w=rng.normal(size=K))


def pin_gradients_fd():
    """Autograd gradients (pose twists, geometry parameters, tau) vs FP64 central
    differences, h = 1e-6."""
    rng = np.random.default_rng(18)
    h = 1e-6
    for kind, seed in (("poly", 7), ("capbox", 8), ("sphpoly", 9)):
        GA, pA, GB, pB = _pair_case(kind, seed)
        tau, K = 0.03, 6
        cot = _cot(rng, K)
        GAg = O.make_geom(GA.kind, params=None if GA.params is None else GA.params.detach().numpy(),
                          points=None if GA.points is None else _orig_points(GA), requires_grad=True)
        GBg = O.make_geom(GB.kind, params=None if GB.params is None else GB.params.detach().numpy(),
                          points=None if GB.points is None else _orig_points(GB), requires_grad=True)
        g = O.pair_grad(GAg, pA, GBg, pB, tau, K, cot)
        z = np.zeros(6)
        for j in range(6):
            e = np.zeros(6); e[j] = h
            fdA = (_loss_fd(GA, pA, GB, pB, tau, K, cot, e, z) - _loss_fd(GA, pA, GB, pB, tau, K, cot, -e, z)) / (2 * h)
            fdB = (_loss_fd(GA, pA, GB, pB, tau, K, cot, z, e) - _loss_fd(GA, pA, GB, pB, tau, K, cot, z, -e)) / (2 * h)
            assert abs(fdA - g["xiA"][j]) <= 1e-5 * (1 + abs(fdA)), (kind, "A", j, fdA, g["xiA"][j])
            assert abs(fdB - g["xiB"][j]) <= 1e-5 * (1 + abs(fdB)), (kind, "B", j, fdB, g["xiB"][j])
        # tau
        def L_tau(tv):
            with torch.no_grad():
                m = O.collide_pair(GA, pA, GB, pB, tv, K)
                return sum(float((m[k] * T(v)).sum()) for k, v in cot.items())
        fd = (L_tau(tau + h) - L_tau(tau - h)) / (2 * h)
        assert abs(fd - g["tau"]) <= 1e-5 * (1 + abs(fd)), (kind, "tau", fd, g["tau"])
        # geometry of A along a random direction
        dirv = rng.normal(size=g["geomA"].shape)
        Lg = []
        for sgn in (1, -1):
            if GA.kind == O.POLYTOPE:
                G2 = O.OGeom(O.POLYTOPE, points=GA.points.detach() + sgn * h * T(dirv), vertex_ids=GA.vertex_ids,
                             edges=GA.edges, tris=GA.tris)
            else:
                G2 = O.make_geom(GA.kind, params=GA.params.detach().numpy() + sgn * h * dirv)
            with torch.no_grad():
                m = O.collide_pair(G2, pA, GB, pB, tau, K)
            Lg.append(sum(float((m[k] * T(v)).sum()) for k, v in cot.items()))
        fd = (Lg[0] - Lg[1]) / (2 * h)
        an = float((g["geomA"] * dirv).sum())
        assert abs(fd - an) <= 1e-5 * (1 + abs(fd)), (kind, "geom", fd, an)


def _orig_points(G):
    return G.points.detach().numpy()


def pin_gradient_joint_motion_identities():
    """Joint translation: sum_b dL/drho_b = sum_k dL/dp_k.  Joint rotation:
    sum_b dL/domega_b = sum_k p_k x dL/dp_k + nu_k x dL/dnu_k."""
    rng = np.random.default_rng(19)
    for kind, seed in (("poly", 10), ("capbox", 11)):
        GA, pA, GB, pB = _pair_case(kind, seed)
        K = 8
        cot = _cot(rng, K)
        g = O.pair_grad(GA, pA, GB, pB, 0.02, K, cot)
        f = g["fwd"]
        jt = g["xiA"][:3] + g["xiB"][:3]
        assert np.allclose(jt, cot["p"].sum(0), atol=1e-9)
        jr = g["xiA"][3:] + g["xiB"][3:]
        ref = np.cross(f["p"], cot["p"]).sum(0) + np.cross(f["nu"], cot["nu"]).sum(0)
        assert np.allclose(jr, ref, atol=1e-9)


def pin_broadphase_f32():
    """Float32 bounding-sphere predicate agrees with an FP64 evaluation away
    from the boundary; offsets are the exclusive scan of per-scene counts."""
    b = W.mixed_scenes(64, seed=3)
    pairs, off = O.broadphase(b)
    sc, a, bb = b.candidate_pairs()
    gs = b.geoms
    R = []
    for g in range(gs.n):
        k = int(gs.types[g]); p = gs.params[g].astype(np.float64)
        if k == O.SPHERE: R.append(p[0])
        elif k == O.CAPSULE: R.append(p[0] + p[1])
        elif k == O.BOX: R.append(np.linalg.norm(p[:3]))
        else: R.append(np.linalg.norm(gs.points_of(g).astype(np.float64), axis=1).max())
    R = np.array(R)
    t = b.pose[4:7].astype(np.float64)
    dist = np.linalg.norm(t[:, bb] - t[:, a], axis=0)
    rr = R[b.body_geom[a]] + R[b.body_geom[bb]] + 10 * b.tau
    keep64 = dist <= rr
    safe = np.abs(dist - rr) > 1e-5
    kept = set(zip(pairs[0].tolist(), pairs[1].tolist()))
    mine = np.array([(x, y) in kept for x, y in zip(a.tolist(), bb.tolist())])
    assert np.array_equal(mine[safe], keep64[safe])
    cnt = np.bincount(sc[mine], minlength=b.n_scenes)
    assert np.array_equal(off, np.concatenate([[0], np.cumsum(cnt)]))


# ----------------------------------------------------------------------------- superquadric unions

def _sq_rec(ax, e1, e2, t=(0.0, 0.0, 0.0), q=(1.0, 0.0, 0.0, 0.0)):
    return T([[ax[0], ax[1], ax[2], e1, e2, t[0], t[1], t[2], q[0], q[1], q[2], q[3]]])


def pin_sq_sphere_limit():
    """eps1 = eps2 = 1 with equal semi-axes is a sphere: phi = |x - t| - r
    exactly, grad phi = (x - t) / |x - t|, and the V-S normal direction
    (grad f) is parallel to it."""
    rng = np.random.default_rng(11)
    for _ in range(3):
        r = rng.uniform(0.1, 0.5)
        t = rng.uniform(-0.5, 0.5, 3)
        q = Rotation.random(random_state=rng).as_quat()[[3, 0, 1, 2]]
        rec = _sq_rec((r, r, r), 1.0, 1.0, t, q)
        x = T(rng.uniform(-1, 1, (40, 3)))
        phi, g, nd = O.sq_union_sdf(rec, x, 0.01)
        d = x - T(t)
        nrm = torch.sqrt((d * d).sum(-1))
        assert torch.allclose(phi, nrm - r, atol=1e-12)
        assert torch.allclose(g, d / nrm[:, None], atol=1e-10)
        ndn = nd / torch.sqrt((nd * nd).sum(-1, keepdim=True))
        assert torch.allclose(ndn, d / nrm[:, None], atol=1e-10)


def pin_sq_axis_distance():
    """Along a primitive's own axes the radial SDF is the exact distance to
    the surface: at s a e_x it is a (s - 1), at s c e_z it is c (s - 1), for
    any exponents (the surface crosses the axes at the semi-axes)."""
    for ax, e1, e2 in [((0.3, 0.2, 0.5), 0.4, 1.3), ((0.15, 0.4, 0.25), 1.7, 0.6)]:
        rec = _sq_rec(ax, e1, e2)
        for s in (0.5, 1.3, 2.0):
            x = T([[s * ax[0], 0, 0], [0, s * ax[1], 0], [0, 0, s * ax[2]]])
            phi, _, _ = O.sq_union_sdf(rec, x, 0.01)
            ref = T([ax[0] * (s - 1), ax[1] * (s - 1), ax[2] * (s - 1)])
            assert torch.allclose(phi, ref, atol=1e-12), (phi, ref)


def pin_sq_surface_and_mesh():
    """Parametric samples lie on their primitive's surface (f = 1, and the
    union of one primitive is that primitive exactly); kept mesh vertices lie
    outside every other primitive; a primitive inside another keeps none."""
    rng = W._rng(6, 5)
    rec = T(W.sq_union_records(rng, 4).reshape(-1, 12).astype(np.float64))
    samples, _ = O.sq_local_topology()
    for i in range(rec.shape[0]):
        pts = O.sq_points(rec[i:i + 1], [(0, k) for k in range(len(samples))])
        ax, e1, e2, R, t = O.sq_unpack(rec[i:i + 1])
        y = ((pts[:, None, :] - t)[:, :, None, :] @ R).squeeze(-2)
        f, _ = O.sq_inside_outside(y, ax, e1, e2)
        assert torch.allclose(f, torch.ones_like(f), atol=1e-12)
        phi, _, _ = O.sq_union_sdf(rec[i:i + 1], pts, 0.01)
        assert phi.abs().max() < 1e-12
    keep, E = O.sq_union_mesh(rec.numpy())
    V = O.sq_points(rec, keep)
    ax, e1, e2, R, t = O.sq_unpack(rec)
    y = ((V[:, None, :] - t)[:, :, None, :] @ R).squeeze(-2)
    f, _ = O.sq_inside_outside(y, ax, e1, e2)
    for j, (i, _) in enumerate(keep):
        others = [m for m in range(rec.shape[0]) if m != i]
        assert bool((f[j, others] >= 1.0).all())
    assert E.max() < len(keep)
    nested = torch.cat([_sq_rec((0.5, 0.5, 0.5), 1.0, 1.0), _sq_rec((0.1, 0.1, 0.1), 0.8, 0.8, (0.05, 0, 0))])
    keep2, _ = O.sq_union_mesh(nested.numpy())
    assert all(i == 0 for i, _ in keep2) and len(keep2) == 32


def pin_sq_gradients_fd():
    """grad phi of a union of 3 superquadrics and grad f of each primitive
    match central finite differences."""
    rng = W._rng(6, 7)
    rec = T(W.sq_union_records(rng, 3).reshape(-1, 12).astype(np.float64))
    x = T(np.random.default_rng(8).uniform(-0.6, 0.6, (25, 3)))
    tau, h = 0.05, 1e-6
    phi, g, _ = O.sq_union_sdf(rec, x, tau)
    ax, e1, e2, R, t = O.sq_unpack(rec)
    ys = ((x[:, None, :] - t)[:, :, None, :] @ R).squeeze(-2)
    f, gf = O.sq_inside_outside(ys, ax, e1, e2)
    for k in range(3):
        dx = torch.zeros(3, dtype=DT); dx[k] = h
        fd = (O.sq_union_sdf(rec, x + dx, tau)[0] - O.sq_union_sdf(rec, x - dx, tau)[0]) / (2 * h)
        assert torch.allclose(fd, g[:, k], rtol=1e-5, atol=1e-6), (fd - g[:, k]).abs().max()
        dy = torch.zeros(3, dtype=DT); dy[k] = h
        fp, _ = O.sq_inside_outside(ys + dy, ax, e1, e2)
        fm, _ = O.sq_inside_outside(ys - dy, ax, e1, e2)
        fdf = (fp - fm) / (2 * h)
        assert torch.allclose(fdf, gf[..., k], rtol=1e-5, atol=1e-5 * float(gf.abs().max())), \
            (fdf - gf[..., k]).abs().max()


def pin_sq_union_bounds():
    """The smooth union lies between min_i phi_i - tau ln M and min_i phi_i,
    and tends to the hard union as tau -> 0."""
    rng = W._rng(6, 9)
    rec = T(W.sq_union_records(rng, 6).reshape(-1, 12).astype(np.float64))
    x = T(np.random.default_rng(10).uniform(-0.8, 0.8, (60, 3)))
    mins = torch.stack([O.sq_union_sdf(rec[i:i + 1], x, 0.01)[0] for i in range(6)]).min(0).values
    for tau in (0.05, 0.01):
        phi, _, _ = O.sq_union_sdf(rec, x, tau)
        assert bool((phi <= mins + 1e-12).all()) and bool((phi >= mins - tau * math.log(6) - 1e-12).all())
    phi0, _, _ = O.sq_union_sdf(rec, x, 1e-7)
    assert torch.allclose(phi0, mins, atol=1e-6)


def pin_sq_rigid_invariance():
    """Moving every primitive and the query points by one rigid motion leaves
    phi unchanged and rotates grad phi and the normal direction."""
    rng = W._rng(6, 12)
    rec = W.sq_union_records(rng, 4).reshape(-1, 12).astype(np.float64)
    Rm = Rotation.random(random_state=np.random.default_rng(13))
    d = np.array([0.3, -0.2, 0.1])
    moved = rec.copy()
    moved[:, 5:8] = Rm.apply(rec[:, 5:8]) + d
    qs = (Rm * Rotation.from_quat(rec[:, [9, 10, 11, 8]])).as_quat()
    moved[:, 8:12] = qs[:, [3, 0, 1, 2]]
    x = np.random.default_rng(14).uniform(-0.6, 0.6, (30, 3))
    p0, g0, n0 = O.sq_union_sdf(T(rec), T(x), 0.01)
    p1, g1, n1 = O.sq_union_sdf(T(moved), T(Rm.apply(x) + d), 0.01)
    Q = T(Rm.as_matrix())
    assert torch.allclose(p0, p1, atol=1e-10)
    assert torch.allclose(g0 @ Q.T, g1, atol=1e-8)
    assert torch.allclose(n0 @ Q.T, n1, rtol=1e-8, atol=1e-8 * float(n0.abs().max()))


# ----------------------------------------------------------------------------- witness sphere tracing

def pin_sphere_trace_metric_one_step():
    """For a metric SDF (sphere, capsule) one tracing step along the unit
    gradient lands exactly on the surface, from outside and from inside."""
    rng = np.random.default_rng(21)
    I = torch.eye(3, dtype=DT)
    z = torch.zeros(3, dtype=DT)
    for kind, prm in ((O.SPHERE, [0.3, 0, 0, 0]), (O.CAPSULE, [0.15, 0.3, 0, 0])):
        G = O.make_geom(kind, params=np.array(prm, np.float32))
        x = T(rng.uniform(-0.7, 0.7, (50, 3)))
        y = O.sphere_trace(G, I, z, x, 0.01, None, 1)
        phi, _ = O.sdf_world(G, I, z, y, 0.01)
        assert phi.abs().max() < 1e-12, phi.abs().max()


def pin_sphere_trace_polytope_converges():
    """On the tau-LSE polytope SDF (metric away from the smoothed edges, not
    on them) tracing from points on the hull's edges converges: every step
    at least halves the largest |phi|, five steps reach below 5e-3 of it."""
    rng = np.random.default_rng(22)
    pts = W.ellipsoid_points(rng, 24, [0.4, 0.3, 0.25]).astype(np.float32)
    G = O.make_geom(O.POLYTOPE, points=pts)
    V = G.vertices()
    E = torch.as_tensor(G.edges)
    al = T(rng.uniform(0.1, 0.9, (len(E), 1)))
    x = V[E[:, 0]] * (1 - al) + V[E[:, 1]] * al
    I = torch.eye(3, dtype=DT)
    z = torch.zeros(3, dtype=DT)
    tau = 0.01
    phi0, _ = O.sdf_world(G, I, z, x, tau)
    assert phi0.min() > 0   # the smoothed surface lies outside the mesh edges
    prev = float(phi0.abs().max())
    for k in range(1, 6):
        y = O.sphere_trace(G, I, z, x, tau, None, k)
        phi, _ = O.sdf_world(G, I, z, y, tau)
        cur = float(phi.abs().max())
        assert cur <= 0.5 * prev, (k, cur, prev)
        prev = cur
    assert prev < 5e-3 * float(phi0.abs().max())


def pin_refined_witnesses_on_own_surfaces():
    """With tracing, each E-E witness lies on its own body's smoothed surface
    (e1 on A, e2 on B), and the QP distances still rank the nearest
    neighbours (the indicators equal the unrefined ones)."""
    b = W.cube_pairs(4, seed=23)
    G = O.make_geom(int(b.geoms.types[0]), params=b.geoms.params[0])
    RA, tA = O.pose_Rt(b.pose[:, 0])
    RB, tB = O.pose_Rt(b.pose[:, 1])
    c0 = O.pair_candidates(G, RA, tA, G, RB, tB, b.tau)
    c1 = O.pair_candidates(G, RA, tA, G, RB, tB, b.tau, refine=6)
    e1, e2 = c1["extra"]["e1"], c1["extra"]["e2"]
    pA, _ = O.sdf_world(G, RA, tA, e1, b.tau)
    pB, _ = O.sdf_world(G, RB, tB, e2, b.tau)
    assert pA.abs().max() < 1e-6 and pB.abs().max() < 1e-6, (pA.abs().max(), pB.abs().max())
    assert torch.equal(c0["extra"]["log_nn1"], c1["extra"]["log_nn1"])
    assert not torch.allclose(c0["d"], c1["d"])


# ----------------------------------------------------------------------------- oriented point clouds

def _opc_rec(p, n, sg):
    p = np.asarray(p, np.float64).reshape(-1, 3)
    n = np.asarray(n, np.float64).reshape(-1, 3)
    sg = np.broadcast_to(np.asarray(sg, np.float64), (len(p),))
    return T(np.concatenate([p, n, sg[:, None], np.zeros((len(p), 2))], axis=1))


def pin_opc_single_point_and_plane():
    """One oriented point is its tangent plane: phi = n . (x - p), grad = n.
    Points on a plane with its normal reproduce the plane exactly for any
    bandwidths (the weights sum to one)."""
    rng = np.random.default_rng(31)
    x = T(rng.uniform(-1, 1, (40, 3)))
    n0 = np.array([0.3, -0.5, 0.8]); n0 /= np.linalg.norm(n0)
    p0 = np.array([0.1, 0.2, -0.1])
    phi, g = O.opc_sdf(_opc_rec(p0, n0, 0.2), x)
    assert torch.allclose(phi, (x - T(p0)) @ T(n0), atol=1e-13)
    assert torch.allclose(g, T(n0).expand_as(g), atol=1e-13)
    pts = np.concatenate([rng.uniform(-1, 1, (30, 2)), np.zeros((30, 1))], axis=1)
    phi, g = O.opc_sdf(_opc_rec(pts, np.tile([0, 0, 1.0], (30, 1)), rng.uniform(0.05, 0.3, 30)), x)
    assert torch.allclose(phi, x[:, 2], atol=1e-12)
    assert torch.allclose(g, T([0, 0, 1.0]).expand_as(g), atol=1e-10)


def pin_opc_sphere_near_surface():
    """Dense samples of a sphere with radial normals approximate its SDF near
    the surface (averaging tangent planes biases it by about sigma^2 / r:
    within 5 % of the radius here) with unit-length gradients."""
    rng = np.random.default_rng(32)
    r = 0.3
    d = W.ellipsoid_points(rng, 400, [1, 1, 1])
    rec = _opc_rec(r * d, d, 0.03)
    u = W.ellipsoid_points(rng, 60, [1, 1, 1])
    x = T(u * rng.uniform(0.9 * r, 1.1 * r, (60, 1)))
    phi, g = O.opc_sdf(rec, x)
    ref = torch.sqrt((x * x).sum(-1)) - r
    assert (phi - ref).abs().max() < 0.05 * r, (phi - ref).abs().max()
    assert ((g.norm(dim=-1) - 1).abs() < 0.1).all()


def pin_opc_gradient_fd():
    """grad phi of an oriented point cloud matches central differences."""
    rng = W._rng(8, 3)
    rec = T(W.opc_torus_records(rng).reshape(-1, 9).astype(np.float64))
    x = T(np.random.default_rng(33).uniform(-0.45, 0.45, (30, 3)))
    phi, g = O.opc_sdf(rec, x)
    h = 1e-6
    for k in range(3):
        dx = torch.zeros(3, dtype=DT); dx[k] = h
        fd = (O.opc_sdf(rec, x + dx)[0] - O.opc_sdf(rec, x - dx)[0]) / (2 * h)
        assert torch.allclose(fd, g[:, k], rtol=1e-5, atol=1e-6), (fd - g[:, k]).abs().max()


def pin_opc_knn_edges():
    """The mesh edges are the undirected 4-nearest-neighbour graph (against
    scipy's k-d tree)."""
    from scipy.spatial import cKDTree
    P = np.random.default_rng(34).uniform(-1, 1, (60, 3))
    E = O.opc_knn_edges(P)
    _, nb = cKDTree(P).query(P, k=O.OPC_KNN + 1)
    ref = sorted({(min(i, j), max(i, j)) for i in range(len(P)) for j in nb[i, 1:]})
    assert sorted(map(tuple, E.tolist())) == ref


def pin_opc_rigid_invariance():
    """Rotating and translating the points, their normals and the query
    leaves phi unchanged and rotates the gradient."""
    rng = W._rng(8, 4)
    rec = W.opc_torus_records(rng).reshape(-1, 9).astype(np.float64)
    Rm = Rotation.random(random_state=np.random.default_rng(35))
    d = np.array([0.2, -0.1, 0.3])
    moved = rec.copy()
    moved[:, 0:3] = Rm.apply(rec[:, 0:3]) + d
    moved[:, 3:6] = Rm.apply(rec[:, 3:6])
    x = np.random.default_rng(36).uniform(-0.4, 0.4, (25, 3))
    p0, g0 = O.opc_sdf(T(rec), T(x))
    p1, g1 = O.opc_sdf(T(moved), T(Rm.apply(x) + d))
    assert torch.allclose(p0, p1, atol=1e-12)
    assert torch.allclose(g0 @ T(Rm.as_matrix()).T, g1, atol=1e-10)


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
