"""Host geometry builder of the library (hull, meshes, planes, bounding radii)
against the oracle's independent construction (scipy Qhull, numpy float32).

The library's geometry.cpp is compiled here with g++ through a test shim, so
this runs without a GPU.  Integer topology must agree exactly."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest
import torch

import workloads as W
from oracle import cm_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_20304_amd", "csrc")


@pytest.fixture(scope="module")
def shim():
    out = os.path.join(tempfile.mkdtemp(), "libmeshshim.so")
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-ffp-contract=off", "-I", CSRC,
           os.path.join(ROOT, "tests", "host", "mesh_shim.cpp"), os.path.join(CSRC, "geometry.cpp"), "-o", out]
    subprocess.run(cmd, check=True)
    lib = C.CDLL(out)
    lib.shim_build_mesh.restype = C.c_int
    return lib


def build(lib, kind, params, pts=None):
    params = np.asarray(params, np.float32)
    P = np.zeros((1, 3), np.float32) if pts is None else np.ascontiguousarray(pts, np.float32)
    n = 0 if pts is None else len(P)
    cap = max(4 * n + 64, 128)
    v = np.zeros(3 * cap, np.float32); e = np.zeros(6 * cap, np.int32); f = np.zeros(6 * cap, np.int32)
    pl = np.zeros(8 * cap, np.float32); nv = C.c_int(); ne = C.c_int(); nf = C.c_int(); br = C.c_float()
    err = C.create_string_buffer(256)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    ok = lib.shim_build_mesh(kind, ptr(params), ptr(P), C.c_long(n), ptr(v), C.byref(nv), ptr(e), C.byref(ne),
                             ptr(f), C.byref(nf), ptr(pl), C.byref(br), err)
    if not ok:
        return None, err.value.decode()
    return dict(v=v[:3 * nv.value].reshape(-1, 3), e=e[:2 * ne.value].reshape(-1, 2),
                f=f[:3 * nf.value].reshape(-1, 3), planes=pl[:4 * nf.value].reshape(-1, 4), bound=br.value), ""


def test_polytope_hulls_match_oracle(shim):
    rng = np.random.default_rng(0)
    for n in [4, 8, 13, 32, 64, 100, 256]:
        for _ in range(3):
            pts = W.ellipsoid_points(rng, n, rng.uniform(0.2, 0.6, 3)).astype(np.float32)
            m, err = build(shim, W.POLYTOPE, [0, 0, 0, 0], pts)
            assert m is not None, err
            vid, tris, edges = O.hull_topology(pts)
            # same vertex set (library keeps input order) and identical triangle / edge sets
            assert np.array_equal(m["v"], pts[vid])
            key = lambda T: sorted(tuple(sorted(t)) for t in T.tolist())
            assert key(m["f"]) == key(tris)
            assert sorted(map(tuple, m["e"].tolist())) == sorted(map(tuple, edges.tolist()))
            # orientation: each library triangle's normal points outward like the oracle's
            G = O.make_geom(O.POLYTOPE, points=pts)
            n_ref, o_ref = (x.detach().numpy() for x in G.planes())
            ref_of = {tuple(sorted(t)): (n_ref[i], o_ref[i]) for i, t in enumerate(G.tris.tolist())}
            for t, pl in zip(m["f"].tolist(), m["planes"]):
                nr, orf = ref_of[tuple(sorted(t))]
                assert np.allclose(pl[:3], nr, atol=2e-7) and abs(pl[3] - orf) < 2e-7
            assert np.float32(m["bound"]) == O.bound_radius_f32(O.POLYTOPE, None, pts)


def test_hull_with_interior_points(shim):
    rng = np.random.default_rng(1)
    pts = np.concatenate([W.ellipsoid_points(rng, 40, [0.5, 0.4, 0.3]),
                          0.1 * rng.uniform(-1, 1, (20, 3))]).astype(np.float32)
    m, err = build(shim, W.POLYTOPE, [0, 0, 0, 0], pts)
    assert m is not None, err
    vid, tris, edges = O.hull_topology(pts)
    assert len(m["v"]) == len(vid) == 40
    assert np.array_equal(m["v"], pts[vid])


def test_degenerate_polytopes_rejected(shim):
    flat = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [0.5, 0.5, 0]], np.float32)
    m, err = build(shim, W.POLYTOPE, [0, 0, 0, 0], flat)
    assert m is None and "coplanar" in err
    m, err = build(shim, W.POLYTOPE, [0, 0, 0, 0], flat[:3])
    assert m is None
    m, err = build(shim, W.POLYTOPE, [0, 0, 0, 0], np.zeros((6, 3), np.float32))
    assert m is None


@pytest.mark.parametrize("kind,params", [(W.SPHERE, [0.3, 0, 0, 0]), (W.CAPSULE, [0.12, 0.35, 0, 0]),
                                         (W.BOX, [0.5, 0.25, 0.125, 0.02])])
def test_analytic_meshes_match_oracle(shim, kind, params):
    m, err = build(shim, kind, params)
    assert m is not None, err
    G = O.make_geom(kind, params=np.float32(params))
    with torch.no_grad():
        V = G.vertices().numpy()
    assert np.array_equal(m["e"], G.edges.astype(np.int32))
    assert np.allclose(m["v"], V, atol=1e-7)
    assert np.float32(m["bound"]) == O.bound_radius_f32(kind, np.float32(params), None)


def test_invalid_analytic_rejected(shim):
    assert build(shim, W.SPHERE, [-1, 0, 0, 0])[0] is None
    assert build(shim, W.BOX, [0.1, 0.1, 0.1, 0.5])[0] is None
    assert build(shim, 7, [0.1, 0.1, 0.1, 0.0])[0] is None


def build_sq(lib, rec):
    """Library mesh of one superquadric union (records: 4 xyz rows per primitive)."""
    P = np.ascontiguousarray(rec, np.float32).reshape(-1, 3)
    M = max(len(P) // 4, 1)
    capv, cape, capf = 32 * M + 8, 90 * M + 8, 5 * M + 8
    v = np.zeros(3 * capv, np.float32); e = np.zeros(2 * cape, np.int32); f = np.zeros(3 * capf, np.int32)
    pl = np.zeros(4 * capf, np.float32); nv = C.c_int(); ne = C.c_int(); nf = C.c_int(); br = C.c_float()
    err = C.create_string_buffer(256)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    params = np.zeros(4, np.float32)
    ok = lib.shim_build_mesh(W.SQ_UNION, ptr(params), ptr(P), C.c_long(len(P)), ptr(v), C.byref(nv), ptr(e),
                             C.byref(ne), ptr(f), C.byref(nf), ptr(pl), C.byref(br), err)
    if not ok:
        return None, err.value.decode()
    return dict(v=v[:3 * nv.value].reshape(-1, 3), e=e[:2 * ne.value].reshape(-1, 2), nf=nf.value,
                slots=pl[:4 * nf.value].reshape(-1, 4), bound=br.value), ""


@pytest.mark.parametrize("n_prims,seed", [(1, 0), (3, 1), (18, 2), (18, 3)])
def test_sq_union_meshes_match_oracle(shim, n_prims, seed):
    """Library and oracle build the same superquadric-union mesh: vertex set
    and order, edge list, float32 bounding radius bit for bit."""
    rec = W.sq_union_records(W._rng(6, seed), n_prims)
    m, err = build_sq(shim, rec)
    assert m is not None, err
    G = O.make_geom(O.SQ_UNION, points=rec)
    with torch.no_grad():
        V = G.vertices().numpy()
    assert m["v"].shape == V.shape
    assert np.allclose(m["v"], V, atol=1e-6)
    assert np.array_equal(m["e"], G.edges.astype(np.int32))
    assert m["nf"] == 5 * n_prims
    assert np.float32(m["bound"]) == O.bound_radius_f32(O.SQ_UNION, None, rec)
    if n_prims == 1:
        assert len(V) == 32 and len(G.edges) == 90


def test_invalid_sq_union_rejected(shim):
    rec = W.sq_union_records(W._rng(6, 0), 2).reshape(-1, 12).copy()
    bad_eps = rec.copy(); bad_eps[0, 3] = 2.5
    bad_axis = rec.copy(); bad_axis[1, 1] = 0.0
    bad_q = rec.copy(); bad_q[0, 8:12] = 0.0
    for r in (bad_eps, bad_axis, bad_q):
        assert build_sq(shim, r.reshape(-1, 3))[0] is None
    assert build_sq(shim, rec.reshape(-1, 3)[:7])[0] is None         # not 4 rows per primitive


@pytest.mark.parametrize("seed", [0, 1])
def test_opc_meshes_match_oracle(shim, seed):
    """Oriented point clouds: the points are the vertices, the edges the
    undirected 4-nearest-neighbour graph, the float32 bound bit for bit."""
    rec = W.opc_torus_records(W._rng(8, seed))
    P = np.ascontiguousarray(rec, np.float32)
    N = len(P) // 3
    v = np.zeros(3 * N, np.float32); e = np.zeros(2 * 4 * N, np.int32); f = np.zeros(3 * 2 * N, np.int32)
    pl = np.zeros(4 * 2 * N, np.float32); nv = C.c_int(); ne = C.c_int(); nf = C.c_int(); br = C.c_float()
    err = C.create_string_buffer(256)
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    ok = shim.shim_build_mesh(W.OPC, ptr(np.zeros(4, np.float32)), ptr(P), C.c_long(len(P)), ptr(v), C.byref(nv),
                              ptr(e), C.byref(ne), ptr(f), C.byref(nf), ptr(pl), C.byref(br), err)
    assert ok, err.value
    G = O.make_geom(O.OPC, points=rec)
    assert nv.value == N and nf.value == 2 * N
    assert np.array_equal(v[:3 * N].reshape(-1, 3), rec.reshape(-1, 9)[:, 0:3])
    assert np.array_equal(e[:2 * ne.value].reshape(-1, 2), G.edges.astype(np.int32))
    assert np.float32(br.value) == O.bound_radius_f32(O.OPC, None, rec)
