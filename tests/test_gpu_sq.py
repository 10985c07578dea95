"""Superquadric-union bodies (the paper's default primitive family) against
the FP64 oracle on an MI355X: broadphase bit for bit, outputs within
|gpu - ref| <= 1e-6 + 2e-5 |ref|, gradients within 1e-3 of the oracle's
autograd; the kernels built for contexts that hold such bodies also handle
every other type."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import cm_oracle as O
from tests.parity import compare_outputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2602_20304_amd.cm import Context
    return Context(0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(ctx, batch, presel=None, flags=0):
    _say(f"[gpu-sq] {batch.name} scenes={batch.n_scenes} K={batch.K} tau={batch.tau} presel={presel} flags={flags}")
    ids = ctx.create_geometry(batch.geoms)
    db = ctx.upload_batch(batch, ids)
    m = ctx.collide(db, batch.tau, batch.K, flags=flags, presel=presel)
    ctx.check_errors()
    return ids, db, m


def check(batch, got, presel=None, flags=0, max_pairs=None):
    pairs, off = O.broadphase(batch)
    assert np.array_equal(got["offsets"], off) and np.array_equal(got["pairs"], pairs)
    n = pairs.shape[1]
    assert n > 0
    sel = np.arange(n)
    if max_pairs is not None and n > max_pairs:
        sel = np.sort(np.random.default_rng(0).choice(n, max_pairs, replace=False))
    _, _, ref = O.collide_batch(batch, pair_list=pairs[:, sel], presel=presel, safeguard=bool(flags & 4),
                                no_ee=bool(flags & 1), one_sided_vs=bool(flags & 2))
    ok, rep = compare_outputs(got, ref, idx=sel)
    _say(f"   parity {batch.name} presel={presel} flags={flags} ({len(sel)} of {n} pairs): {rep}")
    assert ok, rep


def mixed_with_sq(n_scenes, seed, eps=(0.3, 1.5)):
    """Scenes of 3 bodies: a superquadric union, then a sphere, a rounded box
    or a polytope, then another union."""
    rng = W._rng(7, seed)
    recs = [W.sq_union_records(rng, 4, eps=eps) for _ in range(3)]
    pts = W.ellipsoid_points(rng, 24, [0.3, 0.25, 0.2]).astype(np.float32)
    types = [W.SQ_UNION] * 3 + [W.SPHERE, W.BOX, W.POLYTOPE]
    params = [[0] * 4] * 3 + [[0.25, 0, 0, 0], [0.3, 0.2, 0.25, W.BOX_ROUNDING], [0] * 4]
    gs = W._geomset(types, params, recs + [None, None, pts])
    nb = 3 * n_scenes
    body_geom = np.stack([rng.integers(0, 3, n_scenes), rng.integers(3, 6, n_scenes),
                          rng.integers(0, 3, n_scenes)], axis=1).reshape(-1).astype(np.int32)
    t = rng.uniform(-0.4, 0.4, size=(nb, 3))
    q = W.uniform_quats(rng, nb)
    return W.Batch(gs, (np.arange(n_scenes + 1) * 3).astype(np.int32), body_geom, W._pose_array(q, t), 0.01, 8,
                   name="sq_mixed")


def test_sq_small_unions_all_edge_pairs(ctx):
    b = W.sq_scenes(12, seed=1, n_prims=3, n_geoms=3)
    _, _, m = run(ctx, b)
    check(b, m.to_numpy())


@pytest.mark.parametrize("tau", [0.05, 0.003])
def test_sq_tau_sweep(ctx, tau):
    b = W.sq_scenes(8, seed=2, n_prims=4, n_geoms=2, tau=tau)
    _, _, m = run(ctx, b)
    check(b, m.to_numpy())


def test_sq_with_other_types(ctx):
    b = mixed_with_sq(10, seed=3)
    _, _, m = run(ctx, b)
    check(b, m.to_numpy())


def test_sq_eighteen_primitives_preselected(ctx):
    """The stand-in for a decomposed mesh (18 primitives, ~350 V / ~800 E)
    with the paper's benchmark pre-selection (K_V 64, K_E 18), every pair."""
    b = W.sq_scenes(16, seed=4)
    _, _, m = run(ctx, b, presel=(64, 18))
    check(b, m.to_numpy(), presel=(64, 18))


def test_sq_eighteen_primitives_safeguard_sampled(ctx):
    b = W.sq_scenes(24, seed=5)
    _, _, m = run(ctx, b, presel=(32, 12), flags=4)
    check(b, m.to_numpy(), presel=(32, 12), flags=4, max_pairs=12)


def test_sq_eighteen_primitives_all_edge_pairs_sampled(ctx):
    """Full E-E over every edge pair of ~800-edge meshes, a few sampled pairs."""
    b = W.sq_scenes(4, seed=6)
    _, _, m = run(ctx, b)
    check(b, m.to_numpy(), max_pairs=2)


def test_sq_fused_matches_plain_bitwise(ctx):
    """The fused path (cost classes, work queues, replayed graph) on
    superquadric unions mixed with other types, with and without
    pre-selection, equals the plain kernel bit for bit on two replays."""
    b = mixed_with_sq(16, seed=7)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    for presel in (None, (16, 10)):
        _say(f"[gpu-sq] fused vs plain presel={presel}")
        g1 = ctx.collide(db, b.tau, b.K, presel=presel).to_numpy()
        for _ in range(2):
            g2 = ctx.collide(db, b.tau, b.K, fused=True, presel=presel).to_numpy()
            ctx.check_errors()
            for k in ("pairs", "offsets", "p", "nu", "d", "w"):
                assert np.array_equal(g1[k], g2[k]), (presel, k)


# ---- adjoint: pose twists, tau and the other bodies' geometry gradients
# against autograd of the FP64 oracle, 1e-3 relative (superquadric records
# take no gradient: their parameter gradients must stay 0).  Exponents <= 1:
# above 1 the derivative of the normal field is unbounded on a primitive's
# axis planes, where mesh edges lie.

# (each in a fresh context: the adjoint's LDS is sized by the context's
# largest geometry)

@pytest.fixture
def fresh():
    from paper_2602_20304_amd.cm import Context
    return Context(0)


def test_sq_backward_small_unions(fresh):
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, W.sq_scenes(8, seed=11, n_prims=3, n_geoms=3, eps=(0.3, 1.0)))


def test_sq_backward_with_other_types(fresh):
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, mixed_with_sq(6, seed=13, eps=(0.3, 1.0)))


def test_sq_backward_preselected_safeguard(fresh):
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, W.sq_scenes(8, seed=12, n_prims=5, n_geoms=2, eps=(0.3, 1.0)), flags=4, presel=(16, 10))


def test_sq_backward_eighteen_primitives_preselected(fresh):
    """The 18-primitive unions (about 350 vertices / 900 edges, the stand-in
    for the paper's decomposed benchmark body) through the pre-selection
    adjoint, exponents <= 1: gradient parity with the oracle's autograd."""
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, W.sq_scenes(2, seed=14, eps=(0.3, 1.0)), presel=(16, 10))


def test_sq_served_backward_matches_direct(fresh):
    """A served forward + backward request on superquadric unions returns the
    same pose gradient as the direct forward and adjoint calls."""
    import time
    import torch
    from paper_2602_20304_amd.cm import Server
    b = W.sq_scenes(12, seed=15, n_prims=3, n_geoms=3, eps=(0.3, 1.0))
    ids = fresh.create_geometry(b.geoms)
    db = fresh.upload_batch(b, ids)
    _say(f"[gpu-sq] served backward, scenes={b.n_scenes}")
    m = fresh.collide(db, b.tau, b.K)
    cap, K = m.capacity, b.K
    rng = np.random.default_rng(6)
    cd = rng.standard_normal(cap * K).astype(np.float32)
    cn = rng.standard_normal(3 * cap * K).astype(np.float32)
    g = fresh.collide_backward(db, m, b.tau, K, None, torch.as_tensor(cn).to(fresh.device),
                               torch.as_tensor(cd).to(fresh.device), None, want_vertices=False, want_params=False)
    fresh.check_errors()
    ga = g["pose"].cpu().numpy()
    srv = Server(fresh, 1 << 32, n_streams=2)
    t = srv.submit(b.body_offsets, ids[b.body_geom], b.pose, b.tau, K, True, cd, cn, capacity=cap)
    r = None
    for _ in range(4000):
        r = srv.poll(t)
        if r is not None:
            break
        time.sleep(0.005)
    assert r is not None and r["status"] == 0
    assert np.abs(r["g_pose"] - ga).max() <= 1e-4 * (np.abs(ga).max() + 1e-6)
    srv.release(t)
    srv.close()
