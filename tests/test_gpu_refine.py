"""Witness sphere tracing (cm_params.refine_steps) against the FP64 oracle on
an MI355X: broadphase bit for bit, outputs within |gpu - ref| <= 1e-6 +
2e-5 |ref|; the adjoint through the traces against autograd of the oracle
forward within 1e-3 relative (pose twists, hull vertices, analytic
parameters, tau)."""
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


def run_check(ctx, batch, refine, presel=None, flags=0, max_pairs=None):
    _say(f"[gpu-refine] {batch.name} scenes={batch.n_scenes} K={batch.K} tau={batch.tau} refine={refine} "
         f"presel={presel} flags={flags}")
    ids = ctx.create_geometry(batch.geoms)
    db = ctx.upload_batch(batch, ids)
    got = ctx.collide(db, batch.tau, batch.K, flags=flags, presel=presel, refine=refine).to_numpy()
    ctx.check_errors()
    pairs, off = O.broadphase(batch)
    assert np.array_equal(got["offsets"], off) and np.array_equal(got["pairs"], pairs)
    n = pairs.shape[1]
    sel = np.arange(n)
    if max_pairs is not None and n > max_pairs:
        sel = np.sort(np.random.default_rng(0).choice(n, max_pairs, replace=False))
    _, _, ref = O.collide_batch(batch, pair_list=pairs[:, sel], presel=presel, safeguard=bool(flags & 4),
                                no_ee=bool(flags & 1), one_sided_vs=bool(flags & 2), refine=refine)
    ok, rep = compare_outputs(got, ref, idx=sel)
    _say(f"   parity {batch.name} refine={refine} ({len(sel)} of {n} pairs): {rep}")
    assert ok, rep
    return got


@pytest.mark.parametrize("refine", [1, 4])
def test_refine_cube_pairs(ctx, refine):
    run_check(ctx, W.cube_pairs(512, seed=31), refine)


def test_refine_mixed(ctx):
    run_check(ctx, W.mixed_scenes(24, seed=32), 5, max_pairs=80)


def test_refine_polytopes_k16(ctx):
    b = W.polytope_scenes(4, seed=33, tau=0.01)
    b.K = 16
    run_check(ctx, b, 3)


def test_refine_with_preselection_and_safeguard(ctx):
    run_check(ctx, W.mixed_scenes(24, seed=34), 4, presel=(16, 10), flags=4, max_pairs=80)


def test_refine_changes_the_result(ctx):
    """Tracing moves the witnesses onto the smoothed surfaces: the manifold
    differs from the unrefined one (the QP witnesses sit on mesh edges,
    outside the smoothed polytope surface)."""
    b = W.polytope_scenes(3, seed=35)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    m0 = ctx.collide(db, b.tau, b.K).to_numpy()
    m1 = ctx.collide(db, b.tau, b.K, refine=3).to_numpy()
    ctx.check_errors()
    assert np.abs(m0["d"] - m1["d"]).max() > 1e-4


def test_refine_rejected_where_unsupported(ctx):
    import torch
    from paper_2602_20304_amd._lib import CMError
    b = W.cube_pairs(8, seed=36)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    for kw in (dict(refine=9), dict(refine=-1), dict(refine=2, fused=True)):
        with pytest.raises(CMError):
            ctx.collide(db, b.tau, b.K, **kw)
    with pytest.raises(CMError):
        ctx.collide(db, b.tau, 32, refine=2)
    with pytest.raises(CMError):   # the backward shares the forward's parameter checks
        m = ctx.collide(db, b.tau, b.K, refine=2)
        g = torch.zeros(m.dist.shape, device=ctx.device)
        ctx.collide_backward(db, m, b.tau, b.K, None, None, g, None, refine=9)


def test_refine_served_matches_direct(ctx):
    import time
    from paper_2602_20304_amd.cm import Server
    b = W.mixed_scenes(16, seed=37)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    direct = ctx.collide(db, b.tau, b.K, refine=3).to_numpy()
    srv = Server(ctx, 1 << 32, n_streams=2)
    t = srv.submit(b.body_offsets, ids[b.body_geom], b.pose, b.tau, b.K, refine=3)
    r = None
    for _ in range(4000):
        r = srv.poll(t)
        if r is not None:
            break
        time.sleep(0.005)
    assert r is not None and r["status"] == 0
    n = direct["n_pairs"]
    for k in ("d", "w"):
        assert np.array_equal(r[k][:n], direct[k][:n]), k
    srv.release(t)
    srv.close()


# ---- the adjoint through the traces (each reverse step is a wave-wide SDF
# query adjoint; the tracing direction's adjoint runs through the Hessian of
# the SDF at the QP witness)

@pytest.fixture
def fresh():
    from paper_2602_20304_amd.cm import Context
    return Context(0)


@pytest.mark.parametrize("refine", [1, 3])
def test_refine_backward_polytopes(fresh, refine):
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, W.polytope_scenes(2, seed=41, n_points=24, tau=0.02), refine=refine)


def test_refine_backward_mixed(fresh):
    """Spheres, capsules, rounded boxes and polytopes: analytic parameter
    gradients through the traced witnesses."""
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, W.mixed_scenes(6, seed=42, poly_points=16, tau=0.01), refine=2)


def test_refine_backward_k16_eight_steps(fresh):
    from tests.test_gpu_backward import check as grad_check
    b = W.polytope_scenes(1, seed=43, n_points=20, tau=0.01)
    b.K = 16
    grad_check(fresh, b, refine=8)


def test_refine_backward_preselection_safeguard(fresh):
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, W.mixed_scenes(6, seed=44, poly_points=16, tau=0.01), flags=4, presel=(6, 10), refine=2)


def test_refine_backward_simplification_flags(fresh):
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, W.mixed_scenes(6, seed=45, poly_points=16, tau=0.01), flags=2, refine=3)


def test_refine_backward_superquadric_unions(fresh):
    from tests.test_gpu_backward import check as grad_check
    grad_check(fresh, W.sq_scenes(4, seed=46, n_prims=2, n_geoms=3, eps=(0.3, 1.0)), refine=2)


def test_refine_backward_autograd_joint_motion(fresh):
    """Through the autograd wrapper at a larger size: with only normal and
    distance cotangents, the translation gradients of each scene's bodies sum
    to zero (moving every body together changes neither output)."""
    import torch
    from paper_2602_20304_amd.cm import collide_autograd
    b = W.polytope_scenes(32, seed=47, n_points=32)
    ids = fresh.create_geometry(b.geoms)
    db = fresh.upload_batch(b, ids)
    _say(f"[gpu-refine] autograd joint motion, scenes={b.n_scenes}")
    tau_t = torch.tensor(b.tau, device=fresh.device, requires_grad=True)
    xi = torch.zeros(6, db.n_bodies, device=fresh.device, requires_grad=True)
    p, n, d, w, npairs, pairs = collide_autograd(fresh, db, tau_t, b.K, xi=xi, refine=3)
    gen = torch.Generator(device="cpu").manual_seed(5)
    cn = torch.randn(n.shape, generator=gen).to(fresh.device)
    cd = torch.randn(d.shape, generator=gen).to(fresh.device)
    ((n * cn).sum() + (d * cd).sum()).backward()
    fresh.check_errors()
    pose = xi.grad.cpu().numpy()
    bo = b.body_offsets
    sums = np.stack([pose[:3, bo[s]:bo[s + 1]].sum(1) for s in range(b.n_scenes)])
    scale = np.abs(pose[:3]).max()
    assert scale > 0
    assert np.abs(sums).max() <= 1e-4 * scale, (np.abs(sums).max(), scale)


def test_refine_served_backward_matches_direct(fresh):
    """A served forward + backward request with traced witnesses returns the
    same pose, tau and geometry gradients as the direct calls."""
    import time
    import torch
    from paper_2602_20304_amd.cm import Server
    b = W.mixed_scenes(12, seed=48, poly_points=16, tau=0.01)
    ids = fresh.create_geometry(b.geoms)
    db = fresh.upload_batch(b, ids)
    _say(f"[gpu-refine] served backward, scenes={b.n_scenes}")
    m = fresh.collide(db, b.tau, b.K, refine=2)
    cap, K = m.capacity, b.K
    rng = np.random.default_rng(8)
    cd = rng.standard_normal(cap * K).astype(np.float32)
    cn = rng.standard_normal(3 * cap * K).astype(np.float32)
    cp = rng.standard_normal(3 * cap * K).astype(np.float32)
    g = fresh.collide_backward(db, m, b.tau, K, torch.as_tensor(cp).view(3, -1).to(fresh.device),
                               torch.as_tensor(cn).view(3, -1).to(fresh.device),
                               torch.as_tensor(cd).to(fresh.device), None, refine=2)
    fresh.check_errors()
    srv = Server(fresh, 1 << 32, n_streams=2)
    t = srv.submit(b.body_offsets, ids[b.body_geom], b.pose, b.tau, K, True, cd, cn, capacity=cap, refine=2,
                   cot_point=cp, want_geometry=True)
    r = None
    for _ in range(4000):
        r = srv.poll(t)
        if r is not None:
            break
        time.sleep(0.005)
    assert r is not None and r["status"] == 0
    for key, rk in (("pose", "g_pose"), ("tau", "g_tau"), ("vertices", "g_vertices"), ("params", "g_params")):
        a = g[key].cpu().numpy().reshape(-1)
        c = np.asarray(r[rk]).reshape(-1)[:a.size]
        assert np.abs(c - a).max() <= 1e-4 * (np.abs(a).max() + 1e-6), key
    srv.release(t)
    srv.close()
