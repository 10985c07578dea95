"""Witness sphere tracing (cm_params.refine_steps) against the FP64 oracle on
an MI355X: broadphase bit for bit, outputs within |gpu - ref| <= 1e-6 +
2e-5 |ref|."""
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
    m = ctx.collide(db, b.tau, b.K, refine=2)
    g = torch.zeros(m.dist.shape, device=ctx.device)
    with pytest.raises(CMError):
        ctx.collide_backward(db, m, b.tau, b.K, None, None, g, None, refine=2)


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
