"""Soft top-K pre-selection (cm_params.presel_*) against the FP64 oracle.

Same bar as the full method: broadphase pairs bit for bit, outputs within
|gpu - ref| <= 1e-6 + 2e-5 |ref|.
"""
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


def run(ctx, batch, presel, flags=0):
    _say(f"[gpu-presel] {batch.name} scenes={batch.n_scenes} K={batch.K} tau={batch.tau} presel={presel} flags={flags}")
    ids = ctx.create_geometry(batch.geoms)
    db = ctx.upload_batch(batch, ids)
    m = ctx.collide(db, batch.tau, batch.K, flags=flags, presel=presel)
    ctx.check_errors()
    return m.to_numpy()


def check(batch, got, presel, flags=0, max_pairs=None):
    pairs, off = O.broadphase(batch)
    assert np.array_equal(got["offsets"], off) and np.array_equal(got["pairs"], pairs)
    n = pairs.shape[1]
    sel = np.arange(n)
    if max_pairs is not None and n > max_pairs:
        sel = np.sort(np.random.default_rng(0).choice(n, max_pairs, replace=False))
    _, _, ref = O.collide_batch(batch, pair_list=pairs[:, sel], presel=presel,
                                safeguard=bool(flags & 4), no_ee=bool(flags & 1), one_sided_vs=bool(flags & 2))
    ok, rep = compare_outputs(got, ref, idx=sel)
    _say(f"   parity {batch.name} presel={presel} flags={flags}: {rep}")
    assert ok, rep


@pytest.mark.parametrize("presel", [(8, 12), (3, 5)])
def test_presel_mixed(ctx, presel):
    b = W.mixed_scenes(48, seed=61)
    check(b, run(ctx, b, presel), presel)


def test_presel_polytopes_safeguard(ctx):
    b = W.polytope_scenes(6, seed=62, n_points=24, tau=0.01)
    for flags in (0, 4):
        check(b, run(ctx, b, (12, 18), flags), (12, 18), flags)


def test_presel_select_everything(ctx):
    """K_V, K_E above every body's counts: every vertex and edge is selected
    (as soft averages over all of them)."""
    b = W.cube_pairs(512, seed=63)
    check(b, run(ctx, b, (64, 64)), (64, 64))


def test_presel_with_simplifications(ctx):
    b = W.mixed_scenes(24, seed=64)
    check(b, run(ctx, b, (6, 10), 3), (6, 10), 3)


def test_presel_served_forward_matches_direct(ctx):
    from paper_2602_20304_amd.cm import Server
    b = W.mixed_scenes(40, seed=65)
    ids = ctx.create_geometry(b.geoms)
    direct = run(ctx, b, (8, 12))
    srv = Server(ctx, 1 << 32, n_streams=2)
    t = srv.submit(b.body_offsets, ids[b.body_geom], b.pose, b.tau, b.K, presel=(8, 12))
    import time
    r = None
    for _ in range(2000):
        r = srv.poll(t)
        if r is not None:
            break
        time.sleep(0.005)
    assert r is not None and r["status"] == 0
    n = direct["n_pairs"]
    assert r["n_pairs"] == n
    for k in ("d", "w"):
        assert np.array_equal(r[k][:n], direct[k][:n]), k
    srv.release(t)
    srv.close()


def test_presel_rejected_where_unsupported(ctx):
    import torch
    from paper_2602_20304_amd._lib import CMError
    b = W.cube_pairs(8, seed=66)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    with pytest.raises(CMError):
        ctx.collide(db, b.tau, b.K, presel=(0, 4))
    with pytest.raises(CMError):
        ctx.collide(db, b.tau, b.K, presel=(4, 65))
    with pytest.raises(CMError):
        ctx.collide(db, b.tau, b.K, flags=4)
    m = ctx.collide(db, b.tau, b.K, presel=(4, 4))
    g = torch.zeros(m.dist.shape, device=ctx.device)
    with pytest.raises(CMError):
        ctx.collide_backward(db, m, b.tau, b.K, None, None, g, None, presel=(4, 65))
    with pytest.raises(CMError):
        ctx.collide_backward(db, m, b.tau, b.K, None, None, g, None, flags=4)


def test_presel_served_backward_matches_direct(ctx):
    """A served request with pre-selection and a backward pass returns the
    same pose gradient as the direct forward + adjoint calls."""
    import time
    import torch
    from paper_2602_20304_amd.cm import Server
    b = W.mixed_scenes(24, seed=67)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    presel = (6, 10)
    _say(f"[gpu-presel] served backward presel={presel} scenes={b.n_scenes}")
    m = ctx.collide(db, b.tau, b.K, presel=presel)
    cap, K = m.capacity, b.K
    rng = np.random.default_rng(5)
    cd = rng.standard_normal(cap * K).astype(np.float32)
    cn = rng.standard_normal(3 * cap * K).astype(np.float32)
    g = ctx.collide_backward(db, m, b.tau, K, None, torch.as_tensor(cn).to(ctx.device),
                             torch.as_tensor(cd).to(ctx.device), None, want_vertices=False, want_params=False,
                             presel=presel)
    ctx.check_errors()
    ga = g["pose"].cpu().numpy()
    srv = Server(ctx, 1 << 32, n_streams=2)
    t = srv.submit(b.body_offsets, ids[b.body_geom], b.pose, b.tau, K, True, cd, cn, capacity=cap, presel=presel)
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


def test_presel_fused_matches_plain_bitwise(ctx):
    """The fused path (cost classes, work queues, replayed graph) with
    pre-selection equals the plain kernel bit for bit, on two replays."""
    b = W.mixed_scenes(64, seed=68)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    _say(f"[gpu-presel] fused vs plain, presel=(16, 10), scenes={b.n_scenes}")
    g1 = ctx.collide(db, b.tau, b.K, presel=(16, 10)).to_numpy()
    for _ in range(2):
        g2 = ctx.collide(db, b.tau, b.K, fused=True, presel=(16, 10)).to_numpy()
        ctx.check_errors()
        for k in ("pairs", "offsets", "p", "nu", "d", "w"):
            assert np.array_equal(g1[k], g2[k]), k
