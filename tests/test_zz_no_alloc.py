"""cm_collide_noalloc (workspace in the library's static device array, no
allocation) against cm_collide on the same inputs, through the C ABI (needs
an MI355X).

Two calls in a row on one context, the second with a smaller batch, each
compared with cm_collide: pair lists and offsets bit for bit, the manifold
outputs bit for bit too (the same kernels compute every pair in one
workgroup whatever the grid), which is within the float tolerance of the
oracle bar by construction.  The 64-point hulls need 1.7 MB of scratch per
workgroup, so the allocation-free grid is cut to the slots that fit.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _both(ctx, db, tau, K, cap):
    from paper_2602_20304_amd.cm import Manifold
    a = ctx.collide(db, tau, K, cap)
    ctx.check_errors()
    b = Manifold.empty(db.n_scenes, cap, K, ctx.device)
    b.point.fill_(7.0)     # stale values must be overwritten
    ctx.collide(db, tau, K, cap, out=b, noalloc=True)
    ctx.check_errors()
    return a.to_numpy(), b.to_numpy()


def _same(ref, got, name):
    assert got["n_pairs"] == ref["n_pairs"], name
    assert np.array_equal(got["offsets"], ref["offsets"]), name
    assert np.array_equal(got["pairs"], ref["pairs"]), name
    for k in ("p", "nu", "d", "w"):
        assert np.array_equal(got[k], ref[k]), (name, k, float(np.abs(got[k] - ref[k]).max()))


@pytest.mark.parametrize("maker,sizes", [
    (lambda n: W.polytope_scenes(n, seed=5), (24, 5)),
    (lambda n: W.mixed_scenes(n, seed=6), (96, 17)),
    (lambda n: W.cube_pairs(n, seed=7), (4096, 300)),
], ids=["polytopes", "mixed", "cubes"])
def test_noalloc_matches_collide_twice(maker, sizes):
    from paper_2602_20304_amd.cm import Context
    ctx = Context(0)
    big = maker(sizes[0])
    ids = ctx.create_geometry(big.geoms)
    for n in sizes:
        b = W.subset_scenes(big, np.arange(n))
        db = ctx.upload_batch(b, ids)
        cap = db.n_cand_total
        _say(f"[gpu] noalloc {b.name} scenes={b.n_scenes} cap={cap} K={b.K} tau={b.tau}")
        ref, got = _both(ctx, db, b.tau, b.K, cap)
        assert ref["n_pairs"] > 0
        _same(ref, got, f"{b.name}:{n}")
    ctx.close()


def test_noalloc_rejects_oversized_workspace():
    """A hull whose per-workgroup scratch slot exceeds the static array is
    refused on the host with a message (nothing is launched)."""
    from paper_2602_20304_amd import _lib as L
    from paper_2602_20304_amd.cm import Context
    ctx = Context(0)
    rng = np.random.default_rng(3)
    gs = W._geomset([3], [np.zeros(4)], [W.ellipsoid_points(rng, 560, [0.5, 0.4, 0.45])])
    ids = ctx.create_geometry(gs)
    info = ctx.geometry_info(int(ids[0]))
    assert 8 * info["n_edges"] ** 2 * 4 > L.CM_NOALLOC_SCRATCH_BYTES
    b = W.Batch(name="one_big_pair", body_offsets=np.array([0, 2], np.int32),
                body_geom=np.array([0, 0], np.int32),
                pose=np.array([[1, 1], [0, 0], [0, 0], [0, 0], [0, 0.1], [0, 0], [0, 0]], np.float32),
                geoms=gs, tau=0.01, K=8)
    db = ctx.upload_batch(b, ids)
    _say(f"[gpu] noalloc rejection: {info['n_edges']} edges")
    with pytest.raises(L.CMError) as ei:
        ctx.collide(db, 0.01, 8, 1, noalloc=True)
    assert ei.value.status in (-7, -1), ei.value
    assert "B" in str(ei.value)
    ctx.close()
