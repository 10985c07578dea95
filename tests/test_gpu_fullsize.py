"""Parity at the sizes the workloads name (needs an MI355X).

* the adjoint on the differentiation workload's bodies: hulls of 64 points
  (64 V / 186 E / 124 F: two-word face masks), tau 0.1, 0.01, 0.001;
* the adjoint on uneven-workload pairs at K = 16 whose larger body has more
  than 300 edges (the fused path's largest size class, no face culling above
  128 faces, edge arrays outside LDS);
* the forward, plain and fused, on uneven-workload pairs whose bodies both
  have more than 200 vertices (up to 762 edges), beside a random sample;
* the forward, plain and fused, on the differentiation, mixed and uneven
  workloads at their full benchmark sizes (the launch shapes the benchmark
  times), checked on a seeded sample of kept pairs;
* the adjoint over the whole differentiation workload, with cotangents on
  the pairs of two sampled scenes only.

The FP64 oracle is the reference throughout (gradients: its autograd).
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import cm_oracle as O
from tests.parity import compare_outputs
from tests.test_gpu_backward import check as check_grads
from tests.test_gpu_backward import close, oracle_grads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2602_20304_amd.cm import Context
    return Context(0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pairs_batch(b, sel, name):
    """One scene per selected (a, b) body pair of batch b, listed as the
    scene's only candidate; the geometry set is kept whole."""
    bodies = np.array([x for p in sel for x in p], dtype=np.int64)
    n = len(sel)
    return W.Batch(geoms=b.geoms, body_offsets=(2 * np.arange(n + 1)).astype(np.int32),
                   body_geom=b.body_geom[bodies].astype(np.int32), pose=b.pose[:, bodies].copy(),
                   tau=b.tau, K=b.K, cand_offsets=np.arange(n + 1, dtype=np.int32),
                   cand_pairs=np.stack([2 * np.arange(n), 2 * np.arange(n) + 1]).astype(np.int32), name=name)


def _vertex_counts(b):
    return np.diff(b.geoms.pt_off)[b.body_geom]


@pytest.mark.parametrize("tau", [0.1, 0.01, 0.001])
def test_backward_differentiation_hulls(ctx, tau):
    """One scene of the differentiation workload: 4 hulls of 64 points, all 6
    pairs candidates."""
    b = W.polytope_scenes(1, seed=60, tau=tau)
    check_grads(ctx, b, seed=61)


def test_backward_uneven_largest_class(ctx):
    """K = 16 uneven pairs: the first two kept pairs whose larger body has
    more than 300 edges (hulls of more than 102 points) and whose smaller one
    more than 200, and two smaller pairs."""
    b = W.uneven_scenes(300, seed=62)
    pairs, _ = O.broadphase(b)
    nv = _vertex_counts(b)
    eA, eB = 3 * nv[pairs[0]] - 6, 3 * nv[pairs[1]] - 6
    e_max = np.maximum(eA, eB)
    big = np.nonzero((e_max > 300) & (np.minimum(eA, eB) > 200))[0][:2]
    small = np.nonzero((e_max > 0) & (e_max <= 300))[0][:2]
    assert len(big) == 2
    sel = [(int(pairs[0, i]), int(pairs[1, i])) for i in np.concatenate([big, small])]
    _say(f"[gpu-bwd] uneven largest class: edges {[int(e_max[i]) for i in np.concatenate([big, small])]}")
    check_grads(ctx, pairs_batch(b, sel, "uneven_largest_class"), seed=63)


def test_forward_uneven_both_bodies_above_200_vertices(ctx):
    """Forward parity on uneven scenes with hulls of up to 256 points: every
    kept pair whose bodies both exceed 200 vertices (at least one exists for
    this seed) plus 24 random kept pairs, plain and fused."""
    b = W.uneven_scenes(400, seed=41)
    pairs, off = O.broadphase(b)
    nv = _vertex_counts(b)
    big = np.nonzero((nv[pairs[0]] > 200) & (nv[pairs[1]] > 200))[0][:3]
    assert len(big) >= 1
    rng = np.random.default_rng(64)
    rest = np.setdiff1d(np.arange(pairs.shape[1]), big)
    sel = np.sort(np.concatenate([big, rng.choice(rest, 24, replace=False)]))
    _say(f"[gpu] uneven 400 scenes: {pairs.shape[1]} kept pairs, big pairs {list(big)} "
         f"(vertices {[(int(nv[pairs[0, i]]), int(nv[pairs[1, i]])) for i in big]})")
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    _, _, ref = O.collide_batch(b, pair_list=pairs[:, sel])
    for fused in (False, True):
        m = ctx.collide(db, b.tau, b.K, fused=fused)
        ctx.check_errors()
        got = m.to_numpy()
        assert np.array_equal(got["pairs"], pairs) and np.array_equal(got["offsets"], off)
        ok, rep = compare_outputs(got, ref, idx=sel)
        _say(f"   parity uneven (fused={fused}): {rep}")
        assert ok, rep


def _full_size_forward(ctx, b, n_sample, seed, extra=(), bp=None):
    """The workload as the benchmark runs it (plain and fused launches over
    the whole batch), then the FP64 oracle on a seeded sample of kept pairs
    (the first, the last, any listed ones and n_sample random ones):
    broadphase and offsets bit-exact, sampled outputs within the bar."""
    pairs, off = bp if bp is not None else O.broadphase(b)
    rng = np.random.default_rng(seed)
    sel = np.unique(np.concatenate([[0, pairs.shape[1] - 1], np.asarray(extra, dtype=np.int64),
                                    rng.choice(pairs.shape[1], n_sample, replace=False)]))
    _say(f"[gpu] full size {b.name}: {pairs.shape[1]} kept pairs, {len(sel)} sampled for the oracle")
    _, _, ref = O.collide_batch(b, pair_list=pairs[:, sel])
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    for fused in (False, True):
        _say(f"   launch {b.name} fused={fused}")
        m = ctx.collide(db, b.tau, b.K, fused=fused)
        ctx.check_errors()
        got = m.to_numpy()
        assert np.array_equal(got["pairs"], pairs) and np.array_equal(got["offsets"], off)
        ok, rep = compare_outputs(got, ref, idx=sel)
        _say(f"   parity {b.name} (fused={fused}): {rep}")
        assert ok, rep


def test_forward_full_size_differentiation_workload(ctx):
    """16,384 scenes x 4 hulls of 64 points, tau 0.01, K 8 (the headline
    workload, same seed as the benchmark): 30 sampled pairs."""
    _full_size_forward(ctx, W.polytope_scenes(16384, seed=0, tau=0.01), 28, seed=70)


def test_forward_full_size_mixed_workload(ctx):
    """65,536 scenes x 8 mixed bodies (same seed as the benchmark): 34
    sampled pairs."""
    _full_size_forward(ctx, W.mixed_scenes(65536, seed=0), 32, seed=71)


def test_forward_full_size_uneven_workload(ctx):
    """100,000 uneven scenes at K 16 (same seed as the benchmark): the pair
    of the two largest hulls (256 points each for this seed), the first and
    last kept pairs and 8 random ones."""
    b = W.uneven_scenes(100_000, seed=0)
    pairs, off = O.broadphase(b)
    nv = _vertex_counts(b)
    big = int(np.argmax(nv[pairs[0]].astype(np.int64) * nv[pairs[1]]))
    _full_size_forward(ctx, b, 8, seed=72, extra=[big], bp=(pairs, off))


def test_backward_full_size_differentiation_workload(ctx):
    """The adjoint over the whole headline workload (16,384 scenes x 4 hulls
    of 64 points, tau 0.01, K 8, the benchmark's seed and launch shapes),
    with cotangents that are nonzero only on the kept pairs of two sampled
    scenes: the pose, hull-vertex and tau gradients of those scenes' bodies
    equal the FP64 oracle's autograd of those pairs, and every other body's
    gradients are exactly zero (the adjoint is linear in the cotangents)."""
    import torch
    b = W.polytope_scenes(16384, seed=0, tau=0.01)
    K = b.K
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    _say("[gpu-bwd] full size differentiation workload: forward")
    m = ctx.collide(db, b.tau, K)
    ctx.check_errors()
    fwd = m.to_numpy()
    pairs, off = fwd["pairs"], fwd["offsets"]
    rng = np.random.default_rng(73)
    scenes = np.sort(rng.choice(b.n_scenes, 2, replace=False))
    sel = np.concatenate([np.arange(off[s], off[s + 1]) for s in scenes])
    cap = m.capacity
    cot = {k: np.zeros(s, np.float32) for k, s in
           (("p", (3, cap * K)), ("nu", (3, cap * K)), ("d", (cap * K,)), ("w", (cap * K,)))}
    for i in sel:
        sl = slice(int(i) * K, (int(i) + 1) * K)
        cot["p"][:, sl] = rng.standard_normal((3, K))
        cot["nu"][:, sl] = rng.standard_normal((3, K))
        cot["d"][sl] = rng.standard_normal(K)
        cot["w"][sl] = rng.standard_normal(K)
    tt = {k: torch.as_tensor(v).to(ctx.device) for k, v in cot.items()}
    _say(f"[gpu-bwd] adjoint over {pairs.shape[1]} pairs, cotangents on scenes {list(scenes)} ({len(sel)} pairs)")
    g = ctx.collide_backward(db, m, b.tau, K, tt["p"], tt["nu"], tt["d"], tt["w"])
    ctx.check_errors()
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in g.items()}
    sub = {k: (v[:, np.concatenate([np.arange(int(i) * K, (int(i) + 1) * K) for i in sel])] if v.ndim == 2
               else v[np.concatenate([np.arange(int(i) * K, (int(i) + 1) * K) for i in sel])]) for k, v in cot.items()}
    g_pose, g_geom, g_tau, _ = oracle_grads(b, pairs[:, sel], sub, K)
    bodies = np.unique(pairs[:, sel])
    rep = {"pose": close(g["pose"][:, bodies], g_pose[:, bodies])}
    vx, vr = [], []
    for gid, ref in g_geom.items():
        info = ctx.geometry_info(int(ids[gid]))
        o = info["vertex_offset"]
        vx.append(g["vertices"][:, o:o + info["n_vertices"]].T)
        vr.append(ref)
    rep["vertices"] = close(np.concatenate(vx), np.concatenate(vr))
    rep["tau"] = close([g["tau"][0]], [g_tau])
    _say("   full-size grad parity: " +
         ", ".join(f"{k}: excess {v[0]:.2e} maxabs {v[1]:.2e} scale {v[2]:.2e}" for k, v in rep.items()))
    for k, v in rep.items():
        assert v[0] <= 0, (k, v)
    others = np.setdiff1d(np.arange(b.n_bodies), bodies)
    assert not np.any(g["pose"][:, others]), "pose gradients outside the sampled scenes"
    touched = set(int(ids[b.body_geom[x]]) for x in bodies)
    for x in others[:: max(1, len(others) // 64)]:
        gid = int(ids[b.body_geom[x]])
        if gid in touched:
            continue
        info = ctx.geometry_info(gid)
        o = info["vertex_offset"]
        assert not np.any(g["vertices"][:, o:o + info["n_vertices"]]), "vertex gradients outside the sampled scenes"
