"""Forward parity of the HIP path against the FP64 oracle (needs an MI355X).

Broadphase pair lists and per-scene offsets must match bit for bit; the
manifold outputs element-wise within |gpu - ref| <= 1e-6 + 2e-5 |ref|.
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


def run_gpu(ctx, batch, fused=False, capacity=None, flags=0):
    _say(f"[gpu] {batch.name} scenes={batch.n_scenes} fused={fused} K={batch.K} tau={batch.tau} flags={flags}")
    ids = ctx.create_geometry(batch.geoms)
    db = ctx.upload_batch(batch, ids)
    m = ctx.collide(db, batch.tau, batch.K, capacity, fused=fused, flags=flags)
    ctx.check_errors()
    return m.to_numpy()


def check_against_oracle(batch, got, max_pairs=None, seed=0, flags=0):
    pairs, off = O.broadphase(batch)
    assert got["n_pairs"] == pairs.shape[1]
    assert np.array_equal(got["offsets"], off), "pair offsets differ"
    assert np.array_equal(got["pairs"], pairs), "pair lists differ"
    n = pairs.shape[1]
    sel = np.arange(n)
    if max_pairs is not None and n > max_pairs:
        sel = np.sort(np.random.default_rng(seed).choice(n, max_pairs, replace=False))
    _, _, ref = O.collide_batch(batch, pair_list=pairs[:, sel], no_ee=bool(flags & 1), one_sided_vs=bool(flags & 2))
    ok, rep = compare_outputs(got, ref, idx=sel)
    _say(f"   parity {batch.name}: {rep}")
    assert ok, rep


def test_cube_pairs_full(ctx):
    b = W.cube_pairs(4096, seed=0)
    got = run_gpu(ctx, b)
    check_against_oracle(b, got)


def test_mixed_scenes(ctx):
    b = W.mixed_scenes(48, seed=1)
    got = run_gpu(ctx, b)
    check_against_oracle(b, got)


def test_polytope_scenes(ctx):
    b = W.polytope_scenes(6, seed=2)
    got = run_gpu(ctx, b)
    check_against_oracle(b, got)


@pytest.mark.parametrize("tau", [0.1, 0.001])
def test_polytope_tau_sweep(ctx, tau):
    b = W.polytope_scenes(3, seed=3, tau=tau)
    got = run_gpu(ctx, b)
    check_against_oracle(b, got)


def test_uneven_scenes_sampled(ctx):
    b = W.uneven_scenes(40, seed=4, v_max=96)
    got = run_gpu(ctx, b)
    check_against_oracle(b, got, max_pairs=60)


def test_fused_matches_plain_bitwise(ctx):
    b = W.mixed_scenes(64, seed=5)
    g1 = run_gpu(ctx, b, fused=False)
    g2 = run_gpu(ctx, b, fused=True)
    for k in ("pairs", "offsets", "p", "nu", "d", "w"):
        assert np.array_equal(g1[k], g2[k]), k


def test_empty_and_degenerate_scenes(ctx):
    # scenes with 0, 1, 2 bodies; only the 2-body scene has a candidate pair
    b = W.cube_pairs(3, seed=6)
    b.body_offsets = np.array([0, 0, 1, 3], dtype=np.int32)
    b.body_geom = np.zeros(3, np.int32)
    b.pose = np.concatenate([b.pose[:, :1], b.pose[:, :2]], axis=1)
    b.pose[4:7, 2] = [0.2, 0.1, 0.3]
    got = run_gpu(ctx, b)
    check_against_oracle(b, got)
    assert got["n_pairs"] == 1 and list(got["offsets"]) == [0, 0, 0, 1]


def test_zero_scenes(ctx):
    b = W.cube_pairs(1, seed=7)
    b.body_offsets = np.array([0], dtype=np.int32)
    b.body_geom = np.zeros(0, np.int32)
    b.pose = np.zeros((7, 0), np.float32)
    from paper_2602_20304_amd.cm import Manifold
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    m = ctx.collide(db, b.tau, b.K, capacity=4)
    ctx.check_errors()
    assert int(m.n_pairs.item()) == 0


def test_capacity_overflow_reported(ctx):
    from paper_2602_20304_amd._lib import CMError
    b = W.mixed_scenes(8, seed=8)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    pairs, off = O.broadphase(b)
    cap = pairs.shape[1] // 2
    m = ctx.collide(db, b.tau, b.K, capacity=cap)
    with pytest.raises(CMError) as e:
        ctx.check_errors()
    assert e.value.status == -7
    # the pairs that fit are still the oracle's first `cap` pairs
    got = m.to_numpy()
    assert got["n_pairs"] == pairs.shape[1]
    assert np.array_equal(got["pairs"], pairs[:, :cap])


def test_bad_geometry_id_reported(ctx):
    from paper_2602_20304_amd._lib import CMError
    b = W.cube_pairs(4, seed=9)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    db.body_geom[1] = 10 ** 7
    ctx.collide(db, b.tau, b.K)
    with pytest.raises(CMError) as e:
        ctx.check_errors()
    assert e.value.status == -6


def test_fused_graph_replays_match_plain(ctx):
    """The fused path (size classes, cost order, hipGraph) replays the captured
    graph on later calls: every replay must equal the plain kernel bitwise,
    including after the poses change in place between replays."""
    import torch
    from paper_2602_20304_amd.cm import Manifold
    b = W.uneven_scenes(80, seed=31, v_max=160)
    _say(f"[gpu] fused replays: {b.n_scenes} scenes")
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    cap = db.n_cand_total
    outs = {k: Manifold.empty(db.n_scenes, cap, b.K, ctx.device) for k in ("plain", "fused")}
    gen = torch.Generator(device="cpu").manual_seed(5)
    for rep in range(3):
        ctx.collide(db, b.tau, b.K, out=outs["plain"], fused=False)
        ctx.collide(db, b.tau, b.K, out=outs["fused"], fused=True)
        ctx.check_errors()
        gp, gf = outs["plain"].to_numpy(), outs["fused"].to_numpy()
        for k in ("pairs", "offsets", "p", "nu", "d", "w"):
            assert np.array_equal(gp[k], gf[k]), (rep, k)
        shift = (0.02 * torch.randn(3, db.n_bodies, generator=gen)).to(ctx.device)
        db.pose[4:7] += shift
    torch.cuda.synchronize()


def test_kernel_timing_counts_launches(ctx):
    """Opt-in event timing: one forward launch per cm_collide, one graph
    replay per cm_collide_fused, sums reset on enable."""
    b = W.cube_pairs(256, seed=2)
    _say(f"[gpu] kernel timing: {b.n_scenes} scenes")
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    ctx.collide(db, b.tau, b.K, fused=True)        # capture outside the timed calls
    ctx.set_kernel_timing(True)
    for _ in range(3):
        ctx.collide(db, b.tau, b.K)
    ctx.collide(db, b.tau, b.K, fused=True)
    ms, n = ctx.kernel_time("forward")
    assert n == 3 and ms > 0.0
    bp_ms, bp_n = ctx.kernel_time("broadphase")
    assert bp_n == 3 and bp_ms > 0.0
    f_ms, f_n = ctx.kernel_time("fused")
    assert f_n == 1 and f_ms > 0.0
    ctx.set_kernel_timing(True)
    assert ctx.kernel_time("forward") == (0.0, 0)
    ctx.set_kernel_timing(False)
    ctx.collide(db, b.tau, b.K)
    assert ctx.kernel_time("forward") == (0.0, 0)
    ctx.check_errors()


@pytest.mark.parametrize("flags", [1, 3])
def test_simplification_flags(ctx, flags):
    """Ours-NE (no E-E) and Ours-NE-S (one-sided V-S), plain and fused."""
    b = W.mixed_scenes(48, seed=7)
    got = run_gpu(ctx, b, flags=flags)
    check_against_oracle(b, got, flags=flags)
    fused = run_gpu(ctx, b, fused=True, flags=flags)
    for k in ("pairs", "offsets", "p", "nu", "d", "w"):
        assert np.array_equal(fused[k], got[k]), k


def test_fewer_candidates_than_K(ctx):
    """One-sided V-S of a cube (8 vertices) with K = 12: rows 8..11 are empty."""
    b = W.cube_pairs(256, seed=8, K=12)
    b.pose[4:7] += np.array([[0.3], [-0.2], [0.5]], dtype=b.pose.dtype)   # body A off the origin
    got = run_gpu(ctx, b, flags=3)
    check_against_oracle(b, got, flags=3)
    n = got["n_pairs"]
    assert n > 0
    for k in ("p", "nu", "d", "w"):
        assert not np.any(got[k][:n, 8:]), k


def test_calls_on_two_streams_are_ordered(ctx):
    """Forward calls on one context alternating between two streams, with no
    synchronisation between them, share the context's scratch: the library
    orders them, so every result equals the single-stream one bit for bit."""
    import torch
    b = W.polytope_scenes(32, seed=12)
    _say(f"[gpu] two streams: {b.n_scenes} scenes")
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    ref = ctx.collide(db, b.tau, b.K)
    ctx.check_errors()
    r = ref.to_numpy()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = [ctx.collide(db, b.tau, b.K, stream=(s1 if i % 2 == 0 else s2)) for i in range(4)]
    torch.cuda.synchronize()
    ctx.check_errors()
    for m in outs:
        g = m.to_numpy()
        for k in ("pairs", "offsets", "p", "nu", "d", "w"):
            assert np.array_equal(g[k], r[k]), k


def test_fused_autotune_sample_and_cache(tmp_path, monkeypatch):
    """The fused path's autotuner times its size classes on strided samples
    and stores the choices; a fresh context with the same geometry reads them
    back from the cache file instead of timing, with the same results."""
    from paper_2602_20304_amd.cm import Context
    monkeypatch.setenv("CM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    b = W.uneven_scenes(60, seed=33, v_max=160)
    _say(f"[gpu] autotune cache: {b.n_scenes} scenes")
    outs = []
    for run in range(2):
        c = Context(0)
        ids = c.create_geometry(b.geoms)
        db = c.upload_batch(b, ids)
        m = c.collide(db, b.tau, b.K, fused=True)
        c.check_errors()
        t = c.fused_tuning()
        _say(f"   run {run}: {t}")
        if run == 0:
            assert not any(t["from_cache"])
            timed = [i for i in range(3) if t["sample_pairs"][i] > 0]
            assert timed and all(t["sample_ms"][i][0] > 0 for i in timed)
            lines = (tmp_path / "tune.txt").read_text().split("\n")
            assert len([x for x in lines if x.strip()]) == len(timed)
        else:
            assert all(t["from_cache"][i] for i in timed) and not any(t["sample_pairs"])
            assert t["class_blocks"] == first["class_blocks"]
        first = t if run == 0 else first
        outs.append(m.to_numpy())
        c.close()
    for k in ("pairs", "offsets", "p", "nu", "d", "w"):
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_fused_any_block_size_matches_plain_bitwise(tmp_path, monkeypatch):
    """Every reduction whose order could depend on the block size (the column
    LSE's chunks) is chunked the same way in every instantiation, so the fused
    path equals the plain kernel bit for bit whichever block size its classes
    run (forced here through the tuner's cache file: 128, 256 and 64 threads),
    also on hulls of up to 256 points, whose edge arrays move out of LDS."""
    from paper_2602_20304_amd.cm import Context
    for name, b in (("mixed", W.mixed_scenes(64, seed=5)), ("uneven", W.uneven_scenes(40, seed=35, v_max=256))):
        monkeypatch.setenv("CM_TUNE_CACHE", str(tmp_path / f"{name}_tuned.txt"))
        c = Context(0)
        ids = c.create_geometry(b.geoms)
        db = c.upload_batch(b, ids)
        plain = c.collide(db, b.tau, b.K).to_numpy()
        c.collide(db, b.tau, b.K, fused=True)
        c.check_errors()
        c.close()
        keys = [ln.split()[0] for ln in (tmp_path / f"{name}_tuned.txt").read_text().split("\n") if ln.strip()]
        assert keys
        for block in (128, 256, 64):
            path = tmp_path / f"{name}_{block}.txt"
            path.write_text("".join(f"{k} {block}\n" for k in keys))
            monkeypatch.setenv("CM_TUNE_CACHE", str(path))
            _say(f"[gpu] fused at block {block} vs plain: {name}, {b.n_scenes} scenes")
            c = Context(0)
            ids = c.create_geometry(b.geoms)
            db = c.upload_batch(b, ids)
            fused = c.collide(db, b.tau, b.K, fused=True).to_numpy()
            c.check_errors()
            t = c.fused_tuning()
            used = [i for i in range(3) if t["from_cache"][i]]
            assert used and all(t["class_blocks"][i] == block for i in used), t
            for k in ("pairs", "offsets", "p", "nu", "d", "w"):
                assert np.array_equal(plain[k], fused[k]), (name, block, k)
            c.close()
