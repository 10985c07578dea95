"""Oriented point clouds (a non-convex torus stand-in) against the FP64
oracle on an MI355X: broadphase bit for bit, outputs within |gpu - ref| <=
1e-6 + 2e-5 |ref|, gradients within 1e-3 of the oracle's autograd."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import cm_oracle as O
from tests.parity import compare_outputs

pytestmark = pytest.mark.gpu


@pytest.fixture
def ctx():
    from paper_2602_20304_amd.cm import Context
    return Context(0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_check(ctx, batch, presel=None, refine=0, max_pairs=None):
    _say(f"[gpu-opc] {batch.name} scenes={batch.n_scenes} K={batch.K} presel={presel} refine={refine}")
    ids = ctx.create_geometry(batch.geoms)
    db = ctx.upload_batch(batch, ids)
    got = ctx.collide(db, batch.tau, batch.K, presel=presel, refine=refine).to_numpy()
    ctx.check_errors()
    pairs, off = O.broadphase(batch)
    assert np.array_equal(got["offsets"], off) and np.array_equal(got["pairs"], pairs)
    n = pairs.shape[1]
    assert n > 0
    sel = np.arange(n)
    if max_pairs is not None and n > max_pairs:
        sel = np.sort(np.random.default_rng(0).choice(n, max_pairs, replace=False))
    _, _, ref = O.collide_batch(batch, pair_list=pairs[:, sel], presel=presel, refine=refine)
    ok, rep = compare_outputs(got, ref, idx=sel)
    _say(f"   parity {batch.name} ({len(sel)} of {n} pairs): {rep}")
    assert ok, rep


def test_opc_tori_with_analytic(ctx):
    run_check(ctx, W.opc_scenes(12, seed=1), max_pairs=24)


def test_opc_preselected_and_traced(ctx):
    run_check(ctx, W.opc_scenes(12, seed=2), presel=(24, 12), refine=3)


def test_opc_backward(ctx):
    from tests.test_gpu_backward import check as grad_check
    grad_check(ctx, W.opc_scenes(4, seed=3, nu=12, nv=6))


def test_opc_fused_matches_plain_bitwise(ctx):
    b = W.opc_scenes(24, seed=4)
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    _say(f"[gpu-opc] fused vs plain, scenes={b.n_scenes}")
    g1 = ctx.collide(db, b.tau, b.K).to_numpy()
    for _ in range(2):
        g2 = ctx.collide(db, b.tau, b.K, fused=True).to_numpy()
        ctx.check_errors()
        for k in ("pairs", "offsets", "p", "nu", "d", "w"):
            assert np.array_equal(g1[k], g2[k]), k
