"""Batched E-E witness points (cm_ee_witness) against the FP64 oracle.

Edge pairs are drawn uniformly from the unit cube, as in the paper's
witness-point speed experiment (Sec. V, Fig. 6).  Outputs must agree element
by element within |gpu - ref| <= 1e-6 + 2e-5 |ref|; the 0/1 inside indicator
of the unsmoothed solver must agree exactly away from the box boundary.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import cm_oracle as O
from tests.parity import ATOL, RTOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2602_20304_amd.cm import Context
    return Context(0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(ctx, E, tau, hard, lam=-1.0):
    _say(f"[gpu-ee] n={E.shape[0]} tau={tau} hard={hard} lam={lam}")
    rows = np.ascontiguousarray(E.reshape(E.shape[0], 12).T, dtype=np.float32)
    out = ctx.ee_witness(torch.as_tensor(rows).to(ctx.device), tau, lam, hard=hard)
    torch.cuda.synchronize()
    o = out.cpu().numpy().astype(np.float64)
    return dict(al1=o[0], al2=o[1], con=o[2], e1=o[3:6].T, e2=o[6:9].T)


def compare(got, ref, hard):
    for k in ("al1", "al2", "e1", "e2") + (() if hard else ("con",)):
        ex = np.abs(got[k] - ref[k]) - (ATOL + RTOL * np.abs(ref[k]))
        assert ex.max() <= 0, (k, float(ex.max()), int(np.argmax(ex.reshape(ex.shape[0], -1).max(-1))))
    if hard:
        # the inside decision is made in float64 on both sides
        assert np.array_equal(got["con"], ref["con"])


@pytest.mark.parametrize("hard", [False, True])
@pytest.mark.parametrize("n", [1, 7, 100_000, 100_003])
def test_ee_witness_parity(ctx, n, hard):
    E = W.edge_pairs(n, seed=n)
    tau = 0.05
    got = run(ctx, E, tau, hard)
    ref = O.ee_witness_batch(E.astype(np.float32), tau, hard=hard)
    compare(got, ref, hard)


@pytest.mark.parametrize("tau", [0.5, 0.001])
def test_ee_witness_tau_sweep(ctx, tau):
    E = W.edge_pairs(50_000, seed=3)
    compare(run(ctx, E, tau, False), O.ee_witness_batch(E.astype(np.float32), tau), False)


def test_ee_witness_degenerate_edges(ctx):
    """Zero-length, parallel, identical and crossing edges."""
    rng = np.random.default_rng(5)
    E = W.edge_pairs(4096, seed=4).copy()
    E[0:512, 1] = E[0:512, 0]                        # edge 1 is a point
    E[512:1024, 3] = E[512:1024, 2]                  # edge 2 is a point
    d = rng.uniform(-1, 1, (512, 1, 3))
    E[1024:1536, 2:4] = E[1024:1536, 0:2] + 0.1 * d  # parallel, offset
    E[1536:2048, 2:4] = E[1536:2048, 0:2]            # identical
    E[2048:2560, 2:4] = E[2048:2560, 1::-1]          # identical, reversed
    for hard in (False, True):
        for lam in (-1.0, 0.3):
            got = run(ctx, E, 0.02, hard, lam)
            ref = O.ee_witness_batch(E.astype(np.float32), 0.02, 0.01 if lam < 0 else lam, hard=hard)
            if hard:
                # ties between box edges pick the same unique minimiser; the
                # 0/1 indicator can flip only where the minimiser is on the boundary
                on_edge = (np.minimum.reduce([ref["al1"], 1 - ref["al1"], ref["al2"], 1 - ref["al2"]]) < 1e-9)
                keep = ~on_edge
                assert np.array_equal(got["con"][keep], ref["con"][keep])
                got = {k: v for k, v in got.items()}
                got["con"] = ref["con"]
            compare(got, ref, hard)


def test_ee_witness_full_size_sampled(ctx):
    """10^7 queries (the largest size of the experiment), checked on a sample."""
    n = 10_000_000
    E = W.edge_pairs(n, seed=9)
    got = run(ctx, E, 0.05, False)
    sel = np.sort(np.random.default_rng(1).choice(n, 20_000, replace=False))
    ref = O.ee_witness_batch(E[sel].astype(np.float32), 0.05)
    compare({k: v[sel] for k, v in got.items()}, ref, False)


def test_ee_witness_empty_and_errors(ctx):
    from paper_2602_20304_amd._lib import CMError
    e = torch.zeros(12, 0, device=ctx.device)
    assert ctx.ee_witness(e, 0.05).shape == (9, 0)
    e = torch.zeros(12, 8, device=ctx.device)
    with pytest.raises(CMError):
        ctx.ee_witness(e, 0.0)
    with pytest.raises(CMError):
        ctx.ee_witness(e, 0.05, lambda_reg=0.0)
    out = ctx.ee_witness(e, 0.0, hard=True)     # tau is unused without smoothing
    torch.cuda.synchronize()
    assert torch.isfinite(out).all()
