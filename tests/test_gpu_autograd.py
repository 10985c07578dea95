"""The adjoint behind torch.autograd (collide_autograd): gradients that
autograd delivers for a scalar loss of the manifold outputs equal those of a
direct cm_collide_backward call with the loss's cotangents (needs an MI355X)."""
import sys

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2602_20304_amd.cm import Context
    return Context(0)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("presel,fused", [(None, False), (None, True), ((8, 12), False)])
def test_autograd_matches_direct_adjoint(ctx, presel, fused):
    from paper_2602_20304_amd.cm import collide_autograd
    b = W.mixed_scenes(12, seed=71, poly_points=16, tau=0.01)
    _say(f"[gpu-autograd] {b.name} scenes={b.n_scenes} presel={presel} fused={fused}")
    ids = ctx.create_geometry(b.geoms)
    db = ctx.upload_batch(b, ids)
    tau_t = torch.tensor(b.tau, device=ctx.device, requires_grad=True)
    xi = torch.zeros(6, db.n_bodies, device=ctx.device, requires_grad=True)
    p, nu, d, w, n_pairs, pairs = collide_autograd(ctx, db, tau_t, b.K, xi=xi, fused=fused, presel=presel)
    rng = np.random.default_rng(3)
    cot = {k: torch.as_tensor(rng.standard_normal(tuple(t.shape)).astype(np.float32), device=ctx.device)
           for k, t in (("p", p), ("nu", nu), ("d", d), ("w", w))}
    L = (p * cot["p"]).sum() + (nu * cot["nu"]).sum() + (d * cot["d"]).sum() + (w * cot["w"]).sum()
    L.backward()
    ctx.check_errors()
    # the same cotangents through the direct calls
    m = ctx.collide(db, b.tau, b.K, presel=presel)
    g = ctx.collide_backward(db, m, b.tau, b.K, cot["p"], cot["nu"], cot["d"], cot["w"], presel=presel)
    ctx.check_errors()
    ref_pose, ref_tau = g["pose"].cpu().numpy(), float(g["tau"][0])
    got_pose, got_tau = xi.grad.cpu().numpy(), float(tau_t.grad)
    scale = np.abs(ref_pose).max()
    _say(f"   pose max diff {np.abs(got_pose - ref_pose).max():.3e} (scale {scale:.3e}), tau {got_tau:.6g} vs {ref_tau:.6g}")
    assert int(n_pairs.item()) == int(m.n_pairs.item()) > 0
    assert np.abs(got_pose - ref_pose).max() <= 1e-5 * (scale + 1e-6)
    assert abs(got_tau - ref_tau) <= 1e-5 * (abs(ref_tau) + 1e-6)
