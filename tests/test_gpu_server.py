"""Serving loop (continuous batching over resident geometry) on an MI355X:
each result is the same alone and in the mix, admission respects the HBM
budget, oversize requests are rejected, latencies are reported."""
import sys
import time

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    from paper_2602_20304_amd.cm import Context
    ctx = Context(0)
    pool = W.polytope_pool(24, seed=1, n_points=20)
    ids = ctx.create_geometry(pool)
    return ctx, ids


def _alone(ctx, req, ids, tau, K, cot_d=None, cot_n=None):
    from paper_2602_20304_amd.cm import DeviceBatch
    dev = ctx.device
    db = DeviceBatch(req.n_env, int(len(req.body_geom)), torch.as_tensor(req.body_offsets, dtype=torch.int32).to(dev),
                     torch.as_tensor(ids[req.body_geom], dtype=torch.int32).to(dev),
                     torch.as_tensor(req.pose, dtype=torch.float32).contiguous().to(dev))
    m = ctx.collide(db, tau, K)
    ctx.check_errors()
    out = m.to_numpy()
    if cot_d is not None:
        g = ctx.collide_backward(db, m, tau, K, None, torch.as_tensor(cot_n).to(dev), torch.as_tensor(cot_d).to(dev),
                                 None, want_vertices=False, want_params=False)
        ctx.check_errors()
        out["g_pose"] = g["pose"].cpu().numpy()
    return out


def _wait(srv, tickets, budget, timeout=240):
    done = {}
    t0 = time.time()
    peak = 0
    while len(done) < len(tickets):
        st = srv.stats()
        peak = max(peak, st["in_flight_bytes"])
        assert st["in_flight_bytes"] <= budget
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return done, peak


def test_server_results_equal_alone(setup):
    from paper_2602_20304_amd.cm import Server
    ctx, ids = setup
    tau, K = 0.01, 8
    reqs = W.serving_requests(n_requests=10, seed=3, env_min=8, env_max=96, bodies_min=2, bodies_max=6,
                              pool_size=24)
    rng = np.random.default_rng(4)
    budget = 1 << 34
    srv = Server(ctx, budget, n_streams=4)
    tickets, cots = [], {}
    for i, q in enumerate(reqs):
        nb = len(q.body_geom)
        bo = q.body_offsets.astype(np.int64)
        cap = int((np.diff(bo) * (np.diff(bo) - 1) // 2).sum())
        cd = cn = None
        if q.want_bwd:
            cd = rng.standard_normal(cap * K).astype(np.float32)
            cn = rng.standard_normal(3 * cap * K).astype(np.float32)
        _say(f"[gpu-server] submit {i}: envs={q.n_env} bodies={nb} bwd={q.want_bwd}")
        t = srv.submit(q.body_offsets, ids[q.body_geom], q.pose, tau, K, q.want_bwd, cd, cn)
        tickets.append(t)
        cots[t] = (q, cd, cn)
    done, peak = _wait(srv, tickets, budget)
    lat = np.array([done[t]["t_done"] - done[t]["t_submit"] for t in tickets])
    _say(f"   server: p50 {np.percentile(lat, 50) * 1e3:.2f} ms  p99 {np.percentile(lat, 99) * 1e3:.2f} ms  "
         f"peak in-flight {peak / 2**20:.1f} MiB")
    for t in tickets:
        q, cd, cn = cots[t]
        r = done[t]
        assert r["status"] == 0
        a = _alone(ctx, q, ids, tau, K, cd, cn)
        for k in ("pairs", "offsets", "p", "nu", "d", "w"):
            assert np.array_equal(r[k], a[k]), k
        if q.want_bwd:
            g, ga = r["g_pose"], a["g_pose"]
            assert np.abs(g - ga).max() <= 1e-4 * (np.abs(ga).max() + 1e-6)
        srv.release(t)
    srv.close()


def test_server_budget_admission_and_rejection(setup):
    from paper_2602_20304_amd.cm import Server
    from paper_2602_20304_amd._lib import CMError
    ctx, ids = setup
    tau, K = 0.01, 8
    reqs = W.serving_requests(n_requests=8, seed=5, env_min=32, env_max=64, bodies_min=3, bodies_max=4,
                              pool_size=24)
    # probe one footprint with a huge budget, then size the budget for ~2 in flight
    srv = Server(ctx, 1 << 36, n_streams=4)
    q = reqs[0]
    t = srv.submit(q.body_offsets, ids[q.body_geom], q.pose, tau, K)
    done, _ = _wait(srv, [t], 1 << 36)
    fp = done[t]["footprint"]
    srv.release(t)
    srv.close()
    budget = int(2.5 * fp)
    srv = Server(ctx, budget, n_streams=4)
    tickets = [srv.submit(q.body_offsets, ids[q.body_geom], q.pose, tau, K) for q in reqs]
    done, peak = _wait(srv, tickets, budget)
    assert peak <= budget
    assert all(done[t]["status"] == 0 for t in tickets)
    # a request larger than the whole budget is rejected up front: its
    # outputs alone (28 pairs x K x 32 B per 8-body environment) exceed it
    n_big = int(budget // (28 * K * 32)) + 1
    big = W.serving_requests(n_requests=1, seed=6, env_min=n_big, env_max=n_big, bodies_min=8, bodies_max=8,
                             pool_size=24)[0]
    with pytest.raises(CMError) as e:
        srv.submit(big.body_offsets, ids[big.body_geom], big.pose, tau, K)
    assert e.value.status == -5
    for t in tickets:
        srv.release(t)
    srv.close()
