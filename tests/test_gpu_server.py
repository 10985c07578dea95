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


def _oracle_env_check(q, r, pool, tau, K, envs, cot=None):
    """Served outputs of the kept pairs in environments `envs` against the
    FP64 oracle; with cot (host cotangents laid out like the outputs) also
    the pose gradients of those environments' bodies."""
    from oracle import cm_oracle as O
    from tests.parity import excess
    from tests.test_gpu_backward import close
    cache = O.GeomCache(pool, requires_grad=cot is not None)
    off = r["offsets"]
    worst, n = -1.0, 0
    g_ref, bodies = {}, []
    for e in envs:
        for i in range(int(off[e]), int(off[e + 1])):
            a, b = int(r["pairs"][0, i]), int(r["pairs"][1, i])
            GA, GB = cache[q.body_geom[a]], cache[q.body_geom[b]]
            import torch
            with torch.no_grad():
                ref = O.collide_pair(GA, q.pose[:, a], GB, q.pose[:, b], tau, K)
            for k in ("p", "nu", "d", "w"):
                worst = max(worst, float(excess(r[k][i], ref[k].numpy()).max()))
            n += 1
            if cot is not None:
                sl = slice(i * K, (i + 1) * K)
                c = dict(p=cot["p"][:, sl].T, nu=cot["nu"][:, sl].T, d=cot["d"][sl], w=cot["w"][sl])
                g = O.pair_grad(GA, q.pose[:, a], GB, q.pose[:, b], tau, K, c)
                g_ref[a] = g_ref.get(a, 0) + g["xiA"]
                g_ref[b] = g_ref.get(b, 0) + g["xiB"]
        bodies += list(range(int(q.body_offsets[e]), int(q.body_offsets[e + 1])))
    rep = {"pairs": n, "max_excess": worst}
    if cot is not None:
        got = np.stack([r["g_pose"][:, b] for b in bodies])
        ref = np.stack([g_ref.get(b, np.zeros(6)) for b in bodies])
        rep["g_pose"] = close(got, ref)
    return rep


def test_served_results_against_oracle_sample():
    """Served requests over a resident pool of 64-point hulls (the
    differentiation workload's bodies), forward and forward + backward with
    all four cotangents: on a seeded 1 % of each request's environments (at
    least 2) every kept pair matches the FP64 oracle, and so do the pose
    gradients of those environments' bodies."""
    from paper_2602_20304_amd.cm import Context, Server
    ctx = Context(0)
    pool = W.polytope_pool(32, seed=3, n_points=64)
    ids = ctx.create_geometry(pool)
    tau, K = 0.01, 8
    reqs = W.serving_requests(n_requests=4, seed=8, env_min=150, env_max=300, bodies_min=2, bodies_max=5,
                              pool_size=32)
    rng = np.random.default_rng(9)
    srv = Server(ctx, 1 << 34, n_streams=3)
    tickets = []
    for q in reqs:
        nbe = np.diff(q.body_offsets.astype(np.int64))
        cap = int((nbe * (nbe - 1) // 2).sum())
        cot = None
        if q.want_bwd:
            cot = dict(p=rng.standard_normal((3, cap * K)).astype(np.float32),
                       nu=rng.standard_normal((3, cap * K)).astype(np.float32),
                       d=rng.standard_normal(cap * K).astype(np.float32),
                       w=rng.standard_normal(cap * K).astype(np.float32))
        _say(f"[gpu-server] oracle sample: submit envs={q.n_env} bwd={q.want_bwd}")
        t = srv.submit(q.body_offsets, ids[q.body_geom], q.pose, tau, K, q.want_bwd,
                       None if cot is None else cot["d"], None if cot is None else cot["nu"],
                       cot_point=None if cot is None else cot["p"], cot_weight=None if cot is None else cot["w"])
        tickets.append((t, q, cot))
    done, _ = _wait(srv, [t for t, _, _ in tickets], 1 << 34)
    assert any(c is not None for _, _, c in tickets) and any(c is None for _, _, c in tickets)
    for t, q, cot in tickets:
        r = done[t]
        assert r["status"] == 0
        envs = np.sort(rng.choice(q.n_env, size=max(2, q.n_env // 100), replace=False))
        rep = _oracle_env_check(q, r, pool, tau, K, envs, cot)
        _say(f"   served vs oracle ({len(envs)} envs of {q.n_env}): {rep}")
        assert rep["pairs"] > 0 and rep["max_excess"] <= 0, rep
        if cot is not None:
            assert rep["g_pose"][0] <= 0, rep
        srv.release(t)
    srv.close()
    ctx.close()


def test_served_backward_all_gradients_match_direct(setup):
    """A served backward request with all four cotangents and geometry
    gradients equals cm_collide_backward run alone on the same request:
    pose, tau, hull-vertex and parameter gradients (float atomics may
    reorder: 1e-4 relative)."""
    from paper_2602_20304_amd.cm import DeviceBatch, Server
    ctx, ids = setup
    tau, K = 0.01, 8
    q = W.serving_requests(n_requests=1, seed=12, env_min=40, env_max=40, bodies_min=3, bodies_max=5,
                           pool_size=24)[0]
    nbe = np.diff(q.body_offsets.astype(np.int64))
    cap = int((nbe * (nbe - 1) // 2).sum())
    rng = np.random.default_rng(13)
    cot = dict(p=rng.standard_normal((3, cap * K)).astype(np.float32),
               nu=rng.standard_normal((3, cap * K)).astype(np.float32),
               d=rng.standard_normal(cap * K).astype(np.float32),
               w=rng.standard_normal(cap * K).astype(np.float32))
    srv = Server(ctx, 1 << 34, n_streams=2)
    _say(f"[gpu-server] full backward: envs={q.n_env}")
    t = srv.submit(q.body_offsets, ids[q.body_geom], q.pose, tau, K, True, cot["d"], cot["nu"],
                   cot_point=cot["p"], cot_weight=cot["w"], want_geometry=True)
    done, _ = _wait(srv, [t], 1 << 34)
    r = done[t]
    assert r["status"] == 0
    dev = ctx.device
    db = DeviceBatch(q.n_env, int(len(q.body_geom)), torch.as_tensor(q.body_offsets, dtype=torch.int32).to(dev),
                     torch.as_tensor(ids[q.body_geom], dtype=torch.int32).to(dev),
                     torch.as_tensor(q.pose, dtype=torch.float32).contiguous().to(dev))
    m = ctx.collide(db, tau, K)
    tt = {k: torch.as_tensor(v).to(dev) for k, v in cot.items()}
    g = ctx.collide_backward(db, m, tau, K, tt["p"], tt["nu"], tt["d"], tt["w"])
    ctx.check_errors()
    ref = {"g_pose": g["pose"].cpu().numpy(), "g_tau": float(g["tau"].item()),
           "g_vertices": g["vertices"].cpu().numpy(), "g_params": g["params"].cpu().numpy()}
    for k in ("g_pose", "g_vertices", "g_params"):
        a, b = np.asarray(r[k], np.float64), np.asarray(ref[k], np.float64)
        assert a.shape == b.shape, k
        assert np.abs(a - b).max() <= 1e-4 * (np.abs(b).max() + 1e-6), k
    assert abs(r["g_tau"] - ref["g_tau"]) <= 1e-4 * (abs(ref["g_tau"]) + 1e-6)
    srv.release(t)
    srv.close()


def test_served_errors_per_request(setup):
    """A request naming a geometry id the context does not hold is refused at
    submit with CM_ERR_NOT_FOUND and a message on the calling thread; a
    malformed body_offsets is CM_ERR_INVALID_ARG; other requests are
    unaffected."""
    from paper_2602_20304_amd.cm import Server
    from paper_2602_20304_amd._lib import CMError
    ctx, ids = setup
    tau, K = 0.01, 8
    q = W.serving_requests(n_requests=1, seed=14, env_min=8, env_max=8, bodies_min=2, bodies_max=3,
                           pool_size=24)[0]
    srv = Server(ctx, 1 << 34, n_streams=2)
    bad_geom = ids[q.body_geom].copy()
    bad_geom[0] = 10 ** 6
    with pytest.raises(CMError) as e:
        srv.submit(q.body_offsets, bad_geom, q.pose, tau, K)
    assert e.value.status == -6 and "geometry" in str(e.value)
    bad_off = q.body_offsets.copy()
    bad_off[0] = -1
    with pytest.raises(CMError) as e:
        srv.submit(bad_off, ids[q.body_geom], q.pose, tau, K)
    assert e.value.status == -1 and "body_offsets" in str(e.value)
    t = srv.submit(q.body_offsets, ids[q.body_geom], q.pose, tau, K)
    done, _ = _wait(srv, [t], 1 << 34)
    assert done[t]["status"] == 0
    srv.release(t)
    srv.close()
