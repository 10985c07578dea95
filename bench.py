"""Benchmark of the contact-manifold hot path on one MI355X.

A step is one pass of the whole path -- float32 bounding-sphere broadphase,
per-scene compaction, vertex-SDF both ways, all-pairs edge-edge witness
contacts with their indicators, and the SoftSort K-contact manifold -- over
one batch of synthetic scenes already resident in HBM.

Default workload: 65,536 scenes x 8 bodies (2 spheres, 2 capsules, 2 rounded
boxes, 2 convex polytopes of 32 points), all 28 pairs per scene are
candidates, tau = 0.005, K = 8.

Legs, all in one process on the same inputs:
  plain     cm_collide (broadphase + one forward pair kernel)
  fused     cm_collide_fused (cost-ordered work queue, replayed hipGraph)
  fwd_bwd   cm_collide + cm_collide_backward with random cotangents
  plain_ne, plain_ne_s     the no-E-E / one-sided simplification flags
  plain_presel, fwd_bwd_presel   soft top-K pre-selection (K_V 64, K_E 18)
  plain_refine  E-E witnesses sphere-traced onto the smoothed surfaces (3 steps)
  plain_presel_refine   the two together (tracing after pre-selection)
  serving   a short Poisson request stream through cm_server_* (p50 / p99)
The headline value is the forward throughput of --path (fused by default).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "geom-pair contact evals/s (fwd, fwd+bwd) vs plain kernel; p50/p99 query latency"
FWD_KERNEL = "collide_fwd"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "collide_fwd_mixed65536_traffic.md")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_workload(name: str, scenes: int | None):
    import workloads as W
    if name == "mixed":
        b = W.mixed_scenes(scenes or 65536, seed=0)
        desc = (f"mixed_scenes: {b.n_scenes} scenes x 8 bodies (2 sphere, 2 capsule, 2 rounded box, "
                f"2 polytope hull-of-32), all 28 pairs/scene candidates, tau={b.tau:g}, K={b.K}")
    elif name == "cubes":
        b = W.cube_pairs(scenes or 4096, seed=0)
        desc = f"cube_pairs: {b.n_scenes} scenes x 1 cube pair (8 V / 12 E), tau={b.tau:g}, K={b.K}"
    elif name == "polytopes":
        b = W.polytope_scenes(scenes or 16384, seed=0)
        desc = (f"polytope_scenes: {b.n_scenes} scenes x 4 polytopes (hull of 64: 64 V / 186 E / 124 F), "
                f"6 pairs/scene, tau={b.tau:g}, K={b.K}")
    elif name == "uneven":
        b = W.uneven_scenes(scenes or 100_000, seed=0)
        desc = (f"uneven_scenes: {b.n_scenes} scenes, geometric pairs/scene (mean 12), polytopes 8-256 V, "
                f"20% analytic, 30% forced penetration, tau={b.tau:g}, K={b.K}")
    else:
        raise SystemExit(f"unknown workload {name}")
    return b, desc


FWD_SOURCES = ("cm_fwd.hip", "cm_pair.cuh", "cm_device.cuh", "cm_kernels.h", "cm_internal.h")
EE_SOURCES = ("cm_ee.hip", "cm_device.cuh", "cm_kernels.h", "cm_internal.h")
EE_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ee_witness_1e7_traffic.md")


def source_hash(files=FWD_SOURCES) -> str:
    """Hash of a kernel's sources (a stored traffic figure is void once they change)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2602_20304_amd", "csrc")
    for f in sorted(files):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def stored_traffic(path: str, files, key: str = "traffic_bytes_per_launch"):
    """HBM bytes per launch from a committed PMC summary, or None when it is
    absent or was taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_hash = re.search(r"source_hash:\s*([0-9a-f]+)", txt)
    m_bytes = re.search(key + r":\s*([0-9.eE+]+)", txt)
    if not m_hash or not m_bytes or m_hash.group(1) != source_hash(files):
        return None
    return float(m_bytes.group(1))


def cpu_baseline(batch, budget_s: float):
    """Time the FP64 oracle on the host over whole scenes in scene order until
    the time budget is spent.  Only the per-pair evaluations are timed (the
    oracle's mesh and hull construction for a geometry happens before)."""
    import torch
    from oracle import cm_oracle as O
    pairs, offsets = O.broadphase(batch)
    cache = O.GeomCache(batch.geoms)
    threads = int(torch.get_num_threads())
    spent = 0.0
    done = 0
    scenes = 0
    with torch.no_grad():
        for s in range(batch.n_scenes):
            for i in range(int(offsets[s]), int(offsets[s + 1])):
                a, b = int(pairs[0, i]), int(pairs[1, i])
                GA, GB = cache[batch.body_geom[a]], cache[batch.body_geom[b]]
                t0 = time.perf_counter()
                O.collide_pair(GA, batch.pose[:, a], GB, batch.pose[:, b], batch.tau, batch.K)
                spent += time.perf_counter() - t0
                done += 1
            scenes += 1
            if spent > budget_s:
                break
    return dict(value=done / spent, unit="pairs/s", cores=threads, kind="oracle",
                sample=f"first {scenes} scenes ({done} kept pairs) of the same workload, FP64 oracle, "
                       f"{spent:.1f} s of pair evaluation, torch intra-op threads={threads}, "
                       f"mesh builds excluded")


def serving_leg(ctx_cls, n_requests: int, seed: int = 11):
    """Poisson request stream through the serving loop.

    A burst of requests (all submitted at once) first measures the saturated
    request throughput; the stream then arrives at 0.7 of it, so latencies
    reflect service time rather than an ever-growing queue."""
    import workloads as W
    from paper_2602_20304_amd.cm import Server
    ctx = ctx_cls(0)
    pool = W.polytope_pool(64, seed=1, n_points=64)
    ids = ctx.create_geometry(pool)
    tau, K = 0.01, 8
    n_cal = max(4, n_requests // 2)
    reqs = W.serving_requests(n_requests=n_cal + n_requests, seed=seed, rate_hz=1.0, env_min=256, env_max=4096,
                              bodies_min=2, bodies_max=6, pool_size=64)
    rng = np.random.default_rng(seed)
    payload = []
    for q in reqs:
        nbe = np.diff(q.body_offsets.astype(np.int64))
        cap = int((nbe * (nbe - 1) // 2).sum())
        cd = cn = None
        if q.want_bwd:
            cd = rng.standard_normal(cap * K).astype(np.float32)
            cn = rng.standard_normal(3 * cap * K).astype(np.float32)
        payload.append((q, cd, cn))
    srv = Server(ctx, 64 << 30, n_streams=4)

    def run(items, arrivals):
        tickets = []
        t0 = time.perf_counter()
        for (q, cd, cn), at in zip(items, arrivals):
            wait = at - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            tickets.append(srv.submit(q.body_offsets, ids[q.body_geom], q.pose, tau, K, q.want_bwd, cd, cn))
        done = {}
        while len(done) < len(tickets):
            for t in tickets:
                if t not in done:
                    r = srv.poll(t)
                    if r is not None:
                        if r["status"] != 0:
                            raise RuntimeError(f"request {t} failed with status {r['status']}")
                        done[t] = (r["t_submit"], r["t_start"], r["t_done"], r["n_pairs"])
                        srv.release(t)
            time.sleep(0.001)
        return done, time.perf_counter() - t0

    def run_plain(items):
        # the same requests one at a time through cm_collide / cm_collide_backward
        import torch
        from paper_2602_20304_amd.cm import DeviceBatch
        dev = ctx.device
        t0 = time.perf_counter()
        pairs = 0
        for q, cd, cn in items:
            db = DeviceBatch(q.n_env, len(q.body_geom), torch.as_tensor(q.body_offsets, dtype=torch.int32).to(dev),
                             torch.as_tensor(ids[q.body_geom], dtype=torch.int32).to(dev),
                             torch.as_tensor(q.pose, dtype=torch.float32).contiguous().to(dev))
            m = ctx.collide(db, tau, K)
            if q.want_bwd:
                ctx.collide_backward(db, m, tau, K, None, torch.as_tensor(cn).to(dev), torch.as_tensor(cd).to(dev),
                                     None, want_vertices=False, want_params=False)
            out = m.to_numpy()
            pairs += out["n_pairs"]
        torch.cuda.synchronize()
        return pairs / (time.perf_counter() - t0)

    run(payload[:2], [0.0, 0.0])          # warm-up (module loads, first allocations), not timed
    run_plain(payload[:2])
    cal, cal_wall = run(payload[:n_cal], [0.0] * n_cal)
    sat = n_cal / cal_wall
    rate = 0.7 * sat
    gaps = np.random.default_rng(seed + 1).exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    done, wall = run(payload[n_cal:], arrivals)
    srv.close()
    burst_pairs = sum(d[3] for d in cal.values()) / cal_wall
    plain_pairs = run_plain(payload[:n_cal])
    lat = np.array([d[2] - d[0] for d in done.values()])
    pairs = sum(d[3] for d in done.values())
    return dict(requests=len(done), rate_per_s=rate, saturated_per_s=sat, burst_pairs_per_s=burst_pairs,
                plain_sequential_pairs_per_s=plain_pairs, p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), pairs_per_s=pairs / wall, wall_s=wall,
                config=f"{n_requests} Poisson requests at 0.7 x the saturated rate measured on a burst of {n_cal}; "
                       f"256-4096 envs (log-uniform), 2-6 bodies/env from a resident pool of 64 hull-of-64 polytopes, "
                       f"fwd or fwd+bwd 50/50, tau={tau}, K={K}, 4 streams, 64 GiB budget")


EE_BYTES_PER_QUERY = 12 * 4 + 9 * 4   # float32 rows in (a0, a1, b0, b1) and out (alpha, con, e1, e2)


def ee_witness_leg(ctx, trials: int = 100, max_n: int = 10_000_000, tau: float = 0.05):
    """The witness-point speed experiment (Sec. V, Fig. 6): n edge pairs
    uniform in the unit cube, n = 1 .. max_n by decades, `trials` timed
    launches each (mean and standard deviation), smoothed and unsmoothed."""
    import torch
    import workloads as W
    sizes = [10 ** k for k in range(0, 8) if 10 ** k <= max_n]
    E = W.edge_pairs(max_n, seed=2)
    rows = torch.as_tensor(np.ascontiguousarray(E.reshape(max_n, 12).T)).to(ctx.device)
    del E
    stream = torch.cuda.current_stream()
    res = {"sizes": sizes, "trials": trials, "tau": tau}
    for mode in ("smooth", "hard"):
        hard = mode == "hard"
        means, stds = [], []
        for n in sizes:
            ed = rows[:, :n].contiguous()
            out = torch.empty(9, n, dtype=torch.float32, device=ctx.device)
            for _ in range(3):
                ctx.ee_witness(ed, tau, hard=hard, out=out, stream=stream)
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(trials)]
            torch.cuda.synchronize()
            ctx.set_kernel_timing(True)
            for a, b in evs:
                a.record(stream)
                ctx.ee_witness(ed, tau, hard=hard, out=out, stream=stream)
                b.record(stream)
            torch.cuda.synchronize()
            k_ms, k_n = ctx.kernel_time("ee_witness")
            ctx.set_kernel_timing(False)
            t = np.array([a.elapsed_time(b) for a, b in evs])
            means.append(k_ms / k_n)
            stds.append(float(t.std()))
            del ed, out
        res[f"{mode}_ms"] = means
        res[f"{mode}_std_ms"] = stds
        kms = means[-1]
        gbs = EE_BYTES_PER_QUERY * sizes[-1] / (kms * 1e-3) / 1e9
        res[f"{mode}_queries_per_s"] = sizes[-1] / (kms * 1e-3)
        traffic = stored_traffic(EE_TRAFFIC_FILE, EE_SOURCES, f"{mode}_traffic_bytes_per_launch")
        res[f"{mode}_roofline"] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": gbs / HBM_PEAK_GBS, "bytes_per_query": EE_BYTES_PER_QUERY,
                                   "queries_per_launch": sizes[-1], "traffic": traffic}
    return res


def sq_leg(ctx_cls, steps: int = 5, scenes_presel: int = 4096, scenes_all: int = 256):
    """Superquadric-union bodies (the paper's default primitive family): two
    bodies per scene, each a smooth union of 18 superquadrics with a
    ~350-vertex / ~800-edge mesh.  Forward with the paper's benchmark
    pre-selection (K_V 64, K_E 18) and, on fewer scenes, over all edge pairs.
    Its own context: contexts holding superquadric unions run the kernels
    built for them."""
    import torch
    import workloads as W
    ctx = ctx_cls(0)
    stream = torch.cuda.current_stream()
    res = {}
    configs = (("presel_64_18", scenes_presel, (64, 18), "sq"), ("all_edge_pairs", scenes_all, None, "sq"),
               ("opc_tori_all_edge_pairs", scenes_presel // 4, None, "opc"))
    for name, n, presel, kind in configs:
        b = W.sq_scenes(n, seed=3) if kind == "sq" else W.opc_scenes(n, seed=3)
        ids = ctx.create_geometry(b.geoms)
        db = ctx.upload_batch(b, ids)
        out = ctx.collide(db, b.tau, b.K, stream=stream, presel=presel)
        torch.cuda.synchronize()
        ctx.check_errors()
        ctx.set_kernel_timing(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(steps):
            ctx.collide(db, b.tau, b.K, out=out, stream=stream, presel=presel)
        ev1.record(stream)
        torch.cuda.synchronize()
        k_ms, k_n = ctx.kernel_time("forward")
        ctx.set_kernel_timing(False)
        ctx.check_errors()
        ms = ev0.elapsed_time(ev1) / steps
        kept = int(out.n_pairs.item())
        info = [ctx.geometry_info(int(g)) for g in ids]
        res[name] = {"scenes": n, "kept_pairs": kept, "ms_per_step": ms, "forward_kernel_ms": k_ms / max(k_n, 1),
                     "pairs_per_s": kept / (ms * 1e-3), "presel": list(presel) if presel else None,
                     "mesh_vertices": [i["n_vertices"] for i in info], "mesh_edges": [i["n_edges"] for i in info]}
        log(f"sq {name}: {ms:.3f} ms/step, {kept} kept pairs, {kept / (ms * 1e-3):.4g} pairs/s")
    res["config"] = ("2 bodies per scene from a pool of 8 smooth unions of 18 superquadrics (semi-axes U[0.07, 0.16], "
                     "torso x2, exponents U[0.3, 1.5]), centres uniform in [-0.6, 0.6]^3, tau 0.01, K 8; "
                     "opc_tori: 2 oriented-point-cloud tori (128 points, 4-NN mesh edges) and a sphere or rounded box "
                     "per scene, centres uniform in [-0.35, 0.35]^3")
    return res


def copy_calibration(n_bytes: int, reps: int):
    """Plain device copy of a known size (for scaling PMC byte counters)."""
    import torch
    n = n_bytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "bytes_written": 4 * n, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed")
    ap.add_argument("--scenes", type=int, default=None)
    ap.add_argument("--path", default="fused", choices=["plain", "fused"])
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--serve", type=int, default=16, help="requests in the serving leg (0 = skip)")
    ap.add_argument("--no-ee", action="store_true", help="skip the E-E witness microbenchmark")
    ap.add_argument("--ee-only", action="store_true", help="run only the E-E witness microbenchmark")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving leg")
    ap.add_argument("--no-sq", action="store_true", help="skip the superquadric-union leg")
    ap.add_argument("--sq-only", action="store_true", help="run only the superquadric-union leg")
    ap.add_argument("--ee-trials", type=int, default=100, help="timed launches per size in the E-E sweep")
    ap.add_argument("--no-simplifications", action="store_true",
                    help="skip the forward legs without E-E (ne), with one-sided vertex contacts (ne_s) and "
                         "with soft top-K pre-selection (presel)")
    ap.add_argument("--only", default=None,
                    choices=[None, "plain", "fused", "fwd_bwd", "plain_ne", "plain_ne_s", "plain_presel",
                             "fwd_bwd_presel", "plain_refine", "fused_presel", "plain_presel_refine"],
                    help="run one leg only (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (PMC byte calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on exactly one GPU; --gpus must be 1"}), flush=True)
        raise SystemExit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration << 20, 5)
        return

    import torch
    import workloads as W
    from paper_2602_20304_amd.cm import FLAG_NO_EE, FLAG_ONE_SIDED_VS, Context, Manifold
    from paper_2602_20304_amd import opmodel

    if args.serve_only:
        print(json.dumps({"serving": serving_leg(Context, args.serve or 16)}), flush=True)
        return
    if args.sq_only:
        print(json.dumps({"superquadrics": sq_leg(Context, steps=args.steps)}), flush=True)
        return
    if args.ee_only:
        ctx = Context(0)
        print(json.dumps({"ee_witness": ee_witness_leg(ctx, trials=args.ee_trials)}), flush=True)
        return

    batch, desc = build_workload(args.workload, args.scenes)
    log(f"workload: {desc}")
    ctx = Context(0)
    t0 = time.perf_counter()
    ids = ctx.create_geometry(batch.geoms)
    t_geom = time.perf_counter() - t0
    db = ctx.upload_batch(batch, ids)
    cap = db.n_cand_total
    out = Manifold.empty(db.n_scenes, cap, batch.K, ctx.device)
    log(f"geometry build {t_geom:.1f}s; {batch.n_bodies} bodies, {cap} candidate pairs")
    stream = torch.cuda.current_stream()
    cot_d = cot_n = None
    if not args.no_bwd:
        a, b = W.cotangents(cap, batch.K, seed=1)
        cot_d = torch.as_tensor(a).to(ctx.device)
        cot_n = torch.as_tensor(b).to(ctx.device)

    leg_flags = {"plain_ne": FLAG_NO_EE, "plain_ne_s": FLAG_NO_EE | FLAG_ONE_SIDED_VS}
    # the paper's benchmark shape: every vertex (K_V at its cap of 64 covers the
    # meshes here) and the K_E = 18 deepest edges per body
    leg_presel = {"plain_presel": (64, 18), "fwd_bwd_presel": (64, 18), "fused_presel": (64, 18),
                  "plain_presel_refine": (64, 18)}

    leg_refine = {"plain_refine": 3, "plain_presel_refine": 3}

    def step(leg):
        ctx.collide(db, batch.tau, batch.K, out=out, fused=(leg in ("fused", "fused_presel")), stream=stream,
                    flags=leg_flags.get(leg, 0), presel=leg_presel.get(leg), refine=leg_refine.get(leg, 0))
        if leg in ("fwd_bwd", "fwd_bwd_presel"):
            ctx.collide_backward(db, out, batch.tau, batch.K, None, cot_n, cot_d, None, stream=stream,
                                 presel=leg_presel.get(leg))

    legs = ["plain", "fused"] + ([] if args.no_bwd else ["fwd_bwd"])
    legs += [] if args.no_simplifications else ["plain_ne", "plain_ne_s", "plain_presel", "fused_presel",
                                                "plain_refine", "plain_presel_refine"]
    legs += [] if (args.no_simplifications or args.no_bwd) else ["fwd_bwd_presel"]
    if args.only:
        legs = [args.only]
    results = {}
    kernel = {}
    for leg in legs:
        for _ in range(args.warmup):
            step(leg)
        torch.cuda.synchronize()
        ctx.check_errors()
        ctx.set_kernel_timing(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            step(leg)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        kernel[leg] = {t: ctx.kernel_time(t) for t in ("broadphase", "forward", "backward", "fused")}
        ctx.set_kernel_timing(False)
        ctx.check_errors()
        n_pairs = int(out.n_pairs.item())
        results[leg] = dict(ms=ms, n_pairs=n_pairs)
        log(f"{leg}: {ms:.3f} ms/step, {n_pairs} kept pairs, {n_pairs / (ms * 1e-3):.4g} pairs/s; "
            + ", ".join(f"{k} {v[0] / max(v[1], 1):.3f} ms x{v[1]}" for k, v in kernel[leg].items() if v[1]))

    main_leg = args.path if args.path in results else legs[0]
    ms = results[main_leg]["ms"]
    n_pairs = results[main_leg]["n_pairs"]
    kept = min(n_pairs, cap)
    pairs = out.pairs[:, :kept].cpu().numpy()
    G = ctx.geometry_count
    sizes = np.array([[ctx.geometry_info(int(g))[k] for k in ("type", "n_vertices", "n_edges", "n_faces")]
                      for g in range(G)], dtype=np.int64)
    body_geom = ids[batch.body_geom]
    ops = opmodel.batch_ops(sizes[:, 0], sizes[:, 1], sizes[:, 2], sizes[:, 3], pairs[0], pairs[1], body_geom)

    # roofline of the dominant kernel: the forward pair kernel, timed with HIP
    # events on its own stream during the plain leg (one launch = all kept pairs)
    roof_leg = "plain" if "plain" in kernel else main_leg
    k_ms, k_n = kernel[roof_leg]["forward"]
    roofline = None
    if k_n:
        kms = k_ms / k_n
        roof = opmodel.roofline(ops, kms * 1e-3)
        traffic = stored_traffic(TRAFFIC_FILE, FWD_SOURCES) if args.workload == "mixed" else None
        roofline = {"bound": "alu", "kernel": FWD_KERNEL, "achieved": roof["achieved_flops"] / 1e12,
                    "peak": roof["peak_flops"] / 1e12, "unit": "TFLOP/s", "frac": roof["frac"],
                    "traffic": traffic, "kernel_ms": kms, "launches": k_n,
                    "ops_per_launch": {"fma": int(ops[0]), "alu": int(ops[1]), "trans": int(ops[2])}}
        # the fused path does the same algorithmic work; its time is the whole
        # replayed graph (broadphase, classification, class launches) timed
        # with HIP events around the graph launch, so this rate is a lower
        # bound for its pair kernel
        f_ms, f_n = kernel["fused"]["fused"] if "fused" in kernel else (0.0, 0)
        if f_n:
            froof = opmodel.roofline(ops, f_ms / f_n * 1e-3)
            roofline["fused_path"] = {"achieved": froof["achieved_flops"] / 1e12, "frac": froof["frac"],
                                      "graph_ms": f_ms / f_n, "launches": f_n}

    legs_out = {}
    for k, v in results.items():
        legs_out[k] = {"ms_per_step": v["ms"], "pairs_per_s": v["n_pairs"] / (v["ms"] * 1e-3)}
        for t, (tms, tn) in kernel[k].items():
            if tn:
                legs_out[k][f"{t}_kernel_ms"] = tms / tn
    line = {
        "metric": METRIC,
        "value": n_pairs / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": desc, "scenes": batch.n_scenes, "candidate_pairs": cap, "kept_pairs": n_pairs,
                   "tau": batch.tau, "K": batch.K, "path": main_leg, "parallelism": "single-gpu"},
        "legs": legs_out,
        "roofline": roofline,
    }
    if "fwd_bwd" in results:
        v = results["fwd_bwd"]
        line["fwd_bwd_pairs_per_s"] = v["n_pairs"] / (v["ms"] * 1e-3)
    if "plain" in results and main_leg != "plain":
        line["speedup_vs_plain"] = results["plain"]["ms"] / ms
    if "plain" in results and "plain_ne" in results and "plain_ne_s" in results:
        line["simplifications"] = {"ne_speedup": results["plain"]["ms"] / results["plain_ne"]["ms"],
                                   "ne_s_speedup_over_ne": results["plain_ne"]["ms"] / results["plain_ne_s"]["ms"]}
    if "plain" in results and "plain_presel" in results:
        line["preselection"] = {"presel": list(leg_presel["plain_presel"]),
                                "speedup_vs_all_pairs": results["plain"]["ms"] / results["plain_presel"]["ms"]}
        if "fused_presel" in results:
            line["preselection"]["fused_speedup_vs_plain_presel"] = (results["plain_presel"]["ms"]
                                                                     / results["fused_presel"]["ms"])
        if "fwd_bwd" in results and "fwd_bwd_presel" in results:
            line["preselection"]["fwd_bwd_speedup_vs_all_pairs"] = (results["fwd_bwd"]["ms"]
                                                                    / results["fwd_bwd_presel"]["ms"])
    if "plain" in results and "plain_refine" in results:
        line["witness_refinement"] = {"steps": leg_refine["plain_refine"],
                                      "cost_vs_plain": results["plain_refine"]["ms"] / results["plain"]["ms"]}
        if "plain_presel" in results and "plain_presel_refine" in results:
            line["witness_refinement"]["presel_cost_vs_plain_presel"] = (results["plain_presel_refine"]["ms"]
                                                                         / results["plain_presel"]["ms"])
    if args.serve and not args.only:
        log(f"serving leg: {args.serve} requests ...")
        line["serving"] = serving_leg(Context, args.serve)
        log(f"serving: {line['serving']['rate_per_s']:.2f} req/s (saturated {line['serving']['saturated_per_s']:.2f}), "
            f"p50 {line['serving']['p50_ms']:.1f} ms, p99 {line['serving']['p99_ms']:.1f} ms")
    if not args.no_ee:
        log("E-E witness microbenchmark ...")
        ee = ee_witness_leg(ctx)
        line["ee_witness"] = ee
        log("ee_witness: " + ", ".join(f"n={n}: {a:.4f}/{b:.4f} ms" for n, a, b in
                                       zip(ee["sizes"], ee["smooth_ms"], ee["hard_ms"])) +
            f"; 1e7 smooth {ee['smooth_roofline']['achieved']:.0f} GB/s, hard {ee['hard_roofline']['achieved']:.0f} GB/s")
    if not args.no_sq and not args.only:
        log("superquadric-union leg ...")
        line["superquadrics"] = sq_leg(Context, steps=min(args.steps, 5))
    if not args.no_cpu_baseline and not args.only:
        log("timing the FP64 oracle on the host ...")
        line["cpu_baseline"] = cpu_baseline(batch, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
