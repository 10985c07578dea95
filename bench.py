"""Benchmark of the contact-manifold hot path on one MI355X.

A step is one pass of the whole path -- float32 bounding-sphere broadphase,
per-scene compaction, vertex-SDF both ways, all-pairs edge-edge witness
contacts with their indicators, and the SoftSort K-contact manifold -- over
one batch of synthetic scenes already resident in HBM.

Default workload: 65,536 scenes x 8 bodies (2 spheres, 2 capsules, 2 rounded
boxes, 2 convex polytopes of 32 points), all 28 pairs per scene are
candidates, tau = 0.005, K = 8.

Prints ONE JSON line (see the repository's measurement notes for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


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


def cpu_baseline(batch, budget_s: float):
    """Time the FP64 oracle on the host for a bounded prefix of the scenes."""
    import torch
    import workloads as W
    from oracle import cm_oracle as O
    pairs, _ = O.broadphase(batch)
    cache = O.GeomCache(batch.geoms)
    t0 = time.perf_counter()
    done = 0
    with torch.no_grad():
        for i in range(pairs.shape[1]):
            a, b = int(pairs[0, i]), int(pairs[1, i])
            O.collide_pair(cache[batch.body_geom[a]], batch.pose[:, a], cache[batch.body_geom[b]], batch.pose[:, b],
                           batch.tau, batch.K)
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="pairs/s", cores=int(torch.get_num_threads()), kind="oracle",
                sample=f"first {done} kept pairs of the same workload in pair order ({dt:.1f} s, FP64 oracle, "
                       f"geometry build excluded)")


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        raise SystemExit(2)

    import torch
    from paper_2602_20304_amd.cm import Context, Manifold
    from paper_2602_20304_amd import opmodel

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

    def step(path):
        ctx.collide(db, batch.tau, batch.K, out=out, fused=(path == "fused"), stream=stream)

    results = {}
    for path in ("plain", "fused"):
        for _ in range(args.warmup):
            step(path)
        torch.cuda.synchronize()
        ctx.check_errors()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            step(path)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / args.steps
        n_pairs = int(out.n_pairs.item())
        results[path] = dict(ms=ms, n_pairs=n_pairs)
        log(f"{path}: {ms:.3f} ms/step, {n_pairs} kept pairs, {n_pairs / (ms * 1e-3):.4g} pairs/s")
    ctx.check_errors()

    main_path = args.path
    ms = results[main_path]["ms"]
    n_pairs = results[main_path]["n_pairs"]
    pairs = out.pairs[:, :n_pairs].cpu().numpy()
    G = ctx.geometry_count
    sizes = np.array([[ctx.geometry_info(int(g))[k] for k in ("type", "n_vertices", "n_edges", "n_faces")]
                      for g in range(G)], dtype=np.int64)
    body_geom = ids[batch.body_geom]
    ops = opmodel.batch_ops(sizes[:, 0], sizes[:, 1], sizes[:, 2], sizes[:, 3], pairs[0], pairs[1], body_geom)
    roof = opmodel.roofline(ops, ms * 1e-3)
    line = {
        "metric": "geom-pair contact evals/s (fwd)",
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
                   "tau": batch.tau, "K": batch.K, "path": main_path, "parallelism": "single-gpu"},
        "paths": {k: {"ms_per_step": v["ms"], "pairs_per_s": v["n_pairs"] / (v["ms"] * 1e-3)}
                  for k, v in results.items()},
        "roofline": {"bound": "alu", "achieved": roof["achieved_flops"] / 1e12, "peak": roof["peak_flops"] / 1e12,
                     "unit": "TFLOP/s", "frac": roof["frac"], "traffic": None,
                     "ops_per_step": {"fma": int(ops[0]), "alu": int(ops[1]), "trans": int(ops[2])}},
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on the host ...")
        line["cpu_baseline"] = cpu_baseline(batch, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
