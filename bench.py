"""Benchmark of the contact-manifold hot path on one MI355X.

A step is one pass of the whole path -- float32 bounding-sphere broadphase,
per-scene compaction, vertex-SDF both ways, all-pairs edge-edge witness
contacts with their indicators, and the SoftSort K-contact manifold -- over
one batch of synthetic scenes already resident in HBM.

Headline (--steps / --warmup apply to it): the differentiation workload,
16,384 scenes x 4 convex polytopes (hulls of 64 unit-sphere points scaled
per axis by U[0.3, 0.6]: 64 V / 186 E / 124 F), all 6 pairs per scene
candidates, tau = 0.01, K = 8, through the fused batched path
(cm_collide_fused).  The same process then times, with the replay counts
given in parentheses (warm-up + timed):

  cfg3_plain_fwd            cm_collide on the headline batch (1 + 3)
  cfg3_fwd_bwd_tau*         cm_collide + cm_collide_backward at tau 0.1, 0.01,
                            0.001 with L = sum_k a_k w_k d_k + b_k . nu_k
                            (cotangents g_dist = a w, g_weight = a d,
                            g_normal = b, seeded standard normals) (1 + 2)
  cfg3_fused_fwd_bwd        the fused forward + the adjoint at tau 0.01 (1 + 2)
  cfg4_fused_fwd, cfg4_plain_fwd, cfg4_fused_fwd_bwd
                            100,000 uneven scenes (geometric pairs per scene,
                            8-256-point hulls, 20 % analytic bodies, 30 %
                            forced penetration, tau 0.01, K 16) (1 + 1, 0 + 1,
                            0 + 1 after the fused forward's warm-up)
  cfg2_*                    65,536 mixed scenes x 8 bodies (tau 0.005, K 8):
                            plain, fused, fwd+bwd, pre-selected (K_V 64, K_E
                            18) plain and fused, no-E-E and one-sided
                            simplifications (1 + 3)
  cfg1_*                    4,096 cube pairs (tau 0.01, K 8), plain and fused
                            (5 + 20; launch-latency bound)
  serving                   a Poisson request stream through cm_server_*
                            (p50 / p99), a sample of served pairs checked
                            against the FP64 oracle
  ee_witness                the E-E witness routine alone, 1 .. 10^7 queries
  superquadrics             superquadric-union and point-cloud bodies
Legs that would push the run past --budget seconds of wall clock are skipped
and listed under "skipped".  The FP64 oracle is timed on the host cores
first, before the GPU is touched (cpu_baseline).

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
TRAFFIC_FILE_CFG3 = os.path.join(ROOT, "profiles", "collide_fwd_polytopes16384_traffic.md")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


def excess_max(gpu, ref, atol=1e-6, rtol=2e-5) -> float:
    """Largest amount by which |gpu - ref| exceeds atol + rtol |ref| (<= 0: within the bar)."""
    g = np.asarray(gpu, np.float64)
    r = np.asarray(ref, np.float64)
    return float((np.abs(g - r) - (atol + rtol * np.abs(r))).max()) if g.size else 0.0


_CPU_JOB = {}


def _oracle_worker(w: int):
    """Forked worker of the CPU baseline: one intra-op thread, pairs w, w + n,
    w + 2n, ... of the sample until its time budget is spent.  Geometry
    (hull) construction is done before timing each pair."""
    import torch
    from oracle import cm_oracle as O
    torch.set_num_threads(1)
    job = _CPU_JOB
    b, pairs, n, budget = job["batch"], job["pairs"], job["n"], job["budget"]
    cache = O.GeomCache(b.geoms)
    spent, done = 0.0, 0
    t_start = time.perf_counter()
    with torch.no_grad():
        for i in range(w, pairs.shape[1], n):
            a, c = int(pairs[0, i]), int(pairs[1, i])
            GA, GB = cache[b.body_geom[a]], cache[b.body_geom[c]]
            t0 = time.perf_counter()
            O.collide_pair(GA, b.pose[:, a], GB, b.pose[:, c], b.tau, b.K)
            spent += time.perf_counter() - t0
            done += 1
            if time.perf_counter() - t_start > budget:
                break
    return done, spent


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, budget_s: float, max_workers: int = 16):
    """The FP64 oracle on the host, before any GPU call (so the pool's forked
    workers start from a process that has not touched the GPU).  Kept pairs of
    the batch in scene order; one process per core of this process's CPU
    affinity (at most max_workers, the host share of one GPU), each with one
    intra-op thread, for about 2/3 of the budget; then one process with one
    thread for the rest (the 1-thread figure)."""
    import multiprocessing as mp
    from oracle import cm_oracle as O
    pairs, _ = O.broadphase(batch)
    affinity = len(os.sched_getaffinity(0))
    workers = max(1, min(affinity, max_workers))
    _CPU_JOB.update(batch=batch, pairs=pairs, n=workers, budget=budget_s * 2 / 3)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_worker, range(workers))
    wall = time.perf_counter() - t0
    done = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    _CPU_JOB.update(n=1, budget=budget_s / 3)
    d1, s1 = _oracle_worker(0)
    return dict(value=done / busy, unit="pairs/s", cores=workers, kind="oracle",
                sample=f"{done} kept pairs of the headline workload (scene order, strided over {workers} "
                       f"processes x 1 thread), FP64 oracle, {busy:.1f} s of pair evaluation per process "
                       f"({wall:.1f} s wall incl. hull builds); value = pairs / busiest process's evaluation time",
                cpu_model=cpu_model(), affinity_cores=affinity, one_thread_pairs_per_s=d1 / s1,
                one_thread_sample=f"{d1} pairs, {s1:.1f} s")


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
    kept_results = {}

    def run(items, arrivals, keep=0):
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
                        i = tickets.index(t)
                        if i < keep:
                            kept_results[i] = r
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
    done, wall = run(payload[n_cal:], arrivals, keep=4)
    srv.close()
    # FP64 oracle on a seeded sample of served pairs (4 per request, first 4 requests of the stream)
    from oracle import cm_oracle as O
    cache = O.GeomCache(pool)
    worst, checked = -float("inf"), 0
    srng = np.random.default_rng(seed + 2)
    for i, r in sorted(kept_results.items()):
        q = payload[n_cal + i][0]
        m = min(r["n_pairs"], r["capacity"])
        for j in srng.choice(m, size=min(4, m), replace=False):
            a_, b_ = int(r["pairs"][0, j]), int(r["pairs"][1, j])
            with __import__("torch").no_grad():
                ref = O.collide_pair(cache[q.body_geom[a_]], q.pose[:, a_], cache[q.body_geom[b_]], q.pose[:, b_], tau, K)
            for k in ("p", "nu", "d", "w"):
                worst = max(worst, excess_max(r[k][j], ref[k].numpy()))
            checked += 1
    burst_pairs = sum(d[3] for d in cal.values()) / cal_wall
    plain_pairs = run_plain(payload[:n_cal])
    lat = np.array([d[2] - d[0] for d in done.values()])
    pairs = sum(d[3] for d in done.values())
    return dict(requests=len(done), rate_per_s=rate, saturated_per_s=sat, burst_pairs_per_s=burst_pairs,
                plain_sequential_pairs_per_s=plain_pairs, p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), pairs_per_s=pairs / wall, wall_s=wall,
                oracle_check={"pairs": checked, "max_excess": worst if checked else None,
                              "bar": "|gpu - fp64| <= 1e-6 + 2e-5 |fp64| (max_excess <= 0 passes)"},
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


class Timer:
    """HIP-event timing of `steps` calls of fn on the current stream, with
    the library's per-kernel event timers enabled over the timed region."""

    def __init__(self, ctx, stream):
        self.ctx, self.stream = ctx, stream

    def run(self, fn, warmup: int, steps: int) -> dict:
        import torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        self.ctx.check_errors()
        self.ctx.set_kernel_timing(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(self.stream)
        for _ in range(steps):
            fn()
        ev1.record(self.stream)
        torch.cuda.synchronize()
        out = {"ms": ev0.elapsed_time(ev1) / steps, "steps": steps, "warmup": warmup}
        for t in ("broadphase", "forward", "backward", "fused"):
            ms, n = self.ctx.kernel_time(t)
            if n:
                out[f"{t}_kernel_ms"] = ms / n
                out[f"{t}_launches"] = n
        self.ctx.set_kernel_timing(False)
        self.ctx.check_errors()
        return out


def config_ops(ctx, ids, batch, out):
    """Algorithmic (fma, alu, trans) of the kept pairs of `out` (op model)."""
    from paper_2602_20304_amd import opmodel
    kept = min(int(out.n_pairs.item()), out.capacity)
    pairs = out.pairs[:, :kept].cpu().numpy()
    gids = np.unique(ids)
    info = {int(g): ctx.geometry_info(int(g)) for g in gids}
    lut = np.zeros((int(gids.max()) + 1, 4), np.int64)
    for g, i in info.items():
        lut[g] = (i["type"], i["n_vertices"], i["n_edges"], i["n_faces"])
    body_geom = ids[batch.body_geom]
    return opmodel.batch_ops(lut[:, 0], lut[:, 1], lut[:, 2], lut[:, 3], pairs[0], pairs[1], body_geom)


def _geometry_lut(ctx, ids):
    gids = np.unique(ids)
    lut = np.zeros((int(gids.max()) + 1, 4), np.int64)
    for g in gids:
        i = ctx.geometry_info(int(g))
        lut[int(g)] = (i["type"], i["n_vertices"], i["n_edges"], i["n_faces"])
    return lut


def tape_windows(out, nvA, nvB):
    """Per kept pair of `out`: the adjoint-window candidates among A's
    vertices, B's vertices and the edge-edge witnesses, read from the tape
    the forward recorded (layout in include/cm.h).  A pair whose window was
    not recorded counts as all edge-edge."""
    K, cap = out.K, out.capacity
    n = min(int(out.n_pairs.item()), cap)
    stride = 16 + 80 * K
    hdr = (cap * stride + 255) // 256 * 256
    t = out.tape
    used = int(t[:8].cpu().numpy().view(np.uint64)[0])
    recs = t[256:256 + n * stride].cpu().numpy().reshape(n, stride)
    count = recs[:, 0:4].copy().view(np.int32)[:, 0].astype(np.int64)
    form = recs[:, 4:8].copy().view(np.int32)[:, 0]
    off = recs[:, 8:16].copy().view(np.int64)[:, 0]
    pool_n = min(used, (t.numel() - 256 - hdr) // 4)
    pool = t[256 + hdr:256 + hdr + 4 * pool_n].cpu().numpy().view(np.int32)
    nvs = nvA + nvB
    w_a = np.zeros(n, np.int64)
    w_b = np.zeros(n, np.int64)
    w_e = np.where(form == 0, count, 0)
    lp = np.nonzero(form == 1)[0]
    if lp.size:
        lens = count[lp]
        first = np.repeat(off[lp] - np.concatenate(([0], np.cumsum(lens)[:-1])), lens)
        vals = pool[first + np.arange(int(lens.sum()))]
        owner = np.repeat(lp, lens)
        in_a = vals < nvA[owner]
        in_b = ~in_a & (vals < nvs[owner])
        w_a += np.bincount(owner, weights=in_a, minlength=n).astype(np.int64)
        w_b += np.bincount(owner, weights=in_b, minlength=n).astype(np.int64)
        w_e += np.bincount(owner, weights=~(in_a | in_b), minlength=n).astype(np.int64)
    for p in np.nonzero(form == 2)[0]:
        words = (int(nvs[p]) + 63) // 64   # the mask words covering the vertex candidates
        bits = np.unpackbits(pool[off[p]:off[p] + 2 * words].view(np.uint8), bitorder="little")
        a_, b_ = int(nvA[p]), int(nvs[p])
        w_a[p] = int(bits[:a_].sum())
        w_b[p] = int(bits[a_:b_].sum())
        w_e[p] = int(count[p]) - w_a[p] - w_b[p]
    return w_a, w_b, w_e


def adjoint_ops(ctx, ids, batch, out):
    """Algorithmic (fma, alu, trans) of the adjoint launch on `out`'s kept
    pairs, from the op model and each pair's recorded adjoint window."""
    from paper_2602_20304_amd import opmodel
    kept = min(int(out.n_pairs.item()), out.capacity)
    pairs = out.pairs[:, :kept].cpu().numpy()
    lut = _geometry_lut(ctx, ids)
    body_geom = ids[batch.body_geom]
    ga, gb = body_geom[pairs[0]], body_geom[pairs[1]]
    w_a, w_b, w_e = tape_windows(out, lut[ga, 1], lut[gb, 1])
    ops = opmodel.adjoint_batch_ops(lut[:, 0], lut[:, 1], lut[:, 2], lut[:, 3], pairs[0], pairs[1], body_geom,
                                    w_a, w_b, w_e)
    return ops, dict(window_candidates_per_pair=float((w_a + w_b + w_e).mean()) if kept else 0.0,
                     vertex_sdf_share=float((w_a + w_b).sum() / max((w_a + w_b + w_e).sum(), 1)))


ADJOINT_NOTE = ("algorithmic ops = the adjoint's method on each pair's recorded window (candidates within 18 tau "
                "of s_[K]): the window candidates evaluated again and swept in reverse, the distance pass and "
                "nearest-neighbour LSE terms of every edge pair recomputed, the LSE terms swept in reverse "
                "(opmodel.adjoint_batch_ops); duration = the adjoint launch")


def roofline_entry(ops, kernel_ms, kernel, launches, traffic=None, note=None):
    from paper_2602_20304_amd import opmodel
    r = opmodel.roofline(ops, kernel_ms * 1e-3)
    e = {"bound": "alu", "kernel": kernel, "achieved": r["achieved_flops"] / 1e12, "peak": r["peak_flops"] / 1e12,
         "unit": "TFLOP/s", "frac": r["frac"], "traffic": traffic, "kernel_ms": kernel_ms, "launches": launches,
         "ops_per_launch": {"fma": int(ops[0]), "alu": int(ops[1]), "trans": int(ops[2])}}
    if note:
        e["note"] = note
    return e


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--budget", type=float, default=480.0,
                    help="wall-clock seconds after which remaining legs are skipped")
    ap.add_argument("--cpu-budget", type=float, default=18.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--configs", default="3,4,2,1,5,ee,sq",
                    help="comma list of legs to run after the headline: 3 4 2 1 5(serving) ee sq")
    ap.add_argument("--scenes", type=int, default=None, help="override the headline's scene count (testing)")
    ap.add_argument("--cfg4-scenes", type=int, default=100_000)
    ap.add_argument("--serve", type=int, default=24, help="requests in the serving leg")
    ap.add_argument("--ee-trials", type=int, default=20, help="timed launches per size in the E-E sweep")
    ap.add_argument("--only", default=None,
                    choices=[None, "cfg3_fused", "cfg3_plain", "cfg3_bwd", "cfg4_fused", "cfg4_plain", "cfg4_bwd", "cfg2_plain",
                             "cfg2_fused", "cfg2_bwd", "cfg2_refine", "cfg2_all", "ee", "sq"],
                    help="run one leg only, without the headline and the other legs (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of this many MiB (PMC byte calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on exactly one GPU; --gpus must be 1"}), flush=True)
        raise SystemExit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration << 20, 5)
        return
    t_start = time.perf_counter()
    elapsed = lambda: time.perf_counter() - t_start
    wanted = set(args.configs.split(",")) if args.configs else set()

    import workloads as W
    b3 = W.polytope_scenes(args.scenes or 16384, seed=0, tau=0.01)
    desc3 = (f"polytope_scenes (differentiation workload): {b3.n_scenes} scenes x 4 convex polytopes (hull of 64 "
             f"unit-sphere points scaled per axis U[0.3,0.6]: 64 V / 186 E / 124 F), all 6 pairs/scene candidates, "
             f"centres U[-0.5,0.5]^3, tau={b3.tau:g}, K={b3.K}")
    cpu = None
    if not args.no_cpu_baseline and not args.only:
        log("timing the FP64 oracle on the host cores (before any GPU call) ...")
        cpu = cpu_baseline(b3, args.cpu_budget)
        log(f"cpu baseline: {cpu['value']:.3g} pairs/s on {cpu['cores']} processes ({cpu['cpu_model']}), "
            f"1 thread {cpu['one_thread_pairs_per_s']:.3g} pairs/s")

    import torch
    from paper_2602_20304_amd.cm import FLAG_NO_EE, FLAG_ONE_SIDED_VS, Context, Manifold
    from paper_2602_20304_amd import opmodel

    # one context per workload: a plain launch sizes its LDS and face masks by
    # the largest geometry its context holds
    ctx = Context(0)
    stream = torch.cuda.current_stream()
    timer = Timer(ctx, stream)
    legs, skipped, rooflines = {}, {}, {}

    def new_context():
        nonlocal ctx
        ctx.close()
        torch.cuda.empty_cache()
        ctx = Context(0)
        timer.ctx = ctx

    def fits(name, est_s):
        if elapsed() + est_s > args.budget:
            skipped[name] = f"estimated {est_s:.0f} s would pass the {args.budget:.0f} s budget at {elapsed():.0f} s"
            log(f"skip {name}: {skipped[name]}")
            return False
        return True

    def record(name, res, kept, cand):
        res = dict(res)
        res["kept_pairs"] = kept
        res["candidate_pairs"] = cand
        res["pairs_per_s"] = kept / (res["ms"] * 1e-3)
        res["ms_per_step"] = res.pop("ms")
        legs[name] = res
        log(f"{name}: {res['ms_per_step']:.3f} ms/step, {kept} kept pairs, {res['pairs_per_s']:.4g} pairs/s"
            + "".join(f", {k} {v:.3f}" for k, v in res.items() if k.endswith("_kernel_ms")))
        return res

    def upload(batch):
        t0 = time.perf_counter()
        ids = ctx.create_geometry(batch.geoms)
        db = ctx.upload_batch(batch, ids)
        cap = db.n_cand_total
        out = Manifold.empty(db.n_scenes, cap, batch.K, ctx.device)
        log(f"{batch.name}: {batch.n_scenes} scenes, {batch.n_bodies} bodies, {cap} candidate pairs, "
            f"geometry build + upload {time.perf_counter() - t0:.1f} s")
        return ids, db, cap, out

    def loss_cotangents(cap, K, seed):
        """a [cap K], b [3, cap K] seeded standard normals (float32)."""
        a, b = W.cotangents(cap, K, seed=seed)
        return torch.as_tensor(a).to(ctx.device), torch.as_tensor(b).to(ctx.device)

    def fwd_bwd(db, out, tau, K, a, b, fused=False, presel=None):
        ctx.collide(db, tau, K, out=out, fused=fused, stream=stream, presel=presel, record=True)
        # L = sum_k a_k w_k d_k + b_k . nu_k
        gd = a * out.weight
        gw = a * out.dist
        ctx.collide_backward(db, out, tau, K, None, b, gd, gw, stream=stream, presel=presel,
                             want_vertices=True, want_params=True)

    only = args.only
    # ------------------------------------------------------------ headline: cfg 3 fused forward
    ids3, db3, cap3, out3 = upload(b3)
    ops3 = None
    if only in (None, "cfg3_fused"):
        res = timer.run(lambda: ctx.collide(db3, b3.tau, b3.K, out=out3, fused=True, stream=stream),
                        args.warmup, args.steps)
        head = record("cfg3_fused_fwd", res, int(out3.n_pairs.item()), cap3)
        head["tuning"] = ctx.fused_tuning()
        ops3 = config_ops(ctx, ids3, b3, out3)
        rooflines["cfg3_fused_fwd"] = roofline_entry(
            ops3, res["fused_kernel_ms"], "collide_fwd (fused class kernel)", res["fused_launches"],
            stored_traffic(TRAFFIC_FILE_CFG3, FWD_SOURCES),
            "duration = the whole replayed graph (broadphase, pricing, sort, class launches) between HIP events "
            "on the launch stream: an upper bound of the class kernel's, so a lower bound of its rate")
    if only in (None, "cfg3_plain") and ("3" in wanted or only):
        res = timer.run(lambda: ctx.collide(db3, b3.tau, b3.K, out=out3, stream=stream), 1, 3)
        record("cfg3_plain_fwd", res, int(out3.n_pairs.item()), cap3)
        ops3 = ops3 if ops3 is not None else config_ops(ctx, ids3, b3, out3)
        rooflines["cfg3_plain_fwd"] = roofline_entry(ops3, res["forward_kernel_ms"], "collide_fwd (plain)",
                                                     res["forward_launches"])
    if only in (None, "cfg3_bwd") and ("3" in wanted or only):
        a3, bb3 = loss_cotangents(cap3, b3.K, seed=1)
        for tau in (0.01, 0.001, 0.1):
            name = f"cfg3_fwd_bwd_tau{tau:g}"
            # at tau 0.1 nearly every candidate lies inside the adjoint's
            # window: one timed pass, no warm-up (the kernels are loaded)
            wu, st = (0, 1) if tau > 0.05 else (1, 2)
            if not fits(name, 40.0 if tau > 0.05 else 15.0):
                continue
            res = timer.run(lambda: fwd_bwd(db3, out3, tau, b3.K, a3, bb3), wu, st)
            r = record(name, res, int(out3.n_pairs.item()), cap3)
            if tau == 0.01:
                ops, win = adjoint_ops(ctx, ids3, b3, out3)
                rooflines["cfg3_adjoint"] = roofline_entry(ops, r["backward_kernel_ms"], "collide_bwd",
                                                           r["backward_launches"], note=ADJOINT_NOTE)
                rooflines["cfg3_adjoint"].update(win)
        if not only and fits("cfg3_fused_fwd_bwd", 15.0):
            res = timer.run(lambda: fwd_bwd(db3, out3, b3.tau, b3.K, a3, bb3, fused=True), 1, 2)
            record("cfg3_fused_fwd_bwd", res, int(out3.n_pairs.item()), cap3)
        del a3, bb3
    # restore the headline manifold (tau 0.01) for anything that reads it
    # ------------------------------------------------------------ cfg 4 uneven batching
    if (only in ("cfg4_fused", "cfg4_plain", "cfg4_bwd")) or (only is None and "4" in wanted and fits("cfg4", 150.0)):
        del db3, out3
        new_context()
        t0 = time.perf_counter()
        b4 = W.uneven_scenes(args.cfg4_scenes, seed=0)
        log(f"cfg4 generated in {time.perf_counter() - t0:.1f} s")
        ids4, db4, cap4, out4 = upload(b4)
        est = max(30.0, 1e-4 * cap4)
        if only in (None, "cfg4_fused"):
            res = timer.run(lambda: ctx.collide(db4, b4.tau, b4.K, out=out4, fused=True, stream=stream), 1, 1)
            r = record("cfg4_fused_fwd", res, int(out4.n_pairs.item()), cap4)
            r["tuning"] = ctx.fused_tuning()
            est = r["ms_per_step"] * 1e-3
            ops4 = config_ops(ctx, ids4, b4, out4)
            rooflines["cfg4_fused_fwd"] = roofline_entry(ops4, r["fused_kernel_ms"], "collide_fwd (fused graph)",
                                                         r["fused_launches"])
        if only in (None, "cfg4_plain") and (only or fits("cfg4_plain_fwd", 1.5 * est)):
            res = timer.run(lambda: ctx.collide(db4, b4.tau, b4.K, out=out4, stream=stream), 0, 1)
            r = record("cfg4_plain_fwd", res, int(out4.n_pairs.item()), cap4)
            ops4 = config_ops(ctx, ids4, b4, out4)
            rooflines["cfg4_plain_fwd"] = roofline_entry(ops4, r["forward_kernel_ms"], "collide_fwd (plain)",
                                                         r["forward_launches"])
        if only == "cfg4_bwd" or (only is None and fits("cfg4_fused_fwd_bwd", 4.0 * est)):
            a4, bb4 = loss_cotangents(cap4, b4.K, seed=4)
            res = timer.run(lambda: fwd_bwd(db4, out4, b4.tau, b4.K, a4, bb4, fused=True), 0, 1)
            r = record("cfg4_fused_fwd_bwd", res, int(out4.n_pairs.item()), cap4)
            ops4, win = adjoint_ops(ctx, ids4, b4, out4)
            rooflines["cfg4_adjoint"] = roofline_entry(ops4, r["backward_kernel_ms"], "collide_bwd",
                                                       r["backward_launches"], note=ADJOINT_NOTE)
            rooflines["cfg4_adjoint"].update(win)
            del a4, bb4
        legs_cfg4 = dict(workload=f"uneven_scenes: {b4.n_scenes} scenes, geometric pairs/scene (mean 12, clip "
                                  f"[1,64]), polytopes of 8-256 points on random ellipsoids, 20% analytic, 30% forced "
                                  f"penetration U[0,0.05], tau={b4.tau:g}, K={b4.K}", bodies=b4.n_bodies)
        legs["cfg4_config"] = legs_cfg4
        del db4, out4, b4
        torch.cuda.empty_cache()
    # ------------------------------------------------------------ cfg 5 serving
    serving = ee = sq = None
    if only is None and "5" in wanted and fits("serving", 40.0):
        log(f"serving leg: {args.serve} requests ...")
        serving = serving_leg(Context, args.serve)
        log(f"serving: {serving['rate_per_s']:.2f} req/s (saturated {serving['saturated_per_s']:.2f}), "
            f"p50 {serving['p50_ms']:.1f} ms, p99 {serving['p99_ms']:.1f} ms, oracle sample max excess "
            f"{serving['oracle_check']['max_excess']}")
    # ------------------------------------------------------------ cfg 2 mixed scenes
    if (only and only.startswith("cfg2")) or (only is None and "2" in wanted and fits("cfg2", 40.0)):
        new_context()
        b2 = W.mixed_scenes(65536, seed=0)
        ids2, db2, cap2, out2 = upload(b2)
        a2, bb2 = loss_cotangents(cap2, b2.K, seed=1)
        cfg2 = {"cfg2_plain_fwd": dict(), "cfg2_fused_fwd": dict(fused=True),
                "cfg2_plain_presel_fwd": dict(presel=(64, 18)), "cfg2_fused_presel_fwd": dict(fused=True, presel=(64, 18)),
                "cfg2_plain_ne_fwd": dict(flags=FLAG_NO_EE),
                "cfg2_plain_ne_s_fwd": dict(flags=FLAG_NO_EE | FLAG_ONE_SIDED_VS),
                "cfg2_plain_refine_fwd": dict(refine=3)}
        pick = {"cfg2_plain": ["cfg2_plain_fwd"], "cfg2_fused": ["cfg2_fused_fwd"], "cfg2_bwd": [],
                "cfg2_refine": ["cfg2_plain_refine_fwd"], "cfg2_all": list(cfg2)}
        names = pick[only] if only else [n for n in cfg2 if n != "cfg2_plain_refine_fwd"]
        for name in names:
            kw = cfg2[name]
            if not only and not fits(name, 3.0):
                continue
            res = timer.run(lambda: ctx.collide(db2, b2.tau, b2.K, out=out2, stream=stream, **kw), 1, 3)
            r = record(name, res, int(out2.n_pairs.item()), cap2)
            if name == "cfg2_plain_fwd":
                ops2 = config_ops(ctx, ids2, b2, out2)
                rooflines["cfg2_plain_fwd"] = roofline_entry(ops2, r["forward_kernel_ms"], "collide_fwd (plain)",
                                                             r["forward_launches"], stored_traffic(TRAFFIC_FILE, FWD_SOURCES))
            if name == "cfg2_fused_fwd":
                r["tuning"] = ctx.fused_tuning()
                ops2 = config_ops(ctx, ids2, b2, out2)
                rooflines["cfg2_fused_fwd"] = roofline_entry(ops2, r["fused_kernel_ms"], "collide_fwd (fused graph)",
                                                             r["fused_launches"])
        if only in (None, "cfg2_bwd") and (only or fits("cfg2_fwd_bwd", 8.0)):
            for name, presel in (("cfg2_fwd_bwd", None), ("cfg2_fwd_bwd_presel", (64, 18))):
                res = timer.run(lambda: fwd_bwd(db2, out2, b2.tau, b2.K, a2, bb2, presel=presel), 1, 2)
                r = record(name, res, int(out2.n_pairs.item()), cap2)
                if presel is None:
                    ops2, win = adjoint_ops(ctx, ids2, b2, out2)
                    rooflines["cfg2_adjoint"] = roofline_entry(ops2, r["backward_kernel_ms"], "collide_bwd",
                                                               r["backward_launches"], note=ADJOINT_NOTE)
                    rooflines["cfg2_adjoint"].update(win)
        del db2, out2, a2, bb2
        torch.cuda.empty_cache()
    # ------------------------------------------------------------ cfg 1 cube pairs
    if only is None and "1" in wanted and fits("cfg1", 5.0):
        new_context()
        b1 = W.cube_pairs(4096, seed=0)
        ids1, db1, cap1, out1 = upload(b1)
        for name, fused in (("cfg1_plain_fwd", False), ("cfg1_fused_fwd", True)):
            res = timer.run(lambda: ctx.collide(db1, b1.tau, b1.K, out=out1, fused=fused, stream=stream), 5, 20)
            record(name, res, int(out1.n_pairs.item()), cap1)
    # ------------------------------------------------------------ serving, E-E, extended primitives
    if only == "ee" or (only is None and "ee" in wanted and fits("ee_witness", 15.0)):
        log("E-E witness microbenchmark ...")
        ee = ee_witness_leg(ctx, trials=args.ee_trials)
    if only == "sq" or (only is None and "sq" in wanted and fits("superquadrics", 10.0)):
        log("superquadric-union leg ...")
        sq = sq_leg(Context, steps=3)

    if only:
        print(json.dumps({"only": only, "legs": legs, "rooflines": rooflines, "ee_witness": ee, "superquadrics": sq}),
              flush=True)
        return
    line = {
        "metric": METRIC,
        "value": head["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": desc3, "scenes": b3.n_scenes, "candidate_pairs": cap3,
                   "kept_pairs": head["kept_pairs"], "tau": b3.tau, "K": b3.K, "path": "fused",
                   "parallelism": "single-gpu"},
        "roofline": rooflines.get("cfg3_fused_fwd"),
        "rooflines": rooflines,
        "legs": legs,
    }
    if "cfg3_plain_fwd" in legs:
        line["speedup_vs_plain"] = legs["cfg3_plain_fwd"]["ms_per_step"] / head["ms_per_step"]
    if "cfg3_fwd_bwd_tau0.01" in legs:
        line["fwd_bwd_pairs_per_s"] = legs["cfg3_fwd_bwd_tau0.01"]["pairs_per_s"]
    if "cfg4_fused_fwd" in legs and "cfg4_plain_fwd" in legs:
        line["cfg4_fused_speedup_vs_plain"] = legs["cfg4_plain_fwd"]["ms_per_step"] / legs["cfg4_fused_fwd"]["ms_per_step"]
    if serving:
        line["serving"] = serving
    if ee:
        line["ee_witness"] = ee
    if sq:
        line["superquadrics"] = sq
    if cpu:
        line["cpu_baseline"] = cpu
    line["skipped"] = skipped
    line["wall_s"] = elapsed()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
