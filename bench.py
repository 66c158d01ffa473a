"""Benchmark of the RTMC hot path on one MI355X.

One step is one pass of the whole hot path over one batch of synthetic input:
the realistic single-foam workload (128^3 Gaussian-random-field foam at
porosity 0.6, about 1.9M FP32 triangles, BVH built on the device) swept over
E in {50, 100, 250, 500, 1000} eV x theta in {0, 20, 40, 60, 80} deg with
1e7 primaries per point and cascades up to generation 6.  Every primary and
secondary ray is traced, shaded, queued and tallied inside the timed region;
inputs are resident in HBM before it starts.

Prints one JSON line.  The FP64 oracle is timed beside it on a bounded
sample of the same workload (the same primary ids, so the sample is also a
paired parity check).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X published HBM3E bandwidth
Q_READ_BYTES = 24  # traversal reads origin + direction of a queued ray (6 x 32-bit streams)
HIT_BYTES = 28  # one hit record: 7 x 32-bit streams
NODE_BYTES = 64
# LBVH build per triangle: Morton codes (48 read + 12 written), 8 radix passes
# (8 + 24 bytes each), triangle gather (4 + 48 read, 48 sorted + 64 rotated
# written), hierarchy (24 key reads + 16 link writes), bottom-up bounds (48
# triangle read + 64 node write + 12), 4-wide collapse (64 read + 64 written)
# and the breadth-first copy of the reached half (32 read + 32 written)
BUILD_BYTES_PER_TRI = 60 + 8 * 32 + 164 + 40 + 124 + 128 + 64
# one triangle test reads the three vertices in the ray's axis order (3 x 12 B)
# and the caller's index (4 B) from the triangle's rotated 64-byte record
TRI_BYTES = 40
SWEEP_CHUNK = 1 << 28  # primaries per chunk of the batched sweep

CONFIGS = {
    "c1": dict(n=128, porosity=0.6, ell=2.0, seed=1, energies=[50.0, 100.0, 250.0, 500.0, 1000.0],
               thetas=[0.0, 20.0, 40.0, 60.0, 80.0], primaries=10_000_000, max_gen=6, rng=2,
               name="128^3 GRF foam, porosity 0.6; 5 E x 5 theta points; 1e7 primaries/point; max_gen 6"),
    "c0": dict(n=16, porosity=0.5, ell=2.0, seed=0, energies=[500.0], thetas=[0.0], primaries=10_000, max_gen=6,
               rng=1, name="16^3 GRF foam, porosity 0.5; 500 eV normal incidence; 1e4 primaries; max_gen 6"),
    "c3": dict(n=256, porosity=0.8, ell=2.0, seed=4, energies=[250.0], thetas=[-80.0], primaries=100_000_000,
               max_gen=10, rng=4,
               name="256^3 GRF foam, porosity 0.8; 250 eV, theta uniform in [0, 80]; 1e8 primaries; max_gen 10"),
    "c2": dict(n_foams=64, sizes=[64, 96, 128, 192], energies=[50.0, 100.0, 250.0, 500.0, 1000.0],
               thetas=[0.0, 20.0, 40.0, 60.0, 80.0], primaries=1_000_000, max_gen=6, rng=3,
               name="64 GRF foams, porosity ~U[0.2,0.8], grids from {64,96,128,192}^3; 25 points each; "
                    "1e6 primaries/point; one HIP graph"),
}


def source_hash(texts) -> str:
    """sha256 (first 16 hex digits) of C++ sources with comments and blank
    space removed, so that edits to comments keep a counter summary current."""
    h = hashlib.sha256()
    for t in texts:
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(" ".join(t.split()).encode())
    return h.hexdigest()[:16]


def kernel_hash() -> str:
    """Hash of the traversal kernel's sources (trace.hip and rtmc_internal.h)."""
    return source_hash(open(os.path.join(ROOT, "paper_1806_00205_amd", "csrc", f)).read()
                       for f in ("trace.hip", "rtmc_internal.h"))


def load_traffic(cfg_name: str):
    """Measured HBM bytes per algorithmic byte from a committed counter summary, if current."""
    path = os.path.join(ROOT, "profiles", f"k_traverse_{cfg_name}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c1", choices=sorted(CONFIGS))
    ap.add_argument("--primaries", type=int, default=0, help="override primaries per point")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU path (shard primary ids, one "
              "all-reduce of the tally block) is a design, not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import foamgen as fg
    import paper_1806_00205_amd as rt

    cfg = CONFIGS[args.config]
    npp = args.primaries or cfg["primaries"]
    if args.config == "c2":
        return bench_batched(args, cfg, npp)
    t0 = time.time()
    mesh = fg.make_grf_foam(cfg["n"], cfg["porosity"], cfg["ell"], seed=cfg["seed"])
    tab = fg.make_tables("vaughan")
    print(f"[bench] mesh {mesh.n_tris} triangles in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    ctx = rt.Context(0)
    sid = ctx.load_scene(mesh)
    tid = ctx.load_tables(tab)
    info = ctx.scene_info(sid)
    print(f"[bench] BVH built on device in {info['build_ms']:.1f} ms, depth {info['bvh_depth']}",
          file=sys.stderr, flush=True)
    points = [(E, th) for E in cfg["energies"] for th in cfg["thetas"]]

    # the points go through the library as one batch: chunks of up to 2^28
    # primaries span several points, so every generation's launch is large
    # (per-point results are those of single traces, integer tallies equal)
    lc = ctx.get_launch()
    ctx.set_launch(lc["block"], lc["wg_per_cu"], lc["lds_stack"], SWEEP_CHUNK, lc["refill"], lc["occupancy"])
    jobs = [(sid, E, th, npp, cfg["rng"] * 1000 + k) for k, (E, th) in enumerate(points)]

    def step():
        return ctx.trace_batch(tid, jobs, max_gen=cfg["max_gen"])

    for w in range(args.warmup):
        step()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tot = dict(prim=0, rays=0, tests=0, visits=0, spawned=0, kms=0.0, sms=0.0, launches=0)
    t_start = time.perf_counter()
    last = None
    for s in range(args.steps):
        last = step()
        for r in last:
            tot["prim"] += r["n_primaries"]
            tot["rays"] += r["n_rays"]
            tot["tests"] += r["n_tri_tests"]
            tot["visits"] += r["n_node_visits"]
            tot["spawned"] += r["n_spawned"]
        # timing and launch counts are the whole batch's, repeated in every job's result
        assert last[0]["kernel_ms"] > 0.0, "batch was replayed as a graph: no per-launch timing"
        tot["kms"] += last[0]["kernel_ms"]
        tot["sms"] += last[0]["shade_ms"]
        tot["launches"] += last[0]["n_kernel_launches"]
        print(f"[bench] step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps
    prim_s = tot["prim"] / wall
    # algorithmic bytes of the traversal kernel: node and triangle fetches,
    # origin + direction reads of queued (secondary) rays, hit-record writes
    alg_bytes = (NODE_BYTES * tot["visits"] + TRI_BYTES * tot["tests"] +
                 Q_READ_BYTES * (tot["rays"] - tot["prim"]) + HIT_BYTES * tot["rays"])
    achieved = alg_bytes / (tot["kms"] * 1e-3) / 1e9 if tot["kms"] > 0 else 0.0
    achievable = ctx.copy_probe(1 << 32, reps=5)
    traffic = load_traffic(args.config)
    out = {
        "metric": "primaries/s + ray-tri tests/s at <=3 sigma yield error vs FP64 oracle",
        "value": prim_s,
        "unit": "primaries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {cfg['name']}", "n_tris": info["n_tris"],
                   "primaries_per_point": npp, "points": len(points), "bvh_depth": info["bvh_depth"],
                   "call": "rtmc_trace_batch over the points", "launch": ctx.get_launch()},
        "tri_tests_per_s": tot["tests"] / wall,
        "rays_per_s": tot["rays"] / wall,
        "node_visits_per_ray": tot["visits"] / max(tot["rays"], 1),
        "tri_tests_per_ray": tot["tests"] / max(tot["rays"], 1),
        "rays_per_primary": tot["rays"] / max(tot["prim"], 1),
        "yields": {f"{E:g}eV_{th:g}deg": round(r["yield"], 5) for (E, th), r in zip(points, last)},
        "max_yield_sigma": max(r["yield_sigma"] for r in last),
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": PEAK_HBM_GBPS,
            "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBPS,
            "traffic": (traffic["fetch_plus_write_bytes_per_alg_byte"] * alg_bytes / max(tot["launches"], 1)
                        if traffic else None),
            # from the same committed counter summary (null once the kernel has changed)
            "valu_issue": traffic.get("valu_issue") if traffic else None,
            "l2_hit": traffic.get("l2_hit") if traffic else None,
            "kernel": "k_traverse",
            "kernel_ms_total": tot["kms"],
            "shade_ms_total": tot["sms"],
            "kernel_launches": tot["launches"],
            "alg_bytes_per_launch": alg_bytes / max(tot["launches"], 1),
            "achievable_copy_gbps": achievable,
        },
    }
    out["bvh_build"] = bench_build(ctx, mesh)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ctx, sid, tid, mesh, tab, cfg, points, npp, prim_s, args.cpu_seconds)
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_build(ctx, mesh, reps: int = 3):
    """Mesh ingest (host arrays -> device) and the device LBVH build of the
    same mesh, after the timed region; the build time is the library's own
    HIP-event figure."""
    ingest, build = [], []
    for _ in range(reps):
        t = time.perf_counter()
        sid = ctx.load_mesh(mesh.verts, mesh.tris, mesh.box_lo, mesh.box_hi, mesh.flags)
        ingest.append((time.perf_counter() - t) * 1e3)
        ctx.build_bvh(sid)
        build.append(ctx.scene_info(sid)["build_ms"])
    b = sorted(build)[reps // 2]
    n = mesh.n_tris
    return {"n_tris": n, "ingest_ms": sorted(ingest)[reps // 2], "build_ms": b, "tris_per_s": n / (b * 1e-3),
            "alg_bytes_per_tri": BUILD_BYTES_PER_TRI,
            "alg_gbps": BUILD_BYTES_PER_TRI * n / (b * 1e-3) / 1e9}


def bench_batched(args, cfg, npp):
    """Many uneven foams x (E, theta) points in one graph, against the same jobs traced one by one."""
    import numpy as np
    import torch

    import foamgen as fg
    import paper_1806_00205_amd as rt

    rng = np.random.default_rng(cfg["rng"])
    tab = fg.make_tables("vaughan")
    ctx = rt.Context(0)
    tid = ctx.load_tables(tab)
    scenes, tris = [], 0
    t0 = time.time()
    for i in range(cfg["n_foams"]):
        n = int(rng.choice(cfg["sizes"]))
        p = float(rng.uniform(0.2, 0.8))
        m = fg.make_grf_foam(n, p, 2.0, seed=1000 + i)
        scenes.append((ctx.load_scene(m), n, p, m.n_tris))
        tris += m.n_tris
        print(f"[bench] foam {i + 1}/{cfg['n_foams']}: {n}^3, porosity {p:.2f}, {m.n_tris} triangles",
              file=sys.stderr, flush=True)
    print(f"[bench] {len(scenes)} foams, {tris} triangles in {time.time() - t0:.0f} s", file=sys.stderr, flush=True)
    mid = sorted(scenes, key=lambda x: x[3])[len(scenes) // 2][0]
    tuned = ctx.autotune(mid, tid, 250.0, 40.0, 2_000_000)
    print(f"[bench] autotuned launch: {tuned}", file=sys.stderr, flush=True)
    jobs = []
    for sid, _, _, _ in scenes:
        for E in cfg["energies"]:
            for th in cfg["thetas"]:
                jobs.append((sid, E, th, npp, int(rng.integers(1, 2 ** 62))))
    total = len(jobs) * npp
    for w in range(args.warmup):
        ctx.trace_batch(tid, jobs, max_gen=cfg["max_gen"])
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s_ in range(args.steps):
        res = ctx.trace_batch(tid, jobs, max_gen=cfg["max_gen"])
        print(f"[bench] step {s_ + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    tests = sum(r["n_tri_tests"] for r in res)
    rays = sum(r["n_rays"] for r in res)
    # the same jobs, one rtmc_trace each (plain single-foam RTMC)
    t1 = time.perf_counter()
    single = [ctx.trace(sid, tid, E, th, n, seed=sd, max_gen=cfg["max_gen"]) for sid, E, th, n, sd in jobs]
    t_single = time.perf_counter() - t1
    same = all(a["n_escaped"] == b["n_escaped"] and a["n_rays"] == b["n_rays"] for a, b in zip(res, single))
    out = {
        "metric": "primaries/s + ray-tri tests/s at <=3 sigma yield error vs FP64 oracle",
        "value": total * args.steps / wall,
        "unit": "primaries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c2: {cfg['name']}", "jobs": len(jobs), "triangles_total": tris,
                   "launch": tuned},
        "tri_tests_per_s": tests * args.steps / wall,
        "rays_per_s": rays * args.steps / wall,
        "single_jobs_primaries_per_s": total / t_single,
        "batched_over_single": (total * args.steps / wall) / (total / t_single),
        "batched_equals_single_integer_tallies": same,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def cpu_baseline(ctx, sid, tid, mesh, tab, cfg, points, npp, gpu_prim_s, seconds):
    """FP64 oracle on the host cores, on primary ids 0..n-1 of the first point."""
    import numpy as np
    import torch

    import oracle

    oracle.build(force=False)
    cores = len(os.sched_getaffinity(0))
    cores = min(cores, 16)
    E, th = points[len(points) // 2]
    seed = cfg["rng"] * 1000 + len(points) // 2
    # pilot on enough primaries to keep every thread busy, then size the sample
    pilot = 16 * cores
    t = time.perf_counter()
    oracle.trace(mesh, tab, E, th, pilot, seed=seed, max_gen=cfg["max_gen"], n_threads=cores)
    per = (time.perf_counter() - t) / pilot
    n = int(max(64, min(npp, seconds / max(per, 1e-9))))
    t = time.perf_counter()
    o = oracle.trace(mesh, tab, E, th, n, seed=seed, max_gen=cfg["max_gen"], n_threads=cores, per_primary=True)
    dt = time.perf_counter() - t
    # one core, on a prefix of the same ids (about a tenth of the time budget)
    n1 = int(max(8, min(n, 0.1 * seconds / max(per * cores, 1e-9))))
    t = time.perf_counter()
    o1 = oracle.trace(mesh, tab, E, th, n1, seed=seed, max_gen=cfg["max_gen"], n_threads=1)
    dt1 = time.perf_counter() - t
    pp = torch.zeros(n, dtype=torch.int32, device="cuda:0")
    g = ctx.trace(sid, tid, E, th, n, seed=seed, max_gen=cfg["max_gen"], per_primary=pp)
    ppg = pp.cpu().numpy().astype(np.int64)
    ppo = o["per_primary"]["escaped"].astype(np.int64)
    diff = ppg - ppo
    sd = diff.std(ddof=1) if n > 1 else 0.0
    z = diff.mean() / (sd / math.sqrt(n)) if sd > 0 else 0.0
    return {
        "value": n / dt,
        "unit": "primaries/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"primary ids 0..{n - 1} at E={E:g} eV, theta={th:g} deg on the same mesh ({dt:.1f} s)",
        "tri_tests_per_s": o["n_tri_tests"] / dt,
        "one_core": {"primaries_per_s": n1 / dt1, "tri_tests_per_s": o1["n_tri_tests"] / dt1,
                     "sample": f"primary ids 0..{n1 - 1} ({dt1:.1f} s)"},
        "paired_parity": {"oracle_yield": o["yield"], "gpu_yield": g["yield"],
                          "same_escape_count_frac": float((diff == 0).mean()), "paired_z": float(z)},
    }


if __name__ == "__main__":
    main()
