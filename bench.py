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
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X published HBM3E bandwidth
Q_READ_BYTES = 24  # traversal reads origin + direction of a queued ray (6 x 32-bit streams)
HIT_BYTES = 28  # one hit record: 7 x 32-bit streams
NODE_BYTES = 64
TRI_BYTES = 48

CONFIGS = {
    "c1": dict(n=128, porosity=0.6, ell=2.0, seed=1, energies=[50.0, 100.0, 250.0, 500.0, 1000.0],
               thetas=[0.0, 20.0, 40.0, 60.0, 80.0], primaries=10_000_000, max_gen=6, rng=2,
               name="128^3 GRF foam, porosity 0.6; 5 E x 5 theta points; 1e7 primaries/point; max_gen 6"),
    "c0": dict(n=16, porosity=0.5, ell=2.0, seed=0, energies=[500.0], thetas=[0.0], primaries=10_000, max_gen=6,
               rng=1, name="16^3 GRF foam, porosity 0.5; 500 eV normal incidence; 1e4 primaries; max_gen 6"),
    "c3": dict(n=256, porosity=0.8, ell=2.0, seed=4, energies=[250.0], thetas=[-80.0], primaries=100_000_000,
               max_gen=10, rng=4,
               name="256^3 GRF foam, porosity 0.8; 250 eV, theta uniform in [0, 80]; 1e8 primaries; max_gen 10"),
}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in ("trace.hip", "rtmc_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1806_00205_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


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

    def step():
        res = []
        for k, (E, th) in enumerate(points):
            res.append(ctx.trace(sid, tid, E, th, npp, seed=cfg["rng"] * 1000 + k, max_gen=cfg["max_gen"]))
        return res

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
            tot["kms"] += r["kernel_ms"]
            tot["sms"] += r["shade_ms"]
            tot["launches"] += r["n_kernel_launches"]
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
                   "launch": ctx.get_launch()},
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
            "kernel": "k_traverse",
            "kernel_ms_total": tot["kms"],
            "shade_ms_total": tot["sms"],
            "kernel_launches": tot["launches"],
            "alg_bytes_per_launch": alg_bytes / max(tot["launches"], 1),
            "achievable_copy_gbps": achievable,
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ctx, sid, tid, mesh, tab, cfg, points, npp, prim_s, args.cpu_seconds)
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
    t = time.perf_counter()
    oracle.trace(mesh, tab, E, th, 32, seed=seed, max_gen=cfg["max_gen"], n_threads=cores)
    per = (time.perf_counter() - t) / 32
    n = int(max(64, min(npp, seconds / max(per, 1e-9))))
    t = time.perf_counter()
    o = oracle.trace(mesh, tab, E, th, n, seed=seed, max_gen=cfg["max_gen"], n_threads=cores, per_primary=True)
    dt = time.perf_counter() - t
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
        "paired_parity": {"oracle_yield": o["yield"], "gpu_yield": g["yield"],
                          "same_escape_count_frac": float((diff == 0).mean()), "paired_z": float(z)},
    }


if __name__ == "__main__":
    main()
