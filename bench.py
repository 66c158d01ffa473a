"""Benchmark of the RTMC hot path on one MI355X.

The headline step is one pass of the whole hot path over the large-foam
workload: a 256^3 Gaussian-random-field foam at porosity 0.8 (about 11M FP32
triangles, BVH built on the device, ~1 GB of traversal data, larger than the
256 MB last-level cache), 1e8 primaries of 250 eV at polar angles uniform in
[0, 80] deg, cascades up to generation 10.  Every primary and secondary ray
is traced, shaded, queued and tallied inside the timed region; inputs are
resident in HBM before it starts.

The same JSON line carries, as sub-records:
  c1:        the 128^3 foam (porosity 0.6, 1.9M triangles) swept over
             E in {50, 100, 250, 500, 1000} eV x theta in {0, 20, 40, 60, 80}
             deg with 1e7 primaries per point (one batched call), with the
             first ids of every point paired against the FP64 oracle;
  surrogate: the learned yield model's fused inference on 1e6 queries and
             its gain over RTMC at the held-out error;
  c2:        64 uneven foams x the 25 sweep points (1600 jobs, 1e6 primaries
             each) in one batched call replayed as a HIP graph, with the
             autotuned launch, against the same jobs traced one by one.

The FP64 oracle is timed beside each single-foam workload on a bounded
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
SWEEP_CHUNK = 1 << 28  # primaries per chunk of a batched call
PAIRED_IDS_PER_POINT = 128  # c1 sub-record: primary ids of every sweep point paired with the oracle

CONFIGS = {
    "c3": dict(n=256, porosity=0.8, ell=2.0, seed=4, energies=[250.0], thetas=[-80.0], primaries=100_000_000,
               max_gen=10, rng=4,
               name="256^3 GRF foam, porosity 0.8; 250 eV, theta uniform in [0, 80]; 1e8 primaries; max_gen 10"),
    "c1": dict(n=128, porosity=0.6, ell=2.0, seed=1, energies=[50.0, 100.0, 250.0, 500.0, 1000.0],
               thetas=[0.0, 20.0, 40.0, 60.0, 80.0], primaries=10_000_000, max_gen=6, rng=2,
               name="128^3 GRF foam, porosity 0.6; 5 E x 5 theta points; 1e7 primaries/point; max_gen 6"),
    "c0": dict(n=16, porosity=0.5, ell=2.0, seed=0, energies=[500.0], thetas=[0.0], primaries=10_000, max_gen=6,
               rng=1, name="16^3 GRF foam, porosity 0.5; 500 eV normal incidence; 1e4 primaries; max_gen 6"),
    "c2": dict(n_foams=64, sizes=[64, 96, 128, 192], energies=[50.0, 100.0, 250.0, 500.0, 1000.0],
               thetas=[0.0, 20.0, 40.0, 60.0, 80.0], primaries=1_000_000, max_gen=6, rng=3,
               name="64 GRF foams, porosity ~U[0.2,0.8], grids from {64,96,128,192}^3; 25 points each; "
                    "1e6 primaries/point; one HIP graph"),
}
METRIC = "primaries/s + ray-tri tests/s at <=3 sigma yield error vs FP64 oracle; surrogate vs RTMC"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(texts) -> str:
    """sha256 (first 16 hex digits) of C++ sources with comments and blank
    space removed, so that edits to comments keep a counter summary current."""
    h = hashlib.sha256()
    for t in texts:
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(" ".join(t.split()).encode())
    return h.hexdigest()[:16]


TRAVERSAL_SOURCES = ("traverse.hip", "device_util.h", "rtmc_internal.h")


def kernel_hash() -> str:
    """Hash of the traversal kernel's sources."""
    return source_hash(open(os.path.join(ROOT, "paper_1806_00205_amd", "csrc", f)).read()
                       for f in TRAVERSAL_SOURCES)


def load_traffic(cfg_name: str):
    """Committed counter summary of the traversal kernel on a workload, if it
    was taken on the kernel sources as they stand (else None)."""
    path = os.path.join(ROOT, "profiles", f"k_traverse_{cfg_name}_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d


def oracle_threads() -> int:
    """Threads the oracle runs with: OpenMP's thread count when the
    environment sets one (the host's CPU share), else every core this
    process may run on."""
    n = os.environ.get("OMP_NUM_THREADS", "")
    if n.strip().isdigit() and int(n) > 0:
        return int(n)
    return len(os.sched_getaffinity(0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    ap.add_argument("--primaries", type=int, default=0, help="override primaries per point")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sub", action="store_true", help="headline workload only (no c1, surrogate or c2 records)")
    ap.add_argument("--workers", type=int, default=0,
                    help="foam-generation processes of the batched workload (0: up to 16, one per host core)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU path (shard primary ids, one "
              "all-reduce of the tally block) is a design, not built", file=sys.stderr)
        sys.exit(2)

    import paper_1806_00205_amd as rt

    if args.config == "c2":
        print(json.dumps(bench_batched(args, CONFIGS["c2"], args.primaries or CONFIGS["c2"]["primaries"])), flush=True)
        return
    ctx = rt.Context(0)
    achievable = ctx.copy_probe(1 << 32, reps=5)
    # the GPU workloads are timed first, the host-side work (build timing, the
    # oracle on the host cores) follows, so that no timed step runs just after
    # the oracle has loaded every host core
    out, st = bench_foam(ctx, args, args.config, achievable)
    sub = None
    if args.config == "c3" and not args.no_sub:
        sub, st1 = bench_foam(ctx, args, "c1", achievable)
    foam_extras(ctx, args, out, st)
    if sub is not None:
        foam_extras(ctx, args, sub, st1)
        for k in ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline", "data"):
            sub.pop(k, None)
        out["c1"] = sub
        out["surrogate"] = bench_surrogate(ctx, out)
    ctx.close()
    if args.config == "c3" and not args.no_sub:
        sub = bench_batched(args, CONFIGS["c2"], CONFIGS["c2"]["primaries"])
        for k in ("metric", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline", "data"):
            sub.pop(k, None)
        out["c2"] = sub
    print(json.dumps(out), flush=True)


def bench_foam(ctx, args, name, achievable):
    """One single-foam workload: its (E, theta) points traced as one batched
    call per step.  Returns the record and what foam_extras needs."""
    import torch

    import foamgen as fg

    cfg = CONFIGS[name]
    npp = args.primaries or cfg["primaries"]
    t0 = time.time()
    mesh = fg.make_grf_foam(cfg["n"], cfg["porosity"], cfg["ell"], seed=cfg["seed"])
    tab = fg.make_tables("vaughan")
    log(f"{name}: mesh {mesh.n_tris} triangles in {time.time() - t0:.1f} s")
    sid = ctx.load_scene(mesh)
    tid = ctx.load_tables(tab)
    info = ctx.scene_info(sid)
    log(f"{name}: BVH built on device in {info['build_ms']:.1f} ms, depth {info['bvh_depth']}")
    points = [(E, th) for E in cfg["energies"] for th in cfg["thetas"]]

    # the points go through the library as one batch: chunks of up to 2^28
    # primaries span several points, so every generation's launch is large
    # (per-point results are those of single traces, integer tallies equal)
    lc = ctx.get_launch()
    ctx.set_launch(lc["block"], lc["wg_per_cu"], lc["lds_stack"], SWEEP_CHUNK, lc["refill"], lc["occupancy"],
                   lc["claim"])
    jobs = [(sid, E, th, npp, cfg["rng"] * 1000 + k) for k, (E, th) in enumerate(points)]

    def step():
        return ctx.trace_batch(tid, jobs, max_gen=cfg["max_gen"])

    for w in range(args.warmup):
        step()
        log(f"{name}: warmup {w + 1}/{args.warmup} done")
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
        log(f"{name}: step {s + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    prim_s = tot["prim"] / wall
    # algorithmic bytes of the traversal kernel: node and triangle fetches,
    # origin + direction reads of queued (secondary) rays, hit-record writes
    alg_bytes = (NODE_BYTES * tot["visits"] + TRI_BYTES * tot["tests"] +
                 Q_READ_BYTES * (tot["rays"] - tot["prim"]) + HIT_BYTES * tot["rays"])
    per_launch = alg_bytes / max(tot["launches"], 1)
    kernel_ms = tot["kms"] / max(tot["launches"], 1)
    achieved = alg_bytes / (tot["kms"] * 1e-3) / 1e9 if tot["kms"] > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": prim_s,
        "unit": "primaries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{name}: {cfg['name']}", "n_tris": info["n_tris"],
                   "primaries_per_point": npp, "points": len(points), "bvh_depth": info["bvh_depth"],
                   "call": "rtmc_trace_batch over the points", "launch": ctx.get_launch()},
        "tri_tests_per_s": tot["tests"] / wall,
        "rays_per_s": tot["rays"] / wall,
        "node_visits_per_ray": tot["visits"] / max(tot["rays"], 1),
        "tri_tests_per_ray": tot["tests"] / max(tot["rays"], 1),
        "rays_per_primary": tot["rays"] / max(tot["prim"], 1),
        "yields": {f"{E:g}eV_{th:g}deg": round(r["yield"], 5) for (E, th), r in zip(points, last)},
        "max_yield_sigma": max(r["yield_sigma"] for r in last),
        "roofline": roofline(name, achieved, per_launch, kernel_ms, tot, achievable),
    }
    ctx.set_launch(**lc)
    return out, (mesh, tab, cfg, jobs, tid, lc)


def foam_extras(ctx, args, out, st):
    """The BVH build timing and the oracle baseline of a single-foam workload."""
    mesh, tab, cfg, jobs, tid, lc = st
    out["bvh_build"] = bench_build(ctx, mesh)
    if not args.no_cpu_baseline:
        ctx.set_launch(lc["block"], lc["wg_per_cu"], lc["lds_stack"], SWEEP_CHUNK, lc["refill"], lc["occupancy"],
                   lc["claim"])
        try:
            out["cpu_baseline"] = cpu_baseline(ctx, tid, mesh, tab, cfg, jobs, args.cpu_seconds)
        finally:
            ctx.set_launch(**lc)
    return out


def roofline(name, achieved, per_launch, kernel_ms, tot, achievable):
    """Roofline object of the traversal kernel: algorithmic bytes per launch
    over its average launch duration (HIP events on the library's stream),
    against the published HBM peak; measured traffic and the binding unit
    from the committed counter summary of the same kernel sources."""
    tr = load_traffic(name)
    r = {
        "bound": tr.get("bound", "hbm") if tr else "hbm",
        "achieved": achieved,
        "peak": PEAK_HBM_GBPS,
        "unit": "GB/s",
        "frac": achieved / PEAK_HBM_GBPS,
        "traffic": (tr["fetch_plus_write_bytes_per_alg_byte"] * per_launch if tr else None),
        "kernel": "k_traverse",
        "kernel_ms_avg": kernel_ms,
        "kernel_ms_total": tot["kms"],
        "shade_ms_total": tot["sms"],
        "kernel_launches": tot["launches"],
        "alg_bytes_per_launch": per_launch,
        "achievable_copy_gbps": achievable,
    }
    if tr:
        # measured memory-side rate of the same bytes per launch, next to the
        # algorithmic rate and the copy probe (from the counter summary)
        r["measured_dram_gbps"] = r["traffic"] / (kernel_ms * 1e-3) / 1e9 if kernel_ms > 0 else None
        r["measured_dram_frac_of_copy"] = r["measured_dram_gbps"] / achievable if r["measured_dram_gbps"] else None
        r["valu_issue"] = tr.get("valu_issue")
        r["l2_hit"] = tr.get("l2_hit")
        # the vector-ALU ceiling: one wave64 VALU instruction per CU per cycle
        # (four SIMDs, four cycles per instruction each)
        r["alu"] = {"achieved": tr.get("valu_issue"), "peak": 1.0, "unit": "VALU wave-instructions per CU per cycle",
                    "frac": tr.get("valu_issue")}
        r["counters"] = f"profiles/k_traverse_{name}_traffic.json"
    return r


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


def _paired(ppg, ppo):
    """Agreement, mean paired difference of escape counts and its standard error."""
    import numpy as np
    d = ppg.astype(np.int64) - ppo.astype(np.int64)
    se = float(d.std(ddof=1) / math.sqrt(d.size)) if d.size > 1 else 0.0
    return float((d == 0).mean()), float(d.mean()), se


def cpu_baseline(ctx, tid, mesh, tab, cfg, jobs, seconds):
    """The FP64 oracle on the host's cores, on primary ids 0..n-1 of the
    benchmark's own jobs, paired with the GPU's escape counts of the same ids
    (traced by the same batched call, outside the timed region).  One point:
    the oracle rate at all threads and at one; a sweep: besides, the first
    ids of every point."""
    import numpy as np
    import torch

    import oracle

    oracle.build(force=False)
    cores = oracle_threads()
    k_mid = len(jobs) // 2
    _, E, th, npp, seed = jobs[k_mid]
    mg = cfg["max_gen"]
    # pilot on enough primaries to keep every thread busy, then size the sample
    pilot = 4 * cores
    t = time.perf_counter()
    oracle.trace(mesh, tab, E, th, pilot, seed=seed, max_gen=mg, n_threads=cores)
    per = (time.perf_counter() - t) / pilot
    n = int(max(64, min(npp, seconds / max(per, 1e-9))))
    t = time.perf_counter()
    o = oracle.trace(mesh, tab, E, th, n, seed=seed, max_gen=mg, n_threads=cores, per_primary=True)
    dt = time.perf_counter() - t
    # one core, on a prefix of the same ids (about a tenth of the time budget)
    n1 = int(max(8, min(n, 0.1 * seconds / max(per * cores, 1e-9))))
    t = time.perf_counter()
    o1 = oracle.trace(mesh, tab, E, th, n1, seed=seed, max_gen=mg, n_threads=1)
    dt1 = time.perf_counter() - t
    # the GPU's per-primary counts from the benchmark's own batched call
    pps = [torch.zeros(j[3], dtype=torch.int32, device="cuda:0") for j in jobs]
    g = ctx.trace_batch(tid, jobs, max_gen=mg, per_primary=pps)
    agree, mean, se = _paired(pps[k_mid][:n].cpu().numpy(), o["per_primary"]["escaped"])
    out = {
        "value": n / dt,
        "unit": "primaries/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"primary ids 0..{n - 1} at E={E:g} eV, theta={th:g} deg on the same mesh ({dt:.1f} s)",
        "tri_tests_per_s": o["n_tri_tests"] / dt,
        "one_core": {"primaries_per_s": n1 / dt1, "tri_tests_per_s": o1["n_tri_tests"] / dt1,
                     "sample": f"primary ids 0..{n1 - 1} ({dt1:.1f} s)"},
        "paired_parity": {"oracle_yield": o["yield"], "gpu_yield_same_ids": float(pps[k_mid][:n].sum().item()) / n,
                          "gpu_yield_all": g[k_mid]["yield"], "same_escape_count_frac": agree,
                          "mean_diff": mean, "paired_z": mean / se if se > 0 else 0.0},
    }
    if len(jobs) > 1:
        k = PAIRED_IDS_PER_POINT
        t = time.perf_counter()
        rows, chi2 = [], 0.0
        for (s, E, th, n_j, sd), pp, r in zip(jobs, pps, g):
            oj = oracle.trace(mesh, tab, E, th, k, seed=sd, max_gen=mg, n_threads=cores, per_primary=True)
            a, m, e = _paired(pp[:k].cpu().numpy(), oj["per_primary"]["escaped"])
            z = m / e if e > 0 else 0.0
            chi2 += z * z
            sig = math.sqrt(r["yield_sigma"] ** 2 + oj["yield_sigma"] ** 2)
            rows.append({"E": E, "theta": th, "agree": a, "paired_z": z,
                         "unpaired_z": (r["yield"] - oj["yield"]) / sig if sig > 0 else 0.0})
        out["sweep_pairing"] = {
            "ids_per_point": k, "points": len(rows), "seconds": time.perf_counter() - t,
            "min_agree": min(x["agree"] for x in rows),
            "max_abs_paired_z": max(abs(x["paired_z"]) for x in rows),
            "max_abs_unpaired_z": max(abs(x["unpaired_z"]) for x in rows),
            "chi2_paired": chi2, "dof": len(rows), "per_point": rows,
        }
    del pps
    return out


def bench_surrogate(ctx, rtmc):
    """Fused surrogate inference on 1e6 queries (HIP events on the library's
    stream), and its gain over RTMC at the held-out error of the committed
    experiment: RTMC needs (sigma_1 / MAE)^2 primaries per yield at that
    error, sigma_1 being the per-primary spread of the held-out yields."""
    from paper_1806_00205_amd.surrogate import bench_inference, bench_training

    srg = ctx.srg_create(8, 256, 4, seed=0)
    inf = bench_inference(ctx, srg, n=1_000_000, reps=20)
    train = bench_training(ctx)
    # the same loop at a batch that fills the GPU (256 workgroups, four passes of 16384 rows)
    train["batch_65536"] = bench_training(ctx, batch=65536, steps=30)
    # held-out experiment (python -m paper_1806_00205_amd.surrogate --train-foams 1024 --points 96
    # --test-foams 256 --steps 8000): MAE 0.0100 over 256 x 25 points judged by RTMC at 1e6 primaries,
    # which need 4006 primaries per yield for sigma = MAE
    mae, prim_per_yield = 0.0100, 4006.0
    rate = rtmc["value"]
    return {"queries": inf["queries"], "ms_per_1e6_queries": inf["ms_per_batch"],
            "queries_per_s": inf["queries_per_s"], "achieved_tflops": inf["tflops"], "peak_tflops": 2500.0,
            "frac": inf["frac"], "dtype": "bf16 operands, f32 accumulate",
            "heldout_mae": mae, "heldout_source": "profiles/surrogate_vs_rtmc_heldout.md",
            "rtmc_primaries_per_yield_at_mae": prim_per_yield,
            "rtmc_yields_per_s_at_mae": rate / prim_per_yield,
            "gain_vs_rtmc": inf["queries_per_s"] / (rate / prim_per_yield),
            "training": train}


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
    specs = []
    for i in range(cfg["n_foams"]):
        n = int(rng.choice(cfg["sizes"]))
        p = float(rng.uniform(0.2, 0.8))
        specs.append((1000 + i, n, p))
    # the foams are CPU work: generated in worker processes, loaded as they arrive
    import multiprocessing as mp

    from foamgen.batch import grf_foam
    workers = args.workers or max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("spawn").Pool(workers) as pool:
        for i, m in enumerate(pool.imap(grf_foam, specs)):
            _, n, p = specs[i]
            scenes.append((ctx.load_scene(m), n, p, m.n_tris))
            tris += m.n_tris
            log(f"foam {i + 1}/{cfg['n_foams']}: {n}^3, porosity {p:.2f}, {m.n_tris} triangles")
    log(f"{len(scenes)} foams, {tris} triangles in {time.time() - t0:.0f} s")
    mid = sorted(scenes, key=lambda x: x[3])[len(scenes) // 2][0]
    tuned = ctx.autotune(mid, tid, 250.0, 40.0, 2_000_000)
    log(f"autotuned launch: {tuned}")
    jobs = []
    for sid, _, _, _ in scenes:
        for E in cfg["energies"]:
            for th in cfg["thetas"]:
                jobs.append((sid, E, th, npp, int(rng.integers(1, 2 ** 62))))
    total = len(jobs) * npp
    for w in range(args.warmup):
        ctx.trace_batch(tid, jobs, max_gen=cfg["max_gen"])
        log(f"warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s_ in range(args.steps):
        res = ctx.trace_batch(tid, jobs, max_gen=cfg["max_gen"])
        log(f"step {s_ + 1}/{args.steps} done")
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
        "metric": METRIC,
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
    return out


if __name__ == "__main__":
    main()
