"""Learned yield surrogate: data from RTMC, training and evaluation.

The surrogate maps eight inputs -- foam porosity, surface-to-volume ratio,
mean and variance of the surface mean curvature, mean and standard deviation
of the void chord length, ln E and cos(theta) -- to the secondary electron
yield.  Its training targets are yields traced by the library itself
(rtmc_trace_batch); its forward and backward passes and AdamW updates run in
the library's BF16 matrix-core kernels (rtmc_srg_*).  Plain RTMC stays the
reference: it evaluates the surrogate on held-out foams and is the fallback for
inputs outside the training support.

Command line: ``python -m paper_1806_00205_amd.surrogate --out results.json``.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

import foamgen as fg

GRID_E = [50.0, 100.0, 250.0, 500.0, 1000.0]
GRID_THETA = [0.0, 20.0, 40.0, 60.0, 80.0]


def foam_specs(first_seed: int, count: int, rng: np.random.Generator, sizes=(40, 48, 56)):
    """(seed, grid, porosity) of `count` foams of the batched-workload family:
    grid uniform over `sizes`, porosity ~ U[0.2, 0.8]."""
    return [(first_seed + i, int(rng.choice(sizes)), float(rng.uniform(0.2, 0.8))) for i in range(count)]


def generate(specs, pool=None):
    """Meshes and descriptors of the specs, in worker processes when a pool is given."""
    from foamgen.batch import foam_with_descriptors

    if pool is None:
        return [foam_with_descriptors(sp) for sp in specs]
    return pool.map(foam_with_descriptors, specs, chunksize=1)


def features(desc, E, theta_deg):
    """Rows of the eight surrogate inputs (unnormalised)."""
    desc = np.atleast_2d(desc)
    E = np.asarray(E, dtype=np.float64).reshape(-1)
    th = np.asarray(theta_deg, dtype=np.float64).reshape(-1)
    return np.concatenate([desc, np.log(E)[:, None], np.cos(np.deg2rad(th))[:, None]], axis=1)


def rtmc_yields(ctx, table, jobs, max_gen=6, batch=4096):
    """Yields of (scene, E, theta, n, seed) jobs through the batched graph path."""
    out = []
    for i in range(0, len(jobs), batch):
        out.extend(ctx.trace_batch(table, jobs[i:i + batch], max_gen=max_gen))
    return np.array([r["yield"] for r in out]), np.array([r["yield_sigma"] for r in out]), out


class Surrogate:
    """Normalisation + the library's MLP; RTMC fallback outside the training support."""

    def __init__(self, ctx, seed: int = 0):
        self.ctx = ctx
        self.id = ctx.srg_create(8, 256, 4, seed=seed)
        self.mu = None
        self.sd = None
        self.lo = None
        self.hi = None

    def _norm(self, F):
        return ((F - self.mu) / self.sd).astype(np.float32)

    def fit(self, F, y, steps=4000, batch=1024, lr=2e-3, weight_decay=1e-5, seed=0, log=None):
        import torch

        self.mu = F.mean(axis=0)
        self.sd = F.std(axis=0) + 1e-12
        self.lo = F.min(axis=0)
        self.hi = F.max(axis=0)
        Xd = torch.tensor(self._norm(F), device=f"cuda:{self.ctx.device}")
        yd = torch.tensor(np.asarray(y, dtype=np.float32), device=Xd.device)
        # cosine decay to 2 % of lr; the library draws the batches and replays one step as a graph
        frac = np.arange(steps) / max(steps - 1, 1)
        lr_s = lr * (0.02 + 0.49 * (1.0 + np.cos(np.pi * frac)))
        step_losses = self.ctx.srg_train(self.id, Xd, yd, batch, lr_s, weight_decay=weight_decay, seed=seed)
        losses = [(it, float(step_losses[it])) for it in range(steps) if it % 200 == 0 or it == steps - 1]
        if log:
            for it, loss in losses:
                log(f"step {it}: loss {loss:.3e}")
        return losses

    def predict(self, F):
        import torch

        Xd = torch.tensor(self._norm(np.asarray(F, dtype=np.float64)), device=f"cuda:{self.ctx.device}")
        return self.ctx.srg_predict(self.id, Xd).cpu().numpy().astype(np.float64)

    def in_support(self, F, margin=0.05):
        span = self.hi - self.lo
        F = np.atleast_2d(F)
        return np.all((F >= self.lo - margin * span) & (F <= self.hi + margin * span), axis=1)

    def predict_or_trace(self, F, fallback):
        """Surrogate where the inputs lie in the training support, else fallback(row index)."""
        F = np.atleast_2d(F)
        y = self.predict(F)
        ok = self.in_support(F)
        for i in np.nonzero(~ok)[0]:
            y[i] = fallback(int(i))
        return y, ok


def forward_flops(n_in: int = 8, width: int = 256, depth: int = 4) -> int:
    """Multiply-adds x 2 of one forward pass (unpadded layer sizes)."""
    return 2 * (n_in * width + (depth - 1) * width * width + width)


def bench_inference(ctx, srg_id: int, n_in: int = 8, n: int = 1_000_000, reps: int = 20, seed: int = 0):
    """Timed batches of n queries through the fused kernel (HIP events on the
    library's stream); dense BF16 matrix-core peak 2.5 PFLOP/s."""
    import torch

    dev = f"cuda:{ctx.device}"
    X = torch.randn(n, n_in, generator=torch.Generator().manual_seed(seed)).to(dev)
    ctx.srg_predict(srg_id, X)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.srg_predict(srg_id, X)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = forward_flops(n_in) * n
    return {"queries": n, "ms_per_batch": ms, "queries_per_s": n / (ms * 1e-3),
            "tflops": flops / (ms * 1e-3) / 1e12, "peak_tflops": 2500.0,
            "frac": flops / (ms * 1e-3) / 2.5e15}


def bench_training(ctx, n_in: int = 8, batch: int = 1024, steps: int = 500, seed: int = 0):
    """The device training loop (three launches per step, replayed as a graph)
    on synthetic rows: steps per second, samples per second and the
    forward + backward FLOP rate (3 x the forward's per sample)."""
    import torch

    dev = f"cuda:{ctx.device}"
    g = torch.Generator().manual_seed(seed)
    X = torch.randn(65536, n_in, generator=g).to(dev)
    y = (0.5 + 0.3 * torch.sin(X[:, 0])).to(dev)
    s = ctx.srg_create(n_in, 256, 4, seed=seed)
    lr = np.full(steps, 1e-3, dtype=np.float32)
    ctx.srg_train(s, X, y, batch, lr[:8], seed=1)  # captures the step's graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.srg_train(s, X, y, batch, lr, seed=2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flops = 3 * forward_flops(n_in) * batch * steps
    return {"batch": batch, "steps": steps, "us_per_step": dt / steps * 1e6, "samples_per_s": batch * steps / dt,
            "tflops": flops / dt / 1e12, "frac": flops / dt / 2.5e15}


def _traced_batches(device, tab, specs, points, batch_foams, pool, max_gen, log, what):
    """Generate the foams of `specs` in batches, trace each batch's jobs in a
    context of its own (so its scenes are freed), and return per job
    (descriptors, E, theta, yield, sigma, n_primaries) plus the tracing time.
    points(foam index) -> list of (E, theta, n_primaries, seed)."""
    import paper_1806_00205_amd as rt

    rows, t_trace, t_gen, prim = [], 0.0, 0.0, 0
    for b0 in range(0, len(specs), batch_foams):
        t0 = time.time()
        foams = generate(specs[b0:b0 + batch_foams], pool)
        t_gen += time.time() - t0
        ctx = rt.Context(device)
        try:
            tid = ctx.load_tables(tab)
            jobs, meta = [], []
            for k, (mesh, d) in enumerate(foams):
                sid = ctx.load_scene(mesh)
                for E, th, n, sd in points(b0 + k):
                    jobs.append((sid, float(E), float(th), int(n), int(sd)))
                    meta.append((d, float(E), float(th)))
            del foams
            t0 = time.time()
            y, sig, res = rtmc_yields(ctx, tid, jobs, max_gen=max_gen)
            t_trace += time.time() - t0
            prim += sum(r["n_primaries"] for r in res)
        finally:
            ctx.close()
        rows.extend((d, E, th, yy, ss) for (d, E, th), yy, ss in zip(meta, y, sig))
        log(f"[srg] {what}: {min(b0 + batch_foams, len(specs))}/{len(specs)} foams")
    return rows, t_trace, t_gen, prim


def run_experiment(ctx, n_train=256, points_per_foam=64, n_test=64, train_primaries=20000,
                   eval_primaries=100000, steps=4000, seed=0, log=print, sizes=(40, 48, 56), workers=0,
                   batch_foams=64, max_gen=6):
    """Train on RTMC yields of n_train foams, evaluate on n_test held-out foams."""
    rng = np.random.default_rng(seed)
    tab = fg.make_tables("vaughan")
    pool = None
    if workers and workers > 1:
        import multiprocessing as mp

        pool = mp.get_context("spawn").Pool(workers)
    try:
        train_specs = foam_specs(10000, n_train, rng, sizes)
        test_specs = foam_specs(90000, n_test, rng, sizes)
        # training points: E log-uniform in [50, 1000] eV, theta uniform in [0, 80] deg
        tp = []
        for _ in range(n_train):
            E = np.exp(rng.uniform(np.log(50.0), np.log(1000.0), size=points_per_foam))
            th = rng.uniform(0.0, 80.0, size=points_per_foam)
            tp.append([(e, t, train_primaries, int(rng.integers(1, 2 ** 62))) for e, t in zip(E, th)])
        # held-out foams: the 5 x 5 grid
        jp = [[(e, t, eval_primaries, int(rng.integers(1, 2 ** 62))) for e in GRID_E for t in GRID_THETA]
              for _ in range(n_test)]
        train, t_rtmc, t_gen, prim = _traced_batches(ctx.device, tab, train_specs, lambda i: tp[i], batch_foams,
                                                     pool, max_gen, log, "training foams")
        log(f"[srg] {len(train)} training yields traced in {t_rtmc:.2f} s ({prim / t_rtmc:.3g} primaries/s); "
            f"foams generated in {t_gen:.1f} s")
        test, t_eval, t_gen2, prim_t = _traced_batches(ctx.device, tab, test_specs, lambda i: jp[i], batch_foams,
                                                        pool, max_gen, log, "held-out foams")
    finally:
        if pool is not None:
            pool.close()
            pool.join()
    F_train = features(np.array([r[0] for r in train]), [r[1] for r in train], [r[2] for r in train])
    y_train = np.array([r[3] for r in train])
    model = Surrogate(ctx, seed=seed)
    t0 = time.time()
    losses = model.fit(F_train, y_train, steps=steps, seed=seed, log=log)
    t_train = time.time() - t0
    log(f"[srg] trained {steps} steps in {t_train:.2f} s")

    F_test = features(np.array([r[0] for r in test]), [r[1] for r in test], [r[2] for r in test])
    y_test = np.array([r[3] for r in test])
    s_test = np.array([r[4] for r in test])
    test_grid = [sp[1] for sp in test_specs]
    y_hat = model.predict(F_test)
    err = np.abs(y_hat - y_test)
    ok = model.in_support(F_test)
    # one million surrogate queries (the held-out features, repeated), end to end
    Fq = np.repeat(F_test, int(math.ceil(1e6 / len(F_test))), axis=0)[:1_000_000]
    import torch

    Xq = torch.tensor(model._norm(Fq), device=f"cuda:{ctx.device}")
    ctx.srg_predict(model.id, Xq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.srg_predict(model.id, Xq)
    torch.cuda.synchronize()
    t_q = time.perf_counter() - t0
    inf = bench_inference(ctx, model.id)
    # a foam-blind predictor for comparison: the mean training yield of the 32
    # training points nearest in (ln E, cos theta), whatever their foam
    Et, Ft = F_train[:, -2:], F_test[:, -2:]
    d2 = ((Ft[:, None, :] - Et[None, :, :]) ** 2).sum(axis=2)
    nn = np.argpartition(d2, 32, axis=1)[:, :32]
    blind = y_train[nn].mean(axis=1)
    blind_mae = float(np.abs(blind - y_test).mean())
    # RTMC cost of one yield at the surrogate's error: primaries for sigma = MAE
    sd_pp = float(np.median(s_test * math.sqrt(eval_primaries)))
    mae = float(err.mean())
    n_matched = (sd_pp / mae) ** 2
    rtmc_rate = prim_t / t_eval
    rtmc_yield_s = rtmc_rate / n_matched
    out = {
        "n_train_foams": n_train, "train_yields": len(train), "train_primaries_per_yield": train_primaries,
        "foam_grids": list(sizes),
        "n_test_foams": n_test, "test_points": len(test), "eval_primaries_per_yield": eval_primaries,
        "mae": mae, "p95_abs_err": float(np.quantile(err, 0.95)), "max_abs_err": float(err.max()),
        "foam_blind_mae": blind_mae,
        "mae_in_support": float(err[ok].mean()) if ok.any() else None, "in_support_frac": float(ok.mean()),
        "eval_sigma_median": float(np.median(s_test)),
        "train_sigma_median": float(np.median([r[4] for r in train])),
        "mae_by_grid": {str(n): float(err[np.repeat(np.array(test_grid) == n, 25)].mean())
                        for n in sorted(set(test_grid))},
        "final_loss": losses[-1][1], "train_seconds": t_train, "gen_seconds": t_gen + t_gen2,
        "rtmc_train_seconds": t_rtmc, "rtmc_eval_seconds": t_eval,
        "surrogate_queries_per_s": 1e6 / t_q, "rtmc_primaries_per_s": rtmc_rate,
        "rtmc_primaries_for_matched_error": n_matched, "rtmc_yields_per_s_matched_error": rtmc_yield_s,
        "gain": (1e6 / t_q) / rtmc_yield_s,
        "inference_kernel": inf,
        "train_samples_per_s": steps * 1024 / t_train,
    }
    return out, model


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--train-foams", type=int, default=256)
    ap.add_argument("--points", type=int, default=64)
    ap.add_argument("--test-foams", type=int, default=64)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--train-primaries", type=int, default=100000)
    ap.add_argument("--eval-primaries", type=int, default=1000000)
    ap.add_argument("--sizes", default="64,96,128,192", help="foam grids (voxels per side)")
    ap.add_argument("--workers", type=int, default=min(16, len(os.sched_getaffinity(0))))
    ap.add_argument("--batch-foams", type=int, default=32)
    ap.add_argument("--timing", action="store_true",
                    help="only time the kernels: 1e6-query inference and the training loop at batch 1024 and 65536")
    args = ap.parse_args()
    import paper_1806_00205_amd as rt

    ctx = rt.Context(0)
    if args.timing:
        srg = ctx.srg_create(8, 256, 4, seed=0)
        print(json.dumps({"inference": bench_inference(ctx, srg), "training": bench_training(ctx),
                          "training_batch_65536": bench_training(ctx, batch=65536, steps=30)}), flush=True)
        ctx.close()
        return
    res, _ = run_experiment(ctx, n_train=args.train_foams, points_per_foam=args.points, n_test=args.test_foams,
                            train_primaries=args.train_primaries, eval_primaries=args.eval_primaries,
                            steps=args.steps, sizes=tuple(int(x) for x in args.sizes.split(",")),
                            workers=args.workers, batch_foams=args.batch_foams,
                            log=lambda m: print(m, flush=True))
    print(json.dumps(res))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
