"""Experiments of the paper's section 3 on the GPU path.

* ``cage``: the open cubic cage on a substrate (section 3.1, Fig. ashby):
  yield against primary energy at normal incidence for struts of t/l = 0.10,
  0.15, 0.20, 0.25 (the paper's v_f = 1, 2.25, 4, 6.25 % as (t/l)^2), with
  the paper's tungsten fits and emission rule.
* ``penetration``: the absorption-depth profile of a 4 % volume-fraction foam
  at 100 eV for normal and random incidence (section 3.2, Fig. pen): every
  ray of any generation that ends on a surface counts at its depth below the
  top of the cell.

Command line: ``python -m paper_1806_00205_amd.experiments cage --out r.json``
(or ``penetration``).
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

import foamgen as fg

CAGE_T_OVER_L = (0.10, 0.15, 0.20, 0.25)
CAGE_ENERGIES = (50.0, 100.0, 200.0, 300.0, 400.0, 500.0, 600.0, 800.0, 1000.0)


def cage_sweep(ctx, t_over_l=CAGE_T_OVER_L, energies=CAGE_ENERGIES, n_cells: int = 4, cell: float = 16.0,
               primaries: int = 1_000_000, kind: str = "paper_w", seed: int = 7, max_gen: int = 10):
    """Yield of the open cage at normal incidence for each strut thickness and energy."""
    tab = fg.make_tables(kind)
    tid = ctx.load_tables(tab)
    rows = []
    for a in t_over_l:
        m = fg.make_cage(a, cell, n_cells)
        sid = ctx.load_scene(m)
        jobs = [(sid, float(E), 0.0, int(primaries), seed + 1000 * k) for k, E in enumerate(energies)]
        res = ctx.trace_batch(tid, jobs, max_gen=max_gen)
        for E, r in zip(energies, res):
            rows.append(dict(t_over_l=a, v_f_paper=a * a, v_f_solid=fg.cage_solid_fraction(a), E=E,
                             yield_=r["yield"], sigma=r["yield_sigma"], n_tris=m.n_tris))
    return rows


def penetration(ctx, n: int = 128, porosity: float = 0.96, E: float = 100.0, primaries: int = 10_000_000,
                n_zbins: int = 50, seed: int = 1, kind: str = "vaughan", max_gen: int = 10):
    """Absorption-depth histograms of one foam, normal incidence vs theta
    uniform in [0, 80] deg (the random-incidence reading)."""
    m = fg.make_grf_foam(n, porosity, 2.0, seed=seed)
    sid = ctx.load_scene(m)
    tid = ctx.load_tables(fg.make_tables(kind))
    out = dict(n_tris=m.n_tris, porosity=porosity, E=E, n_zbins=n_zbins, tables=kind)
    centres = (np.arange(n_zbins) + 0.5) / n_zbins
    for name, th in (("normal", 0.0), ("random", -80.0)):
        r = ctx.trace(sid, tid, E, th, primaries, seed=seed + 17, max_gen=max_gen, n_zbins=n_zbins)
        z = r["z_hist"].astype(np.float64)
        out[name] = dict(yield_=r["yield"], sigma=r["yield_sigma"], z_hist=r["z_hist"].tolist(),
                         mean_depth=float((z * centres).sum() / z.sum()),
                         median_depth=float(centres[np.searchsorted(np.cumsum(z) / z.sum(), 0.5)]),
                         absorbed=int(z.sum()))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["cage", "penetration"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--primaries", type=int, default=1_000_000)
    ap.add_argument("--cells", type=int, nargs="+", default=[4])
    ap.add_argument("--tables", default="paper_w")
    args = ap.parse_args()
    import paper_1806_00205_amd as rt

    ctx = rt.Context(0)
    out = {}
    t0 = time.time()
    if args.what == "cage":
        for n in args.cells:
            out[f"n_cells={n}"] = cage_sweep(ctx, n_cells=n, primaries=args.primaries, kind=args.tables)
            print(f"[cage] n_cells {n} done in {time.time() - t0:.1f} s", flush=True)
    else:
        for kind in ("vaughan", "paper_w"):
            out[kind] = penetration(ctx, primaries=args.primaries, kind=kind)
            print(f"[penetration] {kind} done in {time.time() - t0:.1f} s", flush=True)
    ctx.close()
    print(json.dumps(out))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
