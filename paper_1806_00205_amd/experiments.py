"""Experiments of the paper's section 3 on the GPU path.

* ``cage``: the open cubic cage on a substrate (section 3.1, Fig. ashby):
  yield against primary energy at normal incidence for struts of t/l = 0.10,
  0.15, 0.20, 0.25 (the paper's v_f = 1, 2.25, 4, 6.25 % as (t/l)^2), with
  the paper's tungsten fits and emission rule.

Command line: ``python -m paper_1806_00205_amd.experiments cage --out r.json``.
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["cage"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--primaries", type=int, default=1_000_000)
    ap.add_argument("--cells", type=int, nargs="+", default=[4])
    ap.add_argument("--tables", default="paper_w")
    args = ap.parse_args()
    import paper_1806_00205_amd as rt

    ctx = rt.Context(0)
    out = {}
    t0 = time.time()
    for n in args.cells:
        out[f"n_cells={n}"] = cage_sweep(ctx, n_cells=n, primaries=args.primaries, kind=args.tables)
        print(f"[cage] n_cells {n} done in {time.time() - t0:.1f} s", flush=True)
    ctx.close()
    print(json.dumps(out))
    if args.out:
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
