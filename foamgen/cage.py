"""Open cubic cage on a substrate (the paper's second verification geometry,
section 3.1): a periodic lattice of square struts of thickness t along the
edges of cubic cells of size l, n_cells cells high, standing on the flat
substrate at z = 0.

The struts of one lattice cell: along x centred on (y, z) = (0, z_k), along y
centred on (x, z) = (0, z_k), along z centred on (x, y) = (0, 0), with
horizontal layers z_k spanning [k l, k l + t] for k = 0 .. n_cells and the
vertical struts spanning [0, n_cells l + t].  The periodic cell is
[0, l) x [0, l) x [0, n_cells l + t + l]: one cell of void above the top.

The surface is the boundary of that union of axis-aligned boxes, built on the
grid whose planes are the strut faces: every grid cell is solid or void, each
solid/void face becomes two triangles oriented towards the void, so the mesh
is watertight (periodically) with no T-junctions.  The substrate plane z = 0
is not meshed (the scene's substrate flag supplies it) and no surface lies on
a face of the periodic cell.

Solid volume fraction of an infinite cage: 3 (t/l)^2 - 2 (t/l)^3.  The paper
quotes v_f = C (t/l)^2 with C about 28 and studies v_f = 1, 2.25, 4 and 6.25 %,
which are (t/l)^2 for t/l = 0.10, 0.15, 0.20, 0.25 (C = 1).
"""
from __future__ import annotations

import numpy as np

from .foam import PERIODIC_XY, SUBSTRATE, Mesh


def cage_solid_fraction(t_over_l: float) -> float:
    """Solid fraction of an infinite cubic cage with square struts."""
    a = float(t_over_l)
    return 3.0 * a * a - 2.0 * a ** 3


def _axis_planes(l: float, t: float):
    # x (and y): strut band centred on 0, periodic: [0, t/2) and [l - t/2, l)
    return np.array([0.0, t / 2.0, l - t / 2.0, l])


def make_cage(t_over_l: float = 0.2, l: float = 16.0, n_cells: int = 4) -> Mesh:
    if not (0.0 < t_over_l < 0.5):
        raise ValueError("t/l must be in (0, 0.5)")
    if n_cells < 1:
        raise ValueError("need at least one cell")
    t = t_over_l * l
    xs = _axis_planes(l, t)
    top = n_cells * l + t
    zs = np.array(sorted(set([0.0] + [k * l for k in range(n_cells + 1)] + [k * l + t for k in range(n_cells + 1)]
                         + [top + l])))
    nx, nz = len(xs) - 1, len(zs) - 1
    band = np.array([True, False, True])  # the x (or y) intervals inside the strut band
    zc = 0.5 * (zs[:-1] + zs[1:])
    layer = np.array([any(k * l <= z < k * l + t for k in range(n_cells + 1)) for z in zc])
    below_top = zc < top
    solid = np.zeros((nx, nx, nz), dtype=bool)
    bx = band[:, None, None]
    by = band[None, :, None]
    solid |= by & layer[None, None, :]  # struts along x
    solid |= bx & layer[None, None, :]  # struts along y
    solid |= bx & by & below_top[None, None, :]  # struts along z
    solid = np.broadcast_to(solid, (nx, nx, nz)).copy()

    verts = {}
    vlist = []
    canon = []  # periodic identification: plane index nx is plane 0 of the next cell

    def vid(i, j, k):
        key = (i, j, k)
        if key not in verts:
            verts[key] = len(vlist)
            vlist.append((xs[i], xs[j], zs[k]))
            canon.append((i % nx, j % nx, k))
        return verts[key]

    tris = []

    def quad(a, b, c, d):
        # a b c d counter-clockwise seen from the void side
        tris.append((a, b, c))
        tris.append((a, c, d))

    for i in range(nx):
        for j in range(nx):
            for k in range(nz):
                if not solid[i, j, k]:
                    continue
                # +x neighbour (periodic)
                if not solid[(i + 1) % nx, j, k]:
                    quad(vid(i + 1, j, k), vid(i + 1, j + 1, k), vid(i + 1, j + 1, k + 1), vid(i + 1, j, k + 1))
                if not solid[(i - 1) % nx, j, k]:
                    quad(vid(i, j, k), vid(i, j, k + 1), vid(i, j + 1, k + 1), vid(i, j + 1, k))
                if not solid[i, (j + 1) % nx, k]:
                    quad(vid(i, j + 1, k), vid(i, j + 1, k + 1), vid(i + 1, j + 1, k + 1), vid(i + 1, j + 1, k))
                if not solid[i, (j - 1) % nx, k]:
                    quad(vid(i, j, k), vid(i + 1, j, k), vid(i + 1, j, k + 1), vid(i, j, k + 1))
                if k + 1 < nz and not solid[i, j, k + 1]:
                    quad(vid(i, j, k + 1), vid(i + 1, j, k + 1), vid(i + 1, j + 1, k + 1), vid(i, j + 1, k + 1))
                if k > 0 and not solid[i, j, k - 1]:
                    quad(vid(i, j, k), vid(i, j + 1, k), vid(i + 1, j + 1, k), vid(i + 1, j, k))
    V = np.array(vlist, dtype=np.float64)
    T = np.array(tris, dtype=np.int32)
    keys = {}
    cid = np.array([keys.setdefault(c, len(keys)) for c in canon], dtype=np.int64)
    return Mesh(verts=V.astype(np.float32), tris=T, box_lo=(0.0, 0.0, 0.0), box_hi=(l, l, float(zs[-1])),
                flags=PERIODIC_XY | SUBSTRATE,
                meta=dict(kind="cage", t_over_l=t_over_l, l=l, t=t, n_cells=n_cells, top=top,
                          v_f_paper=t_over_l ** 2, v_f_solid=cage_solid_fraction(t_over_l), canon=cid))
