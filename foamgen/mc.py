"""Periodic marching cubes with a case table derived in code.

The paper turns a voxel model into a triangle mesh with an iso-surface
routine (section 2.3).  This module is the seeded stand-in used to make
synthetic foams: it extracts the level set ``f = tau`` of a scalar field
sampled on a lattice that is periodic in x and y and open in z.

The case table is not typed in.  For each of the 256 corner sign patterns it
is derived by walking the six cube faces:

* on a face with two sign changes the two crossing edges are joined;
* on a face with four sign changes (diagonal pattern) each solid corner is
  cut off on its own.  The rule depends only on the face's four corner
  values, so the two cubes sharing that face choose the same segments and
  the surface is watertight;
* the face segments form closed loops on the cube boundary; each loop is
  oriented so that its area vector points from the solid corners to the
  void corners of the edges it crosses, then fan-triangulated from an apex
  chosen so that no triangle lies in a cube face.

Triangle vertices are ordered so that ``(V1-V0) x (V2-V0)`` points into the
void, i.e. counter-clockwise seen from the vacuum side (the convention of
the paper's normal footnote in section 2.1).
"""
from __future__ import annotations

import numpy as np

# corner c has offset (c & 1, (c >> 1) & 1, (c >> 2) & 1)
_CORNER_OFF = np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int64)


def _edges():
    """12 edges as (corner_lo, corner_hi, axis); edge index = axis*4 + j."""
    out = []
    for a in range(3):
        others = [b for b in range(3) if b != a]
        for j in range(4):
            c = ((j & 1) << others[0]) | (((j >> 1) & 1) << others[1])
            out.append((c, c | (1 << a), a))
    return out


EDGES = _edges()
_EDGE_OF_PAIR = {}
for _e, (_c0, _c1, _a) in enumerate(EDGES):
    _EDGE_OF_PAIR[(_c0, _c1)] = _e
    _EDGE_OF_PAIR[(_c1, _c0)] = _e


def _faces():
    """6 faces, each as its 4 corners in cyclic order."""
    out = []
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        for s in range(2):
            cyc = []
            for (pb, pc) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                cyc.append((s << a) | (pb << b) | (pc << c))
            out.append(cyc)
    return out


FACES = _faces()


def _case_loops(case: int):
    """Closed, oriented loops of crossing-edge indices for one corner pattern."""
    solid = [(case >> c) & 1 for c in range(8)]
    adj = {}

    def link(e0, e1):
        adj.setdefault(e0, []).append(e1)
        adj.setdefault(e1, []).append(e0)

    for cyc in FACES:
        ring = [_EDGE_OF_PAIR[(cyc[k], cyc[(k + 1) % 4])] for k in range(4)]
        cross = [k for k in range(4) if solid[cyc[k]] != solid[cyc[(k + 1) % 4]]]
        if len(cross) == 2:
            link(ring[cross[0]], ring[cross[1]])
        elif len(cross) == 4:
            # diagonal face: isolate each solid corner (edges k-1 and k meet at corner k)
            for k in range(4):
                if solid[cyc[k]]:
                    link(ring[(k - 1) % 4], ring[k])
    loops = []
    seen = set()
    for start in sorted(adj):
        if start in seen:
            continue
        loop = [start]
        seen.add(start)
        prev, cur = None, start
        while True:
            nxt = [e for e in adj[cur] if e != prev]
            # both neighbours equal only for a 2-cycle, which cannot occur
            n = nxt[0]
            if n == start:
                break
            loop.append(n)
            seen.add(n)
            prev, cur = cur, n
        # orient: Newell area vector of midpoints must point solid -> void
        pts = np.array([(_CORNER_OFF[EDGES[e][0]] + _CORNER_OFF[EDGES[e][1]]) * 0.5 for e in loop])
        area = np.zeros(3)
        for k in range(len(loop)):
            area += np.cross(pts[k], pts[(k + 1) % len(loop)])
        score = 0.0
        for e in loop:
            c0, c1, _ = EDGES[e]
            sc, vc = (c0, c1) if solid[c0] else (c1, c0)
            score += float(np.dot(_CORNER_OFF[vc] - _CORNER_OFF[sc], area))
        if score < 0:
            loop = loop[::-1]
        loops.append(loop)
    return loops


def _on_common_face(e0, e1, e2):
    """True when three cube edges lie on one cube face."""
    for cyc in FACES:
        cs = set(cyc)
        if all(EDGES[e][0] in cs and EDGES[e][1] in cs for e in (e0, e1, e2)):
            return True
    return False


def _fan(loop):
    """Fan triangulation whose apex avoids triangles lying in a cube face.

    A fan triangle with all three vertices on one face would lie in the face
    plane (a lattice plane, possibly the periodic boundary).  The apex is the
    first rotation of the loop with the fewest such triangles.
    """
    best = None
    for r in range(len(loop)):
        rot = loop[r:] + loop[:r]
        tri = [(rot[0], rot[k], rot[k + 1]) for k in range(1, len(rot) - 1)]
        bad = sum(_on_common_face(*t) for t in tri)
        if best is None or bad < best[0]:
            best = (bad, tri)
    return best[1]


def _build_table():
    tris = []
    for case in range(256):
        t = []
        for loop in _case_loops(case):
            t.extend(_fan(loop))
        tris.append(t)
    maxn = max(len(t) for t in tris)
    table = np.full((256, maxn, 3), -1, dtype=np.int64)
    count = np.zeros(256, dtype=np.int64)
    for case, t in enumerate(tris):
        count[case] = len(t)
        if t:
            table[case, : len(t)] = np.array(t)
    return table, count


CASE_TRIS, CASE_COUNT = _build_table()


_T_EDGE = 2.0 ** -12  # smallest distance of a vertex from the ends of its edge, in voxels


def marching_cubes_periodic(field: np.ndarray, tau: float):
    """Extract the surface ``field == tau`` (solid where ``field >= tau``).

    ``field`` has shape (nx, ny, nz), indexed [x, y, z]; lattice point (i, j, k)
    sits at position (i, j, k).  x and y are periodic: cubes with i = nx-1 use
    the lattice point i = 0 as their upper corner but place it at x = nx.  z is
    open: cubes span k in [0, nz-1).

    Returns ``verts`` float32 [V, 3], ``tris`` int32 [T, 3] (CCW seen from the
    void) and ``canon`` int64 [V]: a vertex id that identifies periodic copies
    (vertices on x = nx and x = 0 get the same canon id).
    """
    f = np.asarray(field, dtype=np.float64)
    nx, ny, nz = f.shape
    solid = f >= tau
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz - 1), indexing="ij")
    case = np.zeros(ii.shape, dtype=np.int64)
    for c in range(8):
        ox, oy, oz = _CORNER_OFF[c]
        s = solid[(ii + ox) % nx, (jj + oy) % ny, kk + oz]
        case |= s.astype(np.int64) << c
    case = case.ravel()
    cnt = CASE_COUNT[case]
    cube_idx = np.repeat(np.arange(case.size), cnt)
    # k-th triangle of each cube
    starts = np.cumsum(cnt) - cnt
    kth = np.arange(cube_idx.size) - np.repeat(starts, cnt)
    local = CASE_TRIS[case[cube_idx], kth]  # [T, 3] local edge ids
    ci = ii.ravel()[cube_idx]
    cj = jj.ravel()[cube_idx]
    ck = kk.ravel()[cube_idx]
    # global edge id on the unwrapped (nx+1, ny+1, nz) lattice: lower corner + axis
    ec0 = np.array([e[0] for e in EDGES])
    eax = np.array([e[2] for e in EDGES])
    lo_off = _CORNER_OFF[ec0]  # [12, 3]
    px = ci[:, None] + lo_off[local, 0]
    py = cj[:, None] + lo_off[local, 1]
    pz = ck[:, None] + lo_off[local, 2]
    ax = eax[local]
    gid = ((px * (ny + 1) + py) * nz + pz) * 3 + ax
    uniq, inv = np.unique(gid.ravel(), return_inverse=True)
    tris = inv.reshape(-1, 3).astype(np.int32)
    ux = uniq // 3
    uax = uniq % 3
    uz = ux % nz
    uy = (ux // nz) % (ny + 1)
    uxx = ux // (nz * (ny + 1))
    f0 = f[uxx % nx, uy % ny, uz]
    step = np.stack([(uax == 0), (uax == 1), (uax == 2)], axis=1).astype(np.int64)
    x1 = uxx + step[:, 0]
    y1 = uy + step[:, 1]
    z1 = uz + step[:, 2]
    f1 = f[x1 % nx, y1 % ny, z1]
    t = (tau - f0) / (f1 - f0)
    # keep every vertex strictly inside its edge after rounding to float32
    # (exact for lattice coordinates below 2048): a crossing that rounded onto
    # a lattice corner could put a triangle into the plane of a cube face,
    # and on the periodic boundary that plane is a face of the cell
    t = np.clip(t, _T_EDGE, 1.0 - _T_EDGE)
    pos = np.stack([uxx, uy, uz], axis=1).astype(np.float64) + step * t[:, None]
    verts = pos.astype(np.float32)
    canon = (((uxx % nx) * ny + (uy % ny)) * nz + uz) * 3 + uax
    return verts, tris, canon
