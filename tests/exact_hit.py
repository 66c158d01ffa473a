"""Exact closest hit with rational arithmetic, for tiny meshes.

Written from the geometry, not from the Moller-Trumbore solve: intersect the
ray with the triangle's plane, then test the hit point against the three
edges with exact sign tests.  Every float is a dyadic rational, so
``fractions.Fraction`` evaluates all of this without rounding.
"""
from fractions import Fraction as F


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def exact_first_hit(verts, tris, lo, hi, substrate, ray):
    """Closest front-facing hit of one ray in a NON-periodic box.

    Returns (id, t) with id the triangle index, -1 (leaves through the top
    moving up), -2 (substrate), -3 (leaves through a side or the bottom).
    """
    O = tuple(F(float(x)) for x in ray[:3])
    D = tuple(F(float(x)) for x in ray[3:6])
    lo = [F(float(x)) for x in lo]
    hi = [F(float(x)) for x in hi]
    te = []
    for a in range(3):
        if D[a] > 0:
            te.append(max(F(0), (hi[a] - O[a]) / D[a]))
        elif D[a] < 0:
            te.append(max(F(0), (lo[a] - O[a]) / D[a]))
        else:
            te.append(None)
    texit = min(t for t in te if t is not None)
    best = None
    for j, tri in enumerate(tris):
        V = [tuple(F(float(x)) for x in verts[int(k)]) for k in tri]
        s = _cross(_sub(V[1], V[0]), _sub(V[2], V[0]))
        sd = _dot(s, D)
        if sd >= 0:  # back-facing or parallel
            continue
        t = _dot(s, _sub(V[0], O)) / sd
        if t <= 0 or t > texit:
            continue
        P = tuple(O[a] + t * D[a] for a in range(3))
        inside = all(_dot(_cross(_sub(V[(k + 1) % 3], V[k]), _sub(P, V[k])), s) >= 0 for k in range(3))
        if not inside:
            continue
        if best is None or (t, j) < best:
            best = (t, j)
    if best is not None:
        return best[1], best[0]
    if te[2] is not None and te[2] == texit:
        if D[2] > 0:
            return -1, texit
        return (-2 if substrate else -3), texit
    return -3, texit
