"""Synthetic inputs: foams are watertight, oriented, periodic and porous as asked."""
from collections import Counter

import numpy as np
import pytest

import foamgen as fg


def _directed_edges_pair_up(tris, canon):
    ct = canon[tris]
    de = Counter()
    for a, b, c in ct:
        for x, y in ((a, b), (b, c), (c, a)):
            de[(int(x), int(y))] += 1
    return all(n == 1 and de.get((y, x), 0) == 1 for (x, y), n in de.items())


@pytest.mark.parametrize("n,p,seed", [(8, 0.5, 0), (12, 0.3, 1), (12, 0.8, 2)])
def test_foam_is_watertight_modulo_periodicity(n, p, seed):
    m = fg.make_grf_foam(n, p, 2.0, seed=seed)
    assert _directed_edges_pair_up(m.tris, m.meta["canon"])


def test_foam_normals_point_into_the_void():
    m = fg.make_grf_foam(12, 0.5, 2.0, seed=3)
    f, tau = fg.foam_field(12, 0.5, 2.0, seed=3)
    canon = m.meta["canon"]
    ax = canon % 3
    base = canon // 3
    nx, ny, nz = f.shape
    z = base % nz
    y = (base // nz) % ny
    x = base // (nz * ny)
    step = np.eye(3, dtype=int)[ax]
    f0 = f[x, y, z]
    dirv = step * np.where(f0 >= tau, 1.0, -1.0)[:, None]  # solid -> void along the edge
    V = m.verts[m.tris].astype(np.float64)
    s = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    score = (s[:, None, :] * dirv[m.tris]).sum(-1).sum(-1)
    assert (score > 0).all()


def test_foam_porosity_and_size():
    m = fg.make_grf_foam(16, 0.5, 2.0, seed=0)
    assert abs(m.meta["void_fraction"] - 0.5) < 1e-3
    assert 2500 < m.n_tris < 6000  # "~4k triangles" for the 16^3 foam
    assert m.verts.min() >= 0 and m.verts[:, :2].max() <= 16 and m.verts[:, 2].max() <= 15
    # periodic copies: vertices on x = 16 mirror those on x = 0
    canon = m.meta["canon"]
    on_hi = np.nonzero(m.verts[:, 0] == 16)[0]
    for i in on_hi[:50]:
        j = np.nonzero((canon == canon[i]) & (m.verts[:, 0] == 0))[0]
        assert j.size >= 1
        for k in j:
            assert m.verts[k, 2] == m.verts[i, 2] and (m.verts[k, 1] - m.verts[i, 1]) % 16 == 0


def test_foam_seeded():
    a = fg.make_grf_foam(10, 0.6, 2.0, seed=7)
    b = fg.make_grf_foam(10, 0.6, 2.0, seed=7)
    c = fg.make_grf_foam(10, 0.6, 2.0, seed=8)
    assert np.array_equal(a.verts, b.verts) and np.array_equal(a.tris, b.tris)
    assert a.verts.shape != c.verts.shape or not np.array_equal(a.verts, c.verts)


def test_grf_covariance_length():
    f = fg.grf_field(64, 64, 2.0, seed=1)
    # covariance exp(-r^2 / (2 l^2)): at r = 2 it is exp(-1/2)
    c2 = np.mean(f * np.roll(f, 2, axis=0))
    assert abs(c2 - np.exp(-0.5)) < 0.03


def test_chung_everhart_closed_forms():
    xi = np.linspace(0.001, 0.999, 999)
    E = fg.ce_inverse(xi)
    assert np.allclose(fg.ce_cdf(E), xi, atol=1e-12)
    assert fg.ce_inverse(0.5) == pytest.approx(4.5, rel=1e-12)
    t = fg.make_tables("vaughan")
    assert t.cdf_F[0] == 0 and t.cdf_F[-1] == 1 and np.all(np.diff(t.cdf_F) >= 0)


def test_chord_lengths_match_a_walk_along_every_line():
    """Void chord lengths (a surrogate input) against walking each lattice line."""
    from foamgen.descriptors import chord_lengths
    rng = np.random.default_rng(3)
    v = rng.random((5, 4, 7)) < 0.55
    v[1, 2, :] = True  # an all-void column
    nx, ny, nz = v.shape
    inner = v[:, :, 1:nz - 1]

    def walk(line, periodic):
        if line.all():
            return [len(line)]
        if not line.any():
            return []
        if periodic:
            line = np.roll(line, -int(np.argmin(line)))
        out, c = [], 0
        for x in line:
            if x:
                c += 1
            elif c:
                out.append(c)
                c = 0
        return out + ([c] if c else [])

    ref = []
    for y in range(ny):
        for z in range(nz - 2):
            ref += walk(inner[:, y, z], True)
    for x in range(nx):
        for z in range(nz - 2):
            ref += walk(inner[x, :, z], True)
    for x in range(nx):
        for y in range(ny):
            ref += walk(inner[x, y, :], False)
    assert sorted(chord_lengths(v).tolist()) == sorted(ref)


@pytest.mark.parametrize("a,n", [(0.1, 4), (0.2, 2), (0.25, 1)])
def test_cage_is_the_union_of_its_struts(a, n):
    """Open cubic cage: watertight modulo periodicity except where it stands on
    the substrate, normals into the void, enclosed volume exactly that of the
    struts, no surface on a face of the periodic cell."""
    ell = 16.0
    m = fg.make_cage(a, ell, n)
    V = m.verts.astype(np.float64)
    c = m.meta["canon"]
    e = Counter()
    for tri in m.tris:
        for u, v in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0])):
            e[(c[u], c[v])] += 1
    for (u, v), k in e.items():
        if e.get((v, u), 0) != k:  # open edges only on the substrate plane
            assert V[c == u][0][2] == 0.0 and V[c == v][0][2] == 0.0
    P = V[m.tris]
    s = np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0])
    t = a * ell
    top = n * ell + t
    exact = (n + 1) * t * (2 * t * ell - t * t) + t * t * (top - (n + 1) * t)
    assert (s[:, 2] * P[:, :, 2].mean(axis=1)).sum() / 2 == pytest.approx(exact, rel=1e-5)  # FP32 vertices

    def solid(p):
        band = lambda x: (x % ell < t / 2) | (x % ell > ell - t / 2)
        layer = np.zeros(len(p), dtype=bool)
        for k in range(n + 1):
            layer |= (p[:, 2] > k * ell) & (p[:, 2] < k * ell + t)
        return ((band(p[:, 1]) & layer) | (band(p[:, 0]) & layer)
                | (band(p[:, 0]) & band(p[:, 1]) & (p[:, 2] < top)) | (p[:, 2] < 0))

    cen = P.mean(axis=1)
    nrm = s / np.linalg.norm(s, axis=1, keepdims=True)
    assert not solid(cen + 1e-3 * nrm).any()
    assert solid(cen - 1e-3 * nrm).all()
    # nothing on the periodic cell's faces, the substrate plane included
    assert not np.any(np.all(P[:, :, 0] == 0.0, axis=1) | np.all(P[:, :, 0] == ell, axis=1))
    assert not np.any(np.all(P[:, :, 1] == 0.0, axis=1) | np.all(P[:, :, 1] == ell, axis=1))
    assert not np.any(np.all(P[:, :, 2] == 0.0, axis=1))
    assert m.meta["v_f_paper"] == pytest.approx(a * a)
    assert fg.cage_solid_fraction(a) == pytest.approx(3 * a * a - 2 * a ** 3)
