"""Seeded synthetic nanofoams and simple verification geometries.

The paper's foams come from X-ray tomography (section 2.3); those images are
not available, so foams here are level sets of a seeded Gaussian random field
(GRF):

* white noise N(0, 1) on an (n, n, nz) lattice, PCG64 seeded;
* filtered in Fourier space by exp(-|k|^2 l^2 / 4), so the covariance is
  exp(-r^2 / (2 l^2)) with correlation length l (in voxels);
* normalised to unit variance;
* void where f < tau, tau the porosity quantile of the interior layers;
* the bottom layer is forced solid and the top layer void, so the surface is
  closed from below and open to the vacuum above;
* periodic in x and y (the paper's boundary conditions, section 2.2).

All lengths are in voxel units (pitch 1); the method itself has no length
scale because the flat-surface tables depend only on energy and angle.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .mc import marching_cubes_periodic

# scene flags (same bit values as the C interface)
PERIODIC_XY = 1
SUBSTRATE = 2


@dataclass
class Mesh:
    verts: np.ndarray  # float32 [V, 3]
    tris: np.ndarray  # int32 [T, 3], CCW seen from the vacuum side
    box_lo: tuple  # (x, y, z) float
    box_hi: tuple
    flags: int
    meta: dict

    @property
    def n_tris(self) -> int:
        return int(self.tris.shape[0])


def grf_field(n: int, nz: int, ell: float, seed: int) -> np.ndarray:
    """Unit-variance periodic GRF on an (n, n, nz) lattice, indexed [x, y, z]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((n, n, nz))
    kx = 2.0 * np.pi * np.fft.fftfreq(n)
    kz = 2.0 * np.pi * np.fft.rfftfreq(nz)
    k2 = kx[:, None, None] ** 2 + kx[None, :, None] ** 2 + kz[None, None, :] ** 2
    spec = np.fft.rfftn(w) * np.exp(-k2 * ell * ell / 4.0)
    f = np.fft.irfftn(spec, s=(n, n, nz), axes=(0, 1, 2))
    f -= f.mean()
    f /= f.std()
    return f


def foam_field(n: int, porosity: float, ell: float = 2.0, seed: int = 0, nz: int | None = None):
    """Thresholded GRF ready for meshing: returns (field, tau)."""
    nz = n if nz is None else nz
    if not (0.0 < porosity < 1.0):
        raise ValueError("porosity must be in (0, 1)")
    if n < 2 or nz < 3:
        raise ValueError("grid too small")
    f = grf_field(n, nz, ell, seed)
    interior = f[:, :, 1 : nz - 1]
    tau = float(np.quantile(interior, porosity))
    # keep lattice values off the iso-level so no vertex lands on a corner
    near = np.abs(f - tau) < 1e-9
    f[near] = tau + 1e-9
    f[:, :, 0] = tau + 1.0  # solid substrate layer
    f[:, :, nz - 1] = tau - 1.0  # vacuum layer
    return f, tau


def make_grf_foam(n: int, porosity: float, ell: float = 2.0, seed: int = 0, nz: int | None = None,
                  field=None) -> Mesh:
    """Periodic GRF nanofoam mesh in a box [0, n) x [0, n) x [0, nz-1].
    `field` may pass in foam_field's (field, tau) for the same arguments."""
    nz = n if nz is None else nz
    f, tau = foam_field(n, porosity, ell, seed, nz) if field is None else field
    verts, tris, canon = marching_cubes_periodic(f, tau)
    void_frac = float((f[:, :, 1 : nz - 1] < tau).mean())
    return Mesh(
        verts=verts,
        tris=tris,
        box_lo=(0.0, 0.0, 0.0),
        box_hi=(float(n), float(n), float(nz - 1)),
        flags=PERIODIC_XY | SUBSTRATE,
        meta=dict(kind="grf_foam", n=n, nz=nz, porosity=porosity, ell=ell, seed=seed,
                  tau=tau, void_fraction=void_frac, canon=canon),
    )


def flat_plane(L: float = 4.0, z0: float = 1.0, height: float = 4.0) -> Mesh:
    """Two triangles covering the periodic cell at z = z0, normal +z."""
    v = np.array([[0, 0, z0], [L, 0, z0], [L, L, z0], [0, L, z0]], dtype=np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    return Mesh(v, t, (0.0, 0.0, 0.0), (L, L, z0 + height), PERIODIC_XY, dict(kind="flat", L=L, z0=z0))


def trench(w: float = 2.0, h: float = 3.0, tw: float = 1.0, Ly: float = 4.0) -> Mesh:
    """Infinite slot of width w and depth h between walls of thickness tw.

    The cell is x in [0, tw + w] (periodic), y in [0, Ly] (periodic), z in
    [-1, h + w].  The wall straddles the periodic x boundary (half of it at
    each end of the cell) and the floor sits above the cell bottom, so that
    no surface lies on a cell face (a hit there would race the exit test).  Surfaces:
    wall tops (z = h), slot floor (z = 0, x in [tw/2, tw/2 + w]), the wall
    face at x = tw/2 facing +x and the face at x = tw/2 + w facing -x.  All
    normals point into the vacuum.
    """
    P = tw + w
    a, b = 0.5 * tw, 0.5 * tw + w
    quads = [
        # wall tops, normal +z
        [(0, 0, h), (a, 0, h), (a, Ly, h), (0, Ly, h)],
        [(b, 0, h), (P, 0, h), (P, Ly, h), (b, Ly, h)],
        # slot floor, normal +z
        [(a, 0, 0), (b, 0, 0), (b, Ly, 0), (a, Ly, 0)],
        # wall face at x = a, normal +x
        [(a, 0, 0), (a, Ly, 0), (a, Ly, h), (a, 0, h)],
        # wall face at x = b, normal -x
        [(b, 0, 0), (b, 0, h), (b, Ly, h), (b, Ly, 0)],
    ]
    verts = []
    tris = []
    for q in quads:
        base = len(verts)
        verts.extend(q)
        tris.append([base, base + 1, base + 2])
        tris.append([base, base + 2, base + 3])
    v = np.array(verts, dtype=np.float32)
    t = np.array(tris, dtype=np.int32)
    return Mesh(v, t, (0.0, 0.0, -1.0), (P, Ly, h + w), PERIODIC_XY,
                dict(kind="trench", w=w, h=h, tw=tw, Ly=Ly))


def random_soup(n_tris: int, seed: int, L: float = 4.0, dyadic_bits: int = 6) -> Mesh:
    """Random triangles with dyadic coordinates inside a box (first-hit tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = float(1 << dyadic_bits)
    c = rng.integers(0, int(L * scale) + 1, size=(n_tris, 3, 3)) / scale
    c[:, :, 2] = np.clip(c[:, :, 2], 0.25, L - 0.25)
    v = c.reshape(-1, 3).astype(np.float32)
    t = np.arange(n_tris * 3, dtype=np.int32).reshape(n_tris, 3)
    return Mesh(v, t, (0.0, 0.0, 0.0), (L, L, L), PERIODIC_XY, dict(kind="soup", seed=seed))


def surface_rays(mesh: Mesh, n: int, seed: int, eps: float = 1e-4) -> np.ndarray:
    """Rays leaving random points of random triangles into their front side.

    Returns float64 [n, 6] (origin, unit direction) with a cosine-distributed
    direction about the triangle normal, offset eps along the normal: the
    shape of daughter rays.  Uses its own PCG64 stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    V = mesh.verts[mesh.tris].astype(np.float64)
    s = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    a = np.linalg.norm(s, axis=1)
    ok = np.nonzero(a > 0)[0]
    pick = ok[rng.integers(0, ok.size, size=n)]
    r1 = rng.random(n)
    r2 = rng.random(n)
    sq = np.sqrt(r1)
    b0, b1, b2 = 1 - sq, sq * (1 - r2), sq * r2
    P = b0[:, None] * V[pick, 0] + b1[:, None] * V[pick, 1] + b2[:, None] * V[pick, 2]
    nrm = s[pick] / a[pick, None]
    u = rng.random(n)
    phi = 2 * np.pi * rng.random(n)
    # any orthonormal frame works here: build it by Gram-Schmidt
    helper = np.where(np.abs(nrm[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = helper - (helper * nrm).sum(1, keepdims=True) * nrm
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    sb, cb = np.sqrt(u), np.sqrt(1 - u)
    d = cb[:, None] * nrm + sb[:, None] * (np.cos(phi)[:, None] * t1 + np.sin(phi)[:, None] * t2)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = P + eps * nrm
    lo = np.array(mesh.box_lo)
    hi = np.array(mesh.box_hi)
    o = np.clip(o, lo, hi)
    return np.concatenate([o, d], axis=1)


def top_rays(mesh: Mesh, n: int, seed: int, theta_max_deg: float = 80.0) -> np.ndarray:
    """Downward rays from random points of the top face (primary-like)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo = np.array(mesh.box_lo)
    hi = np.array(mesh.box_hi)
    o = np.empty((n, 3))
    o[:, 0] = lo[0] + (hi[0] - lo[0]) * rng.random(n)
    o[:, 1] = lo[1] + (hi[1] - lo[1]) * rng.random(n)
    o[:, 2] = hi[2]
    th = np.deg2rad(theta_max_deg) * rng.random(n)
    ps = 2 * np.pi * rng.random(n)
    d = np.stack([np.sin(th) * np.cos(ps), np.sin(th) * np.sin(ps), -np.cos(th)], axis=1)
    return np.concatenate([o, d], axis=1)
