"""Geometric descriptors of a synthetic foam (inputs of the yield surrogate).

Six numbers per foam, computed from its field and mesh:
  porosity      void fraction of the interior lattice layers;
  s_over_v      mesh area / cell volume (voxel units);
  h_mean, h_var area-weighted mean and variance of the mean curvature
                H = -1/2 div(grad f / |grad f|) of the field at the triangle
                centroids (nearest lattice point), curvature of the level set;
  chord_mean, chord_std  lengths of void runs along lattice lines in x, y
                (periodic) and z, a pore-size measure.
"""
from __future__ import annotations

import numpy as np


def _grad(f):
    gx = (np.roll(f, -1, 0) - np.roll(f, 1, 0)) * 0.5
    gy = (np.roll(f, -1, 1) - np.roll(f, 1, 1)) * 0.5
    gz = np.gradient(f, axis=2)
    return gx, gy, gz


def mean_curvature(f):
    gx, gy, gz = _grad(f)
    norm = np.sqrt(gx * gx + gy * gy + gz * gz) + 1e-12
    nx, ny, nz = gx / norm, gy / norm, gz / norm
    div = ((np.roll(nx, -1, 0) - np.roll(nx, 1, 0)) * 0.5 + (np.roll(ny, -1, 1) - np.roll(ny, 1, 1)) * 0.5
           + np.gradient(nz, axis=2))
    return -0.5 * div


def _runs(rows, periodic):
    """Lengths of True runs along the last axis of a 2-D boolean array (as a
    multiset: order is not meaningful).  Periodic rows are first rotated to
    start at a solid site so that no run wraps; an all-void row is one run."""
    M = np.asarray(rows, dtype=bool)
    if M.size == 0:
        return np.zeros(0, dtype=np.int64)
    L = M.shape[1]
    full = M.all(axis=1)
    A = M[M.any(axis=1) & ~full]
    if periodic and A.shape[0]:
        k = np.argmin(A, axis=1)
        A = np.take_along_axis(A, (k[:, None] + np.arange(L)[None, :]) % L, axis=1)
    P = np.zeros((A.shape[0], L + 2), dtype=np.int8)
    P[:, 1:-1] = A
    d = np.diff(P, axis=1)
    starts = np.nonzero(d == 1)[1]
    ends = np.nonzero(d == -1)[1]  # row-major order: pairs with starts
    return np.concatenate([ends - starts, np.full(int(full.sum()), L, dtype=np.int64)])


def chord_lengths(void):
    nx, ny, nz = void.shape
    inner = void[:, :, 1:nz - 1]
    runs = [_runs(inner.transpose(1, 2, 0).reshape(-1, nx), True),
            _runs(inner.transpose(0, 2, 1).reshape(-1, ny), True),
            _runs(inner.reshape(-1, nz - 2), False)]
    return np.concatenate(runs).astype(np.float64)


def foam_descriptors(mesh, field, tau):
    """Six descriptors of a foam from its mesh and thresholded field."""
    nz = field.shape[2]
    void = field < tau
    porosity = float(void[:, :, 1:nz - 1].mean())
    V = mesh.verts[mesh.tris].astype(np.float64)
    s = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    area = 0.5 * np.linalg.norm(s, axis=1)
    lo, hi = np.array(mesh.box_lo), np.array(mesh.box_hi)
    vol = float(np.prod(hi - lo))
    s_over_v = float(area.sum() / vol)
    H = mean_curvature(field)
    c = V.mean(axis=1)
    idx = np.rint(c).astype(np.int64)
    idx[:, 0] %= field.shape[0]
    idx[:, 1] %= field.shape[1]
    idx[:, 2] = np.clip(idx[:, 2], 0, nz - 1)
    h = H[idx[:, 0], idx[:, 1], idx[:, 2]]
    w = area / max(area.sum(), 1e-30)
    h_mean = float((w * h).sum())
    h_var = float((w * (h - h_mean) ** 2).sum())
    ch = chord_lengths(void)
    return np.array([porosity, s_over_v, h_mean, h_var, ch.mean(), ch.std()], dtype=np.float64)
