"""Foams of the batched-workload family with their descriptors, for worker
processes (imports nothing but numpy and foamgen)."""
from __future__ import annotations

from .descriptors import foam_descriptors
from .foam import foam_field, make_grf_foam


def foam_with_descriptors(spec):
    """spec = (seed, n, porosity[, ell]) -> (mesh, six descriptors)."""
    seed, n, p = spec[0], int(spec[1]), float(spec[2])
    ell = float(spec[3]) if len(spec) > 3 else 2.0
    field = foam_field(n, p, ell, seed=seed)
    mesh = make_grf_foam(n, p, ell, seed=seed, field=field)
    return mesh, foam_descriptors(mesh, *field)


def grf_foam(spec):
    """spec = (seed, n, porosity) -> the GRF foam mesh (correlation length 2 voxels)."""
    seed, n, p = spec
    return make_grf_foam(int(n), float(p), 2.0, seed=int(seed))
