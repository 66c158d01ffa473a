"""Seeded synthetic inputs for the RTMC hot path.

Foams, verification geometries and flat-surface tables.  This module holds
none of the method's arithmetic: both the FP64 oracle and the GPU library
consume what it produces.
"""
from .foam import (Mesh, PERIODIC_XY, SUBSTRATE, flat_plane, foam_field, grf_field,
                   make_grf_foam, random_soup, surface_rays, top_rays, trench)
from .cage import cage_solid_fraction, make_cage
from .mc import marching_cubes_periodic
from .tables import (Tables, bilinear_reference, ce_cdf, ce_inverse, make_tables,
                     paper_w_yield, vaughan_yield)
