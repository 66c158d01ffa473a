"""FP64 brute-force oracle for the RTMC secondary-electron-yield method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product (the GPU library and its
binding) never imports this package, and this package imports nothing from
the product.

``rtmc_oracle.c`` holds the method (plain C, FP64, OpenMP over primaries,
every ray against every triangle); this module only builds it with gcc and
marshals arguments with ctypes.  ``mlp_ref`` holds the FP64 reference of the
learned surrogate's forward and backward passes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rtmc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ID_ESCAPE = -1
ID_SUBSTRATE = -2
ID_LOST = -3


def compile_source(src: str, out: str) -> str:
    """Compile one oracle source file with gcc (IEEE FP64, no contraction, OpenMP)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Build liboracle.so next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


class _MeshIn(C.Structure):
    _fields_ = [("verts", C.c_void_p), ("n_verts", C.c_int64), ("tris", C.c_void_p), ("n_tris", C.c_int64),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("flags", C.c_uint32)]


class _TablesIn(C.Structure):
    _fields_ = [("yld", C.c_void_p), ("n_E", C.c_int32), ("n_theta", C.c_int32), ("E_min", C.c_double),
                ("E_max", C.c_double), ("cdf_E", C.c_void_p), ("cdf_F", C.c_void_p), ("n_cdf", C.c_int32),
                ("Ec", C.c_double), ("esee", C.c_void_p), ("emission", C.c_int32)]


class _Job(C.Structure):
    _fields_ = [("E0", C.c_double), ("theta_deg", C.c_double), ("pid0", C.c_uint64),
                ("n_primaries", C.c_uint64), ("seed", C.c_uint64), ("max_gen", C.c_int32),
                ("n_ebins", C.c_int32), ("n_abins", C.c_int32), ("n_threads", C.c_int32), ("n_zbins", C.c_int32)]


class _Result(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("n_primaries", "n_rays", "n_escaped", "n_absorbed", "n_truncated",
                                          "n_lost", "n_substrate", "n_wraps", "n_tri_tests", "n_dropped_tris")] + \
               [(n, C.c_double) for n in ("e_escaped", "e_deposited", "yield_", "yield_sigma")]


_lib = None


def _bind(path):
    lib = C.CDLL(path)
    lib.orc_first_hit.argtypes = [C.POINTER(_MeshIn), C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_int32]
    lib.orc_trace.argtypes = [C.POINTER(_MeshIn), C.POINTER(_TablesIn), C.POINTER(_Job), C.POINTER(_Result)] + \
        [C.c_void_p] * 7
    lib.orc_table_yield.argtypes = [C.POINTER(_TablesIn), C.c_double, C.c_double]
    lib.orc_table_yield.restype = C.c_double
    lib.orc_sample_energy.argtypes = [C.POINTER(_TablesIn), C.c_double, C.c_double]
    lib.orc_sample_energy.restype = C.c_double
    lib.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.orc_onb.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.orc_mesh_dropped.argtypes = [C.POINTER(_MeshIn), C.POINTER(C.c_int64)]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _bind(_LIB)
    return _lib


class Variant:
    """The oracle's entry points bound to another build of the source.

    Used by the tests that plant a mistake in a copy of the oracle and check
    that a pin catches it.
    """

    def __init__(self, path):
        self._lib = _bind(path)

    def __getattr__(self, name):
        fn = globals()[name]

        def call(*a, **k):
            return fn(*a, _lib=self._lib, **k)
        return call


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


class _Keep:
    """Holds numpy arrays alive while a ctypes struct points into them."""

    def __init__(self):
        self.refs = []

    def add(self, a):
        self.refs.append(a)
        return a


def _mesh_in(mesh, keep):
    v = keep.add(np.ascontiguousarray(mesh.verts, dtype=np.float32))
    t = keep.add(np.ascontiguousarray(mesh.tris, dtype=np.int32))
    mi = _MeshIn()
    mi.verts = _ptr(v)
    mi.n_verts = v.shape[0]
    mi.tris = _ptr(t)
    mi.n_tris = t.shape[0]
    mi.lo = (C.c_double * 3)(*mesh.box_lo)
    mi.hi = (C.c_double * 3)(*mesh.box_hi)
    mi.flags = int(mesh.flags)
    return mi


def _tables_in(tab, keep):
    y = keep.add(np.ascontiguousarray(tab.yld, dtype=np.float32))
    ce = keep.add(np.ascontiguousarray(tab.cdf_E, dtype=np.float32))
    cf = keep.add(np.ascontiguousarray(tab.cdf_F, dtype=np.float32))
    ti = _TablesIn()
    ti.yld = _ptr(y)
    ti.n_E, ti.n_theta = y.shape
    ti.E_min, ti.E_max = tab.E_min, tab.E_max
    ti.cdf_E = _ptr(ce)
    ti.cdf_F = _ptr(cf)
    ti.n_cdf = ce.shape[0]
    ti.Ec = tab.Ec
    ti.emission = int(getattr(tab, "emission", 0))
    es = getattr(tab, "esee", None)
    if es is not None:
        ti.esee = _ptr(keep.add(np.ascontiguousarray(es, dtype=np.float32)))
    return ti


def philox4x32_10(ctr, key, _lib=None):
    """Philox4x32-10 of one 128-bit counter under a 64-bit key (as uint32 words)."""
    lib = _lib or _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def first_hit(mesh, rays, n_threads: int = 0, _lib=None):
    """First surface reached by each ray (origin, direction rows), FP64 brute force.

    Returns (tri, t, wraps): tri is the caller's triangle index or -1 escape,
    -2 substrate, -3 lost; t is the path length over all periodic segments.
    """
    lib = _lib or _load()
    keep = _Keep()
    mi = _mesh_in(mesh, keep)
    r = np.ascontiguousarray(rays, dtype=np.float64).reshape(-1, 6)
    n = r.shape[0]
    tri = np.zeros(n, dtype=np.int32)
    t = np.zeros(n, dtype=np.float64)
    w = np.zeros(n, dtype=np.int32)
    st = lib.orc_first_hit(C.byref(mi), _ptr(r), n, _ptr(tri), _ptr(t), _ptr(w), int(n_threads))
    if st != 0:
        raise ValueError(f"oracle first_hit failed ({st})")
    return tri, t, w


def trace(mesh, tab, E0: float, theta_deg: float, n_primaries: int, seed: int, max_gen: int = 6,
          pid0: int = 0, n_ebins: int = 256, n_abins: int = 90, n_threads: int = 0, per_primary: bool = False,
          n_zbins: int = 0, _lib=None):
    """FP64 RTMC over primaries pid0 .. pid0 + n - 1; returns a dict."""
    lib = _lib or _load()
    keep = _Keep()
    mi = _mesh_in(mesh, keep)
    ti = _tables_in(tab, keep)
    job = _Job(float(E0), float(theta_deg), int(pid0), int(n_primaries), int(seed), int(max_gen), int(n_ebins),
               int(n_abins), int(n_threads), int(n_zbins))
    res = _Result()
    eh = np.zeros(n_ebins, dtype=np.uint64)
    ah = np.zeros(n_abins, dtype=np.uint64)
    zh = np.zeros(max(n_zbins, 1), dtype=np.uint64)
    pp = None
    if per_primary:
        pp = dict(escaped=np.zeros(n_primaries, dtype=np.uint32), e_esc=np.zeros(n_primaries),
                  e_dep=np.zeros(n_primaries), rays=np.zeros(n_primaries, dtype=np.uint32))
    st = lib.orc_trace(C.byref(mi), C.byref(ti), C.byref(job), C.byref(res), _ptr(eh), _ptr(ah), _ptr(zh),
                       _ptr(pp["escaped"]) if pp else None, _ptr(pp["e_esc"]) if pp else None,
                       _ptr(pp["e_dep"]) if pp else None, _ptr(pp["rays"]) if pp else None)
    if st != 0:
        raise ValueError(f"oracle trace failed ({st})")
    out = {f[0].rstrip("_"): getattr(res, f[0]) for f in _Result._fields_}
    out["e_hist"] = eh
    out["a_hist"] = ah
    if n_zbins:
        out["z_hist"] = zh
    if pp:
        out["per_primary"] = pp
    return out


def table_yield(tab, E: float, alpha: float, _lib=None) -> float:
    keep = _Keep()
    ti = _tables_in(tab, keep)
    return (_lib or _load()).orc_table_yield(C.byref(ti), float(E), float(alpha))


def sample_energy(tab, xi: float, E_avail: float, _lib=None) -> float:
    keep = _Keep()
    ti = _tables_in(tab, keep)
    return (_lib or _load()).orc_sample_energy(C.byref(ti), float(xi), float(E_avail))


def onb(n, _lib=None):
    n = np.ascontiguousarray(n, dtype=np.float64)
    t1 = np.zeros(3)
    t2 = np.zeros(3)
    (_lib or _load()).orc_onb(_ptr(n), _ptr(t1), _ptr(t2))
    return t1, t2


def mesh_dropped(mesh, _lib=None) -> int:
    keep = _Keep()
    mi = _mesh_in(mesh, keep)
    d = C.c_int64(0)
    st = (_lib or _load()).orc_mesh_dropped(C.byref(mi), C.byref(d))
    if st != 0:
        raise ValueError(f"oracle mesh check failed ({st})")
    return int(d.value)
