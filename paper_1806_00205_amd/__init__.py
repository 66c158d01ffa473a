"""MI355X ray-tracing Monte Carlo for secondary electron emission.

Thin ctypes binding of ``librtmc.so`` (declared in ``include/rtmc.h``): it
marshals arguments and nothing else.  Every step of the method runs in the
library's HIP kernels; PyTorch only supplies device memory (through its
caching allocator) and the stream.  Importing this package never loads the
library; constructing a :class:`Context` does, and raises if the library is
missing or was built for another GPU.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtmc.so")

PERIODIC_XY = 1
SUBSTRATE = 2
HIT_ESCAPE = -1
HIT_SUBSTRATE = -2
HIT_LOST = -3

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EOVERFLOW", -6: "ENOTIMPL"}

EXPORTS = [
    "rtmc_create", "rtmc_destroy", "rtmc_last_error", "rtmc_set_stream", "rtmc_load_mesh", "rtmc_build_bvh",
    "rtmc_get_scene_info", "rtmc_bvh_download", "rtmc_bvh_download_wide", "rtmc_load_tables", "rtmc_trace", "rtmc_trace_batch",
    "rtmc_first_hit", "rtmc_first_hit_noalloc", "rtmc_sort_pairs_u64", "rtmc_set_launch", "rtmc_get_launch", "rtmc_autotune",
    "rtmc_copy_probe", "rtmc_srg_create", "rtmc_srg_param_count", "rtmc_srg_get_params", "rtmc_srg_set_params",
    "rtmc_srg_gradient", "rtmc_srg_train_step", "rtmc_srg_train", "rtmc_srg_predict",
]


class RtmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"rtmc {_STATUS.get(status, status)}: {msg}")
        self.status = status


class Allocator(C.Structure):
    _fields_ = [("alloc", C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)),
                ("free", C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)), ("user", C.c_void_p)]


class Tables(C.Structure):
    _fields_ = [("n_E", C.c_int32), ("n_theta", C.c_int32), ("E_min", C.c_double), ("E_max", C.c_double),
                ("yield_", C.c_void_p), ("n_cdf", C.c_int32), ("cdf_E", C.c_void_p), ("cdf_F", C.c_void_p),
                ("Ec", C.c_double), ("esee", C.c_void_p), ("emission", C.c_int32)]


class TraceOpts(C.Structure):
    _fields_ = [("max_gen", C.c_int32), ("n_ebins", C.c_int32), ("n_abins", C.c_int32), ("pid0", C.c_uint64),
                ("e_hist", C.c_void_p), ("a_hist", C.c_void_p), ("pp_escaped", C.c_void_p), ("n_zbins", C.c_int32),
                ("z_hist", C.c_void_p), ("replay", C.c_void_p), ("n_replay", C.c_int64), ("replay_gen", C.c_int32),
                ("n_replay_out", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("yield_", C.c_double), ("yield_sigma", C.c_double)] + \
               [(n, C.c_uint64) for n in ("n_primaries", "n_rays", "n_escaped", "n_absorbed", "n_truncated",
                                          "n_lost", "n_substrate", "n_wraps", "n_node_visits", "n_tri_tests",
                                          "n_spawned")] + \
               [("e_escaped", C.c_double), ("e_deposited", C.c_double), ("ms", C.c_double),
                ("kernel_ms", C.c_double), ("shade_ms", C.c_double), ("n_kernel_launches", C.c_uint64),
                ("n_chunks", C.c_int32)]

    def to_dict(self):
        return {f[0].rstrip("_"): getattr(self, f[0]) for f in self._fields_}


class LaunchCfg(C.Structure):
    _fields_ = [("block", C.c_int32), ("wg_per_cu", C.c_int32), ("lds_stack", C.c_int32), ("chunk", C.c_int32),
                ("refill", C.c_int32), ("occupancy", C.c_int32), ("claim", C.c_int32)]


class SceneInfo(C.Structure):
    _fields_ = [("n_tris_in", C.c_int64), ("n_tris", C.c_int64), ("n_dropped", C.c_int64), ("n_nodes", C.c_int64),
                ("bvh_built", C.c_int32), ("bvh_depth", C.c_int32), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("flags", C.c_uint32), ("build_ms", C.c_double)]


class Job(C.Structure):
    _fields_ = [("scene_id", C.c_int32), ("E_eV", C.c_double), ("theta_deg", C.c_double),
                ("n_primaries", C.c_uint64), ("seed", C.c_uint64), ("pp_escaped", C.c_void_p)]


_lib = None
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    # release device memory while torch's allocator is still alive
    for ctx in list(_live):
        ctx.close()


def load_library(path: str = LIB_PATH):
    """Load librtmc.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librtmc.so not built ({path}); run __graft_entry__.build()")
    lib = C.CDLL(path)
    P = C.c_void_p
    i32, i64, u32, u64, dbl = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    sig = {
        "rtmc_create": ([C.POINTER(P), C.c_int, C.POINTER(Allocator), P], C.c_int),
        "rtmc_destroy": ([P], None),
        "rtmc_last_error": ([P], C.c_char_p),
        "rtmc_set_stream": ([P, P], C.c_int),
        "rtmc_load_mesh": ([P, P, i64, P, i64, C.POINTER(dbl), C.POINTER(dbl), u32, C.POINTER(i32)], C.c_int),
        "rtmc_build_bvh": ([P, i32], C.c_int),
        "rtmc_get_scene_info": ([P, i32, C.POINTER(SceneInfo)], C.c_int),
        "rtmc_bvh_download": ([P, i32, P, P], C.c_int),
        "rtmc_bvh_download_wide": ([P, i32, P], C.c_int),
        "rtmc_load_tables": ([P, C.POINTER(Tables), C.POINTER(i32)], C.c_int),
        "rtmc_trace": ([P, i32, i32, dbl, dbl, u64, u64, C.POINTER(TraceOpts), C.POINTER(Result)], C.c_int),
        "rtmc_trace_batch": ([P, i32, C.POINTER(Job), i64, i32, C.POINTER(Result)], C.c_int),
        "rtmc_first_hit": ([P, i32, P, i64, P, P], C.c_int),
        "rtmc_first_hit_noalloc": ([P, i32, P, i64, P, P], C.c_int),
        "rtmc_sort_pairs_u64": ([P, P, P, i64, i32], C.c_int),
        "rtmc_set_launch": ([P, C.POINTER(LaunchCfg)], C.c_int),
        "rtmc_get_launch": ([P, C.POINTER(LaunchCfg)], C.c_int),
        "rtmc_autotune": ([P, i32, i32, dbl, dbl, u64, C.POINTER(LaunchCfg)], C.c_int),
        "rtmc_copy_probe": ([P, P, P, C.c_size_t, i32, C.POINTER(dbl)], C.c_int),
        "rtmc_srg_create": ([P, i32, i32, i32, u64, C.POINTER(i32)], C.c_int),
        "rtmc_srg_param_count": ([P, i32, C.POINTER(i64)], C.c_int),
        "rtmc_srg_get_params": ([P, i32, P, i64], C.c_int),
        "rtmc_srg_set_params": ([P, i32, P, i64], C.c_int),
        "rtmc_srg_gradient": ([P, i32, P, P, i64, C.POINTER(C.c_float), P], C.c_int),
        "rtmc_srg_train_step": ([P, i32, P, P, i64, C.c_float, C.c_float, C.POINTER(C.c_float)], C.c_int),
        "rtmc_srg_train": ([P, i32, P, P, i64, i64, i32, P, C.c_float, u64, i32, P], C.c_int),
        "rtmc_srg_predict": ([P, i32, P, i64, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


class Context:
    """One library context on one GPU; device memory comes from torch."""

    def __init__(self, device: int = 0, use_torch_allocator: bool = True):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the RTMC library runs only on the GPU")
        self.lib = load_library()
        self.torch = torch
        self.device = device
        torch.cuda.set_device(device)
        stream = torch.cuda.current_stream(device)
        self._alloc = None
        if use_torch_allocator:
            dev = device

            def _a(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, torch.cuda.current_stream(dev))
                except Exception:
                    return None

            def _f(p, user):
                if torch is not None and torch.cuda is not None:
                    torch.cuda.caching_allocator_delete(p)

            self._alloc = Allocator(Allocator._fields_[0][1](_a), Allocator._fields_[1][1](_f), None)
        h = C.c_void_p()
        st = self.lib.rtmc_create(C.byref(h), device, C.byref(self._alloc) if self._alloc else None,
                                  C.c_void_p(stream.cuda_stream))
        if st != 0:
            raise RtmcError(st, "rtmc_create failed")
        self.h = h
        _live.add(self)

    def close(self):
        if getattr(self, "h", None):
            self.lib.rtmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        if st != 0:
            raise RtmcError(st, self.lib.rtmc_last_error(self.h).decode())

    # ---------------------------------------------------------------- scenes
    def load_mesh(self, verts, tris, box_lo, box_hi, flags: int) -> int:
        v = np.ascontiguousarray(verts, dtype=np.float32)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        lo = (C.c_double * 3)(*[float(x) for x in box_lo])
        hi = (C.c_double * 3)(*[float(x) for x in box_hi])
        sid = C.c_int32()
        self._chk(self.lib.rtmc_load_mesh(self.h, _ptr(v), v.shape[0], _ptr(t), t.shape[0], lo, hi, int(flags),
                                          C.byref(sid)))
        return sid.value

    def load_scene(self, mesh, build: bool = True) -> int:
        sid = self.load_mesh(mesh.verts, mesh.tris, mesh.box_lo, mesh.box_hi, mesh.flags)
        if build:
            self.build_bvh(sid)
        return sid

    def build_bvh(self, scene: int):
        self._chk(self.lib.rtmc_build_bvh(self.h, scene))

    def scene_info(self, scene: int) -> dict:
        si = SceneInfo()
        self._chk(self.lib.rtmc_get_scene_info(self.h, scene, C.byref(si)))
        d = {f[0]: getattr(si, f[0]) for f in SceneInfo._fields_}
        d["lo"] = tuple(si.lo)
        d["hi"] = tuple(si.hi)
        return d

    def bvh_download(self, scene: int):
        info = self.scene_info(scene)
        nodes = np.zeros((info["n_nodes"], 16), dtype=np.float32)
        tris = np.zeros((info["n_tris"], 12), dtype=np.float32)
        self._chk(self.lib.rtmc_bvh_download(self.h, scene, _ptr(nodes), _ptr(tris)))
        return nodes, tris

    def bvh_download_wide(self, scene: int):
        """The 4-wide nodes traversal reads, as uint32 [n_nodes, 16]."""
        info = self.scene_info(scene)
        wide = np.zeros((info["n_nodes"], 16), dtype=np.uint32)
        self._chk(self.lib.rtmc_bvh_download_wide(self.h, scene, _ptr(wide)))
        return wide

    # ---------------------------------------------------------------- tables
    def load_tables(self, tab) -> int:
        y = np.ascontiguousarray(tab.yld, dtype=np.float32)
        ce = np.ascontiguousarray(tab.cdf_E, dtype=np.float32)
        cf = np.ascontiguousarray(tab.cdf_F, dtype=np.float32)
        emission = int(getattr(tab, "emission", 0))
        es = getattr(tab, "esee", None)
        es = np.ascontiguousarray(es, dtype=np.float32) if es is not None else None
        t = Tables(y.shape[0], y.shape[1], float(tab.E_min), float(tab.E_max), _ptr(y).value, ce.shape[0],
                   _ptr(ce).value, _ptr(cf).value, float(tab.Ec), _ptr(es).value if es is not None else None,
                   emission)
        tid = C.c_int32()
        self._chk(self.lib.rtmc_load_tables(self.h, C.byref(t), C.byref(tid)))
        return tid.value

    # ---------------------------------------------------------------- tracing
    def trace(self, scene: int, table: int, E: float, theta: float, n_primaries: int, seed: int, max_gen: int = 6,
              n_ebins: int = 256, n_abins: int = 90, pid0: int = 0, per_primary=None, n_zbins: int = 0,
              replay=None, replay_gen: int = 1) -> dict:
        """Full RTMC; per_primary may be a uint32/int32 torch tensor of n_primaries on the GPU;
        n_zbins > 0 adds the absorption-depth histogram ("z_hist"); replay may be a float32
        [n, 6] GPU tensor that receives rays of generation replay_gen as queued ("n_replay")."""
        eh = np.zeros(n_ebins, dtype=np.uint64)
        ah = np.zeros(n_abins, dtype=np.uint64)
        zh = np.zeros(max(n_zbins, 1), dtype=np.uint64)
        pp = per_primary.data_ptr() if per_primary is not None else None
        nrep = C.c_int64(0)
        if replay is not None:
            assert replay.is_cuda and replay.is_contiguous() and replay.dtype == self.torch.float32
            assert replay.dim() == 2 and replay.shape[1] == 6
        o = TraceOpts(int(max_gen), int(n_ebins), int(n_abins), int(pid0), _ptr(eh).value, _ptr(ah).value, pp,
                      int(n_zbins), _ptr(zh).value, replay.data_ptr() if replay is not None else None,
                      int(replay.shape[0]) if replay is not None else 0, int(replay_gen),
                      C.cast(C.pointer(nrep), C.c_void_p).value)
        r = Result()
        self._chk(self.lib.rtmc_trace(self.h, scene, table, float(E), float(theta), int(n_primaries), int(seed),
                                      C.byref(o), C.byref(r)))
        d = r.to_dict()
        d["e_hist"] = eh
        d["a_hist"] = ah
        if n_zbins:
            d["z_hist"] = zh
        if replay is not None:
            d["n_replay"] = int(nrep.value)
        return d

    def trace_batch(self, table: int, jobs, max_gen: int = 6, per_primary=None) -> list:
        """jobs: iterable of (scene, E, theta, n_primaries, seed).  per_primary,
        if given, is a list with one entry per job: None or a uint32/int32
        torch tensor of n_primaries on the GPU for that job's escape counts."""
        jl = list(jobs)
        pps = list(per_primary) if per_primary is not None else [None] * len(jl)
        if len(pps) != len(jl):
            raise ValueError("per_primary needs one entry per job")
        for (s, E, th, n, sd), p in zip(jl, pps):
            if p is not None:
                assert p.is_cuda and p.is_contiguous() and p.numel() >= int(n) and p.element_size() == 4
        arr = (Job * len(jl))(*[Job(int(s), float(E), float(th), int(n), int(sd),
                                    p.data_ptr() if p is not None else None)
                                for (s, E, th, n, sd), p in zip(jl, pps)])
        outs = (Result * len(jl))()
        self._chk(self.lib.rtmc_trace_batch(self.h, table, arr, len(jl), int(max_gen), outs))
        return [o.to_dict() for o in outs]

    def first_hit(self, scene: int, rays):
        """rays: float32 torch tensor [n, 6] on the GPU; returns (tri int32, t float32) tensors."""
        torch = self.torch
        assert rays.is_cuda and rays.dtype == torch.float32 and rays.is_contiguous() and rays.shape[-1] == 6
        n = rays.shape[0]
        tri = torch.empty(n, dtype=torch.int32, device=rays.device)
        t = torch.empty(n, dtype=torch.float32, device=rays.device)
        self._chk(self.lib.rtmc_first_hit(self.h, scene, C.c_void_p(rays.data_ptr()), n, C.c_void_p(tri.data_ptr()),
                                          C.c_void_p(t.data_ptr())))
        return tri, t

    def first_hit_noalloc(self, scene: int, rays, tri, t):
        """rtmc_first_hit_noalloc into caller tensors tri (int32) and t
        (float32) of at least rays.shape[0] entries; asynchronous."""
        torch = self.torch
        assert rays.is_cuda and rays.dtype == torch.float32 and rays.is_contiguous() and rays.shape[-1] == 6
        n = rays.shape[0]
        assert tri.dtype == torch.int32 and t.dtype == torch.float32 and tri.numel() >= n and t.numel() >= n
        self._chk(self.lib.rtmc_first_hit_noalloc(self.h, scene, C.c_void_p(rays.data_ptr()), n,
                                                  C.c_void_p(tri.data_ptr()), C.c_void_p(t.data_ptr())))

    def sort_pairs(self, keys, vals, key_bits: int = 64):
        """In-place device radix sort of int64 keys (as uint64 bits) with int32 values."""
        torch = self.torch
        assert keys.is_cuda and keys.dtype == torch.int64 and vals.dtype == torch.int32
        assert keys.is_contiguous() and vals.is_contiguous() and keys.numel() == vals.numel()
        self._chk(self.lib.rtmc_sort_pairs_u64(self.h, C.c_void_p(keys.data_ptr()), C.c_void_p(vals.data_ptr()),
                                               keys.numel(), int(key_bits)))

    def set_stream(self, stream):
        """Enqueue later work on a torch.cuda.Stream (use it as torch's current
        stream too, so the caching allocator's stream matches)."""
        self._chk(self.lib.rtmc_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def set_launch(self, block: int, wg_per_cu: int, lds_stack: int, chunk: int, refill: int = 48, occupancy: int = 0,
                   claim: int = 0):
        self._chk(self.lib.rtmc_set_launch(self.h, C.byref(LaunchCfg(block, wg_per_cu, lds_stack, chunk, refill,
                                                                     occupancy, claim))))

    def get_launch(self) -> dict:
        c = LaunchCfg()
        self._chk(self.lib.rtmc_get_launch(self.h, C.byref(c)))
        return {f[0]: getattr(c, f[0]) for f in LaunchCfg._fields_}

    def autotune(self, scene: int, table: int, E: float, theta: float, n_primaries: int) -> dict:
        c = LaunchCfg()
        self._chk(self.lib.rtmc_autotune(self.h, scene, table, float(E), float(theta), int(n_primaries),
                                         C.byref(c)))
        return {f[0]: getattr(c, f[0]) for f in LaunchCfg._fields_}

    def copy_probe(self, nbytes: int, reps: int = 10) -> float:
        """Achievable device copy bandwidth in GB/s (read + write bytes)."""
        torch = self.torch
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=f"cuda:{self.device}")
        dst = torch.empty_like(src)
        ms = C.c_double()
        self._chk(self.lib.rtmc_copy_probe(self.h, C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                                           src.numel() * 4, int(reps), C.byref(ms)))
        return 2.0 * nbytes / (ms.value * 1e-3) / 1e9

    # ---------------------------------------------------------------- surrogate
    def srg_create(self, n_in: int = 8, width: int = 256, depth: int = 4, seed: int = 0) -> int:
        sid = C.c_int32()
        self._chk(self.lib.rtmc_srg_create(self.h, n_in, width, depth, int(seed), C.byref(sid)))
        return sid.value

    def srg_params(self, srg: int) -> np.ndarray:
        n = C.c_int64()
        self._chk(self.lib.rtmc_srg_param_count(self.h, srg, C.byref(n)))
        p = np.zeros(n.value, dtype=np.float32)
        self._chk(self.lib.rtmc_srg_get_params(self.h, srg, _ptr(p), p.size))
        return p

    def srg_set_params(self, srg: int, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._chk(self.lib.rtmc_srg_set_params(self.h, srg, _ptr(p), p.size))

    def _dev(self, a):
        torch = self.torch
        t = torch.as_tensor(a, dtype=torch.float32)
        return t.to(f"cuda:{self.device}").contiguous()

    def srg_gradient(self, srg: int, X, y):
        """Loss and gradient (public parameter order) of one batch, no update."""
        Xd, yd = self._dev(X), self._dev(y)
        n = self.srg_params(srg).size
        g = np.zeros(n, dtype=np.float32)
        loss = C.c_float()
        self._chk(self.lib.rtmc_srg_gradient(self.h, srg, C.c_void_p(Xd.data_ptr()), C.c_void_p(yd.data_ptr()),
                                             Xd.shape[0], C.byref(loss), _ptr(g)))
        return loss.value, g

    def srg_train_step(self, srg: int, X, y, lr: float, weight_decay: float = 0.0) -> float:
        """X, y: torch tensors on the GPU (float32) or arrays."""
        Xd = X if getattr(X, "is_cuda", False) else self._dev(X)
        yd = y if getattr(y, "is_cuda", False) else self._dev(y)
        loss = C.c_float()
        self._chk(self.lib.rtmc_srg_train_step(self.h, srg, C.c_void_p(Xd.data_ptr()), C.c_void_p(yd.data_ptr()),
                                               Xd.shape[0], float(lr), float(weight_decay), C.byref(loss)))
        return loss.value

    def srg_train(self, srg: int, X, y, batch: int, lr, weight_decay: float = 0.0, seed: int = 0,
                  use_graph: bool = True):
        """Device training loop: len(lr) AdamW steps on batches drawn from (X, y)
        on the GPU; returns the batch losses (numpy float32, one per step)."""
        Xd = X if getattr(X, "is_cuda", False) else self._dev(X)
        yd = y if getattr(y, "is_cuda", False) else self._dev(y)
        assert Xd.is_contiguous() and yd.is_contiguous() and Xd.shape[0] == yd.shape[0]
        lr_h = np.ascontiguousarray(lr, dtype=np.float32).reshape(-1)
        losses = np.zeros(lr_h.size, dtype=np.float32)
        self._chk(self.lib.rtmc_srg_train(self.h, srg, C.c_void_p(Xd.data_ptr()), C.c_void_p(yd.data_ptr()),
                                          Xd.shape[0], int(batch), lr_h.size, _ptr(lr_h), float(weight_decay),
                                          int(seed), int(bool(use_graph)), _ptr(losses)))
        return losses

    def srg_predict(self, srg: int, X):
        """Returns a float32 GPU tensor of predictions."""
        Xd = X if getattr(X, "is_cuda", False) else self._dev(X)
        y = self.torch.empty(Xd.shape[0], dtype=self.torch.float32, device=Xd.device)
        self._chk(self.lib.rtmc_srg_predict(self.h, srg, C.c_void_p(Xd.data_ptr()), Xd.shape[0],
                                            C.c_void_p(y.data_ptr())))
        return y

