"""Thin Python binding of libsemipar (argument marshalling only).

Every step of the evolution runs in the library's HIP kernels. This module loads the
in-tree ``libsemipar.so`` (built by ``paper_1011_4046_amd.build``) and raises if it is
missing: there is no fallback implementation. PyTorch is used only to hand device
memory and the current stream to the library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .inputs import EVENT_DTYPE, REC_DTYPE

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsemipar.so")

FLAT, MATTER, RADIATION = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
SCREEN_F64, SCREEN_F32 = 0, 1
K_EVOLVE, K_SCAN, K_SCATTER, K_SCREEN, K_CONFIRM, K_RESOLVE = range(6)

ERRORS = {0: "ok", -1: "E_ARG", -2: "E_SURFACE", -3: "E_OOM", -4: "E_HIP",
          -5: "E_OVERFLOW", -6: "E_STATE"}


class SemiparError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({code})")
        self.code = code


class Surface(ctypes.Structure):
    _fields_ = [("recs", ctypes.c_void_p), ("n", ctypes.c_int64), ("face", ctypes.c_int32),
                ("mem", ctypes.c_int32)]


class RegionGeom(ctypes.Structure):
    _fields_ = [("idx", ctypes.c_int32 * 4), ("origin", ctypes.c_double * 4),
                ("inv2g", ctypes.c_double)]


def _geom_struct(geom):
    g = RegionGeom()
    for i in range(4):
        g.origin[i] = float(geom[i])
        g.idx[i] = int(geom[5 + i])
    g.inv2g = float(geom[4])
    return g


class RegionDesc(ctypes.Structure):
    _fields_ = [("cosmology", ctypes.c_int32), ("bounded", ctypes.c_int32),
                ("box", ctypes.c_double), ("capacity", ctypes.c_int64),
                ("stream", ctypes.c_void_p), ("idx", ctypes.c_int32 * 4),
                ("origin", ctypes.c_double * 4), ("inv2g", ctypes.c_double),
                ("n_sub", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("sub", ctypes.c_void_p)]


class EvolveParams(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int64), ("t_end", ctypes.c_double),
                ("screen", ctypes.c_int32), ("intercommute", ctypes.c_int32),
                ("cell_size", ctypes.c_double), ("steps_per_sync", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("cand_per_point", ctypes.c_double),
                ("events_per_point", ctypes.c_double), ("timed_kernel", ctypes.c_int32),
                ("screen_split", ctypes.c_int32)]


class EvolveStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("point_steps", ctypes.c_int64),
                ("candidates", ctypes.c_int64), ("confirmed", ctypes.c_int64),
                ("accepted", ctypes.c_int64), ("large_elements", ctypes.c_int64),
                ("final_step", ctypes.c_int32), ("done", ctypes.c_int32),
                ("elapsed_ms", ctypes.c_double), ("timed_kernel_ms", ctypes.c_double),
                ("timed_kernel_launches", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# exported symbols declared in include/semipar.h
SYMBOLS = ["region_init_from_surfaces", "region_evolve", "region_emit_final_surfaces",
           "region_events", "region_destroy", "semipar_strerror", "semipar_version",
           "semipar_last_error"]

_lib = None


def lib():
    """Load libsemipar.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1011_4046_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.region_init_from_surfaces.argtypes = [ctypes.POINTER(RegionDesc), ctypes.POINTER(Surface),
                                                ctypes.c_int, ctypes.POINTER(P)]
        L.region_init_from_surfaces.restype = ctypes.c_int
        L.region_evolve.argtypes = [P, ctypes.POINTER(EvolveParams), ctypes.POINTER(EvolveStats)]
        L.region_evolve.restype = ctypes.c_int
        L.region_emit_final_surfaces.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64),
                                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
        L.region_emit_final_surfaces.restype = ctypes.c_int
        L.region_events.argtypes = [P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.region_events.restype = ctypes.c_int
        L.region_destroy.argtypes = [P]
        L.region_destroy.restype = None
        L.semipar_strerror.argtypes = [ctypes.c_int]
        L.semipar_strerror.restype = ctypes.c_char_p
        L.semipar_version.argtypes = []
        L.semipar_version.restype = ctypes.c_char_p
        L.semipar_last_error.argtypes = []
        L.semipar_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        if rc == -4:
            what = f"{what} [{lib().semipar_last_error().decode()}]"
        raise SemiparError(rc, what)


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Region:
    """One region on the GPU, built from initial surfaces.

    ``recs``: a numpy REC_DTYPE array (host) or a torch uint8 CUDA tensor holding
    160-byte records (device-resident input).
    """

    @classmethod
    def batch(cls, parts, box, cosmology, stream=None):
        """One region holding many independent bounded regions: parts = [(recs, geom)]."""
        self = cls.__new__(cls)
        L = lib()
        surfs = (Surface * max(len(parts), 1))()
        geoms = (RegionGeom * max(len(parts), 1))()
        keep = []
        total = 0
        for i, (recs, geom) in enumerate(parts):
            recs = np.ascontiguousarray(recs, dtype=REC_DTYPE)
            keep.append(recs)
            surfs[i] = Surface(recs.ctypes.data if len(recs) else None, len(recs), -1, MEM_HOST)
            geoms[i] = _geom_struct(geom)
            total += len(recs)
        d = RegionDesc()
        d.cosmology, d.box, d.bounded = int(cosmology), float(box), 1
        d.stream = stream
        d.n_sub = len(parts)
        d.sub = ctypes.cast(geoms, ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(L.region_init_from_surfaces(ctypes.byref(d), surfs, len(parts), ctypes.byref(h)),
               "region_init_from_surfaces (batch)")
        self.h, self.n, self._keep = h, total, None
        return self

    def __init__(self, recs, box, cosmology, capacity=0, stream=None, geom=None):
        L = lib()
        if isinstance(recs, np.ndarray):
            recs = np.ascontiguousarray(recs, dtype=REC_DTYPE)
            ptr, n, mem = recs.ctypes.data, len(recs), MEM_HOST
            self._keep = recs
        else:  # torch tensor on the GPU
            assert recs.is_cuda and recs.numel() % REC_DTYPE.itemsize == 0
            ptr, n, mem = recs.data_ptr(), recs.numel() // REC_DTYPE.itemsize, MEM_DEVICE
            self._keep = recs
        if stream is None and mem == MEM_DEVICE:
            stream = _current_stream()
        d = RegionDesc()
        d.cosmology = int(cosmology)
        d.box = float(box)
        d.capacity = int(capacity)
        d.stream = stream if stream is not None else None
        if geom is not None:  # (origin[4], inv2g, idx[4])
            d.bounded = 1
            for i in range(4):
                d.origin[i] = float(geom[i])
                d.idx[i] = int(geom[5 + i])
            d.inv2g = float(geom[4])
        surf = Surface(ptr, n, -1, mem)
        h = ctypes.c_void_p()
        _check(L.region_init_from_surfaces(ctypes.byref(d), ctypes.byref(surf), 1, ctypes.byref(h)),
               "region_init_from_surfaces")
        self.h = h
        self.n = n
        self._keep = None

    def evolve(self, max_steps, t_end=float("inf"), screen=SCREEN_F64, intercommute=True,
               cell_size=0.0, steps_per_sync=0, use_graph=False, cand_per_point=0.0,
               events_per_point=0.0, timed_kernel=-1, screen_split=0):
        p = EvolveParams(int(max_steps), float(t_end), int(screen), int(bool(intercommute)),
                         float(cell_size), int(steps_per_sync), int(bool(use_graph)),
                         float(cand_per_point), float(events_per_point), int(timed_kernel),
                         int(screen_split))
        st = EvolveStats()
        _check(lib().region_evolve(self.h, ctypes.byref(p), ctypes.byref(st)), "region_evolve")
        return st.as_dict()

    def emit_faces(self):
        """Output surfaces: list of 4 host record arrays (one per final face)."""
        L = lib()
        n = (ctypes.c_int64 * 4)()
        _check(L.region_emit_final_surfaces(self.h, None, None, n, MEM_HOST), "emit (count)")
        outs = [np.zeros(n[f], dtype=REC_DTYPE) for f in range(4)]
        ptrs = (ctypes.c_void_p * 4)(*[o.ctypes.data if len(o) else None for o in outs])
        cap = (ctypes.c_int64 * 4)(*[len(o) for o in outs])
        _check(L.region_emit_final_surfaces(self.h, ptrs, cap, n, MEM_HOST), "emit")
        return outs

    def emit(self):
        """All output records (host numpy array): slot order for a whole-volume region,
        faces 0..3 concatenated for a bounded one."""
        return np.concatenate(self.emit_faces())

    def emit_device(self, out_tensor):
        """Write the final surface into a torch uint8 CUDA tensor (n*160 bytes)."""
        L = lib()
        n = (ctypes.c_int64 * 4)()
        ptrs = (ctypes.c_void_p * 4)(out_tensor.data_ptr(), None, None, None)
        cap = (ctypes.c_int64 * 4)(out_tensor.numel() // REC_DTYPE.itemsize, 0, 0, 0)
        _check(L.region_emit_final_surfaces(self.h, ptrs, cap, n, MEM_DEVICE), "emit (device)")
        return int(n[0])

    def events(self):
        L = lib()
        n = ctypes.c_int64()
        _check(L.region_events(self.h, None, 0, ctypes.byref(n)), "region_events (count)")
        out = np.zeros(n.value, dtype=EVENT_DTYPE)
        if n.value:
            _check(L.region_events(self.h, out.ctypes.data, n.value, ctypes.byref(n)),
                   "region_events")
        return out

    def close(self):
        if getattr(self, "h", None):
            lib().region_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version():
    return lib().semipar_version().decode()


def strerror(code):
    return lib().semipar_strerror(int(code)).decode()
