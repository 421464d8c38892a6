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

from .inputs import EVENT_DTYPE, LOOP_DTYPE, REC_DTYPE

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsemipar.so")

FLAT, MATTER, RADIATION = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
SCREEN_F64, SCREEN_F32 = 0, 1
FLAG_HAS_R, FLAG_FROZEN, FLAG_ACTIVE, FLAG_REMOVED = 1, 2, 4, 8
EVENT_EXCHANGE, EVENT_PASSED = 0, 1  # semipar_event.kind
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
                ("screen_split", ctypes.c_int32), ("loop_every", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("p", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("cell_factor", ctypes.c_double)]


class EvolveStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("point_steps", ctypes.c_int64),
                ("candidates", ctypes.c_int64), ("confirmed", ctypes.c_int64),
                ("accepted", ctypes.c_int64), ("large_elements", ctypes.c_int64),
                ("final_step", ctypes.c_int32), ("done", ctypes.c_int32),
                ("elapsed_ms", ctypes.c_double), ("timed_kernel_ms", ctypes.c_double),
                ("timed_kernel_launches", ctypes.c_int64), ("loops", ctypes.c_int64),
                ("loop_points", ctypes.c_int64), ("resolve_rounds", ctypes.c_int64),
                ("passed", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Tiling(ctypes.Structure):
    _fields_ = [("n_regions", ctypes.c_int32), ("cosmology", ctypes.c_int32),
                ("box", ctypes.c_double), ("surfaces", ctypes.c_void_p),
                ("geoms", ctypes.c_void_p), ("n_pred", ctypes.c_void_p),
                ("succ_off", ctypes.c_void_p), ("succ", ctypes.c_void_p),
                ("stream", ctypes.c_void_p)]


class SchedParams(ctypes.Structure):
    _fields_ = [("policy", ctypes.c_int32), ("out_mem", ctypes.c_int32),
                ("batch_points", ctypes.c_int64), ("cost", ctypes.c_void_p),
                ("evolve", EvolveParams), ("out", ctypes.c_void_p), ("out_off", ctypes.c_void_p),
                ("events", ctypes.c_void_p), ("events_cap", ctypes.c_int64),
                ("events_off", ctypes.c_void_p), ("region_steps", ctypes.c_void_p),
                ("region_point_steps", ctypes.c_void_p), ("region_batch", ctypes.c_void_p),
                ("region_ms", ctypes.c_void_p), ("lanes", ctypes.c_int32),
                ("pack", ctypes.c_int32), ("loops", ctypes.c_void_p),
                ("loops_cap", ctypes.c_int64), ("loops_off", ctypes.c_void_p),
                ("lane_sleep_ms", ctypes.c_double), ("lane_submit_ms", ctypes.c_double)]


class SchedStats(ctypes.Structure):
    _fields_ = [("regions", ctypes.c_int64), ("empty_regions", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("point_steps", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("events", ctypes.c_int64),
                ("makespan_ms", ctypes.c_double), ("evolve_ms", ctypes.c_double),
                ("timed_kernel_ms", ctypes.c_double), ("timed_kernel_launches", ctypes.c_int64),
                ("loops", ctypes.c_int64), ("passed", ctypes.c_int64),
                ("lane_held_ms", ctypes.c_double), ("lane_busy_ms", ctypes.c_double),
                ("lanes_started", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Handoff(ctypes.Structure):
    _fields_ = [("n_regions", ctypes.c_int32), ("cosmology", ctypes.c_int32),
                ("box", ctypes.c_double), ("geoms", ctypes.c_void_p),
                ("n_pred", ctypes.c_void_p), ("succ_off", ctypes.c_void_p),
                ("succ", ctypes.c_void_p), ("ic", ctypes.c_void_p),
                ("n_points", ctypes.c_int64), ("ic_mem", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("hist", ctypes.c_void_p),
                ("hist_slices", ctypes.c_int64), ("stream", ctypes.c_void_p)]


SCHED_PLAIN, SCHED_BATCHED = 0, 1
PACK_POINTS, PACK_WORK = 0, 1
MLP_IN, MLP_HIDDEN, MLP_PARAMS = 12, 64, 5057
PERSISTENT_MAX = 512  # SEMIPAR_PERSISTENT_MAX
PERSISTENT_EVENTS = 160  # SEMIPAR_PERSISTENT_EVENTS

# exported symbols declared in include/semipar.h
SYMBOLS = ["region_init_from_surfaces", "region_evolve", "region_emit_final_surfaces",
           "region_events", "region_candidates", "region_loops", "region_destroy", "semipar_strerror", "semipar_version",
           "semipar_last_error", "schedule_regions", "schedule_handoff",
           "semipar_region_features",
           "semipar_mlp_forward", "semipar_mlp_loss_grad", "semipar_mlp_loss_grad_noalloc",
           "semipar_mlp_adam_step",
           "semipar_mlp_train", "semipar_mlp_norm"]

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
        L.region_candidates.argtypes = [P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.region_candidates.restype = ctypes.c_int
        L.region_loops.argtypes = [P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.region_loops.restype = ctypes.c_int
        L.region_destroy.argtypes = [P]
        L.region_destroy.restype = None
        L.semipar_strerror.argtypes = [ctypes.c_int]
        L.semipar_strerror.restype = ctypes.c_char_p
        L.semipar_version.argtypes = []
        L.semipar_version.restype = ctypes.c_char_p
        L.semipar_last_error.argtypes = []
        L.semipar_last_error.restype = ctypes.c_char_p
        L.schedule_regions.argtypes = [ctypes.POINTER(Tiling), ctypes.POINTER(SchedParams),
                                       ctypes.POINTER(SchedStats)]
        L.schedule_regions.restype = ctypes.c_int
        L.schedule_handoff.argtypes = [ctypes.POINTER(Handoff), ctypes.POINTER(SchedParams),
                                       ctypes.POINTER(SchedStats)]
        L.schedule_handoff.restype = ctypes.c_int
        L.semipar_region_features.argtypes = [ctypes.POINTER(Tiling), P]
        L.semipar_region_features.restype = ctypes.c_int
        L.semipar_mlp_forward.argtypes = [P, P, P, ctypes.c_int64, P, P]
        L.semipar_mlp_forward.restype = ctypes.c_int
        L.semipar_mlp_loss_grad.argtypes = [P, P, P, P, ctypes.c_int64, P, P, P]
        L.semipar_mlp_loss_grad.restype = ctypes.c_int
        L.semipar_mlp_loss_grad_noalloc.argtypes = [P, P, P, P, ctypes.c_int64, P, P, P]
        L.semipar_mlp_loss_grad_noalloc.restype = ctypes.c_int
        L.semipar_mlp_adam_step.argtypes = [P, P, P, P, ctypes.c_int64, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, ctypes.c_float, P]
        L.semipar_mlp_adam_step.restype = ctypes.c_int
        L.semipar_mlp_train.argtypes = [P, P, P, P, P, P, ctypes.c_int64, ctypes.c_int32,
                                        ctypes.c_int64, ctypes.c_float, P, P]
        L.semipar_mlp_train.restype = ctypes.c_int
        L.semipar_mlp_norm.argtypes = [P, ctypes.c_int64, P]
        L.semipar_mlp_norm.restype = ctypes.c_int
        _lib = L
    return _lib


def last_error():
    """Text of the library's last recorded error on this thread ("" if none)."""
    return lib().semipar_last_error().decode()


def _check(rc, what):
    if rc != 0:
        msg = lib().semipar_last_error().decode()
        if msg:
            what = f"{what} [{msg}]"
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
               events_per_point=0.0, timed_kernel=-1, screen_split=0, loop_every=0, p=1.0,
               seed=0, persistent=0, cell_factor=0.0):
        """p: intercommutation probability in (0, 1]; seed: key of the crossings' draws;
        persistent: evolve a batch of small regions by persistent workgroups;
        cell_factor: cell edge over the largest element extent (0: the default)."""
        prm = EvolveParams(int(max_steps), float(t_end), int(screen), int(bool(intercommute)),
                           float(cell_size), int(steps_per_sync), int(bool(use_graph)),
                           float(cand_per_point), float(events_per_point), int(timed_kernel),
                           int(screen_split), int(loop_every), int(persistent), float(p),
                           int(seed), float(cell_factor))
        st = EvolveStats()
        _check(lib().region_evolve(self.h, ctypes.byref(prm), ctypes.byref(st)), "region_evolve")
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

    def candidates(self):
        """Pairs that passed the screen in the last step, (n, 2) int64 id pairs
        (smaller id first), sorted."""
        L = lib()
        n = ctypes.c_int64()
        _check(L.region_candidates(self.h, None, 0, ctypes.byref(n)), "region_candidates (count)")
        out = np.zeros((n.value, 2), dtype=np.int64)
        if n.value:
            _check(L.region_candidates(self.h, out.ctypes.data, n.value, ctypes.byref(n)),
                   "region_candidates")
        return out[:n.value]

    def loops(self):
        """Loops recorded and removed since init, sorted by (step, rep_id)."""
        L = lib()
        n = ctypes.c_int64()
        _check(L.region_loops(self.h, None, 0, ctypes.byref(n)), "region_loops (count)")
        out = np.zeros(n.value, dtype=LOOP_DTYPE)
        if n.value:
            _check(L.region_loops(self.h, out.ctypes.data, n.value, ctypes.byref(n)),
                   "region_loops")
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


# ---- many regions ----------------------------------------------------------------

class RegionSet:
    """Regions of a tiling, packed for schedule_regions / region_features.

    recs: all regions' records concatenated (numpy REC_DTYPE on the host, or a torch
    uint8 CUDA tensor of 160-byte records); counts[r]: records of region r;
    geoms[r]: (origin[4], inv2g, idx[4]) as produced by inputs.region_geometry.
    n_pred / succ: optional dependency lists (succ[r] = list of successors of r).
    """

    def __init__(self, recs, counts, geoms, box, cosmology, n_pred=None, succ=None):
        self.counts = np.asarray(counts, dtype=np.int64)
        nr = len(self.counts)
        self.box, self.cosmology = float(box), int(cosmology)
        if isinstance(recs, np.ndarray):
            self.recs = np.ascontiguousarray(recs, dtype=REC_DTYPE)
            base, mem = self.recs.ctypes.data, MEM_HOST
        else:
            assert recs.is_cuda and recs.numel() % REC_DTYPE.itemsize == 0
            self.recs = recs
            base, mem = recs.data_ptr(), MEM_DEVICE
        assert int(self.counts.sum()) * REC_DTYPE.itemsize == (
            self.recs.nbytes if mem == MEM_HOST else recs.numel())
        self.mem = mem
        self.surfs = (Surface * max(nr, 1))()
        off = np.concatenate([[0], np.cumsum(self.counts)])
        self.offsets = off
        for r in range(nr):
            n = int(self.counts[r])
            self.surfs[r] = Surface(base + int(off[r]) * REC_DTYPE.itemsize if n else None, n, -1, mem)
        self.geoms = (RegionGeom * max(nr, 1))()
        for r in range(nr):
            self.geoms[r] = _geom_struct(geoms[r])
        self.n_regions = nr
        self._dag = None
        if n_pred is not None:
            npred = np.ascontiguousarray(n_pred, dtype=np.int32)
            so = np.zeros(nr + 1, dtype=np.int32)
            flat = []
            for r in range(nr):
                flat.extend(int(x) for x in succ[r])
                so[r + 1] = len(flat)
            sl = np.ascontiguousarray(flat if flat else [0], dtype=np.int32)
            self._dag = (npred, so, sl)

    def tiling(self, stream=None):
        t = Tiling()
        t.n_regions = self.n_regions
        t.cosmology = self.cosmology
        t.box = self.box
        t.surfaces = ctypes.cast(self.surfs, ctypes.c_void_p)
        t.geoms = ctypes.cast(self.geoms, ctypes.c_void_p)
        if self._dag is not None:
            t.n_pred = self._dag[0].ctypes.data
            t.succ_off = self._dag[1].ctypes.data
            t.succ = self._dag[2].ctypes.data
        if stream is None and self.mem == MEM_DEVICE:
            stream = _current_stream()
        t.stream = stream
        return t

    @classmethod
    def from_parts(cls, parts, box, cosmology, device=False, **kw):
        """parts = [(recs, geom)]; device=True uploads the records to the current GPU."""
        counts = [len(p[0]) for p in parts]
        recs = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, REC_DTYPE)
        if device:
            import torch
            recs = torch.from_numpy(recs.view(np.uint8).copy()).cuda()
        return cls(recs, counts, [p[1] for p in parts], box, cosmology, **kw)


def region_features(rs, stream=None):
    """12 cost-model features per region (numpy float32, n_regions x 12), on the GPU."""
    feat = np.zeros((max(rs.n_regions, 1), MLP_IN), dtype=np.float32)
    t = rs.tiling(stream)
    _check(lib().semipar_region_features(ctypes.byref(t), feat.ctypes.data), "region_features")
    return feat[:rs.n_regions]


def schedule_regions(rs, policy=SCHED_BATCHED, batch_points=0, cost=None, out="host",
                     events=True, stream=None, max_steps=10 ** 7, t_end=float("inf"),
                     screen=SCREEN_F64, intercommute=True, cell_size=0.0, steps_per_sync=0,
                     use_graph=False, cand_per_point=0.0, events_per_point=0.0,
                     screen_split=0, timed_kernel=-1, lanes=1, loop_every=0,
                     pack=PACK_POINTS, p=1.0, seed=0, persistent=0, cell_factor=0.0,
                     lane_sleep_ms=0.0, lane_submit_ms=0.0):
    """Run every region of rs; returns a dict with the stats, per-region logs, output
    records (out = "host": numpy; "device": torch uint8 CUDA tensor; None: not
    written), their offsets (4 per region + 1) and the events with offsets."""
    L = lib()
    nr = rs.n_regions
    p_ic = float(p)  # the name p is the parameter block below
    p = SchedParams()
    p.policy = int(policy)
    p.batch_points = int(batch_points)
    p.lanes = int(lanes)
    p.pack = int(pack)
    p.lane_sleep_ms = float(lane_sleep_ms)
    p.lane_submit_ms = float(lane_submit_ms)
    cost_arr = None
    if cost is not None:
        cost_arr = np.ascontiguousarray(cost, dtype=np.float32)
        assert len(cost_arr) == nr
        p.cost = cost_arr.ctypes.data
    p.evolve = EvolveParams(int(max_steps), float(t_end), int(screen), int(bool(intercommute)),
                            float(cell_size), int(steps_per_sync), int(bool(use_graph)),
                            float(cand_per_point), float(events_per_point), int(timed_kernel),
                            int(screen_split), int(loop_every), int(persistent), p_ic,
                            int(seed), float(cell_factor))
    total = int(rs.counts.sum())
    out_off = np.zeros(4 * nr + 1, dtype=np.int64)
    res = {}
    if out == "host":
        o = np.zeros(total, dtype=REC_DTYPE)
        p.out, p.out_mem = (o.ctypes.data if total else None), MEM_HOST
        res["out"] = o
    elif out == "device":
        import torch
        o = torch.empty(max(total, 1) * REC_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        p.out, p.out_mem = o.data_ptr(), MEM_DEVICE
        res["out"] = o
    p.out_off = out_off.ctypes.data
    ev_off = np.zeros(nr + 1, dtype=np.int64)
    ev_cap = max(2 * total, 4096)
    ev = np.zeros(ev_cap, dtype=EVENT_DTYPE) if events else None
    if events:
        p.events, p.events_cap, p.events_off = ev.ctypes.data, ev_cap, ev_off.ctypes.data
    lp_off = np.zeros(nr + 1, dtype=np.int64)
    lp_cap = max(total, 1024)
    lp = np.zeros(lp_cap, dtype=LOOP_DTYPE) if loop_every else None
    if loop_every:
        p.loops, p.loops_cap, p.loops_off = lp.ctypes.data, lp_cap, lp_off.ctypes.data
    steps = np.zeros(max(nr, 1), dtype=np.int32)
    psteps = np.zeros(max(nr, 1), dtype=np.int64)
    batch = np.zeros(max(nr, 1), dtype=np.int32)
    ms = np.zeros(max(nr, 1), dtype=np.float64)
    p.region_steps, p.region_point_steps = steps.ctypes.data, psteps.ctypes.data
    p.region_batch, p.region_ms = batch.ctypes.data, ms.ctypes.data
    st = SchedStats()
    t = rs.tiling(stream)
    _check(L.schedule_regions(ctypes.byref(t), ctypes.byref(p), ctypes.byref(st)),
           "schedule_regions")
    res.update(stats=st.as_dict(), out_off=out_off, region_steps=steps[:nr],
               region_point_steps=psteps[:nr], region_batch=batch[:nr], region_ms=ms[:nr])
    if events:
        if st.events > ev_cap:
            raise SemiparError(-5, f"schedule_regions: {st.events} events > buffer {ev_cap}")
        res["events"], res["events_off"] = ev[:st.events], ev_off
    if loop_every:
        res["loops"], res["loops_off"] = lp[:st.loops], lp_off
    return res


def schedule_handoff(ic, box, cosmology, geoms, n_pred, succ, hist, batch_points=0,
                     cost=None, events=True, stream=None, max_steps=0, screen=SCREEN_F64,
                     intercommute=True, cell_size=0.0, steps_per_sync=0, use_graph=False,
                     cand_per_point=0.0, events_per_point=0.0, timed_kernel=-1, seed=0,
                     cell_factor=0.0, screen_split=0, lanes=1):
    """Run a periodic tiling region by region with hand-off (schedule_handoff).

    ic: the volume's initial surface (numpy records); geoms: per region (origin[4],
    inv2g, idx[4]); n_pred, succ: predecessor counts and successor lists; hist: a CUDA
    float64 tensor of shape (slices, n_points, 4), the world sheet (filled by the call).
    Returns a dict with the stats, per-region logs and the events with offsets."""
    import torch
    L = lib()
    ic = np.ascontiguousarray(ic, dtype=REC_DTYPE)
    n = len(ic)
    nr = len(geoms)
    assert hist.is_cuda and hist.dtype == torch.float64 and hist.is_contiguous()
    assert hist.dim() == 3 and hist.shape[1] == n and hist.shape[2] == 4
    garr = (RegionGeom * max(nr, 1))()
    for r, gm in enumerate(geoms):
        garr[r] = _geom_struct(gm)
    npred = np.ascontiguousarray(n_pred, dtype=np.int32)
    off = np.zeros(nr + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(x) for x in succ])
    flat = np.ascontiguousarray(np.concatenate([np.asarray(x, np.int32) for x in succ])
                                if off[-1] else np.zeros(1, np.int32))
    h = Handoff()
    h.n_regions, h.cosmology, h.box = nr, int(cosmology), float(box)
    h.geoms = ctypes.addressof(garr)
    h.n_pred, h.succ_off, h.succ = npred.ctypes.data, off.ctypes.data, flat.ctypes.data
    h.ic, h.n_points, h.ic_mem = ic.ctypes.data, n, MEM_HOST
    h.hist, h.hist_slices = hist.data_ptr(), int(hist.shape[0])
    h.stream = stream if stream is not None else _current_stream()
    p = SchedParams()
    p.batch_points = int(batch_points)
    p.lanes = int(lanes)
    cost_arr = None
    if cost is not None:
        cost_arr = np.ascontiguousarray(cost, dtype=np.float32)
        assert len(cost_arr) == nr
        p.cost = cost_arr.ctypes.data
    p.evolve = EvolveParams(int(max_steps), float("inf"), int(screen), int(bool(intercommute)),
                            float(cell_size), int(steps_per_sync), int(bool(use_graph)),
                            float(cand_per_point), float(events_per_point), int(timed_kernel),
                            int(screen_split), 0, 0, 0.0, int(seed), float(cell_factor))
    ev_off = np.zeros(nr + 1, dtype=np.int64)
    ev_cap = max(n, 4096)
    ev = np.zeros(ev_cap, dtype=EVENT_DTYPE) if events else None
    if events:
        p.events, p.events_cap, p.events_off = ev.ctypes.data, ev_cap, ev_off.ctypes.data
    steps = np.zeros(max(nr, 1), dtype=np.int32)
    psteps = np.zeros(max(nr, 1), dtype=np.int64)
    batch = np.zeros(max(nr, 1), dtype=np.int32)
    ms = np.zeros(max(nr, 1), dtype=np.float64)
    p.region_steps, p.region_point_steps = steps.ctypes.data, psteps.ctypes.data
    p.region_batch, p.region_ms = batch.ctypes.data, ms.ctypes.data
    st = SchedStats()
    _check(L.schedule_handoff(ctypes.byref(h), ctypes.byref(p), ctypes.byref(st)),
           "schedule_handoff")
    res = dict(stats=st.as_dict(), region_steps=steps[:nr], region_point_steps=psteps[:nr],
               region_batch=batch[:nr], region_ms=ms[:nr])
    if events:
        if st.events > ev_cap:
            raise SemiparError(-5, f"schedule_handoff: {st.events} events > buffer {ev_cap}")
        res["events"], res["events_off"] = ev[:st.events], ev_off
    return res


# ---- cost model --------------------------------------------------------------------

class CostModel:
    """The 12 -> 64 -> 64 -> 1 ReLU cost model, trained and run by libsemipar's FP32
    kernels on the current GPU. params: numpy float32 (MLP_PARAMS) initial values."""

    def __init__(self, params, norm=None):
        import torch
        self.torch = torch
        self.params = torch.from_numpy(np.ascontiguousarray(params, np.float32)).cuda()
        assert self.params.numel() == MLP_PARAMS
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.norm = None if norm is None else torch.from_numpy(
            np.ascontiguousarray(norm, np.float32)).cuda()
        self.step = 0

    def _dev(self, a):
        return self.torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()

    def _np(self, p):
        return p.data_ptr() if p is not None else None

    def set_norm_from(self, x):
        x = np.ascontiguousarray(x, np.float32)
        norm = np.zeros(2 * MLP_IN, np.float32)
        _check(lib().semipar_mlp_norm(x.ctypes.data, len(x), norm.ctypes.data), "mlp_norm")
        self.norm = self._dev(norm)
        return norm

    def forward(self, x):
        xd = self._dev(x)
        y = self.torch.empty(len(x), dtype=self.torch.float32, device="cuda")
        _check(lib().semipar_mlp_forward(self._np(self.params), self._np(self.norm), self._np(xd),
                                         len(x), self._np(y), _current_stream()), "mlp_forward")
        return y.cpu().numpy()

    def loss_grad(self, x, target):
        xd, td = self._dev(x), self._dev(target)
        g = self.torch.empty(MLP_PARAMS, dtype=self.torch.float32, device="cuda")
        l = self.torch.empty(1, dtype=self.torch.float32, device="cuda")
        _check(lib().semipar_mlp_loss_grad(self._np(self.params), self._np(self.norm), self._np(xd),
                                           self._np(td), len(x), self._np(g), self._np(l),
                                           _current_stream()), "mlp_loss_grad")
        return float(l.cpu()[0]), g.cpu().numpy()

    def loss_grad_noalloc(self, x, target, grad=None, loss=None):
        """The same through semipar_mlp_loss_grad_noalloc: the library allocates
        nothing. x, target (and the optional outputs grad, loss) are device tensors
        the caller owns; returns (grad, loss) device tensors."""
        T = self.torch
        g = grad if grad is not None else T.empty(MLP_PARAMS, dtype=T.float32, device="cuda")
        l = loss if loss is not None else T.empty(1, dtype=T.float32, device="cuda")
        _check(lib().semipar_mlp_loss_grad_noalloc(
            self._np(self.params), self._np(self.norm), self._np(x), self._np(target), len(x),
            self._np(g), self._np(l), _current_stream()), "mlp_loss_grad_noalloc")
        return g, l

    def adam_step(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        gd = self._dev(grad)
        self.step += 1
        _check(lib().semipar_mlp_adam_step(self._np(self.params), self._np(self.m), self._np(self.v),
                                           self._np(gd), self.step, lr, beta1, beta2, eps,
                                           _current_stream()), "mlp_adam_step")

    def train(self, x, target, iters=2000, lr=1e-3):
        xd, td = self._dev(x), self._dev(target)
        loss = np.zeros(iters + 1, np.float32)
        _check(lib().semipar_mlp_train(self._np(self.params), self._np(self.m), self._np(self.v),
                                       self._np(self.norm), self._np(xd), self._np(td), len(x),
                                       int(iters), self.step, float(lr), loss.ctypes.data,
                                       _current_stream()), "mlp_train")
        self.step += iters
        return loss

    def get_params(self):
        return self.params.cpu().numpy()
