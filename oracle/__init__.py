"""CPU oracle for the string-network evolver -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product library (libsemipar) never
loads it. It shares no code with the HIP path: the C source ``oracle.c`` is
compiled by gcc with ``-O2 -ffp-contract=off`` and driven through ctypes.

Record and event layouts are restated here (they are the data format of the
initial and final surfaces, not shared code).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

REC = np.dtype([
    ("id", "<i8"), ("next_id", "<i8"), ("prev_id", "<i8"),
    ("step", "<i4"), ("flags", "<i4"),
    ("x", "<f8", (4,)), ("x_prev", "<f8", (4,)),
    ("r", "<f8", (4,)), ("r_prev", "<f8", (4,)),
])
EVT = np.dtype([
    ("step", "<i4"), ("kind", "<i4"), ("id_a", "<i8"), ("id_b", "<i8"),
    ("t_star", "<f8"), ("x_star", "<f8", (3,)),
])

LOOP = np.dtype([
    ("step", "<i4"), ("n_points", "<i4"), ("rep_id", "<i8"),
    ("energy", "<f8"), ("centre", "<f8", (3,)),
])

GRID, BRUTE = 0, 1
FLAG_HAS_R, FLAG_FROZEN, FLAG_ACTIVE, FLAG_REMOVED = 1, 2, 4, 8


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP for the per-point loops)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_create.argtypes = [P, i64, dbl, ctypes.c_int, dbl, ctypes.POINTER(P)]
        L.orc_create.restype = ctypes.c_int
        L.orc_evolve.argtypes = [P, i64, dbl, ctypes.c_int, ctypes.c_int, i32]
        L.orc_evolve.restype = ctypes.c_int
        L.orc_destroy.argtypes = [P]
        L.orc_destroy.restype = None
        L.orc_n.argtypes = [P]
        L.orc_n.restype = i64
        L.orc_step.argtypes = [P]
        L.orc_step.restype = i32
        L.orc_event_count.argtypes = [P]
        L.orc_event_count.restype = i64
        L.orc_events.argtypes = [P, P]
        L.orc_events.restype = ctypes.c_int
        L.orc_read.argtypes = [P, P]
        L.orc_read.restype = ctypes.c_int
        L.orc_stats.argtypes = [P, P]
        L.orc_stats.restype = None
        L.orc_band_candidates.argtypes = [P, ctypes.c_int, P, i64]
        L.orc_band_candidates.restype = i64
        L.orc_top.argtypes = [ctypes.c_int, dbl, dbl, P, P, P, P]
        L.orc_top.restype = None
        L.orc_det4.argtypes = [P, P, P, P]
        L.orc_det4.restype = dbl
        L.orc_tri_tri.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_tri_tri.restype = ctypes.c_int
        L.orc_last_confirmed.argtypes = [P, P, P, P]
        L.orc_last_confirmed.restype = i64
        L.orc_create_bounded.argtypes = [P, i64, dbl, ctypes.c_int, dbl, P, ctypes.POINTER(P)]
        L.orc_create_bounded.restype = ctypes.c_int
        L.orc_region_coords.argtypes = [P, P, P]
        L.orc_region_coords.restype = None
        L.orc_active.argtypes = [P]
        L.orc_active.restype = i64
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        L.orc_loop_count.argtypes = [P]
        L.orc_loop_count.restype = i64
        L.orc_loops.argtypes = [P, P]
        L.orc_loops.restype = ctypes.c_int
        L.orc_set_coin.argtypes = [P, dbl, ctypes.c_uint64]
        L.orc_set_coin.restype = ctypes.c_int
        L.orc_philox4x64.argtypes = [P, P, P]
        L.orc_philox4x64.restype = None
        L.orc_coin.argtypes = [ctypes.c_uint64, i32, i64, i64]
        L.orc_coin.restype = dbl
        L.orc_region_keys.argtypes = [P, dbl, i32, P, i64, P, P]
        L.orc_region_keys.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleRegion:
    """Region evolved by the oracle (lockstep lattice, periodic box).

    With ``geom`` = (V[4], inv2g, idx[4]) the region is one 4-cube of the tiling:
    points stop when their next diamond's earliest point leaves it."""

    def __init__(self, recs, box, cosmology, hcoef, geom=None):
        recs = np.ascontiguousarray(recs, dtype=REC)
        self._keep = recs
        h = ctypes.c_void_p()
        if geom is None:
            rc = lib().orc_create(_ptr(recs), len(recs), float(box), int(cosmology),
                                  float(hcoef), ctypes.byref(h))
        else:
            g = np.ascontiguousarray(geom, dtype=np.float64)
            assert g.shape == (9,)
            rc = lib().orc_create_bounded(_ptr(recs), len(recs), float(box), int(cosmology),
                                          float(hcoef), _ptr(g), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle rejected the surface (code {rc})")
        self.h = h

    def evolve(self, max_steps, t_end=float("inf"), search=GRID, intercommute=True,
               loop_every=0, p=1.0, seed=0):
        """p: intercommutation probability in [0, 1] (0: every crossing passes
        through); seed: key of the crossings' random numbers (both apply to this call's
        steps)."""
        rc = lib().orc_set_coin(self.h, float(p), int(seed))
        if rc != 0:
            raise ValueError(f"oracle rejected p = {p} (code {rc})")
        rc = lib().orc_evolve(self.h, int(max_steps), float(t_end), int(search),
                              int(bool(intercommute)), int(loop_every))
        if rc != 0:
            raise RuntimeError(f"oracle evolve failed (code {rc})")

    def read(self):
        n = lib().orc_n(self.h)
        out = np.zeros(n, dtype=REC)
        lib().orc_read(self.h, _ptr(out))
        return out

    def loops(self):
        """Loops recorded and removed, in removal order (step, then lowest slot)."""
        n = lib().orc_loop_count(self.h)
        out = np.zeros(n, dtype=LOOP)
        if n:
            lib().orc_loops(self.h, _ptr(out))
        return out

    def events(self):
        n = lib().orc_event_count(self.h)
        out = np.zeros(n, dtype=EVT)
        if n:
            lib().orc_events(self.h, _ptr(out))
        return out

    def stats(self):
        s = np.zeros(6, dtype=np.int64)
        lib().orc_stats(self.h, _ptr(s))
        return dict(point_steps=int(s[0]), candidates=int(s[1]), confirmed=int(s[2]),
                    accepted=int(s[3]), steps=int(s[4]), passed=int(s[5]))

    def last_confirmed(self):
        """Confirmed events of the most recent step, sorted by (t*, id_a, id_b)."""
        n = lib().orc_last_confirmed(self.h, None, None, None)
        t = np.zeros(max(n, 1)); ids = np.zeros((max(n, 1), 2), np.int64); x = np.zeros((max(n, 1), 3))
        lib().orc_last_confirmed(self.h, _ptr(t), _ptr(ids), _ptr(x))
        return t[:n], ids[:n], x[:n]

    @property
    def step(self):
        return lib().orc_step(self.h)

    @property
    def active(self):
        return lib().orc_active(self.h)

    def coords(self, P):
        """Generator coordinates of a spacetime point (x, y, z, t)."""
        P = np.ascontiguousarray(P, dtype=np.float64)
        c = np.zeros(4)
        lib().orc_region_coords(self.h, _ptr(P), _ptr(c))
        return c

    def band_candidates(self, search=GRID):
        """Exact-overlap candidate id pairs of the current band (no state change)."""
        n = lib().orc_band_candidates(self.h, int(search), None, 0)
        out = np.zeros((max(n, 1), 2), dtype=np.int64)
        lib().orc_band_candidates(self.h, int(search), _ptr(out), n)
        return out[:n]

    def close(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run(net, steps, t_end=float("inf"), search=GRID, intercommute=True, loop_every=0, p=1.0,
        seed=0):
    """Convenience: evolve a generated network (or region, when it carries "geom") and
    return (records, events, stats)."""
    hc = {0: 0.0, 1: 2.0, 2: 1.0}[net["cosmology"]]
    r = OracleRegion(net["recs"], net["box"], net["cosmology"], hc, net.get("geom"))
    r.evolve(steps, t_end, search, intercommute, loop_every, p, seed)
    out = (r.read(), r.events(), r.stats())
    r.close()
    return out


def top(cosmology, hcoef, box, L, R, B):
    T = np.zeros(4)
    Lr, Rr, Br = (np.ascontiguousarray(v, dtype=np.float64) for v in (L, R, B))
    lib().orc_top(int(cosmology), float(hcoef), float(box), _ptr(Lr), _ptr(Rr), _ptr(Br), _ptr(T))
    return T


def det4(a, b, c, d):
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d))
    return lib().orc_det4(_ptr(a), _ptr(b), _ptr(c), _ptr(d))


def tri_tri(P, Q):
    """P, Q: 3 x 4 vertex arrays. Returns (hit, t*, X*)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    t = np.zeros(1)
    x = np.zeros(3)
    hit = lib().orc_tri_tri(_ptr(P[0]), _ptr(P[1]), _ptr(P[2]), _ptr(Q[0]), _ptr(Q[1]),
                            _ptr(Q[2]), _ptr(t), _ptr(x))
    return bool(hit), float(t[0]), x


def threads():
    return lib().orc_threads()


def philox4x64(ctr, key):
    """Philox4x64-10 of a 4-word counter under a 2-word key (uint64 words)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    assert c.shape == (4,) and k.shape == (2,)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def coin(seed, step, id_a, id_b):
    """Uniform number in [0, 1) deciding whether crossing (id_a, id_b) of step
    `step` exchanges partners (it does when the number is below p)."""
    return lib().orc_coin(int(seed), int(step), int(id_a), int(id_b))


# --------------------------------------------------------------------------------------
# A periodic spacetime tiling run as one whole volume
# --------------------------------------------------------------------------------------

def region_keys(V, inv2g, K, P):
    """(S, key) of spacetime points P (n x 4: x, y, z, t) in the periodic tiling with
    lattice origin V, 1/(2 g) = inv2g and K = 4 L / (2 g): S the layer and key the past
    vertex's position mod K (orc_region_keys)."""
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(-1, 4))
    Vv = np.ascontiguousarray(V, dtype=np.float64)
    S = np.zeros(len(P), np.int32)
    key = np.zeros(len(P), np.int32)
    if len(P):
        lib().orc_region_keys(_ptr(Vv), float(inv2g), int(K), _ptr(P), len(P), _ptr(S),
                              _ptr(key))
    return S, key


def whole_volume_history(net, t_stop, p=0.0, seed=0, search=GRID):
    """Run a whole-volume network one lattice step at a time until every point of the
    newest slice has t > t_stop, keeping every slice.

    Returns (X, ids, nxt, events): X[s, q] the vertex of the point in slot q on slice
    s0 - 1 + s (s0 the step of the input records, so X[0] and X[1] are the initial
    surface), nxt the next-neighbour slot of each slot at the start (with p = 0 links
    never change) and the event log. With p = 0 every crossing is logged as passed."""
    recs = np.ascontiguousarray(net["recs"], dtype=REC)
    hc = {0: 0.0, 1: 2.0, 2: 1.0}[net["cosmology"]]
    r = OracleRegion(recs, net["box"], net["cosmology"], hc)
    try:
        ids = recs["id"].copy()
        slot = {int(v): q for q, v in enumerate(ids)}
        nxt = np.array([slot[int(v)] for v in recs["next_id"]], dtype=np.int64)
        X = [recs["x_prev"].copy(), recs["x"].copy()]
        while X[-1][:, 3].min() <= t_stop:
            r.evolve(1, search=search, intercommute=True, p=p, seed=seed)
            cur = r.read()
            if not np.array_equal(cur["id"], ids):
                raise RuntimeError("slot order changed")
            X.append(cur["x"].copy())
        return np.stack(X), ids, nxt, r.events()
    finally:
        r.close()


def vertex_homes(X, nxt, V, inv2g, K):
    """Home region name (S << 32 | key) of every vertex of a whole-volume history.

    A vertex's home is the region holding it, except where that region comes before the
    home of a vertex its diamond was built from (the first-order expansion can leave an
    edge slightly outside the light cone, so that a world line steps back across a face):
    then it takes that later home. The vertices a diamond with top X[s, q] is built from
    are X[s-1, q], X[s-1, next q] and X[s-2, next q]; the second initial slice X[1, q] is
    taken as built from X[0, q] and X[0, next q]. "Later" is by layer S; two different
    homes of the latest layer among those inputs cannot be ordered and raise ValueError.
    With every edge inside or on the light cone (flat space) the homes are the regions."""
    ns, n = X.shape[0], X.shape[1]
    S, key = region_keys(V, inv2g, K, X.reshape(-1, 4))
    own = ((S.astype(np.int64) << 32) | key.astype(np.int64)).reshape(ns, n)
    home = own.copy()

    def resolve(o, inputs):
        m = inputs[0]
        for x in inputs[1:]:
            m = np.where((x >> 32) > (m >> 32), x, m)
        later = (o >> 32) > (m >> 32)
        for x in inputs:
            if np.any(((x >> 32) == (m >> 32)) & (x != m) & ~later):
                raise ValueError("inputs with two homes of one layer")
        return np.where((o == m) | later, o, m)

    if ns > 1:
        home[1] = resolve(own[1], [home[0], home[0][nxt]])
    for s in range(2, ns):
        home[s] = resolve(own[s], [home[s - 1], home[s - 1][nxt], home[s - 2][nxt]])
    return home, own


def diamond_owners(X, nxt, V, inv2g, K, region_of):
    """Owner of every diamond of a whole-volume history in a periodic tiling (Section
    "Semi-parallel cosmic string simulation": a diamond is built by the region holding
    its earliest point; vertex_homes gives the reading where a world line steps back
    across a face). The diamond whose top is X[s, q] (s >= 2) has bottom
    X[s - 2, next q]; owner[s, q] is the index that region_of (a dict (S, key) ->
    region) gives that bottom's home, -1 outside the tiling or for s < 2. Also returns
    the region index of every vertex's home."""
    ns, n = X.shape[0], X.shape[1]
    home, _ = vertex_homes(X, nxt, V, inv2g, K)
    rk = np.array([s_ * (1 << 32) + k_ for (s_, k_) in region_of], dtype=np.int64)
    rv = np.array(list(region_of.values()), dtype=np.int64)
    if len(rk) == 0:
        lut = np.full((ns, n), -1, np.int64)
    else:
        order = np.argsort(rk)
        rk, rv = rk[order], rv[order]
        pos = np.minimum(np.searchsorted(rk, home), len(rk) - 1)
        lut = np.where(rk[pos] == home, rv[pos], -1)
    owner = np.full((ns, n), -1, np.int64)
    owner[2:] = lut[:-2][:, nxt]
    return owner, lut
