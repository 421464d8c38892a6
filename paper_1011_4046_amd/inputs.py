"""Seeded synthetic inputs: initial surfaces of cosmic-string networks.

This module is shared by the HIP path (tests, bench) and by the CPU oracle. It holds
none of the evolution, intersection or reconnection arithmetic. It only samples
string shapes and writes them out as initial-surface point records.

Representation (the staggered diamond lattice of the piecewise-linear solution
x = [a(t - sigma) + b(t + sigma)]/2, Section "Semi-parallel cosmic string
simulation", equation for x(sigma, t) and the diamond construction that follows):

* A chain of N points is described by samples A_k = a(-k*delta) and
  B_m = b(m*delta), delta being the sigma spacing.
* Point k on lattice slice n is the world-sheet vertex X_n[k] = (A_k + B_{k+n})/2,
  at time t_n = t0 + n*delta/2.
* The initial surface therefore holds X_0 and X_1. Each record carries X_1 as
  ``x`` (slice ``step`` = 1) and X_0 as ``x_prev``.
* A chain that winds the periodic box carries shift vectors: A_{k+N} = A_k + wA
  and B_{k+N} = B_k + wB. Positions are stored unwrapped along each chain.

Generators:

* :func:`kt_loops`: closed loops with a few Fourier modes, arc-length
  reparametrized to unit speed (flat-space workload).
* :func:`vv_network`: a Vachaspati-Vilenkin-style network from random Z3 phases
  on a periodic cubic lattice, traced through pierced plaquettes, at rest
  (matter-era workload).
* :func:`straight_string`, :func:`circular_loop`, :func:`crossing_strings`:
  analytic shapes used to pin the oracle.
"""
from __future__ import annotations

import numpy as np

# One point record of an initial or final surface (160 bytes, matches the C ABI).
REC_DTYPE = np.dtype([
    ("id", "<i8"), ("next_id", "<i8"), ("prev_id", "<i8"),
    ("step", "<i4"), ("flags", "<i4"),
    ("x", "<f8", (4,)), ("x_prev", "<f8", (4,)),
    ("r", "<f8", (4,)), ("r_prev", "<f8", (4,)),
])
assert REC_DTYPE.itemsize == 160

# Event record of the C ABI (56 bytes).
EVENT_DTYPE = np.dtype([
    ("step", "<i4"), ("kind", "<i4"), ("id_a", "<i8"), ("id_b", "<i8"),
    ("t_star", "<f8"), ("x_star", "<f8", (3,)),
])
assert EVENT_DTYPE.itemsize == 56

# Loop record of the C ABI (48 bytes): a loop recorded and removed.
LOOP_DTYPE = np.dtype([
    ("step", "<i4"), ("n_points", "<i4"), ("rep_id", "<i8"),
    ("energy", "<f8"), ("centre", "<f8", (3,)),
])
assert LOOP_DTYPE.itemsize == 48

FLAT, MATTER, RADIATION = 0, 1, 2
# H = HCOEF / eta in conformal time for a ∝ eta^HCOEF (matter: a ∝ eta^2).
HCOEF = {FLAT: 0.0, MATTER: 2.0, RADIATION: 1.0}


class Network(dict):
    """Initial surface plus the samples it was built from.

    Keys: ``recs`` (REC_DTYPE array), ``box`` (periodic length L), ``delta``,
    ``t0``, ``cosmology``, ``chains`` (list of dicts with A, B, wA, wB, id0).
    """


def records_from_chains(chains, t0, delta):
    """Build the initial surface (slices 0 and 1) for a list of chains.

    Each chain is a dict with ``A`` and ``B`` (N x 3 samples), ``wA`` and ``wB``
    (shift per period; zero for a loop that does not wind the box).
    """
    total = sum(len(c["A"]) for c in chains)
    recs = np.zeros(total, dtype=REC_DTYPE)
    t1 = t0 + 0.5 * delta
    base = 0
    for c in chains:
        A = np.asarray(c["A"], dtype=np.float64)
        B = np.asarray(c["B"], dtype=np.float64)
        n = len(A)
        Bn = np.concatenate([B[1:], (B[0] + np.asarray(c["wB"], np.float64))[None]], axis=0)
        x0 = 0.5 * (A + B)
        x1 = 0.5 * (A + Bn)
        ids = base + np.arange(n, dtype=np.int64)
        sl = slice(base, base + n)
        recs["id"][sl] = ids
        recs["next_id"][sl] = base + (np.arange(n) + 1) % n
        recs["prev_id"][sl] = base + (np.arange(n) - 1) % n
        recs["step"][sl] = 1
        recs["x"][sl, :3] = x1
        recs["x"][sl, 3] = t1
        recs["x_prev"][sl, :3] = x0
        recs["x_prev"][sl, 3] = t0
        c["id0"] = base
        base += n
    return recs


# --------------------------------------------------------------------------------------
# Flat space: closed loops with a few Fourier modes
# --------------------------------------------------------------------------------------

def _fourier_closed_curve(rng, n_modes, n_pts, dense):
    """Closed curve sum_m A_m cos(2 pi m s) + B_m sin(2 pi m s), resampled at n_pts
    equal-arc points after scaling its length to 1 (unit speed in sigma)."""
    coef = rng.standard_normal((2, n_modes, 3))
    s = np.arange(dense, dtype=np.float64) / dense
    m = np.arange(1, n_modes + 1, dtype=np.float64)
    ph = 2.0 * np.pi * np.outer(s, m)                  # dense x modes
    C = np.cos(ph) @ coef[0] + np.sin(ph) @ coef[1]     # dense x 3
    Cc = np.concatenate([C, C[:1]], axis=0)
    seg = np.linalg.norm(np.diff(Cc, axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    total = cum[-1]
    u = np.arange(n_pts, dtype=np.float64) * (total / n_pts)
    i = np.clip(np.searchsorted(cum, u, side="right") - 1, 0, dense - 1)
    f = (u - cum[i]) / np.where(seg[i] > 0, seg[i], 1.0)
    P = Cc[i] + f[:, None] * (Cc[i + 1] - Cc[i])
    P = P / total
    return P - P.mean(axis=0)


def kt_loops(n_loops=8, n_pts=256, n_modes=5, box=1.0, seed=0, t0=0.0, dense=1 << 16):
    """Flat-space workload: closed loops of invariant length 1 in a periodic box.

    Per loop, in this rng order: a-curve coefficients, b-curve coefficients
    (each 2 x n_modes x 3 iid N(0,1)), loop centre uniform in [0, box)^3.
    delta = 1/n_pts, so dt = delta/2.
    """
    rng = np.random.default_rng(seed)
    chains = []
    for _ in range(n_loops):
        a = _fourier_closed_curve(rng, n_modes, n_pts, dense)
        b = _fourier_closed_curve(rng, n_modes, n_pts, dense)
        c = rng.uniform(0.0, box, 3)
        a = a + c
        b = b + c
        k = np.arange(n_pts)
        A = a[(-k) % n_pts]          # A_k = a(-k delta)
        B = b[k]                     # B_m = b(m delta)
        chains.append(dict(A=A, B=B, wA=np.zeros(3), wB=np.zeros(3)))
    delta = 1.0 / n_pts
    recs = records_from_chains(chains, t0, delta)
    return Network(recs=recs, box=float(box), delta=delta, t0=float(t0),
                   cosmology=FLAT, chains=chains)


# --------------------------------------------------------------------------------------
# Matter era: Vachaspati-Vilenkin-style network from Z3 phases
# --------------------------------------------------------------------------------------

def _zdiff(a, b):
    """Minimal Z3 phase difference b - a in {-1, 0, 1} (units of 2 pi / 3)."""
    return ((b - a + 1) % 3) - 1


def vv_faces(phase):
    """Windings (in {-1,0,1}) of the three families of plaquettes of a periodic lattice.

    Face (axis, i, j, k) is the plaquette at coordinate i (resp. j, k) along ``axis``
    with the lower corner at site (i, j, k); its normal is +axis and the winding is
    taken counterclockwise about that normal.
    """
    p = phase
    r = lambda a, ax: np.roll(a, -1, ax)
    pi, pj, pk = r(p, 0), r(p, 1), r(p, 2)
    # normal +x: (j,k) -> (j+1,k) -> (j+1,k+1) -> (j,k+1)
    pjk = r(pj, 2)
    wx = _zdiff(p, pj) + _zdiff(pj, pjk) + _zdiff(pjk, pk) + _zdiff(pk, p)
    # normal +y: (k,i) -> (k+1,i) -> (k+1,i+1) -> (k,i+1)
    pki = r(pk, 0)
    wy = _zdiff(p, pk) + _zdiff(pk, pki) + _zdiff(pki, pi) + _zdiff(pi, p)
    # normal +z: (i,j) -> (i+1,j) -> (i+1,j+1) -> (i,j+1)
    pij = r(pi, 1)
    wz = _zdiff(p, pi) + _zdiff(pi, pij) + _zdiff(pij, pj) + _zdiff(pj, p)
    w = np.stack([wx, wy, wz])
    assert np.all(w % 3 == 0)
    return w // 3


def vv_chains(m, rng, xi=1.0, pts_per_xi=8, jitter=0.15):
    """Trace strings through pierced plaquettes of an m^3 periodic Z3 lattice.

    Path: face centre -> (cube centre + offset) -> face centre. The offset is drawn
    per cube traversal, uniform in [-jitter, jitter]^3 * xi, so that the 2 or 3
    strings crossing one cube do not touch. Each closed polyline is sampled every
    delta = xi/pts_per_xi of arc length from its first face centre; the closing
    chord is the remainder (< delta). Cubes with 2 or 3 strings pair their entry and
    exit faces by ranking seeded random keys. rng order: phases (m^3), pairing keys
    (6 per cube), offsets (3 per pierced face, in face order).
    Returns a list of (P, winding) with P the unwrapped points (n x 3).
    """
    phase = rng.integers(0, 3, size=(m, m, m))
    w = vv_faces(phase)                                   # (3, m, m, m) in {-1,0,1}
    M3 = m * m * m
    I_, J_, K_ = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    cube = (I_ * m + J_) * m + K_
    # the 6 faces of every cube: (axis, lower/upper); face id = axis*M3 + site index
    face_ids, fw, is_hi = [], [], []
    for ax in range(3):
        for hi in (0, 1):
            sh = [I_, J_, K_]
            sh[ax] = (sh[ax] + hi) % m
            site = (sh[0] * m + sh[1]) * m + sh[2]
            face_ids.append(ax * M3 + site)
            fw.append(w[ax].reshape(-1)[site])
            is_hi.append(np.full(cube.shape, hi))
    F = np.stack([f.reshape(-1) for f in face_ids], 1)         # (M3, 6)
    Wf = np.stack([f.reshape(-1) for f in fw], 1)
    H = np.stack([f.reshape(-1) for f in is_hi], 1)
    # flux into the cube: lower face with w=+1 or upper face with w=-1
    incoming = ((H == 0) & (Wf == 1)) | ((H == 1) & (Wf == -1))
    outgoing = ((H == 0) & (Wf == -1)) | ((H == 1) & (Wf == 1))
    assert np.all(incoming.sum(1) == outgoing.sum(1))
    keys = rng.random((M3, 6))
    # rank incoming faces by position, outgoing faces by random key; pair equal ranks
    big = 10.0
    in_order = np.argsort(np.where(incoming, np.arange(6)[None, :], big), axis=1, kind="stable")
    out_order = np.argsort(np.where(outgoing, keys, big), axis=1, kind="stable")
    nio = incoming.sum(1)
    succ = -np.ones(3 * M3, dtype=np.int64)
    out_dir = np.zeros(3 * M3, dtype=np.int64)         # exit sign of the paired face
    rows = np.arange(M3)
    for r in range(3):
        sel = nio > r
        fi = F[rows[sel], in_order[sel, r]]
        slot = out_order[sel, r]
        fo = F[rows[sel], slot]
        succ[fi] = fo
        out_dir[fi] = np.where(H[rows[sel], slot] == 1, 1, -1)
    pierced = np.nonzero(succ >= 0)[0]
    offsets = np.zeros((3 * M3, 3))
    offsets[pierced] = rng.uniform(-jitter, jitter, (len(pierced), 3))
    # chains = cycles of the permutation succ over pierced faces, each started at its
    # smallest face id, in increasing order of that id
    F = len(pierced)
    cidx = -np.ones(3 * M3, dtype=np.int64)
    cidx[pierced] = np.arange(F)
    nxt = cidx[succ[pierced]]
    lab = np.arange(F)
    jump = nxt.copy()
    for _ in range(max(1, int(np.ceil(np.log2(max(F, 2))))) + 1):
        lab = np.minimum(lab, lab[jump])
        jump = jump[jump]
    # distance from the cycle start: break each cycle before its start, rank the lists
    tail = nxt == lab
    dist = np.where(tail, 0, 1)
    jump = np.where(tail, np.arange(F), nxt)
    for _ in range(max(1, int(np.ceil(np.log2(max(F, 2))))) + 1):
        dist = dist + np.where(jump == np.arange(F), 0, dist[jump])
        jump = jump[jump]
    length = np.bincount(lab, minlength=F)
    rank = length[lab] - 1 - dist
    order = np.lexsort((rank, lab))
    starts = np.nonzero(rank[order] == 0)[0]
    ends = np.append(starts[1:], F)
    chains = []
    step = 1.0 / pts_per_xi
    axis_of = lambda f: f // M3
    for a0, a1 in zip(starts, ends):
        cyc = pierced[order[a0:a1]]
        ax = axis_of(cyc)
        site = cyc % M3
        fi_, rest = np.divmod(site, m * m)
        fj_, fk_ = np.divmod(rest, m)
        start = np.array([fi_[0] + 0.5, fj_[0] + 0.5, fk_[0] + 0.5])
        start[ax[0]] -= 0.5
        din = np.zeros((len(cyc), 3))
        din[np.arange(len(cyc)), ax] = w[ax, fi_, fj_, fk_]
        dout = np.zeros((len(cyc), 3))
        nxt = np.roll(cyc, -1)
        dout[np.arange(len(cyc)), axis_of(nxt)] = out_dir[cyc]
        # face centres along the unwrapped path: F_{i+1} = F_i + din_i/2 + dout_i/2
        moves = 0.5 * din + 0.5 * dout
        Fc = start + np.concatenate([np.zeros((1, 3)), np.cumsum(moves, axis=0)])
        C = Fc[:-1] + 0.5 * din + offsets[cyc]
        V = np.empty((2 * len(cyc) + 1, 3))
        V[0:-1:2] = Fc[:-1]
        V[1::2] = C
        V[-1] = Fc[-1]
        seg = np.linalg.norm(np.diff(V, axis=0), axis=1)
        cum = np.concatenate([[0.0], np.cumsum(seg)])
        n = int(np.floor(cum[-1] / step))
        if cum[-1] - n * step < 1e-9:
            n -= 1
        u = np.arange(n + 1, dtype=np.float64) * step
        i = np.clip(np.searchsorted(cum, u, side="right") - 1, 0, len(seg) - 1)
        fr = (u - cum[i]) / seg[i]
        P = V[i] + fr[:, None] * (V[i + 1] - V[i])
        wind = np.rint((V[-1] - V[0]) / m).astype(np.int64)
        chains.append((P * xi, wind))
    return chains


def vv_network(m=32, xi=1.0, pts_per_xi=8, seed=0, t0=8.0, cosmology=MATTER, jitter=0.15):
    """Matter-era workload: a VV-style network at rest in a periodic box L = m*xi.

    Zero initial velocity: a(-sigma) = b(sigma) = x0(sigma), i.e. A = B = P.
    delta = xi / pts_per_xi. Ids are chain-major in tracing order.
    A jitter of 0 gives the undisplaced face-centre / cube-centre path.
    """
    rng = np.random.default_rng(seed)
    L = m * xi
    raw = vv_chains(m, rng, xi, pts_per_xi, jitter)
    chains = []
    for P, wind in raw:
        wv = wind.astype(np.float64) * L
        chains.append(dict(A=P, B=P, wA=wv, wB=wv))
    delta = xi / pts_per_xi
    recs = records_from_chains(chains, t0, delta)
    return Network(recs=recs, box=float(L), delta=delta, t0=float(t0),
                   cosmology=cosmology, chains=chains)


# --------------------------------------------------------------------------------------
# Analytic shapes
# --------------------------------------------------------------------------------------

def straight_string(n_pts, box, v=0.0, origin=(0.0, 0.0, 0.0), axis=0, vdir=1):
    """A straight string along ``axis`` winding the box once, moving with speed v
    along ``vdir``. x(sigma,t) = sigma*sqrt(1-v^2) e_axis + v t e_vdir, hence
    a(u) = -u*sqrt(1-v^2) e_axis + v u e_vdir and b(u) = u*sqrt(1-v^2) e_axis + v u e_vdir.
    delta = box / (n_pts*sqrt(1-v^2)), so the chain closes on the box period."""
    g = np.sqrt(1.0 - v * v)
    delta = box / (n_pts * g)
    k = np.arange(n_pts, dtype=np.float64)
    ea = np.zeros(3); ea[axis] = 1.0
    ev = np.zeros(3); ev[vdir] = 1.0
    o = np.asarray(origin, np.float64)
    # A_k = a(-k delta), B_m = b(m delta)
    A = o + np.outer(k * delta * g, ea) + np.outer(-v * k * delta, ev)
    B = o + np.outer(k * delta * g, ea) + np.outer(v * k * delta, ev)
    wA = n_pts * delta * g * ea - v * n_pts * delta * ev
    wB = n_pts * delta * g * ea + v * n_pts * delta * ev
    return dict(A=A, B=B, wA=wA, wB=wB), delta


def circular_loop(n_pts, radius, centre=(0.0, 0.0, 0.0)):
    """A static regular polygon inscribed in a circle (A = B = P, zero velocity).
    The sigma spacing is the chord length, so the lattice edges are null."""
    th = 2.0 * np.pi * np.arange(n_pts) / n_pts
    P = np.asarray(centre, np.float64) + radius * np.stack([np.cos(th), np.sin(th), np.zeros(n_pts)], 1)
    delta = 2.0 * radius * np.sin(np.pi / n_pts)
    return dict(A=P, B=P, wA=np.zeros(3), wB=np.zeros(3)), delta


def make_network(chains, box, delta, t0, cosmology):
    recs = records_from_chains(chains, t0, delta)
    return Network(recs=recs, box=float(box), delta=float(delta), t0=float(t0),
                   cosmology=cosmology, chains=chains)


def crossing_strings(n_pts=64, box=1.0, v=0.5, y0=0.1, x0=0.30078125, z_off=0.0057):
    """Two straight strings in flat space whose world sheets meet at one point.

    String 1 lies along x at rest through (., 0, 0). String 2 lies along z through
    (x0, y0, .) moving with speed v in -y. They cross at t* = y0/v at X* = (x0, 0, 0).
    """
    s1, d1 = straight_string(n_pts, box, v=0.0, origin=(0.0, 0.0, 0.0), axis=0, vdir=1)
    g = np.sqrt(1.0 - v * v)
    # string 2 must share the same delta: choose its point count so that it closes
    n2 = int(round(box / (d1 * g)))
    # pick v so that n2 * d1 * g == box exactly as far as possible: recompute g from n2
    g2 = box / (n2 * d1)
    v2 = np.sqrt(1.0 - g2 * g2)
    k = np.arange(n2, dtype=np.float64)
    ez = np.array([0.0, 0.0, 1.0]); ey = np.array([0.0, 1.0, 0.0])
    o = np.array([x0, y0, z_off])
    A = o + np.outer(k * d1 * g2, ez) + np.outer(v2 * k * d1, ey)
    B = o + np.outer(k * d1 * g2, ez) - np.outer(v2 * k * d1, ey)
    wA = n2 * d1 * g2 * ez + v2 * n2 * d1 * ey
    wB = n2 * d1 * g2 * ez - v2 * n2 * d1 * ey
    s2 = dict(A=A, B=B, wA=wA, wB=wB)
    net = make_network([s1, s2], box, d1, 0.0, FLAT)
    net["v2"] = v2
    net["t_star"] = y0 / v2
    net["x_star"] = np.array([x0, 0.0, 0.0])
    return net


# --------------------------------------------------------------------------------------
# Standalone regions of the tiling (first layer: they generate their own initial data)
# --------------------------------------------------------------------------------------

def region_geometry(size, t_mid, centre=(0.0, 0.0, 0.0)):
    """One 4-cube region of the spacetime tiling (Section "Geometry").

    Generators g/2 (1,1,1,1), g/2 (1,-1,-1,1), g/2 (-1,1,-1,1), g/2 (-1,-1,1,1) in
    (x, y, z, tau) with tau = sqrt(3) t, region "size" s = rhombohedron edge, so
    g = s / sqrt(2). The region with index 0 and lattice origin V has its mid-time
    centre at (centre, tau = sqrt(3) t_mid) when V = (centre, sqrt(3) t_mid - g).
    Returns geom = [V0, V1, V2, V3, 1/(2g), 0, 0, 0, 0] and g.
    """
    g = size / np.sqrt(2.0)
    V = [float(centre[0]), float(centre[1]), float(centre[2]), float(np.sqrt(3.0) * t_mid - g)]
    return np.array(V + [1.0 / (2.0 * g), 0.0, 0.0, 0.0, 0.0]), g


def region_network(n_target, size, seed, t_mid=8.0, centre=(0.0, 0.0, 0.0), pts_per_xi=8,
                   jitter=0.15, cosmology=MATTER, box=None):
    """Initial data of a first-layer region: a VV-style network at rest cut to the
    region's spatial cross-section at its mid-time (the octahedron |x|+|y|+|z| < g
    around the centre, the middle slice of a 4-cube standing on a vertex).

    The lattice spacing xi is chosen so that about n_target points fall inside.
    Points are kept when their slice-0 position lies inside the octahedron by more than
    one sigma spacing; links to dropped points become -1 (dangling). box is the periodic
    length used by the evolver (default: a power of two larger than 4 g, so that no
    difference inside the region is ever folded).
    """
    rng = np.random.default_rng(seed)
    geom, g = region_geometry(size, t_mid, centre)
    if n_target <= 0:
        recs = np.zeros(0, dtype=REC_DTYPE)
        L = box or 2.0 ** np.ceil(np.log2(4 * g))
        return Network(recs=recs, box=float(L), delta=1.0, t0=float(t_mid), cosmology=cosmology,
                       chains=[], geom=geom, g=g)
    xi = g * (9.48 / n_target) ** (1.0 / 3.0)
    m = int(np.ceil((2 * g + 2 * xi) / xi))
    W = m * xi
    delta = xi / pts_per_xi
    raw = vv_chains(m, rng, xi, pts_per_xi, jitter)
    c = np.asarray(centre, np.float64)
    pts, nxt_ok = [], []
    X0s, X1s = [], []
    for P, wind in raw:
        n = len(P)
        Pn = np.concatenate([P[1:], (P[0] + wind * W)[None]], axis=0)
        step = 0.5 * (Pn - P)
        w = P - W * np.floor(P / W) - 0.5 * W + c      # wrapped into the box around the centre
        X0s.append(w)
        X1s.append(w + step)
    lim = g - delta
    recs_list = []
    base = 0
    for X0, X1 in zip(X0s, X1s):
        inside = np.abs(X0 - c).sum(axis=1) < lim
        n = len(X0)
        keep_idx = np.nonzero(inside)[0]
        if len(keep_idx) == 0:
            continue
        new_id = -np.ones(n, dtype=np.int64)
        new_id[keep_idx] = base + np.arange(len(keep_idx))
        r = np.zeros(len(keep_idx), dtype=REC_DTYPE)
        r["id"] = new_id[keep_idx]
        r["next_id"] = new_id[(keep_idx + 1) % n]
        r["prev_id"] = new_id[(keep_idx - 1) % n]
        r["step"] = 1
        r["x"][:, :3] = X1[keep_idx]
        r["x"][:, 3] = t_mid + 0.5 * delta
        r["x_prev"][:, :3] = X0[keep_idx]
        r["x_prev"][:, 3] = t_mid
        recs_list.append(r)
        base += len(keep_idx)
    recs = np.concatenate(recs_list) if recs_list else np.zeros(0, dtype=REC_DTYPE)
    L = box or float(2.0 ** np.ceil(np.log2(4 * g)))
    return Network(recs=recs, box=float(L), delta=float(delta), t0=float(t_mid),
                   cosmology=cosmology, chains=[], geom=geom, g=g)


def lognormal_regions(n_regions=512, median=2e4, sigma=1.5, cap=2e5, p_empty=0.2, seed=0):
    """Per-region point targets of the batched workload: empty with probability p_empty,
    else min(LogNormal(ln median, sigma), cap)."""
    rng = np.random.default_rng(seed)
    empty = rng.random(n_regions) < p_empty
    n = np.minimum(np.exp(np.log(median) + sigma * rng.standard_normal(n_regions)), cap)
    n = np.where(empty, 0, np.round(n)).astype(np.int64)
    return n


def region_batch(n_targets, size=4.0, seed=0, t_mid=8.0, slots=8, cosmology=MATTER,
                 pts_per_xi=None, workers=0, progress=None):
    """Independent first-layer regions on the slots of a periodic box (slots^3 slots,
    slot spacing >= 2 g + 1, so regions never overlap). Region r has point target
    n_targets[r], seed seed + r and pts_per_xi[r] points per correlation length
    (default 8); its ids are offset to be unique in the batch. workers > 1 generates
    the regions in that many worker processes (same result): forked while no GPU
    runtime is mapped in this process, spawned otherwise; progress(i) is called after
    every region generated serially.
    Returns (parts, box) with parts = [(recs, geom), ...]."""
    g = size / np.sqrt(2.0)
    nr = len(n_targets)
    assert nr <= slots ** 3
    box = float(2.0 ** np.ceil(np.log2(slots * (2 * g + 1.0))))
    spacing = box / slots
    ppx = [8] * nr if pts_per_xi is None else [int(v) for v in pts_per_xi]
    jobs = []
    for r, nt in enumerate(n_targets):
        i, j, k = r // (slots * slots), (r // slots) % slots, r % slots
        centre = (spacing * (i + 0.5), spacing * (j + 0.5), spacing * (k + 0.5))
        jobs.append((int(nt), size, seed + r, t_mid, centre, ppx[r], cosmology, box))
    if workers and workers > 1 and nr > 1:
        # pure NumPy work in worker processes: forked copies of this process while it
        # holds no GPU runtime state, freshly started interpreters otherwise
        import multiprocessing as mp
        ctx = mp.get_context("spawn" if _gpu_in_use() else "fork")
        with ctx.Pool(workers) as pool:
            nets = pool.map(_region_job, jobs, chunksize=1)
    else:
        nets = []
        for i, j in enumerate(jobs):
            nets.append(_region_job(j))
            if progress:
                progress(i)
    parts = []
    id_off = 0
    for recs, geom in nets:
        recs["id"] += id_off
        for f in ("next_id", "prev_id"):
            recs[f] = np.where(recs[f] >= 0, recs[f] + id_off, -1)
        parts.append((recs, geom))
        id_off += len(recs)
    return parts, box


# spatial part (x, y, z) of the four generators, in units of g/2
_GEN_XYZ = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.int64)


def _gen_coords(P, t, V, inv2g):
    """Generator coordinates c of points (P, t) about the lattice origin V (x, y, z,
    tau), written in the same operation order as the library's region test."""
    dx, dy, dz = P[:, 0] - V[0], P[:, 1] - V[1], P[:, 2] - V[2]
    dtau = np.sqrt(3.0) * t - V[3]
    a, b, cc, d = dx + dy, dz + dtau, dx - dy, dtau - dz
    return np.stack([(a + b) * inv2g, (cc + d) * inv2g, (d - cc) * inv2g, (b - a) * inv2g], 1)


def tiling_regions(net, M=4, layers=16, lead=1.75):
    """Cut a whole-volume network at its initial slice into the regions of a periodic
    spacetime tiling (Section "Geometry": 4-cubes spanned by four null generators; its
    subsection "Boundary conditions": the tiling repeats with the box).

    The box L holds M steps of 2 g per axis (g = L / 2M, region size s = g sqrt 2), so
    a layer -- the regions whose indices sum to S -- has 4 M^3 regions. Layers
    S = 0 .. layers-1 are kept. The lattice origin puts the initial slice `lead` g
    above the past vertex of layer 0 in tau, so the slice crosses layers 0 .. 3.
    A region is named by (S, p mod 4M) with p = the past vertex's spatial position in
    units of g/2; every point is moved by whole boxes into its region's canonical image
    (p in [0, 4M)^3). Region r's predecessors are the four regions r - e_m of layer
    S - 1 (none for layer 0). Links to points of other regions become -1. Regions cut
    by the initial slice take the points inside them; the others start empty.

    Returns (parts, box, n_pred, succ, layer) with parts = [(recs, geom)] in
    (layer, spatial key) order and geom = (origin[4], 1/(2 g), idx[4])."""
    L = float(net["box"])
    g = L / (2 * M)
    inv2g = 1.0 / (2.0 * g)
    recs = net["recs"]
    t0 = float(recs["x_prev"][0, 3]) if len(recs) else float(net["t0"])
    V = np.array([0.0, 0.0, 0.0, np.sqrt(3.0) * t0 - lead * g])
    K = 4 * M
    A = _GEN_XYZ.T                                    # p = A @ i
    # regions of one layer: canonical index for every spatial key in [0, K)^3
    rng_i = np.arange(-K, K + 1)
    I1, I2, I3 = np.meshgrid(rng_i, rng_i, rng_i, indexing="ij")
    cand = np.stack([I1.ravel(), I2.ravel(), I3.ravel()], 1)
    keys_of_layer = []
    for S in range(layers):
        i = np.concatenate([cand, (S - cand.sum(1))[:, None]], 1)
        p = i @ A.T
        ok = np.all((p >= 0) & (p < K), axis=1)
        i, p = i[ok], p[ok]
        key = (p[:, 0] * K + p[:, 1]) * K + p[:, 2]
        order = np.argsort(key)
        i, key = i[order], key[order]
        assert len(key) == 4 * M ** 3 and len(np.unique(key)) == len(key)
        keys_of_layer.append((key, i))
    per = 4 * M ** 3
    nr = layers * per
    # points: region index from the initial-slice position, moved to the canonical image
    # (a point within rounding of a region boundary may land in the neighbouring region
    # after a move; it is moved again until its own coordinates put it in a canonical one)
    x0, x1 = recs["x_prev"][:, :3].copy(), recs["x"][:, :3].copy()
    for _ in range(4):
        c2 = _gen_coords(x0, recs["x_prev"][:, 3], V, inv2g)
        i2 = np.floor(c2).astype(np.int64)
        wrap = np.floor_divide(i2 @ A.T, K)
        if not wrap.any():
            break
        x0 -= wrap * L
        x1 -= wrap * L
    else:
        raise AssertionError("points do not settle in a canonical region image")
    S_pt = i2.sum(1)
    p2 = i2 @ A.T
    assert np.all((p2 >= 0) & (p2 < K))
    inside = (S_pt >= 0) & (S_pt < layers)
    key_pt = (p2[:, 0] * K + p2[:, 1]) * K + p2[:, 2]
    rid = -np.ones(len(recs), dtype=np.int64)
    for S in range(layers):
        sel = inside & (S_pt == S)
        key, _ = keys_of_layer[S]
        rid[sel] = S * per + np.searchsorted(key, key_pt[sel])
    moved = recs.copy()
    moved["x"][:, :3] = x1
    moved["x_prev"][:, :3] = x0
    # links across regions dangle
    pos = {int(v): k for k, v in enumerate(recs["id"])}
    nxt = np.array([pos.get(int(v), -1) for v in recs["next_id"]], dtype=np.int64)
    prv = np.array([pos.get(int(v), -1) for v in recs["prev_id"]], dtype=np.int64)
    same_n = (nxt >= 0) & (rid[np.maximum(nxt, 0)] == rid)
    same_p = (prv >= 0) & (rid[np.maximum(prv, 0)] == rid)
    moved["next_id"] = np.where(same_n, moved["next_id"], -1)
    moved["prev_id"] = np.where(same_p, moved["prev_id"], -1)
    order = np.argsort(rid, kind="stable")
    counts = np.bincount(rid[rid >= 0], minlength=nr)
    sorted_recs = moved[order][rid[order] >= 0]
    off = np.concatenate([[0], np.cumsum(counts)])
    parts, n_pred, succ, layer = [], np.zeros(nr, np.int64), [[] for _ in range(nr)], []
    for S in range(layers):
        key, idx = keys_of_layer[S]
        for q in range(per):
            r = S * per + q
            geom = np.array([V[0], V[1], V[2], V[3], inv2g] + [float(v) for v in idx[q]])
            parts.append((sorted_recs[off[r]:off[r + 1]].copy(), geom))
            layer.append(S)
            if S + 1 < layers:
                pk = np.array([key[q] // (K * K), (key[q] // K) % K, key[q] % K])
                nkey, _ = keys_of_layer[S + 1]
                for m in range(4):
                    qp = (pk + _GEN_XYZ[m]) % K
                    s_id = (S + 1) * per + int(np.searchsorted(nkey, (qp[0] * K + qp[1]) * K + qp[2]))
                    succ[r].append(s_id)
                    n_pred[s_id] += 1
    return parts, L, n_pred, succ, np.array(layer)


def _gpu_in_use():
    """True when this process may hold GPU runtime state that a forked child must not
    inherit: torch has initialised its GPU context, or the HSA runtime is mapped at all
    (libsemipar was loaded, or a profiler preloaded its library before the program
    started)."""
    import sys
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        return True
    try:
        with open("/proc/self/maps") as f:
            return any("libhsa-runtime64" in line for line in f)
    except OSError:
        return True  # cannot tell: do not fork


def _region_job(job):
    nt, size, seed, t_mid, centre, ppx, cosmology, box = job
    net = region_network(nt, size, seed, t_mid, centre, pts_per_xi=ppx, cosmology=cosmology,
                         box=box)
    return net["recs"].copy(), net["geom"]


def mixed_regions(n_regions=256, median=2000, sigma=1.0, cap=50000, p_empty=0.1, seed=0,
                  ppx_choices=(4, 6, 8, 12, 16)):
    """Point targets and resolutions of a workload whose region cost is not a function
    of the point count: targets as in lognormal_regions, and each region's points per
    correlation length drawn uniformly from ppx_choices (seeded), which sets its sigma
    spacing and hence the number of lattice steps it needs."""
    n = lognormal_regions(n_regions, median, sigma, cap, p_empty, seed)
    rng = np.random.default_rng(seed + 7919)
    ppx = rng.choice(np.asarray(ppx_choices), size=n_regions)
    return n, ppx
