"""Pins of the oracle's region geometry and bounded-region evolution.

Geometry against the values the paper prints (tests/golden/geometry.json); bounded
evolution against the whole-volume evolution of the same strings: a region computes a
subset of the world-sheet diamonds, each of which must equal the whole-volume one.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1011_4046_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "geometry.json")))
SQ3 = np.sqrt(3.0)


def unit_region():
    """Region with unit-edge generators (g = 1), origin 0, index 0 (paper's example)."""
    recs = np.zeros(0, dtype=O.REC)
    geom = np.array([0.0, 0.0, 0.0, 0.0, 0.5, 0, 0, 0, 0])
    return O.OracleRegion(recs, 64.0, 0, 0.0, geom)


def at(r, xyz, tau):
    """Generator coordinates of the point with lattice time tau (t = tau / sqrt 3)."""
    return r.coords(np.array([xyz[0], xyz[1], xyz[2], tau / SQ3]))


def test_generators_and_vertices_match_paper():
    r = unit_region()
    G = np.array(GOLD["unit_edge_generators"])
    for i, gvec in enumerate(G):
        c = at(r, gvec[:3], gvec[3])
        assert np.allclose(c, np.eye(4)[i], atol=1e-15)
    assert np.allclose(at(r, GOLD["past_vertex"][:3], 0.0), 0.0)
    fv = GOLD["future_vertex"]
    assert np.allclose(G.sum(axis=0), fv)
    assert np.allclose(at(r, fv[:3], fv[3]), 1.0, atol=1e-15)
    # the four initial surfaces are 3-cubes ending at time 3/2 at the printed corners
    tau = GOLD["initial_surface_corners_time"]
    for xyz in GOLD["initial_surface_corners_xyz"]:
        c = at(r, xyz, tau)
        assert np.isclose(c.sum(), 3.0) and sorted(np.round(c, 12)) == [0.0, 1.0, 1.0, 1.0]
    # diagonal of an initial 3-cube, past vertex to its far corner: spatial length
    # sqrt(3)/2 and temporal 3/2, made null by shrinking time by sqrt(3)
    corner = G[1:].sum(axis=0)
    assert np.isclose(np.linalg.norm(corner[:3]), GOLD["main_diagonal_spatial_length"])
    assert np.isclose(corner[3], GOLD["main_diagonal_temporal_length"])
    assert np.isclose(corner[3] / GOLD["main_diagonal_spatial_length"], GOLD["time_shrink_factor"])


def test_faces_are_null_after_time_shrink():
    """The face spanned by three generators is a null 3-surface once t = tau/sqrt(3)."""
    G = np.array(GOLD["unit_edge_generators"])
    for i in range(4):
        F = np.delete(G, i, axis=0).copy()
        F[:, 3] /= SQ3                      # physical time
        # normal n with n.v = 0 for the three spanning vectors (Minkowski: (n_x,n_y,n_z,-n_t))
        M = np.column_stack([F[:, :3], -F[:, 3]])
        n = np.linalg.svd(M)[2][-1]
        assert abs(n[0] ** 2 + n[1] ** 2 + n[2] ** 2 - n[3] ** 2) < 1e-12


def test_twelve_periodicity_vectors_and_region_counts():
    G = np.array(GOLD["unit_edge_generators"])
    vecs = {tuple(np.round(G[i] - G[j], 12)) for i, j in itertools.permutations(range(4), 2)}
    assert len(vecs) == GOLD["n_periodicity_vectors"]
    for v in vecs:
        assert v[3] == 0.0
        comps = sorted(abs(c) for c in v[:3])
        assert comps == [0.0, 1.0, 1.0]
    assert 50 ** 3 == GOLD["regions_per_layer_N50"]
    # size = rhombohedron edge s: spatial periodicity vectors g (0,1,1) etc. with g = s/sqrt 2
    s = 40.0
    g = s / np.sqrt(2.0)
    P = g * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], dtype=float)
    assert np.isclose(np.linalg.norm(P[0]), s)
    assert np.isclose(abs(np.linalg.det(P)), GOLD["size40_volume"])
    assert np.isclose(12 * np.sqrt(2.0), GOLD["min_vv_region_size"])


def test_membership_partitions_spacetime():
    """Every point lies in exactly one region: floor(c) is its index, and stepping along
    a generator moves to the successor across that face."""
    r = unit_region()
    rng = np.random.default_rng(0)
    G = np.array(GOLD["unit_edge_generators"])
    for _ in range(500):
        P = rng.uniform(-3, 3, 4)
        c = at(r, P[:3], P[3])
        i = rng.integers(4)
        c2 = at(r, P[:3] + G[i][:3], P[3] + G[i][3])
        assert np.allclose(c2 - c, np.eye(4)[i], atol=1e-12)


def _loops_in_region(size, t_mid, n_loops=3, n_pts=64, seed=0):
    """Closed KT loops small enough to sit inside the region's mid-time octahedron."""
    geom, g = I.region_geometry(size, t_mid)
    rng = np.random.default_rng(seed)
    chains = []
    for _ in range(n_loops):
        a = I._fourier_closed_curve(rng, 3, n_pts, 1 << 12) * (0.6 * g)
        b = I._fourier_closed_curve(rng, 3, n_pts, 1 << 12) * (0.6 * g)
        c = rng.uniform(-0.15 * g, 0.15 * g, 3)
        k = np.arange(n_pts)
        chains.append(dict(A=a[(-k) % n_pts] + c, B=b[k] + c, wA=np.zeros(3), wB=np.zeros(3)))
    delta = 0.6 * g / n_pts
    net = I.make_network(chains, 64.0, delta, t_mid, I.FLAT)
    net["geom"] = geom
    return net


@pytest.mark.parametrize("cosmo", [I.FLAT, I.MATTER])
def test_bounded_region_diamonds_equal_whole_volume(cosmo):
    net = _loops_in_region(4.0, 8.0)
    hc = I.HCOEF[cosmo]
    br = O.OracleRegion(net["recs"], net["box"], cosmo, hc, net["geom"])
    br.evolve(100000, intercommute=False)
    assert br.active == 0
    frz = br.read()
    assert np.all(frz["flags"] & O.FLAG_FROZEN)
    # whole-volume run, recording every slice
    wr = O.OracleRegion(net["recs"], net["box"], cosmo, hc)
    hist = {}
    smax = int(frz["step"].max())
    while wr.step <= smax:
        rec = wr.read()
        hist[wr.step] = rec[np.argsort(rec["id"])]
        wr.evolve(1, intercommute=False)
    for f in frz:
        h = hist[int(f["step"])][f["id"]]
        assert h["x"].tobytes() == f["x"].tobytes()
        assert h["x_prev"].tobytes() == f["x_prev"].tobytes()
        if f["flags"] & O.FLAG_HAS_R:
            hj = hist[int(f["step"])][f["next_id"]]
            assert hj["x"].tobytes() == f["r"].tobytes()
            assert hj["x_prev"].tobytes() == f["r_prev"].tobytes()
    # points stop one step after the bottom of their next diamond leaves the region:
    # check the exit face against the generator coordinates of that bottom
    nstop = 0
    for f in frz:
        if not f["flags"] & O.FLAG_HAS_R:
            continue
        c = br.coords(f["r_prev"])
        face = (int(f["flags"]) >> 8) - 1
        assert np.floor(c[face]) > 0 and np.all(np.floor(c[:face]) <= 0)
        nstop += 1
    assert nstop > 0


def test_bounded_region_cut_network_runs_to_completion():
    net = I.region_network(2000, 4.0, seed=3)
    assert np.any(net["recs"]["next_id"] < 0)
    rec, ev, st = O.run(net, 100000)
    assert np.all(rec["flags"] & O.FLAG_FROZEN)
    faces = (rec["flags"] >> 8) - 1
    assert set(np.unique(faces)) <= {-1, 0, 1, 2, 3}
    assert st["point_steps"] > len(rec)
