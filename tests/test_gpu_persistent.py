"""GPU tests of the persistent evolution of small regions (one workgroup per region,
pulled from a device counter, every step inside the kernel) against the oracle, region
by region, and of the step-kernel fallback when a step holds more crossings than a
workgroup keeps.

Bar: per region, records and events identical to the oracle's run of that region alone
(bitwise), as for the step kernels.
"""
import numpy as np
import pytest

import oracle as O
from paper_1011_4046_amd import inputs as I
from test_gpu_parity import assert_same_events, assert_same_records, say
from test_gpu_schedule import check_against_oracle, oracle_regions

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1011_4046_amd import semipar
    semipar.lib()
    return semipar


SMALL = [300, 0, 420, 120, 40, 380, 8, 250, 0, 160, 60, 400]


@pytest.mark.parametrize("lanes", [1, 3])
def test_persistent_small_regions_equal_oracle(S, lanes):
    say(f"case: persistent workgroups, sizes {SMALL}, seed 300, lanes {lanes}")
    parts, box = I.region_batch(SMALL, seed=300)
    assert max(len(p[0]) for p in parts) <= S.PERSISTENT_MAX
    orc = oracle_regions(parts, box, "small300")
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=1200, lanes=lanes,
                             screen=S.SCREEN_F32, persistent=1)
    check_against_oracle(res, parts, orc)


def test_persistent_regions_with_probability(S):
    say("case: persistent workgroups, p = 0.4, seed 9, sizes seed 301")
    parts, box = I.region_batch(SMALL, seed=301)
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, screen=S.SCREEN_F32, persistent=1, p=0.4,
                             seed=9)
    passed = 0
    for r, (recs, geom) in enumerate(parts):
        mine = res["out"][res["out_off"][4 * r]:res["out_off"][4 * r + 4]]
        ev = res["events"][res["events_off"][r]:res["events_off"][r + 1]]
        if len(recs) == 0:
            continue
        o, oe, ost = O.run(dict(recs=recs, box=box, cosmology=I.MATTER, geom=geom), 100000,
                           p=0.4, seed=9)
        assert_same_events(ev, oe)
        assert_same_records(mine, o)
        passed += int((oe["kind"] == 1).sum())
    assert passed > 0


def test_persistent_next_to_step_kernels(S):
    """Small regions run persistently while large ones in the same schedule take the step
    kernels: every region still equals the oracle's run of it alone."""
    sizes = [300, 5000, 120, 0, 2500, 60, 450]
    say(f"case: mixed small and large regions {sizes}, seed 302, persistent, 2 lanes")
    parts, box = I.region_batch(sizes, seed=302)
    orc = oracle_regions(parts, box, "mixed302")
    rs = S.RegionSet.from_parts(parts, box, I.MATTER, device=True)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, lanes=2, use_graph=True, screen=S.SCREEN_F32,
                             persistent=1)
    check_against_oracle(res, parts, orc)
    b = res["region_batch"]
    small = [r for r in range(len(sizes)) if 0 < len(parts[r][0]) <= S.PERSISTENT_MAX]
    large = [r for r in range(len(sizes)) if len(parts[r][0]) > S.PERSISTENT_MAX]
    assert not set(b[small]) & set(b[large])  # never in one batch


def test_persistent_tiling_in_dependency_order(S):
    say("case: tiling of VV 8^3 seed 3 (M=2, 6 layers), persistent, 2 lanes")
    net = I.vv_network(m=8, seed=3)
    parts, box, n_pred, succ, layer = I.tiling_regions(net, M=2, layers=6)
    orc = oracle_regions(parts, box, "tiling8")
    rs = S.RegionSet.from_parts(parts, box, I.MATTER, n_pred=n_pred, succ=succ)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, lanes=2, screen=S.SCREEN_F32, persistent=1)
    check_against_oracle(res, parts, orc)
    bb = res["region_batch"]
    for r in range(len(parts)):
        for q in succ[r]:
            if bb[r] >= 0 and bb[q] >= 0:
                assert bb[q] > bb[r], (r, q)


def grid_region(nx=18, n_keep=14, n_pts=64, v=0.5, z0=0.02, span=0.6):
    """nx open strings along x moving -z and nx along y moving +z, each the n_keep points
    of a straight string nearest the region's centre: nx^2 crossings within two steps,
    more in one step than a persistent workgroup keeps."""
    chains = []
    for i in range(nx):
        y = (i + 0.5) * span / nx - span / 2 + 0.0123
        c, d = I.straight_string(n_pts, 4.0, v=-v, origin=(-2.0 + 0.0071, y, z0), axis=0, vdir=2)
        chains.append(c)
    for j in range(nx):
        x = (j + 0.5) * span / nx - span / 2 + 0.0311
        c, d = I.straight_string(n_pts, 4.0, v=v, origin=(x, -2.0 + 0.0053, -z0), axis=1,
                                 vdir=2)
        chains.append(c)
    recs = I.records_from_chains(chains, 8.0, d)
    keep = np.zeros(len(recs), bool)
    for ci in range(2 * nx):
        axis = 0 if ci < nx else 1
        coord = recs["x_prev"][ci * n_pts:(ci + 1) * n_pts, axis]
        keep[ci * n_pts + np.argsort(np.abs(coord))[:n_keep]] = True
    out = recs[keep].copy()
    ids = out["id"]
    out["next_id"] = np.where(np.isin(out["next_id"], ids), out["next_id"], -1)
    out["prev_id"] = np.where(np.isin(out["prev_id"], ids), out["prev_id"], -1)
    geom, _ = I.region_geometry(4.0, 8.0, (0.0, 0.0, 0.0))
    return out, geom


def test_persistent_overflow_falls_back_to_step_kernels(S):
    say("case: 18 x 18 open strings in one region (504 points): too many crossings in a step "
        "for a persistent workgroup")
    recs, geom = grid_region()
    assert len(recs) <= S.PERSISTENT_MAX
    box = 16.0
    o, oe, ost = O.run(dict(recs=recs, box=box, cosmology=I.FLAT, geom=geom), 100000)
    assert np.bincount(oe["step"]).max() > S.PERSISTENT_EVENTS
    reg = S.Region.batch([(recs, geom)], box, I.FLAT)
    with pytest.raises(S.SemiparError) as e:
        reg.evolve(100000, screen=S.SCREEN_F32, persistent=1)
    assert e.value.code == -5
    reg.close()
    # the scheduler runs such a batch again from its surfaces on the step kernels
    rs = S.RegionSet.from_parts([(recs, geom)], box, I.FLAT)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, screen=S.SCREEN_F32, persistent=1)
    assert_same_events(res["events"], oe)
    assert_same_records(res["out"], o)
