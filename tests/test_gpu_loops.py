"""GPU parity of loop record and removal (through the C ABI) against the oracle: the
same loops removed at the same steps (step, size and representative exact; energy and
centre to 1e-12), the same events, and the same final records, bit for bit, in
whole-volume regions, bounded regions, batches and the scheduler, over one evolve call
or several."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1011_4046_amd import inputs as I

pytestmark = pytest.mark.gpu

REL_TOL = 1e-12


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1011_4046_amd import semipar
    semipar.lib()
    return semipar


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def by_id(recs):
    return recs[np.argsort(recs["id"], kind="stable")]


def sort_loops(lp):
    return lp[np.lexsort((lp["rep_id"], lp["step"]))]


def assert_same_loops(g, o, box):
    o = sort_loops(o)
    assert len(g) == len(o), (len(g), len(o))
    for f in ("step", "n_points", "rep_id"):
        assert np.array_equal(g[f], o[f]), f
    if len(o):
        err = np.abs(g["energy"] - o["energy"]) / np.maximum(np.abs(o["energy"]), 1e-300)
        assert float(err.max()) <= REL_TOL
        assert float(np.abs(g["centre"] - o["centre"]).max()) <= REL_TOL * box


def assert_same_records(g, o):
    g, o = by_id(g), by_id(o)
    assert len(g) == len(o)
    for f in ("id", "next_id", "prev_id", "step", "flags"):
        assert np.array_equal(g[f], o[f]), f
    assert g.tobytes() == o.tobytes()


def assert_same_events(ge, oe):
    assert len(ge) == len(oe), (len(ge), len(oe))
    assert ge.tobytes() == oe.tobytes()


def oracle_region(net):
    hc = {0: 0.0, 1: 2.0, 2: 1.0}[net["cosmology"]]
    return O.OracleRegion(net["recs"], net["box"], net["cosmology"], hc, net.get("geom"))


def run_both(S, net, calls, every, intercommute=True, **kw):
    """Evolve on the GPU and in the oracle with the same sequence of calls, each
    (max_steps, t_end). Returns (gpu records, events, loops, stats list) and the same
    for the oracle."""
    r = S.Region(net["recs"], net["box"], net["cosmology"], geom=net.get("geom"))
    o = oracle_region(net)
    sts = []
    for steps, t_end in calls:
        sts.append(r.evolve(steps, t_end, intercommute=intercommute, loop_every=every, **kw))
        o.evolve(steps, t_end, O.GRID, intercommute, every)
    g = (r.emit(), r.events(), r.loops(), sts)
    r.close()
    oo = (o.read(), o.events(), o.loops(), o.stats())
    o.close()
    return g, oo


def test_flat_loops_removed_after_one_period(S):
    say("case: 8 KT loops x 256, flat, no intercommutation, loop_every 64, 300 steps")
    net = I.kt_loops(n_loops=8, n_pts=256, box=4.0, seed=3)
    g, o = run_both(S, net, [(300, float("inf"))], 64, intercommute=False)
    assert len(o[2]) == 8 and np.all(o[2]["step"] == 257)
    assert_same_loops(g[2], o[2], 4.0)
    assert_same_records(g[0], o[0])
    assert np.all(g[0]["flags"] == S.FLAG_REMOVED)
    st = g[3][0]
    assert st["loops"] == 8 and st["loop_points"] == 2048
    # the evolution stops once no point advances: 256 steps taken
    assert st["steps"] == 256 and st["point_steps"] == 256 * 2048


@pytest.mark.parametrize("graph,sync", [(False, 0), (True, 32), (True, 7)])
def test_flat_kt_with_intercommutation(S, graph, sync):
    say(f"case: 8 KT loops x 256, flat, p=1, loop_every 16, 600 steps, graph {graph}, "
        f"sync {sync}")
    net = I.kt_loops()
    g, o = run_both(S, net, [(600, float("inf"))], 16, use_graph=graph, steps_per_sync=sync)
    assert len(o[2]) > 100
    assert_same_events(g[1], o[1])
    assert_same_loops(g[2], o[2], net["box"])
    assert_same_records(g[0], o[0])


@pytest.mark.parametrize("m,seed,every", [(6, 1, 8), (8, 2, 5), (5, 3, 1)])
def test_matter_vv_until_t_end(S, m, seed, every):
    say(f"case: VV {m}^3 seed {seed}, matter era, loop_every {every}, until min t >= 16")
    net = I.vv_network(m=m, seed=seed)
    g, o = run_both(S, net, [(100000, 16.0)], every, use_graph=True)
    assert len(o[2]) > 10
    assert g[3][0]["steps"] == o[3]["steps"]
    assert_same_events(g[1], o[1])
    assert_same_loops(g[2], o[2], net["box"])
    assert_same_records(g[0], o[0])


def test_full_size_network_in_bench_launch_configuration(S):
    """Full-size matter-era workload (32^3 VV, ~2.4e5 points), 80 steps with a check
    every 8 (thousands of loops), graph-captured blocks of 32 steps, FP32 screen."""
    say("case: VV 32^3 seed 0, matter, loop_every 8, 80 steps, graph, sync 32, f32 screen")
    net = I.vv_network()
    g, o = run_both(S, net, [(80, np.inf)], 8, use_graph=True, steps_per_sync=32,
                    screen=S.SCREEN_F32, screen_split=1)
    assert len(o[2]) > 1000
    assert_same_events(g[1], o[1])
    assert_same_loops(g[2], o[2], net["box"])
    assert_same_records(g[0], o[0])


def test_several_calls_equal_the_oracle_with_the_same_calls(S):
    """Calls that end on, before and after check steps, and one cut by t_end: the
    checks fall at the same steps as in the oracle driven by the same calls."""
    say("case: VV 6^3 seed 1, matter era, loop_every 8, calls of 7, 8, 1, 37, 100 steps")
    net = I.vv_network(m=6, seed=1)
    calls = [(7, np.inf), (8, np.inf), (1, np.inf), (37, np.inf), (100, 12.0), (300, 16.0)]
    g, o = run_both(S, net, calls, 8, use_graph=True, steps_per_sync=5)
    assert len(o[2]) > 10
    assert_same_events(g[1], o[1])
    assert_same_loops(g[2], o[2], net["box"])
    assert_same_records(g[0], o[0])


def test_removal_enabled_in_a_later_call(S):
    """Events are tracked from init: removal switched on after 40 steps without it."""
    say("case: VV 6^3 seed 1, matter, 40 steps without removal, then loop_every 8")
    net = I.vv_network(m=6, seed=1)
    r = S.Region(net["recs"], net["box"], net["cosmology"])
    o = oracle_region(net)
    r.evolve(40)
    o.evolve(40, np.inf, O.GRID, True, 0)
    r.evolve(200, loop_every=8)
    o.evolve(200, np.inf, O.GRID, True, 8)
    assert len(o.loops()) > 0
    assert_same_loops(r.loops(), o.loops(), net["box"])
    assert_same_events(r.events(), o.events())
    assert_same_records(r.emit(), o.read())
    r.close()
    o.close()


def test_winding_string_is_never_removed(S):
    say("case: straight string winding the box, flat, loop_every 16, 400 steps")
    chain, delta = I.straight_string(128, 4.0, v=0.3)
    net = I.make_network([chain], 4.0, delta, 0.0, I.FLAT)
    g, o = run_both(S, net, [(400, np.inf)], 16, intercommute=False)
    assert len(g[2]) == 0 and len(o[2]) == 0
    assert_same_records(g[0], o[0])


def _loops_in_region(size, t_mid, n_loops, n_pts, seed, cosmology):
    geom, g = I.region_geometry(size, t_mid)
    rng = np.random.default_rng(seed)
    chains = []
    for _ in range(n_loops):
        a = I._fourier_closed_curve(rng, 3, n_pts, 1 << 12) * (0.6 * g)
        b = I._fourier_closed_curve(rng, 3, n_pts, 1 << 12) * (0.6 * g)
        c = rng.uniform(-0.15 * g, 0.15 * g, 3)
        k = np.arange(n_pts)
        chains.append(dict(A=a[(-k) % n_pts] + c, B=b[k] + c, wA=np.zeros(3), wB=np.zeros(3)))
    net = I.make_network(chains, 64.0, 0.6 * g / n_pts, t_mid, cosmology)
    net["geom"] = geom
    return net


@pytest.mark.parametrize("cosmo,n_pts,every", [(I.FLAT, 32, 4), (I.MATTER, 64, 4),
                                               (I.MATTER, 16, 2)])
def test_bounded_region(S, cosmo, n_pts, every):
    say(f"case: bounded region, 6 loops x {n_pts}, cosmology {cosmo}, loop_every {every}")
    net = _loops_in_region(4.0, 8.0, 6, n_pts, 11, cosmo)
    r = S.Region(net["recs"], net["box"], net["cosmology"], geom=net["geom"])
    r.evolve(100000, loop_every=every)
    faces, ge, gl = r.emit_faces(), r.events(), r.loops()
    r.close()
    o = oracle_region(net)
    o.evolve(100000, np.inf, O.GRID, True, every)
    assert len(o.loops()) > 10
    assert_same_events(ge, o.events())
    assert_same_loops(gl, o.loops(), net["box"])
    assert_same_records(np.concatenate(faces), o.read())
    # removed points go to stream 0 with no owning face
    rem = np.concatenate(faces[1:])
    assert not np.any(rem["flags"] & S.FLAG_REMOVED)
    assert np.any(faces[0]["flags"] & S.FLAG_REMOVED)
    o.close()


SIZES = [0, 300, 1200, 40, 800, 2500]


@pytest.fixture(scope="module")
def batch_oracle():
    parts, box = I.region_batch(SIZES, seed=100)
    out = []
    for recs_i, geom in parts:
        if len(recs_i) == 0:
            out.append((recs_i, np.zeros(0, I.EVENT_DTYPE), np.zeros(0, I.LOOP_DTYPE)))
            continue
        o = O.OracleRegion(recs_i, box, I.MATTER, 2.0, geom)
        o.evolve(100000, np.inf, O.GRID, True, 4)
        out.append((o.read(), o.events(), o.loops()))
        o.close()
    return parts, box, out


def test_batch_equals_separate_regions(S, batch_oracle):
    say(f"case: batch of {len(SIZES)} bounded regions {SIZES}, matter, loop_every 4")
    parts, box, ref = batch_oracle
    r = S.Region.batch(parts, box, I.MATTER)
    st = r.evolve(100000, loop_every=4, use_graph=True)
    faces, ge, gl = r.emit_faces(), r.events(), r.loops()
    r.close()
    recs = np.concatenate([x[0] for x in ref])
    evs = np.concatenate([x[1] for x in ref])
    lps = np.concatenate([x[2] for x in ref])
    assert len(lps) > 10 and st["loops"] == len(lps)
    assert_same_loops(gl, lps, box)
    assert_same_records(np.concatenate(faces), recs)
    key = lambda e: np.lexsort((e["id_b"], e["id_a"], e["t_star"], e["step"]))
    assert ge[key(ge)].tobytes() == evs[key(evs)].tobytes()


@pytest.mark.parametrize("policy,batch_points,lanes", [(0, 0, 1), (1, 0, 1), (1, 1500, 2)])
def test_schedule_regions_loops_per_region(S, batch_oracle, policy, batch_points, lanes):
    say(f"case: schedule_regions policy {policy}, batch_points {batch_points}, lanes {lanes}, "
        f"loop_every 4")
    parts, box, ref = batch_oracle
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    res = S.schedule_regions(rs, policy, batch_points=batch_points, lanes=lanes, loop_every=4,
                             use_graph=True)
    off = res["loops_off"]
    assert res["stats"]["loops"] == sum(len(x[2]) for x in ref)
    for q, (recs, evs, lps) in enumerate(ref):
        assert_same_loops(res["loops"][off[q]:off[q + 1]], lps, box)
        oo = res["out_off"]
        assert_same_records(res["out"][oo[4 * q]:oo[4 * q + 4]], recs)
