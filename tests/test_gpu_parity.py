"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar (written here): events identical bit for bit (integer/topology), positions
within 1e-12 relative (bitwise equality expected, since both sides evaluate the same
FP64 expressions without contraction). Every test prints the case it runs first.
"""
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


def assert_same_state(gpu, orc):
    g, o = by_id(gpu), by_id(orc)
    assert np.array_equal(g["id"], o["id"])
    assert np.array_equal(g["next_id"], o["next_id"])
    assert np.array_equal(g["prev_id"], o["prev_id"])
    assert np.array_equal(g["step"], o["step"])
    for f in ("x", "x_prev"):
        scale = max(1.0, float(np.abs(o[f]).max()))
        err = float(np.abs(g[f] - o[f]).max()) / scale
        assert err <= REL_TOL, (f, err)
    # bitwise is what the design delivers; report if it ever is not
    assert g["x"].tobytes() == o["x"].tobytes()
    assert g["x_prev"].tobytes() == o["x_prev"].tobytes()


def assert_same_events(ge, oe):
    assert len(ge) == len(oe), (len(ge), len(oe))
    assert np.array_equal(ge["step"], oe["step"])
    assert np.array_equal(ge["id_a"], oe["id_a"])
    assert np.array_equal(ge["id_b"], oe["id_b"])
    assert ge.tobytes() == oe.tobytes()


def run_gpu(S, net, steps, t_end=float("inf"), **kw):
    r = S.Region(net["recs"], net["box"], net["cosmology"])
    st = r.evolve(steps, t_end, **kw)
    out = r.emit(), r.events(), st
    r.close()
    return out


def run_oracle(net, steps, t_end=float("inf"), intercommute=True):
    return O.run(net, steps, t_end, O.GRID, intercommute)


# ---------------------------------------------------------------------------------
def test_flat_kt_loops_no_intercommutation_closed_form(S):
    say("case: 8 KT loops x 256, flat, 2000 steps, intercommutation off")
    net = I.kt_loops()
    g, ge, st = run_gpu(S, net, 2000, intercommute=False)
    o, oe, _ = run_oracle(net, 2000, intercommute=False)
    assert len(ge) == 0 and st["steps"] == 2000 and st["point_steps"] == 2000 * 2048
    assert_same_state(g, o)


@pytest.mark.parametrize("screen", [0, 1])
def test_flat_kt_loops_full(S, screen):
    say(f"case: 8 KT loops x 256, flat, 2000 steps, p=1, screen={'f64' if screen == 0 else 'f32'}")
    net = I.kt_loops()
    g, ge, st = run_gpu(S, net, 2000, screen=screen)
    o, oe, ost = run_oracle(net, 2000)
    assert len(oe) > 100
    assert_same_events(ge, oe)
    assert_same_state(g, o)
    assert st["accepted"] == ost["accepted"] and st["confirmed"] == ost["confirmed"]


@pytest.mark.parametrize("m,seed", [(4, 0), (6, 1), (8, 2), (5, 3)])
def test_matter_vv_small_full_run(S, m, seed):
    say(f"case: VV {m}^3 seed {seed}, matter era, until min t >= 16")
    net = I.vv_network(m=m, seed=seed)
    g, ge, st = run_gpu(S, net, 100000, t_end=16.0)
    o, oe, ost = run_oracle(net, 100000, t_end=16.0)
    assert ost["steps"] == st["steps"] and st["steps"] > 100
    assert_same_events(ge, oe)
    assert_same_state(g, o)


def test_matter_vv_full_size_first_steps(S):
    """Full-size matter-era workload (32^3 VV, ~2.4e5 points), first 30 steps, in the
    benchmark's launch configuration (graph-captured step blocks)."""
    say("case: VV 32^3 seed 0, matter era, 30 steps, graph")
    net = I.vv_network()
    g, ge, st = run_gpu(S, net, 30, use_graph=True, steps_per_sync=30)
    o, oe, _ = run_oracle(net, 30)
    assert len(oe) > 1000
    assert_same_events(ge, oe)
    assert_same_state(g, o)


def test_screen_precision_does_not_change_events_full_run(S):
    """Property at full size: the FP32 screen only adds false positives, so the whole
    matter-era run gives the same events and positions as the FP64 screen."""
    say("case: VV 32^3 seed 0, matter era, 200 steps, f32 vs f64 screen")
    net = I.vv_network()
    a = run_gpu(S, net, 200, screen=0, use_graph=True)
    b = run_gpu(S, net, 200, screen=1, use_graph=True)
    assert_same_events(a[1], b[1])
    assert a[0].tobytes() == b[0].tobytes()
    assert b[2]["candidates"] >= a[2]["candidates"]


def test_screen_precision_dense_64_network_false_positive_rate(S):
    """The dense 64^3 network (about 1.9e6 points, L = 64 correlation lengths), 500 steps:
    the FP32 screen with its conservative margin gives the same events and positions as
    the FP64 screen. Its false-positive rate is (cand_f32 - cand_f64) / cand_f32; both
    screens test the same spatial boxes and the FP32 ones are rounded outward by a few
    ulps, so it must stay small."""
    say("case: VV 64^3 seed 0, matter era, 500 steps, f32 vs f64 screen")
    net = I.vv_network(m=64, seed=0)
    a = run_gpu(S, net, 500, screen=0, use_graph=True)
    b = run_gpu(S, net, 500, screen=1, use_graph=True)
    assert_same_events(a[1], b[1])
    assert a[0].tobytes() == b[0].tobytes()
    c64, c32 = a[2]["candidates"], b[2]["candidates"]
    assert c32 >= c64 > 0
    rate = (c32 - c64) / c32
    say(f"  {len(net['recs'])} points, candidates f64 {c64} f32 {c32}, "
        f"false-positive rate {rate:.2e}, events {len(a[1])}")
    assert rate < 1e-2


def test_radiation_era_parity(S):
    """Radiation era (H = 1/eta) against the oracle: same first-order diamond with the
    other Hubble coefficient."""
    say("case: VV 6^3 seed 4, radiation era, 150 steps")
    net = I.vv_network(m=6, seed=4, cosmology=I.RADIATION)
    g, ge, st = run_gpu(S, net, 150, use_graph=True)
    o, oe, _ = run_oracle(net, 150)
    assert_same_events(ge, oe)
    assert_same_state(g, o)


@pytest.mark.parametrize("split", [1, 2, 5, 7])
def test_screen_split_variants(S, split):
    say(f"case: VV 8^3 seed 2, matter era, 150 steps, screen split {split}")
    net = I.vv_network(m=8, seed=2)
    g, ge, st = run_gpu(S, net, 150, screen_split=split)
    o, oe, _ = run_oracle(net, 150)
    assert_same_events(ge, oe)
    assert_same_state(g, o)


def test_graph_and_eager_identical(S):
    say("case: 8 KT loops, 600 steps, eager vs graph (K=7)")
    net = I.kt_loops()
    a = run_gpu(S, net, 600)
    b = run_gpu(S, net, 600, use_graph=True, steps_per_sync=7)
    assert_same_events(a[1], b[1])
    assert a[0].tobytes() == b[0].tobytes()


@pytest.mark.parametrize("cell", [1e-6, 0.9])
def test_large_element_path(S, cell):
    """Tiny cells (every element larger than a cell) and one huge cell (no hash at
    all) must still find exactly the oracle's events."""
    say(f"case: 3 KT loops x 64, flat, 300 steps, cell={cell}")
    net = I.kt_loops(n_loops=3, n_pts=64, seed=4)
    g, ge, st = run_gpu(S, net, 300, cell_size=cell)
    o, oe, _ = run_oracle(net, 300)
    assert st["large_elements"] > 0
    assert_same_events(ge, oe)
    assert_same_state(g, o)


def test_buffer_overflow_retakes_step(S):
    say("case: VV 6^3, matter, tiny candidate/event buffers (deferred steps)")
    net = I.vv_network(m=6, seed=1)
    g, ge, st = run_gpu(S, net, 120, cand_per_point=1e-4, events_per_point=1e-4)
    o, oe, _ = run_oracle(net, 120)
    assert_same_events(ge, oe)
    assert_same_state(g, o)


def test_ragged_and_degenerate_inputs(S):
    say("case: ragged sizes: loops of 3, 5, 257 points; 2-point loop")
    rng = np.random.default_rng(9)
    chains = []
    for n in (3, 5, 257, 2):
        P = rng.uniform(0.3, 0.7, (n, 3))
        chains.append(dict(A=P, B=P[::-1].copy(), wA=np.zeros(3), wB=np.zeros(3)))
    net = I.make_network(chains, 1.0, 1.0 / 64, 0.0, I.FLAT)
    g, ge, st = run_gpu(S, net, 150)
    o, oe, _ = run_oracle(net, 150)
    assert_same_events(ge, oe)
    assert_same_state(g, o)


def test_empty_region(S):
    say("case: empty region")
    net = I.kt_loops(n_loops=1, n_pts=8)
    r = S.Region(net["recs"][:0], 1.0, I.FLAT)
    st = r.evolve(100)
    assert st["steps"] == 0 and st["point_steps"] == 0
    assert len(r.emit()) == 0 and len(r.events()) == 0
    r.close()


def test_surface_errors(S):
    say("case: invalid surfaces")
    net = I.kt_loops(n_loops=2, n_pts=16)
    recs = net["recs"].copy()
    recs["id"][3] = recs["id"][4]
    with pytest.raises(S.SemiparError) as e:
        S.Region(recs, 1.0, I.FLAT)
    assert e.value.code == -2
    recs = net["recs"].copy()
    recs["next_id"][2] = 12345
    with pytest.raises(S.SemiparError):
        S.Region(recs, 1.0, I.FLAT)


def test_device_resident_input_and_output(S):
    import torch
    say("case: device-resident records in and out (VV 8^3, matter, 80 steps)")
    net = I.vv_network(m=8, seed=5)
    raw = torch.from_numpy(net["recs"].view(np.uint8).copy()).cuda()
    r = S.Region(raw, net["box"], net["cosmology"])
    st = r.evolve(80)
    out = torch.zeros_like(raw)
    n = r.emit_device(out)
    torch.cuda.synchronize()
    g = out.cpu().numpy().view(I.REC_DTYPE)[:n]
    ge = r.events()
    r.close()
    o, oe, _ = run_oracle(net, 80)
    assert_same_events(ge, oe)
    assert_same_state(g, o)


def test_matter_static_string_bitwise_static_gpu(S):
    say("case: static straight string, matter era")
    chain, delta = I.straight_string(32, 4.0, v=0.0)
    net = I.make_network([chain], 4.0, delta, 8.0, I.MATTER)
    g, ge, st = run_gpu(S, net, 100)
    g = by_id(g)
    n = int(g["step"][0])
    assert np.all(g["x"][:, 0] == (np.arange(32) + n / 2) * delta)
    assert np.all(g["x"][:, 1:3] == 0.0)
    assert np.all(g["x"][:, 3] == 8.0 + n * delta / 2)


def test_repeat_runs_identical(S):
    say("case: determinism, VV 8^3 twice")
    net = I.vv_network(m=8, seed=7)
    a = run_gpu(S, net, 150)
    b = run_gpu(S, net, 150)
    assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()


# ---------------------------------------------------------------------------------
# bounded regions (one 4-cube of the tiling)
# ---------------------------------------------------------------------------------
def run_gpu_region(S, net, steps=100000, **kw):
    r = S.Region(net["recs"], net["box"], net["cosmology"], geom=net["geom"])
    st = r.evolve(steps, **kw)
    faces, ev = r.emit_faces(), r.events()
    r.close()
    return faces, ev, st


def assert_same_records(g, o):
    g, o = by_id(g), by_id(o)
    assert len(g) == len(o)
    for f in ("id", "next_id", "prev_id", "step", "flags"):
        assert np.array_equal(g[f], o[f]), f
    for f in ("x", "x_prev", "r", "r_prev"):
        scale = max(1.0, float(np.abs(o[f]).max()) if len(o) else 1.0)
        assert float(np.abs(g[f] - o[f]).max() if len(o) else 0.0) / scale <= REL_TOL, f
    assert g.tobytes() == o.tobytes()


def check_faces(faces):
    for f, recs in enumerate(faces):
        face = (recs["flags"] >> 8) - 1
        frozen = (recs["flags"] & 2) != 0
        if f == 0:
            assert np.all(~frozen | (face <= 0))
        else:
            assert np.all(frozen & (face == f))


@pytest.mark.parametrize("n_target,seed,screen", [(600, 1, 0), (3000, 2, 1), (20000, 3, 1),
                                                  (20000, 4, 0)])
def test_bounded_region_matter_parity(S, n_target, seed, screen):
    say(f"case: bounded region, VV cut to the octahedron, ~{n_target} points, seed {seed}, "
        f"screen {screen}")
    net = I.region_network(n_target, 4.0, seed=seed)
    faces, ge, st = run_gpu_region(S, net, screen=screen)
    o, oe, ost = run_oracle(net, 100000)
    assert st["steps"] == ost["steps"] and st["point_steps"] == ost["point_steps"]
    assert_same_events(ge, oe)
    assert_same_records(np.concatenate(faces), o)
    check_faces(faces)


def _loops_in_region(size, t_mid, n_loops=3, n_pts=64, seed=0, cosmology=I.FLAT):
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


@pytest.mark.parametrize("cosmo", [I.FLAT, I.MATTER])
def test_bounded_region_loops_parity(S, cosmo):
    say(f"case: bounded region with closed loops, cosmology {cosmo}")
    net = _loops_in_region(4.0, 8.0, n_loops=6, n_pts=128, seed=11, cosmology=cosmo)
    faces, ge, st = run_gpu_region(S, net)
    o, oe, _ = run_oracle(net, 100000)
    assert_same_events(ge, oe)
    assert_same_records(np.concatenate(faces), o)


def test_bounded_region_stopped_early_emits_active(S):
    say("case: bounded region stopped after 10 steps")
    net = I.region_network(3000, 4.0, seed=5)
    faces, ge, st = run_gpu_region(S, net, steps=10)
    o, oe, _ = run_oracle(net, 10)
    g = np.concatenate(faces)
    assert np.any(g["flags"] & 4) and np.any(g["flags"] & 2)
    assert_same_events(ge, oe)
    assert_same_records(g, o)


def test_bounded_empty_region(S):
    say("case: empty bounded region")
    net = I.region_network(0, 4.0, seed=0)
    faces, ge, st = run_gpu_region(S, net)
    assert st["steps"] == 0 and sum(len(f) for f in faces) == 0 and len(ge) == 0


_batch_oracle = {}


BATCH_SIZES = {"big": [0, 300, 5000, 1200, 0, 20000, 800, 2500, 40, 9000],
               "small": [0, 300, 1200, 40, 800]}


@pytest.mark.parametrize("which,cell,screen", [("big", 0.0, 0), ("big", 0.0, 1),
                                               ("small", 1e-6, 1), ("small", 0.9, 0),
                                               ("big", 0.05, 1)])
def test_region_batch_equals_separate_regions(S, which, cell, screen):
    """A batch of independent regions evolved in one set of launches gives exactly the
    union of the regions' separate results (oracle, one region at a time), with each
    region's own adaptive grid or a fixed cell size (tiny: elements go to the
    large-element path; coarse: many elements per cell)."""
    sizes = BATCH_SIZES[which]
    say(f"case: batch of {len(sizes)} regions, sizes {sizes}, cell {cell}, screen {screen}")
    parts, box = I.region_batch(sizes, seed=100)
    r = S.Region.batch(parts, box, I.MATTER)
    st = r.evolve(100000, cell_size=cell, screen=screen, use_graph=cell > 0)
    faces, ge = r.emit_faces(), r.events()
    r.close()
    if which not in _batch_oracle:
        recs, evs, psteps, steps = [], [], 0, 0
        for recs_i, geom in parts:
            if len(recs_i) == 0:
                continue
            net = dict(recs=recs_i, box=box, cosmology=I.MATTER, geom=geom)
            o, oe, ost = run_oracle(net, 100000)
            recs.append(o)
            evs.append(oe)
            psteps += ost["point_steps"]
            steps = max(steps, ost["steps"])
        _batch_oracle[which] = dict(recs=recs, evs=evs, psteps=psteps, steps=steps)
    cached = _batch_oracle[which]
    recs, evs = cached["recs"], cached["evs"]
    psteps, steps = cached["psteps"], cached["steps"]
    oe = np.concatenate(evs)
    oe = oe[np.lexsort((oe["id_b"], oe["id_a"], oe["t_star"], oe["step"]))]
    assert st["point_steps"] == psteps and st["steps"] == steps
    assert_same_events(ge, oe)
    assert_same_records(np.concatenate(faces), np.concatenate(recs))


def _pair_keys(pairs, base):
    return pairs[:, 0].astype(np.int64) * base + pairs[:, 1].astype(np.int64)


def test_screen_candidates_per_step_nest(S):
    """P6 per step, on a mid-size network (VV 16^3, about 3e4 points, 60 steps): the
    oracle's exact 4-D box-overlap pairs of the band are among the FP64 screen's pairs,
    which are among the FP32 screen's pairs (outward-rounded boxes with a margin only
    add false positives). Events and positions stay identical."""
    say("case: VV 16^3 seed 5, matter era, 60 single steps, oracle exact ⊆ f64 ⊆ f32")
    net = I.vv_network(m=16, seed=5)
    base = int(net["recs"]["id"].max()) + 1
    a = S.Region(net["recs"], net["box"], net["cosmology"])
    b = S.Region(net["recs"], net["box"], net["cosmology"])
    o = O.OracleRegion(net["recs"], net["box"], I.MATTER, I.HCOEF[I.MATTER])
    n64 = n32 = nex = 0
    for step in range(60):
        exact = o.band_candidates(O.GRID)
        o.evolve(1)
        a.evolve(1, screen=0)
        b.evolve(1, screen=1)
        c64, c32 = a.candidates(), b.candidates()
        k_ex, k64, k32 = (_pair_keys(c, base) for c in (exact, c64, c32))
        assert len(np.unique(k64)) == len(k64) and len(np.unique(k32)) == len(k32), step
        assert np.isin(k_ex, k64).all(), f"step {step}: the FP64 screen missed an overlap"
        assert np.isin(k64, k32).all(), f"step {step}: the FP32 screen missed an FP64 pair"
        n64, n32, nex = n64 + len(k64), n32 + len(k32), nex + len(k_ex)
    assert nex > 0
    ge, be = a.events(), b.events()
    assert_same_events(ge, o.events())
    assert_same_events(be, ge)
    ga, gb = a.emit(), b.emit()
    assert_same_state(ga, o.read())
    assert ga.tobytes() == gb.tobytes()
    say(f"  pairs over 60 steps: exact {nex}, f64 screen {n64}, f32 screen {n32} "
        f"(f32 false-positive rate over f64 {(n32 - n64) / max(n32, 1):.2e})")
    for r in (a, b):
        r.close()
    o.close()


@pytest.mark.parametrize("screen", [0, 1])
def test_buffer_overflow_retakes_step_bounded_region(S, screen):
    """A bounded region with candidate and event buffers far too small: overflowing
    steps are retaken after the buffers grow, although the first attempt already wrote
    stop steps, faces, stopped records and wave flags. Results equal the oracle's."""
    say(f"case: bounded region ~3000 points seed 2, tiny buffers, screen {screen}")
    net = I.region_network(3000, 4.0, seed=2)
    faces, ge, st = run_gpu_region(S, net, screen=screen, cand_per_point=1e-5,
                                   events_per_point=1e-5, use_graph=True, steps_per_sync=8)
    o, oe, ost = run_oracle(net, 100000)
    assert st["steps"] == ost["steps"] and st["point_steps"] == ost["point_steps"]
    assert_same_events(ge, oe)
    assert_same_records(np.concatenate(faces), o)
    check_faces(faces)


def test_buffer_overflow_retakes_step_batch(S):
    """The same for a batch of regions through schedule_regions (one batch)."""
    say("case: batch of 6 regions (seed 41), tiny buffers, one batch, f32 screen")
    sizes = [900, 0, 2500, 300, 1600, 50]
    parts, box = I.region_batch(sizes, seed=41)
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=0, use_graph=True,
                             screen=S.SCREEN_F32, steps_per_sync=8, cand_per_point=1e-5,
                             events_per_point=1e-5)
    assert res["stats"]["batches"] == 1
    for r, (recs, geom) in enumerate(parts):
        mine = res["out"][res["out_off"][4 * r]:res["out_off"][4 * r + 4]]
        ev = res["events"][res["events_off"][r]:res["events_off"][r + 1]]
        if len(recs) == 0:
            assert len(mine) == 0 and len(ev) == 0
            continue
        o, oe, ost = O.run(dict(recs=recs, box=box, cosmology=I.MATTER, geom=geom), 100000)
        assert_same_events(ev, oe)
        assert_same_records(mine, o)
        assert res["region_point_steps"][r] == ost["point_steps"]


@pytest.mark.parametrize("screen", [0, 1])
def test_precomputed_pencil_screen_bounded_and_wrapping(S, screen):
    """The screen variant whose pencil ranges are written by the bucket sort: a bounded
    region (local grid, no wrap) and a whole-volume network in a small periodic box
    (the z-pencils wrap, so some pencils are looked up cell by cell) equal the oracle."""
    say(f"case: precomputed pencils, screen {screen}: bounded ~3000 seed 2; VV 4^3 seed 1")
    net = I.region_network(3000, 4.0, seed=2)
    faces, ge, st = run_gpu_region(S, net, screen=screen, screen_split=2, use_graph=True)
    o, oe, ost = run_oracle(net, 100000)
    assert_same_events(ge, oe)
    assert_same_records(np.concatenate(faces), o)
    small = I.vv_network(m=4, seed=1)
    g, ge, st = run_gpu(S, small, 200, screen=screen, screen_split=2)
    o, oe, _ = run_oracle(small, 200)
    assert_same_events(ge, oe)
    assert_same_state(g, o)
