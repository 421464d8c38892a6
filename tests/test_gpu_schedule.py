"""GPU tests of the many-region path: schedule_regions against the oracle run region by
region, the cost-model features and FP32 kernels against the FP64 oracle, and the
gain of the trained cost model over the point-count heuristic.

Bars: per region, records and events identical to the oracle's run of that region
alone (bitwise), under every policy and packing; features within FP32 rounding of the
FP64 oracle (1e-5 relative); forward within 1e-5, gradient within 1e-3 (norm-wise,
FP32 against FP64) and the Adam update within 1e-6 relative.
"""
import numpy as np
import pytest

import oracle as O
from oracle import costmodel as C
from paper_1011_4046_amd import inputs as I
from test_gpu_parity import assert_same_events, assert_same_records, check_faces, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1011_4046_amd import semipar
    semipar.lib()
    return semipar


_oracle_cache = {}


def oracle_regions(parts, box, key):
    """Each region run alone by the oracle: (records, events, stats, steps advanced)."""
    if key in _oracle_cache:
        return _oracle_cache[key]
    res = []
    for recs, geom in parts:
        if len(recs) == 0:
            res.append(None)
            continue
        net = dict(recs=recs, box=box, cosmology=I.MATTER, geom=geom)
        o, oe, ost = O.run(net, 100000)
        res.append((o, oe, ost, int(o["step"].max()) - int(recs["step"][0])))
    _oracle_cache[key] = res
    return res


def check_against_oracle(res, parts, orc):
    out, off = res["out"], res["out_off"]
    ev, eoff = res["events"], res["events_off"]
    total_ps = 0
    for r, (recs, geom) in enumerate(parts):
        mine = out[off[4 * r]:off[4 * r + 4]]
        mine_ev = ev[eoff[r]:eoff[r + 1]]
        if orc[r] is None:
            assert len(mine) == 0 and len(mine_ev) == 0
            assert res["region_batch"][r] == -1
            continue
        o, oe, ost, steps = orc[r]
        assert_same_records(mine, o)
        assert_same_events(mine_ev, oe)
        check_faces([out[off[4 * r + f]:off[4 * r + f + 1]] for f in range(4)])
        assert res["region_point_steps"][r] == ost["point_steps"]
        assert res["region_steps"][r] == steps
        total_ps += ost["point_steps"]
    assert res["stats"]["point_steps"] == total_ps


SIZES = [0, 300, 5000, 1200, 0, 20000, 800, 2500, 40, 9000, 150, 3000]


@pytest.mark.parametrize("case", ["plain", "batched-heuristic", "batched-cost", "one-batch-f32",
                                  "lanes", "lanes-small-batches", "work-packing",
                                  "precomputed-pencils"])
def test_schedule_policies_equal_oracle_region_by_region(S, case):
    say(f"case: schedule_regions {case}, sizes {SIZES}, seed 200")
    parts, box = I.region_batch(SIZES, seed=200)
    orc = oracle_regions(parts, box, "sizes200")
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    if case == "plain":
        res = S.schedule_regions(rs, S.SCHED_PLAIN, steps_per_sync=1)
        assert res["stats"]["batches"] == 10
    elif case == "batched-heuristic":
        res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=6000, use_graph=True,
                                 screen=S.SCREEN_F32)
        assert res["stats"]["batches"] >= 4
        # point-count order: the batch index never decreases as regions get smaller
        nz = [r for r in range(len(SIZES)) if len(parts[r][0])]
        order = sorted(nz, key=lambda r: -len(parts[r][0]))
        b = [res["region_batch"][r] for r in order]
        assert b == sorted(b)
    elif case == "batched-cost":
        cost = np.random.default_rng(5).permutation(len(SIZES)).astype(np.float32)
        res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=8000, cost=cost)
        nz = [r for r in range(len(SIZES)) if len(parts[r][0])]
        order = sorted(nz, key=lambda r: -cost[r])
        b = [res["region_batch"][r] for r in order]
        assert b == sorted(b)
    elif case == "work-packing":
        # equal shares of predicted point-steps (points x cost) over 3 batches (one lane,
        # so that the batches run, and are numbered, in cut order)
        cost = np.random.default_rng(6).uniform(10, 300, len(SIZES)).astype(np.float32)
        bp = -(-int(rs.counts.sum()) // 3)
        res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=bp, cost=cost, lanes=1,
                                 pack=S.PACK_WORK, use_graph=True, screen=S.SCREEN_F32)
        nz = [r for r in range(len(SIZES)) if len(parts[r][0])]
        order = sorted(nz, key=lambda r: -cost[r])
        b = [res["region_batch"][r] for r in order]
        assert res["stats"]["batches"] == 3
        # cut in cost order: region i opens a new batch when the predicted work before it
        # has reached (batches so far) shares and fewer than 3 batches exist
        wk = [len(parts[r][0]) * float(cost[r]) for r in order]
        share = sum(wk) / 3
        want, done = [], 0.0
        for w in wk:
            if not want or (want[-1] + 1 < 3 and done >= share * (want[-1] + 1)):
                want.append(len(want) and want[-1] + 1)
            else:
                want.append(want[-1])
            done += w
        assert [x - b[0] for x in b] == want
    elif case == "precomputed-pencils":
        # the screen variant reading pencil ranges written by the bucket sort
        res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=6000, use_graph=True,
                                 screen=S.SCREEN_F32, screen_split=2, lanes=2)
        assert res["stats"]["batches"] >= 4
    elif case == "lanes-small-batches":
        # many small batches on three lanes: one lane builds a batch (copies, fills) while
        # another captures its step graph, which must not disturb the capture
        res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=1500, use_graph=True,
                                 screen=S.SCREEN_F32, lanes=3)
        assert res["stats"]["batches"] >= 6
    elif case == "lanes":
        # batches evolved concurrently by three host threads on streams of their own
        res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=6000, use_graph=True,
                                 screen=S.SCREEN_F32, lanes=3)
        assert res["stats"]["batches"] >= 4
    else:
        res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=0, use_graph=True,
                                 screen=S.SCREEN_F32, steps_per_sync=16)
        assert res["stats"]["batches"] == 1
    assert res["stats"]["empty_regions"] == 2 and res["stats"]["regions"] == len(SIZES)
    check_against_oracle(res, parts, orc)


@pytest.mark.parametrize("factor", [1.0, 1.3, 2.5, 4.0])
def test_cell_factor_changes_nothing(S, factor):
    """Cells of any edge from 1 to 4 times the largest element extent give the oracle's
    results: the cell factor (which the autotuner searches) is performance only."""
    say(f"case: schedule_regions BATCHED with cell factor {factor}, sizes {SIZES}, seed 200")
    parts, box = I.region_batch(SIZES, seed=200)
    orc = oracle_regions(parts, box, "sizes200")
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=6000, use_graph=True,
                             screen=S.SCREEN_F32, lanes=2, cell_factor=factor)
    check_against_oracle(res, parts, orc)


def test_cell_factor_outside_its_range_is_refused(S):
    parts, box = I.region_batch([400], seed=201)
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    for bad in (0.5, 4.5, -1.0, float("nan")):
        with pytest.raises(S.SemiparError) as e:
            S.schedule_regions(rs, S.SCHED_BATCHED, cell_factor=bad)
        assert e.value.code == -1


def test_schedule_device_resident_io_and_dependencies(S):
    """Device-resident input and output, and a dependency order: a region starts only
    in a later wave than all its predecessors; results unchanged."""
    import torch
    say("case: schedule_regions device I/O with a dependency DAG, sizes[:8], seed 200")
    sizes = SIZES[:8]
    parts, box = I.region_batch(sizes, seed=200)
    orc = oracle_regions(parts, box, "sizes200")[:8]
    succ = [[1, 2], [3], [3, 4], [5], [6], [7], [7], []]
    npred = [0] * 8
    for r in range(8):
        for q in succ[r]:
            npred[q] += 1
    rs = S.RegionSet.from_parts(parts, box, I.MATTER, device=True, n_pred=npred, succ=succ)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, out="device", use_graph=True,
                             screen=S.SCREEN_F32)
    torch.cuda.synchronize()
    res["out"] = res["out"].cpu().numpy().view(I.REC_DTYPE)[:int(rs.counts.sum())]
    check_against_oracle(res, parts, orc)
    b = res["region_batch"]
    for r in range(8):
        for q in succ[r]:
            if b[r] >= 0 and b[q] >= 0:
                assert b[q] > b[r], (r, q)


@pytest.mark.parametrize("policy,lanes", [(0, 1), (1, 1), (1, 3)])
def test_spacetime_tiling_in_dependency_order(S, policy, lanes):
    """A matter-era network cut at its initial slice into a periodic spacetime tiling
    (6 layers x 32 regions), run in dependency order: every region equals the
    oracle's run of that region alone, and no region runs before a predecessor."""
    say(f"case: tiling of VV 8^3 seed 3 (M=2, 6 layers), policy {policy}, lanes {lanes}")
    net = I.vv_network(m=8, seed=3)
    parts, box, n_pred, succ, layer = I.tiling_regions(net, M=2, layers=6)
    orc = oracle_regions(parts, box, "tiling8")
    rs = S.RegionSet.from_parts(parts, box, I.MATTER, n_pred=n_pred, succ=succ)
    res = S.schedule_regions(rs, policy, batch_points=1500 if lanes > 1 else 0, lanes=lanes,
                             use_graph=True, screen=S.SCREEN_F32)
    check_against_oracle(res, parts, orc)
    assert res["stats"]["regions"] == len(parts)
    assert res["stats"]["empty_regions"] == sum(1 for p in parts if len(p[0]) == 0)
    b = res["region_batch"]
    for r in range(len(parts)):
        for q in succ[r]:
            if b[r] >= 0 and b[q] >= 0:
                assert b[q] > b[r], (r, q)


@pytest.mark.parametrize("sleep_ms,submit_ms", [(0.0, 0.0), (0.5, 0.2), (5.0, 0.0)])
def test_worker_pool_policies_change_nothing(S, sleep_ms, submit_ms):
    """The paper's variable-size worker pool (lanes that sleep, exit when nothing comes,
    and are started again when batches wait) gives the same per-region results in
    dependency order as lanes held throughout; its time accounting is consistent:
    busy <= held <= lanes x makespan, and a held pool holds every lane for the run."""
    say(f"case: tiling of VV 8^3 seed 3 (M=2, 6 layers), 3 lanes, lane sleep {sleep_ms} ms, "
        f"submit {submit_ms} ms")
    net = I.vv_network(m=8, seed=3)
    parts, box, n_pred, succ, layer = I.tiling_regions(net, M=2, layers=6)
    orc = oracle_regions(parts, box, "tiling8")
    rs = S.RegionSet.from_parts(parts, box, I.MATTER, n_pred=n_pred, succ=succ)
    res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=1500, lanes=3, use_graph=True,
                             screen=S.SCREEN_F32, lane_sleep_ms=sleep_ms,
                             lane_submit_ms=submit_ms)
    check_against_oracle(res, parts, orc)
    st = res["stats"]
    b = res["region_batch"]
    for r in range(len(parts)):
        for q in succ[r]:
            if b[r] >= 0 and b[q] >= 0:
                assert b[q] > b[r], (r, q)
    assert st["lanes_started"] >= 3
    assert 0.0 < st["lane_busy_ms"] <= st["lane_held_ms"] + 1e-6
    assert st["lane_held_ms"] <= 3 * st["makespan_ms"] + 1e-6
    if sleep_ms == 0.0:
        assert st["lanes_started"] == 3
    with pytest.raises(S.SemiparError) as e:
        S.schedule_regions(rs, S.SCHED_BATCHED, lanes=3, lane_sleep_ms=-1.0)
    assert e.value.code == -1


@pytest.mark.parametrize("device", [False, True])
def test_region_features_match_oracle(S, device):
    """Host surfaces go through a batch region of all regions; device surfaces are read
    in place. Both give the oracle's features."""
    say(f"case: cost-model features of 12 regions (seed 200) and two strings, device {device}")
    parts, box = I.region_batch(SIZES, seed=200)
    chain, delta = I.straight_string(200, 16.0, v=0.6)
    s1 = I.make_network([chain], 16.0, delta, 8.0, I.MATTER)
    geom, _ = I.region_geometry(4.0, 8.0, (0.3, 0.2, 0.1))
    rs = S.RegionSet.from_parts(parts, box, I.MATTER, device=device)
    f = S.region_features(rs)
    for r, (recs, geom_r) in enumerate(parts):
        want = C.features(recs, geom_r, box)
        assert np.allclose(f[r], want, rtol=1e-5, atol=1e-6), (r, f[r], want)
    rs1 = S.RegionSet.from_parts([(s1["recs"], geom)], 16.0, I.MATTER, device=device)
    f1 = S.region_features(rs1)[0]
    assert np.allclose(f1, C.features(s1["recs"], geom, 16.0), rtol=1e-5, atol=1e-6)
    assert f1[2] == pytest.approx(0.6, rel=1e-5)
    # regions of a spacetime tiling: nonzero indices, one shared lattice origin, empty
    # regions among them (also the last ones)
    net = I.vv_network(m=8, seed=3)
    tparts, tbox, _, _, _ = I.tiling_regions(net, M=2, layers=6)
    assert len(tparts[-1][0]) == 0
    ft = S.region_features(S.RegionSet.from_parts(tparts, tbox, I.MATTER, device=device))
    for r, (recs, geom_r) in enumerate(tparts):
        want = C.features(recs, geom_r, tbox)
        assert np.allclose(ft[r], want, rtol=1e-5, atol=1e-6), (r, ft[r], want)


def test_region_features_in_place_equal_the_batch_path(S):
    say("case: features of the 512-region workload's first 64 regions, host vs device surfaces")
    nt = I.lognormal_regions(64, median=2e3, sigma=1.0, cap=2e4, p_empty=0.2, seed=5)
    parts, box = I.region_batch(nt, size=4.0, seed=5, slots=4)
    fh = S.region_features(S.RegionSet.from_parts(parts, box, I.MATTER))
    fd = S.region_features(S.RegionSet.from_parts(parts, box, I.MATTER, device=True))
    assert np.allclose(fh, fd, rtol=1e-6, atol=1e-7)
    assert np.all(fd[[len(p[0]) == 0 for p in parts]] == 0)


def test_region_features_reject_duplicate_ids_in_place(S):
    say("case: device surfaces with a duplicated id are rejected")
    parts, box = I.region_batch([300, 200], seed=7)
    recs = parts[1][0].copy()
    recs["id"][5] = parts[0][0]["id"][3]
    bad = [parts[0], (recs, parts[1][1])]
    with pytest.raises(S.SemiparError):
        S.region_features(S.RegionSet.from_parts(bad, box, I.MATTER, device=True))


def _mlp_case(seed, n=700):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.25, C.NP).astype(np.float32)
    x = rng.normal(1.0, 2.0, (n, 12)).astype(np.float32)
    t = (0.5 * x[:, 0] - 0.2 * x[:, 4] + 0.1 * x[:, 7] ** 2).astype(np.float32)
    return p, x, t


def test_mlp_forward_and_gradient_against_fp64_oracle(S):
    say("case: cost MLP forward / gradient / Adam vs FP64 oracle, n = 700 and 33")
    for n in (700, 33):
        p, x, t = _mlp_case(1, n)
        m = S.CostModel(p)
        norm = m.set_norm_from(x)
        assert np.allclose(norm, C.norm_of(x), rtol=1e-5)
        y = m.forward(x)
        yo, _ = C.forward(p, x, norm)
        assert np.max(np.abs(y - yo)) <= 1e-5 * max(1.0, np.max(np.abs(yo)))
        l, g = m.loss_grad(x, t)
        lo, go = C.loss_grad(p, x, t, norm)
        assert l == pytest.approx(lo, rel=1e-5)
        assert np.linalg.norm(g - go) <= 1e-3 * np.linalg.norm(go)
        assert np.max(np.abs(g - go)) <= 1e-3 * np.max(np.abs(go))
        # the FP64 gradient is itself pinned to central differences; spot-check here too
        for i in (0, 800, 4930, 5056):
            e = np.zeros(C.NP)
            e[i] = 1e-6
            fd = (C.loss(p + e, x, t, norm) - C.loss(p - e, x, t, norm)) / 2e-6
            assert abs(g[i] - fd) <= 1e-3 * max(abs(fd), 1e-3 * np.max(np.abs(go)))


def test_mlp_adam_and_training_against_fp64_oracle(S):
    say("case: cost MLP Adam step and 200 training steps vs FP64 oracle")
    p, x, t = _mlp_case(2)
    m = S.CostModel(p)
    norm = m.set_norm_from(x)
    _, g = m.loss_grad(x, t)
    # two steps: the second uses non-zero moments
    po, mo, vo = p.astype(np.float64), np.zeros(C.NP), np.zeros(C.NP)
    for k in (1, 2):
        m.adam_step(g, lr=1e-3)
        po, mo, vo = C.adam_step(po, mo, vo, g.astype(np.float64), k, lr=1e-3)
    got = m.get_params()
    assert np.max(np.abs(got - po)) <= 1e-6 * max(1.0, np.max(np.abs(po)))
    m2 = S.CostModel(p, norm)
    losses = m2.train(x, t, iters=200, lr=1e-3)
    _, lo = C.train(p, x, t, 200, lr=1e-3, norm=norm)
    assert np.allclose(losses, lo, rtol=2e-3, atol=1e-6)
    assert losses[-1] < 0.5 * losses[0]


def _work(steps, counts, batch):
    """Point-steps the batched kernels visit: every point of a batch, every step of the
    batch (the batch runs as long as its longest region)."""
    tot = 0
    for b in np.unique(batch[batch >= 0]):
        sel = batch == b
        tot += int(steps[sel].max()) * int(counts[sel].sum())
    return tot


def test_learned_packing_beats_point_count_heuristic(S):
    """Regions of random resolution: the point count says little about how many steps a
    region needs, the features do. Trained on one workload's logged steps, the model
    packs another workload with less wasted work than the point-count heuristic, and
    the results are identical under both packings."""
    say("case: learned packing, mixed workloads seeds 11 (train) and 12 (test), 160 regions")
    runs = {}
    for seed in (11, 12):
        n, ppx = I.mixed_regions(160, median=800, sigma=1.0, cap=20000, p_empty=0.1, seed=seed)
        parts, box = I.region_batch(n, seed=1000 * seed, pts_per_xi=ppx)
        rs = S.RegionSet.from_parts(parts, box, I.MATTER, device=True)
        runs[seed] = (rs, parts, box, S.region_features(rs))
    rs, parts, box, feat = runs[11]
    log = S.schedule_regions(rs, S.SCHED_BATCHED, use_graph=True, screen=S.SCREEN_F32,
                             out=None, events=False)
    live = rs.counts > 0
    target = np.log(np.maximum(log["region_steps"][live], 1)).astype(np.float32)
    p0 = np.random.default_rng(0).normal(0.0, 0.1, C.NP).astype(np.float32)
    model = S.CostModel(p0)
    model.set_norm_from(feat[live])
    losses = model.train(feat[live], target, iters=2000, lr=3e-3)
    say(f"  training loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.25 * losses[0]
    rs, parts, box, feat = runs[12]
    pred = np.exp(model.forward(feat)).astype(np.float32)
    budget = int(rs.counts.sum() // 6)
    out = {}
    for name, cost in (("heuristic", None), ("learned", pred)):
        out[name] = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=budget, cost=cost,
                                       use_graph=True, screen=S.SCREEN_F32)
    steps = out["heuristic"]["region_steps"]
    assert np.array_equal(steps, out["learned"]["region_steps"])
    live = rs.counts > 0
    corr = np.corrcoef(np.log(pred[live]), np.log(np.maximum(steps[live], 1)))[0, 1]
    corr_n = np.corrcoef(np.log(rs.counts[live]), np.log(np.maximum(steps[live], 1)))[0, 1]
    w = {k: _work(steps, rs.counts, v["region_batch"]) for k, v in out.items()}
    ms = {k: v["stats"]["makespan_ms"] for k, v in out.items()}
    say(f"  corr(pred, steps) {corr:.3f}  corr(log n, steps) {corr_n:.3f}  "
        f"visited point-steps {w}  makespan ms {ms}")
    assert corr > 0.9
    assert w["learned"] < 0.9 * w["heuristic"]
    # identical results under both packings
    for r in range(rs.n_regions):
        a = out["heuristic"]
        b = out["learned"]
        ra = a["out"][a["out_off"][4 * r]:a["out_off"][4 * r + 4]]
        rb = b["out"][b["out_off"][4 * r]:b["out_off"][4 * r + 4]]
        assert ra.tobytes() == rb.tobytes()
        ea = a["events"][a["events_off"][r]:a["events_off"][r + 1]]
        eb = b["events"][b["events_off"][r]:b["events_off"][r + 1]]
        assert ea.tobytes() == eb.tobytes()


def test_autotuner_choice_is_valid_cached_and_changes_no_result(S, tmp_path):
    """The autotuner's coordinate search returns one value of every tunable, reuses
    its cached choice for the same workload, and the schedule it picks gives exactly
    the records and events of the default launch shape."""
    from paper_1011_4046_amd import scheduler as SC
    say("case: autotune on sizes seed 200, max_steps 24, cache in tmp")
    parts, box = I.region_batch(SIZES, seed=200)
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    cost = rs.counts.astype(np.float32)
    cache = str(tmp_path / "tune.json")
    cfg = SC.autotune(rs, cost, screen=S.SCREEN_F32, cache=cache, max_steps=24)
    for k, vals in SC.TUNABLE.items():
        assert cfg[k] in vals, k
    assert cfg["ns_per_point_step"] > 0 and not cfg.get("cached")
    again = SC.autotune(rs, cost, screen=S.SCREEN_F32, cache=cache, max_steps=24)
    assert again["cached"] and all(again[k] == cfg[k] for k in SC.TUNABLE)
    kw = dict(use_graph=True, screen=S.SCREEN_F32)
    base = S.schedule_regions(rs, S.SCHED_BATCHED, cost=cost, **kw)
    tuned = S.schedule_regions(rs, S.SCHED_BATCHED, cost=cost,
                               batch_points=SC.batch_points_for(rs, cfg),
                               screen_split=cfg["screen_split"],
                               steps_per_sync=cfg["steps_per_sync"], lanes=cfg["lanes"],
                               pack=cfg["pack"], **kw)
    for r in range(rs.n_regions):
        a = base["out"][base["out_off"][4 * r]:base["out_off"][4 * r + 4]]
        b = tuned["out"][tuned["out_off"][4 * r]:tuned["out_off"][4 * r + 4]]
        assert a.tobytes() == b.tobytes()
        ea = base["events"][base["events_off"][r]:base["events_off"][r + 1]]
        eb = tuned["events"][tuned["events_off"][r]:tuned["events_off"][r + 1]]
        assert ea.tobytes() == eb.tobytes()


def test_learned_cost_fit_and_predict(S):
    """LearnedCost trains on logged step counts of non-empty regions (log steps) and
    predicts zero for empty regions; the learned schedule equals the plain batched one
    region by region."""
    from paper_1011_4046_amd import scheduler as SC
    say("case: LearnedCost on sizes seed 200")
    parts, box = I.region_batch(SIZES, seed=200)
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    log = S.schedule_regions(rs, S.SCHED_BATCHED, use_graph=True, screen=S.SCREEN_F32)
    feat = S.region_features(rs)
    cm = SC.LearnedCost(seed=0).fit(feat, log["region_steps"], iters=500, lr=3e-3)
    assert cm.losses[-1] < 0.1 * cm.losses[0]
    pred = cm.predict(feat)
    live = rs.counts > 0
    assert np.all(pred[~live] == 0) and np.all(pred[live] > 0)
    steps = log["region_steps"][live]
    assert np.allclose(np.log(pred[live]), np.log(steps), atol=0.35)
    res = SC.learned_schedule(rs, cm, use_graph=True, screen=S.SCREEN_F32, lanes=2,
                              batch_points=8000)
    assert np.array_equal(res["pred"], pred)
    for r in range(rs.n_regions):
        a = log["out"][log["out_off"][4 * r]:log["out_off"][4 * r + 4]]
        b = res["out"][res["out_off"][4 * r]:res["out_off"][4 * r + 4]]
        assert a.tobytes() == b.tobytes()


def _cross_linked(parts):
    """The same regions with surfaces that name points of other regions: every region's
    first dangling right end is joined (both ways) to the next region's first dangling
    left end. A region run alone never sees the other region's points, so these links
    dangle there."""
    parts = [(recs.copy(), geom) for recs, geom in parts]
    live = [r for r in range(len(parts)) if len(parts[r][0])]
    joined = 0
    for a, b in zip(live, live[1:] + live[:1]):
        ra, rb = parts[a][0], parts[b][0]
        ia = np.nonzero(ra["next_id"] < 0)[0]
        ib = np.nonzero(rb["prev_id"] < 0)[0]
        if len(ia) == 0 or len(ib) == 0 or a == b:
            continue
        ra["next_id"][ia[0]] = rb["id"][ib[0]]
        rb["prev_id"][ib[0]] = ra["id"][ia[0]]
        joined += 1
    return parts, joined


def test_links_between_regions_of_a_batch_are_cut(S):
    """Surfaces whose links name points of other regions: under every policy, and for
    the features, each region behaves as when run alone (links never leave a region)."""
    say("case: cross-region links, sizes[:8] seed 200, plain vs batched vs oracle")
    parts, box = I.region_batch(SIZES[:8], seed=200)
    orc = oracle_regions(parts, box, "sizes200")[:8]
    xparts, joined = _cross_linked(parts)
    assert joined >= 4
    rs = S.RegionSet.from_parts(xparts, box, I.MATTER)
    for policy in (S.SCHED_PLAIN, S.SCHED_BATCHED):
        res = S.schedule_regions(rs, policy, batch_points=0, use_graph=True,
                                 screen=S.SCREEN_F32)
        if policy == S.SCHED_BATCHED:
            assert res["stats"]["batches"] == 1
        # the oracle ran the surfaces without the extra links: every field must agree
        for r in range(len(parts)):
            mine = res["out"][res["out_off"][4 * r]:res["out_off"][4 * r + 4]]
            ev = res["events"][res["events_off"][r]:res["events_off"][r + 1]]
            if orc[r] is None:
                assert len(mine) == 0 and len(ev) == 0
                continue
            o, oe, _, _ = orc[r]
            a, b = mine[np.argsort(mine["id"])], o[np.argsort(o["id"])]
            assert a.tobytes() == b.tobytes(), (policy, r)
            assert ev.tobytes() == oe.tobytes(), (policy, r)
    for device in (False, True):
        f = S.region_features(S.RegionSet.from_parts(xparts, box, I.MATTER, device=device))
        for r, (recs, geom_r) in enumerate(parts):
            want = C.features(recs, geom_r, box)
            assert np.allclose(f[r], want, rtol=1e-5, atol=1e-6), (device, r, f[r], want)


def _twins(parts, shift=10 ** 9):
    """Each region followed by its twin: the same geometry and positions, ids shifted."""
    out = []
    for recs, geom in parts:
        twin = recs.copy()
        for f in ("id", "next_id", "prev_id"):
            twin[f] = np.where(recs[f] >= 0, recs[f] + shift, recs[f])
        out += [(recs, geom), (twin, geom)]
    return out


@pytest.mark.parametrize("case", ["coarse", "tiny-cells"])
def test_twin_regions_with_large_elements_do_not_meet_in_a_batch(S, case):
    """Regions of one batch never pair elements of two regions, also on the screen's
    path for elements larger than their cells (tested all against all). Each region is
    batched with a twin at the same place (same geometry and positions, other ids), so
    that every element of a region overlaps its twin's copy; each must end exactly as
    the oracle's run of it alone. coarse: strings of one point per correlation length in
    small regions, whose elements exceed a third of the local grid and are all large
    (12-17 points, 10-23 point-steps per region); tiny-cells: two regions of 1355 and
    774 points with 24 and 4 crossings, under a fixed cell edge of 1e-3, which makes
    every element large."""
    if case == "coarse":
        say("case: twin coarse regions (size 1, 1 point per correlation length), one batch")
        base, box = I.region_batch([300] * 4, size=1.0, seed=7, pts_per_xi=[1] * 4, slots=2)
        kw = {}
    else:
        say("case: twin regions (seed 33) with a fixed cell edge of 1e-3, one batch")
        base, box = I.region_batch([1500, 800], seed=33, slots=2)
        kw = dict(cell_size=1e-3)
    parts = _twins(base)
    assert sum(len(r) for r, _ in parts) >= 40
    orc = oracle_regions(parts, box, f"twins-{case}")
    if case == "tiny-cells":
        assert sum(len(o[1]) for o in orc) == 2 * (24 + 4)
    rs = S.RegionSet.from_parts(parts, box, I.MATTER)
    for policy in (S.SCHED_PLAIN, S.SCHED_BATCHED):
        for screen in (S.SCREEN_F32, S.SCREEN_F64):
            res = S.schedule_regions(rs, policy, batch_points=0, use_graph=True, screen=screen,
                                     **kw)
            if policy == S.SCHED_BATCHED:
                assert res["stats"]["batches"] == 1
            check_against_oracle(res, parts, orc)
            # a twin's events are its original's with the ids shifted
            for r in range(0, len(parts), 2):
                ea = res["events"][res["events_off"][r]:res["events_off"][r + 1]]
                eb = res["events"][res["events_off"][r + 1]:res["events_off"][r + 2]]
                assert len(ea) == len(eb)
                assert np.array_equal(ea["id_a"] + 10 ** 9, eb["id_a"])
                assert np.array_equal(ea["t_star"], eb["t_star"])
