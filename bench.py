#!/usr/bin/env python3
"""Benchmark: string point-steps/s on one MI355X, batched + learned scheduling against
the plain per-region path.

Default workload (--workload batched): 512 independent first-layer regions of an
8x8x8 tiling (region size 4, matter era), each an independent Vachaspati-Vilenkin-
style network at rest cut to the region's mid-time cross-section; point counts
lognormal (median 2e4, sigma 1.5, capped at 2e5) with 20% of the regions empty, 8
points per correlation length, about 1.6e7 points in about 410 non-empty regions.
Every region runs until all of its points have stopped (left the region).

One benchmark step = one whole schedule of all regions with inputs resident in HBM:
cost-model features (GPU) + cost-model inference (GPU) + schedule_regions(BATCHED)
ordered and packed by the predicted steps, FP32 screen with FP64 confirmation,
graph-captured step blocks, output surfaces written to HBM, event lists to the host.
The cost model is trained beforehand on the logged steps of a separate workload of
the same recipe (seed 1), by the library's own kernels.

Also reported: the point-count heuristic (same pipeline, no model), the plain
per-region path (one region at a time, FP64 screen, one host check per step, no
graphs, no batching), the roofline of the dominant kernel and the oracle on the host.

--workload tiling: a 32^3 matter-era VV network (seed 1, ~2.4e5 points, eta 8) in a
periodic spacetime tiling of 4M layers x 4M^3 regions (M = 4: 16 x 256 = 4096), run region by region in
dependency order with hand-off (schedule_handoff): every region builds the diamonds
whose earliest point it holds from what its predecessors and the initial surface built,
searches the crossings of its own elements (they pass through: intercommutation
probability 0, so that the run equals one whole-volume run), and starts its successors'
work. One step = the whole tiling, world sheet resident in HBM. Reported against the
plain per-region hand-off path (one region per launch sequence, FP64 screen, a host
check every step, no graphs) and the oracle's whole-volume run on the host.

--workload vv32: one whole-volume matter-era region (32^3 VV network, ~2.4e5 points,
eta 8 -> 16), as before.

Prints one JSON line. --gpus N > 1 is refused: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "string point-steps/s (evolve+intersect), batched+learned vs plain per-region"
HBM_PEAK_GBS = 8000.0


def evolve_bytes_per_point(screen_f32, bounded):
    """Compulsory HBM bytes of k_evolve per point-step: read X[n], X[n-1] (4 x FP64
    each) and next (int32); write X[n+1] (4 x FP64), the element box (8 x FP32 or
    8 x FP64), cell id and bucket slot (int32 each), one read-modify-write of a bucket
    counter (int32); bounded regions also read the stop step and sub-region (int32)."""
    box = 32 if screen_f32 else 64
    return 32 + 32 + 4 + 32 + box + 4 + 4 + 8 + (8 if bounded else 0)


def screen_bytes_per_element(screen_f32):
    """Compulsory HBM bytes of k_screen per element, its cell-sorted entry read once:
    FP32, the spatial box with the cell key and slot packed in (8 x 4 B); FP64, the
    (cell, slot) pair (2 x int32) and the box (8 x FP64)."""
    return 32 if screen_f32 else 8 + 64


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1011_4046_amd", "csrc", "semipar.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def counted_traffic(kernel, launch_config):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summaries
    (profiles/*.txt lines 'traffic-per-launch: ...'), when they were taken on the same
    kernel source and launch configuration; else None."""
    want = kernel_source_hash()
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".txt"):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                if not line.startswith("traffic-per-launch:"):
                    continue
                kv = dict(tok.split("=", 1) for tok in line.split()[1:])
                if (kv.get("kernel") == kernel and kv.get("source") == want
                        and kv.get("config") == launch_config):
                    return int(float(kv["fetch_bytes"]) + float(kv["write_bytes"]))
    return None


def table1(st):
    """The six metrics of the paper's comparison table (Section "Performance"), with lanes
    in the place of processors: total busy time of the lanes on batches ("CPU time"),
    makespan ("elapsed time"), the lanes' summed lifetimes ("total real time"), their
    time average ("average number of processors"), busy over held ("utilization") and
    busy over elapsed ("degree of parallelism")."""
    el = max(st["makespan_ms"], 1e-9)
    held = max(st["lane_held_ms"], 1e-9)
    return {"cpu_ms": round(st["lane_busy_ms"], 2), "elapsed_ms": round(st["makespan_ms"], 2),
            "real_ms": round(st["lane_held_ms"], 2), "avg_lanes": round(held / el, 3),
            "utilisation_pct": round(100.0 * st["lane_busy_ms"] / held, 2),
            "parallelism": round(st["lane_busy_ms"] / el, 3),
            "lanes_started": st["lanes_started"]}


def make_inputs(args):
    from paper_1011_4046_amd import inputs as I
    t = time.perf_counter()
    nt = I.lognormal_regions(args.regions, median=2e4, sigma=1.5, cap=2e5, p_empty=0.2, seed=0)
    prog = lambda i: (i % 64 == 63) and log(f"  generated {i + 1} regions")
    parts, box = I.region_batch(nt, size=4.0, seed=0, slots=8, workers=args.workers,
                                progress=prog)
    log(f"workload: {len(parts)} regions, {sum(len(p[0]) for p in parts)} points "
        f"({time.perf_counter() - t:.1f} s)")
    t = time.perf_counter()
    nt = I.lognormal_regions(args.train_regions, median=2e4, sigma=1.5, cap=2e5, p_empty=0.2,
                             seed=1)
    train, tbox = I.region_batch(nt, size=4.0, seed=100000, slots=8, workers=args.workers,
                                 progress=prog)
    log(f"training workload: {len(train)} regions, {sum(len(p[0]) for p in train)} points "
        f"({time.perf_counter() - t:.1f} s)")
    return parts, box, train, tbox


def handoff_inputs(args, seed=1):
    """Network, tiling geometry and dependency lists of the hand-off workload, and the
    number of world-sheet slices its last layer needs."""
    import numpy as np
    from paper_1011_4046_amd import inputs as I
    t = time.perf_counter()
    net = I.vv_network(m=args.m, seed=seed)
    layers = args.layers or 4 * args.split_m
    parts, box, n_pred, succ, _ = I.tiling_regions(net, M=args.split_m, layers=layers)
    geoms = [g for _, g in parts]
    V, inv2g = geoms[0][:4], geoms[0][4]
    g = 0.5 / inv2g
    t_last = (V[3] + 0.5 * g * (layers - 1) + 2 * g) / np.sqrt(3.0)
    # the initial slices are dt apart in t; in an expanding universe later slices of a
    # moving string advance t by less, so twice that many slices, grown on overflow
    rec = net["recs"][0]
    dt = float(rec["x"][3] - rec["x_prev"][3])
    slices = 2 * int(np.ceil((t_last - float(rec["x_prev"][3])) / dt)) + 8
    log(f"hand-off tiling (seed {seed}): {len(net['recs'])} points, {len(geoms)} regions in "
        f"{layers} layers, {slices} slices ({time.perf_counter() - t:.1f} s)")
    return net, box, geoms, n_pred, succ, slices, layers


def bench_handoff(args):
    import numpy as np
    import torch
    from paper_1011_4046_amd import semipar as S
    net, box, geoms, n_pred, succ, slices, layers = handoff_inputs(args)
    n = len(net["recs"])
    torch.cuda.set_device(0)
    screen = S.SCREEN_F32 if args.screen == "f32" else S.SCREEN_F64
    kw = dict(use_graph=True, screen=screen, steps_per_sync=args.sync_steps,
              batch_points=0, cell_factor=args.cell_factor, screen_split=args.split)
    hist = None
    run = lambda **k: S.schedule_handoff(net["recs"], box, net["cosmology"], geoms, n_pred, succ,
                                         hist, **k)
    for _ in range(4):
        hist = torch.empty((slices, n, 4), dtype=torch.float64, device="cuda")
        try:
            r = run(**kw)
            break
        except S.SemiparError as e:
            if e.code != -5:
                raise
            log(f"world sheet of {slices} slices too short: doubled")
            del hist
            slices *= 2
    log(f"first run: {r['stats']['batches']} batches, {r['stats']['makespan_ms']:.0f} ms")
    for w in range(args.warmup):
        r = run(**kw)
        log(f"warmup {w}: {r['stats']['batches']} batches, {r['stats']['makespan_ms']:.0f} ms")
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runs.append(run(**kw))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    point_steps = sum(r["stats"]["point_steps"] for r in runs)
    value = point_steps / elapsed
    st = runs[0]["stats"]
    log(f"timed {args.steps} tilings: {elapsed * 1e3:.0f} ms, {point_steps} point-steps, "
        f"{st['batches']} batches, {st['events']} crossings per tiling")
    extra = {"handoff": {"batches": st["batches"], "empty_regions": st["empty_regions"],
                         "makespan_ms": st["makespan_ms"], "evolve_ms": st["evolve_ms"],
                         "crossings": st["events"]}}
    if args.plain:
        t = time.perf_counter()
        rp = run(use_graph=False, screen=S.SCREEN_F64, steps_per_sync=1, batch_points=1)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        pv = rp["stats"]["point_steps"] / tp
        assert rp["stats"]["point_steps"] == st["point_steps"]
        extra["plain_per_region"] = {"point_steps_per_s": pv, "ms": tp * 1e3,
                                     "batches": rp["stats"]["batches"],
                                     "speedup_batched": value / pv, "steps_per_sync": 1}
        log(f"plain per-region hand-off: {tp * 1e3:.0f} ms, speed-up {value / pv:.2f}x")
    del hist
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_whole_volume(net)
    return {
        "value": value, "ms_per_step": elapsed * 1e3 / args.steps,
        "config": {"workload": f"hand-off tiling: {args.m}^3 matter-era VV network (seed 1) in "
                               f"a periodic spacetime tiling of {layers} layers x "
                               f"{4 * args.split_m ** 3} regions, run in dependency order, "
                               f"crossings of each region's elements searched (pass through)",
                   "regions": len(geoms), "points": n, "slices": slices,
                   "point_steps_per_tiling": st["point_steps"], "screen": args.screen,
                   "graph": True, "steps_per_sync": args.sync_steps, "lanes": 1,
                   "screen_split": args.split,
                   "path": "schedule_handoff: each layer's regions in one batch, layer after "
                           "layer, world sheet in HBM"},
        "roofline": None, "cpu_baseline": cpu, **extra,
    }


def cpu_baseline_whole_volume(net, budget_s=20.0):
    """The oracle's whole-volume run of the same network (crossing search on, every
    crossing passing through), stepped for about budget_s seconds."""
    import oracle as O
    hc = {0: 0.0, 1: 2.0, 2: 1.0}[net["cosmology"]]
    ro = O.OracleRegion(net["recs"], net["box"], net["cosmology"], hc)
    t = time.perf_counter()
    while time.perf_counter() - t < budget_s:
        ro.evolve(1, p=0.0)
    tc = time.perf_counter() - t
    st = ro.stats()
    ro.close()
    log(f"cpu baseline: whole volume, {st['steps']} steps in {tc:.1f} s")
    return {"value": st["point_steps"] / tc, "unit": "point-steps/s", "cores": O.threads(),
            "kind": "oracle",
            "sample": f"the whole-volume run of the same network ({len(net['recs'])} points), "
                      f"first {st['steps']} lattice steps ({st['point_steps']} point-steps in "
                      f"{tc:.1f} s)"}


def bench_batched(args):
    parts, box, train, tbox = make_inputs(args)   # before any GPU use (process pool)
    dag, dag_tr = {}, {}
    desc = ("512 independent matter-era regions (8x8x8 first layer, size 4), "
            "lognormal points median 2e4 sigma 1.5 cap 2e5, 20% empty, "
            "each run until all its points stop")
    import numpy as np
    import torch
    from paper_1011_4046_amd import inputs as I
    from paper_1011_4046_amd import scheduler as SC
    from paper_1011_4046_amd import semipar as S
    torch.cuda.set_device(0)
    rs = S.RegionSet.from_parts(parts, box, I.MATTER, device=True, **dag)
    rs_tr = S.RegionSet.from_parts(train, tbox, I.MATTER, device=True, **dag_tr)
    torch.cuda.synchronize()
    screen = S.SCREEN_F32 if args.screen == "f32" else S.SCREEN_F64
    coin = dict(p=args.p, seed=args.seed)
    fast = dict(use_graph=True, screen=screen, out="device", events=True, **coin)

    # cost model: trained on the logged steps of the training workload
    t = time.perf_counter()
    logrun = S.schedule_regions(rs_tr, S.SCHED_BATCHED, use_graph=True, screen=screen,
                                out=None, events=False, **coin)
    cm = SC.LearnedCost(seed=0).fit(S.region_features(rs_tr), logrun["region_steps"],
                                    iters=2000, lr=3e-3)
    log(f"cost model: trained on {int((rs_tr.counts > 0).sum())} logged regions, loss "
        f"{cm.losses[0]:.3f} -> {cm.losses[-1]:.4f} ({time.perf_counter() - t:.1f} s)")
    del rs_tr

    feat = S.region_features(rs)
    pred = cm.predict(feat)
    cfg = {"batch_frac": args.batch_frac, "screen_split": args.split,
           "steps_per_sync": args.sync_steps, "lanes": args.lanes, "pack": args.pack,
           "cell_factor": args.cell_factor}
    if args.tune:
        cfg = SC.autotune(rs, pred, screen=screen, cache=args.tune_cache or None, log=log)
        log(f"autotune: {cfg}")
    bp = SC.batch_points_for(rs, cfg)
    kw = dict(fast, batch_points=bp, screen_split=cfg["screen_split"],
              steps_per_sync=cfg["steps_per_sync"], lanes=cfg["lanes"],
              cell_factor=cfg.get("cell_factor", 0.0))
    kw_learned = dict(kw, pack=cfg.get("pack", S.PACK_POINTS))

    for w in range(args.warmup):
        r = SC.learned_schedule(rs, cm, **kw_learned)
        log(f"warmup {w}: {r['stats']['batches']} batches, {r['stats']['makespan_ms']:.0f} ms")
        del r
    torch.cuda.synchronize()
    runs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        runs.append(SC.learned_schedule(rs, cm, **kw_learned))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    point_steps = sum(r["stats"]["point_steps"] for r in runs)
    value = point_steps / elapsed
    st = runs[0]["stats"]
    steps = runs[0]["region_steps"]
    live = rs.counts > 0
    corr = float(np.corrcoef(np.log(pred[live]), np.log(np.maximum(steps[live], 1)))[0, 1])
    log(f"timed {args.steps} schedules: {elapsed * 1e3:.0f} ms, {point_steps} point-steps, "
        f"{st['batches']} batches, {st['events']} events per schedule")
    # the paper's split-factor metrics, with lanes in the place of processors: busy
    # device time of the evolve calls ("CPU time"), makespan ("elapsed"), their ratio
    # (degree of parallelism) and its share of the lanes (utilisation)
    busy = st["evolve_ms"]
    extra = {"learned": {"batches": st["batches"], "makespan_ms": st["makespan_ms"],
                         "evolve_busy_ms": busy,
                         "parallelism": busy / max(st["makespan_ms"], 1e-9),
                         "lane_utilisation": busy / max(cfg["lanes"] * st["makespan_ms"], 1e-9),
                         "predict_ms": runs[0]["predict_ms"],
                         "corr_log_pred_log_steps": round(corr, 4),
                         "table1_held_pool": table1(st)}}
    del runs
    # the same schedule under the paper's variable-size worker pool (lanes sleep, exit
    # when nothing comes for lane_sleep_ms, are started again when batches wait
    # lane_submit_ms): Table 1's six metrics, not part of the timed value
    re_ = SC.learned_schedule(rs, cm, lane_sleep_ms=args.lane_sleep_ms,
                              lane_submit_ms=args.lane_submit_ms, **kw_learned)
    torch.cuda.synchronize()
    extra["learned"]["table1_elastic_pool"] = dict(
        table1(re_["stats"]), lane_sleep_ms=args.lane_sleep_ms,
        lane_submit_ms=args.lane_submit_ms)
    del re_

    # point-count heuristic, same batch size
    t = time.perf_counter()
    rh = S.schedule_regions(rs, S.SCHED_BATCHED, **kw)
    torch.cuda.synchronize()
    th = time.perf_counter() - t
    extra["heuristic"] = {"point_steps_per_s": rh["stats"]["point_steps"] / th,
                          "batches": rh["stats"]["batches"], "ms": th * 1e3}
    log(f"heuristic: {th * 1e3:.0f} ms")
    del rh

    # plain per-region path
    if args.plain:
        t = time.perf_counter()
        rp = S.schedule_regions(rs, S.SCHED_PLAIN, screen=S.SCREEN_F64, use_graph=False,
                                steps_per_sync=1, out="device", events=True, **coin)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        pv = rp["stats"]["point_steps"] / tp
        assert rp["stats"]["point_steps"] == st["point_steps"]
        extra["plain_per_region"] = {"point_steps_per_s": pv, "ms": tp * 1e3,
                                     "speedup_batched_learned": value / pv,
                                     "steps_per_sync": 1}
        log(f"plain per-region: {tp * 1e3:.0f} ms, speed-up {value / pv:.2f}x")
        del rp
        # the same plain path with a host check every 32 steps (still no graphs, FP64
        # screen, one region at a time): what batching alone gains
        t = time.perf_counter()
        rp = S.schedule_regions(rs, S.SCHED_PLAIN, screen=S.SCREEN_F64, use_graph=False,
                                steps_per_sync=32, out="device", events=True, **coin)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t
        pv = rp["stats"]["point_steps"] / tp
        extra["plain_per_region_sync32"] = {"point_steps_per_s": pv, "ms": tp * 1e3,
                                            "speedup_batched_learned": value / pv,
                                            "steps_per_sync": 32}
        log(f"plain per-region, 32 steps per host check: {tp * 1e3:.0f} ms, "
            f"speed-up {value / pv:.2f}x")
        del rp

    roof, other = roofline_runs(S, rs, bp, cfg, screen, coin, args.screen)

    if args.workload == "batched" and args.mixed:
        extra["mixed_resolution"] = mixed_leg(S, SC, I, screen, coin, args)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on a sample of the regions")
        cpu = cpu_baseline_regions(parts, box, coin=coin)
    return {
        "value": value, "ms_per_step": elapsed * 1e3 / args.steps,
        "config": {"workload": desc,
                   "regions": rs.n_regions, "points": int(rs.counts.sum()),
                   "point_steps_per_schedule": st["point_steps"],
                   "screen": args.screen, "graph": True, "batch_points": bp,
                   "screen_split": cfg["screen_split"], "steps_per_sync": cfg["steps_per_sync"],
                   "lanes": cfg["lanes"], "pack": cfg.get("pack", 0),
                   "cell_factor": cfg.get("cell_factor", 0.0) or 1.15,
                   "p_intercommute": args.p,
                   "path": "batched + learned cost model (features, inference and schedule "
                           "inside the timed region)"},
        "roofline": roof, "roofline_other": other, "cpu_baseline": cpu, **extra,
    }


def roofline_runs(S, rs, bp, cfg, screen, coin, screen_name):
    """Roofline of the evolve and screen kernels: one eager schedule per timed kernel
    (HIP events around every launch of it, on the batch's stream; events cannot be
    recorded inside graphs), one lane so that no other batch's kernels run beside the
    timed ones, batches of the timed configuration's size in point-count order.
    `bench.py --roofline-only` runs exactly these schedules, for the profiler."""
    roofs = {}
    launch_config = (f"eager-1lane-bp{bp}-split{cfg['screen_split']}-sync{cfg['steps_per_sync']}"
                     f"-{screen_name}")
    if cfg.get("cell_factor", 0.0):
        launch_config += f"-cf{cfg['cell_factor']:g}"  # the default 1.15 goes unnamed
    for kname, kid in (("k_evolve", S.K_EVOLVE), ("k_screen", S.K_SCREEN)):
        rr = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=bp, cost=None, out=None,
                                events=False, use_graph=False, screen=screen,
                                screen_split=cfg["screen_split"],
                                steps_per_sync=cfg["steps_per_sync"], timed_kernel=kid, lanes=1,
                                cell_factor=cfg.get("cell_factor", 0.0), **coin)
        s2 = rr["stats"]
        ms, nl = s2["timed_kernel_ms"], max(s2["timed_kernel_launches"], 1)
        if kname == "k_evolve":
            unit = evolve_bytes_per_point(screen == S.SCREEN_F32, True)
        else:
            unit = screen_bytes_per_element(screen == S.SCREEN_F32)
        # one element per point-step (the band piece to the right neighbour)
        alg = unit * s2["point_steps"]
        ach = alg / (ms / 1e3) / 1e9 if ms > 0 else 0.0
        roofs[kname] = {"bound": "hbm", "kernel": kname, "achieved": round(ach, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "traffic": counted_traffic(kname, launch_config),
                        "bytes_per_point_step": unit,
                        "avg_launch_us": round(ms / nl * 1e3, 3), "launches": nl,
                        "total_ms": round(ms, 2),
                        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, "
                                        "copy-calibrated)",
                        "launch_config": launch_config,
                        "timing": "HIP events around every launch of this kernel in eager "
                                  "one-lane schedules"}
        log(f"{kname}: {nl} launches, {ms:.1f} ms, {ach:.0f} GB/s algorithmic")
    dom = max(roofs, key=lambda k: roofs[k]["total_ms"])
    return roofs[dom], {k: v for k, v in roofs.items() if k != dom}


def mixed_leg(S, SC, I, screen, coin, args):
    """Learned packing where it should pay: regions of random resolution (points per
    correlation length from {4, 6, 8, 12, 16}), so that the point count says little about
    the steps a region needs. The model trains on one such workload's logged steps
    (seed 11) and packs another (seed 12) into batches of a sixth of the points, one
    lane; makespans are the best of three runs of each order."""
    import numpy as np
    out = {}
    work = {}
    for seed in (11, 12):
        n, ppx = I.mixed_regions(args.mixed_regions, median=args.mixed_median, sigma=1.0,
                                 cap=50000, p_empty=0.1, seed=seed)
        parts, box = I.region_batch(n, seed=1000 * seed, pts_per_xi=ppx, workers=args.workers)
        work[seed] = S.RegionSet.from_parts(parts, box, I.MATTER, device=True)
    rs_tr, rs = work[11], work[12]
    logrun = S.schedule_regions(rs_tr, S.SCHED_BATCHED, use_graph=True, screen=screen, out=None,
                                events=False, **coin)
    cm = SC.LearnedCost(seed=0).fit(S.region_features(rs_tr), logrun["region_steps"], iters=2000,
                                    lr=3e-3)
    pred = cm.predict(S.region_features(rs))
    bp = int(rs.counts.sum() // 6)
    kw = dict(batch_points=bp, use_graph=True, screen=screen, out="device", events=True,
              lanes=1, **coin)
    for name, cost in (("heuristic", None), ("learned", pred)):
        best = None
        for _ in range(3):
            r = S.schedule_regions(rs, S.SCHED_BATCHED, cost=cost, **kw)
            if best is None or r["stats"]["makespan_ms"] < best["stats"]["makespan_ms"]:
                best = r
        st = best["stats"]
        steps = best["region_steps"]
        visited = 0
        for b in np.unique(best["region_batch"][best["region_batch"] >= 0]):
            sel = best["region_batch"] == b
            visited += int(steps[sel].max()) * int(rs.counts[sel].sum())
        out[name] = {"makespan_ms": round(st["makespan_ms"], 2),
                     "point_steps_per_s": st["point_steps"] / (st["makespan_ms"] / 1e3),
                     "batches": st["batches"], "visited_point_steps": visited}
        log(f"mixed workload, {name}: {st['makespan_ms']:.1f} ms, {st['batches']} batches, "
            f"visited point-steps {visited}")
    live = rs.counts > 0
    out["regions"] = rs.n_regions
    out["points"] = int(rs.counts.sum())
    out["point_steps"] = int(st["point_steps"])
    out["corr_log_pred_log_steps"] = round(float(np.corrcoef(
        np.log(pred[live]), np.log(np.maximum(steps[live], 1)))[0, 1]), 4)
    out["learned_gain"] = round(out["heuristic"]["makespan_ms"] / out["learned"]["makespan_ms"], 4)
    return out


def cpu_baseline_regions(parts, box, every=50, budget_s=20.0, coin=None):
    """The oracle on a bounded sample of the same regions: every `every`-th non-empty
    region, each stepped one lattice step at a time for an equal share of `budget_s`
    seconds (or until it has stopped)."""
    import numpy as np
    import oracle as O
    from paper_1011_4046_amd import inputs as I
    live = [i for i, p in enumerate(parts) if len(p[0])]
    sample = live[::every]
    share = budget_s / max(len(sample), 1)
    t = time.perf_counter()
    ps, steps, npts = 0, 0, 0
    for i in sample:
        recs, geom = parts[i]
        ro = O.OracleRegion(recs, box, I.MATTER, I.HCOEF[I.MATTER], geom)
        t1 = time.perf_counter()
        while time.perf_counter() - t1 < share and ro.active > 0:
            ro.evolve(1, **(coin or {}))
        st = ro.stats()
        ps += st["point_steps"]
        steps += st["steps"]
        npts += len(recs)
        ro.close()
        log(f"cpu baseline: region {i} ({len(recs)} points), {st['steps']} steps, "
            f"{time.perf_counter() - t:.1f} s")
    tc = time.perf_counter() - t
    return {"value": ps / tc, "unit": "point-steps/s", "cores": O.threads(), "kind": "oracle",
            "sample": f"{len(sample)} of the {len(live)} non-empty regions (every {every}th, "
                      f"{npts} points), each stepped for {share:.1f} s: {steps} lattice steps, "
                      f"{ps} point-steps in {tc:.1f} s"}


def cached_region_batch(path, nt, workers):
    """The batched workload's regions (seed 0), read from `path` when it holds them, else
    generated and, when `path` is set, saved there (so that profiler passes over the same
    workload generate it once, outside the profiler)."""
    import numpy as np
    from paper_1011_4046_amd import inputs as I
    if path and os.path.exists(path):
        with np.load(path) as z:
            assert np.array_equal(z["nt"], np.asarray(nt)), "cached workload differs"
            recs, cnt = z["recs"], z["counts"]
            off = np.concatenate([[0], np.cumsum(cnt)])
            parts = [(recs[off[r]:off[r + 1]].copy(), z["geoms"][r].copy())
                     for r in range(len(cnt))]
            return parts, float(z["box"])
    parts, box = I.region_batch(nt, size=4.0, seed=0, slots=8, workers=workers)
    if path:
        np.savez(path, nt=np.asarray(nt), recs=np.concatenate([p[0] for p in parts]),
                 counts=np.array([len(p[0]) for p in parts], np.int64),
                 geoms=np.array([p[1] for p in parts], np.float64), box=box)
    return parts, box


def roofline_only(args):
    """The roofline schedules of the batched workload alone (no training, no timed
    schedules): what a profiler run of the kernels the roofline describes should see."""
    from paper_1011_4046_amd import inputs as I
    nt = I.lognormal_regions(args.regions, median=2e4, sigma=1.5, cap=2e5, p_empty=0.2, seed=0)
    parts, box = cached_region_batch(args.inputs_cache, nt, args.workers)
    if args.inputs_only:
        return {"mode": "inputs-only", "regions": len(parts)}
    import torch
    from paper_1011_4046_amd import semipar as S
    torch.cuda.set_device(0)
    rs = S.RegionSet.from_parts(parts, box, I.MATTER, device=True)
    screen = S.SCREEN_F32 if args.screen == "f32" else S.SCREEN_F64
    cfg = {"batch_frac": args.batch_frac, "screen_split": args.split,
           "steps_per_sync": args.sync_steps, "cell_factor": args.cell_factor}
    from paper_1011_4046_amd import scheduler as SC
    bp = SC.batch_points_for(rs, cfg)
    roof, other = roofline_runs(S, rs, bp, cfg, screen, dict(p=args.p, seed=args.seed),
                                args.screen)
    return {"mode": "roofline-only", "roofline": roof, "roofline_other": other}


def bench_vv32(args):
    import numpy as np
    import torch
    from paper_1011_4046_amd import inputs as I
    from paper_1011_4046_amd import semipar as S
    torch.cuda.set_device(0)
    net = I.vv_network(m=args.m, seed=0)
    n = len(net["recs"])
    t0, t_end = net["t0"], 2.0 * net["t0"]
    raw = torch.from_numpy(net["recs"].view(np.uint8).copy()).cuda()
    screen = S.SCREEN_F32 if args.screen == "f32" else S.SCREEN_F64
    coin = dict(p=args.p, seed=args.seed)
    kw = dict(screen=screen, use_graph=True, steps_per_sync=64, **coin)
    log(f"VV {args.m}^3 matter era, {n} points, eta {t0} -> {t_end}")

    def fresh():
        return S.Region(raw, net["box"], net["cosmology"])

    for _ in range(args.warmup):
        r = fresh()
        r.evolve(args.max_steps, t_end, **kw)
        r.close()
    regions = [fresh() for _ in range(args.steps)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    stats = [r.evolve(args.max_steps, t_end, **kw) for r in regions]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t
    for r in regions:
        r.close()
    ps = sum(s["point_steps"] for s in stats)
    r = fresh()
    tst = r.evolve(args.max_steps, t_end, screen=screen, use_graph=False, steps_per_sync=64,
                   timed_kernel=S.K_EVOLVE, **coin)
    r.close()
    unit = evolve_bytes_per_point(screen == S.SCREEN_F32, False)
    ms, nl = tst["timed_kernel_ms"], max(tst["timed_kernel_launches"], 1)
    ach = unit * tst["point_steps"] / (ms / 1e3) / 1e9 if ms > 0 else 0.0
    roof = {"bound": "hbm", "kernel": "k_evolve", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_point_step": unit, "avg_launch_us": round(ms / nl * 1e3, 3)}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        ro = O.OracleRegion(net["recs"], net["box"], net["cosmology"], I.HCOEF[net["cosmology"]])
        tc = time.perf_counter()
        ro.evolve(30, **coin)
        tcpu = time.perf_counter() - tc
        cst = ro.stats()
        ro.close()
        cpu = {"value": cst["point_steps"] / tcpu, "unit": "point-steps/s", "cores": O.threads(),
               "kind": "oracle", "sample": f"first 30 lattice steps ({cst['point_steps']} "
                                           f"point-steps, {tcpu:.1f} s)"}
    return {"value": ps / elapsed, "ms_per_step": elapsed * 1e3 / args.steps,
            "config": {"workload": f"matter-era VV network {args.m}^3, one whole-volume region, "
                                   f"eta 8 -> 16", "points": n,
                       "lattice_steps_per_run": stats[0]["steps"], "screen": args.screen,
                       "p_intercommute": args.p},
            "roofline": roof, "cpu_baseline": cpu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["batched", "tiling", "vv32"], default="batched")
    ap.add_argument("--screen", choices=["f32", "f64"], default="f32")
    ap.add_argument("--regions", type=int, default=512)
    ap.add_argument("--train-regions", type=int, default=128)
    ap.add_argument("--workers", type=int, default=8,
                    help="forked processes generating the inputs (0 under a profiler, which "
                         "loads the GPU runtime before the program starts)")
    ap.add_argument("--batch-frac", type=float, default=0.34,
                    help="batch size as a fraction of all points (1 = one batch)")
    ap.add_argument("--split", type=int, default=1, help="screen threads per element (1 or 5)")
    ap.add_argument("--lanes", type=int, default=3, help="batches evolved concurrently")
    ap.add_argument("--sync-steps", type=int, default=32, help="lattice steps per host check")
    ap.add_argument("--lane-sleep-ms", type=float, default=2.0,
                    help="elastic worker pool leg: a lane exits after sleeping this long")
    ap.add_argument("--lane-submit-ms", type=float, default=1.0,
                    help="elastic worker pool leg: lanes are started again once batches have "
                         "waited this long")
    ap.add_argument("--cell-factor", type=float, default=0.0,
                    help="cell edge over the largest element extent (0: the library's 1.15)")
    ap.add_argument("--pack", type=int, default=0,
                    help="learned schedule: 0 = batches of equal points, 1 = of equal "
                         "predicted point-steps")
    ap.add_argument("--tune", type=int, default=0,
                    help="run the autotuner first (the defaults are its choice for this "
                         "workload)")
    ap.add_argument("--tune-cache", default="")
    ap.add_argument("--plain", type=int, default=1, help="also time the plain per-region path")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--split-m", type=int, default=4,
                    help="tiling workload: regions per layer 4 M^3 (the split factor)")
    ap.add_argument("--layers", type=int, default=0,
                    help="tiling workload: layers (0: 4 M, the same spacetime volume for every "
                         "split factor)")
    ap.add_argument("--max-steps", type=int, default=10 ** 7)
    ap.add_argument("--p", type=float, default=1.0,
                    help="intercommutation probability in (0, 1] (1: every crossing exchanges)")
    ap.add_argument("--seed", type=int, default=0, help="key of the crossings' draws (p < 1)")
    ap.add_argument("--mixed", type=int, default=1,
                    help="also time learned against point-count packing on a workload of "
                         "random resolution")
    ap.add_argument("--mixed-regions", type=int, default=160)
    ap.add_argument("--mixed-median", type=float, default=4000.0)
    ap.add_argument("--inputs-cache", default="",
                    help="file holding the batched workload (--roofline-only): read when "
                         "present, written after generating it otherwise")
    ap.add_argument("--inputs-only", action="store_true",
                    help="with --roofline-only: generate (and cache) the workload, run nothing")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the eager one-lane roofline schedules of the batched workload "
                         "(for a profiler); prints their roofline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)
    if not 0.0 < args.p <= 1.0:
        print(f"bench.py: --p {args.p} is outside (0, 1]", file=sys.stderr)
        sys.exit(2)
    if args.roofline_only:
        print(json.dumps(roofline_only(args)), flush=True)
        return
    if args.workload == "vv32":
        res = bench_vv32(args)
    elif args.workload == "tiling":
        res = bench_handoff(args)
    else:
        res = bench_batched(args)
    out = {"metric": METRIC, "value": res.pop("value"), "unit": "point-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res.pop("ms_per_step"),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", **res}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
