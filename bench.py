#!/usr/bin/env python3
"""Benchmark: string point-steps/s of one whole-volume matter-era region on one MI355X.

Workload: a Vachaspati-Vilenkin-style network from Z3 phases on a periodic 32^3
lattice (box L = 32 correlation lengths, 8 points per correlation length,
~2.4e5 points, at rest), evolved in the matter era from conformal time 8 until the
smallest time on the current slice reaches 16. One benchmark step = one such run
(diamond tops, element boxes, spatial hash, screen, FP64 confirmation, resolution,
partner exchange) from the initial surface already resident in HBM.

Prints one JSON line. --gpus N > 1 is refused: this build runs on one GPU.
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


def evolve_bytes_per_point(screen_f32):
    """Compulsory HBM bytes of one k_evolve launch per point: read X[n], X[n-1]
    (4 x FP64 each) and next (int32); write X[n+1] (4 x FP64), the element box
    (8 x FP32 or 8 x FP64), cell id and bucket slot (int32 each), and one
    read-modify-write of a bucket counter (int32)."""
    box = 32 if screen_f32 else 64
    return 32 + 32 + 4 + 32 + box + 4 + 4 + 8


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--screen", choices=["f32", "f64"], default="f32")
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--sync-steps", type=int, default=64)
    ap.add_argument("--m", type=int, default=32, help="lattice size of the VV network")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain", type=int, default=1, help="also time the plain per-step path")
    ap.add_argument("--max-steps", type=int, default=10 ** 7,
                    help="cap on lattice steps per run (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1011_4046_amd import inputs as I
    from paper_1011_4046_amd import semipar as S

    torch.cuda.set_device(0)
    net = I.vv_network(m=args.m, seed=0)
    n = len(net["recs"])
    t0, t_end = net["t0"], 2.0 * net["t0"]
    raw = torch.from_numpy(net["recs"].view(np.uint8).copy()).cuda()
    stream = torch.cuda.current_stream()
    screen = S.SCREEN_F32 if args.screen == "f32" else S.SCREEN_F64
    kw = dict(screen=screen, use_graph=bool(args.graph), steps_per_sync=args.sync_steps)
    print(f"bench: VV {args.m}^3 matter era, {n} points, eta {t0} -> {t_end}, "
          f"screen {args.screen}, graph {args.graph}", file=sys.stderr, flush=True)

    def fresh():
        return S.Region(raw, net["box"], net["cosmology"])

    for w in range(args.warmup):
        r = fresh()
        st = r.evolve(args.max_steps, t_end, **kw)
        r.close()
        print(f"bench: warmup {w}: {st['steps']} steps, {st['elapsed_ms']:.1f} ms",
              file=sys.stderr, flush=True)

    regions = [fresh() for _ in range(args.steps)]
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for r in regions:
        stats.append(r.evolve(args.max_steps, t_end, **kw))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    for r in regions:
        r.close()
    point_steps = sum(s["point_steps"] for s in stats)
    value = point_steps / elapsed
    lattice_steps = stats[0]["steps"]
    print(f"bench: timed {args.steps} runs: {elapsed * 1e3:.1f} ms, {point_steps} point-steps, "
          f"{lattice_steps} lattice steps per run", file=sys.stderr, flush=True)

    # roofline of the dominant kernel (k_evolve): HIP events around each of its launches,
    # recorded on the region's stream during one more full run (events cannot be timed
    # inside a captured graph, so this run issues its steps eagerly)
    r = fresh()
    tst = r.evolve(args.max_steps, t_end, screen=screen, use_graph=False,
                   steps_per_sync=args.sync_steps, timed_kernel=S.K_EVOLVE)
    r.close()
    ev_ms = tst["timed_kernel_ms"]
    ev_n = tst["timed_kernel_launches"]
    bpp = evolve_bytes_per_point(args.screen == "f32")
    avg_s = ev_ms / max(ev_n, 1) / 1e3
    achieved = bpp * n / avg_s / 1e9 if avg_s > 0 else 0.0
    roof = {"bound": "hbm", "kernel": "k_evolve", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None, "bytes_per_point": bpp, "avg_launch_us": round(avg_s * 1e6, 3)}

    extra = {}
    if args.plain:
        r = fresh()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        sp = r.evolve(args.max_steps, t_end, screen=S.SCREEN_F64, use_graph=False, steps_per_sync=1)
        torch.cuda.synchronize()
        te = time.perf_counter() - ts
        r.close()
        extra["plain_per_region_point_steps_per_s"] = sp["point_steps"] / te
        extra["plain_ms"] = te * 1e3

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        sample_steps = 30
        ro = O.OracleRegion(net["recs"], net["box"], net["cosmology"], I.HCOEF[net["cosmology"]])
        tc = time.perf_counter()
        ro.evolve(sample_steps)
        tcpu = time.perf_counter() - tc
        cst = ro.stats()
        ro.close()
        cpu = {"value": cst["point_steps"] / tcpu, "unit": "point-steps/s", "cores": O.threads(),
               "kind": "oracle",
               "sample": f"first {sample_steps} lattice steps of the same network "
                         f"({cst['point_steps']} point-steps, {tcpu:.1f} s)"}

    out = {
        "metric": METRIC, "value": value, "unit": "point-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"matter-era VV network {args.m}^3 (L={args.m}, 8 points per "
                               f"correlation length), one whole-volume region, eta 8 -> 16",
                   "points": n, "lattice_steps_per_run": lattice_steps,
                   "screen": args.screen, "graph": bool(args.graph),
                   "path": "plain per-region (single region, graph-captured step blocks)"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "events_per_run": stats[0]["accepted"],
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
