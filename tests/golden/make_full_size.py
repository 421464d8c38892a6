"""Write full_size.json: digests of the oracle's results on the full-size workloads.

Calls only the oracle and the seeded input generators (no GPU code). The GPU parity
tests in tests/test_gpu_full_size.py compare the HIP path's results with these
digests; the per-step event counts show the first step at which two runs differ.

Workloads (the survey's configurations at their real sizes):
  * matter32: the 32^3 matter-era VV network (seed 0, L = 32 correlation lengths,
    8 points per correlation length, at rest at eta = 8), run until the smallest t of
    the slice reaches 16 (conformal time doubles);
  * matter64_20: the dense 64^3 network (seed 0, L = 64), its first 20 steps;
  * batched512: sixteen regions of the 512-region batched workload (lognormal point
    targets, median 2e4, sigma 1.5, cap 2e5, 20% empty, seed 0 + region index), each
    run alone until all its points stop: the 8 with the most points and 8 more drawn
    (seeded) from the other non-empty regions.

A digest is the SHA-256 of the records sorted by id (for a whole-volume run the
fields id, next_id, prev_id, step, x, x_prev; for a bounded region every byte of the
160-byte record) and of the event list in listing order.

Run from the repository root: python tests/golden/make_full_size.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1011_4046_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "full_size.json")
STATE_FIELDS = ("id", "next_id", "prev_id", "step", "x", "x_prev")
BATCH_SAMPLE_SEED = 2024


def sha(b):
    return hashlib.sha256(b).hexdigest()


def state_digest(recs):
    """Digest of a whole-volume run's state: the fields that define it, by id."""
    r = recs[np.argsort(recs["id"], kind="stable")]
    parts = [np.ascontiguousarray(r[f]).tobytes() for f in STATE_FIELDS]
    return sha(b"".join(parts))


def record_digest(recs):
    """Digest of a bounded region's output surfaces: every record byte, by id."""
    return sha(recs[np.argsort(recs["id"], kind="stable")].tobytes())


def step_counts(ev, step0):
    """Events per step, as [[step - step0, count], ...] for the steps that have any."""
    if len(ev) == 0:
        return []
    s, c = np.unique(ev["step"], return_counts=True)
    return [[int(a) - int(step0), int(b)] for a, b in zip(s, c)]


def summary(recs, ev, st, step0, bounded):
    return dict(
        records=int(len(recs)), events=int(len(ev)),
        records_sha256=record_digest(recs) if bounded else state_digest(recs),
        events_sha256=sha(ev.tobytes()),
        step_counts=step_counts(ev, step0),
        point_steps=int(st["point_steps"]), candidates=int(st["candidates"]),
        confirmed=int(st["confirmed"]), accepted=int(st["accepted"]), steps=int(st["steps"]))


def batch_sample(counts):
    """Region indices of the batched sample: the 8 largest (ties by index), then 8
    drawn without replacement from the other non-empty regions."""
    live = np.nonzero(counts > 0)[0]
    big = sorted(live, key=lambda r: (-int(counts[r]), int(r)))[:8]
    rest = np.array([r for r in live if r not in set(big)])
    rng = np.random.default_rng(BATCH_SAMPLE_SEED)
    extra = rng.choice(rest, size=8, replace=False)
    return [int(r) for r in big] + sorted(int(r) for r in extra)


def main():
    out = {"description": __doc__.strip().splitlines()[0], "oracle_threads": O.threads()}
    t = time.time()
    net = I.vv_network(m=32, seed=0)
    o, oe, st = O.run(net, 100000, t_end=16.0)
    out["matter32"] = dict(config="VV 32^3 seed 0, matter era, eta 8 -> 16",
                           points=int(len(net["recs"])),
                           **summary(o, oe, st, net["recs"]["step"][0], False))
    print(f"matter32: {st['steps']} steps, {len(oe)} events ({time.time() - t:.0f} s)", flush=True)

    t = time.time()
    net = I.vv_network(m=64, seed=0)
    o, oe, st = O.run(net, 20)
    out["matter64_20"] = dict(config="VV 64^3 seed 0, matter era, first 20 steps",
                              points=int(len(net["recs"])),
                              **summary(o, oe, st, net["recs"]["step"][0], False))
    print(f"matter64_20: {len(net['recs'])} points, {len(oe)} events "
          f"({time.time() - t:.0f} s)", flush=True)

    t = time.time()
    nt = I.lognormal_regions(512, median=2e4, sigma=1.5, cap=2e5, p_empty=0.2, seed=0)
    parts, box = I.region_batch(nt, size=4.0, seed=0, slots=8, workers=8)
    counts = np.array([len(p[0]) for p in parts])
    sample = batch_sample(counts)
    print(f"batched512: {int(counts.sum())} points, sample {sample} "
          f"({time.time() - t:.0f} s)", flush=True)
    regions = {}
    for r in sample:
        t = time.time()
        recs, geom = parts[r]
        o, oe, st = O.run(dict(recs=recs, box=box, cosmology=I.MATTER, geom=geom), 100000)
        regions[str(r)] = dict(points=int(len(recs)),
                               **summary(o, oe, st, recs["step"][0], True))
        print(f"  region {r}: {len(recs)} points, {st['steps']} steps, {len(oe)} events "
              f"({time.time() - t:.0f} s)", flush=True)
    out["batched512"] = dict(
        config="512 regions, lognormal targets median 2e4 sigma 1.5 cap 2e5, 20% empty, "
               "seed 0, size 4, 8x8x8 slots; each sampled region run alone",
        total_points=int(counts.sum()), sample_seed=BATCH_SAMPLE_SEED, regions=regions)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
