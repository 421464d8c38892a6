"""Scheduling pipeline over libsemipar: learned cost model and autotuner.

Paper, Section "Performance": the elapsed time is set by the most difficult regions,
which a scheduler can start first and group with regions of similar cost. Here:

* features of every region's initial surface come from the library's GPU kernel;
* the cost model (12 -> 64 -> 64 -> 1, FP32) is trained by the library's own forward,
  gradient and Adam kernels on logged per-region step counts (log steps);
* the scheduler orders regions by the predicted steps and cuts them into launch
  batches (schedule_regions with a cost vector); without a model it falls back to the
  point-count order;
* an autotuner picks the batch size, the number of concurrent lanes, the screen split
  and the steps per host check by timing capped schedules of the whole workload, and
  caches the choice per workload.

Nothing here changes results: every choice only orders or groups regions, or sets
launch shapes.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import semipar as S


def init_params(seed=0):
    """He-uniform initial weights (seeded), zero biases, in the library's layout."""
    rng = np.random.default_rng(seed)
    ni, nh = S.MLP_IN, S.MLP_HIDDEN
    w1 = rng.uniform(-1, 1, (nh, ni)) * np.sqrt(6.0 / ni)
    w2 = rng.uniform(-1, 1, (nh, nh)) * np.sqrt(6.0 / nh)
    w3 = rng.uniform(-1, 1, nh) * np.sqrt(6.0 / nh)
    p = np.concatenate([w1.ravel(), np.zeros(nh), w2.ravel(), np.zeros(nh), w3, [0.0]])
    assert p.size == S.MLP_PARAMS
    return p.astype(np.float32)


class LearnedCost:
    """Cost model trained on logged (features, steps) pairs of earlier runs."""

    def __init__(self, seed=0):
        self.seed = seed
        self.model = S.CostModel(init_params(seed))
        self.losses = None
        self.val_losses = None
        self.best_iter = None

    def fit(self, feat, steps, iters=2000, lr=3e-3, holdout=0.0, chunk=100):
        """Train on log steps. holdout > 0: that share of the logged regions (seeded) is
        kept out of training; every `chunk` iterations the loss on it is measured, and the
        parameters with the lowest held-out loss are kept (early stopping)."""
        live = np.asarray(feat)[:, 0] > 0  # log1p(points) > 0: non-empty regions
        x = np.asarray(feat, np.float32)[live]
        y = np.log(np.maximum(np.asarray(steps, np.float64)[live], 1.0)).astype(np.float32)
        n_val = int(round(holdout * len(x))) if holdout > 0 and len(x) >= 10 else 0
        if n_val == 0:
            self.model.set_norm_from(x)
            self.losses = self.model.train(x, y, iters=iters, lr=lr)
            return self
        perm = np.random.default_rng(self.seed + 1).permutation(len(x))
        va, tr = perm[:n_val], perm[n_val:]
        self.model.set_norm_from(x[tr])
        losses, vals = [], []
        best, best_params, done = np.inf, None, 0
        while done < iters:
            k = min(chunk, iters - done)
            losses.append(self.model.train(x[tr], y[tr], iters=k, lr=lr)[:k])
            done += k
            v = float(np.mean((self.model.forward(x[va]) - y[va]) ** 2))
            vals.append(v)
            if v < best:
                best, best_params, self.best_iter = v, self.model.params.clone(), done
        self.model.params.copy_(best_params)
        self.losses = np.concatenate(losses)
        self.val_losses = np.array(vals)
        return self

    def predict(self, feat):
        """Predicted lattice steps per region (empty regions: 0)."""
        feat = np.asarray(feat, np.float32)
        y = np.exp(self.model.forward(feat)).astype(np.float32)
        return np.where(feat[:, 0] > 0, y, 0.0).astype(np.float32)


def learned_schedule(rs, cost_model, **kw):
    """Features on the GPU, cost-model inference, then the batched schedule."""
    t0 = time.perf_counter()
    feat = S.region_features(rs)
    pred = cost_model.predict(feat)
    t1 = time.perf_counter()
    res = S.schedule_regions(rs, S.SCHED_BATCHED, cost=pred, **kw)
    res["predict_ms"] = (t1 - t0) * 1e3
    res["pred"] = pred
    return res


# ---- autotuner ------------------------------------------------------------------

TUNABLE = {
    "batch_frac": [1.0, 0.5, 0.34, 0.25, 0.125],  # batch_points as a fraction of all points
    "lanes": [1, 2, 3],                            # batches evolved concurrently
    "screen_split": [5, 1],
    "steps_per_sync": [64, 32, 128],
    "pack": [S.PACK_POINTS, S.PACK_WORK],         # equal points / equal predicted work
    "cell_factor": [1.15, 1.0, 1.3, 1.6],         # cell edge / largest element extent
}


def workload_key(rs, screen):
    n = rs.counts[rs.counts > 0]
    return (f"r{rs.n_regions}-n{int(np.log2(max(int(n.sum()), 1)))}-"
            f"m{int(np.log2(max(int(np.median(n)) if len(n) else 1, 1)))}-c{rs.cosmology}-s{screen}")


def autotune(rs, cost=None, screen=S.SCREEN_F32, cache=None, max_steps=96, log=None):
    """Coordinate search over TUNABLE, timing one batched schedule of all regions per
    candidate, each batch cut after max_steps lattice steps (the per-step costs, not the
    tails, decide launch shapes; a batch size that splits regions of different length
    shows its cost as more batches). Returns the parameter dict; with `cache` (a JSON
    path) a previous choice for the same workload key is reused."""
    key = workload_key(rs, screen)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            got = json.load(f).get(key)
        if got:
            return dict(got, cached=True)
    total = int(rs.counts.sum())
    best = {k: v[0] for k, v in TUNABLE.items()}

    def run(cfg):
        bp = int(total * cfg["batch_frac"]) if cfg["batch_frac"] < 1.0 else 0
        res = S.schedule_regions(rs, S.SCHED_BATCHED, batch_points=bp, cost=cost,
                                 out=None, events=False, use_graph=True, screen=screen,
                                 screen_split=cfg["screen_split"],
                                 steps_per_sync=cfg["steps_per_sync"], max_steps=max_steps,
                                 lanes=cfg["lanes"], pack=cfg["pack"] if cost is not None else 0,
                                 cell_factor=cfg["cell_factor"])
        st = res["stats"]
        # time per point-step of the truncated schedule
        return st["makespan_ms"] / max(st["point_steps"], 1) * 1e6

    run(best)  # warm-up (graph instantiation, allocator)
    best_ms = run(best)
    for k, vals in TUNABLE.items():
        for v in vals[1:]:
            cfg = dict(best, **{k: v})
            ms = run(cfg)
            if log:
                log(f"autotune {key}: {cfg} -> {ms:.3f} ns per point-step")
            if ms < best_ms:
                best, best_ms = cfg, ms
    out = dict(best, ns_per_point_step=best_ms)
    if cache:
        data = {}
        if os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
        data[key] = out
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return out


def batch_points_for(rs, cfg):
    f = cfg.get("batch_frac", 1.0)
    return int(int(rs.counts.sum()) * f) if f < 1.0 else 0
