"""CPU oracle of the region cost model -- TEST INFRASTRUCTURE ONLY.

Plain FP64 NumPy versions of what the library's cost-model path computes: the 12
features of a region's initial surface, the 12 -> 64 -> 64 -> 1 ReLU perceptron, its
mean-squared-error gradient (backpropagation written out layer by layer), and Adam
(Kingma and Ba, "Adam: a method for stochastic optimization", 2015, Algorithm 1).
Paper, Section "Performance": the elapsed time is set by the most difficult regions,
so the scheduler orders and groups regions by a predicted cost.

Only tests and the CPU baseline may import this module. It shares no code with the
HIP path.

Parameter block (5057 values, row-major): W1[64][12], b1[64], W2[64][64], b2[64],
w3[64], b3.
"""
from __future__ import annotations

import numpy as np

NI, NH = 12, 64
SIZES = [("W1", (NH, NI)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)),
         ("b3", ())]
NP = sum(int(np.prod(s)) if s else 1 for _, s in SIZES)


def unpack(params):
    """Views of the parameter block as named arrays (FP64 copies)."""
    p = np.asarray(params, dtype=np.float64).ravel()
    assert p.size == NP
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape)) if shape else 1
        out[name] = p[o:o + n].reshape(shape) if shape else p[o]
        o += n
    return out


def pack(d):
    return np.concatenate([np.atleast_1d(np.asarray(d[name], np.float64)).ravel()
                           for name, _ in SIZES])


def normalise(x, norm):
    x = np.asarray(x, dtype=np.float64)
    if norm is None:
        return x
    norm = np.asarray(norm, dtype=np.float64)
    return (x - norm[:NI]) * norm[NI:]


def forward(params, x, norm=None):
    """y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 for every row of x."""
    P = unpack(params)
    xn = normalise(x, norm)
    z1 = xn @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["w3"] + P["b3"]
    return y, (xn, z1, h1, z2, h2)


def loss(params, x, target, norm=None):
    y, _ = forward(params, x, norm)
    return float(np.mean((y - np.asarray(target, np.float64)) ** 2))


def loss_grad(params, x, target, norm=None):
    """Mean squared error and its gradient with respect to the parameter block."""
    P = unpack(params)
    y, (xn, z1, h1, z2, h2) = forward(params, x, norm)
    n = len(y)
    e = y - np.asarray(target, np.float64)
    dy = 2.0 * e / n                         # dL/dy
    g = {"b3": dy.sum(), "w3": dy @ h2}
    d2 = np.outer(dy, P["w3"]) * (z2 > 0)    # dL/dz2
    g["b2"] = d2.sum(0)
    g["W2"] = d2.T @ h1
    d1 = (d2 @ P["W2"]) * (z1 > 0)           # dL/dz1
    g["b1"] = d1.sum(0)
    g["W1"] = d1.T @ xn
    return float(np.mean(e ** 2)), pack(g)


def adam_step(params, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at 1-based step number `step`; returns new (params, m, v)."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def train(params, x, target, iters, lr=1e-3, norm=None):
    """Full-batch Adam on the mean squared error; returns params and the losses before
    each step plus the final one."""
    p = np.asarray(params, np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for it in range(iters):
        l, g = loss_grad(p, x, target, norm)
        losses.append(l)
        p, m, v = adam_step(p, m, v, g, it + 1, lr)
    losses.append(loss(p, x, target, norm))
    return p, np.array(losses)


def norm_of(x):
    """Per-feature mean and inverse standard deviation (scale 1 below 1e-6)."""
    x = np.asarray(x, np.float64)
    mu, sd = x.mean(0), x.std(0)
    return np.concatenate([mu, np.where(sd > 1e-6, 1.0 / np.where(sd > 0, sd, 1.0), 1.0)])


# ---- features of a region's initial surface -------------------------------------

def features(recs, geom, box):
    """The 12 features of one region's records (FP64):
      0 log1p(points), 1 log1p(points without a left neighbour),
      2 RMS over points with a right neighbour j of |(L - B) + (R - B)| / (dt_L + dt_R)
        (L = x_k, R = x_j, B = x_prev_j; spatial parts by minimum image),
      3..10 fraction of the points in 16^3 grid cells over the cube of side 2g around the
        region's spatial centre whose count relative to n / 4096 has
        floor(log2) + 4 = b (clamped to 0..7),
      11 log1p(mean |R - L| / size), size = sqrt(2) g."""
    n = len(recs)
    f = np.zeros(12)
    if n == 0:
        return f
    ids = recs["id"]
    order = np.argsort(ids)
    sid = ids[order]

    def find(q):
        pos = np.searchsorted(sid, q)
        pos = np.clip(pos, 0, n - 1)
        ok = (q >= 0) & (sid[pos] == q)
        return np.where(ok, order[pos], -1)

    j = find(recs["next_id"])
    pv = find(recs["prev_id"])
    x, xp = recs["x"], recs["x_prev"]
    L = x[:, :3]
    has = j >= 0
    jj = np.where(has, j, 0)
    R, B = x[jj, :3], xp[jj, :3]

    def mi(d):
        return d - box * np.rint(d / box)

    a = mi(L - B)
    vv = a + (R - B)
    dt = (x[:, 3] - xp[jj, 3]) + (x[jj, 3] - xp[jj, 3])
    okv = has & (dt > 0)
    v2 = np.where(okv, (vv ** 2).sum(1) / np.where(okv, dt, 1.0) ** 2, 0.0)
    e = np.sqrt((mi(R - L) ** 2).sum(1))
    g = 0.5 / geom[4]
    size = np.sqrt(2.0) * g
    # the region's spatial centre: the lattice origin plus g/2 times the index summed
    # along the generators' spatial parts (1,1,1), (1,-1,-1), (-1,1,-1), (-1,-1,1)
    i1, i2, i3, i4 = (float(v) for v in geom[5:9])
    steps = np.array([i1 + i2 - i3 - i4, i1 - i2 + i3 - i4, i1 - i2 - i3 + i4])
    centre = np.asarray(geom[:3], dtype=np.float64) + (0.25 / geom[4]) * steps
    c = mi(L - centre)
    ci = np.floor((c + g) * (16 / (2.0 * g))).astype(np.int64)
    ci = np.clip(ci, 0, 15)
    cell = (ci[:, 0] * 16 + ci[:, 1]) * 16 + ci[:, 2]
    occ = np.bincount(cell, minlength=4096)
    f[0] = np.log1p(n)
    f[1] = np.log1p(np.count_nonzero(pv < 0))
    f[2] = np.sqrt(v2[okv].sum() / okv.sum()) if okv.any() else 0.0
    for o in occ[occ > 0]:
        b = int(np.floor(np.log2(o * 4096.0 / n))) + 4
        f[3 + min(max(b, 0), 7)] += o / n
    f[11] = np.log1p(e[has].sum() / has.sum() / size) if has.any() else 0.0
    return f
