"""Pins of the cost-model oracle (CPU): its gradient against central finite differences,
its forward pass against closed forms, Adam's first step against its closed form, and
its features against strings whose speed, spacing and layout are known exactly."""
import numpy as np
import pytest

from oracle import costmodel as C
from paper_1011_4046_amd import inputs as I


def rand_params(rng, scale=0.3):
    return rng.normal(0.0, scale, C.NP)


def test_parameter_count_and_layout():
    assert C.NP == 64 * 12 + 64 + 64 * 64 + 64 + 64 + 1 == 5057
    p = np.arange(C.NP, dtype=np.float64)
    d = C.unpack(p)
    assert d["W1"][1, 0] == 12 and d["b1"][0] == 768 and d["W2"][0, 1] == 833
    assert d["b2"][0] == 4928 and d["w3"][0] == 4992 and d["b3"] == 5056
    assert np.array_equal(C.pack(d), p)


def test_forward_closed_forms():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(50, 12))
    # all weights zero: the output is the last bias
    d = {k: np.zeros(s) for k, s in C.SIZES}
    d["b3"] = 2.5
    y, _ = C.forward(C.pack(d), x)
    assert np.all(y == 2.5)
    # |x0| = relu(x0) + relu(-x0), passed through an identity second layer
    d = {k: np.zeros(s) for k, s in C.SIZES}
    d["W1"][0, 0], d["W1"][1, 0] = 1.0, -1.0
    d["W2"][0, 0], d["W2"][1, 1] = 1.0, 1.0
    d["w3"][0], d["w3"][1] = 1.0, 1.0
    y, _ = C.forward(C.pack(d), x)
    assert np.array_equal(y, np.abs(x[:, 0]))
    # normalisation: (x - mu) * s applied before the first layer
    norm = np.concatenate([np.full(12, 3.0), np.full(12, 0.5)])
    y2, _ = C.forward(C.pack(d), x, norm)
    assert np.allclose(y2, np.abs((x[:, 0] - 3.0) * 0.5), rtol=0, atol=1e-15)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    p = rand_params(rng)
    x = rng.normal(size=(40, 12))
    t = rng.normal(size=40)
    norm = C.norm_of(x)
    l0, g = C.loss_grad(p, x, t, norm)
    assert l0 == pytest.approx(C.loss(p, x, t, norm), rel=1e-14)
    idx = np.concatenate([rng.choice(C.NP, 300, replace=False), [C.NP - 1, 768, 4928]])
    h = 1e-6
    for i in idx:
        e = np.zeros(C.NP)
        e[i] = h
        fd = (C.loss(p + e, x, t, norm) - C.loss(p - e, x, t, norm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(g[i]), (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.normal(size=C.NP)
    g = rng.normal(size=C.NP)
    z = np.zeros(C.NP)
    p1, m, v = C.adam_step(p, z, z, g, 1, lr=0.01)
    # after bias correction m_hat = g, v_hat = g^2
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_fits_a_smooth_target():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(256, 12))
    t = 0.7 * x[:, 0] - 0.4 * x[:, 3] + 0.2 * np.abs(x[:, 5])
    p, losses = C.train(rand_params(rng, 0.1), x, t, 400, lr=3e-3)
    assert losses[-1] < 0.02 * losses[0]


def _geom(size=4.0, centre=(0.0, 0.0, 0.0)):
    geom, g = I.region_geometry(size, 8.0, centre)
    return geom, g


def test_features_of_a_moving_straight_string():
    """A straight string moving uniformly at speed v: RMS transverse speed v, spatial
    spacing of neighbours delta sqrt(1 - v^2), one closed string (no open piece)."""
    box = 8.0
    for v in (0.0, 0.6):
        chain, delta = I.straight_string(256, box, v=v)
        net = I.make_network([chain], box, delta, 8.0, I.MATTER)
        geom, g = _geom()
        f = C.features(net["recs"], geom, box)
        assert f[0] == pytest.approx(np.log1p(256))
        assert f[1] == 0.0
        assert f[2] == pytest.approx(v, abs=1e-12)
        edge = delta * np.sqrt(1.0 - v * v)
        assert f[11] == pytest.approx(np.log1p(edge / (np.sqrt(2.0) * g)), rel=1e-12)
        assert f[3:11].sum() == pytest.approx(1.0)


def test_features_occupancy_histogram_by_hand():
    """Points placed by hand in known cells: 48 in one cell, 16 in another, with no
    links (every point is an open piece of its own)."""
    geom, g = _geom()
    h = 2 * g / 16
    recs = np.zeros(64, dtype=I.REC_DTYPE)
    recs["id"] = np.arange(64)
    recs["next_id"] = -1
    recs["prev_id"] = -1
    recs["step"] = 1
    pos = np.zeros((64, 3))
    pos[:48] = [-g + 0.5 * h, -g + 0.5 * h, -g + 0.5 * h]   # cell (0, 0, 0)
    pos[48:] = [0.25 * h, 0.25 * h, 0.25 * h]               # cell (8, 8, 8)
    recs["x"][:, :3] = pos
    recs["x"][:, 3] = 8.0
    recs["x_prev"][:, :3] = pos
    recs["x_prev"][:, 3] = 7.9
    f = C.features(recs, geom, 64.0)
    # relative occupancy 48 * 4096 / 64 = 3072 -> bin 7 (clamped); 16 * 64 = 1024 -> bin 7
    assert f[1] == pytest.approx(np.log1p(64))
    assert f[2] == 0.0 and f[11] == 0.0
    assert f[10] == pytest.approx(1.0)
    # a sparse region: one point per cell in 64 distinct cells -> rel = 64, bin 7 too;
    # 4096 points one per cell -> rel 1 -> bin 4
    recs2 = np.zeros(4096, dtype=I.REC_DTYPE)
    recs2["id"] = np.arange(4096)
    recs2["next_id"] = recs2["prev_id"] = -1
    ii = np.arange(4096)
    c = np.stack([ii // 256, (ii // 16) % 16, ii % 16], 1)
    p2 = -g + (c + 0.5) * h
    recs2["x"][:, :3] = p2
    recs2["x_prev"][:, :3] = p2
    f2 = C.features(recs2, geom, 64.0)
    assert f2[3 + 4] == pytest.approx(1.0) and f2[3:11].sum() == pytest.approx(1.0)


def test_features_follow_the_region_index():
    """Moving a region by whole generator steps (index + k e_m) and its points by the
    generators' spatial part leaves every feature unchanged: the occupancy grid is
    centred on the region, not on the tiling's lattice origin."""
    net = I.region_network(3000, 4.0, seed=5)
    recs, geom, g, box = net["recs"], net["geom"], net["g"], net["box"]
    f0 = C.features(recs, geom, box)
    gens = 0.5 * g * np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    for m in range(4):
        for k in (1, -2, 3):
            geom2 = geom.copy()
            geom2[5 + m] += k
            r2 = recs.copy()
            r2["x"][:, :3] += k * gens[m]
            r2["x_prev"][:, :3] += k * gens[m]
            assert np.allclose(C.features(r2, geom2, box), f0, rtol=1e-12, atol=1e-12), (m, k)
    # a region displaced without moving its index sees its points off-centre
    geom3 = geom.copy()
    geom3[5] += 1
    assert not np.allclose(C.features(recs, geom3, box), f0)
