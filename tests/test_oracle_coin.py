"""Pins of the oracle's intercommutation probability p (CPU). Section "Semi-parallel
cosmic string simulation": strings that cross exchange partners with probability p,
1 for field-theory strings and down to 1e-3 for superstrings.

The generator is pinned to numpy's own Philox4x64-10; each step's decisions are pinned
to a greedy matching recomputed here from that step's confirmed crossings and numpy's
numbers; the fraction of crossings that pass through is pinned to 1 - p by a binomial
bound; p = 1 is pinned to the default run."""
import numpy as np
import pytest

import oracle as O
from paper_1011_4046_amd import inputs as I

M64 = (1 << 64) - 1


def numpy_philox(ctr, key):
    """Philox4x64-10 of one counter from numpy's bit generator, which steps its
    counter by one before each block: start it one below."""
    c = [int(v) for v in ctr]
    i = 0
    while True:
        c[i] = (c[i] - 1) & M64
        if c[i] != M64 or i == 3:
            break
        i += 1
    g = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                         key=np.array([int(v) for v in key], dtype=np.uint64))
    return g.random_raw(4)


def numpy_coin(seed, step, ida, idb):
    w = int(numpy_philox([ida, idb, step & M64, 0], [seed, 0])[0])
    return (w >> 11) * 2.0 ** -53


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 11, 13), (123456789, 987654321)),
    ((0, 1, 0, 0), (1, 2)),                       # numpy's counter borrows into word 1
    ((M64, M64, M64, M64), (M64, M64)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_philox_matches_numpy(ctr, key):
    assert np.array_equal(O.philox4x64(ctr, key), numpy_philox(ctr, key))


def test_coin_is_the_top_53_bits_of_the_first_word():
    rng = np.random.default_rng(5)
    for _ in range(200):
        seed = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        step = int(rng.integers(-5, 1 << 20))
        ida, idb = sorted(int(v) for v in rng.integers(0, 1 << 40, 2))
        u = O.coin(seed, step, ida, idb)
        assert u == numpy_coin(seed, step, ida, idb)
        assert 0.0 <= u < 1.0


def test_p_out_of_range_is_rejected():
    net = I.vv_network(m=4, seed=1)
    r = O.OracleRegion(net["recs"], net["box"], I.MATTER, 2.0)
    for p in (-1e-300, -0.5, 1.5, float("nan")):
        with pytest.raises(ValueError):
            r.evolve(1, p=p)
    r.evolve(1, p=0.0)  # every crossing passes through
    r.close()


def test_p_one_is_the_default_run():
    net = I.vv_network(m=6, seed=2)
    a = O.run(net, 120)
    b = O.run(net, 120, p=1.0, seed=99)
    assert a[0].tobytes() == b[0].tobytes() and a[1].tobytes() == b[1].tobytes()
    assert len(a[1]) > 0 and np.all(a[1]["kind"] == 0) and b[2]["passed"] == 0


def greedy(conf_ids, exchange):
    """Greedy matching over the crossings that exchange, in key order: one per element
    (an element is named by its left point's id)."""
    used, out = set(), []
    for (a, b), x in zip(conf_ids, exchange):
        if not x or a in used or b in used:
            continue
        used.update((a, b))
        out.append((a, b))
    return out


@pytest.mark.parametrize("p,seed", [(0.5, 11), (0.15, 3)])
def test_each_step_follows_the_coins_and_the_greedy_order(p, seed):
    net = I.vv_network(m=6, seed=1)
    r = O.OracleRegion(net["recs"], net["box"], I.MATTER, 2.0)
    n_ev = 0
    seen_pass = 0
    for _ in range(90):
        before = r.read()
        nxt0 = dict(zip(before["id"].tolist(), before["next_id"].tolist()))
        step = r.step
        r.evolve(1, p=p, seed=seed)
        t, ids, _ = r.last_confirmed()
        ev = r.events()[n_ev:]
        n_ev += len(ev)
        assert np.all(ev["step"] == step)
        u = np.array([numpy_coin(seed, step, a, b) for a, b in ids])
        exch = u < p
        acc = greedy([tuple(x) for x in ids.tolist()], exch)
        # logged in key order: every crossing that passes through, and the matching
        want = [(int(a), int(b), 0 if x else 1) for (a, b), x in zip(ids.tolist(), exch)
                if not x or (int(a), int(b)) in set(acc)]
        got = list(zip(ev["id_a"].tolist(), ev["id_b"].tolist(), ev["kind"].tolist()))
        assert got == want
        assert np.array_equal(ev["t_star"], t[[i for i, (a, b) in enumerate(ids.tolist())
                                               if not exch[i] or (a, b) in set(acc)]])
        # exchanges swap the right neighbours; crossings that pass leave them alone
        after = r.read()
        nxt1 = dict(zip(after["id"].tolist(), after["next_id"].tolist()))
        moved = {}
        for a, b in acc:
            moved[a], moved[b] = nxt0[b], nxt0[a]
        for k in nxt0:
            assert nxt1[k] == moved.get(k, nxt0[k])
        seen_pass += int((~exch).sum())
    st = r.stats()
    assert st["passed"] == seen_pass > 0
    assert st["accepted"] + st["passed"] == len(r.events())
    r.close()


def test_fraction_passing_through_is_one_minus_p():
    p = 0.3
    net = I.vv_network(m=12, seed=4)
    _, ev, st = O.run(net, 300, p=p, seed=1234)
    n, k = st["confirmed"], st["passed"]
    assert n > 1500
    sd = np.sqrt(n * p * (1 - p))
    assert abs(k - n * (1 - p)) < 5 * sd
    assert k == int((ev["kind"] == 1).sum())


def test_removed_loops_saw_no_crossing_of_either_kind_in_their_last_period():
    net = I.vv_network(m=6, seed=1)
    box = net["box"]
    r = O.OracleRegion(net["recs"], box, I.MATTER, 2.0)
    r.evolve(300, loop_every=8, p=0.2, seed=8)
    lp, ev, rec = r.loops(), r.events(), r.read()
    assert len(lp) > 0 and np.any(ev["kind"] == 1)
    removed = rec[(rec["flags"] & O.FLAG_REMOVED) != 0]
    by_id = {int(x["id"]): x for x in removed}
    for L in lp:
        ids, k = [], int(L["rep_id"])
        while True:
            ids.append(k)
            k = int(by_id[k]["next_id"])
            if k == int(L["rep_id"]):
                break
        s = set(ids)
        recent = ev[ev["step"] >= L["step"] - L["n_points"]]
        assert not any(int(a) in s or int(b) in s for a, b in zip(recent["id_a"], recent["id_b"]))
    r.close()
