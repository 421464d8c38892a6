"""Pins of the oracle's loop record and removal (CPU): in flat space a loop that never
intersects is removed after exactly one period with its exact energy and centre of
mass; a string winding the box is never removed; every removed loop of a matter-era
network is a closed, compact chain with no event during its last period."""
import numpy as np
import pytest

import oracle as O
from paper_1011_4046_amd import inputs as I


def flat_energy_and_centre(recs, box):
    """Energy sum |X[n][k] - X[n-1][j]| + |X[n][j] - X[n-1][j]| and mean position of each
    closed chain of the records, keyed by the chain's lowest record index."""
    idx = {int(i): k for k, i in enumerate(recs["id"])}
    seen = np.zeros(len(recs), bool)
    out = {}
    for k0 in range(len(recs)):
        if seen[k0]:
            continue
        cyc, k = [], k0
        while not seen[k]:
            seen[k] = True
            cyc.append(k)
            k = idx[int(recs["next_id"][k])]
        e, acc = 0.0, np.zeros(3)
        rep = min(cyc)
        for a in cyc:
            j = idx[int(recs["next_id"][a])]
            da = recs["x"][a, :3] - recs["x_prev"][j, :3]
            da -= box * np.rint(da / box)
            db = recs["x"][j, :3] - recs["x_prev"][j, :3]
            e += np.linalg.norm(da) + np.linalg.norm(db)
            d = recs["x"][a, :3] - recs["x"][rep, :3]
            acc += d - box * np.rint(d / box)
        out[rep] = (len(cyc), e, recs["x"][rep, :3] + acc / len(cyc))
    return out


def test_flat_loops_removed_after_one_period_with_exact_energy_and_centre():
    net = I.kt_loops(n_loops=8, n_pts=256, box=4.0, seed=3)
    init = flat_energy_and_centre(net["recs"], 4.0)
    r = O.OracleRegion(net["recs"], 4.0, I.FLAT, 0.0)
    # no intersection search: the loops never intercommute
    r.evolve(300, intercommute=False, loop_every=64)
    lp = r.loops()
    assert len(lp) == 8
    # step0 = 1; checks at 65, 129, 193, 257: the first with n - step0 >= 256 is 257
    assert np.all(lp["step"] == 257) and np.all(lp["n_points"] == 256)
    ids = net["recs"]["id"]
    for L in lp:
        rep = int(np.nonzero(ids == L["rep_id"])[0][0])
        n, e, c = init[rep]
        assert L["energy"] == pytest.approx(e, rel=1e-12)
        assert np.allclose(L["centre"], c, rtol=0, atol=1e-12)
    rec = r.read()
    assert np.all(rec["flags"] == O.FLAG_REMOVED) and np.all(rec["step"] == 257)
    assert r.active == 0


def test_winding_string_is_never_removed():
    chain, delta = I.straight_string(128, 4.0, v=0.3)
    net = I.make_network([chain], 4.0, delta, 0.0, I.FLAT)
    r = O.OracleRegion(net["recs"], 4.0, I.FLAT, 0.0)
    r.evolve(400, intercommute=False, loop_every=16)
    assert len(r.loops()) == 0 and r.active == len(net["recs"])


def test_removed_loops_are_quiet_closed_and_compact():
    net = I.vv_network(m=6, seed=1)
    box = net["box"]
    r = O.OracleRegion(net["recs"], box, I.MATTER, 2.0)
    r.evolve(300, loop_every=8)
    lp, ev, rec = r.loops(), r.events(), r.read()
    assert len(lp) > 0
    removed = rec[(rec["flags"] & O.FLAG_REMOVED) != 0]
    by_id = {int(x["id"]): x for x in removed}
    total = 0
    for L in lp:
        # the loop: follow next from its representative through removed points
        ids, k = [], int(L["rep_id"])
        while True:
            ids.append(k)
            x = by_id[k]
            assert x["step"] == L["step"]
            k = int(x["next_id"])
            if k == int(L["rep_id"]):
                break
        assert len(ids) == L["n_points"]
        total += len(ids)
        s = set(ids)
        recent = ev[ev["step"] >= L["step"] - L["n_points"]]
        assert not any(int(a) in s or int(b) in s for a, b in zip(recent["id_a"], recent["id_b"]))
        x0 = by_id[int(L["rep_id"])]["x"][:3]
        for i in ids:
            d = by_id[i]["x"][:3] - x0
            d -= box * np.rint(d / box)
            assert np.all(np.abs(d) < 0.25 * box)
    assert total == len(removed)
