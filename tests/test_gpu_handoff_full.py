"""GPU parity of the hand-off tiling at full size: the 32^3 matter-era network's 4096-region
tiling run by schedule_handoff in the benchmark's launch shape (every ready region in one
batch per wave, graph-captured blocks of 32 steps, FP32 screen with FP64 confirmation,
one thread per element in the screen), against digests of the oracle's whole-volume run
(tests/golden/handoff.json, written by tests/golden/make_handoff.py from the oracle
alone): the set of vertices built, their values bit for bit, the diamonds per region and
the crossings found in each region.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from test_gpu_parity import say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def sha(b):
    return hashlib.sha256(b).hexdigest()


def test_hand_off_tiling_of_the_32_cubed_network():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1011_4046_amd import semipar as S
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    import make_handoff as MH
    with open(os.path.join(HERE, "golden", "handoff.json")) as f:
        gold = json.load(f)
    net, box, geoms, n_pred, succ, layer = MH.tiling()
    n = len(net["recs"])
    ns = gold["whole_volume_slices"] + 4
    say(f"hand-off 32^3 tiling: {n} points, {len(geoms)} regions, {ns} slices")
    hist = torch.empty((ns, n, 4), dtype=torch.float64, device="cuda")
    res = S.schedule_handoff(net["recs"], box, net["cosmology"], geoms, n_pred, succ, hist,
                             use_graph=True, screen=S.SCREEN_F32, steps_per_sync=32,
                             screen_split=1)
    torch.cuda.synchronize()
    st = res["stats"]
    say(f"  {st['point_steps']} point-steps, {st['events']} crossings, "
        f"{st['makespan_ms']:.0f} ms")
    assert st["point_steps"] == gold["point_steps"]
    ps = np.asarray(res["region_point_steps"], dtype=np.int64)
    assert sha(ps.tobytes()) == gold["point_steps_sha256"]
    built = ~torch.isnan(hist[:, :, 3]).reshape(-1)
    flat = torch.nonzero(built).reshape(-1)
    del built
    assert flat.numel() == gold["built"]
    assert sha(flat.cpu().numpy().astype(np.int64).tobytes()) == gold["built_sha256"]
    vals = hist.reshape(-1, 4)[flat].cpu().numpy()
    del flat, hist
    assert sha(np.ascontiguousarray(vals).tobytes()) == gold["vertices_sha256"]
    del vals
    ev, off = res["events"], res["events_off"]
    chunks = []
    for r in range(len(geoms)):
        w = ev[off[r]:off[r + 1]]
        if len(w):
            chunks.append(w[np.lexsort((w["id_b"], w["id_a"], w["t_star"], w["step"]))].tobytes())
    assert len(ev) == gold["events"]
    assert sha(b"".join(chunks)) == gold["events_sha256"]
