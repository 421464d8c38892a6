"""CPU checks of the C ABI: the library loads and exports every declared symbol, and
argument errors are reported without touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1011_4046_amd import semipar as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semipar.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char\s*\*|const char\s*\*)\s*\**\s*(\w+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ("region_init_from_surfaces", "region_evolve", "region_emit_final_surfaces",
              "region_events", "region_destroy", "semipar_strerror"):
        assert n in names
    assert sorted(S.SYMBOLS) == names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(S.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_every_call_has_a_ctypes_signature():
    """Without argtypes ctypes passes Python ints as C int: 64-bit pointers and sizes
    would be truncated."""
    L = S.lib()
    for name in S.SYMBOLS:
        assert getattr(L, name).argtypes is not None, name


LAYOUT_C = r"""
#include <stdio.h>
#include <stddef.h>
#include "semipar.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
#define Z(T) printf(#T " %zu\n", sizeof(T));
int main(void) {
  Z(semipar_point_rec) Z(semipar_event) Z(semipar_surface) Z(semipar_region_geom)
  Z(semipar_region_desc) Z(semipar_evolve_params) Z(semipar_evolve_stats)
  Z(semipar_tiling) Z(semipar_sched_params) Z(semipar_sched_stats) Z(semipar_loop)
  Z(semipar_handoff)
  F(semipar_handoff, geoms) F(semipar_handoff, ic) F(semipar_handoff, n_points)
  F(semipar_handoff, ic_mem) F(semipar_handoff, hist) F(semipar_handoff, hist_slices)
  F(semipar_handoff, stream)
  F(semipar_region_desc, stream) F(semipar_region_desc, inv2g) F(semipar_region_desc, sub)
  F(semipar_evolve_params, screen_split) F(semipar_evolve_params, loop_every)
  F(semipar_evolve_stats, timed_kernel_launches) F(semipar_evolve_stats, loop_points)
  F(semipar_evolve_stats, resolve_rounds) F(semipar_sched_params, pack)
  F(semipar_evolve_params, p) F(semipar_evolve_params, seed) F(semipar_evolve_params, cell_factor)
  F(semipar_evolve_stats, passed)
  F(semipar_loop, rep_id) F(semipar_loop, energy) F(semipar_loop, centre)
  F(semipar_tiling, surfaces) F(semipar_tiling, stream)
  F(semipar_sched_params, cost) F(semipar_sched_params, evolve) F(semipar_sched_params, out)
  F(semipar_sched_params, lane_sleep_ms) F(semipar_sched_params, lane_submit_ms)
  F(semipar_sched_stats, lane_held_ms) F(semipar_sched_stats, lanes_started)
  F(semipar_sched_params, events_cap) F(semipar_sched_params, region_ms)
  F(semipar_sched_params, lanes) F(semipar_sched_params, loops)
  F(semipar_sched_params, loops_off)
  F(semipar_sched_stats, makespan_ms) F(semipar_sched_stats, timed_kernel_launches)
  F(semipar_sched_stats, loops) F(semipar_sched_stats, passed)
  printf("SEMIPAR_FLAG_REMOVED %d\n", SEMIPAR_FLAG_REMOVED);
  return 0;
}
"""


def c_layout(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(LAYOUT_C)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (line.split() for line in out.splitlines())}


def test_record_layouts_match_header(tmp_path):
    from paper_1011_4046_amd.inputs import EVENT_DTYPE, LOOP_DTYPE, REC_DTYPE
    c = c_layout(tmp_path)
    assert c["semipar_point_rec"] == REC_DTYPE.itemsize == 160
    assert c["semipar_event"] == EVENT_DTYPE.itemsize == 56
    assert c["semipar_loop"] == LOOP_DTYPE.itemsize == 48
    assert c.pop("SEMIPAR_FLAG_REMOVED") == S.FLAG_REMOVED
    for f in ("rep_id", "energy", "centre"):
        assert c.pop(f"semipar_loop.{f}") == LOOP_DTYPE.fields[f][1]
    pairs = {"semipar_surface": S.Surface, "semipar_region_geom": S.RegionGeom,
             "semipar_region_desc": S.RegionDesc, "semipar_evolve_params": S.EvolveParams,
             "semipar_evolve_stats": S.EvolveStats, "semipar_tiling": S.Tiling,
             "semipar_sched_params": S.SchedParams, "semipar_sched_stats": S.SchedStats,
             "semipar_handoff": S.Handoff}
    for cname, py in pairs.items():
        assert c[cname] == ctypes.sizeof(py), cname
    fields = {"semipar_region_desc": S.RegionDesc, "semipar_evolve_params": S.EvolveParams,
              "semipar_evolve_stats": S.EvolveStats, "semipar_tiling": S.Tiling,
              "semipar_sched_params": S.SchedParams, "semipar_sched_stats": S.SchedStats,
              "semipar_handoff": S.Handoff}
    for key, off in c.items():
        if "." in key:
            cname, f = key.split(".")
            assert getattr(fields[cname], f).offset == off, key
    for n, name in ((S.MLP_IN, "IN"), (S.MLP_HIDDEN, "HIDDEN"), (S.MLP_PARAMS, "PARAMS")):
        assert re.search(rf"#define SEMIPAR_MLP_{name} {n}\b", open(HEADER).read())
    assert S.MLP_PARAMS == 64 * 12 + 64 + 64 * 64 + 64 + 64 + 1


def test_scheduler_without_gpu_work():
    """Empty regions are only noted (no launch), and predecessor counts that leave a
    region never ready are an argument error."""
    import numpy as np
    from paper_1011_4046_amd import inputs as I
    geom, _ = I.region_geometry(4.0, 8.0)
    empty = np.zeros(0, dtype=I.REC_DTYPE)
    rs = S.RegionSet(empty, [0, 0, 0], [geom] * 3, 16.0, I.MATTER,
                     n_pred=[0, 1, 1], succ=[[1, 2], [], []])
    res = S.schedule_regions(rs, policy=S.SCHED_BATCHED)
    st = res["stats"]
    assert st["regions"] == 3 and st["empty_regions"] == 3 and st["batches"] == 0
    assert list(res["region_batch"]) == [-1, -1, -1]
    assert list(res["out_off"]) == [0] * 13
    cyc = S.RegionSet(empty, [0, 0], [geom] * 2, 16.0, I.MATTER, n_pred=[1, 1], succ=[[1], [0]])
    with pytest.raises(S.SemiparError):
        S.schedule_regions(cyc)
    L = S.lib()
    t = rs.tiling()
    p = S.SchedParams()
    p.policy = 7
    assert L.schedule_regions(ctypes.byref(t), ctypes.byref(p), None) == -1
    assert L.schedule_regions(None, ctypes.byref(p), None) == -1
    t.box = -1.0
    p.policy = 0
    assert L.schedule_regions(ctypes.byref(t), ctypes.byref(p), None) == -1


def test_mlp_host_normalisation_and_argument_errors():
    import numpy as np
    rng = np.random.default_rng(0)
    x = rng.normal(3.0, 2.0, (500, 12)).astype(np.float32)
    x[:, 5] = 1.0  # constant feature: scale 1
    norm = np.zeros(24, np.float32)
    L = S.lib()
    assert L.semipar_mlp_norm(x.ctypes.data, len(x), norm.ctypes.data) == 0
    xd = x.astype(np.float64)
    assert np.allclose(norm[:12], xd.mean(0), rtol=1e-6)
    sd = xd.std(0)
    expect = np.where(sd > 1e-6, 1.0 / np.where(sd > 0, sd, 1), 1.0)
    assert np.allclose(norm[12:], expect, rtol=1e-5)
    assert L.semipar_mlp_norm(None, 3, norm.ctypes.data) == -1
    assert L.semipar_mlp_forward(None, None, None, 1, None, None) == -1
    assert L.semipar_mlp_loss_grad(None, None, None, None, 0, None, None, None) == -1
    assert L.semipar_mlp_adam_step(None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.semipar_mlp_train(None, None, None, None, None, None, 0, 1, 0, 1e-3, None, None) == -1


def test_argument_errors_without_gpu():
    L = S.lib()
    h = ctypes.c_void_p()
    assert L.region_init_from_surfaces(None, None, 0, ctypes.byref(h)) == -1
    d = S.RegionDesc()
    d.box = -1.0
    assert L.region_init_from_surfaces(ctypes.byref(d), None, 0, ctypes.byref(h)) == -1
    d = S.RegionDesc()
    d.cosmology, d.box = 7, 1.0
    assert L.region_init_from_surfaces(ctypes.byref(d), None, 0, ctypes.byref(h)) == -1
    assert L.region_evolve(None, None, None) == -1
    n = (ctypes.c_int64 * 4)()
    assert L.region_emit_final_surfaces(None, None, None, n, 0) == -1
    L.region_destroy(None)
    # the hand-off run checks its tiling before touching the device
    import numpy as np
    from paper_1011_4046_amd import inputs as I
    p = S.SchedParams()
    assert L.schedule_handoff(None, ctypes.byref(p), None) == -1
    geom, _ = I.region_geometry(4.0, 8.0)
    g = (S.RegionGeom * 2)(S._geom_struct(geom), S._geom_struct(geom))
    npred = np.zeros(2, np.int32)
    off = np.zeros(3, np.int32)
    rec = np.zeros(4, I.REC_DTYPE)
    fake = np.zeros(8)
    h = S.Handoff()
    h.n_regions, h.cosmology, h.box = 2, I.MATTER, 16.0 * np.sqrt(2.0) / 4.0 * 1.01
    h.geoms, h.n_pred, h.succ_off = ctypes.addressof(g), npred.ctypes.data, off.ctypes.data
    h.ic, h.n_points, h.ic_mem = rec.ctypes.data, 4, S.MEM_HOST
    h.hist, h.hist_slices = fake.ctypes.data, 2
    assert L.schedule_handoff(ctypes.byref(h), ctypes.byref(p), None) == -1  # box
    h.box = 4.0 / (2.0 * geom[4])
    assert L.schedule_handoff(ctypes.byref(h), ctypes.byref(p), None) == -1  # one name twice
    h.hist_slices = 1
    assert L.schedule_handoff(ctypes.byref(h), ctypes.byref(p), None) == -1
    assert S.strerror(-2).startswith("inconsistent surface")
    assert "gfx950" in S.version()


def test_fork_guard_sees_a_loaded_gpu_runtime():
    """The input generators fork worker processes only while no GPU runtime is mapped
    in this process: loading libsemipar (which maps the HSA runtime) or a profiler's
    preload turns the guard on even when torch never touched the GPU."""
    import subprocess
    import sys
    code = (
        "import ctypes, sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from paper_1011_4046_amd import inputs as I, build as B\n"
        "before = I._gpu_in_use()\n"
        "ctypes.CDLL(B.LIB)\n"
        "print(before, I._gpu_in_use())\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         check=True).stdout.split()
    assert out == ["False", "True"], out
