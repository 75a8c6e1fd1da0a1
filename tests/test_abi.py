"""The C-ABI library loads, exports every function that include/sf.h declares,
and validates arguments before touching the GPU (runs without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "sf.h")


@pytest.fixture(scope="module")
def L():
    from paper_2605_08528_amd import sf
    if not os.path.exists(sf.LIB_PATH):
        from paper_2605_08528_amd import build
        build.build()
    return sf.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sf_[a-z_]+)\s*\(", src)) - {"sf_sim"})


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sf_create", "sf_step", "sf_observe", "sf_reset", "sf_destroy",
                 "sf_get_state", "sf_set_state", "sf_get_contacts"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_defaults_and_status_strings(L):
    from paper_2605_08528_amd import sf
    p = sf.VehicleParams()
    assert L.sf_default_params(C.byref(p)) == 0
    assert abs(p.mass - 1500.0) < 1e-6 and abs(p.inertia[2] - 2800.0) < 1e-6
    o = sf.Options()
    assert L.sf_default_options(C.byref(o)) == 0
    assert o.max_episode_steps == 1500 and o.collision_warmup == 24
    assert L.sf_status_str(1) == b"invalid argument"
    assert L.sf_default_params(None) == 1


def _desc(sf, worlds, keep):
    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(C.c_void_p)
    d = sf.WorldDesc()
    d.num_worlds = worlds.num_worlds
    d.agent_offsets = arr(worlds.agent_offsets, np.int32)
    d.road_offsets = arr(worlds.road_offsets, np.int32)
    d.road_xy = arr(worlds.road_xy, np.float32)
    d.road_type = arr(worlds.road_type, np.uint8)
    d.tri_offsets = arr(worlds.tri_offsets, np.int32)
    d.tri_verts = arr(worlds.tri_verts, np.float32)
    d.tri_surface = arr(worlds.tri_surface, np.uint8)
    d.num_surfaces = worlds.num_surfaces
    d.mu_class = arr(worlds.mu_class, np.float32)
    d.spawn_offsets = arr(worlds.spawn_offsets, np.int32)
    d.spawn = arr(worlds.spawn, np.float32)
    return d


def test_create_rejects_bad_arguments_without_touching_the_gpu(L):
    from paper_2605_08528_amd import sf, inputs as I
    p = sf.make_params(I.VEHICLE_DEFAULTS)
    h = C.c_void_p()
    keep = []
    w = I.flat_plane(2)
    d = _desc(sf, w, keep)
    assert L.sf_create(None, C.byref(p), None, C.byref(h)) == 1
    assert L.sf_create(C.byref(d), C.byref(p), None, None) == 1
    # non-monotone offsets
    bad = I.flat_plane(2)
    bad.agent_offsets = np.array([0, -1], np.int32)
    assert L.sf_create(C.byref(_desc(sf, bad, keep)), C.byref(p), None, C.byref(h)) == 1
    assert b"non-decreasing" in L.sf_last_error()
    # too many agents in one world
    big = I.flat_plane(65)
    assert L.sf_create(C.byref(_desc(sf, big, keep)), C.byref(p), None, C.byref(h)) == 5
    # agents but no spawn entries
    nos = I.flat_plane(2)
    nos.spawn_offsets = np.array([0, 0], np.int32)
    assert L.sf_create(C.byref(_desc(sf, nos, keep)), C.byref(p), None, C.byref(h)) == 1
    # surface id out of range
    srf = I.flat_plane(2)
    srf.tri_surface = np.array([1, 7], np.uint8)
    assert L.sf_create(C.byref(_desc(sf, srf, keep)), C.byref(p), None, C.byref(h)) == 1
    # non-finite road data
    nan = I.flat_plane(2)
    nan.tri_verts = nan.tri_verts.copy()
    nan.tri_verts[0, 0, 0] = np.nan
    assert L.sf_create(C.byref(_desc(sf, nan, keep)), C.byref(p), None, C.byref(h)) == 1
    # bad vehicle parameter
    p2 = sf.make_params(dict(I.VEHICLE_DEFAULTS, mass=-1.0))
    assert L.sf_create(C.byref(d), C.byref(p2), None, C.byref(h)) == 1
    assert not h.value


def test_calls_on_null_handle(L):
    assert L.sf_step(None, None, C.c_float(0.1), 1) == 1
    assert L.sf_reset(None, None) == 1
    assert L.sf_observe(None, None, None, None, None) == 1
    assert L.sf_destroy(None) == 1
    assert L.sf_state_bytes(None) == 0
    for name in ("sf_sur_log", "sf_sur_enable"):
        assert getattr(L, name)(None, 0) == 1
    assert L.sf_sur_counts(None, None, 0) == 1
    assert L.sf_sur_set(None, None, None, None) == 1
    assert L.sf_get_tuning(None, None) == 1 and L.sf_set_tuning(None, None) == 1
    assert L.sf_autotune(None, C.c_float(0.1), 1, 1, None, None) == 1


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the ABI structs have the C compiler's sizes and
    field offsets (a C program built from include/sf.h prints them)."""
    import shutil
    import subprocess
    from paper_2605_08528_amd import sf
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"sf_vehicle_params": sf.VehicleParams, "sf_world_desc": sf.WorldDesc,
               "sf_options": sf.Options, "sf_sur_train_opts": sf.SurTrainOpts, "sf_tuning": sf.Tuning}
    header_fields = {
        "sf_vehicle_params": ["mass", "inertia", "wheel_radius", "mount", "jacobi_iters", "slop"],
        "sf_world_desc": ["num_worlds", "agent_offsets", "num_surfaces", "spawn", "seed"],
        "sf_options": ["stream", "alloc", "max_episode_steps", "flags", "tri_cell", "step_grid", "reserved"],
        "sf_sur_train_opts": ["steps", "batch", "lr", "eps", "seed", "init_seed", "set_envelope"],
        "sf_tuning": ["step_block", "step_grid", "obs_waves", "policy_rows", "step_us", "policy_us", "grid_cell",
                      "tri_cell"],
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sf.h"', "int main(void) {"]
    for s, fields in header_fields.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fields:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for s, cls in structs.items():
        assert int(got[s]) == C.sizeof(cls), s
        for f in header_fields[s]:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)
