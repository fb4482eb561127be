"""The C-ABI library loads and exports every symbol that include/ovl.h declares.

No compute call is made here: only host-side argument validation that fails
before the library touches the device.
"""
import ctypes as C

import numpy as np
import pytest

import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes


def test_library_exports_every_header_symbol():
    L = ovl.lib()
    names = ovl.header_symbols()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version_string():
    assert "gfx950" in ovl.ovl_version()


def test_binding_names_match_the_header():
    for n in ["ovl_create_world", "ovl_set_partitions", "ovl_step", "ovl_read_state"]:
        assert n in ovl.header_symbols()
    assert callable(ovl.ovl_create_world)


def _desc_with(sc, **over):
    keep = []

    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a.ctypes.data if a.size else None

    d = ovl.ovl_world_desc()
    d.n_bodies, d.n_scenes, d.n_joints = sc.n_bodies, sc.n_scenes, int(sc.joint_ab.shape[0])
    for name, dt in [("scene", np.int32), ("shape", np.int32), ("radius", np.float32), ("halflen", np.float32),
                     ("mass", np.float32), ("inertia", np.float32), ("state", np.float32), ("mu", np.float32),
                     ("margin", np.float32), ("plane_off", np.int32), ("planes", np.float32), ("ssph_off", np.int32),
                     ("ssph", np.float32), ("joint_ab", np.int32), ("joint_anchor", np.float32)]:
        setattr(d, name, arr(over.get(name, getattr(sc, name)), dt))
    for k in ("n_bodies", "n_scenes", "n_joints"):
        if k in over:
            setattr(d, k, over[k])
    return d, keep


@pytest.mark.parametrize("what,over", [
    ("no scenes", dict(n_scenes=0)),
    ("negative bodies", dict(n_bodies=-1)),
    ("capsule without half-length", "capsule"),
    ("unknown shape", "shape2"),
    ("capsule inertia not symmetric about its axis", "cap_aniso"),
    ("anisotropic inertia", "aniso"),
    ("zero mass", "mass0"),
    ("nan state", "nan"),
    ("unsorted scenes", "unsorted"),
])
def test_create_world_rejects_bad_input_before_touching_the_device(what, over):
    sc = scenes.config1(0)
    if over == "capsule":
        over = dict(shape=np.r_[1, np.zeros(63)].astype(np.int32))
    elif over == "shape2":
        over = dict(shape=np.r_[2, np.zeros(63)].astype(np.int32))
    elif over == "cap_aniso":
        I = sc.inertia.copy()
        I[0, 1] *= 2
        over = dict(shape=np.r_[1, np.zeros(63)].astype(np.int32), halflen=np.r_[0.3, np.zeros(63)].astype(np.float32),
                    inertia=I)
    elif over == "aniso":
        I = sc.inertia.copy()
        I[3, 2] *= 2
        over = dict(inertia=I)
    elif over == "mass0":
        m = sc.mass.copy()
        m[5] = 0
        over = dict(mass=m)
    elif over == "nan":
        s = sc.state.copy()
        s[7, 8] = np.nan
        over = dict(state=s)
    elif over == "unsorted":
        sc = scenes.concat_scenes([scenes.config1(0), scenes.config1(1)])
        s = sc.scene.copy()
        s[0] = 1
        over = dict(scene=s)
    d, keep = _desc_with(sc, **over)
    p = ovl.make_params()
    h = C.c_void_p()
    st = ovl.lib().ovl_create_world(C.byref(d), C.byref(p), None, C.byref(h))
    assert st == ovl.ERR_INVALID_ARG, what
    assert not h.value
    assert ovl.lib().ovl_last_error(None).decode()


@pytest.mark.parametrize("field,val", [("dt", 0.0), ("erp", 1.5), ("max_iters", 0), ("mode", 7), ("cfm", -1.0),
                                       ("weights", 2), ("coupling", 3), ("coupling", -1)])
def test_create_world_rejects_bad_params(field, val):
    sc = scenes.config1(0)
    d, keep = _desc_with(sc)
    p = ovl.make_params()
    setattr(p, field, val)
    h = C.c_void_p()
    assert ovl.lib().ovl_create_world(C.byref(d), C.byref(p), None, C.byref(h)) == ovl.ERR_INVALID_ARG


def test_null_world_is_rejected():
    L = ovl.lib()
    assert L.ovl_step(None, 1, None, 0) == ovl.ERR_INVALID_ARG
    assert L.ovl_set_partitions(None, None, 0, None, 0, 1, 1) == ovl.ERR_INVALID_ARG
    assert L.ovl_read_state(None, None, 0, 0) == ovl.ERR_INVALID_ARG
    assert L.ovl_set_load_balance(None, 1, 0, None, 0) == ovl.ERR_INVALID_ARG
    L.ovl_destroy_world(None)


def test_launch_candidates_and_launch_validation():
    L = ovl.lib()
    cands = ovl.launch_candidates()
    assert len(cands) == L.ovl_launch_candidates(None, 0) == 8
    pairs = {(c["pgs_block"], c["pgs_lds_reps"]) for c in cands}
    assert pairs == {(1024, 4800), (512, 2400), (256, 1200), (256, 2400)}
    assert {c["persistent"] for c in cands} == {0, 1} and all(c["graph"] == 0 for c in cands)
    # every LDS tile (two float4 per replica, plus the kernel's static LDS) fits the 160 KiB of a CU
    for b, r in pairs:
        assert 2 * r * 16 + 1024 <= 160 * 1024
    cfg = ovl.ovl_launch_cfg(1024, 4800, 0, 0)
    assert L.ovl_set_launch(None, C.byref(cfg)) == ovl.ERR_INVALID_ARG
    assert L.ovl_get_launch(None, C.byref(cfg)) == ovl.ERR_INVALID_ARG
    assert L.ovl_autotune(None, 1, None, None, 0) == ovl.ERR_INVALID_ARG
