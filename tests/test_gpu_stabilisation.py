"""The GPU path against the closed forms of Eq. 2's stabilisation and of the
residual's velocity scale (the same cases as the oracle pins in
test_oracle_stabilisation.py), at float32 tolerances, and each case against
the oracle as every parity test does.

A sphere sunk d into the ground leaves a converged step rising at erp d / h; a
fast sphere over an open gap phi inside the margin lands at phi / h; a ball
joint whose anchors are C apart closes at -erp C / h (anchor of a relative to
b); one corrective sweep of size delta stops the adaptive sweeps at tolerance
1e-4 after one sweep for a heavy sphere and after two for a light one.
"""
import numpy as np
import pytest

import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes
from parity import compare_step

pytestmark = pytest.mark.gpu

G = 9.81
H = 1.0 / 60.0


def _world(sc, **kw):
    # fixed sweeps, enough for these one- and two-body problems to converge in float32
    kw.setdefault("max_iters", 100)
    kw.setdefault("mode", ovl.MODE_FIXED)
    p = ovl.make_params(dt=sc.dt, **kw)
    w = ovl.World(sc, p)
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
    return w, p


@pytest.mark.parametrize("erp", [0.2, 1.0])
def test_penetration_is_corrected_by_erp(erp):
    m, r, depth = 3.0, 0.5, 0.02
    sc = scenes.custom_spheres([[0.3, -0.2, r - depth]], r, m, planes=scenes.GROUND, mu=0.5, dt=H, iters=200)
    w, p = _world(sc, erp=erp)
    st, o = compare_step(sc, w, p, label=f"penetration erp {erp}")
    d = r - float(sc.state[0, 2])
    s = w.read_state()[0]
    assert s[9] == pytest.approx(erp * d / H, rel=1e-5)
    assert w.debug("copy_lambda")[0, 0] == pytest.approx(m * (G * H + erp * d / H), rel=1e-5)
    w.close()


def test_open_gap_closes_at_gap_over_h():
    m, r, gap, v = 2.0, 0.5, 0.012, 3.0
    sc = scenes.custom_spheres([[0, 0, r + gap]], r, m, vel=[[0, 0, -v]], planes=scenes.GROUND, mu=0.5, dt=H,
                               iters=200)
    w, p = _world(sc)
    st, o = compare_step(sc, w, p, label="open gap")
    phi = float(sc.state[0, 2]) - r
    s = w.read_state()[0]
    assert s[9] == pytest.approx(-phi / H, rel=1e-5)
    assert s[2] == pytest.approx(r, abs=1e-6)
    w.close()


@pytest.mark.parametrize("C", [(0.01, 0.0, 0.0), (-0.004, 0.007, 0.02)])
def test_joint_displacement_is_driven_back(C):
    ma, mb, r, erp = 1.0, 4.0, 0.5, 0.2
    aa, ab = np.array([0.5, 0.1, 0.0]), np.array([-0.5, 0.0, -0.1])
    xa = np.array([0.0, 0.0, 5.0])
    xb = xa + aa - ab - np.asarray(C)
    sc = scenes.custom_spheres([xa, xb], r, [ma, mb], mu=0.0, dt=H, iters=200, joint_ab=[[0, 1]],
                               joint_anchor=[np.concatenate([aa, ab])])
    w, p = _world(sc, erp=erp)
    st, o = compare_step(sc, w, p, label=f"joint C={C}")
    st0 = sc.state.astype(np.float64)
    Cs = (st0[0, :3] + sc.joint_anchor[0, :3]) - (st0[1, :3] + sc.joint_anchor[0, 3:])
    s = w.read_state().astype(np.float64)
    ua = s[0, 7:10] + np.cross(s[0, 10:13], sc.joint_anchor[0, :3].astype(np.float64))
    ub = s[1, 7:10] + np.cross(s[1, 10:13], sc.joint_anchor[0, 3:].astype(np.float64))
    assert np.allclose(ua - ub, -erp * Cs / H, rtol=1e-4, atol=2e-6)
    w.close()


@pytest.mark.parametrize("m,delta,sweeps", [(100.0, 1e-3, 1), (0.01, 1e-5, 2)])
def test_adaptive_stop_uses_velocity_units(m, delta, sweeps):
    """A resting sphere warm-started from m g h + delta: the first sweep moves the
    normal impulse by -delta, a residual of |delta| / m in m/s."""
    sc = scenes.custom_spheres([[0.0, 0.0, 0.5]], 0.5, m, planes=scenes.GROUND, mu=0.5, dt=H, iters=50)
    w, p = _world(sc, mode=ovl.MODE_ADAPTIVE, tol=1e-4, max_iters=50)
    w.step(1, stats=True)                               # a cache entry for the contact
    cache = w.cache()
    mm = float(sc.mass[0])
    cache["cache_val"][0] = [np.float32(mm * G * H + delta), 0.0, 0.0, 0.0]
    w.write_state(sc.state, keep_cache=False)
    w.write_cache(cache)
    w.step(1, stats=True)
    assert int(w.debug("part_iters")[0]) == sweeps
    assert w.debug("copy_lambda")[0, 0] == pytest.approx(mm * G * H, rel=1e-5)
    w.close()
