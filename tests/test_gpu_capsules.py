"""GPU parity of the capsule path (shape 1) against the oracle.

Contact lists and every integer structure bit for bit; contact geometry (normal,
gap, lever arms) within float rounding of the double-precision oracle;
velocities within the tolerances of tests/parity.py after one step.
"""
import math

import numpy as np
import pytest

import oracle
import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes
from parity import check_state, compare_step, log, next_start, oracle_kwargs, oracle_run

pytestmark = pytest.mark.gpu
G = 9.81
Q_AXIS_X = [0.5, 0.5, 0.5, 0.5]          # body z onto world x, exact in float


def _world(sc, **pkw):
    p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, **pkw)
    w = ovl.World(sc, p)
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
    return w, p


def _axes(state):
    q = state[:, 3:7].astype(np.float64)
    qw, qx, qy, qz = q.T
    return np.stack([2 * (qx * qz + qw * qy), 2 * (qy * qz - qw * qx), 1 - 2 * (qx * qx + qy * qy)], 1)


def _check_geometry(sc, s0, geom, o):
    """GPU (n, phi, l_a, l_b, s_a, t_b) against the oracle's normal, gap and lever arms."""
    keys = o["contact_key"].astype(np.int64)
    a = keys >> 32
    b = (keys >> 1) & 0x7FFFFFFF
    u = _axes(s0)
    n = geom[:, 0:3].astype(np.float64)
    ra = geom[:, 6:7] * u[a] + geom[:, 4:5] * n
    dyn = b < sc.n_bodies
    ub = np.zeros_like(ra)
    ub[dyn] = u[b[dyn]]
    rb = geom[:, 7:8] * ub - geom[:, 5:6] * n
    rb[~dyn & (b < sc.n_bodies + sc.planes.shape[0])] = 0.0
    en = np.abs(n - o["contact_n"]).max(initial=0)
    ep = np.abs(geom[:, 3] - o["contact_phi"]).max(initial=0)
    era = np.abs(ra - o["contact_ra"]).max(initial=0)
    erb = np.abs(rb[dyn] - o["contact_rb"][dyn]).max(initial=0)
    log(f"  geometry: max |dn| {en:.2e}, |dphi| {ep:.2e}, |dr_a| {era:.2e}, |dr_b| {erb:.2e}")
    assert en < 1e-5 and ep < 1e-5 and era < 1e-5 and erb < 1e-5


def _squeezed_pile(n, seed, parts, factor=0.4):
    sc = scenes.capsule_pile(n, seed, parts, scale=(n / 20000.0) ** (1 / 3))
    st = sc.state.copy()
    rng = np.random.default_rng(seed)
    st[:, :3] *= np.float32(factor)
    st[:, 2] += np.float32(0.6)
    st[:, :3] += rng.normal(0, 0.05, st[:, :3].shape).astype(np.float32)
    return sc, st


def test_capsule_pile_first_step():
    sc, st = _squeezed_pile(1500, 4, 4)
    w, p = _world(sc)
    s0 = st
    stats, o = compare_step(sc, w, p, start=(st, None), label="capsule pile squeezed")
    keys = o["contact_key"].astype(np.int64)
    caps = sc.shape == 1
    a, b = keys >> 32, (keys >> 1) & 0x7FFFFFFF
    dyn = b < sc.n_bodies
    n_cc = int((caps[a[dyn]] & caps[b[dyn]]).sum())
    log(f"  contacts {len(keys)}, capsule-capsule {n_cc}")
    assert n_cc > 100
    _check_geometry(sc, s0, w.debug("contact_geom"), o)


def test_capsule_pile_trajectory():
    sc = scenes.capsule_pile(2000, 5, 4, scale=(2000 / 20000.0) ** (1 / 3))
    w, p = _world(sc)
    _, o = compare_step(sc, w, p, label="capsule pile t=0")
    s, c = next_start(o)
    st, o = compare_step(sc, w, p, start=oracle_run(sc, p, 150, state=s, cache=c), label="capsule pile t=151")
    plane_caps = sum(1 for k in o["contact_key"].astype(np.int64)
                     if sc.n_bodies <= ((k >> 1) & 0x7FFFFFFF) < sc.n_bodies + sc.planes.shape[0] and
                     sc.shape[k >> 32] == 1)
    log(f"  capsule-plane contacts {plane_caps}")
    assert st["n_contacts"] > 500 and plane_caps > 50


def test_horizontal_capsule_rests_on_two_ends():
    h, m, r, hl = 1.0 / 60.0, 2.0, 0.25, 0.5
    sc = scenes.custom_spheres([[0, 0, r]], r, m, quat=[Q_AXIS_X], halflen=[hl], planes=scenes.GROUND, mu=0.5,
                               dt=h, iters=400)
    w, p = _world(sc, warmstart=ovl.WARM_NONE)
    w.step(1)
    lam = w.debug("copy_lambda")
    log(f"  lambda {lam.tolist()}")
    assert lam[:, 0] == pytest.approx([m * G * h / 2] * 2, rel=1e-4)
    assert np.abs(lam[:, 1:].sum(0)).max() < 1e-6
    assert np.abs(w.read_state()[0, 7:13]).max() < 1e-5


def test_capsule_chain_with_joints():
    """Capsules joined end to end by ball joints, draped over a static sphere:
    the capsule joint rows (full inertia) against the oracle."""
    n, r, hl = 24, 0.08, 0.2
    L = 2 * (hl + r)
    pos = [[(i - n / 2) * L, 0.0, 2.0] for i in range(n)]
    owner = (np.arange(n) * 3 // n).astype(np.int32)
    sc = scenes.custom_spheres(pos, r, 0.4, quat=[Q_AXIS_X] * n, halflen=[hl] * n, planes=scenes.GROUND,
                               ssph=[[0.3, 0.0, 1.2, 0.6]], joint_ab=[[i, i + 1] for i in range(n - 1)],
                               joint_anchor=[[0, 0, hl + r, 0, 0, -(hl + r)] for _ in range(n - 1)],
                               owner=owner, n_parts=3, halo_k=2, beta=4, dt=1 / 120.0, iters=40)
    w, p = _world(sc)
    _, o = compare_step(sc, w, p, label="capsule chain t=0")
    s, c = next_start(o)
    st, o = compare_step(sc, w, p, start=oracle_run(sc, p, 80, state=s, cache=c), label="capsule chain t=81")
    log(f"  joint violation {float(o['joint_violation']):.2e}")
    assert st["n_contacts"] > 0
