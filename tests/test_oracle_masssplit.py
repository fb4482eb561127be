"""Pins of the oracle's mass splitting at the interface (coupling mode 2).

Section 2 likens the blend to the mass splitting of [TBV12]: the workers
share a body's mass.  The variant makes the share explicit in every solve:
the replica of an overlap body in partition i carries w_i of its mass and of
its inertia, w_i being its blend weight.  The pins fix it by physics:

* a row of spheres resting on the ground, split between two partitions: the
  ground impulse of a replica is its share of the body's weight over one
  step, w_i m g h (closed form), where the unsplit solve gives m g h in
  every partition; with equal weights the share is 1/|W|; a replica of
  weight 0 (its partition reached by no geodesic search) keeps the whole
  body and so m g h;
* the blend of split replicas applies the sum of the partitions' impulses to
  the whole body.  Every constraint pushes its two bodies with equal and
  opposite impulses, so with gravity off and no statics one partitioned step
  conserves linear momentum (contacts with friction), and angular momentum
  about the origin where the constraint points coincide (exactly assembled
  ball joints, spheres and turned capsules, the latter pinning the scaled
  inertia tensor).  The same steps without splitting do not conserve them;
* a single partition has every weight 1: splitting changes nothing.
"""
import numpy as np
import pytest

import oracle
from paper_2403_17261_amd import scenes

G = 9.81
H = 1.0 / 60.0


def _run(sc, coupling, **kw):
    args = dict(halo_k=1, warmstart=False, adaptive=True, tol=1e-12, max_iters=5000)
    args.update(kw)
    return oracle.step(sc, coupling=coupling, **args)


def _ground_impulses(o):
    """{(partition, body): normal impulse of its ground contact}"""
    off, ro = o["part_copy_off"], o["part_rep_off"]
    out = {}
    for p in range(len(off) - 1):
        for m in range(off[p], off[p + 1]):
            if o["copy_ib"][m] < 0:
                out[(p, int(o["rep_body"][ro[p] + o["copy_ia"][m]]))] = float(o["copy_lambda"][m][0])
    return out


def _row(owner):
    """Four unit spheres (r 0.5, m 1) in a row on the ground, 1 cm apart."""
    pos = [[1.01 * k, 0.0, 0.5] for k in range(4)]
    return scenes.custom_spheres(pos, 0.5, 1.0, planes=[[0.0, 0.0, 1.0, 0.0]], owner=owner, n_parts=2,
                                 dt=H, iters=20, halo_k=1, beta=4)


def test_resting_row_shares_the_weight_by_blend_weight():
    sc = _row([0, 0, 1, 1])
    w = {(0, 0): 1.0, (0, 1): 2 / 3, (0, 2): 1 / 3, (1, 1): 1 / 3, (1, 2): 2 / 3, (1, 3): 1.0}
    split = _ground_impulses(_run(sc, 2))
    plain = _ground_impulses(_run(sc, 0))
    assert sorted(split) == sorted(w) == sorted(plain)
    for k, wk in w.items():
        assert split[k] == pytest.approx(wk * G * H, rel=1e-9, abs=1e-12)
        assert plain[k] == pytest.approx(G * H, rel=1e-9)
    # each body's shares add up to its weight over the step
    for b in range(4):
        assert sum(v for (p, bb), v in split.items() if bb == b) == pytest.approx(G * H, rel=1e-9)
    o = _run(sc, 2)
    np.testing.assert_allclose(o["state"][:, 7:13], 0.0, atol=1e-6)


def test_resting_row_equal_weights_share_evenly():
    sc = _row([0, 0, 1, 1])
    split = _ground_impulses(_run(sc, 2, equal_weights=True))
    for (p, b), v in split.items():
        share = 0.5 if b in (1, 2) else 1.0
        assert v == pytest.approx(share * G * H, rel=1e-9)


def test_replica_of_weight_zero_keeps_the_whole_body():
    # owners 0 0 0 1 with a 2-hop halo: partition 1 has no body of its own, so
    # no search reaches it and its replicas have weight 0
    sc = _row([0, 0, 0, 1])
    o = _run(sc, 2, halo_k=2)
    ro = o["part_rep_off"]
    assert np.all(o["rep_w"][ro[1]:ro[2]] == 0.0)
    np.testing.assert_array_equal(o["rep_invm"][ro[1]:ro[2]], 1.0)
    split = _ground_impulses(o)
    for v in split.values():
        assert v == pytest.approx(G * H, rel=1e-9)
    assert np.all(np.isfinite(o["state"]))


def _momenta(sc, state_in, state_out):
    """Linear momentum and angular momentum about the origin, with the
    inertia of the start of the step (the orientation the solve used)."""
    m = sc.mass.astype(np.float64)
    x = state_in[:, 0:3].astype(np.float64)
    v = state_out[:, 7:10].astype(np.float64)
    om = state_out[:, 10:13].astype(np.float64)
    P = (m[:, None] * v).sum(0)
    L = np.cross(x, m[:, None] * v).sum(0)
    for i in range(len(m)):
        q = state_in[i, 3:7].astype(np.float64)
        R = _quat_mat(q)
        Ib = np.diag(sc.inertia[i].astype(np.float64))
        L += R @ Ib @ R.T @ om[i]
    return P, L


def _quat_mat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _pile(seed):
    """A loose 3x3x3 pile of spheres with random velocities and spins, no
    gravity and no statics, in three x slabs."""
    rng = np.random.default_rng(seed)
    pos = [[0.98 * i, 0.98 * j, 0.98 * k] for i in range(3) for j in range(3) for k in range(3)]
    pos = np.asarray(pos) + rng.uniform(-0.005, 0.005, (27, 3))
    vel = rng.normal(0.0, 1.0, (27, 3))
    om = rng.normal(0.0, 2.0, (27, 3))
    owner = np.minimum((pos[:, 0] / 0.98 + 0.5).astype(int), 2)
    return scenes.custom_spheres(pos, 0.5, rng.uniform(0.5, 2.0, 27), vel=vel, omega=om, owner=owner, n_parts=3,
                                 mu=0.6, dt=H, iters=20, halo_k=1, beta=8)


def _chain(capsules, seed):
    """A straight chain of 12 bodies along z joined by ball joints at exactly
    coincident anchors, random velocities and spins, no gravity, no statics,
    four partitions of three bodies."""
    rng = np.random.default_rng(seed)
    r, hl = 0.125, (0.25 if capsules else 0.0)
    step = 2 * (r + hl)
    pos = [[0.0, 0.0, step * k] for k in range(12)]
    kw = {}
    if capsules:
        kw = dict(halflen=hl)
    sc = scenes.custom_spheres(pos, r, rng.uniform(0.5, 2.0, 12), vel=rng.normal(0, 1, (12, 3)),
                               omega=rng.normal(0, 3, (12, 3)), owner=np.arange(12) // 3, n_parts=4,
                               joint_ab=[[k, k + 1] for k in range(11)],
                               joint_anchor=[[0, 0, step / 2, 0, 0, -step / 2]] * 11, dt=H, iters=20,
                               halo_k=1, beta=8, **kw)
    return sc


def _conservation(sc, **kw):
    out = {}
    for cpl in (0, 2):
        o = _run(sc, cpl, gravity=(0.0, 0.0, 0.0), **kw)
        assert o["n_overlap"] > 0
        # every replica takes part in the blend (a replica of weight 0 would
        # keep the whole body and its partition's impulses would be lost)
        assert np.all(o["rep_w"] > 0.0)
        out[cpl] = _momenta(sc, sc.state, o["state"])
    P0, L0 = _momenta(sc, sc.state, sc.state)
    return P0, L0, out


@pytest.mark.parametrize("seed", [0, 1])
def test_split_pile_conserves_linear_momentum(seed):
    sc = _pile(seed)
    P0, _, out = _conservation(sc, halo_k=1, max_iters=30, adaptive=False)
    scale = float((sc.mass[:, None] * np.abs(sc.state[:, 7:10])).sum())
    np.testing.assert_allclose(out[2][0], P0, atol=2e-6 * scale)
    # the unsplit blend averages impulses where it should add them
    assert np.abs(out[0][0] - P0).max() > 100 * 2e-6 * scale


@pytest.mark.parametrize("capsules", [False, True])
def test_split_chain_conserves_linear_and_angular_momentum(capsules):
    sc = _chain(capsules, seed=3)
    P0, L0, out = _conservation(sc, halo_k=1, max_iters=40, adaptive=False)
    scale_p = float((sc.mass[:, None] * np.abs(sc.state[:, 7:10])).sum())
    scale_l = scale_p * float(np.abs(sc.state[:, 0:3]).max()) + float(
        (sc.inertia * np.abs(sc.state[:, 10:13])).sum())
    np.testing.assert_allclose(out[2][0], P0, atol=2e-6 * scale_p)
    np.testing.assert_allclose(out[2][1], L0, atol=2e-6 * scale_l)
    assert np.abs(out[0][1] - L0).max() > 100 * 2e-6 * scale_l


def test_turned_capsule_chain_conserves_angular_momentum():
    # the chain of capsules lies along x: body z axes turned by 90 degrees
    # about y, so the world inertia is not the body's diagonal
    sc = _chain(True, seed=4)
    c, s = np.cos(np.pi / 4), np.sin(np.pi / 4)
    st = sc.state.copy()
    st[:, 0], st[:, 2] = st[:, 2].copy(), 0.0
    st[:, 3:7] = np.array([c, 0.0, s, 0.0], np.float32)
    sc.state[:] = st
    P0, L0, out = _conservation(sc, halo_k=1, max_iters=40, adaptive=False)
    scale_p = float((sc.mass[:, None] * np.abs(st[:, 7:10])).sum())
    scale_l = scale_p * float(np.abs(st[:, 0:3]).max()) + float((sc.inertia * np.abs(st[:, 10:13])).sum())
    np.testing.assert_allclose(out[2][0], P0, atol=2e-6 * scale_p)
    np.testing.assert_allclose(out[2][1], L0, atol=2e-6 * scale_l)


def test_single_partition_is_unchanged_by_splitting():
    sc = _pile(5)
    sc.owner[:] = 0
    a = _run(sc, 0, parts_per_scene=[1], max_iters=20, adaptive=False)
    b = _run(sc, 2, parts_per_scene=[1], max_iters=20, adaptive=False)
    np.testing.assert_array_equal(a["state"], b["state"])
    np.testing.assert_array_equal(a["copy_lambda"], b["copy_lambda"])
