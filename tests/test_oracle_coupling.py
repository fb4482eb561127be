"""Pins of the oracle's interface coupling (section 7's proposal: the previous
step's constraint impulses couple the partitions beyond the overlap).

The cut constraint of a partition is one whose two dynamic bodies are not
both active in it; with coupling on, its impulse of the previous step (from
the cache of the lowest partition active in both bodies) acts on the body
inside the partition.  The pins fix it by physics, not by its own formula:

* a resting stack split between two partitions: the upper partition lacks
  the support of its lowest body.  Given the support's static impulse (the
  weight above it over one step, m g h per body) the upper partition's stack
  stays at rest, where without coupling it falls freely.  Contacts and ball
  joints each pin the sign of their impulse this way; the same cache entry
  stored under the other partition does nothing (the source is the lowest
  partition active in both bodies);
* one free body in zero gravity with no sweeps: the impulse F at lever r
  changes the linear momentum by F and the angular momentum about the
  centre by r x F (checked with the inertia tensor, not its inverse, on a
  turned capsule), and a contact's cached friction is projected on the
  tangent plane, a negative normal impulse pushes nothing;
* nothing is cut in a single partition: coupling changes nothing.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2403_17261_amd import scenes

G = 9.81
H = 1.0 / 60.0


def _quat_mat(q):
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _cache(entries):
    """entries: (partition, kind, key, (v0, v1, v2, v3)); sorted as the cache is."""
    entries = sorted(entries, key=lambda e: (e[0], e[1], e[2]))
    return dict(cache_part=np.array([e[0] for e in entries], np.int32),
                cache_kind=np.array([e[1] for e in entries], np.int32),
                cache_key=np.array([e[2] for e in entries], np.uint64),
                cache_val=np.array([e[3] for e in entries], np.float32).reshape(-1, 4))


def _rep(o, body, part):
    lo, hi = o["part_rep_off"][part], o["part_rep_off"][part + 1]
    idx = [r for r in range(lo, hi) if o["rep_body"][r] == body]
    assert len(idx) == 1
    return idx[0]


def _stack(joints):
    """Four unit spheres (r 0.5, m 1) stacked on the ground, owners 0 0 1 1."""
    pos = [[0.0, 0.0, 0.5 + k] for k in range(4)]
    kw = {}
    if joints:
        kw = dict(joint_ab=[[0, 1], [1, 2], [2, 3]], joint_anchor=[[0, 0, 0.5, 0, 0, -0.5]] * 3)
    return scenes.custom_spheres(pos, 0.5, 1.0, planes=[[0.0, 0.0, 1.0, 0.0]], owner=[0, 0, 1, 1], n_parts=2,
                                 dt=H, iters=20, halo_k=1, beta=4, **kw)


def _run(sc, cache, coupling, **kw):
    args = dict(halo_k=1, warmstart=False, adaptive=True, tol=1e-10, max_iters=5000, erp=0.2)
    args.update(kw)
    return oracle.step(sc, cache=cache, coupling=coupling, **args)


def test_stack_of_contacts_rests_with_its_cut_support():
    sc = _stack(joints=False)
    keys = [int(k) for k in oracle.step(sc, halo_k=1)["contact_key"]]
    k01 = [k for k in keys if k >> 32 == 0 and (k >> 1) & 0x7FFFFFFF == 1][0]
    k23 = [k for k in keys if k >> 32 == 2 and (k >> 1) & 0x7FFFFFFF == 3][0]
    # the weight above each cut contact over one step; the contact (0,1) is
    # solved in partition 0 only, (2,3) in partition 1 only
    cache = _cache([(0, 1, k01, (3 * G * H, 0, 0, 0)), (1, 1, k23, (G * H, 0, 0, 0))])
    o = _run(sc, cache, True)
    m = o["mask"]
    assert list(m) == [1, 3, 3, 2]
    assert np.allclose(o["rep_cpl"][_rep(o, 1, 1)], [0, 0, 3 * G * H, 0, 0, 0], atol=1e-6)
    assert np.allclose(o["rep_cpl"][_rep(o, 2, 0)], [0, 0, -G * H, 0, 0, 0], atol=1e-6)
    # every replica, and so every body, stays at rest
    assert np.abs(o["rep_state"][:, 7:13]).max() < 1e-7
    assert np.abs(o["state"][:, 7:13]).max() < 1e-7
    # without coupling the upper partition's three bodies fall freely
    f = _run(sc, cache, False)
    for b in (1, 2, 3):
        assert f["rep_state"][_rep(f, b, 1), 9] == pytest.approx(-G * H, rel=1e-6)
    assert np.abs(f["rep_cpl"]).max() == 0.0


def test_cut_impulse_comes_from_the_lowest_partition_in_both_bodies():
    sc = _stack(joints=False)
    keys = [int(k) for k in oracle.step(sc, halo_k=1)["contact_key"]]
    k01 = [k for k in keys if k >> 32 == 0 and (k >> 1) & 0x7FFFFFFF == 1][0]
    # the entry stored under partition 1, which is not active in body 0
    o = _run(sc, _cache([(1, 1, k01, (3 * G * H, 0, 0, 0))]), True)
    assert np.abs(o["rep_cpl"]).max() == 0.0
    assert o["rep_state"][_rep(o, 1, 1), 9] == pytest.approx(-G * H, rel=1e-6)


def test_stack_of_ball_joints_rests_with_its_cut_support():
    sc = _stack(joints=True)
    # ball-joint rows point along -e_k, so body b of a joint receives -lambda:
    # holding up the weight above it takes lambda_z = -(that weight)
    cache = _cache([(0, 0, 0, (0, 0, -3 * G * H, 0)), (1, 0, 2, (0, 0, -G * H, 0))])
    o = _run(sc, cache, True)
    assert list(o["mask"]) == [1, 3, 3, 2]
    assert np.abs(o["rep_state"][:, 7:13]).max() < 1e-7
    f = _run(sc, cache, False)
    assert f["rep_state"][_rep(f, 3, 1), 9] == pytest.approx(-G * H, rel=1e-6)


def test_joint_impulse_on_a_turned_capsule_is_a_rigid_body_impulse():
    # chain 0-1-2-3 along x in zero gravity; body 1 is a capsule turned about
    # (1, 1, 1) / sqrt 3 by 50 degrees; the joint (0, 1) is cut from partition 1
    ang = math.radians(50.0)
    ax = np.ones(3) / math.sqrt(3.0)
    q1 = [math.cos(ang / 2)] + list(math.sin(ang / 2) * ax)
    quat = [[1, 0, 0, 0], q1, [1, 0, 0, 0], [1, 0, 0, 0]]
    pos = [[0.0, 0, 5], [3.0, 0, 5], [6.0, 0, 5], [9.0, 0, 5]]
    anchors = [[1.5, 0, 0, 0.2, -0.3, 0.4], [1.5, 0, 0, -1.5, 0, 0], [1.5, 0, 0, -1.5, 0, 0]]
    sc = scenes.custom_spheres(pos, 0.5, 1.0, quat=quat, halflen=[0, 0.6, 0, 0], joint_ab=[[0, 1], [1, 2], [2, 3]],
                               joint_anchor=anchors, owner=[0, 0, 1, 1], n_parts=2, dt=H, iters=0, halo_k=1,
                               beta=4)
    lam = np.array([0.7, -1.1, 0.4], np.float32).astype(np.float64)   # the cache holds float32
    o = _run(sc, _cache([(0, 0, 0, tuple(lam) + (0.0,))]), True, gravity=(0.0, 0.0, 0.0), adaptive=False,
             forced_iters=np.array([0, 0], np.int32))
    r = _rep(o, 1, 1)
    v, w = o["rep_state"][r, 7:10], o["rep_state"][r, 10:13]
    F = -lam                                   # body b of the joint
    R1 = _quat_mat(np.array(q1, np.float32).astype(np.float64))
    lever = R1 @ np.array([0.2, -0.3, 0.4])
    I_world = R1 @ np.diag(sc.inertia[1].astype(np.float64)) @ R1.T
    assert sc.mass[1] * v == pytest.approx(F, abs=1e-12)
    # the stored quaternion is float32 (|q| - 1 ~ 3e-8): rotations agree to ~1e-7
    assert I_world @ w == pytest.approx(np.cross(lever, F), abs=2e-7)
    # the other replicas of the chain feel nothing
    for b, p in [(2, 1), (3, 1), (0, 0), (1, 0), (2, 0)]:
        assert np.abs(o["rep_state"][_rep(o, b, p), 7:13]).max() == 0.0


@pytest.mark.parametrize("val, push", [
    ((2.0, 0.0, 0.3, 0.4), (2.0, 0.3, 0.4)),     # friction in the tangent plane, inside the box
    ((2.0, 5.0, 0.3, 0.4), (2.0, 0.3, 0.4)),     # its normal part is not friction
    ((-1.0, 0.0, 0.3, 0.4), (0.0, 0.0, 0.0)),    # a pulling normal impulse is no contact impulse
])
def test_contact_impulse_projection(val, push):
    # spheres touching along x: contact (0, 1) has n = +x and its point at x = 1
    pos = [[0.5, 0, 5], [1.5, 0, 5], [2.5, 0, 5], [3.5, 0, 5]]
    sc = scenes.custom_spheres(pos, 0.5, 1.0, owner=[0, 0, 1, 1], n_parts=2, dt=H, iters=0, halo_k=1, beta=4, mu=0.5)
    keys = [int(k) for k in oracle.step(sc, halo_k=1, gravity=(0.0, 0.0, 0.0))["contact_key"]]
    k01 = [k for k in keys if k >> 32 == 0 and (k >> 1) & 0x7FFFFFFF == 1][0]
    o = _run(sc, _cache([(0, 1, k01, val)]), True, gravity=(0.0, 0.0, 0.0), adaptive=False,
             forced_iters=np.array([0, 0], np.int32))
    r = _rep(o, 1, 1)
    P = np.array(push)
    lever = np.array([1.0, 0.0, 5.0]) - np.array(pos[1])
    I = sc.inertia[1].astype(np.float64)
    assert sc.mass[1] * o["rep_state"][r, 7:10] == pytest.approx(P, abs=1e-7)
    assert I * o["rep_state"][r, 10:13] == pytest.approx(np.cross(lever, P), abs=1e-7)


def test_single_partition_is_unchanged():
    sc = scenes.config1(0)
    o0 = oracle.step(sc)
    one = np.zeros(sc.n_bodies, np.int32)
    base = oracle.step(sc, owner=one, parts_per_scene=[1], cache=o0, warmstart=True)
    cpl = oracle.step(sc, owner=one, parts_per_scene=[1], cache=o0, warmstart=True, coupling=True)
    assert np.array_equal(base["state"], cpl["state"])
    assert np.abs(cpl["rep_cpl"]).max() == 0.0


def test_source_is_the_lowest_of_two_partitions_holding_the_pair():
    # six spheres touching along x, owners 0 0 1 1 2 2, 2-hop overlap: the
    # contact (3, 4) is solved in partitions 1 and 2 and cut from partition 0
    # (body 4 is not active there); the impulse stored under partition 1 acts
    pos = [[0.5 + k, 0, 5] for k in range(6)]
    sc = scenes.custom_spheres(pos, 0.5, 1.0, owner=[0, 0, 1, 1, 2, 2], n_parts=3, dt=H, iters=0, halo_k=2, beta=4,
                               mu=0.5)
    base = oracle.step(sc, halo_k=2, gravity=(0.0, 0.0, 0.0))
    assert [int(m) for m in base["mask"]] == [3, 3, 7, 7, 6, 6]
    k34 = [int(k) for k in base["contact_key"] if int(k) >> 32 == 3 and (int(k) >> 1) & 0x7FFFFFFF == 4][0]
    cache = _cache([(1, 1, k34, (2.0, 0, 0, 0)), (2, 1, k34, (5.0, 0, 0, 0))])
    o = _run(sc, cache, True, halo_k=2, gravity=(0.0, 0.0, 0.0), adaptive=False,
             forced_iters=np.array([0, 0, 0], np.int32))
    # body 3 is body a of the contact: the normal impulse 2 pushes it along -x
    v = o["rep_state"][_rep(o, 3, 0), 7:10]
    assert v == pytest.approx([-2.0, 0.0, 0.0], abs=1e-7)
    assert np.abs(o["rep_cpl"][_rep(o, 3, 1)]).max() == 0.0   # solved in partition 1: nothing cut there
