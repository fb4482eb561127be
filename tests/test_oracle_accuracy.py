"""Pins of the oracle's accuracy-study options against closed forms.

* equal blending weights (the naive choice of section 5.3): every overlap
  body gets 1/|W| per replica, and its blended position and velocities are
  the plain mean of its replicas';
* joint violation of the blended state (section 6 reports it for the
  bridges): the largest and the summed norm of C = (x_a + R_a a_a) -
  (x_b + R_b a_b) over the ball joints, on a configuration the step leaves
  unchanged (no gravity, no stabilisation, bodies at rest), including a body
  turned 90 degrees about z.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2403_17261_amd import scenes


def _weights(o):
    w = {}
    for r in range(len(o["rep_body"])):
        p = int(np.searchsorted(o["part_rep_off"], r, side="right") - 1)
        w[(int(o["rep_body"][r]), p)] = o["rep_w"][r]
    return w


def test_equal_weights_on_a_split_chain():
    sc = scenes.chain_line(10, 2, split=[0] * 5 + [1] * 5)
    geo = _weights(oracle.step(sc, halo_k=1))
    eq = _weights(oracle.step(sc, halo_k=1, equal_weights=True))
    assert geo[(4, 0)] == pytest.approx(2 / 3) and geo[(5, 1)] == pytest.approx(2 / 3)
    for b in (4, 5):
        assert eq[(b, 0)] == 0.5 and eq[(b, 1)] == 0.5
    for (b, p), v in eq.items():
        if b not in (4, 5):
            assert v == 1.0


def test_equal_weights_blend_is_the_replica_mean():
    sc = scenes.chain_line(12, 3, split=[0] * 4 + [1] * 4 + [2] * 4)
    o = oracle.step(sc, halo_k=2, equal_weights=True)
    rep = o["rep_state"]
    for v in range(sc.n_bodies):
        rows = np.nonzero(o["rep_body"] == v)[0]
        if len(rows) < 2:
            continue
        mean = rep[rows].mean(axis=0)
        assert np.allclose(o["state"][v, 0:3], mean[0:3], rtol=0, atol=1e-13)
        assert np.allclose(o["state"][v, 7:13], mean[7:13], rtol=0, atol=1e-13)


def test_joint_violation_closed_form():
    c, s = math.cos(math.pi / 4), math.sin(math.pi / 4)
    pos = [[0.0, 0.0, 5.0], [0.0, 0.7, 5.0], [10.0, 0.0, 5.0], [11.0, 0.0, 5.0]]
    quat = [[c, 0.0, 0.0, s], [1, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0]]
    # body 0 turned 90 degrees about z: its anchor (0.5, 0, 0) sits at (0, 0.5, 0)
    anchors = [[0.5, 0.0, 0.0, 0.0, -0.1, 0.0],       # C = (0, 0.5) - (0, 0.6): |C| = 0.1
               [0.5, 0.0, 0.0, -0.3, 0.0, 0.0]]       # C = 10.5 - 10.7:        |C| = 0.2
    sc = scenes.custom_spheres(pos, 0.5, 1.0, quat=quat, joint_ab=[[0, 1], [2, 3]], joint_anchor=anchors,
                               dt=1 / 60.0, iters=10)
    o = oracle.step(sc, gravity=(0.0, 0.0, 0.0), erp=0.0)
    assert len(o["contact_key"]) == 0
    assert np.abs(o["state"][:, 7:13]).max() < 1e-12
    assert o["joint_violation"] == pytest.approx(0.2, abs=1e-7)
    assert o["joint_violation_sum"] == pytest.approx(0.3, abs=1e-7)
