"""Pins of the oracle's dynamic load balancing (section 5.4, Alg. 6 with the
bridge test of Alg. 7) against the scenarios of Figure 9, worked by hand.

Each case places a few unit spheres on a line so that exactly the listed pairs
touch, gives every body a worker set, and reads the worker sets the oracle
hands to the rest of the step.  Every contact of the step between two dynamic
bodies is taken, in key order (Alg. 1 hands the step's contact list to Alg. 6,
and the text has an isolated collision of one step become scenario (iii) in
the next).  The expected sets follow from the text of section 5.4 and from the
readings the oracle states (load of a set of workers = the number of bodies
active in it, summed over its workers; ties go to A's side and to the lowest
worker index; the BFS of the growth step includes its root):

* (i)   inter-worker collision in isolation: the lighter side's workers are
        activated on the other body, nothing is taken away;
* (ii)  the same with a body already touching others: growth to depth gamma,
        then the remaining contacts of the chain, depths 0 to 3;
* (iii) an overlap body hit by a single-worker body with no other neighbour
        drops its other workers;
* (iv)  the same when the overlap body bridges two workers: nothing changes;
* (v)   two overlap bodies with the same workers keep only the least loaded;
* (i) followed by (iii) in the next step: the body ends in one worker;
* contacts are taken in key order and loads change as they are taken;
* statics never take part.
"""
import numpy as np
import pytest

import oracle
from paper_2403_17261_amd import scenes

R = 0.5
STEP = 0.98          # centre spacing of touching spheres (2 R minus a small overlap)


def _key(a, b):
    a, b = min(a, b), max(a, b)
    return np.uint64((a << 32) | (b << 1))


def _scene(xs, owner, n_parts, planes=None):
    pos = [[x, 0.0, 5.0] for x in xs]
    return scenes.custom_spheres(pos, R, 1.0, owner=np.asarray(owner, np.int32), n_parts=n_parts, planes=planes,
                                 dt=1 / 60.0, iters=10)


def _masks(sc, masks, depth=0, state=None):
    out = oracle.step(sc, state=state, lb_masks=np.asarray(masks, np.uint64), lb_depth=depth)
    return [int(m) for m in out["mask"]], out


def _touching(out):
    k = out["contact_key"].astype(np.int64)
    return sorted((int(a), int(b)) for a, b in zip(k >> 32, (k >> 1) & 0x7FFFFFFF))


# body layout used below: touching clusters near x = 0, lone bodies far away
FAR = [100.0, 110.0, 120.0, 130.0, 140.0, 150.0]


def test_scenario_i_lighter_side_is_activated_on_the_other_body():
    # A = 0 (worker 0), B = 1 (worker 1); worker 0 holds two more lone bodies
    sc = _scene([0.0, STEP] + FAR[:2], [0, 1, 0, 0], 2)
    m, out = _masks(sc, [1, 2, 1, 1])
    assert _touching(out) == [(0, 1)]
    # <W_A> = 3 > <W_B> = 1: worker 1 is activated on A, B keeps its set
    assert m == [0b11, 0b10, 1, 1]
    # loads swapped: worker 0 is activated on B
    sc = _scene([0.0, STEP] + FAR[:2], [0, 1, 1, 1], 2)
    m, _ = _masks(sc, [1, 2, 2, 2])
    assert m == [0b01, 0b11, 2, 2]
    # a tie goes to A's side (the test of line 5 is <=)
    sc = _scene([0.0, STEP], [0, 1], 2)
    m, _ = _masks(sc, [1, 2])
    assert m == [0b01, 0b11]


def test_scenario_ii_growth_to_depth_gamma():
    # chain A(0) - B(1) - C(1) - D(1) - E(1), contacts (0,1), (1,2), (2,3), (3,4)
    xs = [i * STEP for i in range(5)]
    own = [0, 1, 1, 1, 1]
    sc = _scene(xs, own, 2)
    expect = {
        # (0,1): B enters worker 0; (1,2): B bridges A and C, kept; the rest single-worker
        0: [0b01, 0b11, 0b10, 0b10, 0b10],
        # (0,1): A, B, C in both (loads 3 : 5); (1,2): B, C keep worker 0 (3 : 3);
        # (2,3): tie, D enters worker 0 and C, D, E grow to both (5 : 4); (3,4): D, E keep worker 1
        1: [0b11, 0b01, 0b11, 0b10, 0b10],
        # (0,1): A..D in both (4 : 5); (1,2): B, C keep worker 0 (4 : 3); (2,3), (3,4): D bridges
        2: [0b11, 0b01, 0b01, 0b11, 0b10],
        # (0,1): all in both (5 : 5); (1,2): tie, B, C keep worker 0 (5 : 3); (2,3): D bridges;
        # (3,4): D, E keep worker 1
        3: [0b11, 0b01, 0b01, 0b10, 0b10],
    }
    for depth, want in expect.items():
        m, out = _masks(sc, [1 << o for o in own], depth=depth)
        assert _touching(out) == [(0, 1), (1, 2), (2, 3), (3, 4)]
        assert m == want, depth


def test_scenario_iii_overlap_body_without_other_neighbours_leaves():
    # B = 0 in both workers, A = 1 in worker 0 only, touching only each other
    sc = _scene([0.0, STEP] + FAR[:1], [0, 0, 1], 2)
    m, _ = _masks(sc, [0b11, 0b01, 0b10])
    assert m == [0b01, 0b01, 0b10]
    # the mirror case (the overlap body second in the pair, lines 18-19)
    m, _ = _masks(sc, [0b01, 0b11, 0b10])
    assert m == [0b01, 0b01, 0b10]


def test_scenario_iv_bridge_body_is_kept():
    # A(0) - B(0,1) - C(1): B's neighbours span both workers, both contacts keep it
    sc = _scene([0.0, STEP, 2 * STEP], [0, 0, 1], 2)
    masks = [0b01, 0b11, 0b10]
    m, _ = _masks(sc, masks)
    assert m == masks
    # without C's contact B is no bridge and drops worker 1
    sc2 = _scene([0.0, STEP, 50.0], [0, 0, 1], 2)
    m, _ = _masks(sc2, masks)
    assert m == [0b01, 0b01, 0b10]


def test_scenario_v_two_overlap_bodies_keep_the_least_loaded_worker():
    # A, B both in workers {0, 1}; loads w0 = 2 + 3 lone, w1 = 2 + 1 lone
    sc = _scene([0.0, STEP] + FAR[:4], [0, 0, 0, 0, 0, 1], 2)
    m, _ = _masks(sc, [0b11, 0b11, 1, 1, 1, 2])
    assert m == [0b10, 0b10, 1, 1, 1, 2]
    # equal loads: the lowest worker index
    sc = _scene([0.0, STEP], [0, 1], 2)
    m, _ = _masks(sc, [0b11, 0b11])
    assert m == [0b01, 0b01]
    # three workers, both bodies in {1, 2}: worker 0 never comes into it
    sc = _scene([0.0, STEP] + FAR[:3], [1, 1, 0, 0, 0], 3)
    m, _ = _masks(sc, [0b110, 0b110, 1, 1, 1])
    assert m == [0b010, 0b010, 1, 1, 1]


def test_isolated_collision_becomes_scenario_iii_next_step():
    # step 1: (i), a tie, so worker 0 is activated on B; step 2: the same contact
    # is (iii) and B, touching nothing else, keeps only worker 0
    sc = _scene([0.0, STEP], [0, 1], 2)
    m1, o1 = _masks(sc, [1, 2])
    assert m1 == [0b01, 0b11]
    m2, o2 = _masks(sc, m1, state=o1["state"].astype(np.float32))
    assert _touching(o2) == [(0, 1)]
    assert m2 == [0b01, 0b01]


def test_contacts_are_taken_in_key_order_with_running_loads():
    # pairs (0, 2) and (1, 3): bodies 0, 1 in worker 0, bodies 2, 3 in worker 1
    sc = _scene([0.0, 20.0, STEP, 20.0 + STEP], [0, 0, 1, 1], 2)
    m, out = _masks(sc, [1, 1, 2, 2])
    assert _touching(out) == [(0, 2), (1, 3)]
    # (0, 2): tie 2 <= 2, worker 0 activated on body 2 (loads now 3 : 2);
    # (1, 3): 3 > 2, worker 1 activated on body 1
    assert m == [0b01, 0b11, 0b11, 0b10]


def test_load_of_a_worker_set_is_the_sum_over_its_workers():
    # A = 0 in {0, 1}, B = 1 in {2}; loads w0 = 2, w1 = 2, w2 = 3.
    # Sum: 4 > 3, so worker 2 is activated on A (a max or min reading would
    # activate workers 0 and 1 on B instead).
    sc = _scene([0.0, STEP] + FAR[:3], [0, 2, 0, 1, 2], 3)
    m, _ = _masks(sc, [0b011, 0b100, 0b001, 0b010, 0b100])
    assert m == [0b111, 0b100, 0b001, 0b010, 0b100]


def test_statics_take_no_part():
    # a sphere resting on the ground in worker 0, touching nothing else
    sc = _scene([0.0], [0], 2, planes=scenes.GROUND)
    sc.state[0, 2] = np.float32(R - 0.01)
    m, out = _masks(sc, [0b11])
    assert len(out["contact_key"]) == 1 and m == [0b11]


def test_rejects_empty_or_out_of_range_sets():
    sc = _scene([0.0, STEP], [0, 1], 2)
    with pytest.raises(RuntimeError):
        _masks(sc, [0, 2])
    with pytest.raises(RuntimeError):
        _masks(sc, [1, 4])


def test_several_steps_keep_sets_valid():
    """Over a settling pile the sets stay non-empty and within the scene's
    workers, every worker keeps bodies, and a body with no dynamic contact
    keeps its set."""
    sc = scenes.bowl_naive(300, 7, 4, squeeze=0.35)
    st, m = sc.state, oracle.initial_masks(sc)
    changed_steps = 0
    for t in range(12):
        out = oracle.step(sc, state=st, lb_masks=m, lb_depth=1)
        m2 = out["mask"].astype(np.uint64)
        assert (m2 != 0).all() and (m2 >> np.uint64(4) == 0).all()
        keys = out["contact_key"].astype(np.uint64)
        a = (keys >> np.uint64(32)).astype(np.int64)
        b = ((keys >> np.uint64(1)) & np.uint64(0x7FFFFFFF)).astype(np.int64)
        dyn = b < sc.n_bodies
        touched = np.zeros(sc.n_bodies, bool)
        touched[a[dyn]] = touched[b[dyn]] = True
        assert np.array_equal(m2[~touched], m[~touched])
        changed_steps += int((m2 != m).any())
        st, m = out["state"].astype(np.float32), m2
    load = [int(((m >> np.uint64(b)) & np.uint64(1)).sum()) for b in range(4)]
    assert min(load) > 0 and changed_steps > 0
