"""GPU parity of the dynamic load balancing (section 5.4, Alg. 6 with the
bridge test of Alg. 7) against the oracle.

The carried worker sets are an input of a step; every case hands the same
sets to both sides and compares the sets the step produces bit for bit, then
the rest of the step (replica tables, weights, velocities) as every other
parity test does.  Start states and sets come from the scene or from oracle
runs (oracle.run_lb); no oracle input is read back from the library.  The
graph-replay test checks replayed steps against eager GPU steps, then one step
against the oracle from the oracle's own run of the same length.

Cases: the Figure 9 scenarios on hand-placed spheres, including the chain at
growth depths 0 to 3 and an isolated collision over two steps; a settling bowl
from the naive start at depths 0 and 2 (scenes kept in LDS); a bowl larger
than the LDS limit (scene kept in global memory); several scenes at once; the
graph-replayed step against the eager one.
"""
import numpy as np
import pytest

import oracle
import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes
from parity import compare_step, log, next_start

pytestmark = pytest.mark.gpu

R = 0.5
STEP = 0.98
FAR = [100.0, 110.0, 120.0, 130.0, 140.0, 150.0]


def _world(sc, **pkw):
    p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, **pkw)
    w = ovl.World(sc, p)
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=max(sc.halo_k, 1), beta=sc.beta)
    return w, p


def _line(xs, owner, n_parts):
    return scenes.custom_spheres([[x, 0.0, 5.0] for x in xs], R, 1.0, owner=np.asarray(owner, np.int32),
                                 n_parts=n_parts, dt=1 / 60.0, iters=10)


FIG9 = [
    # (label, xs, owner, n_parts, sets, depth)
    ("i lighter side", [0.0, STEP] + FAR[:2], [0, 1, 0, 0], 2, [1, 2, 1, 1], 0),
    ("i tie", [0.0, STEP], [0, 1], 2, [1, 2], 0),
    ("ii depth 0", [i * STEP for i in range(5)], [0, 1, 1, 1, 1], 2, [1, 2, 2, 2, 2], 0),
    ("ii depth 1", [i * STEP for i in range(5)], [0, 1, 1, 1, 1], 2, [1, 2, 2, 2, 2], 1),
    ("ii depth 2", [i * STEP for i in range(5)], [0, 1, 1, 1, 1], 2, [1, 2, 2, 2, 2], 2),
    ("ii depth 3", [i * STEP for i in range(5)], [0, 1, 1, 1, 1], 2, [1, 2, 2, 2, 2], 3),
    ("iii", [0.0, STEP] + FAR[:1], [0, 0, 1], 2, [3, 1, 2], 0),
    ("iii mirror", [0.0, STEP] + FAR[:1], [0, 0, 1], 2, [1, 3, 2], 0),
    ("iv bridge", [0.0, STEP, 2 * STEP], [0, 0, 1], 2, [1, 3, 2], 0),
    ("v", [0.0, STEP] + FAR[:4], [0, 0, 0, 0, 0, 1], 2, [3, 3, 1, 1, 1, 2], 0),
    ("v three workers", [0.0, STEP] + FAR[:3], [1, 1, 0, 0, 0], 3, [6, 6, 1, 1, 1], 0),
    ("key order", [0.0, 20.0, STEP, 20.0 + STEP], [0, 0, 1, 1], 2, [1, 1, 2, 2], 0),
    ("set load is a sum", [0.0, STEP] + FAR[:3], [0, 2, 0, 1, 2], 3, [3, 4, 1, 2, 4], 0),
]


@pytest.mark.parametrize("case", FIG9, ids=[c[0] for c in FIG9])
def test_figure9_scenarios(case):
    label, xs, owner, n_parts, sets, depth = case
    sc = _line(xs, owner, n_parts)
    w, p = _world(sc)
    sets = np.asarray(sets, np.uint64)
    w.set_load_balance(True, depth, sets=sets)
    _, o = compare_step(sc, w, p, label=f"fig 9 {label}", lb=dict(sets=sets, depth=depth))
    log(f"  sets {sets.tolist()} -> {o['mask'].tolist()}")


def test_isolated_collision_over_two_steps():
    """(i) in the first step, (iii) in the second: the library carries its own sets."""
    sc = _line([0.0, STEP], [0, 1], 2)
    w, p = _world(sc)
    w.set_load_balance(True, 0)
    _, o1 = compare_step(sc, w, p, label="(i)", lb=dict(sets=[1, 2], depth=0))
    assert o1["mask"].tolist() == [1, 3]
    _, o2 = compare_step(sc, w, p, start=next_start(o1), label="(iii)",
                         lb=dict(sets=o1["mask"], depth=0, carried=True))
    assert o2["mask"].tolist() == [1, 1]


def _oracle_start(sc, steps, depth):
    """State and sets after `steps` oracle steps from the naive start."""
    st, out, _ = oracle.run_lb(sc, steps, depth, dt=sc.dt, max_iters=sc.iters, beta=sc.beta)
    return st, out["mask"].astype(np.uint64), out


@pytest.mark.parametrize("depth", [0, 2])
def test_bowl_from_oracle_state(depth):
    sc = scenes.bowl_naive(1200, 3, 5, squeeze=0.35)
    st, sets, o_prev = _oracle_start(sc, 4, depth)
    w, p = _world(sc)
    _, o = compare_step(sc, w, p, start=(st, o_prev), label=f"bowl 1200 depth {depth}", lb=dict(sets=sets, depth=depth))
    changed = int((o["mask"] != sets).sum())
    log(f"  sets changed on {changed} bodies, overlap {o['n_overlap']}")
    assert changed > 0


def test_bowl_naive_start_first_step():
    sc = scenes.bowl_naive(1200, 4, 6, squeeze=0.35)
    w, p = _world(sc)
    sets = oracle.initial_masks(sc)
    w.set_load_balance(True, 1)
    _, o = compare_step(sc, w, p, label="bowl naive first step", lb=dict(sets=sets, depth=1))
    assert int((o["mask"] != sets).sum()) > 0


def test_scene_beyond_lds_limit():
    """A scene kept in global memory.  Its replicas exceed the initial replica
    capacity, so the step also grows the per-step buffers and runs again; the
    warm-start cache written beforehand must survive that."""
    sc = scenes.bowl_naive(13000, 5, 7, squeeze=0.35)
    assert sc.n_bodies > 12288
    st, sets, o_prev = _oracle_start(sc, 2, 1)
    w, p = _world(sc)
    _, o = compare_step(sc, w, p, start=(st, o_prev), label="bowl 13000 (global memory)", lb=dict(sets=sets, depth=1))
    assert int((o["mask"] != sets).sum()) > 0


def test_several_scenes():
    parts = [scenes.bowl_naive(n, 10 + i, k, squeeze=0.35) for i, (n, k) in enumerate([(300, 2), (700, 5), (450, 3)])]
    sc = scenes.concat_scenes(parts, halo_k=0, beta=4, dt=1 / 60, iters=30)
    w, p = _world(sc)
    sets = oracle.initial_masks(sc)
    w.set_load_balance(True, 0)
    _, o = compare_step(sc, w, p, label="three bowls", lb=dict(sets=sets, depth=0))
    # the next step with the sets the library carried from this one
    _, o2 = compare_step(sc, w, p, start=next_start(o), label="three bowls, carried",
                         lb=dict(sets=o["mask"].astype(np.uint64), depth=0, carried=True))


def test_trajectory_and_graph_replay():
    """60 steps from the naive start, eager and graph-replayed: the same bits;
    then one step against the oracle from the run's state and sets."""
    sc = scenes.bowl_naive(1500, 6, 7, squeeze=0.35)
    out = []
    for graph in (0, 1):
        w, p = _world(sc)
        cfg = w.get_launch()
        cfg["graph"] = graph
        w.set_launch(**cfg)
        w.set_load_balance(True, 0)
        for _ in range(3):
            w.step(20)
        out.append((w.read_state(), w.debug("mask").astype(np.uint64), w))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    st, sets, w = out[0]
    assert (sets != 0).all()
    load = [int(((sets >> np.uint64(b)) & np.uint64(1)).sum()) for b in range(7)]
    log(f"  bodies per worker after 60 steps {load}")
    # one step against the oracle from the oracle's own 60-step run
    ost, oout, _ = oracle.run_lb(sc, 60, 0, dt=sc.dt, max_iters=sc.iters, beta=sc.beta)
    compare_step(sc, w, p, start=(ost, oout), label="bowl 1500 t=61",
                 lb=dict(sets=oout["mask"].astype(np.uint64), depth=0))
