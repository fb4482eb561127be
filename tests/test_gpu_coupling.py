"""GPU parity of the interface coupling (previous-step impulses of cut
constraints, the coupling section 7 proposes) against the oracle.

Each case starts from a state and warm-start cache the oracle produced with
coupling on, written into the world; then whole steps are compared as in
every parity test, plus the coupling impulse of every replica (float32
against double, within 1e-5 of the largest).  Cases: jointed chains with
links displaced by up to 2 cm (ball joints cut at the halo's edge carry
impulses well above rounding), a sphere lattice on the ground (contacts with
friction), a squeezed pile of capsules (lever arms and the capsule inverse
inertia), dynamically balanced worker sets (depth 0 leaves many constraints
cut), and two chain scenes in one world (partition ids offset per scene).
"""
import numpy as np
import pytest

import oracle
import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes
from parity import compare_step, log, next_start, oracle_run

pytestmark = pytest.mark.gpu


def _world(sc, halo_k, **pkw):
    p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, coupling=ovl.COUPLING_PREV_IMPULSE, **pkw)
    w = ovl.World(sc, p)
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=halo_k, beta=sc.beta)
    return w, p


def _displaced(sc, seed):
    rng = np.random.default_rng(seed)
    st = sc.state.copy()
    st[:, :3] += rng.uniform(-0.02, 0.02, (sc.n_bodies, 3)).astype(np.float32)
    return st


def test_chains():
    sc = scenes.config3(0, n_chains=16, links=50)
    w, p = _world(sc, sc.halo_k)
    start = oracle_run(sc, p, 2, state=_displaced(sc, 7))
    for t in range(2):
        _, o = compare_step(sc, w, p, start=start, label=f"chains coupled step {t + 3}")
        start = next_start(o)
    assert (np.abs(o["rep_cpl"]).max(axis=1) > 0).sum() > 20 and np.abs(o["rep_cpl"]).max() > 1e-2


@pytest.mark.parametrize("halo_k", [1, 2])
def test_lattice_contacts(halo_k):
    blk = scenes.lattice_stack(8, 8, 6, seed=3, n_parts=6,
                               owner_fn=lambda x: scenes.kmeans_owner(x, 6, seed=1)[0])
    sc = scenes._assemble([blk], "lattice-384", halo_k=halo_k, beta=4, dt=1 / 60, iters=30)
    w, p = _world(sc, halo_k)
    start = oracle_run(sc, p, 2)
    for t in range(2):
        _, o = compare_step(sc, w, p, start=start, label=f"lattice k={halo_k} coupled step {t + 3}")
        start = next_start(o)
    assert (np.abs(o["rep_cpl"]).max(axis=1) > 0).sum() > 20


def test_capsule_pile():
    n, seed = 1200, 6
    sc = scenes.capsule_pile(n, seed, 4, scale=(n / 20000.0) ** (1 / 3))
    st = sc.state.copy()
    rng = np.random.default_rng(seed)
    st[:, :3] *= np.float32(0.4)
    st[:, 2] += np.float32(0.6)
    st[:, :3] += rng.normal(0, 0.05, st[:, :3].shape).astype(np.float32)
    w, p = _world(sc, 1)
    start = oracle_run(sc, p, 1, state=st, halo_k=1)
    _, o = compare_step(sc, w, p, start=start, halo_k=1, label="capsule pile coupled")
    caps = sc.shape[o["rep_body"]] == 1
    assert ((np.abs(o["rep_cpl"]).max(axis=1) > 0) & caps).sum() > 10


def test_with_load_balancing():
    sc = scenes.bowl_naive(1200, 3, 5, squeeze=0.35)
    st, out, _ = oracle.run_lb(sc, 4, 0, dt=sc.dt, max_iters=sc.iters, beta=sc.beta)
    sets = out["mask"].astype(np.uint64)
    w, p = _world(sc, 1)
    _, o = compare_step(sc, w, p, start=(st, out), label="bowl, balanced sets, coupled", lb=dict(sets=sets, depth=0))
    n = int((np.abs(o["rep_cpl"]).max(axis=1) > 0).sum())
    log(f"  coupled replicas {n}")
    assert n > 20


def test_several_scenes():
    parts = [scenes.config3(0, n_chains=4, links=40), scenes.config3(1, n_chains=6, links=30)]
    sc = scenes.concat_scenes(parts, halo_k=2, beta=4, dt=1 / 120, iters=40)
    w, p = _world(sc, 2)
    _, o = compare_step(sc, w, p, start=oracle_run(sc, p, 2, state=_displaced(sc, 8)), label="two chain scenes coupled")
    assert (np.abs(o["rep_cpl"]).max(axis=1) > 0).sum() > 10


def test_single_partition_unchanged():
    sc = scenes.config1(0)
    one = np.zeros(sc.n_bodies, np.int32)
    res = []
    for c in (ovl.COUPLING_NONE, ovl.COUPLING_PREV_IMPULSE):
        p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, coupling=c)
        w = ovl.World(sc, p)
        w.set_partitions(one, [1], halo_k=1, beta=4)
        w.step(3)
        res.append(w.read_state())
        if c:
            assert np.abs(w.debug("rep_cpl")).max() == 0.0
    assert np.array_equal(res[0], res[1])
