"""GPU parity of mass splitting at the interface (coupling mode 2: the replica
of an overlap body carries the share w_i of the body's mass and inertia)
against the oracle, and its conservation property at full size.

Parity cases start from oracle-made states and compare whole steps as every
parity test does: jointed chains with displaced links (ball-joint rows with
scaled inverse masses and inertias), a sphere lattice on the ground with one-
and two-hop halos (contacts with friction), a squeezed pile of capsules (the
scaled inverse inertia tensor), dynamically balanced worker sets, and two
scenes in one world.  Every launch configuration gives the same bits, the
global-memory variant of the split sweeps included.

At the size of the 100k tower (no ground, no gravity, random velocities, a
geodesic search deep enough that every replica has a weight) one step
conserves linear momentum to float rounding, which the unsplit step does
not: the blend of split replicas applies the sum of the partitions'
impulses, and every constraint's impulses are equal and opposite.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes
from parity import compare_step, log, next_start, oracle_run

pytestmark = pytest.mark.gpu


def _world(sc, halo_k, **pkw):
    p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, coupling=ovl.COUPLING_MASS_SPLIT, **pkw)
    w = ovl.World(sc, p)
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=halo_k, beta=sc.beta)
    return w, p


def _displaced(sc, seed):
    rng = np.random.default_rng(seed)
    st = sc.state.copy()
    st[:, :3] += rng.uniform(-0.02, 0.02, (sc.n_bodies, 3)).astype(np.float32)
    return st


def _split_replicas(o):
    """replicas whose share is below the whole body (weight in (0, 1))"""
    return int(((o["rep_w"] > 0.0) & (o["rep_w"] < 1.0)).sum())


def test_chains():
    sc = scenes.config3(0, n_chains=16, links=50)
    w, p = _world(sc, sc.halo_k)
    start = oracle_run(sc, p, 2, state=_displaced(sc, 7))
    for t in range(2):
        _, o = compare_step(sc, w, p, start=start, label=f"chains mass split step {t + 3}")
        start = next_start(o)
    assert _split_replicas(o) > 50


@pytest.mark.parametrize("halo_k", [1, 2])
def test_lattice_contacts(halo_k):
    blk = scenes.lattice_stack(8, 8, 6, seed=3, n_parts=6,
                               owner_fn=lambda x: scenes.kmeans_owner(x, 6, seed=1)[0])
    sc = scenes._assemble([blk], "lattice-384", halo_k=halo_k, beta=4, dt=1 / 60, iters=30)
    w, p = _world(sc, halo_k)
    start = oracle_run(sc, p, 2)
    for t in range(2):
        _, o = compare_step(sc, w, p, start=start, label=f"lattice k={halo_k} mass split step {t + 3}")
        start = next_start(o)
    assert _split_replicas(o) > 50


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
    _, o = compare_step(sc, w, p, start=start, halo_k=1, label="capsule pile mass split")
    caps = sc.shape[o["rep_body"]] == 1
    assert (caps & (o["rep_w"] > 0.0) & (o["rep_w"] < 1.0)).sum() > 10


def test_with_load_balancing():
    sc = scenes.bowl_naive(1200, 3, 5, squeeze=0.35)
    st, out, _ = oracle.run_lb(sc, 4, 0, dt=sc.dt, max_iters=sc.iters, beta=sc.beta)
    sets = out["mask"].astype(np.uint64)
    w, p = _world(sc, 1)
    _, o = compare_step(sc, w, p, start=(st, out), label="bowl, balanced sets, mass split", lb=dict(sets=sets, depth=0))
    log(f"  split replicas {_split_replicas(o)}")
    assert _split_replicas(o) > 20


def test_several_scenes():
    parts = [scenes.config3(0, n_chains=4, links=40), scenes.config3(1, n_chains=6, links=30)]
    sc = scenes.concat_scenes(parts, halo_k=2, beta=4, dt=1 / 120, iters=40)
    w, p = _world(sc, 2)
    _, o = compare_step(sc, w, p, start=oracle_run(sc, p, 2, state=_displaced(sc, 8)),
                        label="two chain scenes mass split")
    assert _split_replicas(o) > 10


def test_single_partition_unchanged():
    sc = scenes.config1(0)
    one = np.zeros(sc.n_bodies, np.int32)
    res = []
    for c in (ovl.COUPLING_NONE, ovl.COUPLING_MASS_SPLIT):
        p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, coupling=c)
        w = ovl.World(sc, p)
        w.set_partitions(one, [1], halo_k=1, beta=4)
        w.step(3)
        res.append(w.read_state())
    assert np.array_equal(res[0], res[1])


def test_tower_conserves_momentum_at_full_size():
    sc = scenes.config5(0)
    n = sc.n_bodies
    sc = dataclasses.replace(sc, planes=np.zeros((0, 4), np.float32),
                             plane_off=np.zeros_like(sc.plane_off))
    rng = np.random.default_rng(11)
    st = sc.state.copy()
    st[:, 7:10] = rng.normal(0.0, 0.5, (n, 3)).astype(np.float32)
    st[:, 10:13] = rng.normal(0.0, 1.0, (n, 3)).astype(np.float32)
    m = sc.mass.astype(np.float64)
    P0 = (m[:, None] * st[:, 7:10].astype(np.float64)).sum(0)
    scale = float((m[:, None] * np.abs(st[:, 7:10].astype(np.float64))).sum())
    err = {}
    for c in (ovl.COUPLING_NONE, ovl.COUPLING_MASS_SPLIT):
        p = ovl.make_params(dt=sc.dt, gravity=(0.0, 0.0, 0.0), max_iters=30, coupling=c)
        w = ovl.World(sc, p)
        w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=2, beta=16)
        w.write_state(st, keep_cache=False)
        st1 = w.step(1, stats=True)
        out = w.read_state().astype(np.float64)
        wts = w.debug("rep_w")
        assert np.all(wts > 0.0), "a replica without weight would keep the whole body"
        assert np.isfinite(out).all()
        P = (m[:, None] * out[:, 7:10]).sum(0)
        err[c] = float(np.abs(P - P0).max()) / scale
        log(f"  tower 100k coupling {c}: contacts {st1['n_contacts']}, split replicas "
            f"{int(((wts > 0) & (wts < 1)).sum())}, |dP| / sum m|v| = {err[c]:.2e}")
    # float32 rounding of 30 sweeps over 1.2M copies stays far below 1e-7 of
    # the momentum scale; without splitting the blend loses 1e-4 of it
    assert err[ovl.COUPLING_MASS_SPLIT] < 1e-7
    assert err[ovl.COUPLING_NONE] > 100 * 1e-7


def test_every_launch_configuration_gives_the_same_bits():
    # chains in four slabs: partitions above the 1200- and 2400-replica LDS
    # tiles, so the global-memory variant of the split sweeps takes part
    sc = scenes.config3(0, n_chains=64, links=200)
    owner = (sc.owner // 4).astype(np.int32)
    pps = np.array([4], np.int32)
    ref = None
    for c in ovl.launch_candidates():
        for graph in (0, 1):
            p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, coupling=ovl.COUPLING_MASS_SPLIT)
            w = ovl.World(sc, p)
            w.set_partitions(owner, pps, halo_k=3, beta=sc.beta)
            w.set_launch(**dict(c, graph=graph))
            w.step(20)
            st = w.read_state()
            if ref is None:
                ref = st
                big = int(np.diff(w.debug("part_rep_off").astype(np.int64)).max())
                log(f"  {sc.n_bodies} bodies in 4 partitions, largest {big} replicas")
                assert big > 2400
            assert np.array_equal(st, ref), (c, graph)
            w.close()
