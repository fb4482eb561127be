"""GPU tests of the batched execution path: many uneven scenes in one world,
the launch configurations of the solve (block size, LDS tile, persistent
queue), HIP-graph replay and the autotuner.

Every configuration must compute the same bits, the graph must replay the
eager step exactly (checked over many replays with eager work in between),
and a batched world stepped through the graph must match the oracle.
"""
import numpy as np
import pytest

import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes
from parity import compare_step, log, oracle_run

pytestmark = pytest.mark.gpu


def _batched(n_scenes=16, seed=3, nmax=1200):
    return scenes.config4(seed, n_scenes=n_scenes, nmin=200, nmax=nmax)


def _uneven(sizes, seed):
    """Bowl scenes of the given (spheres, partitions): single-partition scenes of
    a few thousand spheres exceed the smaller LDS tiles."""
    parts = [scenes.bowl_scene(n, seed * 1000 + i, k, scale=(n / 20000.0) ** (1 / 3))
             for i, (n, k) in enumerate(sizes)]
    return scenes._assemble(parts, "uneven", halo_k=2, beta=4, dt=1 / 60, iters=30, steps=200)


def _world(sc, **launch):
    p = ovl.make_params(dt=sc.dt, max_iters=sc.iters)
    w = ovl.World(sc, p)
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
    if launch:
        w.set_launch(**launch)
    return w


def _largest_partition(w):
    off = w.debug("part_rep_off")
    return int(np.diff(off).max())


def test_every_launch_configuration_gives_the_same_bits():
    # scenes up to 3000 spheres: some partitions exceed the 1200- and 2400-replica LDS tiles,
    # so the global-memory variant takes part in those configurations
    sc = _uneven([(3000, 1), (1800, 1), (900, 2), (400, 3), (2500, 2), (250, 1), (1200, 6)], 3)
    ref = None
    for c in ovl.launch_candidates():
        for graph in (0, 1):
            w = _world(sc, **dict(c, graph=graph))
            w.step(90)
            st = w.read_state()
            if ref is None:
                ref = st
                big = _largest_partition(w)
                log(f"  {sc.n_bodies} bodies in {sc.n_scenes} scenes, {int(sc.parts_per_scene.sum())} partitions, "
                    f"largest {big} replicas")
                assert big > 2400
            assert np.array_equal(st, ref), (c, graph)
            w.close()


def test_graph_replays_match_eager_steps():
    sc = _batched(seed=4)
    we = _world(sc)
    wg = _world(sc, pgs_block=256, pgs_lds_reps=1200, persistent=1, graph=1)
    for chunk in range(6):
        we.step(7)
        wg.step(7)
        a, b = we.read_state(), wg.read_state()         # eager work between the replays
        assert np.array_equal(a, b), chunk
        if chunk == 3:                                   # a parameter change forces a new capture
            for w in (we, wg):                           # (and the coupling kernel joins the step)
                w.set_params(erp=0.25, coupling=ovl.COUPLING_PREV_IMPULSE)
    sa, sb = we.step(1, stats=True), wg.step(1, stats=True)
    assert sa["n_contacts"] == sb["n_contacts"] > 100
    assert np.array_equal(we.read_state(), wg.read_state())


def test_autotune_advances_one_step_with_the_fastest_candidate():
    sc = _batched(seed=5, n_scenes=24, nmax=3000)
    w0 = _world(sc)
    wt = _world(sc, graph=1)
    w0.step(40)
    wt.step(40)
    chosen, ms = wt.autotune(trials=2)
    w0.step(1)
    log(f"  chosen {chosen}; candidate ms {np.round(ms, 3).tolist()}")
    cands = ovl.launch_candidates()
    assert dict(chosen, graph=0) in cands and chosen["graph"] == 1
    assert np.all(ms > 0) and ms[cands.index(dict(chosen, graph=0))] == ms.min()
    assert wt.get_launch() == chosen
    assert np.array_equal(w0.read_state(), wt.read_state())
    w0.step(5)
    wt.step(5)
    assert np.array_equal(w0.read_state(), wt.read_state())


def test_batched_world_through_graph_matches_oracle():
    sc = _uneven([(1900, 1), (700, 3), (300, 1), (1000, 2)], 6)
    w = ovl.World(sc, ovl.make_params(dt=sc.dt, max_iters=sc.iters))
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
    w.set_launch(pgs_block=256, pgs_lds_reps=1200, persistent=1, graph=1)
    p = w.params
    w.step(2)                       # the graph is captured and replayed before the compared step
    st, o = compare_step(sc, w, p, start=oracle_run(sc, p, 150), label="batched t=151 (graph, persistent)")
    big = _largest_partition(w)
    log(f"  largest partition {big} replicas (LDS tile 1200)")
    assert st["n_contacts"] > 300 and big > 1200


def test_more_partitions_than_compute_units_matches_oracle():
    """Over one partition per compute unit the small partitions colour in the
    256-thread variant, several to a compute unit; colours must still equal
    the oracle's bit for bit."""
    import torch
    sc = _batched(n_scenes=110, seed=9, nmax=700)
    G = int(sc.parts_per_scene.sum())
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    log(f"  {sc.n_bodies} bodies, {G} partitions, {n_cu} compute units")
    assert G > n_cu
    w = ovl.World(sc, ovl.make_params(dt=sc.dt, max_iters=sc.iters))
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
    # every scene's pile squeezed to 30% of its height, so contacts come at once
    st0 = sc.state.copy()
    for s in range(sc.n_scenes):
        m = sc.scene == s
        z0 = st0[m, 2].min()
        st0[m, 2] = (z0 + (st0[m, 2] - z0) * 0.3).astype(np.float32)
    st, o = compare_step(sc, w, w.params, start=oracle_run(sc, w.params, 3, state=st0), label=f"{G} partitions t=4")
    assert st["n_contacts"] > 10000
