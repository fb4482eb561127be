"""GPU parity for the solver's less common paths, against the oracle step by
step: a colour of more than twice the workgroup (a thread's third slot, loaded
where it is solved, after the second slot loaded while the first is solved),
and a partition of more than 16,384 replicas (replica ids read from their own
array rather than packed into the impulse's fourth component, velocities in
global memory).
"""
import numpy as np
import pytest

import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes
from parity import compare_step, log, next_start, oracle_run

pytestmark = pytest.mark.gpu


def make_world(sc, **pkw):
    p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, **pkw)
    w = ovl.World(sc, p)
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
    return w, p


def test_colours_beyond_twice_the_workgroup():
    """A 64 x 64 layer of touching spheres on the ground, one partition of 4,096
    replicas (velocities in LDS, 1,024-thread workgroup): its largest colour
    holds about 2,900 contacts, so some threads solve three slots of it."""
    n = 64
    r = 0.5
    xs = np.arange(n) * (2 * r - 0.002)
    pos = np.array([[x, y, r - 0.001] for x in xs for y in xs], np.float32)
    sc = scenes.custom_spheres(pos, r, 1.0, planes=scenes.GROUND, mu=0.5, dt=1 / 60, iters=12)
    w, p = make_world(sc)
    assert w.get_launch()["pgs_block"] == 1024
    st, o = compare_step(sc, w, p, label="sphere layer t=0")
    col = w.debug("copy_colour")
    sizes = np.bincount(col)
    log(f"  {len(col)} copies in {len(sizes)} colours, largest {sizes.max()}")
    assert sizes.max() > 2 * 1024 and len(sizes) > 1
    s, c = next_start(o)
    compare_step(sc, w, p, start=oracle_run(sc, p, 3, state=s, cache=c), label="sphere layer t=4")


def test_partition_beyond_packed_ids():
    """96 chains of 200 ball-jointed links in one partition: 19,200 replicas,
    above both the LDS tile and the 16,384 replicas whose ids fit the
    impulse's fourth component."""
    sc = scenes.config3(0, n_chains=96, links=200)
    sc.owner = np.zeros(sc.n_bodies, np.int32)
    sc.parts_per_scene = np.array([1], np.int32)
    w, p = make_world(sc)
    st, o = compare_step(sc, w, p, label="96 chains, one partition, t=0")
    assert int(w.debug("part_rep_off")[-1]) > 16384
    s, c = next_start(o)
    compare_step(sc, w, p, start=oracle_run(sc, p, 5, state=s, cache=c), label="96 chains, one partition, t=6")
