"""GPU parity of the accuracy-study options against the oracle.

* equal blending weights (the naive weights of section 5.3) on jointed
  chains: weights exactly 1/|W|, then the whole step as every parity test;
* the diagnostics of a step computed with the exact residual: the natural-map
  residual summed over all rows (the paper's total residual, section 6) and
  the largest and summed joint violation of the blended state, against the
  oracle's from the same state and warm-start cache.

The diagnostics are compared on a state whose links are displaced by up to
2 cm, so that the violations (about 1e-2 m per joint) and the residual of the
unconverged chain solve stand far above what float32 positions resolve
(about 2e-6 m at 20 m): joint violations within 1e-3 relative, residuals
(each side's own final iterate after the same 40 sweeps) within 2%.
"""
import numpy as np
import pytest

import oracle
import paper_2403_17261_amd as ovl
from paper_2403_17261_amd import scenes
from parity import compare_step, log, next_start, oracle_kwargs, oracle_run

pytestmark = pytest.mark.gpu


def _chains(weights):
    sc = scenes.config3(0, n_chains=32, links=50)
    p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, weights=weights)
    w = ovl.World(sc, p)
    w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
    return sc, w, p


def test_equal_weights_parity():
    sc, w, p = _chains(ovl.WEIGHTS_EQUAL)
    _, o = compare_step(sc, w, p, label="chains, equal weights t=0")
    nw = np.bitwise_count(o["mask"].astype(np.uint64))[o["rep_body"]]
    assert np.array_equal(o["rep_w"], 1.0 / nw)
    assert (nw > 1).sum() > 100
    s, c = next_start(o)
    compare_step(sc, w, p, start=oracle_run(sc, p, 60, state=s, cache=c), label="chains, equal weights t=61")


@pytest.mark.parametrize("weights", [ovl.WEIGHTS_GEODESIC, ovl.WEIGHTS_EQUAL])
def test_step_diagnostics_against_oracle(weights):
    sc, w, p = _chains(weights)
    rng = np.random.default_rng(5)
    s0 = sc.state.copy()
    s0[:, :3] += rng.uniform(-0.02, 0.02, (sc.n_bodies, 3)).astype(np.float32)
    w.write_state(s0, keep_cache=False)
    st = w.step(1, stats=True, exact=True)
    o = oracle.step(sc, state=s0, **oracle_kwargs(sc, p, sc.halo_k, sc.beta))
    log(f"  joint violation max {st['joint_violation_max']:.3e} / {o['joint_violation']:.3e}, "
        f"sum {st['joint_violation_sum']:.4e} / {o['joint_violation_sum']:.4e}; residual sum "
        f"{st['resid_exact_sum']:.4e} / {o['rho_sum']:.4e}, max {st['resid_exact']:.3e} / {o['rho_exact']:.3e}")
    assert o["joint_violation"] > 1e-2 and o["rho_exact"] > 1e-3
    assert st["joint_violation_max"] == pytest.approx(o["joint_violation"], rel=1e-3)
    assert st["joint_violation_sum"] == pytest.approx(o["joint_violation_sum"], rel=1e-3)
    assert st["resid_exact_sum"] == pytest.approx(o["rho_sum"], rel=2e-2)
    assert st["resid_exact"] == pytest.approx(o["rho_exact"], rel=2e-2)
