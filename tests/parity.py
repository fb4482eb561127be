"""Helpers for the GPU-vs-oracle parity tests (no method arithmetic here).

compare_step() writes a start into a GPU world -- the scene's synthetic
initial state, or a state and warm-start cache the oracle produced
(oracle_run) -- advances the world by one step, runs the oracle from the same
start, and compares every intermediate result: integer structures bit for
bit, floating point within the tolerances stated below.  No oracle input is
read back from the GPU library.

Tolerances (FP32 GPU path against the FP64 oracle after one step):
  velocity   |v - v_ref| <= 1e-4 * max(|v_ref|, g h)          per body
  spin       |w - w_ref| <= 1e-4 * max(|w_ref|, g h / r)      per body
  position   |x - x_ref| <= 1e-6 * (1 + |x_ref|) + h * (velocity bound)
  weights    |w - w_ref| <= 1e-6
"""
import sys

import numpy as np

import oracle

G_ACC = 9.81


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def adjacency_sets(off, adj):
    return [tuple(sorted(int(u) for u in adj[off[v]:off[v + 1]] if u >= 0)) for v in range(len(off) - 1)]


def oracle_kwargs(sc, params, halo_k, beta):
    return dict(dt=params.dt, gravity=tuple(params.gravity), cfm=params.cfm, erp=params.erp,
                max_iters=params.max_iters, tol=params.tol, adaptive=params.mode == 1,
                warmstart=params.warmstart == 1, seed=params.seed, halo_k=halo_k, beta=beta,
                equal_weights=params.weights == 1, coupling=int(params.coupling))


def check_state(sc, gpu, ref, dt, label=""):
    r = sc.radius.astype(np.float64)
    gh = G_ACC * dt
    v, vr = gpu[:, 7:10].astype(np.float64), ref[:, 7:10]
    w, wr = gpu[:, 10:13].astype(np.float64), ref[:, 10:13]
    ev = np.linalg.norm(v - vr, axis=1) / np.maximum(np.linalg.norm(vr, axis=1), gh)
    ew = np.linalg.norm(w - wr, axis=1) / np.maximum(np.linalg.norm(wr, axis=1), gh / r)
    vb = 1e-4 * np.maximum(np.linalg.norm(vr, axis=1), gh)
    ex = np.linalg.norm(gpu[:, 0:3] - ref[:, 0:3], axis=1) - (1e-6 * (1 + np.linalg.norm(ref[:, 0:3], axis=1)) + dt * vb)
    qd = np.minimum(np.linalg.norm(gpu[:, 3:7] - ref[:, 3:7], axis=1), np.linalg.norm(gpu[:, 3:7] + ref[:, 3:7], axis=1))
    worst = dict(v=float(ev.max(initial=0)), w=float(ew.max(initial=0)), x=float(ex.max(initial=-1)),
                 q=float(qd.max(initial=0)))
    log(f"  {label} worst rel dv={worst['v']:.2e} dw={worst['w']:.2e} x-excess={worst['x']:.2e} dq={worst['q']:.2e}")
    bad_v = np.where(ev > 1e-4)[0]
    bad_w = np.where(ew > 1e-4)[0]
    assert len(bad_v) == 0, f"{label}: {len(bad_v)} bodies exceed the velocity tolerance, e.g. {bad_v[:5]} {ev[bad_v[:5]]}"
    assert len(bad_w) == 0, f"{label}: {len(bad_w)} bodies exceed the spin tolerance, e.g. {bad_w[:5]} {ew[bad_w[:5]]}"
    assert worst["x"] <= 0.0, f"{label}: position error {worst['x']}"
    assert worst["q"] <= 1e-5, f"{label}: quaternion error {worst['q']}"


def oracle_run(sc, params, steps, state=None, cache=None, owner=None, pps=None, halo_k=None, beta=None, lb=None,
               **extra):
    """`steps` oracle steps from `state` (default: the scene's initial state)
    and `cache`, each fed its own output.  Returns (state as float32, the last
    output: its warm-start cache, and with lb its worker sets in "mask").
    lb: dict(sets=, depth=) carries the worker sets of dynamic load balancing."""
    halo_k = sc.halo_k if halo_k is None else halo_k
    beta = sc.beta if beta is None else beta
    kw = oracle_kwargs(sc, params, halo_k, beta)
    kw.update(extra)
    st = (sc.state if state is None else state).astype(np.float32)
    out = cache
    sets = None if lb is None else np.asarray(lb["sets"], np.uint64)
    for _ in range(steps):
        if lb is not None:
            kw.update(lb_masks=sets, lb_depth=int(lb["depth"]))
        out = oracle.step(sc, state=st, owner=owner, parts_per_scene=pps, cache=out, **kw)
        st = out["state"].astype(np.float32)
        if lb is not None:
            sets = out["mask"].astype(np.uint64)
    return st, out


def next_start(o):
    """The start of the step after an oracle step: its state and cache."""
    return o["state"].astype(np.float32), o


def compare_step(sc, w, params, start=None, owner=None, pps=None, halo_k=None, beta=None, forced=None, label="",
                 check_lambda0=True, lb=None):
    """One GPU step against one oracle step from the same start.

    start: None (the scene's initial state, no warm-start cache) or
    (state, cache) from the oracle; it is written into the world first.
    lb: None (k-hop halo sets), or dict(sets=, depth=) giving the carried worker
    sets for this step and the growth depth; they are written into the world
    too, unless lb["carried"] says the world holds them from its last step
    (which the previous comparison found equal to the oracle's)."""
    halo_k = sc.halo_k if halo_k is None else halo_k
    beta = sc.beta if beta is None else beta
    owner = sc.owner if owner is None else owner
    pps = sc.parts_per_scene if pps is None else pps
    s0, cache = (sc.state.astype(np.float32), None) if start is None else start
    s0 = np.ascontiguousarray(s0, np.float32)
    w.write_state(s0, keep_cache=False)
    if cache is not None and len(cache["cache_part"]):
        w.write_cache(cache)
    else:
        cache = None
    if lb is not None and not lb.get("carried", False):
        w.set_load_balance(True, int(lb["depth"]), sets=np.asarray(lb["sets"], np.uint64))
    if forced is not None:
        w.force_iters(forced)
    stats = w.step(1, stats=True)
    g = {k: w.debug(k) for k in ("contact_key", "adj_off", "adj", "mask", "part_rep_off", "rep_body", "rep_d",
                                 "rep_w", "part_copy_off", "copy_kind", "copy_key", "copy_ia", "copy_ib",
                                 "copy_colour", "copy_lambda0", "part_iters")}
    gs = w.read_state()
    kw = oracle_kwargs(sc, params, halo_k, beta)
    if lb is not None:
        kw.update(lb_masks=np.asarray(lb["sets"], np.uint64), lb_depth=int(lb["depth"]))
    o = oracle.step(sc, state=s0, owner=owner, parts_per_scene=pps, cache=cache,
                    forced_iters=forced if forced is not None else None, **kw)
    log(f"  {label} contacts={len(o['contact_key'])} copies={len(o['copy_key'])} replicas={len(o['rep_body'])} "
        f"overlap={o['n_overlap']} colours={o['max_colours']} gpu_iters={stats['max_iters']}")
    assert np.array_equal(g["contact_key"], o["contact_key"]), "contact lists differ"
    assert adjacency_sets(g["adj_off"], g["adj"]) == adjacency_sets(o["adj_off"], o["adj"]), "graphs differ"
    assert np.array_equal(g["mask"], o["mask"]), "overlap masks differ"
    assert np.array_equal(g["part_rep_off"], o["part_rep_off"]), "replica offsets differ"
    assert np.array_equal(g["rep_body"], o["rep_body"]), "replica tables differ"
    assert np.array_equal(g["rep_d"], o["rep_d"]), "geodesic distances differ"
    assert np.abs(g["rep_w"] - o["rep_w"]).max(initial=0) <= 1e-6, "weights differ"
    for k in ("part_copy_off", "copy_kind", "copy_key", "copy_ia", "copy_ib", "copy_colour"):
        assert np.array_equal(g[k], o[k]), f"{k} differs"
    if check_lambda0 and len(o["copy_lambda0"]):
        diff = np.abs(g["copy_lambda0"] - o["copy_lambda0"])
        d0 = diff.max()
        scale = max(1.0, np.abs(o["copy_lambda0"]).max())
        if d0 > 1e-5 * scale:
            bad = np.nonzero(diff.max(axis=1) > 1e-5 * scale)[0]
            u = int(bad[0])
            log(f"  warm start: {len(bad)} copies beyond {1e-5 * scale:.3e}; first uid {u} kind {g['copy_kind'][u]} "
                f"key {int(g['copy_key'][u]):#x} gpu {g['copy_lambda0'][u]} oracle {o['copy_lambda0'][u]}")
        assert d0 <= 1e-5 * scale, f"warm start differs by {d0}"
    if params.coupling == 1:
        # interface-coupling impulses per replica: float32 sums of a few
        # float32 impulses against the oracle's double ones
        gc, oc = w.debug("rep_cpl").astype(np.float64), o["rep_cpl"]
        scale = max(np.abs(oc).max(initial=0.0), G_ACC * params.dt)
        dc = np.abs(gc - oc).max(initial=0.0)
        log(f"  {label} coupled replicas {int((np.abs(oc).max(axis=1) > 0).sum())}, largest impulse {scale:.3e}, "
            f"worst difference {dc:.2e}")
        assert dc <= 1e-5 * scale, f"coupling impulses differ by {dc}"
    if forced is None and not params.mode:
        assert np.all(g["part_iters"] == params.max_iters)
    check_state(sc, gs, o["state"], params.dt, label)
    return stats, o
