#!/usr/bin/env python3
"""Benchmark: body-steps/s at projected Gauss-Seidel residual <= 1e-4, learned
against plain warm start.

Default workload (--workload tower): the 100,000-sphere tower collapse, a
50x50x40 lattice of spheres (r = 0.25 m, density 1000 kg/m^3, jitter
U(+-0.005) m) on a ground plane, mu = 0.5, h = 1/60 s, 64 column partitions
(8x8) with a 2-hop overlap, geodesic search depth 4, adaptive sweeps to a
residual of 1e-4 m/s with a cap of 1000, the first --steps steps from the
initial state (the warm-up steps run first and the state is then reset).
Plain and learned warm starts are timed at 1e-4 and again at the looser
tolerances 1e-2, 3e-3 and 1e-3 (the ladder); the line states the share of
partition-steps that reach each tolerance before the cap, and compares the
two starts at the tightest tolerance both reach in at least 95% of
partition-steps.  The other four configurations (the 64-sphere lattice, the
bowl pile, the chains and the 512 batched bowls) are timed at their fixed
sweep counts over their stated step counts and reported beside the headline.

--workload bowl: the 20,000-sphere bowl pile (8 k-means partitions recomputed
every 10 steps, 2-hop overlap), 1000 steps.

--workload bowl-lb: the paper's Bowl scene with dynamic load balancing
(section 5.4): 5,040 spheres dropped into the bowl, 7 workers starting from
the naive division of the body list, growth depth 0, worker sets updated
with every contact of the step; first 600 steps.  Also reports the per-worker body
and contact distributions over the run and the same run without balancing.

--workload accuracy: the accuracy study on the 51,200-link chains (256
chains of 200 ball-jointed spheres over 16 static spheres, 16 x-slabs, h
1/120 s, 40 sweeps, 500 steps, seeds 0-2): overlap depth k = 1..4 (gamma = k - 1) with
geodesic and with equal blend weights, with geodesic weights plus interface
coupling by the previous step's impulses of cut constraints (section 7) or by
splitting the mass of overlap bodies by blend weight (section 2's comparison
with mass splitting), and one partition as the reference; joint violation and
total residual sampled every 25 steps.

--workload batched: 512 independent bowl scenes (log-uniform 200..5000
spheres, 1..6 k-means partitions each, fixed at the start), 30 sweeps per
step, all in one world: the autotuned, graph-replayed launch against the
default launch and against a loop that steps one world per scene.

One GPU only.  Prints one JSON line.  The roofline entry is for the
Gauss-Seidel kernel, whose binding resource is vector-instruction issue on the
compute units that hold a partition: the algorithmic FP32 operations of all
sweeps of the timed steps (per sweep and constraint copy: 88 for a sphere
contact between two bodies, 74 with a static body, 63 for a ball joint) over
the kernel's summed duration from HIP events recorded on the stream it runs
on, against the chip's VALU issue rate without packed FP32.  The algorithmic
byte rate (220 / 164 / 192 B per copy and sweep) is reported beside it.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# interface coupling modes (the library's OVL_COUPLING_* values)
COUPLING_NAMES = {0: "none", 1: "previous-step impulses", 2: "mass splitting"}
COUPLING_FLAGS = {"none": 0, "impulse": 1, "split": 2}
SOLVER_SRC = os.path.join(ROOT, "paper_2403_17261_amd", "csrc", "solve.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solver_hash():
    with open(SOLVER_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def run_loop(w, sc, steps, state0, owner0, cent0, rebalance_iters=3):
    """steps steps of the scene, rebalancing the k-means owners every sc.rebalance_every steps."""
    from paper_2403_17261_amd import scenes

    owner, cent = owner0, cent0
    t = 0
    every = sc.rebalance_every or steps
    while t < steps:
        if t > 0 and t % every == 0 and sc.rebalance_every:
            st = w.read_state()
            owner, cent = scenes.kmeans_owner(st[:, :3], int(sc.parts_per_scene[0]), iters=rebalance_iters,
                                              centroids=cent)
            w.set_partitions(owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
        n = min(every - t % every, steps - t)
        w.step(n)
        t += n
    return owner, cent


def host_cpu():
    """CPU model, online CPUs and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc_online": os.cpu_count(), "nproc_usable": usable}


def cpu_baseline(workload, n_steps, tol, cap, max_threads=16):
    """The oracle (double precision) on a bounded sample of the workload, on one
    thread and on T = min(partitions, usable cores, max_threads) threads, one
    partition per thread at a time (the paper's worker per core)."""
    import oracle
    from paper_2403_17261_amd import scenes

    kw = dict(adaptive=True, tol=tol, max_iters=cap)
    if workload == "tower":
        # a 25x25x40 sub-tower in 4x4 columns: partitions of the benchmark's size, from t = 0
        sc = scenes.config5(0, nx=25, ny=25, nz=40, cols=4)
        st0, owner, o0 = sc.state, sc.owner, None
        what = (f"the first {n_steps} steps of a 25x25x40 sub-tower (25,000 spheres, 4x4 column partitions of the "
                f"benchmark's partition size) from t = 0")
    else:
        path = os.path.join(ROOT, "oracle", "data", "bowl20k_seed0_t300.npz")
        if not os.path.exists(path):
            return None
        d = np.load(path)
        sc = scenes.config2(0)
        owner = d["owner"]
        o0 = oracle.step(sc, state=d["state"], owner=owner, **kw)         # untimed: fills the warm-start cache
        st0 = o0["state"].astype(np.float32)
        what = f"{n_steps} steps of the 20,000-sphere bowl pile from its oracle-computed state at step 300"
    host = host_cpu()
    G = int(sc.parts_per_scene.sum())
    T = max(1, min(G, host["nproc_usable"], max_threads))

    def leg(threads):
        st, o = st0, o0
        t0 = time.perf_counter()
        sweeps = 0
        for _ in range(n_steps):
            o = oracle.step(sc, state=st, owner=owner, cache=o, threads=threads, **kw)
            st = o["state"].astype(np.float32)
            sweeps += int(o["max_iters"])
        dt = time.perf_counter() - t0
        return {"value": sc.n_bodies * n_steps / dt, "unit": "body-steps/s", "threads": threads,
                "secs": round(dt, 2), "sweeps_per_step": sweeps / n_steps}

    one = leg(1)
    many = leg(T) if T > 1 else one
    return {
        "value": many["value"], "unit": "body-steps/s", "cores": T, "kind": "oracle",
        "sample": f"oracle (double precision, adaptive sweeps to {tol:g}, cap {cap}): {what}; {G} partitions "
                  f"solved on {T} threads, one partition per thread at a time (the paper's worker per core); "
                  f"contacts, graph, weights and blending sequential; mean {many['sweeps_per_step']:.0f} sweeps "
                  f"per step (largest partition), {many['secs']:.1f} s",
        "single_thread": one, "worker_per_core": many, **host,
    }


def bench_batched(args):
    """Many uneven scenes: one batched world (default launch; autotuned + graph) against a per-scene loop."""
    import torch

    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    sc = scenes.config4(0)
    steps = args.steps or 50
    p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, mode=ovl.MODE_FIXED, warmstart=ovl.WARM_PLAIN)
    N = sc.n_bodies
    res = {}

    def timed(step_fn, sync_fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step_fn()
        sync_fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    from paper_2403_17261_amd import tuning

    # one world holding every scene: the default launch and the autotuned,
    # graph-replayed one (the tuner's choice cached per architecture and world
    # shape), each timed args.repeats times in alternation
    reps = {"default": [], "tuned": []}
    for rep_i in range(args.repeats):
        for name in ("default", "tuned"):
            w = ovl.World(sc, p)
            w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
            w.step(args.warmup)
            cand_ms, cached = None, None
            if name == "tuned":
                w.set_launch(graph=1)
                chosen, cand_ms, cached = tuning.tuned_launch(w, sc, trials=3)
                log(f"[batched] launch {chosen} ({'cached' if cached else 'tuned now'})"
                    + ("" if cand_ms is None else f"; candidate ms {np.round(cand_ms, 3).tolist()}"))
            w.sync()
            w.profile(True)
            c0 = w.counters()
            w.profile(False)            # profiled steps bypass the graph; time the launch itself
            secs = timed(lambda: w.step(1), w.sync)
            c1 = w.counters()
            if c1["steps"] - c0["steps"] != steps:
                raise RuntimeError("not every step committed")
            r = {"secs": secs, "value": N * steps / secs, "ms_per_step": 1e3 * secs / steps,
                 "launch": w.get_launch(), "candidates_ms": None if cand_ms is None else
                 [round(float(x), 4) for x in cand_ms], "from_cache": cached}
            reps[name].append(r)
            log(f"[batched {name} {rep_i}] {r['value']:.3e} body-steps/s, {r['ms_per_step']:.3f} ms/step")
            w.close()
    for name, rs in reps.items():
        ms = np.array([r["ms_per_step"] for r in rs])
        best = rs[int(np.argmin(ms))]
        res[name] = {**best, "ms_per_step_runs": [round(float(x), 4) for x in ms],
                     "ms_per_step_mean": float(ms.mean()), "ms_per_step_spread": float(ms.max() - ms.min())}
    if args.skip_loop:
        res["per_scene_loop"] = None
    else:
        res["per_scene_loop"] = per_scene_loop(sc, p, args, timed)
    head = res["tuned"]
    loop = res["per_scene_loop"]
    out = {
        "metric": "body-steps/s, batched scenes, 30 sweeps per step",
        "value": head["value"], "unit": "body-steps/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": (f"512 bowl scenes, spheres log-uniform 200..5000 per scene ({N} in all), r~U(0.2,0.5) m, "
                         f"1..6 k-means partitions per scene ({int(sc.parts_per_scene.sum())} in all, fixed), "
                         f"2-hop overlap, h 1/60 s, 30 sweeps per step, steps {args.warmup + 1}..."
                         f"{args.warmup + steps} of the drop"),
            "batched_tuned": res["tuned"], "batched_default": res["default"], "per_scene_loop": loop,
            "tuned_minus_default_ms_mean": res["tuned"]["ms_per_step_mean"] - res["default"]["ms_per_step_mean"],
            "speedup_vs_per_scene_loop": None if loop is None else loop["secs"] / head["secs"],
        },
    }
    print(json.dumps(out), flush=True)


def bench_bowl_lb(args):
    """The Bowl scene of section 6 with the load balancing of section 5.4."""
    import torch

    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    sc = scenes.bowl_naive(5040, 0, 7)
    steps = args.steps or 600
    G = int(sc.parts_per_scene[0])
    p = ovl.make_params(dt=sc.dt, max_iters=args.cap, mode=ovl.MODE_ADAPTIVE, tol=args.tol,
                        warmstart=ovl.WARM_PLAIN)

    p_cpl = ovl.make_params(dt=sc.dt, max_iters=args.cap, mode=ovl.MODE_ADAPTIVE, tol=args.tol,
                            warmstart=ovl.WARM_PLAIN, coupling=ovl.COUPLING_PREV_IMPULSE)
    p_split = ovl.make_params(dt=sc.dt, max_iters=args.cap, mode=ovl.MODE_ADAPTIVE, tol=args.tol,
                              warmstart=ovl.WARM_PLAIN, coupling=ovl.COUPLING_MASS_SPLIT)

    def restart(w, lb):
        w.write_state(sc.state, keep_cache=False)
        w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=1, beta=sc.beta)
        w.set_load_balance(lb, 0)

    def exact_replay(w, lb):
        """The same run again, untimed: the exact residual of every 10th step of its second half."""
        restart(w, lb)
        w.step(steps // 2)
        out = []
        for _ in range(steps // 2, steps, 10):
            w.step(9)
            out.append(float(w.step(1, stats=True, exact=True)["resid_exact"]))
        return out

    def timed_run(lb, params=p):
        w = ovl.World(sc, params)
        restart(w, lb)
        log(f"[bowl-lb {'on' if lb else 'off'}] warm-up: the {steps} steps once (buffers grow here)")
        w.step(steps, stats=True)
        restart(w, lb)
        w.profile(True)
        c0 = w.counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w.step(steps)
        w.sync()
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        c1 = w.counters()
        if c1["steps"] - c0["steps"] != steps:
            raise RuntimeError("not every step committed")
        r = {"secs": secs, "value": sc.n_bodies * steps / secs, "ms_per_step": 1e3 * secs / steps,
             "pgs_ms": c1["pgs_ms"] - c0["pgs_ms"], "pgs_launches": c1["pgs_launches"] - c0["pgs_launches"],
             "pgs_bytes": c1["pgs_bytes"] - c0["pgs_bytes"], "pgs_ops": c1["pgs_ops"] - c0["pgs_ops"],
             "sweeps_mean": (c1["sweeps_max_total"] - c0["sweeps_max_total"]) / steps,
             "unconverged": c1["unconverged_total"] - c0["unconverged_total"]}
        log(f"[bowl-lb {'on' if lb else 'off'}] {r['value']:.3e} body-steps/s, {r['ms_per_step']:.3f} ms/step, "
            f"sweeps/step {r['sweeps_mean']:.1f}")
        return w, r

    w, on = timed_run(True)
    # per-worker distributions (Figures 13 and 14): the same trajectory again, sampled every 10 steps
    restart(w, True)
    bodies, contacts, overlap, changes = [], [], [], []
    for t in range(0, steps, 10):
        w.step(9)
        changes.append(int(w.step(1, stats=True)["n_lb_changes"]))
        ro = w.debug("part_rep_off").astype(np.int64)
        co = w.debug("part_copy_off").astype(np.int64)
        bodies.append(np.diff(ro))
        contacts.append(np.diff(co))
        overlap.append(int((np.bitwise_count(w.debug("mask").astype(np.uint64)) >= 2).sum()))
    w.close()
    bodies, contacts = np.array(bodies), np.array(contacts)
    half = len(bodies) // 2

    def quart(x):
        return [[int(v) for v in np.percentile(x[:, g], [25, 50, 75])] for g in range(G)]

    def imbalance(x):
        m = x.mean(axis=1)
        ok = m > 0
        return float(np.mean(x.max(axis=1)[ok] / m[ok])) if ok.any() else None

    _, off = timed_run(False)
    w, cpl = timed_run(True, p_cpl)
    cpl["exact"] = exact_replay(w, True)
    w.close()
    w, split = timed_run(True, p_split)
    split["exact"] = exact_replay(w, True)
    w.close()
    w = ovl.World(sc, p)
    on["exact"] = exact_replay(w, True)
    w.close()
    pgs_ms, pgs_launches, pgs_bytes = on["pgs_ms"], on["pgs_launches"], on["pgs_bytes"]
    ops_rate = on["pgs_ops"] / (pgs_ms * 1e-3) / 1e12 if pgs_ms > 0 else 0.0
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_lb(sc, args.tol, args.cap)
    out = {
        "metric": "body-steps/s at PGS residual <=1e-4, dynamic load balancing",
        "value": on["value"], "unit": "body-steps/s", "n_gpus": 1, "steps": steps, "warmup": steps,
        "ms_per_step": on["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": (f"bowl with load balancing: {sc.n_bodies} spheres r~U(0.2,0.5) m, density 1000, "
                         f"five-plane bowl, mu 0.6, h 1/60 s, {G} workers from the naive division of the body "
                         f"list, growth depth 0, beta 4, adaptive sweeps to {args.tol:g} (cap {args.cap}), "
                         f"first {steps} steps of the drop"),
            "mean_sweeps_per_step": round(on["sweeps_mean"], 2), "unconverged_partition_steps": int(on["unconverged"]),
            "bodies_per_worker_quartiles_second_half": quart(bodies[half:]),
            "contact_copies_per_worker_quartiles_second_half": quart(contacts[half:]),
            "max_over_mean_bodies_second_half": imbalance(bodies[half:]),
            "max_over_mean_contacts_second_half": imbalance(contacts[half:]),
            "overlap_bodies_last": overlap[-1],
            "rule_changes_per_step_second_half": float(np.mean(changes[half:])),
            "without_balancing": {"ms_per_step": off["ms_per_step"], "body_steps_per_s": off["value"],
                                  "sweeps_per_step": round(off["sweeps_mean"], 2),
                                  "note": "same owners, 1-hop halo of the naive division every step"},
            "exact_residual_second_half_mean": float(np.mean(on["exact"])),
            "with_interface_coupling": {"ms_per_step": cpl["ms_per_step"], "body_steps_per_s": cpl["value"],
                                        "sweeps_per_step": round(cpl["sweeps_mean"], 2),
                                        "exact_residual_second_half_mean": float(np.mean(cpl["exact"])),
                                        "note": "balancing on, plus the previous step's impulses of cut "
                                                "constraints"},
            "with_mass_splitting": {"ms_per_step": split["ms_per_step"], "body_steps_per_s": split["value"],
                                    "sweeps_per_step": round(split["sweeps_mean"], 2),
                                    "exact_residual_second_half_mean": float(np.mean(split["exact"])),
                                    "note": "balancing on, overlap replicas carry their blend weight's share of "
                                            "the body's mass and inertia"},
        },
        "roofline": {
            "bound": "alu", "achieved": ops_rate, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": ops_rate / VALU_PEAK_TOPS, "traffic": None,
            "kernel": "k_pgs (coloured projected Gauss-Seidel, one workgroup per partition)",
            "launches": int(pgs_launches), "ms_per_launch": pgs_ms / max(1, pgs_launches),
            "alg_ops_per_launch": on["pgs_ops"] / max(1, pgs_launches),
            "busy_cus": min(G, N_CUS),
            "alg_bytes_per_launch": pgs_bytes / max(1, pgs_launches),
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_accuracy(args):
    """Section 6's error measures on the chains, seeds 0-2: geodesic against equal
    weights, the overlap depth, and the two interface couplings."""
    import torch

    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    seeds = tuple(int(x) for x in args.seeds.split(","))
    every = 25
    # (overlap depth k, blend weights, interface coupling mode); k = 0: one partition
    variants = ([(k, wmode, ovl.COUPLING_NONE) for k in (1, 2, 3, 4) for wmode in ("geodesic", "equal")] +
                [(k, "geodesic", c) for c in (ovl.COUPLING_PREV_IMPULSE, ovl.COUPLING_MASS_SPLIT)
                 for k in (1, 2, 3, 4)] + [(0, "one partition", ovl.COUPLING_NONE)])
    per_seed = {v: [] for v in variants}
    steps = None
    for seed in seeds:
        sc = scenes.config3(seed)
        steps = args.steps or sc.steps
        for k, wmode, cpl in variants:
            p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, mode=ovl.MODE_FIXED, warmstart=ovl.WARM_PLAIN,
                                weights=ovl.WEIGHTS_EQUAL if wmode == "equal" else ovl.WEIGHTS_GEODESIC,
                                coupling=cpl)
            w = ovl.World(sc, p)
            if k == 0:
                w.set_partitions(np.zeros(sc.n_bodies, np.int32), np.array([1], np.int32), halo_k=1, beta=sc.beta)
            else:
                w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=k, beta=sc.beta)
            samples = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for t in range(every, steps + 1, every):
                w.step(every - 1)
                st = w.step(1, stats=True, exact=True)
                samples.append((t, st["joint_violation_max"], st["joint_violation_sum"], st["resid_exact_sum"],
                                st["resid_exact"], st["n_overlap"], st["n_replicas"]))
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            w.close()
            a = np.array(samples, np.float64)
            half = a[len(a) // 2:]
            r = {"seed": seed, "ms_per_step": 1e3 * secs / steps,
                 "joint_violation_sum_mean_second_half": float(half[:, 2].mean()),
                 "joint_violation_max_mean_second_half": float(half[:, 1].mean()),
                 "joint_violation_max_worst": float(a[:, 1].max()),
                 "total_residual_mean_second_half": float(half[:, 3].mean()),
                 "overlap_bodies_mean": float(a[:, 5].mean()), "replicas_mean": float(a[:, 6].mean())}
            per_seed[(k, wmode, cpl)].append(r)
            log(f"[accuracy seed {seed} k={k} {wmode} {COUPLING_NAMES[cpl]}] joint violation sum "
                f"{r['joint_violation_sum_mean_second_half']:.4e} m (max {r['joint_violation_max_mean_second_half']:.3e}), "
                f"total residual {r['total_residual_mean_second_half']:.4e} m/s, overlap "
                f"{r['overlap_bodies_mean']:.0f}, {r['ms_per_step']:.2f} ms/step")
    runs = []
    keys = ("ms_per_step", "joint_violation_sum_mean_second_half", "joint_violation_max_mean_second_half",
            "joint_violation_max_worst", "total_residual_mean_second_half", "overlap_bodies_mean", "replicas_mean")
    for (k, wmode, cpl), rs in per_seed.items():
        r = {"k": k, "weights": wmode, "coupling": COUPLING_NAMES[cpl]}
        for key in keys:
            vals = [x[key] for x in rs]
            r[key] = float(np.max(vals)) if key == "joint_violation_max_worst" else float(np.mean(vals))
        r["per_seed_joint_violation_sum"] = [round(x["joint_violation_sum_mean_second_half"], 3) for x in rs]
        r["per_seed_joint_violation_max_mean"] = [round(x["joint_violation_max_mean_second_half"], 4) for x in rs]
        runs.append(r)
    head = next(r for r in runs if r["k"] == 3 and r["weights"] == "geodesic" and r["coupling"] == "none")
    out = {
        "metric": "summed ball-joint violation |C| of the blended state, mean over the second half of the steps "
                  "and over the seeds (lower is better)",
        "value": head["joint_violation_sum_mean_second_half"], "unit": "m", "n_gpus": 1, "steps": steps,
        "warmup": 0, "ms_per_step": head["ms_per_step"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": (f"chains: 256 chains of 200 ball-jointed spheres r 0.1 m, m 0.5 kg, over 16 static "
                         f"spheres, 16 x-slab partitions, h 1/120 s, 40 sweeps (fixed), beta 4, {steps} steps, "
                         f"seeds {list(seeds)}; exact diagnostics every {every} steps"),
            "reported": f"k = 3, geodesic weights, no interface coupling, mean over seeds {list(seeds)}",
            "runs": runs,
        },
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_lb(sc, tol, cap, n_steps=130):
    """The oracle on the first n_steps steps of the same run (carried sets and warm-start cache)."""
    import oracle

    st, m, o = sc.state, oracle.initial_masks(sc), None
    t0 = time.perf_counter()
    sweeps = 0
    for _ in range(n_steps):
        o = oracle.step(sc, state=st, cache=o, lb_masks=m, lb_depth=0, adaptive=True, tol=tol, max_iters=cap)
        st, m = o["state"].astype(np.float32), o["mask"].astype(np.uint64)
        sweeps += int(o["max_iters"])
    dt = time.perf_counter() - t0
    return {"value": sc.n_bodies * n_steps / dt, "unit": "body-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (double precision, one thread, adaptive sweeps to {tol:g}, cap {cap}) on the first "
                      f"{n_steps} steps of the same run (contacts begin near step 20, the pile forms after 100); mean "
                      f"{sweeps / n_steps:.0f} sweeps per step, {dt:.1f} s"}


def per_scene_loop(sc, p, args, timed):
    """One world per scene, stepped one after the other (default launch, no graph)."""
    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    steps = args.steps or 50
    N = sc.n_bodies
    parts = []
    off = np.searchsorted(sc.scene, np.arange(sc.n_scenes + 1))
    poff = np.concatenate([[0], np.cumsum(sc.parts_per_scene)])
    for s_ in range(sc.n_scenes):
        a, b = off[s_], off[s_ + 1]
        sub = scenes.Scene(
            scene=np.zeros(b - a, np.int32), shape=sc.shape[a:b], radius=sc.radius[a:b], halflen=sc.halflen[a:b],
            mass=sc.mass[a:b], inertia=sc.inertia[a:b], state=sc.state[a:b], mu=sc.mu[s_:s_ + 1],
            margin=sc.margin[s_:s_ + 1], plane_off=np.array([0, sc.plane_off[s_ + 1] - sc.plane_off[s_]], np.int32),
            planes=sc.planes[sc.plane_off[s_]:sc.plane_off[s_ + 1]], ssph_off=np.zeros(2, np.int32),
            ssph=np.zeros((0, 4), np.float32), joint_ab=np.zeros((0, 2), np.int32),
            joint_anchor=np.zeros((0, 6), np.float32), owner=(sc.owner[a:b] - poff[s_]).astype(np.int32),
            parts_per_scene=sc.parts_per_scene[s_:s_ + 1].copy(), name=f"scene{s_}", halo_k=sc.halo_k,
            beta=sc.beta, dt=sc.dt, iters=sc.iters, steps=sc.steps)
        wsub = ovl.World(sub, p)
        wsub.set_partitions(sub.owner, sub.parts_per_scene, halo_k=sub.halo_k, beta=sub.beta)
        parts.append(wsub)
    for wsub in parts:
        wsub.step(args.warmup)

    def step_all():
        for wsub in parts:
            wsub.step(1)

    secs = timed(step_all, lambda: [wsub.sync() for wsub in parts])
    r = {"secs": secs, "value": N * steps / secs, "ms_per_step": 1e3 * secs / steps}
    log(f"[per-scene loop] {r['value']:.3e} body-steps/s, {r['ms_per_step']:.3f} ms/step")
    for wsub in parts:
        wsub.close()
    return r


LADDER = (1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 1e-4)
# VALU issue of MI355X without packed FP32: 256 compute units, each issuing one
# wave64 vector instruction per clock (four 16-lane SIMDs, four clocks each),
# at 2.4 GHz: 256 * 64 * 2.4e9 single-precision lane operations per second.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
N_CUS = 256
COUNTERS_FILE = os.path.join(ROOT, "profiles", "pgs_counters.json")


def measured_counters():
    """rocprofv3 counters of the solver kernel on this workload (profiles/), if
    they were taken from this solver source; else None."""
    try:
        with open(COUNTERS_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    return t if t.get("solver_sha") == solver_hash() else None


def reset_run(w, sc, owner0):
    w.write_state(sc.state, keep_cache=False)
    w.set_partitions(owner0, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)


def timed_run(w, sc, steps, owner0, cent0):
    """steps steps from the scene's initial state (warm-start cache cleared), timed
    with the device idle on both sides; solver launches timed with HIP events."""
    import torch

    reset_run(w, sc, owner0)
    w.profile(True)
    c0 = w.counters()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_loop(w, sc, steps, sc.state, owner0, cent0)
    w.sync()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    c1 = w.counters()
    w.profile(False)
    done = c1["steps"] - c0["steps"]
    if done != steps:
        raise RuntimeError(f"only {done} of {steps} steps committed")
    G = int(np.sum(sc.parts_per_scene))
    d = {k: c1[k] - c0[k] for k in ("pgs_ms", "pgs_launches", "pgs_bytes", "pgs_ops", "sweeps_max_total",
                                     "sweeps_part_total", "unconverged_total", "steps_capped")}
    return {"secs": secs, "value": sc.n_bodies * steps / secs, "ms_per_step": 1e3 * secs / steps,
            "pgs_ms": d["pgs_ms"], "pgs_launches": d["pgs_launches"], "pgs_bytes": d["pgs_bytes"],
            "pgs_ops": d["pgs_ops"], "sweeps_mean": d["sweeps_max_total"] / steps,
            "sweeps_part_mean": d["sweeps_part_total"] / (steps * G), "unconverged": d["unconverged_total"],
            "steps_capped": d["steps_capped"], "partition_steps": steps * G,
            "pct_converged": 100.0 * (1.0 - d["unconverged_total"] / (steps * G))}


def rung_summary(r):
    return {"body_steps_per_s": r["value"], "ms_per_step": r["ms_per_step"],
            "partition_sweeps_per_step": round(r["sweeps_part_mean"], 2),
            "largest_partition_sweeps_per_step": round(r["sweeps_mean"], 2),
            "partition_steps_converged_pct": round(r["pct_converged"], 2),
            "steps_with_a_capped_partition_pct": round(100.0 * r["steps_capped"] / max(1, r["steps"]), 2)}


def bench_tower(args):
    """The headline: body-steps/s at residual <= tol (cap) on the tower collapse,
    learned and plain warm starts, with a ladder of looser tolerances."""
    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    sc = scenes.config5(0) if args.workload == "tower" else scenes.config2(0)
    if args.steps is None:
        args.steps = sc.steps
    mode = ovl.MODE_ADAPTIVE if args.mode == "adaptive" else ovl.MODE_FIXED
    cap = args.cap if mode == ovl.MODE_ADAPTIVE else sc.iters
    G = int(np.sum(sc.parts_per_scene))
    owner0 = sc.owner.copy()
    cent0 = sc.centroids[0].copy() if sc.rebalance_every else None
    modes = ["plain", "learned"] if args.warm == "both" else [args.warm]
    weights = None
    if "learned" in modes:
        if os.path.exists(args.weights):
            weights = np.load(args.weights, allow_pickle=False)["params"]
        else:
            log(f"no network weights at {args.weights}: timing the plain warm start only")
            modes = ["plain"]
    ladder = [t for t in LADDER if t != args.tol] if (mode == ovl.MODE_ADAPTIVE and not args.no_ladder) else []
    runs, rungs = {}, {}
    for mode_name in modes:
        p = ovl.make_params(dt=sc.dt, max_iters=cap, mode=mode, tol=args.tol, warmstart=ovl.WARM_PLAIN,
                            coupling=COUPLING_FLAGS[args.coupling])
        w = ovl.World(sc, p)
        w.set_partitions(owner0, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
        if mode_name == "learned":
            w.set_warmstart(ovl.WARM_LEARNED, weights)
        log(f"[{mode_name}] warm-up: {args.warmup} steps")
        run_loop(w, sc, args.warmup, sc.state, owner0, cent0)
        w.sync()
        log(f"[{mode_name}] timed: {args.steps} steps at tol {args.tol:g}, cap {cap}")
        r = timed_run(w, sc, args.steps, owner0, cent0)
        r["steps"] = args.steps
        # untimed: the same run again, the exact residual of every exact_every-th step
        exact = []
        if args.exact_every and mode == ovl.MODE_ADAPTIVE:
            reset_run(w, sc, owner0)
            for _ in range(args.exact_every, args.steps + 1, args.exact_every):
                w.step(args.exact_every - 1)
                exact.append(w.step(1, stats=True, exact=True)["resid_exact"])
        r["exact_sampled"] = exact
        r["last"] = w.step(0, stats=True)
        runs[mode_name] = r
        log(f"[{mode_name}] {r['value']:.3e} body-steps/s, {r['ms_per_step']:.3f} ms/step, solver "
            f"{r['pgs_ms'] / max(1, r['pgs_launches']):.3f} ms/launch, partition sweeps/step "
            f"{r['sweeps_part_mean']:.1f}, converged {r['pct_converged']:.1f}%")
        rungs[mode_name] = {args.tol: rung_summary(r)}
        for tol in ladder:
            w.set_params(tol=tol)
            q = timed_run(w, sc, args.steps, owner0, cent0)
            q["steps"] = args.steps
            rungs[mode_name][tol] = rung_summary(q)
            log(f"[{mode_name} tol {tol:g}] {q['value']:.3e} body-steps/s, partition sweeps/step "
                f"{q['sweeps_part_mean']:.1f}, converged {q['pct_converged']:.1f}%")
        w.close()
    head_name = "learned" if "learned" in runs else "plain"
    head = runs[head_name]
    # equal accuracy: the tightest tolerance that both starts reach in >= 95% of partition-steps
    equal = None
    if len(rungs) == 2:
        both = [t for t in sorted(rungs["plain"]) if t in rungs["learned"] and
                rungs["plain"][t]["partition_steps_converged_pct"] >= 95.0 and
                rungs["learned"][t]["partition_steps_converged_pct"] >= 95.0]
        if both:
            t = both[0]
            pl, le = rungs["plain"][t], rungs["learned"][t]
            equal = {"tol": t, "plain": pl, "learned": le,
                     "learned_over_plain_body_steps_per_s": le["body_steps_per_s"] / pl["body_steps_per_s"],
                     "learned_over_plain_partition_sweeps": (le["partition_sweeps_per_step"] /
                                                             max(1e-9, pl["partition_sweeps_per_step"]))}
    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: {args.cpu_steps} oracle steps, one thread and one thread per partition")
        cpu = cpu_baseline(args.workload, args.cpu_steps, args.tol, args.cap)
    others = None if args.no_configs else other_configs()
    pgs_ms, launches = head["pgs_ms"], max(1, head["pgs_launches"])
    ms_launch = pgs_ms / launches
    ops_rate = head["pgs_ops"] / (pgs_ms * 1e-3) / 1e12 if pgs_ms > 0 else 0.0
    busy = min(G, N_CUS)
    cnt = measured_counters()
    capped = head["steps_capped"] > 0
    out = {
        "metric": "body-steps/s at PGS residual <=1e-4; learned warm-start vs plain PGS",
        "value": head["value"],
        "unit": "body-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"tower collapse: 50x50x40 spheres r 0.25 m, density 1000, jitter 0.005 m, mu 0.5, "
                         f"h 1/60 s, 64 column partitions, 2-hop overlap, beta 4, first {args.steps} steps"
                         if args.workload == "tower" else
                         f"bowl pile: 20,000 spheres r~U(0.2,0.5) m, density 1000, five-plane bowl, mu 0.6, "
                         f"h 1/60 s, 8 k-means partitions (recomputed every 10 steps), 2-hop overlap, beta 4, "
                         f"first {args.steps} steps from the initial drop"),
            "n_bodies": sc.n_bodies, "partitions": G, "halo_k": sc.halo_k, "beta": sc.beta,
            "sweeps": f"{args.mode}, tol {args.tol:g}, cap {cap}",
            "warm_start": "learned (guarded per partition)" if head_name == "learned" else "plain",
            "interface_coupling": COUPLING_NAMES[COUPLING_FLAGS[args.coupling]],
            "accuracy": {
                "capped": capped,
                "label": (f"capped at {cap} sweeps: {head['pct_converged']:.1f}% of partition-steps reach "
                          f"residual {args.tol:g}; the rest stop at the cap" if capped else
                          f"every partition-step reaches residual {args.tol:g} within {cap} sweeps"),
                "partition_steps_converged_pct": round(head["pct_converged"], 2),
                "unconverged_partition_steps": int(head["unconverged"]),
                "partition_steps": int(head["partition_steps"]),
                "exact_residual_sampled_mean": float(np.mean(head["exact_sampled"])) if head["exact_sampled"] else None,
                "exact_residual_sampled_median": (float(np.median(head["exact_sampled"]))
                                                  if head["exact_sampled"] else None),
                "exact_residual_samples": len(head["exact_sampled"]),
            },
            "learned_vs_plain": {k: {**rung_summary(v),
                                     "exact_residual_sampled_mean": (float(np.mean(v["exact_sampled"]))
                                                                     if v["exact_sampled"] else None)}
                                 for k, v in runs.items()},
            "tolerance_ladder": {k: {f"{t:g}": v[t] for t in sorted(v, reverse=True)} for k, v in rungs.items()},
            "equal_accuracy": equal,
            "last_step": {k: head["last"][k] for k in ("n_contacts", "n_copies", "n_replicas", "n_overlap",
                                                       "max_colours")},
            "other_configs": others,
        },
        "roofline": {
            "bound": "alu", "achieved": ops_rate, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": ops_rate / VALU_PEAK_TOPS,
            "traffic": None if cnt is None else cnt.get("hbm_bytes_per_launch"),
            "kernel": "k_pgs (coloured projected Gauss-Seidel, one workgroup per partition)",
            "peak_basis": "FP32 vector lane operations: 256 CUs x 64 lanes x 2.4 GHz (one wave64 VALU "
                          "instruction per CU per clock, no packed FP32)",
            "achieved_basis": "algorithmic FP32 operations of the sweeps (88 per sphere-contact copy, 74 with a "
                              "static body, 63 per ball joint) over the kernel's HIP-event time",
            "launches": int(head["pgs_launches"]), "ms_per_launch": ms_launch,
            "alg_ops_per_launch": head["pgs_ops"] / launches,
            "busy_cus": busy, "frac_of_busy_cus": ops_rate / (VALU_PEAK_TOPS * busy / N_CUS),
            "alg_bytes_per_launch": head["pgs_bytes"] / launches,
            "alg_bytes_rate_gbs": head["pgs_bytes"] / (pgs_ms * 1e-3) / 1e9 if pgs_ms > 0 else 0.0,
            "measured": None if cnt is None else cnt.get("summary"),
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def other_configs():
    """Fixed-sweep throughput of the four other configurations, each over its
    stated number of steps from its initial state (after 10 warm-up steps)."""
    import torch

    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    out = {}
    for name, make in (("small", scenes.config1), ("bowl", scenes.config2), ("chains", scenes.config3),
                       ("batched", scenes.config4)):
        sc = make(0)
        p = ovl.make_params(dt=sc.dt, max_iters=sc.iters, mode=ovl.MODE_FIXED, warmstart=ovl.WARM_PLAIN)
        w = ovl.World(sc, p)
        owner0 = sc.owner.copy()
        batched = name == "batched"
        cent0 = sc.centroids[0].copy() if (sc.rebalance_every and not batched) else None
        if batched:
            w.set_launch(graph=1)
        w.set_partitions(owner0, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
        w.step(10)
        w.sync()
        reset_run(w, sc, owner0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if batched:
            w.step(sc.steps)         # partitions fixed at the start (one graph-replayed world)
        else:
            run_loop(w, sc, sc.steps, sc.state, owner0, cent0)
        w.sync()
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        st = w.step(0, stats=True)
        w.close()
        out[name] = {"n_bodies": sc.n_bodies, "partitions": int(np.sum(sc.parts_per_scene)),
                     "halo_k": sc.halo_k, "sweeps": sc.iters, "steps": sc.steps, "dt": sc.dt,
                     "body_steps_per_s": sc.n_bodies * sc.steps / secs, "ms_per_step": 1e3 * secs / sc.steps,
                     "contacts_last": st["n_contacts"], "copies_last": st["n_copies"],
                     "note": ("k-means owners recomputed on the host every 10 steps (inside the timed loop)"
                              if cent0 is not None else ("one world, graph-replayed steps, default launch"
                                                         if batched else "owners fixed"))}
        log(f"[{name}] {out[name]['body_steps_per_s']:.3e} body-steps/s, {out[name]['ms_per_step']:.3f} ms/step")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["tower", "bowl", "bowl-lb", "batched", "accuracy"], default="tower")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps first (default 10; batched: 150, so the piles have formed)")
    ap.add_argument("--mode", choices=["adaptive", "fixed"], default="adaptive")
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--cap", type=int, default=1000)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--no-ladder", action="store_true", help="tower/bowl: time only the head tolerance")
    ap.add_argument("--no-configs", action="store_true", help="tower/bowl: leave out the other configurations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--warm", choices=["plain", "learned", "both"], default="both",
                    help="warm start of the timed run; 'both' times plain then learned and reports learned")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2403_17261_amd", "data", "warmstart_mlp.npz"))
    ap.add_argument("--skip-loop", action="store_true", help="batched: leave out the per-scene loop")
    ap.add_argument("--repeats", type=int, default=3, help="batched: timed runs per launch, in alternation")
    ap.add_argument("--seeds", default="0,1,2", help="accuracy: scene seeds, comma-separated")
    ap.add_argument("--coupling", nargs="?", const="impulse", default="none", choices=["none", "impulse", "split"],
                    help="tower/bowl: interface coupling, by the previous step's impulses of cut constraints "
                         "(impulse) or by splitting the mass of overlap bodies (split)")
    ap.add_argument("--exact-every", type=int, default=5,
                    help="tower/bowl: after timing, replay the run untimed with the exact residual every this many "
                         "steps (0: off)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB five times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU; a run on several GPUs is not provided "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 5}))
        return
    if args.workload == "bowl-lb":
        bench_bowl_lb(args)
        return
    if args.workload == "accuracy":
        bench_accuracy(args)
        return
    if args.workload == "batched":
        if args.warmup is None:
            args.warmup = 150
        bench_batched(args)
        return
    if args.warmup is None:
        args.warmup = 10
    bench_tower(args)


if __name__ == "__main__":
    main()
