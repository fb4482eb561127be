"""Training pipeline of the learned warm start (runs on the GPU).

1. collect(): step bowl-pile scenes (seeded 100..131) in adaptive mode with
   the feature export on and keep, every few steps, each contact copy's
   twelve features and its final impulses divided by the impulse scale s,
   from the partitions whose sweeps reached the tolerance (a partition stopped
   by the sweep cap has impulses that are not the solution it should learn).
2. fit(): Adam on the device trainer (``ovl_mlp_train_step``); PyTorch only
   holds the rows on the device and draws the shuffles.
3. The parameters go to ``data/warmstart_mlp.npz`` with the training record.

    python -m paper_2403_17261_amd.warmstart [--seeds 100-131] [--bodies 4000] [--tol 1e-2]

4. The record also holds the sweeps to tolerance of the plain and the learned
   start from the same states of held-out bowls (evaluate()).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "data", "warmstart_mlp.npz")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def converged_rows(w, tol):
    """Mask over the last step's training rows (contact copies in uid order):
    True where the copy's partition stopped with its sweep residual <= tol."""
    kind = w.debug("copy_kind")
    pco = w.debug("part_copy_off")
    resid = w.debug("part_resid")
    contacts = np.nonzero(kind == 1)[0]
    part = np.searchsorted(pco, contacts, side="right") - 1
    return resid[part] <= tol


def bowl(n_bodies, seed, parts=4, steps=300):
    """A config-2-style bowl pile of n_bodies spheres (geometry scaled to the count)."""
    from paper_2403_17261_amd import scenes

    blk = scenes.bowl_scene(n_bodies, seed, parts, scale=(n_bodies / 20000.0) ** (1.0 / 3.0))
    sc = scenes._assemble([blk], f"bowl-{n_bodies}-seed{seed}", halo_k=2, beta=4, dt=1 / 60, iters=30,
                          steps=steps, rebalance_every=10)
    return sc, blk["centroids"]


def collect(seeds, n_bodies=4000, steps=300, start=140, every=10, tol=1e-4, cap=1000, converged_only=True):
    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    Xs, Ts = [], []
    for sd in seeds:
        sc, cent = bowl(n_bodies, sd, steps=steps)
        p = ovl.make_params(dt=sc.dt, max_iters=cap, mode=ovl.MODE_ADAPTIVE, tol=tol, warmstart=ovl.WARM_PLAIN)
        w = ovl.World(sc, p)
        w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
        w.set_feature_export(True)
        owner = sc.owner
        t0 = time.time()
        rows = dropped = 0
        for t in range(steps):
            if t > 0 and t % 10 == 0:
                st = w.read_state()
                owner, cent = scenes.kmeans_owner(st[:, :3], 4, iters=3, centroids=cent)
                w.set_partitions(owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
            w.step(1)
            if t >= start and (t - start) % every == 0:
                X, T = w.training_rows()
                ok = np.isfinite(X).all(1) & np.isfinite(T).all(1)
                if converged_only:
                    conv = converged_rows(w, tol)
                    dropped += int((ok & ~conv).sum())
                    ok &= conv
                Xs.append(X[ok])
                Ts.append(T[ok])
                rows += int(ok.sum())
        w.close()
        log(f"seed {sd}: {rows} rows ({dropped} from unconverged partitions left out) in {time.time() - t0:.1f} s")
    return np.concatenate(Xs), np.concatenate(Ts)


def ab_sweeps(w, params):
    """From the world's current state and warm-start cache, one step with the
    plain start and one with the learned start (guarded), each from the same
    state and cache; the state and cache are restored.  Returns the partitions'
    sweep counts and sweep residuals (plain, learned)."""
    import paper_2403_17261_amd as ovl

    s, c = w.read_state(), w.cache()
    out = []
    for mode in (ovl.WARM_PLAIN, ovl.WARM_LEARNED):
        w.set_warmstart(mode, params if mode == ovl.WARM_LEARNED else None)
        w.step(1, stats=True)
        out.append((w.debug("part_iters").copy(), w.debug("part_resid").copy()))
        w.write_state(s, keep_cache=False)
        w.write_cache(c)
    w.set_warmstart(ovl.WARM_PLAIN)
    return out


def evaluate(params, seeds, n_bodies=4000, steps=300, start=140, every=5, tol=1e-4, cap=1000):
    """Sweeps to tol of the plain and the learned start on the same states: bowl
    piles of the given seeds stepped with the plain start; every `every` steps
    from `start` on, the next step is taken both ways from the same state and
    cache.  Returns per-partition-step sweep counts and convergence flags."""
    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    res = {"plain": [], "learned": [], "plain_conv": [], "learned_conv": []}
    for sd in seeds:
        sc, cent = bowl(n_bodies, sd, steps=steps)
        p = ovl.make_params(dt=sc.dt, max_iters=cap, mode=ovl.MODE_ADAPTIVE, tol=tol, warmstart=ovl.WARM_PLAIN)
        w = ovl.World(sc, p)
        w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
        G = int(np.sum(sc.parts_per_scene))
        for t in range(steps):
            if t > 0 and t % 10 == 0:
                owner, cent = scenes.kmeans_owner(w.read_state()[:, :3], G, iters=3, centroids=cent)
                w.set_partitions(owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
            if t >= start and (t - start) % every == 0:
                (ip, rp), (il, rl) = ab_sweeps(w, params)
                res["plain"] += ip.tolist()
                res["learned"] += il.tolist()
                res["plain_conv"] += (rp <= tol).tolist()
                res["learned_conv"] += (rl <= tol).tolist()
            w.step(1)
        w.close()
    return {k: np.array(v) for k, v in res.items()}


def _val_loss(params, Xv, Tv):
    import paper_2403_17261_amd as ovl

    y = ovl.ovl_mlp_infer(params, Xv)
    return float(((y - Tv) ** 2).mean())


def fit(X, T, Xv, Tv, init_seed=0, epochs=4, batch=4096, lr=1e-3, seed=0):
    """Adam on the device trainer; returns (params, record)."""
    import torch

    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    dev = torch.device("cuda", torch.cuda.current_device())
    Xd = torch.from_numpy(X).to(dev)
    Td = torch.from_numpy(T).to(dev)
    tr = ovl.Trainer(scenes.mlp_initial_weights(init_seed), stream=torch.cuda.current_stream().cuda_stream)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    n = X.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, device=dev, generator=g)
        losses = []
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            xb = Xd.index_select(0, idx).contiguous()
            tb = Td.index_select(0, idx).contiguous()
            losses.append(tr.step(xb, tb, lr * (0.5 ** ep)))
        params = tr.params()
        vl = _val_loss(params, Xv, Tv)
        hist.append({"epoch": ep, "train_loss": float(np.mean(losses)), "val_loss": vl})
        log(f"epoch {ep}: train {np.mean(losses):.5f} val {vl:.5f}")
    return tr.params(), hist


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", default="100-131")
    ap.add_argument("--val", type=int, default=4, help="the last this many seeds are held out")
    ap.add_argument("--bodies", type=int, default=4000)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--tol", type=float, default=1e-2,
                    help="sweep tolerance of the collection runs; rows come only from partitions that reach it")
    ap.add_argument("--eval-seeds", default="140-143", help="held-out bowls for the sweep comparison")
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    a, b = (int(x) for x in args.seeds.split("-"))
    seeds = list(range(a, b + 1))
    tr_seeds, va_seeds = seeds[:-args.val], seeds[-args.val:]
    a, b = (int(x) for x in args.eval_seeds.split("-"))
    ev_seeds = list(range(a, b + 1))
    t0 = time.time()
    X, T = collect(tr_seeds, args.bodies, tol=args.tol)
    Xv, Tv = collect(va_seeds, args.bodies, tol=args.tol)
    log(f"collected {len(X)} training and {len(Xv)} validation rows in {time.time() - t0:.0f} s")
    # baseline: predicting the plain start (lambda_n from the previous step, no friction)
    base = np.zeros_like(Tv)
    base[:, 0] = Xv[:, 9]
    base_loss = float(((base - Tv) ** 2).mean())
    params, hist = fit(X, T, Xv, Tv, epochs=args.epochs)
    # what the network changes: sweeps to the tolerance from the same states, plain against learned
    sweeps = {}
    for tol in sorted({args.tol, 3e-3}, reverse=True):
        r = evaluate(params, ev_seeds, n_bodies=args.bodies, every=10, tol=tol)
        sweeps[f"{tol:g}"] = {"partition_steps": int(len(r["plain"])),
                              "plain_mean_sweeps": float(r["plain"].mean()),
                              "learned_mean_sweeps": float(r["learned"].mean()),
                              "plain_converged": float(r["plain_conv"].mean()),
                              "learned_converged": float(r["learned_conv"].mean())}
        log(f"held-out sweeps at {tol:g}: {json.dumps(sweeps[f'{tol:g}'])}")
    rec = {"train_seeds": tr_seeds, "val_seeds": va_seeds, "eval_seeds": ev_seeds, "bodies": args.bodies,
           "collection_tol": args.tol, "converged_rows_only": True, "rows": int(len(X)),
           "val_rows": int(len(Xv)), "history": hist, "val_loss_plain_start": base_loss,
           "held_out_sweeps": sweeps, "seconds": time.time() - t0}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.savez(args.out, params=params.astype(np.float32), record=json.dumps(rec))
    log(json.dumps(rec))
    print(json.dumps({"weights": args.out, **{k: rec[k] for k in ("rows", "val_rows", "val_loss_plain_start")},
                      "val_loss": hist[-1]["val_loss"], "held_out_sweeps": sweeps}))


def load(path=WEIGHTS):
    d = np.load(path, allow_pickle=False)
    return d["params"], json.loads(str(d["record"]))


if __name__ == "__main__":
    main()
