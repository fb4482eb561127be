"""Training pipeline of the learned warm start (runs on the GPU).

1. collect(): step bowl-pile scenes (seeded 100..131) in adaptive mode with
   the feature export on and keep, every few steps, each contact copy's
   twelve features and its final impulses divided by the impulse scale s.
2. fit(): Adam on the device trainer (``ovl_mlp_train_step``); PyTorch only
   holds the rows on the device and draws the shuffles.
3. The parameters go to ``data/warmstart_mlp.npz`` with the training record.

    python -m paper_2403_17261_amd.warmstart [--seeds 100-131] [--bodies 4000]
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


def collect(seeds, n_bodies=4000, steps=300, start=140, every=10, tol=1e-4, cap=1000):
    import paper_2403_17261_amd as ovl
    from paper_2403_17261_amd import scenes

    Xs, Ts = [], []
    for sd in seeds:
        blk = scenes.bowl_scene(n_bodies, sd, 4, scale=(n_bodies / 20000.0) ** (1.0 / 3.0))
        sc = scenes._assemble([blk], f"bowl-{n_bodies}-seed{sd}", halo_k=2, beta=4, dt=1 / 60, iters=30,
                              steps=steps, rebalance_every=10)
        p = ovl.make_params(dt=sc.dt, max_iters=cap, mode=ovl.MODE_ADAPTIVE, tol=tol, warmstart=ovl.WARM_PLAIN)
        w = ovl.World(sc, p)
        w.set_partitions(sc.owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
        w.set_feature_export(True)
        owner, cent = sc.owner, blk["centroids"]
        t0 = time.time()
        rows = 0
        for t in range(steps):
            if t > 0 and t % 10 == 0:
                st = w.read_state()
                owner, cent = scenes.kmeans_owner(st[:, :3], 4, iters=3, centroids=cent)
                w.set_partitions(owner, sc.parts_per_scene, halo_k=sc.halo_k, beta=sc.beta)
            w.step(1)
            if t >= start and (t - start) % every == 0:
                X, T = w.training_rows()
                ok = np.isfinite(X).all(1) & np.isfinite(T).all(1)
                Xs.append(X[ok])
                Ts.append(T[ok])
                rows += int(ok.sum())
        w.close()
        log(f"seed {sd}: {rows} rows in {time.time() - t0:.1f} s")
    return np.concatenate(Xs), np.concatenate(Ts)


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
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    a, b = (int(x) for x in args.seeds.split("-"))
    seeds = list(range(a, b + 1))
    tr_seeds, va_seeds = seeds[:-args.val], seeds[-args.val:]
    t0 = time.time()
    X, T = collect(tr_seeds, args.bodies)
    Xv, Tv = collect(va_seeds, args.bodies)
    log(f"collected {len(X)} training and {len(Xv)} validation rows in {time.time() - t0:.0f} s")
    # baseline: predicting the plain start (lambda_n from the previous step, no friction)
    base = np.zeros_like(Tv)
    base[:, 0] = Xv[:, 9]
    base_loss = float(((base - Tv) ** 2).mean())
    params, hist = fit(X, T, Xv, Tv, epochs=args.epochs)
    rec = {"train_seeds": tr_seeds, "val_seeds": va_seeds, "bodies": args.bodies, "rows": int(len(X)),
           "val_rows": int(len(Xv)), "history": hist, "val_loss_plain_start": base_loss,
           "seconds": time.time() - t0}
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.savez(args.out, params=params.astype(np.float32), record=json.dumps(rec))
    log(json.dumps(rec))
    print(json.dumps({"weights": args.out, **{k: rec[k] for k in ("rows", "val_rows", "val_loss_plain_start")},
                      "val_loss": hist[-1]["val_loss"]}))


def load(path=WEIGHTS):
    d = np.load(path, allow_pickle=False)
    return d["params"], json.loads(str(d["record"]))


if __name__ == "__main__":
    main()
