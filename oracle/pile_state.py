"""Write the settled bowl-pile state used as the CPU-baseline sample.

Runs the oracle alone (no GPU code) on the 20,000-sphere bowl pile (seed 0)
for STEPS steps with the scene's fixed sweep count, the warm-start cache
carried along and k-means owners recomputed every 10 steps, and stores the
final float32 state, owners and centroids in ``oracle/data/``.

    python oracle/pile_state.py [steps]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2403_17261_amd import scenes  # noqa: E402

OUT = os.path.join(ROOT, "oracle", "data")


def main(steps: int = 300, seed: int = 0, n: int = 20000):
    sc = scenes.config2(seed, n=n)
    st = sc.state.copy()
    owner = sc.owner.copy()
    cent = sc.centroids[0]
    cache = None
    t0 = time.time()
    for t in range(steps):
        if t > 0 and t % sc.rebalance_every == 0:
            owner, cent = scenes.kmeans_owner(st[:, :3], int(sc.parts_per_scene[0]), centroids=cent)
        o = oracle.step(sc, state=st, owner=owner, cache=cache)
        st = o["state"].astype(np.float32)
        cache = o
        if t % 25 == 0:
            print(f"step {t} contacts {len(o['contact_key'])} t={time.time() - t0:.1f}s", flush=True)
    os.makedirs(OUT, exist_ok=True)
    path = os.path.join(OUT, f"bowl{n // 1000}k_seed{seed}_t{steps}.npz")
    np.savez_compressed(path, state=st, owner=owner.astype(np.int32), centroids=cent, steps=steps, seed=seed)
    print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 300)
