"""Per-architecture cache of the solver's autotuned launch configuration.

``ovl_autotune`` times every candidate launch configuration of the solve
(threads per partition workgroup and LDS tile, each with and without the
persistent queue) on one step of a world and keeps the fastest; every
candidate must give the same bits.  This module keeps its choice in a JSON file
per GPU architecture, keyed by the world's shape (scenes, partitions, bodies
to two significant digits, capsules, joints), so that a world of the same
shape starts from the cached launch instead of tuning again.

    launch = tuned_launch(world, scene)        # tunes on a miss, else applies the cached entry
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_DIR = os.path.join(HERE, "data")


def arch_name(device: int = 0) -> str:
    """The GPU architecture (e.g. gfx950), without feature suffixes."""
    import torch

    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def signature(scene) -> str:
    n = int(scene.n_bodies)
    n2 = 0 if n == 0 else int(round(n, 1 - int(math.floor(math.log10(n)))))
    caps = int(np.any(np.asarray(scene.shape) == 1))
    joints = int(np.asarray(scene.joint_ab).reshape(-1, 2).shape[0])
    return (f"scenes={int(scene.n_scenes)} partitions={int(np.sum(scene.parts_per_scene))} bodies~{n2} "
            f"capsules={caps} joints={'yes' if joints else 'no'}")


def cache_path(arch: str, directory: str = DEFAULT_DIR) -> str:
    return os.path.join(directory, f"autotune_{arch}.json")


def load(arch: str, directory: str = DEFAULT_DIR) -> dict:
    try:
        with open(cache_path(arch, directory)) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned_launch(world, scene, trials: int = 3, directory: str = DEFAULT_DIR, graph: int | None = None):
    """Apply the cached launch of this architecture and world shape, or tune and
    record it.  Returns (launch config dict, candidate times in ms or None when
    cached, True if it came from the cache)."""
    arch = arch_name()
    key = signature(scene)
    cache = load(arch, directory)
    g = world.get_launch()["graph"] if graph is None else int(graph)
    if key in cache:
        c = cache[key]
        world.set_launch(pgs_block=c["pgs_block"], pgs_lds_reps=c["pgs_lds_reps"], persistent=c["persistent"],
                         graph=g)
        return world.get_launch(), None, True
    chosen, ms = world.autotune(trials=trials)
    cache[key] = {k: int(chosen[k]) for k in ("pgs_block", "pgs_lds_reps", "persistent")}
    cache[key]["candidates_ms"] = [round(float(x), 4) for x in ms]
    os.makedirs(directory, exist_ok=True)
    tmp = cache_path(arch, directory) + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, cache_path(arch, directory))
    return world.get_launch(), ms, False
