"""Seeded synthetic scene generators (inputs only).

This module produces the inputs that both the GPU library and the CPU oracle
consume: body geometry and mass properties, initial states, static geometry,
ball joints and an initial partition ("owner") per body.  It contains none of
the method's arithmetic (no contacts, no graph, no solve, no blending).

The scenes stand in for the paper's Bowl, articulated-chain and collapse
workloads (section 6, Table 2), whose assets are not published.  Every draw
comes from ``numpy.random.Generator(PCG64(seed))``.

State layout per body (13 float32): x(3), q(4; w first), v(3), w(3), all in
the world frame, as in the paper's generalised state (section 4, Eq. 8).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SHAPE_SPHERE = 0
SHAPE_CAPSULE = 1


@dataclasses.dataclass
class Scene:
    """A world: one or more independent scenes stored back to back.

    Bodies are sorted by ``scene``.  Static planes and static spheres are
    listed per scene through CSR offsets.  Joints join two bodies of the same
    scene and are sorted by scene.
    """

    scene: np.ndarray          # int32 [N]
    shape: np.ndarray          # int32 [N]
    radius: np.ndarray         # float32 [N]
    halflen: np.ndarray        # float32 [N]   (capsules: half segment length along body z)
    mass: np.ndarray           # float32 [N]
    inertia: np.ndarray        # float32 [N,3] body-frame principal moments
    state: np.ndarray          # float32 [N,13]
    mu: np.ndarray             # float32 [S]
    margin: np.ndarray         # float32 [S]
    plane_off: np.ndarray      # int32 [S+1]
    planes: np.ndarray         # float32 [P,4]  (nx, ny, nz, c): n.x = c, n points into the free side
    ssph_off: np.ndarray       # int32 [S+1]
    ssph: np.ndarray           # float32 [Q,4]  (x, y, z, r)
    joint_ab: np.ndarray       # int32 [J,2]
    joint_anchor: np.ndarray   # float32 [J,6]  body-frame anchors on a then b
    owner: np.ndarray          # int32 [N] global partition id of every body
    parts_per_scene: np.ndarray  # int32 [S]
    halo_k: int = 1
    beta: int = 4
    dt: float = 1.0 / 60.0
    iters: int = 20
    steps: int = 200
    name: str = ""
    rebalance_every: int = 0   # >0: k-means owners are recomputed every this many steps

    @property
    def n_bodies(self) -> int:
        return int(self.radius.shape[0])

    @property
    def n_scenes(self) -> int:
        return int(self.mu.shape[0])

    @property
    def n_parts(self) -> int:
        return int(self.parts_per_scene.sum())

    def copy(self) -> "Scene":
        return dataclasses.replace(
            self, **{f.name: (getattr(self, f.name).copy() if isinstance(getattr(self, f.name), np.ndarray)
                              else getattr(self, f.name)) for f in dataclasses.fields(self)})


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sphere_inertia(mass: np.ndarray, radius: np.ndarray) -> np.ndarray:
    """Principal moments of a solid sphere, 2/5 m r^2 on every axis."""
    i = (0.4 * mass.astype(np.float64) * radius.astype(np.float64) ** 2)
    return np.repeat(i[:, None], 3, axis=1).astype(np.float32)


def capsule_mass_inertia(radius: float, halflen: float, density: float):
    """Mass and body-frame principal moments of a solid capsule (axis = body z).

    Cylinder of length 2*halflen plus two hemispherical caps (standard
    composite-body formula with the parallel-axis shift of each cap).
    """
    r, h = float(radius), 2.0 * float(halflen)
    mc = density * math.pi * r * r * h
    ms = density * 4.0 / 3.0 * math.pi * r ** 3          # both caps together
    izz = mc * r * r / 2.0 + ms * 2.0 * r * r / 5.0
    # caps: each hemisphere (mass ms/2) about its own centroid, shifted to the capsule centre
    ihem_c = (83.0 / 320.0) * (ms / 2.0) * r * r          # hemisphere about centroid, transverse axis
    d = h / 2.0 + 3.0 * r / 8.0
    ixx = mc * (r * r / 4.0 + h * h / 12.0) + 2.0 * (ihem_c + (ms / 2.0) * d * d)
    return mc + ms, np.array([ixx, ixx, izz], dtype=np.float64)


def capsule_inertia_for_mass(mass: float, radius: float, halflen: float) -> np.ndarray:
    """Principal moments of a uniform solid capsule of the given mass."""
    m1, i1 = capsule_mass_inertia(radius, halflen, 1.0)
    return (i1 * (float(mass) / m1)).astype(np.float32)


def random_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniformly distributed unit quaternions (w, x, y, z): normalised 4-D Gaussians, w >= 0."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1.0
    return q.astype(np.float32)


def _identity_state(pos: np.ndarray) -> np.ndarray:
    n = pos.shape[0]
    st = np.zeros((n, 13), dtype=np.float32)
    st[:, 0:3] = pos.astype(np.float32)
    st[:, 3] = 1.0
    return st


def _empty_statics(n_scenes: int):
    return (np.zeros(n_scenes + 1, np.int32), np.zeros((0, 4), np.float32))


def _assemble(parts: list, name: str, **kw) -> Scene:
    """Concatenate per-scene dicts into one world (bodies sorted by scene)."""
    S = len(parts)
    n_off = np.cumsum([0] + [p["radius"].shape[0] for p in parts])
    part_off = np.cumsum([0] + [p["n_parts"] for p in parts])
    cat = lambda k, dt: np.concatenate([p[k] for p in parts]).astype(dt) if parts else np.zeros(0, dt)
    scene = np.concatenate([np.full(p["radius"].shape[0], s, np.int32) for s, p in enumerate(parts)])
    planes = [p.get("planes", np.zeros((0, 4), np.float32)) for p in parts]
    ssph = [p.get("ssph", np.zeros((0, 4), np.float32)) for p in parts]
    joints = [p.get("joint_ab", np.zeros((0, 2), np.int32)) + n_off[s] for s, p in enumerate(parts)]
    janch = [p.get("joint_anchor", np.zeros((0, 6), np.float32)) for p in parts]
    owner = np.concatenate([p["owner"].astype(np.int64) + part_off[s] for s, p in enumerate(parts)])
    return Scene(
        scene=scene,
        shape=cat("shape", np.int32),
        radius=cat("radius", np.float32),
        halflen=cat("halflen", np.float32),
        mass=cat("mass", np.float32),
        inertia=np.concatenate([p["inertia"] for p in parts]).astype(np.float32).reshape(-1, 3),
        state=np.concatenate([p["state"] for p in parts]).astype(np.float32).reshape(-1, 13),
        mu=np.array([p["mu"] for p in parts], np.float32),
        margin=np.array([p["margin"] for p in parts], np.float32),
        plane_off=np.cumsum([0] + [x.shape[0] for x in planes]).astype(np.int32),
        planes=(np.concatenate(planes) if S else np.zeros((0, 4))).astype(np.float32).reshape(-1, 4),
        ssph_off=np.cumsum([0] + [x.shape[0] for x in ssph]).astype(np.int32),
        ssph=(np.concatenate(ssph) if S else np.zeros((0, 4))).astype(np.float32).reshape(-1, 4),
        joint_ab=np.concatenate(joints).astype(np.int32).reshape(-1, 2),
        joint_anchor=np.concatenate(janch).astype(np.float32).reshape(-1, 6),
        owner=owner.astype(np.int32),
        parts_per_scene=np.array([p["n_parts"] for p in parts], np.int32),
        name=name,
        **kw,
    )


def _sphere_block(pos, radius, mass):
    n = pos.shape[0]
    radius = np.broadcast_to(np.asarray(radius, np.float32), (n,)).copy()
    mass = np.broadcast_to(np.asarray(mass, np.float32), (n,)).copy()
    return dict(
        shape=np.zeros(n, np.int32), radius=radius, halflen=np.zeros(n, np.float32), mass=mass,
        inertia=sphere_inertia(mass, radius), state=_identity_state(pos))


GROUND = np.array([[0.0, 0.0, 1.0, 0.0]], np.float32)


# --------------------------------------------------------------------------------------------
# Partitioners (inputs: the paper starts from an approximate, user- or naively-chosen division)
# --------------------------------------------------------------------------------------------

def kmeans_owner(pos: np.ndarray, k: int, iters: int = 10, centroids: Optional[np.ndarray] = None,
                 seed: int = 0):
    """Spatial k-means (Lloyd) in float64, used only to produce owner arrays.

    Initial centroids are the positions of the first ``k`` bodies of a seeded
    permutation; later calls pass the previous centroids.  Ties go to the
    lowest centroid index (``argmin``).  Returns (owner int32, centroids).
    """
    p = pos.astype(np.float64)
    n = p.shape[0]
    k = max(1, min(k, n)) if n else max(1, k)
    if n == 0:
        return np.zeros(0, np.int32), np.zeros((k, 3))
    if centroids is None:
        perm = _rng(seed).permutation(n)
        centroids = p[perm[:k]].copy()
    c = centroids.astype(np.float64).copy()
    lab = np.zeros(n, np.int64)
    p2 = (p * p).sum(1)
    for _ in range(iters):
        d2 = p2[:, None] - 2.0 * (p @ c.T) + (c * c).sum(1)[None, :]
        lab = np.argmin(d2, axis=1)
        cnt = np.bincount(lab, minlength=c.shape[0])
        for ax in range(3):
            s_ = np.bincount(lab, weights=p[:, ax], minlength=c.shape[0])
            c[:, ax] = np.where(cnt > 0, s_ / np.maximum(cnt, 1), c[:, ax])
    return lab.astype(np.int32), c


# --------------------------------------------------------------------------------------------
# Configurations
# --------------------------------------------------------------------------------------------

def lattice_stack(nx=4, ny=4, nz=4, spacing=1.0, radius=0.5, mass=1.0, jitter=0.01, mu=0.5,
                  seed=0, owner_fn=None, n_parts=2, margin=None):
    rng = _rng(seed)
    ii, jj, ll = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = np.stack([ii.ravel(), jj.ravel(), ll.ravel()], 1).astype(np.float64)
    pos = radius + spacing * base + rng.uniform(-jitter, jitter, size=base.shape)
    blk = _sphere_block(pos.astype(np.float32), radius, mass)
    owner = owner_fn(pos) if owner_fn is not None else np.zeros(pos.shape[0], np.int32)
    blk.update(planes=GROUND.copy(), mu=mu, margin=np.float32(0.05 * radius if margin is None else margin),
               owner=np.asarray(owner, np.int32), n_parts=n_parts)
    return blk


def config1(seed: int = 0) -> Scene:
    """64 unit spheres in a 4x4x4 stacked lattice on a ground plane, two slabs split at x = 2."""
    blk = lattice_stack(4, 4, 4, 1.0, 0.5, 1.0, 0.01, 0.5, seed,
                        owner_fn=lambda p: (p[:, 0] >= 2.0).astype(np.int32), n_parts=2)
    return _assemble([blk], "small-lattice-64", halo_k=1, beta=4, dt=1 / 60, iters=20, steps=200)


def bowl_planes(half=20.0, incline_deg=60.0) -> np.ndarray:
    """Floor z = 0 plus four walls through the base edges leaning outward."""
    s, c = math.sin(math.radians(incline_deg)), math.cos(math.radians(incline_deg))
    return np.array([
        [0.0, 0.0, 1.0, 0.0],
        [-s, 0.0, c, -s * half],
        [s, 0.0, c, -s * half],
        [0.0, -s, c, -s * half],
        [0.0, s, c, -s * half],
    ], np.float32)


def bowl_scene(n: int, seed: int, n_parts: int, scale: float = 1.0, mu: float = 0.6,
               rmin=0.2, rmax=0.5, density=1000.0, spacing=1.2):
    """Spheres with radius U(rmin, rmax) dropped from random, non-overlapping positions.

    Positions: a random subset of the sites of a lattice with the given spacing
    covering |x|,|y| <= 19.5 s, z in [1, 60 s] (s = scale), each jittered by
    U(+-(spacing - 2 rmax - margin)/2) per axis, so no two spheres start
    closer than 2 rmax + margin.
    """
    rng = _rng(seed)
    margin = 0.05 * rmin
    hx, z0, z1 = 19.5 * scale, 1.0, 1.0 + 59.0 * scale
    gx = np.arange(-hx + rmax, hx - rmax + 1e-9, spacing)
    gz = np.arange(z0 + rmax, z1 - rmax + 1e-9, spacing)
    nsite = gx.size * gx.size * gz.size
    while nsite < n:  # tiny scales: densify the lattice (still overlap-free: spacing >= 2 rmax + margin)
        spacing = max(2 * rmax + margin + 1e-3, spacing * 0.95)
        gx = np.arange(-hx + rmax, hx - rmax + 1e-9, spacing)
        gz = np.arange(z0 + rmax, z1 - rmax + 1e-9, spacing)
        nsite = gx.size * gx.size * gz.size
        if spacing <= 2 * rmax + margin + 1e-3 and nsite < n:
            z1 *= 1.25
    sites = rng.choice(nsite, size=n, replace=False)
    iz, rem = np.divmod(sites, gx.size * gx.size)
    iy, ix = np.divmod(rem, gx.size)
    pos = np.stack([gx[ix], gx[iy], gz[iz]], 1)
    jit = max(0.0, (spacing - 2 * rmax - margin) / 2.0 - 1e-4)
    pos = pos + rng.uniform(-jit, jit, size=pos.shape)
    radius = rng.uniform(rmin, rmax, size=n)
    mass = density * 4.0 / 3.0 * math.pi * radius ** 3
    blk = _sphere_block(pos.astype(np.float32), radius.astype(np.float32), mass.astype(np.float32))
    owner, cent = kmeans_owner(blk["state"][:, :3], n_parts, seed=seed)
    blk.update(planes=bowl_planes(20.0 * scale), mu=mu, margin=np.float32(margin), owner=owner,
               n_parts=int(n_parts))
    blk["centroids"] = cent
    return blk


def capsule_pile(n: int, seed: int, n_parts: int, frac: float = 0.5, scale: float = 1.0, mu: float = 0.6,
                 rmin=0.15, rmax=0.35, hmin=0.15, hmax=0.45, density=1000.0) -> Scene:
    """Bowl pile of mixed spheres and capsules, random orientations.

    Each body is a capsule with probability `frac` (radius U(rmin, rmax),
    half-length U(hmin, hmax)), else a sphere of radius U(rmin, rmax).  Bodies
    start on a jittered lattice whose spacing exceeds twice the largest
    bounding radius (radius + half-length) plus the margin, so none overlap.
    """
    rng = _rng(seed)
    margin = 0.05 * rmin
    R = rmax + hmax
    spacing = 2.0 * R + margin + 0.05
    hx, z0 = 19.5 * scale, 1.0
    gx = np.arange(-hx + R, hx - R + 1e-9, spacing)
    if gx.size == 0:
        gx = np.zeros(1)
    per_layer = gx.size * gx.size
    nz = -(-n // per_layer) + 1
    gz = z0 + R + spacing * np.arange(nz)
    sites = rng.choice(per_layer * nz, size=n, replace=False)
    iz, rem = np.divmod(sites, per_layer)
    iy, ix = np.divmod(rem, gx.size)
    pos = np.stack([gx[ix], gx[iy], gz[iz]], 1)
    pos = pos + rng.uniform(-0.02, 0.02, size=pos.shape)
    radius = rng.uniform(rmin, rmax, size=n)
    is_cap = rng.uniform(size=n) < frac
    hl = np.where(is_cap, rng.uniform(hmin, hmax, size=n), 0.0)
    mass = np.empty(n)
    inertia = np.empty((n, 3))
    for i in range(n):
        if is_cap[i]:
            mass[i], inertia[i] = capsule_mass_inertia(radius[i], hl[i], density)
        else:
            mass[i] = density * 4.0 / 3.0 * math.pi * radius[i] ** 3
            inertia[i] = 0.4 * mass[i] * radius[i] ** 2
    st = _identity_state(pos.astype(np.float32))
    st[:, 3:7] = random_quaternions(rng, n)
    blk = dict(shape=is_cap.astype(np.int32), radius=radius.astype(np.float32), halflen=hl.astype(np.float32),
               mass=mass.astype(np.float32), inertia=inertia.astype(np.float32), state=st)
    owner, cent = kmeans_owner(st[:, :3], n_parts, seed=seed)
    blk.update(planes=bowl_planes(20.0 * scale), mu=mu, margin=np.float32(margin), owner=owner,
               n_parts=int(n_parts))
    sc = _assemble([blk], f"capsule-pile-{n}-seed{seed}", halo_k=2, beta=4, dt=1 / 60, iters=30, steps=300,
                   rebalance_every=10)
    sc.centroids = [cent]
    return sc


def config2(seed: int = 0, n: int = 20000) -> Scene:
    """Bowl pile: spheres r ~ U(0.2, 0.5), density 1000, in a five-plane bowl, 8 k-means parts."""
    blk = bowl_scene(n, seed, 8)
    sc = _assemble([blk], f"bowl-pile-{n}", halo_k=2, beta=4, dt=1 / 60, iters=30, steps=1000,
                   rebalance_every=10)
    sc.centroids = [blk["centroids"]]
    return sc


def bowl_naive(n: int = 5040, seed: int = 0, n_parts: int = 7, scale: Optional[float] = None,
               squeeze: float = 1.0) -> Scene:
    """Bowl pile started from the naive division of section 5.4 (the body list
    cut into equal runs, one per worker), for dynamic load balancing with
    growth depth 0.  Default size: 5040 spheres and 7 workers.  ``squeeze`` < 1
    pulls the drop positions towards the bowl's floor centre so that the pile
    is in contact from the first step (small test cases)."""
    if scale is None:
        scale = (n / 20000.0) ** (1.0 / 3.0)
    blk = bowl_scene(n, seed, n_parts, scale=scale)
    if squeeze != 1.0:
        st = blk["state"]
        st[:, :3] *= np.float32(squeeze)
        st[:, 2] += np.float32(0.5)
    blk["owner"] = (np.arange(n, dtype=np.int64) * n_parts // max(n, 1)).astype(np.int32)
    return _assemble([blk], f"bowl-naive-{n}", halo_k=0, beta=4, dt=1 / 60, iters=30, steps=1000)


def chains_scene(n_chains=256, links=200, seed=0, n_parts=16, radius=0.1, mass=0.5,
                 x_extent=20.0, n_static=16):
    rng = _rng(seed)
    spacing = 2 * radius
    xs = -x_extent + radius + spacing * np.arange(links)
    pos, ab = [], []
    for j in range(n_chains):
        y = -8.0 + (j % 16) + rng.uniform(-0.1, 0.1)
        z = 12.0 + 0.4 * (j // 16)
        p = np.stack([xs, np.full(links, y), np.full(links, z)], 1)
        pos.append(p)
        base = j * links
        ab.append(np.stack([base + np.arange(links - 1), base + np.arange(1, links)], 1))
    pos = np.concatenate(pos) if pos else np.zeros((0, 3))
    ab = np.concatenate(ab) if ab else np.zeros((0, 2), np.int64)
    blk = _sphere_block(pos.astype(np.float32), radius, mass)
    anchors = np.zeros((ab.shape[0], 6), np.float32)
    anchors[:, 0] = radius
    anchors[:, 3] = -radius
    sr = rng.uniform(1.0, 3.0, size=n_static)
    sxy = np.stack([rng.uniform(-16, 16, n_static), rng.uniform(-8, 8, n_static)], 1)
    ssph = np.concatenate([sxy, sr[:, None], sr[:, None]], 1).astype(np.float32)
    width = 2 * x_extent / n_parts
    owner = np.clip(np.floor((pos[:, 0] + x_extent) / width), 0, n_parts - 1).astype(np.int32)
    blk.update(planes=GROUND.copy(), ssph=ssph, joint_ab=ab.astype(np.int32), joint_anchor=anchors,
               mu=0.5, margin=np.float32(0.05 * radius), owner=owner, n_parts=n_parts)
    return blk


def config3(seed: int = 0, n_chains: int = 256, links: int = 200) -> Scene:
    """256 chains of 200 ball-jointed spheres draped over 16 static spheres, 16 x-slabs."""
    blk = chains_scene(n_chains, links, seed)
    return _assemble([blk], f"chains-{n_chains}x{links}", halo_k=3, beta=4, dt=1 / 120, iters=40,
                     steps=500)


def config4(seed: int = 0, n_scenes: int = 512, nmin: int = 200, nmax: int = 5000) -> Scene:
    """Many independent bowl scenes of log-uniform size with 1..6 k-means partitions each."""
    rng = _rng(seed)
    ns = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_scenes))).astype(int)
    ps = rng.integers(1, 7, n_scenes)
    parts = [bowl_scene(int(ns[s]), seed * 100003 + s + 1, int(ps[s]), scale=(ns[s] / 20000.0) ** (1 / 3))
             for s in range(n_scenes)]
    sc = _assemble(parts, f"batched-bowls-{n_scenes}", halo_k=2, beta=4, dt=1 / 60, iters=30, steps=200,
                   rebalance_every=10)
    sc.centroids = [p["centroids"] for p in parts]
    return sc


def config5(seed: int = 0, nx=50, ny=50, nz=40, cols=8) -> Scene:
    """Tower of nx*ny*nz spheres (r = 0.25, density 1000) in 8x8 x-y column partitions."""
    r = 0.25
    m = 1000.0 * 4.0 / 3.0 * math.pi * r ** 3
    lx, ly = nx * 2 * r, ny * 2 * r

    def owner_fn(p):
        cx = np.clip(np.floor(p[:, 0] / (lx / cols)), 0, cols - 1)
        cy = np.clip(np.floor(p[:, 1] / (ly / cols)), 0, cols - 1)
        return (cx * cols + cy).astype(np.int32)

    blk = lattice_stack(nx, ny, nz, 2 * r, r, m, 0.005, 0.5, seed, owner_fn=owner_fn, n_parts=cols * cols)
    return _assemble([blk], f"tower-{nx}x{ny}x{nz}", halo_k=2, beta=4, dt=1 / 60, iters=50, steps=300)


def chain_line(n: int, n_parts: int = 2, split: Optional[list] = None, radius=0.5, mass=1.0,
               joints: bool = True, z: float = 5.0) -> Scene:
    """A straight ball-jointed chain along x (no ground contact), for membership/weight pins."""
    pos = np.stack([radius + 2 * radius * np.arange(n), np.zeros(n), np.full(n, z)], 1)
    blk = _sphere_block(pos.astype(np.float32), radius, mass)
    if split is None:
        owner = (np.arange(n) * n_parts // max(n, 1)).astype(np.int32)
    else:
        owner = np.asarray(split, np.int32)
    ab = np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32) if joints else np.zeros((0, 2), np.int32)
    anch = np.zeros((ab.shape[0], 6), np.float32)
    anch[:, 0] = radius
    anch[:, 3] = -radius
    blk.update(planes=np.zeros((0, 4), np.float32), joint_ab=ab, joint_anchor=anch, mu=0.5,
               margin=np.float32(0.05 * radius), owner=owner, n_parts=n_parts)
    return _assemble([blk], f"chain-{n}", halo_k=1, beta=4)


def custom_spheres(pos, radius, mass, vel=None, omega=None, planes=None, ssph=None, mu=0.5,
                   margin=None, owner=None, n_parts=1, joint_ab=None, joint_anchor=None, quat=None,
                   halflen=None, **kw) -> Scene:
    """Hand-placed spheres (small test problems).  Bodies with halflen > 0 are
    capsules along their body z axis, with the solid-capsule inertia of their mass."""
    pos = np.asarray(pos, np.float32).reshape(-1, 3)
    n = pos.shape[0]
    blk = _sphere_block(pos, radius, mass)
    if halflen is not None:
        hl = np.broadcast_to(np.asarray(halflen, np.float32), (n,)).copy()
        for i in np.nonzero(hl > 0)[0]:
            blk["shape"][i] = 1
            blk["halflen"][i] = hl[i]
            blk["inertia"][i] = capsule_inertia_for_mass(blk["mass"][i], blk["radius"][i], hl[i])
    if vel is not None:
        blk["state"][:, 7:10] = np.asarray(vel, np.float32).reshape(-1, 3)
    if omega is not None:
        blk["state"][:, 10:13] = np.asarray(omega, np.float32).reshape(-1, 3)
    if quat is not None:
        blk["state"][:, 3:7] = np.asarray(quat, np.float32).reshape(-1, 4)
    blk.update(planes=np.zeros((0, 4), np.float32) if planes is None else np.asarray(planes, np.float32),
               ssph=np.zeros((0, 4), np.float32) if ssph is None else np.asarray(ssph, np.float32),
               mu=mu, margin=np.float32((0.05 * float(np.min(blk["radius"])) if n else 0.025) if margin is None
                                        else margin),
               owner=np.zeros(n, np.int32) if owner is None else np.asarray(owner, np.int32),
               n_parts=n_parts)
    if joint_ab is not None:
        blk["joint_ab"] = np.asarray(joint_ab, np.int32).reshape(-1, 2)
        blk["joint_anchor"] = np.asarray(joint_anchor, np.float32).reshape(-1, 6)
    return _assemble([blk], "custom", **kw)


def concat_scenes(scenes: list, name: str = "concat", **kw) -> Scene:
    """Put several single-scene worlds side by side as independent scenes of one world."""
    parts = []
    for sc in scenes:
        assert sc.n_scenes == 1
        parts.append(dict(shape=sc.shape, radius=sc.radius, halflen=sc.halflen, mass=sc.mass,
                          inertia=sc.inertia, state=sc.state, planes=sc.planes, ssph=sc.ssph,
                          joint_ab=sc.joint_ab, joint_anchor=sc.joint_anchor, mu=float(sc.mu[0]),
                          margin=float(sc.margin[0]), owner=sc.owner, n_parts=int(sc.parts_per_scene[0])))
    return _assemble(parts, name, **kw)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


# --------------------------------------------------------------------------------------------
# Initial weights of the warm-start network (random numbers passed in as inputs)
# --------------------------------------------------------------------------------------------

MLP_SHAPES = [(12, 64), (64,), (64, 64), (64,), (64, 3), (3,)]


def mlp_initial_weights(seed: int = 0) -> np.ndarray:
    """Flat float32 parameters W1, b1, W2, b2, W3, b3: He-normal weights, zero biases."""
    rng = _rng(seed)
    parts = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            parts.append(rng.normal(0.0, math.sqrt(2.0 / shape[0]), size=shape).reshape(-1))
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)
