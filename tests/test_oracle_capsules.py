"""Pins of the oracle's capsule contacts (shape 1) against facts other than itself.

* the closest points of two segments, against an enumeration of the
  candidates of the box-constrained quadratic (interior stationary point and
  the four edges), which is exact and shares nothing with the oracle's
  clamp-and-recompute sequence;
* the reading for parallel segments (contact at the middle of the overlap);
* a horizontal capsule resting on a plane (two end contacts of m g h / 2);
* a tilted capsule touching a plane with one end;
* conservation of linear and angular momentum with gravity off;
* the grid against brute force on a capsule pile;
* the solid-capsule mass properties against numerical integration.
"""
import math

import numpy as np
import pytest

from paper_2403_17261_amd import scenes

G = 9.81
# quaternion (w, x, y, z) = (1/2, 1/2, 1/2, 1/2): a 120 degree turn about (1, 1, 1)
# that maps body z exactly onto world x (every component is exact in float)
Q_AXIS_X = [0.5, 0.5, 0.5, 0.5]


def _axis(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([2 * (x * z + w * y), 2 * (y * z - w * x), 1 - 2 * (x * x + y * y)])


def _segment_distance(xa, ua, ha, xb, ub, hb):
    """Minimum of |x_a + s u_a - x_b - t u_b| over |s| <= ha, |t| <= hb, by
    enumerating the candidates of the convex quadratic: the interior
    stationary point (if inside) and the minimum along each of the four edges."""
    r = xa - xb
    a, e, b, c, f = ua @ ua, ub @ ub, ua @ ub, ua @ r, ub @ r
    cands = []
    den = a * e - b * b
    if den > 1e-14:
        s = (b * f - c * e) / den
        t = (a * f - b * c) / den
        if abs(s) <= ha and abs(t) <= hb:
            cands.append((s, t))
    for s in (-ha, ha):
        cands.append((s, float(np.clip((b * s + f) / e, -hb, hb)) if e > 0 else 0.0))
    for t in (-hb, hb):
        cands.append((float(np.clip((b * t - c) / a, -ha, ha)) if a > 0 else 0.0, t))
    best = min(cands, key=lambda st: np.linalg.norm(r + st[0] * ua - st[1] * ub))
    return np.linalg.norm(r + best[0] * ua - best[1] * ub)


def _point_segment_distance(p, x, u, h):
    t = np.clip((p - x) @ u / (u @ u), -h, h)
    return np.linalg.norm(p - (x + t * u))


def _pair(orc, xa, qa, ra, ha, xb, qb, rb, hb, margin=0.02):
    sc = scenes.custom_spheres([xa, xb], [ra, rb], [1.0, 2.0], quat=[qa, qb], halflen=[ha, hb], margin=margin,
                               iters=1)
    return sc, orc.step(sc, gravity=(0, 0, 0), warmstart=False, max_iters=1)


@pytest.mark.parametrize("seed", range(6))
def test_swept_pair_geometry_matches_enumeration(orc, seed):
    rng = np.random.default_rng(100 + seed)
    checked = hits = 0
    for trial in range(60):
        ra, rb = rng.uniform(0.1, 0.4, 2)
        # a capsule against a capsule, a sphere against a capsule, a capsule against a sphere
        kind = trial % 3
        ha = 0.0 if kind == 1 else rng.uniform(0.1, 0.6)
        hb = 0.0 if kind == 2 else rng.uniform(0.1, 0.6)
        qa = scenes.random_quaternions(rng, 1)[0]
        qb = scenes.random_quaternions(rng, 1)[0]
        xa = np.zeros(3, np.float32)
        xb = (rng.normal(size=3) * 0.6).astype(np.float32)
        sc, o = _pair(orc, xa, qa, ra, ha, xb, qb, rb, hb)
        ua, ub = _axis(qa), _axis(qb)
        x64a, x64b = xa.astype(np.float64), xb.astype(np.float64)
        dmin = _segment_distance(x64a, ua, ha, x64b, ub, hb)
        gap = dmin - float(np.float32(ra)) - float(np.float32(rb))
        keys = o["contact_key"]
        if abs(gap - 0.02) < 1e-5:
            continue                                   # too close to the margin to call
        checked += 1
        assert (len(keys) == 1) == (gap < 0.02), (trial, gap, keys)
        if not len(keys):
            continue
        hits += 1
        assert int(keys[0]) == (0 << 32) | (1 << 1)
        phi, n = o["contact_phi"][0], o["contact_n"][0]
        ra_v, rb_v = o["contact_ra"][0], o["contact_rb"][0]
        assert phi == pytest.approx(gap, abs=2e-6)
        assert np.linalg.norm(n) == pytest.approx(1.0, abs=1e-12)
        # the segment points behind the lever arms lie on the segments and are dmin apart along n
        pa = x64a + ra_v - (float(np.float32(ra)) + 0.5 * phi) * n
        pb = x64b + rb_v + (float(np.float32(rb)) + 0.5 * phi) * n
        assert _point_segment_distance(pa, x64a, ua, ha) < 2e-6
        assert _point_segment_distance(pb, x64b, ub, hb) < 2e-6
        assert np.linalg.norm(pb - pa) == pytest.approx(dmin, abs=2e-6)
        if dmin > 1e-3:
            assert np.abs((pb - pa) / np.linalg.norm(pb - pa) - n).max() < 1e-4
        # both lever arms end at the same point (the midpoint of the surface points)
        assert np.abs((x64a + ra_v) - (x64b + rb_v)).max() < 1e-12
    assert checked > 50 and hits > 10


def test_parallel_capsules_touch_at_middle_of_overlap(orc):
    """Reading for parallel segments: the contact sits at the middle of the
    stretch of A that B covers."""
    r, hl, d = 0.2, 0.5, 0.3
    # both along world x; B shifted by d along the axis and 2r - 0.005 sideways
    sc, o = _pair(orc, [0, 0, 0], Q_AXIS_X, r, hl, [d, 0, 2 * r - 0.005], Q_AXIS_X, r, hl)
    assert len(o["contact_key"]) == 1
    mid_s = 0.5 * ((d - hl) + hl)                      # overlap of [-hl, hl] and [d - hl, d + hl]
    ra_v = o["contact_ra"][0]
    assert ra_v[0] == pytest.approx(mid_s, abs=1e-7)
    assert o["contact_n"][0] == pytest.approx([0, 0, 1], abs=1e-7)
    assert o["contact_phi"][0] == pytest.approx(-0.005, abs=1e-7)


def test_horizontal_capsule_rests_on_two_end_contacts(orc):
    h, m, r, hl = 1.0 / 60.0, 2.0, 0.25, 0.5
    sc = scenes.custom_spheres([[0, 0, r]], r, m, quat=[Q_AXIS_X], halflen=[hl], planes=scenes.GROUND, mu=0.5,
                               dt=h, iters=400)
    o = orc.step(sc, warmstart=False)
    keys = o["contact_key"]
    assert len(keys) == 2
    assert [int(k) & 1 for k in keys] == [0, 1]        # sub 0: end at -hl, sub 1: end at +hl
    lam = o["copy_lambda"]
    assert lam[:, 0] == pytest.approx([m * G * h / 2] * 2, rel=1e-9)
    # the friction impulses may hold an internal squeeze along the axis (A is only
    # semi-definite there, so lambda is not unique): only their sum is fixed
    assert np.abs(lam[:, 1:].sum(0)).max() < 1e-12
    assert np.abs(lam[:, 1:]).max() <= 0.5 * m * G * h * 0.5 * (1 + 1e-12)
    assert np.abs(o["state"][0, 7:13]).max() < 1e-10
    # the lever arms of the two contacts: the segment ends, then radius along -z
    assert o["contact_ra"][0] == pytest.approx([-hl, 0, -r], abs=1e-12)
    assert o["contact_ra"][1] == pytest.approx([hl, 0, -r], abs=1e-12)


def test_tilted_capsule_touches_with_lower_end(orc):
    r, hl, ang = 0.2, 0.6, math.radians(30)
    q = [math.cos(ang / 2), 0.0, math.sin(ang / 2), 0.0]      # axis tilted 30 degrees about y
    u = _axis(np.float32(q))
    z = r + hl * abs(u[2]) - 0.001                            # lower end 1 mm into the plane
    sc = scenes.custom_spheres([[0, 0, z]], r, 1.0, quat=[q], halflen=[hl], planes=scenes.GROUND, iters=1)
    o = orc.step(sc, max_iters=1, warmstart=False)
    keys = o["contact_key"]
    assert len(keys) == 1
    lower_sub = 0 if u[2] > 0 else 1                          # the end at -hl u is lower when u_z > 0
    assert int(keys[0]) & 1 == lower_sub
    assert o["contact_phi"][0] == pytest.approx(float(np.float32(z)) - hl * abs(u[2]) - float(np.float32(r)),
                                                abs=1e-7)


def test_capsule_momentum_conserved_one_partition(orc):
    rng = np.random.default_rng(11)
    n = 40
    pos = rng.uniform(0, 3.0, (n, 3)).astype(np.float32)
    rad = rng.uniform(0.25, 0.4, n).astype(np.float32)
    hl = np.where(rng.uniform(size=n) < 0.6, rng.uniform(0.2, 0.5, n), 0.0).astype(np.float32)
    mass = rng.uniform(0.5, 3.0, n).astype(np.float32)
    quat = scenes.random_quaternions(rng, n)
    sc = scenes.custom_spheres(pos, rad, mass, vel=rng.normal(0, 1, (n, 3)), omega=rng.normal(0, 1, (n, 3)),
                               quat=quat, halflen=hl, mu=0.6, iters=30)

    def world_inertia(q, I):
        q = q.astype(np.float64)
        q = q / np.linalg.norm(q)
        w, x, y, z = q
        R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                      [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                      [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
        return R @ np.diag(I.astype(np.float64)) @ R.T

    Iw = [world_inertia(sc.state[i, 3:7], sc.inertia[i]) for i in range(n)]

    def mom(st):
        # angular momentum with the start-of-step orientations: the impulses act at those
        st = st.astype(np.float64)
        p = (mass[:, None] * st[:, 7:10]).sum(0)
        L = (mass[:, None] * np.cross(sc.state[:, 0:3].astype(np.float64), st[:, 7:10])).sum(0)
        L += sum(Iw[i] @ st[i, 10:13] for i in range(n))
        return p, L

    o = orc.step(sc, gravity=(0, 0, 0), warmstart=False)
    keys = o["contact_key"]
    caps = set(np.nonzero(hl > 0)[0])
    assert sum(1 for k in keys if (int(k) >> 32) in caps or ((int(k) >> 1) & 0x7fffffff) in caps) > 10
    p0, L0 = mom(sc.state)
    p1, L1 = mom(o["state"])
    assert np.abs(p1 - p0).max() < 1e-11
    assert np.abs(L1 - L0).max() < 1e-10


def test_capsule_pile_grid_equals_brute_force(orc):
    sc = scenes.capsule_pile(400, 3, 4, scale=(400 / 20000.0) ** (1 / 3))
    st = sc.state.copy()
    rng = np.random.default_rng(1)
    st[:, :3] *= np.float32(0.4)               # squeeze the lattice so bodies touch
    st[:, 2] += np.float32(0.5)
    st[:, :3] += rng.normal(0, 0.05, st[:, :3].shape).astype(np.float32)
    a = orc.step(sc, state=st, max_iters=1)
    b = orc.step(sc, state=st, max_iters=1, brute_force=True)
    assert np.array_equal(a["contact_key"], b["contact_key"])
    keys = a["contact_key"].astype(np.int64)
    dyn = ((keys >> 1) & 0x7fffffff) < sc.n_bodies
    cap_cap = [(int(k) >> 32) for k in keys[dyn] if sc.shape[int(k) >> 32] == 1 and
               sc.shape[(int(k) >> 1) & 0x7fffffff] == 1]
    assert dyn.sum() > 100 and len(cap_cap) > 20


def test_capsule_mass_properties_by_integration():
    r, hl, rho = 0.3, 0.45, 1000.0
    m, I = scenes.capsule_mass_inertia(r, hl, rho)
    n = 160
    L = hl + r
    xs = (np.arange(n) + 0.5) / n * 2 * r - r
    zs = (np.arange(2 * n) + 0.5) / (2 * n) * 2 * L - L
    dv = (2 * r / n) ** 2 * (2 * L / (2 * n))
    X, Y, Z = np.meshgrid(xs, xs, zs, indexing="ij")
    zc = np.clip(Z, -hl, hl)
    inside = X * X + Y * Y + (Z - zc) ** 2 <= r * r
    mass = rho * dv * inside.sum()
    ixx = rho * dv * ((Y * Y + Z * Z) * inside).sum()
    izz = rho * dv * ((X * X + Y * Y) * inside).sum()
    assert mass == pytest.approx(m, rel=5e-3)
    assert ixx == pytest.approx(I[0], rel=1e-2)
    assert izz == pytest.approx(I[2], rel=1e-2)
    assert I[0] == I[1]
