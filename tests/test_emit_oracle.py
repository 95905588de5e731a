"""Pins of the light-vertex generation oracle for the box scene: the random numbers against the
generator's published known-answer vectors and numpy's own Philox, the directions against the
uniform distribution on the sphere, and the first hits against closed-form solid angles and the
sphere's shadow."""
import math
import os

import numpy as np
from scipy import stats

from oracle import emit as E

HERE = os.path.dirname(os.path.abspath(__file__))
F32 = np.float32


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                w = [int(x, 16) for x in line.split()]
                rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox4x32_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert E.philox4_scalar(ctr, key, 32) == out
        got = E.philox4x32_10(*(np.array([c], dtype=np.uint32) for c in ctr), *key)
        assert [int(g[0]) for g in got] == out


def test_philox4x64_matches_numpy():
    """The same round structure at 64-bit words is numpy's Philox bit generator (which advances its
    counter by one before producing each block)."""
    rng = np.random.default_rng(5)
    for _ in range(4):
        key = [int(x) for x in rng.integers(0, 2 ** 63, 2, dtype=np.int64)]
        ctr = [int(x) for x in rng.integers(0, 2 ** 62, 4, dtype=np.int64)]
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
        raw = [int(v) for v in bg.random_raw(8)]
        c1 = [ctr[0] + 1] + ctr[1:]
        c2 = [ctr[0] + 2] + ctr[1:]
        assert E.philox4_scalar(c1, key, 64) == raw[:4]
        assert E.philox4_scalar(c2, key, 64) == raw[4:]


def test_vectorised_philox_equals_scalar():
    rng = np.random.default_rng(6)
    c = rng.integers(0, 2 ** 32, (4, 64), dtype=np.uint64).astype(np.uint32)
    k = rng.integers(0, 2 ** 32, 2, dtype=np.uint64)
    vec = E.philox4x32_10(c[0], c[1], c[2], c[3], int(k[0]), int(k[1]))
    for i in range(64):
        assert [int(v[i]) for v in vec] == E.philox4_scalar([int(x) for x in c[:, i]], [int(x) for x in k], 32)


def test_uniform_is_exact_and_in_range():
    x = np.array([0, 255, 256, 2 ** 32 - 1, 2 ** 31], dtype=np.uint32)
    u = E.uniform(x)
    assert u.dtype == F32
    assert list(u) == [0.0, 0.0, 2.0 ** -24, 1.0 - 2.0 ** -24, 0.5]


def test_directions_uniform_on_sphere():
    J = 400_000
    d, drawn = E.directions(J, it=3, set_id=1, seed=77)
    assert drawn.all()                       # a failure of all 16 attempts has probability 5e-11
    n2 = (d.astype(float) ** 2).sum(0)
    assert np.max(np.abs(n2 - 1.0)) < 4e-7
    # Archimedes: the z coordinate of a uniform point on the sphere is uniform on [-1, 1]
    assert stats.kstest(d[2].astype(float), "uniform", args=(-1.0, 2.0)).pvalue > 1e-4
    az = np.arctan2(d[1].astype(float), d[0].astype(float))
    assert stats.kstest(az, "uniform", args=(-math.pi, 2 * math.pi)).pvalue > 1e-4
    # the three axes are exchangeable: the same holds for x
    assert stats.kstest(d[0].astype(float), "uniform", args=(-1.0, 2.0)).pvalue > 1e-4
    assert np.all(np.abs(d.astype(float).mean(1)) < 5.0 / math.sqrt(3 * J))


def test_slots_are_counter_based():
    """Slot j depends on (seed, set, iteration, j) only: a shorter run is a prefix of a longer one,
    and any change of seed, set or iteration changes the stream."""
    b = E.Box()
    p1, n1, f1 = E.emit(b, 1000, it=2, set_id=0, seed=9)
    p2, n2, f2 = E.emit(b, 37, it=2, set_id=0, seed=9)
    assert np.array_equal(p1[:, :37], p2, equal_nan=True) and np.array_equal(n1[:, :37], n2)
    for kw in (dict(it=3, set_id=0, seed=9), dict(it=2, set_id=1, seed=9), dict(it=2, set_id=0, seed=10),
               dict(it=2, set_id=0, seed=9 + (1 << 32))):
        p3, _, _ = E.emit(b, 1000, **kw)
        assert not np.array_equal(p1, p3, equal_nan=True)


def _rect_solid_angle(h, x1, x2, y1, y2):
    """Solid angle of the rectangle [x1, x2] x [y1, y2] in a plane at distance h, coordinates taken
    from the foot of the perpendicular (sum of four corner terms atan(x y / (h sqrt(x^2+y^2+h^2))))."""
    def g(x, y):
        return math.atan(x * y / (h * math.sqrt(x * x + y * y + h * h)))
    return g(x2, y2) - g(x1, y2) - g(x2, y1) + g(x1, y1)


def _face_solid_angles(L):
    Lx, Ly, Lz = L
    return {
        "x0": _rect_solid_angle(Lx, -Ly, 1 - Ly, -Lz, 1 - Lz),
        "x1": _rect_solid_angle(1 - Lx, -Ly, 1 - Ly, -Lz, 1 - Lz),
        "y0": _rect_solid_angle(Ly, -Lx, 1 - Lx, -Lz, 1 - Lz),
        "y1": _rect_solid_angle(1 - Ly, -Lx, 1 - Lx, -Lz, 1 - Lz),
        "z0": _rect_solid_angle(Lz, -Lx, 1 - Lx, -Ly, 1 - Ly),
        "z1": _rect_solid_angle(1 - Lz, -Lx, 1 - Lx, -Ly, 1 - Ly),
    }


def _faces(pos, nrm):
    lab = np.full(pos.shape[1], "none", dtype=object)
    for ax, name in enumerate("xyz"):
        lab[nrm[ax] > 0] = name + "0"
        lab[nrm[ax] < 0] = name + "1"
    return lab


def test_first_hits_follow_solid_angles_and_shadow():
    box = E.Box()
    L = box.light
    om = _face_solid_angles(L)
    assert abs(sum(om.values()) - 4 * math.pi) < 1e-12            # the six faces close the box
    dist = math.dist(L, box.sphere_c)
    om_s = 2 * math.pi * (1 - math.sqrt(1 - (box.sphere_r / dist) ** 2))
    J = 1_000_000
    pos, nrm, flux = E.emit(box, J, it=0, set_id=0, seed=1)
    lab = _faces(pos, nrm)
    kept = np.isfinite(pos[0])
    assert np.array_equal(kept, lab != "none")
    # the shadow of the sphere falls entirely inside the floor y = 0 (cone axis along -y)
    p = {k: v / (4 * math.pi) for k, v in om.items()}
    p["y0"] -= om_s / (4 * math.pi)
    p["none"] = p.pop("z1") + om_s / (4 * math.pi)
    cats = ["x0", "x1", "y0", "y1", "z0", "none"]
    obs = np.array([(lab == c).sum() for c in cats])
    exp = np.array([p[c] for c in cats]) * J
    assert abs(sum(p.values()) - 1.0) < 1e-12
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    # every kept vertex lies on its face, carries the power and no other normal component
    for ax in range(3):
        on = (nrm[ax] != 0)
        assert np.all((pos[ax][on] == 0.0) | (pos[ax][on] == 1.0))
        assert np.all((pos[ax][kept] >= 0.0) & (pos[ax][kept] <= 1.0))
    assert np.all(np.abs(nrm[:, kept]).sum(0) == 1.0)
    assert np.all(flux[:, kept] == F32(4 * math.pi)) and np.all(flux[:, ~kept] == 0.0)
    assert np.all(np.isnan(pos[:, ~kept])) and np.all(nrm[:, ~kept] == 0.0)
    # the shadow disk on y = 0: centre below the sphere, radius h tan(theta)
    tan_t = (box.sphere_r / dist) / math.sqrt(1 - (box.sphere_r / dist) ** 2)
    rad = L[1] * tan_t
    floor = lab == "y0"
    rr = np.hypot(pos[0][floor] - 0.5, pos[2][floor] - 0.5)
    assert np.sum(rr < rad * (1 - 1e-4)) == 0
    ring = np.sum((rr > rad * (1 + 1e-4)) & (rr < rad * 1.05))
    assert ring > 1000


def test_hits_are_on_the_rays():
    """Each kept vertex lies on the ray from the light along its drawn direction, at the distance a
    float64 intersection gives, up to float32 rounding."""
    box = E.Box()
    J = 200_000
    d, _ = E.directions(J, it=5, set_id=2, seed=3)
    pos, nrm, _ = E.emit(box, J, it=5, set_id=2, seed=3)
    kept = np.isfinite(pos[0])
    L = np.array(box.light)[:, None]
    v = pos[:, kept].astype(float) - L
    dd = d[:, kept].astype(float)
    cross = np.cross(v.T, dd.T).T
    assert np.max(np.linalg.norm(cross, axis=0)) < 5e-6
    assert np.all((v * dd).sum(0) > 0)
    # float64 exit distance of the same direction
    with np.errstate(divide="ignore"):
        t = np.min(np.where(dd > 0, (1 - L) / dd, np.where(dd < 0, -L / dd, np.inf)), axis=0)
    assert np.max(np.abs(np.linalg.norm(v, axis=0) - t)) < 5e-6


def test_merging_partial_is_the_reciprocal_area_density():
    """dVCM of a kept vertex is 1 / p_L with p_L = cos(theta) / (4 pi |y - L|^2), the area density of
    the light pass at the vertex; here recomputed in float64 from the vertex position and normal."""
    box = E.Box()
    J = 100_000
    pos, nrm, flux, mis = E.emit(box, J, it=1, set_id=0, seed=4, with_mis=True)
    kept = np.isfinite(pos[0])
    L = np.array(box.light)[:, None]
    v = pos[:, kept].astype(float) - L
    d2 = (v * v).sum(0)
    cos = np.abs((v * nrm[:, kept]).sum(0)) / np.sqrt(d2)
    pl = cos / (4 * math.pi * d2)
    ok = cos > 1e-3
    assert np.max(np.abs(mis[0, kept][ok] * pl[ok] - 1.0)) < 2e-5
    assert np.all(mis[1:] == 0.0) and np.all(mis[0, ~kept] == 0.0)
    # the same slots as without the partials
    p2, n2, f2 = E.emit(box, J, it=1, set_id=0, seed=4)
    assert np.array_equal(p2, pos, equal_nan=True) and np.array_equal(n2, nrm) and np.array_equal(f2, flux)
