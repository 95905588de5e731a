"""Seeded synthetic inputs: hit points (kernels), light vertices (photons) and run parameters.

The paper's scenes are not available, so these synthetic configurations stand in for them. Every
array is drawn with numpy's Philox generator from ``SeedSequence(seed, spawn_key=(set, iteration))``
so a batch can be regenerated independently of the others. Layout is structure-of-arrays: a
``(3, n)`` float32 array holds x, y and z (or R, G, B) as contiguous rows.

Nothing here computes any part of the estimator (no gather, grouping, statistic or update).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

F32 = np.float32


@dataclass
class Params:
    """Run parameters of the estimator (Sec. 5.1, Sec. 6 settings)."""
    r1: float                 # initial radius
    k: float = 0.7            # shrink ratio
    alpha_f: float = 0.05     # significance level of the F-test
    alpha: float = 0.75       # lower-bound exponent
    rmin: Optional[float] = None   # lower-bound scale; default 0.001 * r1
    n_a: int = 2              # equi-areal annuli
    n_s: int = 6              # equi-angular sectors per annulus
    mode: str = "ppm"         # "ppm" or "vcm"
    n_iter: int = 16
    stats: str = "luma"       # test sample: "luma" (luminance) or "rgb" (one test per channel)

    def __post_init__(self):
        if self.rmin is None:
            self.rmin = 0.001 * self.r1


@dataclass
class KernelSet:
    """Hit points (eye vertices). ``nrm`` None means +z for every kernel."""
    pos: np.ndarray
    nrm: Optional[np.ndarray] = None
    cam_beta: Optional[np.ndarray] = None   # VCM camera throughput RGB
    cam_mis: Optional[np.ndarray] = None    # VCM camera partials dVCM, dVC, dVM

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    def subset(self, idx) -> "KernelSet":
        take = lambda a: None if a is None else np.ascontiguousarray(a[:, idx])
        return KernelSet(pos=take(self.pos), nrm=take(self.nrm), cam_beta=take(self.cam_beta),
                         cam_mis=take(self.cam_mis))


@dataclass
class PhotonBatch:
    """Light vertices stored in one iteration. ``J`` counts every emitted sub-path, stored or not."""
    J: int
    pos: np.ndarray
    flux: np.ndarray
    nrm: Optional[np.ndarray] = None
    mis: Optional[np.ndarray] = None        # VCM light partials dVCM, dVC, dVM

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])


@dataclass
class Workload:
    name: str
    params: Params
    kernels: KernelSet
    photon_fn: Callable[[int], PhotonBatch]
    seed: int
    set_id: int = 0
    info: dict = field(default_factory=dict)

    def photons(self, it: int) -> PhotonBatch:
        """Photon batch of iteration ``it`` (0-based)."""
        return self.photon_fn(it)


def rng_for(seed: int, set_id: int, key: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(np.random.SeedSequence(seed, spawn_key=(set_id, key))))


META_KEY = 1 << 30   # spawn key reserved for per-set constants (kernels, edge and caustic placement)


# ---------------------------------------------------------------------------------------------
# Planar photon density: uniform with a darker half-plane (shadow edge) plus a Gaussian caustic
# ---------------------------------------------------------------------------------------------

def mixture_positions(rng: np.random.Generator, n: int, edge: float = 0.5, dark: float = 0.2,
                      caustic=(0.7, 0.3), sigma: float = 0.03, w_caustic: float = 0.3) -> np.ndarray:
    """(2, n) float64 positions in [0,1]^2 from (1-w) * U' + w * N(caustic, sigma^2 I).

    U' has density proportional to ``dark`` left of x = edge and to 1 right of it. Gaussian draws
    that leave the unit square are redrawn.
    """
    comp = rng.random(n) < w_caustic
    out = np.empty((2, n))
    nu = int((~comp).sum())
    m_left, m_right = dark * edge, 1.0 - edge
    left = rng.random(nu) < m_left / (m_left + m_right)
    u = rng.random(nu)
    x = np.where(left, u * edge, edge + u * (1.0 - edge))
    out[0, ~comp] = x
    out[1, ~comp] = rng.random(nu)
    nc = int(comp.sum())
    g = rng.normal(size=(2, nc)) * sigma + np.asarray(caustic, dtype=float)[:, None]
    bad = (g < 0).any(0) | (g > 1).any(0)
    while bad.any():
        nb = int(bad.sum())
        g[:, bad] = rng.normal(size=(2, nb)) * sigma + np.asarray(caustic, dtype=float)[:, None]
        bad = (g < 0).any(0) | (g > 1).any(0)
    out[:, comp] = g
    return out


def mixture_density(x, y, edge=0.5, dark=0.2, caustic=(0.7, 0.3), sigma=0.03, w_caustic=0.3):
    """Probability density of ``mixture_positions`` (Gaussian truncation ignored: ~1e-23 mass)."""
    m_left, m_right = dark * edge, 1.0 - edge
    z = m_left + m_right
    du = np.where(x < edge, dark / z, 1.0 / z)
    g = np.exp(-((x - caustic[0]) ** 2 + (y - caustic[1]) ** 2) / (2 * sigma ** 2)) / (2 * math.pi * sigma ** 2)
    return (1 - w_caustic) * du + w_caustic * g


def grid_kernels(nx: int, ny: int) -> np.ndarray:
    """(3, nx*ny) float32 pixel centres ((i+1/2)/nx, (j+1/2)/ny, 0), x fastest."""
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    pos = np.zeros((3, nx * ny), dtype=F32)
    pos[0] = ((i.ravel() + 0.5) / nx).astype(F32)
    pos[1] = ((j.ravel() + 0.5) / ny).astype(F32)
    return pos


def _planar_batch(rng, J, n_store, edge, caustic, flux_sigma, with_nrm=False, with_mis=False):
    p = mixture_positions(rng, n_store, edge=edge, caustic=caustic)
    pos = np.zeros((3, n_store), dtype=F32)
    pos[0] = p[0].astype(F32)
    pos[1] = p[1].astype(F32)
    flux = np.exp(rng.normal(size=(3, n_store)) * flux_sigma).astype(F32)
    nrm = None
    if with_nrm:
        nrm = np.zeros((3, n_store), dtype=F32)
        nrm[2] = 1.0
    mis = rng.random((3, n_store)).astype(F32) if with_mis else None
    return PhotonBatch(J=J, pos=pos, flux=flux, nrm=nrm, mis=mis)


# ---------------------------------------------------------------------------------------------
# Config 0: plane with shadow edge and caustic
# ---------------------------------------------------------------------------------------------

def config0(seed: int = 0, n_side: int = 64, J: int = 100_000, n_iter: int = 16, r1: float = 0.05,
            alpha_f: float = 0.05, set_id: int = 0) -> Workload:
    """64x64 hit points on z=0, 100k photons per iteration, r1 = 0.05, 16 iterations."""
    ks = KernelSet(pos=grid_kernels(n_side, n_side))

    def photons(it: int) -> PhotonBatch:
        rng = rng_for(seed, set_id, it)
        return _planar_batch(rng, J, J, 0.5, (0.7, 0.3), 0.5)

    return Workload("plane-edge-caustic", Params(r1=r1, n_iter=n_iter, alpha_f=alpha_f), ks, photons,
                    seed, set_id, info=dict(H=n_side * n_side, J=J, edge=0.5, caustic=(0.7, 0.3)))


def small_config0(seed: int = 0, n_side: int = 16, J: int = 6000, n_iter: int = 6, r1: float = 0.08):
    """Config 0's density at oracle-friendly size (several tiles and a ragged tail when n_side=23)."""
    return config0(seed=seed, n_side=n_side, J=J, n_iter=n_iter, r1=r1)


def uniform_config(seed: int, n_kernels_side: int, J: int, r1: float, n_iter: int = 1,
                   spacing_margin: float = 2.2, alpha_f: float = 0.05, flux_sigma: float = 0.5) -> Workload:
    """Uniform photon density on the unit square; kernels on a lattice in the interior, more than
    2 r1 apart (independent disks) and at least r1 from the border."""
    lo, hi = r1 * 1.01, 1.0 - r1 * 1.01
    step = (hi - lo) / max(n_kernels_side - 1, 1)
    if n_kernels_side > 1 and step < spacing_margin * r1:
        raise ValueError("kernels would overlap")
    g = lo + step * np.arange(n_kernels_side)
    yy, xx = np.meshgrid(g, g, indexing="ij")
    pos = np.zeros((3, xx.size), dtype=F32)
    pos[0] = xx.ravel().astype(F32)
    pos[1] = yy.ravel().astype(F32)

    def photons(it: int) -> PhotonBatch:
        rng = rng_for(seed, 0, it)
        p = np.zeros((3, J), dtype=F32)
        p[0] = rng.random(J).astype(F32)
        p[1] = rng.random(J).astype(F32)
        flux = np.exp(rng.normal(size=(3, J)) * flux_sigma).astype(F32)
        return PhotonBatch(J=J, pos=p, flux=flux)

    return Workload("uniform", Params(r1=r1, n_iter=n_iter, alpha_f=alpha_f), KernelSet(pos=pos), photons, seed)


# ---------------------------------------------------------------------------------------------
# Config 1: unit box with a point light and a spherical occluder
# ---------------------------------------------------------------------------------------------

@dataclass
class BoxScene:
    light: tuple = (0.5, 0.9, 0.5)
    sphere_c: tuple = (0.5, 0.5, 0.5)
    sphere_r: float = 0.15
    cam: tuple = (0.5, 0.5, 2.0)
    res: int = 512
    intensity: float = 1.0     # W/sr; each photon carries 4*pi*intensity

    # ---- hit points ------------------------------------------------------------------------
    def hit_points(self):
        """Primary hits of pixel-centre rays through the z=1 opening (x faces win exact ties).

        Returns (pos (3,H) f32, nrm (3,H) f32, face (H,) int8) with faces 0:x=0 1:x=1 2:y=0 3:y=1 4:z=0.
        """
        n = self.res
        jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        px = (ii.ravel() + 0.5) / n
        py = (jj.ravel() + 0.5) / n
        cx, cy, cz = self.cam
        dx, dy, dz = px - cx, py - cy, 1.0 - cz
        big = np.inf
        tx = np.where(dx < 0, (0.0 - cx) / np.where(dx == 0, 1, dx), np.where(dx > 0, (1.0 - cx) / np.where(dx == 0, 1, dx), big))
        ty = np.where(dy < 0, (0.0 - cy) / np.where(dy == 0, 1, dy), np.where(dy > 0, (1.0 - cy) / np.where(dy == 0, 1, dy), big))
        tz = np.full(px.shape, (0.0 - cz) / dz)
        face = np.full(px.shape, 4, dtype=np.int8)
        use_x = tx <= np.minimum(ty, tz)
        use_y = (~use_x) & (ty < tz)
        face[use_x] = np.where(dx[use_x] < 0, 0, 1)
        face[use_y] = np.where(dy[use_y] < 0, 2, 3)
        t = np.where(use_x, tx, np.where(use_y, ty, tz))
        X = cx + t * dx
        Y = cy + t * dy
        Z = cz + t * dz
        pos = np.stack([X, Y, Z]).astype(F32)
        nrm = np.zeros((3, px.size), dtype=F32)
        for f, (ax, val, nv) in enumerate([(0, 0.0, 1.0), (0, 1.0, -1.0), (1, 0.0, 1.0), (1, 1.0, -1.0), (2, 0.0, 1.0)]):
            sel = face == f
            pos[ax, sel] = val
            nrm[ax, sel] = nv
        np.clip(pos, 0.0, 1.0, out=pos)
        return pos, nrm, face

    # ---- light vertices ----------------------------------------------------------------------
    def emit(self, rng: np.random.Generator, J: int):
        """Trace J isotropic sub-paths from the point light; keep first hits on the five quads."""
        u = rng.random(J)
        v = rng.random(J)
        dz = 1.0 - 2.0 * u
        s = np.sqrt(np.maximum(0.0, 1.0 - dz * dz))
        phi = 2.0 * math.pi * v
        dx = s * np.cos(phi)
        dy = s * np.sin(phi)
        Lx, Ly, Lz = self.light
        # exit face of the unit box along the ray
        with np.errstate(divide="ignore", invalid="ignore"):
            tx = np.where(dx > 0, (1.0 - Lx) / dx, np.where(dx < 0, (0.0 - Lx) / dx, np.inf))
            ty = np.where(dy > 0, (1.0 - Ly) / dy, np.where(dy < 0, (0.0 - Ly) / dy, np.inf))
            tz = np.where(dz > 0, (1.0 - Lz) / dz, np.where(dz < 0, (0.0 - Lz) / dz, np.inf))
        t = np.minimum(np.minimum(tx, ty), tz)
        ax = np.where(tx == t, 0, np.where(ty == t, 1, 2))
        # sphere occluder
        ocx, ocy, ocz = Lx - self.sphere_c[0], Ly - self.sphere_c[1], Lz - self.sphere_c[2]
        b = dx * ocx + dy * ocy + dz * ocz
        c = ocx * ocx + ocy * ocy + ocz * ocz - self.sphere_r ** 2
        disc = b * b - c
        ts = -b - np.sqrt(np.maximum(disc, 0.0))
        occluded = (disc > 0) & (ts > 0) & (ts < t)
        X, Y, Z = Lx + t * dx, Ly + t * dy, Lz + t * dz
        escaped = (ax == 2) & (dz > 0)
        keep = ~(occluded | escaped)
        X, Y, Z, ax, dx, dy, dz = X[keep], Y[keep], Z[keep], ax[keep], dx[keep], dy[keep], dz[keep]
        n = X.size
        pos = np.stack([X, Y, Z]).astype(F32)
        nrm = np.zeros((3, n), dtype=F32)
        for a, d in ((0, dx), (1, dy), (2, dz)):
            sel = ax == a
            pos[a, sel] = np.where(d[sel] > 0, 1.0, 0.0).astype(F32)
            nrm[a, sel] = np.where(d[sel] > 0, -1.0, 1.0).astype(F32)
        np.clip(pos, 0.0, 1.0, out=pos)
        flux = np.full((3, n), 4.0 * math.pi * self.intensity, dtype=F32)
        return PhotonBatch(J=J, pos=pos, flux=flux, nrm=nrm)

    # ---- analytic direct lighting ------------------------------------------------------------
    def irradiance(self, pos: np.ndarray, nrm: np.ndarray) -> np.ndarray:
        """E = I cos(theta) / d^2 with analytic sphere visibility, float64, shape (H,)."""
        L = np.asarray(self.light, dtype=float)[:, None]
        p = pos.astype(float)
        w = L - p
        d2 = (w * w).sum(0)
        d = np.sqrt(d2)
        wn = w / d
        cos = np.maximum(0.0, (wn * nrm.astype(float)).sum(0))
        oc = p - np.asarray(self.sphere_c, dtype=float)[:, None]
        b = (wn * oc).sum(0)
        c = (oc * oc).sum(0) - self.sphere_r ** 2
        disc = b * b - c
        t0 = -b - np.sqrt(np.maximum(disc, 0.0))
        vis = ~((disc > 0) & (t0 > 0) & (t0 < d))
        return self.intensity * cos / d2 * vis


def box_scene(seed: int = 1, res: int = 512, J: int = 2_000_000, n_iter: int = 64, r1: float = 0.05,
              light=(0.5, 0.9, 0.5), sphere_c=(0.5, 0.5, 0.5), set_id: int = 0) -> Workload:
    scene = BoxScene(light=tuple(light), sphere_c=tuple(sphere_c), res=res)
    pos, nrm, face = scene.hit_points()

    def photons(it: int) -> PhotonBatch:
        return scene.emit(rng_for(seed, set_id, it), J)

    return Workload("box-point-light", Params(r1=r1, n_iter=n_iter), KernelSet(pos=pos, nrm=nrm), photons,
                    seed, set_id, info=dict(H=res * res, J=J, scene=scene, face=face))


def config1(seed: int = 1, **kw) -> Workload:
    """512x512 hit points on five quads of the unit box, 2M photons per iteration, 64 iterations."""
    return box_scene(seed=seed, **kw)


# ---------------------------------------------------------------------------------------------
# Config 3: box scenes with jittered light and occluder (training and held-out scenes of the
# learned radius proposal)
# ---------------------------------------------------------------------------------------------

def config3(seed: int, res: int = 512, J: int = 2_000_000, n_iter: int = 64, r1: float = 0.05) -> Workload:
    """Config 1's box with the light and the occluder centre each moved by U(-0.1, 0.1) per axis
    (the light's height capped at 0.92, below the ceiling). Seeds 30-33 are the training scenes,
    seed 39 the held-out one."""
    meta = rng_for(seed, 0, META_KEY)
    dl = meta.uniform(-0.1, 0.1, 3)
    ds = meta.uniform(-0.1, 0.1, 3)
    light = (float(0.5 + dl[0]), float(min(0.9 + dl[1], 0.92)), float(0.5 + dl[2]))
    sphere = (float(0.5 + ds[0]), float(0.5 + ds[1]), float(0.5 + ds[2]))
    w = box_scene(seed=seed, res=res, J=J, n_iter=n_iter, r1=r1, light=light, sphere_c=sphere)
    w.name = f"box-jittered-{seed}"
    return w


# ---------------------------------------------------------------------------------------------
# Config 2: many independent sets of uneven size
# ---------------------------------------------------------------------------------------------

def config2_sets(seed: int = 2, n_sets: int = 16, side_range=(64, 1024), J_range=(500_000, 8_000_000),
                 scale: float = 1.0):
    """Per-set (side, J, edge, caustic centre) of config 2, drawn from the seed's meta stream."""
    meta = rng_for(seed, 0, META_KEY)
    lo, hi = np.log(side_range[0]), np.log(side_range[1])
    sides = np.exp(meta.uniform(lo, hi, n_sets))
    Js = np.exp(meta.uniform(np.log(J_range[0]), np.log(J_range[1]), n_sets))
    edges = meta.uniform(0.2, 0.8, n_sets)
    caus = meta.uniform(0.2, 0.8, (n_sets, 2))
    out = []
    for s in range(n_sets):
        side = max(4, int(round(sides[s] * math.sqrt(scale))))
        J = max(1000, int(round(Js[s] * scale)))
        out.append((side, J, float(edges[s]), (float(caus[s, 0]), float(caus[s, 1]))))
    return out


def config2_photons(seed: int, s: int, it: int, J: int, edge: float, ca) -> PhotonBatch:
    """Light vertices of set s of config 2 at iteration it (every emitted path is stored)."""
    return _planar_batch(rng_for(seed, s, it), J, J, edge, ca, 0.5)


def config2(seed: int = 2, n_sets: int = 16, side_range=(64, 1024), J_range=(500_000, 8_000_000),
            n_iter: int = 16, scale: float = 1.0) -> List[Workload]:
    """Independent planar sets; side and J log-uniform, r1 = 0.05 * sqrt(1e5 / J) keeps about 785
    photons per disk. ``scale`` < 1 shrinks every side and J for quick runs."""
    out = []
    for s, (side, J, edge, ca) in enumerate(config2_sets(seed, n_sets, side_range, J_range, scale)):
        r1 = 0.05 * math.sqrt(1e5 / J)
        ks = KernelSet(pos=grid_kernels(side, side))

        def photons(it, s=s, J=J, edge=edge, ca=ca):
            return config2_photons(seed, s, it, J, edge, ca)

        out.append(Workload(f"set{s}", Params(r1=r1, n_iter=n_iter), ks, photons, seed, s,
                            info=dict(H=side * side, J=J, edge=edge, caustic=ca)))
    return out


# ---------------------------------------------------------------------------------------------
# Config 4: vertex merging at scale (camera vertices with throughput and MIS partials)
# ---------------------------------------------------------------------------------------------

def config4(seed: int = 4, nx: int = 1920, ny: int = 1080, J: int = 4_000_000, n_iter: int = 256,
            r1: float = 0.00212) -> Workload:
    """1920x1080 camera vertices on pixel centres of [0,1]^2 (z=0, +z), 4M light vertices per
    iteration from config 0's density; throughputs lognormal(0,1), partials U[0,1]."""
    meta = rng_for(seed, 0, META_KEY)
    pos = grid_kernels(nx, ny)
    H = nx * ny
    nrm = np.zeros((3, H), dtype=F32)
    nrm[2] = 1.0
    beta = np.exp(meta.normal(size=(3, H))).astype(F32)
    mis = meta.random((3, H)).astype(F32)
    ks = KernelSet(pos=pos, nrm=nrm, cam_beta=beta, cam_mis=mis)

    def photons(it: int) -> PhotonBatch:
        return config4_photons(seed, it, J)

    return Workload("vcm-merge", Params(r1=r1, n_iter=n_iter, mode="vcm"), ks, photons, seed,
                    info=dict(H=H, J=J))


def config4_photons(seed: int, it: int, J: int = 4_000_000) -> PhotonBatch:
    """Light vertices of config 4 at iteration it: config 0's density, normal +z, throughput
    lognormal(0, 1), partials U[0, 1]; every emitted path is stored."""
    return _planar_batch(rng_for(seed, 0, it), J, J, 0.5, (0.7, 0.3), 1.0, with_nrm=True, with_mis=True)


# ---------------------------------------------------------------------------------------------
# Batches by picklable description, for generation in worker processes
# ---------------------------------------------------------------------------------------------

def batch(spec) -> PhotonBatch:
    """The batch a tuple describes: ("box", seed, it, J, res) for config 1's box scene,
    ("jittered", seed, it, J, res) for config 3's scenes, ("sets", seed, s, it, J, edge, caustic)
    for set s of config 2, ("merge", seed, it, J) for config 4."""
    kind = spec[0]
    if kind == "box":
        _, seed, it, J, res = spec
        return box_scene(seed=seed, res=res, J=J).photons(it)
    if kind == "jittered":
        _, seed, it, J, res = spec
        return config3(seed, res=res, J=J).photons(it)
    if kind == "sets":
        _, seed, s, it, J, edge, ca = spec
        return config2_photons(seed, s, it, J, edge, ca)
    if kind == "merge":
        _, seed, it, J = spec
        return config4_photons(seed, it, J)
    raise ValueError(f"unknown batch kind {kind!r}")


class InProcess:
    """The executor interface of ``spawn_pool`` run in the calling process (no worker processes)."""

    def map(self, fn, items):
        return map(fn, items)

    def shutdown(self):
        pass


def spawn_pool(workers: int):
    """Worker processes for ``batch``, started with the spawn method: fresh interpreters that share
    nothing with a parent that may already hold a GPU (no fork of such a process). With workers <= 0
    the batches are generated in the calling process instead."""
    if workers <= 0:
        return InProcess()
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    ex = ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn"))
    list(ex.map(int, range(workers)))          # start the workers now
    return ex
