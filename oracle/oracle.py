"""CPU oracle of the hypothesis-tested progressive kernel estimator (arXiv 2504.04411).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg are
the only callers. It shares no code with the GPU library and never imports it.

Per-pair work (inside-disk test, grouping, test sample, float64 sums) is done by the C library
``liboracle.so`` built from ``hk_oracle.c``. This module does the rest of one iteration in float64:

* retention of sector statistics while the radius is kept (Sec. 5.1: t kept iterations give tJ
  samples per sector),
* the ANOVA F statistic for equal group sizes (Eq. f-statistic),
* the critical value, the (1 - alpha_F) quantile of F(n - 1, n (m - 1)) (Sec. 3.2.2), solved from
  mpmath's regularised incomplete beta function in 40-digit arithmetic,
* the radius update (Eq. radiusupdate) and the progressive estimate (Eq. progressive-VCM-estimator).

Readings where the paper is silent are listed in the design notes and repeated where they are used.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import mpmath as mp
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "hk_oracle.c")
NG = 12
F32 = np.float32


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no contraction of a*b+c, so every float32 op is as written)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", SRC_PATH, "-o", LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_P = ctypes.POINTER(ctypes.c_float)


class _Args(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_int64),
        ("kx", _P), ("ky", _P), ("kz", _P),
        ("knx", _P), ("kny", _P), ("knz", _P),
        ("ux", _P), ("uy", _P), ("uz", _P), ("vx", _P), ("vy", _P), ("vz", _P),
        ("r", _P),
        ("cbR", _P), ("cbG", _P), ("cbB", _P),
        ("cdvcm", _P), ("cdvm", _P),
        ("J", ctypes.c_int64), ("J_emitted", ctypes.c_int64),
        ("px", _P), ("py", _P), ("pz", _P),
        ("pnx", _P), ("pny", _P), ("pnz", _P),
        ("fR", _P), ("fG", _P), ("fB", _P),
        ("pdvcm", _P), ("pdvm", _P),
        ("vcm", ctypes.c_int),
        ("cos_min", ctypes.c_float),
        ("rgb", ctypes.c_int),
        ("count", ctypes.POINTER(ctypes.c_uint32)),
        ("S", ctypes.POINTER(ctypes.c_double)), ("Q", ctypes.POINTER(ctypes.c_double)),
        ("flux", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        L.oracle_gather_allpairs.argtypes = [ctypes.POINTER(_Args), ctypes.c_int]
        L.oracle_gather_grid.argtypes = [ctypes.POINTER(_Args), ctypes.c_int]
        L.oracle_group.argtypes = [ctypes.c_float] * 4
        L.oracle_group.restype = ctypes.c_int
        L.oracle_frame.argtypes = [ctypes.c_int64] + [_P] * 9
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _fp(a: Optional[np.ndarray]):
    if a is None:
        return ctypes.cast(None, _P)
    assert a.dtype == F32 and a.flags.c_contiguous
    return a.ctypes.data_as(_P)


def _rows(a):
    return [np.ascontiguousarray(a[i], dtype=F32) for i in range(a.shape[0])]


# ------------------------------------------------------------------------------------------------
# Building blocks
# ------------------------------------------------------------------------------------------------

def frames(nrm: Optional[np.ndarray], n: int):
    """Tangent frames (u, v) of the kernel normals (+z when ``nrm`` is None); two (3, n) arrays."""
    if nrm is None:
        nrm = np.zeros((3, n), dtype=F32)
        nrm[2] = 1.0
    nx, ny, nz = _rows(nrm)
    out = [np.empty(n, dtype=F32) for _ in range(6)]
    lib().oracle_frame(n, _fp(nx), _fp(ny), _fp(nz), *[_fp(o) for o in out])
    return np.stack(out[:3]), np.stack(out[3:])


def group_of(yu: float, yv: float, d2: float, r2: float) -> int:
    return int(lib().oracle_group(F32(yu), F32(yv), F32(d2), F32(r2)))


@dataclass
class GatherResult:
    count: np.ndarray      # (H,) uint32
    S: np.ndarray          # (H, 12) float64; (H, 36) with one test per channel (R groups, G, B)
    Q: np.ndarray          # like S
    flux: np.ndarray       # (H, 3) float64


def gather(kernels, photons, r: np.ndarray, vcm: bool = False, use_grid: bool = True, cos_min: float = 0.5,
           idx: Optional[np.ndarray] = None, nthreads: int = 0, rgb: bool = False) -> GatherResult:
    """Per-kernel sums of one iteration for the kernels ``idx`` (all when None) at radii ``r``."""
    sel = np.arange(kernels.n) if idx is None else np.asarray(idx)
    H = sel.size
    kp = _rows(kernels.pos[:, sel])
    kn = _rows(kernels.nrm[:, sel]) if kernels.nrm is not None else [None] * 3
    u, v = frames(kernels.nrm[:, sel] if kernels.nrm is not None else None, H)
    u, v = _rows(u), _rows(v)
    rr = np.ascontiguousarray(np.asarray(r, dtype=F32)[sel] if np.ndim(r) else np.full(kernels.n, r, F32)[sel])
    pp = _rows(photons.pos)
    pn = _rows(photons.nrm) if (photons.nrm is not None and kernels.nrm is not None) else [None] * 3
    if photons.nrm is None or kernels.nrm is None:
        kn = [None] * 3
    fl = _rows(photons.flux)
    cb = _rows(kernels.cam_beta[:, sel]) if vcm else [None] * 3
    cm = _rows(kernels.cam_mis[:, sel]) if vcm else [None] * 3
    pm = _rows(photons.mis) if vcm else [None] * 3
    w = 3 * NG if rgb else NG
    out = GatherResult(np.zeros(H, np.uint32), np.zeros((H, w)), np.zeros((H, w)), np.zeros((H, 3)))
    a = _Args()
    a.H = H
    a.kx, a.ky, a.kz = map(_fp, kp)
    a.knx, a.kny, a.knz = map(_fp, kn)
    a.ux, a.uy, a.uz = map(_fp, u)
    a.vx, a.vy, a.vz = map(_fp, v)
    a.r = _fp(rr)
    a.cbR, a.cbG, a.cbB = map(_fp, cb)
    a.cdvcm, a.cdvm = _fp(cm[0]), _fp(cm[2])
    a.J = photons.n
    a.J_emitted = photons.J
    a.px, a.py, a.pz = map(_fp, pp)
    a.pnx, a.pny, a.pnz = map(_fp, pn)
    a.fR, a.fG, a.fB = map(_fp, fl)
    a.pdvcm, a.pdvm = _fp(pm[0]), _fp(pm[2])
    a.vcm = 1 if vcm else 0
    a.cos_min = F32(cos_min)
    a.rgb = 1 if rgb else 0
    a.count = out.count.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    a.S = out.S.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    a.Q = out.Q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    a.flux = out.flux.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fn = lib().oracle_gather_grid if use_grid else lib().oracle_gather_allpairs
    rc = fn(ctypes.byref(a), int(nthreads))
    if rc != 0:
        raise MemoryError("oracle gather failed")
    return out


def f_statistic(S: np.ndarray, Q: np.ndarray, m) -> np.ndarray:
    """ANOVA F for n groups of equal size m (Eq. f-statistic), from per-group sums S and sums of
    squares Q; float64, shape (H,). Groups are the last axis.

    between = m * sum_i (mean_i - mean)^2 / (n - 1),  within = sum_i sum_j (x_ij - mean_i)^2 / (n (m - 1)),
    with sum_j (x_ij - mean_i)^2 = Q_i - S_i^2 / m and m * (mean_i - mean)^2 = (S_i - S / n)^2 / m.
    """
    S = np.asarray(S, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n = S.shape[-1]
    m = np.asarray(m, dtype=np.float64)
    tot = S.sum(-1)
    ssb = ((S - tot[..., None] / n) ** 2).sum(-1) / m
    ssw = (Q - S * S / m[..., None]).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        return (ssb / (n - 1)) / (ssw / (n * (m - 1)))


def within_ss(S, Q, m):
    m = np.asarray(m, dtype=np.float64)
    return (np.asarray(Q, np.float64) - np.asarray(S, np.float64) ** 2 / m[..., None]).sum(-1)


_FC_CACHE = {}


def _f_quantile_mp(p_lo: str, d1: int, d2: float) -> float:
    """(1 - alpha) quantile of F(d1, d2) to float64 accuracy: root of the regularised incomplete beta
    I_x(d1/2, d2/2) = 1 - alpha at x = d1 F / (d1 F + d2), in 40-digit arithmetic (mpmath).

    scipy's own F quantile drifts by 1e-9..1e-5 for d2 beyond 1e10, too close to the decision band."""
    with mp.workdps(40):
        a, b = mp.mpf(d1) / 2, mp.mpf(d2) / 2
        target = 1 - mp.mpf(p_lo)
        fn = lambda F: mp.betainc(a, b, 0, d1 * F / (d1 * F + d2), regularized=True) - target
        x0 = mp.mpf(stats.chi2.ppf(1.0 - float(p_lo), d1) / d1)
        return float(mp.findroot(fn, x0, tol=mp.mpf(10) ** -32))


def f_critical(m, alpha_f: float, n_groups: int = NG) -> np.ndarray:
    """(1 - alpha_F) quantile of F(n - 1, n (m - 1)) (Sec. 3.2.2), float64, elementwise over m."""
    m = np.asarray(m, dtype=np.float64)
    out = np.empty(m.shape)
    flat = m.reshape(-1)
    res = out.reshape(-1)
    for i, mv in enumerate(flat):
        if not mv >= 2.0:                 # n (m - 1) = 0 within-group degrees of freedom: no test
            res[i] = np.nan
            continue
        key = (float(mv), repr(alpha_f), n_groups)
        if key not in _FC_CACHE:
            _FC_CACHE[key] = _f_quantile_mp(repr(alpha_f), n_groups - 1, n_groups * (float(mv) - 1.0))
        res[i] = _FC_CACHE[key]
    return out


def lower_bound(rmin: float, alpha: float, i_next: int) -> np.float32:
    """r_min sqrt((i+1)^(alpha-1)) of Eq. radiusupdate, evaluated in float64 and rounded once."""
    return F32(rmin * math.sqrt(float(i_next) ** (alpha - 1.0)))


# ------------------------------------------------------------------------------------------------
# Iteration driver
# ------------------------------------------------------------------------------------------------

@dataclass
class OracleState:
    r: np.ndarray                      # float32 radius used by the next iteration
    t: np.ndarray                      # kept iterations since the last shrink
    nseen: np.ndarray                  # in-disk photons since the last shrink
    S: np.ndarray                      # (H, 12) retained sums
    Q: np.ndarray                      # (H, 12) retained sums of squares
    tau: np.ndarray                    # (H, 3) sum over iterations of the per-iteration estimate
    iters: int = 0
    J_hist: list = field(default_factory=list)
    # last iteration, for comparison
    count: Optional[np.ndarray] = None
    F: Optional[np.ndarray] = None
    Fc: Optional[np.ndarray] = None
    shrink: Optional[np.ndarray] = None
    m: Optional[np.ndarray] = None
    F_channels: Optional[np.ndarray] = None   # (H, 3) per-channel F with one test per channel


def init_state(H: int, r1: float, r_init: Optional[np.ndarray] = None, rgb: bool = False) -> OracleState:
    r = np.full(H, F32(r1), dtype=F32) if r_init is None else np.asarray(r_init, dtype=F32).copy()
    w = 3 * NG if rgb else NG
    return OracleState(r=r, t=np.zeros(H, np.int64), nseen=np.zeros(H, np.int64),
                       S=np.zeros((H, w)), Q=np.zeros((H, w)), tau=np.zeros((H, 3)))


def iterate(params, kernels, st: OracleState, photons, use_grid: bool = True, nthreads: int = 0,
            fcrit_override=None, gathered: Optional[GatherResult] = None,
            connect: Optional[np.ndarray] = None) -> OracleState:
    """One iteration for every kernel (Sec. 5.1 steps 1-4, Eq. radiusupdate, Eq. progressive-VCM-estimator).

    ``fcrit_override`` (callable m -> F_c) replaces the quantile, for forced-decision tests.
    ``connect`` ((H, 3), the vertex-connection term of Eq. VCM-estimator for this iteration, computed
    with the radius this iteration merges with) is added to the iteration's estimate.
    """
    vcm = params.mode == "vcm"
    rgb = getattr(params, "stats", "luma") == "rgb"
    H = kernels.n
    g = gathered if gathered is not None else gather(kernels, photons, st.r, vcm=vcm, use_grid=use_grid,
                                                      nthreads=nthreads, rgb=rgb)
    i = st.iters + 1                                  # 1-based global iteration index
    J = int(photons.J)
    st.J_hist.append(J)
    # retain the statistics of the iterations since the last shrink (Sec. 5.1)
    st.S += g.S
    st.Q += g.Q
    st.t += 1
    st.nseen += g.count.astype(np.int64)
    # m = sum of J over the kept iterations; zero samples included (one sample per light sub-path)
    cumJ = np.concatenate([[0], np.cumsum(st.J_hist[::-1])]).astype(np.float64)
    m = cumJ[st.t]
    Fc = fcrit_override(m) if fcrit_override is not None else f_critical(m, params.alpha_f, NG)
    Fch = None
    if not rgb:
        F = f_statistic(st.S, st.Q, m)
        ssw = within_ss(st.S, st.Q, m)
        valid = (st.nseen > 0) & (ssw > 0) & (m >= 2)
        shrink = valid & (F > Fc)                      # NaN compares false: keep
    else:
        # one test per channel (Sec. 5.1, chromatic light): reject when any channel rejects; the
        # reported F is the largest channel F (NaN channels ignored)
        Fch = np.stack([f_statistic(st.S[:, c * NG:(c + 1) * NG], st.Q[:, c * NG:(c + 1) * NG], m)
                        for c in range(3)], 1)
        sswc = np.stack([within_ss(st.S[:, c * NG:(c + 1) * NG], st.Q[:, c * NG:(c + 1) * NG], m)
                         for c in range(3)], 1)
        col = lambda x: np.asarray(x)[..., None] if np.ndim(x) else x  # noqa: E731
        validc = (st.nseen[:, None] > 0) & (sswc > 0) & col(m >= 2)
        shrink = np.any(validc & (Fch > col(Fc)), axis=1)
        F = np.fmax.reduce(Fch, axis=1)
    F = np.where(st.nseen > 0, F, np.nan)
    # progressive estimate: each iteration with its own radius r_i (Eq. progressive-VCM-estimator)
    r64 = st.r.astype(np.float64)
    norm = 1.0 / (J * math.pi * r64 * r64)
    if vcm:
        st.tau += kernels.cam_beta.T.astype(np.float64) * g.flux * norm[:, None]
    else:
        st.tau += g.flux * norm[:, None]
    if connect is not None:
        st.tau += connect
    # radius update (Eq. radiusupdate); float32 as the radius is a float32 quantity on both sides
    lb = lower_bound(params.rmin, params.alpha, i + 1)
    r_new = np.maximum(F32(params.k) * st.r, lb).astype(F32)
    st.r = np.where(shrink, r_new, st.r).astype(F32)
    st.S[shrink] = 0.0
    st.Q[shrink] = 0.0
    st.t[shrink] = 0
    st.nseen[shrink] = 0
    st.iters = i
    st.count, st.F, st.Fc, st.shrink, st.m = g.count, F, np.broadcast_to(Fc, F.shape).copy(), shrink, m
    st.F_channels = Fch
    return st


def radiance(st: OracleState) -> np.ndarray:
    """L = f_r tau / N per channel with a Lambertian f_r = 1/pi; (H, 3) float64."""
    return st.tau / (math.pi * max(st.iters, 1))


def run(workload, n_iter: Optional[int] = None, use_grid: bool = True, nthreads: int = 0, callback=None):
    p = workload.params
    st = init_state(workload.kernels.n, p.r1)
    for it in range(n_iter if n_iter is not None else p.n_iter):
        ph = workload.photons(it)
        iterate(p, workload.kernels, st, ph, use_grid=use_grid, nthreads=nthreads)
        if callback is not None:
            callback(it, st, ph)
    return st
