"""Pins of the CPU oracle against things other than itself: printed constants of the paper, textbook
routines (one-way ANOVA), closed forms, distribution laws, invariants and exact brute force."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from tests import f32exact as X
from workloads import generators as G

F32 = np.float32
HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    out = {}
    with open(os.path.join(HERE, "golden", "paper_constants.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                k, v = line.split()
                out[k] = float(v)
    return out


# ---------------------------------------------------------------------------------------------
# grouping of the disk (Sec. 3.2.1; 2 annuli x 6 sectors, Sec. 6.1.1)
# ---------------------------------------------------------------------------------------------

def exact_sector(yu: float, yv: float) -> int:
    """Sector by the polar angle of the float32 point taken as an exact real, [60 s, 60 (s+1))."""
    ang = math.atan2(float(yv), float(yu))
    if ang < 0:
        ang += 2 * math.pi
    return min(int(ang // (math.pi / 3)), 5)


def test_group_on_exact_rays(oracle_mod):
    r2 = F32(1.0)
    d2 = F32(0.1)
    assert oracle_mod.group_of(1.0, 0.0, d2, r2) == 0        # 0 deg belongs to sector 0
    assert oracle_mod.group_of(0.0, 1.0, d2, r2) == 1        # 90 deg
    assert oracle_mod.group_of(-1.0, 0.0, d2, r2) == 3       # 180 deg opens sector 3
    assert oracle_mod.group_of(-1.0, -0.0, d2, r2) == 3
    assert oracle_mod.group_of(0.0, -1.0, d2, r2) == 4       # 270 deg
    assert oracle_mod.group_of(0.0, 0.0, F32(0.0), r2) == 0  # centre
    # just inside/outside the 60 and 120 degree lines (no float32 point lies exactly on them)
    for deg, below, above in ((60, 0, 1), (120, 1, 2), (240, 3, 4), (300, 4, 5)):
        for eps, want in ((-1e-4, below), (1e-4, above)):
            a = math.radians(deg) + eps
            assert oracle_mod.group_of(math.cos(a), math.sin(a), d2, r2) == want, (deg, eps)


def test_group_annulus_and_centres(oracle_mod):
    r = F32(0.05)
    r2 = F32(r * r)
    for s in range(6):
        a = math.radians(30 + 60 * s)
        for frac, ann in ((0.5, 0), (0.9, 1), (0.70, 0), (0.72, 1)):
            yu, yv = F32(frac * r * math.cos(a)), F32(frac * r * math.sin(a))
            d2 = X.fma(yv, yv, X.mul(yu, yu))
            assert oracle_mod.group_of(yu, yv, d2, r2) == 6 * ann + s


def test_group_matches_exact_angle_and_symmetry(oracle_mod):
    rng = np.random.default_rng(5)
    pts = rng.uniform(-1, 1, size=(4000, 2)).astype(F32)
    bad = 0
    for yu, yv in pts:
        ang = math.atan2(float(yv), float(yu)) % (math.pi / 3)
        if min(ang, math.pi / 3 - ang) < 1e-6:
            continue                                      # too close to a boundary for atan2
        g = oracle_mod.group_of(yu, yv, F32(0.1), F32(1.0))
        bad += g != exact_sector(yu, yv)
        gm = oracle_mod.group_of(-yu, -yv, F32(0.1), F32(1.0))
        assert gm == (g + 3) % 6                          # 180 degree rotation relabels s -> s+3
    assert bad == 0


def test_groups_are_equal_area(oracle_mod):
    """Uniform points in the disk fall in the 12 groups with probability 1/12 each."""
    rng = np.random.default_rng(11)
    n = 60000
    p = rng.uniform(-1, 1, size=(3 * n, 2)).astype(F32)
    p = p[(p.astype(float) ** 2).sum(1) < 1][:n]
    counts = np.zeros(12, int)
    for yu, yv in p:
        d2 = X.fma(yv, yv, X.mul(yu, yu)) if False else F32(yu * yu + yv * yv)
        counts[oracle_mod.group_of(yu, yv, d2, F32(1.0))] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


def test_frames_orthonormal(oracle_mod):
    rng = np.random.default_rng(3)
    n = rng.normal(size=(3, 500))
    n /= np.linalg.norm(n, axis=0)
    n = n.astype(F32)
    u, v = oracle_mod.frames(n, 500)
    u, v, n64 = u.astype(float), v.astype(float), n.astype(float)
    assert np.allclose((u * v).sum(0), 0, atol=1e-6)
    assert np.allclose((u * n64).sum(0), 0, atol=1e-6)
    assert np.allclose((u * u).sum(0), 1, atol=1e-6)
    assert np.allclose(np.cross(u.T, v.T).T, n64, atol=1e-6)
    ax = np.zeros((3, 6), F32)
    for i in range(3):
        ax[i, 2 * i], ax[i, 2 * i + 1] = 1, -1
    u, v = oracle_mod.frames(ax, 6)
    assert set(np.unique(np.abs(np.concatenate([u.ravel(), v.ravel()])))) <= {0.0, 1.0}
    assert np.array_equal(np.cross(u.T, v.T).T, ax)


# ---------------------------------------------------------------------------------------------
# gather: exact brute force and the grid against all pairs
# ---------------------------------------------------------------------------------------------

def _brute_pair(k, kn, u, v, r, p, pn, f):
    """Exact float32 evaluation of one pair, written from the definitions (disk, map, luminance)."""
    d = [X.sub(k[a], p[a]) for a in range(3)]
    d2 = X.fma(d[2], d[2], X.fma(d[1], d[1], X.mul(d[0], d[0])))
    r2 = X.mul(r, r)
    if not d2 < r2:
        return None
    if kn is not None:
        c = X.fma(kn[2], pn[2], X.fma(kn[1], pn[1], X.mul(kn[0], pn[0])))
        if not c >= F32(0.5):
            return None
    yu = X.fma(d[2], u[2], X.fma(d[1], u[1], X.mul(d[0], u[0])))
    yv = X.fma(d[2], v[2], X.fma(d[1], v[1], X.mul(d[0], v[0])))
    ann = 1 if X.Fr(d2) * 2 >= X.Fr(r2) else 0
    psi = X.fma(F32(0.0722), f[2], X.fma(F32(0.7152), f[1], X.mul(F32(0.2126), f[0])))
    ang = math.atan2(float(yv), float(yu)) % (math.pi / 3)
    ambiguous = min(ang, math.pi / 3 - ang) < 1e-6 and not (yv == 0)
    return 6 * ann + exact_sector(yu, yv), psi, ambiguous


@pytest.mark.parametrize("box", [False, True])
def test_gather_exact_brute_force(oracle_mod, box):
    if box:
        w = G.box_scene(seed=7, res=6, J=900)
    else:
        w = G.small_config0(seed=7, n_side=5, J=400, r1=0.2)
    ks = w.kernels
    ph = w.photons(0)
    r = np.full(ks.n, F32(w.params.r1))
    r[::3] = F32(w.params.r1 * 0.6)
    g = oracle_mod.gather(ks, ph, r, use_grid=False)
    u, v = oracle_mod.frames(ks.nrm, ks.n)
    for h in range(ks.n):
        cnt, S, Q = 0, np.zeros(12), np.zeros(12)
        for j in range(ph.n):
            res = _brute_pair(ks.pos[:, h], None if ks.nrm is None else ks.nrm[:, h], u[:, h], v[:, h], r[h],
                              ph.pos[:, j], None if ph.nrm is None else ph.nrm[:, j], ph.flux[:, j])
            if res is None:
                continue
            grp, psi, amb = res
            assert not amb
            cnt += 1
            S[grp] += float(psi)
            Q[grp] += float(psi) ** 2
        assert g.count[h] == cnt
        np.testing.assert_allclose(g.S[h], S, rtol=1e-12, atol=0)
        np.testing.assert_allclose(g.Q[h], Q, rtol=1e-12, atol=0)


@pytest.mark.parametrize("which", ["plane", "box", "vcm"])
def test_grid_matches_all_pairs(oracle_mod, which):
    vcm = which == "vcm"
    if which == "plane":
        w = G.small_config0(seed=3, n_side=23, J=8000)
    elif which == "box":
        w = G.box_scene(seed=3, res=24, J=20000, r1=0.08)
    else:
        w = G.config4(seed=3, nx=40, ny=24, J=20000, r1=0.03)
    ph = w.photons(0)
    rng = np.random.default_rng(0)
    r = (w.params.r1 * rng.uniform(0.3, 1.0, w.kernels.n)).astype(F32)
    a = oracle_mod.gather(w.kernels, ph, r, vcm=vcm, use_grid=False)
    b = oracle_mod.gather(w.kernels, ph, r, vcm=vcm, use_grid=True)
    assert np.array_equal(a.count, b.count)
    assert a.count.sum() > 0
    for x, y in ((a.S, b.S), (a.Q, b.Q), (a.flux, b.flux)):
        np.testing.assert_allclose(x, y, rtol=1e-12, atol=1e-300)


def test_counts_invariant_under_photon_permutation(oracle_mod):
    w = G.small_config0(seed=4, n_side=12, J=5000)
    ph = w.photons(0)
    perm = np.random.default_rng(1).permutation(ph.n)
    ph2 = G.PhotonBatch(J=ph.J, pos=np.ascontiguousarray(ph.pos[:, perm]), flux=np.ascontiguousarray(ph.flux[:, perm]))
    a = oracle_mod.gather(w.kernels, ph, w.params.r1)
    b = oracle_mod.gather(w.kernels, ph2, w.params.r1)
    assert np.array_equal(a.count, b.count)
    np.testing.assert_allclose(a.S, b.S, rtol=1e-12)


# ---------------------------------------------------------------------------------------------
# F statistic (Eq. f-statistic) and critical value (Sec. 3.2.2)
# ---------------------------------------------------------------------------------------------

def test_f_statistic_matches_one_way_anova(oracle_mod):
    """Explicit 12 x m sample matrix, zeros included, through scipy's one-way ANOVA."""
    rng = np.random.default_rng(2)
    r = F32(0.1)
    k = np.array([0.5, 0.5, 0.0], F32)
    J, T = 7, 3
    st = oracle_mod.init_state(1, float(r))
    ks = G.KernelSet(pos=k[:, None].copy())
    samples = [[] for _ in range(12)]
    for it in range(T):
        pos = np.zeros((3, J), F32)
        flux = np.zeros((3, J), F32)
        groups = []
        for j in range(J):
            grp = int(rng.integers(0, 13))                 # 12 = outside the disk
            if grp < 12:
                s, ann = grp % 6, grp // 6
                rad = (0.45 if ann == 0 else 0.85) * float(r)
                a = math.radians(60 * s + 10 + 40 * rng.random())
                pos[0, j] = F32(0.5 - rad * math.cos(a))    # y = x - x*, so x* = x - y
                pos[1, j] = F32(0.5 - rad * math.sin(a))
            else:
                pos[0, j], pos[1, j] = F32(0.9), F32(0.9)
            flux[:, j] = F32(rng.lognormal(0, 0.7))
            groups.append(grp)
        ph = G.PhotonBatch(J=J, pos=pos, flux=flux)
        oracle_mod.iterate(G.Params(r1=float(r)), ks, st, ph, fcrit_override=lambda m: np.full_like(m, np.inf))
        for j in range(J):
            psi = float(X.fma(F32(0.0722), flux[2, j], X.fma(F32(0.7152), flux[1, j], X.mul(F32(0.2126), flux[0, j]))))
            for grp in range(12):
                samples[grp].append(psi if groups[j] == grp else 0.0)
    want = stats.f_oneway(*[np.array(s) for s in samples]).statistic
    assert st.t[0] == T and st.m[0] == T * J
    np.testing.assert_allclose(st.F[0], want, rtol=1e-12)


def test_f_invariances(oracle_mod):
    rng = np.random.default_rng(8)
    S = rng.uniform(1, 5, size=(20, 12))
    Q = S ** 2 + rng.uniform(1, 3, size=(20, 12))
    m = np.full(20, 1000.0)
    F = oracle_mod.f_statistic(S, Q, m)
    np.testing.assert_allclose(oracle_mod.f_statistic(3 * S, 9 * Q, m), F, rtol=1e-12)
    perm = rng.permutation(12)
    np.testing.assert_allclose(oracle_mod.f_statistic(S[:, perm], Q[:, perm], m), F, rtol=1e-12)


def test_f_critical_paper_constants(oracle_mod):
    g = _golden()
    fc_inf = float(oracle_mod.f_critical(1e13, g["alpha"], int(g["n_groups"])))
    assert round(fc_inf, int(g["fc_limit_printed_decimals"])) == g["fc_limit_printed"]
    chi = fc_inf * (g["n_groups"] - 1)                    # F(11, inf) = chi2_11 / 11
    dec = int(g["chi_c_printed_decimals"])
    assert math.floor(chi * 10 ** dec) / 10 ** dec == g["chi_c_printed"]


def test_f_critical_closed_forms(oracle_mod):
    for d2 in (6.0, 120.0, 1.2e5, 1.2e6):
        for p in (0.95, 0.99):
            want = (d2 / 2) * math.expm1(-(2 / d2) * math.log1p(-p))    # F(2, d2) quantile
            got = float(oracle_mod.f_critical(d2 / 3 + 1, 1 - p, n_groups=3))
            assert abs(got - want) <= 1e-9 * want
            tq = stats.t.ppf((1 + p) / 2, d2)                          # F(1, d2) = t^2
            got1 = float(oracle_mod.f_critical(d2 / 2 + 1, 1 - p, n_groups=2))
            assert abs(got1 - tq * tq) <= 1e-9 * got1


def _f_samples(oracle_mod, t_keep, n_batches, seed):
    w = G.uniform_config(seed=seed, n_kernels_side=9, J=30000, r1=0.045)
    Fs = []
    for b in range(n_batches):
        st = oracle_mod.init_state(w.kernels.n, w.params.r1)
        for t in range(t_keep):
            oracle_mod.iterate(w.params, w.kernels, st, w.photons(b * t_keep + t),
                               fcrit_override=lambda m: np.full_like(m, np.inf))
        Fs.append(st.F.copy())
    return np.concatenate(Fs), st.m[0]


@pytest.mark.parametrize("t_keep,n_batches", [(1, 24), (4, 8)])
def test_f_law_under_uniform_density(oracle_mod, t_keep, n_batches):
    """Constant contribution over the disk (H0 holds): F ~ F(11, 12 (m - 1)), m = t J; the rejection
    rate at alpha_F = 0.05 stays in its binomial range. A wrong m, n or scale fails the KS test."""
    F, m = _f_samples(oracle_mod, t_keep, n_batches, seed=40 + t_keep)
    assert np.isfinite(F).all()
    d2 = 12 * (m - 1)
    assert stats.kstest(F, stats.f(11, d2).cdf).pvalue > 1e-3
    rej = int((F > oracle_mod.f_critical(m, 0.05)).sum())
    assert stats.binomtest(rej, F.size, 0.05).pvalue > 1e-4


# ---------------------------------------------------------------------------------------------
# radius update (Eq. radiusupdate) and estimate (Eq. progressive-VCM-estimator)
# ---------------------------------------------------------------------------------------------

def test_forced_reject_follows_closed_form(oracle_mod):
    w = G.uniform_config(seed=5, n_kernels_side=4, J=20000, r1=0.05)
    p = G.Params(r1=0.05, k=0.7, alpha=0.75, rmin=0.02)       # large r_min so the bound binds
    st = oracle_mod.init_state(w.kernels.n, p.r1)
    for it in range(12):
        oracle_mod.iterate(p, w.kernels, st, w.photons(it), fcrit_override=lambda m: np.zeros_like(m))
        i = it + 2                                            # radius used by iteration i
        want = max(p.k ** (i - 1) * p.r1, p.rmin * (i ** ((p.alpha - 1) / 2)))
        np.testing.assert_allclose(st.r, want, rtol=2e-6)


def test_radius_never_grows_and_empty_disk_keeps(oracle_mod):
    w = G.small_config0(seed=9, n_side=20, J=4000, n_iter=8)
    # one kernel far outside the photon support keeps r1 with an undefined statistic
    pos = np.concatenate([w.kernels.pos, np.array([[3.0], [3.0], [0.0]], F32)], axis=1)
    ks = G.KernelSet(pos=pos)
    st = oracle_mod.init_state(ks.n, w.params.r1)
    prev = st.r.copy()
    for it in range(8):
        oracle_mod.iterate(w.params, ks, st, w.photons(it))
        assert (st.r <= prev).all()
        prev = st.r.copy()
        assert np.isnan(st.F[-1]) and not st.shrink[-1] and st.r[-1] == F32(w.params.r1)
    assert (st.r < F32(w.params.r1)).any()


def _hold_radius(oracle_mod, w, n_iter):
    st = oracle_mod.init_state(w.kernels.n, w.params.r1)
    for it in range(n_iter):
        oracle_mod.iterate(w.params, w.kernels, st, w.photons(it), fcrit_override=lambda m: np.full_like(m, np.inf))
    return st


def test_radiance_uniform_density_closed_form(oracle_mod):
    """Uniform density, interior kernels: E[L] = f_r E[Phi] = exp(0.125) / pi per channel."""
    w = G.uniform_config(seed=12, n_kernels_side=9, J=40000, r1=0.045)
    N = 6
    st = _hold_radius(oracle_mod, w, N)
    L = oracle_mod.radiance(st)
    truth = math.exp(0.125) / math.pi
    r = 0.045
    var_one = math.exp(0.5) / (40000 * math.pi * r * r) / math.pi ** 2       # per kernel, per iteration
    se = math.sqrt(var_one / (N * w.kernels.n))
    assert np.all(np.abs(L.mean(0) - truth) < 4.5 * se)


def _disk_mass(density, cx, cy, r, n=400):
    """Integral of the density over the disk intersected with the unit square (polar midpoint rule)."""
    rr = (np.arange(n) + 0.5) / n * r
    th = (np.arange(n) + 0.5) / n * 2 * math.pi
    R, T = np.meshgrid(rr, th, indexing="ij")
    x, y = cx + R * np.cos(T), cy + R * np.sin(T)
    inside = (x >= 0) & (x <= 1) & (y >= 0) & (y <= 1)
    return float((density(x, y) * inside * R).sum() * (r / n) * (2 * math.pi / n))


def test_radiance_config0_density_kernel_smoothed(oracle_mod):
    """Per kernel, E[L] = f_r E[Phi] (1 / pi r^2) * (density mass in the disk); z-scores ~ N(0, 1)."""
    w = G.config0(seed=13, n_side=12, J=60000, n_iter=4)
    N = 4
    st = _hold_radius(oracle_mod, w, N)
    L = oracle_mod.radiance(st)[:, 0]
    r = float(F32(0.05))
    ePhi, ePhi2 = math.exp(0.125), math.exp(0.5)
    z = []
    for h in range(w.kernels.n):
        mass = _disk_mass(G.mixture_density, float(w.kernels.pos[0, h]), float(w.kernels.pos[1, h]), r)
        mean = ePhi * mass / (math.pi * r * r) / math.pi
        var = ePhi2 * mass / (60000 * (math.pi * r * r) ** 2) / math.pi ** 2 / N
        z.append((L[h] - mean) / math.sqrt(var))
    z = np.array(z)
    assert abs(z.mean()) < 4.5 / math.sqrt(z.size)
    assert 0.6 < (z ** 2).mean() < 1.6


def test_box_direct_lighting_estimate(oracle_mod):
    """Box scene at held radius: far from shadow and face edges the estimate matches E/pi of the point
    light to within the O(r^2) smoothing bias and the noise."""
    w = G.box_scene(seed=14, res=32, J=400000, r1=0.03)
    N = 3
    st = _hold_radius(oracle_mod, w, N)
    L = oracle_mod.radiance(st)[:, 0]
    sc = w.info["scene"]
    E = sc.irradiance(w.kernels.pos, w.kernels.nrm) / math.pi
    pos = w.kernels.pos.astype(float)
    edge = np.minimum(pos, 1 - pos)
    on_face = np.abs(w.kernels.nrm.astype(float))
    dist_edge = np.where(on_face > 0, np.inf, edge).min(0)
    far = dist_edge > 0.08
    # no shadow boundary within the kernel: visibility equal at the centre and along a ring
    ring_ok = np.ones(w.kernels.n, bool)
    u, v = oracle_mod.frames(w.kernels.nrm, w.kernels.n)
    for a in np.linspace(0, 2 * math.pi, 16, endpoint=False):
        q = (pos + 0.03 * (math.cos(a) * u + math.sin(a) * v)).astype(F32)
        ring_ok &= (sc.irradiance(q, w.kernels.nrm) > 0) == (E > 0)
    sel = far & ring_ok & (E > 0)
    assert sel.sum() > 100
    rel = L[sel] / E[sel] - 1
    assert abs(np.median(rel)) < 0.03
    # fully shadowed kernels receive nothing
    dark = far & ring_ok & (E == 0)
    if dark.any():
        assert np.all(L[dark] == 0)


# ---------------------------------------------------------------------------------------------
# vertex merging weight (Eq. mis-weight, beta = 1): special cases only
# ---------------------------------------------------------------------------------------------

def test_vcm_zero_partials_reduce_to_ppm(oracle_mod):
    w = G.config4(seed=21, nx=24, ny=16, J=20000, r1=0.03, n_iter=3)
    ks = w.kernels
    ks0 = G.KernelSet(pos=ks.pos, nrm=ks.nrm, cam_beta=np.ones_like(ks.cam_beta), cam_mis=np.zeros_like(ks.cam_mis))
    sv = oracle_mod.init_state(ks.n, w.params.r1)
    sp = oracle_mod.init_state(ks.n, w.params.r1)
    pp = G.Params(r1=w.params.r1)
    for it in range(3):
        ph = w.photons(it)
        ph0 = G.PhotonBatch(J=ph.J, pos=ph.pos, flux=ph.flux, nrm=ph.nrm, mis=np.zeros_like(ph.mis))
        oracle_mod.iterate(w.params, ks0, sv, ph0)
        oracle_mod.iterate(pp, ks0, sp, ph0)
        assert np.array_equal(sv.count, sp.count)
        assert np.array_equal(sv.r, sp.r)
        np.testing.assert_array_equal(sv.tau, sp.tau)
        np.testing.assert_array_equal(np.nan_to_num(sv.F), np.nan_to_num(sp.F))


def test_vcm_weight_limits(oracle_mod):
    """One light vertex at the kernel: w from the gathered sum; w grows with r, -> 1 for large r when
    dVM = 0, and falls like r^2 for small r."""
    ks = G.KernelSet(pos=np.array([[0.5], [0.5], [0.0]], F32), nrm=np.array([[0.0], [0.0], [1.0]], F32),
                     cam_beta=np.ones((3, 1), F32), cam_mis=np.array([[0.7], [0.2], [0.0]], F32))
    ph = G.PhotonBatch(J=1000, pos=np.array([[0.5], [0.5], [0.0]], F32), flux=np.ones((3, 1), F32),
                       nrm=np.array([[0.0], [0.0], [1.0]], F32), mis=np.array([[0.4], [0.3], [0.0]], F32))
    rs = np.geomspace(1e-4, 10.0, 30)
    ws = np.array([oracle_mod.gather(ks, ph, np.array([r], F32), vcm=True).flux[0, 0] for r in rs])
    assert np.all(np.diff(ws) > 0)
    assert abs(ws[-1] - 1.0) < 1e-5
    small = ws[:3] / rs[:3] ** 2
    np.testing.assert_allclose(small, small[0], rtol=1e-3)
    eta = 1000 * math.pi * rs[0] ** 2
    np.testing.assert_allclose(ws[0], eta / (eta + 0.7 + 0.4), rtol=1e-4)


def _one_pair_weight(oracle_mod, r, J, cam, light):
    """Merge weight w of a single light vertex lying on a single camera vertex, read back from the
    gathered flux (throughputs of one, so the flux sum is w itself). cam and light are the partials
    (dVCM, dVC, dVM)."""
    ks = G.KernelSet(pos=np.array([[0.5], [0.5], [0.0]], F32), nrm=np.array([[0.0], [0.0], [1.0]], F32),
                     cam_beta=np.ones((3, 1), F32), cam_mis=np.array(cam, F32).reshape(3, 1))
    ph = G.PhotonBatch(J=J, pos=np.array([[0.5], [0.5], [0.0]], F32), flux=np.ones((3, 1), F32),
                       nrm=np.array([[0.0], [0.0], [1.0]], F32), mis=np.array(light, F32).reshape(3, 1))
    g = oracle_mod.gather(ks, ph, np.array([r], F32), vcm=True)
    assert g.count[0] == 1
    return g.flux[0, 0]


def test_vcm_weight_merging_partial_term(oracle_mod):
    """Eq. mis-weight with the vertex-connection partials dVCM zero on both sides: only the dVM p
    terms remain, and with a direction pdf of 1/pi (Lambertian at normal incidence) the weight is
    1 / (1 + (dVM_L + dVM_C) / pi) whatever the radius (no eta left in it). Dropping the dVM term
    would give 1; a pdf of 1 would give 1 / (1 + dVM_L + dVM_C)."""
    for dvm_l, dvm_c in ((0.3, 0.2), (1.0, 0.0), (0.0, 2.5), (0.9, 0.6)):
        want = 1.0 / (1.0 + (dvm_l + dvm_c) / math.pi)
        for r in (1e-4, 3e-3, 0.05, 2.0):
            for J in (1, 1000, 4_000_000):
                got = _one_pair_weight(oracle_mod, r, J, (0.0, 0.9, dvm_c), (0.0, 0.8, dvm_l))
                assert abs(got - want) <= 4e-7 * want, (dvm_l, dvm_c, r, J, got, want)


def test_vcm_weight_mixed_hand_evaluated(oracle_mod):
    """All four partials non-zero, evaluated by hand: J = 1000, r = 0.01 give eta = J pi r^2 = pi/10;
    W_L = 0.4 / eta + 0.3 / pi = 4.3 / pi and W_C = 0.7 / eta + 0.2 / pi = 7.2 / pi, so
    w = 1 / (1 + 11.5 / pi) = pi / (pi + 11.5) ~ 0.2145663. dVC (0.55, 0.45 here) plays no part in
    merging."""
    got = _one_pair_weight(oracle_mod, 0.01, 1000, (0.7, 0.55, 0.2), (0.4, 0.45, 0.3))
    want = math.pi / (math.pi + 11.5)
    assert abs(want - 0.2145663) < 1e-7
    assert abs(got - want) <= 4e-7 * want, (got, want)


# ---------------------------------------------------------------------------------------------
# no test while the within-group degrees of freedom vanish (Sec. 3.2.2: d2 = n (m - 1))
# ---------------------------------------------------------------------------------------------

def test_single_emitted_subpath_has_no_test(oracle_mod):
    """J_emitted = 1 gives m = 1 sample per group, so F(n - 1, n (m - 1)) has no within-group degrees
    of freedom: no critical value (NaN), no F, the radius is kept. The estimate still takes the
    light vertex: tau = flux / (J pi r^2). One more iteration with J = 1 gives m = 2 and the test
    resumes against the quantile of F(11, 12) (d2 = 12, not 24 or 11)."""
    ks = G.KernelSet(pos=np.array([[0.5], [0.5], [0.0]], F32))
    p = G.Params(r1=0.05)
    st = oracle_mod.init_state(1, p.r1)
    ph1 = G.PhotonBatch(J=1, pos=np.array([[0.51], [0.5], [0.0]], F32), flux=np.array([[2.0], [1.0], [0.5]], F32))
    oracle_mod.iterate(p, ks, st, ph1)
    assert st.count[0] == 1 and st.m[0] == 1.0
    assert np.isnan(st.Fc[0]) and np.isnan(st.F[0]) and not st.shrink[0]
    assert st.r[0] == F32(0.05) and st.t[0] == 1
    np.testing.assert_allclose(st.tau[0], np.array([2.0, 1.0, 0.5]) / (math.pi * float(F32(0.05)) ** 2), rtol=1e-12)
    # second sub-path in another sector: m = 2, d2 = 12
    ph2 = G.PhotonBatch(J=1, pos=np.array([[0.49], [0.5], [0.0]], F32), flux=np.array([[2.0], [1.0], [0.5]], F32))
    oracle_mod.iterate(p, ks, st, ph2)
    assert st.m[0] == 2.0
    np.testing.assert_allclose(st.Fc[0], stats.f.ppf(0.95, 11, 12), rtol=1e-9)
    # two equal samples in two of the 12 groups (sectors 3 and 0 of the inner annulus), zero padding
    # elsewhere: one-way ANOVA of the explicit 12 x 2 matrix (F is scale-invariant and does not
    # depend on which two groups)
    groups = [np.zeros(2) for _ in range(12)]
    groups[0][0] = 1.0
    groups[1][1] = 1.0
    np.testing.assert_allclose(st.F[0], stats.f_oneway(*groups).statistic, rtol=1e-6)
