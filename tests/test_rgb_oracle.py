"""Pins of the oracle's one-test-per-channel mode (Sec. 5.1: the luminance test can miss chromatic
structure; a kernel then rejects when any RGB channel rejects)."""
import numpy as np
from scipy import stats

from workloads import generators as G

F32 = np.float32


def _gray(ph):
    f = np.repeat(ph.flux[:1], 3, 0)
    return G.PhotonBatch(J=ph.J, pos=ph.pos, flux=f, nrm=ph.nrm, mis=ph.mis)


def test_gray_light_gives_three_equal_channel_tests(oracle_mod):
    """R = G = B: the three channel statistics coincide, and they match the luminance test up to the
    float32 rounding of the luminance (F is scale-invariant)."""
    w = G.config0(seed=5, n_side=20, J=30_000, n_iter=3, r1=0.06)
    pl = G.Params(r1=w.params.r1)
    pc = G.Params(r1=w.params.r1, stats="rgb")
    sl = oracle_mod.init_state(w.kernels.n, w.params.r1)
    sc = oracle_mod.init_state(w.kernels.n, w.params.r1, rgb=True)
    for it in range(3):
        ph = _gray(w.photons(it))
        oracle_mod.iterate(pl, w.kernels, sl, ph)
        oracle_mod.iterate(pc, w.kernels, sc, ph)
        Fc = sc.F_channels
        assert np.array_equal(np.nan_to_num(Fc[:, 0]), np.nan_to_num(Fc[:, 1]))
        assert np.array_equal(np.nan_to_num(Fc[:, 0]), np.nan_to_num(Fc[:, 2]))
        ok = np.isfinite(sl.F)
        assert np.all(np.abs(sc.F[ok] - sl.F[ok]) <= 1e-5 * np.maximum(1.0, sl.F[ok]))
        far = ok & (np.abs(sl.F - sl.Fc) > 1e-4)
        assert np.array_equal(sc.shrink[far], sl.shrink[far])
        assert np.array_equal(sc.r[far], sl.r[far])


def _isoluminant(seed, n_kernels_side=12, J=200_000, r1=0.03):
    """Uniform density; stripes of width r1 along x alternate red (R = a) and blue (B = b) light with
    0.2126 a = 0.0722 b: every photon has the same float32 luminance, the colours do not."""
    w = G.uniform_config(seed, n_kernels_side, J, r1)
    a = F32(0.0722) * F32(4.0)          # exact scalings: 0.2126 a and 0.0722 b are the same product
    b = F32(0.2126) * F32(4.0)

    def photons(it):
        ph = w.photons(it)
        red = (np.floor(ph.pos[0] / r1).astype(np.int64) % 2) == 0
        f = np.zeros_like(ph.flux)
        f[0] = np.where(red, a, 0.0)
        f[2] = np.where(red, 0.0, b)
        return G.PhotonBatch(J=ph.J, pos=ph.pos, flux=f)
    return w, photons


def test_isoluminant_stripes_only_the_channel_test_sees():
    from oracle import oracle as O
    from tests import f32exact as X
    w, photons = _isoluminant(7)

    def lum(R, G_, B):
        return X.fma(0.0722, B, X.fma(0.7152, G_, X.mul(0.2126, R)))
    a, b = F32(0.0722) * F32(4.0), F32(0.2126) * F32(4.0)
    assert lum(a, 0.0, 0.0) == lum(0.0, 0.0, b)     # the two colours have equal float32 luminance
    pl = G.Params(r1=w.params.r1)
    pc = G.Params(r1=w.params.r1, stats="rgb")
    sl = O.init_state(w.kernels.n, w.params.r1)
    sc = O.init_state(w.kernels.n, w.params.r1, rgb=True)
    ph = photons(0)
    O.iterate(pl, w.kernels, sl, ph)
    O.iterate(pc, w.kernels, sc, ph)
    # luminance: constant samples, so only position noise between groups -> rejects at about alpha_F
    rl = int(sl.shrink.sum())
    assert stats.binomtest(rl, sl.shrink.size, 0.05).pvalue > 1e-4
    # channels: red and blue fill different sectors -> every kernel rejects
    assert sc.shrink.mean() > 0.95
    assert np.all(sc.F[sc.shrink] > sc.Fc[sc.shrink])


def test_vcm_channel_test_with_zero_partials_reduces_to_ppm(oracle_mod):
    w = G.config4(seed=22, nx=20, ny=12, J=20000, r1=0.03, n_iter=2)
    ks = w.kernels
    ks0 = G.KernelSet(pos=ks.pos, nrm=ks.nrm, cam_beta=np.ones_like(ks.cam_beta), cam_mis=np.zeros_like(ks.cam_mis))
    pv = G.Params(r1=w.params.r1, mode="vcm", stats="rgb")
    pp = G.Params(r1=w.params.r1, stats="rgb")
    sv = oracle_mod.init_state(ks.n, w.params.r1, rgb=True)
    sp = oracle_mod.init_state(ks.n, w.params.r1, rgb=True)
    for it in range(2):
        ph = w.photons(it)
        ph0 = G.PhotonBatch(J=ph.J, pos=ph.pos, flux=ph.flux, nrm=ph.nrm, mis=np.zeros_like(ph.mis))
        oracle_mod.iterate(pv, ks0, sv, ph0)
        oracle_mod.iterate(pp, ks0, sp, ph0)
        assert np.array_equal(sv.r, sp.r)
        np.testing.assert_array_equal(np.nan_to_num(sv.F_channels), np.nan_to_num(sp.F_channels))
