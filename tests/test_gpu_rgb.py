"""One F-test per RGB channel on the GPU against the oracle (same parity bar as the luminance test:
counts and radii bit-exact, decisions exact outside the 1e-6 band of any channel, F within its
rounding bound, radiance 1e-5)."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_04411_amd import hk
    hk.lib()
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _rgb(w):
    return dataclasses.replace(w, params=dataclasses.replace(w.params, stats="rgb"))


def _G():
    from workloads import generators as G
    return G


def _parity():
    from tests import gpu_parity
    return gpu_parity


def test_rgb_chromatic_caustic_plane():
    """Config 0's density with a chromatic caustic: red-shifted at its centre, blue-shifted around."""
    G = _G()
    w0 = G.config0(seed=3, n_side=32, J=60_000, n_iter=6, r1=0.06)
    F32 = np.float32

    def photons(it):
        ph = w0.photons(it)
        d2 = (ph.pos[0] - 0.7) ** 2 + (ph.pos[1] - 0.3) ** 2
        wgt = np.exp(-d2 / (2 * 0.03 ** 2))
        f = ph.flux.copy()
        f[0] = (f[0] * (1.0 + 0.8 * wgt)).astype(F32)
        f[2] = (f[2] * (1.0 - 0.8 * wgt)).astype(F32)
        return G.PhotonBatch(J=ph.J, pos=ph.pos, flux=f)

    w = _rgb(dataclasses.replace(w0, photon_fn=photons))
    rep = _parity().run_parity(w, 6)
    assert rep.shrinks > 300


def test_rgb_isoluminant_stripes():
    """Equal luminance everywhere, alternating red and blue stripes: the channel test rejects almost
    every kernel at once, on the GPU as in the oracle."""
    G = _G()
    r1 = 0.03
    w0 = G.uniform_config(7, 12, 200_000, r1, n_iter=2)
    F32 = np.float32
    a, b = F32(0.0722) * F32(4.0), F32(0.2126) * F32(4.0)

    def photons(it):
        ph = w0.photons(it)
        red = (np.floor(ph.pos[0] / r1).astype(np.int64) % 2) == 0
        f = np.zeros_like(ph.flux)
        f[0] = np.where(red, a, 0.0)
        f[2] = np.where(red, 0.0, b)
        return G.PhotonBatch(J=ph.J, pos=ph.pos, flux=f)

    w = _rgb(dataclasses.replace(w0, photon_fn=photons))
    rep = _parity().run_parity(w, 2)
    assert rep.shrinks > 0.95 * rep.kernels


def test_rgb_box_with_normals():
    G = _G()
    w = _rgb(G.box_scene(seed=1, res=32, J=150_000, n_iter=4))
    _parity().run_parity(w, 4)


def test_rgb_vertex_merging():
    G = _G()
    w = _rgb(G.config4(seed=4, nx=96, ny=54, J=150_000, r1=0.012, n_iter=4))
    _parity().run_parity(w, 4)


def test_rgb_batched_sets_match_solo():
    """The per-channel gather in a batch of uneven sets is bit-identical to the sets run alone."""
    G = _G()
    GP = _parity()
    from paper_2504_04411_amd.estimator import DevicePhotons
    ws = [_rgb(w) for w in G.config2(seed=2, n_sets=6, scale=0.01, n_iter=2)]
    a, b = GP.make_estimator(ws[0]), GP.make_estimator(ws[0])
    for s, w in enumerate(ws):
        for e in (a, b):
            e.set_kernels(s, w.kernels.pos, r1=w.params.r1, rmin=w.params.rmin)
    ids = list(range(len(ws)))
    for it in range(2):
        dps = [DevicePhotons.upload(w.photons(it)) for w in ws]
        a.iterate(ids, dps)
        for s in ids:
            b.iterate([s], [dps[s]])
        for s in ids:
            Sa, Qa, Ta = (x.cpu().numpy() for x in a.sums(s))
            Sb, Qb, Tb = (x.cpu().numpy() for x in b.sums(s))
            assert Sa.shape[1] == 36
            assert np.array_equal(Sa, Sb) and np.array_equal(Qa, Qb) and np.array_equal(Ta, Tb)
            assert np.array_equal(a.radii(s).cpu().numpy(), b.radii(s).cpu().numpy())
