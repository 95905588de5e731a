"""GPU parity of the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_04411_amd import hk
    hk.lib()          # fails loudly when libhk.so is missing
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _parity():
    from tests import gpu_parity
    return gpu_parity


def _G():
    from workloads import generators as G
    return G


def test_plane_small_ragged_tiles():
    """529 kernels = 8 full tiles + a ragged tile of 17; 6 iterations."""
    G = _G()
    w = G.small_config0(seed=0, n_side=23, J=6000, n_iter=6)
    _parity().run_parity(w, 6)


def test_plane_config0_full_trajectory():
    """64 x 64 kernels, 100k photons per iteration, 16 iterations, every kernel compared."""
    G = _G()
    rep = _parity().run_parity(G.config0(seed=0), 16)
    assert rep.shrinks > 1000


def test_box_small_with_normals():
    G = _G()
    w = G.box_scene(seed=1, res=40, J=200_000, n_iter=8)
    rep = _parity().run_parity(w, 8)
    assert rep.shrinks > 100


def test_box_config1_full_size_sampled():
    """Full box workload (512 x 512 kernels, 2M photons): all kernels on the GPU, 2048 sampled kernels
    (random plus the hottest ceiling kernels near the light) through the oracle."""
    G = _G()
    w = G.config1(seed=1)
    rng = np.random.default_rng(0)
    pos = w.kernels.pos
    d2 = ((pos - np.array([[0.5], [0.9], [0.5]], np.float32)) ** 2).sum(0)
    hot = np.argsort(d2)[:128]
    idx = np.unique(np.concatenate([rng.choice(w.kernels.n, 1920, replace=False), hot]))
    _parity().run_parity(w, 3, idx=idx)


def test_vcm_small():
    G = _G()
    w = G.config4(seed=4, nx=120, ny=68, J=200_000, r1=0.01, n_iter=6)
    rep = _parity().run_parity(w, 6)
    assert rep.shrinks > 0


def test_vcm_config4_full_size_sampled():
    """1920 x 1080 camera vertices, 4M light vertices: 2048 sampled kernels through the oracle."""
    G = _G()
    w = G.config4(seed=4)
    idx = np.sort(np.random.default_rng(1).choice(w.kernels.n, 2048, replace=False))
    _parity().run_parity(w, 2, idx=idx)


def test_edge_cases_empty_outside_single():
    """No stored photons, photons all outside the domain, one kernel, a tile-multiple and +1."""
    G = _G()
    base = G.small_config0(seed=5, n_side=8, J=3000)
    empty = G.PhotonBatch(J=500, pos=np.zeros((3, 0), np.float32), flux=np.zeros((3, 0), np.float32))
    far = base.photons(1)
    far = G.PhotonBatch(J=far.J, pos=far.pos + np.float32(5.0), flux=far.flux)
    seq = [empty, base.photons(0), far, base.photons(2), empty, base.photons(3)]
    _parity().run_parity(base, len(seq), photons_fn=lambda it: seq[it])
    for n in (1, 64, 65):
        pos = G.grid_kernels(n, 1)
        w = G.Workload("line", base.params, G.KernelSet(pos=pos), base.photon_fn, 5)
        _parity().run_parity(w, 3)


def test_varying_J_and_partial_storage():
    """J_emitted changes between iterations (critical values recomputed for every kept t) and only part
    of the emitted sub-paths are stored."""
    G = _G()
    w = G.small_config0(seed=6, n_side=20, J=8000, n_iter=6, r1=0.06)

    def photons(it):
        ph = w.photons(it)
        keep = ph.n - 1000 * (it % 3)
        return G.PhotonBatch(J=ph.J + 7 * it, pos=np.ascontiguousarray(ph.pos[:, :keep]),
                             flux=np.ascontiguousarray(ph.flux[:, :keep]))

    _parity().run_parity(w, 6, photons_fn=photons)


def test_non_finite_flux_keeps_radius():
    """A NaN flux inside a disk makes that kernel's F undefined, which keeps the radius (both sides)."""
    G = _G()
    w = G.small_config0(seed=7, n_side=12, J=4000, n_iter=3)

    def photons(it):
        ph = w.photons(it)
        f = ph.flux.copy()
        f[:, :5] = np.nan
        return G.PhotonBatch(J=ph.J, pos=ph.pos, flux=f)

    _parity().run_parity(w, 3, photons_fn=photons)


def test_determinism_bitwise():
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    G = _G()
    w = G.small_config0(seed=8, n_side=30, J=20000, n_iter=4)
    outs = []
    for _ in range(2):
        est = Estimator(w.params.r1)
        est.set_kernels(0, w.kernels.pos)
        for it in range(4):
            est.iterate([0], [DevicePhotons.upload(w.photons(it))])
        S, Q, tau = est.sums(0)
        outs.append((est.radii(0).cpu().numpy(), S.cpu().numpy(), Q.cpu().numpy(), tau.cpu().numpy()))
        est.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_group_sums_error_against_float64_oracle():
    """Retained group sums and the estimate against the oracle after 16 iterations of config 0.

    Bound: the group sums are float64 on both sides, the float32 samples and their squares exact in
    float64, and every addition of a nonnegative term rounds by at most e = 2^-53 of the running sum.
    A kernel's sum takes at most N = 16 x 100k samples, 64 lane partials and one retained sum per
    iteration, the oracle's at most N samples, so |dS| <= (2 N + 65 x 16) e S. The estimate is a
    compensated float32 pair updated once per iteration with a float32 quotient (a few u = 2^-24
    relative each)."""
    from oracle import oracle as O
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    G = _G()
    w = G.config0(seed=0)
    est = Estimator(w.params.r1)
    est.set_kernels(0, w.kernels.pos)
    st = O.init_state(w.kernels.n, w.params.r1)
    for it in range(16):
        ph = w.photons(it)
        est.iterate([0], [DevicePhotons.upload(ph)])
        O.iterate(w.params, w.kernels, st, ph)
    S, Q, tau = (x.cpu().numpy() for x in est.sums(0))
    same = est.radii(0).cpu().numpy() == st.r
    eS = np.abs(S - st.S)[same].max() / max(np.abs(st.S[same]).max(), 1e-300)
    eQ = np.abs(Q - st.Q)[same].max() / max(np.abs(st.Q[same]).max(), 1e-300)
    rel_tau = (np.abs(tau - st.tau) / np.maximum(np.abs(st.tau), 1e-300))[same].max()
    print(f"float64 group sums vs the oracle: max |dS|/max|S| = {eS:.3e}, |dQ|/max|Q| = {eQ:.3e}, "
          f"max rel tau = {rel_tau:.3e}", flush=True)
    bound = (2 * 16 * 100_000 + 65 * 16) * 2.0 ** -53
    assert eS <= bound and eQ <= bound and rel_tau < 1e-6
    est.close()


def test_lower_bound_binds():
    """Eq. radiusupdate's lower bound r_min sqrt((i+1)^(alpha-1)) reached on the device: box 40 x 40
    with r_min = 0.3 r1 and k = 0.5, 12 iterations. Radii are compared bit for bit every iteration,
    and many kernels must sit exactly on the bound of the iteration that shrank them."""
    from oracle import oracle as O
    from paper_2504_04411_amd.estimator import DevicePhotons
    G = _G()
    P = _parity()
    w = G.box_scene(seed=1, res=40, J=200_000, n_iter=12)
    w.params.k = 0.5
    w.params.rmin = 0.3 * w.params.r1
    est = P.make_estimator(w)
    est.set_kernels(0, w.kernels.pos, w.kernels.nrm)
    tr = P.Tracker(w)
    on_bound = 0
    for it in range(12):
        ph = w.photons(it)
        est.iterate([0], [DevicePhotons.upload(ph)])
        tr.step(est, 0, ph)
        lb = O.lower_bound(w.params.rmin, w.params.alpha, it + 2)
        r = est.radii(0).cpu().numpy()
        on_bound += int((tr.ost.shrink & (r == lb)).sum())
        assert np.all(r >= lb)
    rep = tr.finish(est, 0)
    est.close()
    print(f"  shrinks onto the lower bound: {on_bound}; {rep}", flush=True)
    assert on_bound > 100


def test_single_emitted_subpath_no_test():
    """J_emitted = 1: m = 1 leaves F(11, 12 (m - 1)) without within-group degrees of freedom, so no
    kernel is tested (critical value NaN) and every radius is kept; the next iteration with J = 1
    (m = 2) tests against F(11, 12). Mixed with ordinary batches before and after."""
    G = _G()
    base = G.small_config0(seed=14, n_side=10, J=3000)
    k = base.kernels.pos
    one = lambda j: G.PhotonBatch(J=1, pos=np.ascontiguousarray(k[:, j:j + 1] + np.float32(0.004)),  # noqa: E731
                                  flux=np.ones((3, 1), np.float32))
    none = G.PhotonBatch(J=1, pos=np.zeros((3, 0), np.float32), flux=np.zeros((3, 0), np.float32))
    seq = [one(11), one(12), none, base.photons(0), one(40), base.photons(1), one(41)]
    _parity().run_parity(base, len(seq), photons_fn=lambda it: seq[it])
