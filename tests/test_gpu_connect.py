"""The vertex-connection half on the GPU (hk_connect_box, the emission's merging partials, the
graph with HK_BOX_CONNECT) against the oracle: partials bit-identical, the connection term within
float32 rounding with identical shadow decisions, and the whole vertex-merging iteration with the
connection in parity with the oracle's."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

F32 = np.float32


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_04411_amd import hk
    hk.lib()
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _scene(box):
    from paper_2504_04411_amd import hk
    return hk.box_scene(box.light, box.sphere_c, box.sphere_r, box.power)


def _vcm_box(res, seed=0, r1=0.02, beta="ones"):
    from workloads import generators as G
    scene = G.BoxScene(res=res)
    pos, nrm, _ = scene.hit_points()
    H = pos.shape[1]
    if beta == "ones":
        cb = np.ones((3, H), F32)
    else:
        cb = np.random.default_rng(seed).lognormal(0.0, 0.5, (3, H)).astype(F32)
    ks = G.KernelSet(pos=pos, nrm=nrm, cam_beta=cb, cam_mis=np.zeros((3, H), F32))
    w = G.Workload("box-vcm", G.Params(r1=r1, mode="vcm"), ks, None, seed, 0, info=dict(scene=scene))
    return w


def _estimator(w):
    from tests import gpu_parity as GP
    est = GP.make_estimator(w)
    ks = w.kernels
    est.set_kernels(0, ks.pos, ks.nrm, None, ks.cam_beta, ks.cam_mis)
    return est


def _compact(pos, nrm, flux, mis, J):
    from workloads import generators as G
    keep = np.isfinite(pos[0])
    return G.PhotonBatch(J=J, pos=pos[:, keep], flux=flux[:, keep], nrm=nrm[:, keep], mis=mis[:, keep])


def test_emitted_partials_match_oracle():
    from oracle import emit as OE
    w = _vcm_box(16)
    est = _estimator(w)
    box = OE.Box()
    J = 300_000
    out = est.emit_box(0, _scene(box), 11, J)
    torch.cuda.synchronize()
    pos, nrm, flux, mis = OE.emit(box, J, it=0, set_id=0, seed=11, with_mis=True)
    gp, gm = out.pos.cpu().numpy(), out.mis.cpu().numpy()
    assert np.array_equal(np.isnan(gp[0]), np.isnan(pos[0]))
    assert np.array_equal(gm, mis)
    est.close()


def test_connection_term_matches_oracle():
    """On a fresh set (radius r1 everywhere) the connection is the whole running estimate."""
    from oracle import emit as OE
    from oracle import vc as VC
    w = _vcm_box(32, seed=3, r1=0.015, beta="lognormal")
    est = _estimator(w)
    box = OE.Box(light=(0.42, 0.8, 0.55), sphere_c=(0.5, 0.45, 0.5), sphere_r=0.18, power=5.0)
    J = 1_234_567
    est.connect_box(0, _scene(box), J)
    torch.cuda.synchronize()
    got = est.radiance(0).cpu().numpy().T.astype(np.float64) * math.pi       # (H, 3), iterations = 0
    r = np.full(w.kernels.n, F32(0.015), F32)
    ref = VC.connect(box.light, box.sphere_c, box.sphere_r, box.power, w.kernels, r, J)
    V = VC.visible(box.light, box.sphere_c, box.sphere_r, w.kernels.pos)
    assert np.array_equal(got[:, 0] == 0.0, ref[:, 0] == 0.0)
    assert (~V).sum() > 20                                    # some camera vertices lie in the shadow
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)
    rel[ref == 0.0] = 0.0
    _say(f"connection term: max rel {rel.max():.2e}")
    assert rel.max() < 2e-6
    est.close()


def test_vertex_merging_with_connection_matches_oracle():
    """Emission with partials, connection and iteration on the GPU; emission oracle, connection
    oracle and iteration oracle on the CPU; compared after every iteration."""
    from oracle import emit as OE
    from oracle import vc as VC
    from tests import gpu_parity as GP
    w = _vcm_box(24, r1=0.03)
    est = _estimator(w)
    tr = GP.Tracker(w, name="box-vcm-connect")
    box = OE.Box()
    J = 120_000
    for it in range(6):
        _say(f"merging + connection: iteration {it + 1}/6")
        dev = est.emit_box(0, _scene(box), 9, J)
        est.connect_box(0, _scene(box), J)
        est.iterate([0], [dev])
        ph = _compact(*OE.emit(box, J, it=it, set_id=0, seed=9, with_mis=True), J)
        tr.step(est, 0, ph, connect_fn=lambda ks, r: VC.connect(box.light, box.sphere_c, box.sphere_r,
                                                                 box.power, ks, r, J))
    rep = tr.finish(est, 0)
    _say(f"parity ok: {rep}")
    assert rep.shrinks > 0
    est.close()


def test_graph_with_connection_replays_like_eager_calls():
    from oracle import emit as OE
    from paper_2504_04411_amd.estimator import DevicePhotons
    w = _vcm_box(32, r1=0.03)
    ga, eb = _estimator(w), _estimator(w)
    box = OE.Box()
    J = 200_000
    mk = lambda: torch.empty((3, J), dtype=torch.float32, device="cuda")  # noqa: E731
    buf = DevicePhotons(J=J, pos=mk(), flux=mk(), nrm=mk(), mis=mk())
    g = ga.capture_box([0], [_scene(box)], [5], [buf], connect=True)
    for it in range(4):
        _say(f"graph with connection: replay {it + 1}/4")
        g.launch()
        dev = eb.emit_box(0, _scene(box), 5, J)
        eb.connect_box(0, _scene(box), J)
        eb.iterate([0], [dev])
        torch.cuda.synchronize()
        assert torch.equal(ga.radii(0), eb.radii(0))
        assert torch.equal(ga.radiance(0), eb.radiance(0))
        for x, y in zip(ga.sums(0), eb.sums(0)):
            assert torch.equal(x, y)
    g.close()
    ga.close()
    eb.close()


def test_connection_errors():
    from paper_2504_04411_amd import hk
    from paper_2504_04411_amd.estimator import Estimator
    from oracle import emit as OE
    from workloads import generators as G
    scene = G.BoxScene(res=8)
    pos, nrm, _ = scene.hit_points()
    est = Estimator(0.05)                                     # merging needs VCM mode
    est.set_kernels(0, pos, nrm)
    with pytest.raises(hk.HKError):
        est.connect_box(0, _scene(OE.Box()), 1000)
    est.close()
    w = _vcm_box(8)
    est = _estimator(w)
    with pytest.raises(hk.HKError):
        est.connect_box(0, _scene(OE.Box()), 0)               # J must be >= 1
    with pytest.raises(hk.HKError):                           # a set without kernels
        hk.hk_connect_box(est.ctx, 3, est.states[0].data_ptr(), _scene(OE.Box()), 1000, est.stream)
    torch.cuda.synchronize()
    est.close()
