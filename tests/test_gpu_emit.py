"""Light-vertex generation on the GPU (hk_emit_box, hk_graph_create_box) against the oracle: every
slot bit-identical (integer random numbers, then float32 operations with one rounding each), the
iteration index taken from the device state, the estimator on generated slots in parity with the
oracle on the oracle's own batches, and graph replays equal to eager calls."""
import math
import sys

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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _scene(box):
    from paper_2504_04411_amd import hk
    return hk.box_scene(box.light, box.sphere_c, box.sphere_r, box.power)


def _same_slots(dev, host):
    pos, nrm, flux = host
    gp, gn, gf = (t.cpu().numpy() for t in (dev.pos, dev.nrm, dev.flux))
    dead_o = np.isnan(pos[0])
    for a in range(3):
        assert np.array_equal(np.isnan(gp[a]), dead_o), "empty slots differ"
    live = ~dead_o
    for a in range(3):
        bad = np.flatnonzero(live & (gp[a] != pos[a]))
        assert bad.size == 0, f"axis {a}: {bad.size} positions differ, first {bad[:4]}: {gp[a][bad[:4]]} vs {pos[a][bad[:4]]}"
    assert np.array_equal(gn, nrm) and np.array_equal(gf, flux)
    return int(live.sum())


def _box_estimator(res=16, r1=0.05, **kw):
    from paper_2504_04411_amd.estimator import Estimator
    from workloads import generators as G
    w = G.box_scene(seed=1, res=res, J=1, r1=r1)
    est = Estimator(r1, **kw)
    est.set_kernels(0, w.kernels.pos, w.kernels.nrm)
    return est, w


@pytest.mark.parametrize("J", [0, 1, 255, 257, 12_345])
def test_emit_small_and_ragged_matches_oracle(J):
    from oracle import emit as OE
    est, _ = _box_estimator()
    box = OE.Box()
    _say(f"emit J={J}")
    if J == 0:
        from paper_2504_04411_amd import hk
        hk.hk_emit_box(est.ctx, 0, est.states[0].data_ptr(), _scene(box), 7, 0, None, None, None, est.stream)
        torch.cuda.synchronize()
        est.close()
        return
    out = est.emit_box(0, _scene(box), 7, J)
    torch.cuda.synchronize()
    _same_slots(out, OE.emit(box, J, it=0, set_id=0, seed=7))
    est.close()


def test_emit_full_size_three_iterations_and_seeds():
    """2M slots per iteration, the iteration index read from the set's state as the estimator
    advances it, a 64-bit seed and another set id."""
    from oracle import emit as OE
    from paper_2504_04411_amd.estimator import DevicePhotons
    from workloads import generators as G
    est, w = _box_estimator(res=64)
    est.set_kernels(3, w.kernels.pos, w.kernels.nrm)
    box = OE.Box()
    J = 2_000_000
    seed = (5 << 32) | 11
    for it in range(3):
        _say(f"full-size emission, iteration {it}")
        out = est.emit_box(0, _scene(box), seed, J)
        out3 = est.emit_box(3, _scene(box), seed, J)
        torch.cuda.synchronize()
        live = _same_slots(out, OE.emit(box, J, it=it, set_id=0, seed=seed))
        _same_slots(out3, OE.emit(box, J, it=it, set_id=3, seed=seed))
        assert 0.5 * J < live < J
        est.iterate([0, 3], [out, out3])
    torch.cuda.synchronize()
    est.close()


def test_emit_jittered_scene_and_no_occluder():
    from oracle import emit as OE
    est, _ = _box_estimator()
    for box in (OE.Box(light=(0.31, 0.77, 0.42), sphere_c=(0.55, 0.4, 0.3), sphere_r=0.21, power=3.5),
                OE.Box(light=(0.5, 0.5, 0.05), sphere_c=(0.5, 0.5, 0.5), sphere_r=0.0, power=1.0)):
        _say(f"emit scene {box}")
        out = est.emit_box(0, _scene(box), 99, 300_000)
        torch.cuda.synchronize()
        _same_slots(out, OE.emit(box, 300_000, it=0, set_id=0, seed=99))
    est.close()


def _compact(pos, nrm, flux, J):
    from workloads import generators as G
    keep = np.isfinite(pos[0])
    return G.PhotonBatch(J=J, pos=pos[:, keep], flux=flux[:, keep], nrm=nrm[:, keep])


def test_estimator_on_generated_batches_matches_oracle():
    """The GPU estimator on the generated slots (empty ones included) against the oracle estimator
    on the oracle's generated batches, compacted."""
    from oracle import emit as OE
    from tests import gpu_parity as GP
    from workloads import generators as G
    w = G.box_scene(seed=1, res=32, J=1, r1=0.05, n_iter=5)
    est = GP.make_estimator(w)
    est.set_kernels(0, w.kernels.pos, w.kernels.nrm)
    tr = GP.Tracker(w, name="box-generated")
    box = OE.Box()
    J = 150_000
    for it in range(5):
        _say(f"generated batches: iteration {it + 1}/5")
        dev = est.emit_box(0, _scene(box), 21, J)
        est.iterate([0], [dev])
        tr.step(est, 0, _compact(*OE.emit(box, J, it=it, set_id=0, seed=21), J))
    rep = tr.finish(est, 0)
    _say(f"parity ok: {rep}")
    assert rep.shrinks > 0
    est.close()


def test_generated_slots_equal_compacted_upload():
    """Empty slots change nothing: the estimator on the generated slots is bit-identical to the
    estimator on the same vertices compacted and uploaded."""
    from oracle import emit as OE
    from paper_2504_04411_amd.estimator import DevicePhotons
    a, w = _box_estimator(res=48)
    b, _ = _box_estimator(res=48)
    box = OE.Box()
    J = 400_000
    for it in range(3):
        _say(f"slots vs compacted: iteration {it + 1}/3")
        dev = a.emit_box(0, _scene(box), 5, J)
        torch.cuda.synchronize()
        pos, nrm, flux = (t.cpu().numpy() for t in (dev.pos, dev.nrm, dev.flux))
        a.iterate([0], [dev])
        b.iterate([0], [DevicePhotons.upload(_compact(pos, nrm, flux, J))])
        torch.cuda.synchronize()
        for x, y in zip(a.sums(0), b.sums(0)):
            assert torch.equal(x, y)
        assert torch.equal(a.radii(0), b.radii(0))
        assert torch.equal(a.radiance(0), b.radiance(0))
    a.close()
    b.close()


def test_graph_with_generation_replays_like_eager_calls():
    """hk_graph_create_box: each replay generates the next iteration's batch on the device and runs
    the iteration; results equal eager hk_emit_box + hk_iterate after every replay."""
    from oracle import emit as OE
    from paper_2504_04411_amd.estimator import DevicePhotons
    box = OE.Box(light=(0.45, 0.85, 0.55))
    J = 300_000
    ga, w = _box_estimator(res=48)
    eb, _ = _box_estimator(res=48)
    mk = lambda: torch.empty((3, J), dtype=torch.float32, device="cuda")  # noqa: E731
    buf = DevicePhotons(J=J, pos=mk(), flux=mk(), nrm=mk())
    g = ga.capture_box([0], [_scene(box)], [77], [buf])
    for it in range(4):
        _say(f"graph replay {it + 1}/4")
        g.launch()
        eb.iterate([0], [eb.emit_box(0, _scene(box), 77, J)])
        torch.cuda.synchronize()
        _same_slots(buf, OE.emit(box, J, it=it, set_id=0, seed=77))
        for x, y in zip(ga.sums(0), eb.sums(0)):
            assert torch.equal(x, y)
        assert torch.equal(ga.radii(0), eb.radii(0))
        assert torch.equal(ga.radiance(0), eb.radiance(0))
        torch.cuda.synchronize()
    g.close()
    ga.close()
    eb.close()


def test_emit_argument_errors():
    from paper_2504_04411_amd import hk
    from oracle import emit as OE
    est, _ = _box_estimator()
    st = est.states[0].data_ptr()
    t = torch.empty((3, 8), dtype=torch.float32, device="cuda")
    rows = [t[i].data_ptr() for i in range(3)]
    bad = [
        dict(scene=hk.box_scene((0.5, 1.0, 0.5), (0.5, 0.5, 0.5), 0.1, 1.0)),      # light on a wall
        dict(scene=hk.box_scene((0.5, 0.5, 0.5), (0.5, 0.5, 0.5), -0.1, 1.0)),     # negative radius
        dict(scene=hk.box_scene((0.5, 0.5, 0.5), (0.5, 0.5, math.nan), 0.1, 1.0)),
        dict(J=-1), dict(J=1 << 27), dict(set_id=5), dict(pos=None),
    ]
    for case in bad:
        a = dict(scene=_scene(OE.Box()), J=8, set_id=0, pos=rows)
        a.update(case)
        with pytest.raises(hk.HKError):
            hk.hk_emit_box(est.ctx, a["set_id"], st, a["scene"], 1, a["J"], a["pos"], rows, rows, est.stream)
    torch.cuda.synchronize()
    est.close()
