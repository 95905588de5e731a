"""Batched launches over many uneven hit-point sets, captured graphs and the autotuner (GPU).

* Batched sets must give, per set, exactly (bit for bit) what the set gives alone: the gather of a
  kernel does not depend on which other kernels share its launch. Every set is also checked against
  the oracle with the parity rules of tests/gpu_parity.py.
* Graph replays are compared, replay by replay, with eager hk_iterate calls on a twin state, with
  eager work (reads, synchronisations) between the replays.
* The autotuner must leave the states untouched and pick one of its candidate settings; results
  under other settings still meet the oracle parity bar.
"""
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


def _mods():
    from paper_2504_04411_amd.estimator import DevicePhotons
    from tests import gpu_parity as GP
    from workloads import generators as G
    return G, GP, DevicePhotons


def _snapshot(est, sid):
    d = {k: v.cpu().numpy().copy() for k, v in est.debug(sid).items()}
    d["r"] = est.radii(sid).cpu().numpy().copy()
    S, Q, tau = est.sums(sid)
    d["S"], d["Q"], d["tau"] = S.cpu().numpy(), Q.cpu().numpy(), tau.cpu().numpy()
    d["L"] = est.radiance(sid).cpu().numpy()
    return d


def _same(a, b, what):
    for k in a:
        x, y = a[k], b[k]
        eq = (x == y) | (np.isnan(x) & np.isnan(y)) if x.dtype.kind == "f" else (x == y)
        assert np.all(eq), f"{what}: '{k}' differs at {np.argwhere(~eq)[:5].ravel()}"


def _add_set(est, sid, w):
    ks, p = w.kernels, w.params
    est.set_kernels(sid, ks.pos, ks.nrm, None, ks.cam_beta, ks.cam_mis, r1=p.r1, rmin=p.rmin)


def test_batched_uneven_sets_match_solo_and_oracle():
    """16 planar sets of uneven size, J and radius in one call per iteration (one gather launch):
    bit-identical to running each set alone, and each set within the oracle parity bar."""
    G, GP, DP = _mods()
    ws = G.config2(seed=2, n_sets=16, scale=0.01, n_iter=4)
    p0 = ws[0].params
    batched = GP.make_estimator(ws[0])
    solo = GP.make_estimator(ws[0])
    trackers = []
    for s, w in enumerate(ws):
        _add_set(batched, s, w)
        _add_set(solo, s, w)
        trackers.append(GP.Tracker(w, name=f"set{s}"))
        assert w.params.k == p0.k and w.params.alpha_f == p0.alpha_f and w.params.alpha == p0.alpha
    sizes = [w.kernels.n for w in ws]
    print(f"  sets: H = {sizes}", flush=True)
    assert len(set(sizes)) > 8
    for it in range(4):
        phs = [w.photons(it) for w in ws]
        dps = [DP.upload(ph) for ph in phs]
        print(f"  iteration {it + 1}: stored = {[d.n for d in dps]}", flush=True)
        batched.iterate(list(range(len(ws))), dps)
        for s in range(len(ws)):
            solo.iterate([s], [dps[s]])
        for s in range(len(ws)):
            _same(_snapshot(batched, s), _snapshot(solo, s), f"iteration {it + 1} set {s}")
            trackers[s].step(batched, s, phs[s])
    shrinks = 0
    for s in range(len(ws)):
        rep = trackers[s].finish(batched, s)
        shrinks += rep.shrinks
        assert batched.stats(s)["iterations"] == 4
    assert shrinks > 0


def test_batch_more_than_64_sets_and_mixed_normals():
    """70 tiny planar sets (two gather launches of at most 64 sets) plus two box sets with normals
    (their own launch) in one call; bit-identical to solo runs."""
    G, GP, DP = _mods()
    ws = [G.config0(seed=10 + s, n_side=5 + (s % 7), J=2000 + 97 * s, n_iter=3, r1=0.1, set_id=s)
          for s in range(70)]
    ws += [G.box_scene(seed=80 + s, res=12 + 4 * s, J=20_000, n_iter=3, set_id=70 + s) for s in range(2)]
    batched = GP.make_estimator(ws[0])
    solo = GP.make_estimator(ws[0])
    for s, w in enumerate(ws):
        _add_set(batched, s, w)
        _add_set(solo, s, w)
    ids = list(range(len(ws)))
    for it in range(3):
        dps = [DP.upload(w.photons(it)) for w in ws]
        print(f"  iteration {it + 1}: {len(ws)} sets", flush=True)
        batched.iterate(ids, dps)
        for s in ids:
            solo.iterate([s], [dps[s]])
        for s in ids:
            _same(_snapshot(batched, s), _snapshot(solo, s), f"iteration {it + 1} set {s}")


@pytest.mark.parametrize("mode", ["ppm", "vcm"])
def test_graph_replay_matches_eager(mode):
    """One iteration captured into a graph and replayed 5 times, photons refilled in place before each
    replay; every replay is compared with the eager call on a twin state."""
    G, GP, DP = _mods()
    if mode == "ppm":
        ws = [G.config0(seed=5, n_side=40, J=40_000, n_iter=5, r1=0.05),
              G.config0(seed=6, n_side=23, J=9_000, n_iter=5, r1=0.08, set_id=1)]
    else:
        ws = [G.config4(seed=4, nx=64, ny=36, J=60_000, r1=0.02, n_iter=5)]
    eager = GP.make_estimator(ws[0])
    graph = GP.make_estimator(ws[0])
    for s, w in enumerate(ws):
        _add_set(eager, s, w)
        _add_set(graph, s, w)
    ids = list(range(len(ws)))
    bufs = [DP.upload(w.photons(0)) for w in ws]      # the graph reads these buffers
    for b, w in zip(bufs, ws):
        assert b.n == w.photons(1).n, "the graph needs a fixed stored count"
    g = graph.capture(ids, bufs)
    torch.cuda.synchronize()
    # capture runs nothing: the sets are still at iteration 0
    assert all(graph.stats(s)["iterations"] == 0 for s in ids)
    for it in range(5):
        phs = [DP.upload(w.photons(it)) for w in ws]
        for b, ph in zip(bufs, phs):
            b.pos.copy_(ph.pos)
            b.flux.copy_(ph.flux)
            if ph.nrm is not None:
                b.nrm.copy_(ph.nrm)
            if ph.mis is not None:
                b.mis.copy_(ph.mis)
        g.launch()
        eager.iterate(ids, phs)
        torch.cuda.synchronize()
        print(f"  replay {it + 1}", flush=True)
        for s in ids:
            _same(_snapshot(graph, s), _snapshot(eager, s), f"replay {it + 1} set {s}")
    assert all(graph.stats(s)["iterations"] == 5 for s in ids)
    g.close()


def test_two_gather_phases_graph_and_eager():
    """Eight planar sets at 0.3 of the 16-set workload's sizes (5.9M light vertices, 370k hit points):
    large enough that the batch is gathered in two phases (the second phase's grids built while the
    first gather runs), checked by the launch count. A captured graph is replayed three times against
    eager calls on a twin state, bit for bit, and 128 sampled kernels of every set of the eager
    state against the oracle."""
    G, GP, DP = _mods()
    ws = G.config2(seed=2, n_sets=8, n_iter=3, scale=0.3)
    eager = GP.make_estimator(ws[0])
    graph = GP.make_estimator(ws[0])
    for s, w in enumerate(ws):
        _add_set(eager, s, w)
        _add_set(graph, s, w)
    ids = list(range(len(ws)))
    rng = np.random.default_rng(21)
    trackers = [GP.Tracker(w, np.sort(rng.choice(w.kernels.n, min(128, w.kernels.n), replace=False)),
                           name=f"set{s}") for s, w in enumerate(ws)]
    bufs = [DP.upload(w.photons(0)) for w in ws]
    g = graph.capture(ids, bufs)
    torch.cuda.synchronize()
    eager.profile(True)
    for it in range(3):
        phs_host = [w.photons(it) for w in ws]
        phs = [DP.upload(ph) for ph in phs_host]
        for b, ph in zip(bufs, phs):
            b.pos.copy_(ph.pos)
            b.flux.copy_(ph.flux)
        g.launch()
        eager.iterate(ids, phs)
        torch.cuda.synchronize()
        for s in ids:
            _same(_snapshot(graph, s), _snapshot(eager, s), f"replay {it + 1} set {s}")
            trackers[s].step(eager, s, phs_host[s])
    prof = eager.profile_read()
    eager.profile(False)
    print(f"  gather launches over 3 iterations: {prof['launches']}", flush=True)
    assert prof["launches"] == 6, "the batch was expected to be gathered in two phases"
    assert prof["launches_phase"] == [3, 3]
    phases = eager.gather_phases(ids, bufs)
    assert sorted(set(phases)) == [0, 1], phases
    print(f"  gather phase per set: {phases}", flush=True)
    for s in ids:
        trackers[s].finish(eager, s)
    g.close()


def test_two_phases_on_a_side_stream_match_the_default_stream():
    """The eight-set batch of the test above (two gather phases, the second phase's grids built beside
    the first gather) called on a stream of the caller's own, with unrelated work queued on the
    default stream meanwhile, leaves every set bit-identical to the same calls on the default stream:
    the library's forks and joins follow whichever stream it is given."""
    G, GP, DP = _mods()
    ws = G.config2(seed=2, n_sets=8, n_iter=3, scale=0.3)
    on_default = GP.make_estimator(ws[0])
    on_side = GP.make_estimator(ws[0])
    for s, w in enumerate(ws):
        _add_set(on_default, s, w)
        _add_set(on_side, s, w)
    ids = list(range(len(ws)))
    side = torch.cuda.Stream()
    for it in range(2):
        phs = [DP.upload(w.photons(it)) for w in ws]
        torch.cuda.synchronize()
        on_default.iterate(ids, phs)
        with torch.cuda.stream(side):
            on_side.iterate(ids, phs)
        x = torch.randn(1 << 22, device="cuda")
        (x * 2.0).sum()
        torch.cuda.synchronize()
    for s in ids:
        _same(_snapshot(on_side, s), _snapshot(on_default, s), f"side stream, set {s}")
    on_default.close()
    on_side.close()


def test_graph_refuses_stale_sets():
    """A graph whose set was re-initialised, or that reached max_iters, is refused on the host."""
    G, GP, DP = _mods()
    from paper_2504_04411_amd import hk
    w = G.config0(seed=7, n_side=12, J=5000, n_iter=2, r1=0.08)
    est = GP.make_estimator(w, max_iters=2)
    _add_set(est, 0, w)
    buf = DP.upload(w.photons(0))
    g = est.capture([0], [buf])
    g.launch()
    g.launch()
    with pytest.raises(hk.HKError) as e:
        g.launch()
    assert e.value.code == hk.HK_E_BAD_STATE
    _add_set(est, 0, w)
    with pytest.raises(hk.HKError) as e:
        g.launch()
    assert e.value.code == hk.HK_E_BAD_STATE
    torch.cuda.synchronize()
    g.close()


def test_autotune_keeps_state_and_picks_a_candidate():
    G, GP, DP = _mods()
    w = G.box_scene(seed=1, res=64, J=300_000, n_iter=4)
    est = GP.make_estimator(w)
    _add_set(est, 0, w)
    est.iterate([0], [DP.upload(w.photons(0))])
    before = est.states[0].clone()
    dp = DP.upload(w.photons(1))
    t = est.autotune([0], [dp])
    torch.cuda.synchronize()
    print(f"  chosen: {t}", flush=True)
    assert torch.equal(before, est.states[0])
    assert t["cell_scale"] in [np.float32(c) for c in (0.35, 0.5, 0.7, 1.0)]
    assert t["lanes_light"] in (4, 8, 16) and t["heavy_cost"] in (1024, 2048, 4096, 16384)
    assert est.tuning() == t
    assert est.stats(0)["iterations"] == 1


@pytest.mark.parametrize("tuning", [dict(cell_scale=0.7, heavy_cost=1024, lanes_light=4, lanes_heavy=16),
                                    dict(cell_scale=1.4, heavy_cost=16384, lanes_light=16, lanes_heavy=64),
                                    dict(cell_scale=0.35, heavy_cost=2048, lanes_light=8, lanes_heavy=64)])
def test_other_tunings_meet_oracle_parity(tuning):
    G, GP, DP = _mods()
    w = G.box_scene(seed=1, res=40, J=200_000, n_iter=6)
    rep = GP.run_parity(w, 6, est_kw=tuning)
    assert rep.shrinks > 100
