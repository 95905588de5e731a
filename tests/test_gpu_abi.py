"""Status codes of the C ABI that need a device context: calls out of order, buffers too small, sizes
beyond the supported range, duplicate set ids, the iteration limit, and caller radii (r_init)."""
import ctypes

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


def _mods():
    from paper_2504_04411_amd import hk
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    from workloads import generators as G
    return hk, DevicePhotons, Estimator, G


def _code(fn, *a):
    hk = _mods()[0]
    with pytest.raises(hk.HKError) as ei:
        fn(*a)
    return ei.value.code


def test_iterate_before_set_kernels_is_bad_state():
    hk, DevicePhotons, Estimator, G = _mods()
    est = Estimator(0.05)
    ph = DevicePhotons.upload(G.small_config0(seed=1, n_side=4, J=100).photons(0))
    est.n[3] = 16                                 # the binding's size bookkeeping only; no state exists
    est.states[3] = torch.empty(256, dtype=torch.uint8, device="cuda")
    assert _code(est.iterate, [3], [ph]) == hk.HK_E_BAD_STATE
    assert "hk_set_kernels" in hk.hk_last_error()
    est.close()


def test_small_workspace_is_refused():
    hk, DevicePhotons, Estimator, G = _mods()
    w = G.small_config0(seed=1, n_side=8, J=2000)
    est = Estimator(w.params.r1)
    pos = torch.from_numpy(w.kernels.pos).cuda()
    st = torch.empty(hk.hk_state_bytes(est.ctx, w.kernels.n), dtype=torch.uint8, device="cuda")
    need = hk.hk_workspace_bytes(est.ctx, 0, w.kernels.n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    rows = [pos[i].data_ptr() for i in range(3)]
    code = _code(hk.hk_set_kernels, est.ctx, 0, w.kernels.n, -1.0, -1.0, rows, None, None, None, None,
                 st.data_ptr(), ws.data_ptr(), need - 1, est.stream)
    assert code == hk.HK_E_SMALL_BUFFER
    est.set_kernels(0, w.kernels.pos)
    ph = DevicePhotons.upload(w.photons(0))
    need = est.workspace_for([ph], [0])
    small = torch.empty(need, dtype=torch.uint8, device="cuda")
    code = _code(hk.hk_iterate, est.ctx, [0], [ph.struct()], [est.states[0].data_ptr()], small.data_ptr(), need - 256,
                 est.stream)
    assert code == hk.HK_E_SMALL_BUFFER
    hk.hk_iterate(est.ctx, [0], [ph.struct()], [est.states[0].data_ptr()], small.data_ptr(), need, est.stream)
    torch.cuda.synchronize()
    est.close()


def test_too_many_stored_vertices_is_unsupported():
    """2^27 stored light vertices in one set, and 2^27 - 64 (one more than the largest set without
    normals: its 32-byte records, and a cursor passing the last row by up to 63 records, must keep
    32-bit byte offsets), are refused before anything is enqueued (the pointers are never read)."""
    hk, DevicePhotons, Estimator, G = _mods()
    w = G.small_config0(seed=1, n_side=4, J=100)
    est = Estimator(w.params.r1)
    est.set_kernels(0, w.kernels.pos)
    dummy = torch.empty(64, dtype=torch.float32, device="cuda")
    rows = [dummy.data_ptr()] * 3
    ws = est._workspace(1 << 20)
    for n in (1 << 27, (1 << 27) - 64):
        ph = hk.make_photons(n, n, rows, rows)
        code = _code(hk.hk_iterate, est.ctx, [0], [ph], [est.states[0].data_ptr()], ws.data_ptr(), ws.numel(),
                     est.stream)
        assert code == hk.HK_E_UNSUPPORTED, n
    n = 1 << 27
    ph = hk.make_photons(n - 2, n - 1, rows, rows)          # more stored than emitted
    code = _code(hk.hk_iterate, est.ctx, [0], [ph], [est.states[0].data_ptr()], ws.data_ptr(), ws.numel(),
                 est.stream)
    assert code == hk.HK_E_INVALID_ARG
    est.close()


def test_duplicate_set_ids_are_refused():
    hk, DevicePhotons, Estimator, G = _mods()
    w = G.small_config0(seed=1, n_side=4, J=100)
    est = Estimator(w.params.r1)
    est.set_kernels(2, w.kernels.pos)
    ph = DevicePhotons.upload(w.photons(0))
    assert _code(est.iterate, [2, 2], [ph, ph]) == hk.HK_E_INVALID_ARG
    assert "twice" in hk.hk_last_error()
    est.close()


def test_gather_phases_query():
    """hk_gather_phases (host-side): one set takes one phase; a set without kernels is refused with
    HK_E_BAD_STATE, an id out of range, a repeated id and a NULL output with HK_E_INVALID_ARG."""
    hk, DevicePhotons, Estimator, G = _mods()
    w = G.small_config0(seed=1, n_side=4, J=100)
    est = Estimator(w.params.r1)
    est.set_kernels(0, w.kernels.pos)
    ph = DevicePhotons.upload(w.photons(0))
    assert est.gather_phases([0], [ph]) == [0]
    assert _code(est.gather_phases, [1], [ph]) == hk.HK_E_BAD_STATE
    assert _code(est.gather_phases, [300], [ph]) == hk.HK_E_INVALID_ARG
    assert _code(est.gather_phases, [0, 0], [ph, ph]) == hk.HK_E_INVALID_ARG
    ids = (ctypes.c_int * 1)(0)
    phs = (hk.hk_photons * 1)(ph.struct())
    assert hk.lib().hk_gather_phases(est.ctx, 1, ids, phs, None) == hk.HK_E_INVALID_ARG
    est.close()


def test_max_iters_reached_is_bad_state():
    hk, DevicePhotons, Estimator, G = _mods()
    w = G.small_config0(seed=1, n_side=4, J=500)
    est = Estimator(w.params.r1, max_iters=2)
    est.set_kernels(0, w.kernels.pos)
    for it in range(2):
        est.iterate([0], [DevicePhotons.upload(w.photons(it))])
    assert _code(est.iterate, [0], [DevicePhotons.upload(w.photons(2))]) == hk.HK_E_BAD_STATE
    assert "max_iters" in hk.hk_last_error()
    est.set_kernels(0, w.kernels.pos)              # a fresh set-up starts the count again
    est.iterate([0], [DevicePhotons.upload(w.photons(0))])
    torch.cuda.synchronize()
    est.close()


@pytest.mark.parametrize("bad", [float("nan"), float("inf"), 0.0, -0.01, 4.0e-5])
def test_invalid_caller_radii_are_refused(bad):
    """r_init must hold finite radii at or above r_min (5e-5 here): below it a shrink to the lower
    bound of Eq. radiusupdate would make the radius grow."""
    hk, DevicePhotons, Estimator, G = _mods()
    w = G.small_config0(seed=1, n_side=6, J=500)
    est = Estimator(w.params.r1, rmin=5e-5)
    r = np.full(w.kernels.n, 0.03, np.float32)
    r[7] = bad
    assert _code(est.set_kernels, 0, w.kernels.pos, None, r) == hk.HK_E_INVALID_ARG
    assert "1 of 36" in hk.hk_last_error()
    ph = DevicePhotons.upload(w.photons(0))
    est.n[0] = w.kernels.n                          # the binding registers a set only on success
    est.states[0] = torch.empty(hk.hk_state_bytes(est.ctx, w.kernels.n), dtype=torch.uint8, device="cuda")
    assert _code(est.iterate, [0], [ph]) == hk.HK_E_BAD_STATE       # the set stayed uninitialised
    r[7] = 5e-5
    est.set_kernels(0, w.kernels.pos, None, r)
    est.iterate([0], [ph])
    torch.cuda.synchronize()
    est.close()


def test_caller_radii_follow_the_oracle():
    """Per-kernel starting radii (spread over two decades, down to r_min itself) in parity with the
    oracle started from the same radii."""
    from oracle import oracle as O
    from tests import gpu_parity as GP
    hk, DevicePhotons, Estimator, G = _mods()
    w = G.small_config0(seed=12, n_side=24, J=20000, n_iter=6, r1=0.06)
    rng = np.random.default_rng(3)
    r0 = (w.params.r1 * np.exp(rng.uniform(np.log(0.01), 0.0, w.kernels.n))).astype(np.float32)
    r0[:5] = np.float32(w.params.rmin)
    est = GP.make_estimator(w)
    est.set_kernels(0, w.kernels.pos, None, r0)
    tr = GP.Tracker(w)
    tr.ost = O.init_state(w.kernels.n, w.params.r1, r_init=r0)
    for it in range(6):
        ph = w.photons(it)
        est.iterate([0], [DevicePhotons.upload(ph)])
        tr.step(est, 0, ph)
    rep = tr.finish(est, 0)
    assert rep.shrinks > 50
    est.close()
