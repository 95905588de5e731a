"""hk_iterate_static (no workspace argument: the library's static per-GPU scratch) against hk_iterate
with a caller workspace, through the C ABI: two calls in a row, the second with a smaller input, the
states compared bit for bit; a call beyond the static scratch is refused before any work."""
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


def _snap(est, sid):
    d = {k: v.cpu().numpy().copy() for k, v in est.debug(sid).items()}
    d["r"] = est.radii(sid).cpu().numpy()
    S, Q, tau = est.sums(sid)
    d["S"], d["Q"], d["tau"] = S.cpu().numpy(), Q.cpu().numpy(), tau.cpu().numpy()
    return d


def _same(a, b, what):
    for k in a:
        x, y = a[k], b[k]
        eq = (x == y) | (np.isnan(x) & np.isnan(y)) if x.dtype.kind == "f" else (x == y)
        assert np.all(eq), f"{what}: '{k}' differs at {np.argwhere(~eq)[:5].ravel()}"


def test_static_scratch_matches_workspace_calls():
    from paper_2504_04411_amd import hk
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    from workloads import generators as G
    big = G.config0(seed=0)                                    # 4096 hit points, 100k light paths
    small = G.small_config0(seed=3, n_side=23, J=30_000)       # 529 hit points, 30k light paths
    ref = Estimator(big.params.r1)
    sta = Estimator(big.params.r1)
    for est in (ref, sta):
        est.set_kernels(0, big.kernels.pos)
        est.set_kernels(1, small.kernels.pos, r1=small.params.r1, rmin=small.params.rmin)
    torch.cuda.synchronize()
    calls = [([0], [big.photons(0)]), ([1], [small.photons(0)]), ([0, 1], [big.photons(1), small.photons(1)]),
             ([1], [small.photons(2)])]
    for c, (ids, phs) in enumerate(calls):
        dps = [DevicePhotons.upload(p) for p in phs]
        need = hk.hk_workspace_bytes_batch(sta.ctx, [d.n for d in dps], [sta.n[s] for s in ids])
        assert need <= hk.HK_STATIC_SCRATCH_BYTES
        print(f"  call {c + 1}: sets {ids}, stored {[d.n for d in dps]}, scratch {need} bytes", flush=True)
        ref.iterate(ids, dps)
        hk.hk_iterate_static(sta.ctx, ids, [d.struct() for d in dps], [sta.states[s].data_ptr() for s in ids],
                             sta.stream)
        torch.cuda.synchronize()
        for s in (0, 1):
            _same(_snap(ref, s), _snap(sta, s), f"call {c + 1} set {s}")
    # beyond the static scratch: refused before anything is enqueued (pointers never read)
    dummy = torch.empty(64, dtype=torch.float32, device="cuda")
    rows = [dummy.data_ptr()] * 3
    n = 2_000_000
    with pytest.raises(hk.HKError) as ei:
        hk.hk_iterate_static(sta.ctx, [0], [hk.make_photons(n, n, rows, rows)], [sta.states[0].data_ptr()],
                             sta.stream)
    assert ei.value.code == hk.HK_E_SMALL_BUFFER
    ref.close()
    sta.close()
