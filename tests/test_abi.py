"""CPU tests of the C ABI: the library loads, exports every declared entry point, validates arguments
without a GPU, and its float64 critical-value routine matches an independent 40-digit evaluation."""
import math

import mpmath as mp
import pytest

hk = pytest.importorskip("paper_2504_04411_amd.hk")


@pytest.fixture(scope="module")
def L():
    try:
        return hk.lib()
    except ImportError as e:
        pytest.skip(str(e))


def test_every_declared_symbol_is_exported(L):
    names = hk.header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert hk.hk_version() >= 100


def test_default_params_and_validation(L):
    p = hk.hk_default_params(0.05)
    assert abs(p.k - 0.7) < 1e-7 and abs(p.alpha_f - 0.05) < 1e-9 and abs(p.alpha - 0.75) < 1e-7
    assert p.rmin == 0.001 * 0.05 and p.n_a == 2 and p.n_s == 6
    bad = [("k", 1.0), ("k", 0.0), ("alpha_f", 1.0), ("alpha", 0.0), ("r1", -1.0), ("r1", float("nan")),
           ("rmin", 1.0), ("max_iters", 0), ("normal_cos_min", 2.0)]
    for field, val in bad:
        q = hk.hk_default_params(0.05)
        setattr(q, field, val)
        with pytest.raises(hk.HKError) as ei:
            hk.hk_create(q)
        assert ei.value.code == hk.HK_E_INVALID_ARG, field
    q = hk.hk_default_params(0.05)
    q.n_s = 8
    with pytest.raises(hk.HKError) as ei:
        hk.hk_create(q)
    assert ei.value.code == hk.HK_E_UNSUPPORTED


def test_null_arguments_are_rejected(L):
    import ctypes
    assert L.hk_destroy(None) == hk.HK_E_INVALID_ARG
    assert L.hk_create(None, None) == hk.HK_E_INVALID_ARG
    out = ctypes.c_size_t()
    assert L.hk_state_bytes(None, 10, ctypes.byref(out)) == hk.HK_E_INVALID_ARG
    assert L.hk_iterate(None, 1, None, None, None, None, 0, None) == hk.HK_E_INVALID_ARG
    assert "NULL" in hk.hk_last_error()


def _mp_quantile(d1, d2, alpha):
    with mp.workdps(40):
        a, b = mp.mpf(d1) / 2, mp.mpf(d2) / 2
        fn = lambda F: mp.betainc(a, b, 0, d1 * F / (d1 * F + d2), regularized=True) - (1 - mp.mpf(alpha))
        return mp.findroot(fn, mp.mpf(2.0), tol=mp.mpf(10) ** -30)


@pytest.mark.parametrize("d2", [12.0, 240.0, 1199988.0, 1.536e9, 1.2288e10, 1.2e14])
@pytest.mark.parametrize("alpha", [0.05, 0.01, 0.1])
def test_f_quantile_matches_40_digit_reference(L, d2, alpha):
    q = hk.hk_f_quantile(11, d2, alpha)
    ref = _mp_quantile(11, d2, alpha)
    assert abs(float((q - ref) / ref)) < 1e-11


def test_f_quantile_closed_forms(L):
    for d2 in (6.0, 120.0, 1.2e6):
        for p in (0.95, 0.99):
            want = (d2 / 2) * math.expm1(-(2 / d2) * math.log1p(-p))
            assert abs(hk.hk_f_quantile(2, d2, 1 - p) / want - 1) < 1e-12
    assert math.isnan(hk.hk_f_quantile(11, 0.0, 0.05))
    assert math.isnan(hk.hk_f_quantile(11, 100.0, 1.5))
