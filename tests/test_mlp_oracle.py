"""Pins of the learned-proposal oracle (oracle/mlp.py) against facts that do not depend on it:
exact bfloat16 rounding cases, hand-placed light vertices on ring boundaries, the equi-areal
property of the rings, closed-form networks, finite differences of the loss, the closed form of a
first Adam step, and the fit of a realisable target."""
import math

import numpy as np
import pytest

from oracle import mlp as M
from workloads.generators import KernelSet, PhotonBatch

F32 = np.float32


def test_bf16_rounding_cases():
    u = 2.0 ** -8
    cases = [(1.0, 1.0), (1.0 + u, 1.0),                       # tie -> even (mantissa 0)
             (1.0 + 3 * u, 1.0 + 4 * u),                        # tie -> even (mantissa 2)
             (1.0 + u + 2.0 ** -20, 1.0 + 2 * u),               # above the tie -> up
             (2.0 - u, 2.0),                                    # tie -> even carries into the exponent
             (-(1.0 + 3 * u), -(1.0 + 4 * u)), (0.0, 0.0), (3.0, 3.0)]
    for x, want in cases:
        assert M.bf16(x) == want, (x, M.bf16(x), want)
    b = M.bf16_bits([1.0, -2.0, 0.5])
    assert list(b) == [0x3F80, 0xC000, 0x3F00]
    assert np.array_equal(M.from_bf16_bits(b), [1.0, -2.0, 0.5])


def _one_kernel(nrm=None):
    return KernelSet(pos=np.zeros((3, 1), F32), nrm=nrm)


def _photons(xy, nrm=None):
    xy = np.asarray(xy, np.float64)
    pos = np.zeros((3, len(xy)), F32)
    pos[0], pos[1] = xy[:, 0], xy[:, 1]
    return PhotonBatch(J=len(xy), pos=pos, flux=np.ones((3, len(xy)), F32), nrm=nrm)


def test_feature_rings_hand_placed():
    """r1 = 1: scales R = 1, 1/2, 1/4, 1/8; ring b of scale s holds b/8 <= d2/R^2 < (b+1)/8."""
    ph = _photons([(0.0, 0.0),          # centre: ring 0 of every scale
                   (0.25, 0.25),        # d2 = 1/8 exactly: ring 1 of scale 0, ring 4 of scale 1
                   (1.0, 0.0),          # d2 = 1: outside (strict)
                   (0.5, 0.0),          # d2 = 1/4: ring 2 of scale 0; on scale 1's boundary -> outside
                   (0.0, 0.125)])       # d2 = 1/64: ring 0 of s0, ring 0 of s1 (1/16), ring 2 of s2, outside s3
    c = M.feature_counts(_one_kernel(), ph, 1.0)[0].reshape(4, 8)
    want = np.zeros((4, 8), np.uint32)
    want[:, 0] += 1                      # centre
    want[0, 1] += 1
    want[1, 4] += 1
    want[0, 2] += 1
    want[0, 0] += 1
    want[1, 0] += 1
    want[2, 2] += 1
    assert np.array_equal(c, want), c


def test_feature_normal_consistency():
    nk = np.zeros((3, 1), F32)
    nk[2] = 1.0
    pn = np.zeros((3, 2), F32)
    pn[2] = [1.0, -1.0]                  # second light vertex faces away: not counted
    ph = _photons([(0.1, 0.0), (0.1, 0.0)], nrm=pn)
    c = M.feature_counts(_one_kernel(nk), ph, 1.0)[0]
    assert c.sum() == 4                  # one vertex, counted at all four scales


def test_feature_rings_equal_area():
    """Uniform points in the unit disk land in the 8 rings of scale 0 with probability 1/8 each."""
    from scipy import stats
    rng = np.random.default_rng(5)
    n = 40000
    rad = np.sqrt(rng.random(n)) * 0.999
    ang = rng.random(n) * 2 * math.pi
    ph = _photons(np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1))
    c = M.feature_counts(_one_kernel(), ph, 1.0)[0].reshape(4, 8)
    assert c[0].sum() == n
    assert stats.chisquare(c[0]).pvalue > 1e-3
    # scale 1 sees the quarter of the points inside radius 1/2, again equally spread
    assert abs(c[1].sum() / n - 0.25 / 0.998) < 0.01
    assert stats.chisquare(c[1]).pvalue > 1e-3


def test_encode_values():
    counts = np.zeros((2, 32), np.uint32)
    counts[1, 3] = 2980                   # log1p(2980) = 7.99999... -> 1.0 after bfloat16 rounding
    f = M.encode(counts, None, M.iteration_code(8))
    assert f.shape == (2, 36)
    assert np.all(f[:, :32][counts == 0] == 0.0)
    assert f[1, 3] == 1.0
    assert np.array_equal(f[:, 32:35], [[0, 0, 1], [0, 0, 1]])
    assert f[0, 35] == 0.5                # log2(8) / 6


def _theta(**kw):
    d = {name: np.zeros(shape) for name, shape in M.SIZES}
    d.update(kw)
    return M.pack(d)


def test_forward_closed_forms():
    X = M.bf16(np.random.default_rng(0).uniform(-1, 1, (9, 36)))
    c = M.forward(_theta(b3=np.array([0.75])), X)
    assert np.all(c.y == 0.75)
    W1 = np.zeros((36, 64))
    W1[5, 7] = 1.0                        # input 5 -> hidden 7 (row = input)
    W2 = np.zeros((64, 64))
    W2[7, 3] = 1.0                        # hidden 7 -> hidden 3
    w3 = np.zeros(64)
    w3[3] = 2.0
    c = M.forward(_theta(W1=W1, W2=W2, w3=w3, b3=np.array([0.5])), X)
    assert np.array_equal(c.y, 2.0 * np.maximum(X[:, 5], 0.0) + 0.5)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = M.init_params(3)
    theta[M.N_PARAMS - 1] = 0.3
    X = rng.uniform(0, 1, (7, 36))
    t = rng.normal(size=7)
    p = M.unpack(theta)
    z1 = X @ p["W1"] + p["b1"]
    z2 = np.maximum(z1, 0) @ p["W2"] + p["b2"]
    assert np.abs(z1).min() > 1e-3 and np.abs(z2).min() > 1e-3      # away from the ReLU kinks
    g, _ = M.gradient(theta, X, t, emulate=False)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd[k] = (M.loss(theta + e, X, t, False) - M.loss(theta - e, X, t, False)) / (2 * h)
    o = 0
    for name, shape in M.SIZES:
        k = int(np.prod(shape))
        a, b = g[o:o + k], fd[o:o + k]
        assert np.abs(a - b).max() <= 1e-6 * max(np.abs(b).max(), 1e-3), name
        o += k


def test_adam_first_step_closed_form():
    theta = M.init_params(4)
    g = np.random.default_rng(2).normal(size=theta.size)
    opt = M.Adam(lr=1e-3)
    th, m, v = M.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), 1, g, opt)
    want = (theta - 1e-3 * g / (np.abs(g) + 1e-8)).astype(F32).astype(np.float64)
    assert np.array_equal(th, want)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_fits_a_realisable_target():
    """A teacher network of the same shape labels random inputs; Adam on the student drives the
    loss down by two orders of magnitude (float64 mode)."""
    rng = np.random.default_rng(7)
    X = rng.uniform(0, 1, (256, 36))
    teacher = M.init_params(11)
    t = M.forward(teacher, X, emulate=False).y
    theta = M.init_params(12)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = M.loss(theta, X, t, False)
    opt = M.Adam(lr=3e-3)
    for step in range(1, 401):
        g, _ = M.gradient(theta, X, t, emulate=False)
        theta, m, v = M.adam_step(theta, m, v, step, g, opt)
    assert M.loss(theta, X, t, False) < l0 / 100


def test_emulated_gradient_close_to_exact():
    """bfloat16 rounding perturbs the gradient by about 2^-8 relative, not more."""
    rng = np.random.default_rng(3)
    theta = M.init_params(5)
    X = M.bf16(rng.uniform(0, 1, (64, 36)))
    t = rng.normal(size=64)
    ge, _ = M.gradient(theta, X, t, emulate=True)
    gx, _ = M.gradient(theta, X, t, emulate=False)
    assert np.linalg.norm(ge - gx) <= 0.03 * np.linalg.norm(gx)


def test_proposal_clamp():
    r = M.propose(np.array([0.0, -1.0, -50.0, 1.0]), 0.05, 1e-4, np.full(4, 0.04, F32))
    assert r[0] == F32(0.04)                          # never above the current radius
    assert r[1] == F32(0.05 * math.exp(-1.0))
    assert r[2] == F32(1e-4)                          # never below the bound
    assert r[3] == F32(0.04)
