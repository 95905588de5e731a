"""CPU oracle of the learned radius proposal (an addition to the paper's method, not part of it).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg are
the only callers. It shares no code with the GPU library and never imports it.

What it defines (the GPU library must reproduce it):

* features of a hit point: light-vertex counts in 8 equi-areal rings at 4 radii r1 / 2^s (computed
  by ``oracle_features`` in hk_oracle.c), encoded as log1p(count) / 8, then the hit point's normal
  and a per-call iteration code, 36 inputs in all, each rounded to bfloat16;
* a multilayer perceptron 36 -> 64 -> 64 -> 1 with ReLU, weights used in bfloat16, biases and
  accumulation in float32 on the GPU (float64 here), predicting log(r_final / r1);
* its gradient for the mean squared error, with the activations and back-propagated errors rounded
  to bfloat16 exactly where the GPU rounds them (``emulate=True``), or in plain float64
  (``emulate=False``, for finite-difference checks);
* Adam (Kingma and Ba 2015) on float32-rounded master parameters;
* the proposal: r = clamp(r1 exp(y + margin), lb, r_current).

Parameter vector order: W1 (36 x 64, row = input), b1 (64), W2 (64 x 64, row = input), b2 (64),
w3 (64), b3 (1) -- 6593 values.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np

from . import oracle as O

N_IN, N_H = 36, 64
SIZES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("w3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)
F32 = np.float32


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SIZES])


def bf16(x) -> np.ndarray:
    """Round to bfloat16, nearest-even, from the float32 value of x (returned as float64)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(F32))
    b = f.view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(F32).astype(np.float64)


def bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of round-to-nearest-even of float32(x)."""
    return (bf16(x).astype(F32).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, np.uint32) << 16).astype(np.uint32).view(F32).astype(np.float64)


# ---------------------------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------------------------

def feature_counts(kernels, photons, r1: float, cos_min: float = 0.5, nthreads: int = 0) -> np.ndarray:
    """H x 32 ring counts (uint32) of every kernel against every stored light vertex."""
    H = kernels.n
    kp = [np.ascontiguousarray(kernels.pos[a], F32) for a in range(3)]
    use_n = kernels.nrm is not None and photons.nrm is not None
    kn = [np.ascontiguousarray(kernels.nrm[a], F32) for a in range(3)] if use_n else [None] * 3
    pp = [np.ascontiguousarray(photons.pos[a], F32) for a in range(3)]
    pn = [np.ascontiguousarray(photons.nrm[a], F32) for a in range(3)] if use_n else [None] * 3
    out = np.zeros((H, 32), np.uint32)
    fp = ctypes.POINTER(ctypes.c_float)
    P = lambda a: None if a is None else a.ctypes.data_as(fp)  # noqa: E731
    L = O.lib()
    fn = L.oracle_features
    fn.restype = ctypes.c_int
    fn(ctypes.c_int64(H), P(kp[0]), P(kp[1]), P(kp[2]), P(kn[0]), P(kn[1]), P(kn[2]),
       ctypes.c_int64(photons.n), P(pp[0]), P(pp[1]), P(pp[2]), P(pn[0]), P(pn[1]), P(pn[2]),
       ctypes.c_float(r1), ctypes.c_float(cos_min), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
       ctypes.c_int(nthreads))
    return out


def encode(counts: np.ndarray, normals, it_code: float) -> np.ndarray:
    """36 inputs per kernel, as float64 values of bfloat16 numbers."""
    H = counts.shape[0]
    f = np.zeros((H, N_IN))
    f[:, :32] = np.log1p(counts.astype(np.float64)) / 8.0
    if normals is None:
        f[:, 34] = 1.0
    else:
        f[:, 32:35] = np.asarray(normals, np.float64).T
    f[:, 35] = float(np.float32(it_code))
    return bf16(f)


def iteration_code(i: int) -> float:
    """Iteration input of the network: log2(i) / 6, as float32."""
    return float(np.float32(math.log2(i) / 6.0))


# ---------------------------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------------------------

@dataclass
class Cache:
    X: np.ndarray
    H1: np.ndarray
    H2: np.ndarray
    y: np.ndarray


def _weights(p: dict, emulate: bool):
    r = bf16 if emulate else (lambda a: np.asarray(a, np.float64))
    return r(p["W1"]), r(p["W2"]), r(p["w3"])


def forward(theta: np.ndarray, X: np.ndarray, emulate: bool = True) -> Cache:
    """y = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3 for every row x of X."""
    p = unpack(theta)
    W1, W2, w3 = _weights(p, emulate)
    r = bf16 if emulate else (lambda a: a)
    X = np.asarray(X, np.float64)
    H1 = r(np.maximum(X @ W1 + p["b1"], 0.0))
    H2 = r(np.maximum(H1 @ W2 + p["b2"], 0.0))
    y = H2 @ w3 + p["b3"][0]
    return Cache(X, H1, H2, y)


def loss(theta, X, t, emulate: bool = True) -> float:
    c = forward(theta, X, emulate)
    return float(np.mean((c.y - np.asarray(t, np.float64)) ** 2))


def gradient(theta: np.ndarray, X: np.ndarray, t: np.ndarray, emulate: bool = True):
    """Gradient of the mean squared error (back-propagation; with ``emulate`` the back-propagated
    errors entering the two matrix products are rounded to bfloat16, as on the GPU)."""
    p = unpack(theta)
    W1, W2, w3 = _weights(p, emulate)
    r = bf16 if emulate else (lambda a: a)
    c = forward(theta, X, emulate)
    n = X.shape[0]
    dy = (2.0 / n) * (c.y - np.asarray(t, np.float64))
    g = {"w3": c.H2.T @ dy, "b3": np.array([dy.sum()])}
    dZ2 = r(np.outer(dy, w3) * (c.H2 > 0))
    g["W2"] = c.H1.T @ dZ2
    g["b2"] = dZ2.sum(0)
    dZ1 = r((dZ2 @ W2.T) * (c.H1 > 0))
    g["W1"] = c.X.T @ dZ1
    g["b1"] = dZ1.sum(0)
    return pack(g), float(np.mean((c.y - t) ** 2))


@dataclass
class Adam:
    lr: float
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


def adam_step(theta, m, v, step: int, grad, opt: Adam):
    """One Adam update (step counts from 1); master parameters are float32 numbers."""
    m = opt.beta1 * m + (1.0 - opt.beta1) * grad
    v = opt.beta2 * v + (1.0 - opt.beta2) * grad * grad
    mh = m / (1.0 - opt.beta1 ** step)
    vh = v / (1.0 - opt.beta2 ** step)
    theta = theta - opt.lr * mh / (np.sqrt(vh) + opt.eps)
    return theta.astype(F32).astype(np.float64), m, v


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (float32 values)."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence(seed)))
    d = {"W1": rng.normal(0, math.sqrt(2.0 / N_IN), (N_IN, N_H)), "b1": np.zeros(N_H),
         "W2": rng.normal(0, math.sqrt(2.0 / N_H), (N_H, N_H)), "b2": np.zeros(N_H),
         "w3": rng.normal(0, math.sqrt(1.0 / N_H), N_H), "b3": np.zeros(1)}
    return pack(d).astype(F32).astype(np.float64)


def propose(y: np.ndarray, r1: float, lb: float, r_cur: np.ndarray, margin: float = 0.0) -> np.ndarray:
    """Proposed radii: r1 exp(y + margin) (the sum in float32), clamped to [lb, r_current] (never
    larger than the current radius)."""
    e = (np.asarray(y, F32) + F32(margin)).astype(np.float64)
    r = (np.float64(F32(r1)) * np.exp(e)).astype(F32)
    return np.minimum(np.maximum(r, F32(lb)), np.asarray(r_cur, F32))
