"""CPU oracle of the vertex-connection half of the VCM estimator for the box scene (Eq.
`VCM-estimator`: the VC sum next to the VM sum), restricted to what the box scene holds: camera
vertices at the first hit and a point light, so the VC technique is the connection of the camera
vertex to the light (next-event estimation, s = 1 light vertices).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg are
the only callers. It shares no code with the GPU library and never imports it.

With the balance heuristic (Eq. `mis-weight`, beta = 1), one light sub-path for connections
(n_VC = 1) and J for merging (n_VM = J), a path light -> x -> camera has two techniques here:

    VC   connect x to the light:    density p_C(x)                       (the light is a point)
    VM   merge a light vertex at x: density p_C(x) p_L(x) pi r^2

with p_L(x) = cos(theta_x) / (4 pi d^2) the area density of the light pass reaching x from an
isotropic point light at distance d. So the connection's weight is w_VC = 1 / (1 + eta p_L(x)) with
eta = J pi r^2, and the merge weight of a light vertex y is w_VM = eta p_L(y) / (1 + eta p_L(y)),
which is the merge weight 1 / (1 + W_L + W_C) with the light partial dVCM_L = 1 / p_L(y), dVM_L = 0
and zero camera partials (no other camera-side technique). The two weights sum to one at y = x.

The connection adds w_VC beta_C I cos(theta_x) V(x) / d^2 (per channel; I = power / (4 pi), the
point light's intensity; V the sphere's visibility) to the iteration's flux-density estimate, with
the radius r the iteration merges with; the radiance is f_r = 1 / pi times the progressive average.
The visibility decision is taken in float32 with the operation order stated in `visible`, the same
decision the kernel takes; the value is float64.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32


def visible(light, sphere_c, sphere_r, pos: np.ndarray) -> np.ndarray:
    """Float32 shadow test of the segment x -> light against the sphere: with w = L - x, dist =
    sqrt(w.w), u = w / dist, o = x - C, B = (u_x o_x + u_y o_y) + u_z o_z and
    Q = ((o_x o_x + o_y o_y) + o_z o_z) - R R, the segment is blocked when D = B B - Q > 0 and the
    near root -B - sqrt(D) lies in (0, dist)."""
    L = np.asarray(light, dtype=F32)
    C = np.asarray(sphere_c, dtype=F32)
    R = F32(sphere_r)
    p = np.asarray(pos, dtype=F32)
    w = (L[:, None] - p).astype(F32)
    d2 = (w[0] * w[0] + w[1] * w[1]) + w[2] * w[2]
    dist = np.sqrt(d2)
    u = (w / dist).astype(F32)
    o = (p - C[:, None]).astype(F32)
    B = (u[0] * o[0] + u[1] * o[1]) + u[2] * o[2]
    Q = ((o[0] * o[0] + o[1] * o[1]) + o[2] * o[2]) - R * R
    D = B * B - Q
    t0 = -B - np.sqrt(np.maximum(D, F32(0.0)))
    return ~((D > 0) & (t0 > 0) & (t0 < dist))


def connect_weight(light, pos: np.ndarray, nrm: np.ndarray, r: np.ndarray, J: int):
    """(w_VC, cos, d^2) per camera vertex in float64."""
    L = np.asarray(light, dtype=np.float64)[:, None]
    p = np.asarray(pos, dtype=np.float64)
    w = L - p
    d2 = (w * w).sum(0)
    cos = np.maximum(0.0, (w * np.asarray(nrm, dtype=np.float64)).sum(0) / np.sqrt(d2))
    eta = J * math.pi * np.asarray(r, dtype=np.float64) ** 2
    pL = cos / (4.0 * math.pi * d2)
    return 1.0 / (1.0 + eta * pL), cos, d2


def connect(light, sphere_c, sphere_r, power, kernels, r: np.ndarray, J: int) -> np.ndarray:
    """The connection's contribution to one iteration's flux-density estimate, (H, 3) float64."""
    wvc, cos, d2 = connect_weight(light, kernels.pos, kernels.nrm, r, J)
    V = visible(light, sphere_c, sphere_r, kernels.pos)
    I = float(power) / (4.0 * math.pi)
    e = wvc * I * cos / d2 * V
    beta = np.ones((kernels.n, 3)) if kernels.cam_beta is None else kernels.cam_beta.T.astype(np.float64)
    return beta * e[:, None]
