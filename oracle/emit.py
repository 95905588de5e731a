"""CPU oracle of light-vertex generation for the box scene (the step before the estimator: light
sub-paths from an isotropic point light, first hits on the five walls of a unit box open at z = 1,
an opaque sphere inside).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg are
the only callers. It shares no code with the GPU library and never imports it.

The paper's renderer traces light sub-paths (Sec. 4, the light pass of VCM); it fixes neither the
random numbers nor the scene, so this generator is a definition of our own, stated here in full and
computed in float32 with one rounding per operation (no fused multiply-add), so that any
implementation that performs the same correctly rounded operations in the same order produces the
same bits:

Random numbers. Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC 2011): counter (j, i, s, b) and key (seed mod 2^32, seed div 2^32) for sub-path j of
iteration i (0-based) of set s, block b = 0..7. A 32-bit output x becomes u = (x >> 8) 2^-24.

Direction (Marsaglia 1972, rejection from the square). Block b gives attempts 2b (words 0, 1) and
2b + 1 (words 2, 3): a = 2u - 1, c = 2u' - 1, q = a a + c c. The first attempt with 0 < q < 1 gives
d = (a f, c f, 1 - 2q) with f = 2 sqrt(1 - q), uniform on the unit sphere. Sixteen failed attempts
(probability (1 - pi/4)^16, about 5e-11) leave the sub-path without a vertex.

First hit. Per axis, t_a = (1 - L_a) / d_a for d_a > 0, (0 - L_a) / d_a for d_a < 0, infinity for
d_a = 0; t is the smallest, on the first axis (x, then y, then z) that attains it. The path escapes
when that axis is z with d_z > 0 (the open top). The sphere (centre C, radius R) occludes when,
with o = L - C, B = (d_x o_x + d_y o_y) + d_z o_z and Q = ((o_x o_x + o_y o_y) + o_z o_z) - R R,
the discriminant D = B B - Q is positive and t_s = -B - sqrt(D) lies in (0, t). A kept vertex sits
at L_a + t d_a clamped to [0, 1], with the hit axis set to exactly 1 (d_a > 0) or 0; its normal is
-1 (d_a > 0) or +1 on the hit axis and 0 elsewhere, and it carries the scene's power in R, G and B.
A sub-path without a vertex leaves NaN positions, zero normal and zero flux in its slot.

For vertex merging with the vertex-connection half (the next-event connection to the point light),
a kept vertex also carries dVCM = (4 pi t^2) / |d_a| in float32, computed as (F(4 pi) (t t)) / |d_a|.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

F32 = np.float32
U32 = np.uint32
U64 = np.uint64

# Philox constants (Salmon et al. 2011, Table 2 and the Weyl key schedule)
PHILOX = {
    32: dict(M=(0xD2511F53, 0xCD9E8D57), W=(0x9E3779B9, 0xBB67AE85)),
    64: dict(M=(0xD2E7470EE14C6C93, 0xCA5A826395121157), W=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}
ATTEMPT_BLOCKS = 8


def philox4_scalar(ctr, key, width: int = 32, rounds: int = 10):
    """One Philox4xW block with Python integers: each round multiplies words 0 and 2 by the round
    multipliers, and the new words are (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
    lo(M0 c0)); the key is bumped by the Weyl constants between rounds."""
    mask = (1 << width) - 1
    M0, M1 = PHILOX[width]["M"]
    W0, W1 = PHILOX[width]["W"]
    c = [int(v) & mask for v in ctr]
    k0, k1 = int(key[0]) & mask, int(key[1]) & mask
    for r in range(rounds):
        if r:
            k0, k1 = (k0 + W0) & mask, (k1 + W1) & mask
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [((p1 >> width) ^ c[1] ^ k0) & mask, p1 & mask, ((p0 >> width) ^ c[3] ^ k1) & mask, p0 & mask]
    return c


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over uint32 arrays (broadcast); returns four uint32 arrays."""
    M0, M1 = (U64(m) for m in PHILOX[32]["M"])
    W0, W1 = (U32(w) for w in PHILOX[32]["W"])
    c0, c1, c2, c3 = (np.asarray(v, dtype=U32) for v in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0, k1 = U32(k0), U32(k1)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0, k1 = U32(k0 + W0), U32(k1 + W1)
            p0 = c0.astype(U64) * M0
            p1 = c2.astype(U64) * M1
            c0, c1, c2, c3 = ((p1 >> U64(32)).astype(U32) ^ c1 ^ k0, (p1 & U64(0xFFFFFFFF)).astype(U32),
                              (p0 >> U64(32)).astype(U32) ^ c3 ^ k1, (p0 & U64(0xFFFFFFFF)).astype(U32))
    return c0, c1, c2, c3


def uniform(x):
    """u = (x >> 8) 2^-24 in [0, 1), exact in float32."""
    return (np.asarray(x, dtype=U32) >> U32(8)).astype(F32) * F32(2.0 ** -24)


@dataclass(frozen=True)
class Box:
    light: tuple = (0.5, 0.9, 0.5)
    sphere_c: tuple = (0.5, 0.5, 0.5)
    sphere_r: float = 0.15
    power: float = float(F32(4.0 * np.pi))   # per kept vertex and channel (4 pi I with I = 1 W/sr)


def directions(J: int, it: int, set_id: int, seed: int):
    """Unit directions (3, J) float32 and the mask of sub-paths that drew one."""
    j = np.arange(J, dtype=np.int64).astype(U32)
    k0, k1 = U32(seed & 0xFFFFFFFF), U32((seed >> 32) & 0xFFFFFFFF)
    a = np.zeros(J, F32)
    c = np.zeros(J, F32)
    q = np.zeros(J, F32)
    done = np.zeros(J, bool)
    for b in range(ATTEMPT_BLOCKS):
        todo = np.nonzero(~done)[0]
        if todo.size == 0:
            break
        x = philox4x32_10(j[todo], U32(it), U32(set_id), U32(b), k0, k1)
        for w in (0, 2):
            left = ~done[todo]
            aa = F32(2.0) * uniform(x[w]) - F32(1.0)
            cc = F32(2.0) * uniform(x[w + 1]) - F32(1.0)
            qq = aa * aa + cc * cc
            ok = left & (qq > F32(0.0)) & (qq < F32(1.0))
            sel = todo[ok]
            a[sel], c[sel], q[sel] = aa[ok], cc[ok], qq[ok]
            done[sel] = True
    f = F32(2.0) * np.sqrt(F32(1.0) - q)
    d = np.stack([a * f, c * f, F32(1.0) - F32(2.0) * q]).astype(F32)
    return d, done


def emit(box: Box, J: int, it: int, set_id: int = 0, seed: int = 1, with_mis: bool = False):
    """The J slots of iteration `it`: pos (3, J), nrm (3, J), flux (3, J) float32 (see the module
    docstring for the definition); with `with_mis` also the vertex-merging partials (3, J): dVCM =
    (4 pi t^2) / |d_a| on the hit axis a, the reciprocal of the area density with which the light
    pass reaches the vertex (isotropic emission 1 / (4 pi), times cos / t^2 with t the distance and
    d a unit direction), and dVC = dVM = 0 (nothing precedes a vertex reached from a point light)."""
    d, drawn = directions(J, it, set_id, seed)
    L = np.asarray(box.light, dtype=F32)
    Cs = np.asarray(box.sphere_c, dtype=F32)
    R = F32(box.sphere_r)
    t_ax = np.full((3, J), np.inf, dtype=F32)
    with np.errstate(divide="ignore", invalid="ignore"):
        for ax in range(3):
            pos_side = d[ax] > 0
            neg_side = d[ax] < 0
            num = np.where(pos_side, F32(1.0) - L[ax], F32(0.0) - L[ax]).astype(F32)
            t_ax[ax] = np.where(pos_side | neg_side, num / d[ax], F32(np.inf))
    t = np.minimum(np.minimum(t_ax[0], t_ax[1]), t_ax[2])
    hit_ax = np.where(t_ax[0] == t, 0, np.where(t_ax[1] == t, 1, 2))
    escaped = (hit_ax == 2) & (d[2] > 0)
    o = (L - Cs).astype(F32)
    B = (d[0] * o[0] + d[1] * o[1]) + d[2] * o[2]
    Q = ((o[0] * o[0] + o[1] * o[1]) + o[2] * o[2]) - R * R
    D = B * B - Q
    with np.errstate(invalid="ignore"):
        ts = -B - np.sqrt(np.maximum(D, F32(0.0)))
    occluded = (D > 0) & (ts > 0) & (ts < t)
    keep = drawn & ~escaped & ~occluded
    pos = np.full((3, J), np.nan, dtype=F32)
    nrm = np.zeros((3, J), dtype=F32)
    flux = np.zeros((3, J), dtype=F32)
    for ax in range(3):
        p = np.clip(L[ax] + t * d[ax], F32(0.0), F32(1.0))
        on = hit_ax == ax
        p = np.where(on, np.where(d[ax] > 0, F32(1.0), F32(0.0)), p)
        pos[ax] = np.where(keep, p, F32(np.nan))
        nrm[ax] = np.where(keep & on, np.where(d[ax] > 0, F32(-1.0), F32(1.0)), F32(0.0))
        flux[ax] = np.where(keep, F32(box.power), F32(0.0))
    if not with_mis:
        return pos, nrm, flux
    dh = np.abs(np.choose(np.where(keep, hit_ax, 0), d)).astype(F32)
    with np.errstate(divide="ignore", invalid="ignore"):
        dvcm = (F32(4.0 * np.pi) * (t * t)) / dh
    mis = np.zeros((3, J), dtype=F32)
    mis[0] = np.where(keep, dvcm, F32(0.0))
    return pos, nrm, flux, mis
