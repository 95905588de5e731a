"""Pins of the vertex-connection oracle for the box scene (the VC half of Eq. VCM-estimator with the
balance heuristic of Eq. mis-weight): the connection and merge weights are complementary, the
shadow test reproduces the sphere's shadow disk, the r -> 0 limit is the analytic direct light, and
and with the connection the merge share of the light is completed."""
import math

import numpy as np

from oracle import emit as E
from oracle import vc as VC
from workloads import generators as G

F32 = np.float32


def _box_kernels(res):
    scene = G.BoxScene(res=res)
    pos, nrm, _ = scene.hit_points()
    H = pos.shape[1]
    return scene, G.KernelSet(pos=pos, nrm=nrm, cam_beta=np.ones((3, H), F32), cam_mis=np.zeros((3, H), F32))


def test_connection_and_merge_weights_sum_to_one(oracle_mod):
    """A light vertex placed on a camera vertex, carrying the emission's dVCM for that point: its
    merge weight (C oracle) plus the connection weight (vc.py) is one."""
    box = E.Box()
    scene, ks = _box_kernels(16)
    sel = np.arange(0, ks.n, 7)
    sub = G.KernelSet(pos=ks.pos[:, sel], nrm=ks.nrm[:, sel], cam_beta=ks.cam_beta[:, sel], cam_mis=ks.cam_mis[:, sel])
    L = np.asarray(box.light, dtype=np.float64)[:, None]
    p = sub.pos.astype(np.float64)
    d2 = ((L - p) ** 2).sum(0)
    cos = np.maximum(((L - p) * sub.nrm).sum(0) / np.sqrt(d2), 1e-3)
    J = 50_000
    r = np.full(sub.n, F32(0.03), F32)
    for k in range(sub.n):
        one = G.KernelSet(pos=sub.pos[:, k:k + 1], nrm=sub.nrm[:, k:k + 1], cam_beta=sub.cam_beta[:, k:k + 1],
                          cam_mis=sub.cam_mis[:, k:k + 1])
        ph = G.PhotonBatch(J=J, pos=sub.pos[:, k:k + 1].copy(), flux=np.ones((3, 1), F32), nrm=sub.nrm[:, k:k + 1].copy(),
                           mis=np.array([[4 * math.pi * d2[k] / cos[k]], [0.0], [0.0]], F32))
        g = oracle_mod.gather(one, ph, r[k:k + 1], vcm=True)
        w_vm = g.flux[0, 0]
        w_vc, _, _ = VC.connect_weight(box.light, one.pos, one.nrm, r[k:k + 1], J)
        if cos[k] > 1e-3:
            assert abs(w_vm + w_vc[0] - 1.0) < 2e-6, (k, w_vm, w_vc)


def test_shadow_disk_on_the_floor():
    box = E.Box()
    g = np.linspace(0.02, 0.98, 200)
    X, Z = np.meshgrid(g, g)
    pos = np.stack([X.ravel(), np.zeros(X.size), Z.ravel()]).astype(F32)
    V = VC.visible(box.light, box.sphere_c, box.sphere_r, pos)
    dist = math.dist(box.light, box.sphere_c)
    rad = box.light[1] * (box.sphere_r / dist) / math.sqrt(1 - (box.sphere_r / dist) ** 2)
    rr = np.hypot(pos[0] - 0.5, pos[2] - 0.5)
    assert not V[rr < rad * (1 - 1e-4)].any()
    assert V[rr > rad * (1 + 1e-4)].all()
    # nothing else on the walls is shadowed: the sphere lies below the light
    side = np.stack([np.zeros(X.size), X.ravel(), Z.ravel()]).astype(F32)
    assert VC.visible(box.light, box.sphere_c, box.sphere_r, side).sum() > 0.9 * side.shape[1]


def test_zero_radius_limit_is_the_analytic_direct_light():
    """r -> 0: the connection weight tends to one and the connection alone is the direct light."""
    box = E.Box()
    scene, ks = _box_kernels(24)
    r = np.full(ks.n, F32(1e-7), F32)
    c = VC.connect(box.light, box.sphere_c, box.sphere_r, box.power, ks, r, J=1_000_000)
    truth = scene.irradiance(ks.pos, ks.nrm)                 # I cos / d^2 with the sphere's visibility
    assert np.max(np.abs(c[:, 0] - truth) / np.maximum(truth, 1e-12)) < 1e-4
    assert np.array_equal(c[:, 0], c[:, 2])


def test_connection_completes_the_merge_share(oracle_mod):
    """The box scene through the oracle in vertex-merging mode with the emission's partials. Merging
    alone carries only its MIS share (1 - w_VC) of the direct light; with the connection the two
    shares add up to the whole light (small radius, so the kernel's smoothing bias is small)."""
    box = E.Box()
    scene, ks = _box_kernels(20)
    truth = scene.irradiance(ks.pos, ks.nrm) / math.pi
    p = G.Params(r1=0.01, mode="vcm")
    J = 40_000
    s_vm = oracle_mod.init_state(ks.n, p.r1)
    s_vc = oracle_mod.init_state(ks.n, p.r1)
    share = np.zeros(ks.n)
    n_it = 8
    for it in range(n_it):
        pos, nrm, flux, mis = E.emit(box, J, it, 0, 3, with_mis=True)
        keep = np.isfinite(pos[0])
        ph = G.PhotonBatch(J=J, pos=pos[:, keep], flux=flux[:, keep], nrm=nrm[:, keep], mis=mis[:, keep])
        c = VC.connect(box.light, box.sphere_c, box.sphere_r, box.power, ks, s_vc.r, J)
        w, _, _ = VC.connect_weight(box.light, ks.pos, ks.nrm, s_vm.r, J)
        share += 1.0 - w
        oracle_mod.iterate(p, ks, s_vm, ph)
        oracle_mod.iterate(p, ks, s_vc, ph, connect=c)
    share /= n_it
    lit = truth > 0.1
    ratio_vc = oracle_mod.radiance(s_vc)[lit, 0] / truth[lit]
    ratio_vm = oracle_mod.radiance(s_vm)[lit, 0] / (truth[lit] * share[lit])
    assert abs(np.median(ratio_vc) - 1.0) < 0.03, np.median(ratio_vc)
    assert abs(np.median(ratio_vm) - 1.0) < 0.05, np.median(ratio_vm)
    assert np.median(share[lit]) < 0.9                      # the connection's share is material here
    e_vc = ((oracle_mod.radiance(s_vc)[:, 0] - truth) ** 2).mean()
    e_vm = ((oracle_mod.radiance(s_vm)[:, 0] - truth) ** 2).mean()
    assert e_vc < e_vm
