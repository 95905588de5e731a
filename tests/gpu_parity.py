"""Side-by-side runs of the HIP path (through the C ABI) and the CPU oracle, compared per iteration.

Rules (parity bar):
  * per-kernel in-disk counts: bit-exact;
  * shrink decisions: exact, except where the oracle's |F - Fc| < 1e-6 (either outcome is correct);
    a kernel whose decision differs inside that band leaves the comparison from then on;
  * radii: bit-exact for kernels still compared (both sides update in float32);
  * F: per kernel, |dF| <= max(1, F) (2 sqrt(n / 132) + 2) (2 n + 65 k) e + 1e-13, with n the
    samples in the retained sums, k the iterations so far and e = 2^-53. The group sums are float64
    on both sides: a float32 sample and its square are exact in float64, and each addition of a
    nonnegative term rounds by at most e of the running sum, so a kernel's group sum that took at
    most n samples, 64 lane partials and one retained sum per iteration is off by at most
    (n + 65 k) e of its value, the oracle's by at most n e. F's
    sensitivity to such relative errors is about 2 S_g / sqrt(sum_g d_g^2) through the
    between-group term (d_g = S_g - mean; near the null hypothesis this is 2 sqrt(n_g / 11) with
    n_g = n / 12 samples per group) plus about 2 through the within-group term; 1e-13 covers F's
    own float64 evaluation. At the workloads' sizes this stays below 1e-10, far inside the 1e-6
    decision band;
  * critical values: relative 1e-10;
  * radiance: relative 1e-5.
"""
from __future__ import annotations

import sys
from dataclasses import dataclass, field

import numpy as np
import torch

from oracle import oracle as O
from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
from workloads import generators as G

BAND = 1e-6


@dataclass
class ParityReport:
    iterations: int = 0
    kernels: int = 0
    band_flips: int = 0
    band_cases: int = 0
    shrinks: int = 0
    max_F_rel: float = 0.0
    max_Fc_rel: float = 0.0
    max_L_rel: float = 0.0
    excluded: int = 0
    worst_F: dict = field(default_factory=dict)
    notes: list = field(default_factory=list)


def sub_kernels(ks: G.KernelSet, idx):
    return ks.subset(idx)


def _err_F(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    d = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    d[np.isnan(a) & np.isnan(b)] = 0.0
    return d


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    both_nan = np.isnan(a) & np.isnan(b)
    d = np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
    d[both_nan] = 0.0
    d[(a == b)] = 0.0
    return d


class Tracker:
    """Oracle run of one set (kernels idx) checked against the GPU set `set_id` after each iteration."""

    def __init__(self, w: G.Workload, idx=None, name=None):
        self.w, self.p = w, w.params
        ks = w.kernels
        self.idx = np.arange(ks.n) if idx is None else np.asarray(idx)
        self.oks = sub_kernels(ks, self.idx)
        self.ost = O.init_state(self.idx.size, self.p.r1, rgb=self.p.stats == "rgb")
        self.alive = np.ones(self.idx.size, bool)
        self.rep = ParityReport(kernels=self.idx.size)
        self.name = name or w.name
        self.nseen = np.zeros(self.idx.size, np.int64)     # retained samples before this iteration

    def step(self, est: Estimator, set_id: int, ph, connect_fn=None):
        """Advances the oracle by the iteration the GPU just ran with photons ph and compares.
        `connect_fn(kernels, r)` gives the oracle's vertex-connection term for the tracked kernels at
        the oracle's own radii, when the GPU iteration had one."""
        idx, ost, alive, rep = self.idx, self.ost, self.alive, self.rep
        it = rep.iterations
        extra = connect_fn(self.oks, ost.r) if connect_fn is not None else None
        O.iterate(self.p, self.oks, ost, ph, connect=extra)
        d = {k: v.cpu().numpy()[idx] for k, v in est.debug(set_id).items()}
        rg = est.radii(set_id).cpu().numpy()[idx]
        cnt = d["count"].astype(np.uint32)
        bad = np.flatnonzero(alive & (cnt != ost.count))
        assert bad.size == 0, (f"[{self.name}] iteration {it + 1}: count mismatch at {idx[bad[:5]]}: "
                               f"{cnt[bad[:5]]} vs {ost.count[bad[:5]]}")
        band = np.abs(ost.F - ost.Fc) < BAND
        if ost.F_channels is not None:             # one test per channel: any channel in the band
            band = np.any(np.abs(ost.F_channels - ost.Fc[:, None]) < BAND, axis=1)
        dg = d["decision"].astype(bool)
        diff = alive & (dg != ost.shrink)
        assert not np.any(diff & ~band), \
            f"[{self.name}] iteration {it + 1}: decision mismatch outside the band at {idx[diff & ~band][:5]}"
        rep.band_cases += int((alive & band).sum())
        rep.band_flips += int(diff.sum())
        alive &= ~diff
        rep.shrinks += int((alive & ost.shrink).sum())
        badr = np.flatnonzero(alive & (rg != ost.r))
        assert badr.size == 0, (f"[{self.name}] iteration {it + 1}: radius mismatch at {idx[badr[:5]]}: "
                                f"{rg[badr[:5]]} vs {ost.r[badr[:5]]}")
        n_ret = (self.nseen + ost.count).astype(np.float64)
        self.nseen = ost.nseen.astype(np.int64).copy()
        e = 2.0 ** -53
        adds = 2.0 * n_ret + 65.0 * (it + 1)
        tol = np.maximum(1.0, np.abs(ost.F)) * (2.0 * np.sqrt(n_ret / 132.0) + 2.0) * adds * e + 1e-13
        dF = np.abs(d["F"] - ost.F)
        badF = np.flatnonzero(alive & np.isfinite(ost.F) & ~(dF <= tol))
        assert badF.size == 0, (f"[{self.name}] iteration {it + 1}: F beyond its rounding bound at {idx[badF[:5]]}: "
                                f"{d['F'][badF[:5]]} vs {ost.F[badF[:5]]} (bound {tol[badF[:5]]})")
        fr = _err_F(d["F"], ost.F)[alive]
        assert np.all(np.isnan(d["F"][alive]) == np.isnan(ost.F[alive])), f"[{self.name}] F defined on one side only"
        if fr.size and np.nanmax(fr) > rep.max_F_rel:
            k = np.flatnonzero(alive)[int(np.nanargmax(fr))]
            rep.max_F_rel = float(fr[int(np.nanargmax(fr))])
            rep.worst_F = dict(iteration=it + 1, kernel=int(idx[k]), F_gpu=float(d["F"][k]), F_oracle=float(ost.F[k]),
                               Fc=float(ost.Fc[k]), count=int(ost.count[k]), m=float(ost.m[k]))
        fin = alive & np.isfinite(ost.Fc)
        if fin.any():
            rep.max_Fc_rel = max(rep.max_Fc_rel, float(_rel(d["Fc"][fin], ost.Fc[fin]).max()))
        rep.iterations += 1

    def finish(self, est: Estimator, set_id: int) -> ParityReport:
        rep, alive, idx = self.rep, self.alive, self.idx
        assert rep.max_F_rel < 1e-8, rep
        assert rep.max_Fc_rel < 1e-10, rep
        Lg = est.radiance(set_id).cpu().numpy()[:, idx].T
        Lo = O.radiance(self.ost)
        lr = _rel(Lg[alive], Lo[alive])
        rep.max_L_rel = float(lr.max()) if lr.size else 0.0
        assert rep.max_L_rel < 1e-5, rep
        rep.excluded = int((~alive).sum())
        assert rep.excluded <= max(2, idx.size // 1000), rep
        return rep


def make_estimator(w: G.Workload, **est_kw) -> Estimator:
    p = w.params
    return Estimator(p.r1, mode=p.mode, k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin, stats=p.stats, **est_kw)


def run_parity(w: G.Workload, n_iter: int, idx=None, photons_fn=None, est_kw=None, verbose=True) -> ParityReport:
    """Runs n_iter iterations on the GPU (all kernels) and on the oracle (kernels idx, default all)."""
    ks = w.kernels
    est = make_estimator(w, **(est_kw or {}))
    est.set_kernels(0, ks.pos, ks.nrm, None, ks.cam_beta, ks.cam_mis)
    tr = Tracker(w, idx)
    get = photons_fn or w.photons
    for it in range(n_iter):
        ph = get(it)
        if verbose:
            print(f"  [{w.name}] iteration {it + 1}/{n_iter}: H={ks.n} J={ph.J} stored={ph.n}", flush=True)
        est.iterate([0], [DevicePhotons.upload(ph)])
        tr.step(est, 0, ph)
    rep = tr.finish(est, 0)
    est.close()
    if verbose:
        print(f"  parity ok: {rep}", flush=True)
    sys.stdout.flush()
    return rep
