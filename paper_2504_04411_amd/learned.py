"""Learned radius proposal on top of the estimator (torch-side buffer owner, like estimator.py).

Every computation runs in libhk's kernels (features, forward, gradient, Adam, proposal); this module
owns the device buffers, shuffles mini-batch indices and sequences the calls.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import hk
from .estimator import DevicePhotons, Estimator

N_IN = 36


def iteration_code(i: int) -> float:
    """Iteration input of the network: log2(i) / 6 (float32)."""
    return float(np.float32(math.log2(i) / 6.0))


class Network:
    """Device state of one 36-64-64-1 network (parameters, Adam moments, bfloat16 weight copies)."""

    def __init__(self, est: Estimator, theta: np.ndarray):
        self.est = est
        self.P = hk.hk_mlp_param_count()
        self.state = torch.zeros(hk.hk_mlp_state_bytes(), dtype=torch.uint8, device=est.device)
        self.ws = torch.empty(0, dtype=torch.uint8, device=est.device)
        self.set_params(theta)

    @property
    def ctx(self):
        return self.est.ctx

    @property
    def stream(self):
        return self.est.stream

    def set_params(self, theta: np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(theta, dtype=np.float32)).to(self.est.device)
        assert t.numel() == self.P
        hk.hk_mlp_set_params(self.ctx, self.state.data_ptr(), t.data_ptr(), self.stream)
        self._keep = t

    def params(self) -> np.ndarray:
        out = torch.empty(self.P, dtype=torch.float32, device=self.est.device)
        hk.hk_mlp_get_params(self.ctx, self.state.data_ptr(), out.data_ptr(), self.stream)
        return out.cpu().numpy()

    def _workspace(self, n: int) -> torch.Tensor:
        need = hk.hk_mlp_workspace_bytes(n)
        if self.ws.numel() < need:
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.est.device)
        return self.ws

    def forward(self, feat: torch.Tensor) -> torch.Tensor:
        n = feat.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=self.est.device)
        hk.hk_mlp_forward(self.ctx, self.state.data_ptr(), feat.data_ptr(), n, y.data_ptr(), self.stream)
        return y

    def grad(self, feat: torch.Tensor, label: torch.Tensor):
        """(gradient of the mean squared error, sum of squared errors) over all rows."""
        n = feat.shape[0]
        ws = self._workspace(n)
        out = torch.empty(self.P + 1, dtype=torch.float32, device=self.est.device)
        hk.hk_mlp_grad(self.ctx, self.state.data_ptr(), feat.data_ptr(), label.data_ptr(), n, out.data_ptr(),
                       ws.data_ptr(), ws.numel(), self.stream)
        v = out.cpu().numpy()
        return v[:self.P].astype(np.float64), float(v[self.P])

    def train_step(self, feat: torch.Tensor, label: torch.Tensor, lr: float):
        n = feat.shape[0]
        ws = self._workspace(n)
        hk.hk_mlp_train_step(self.ctx, self.state.data_ptr(), feat.data_ptr(), label.data_ptr(), n, lr,
                             ws.data_ptr(), ws.numel(), self.stream)

    def train(self, feat: torch.Tensor, label: torch.Tensor, epochs: int, batch: int, lr: float, seed: int = 0,
              lr_final: Optional[float] = None):
        """Mini-batch Adam over shuffled rows; the learning rate decays geometrically to lr_final."""
        n = feat.shape[0]
        rng = np.random.Generator(np.random.Philox(np.random.SeedSequence(seed)))
        steps = epochs * max(1, n // batch)
        decay = (lr_final / lr) ** (1.0 / max(steps - 1, 1)) if lr_final else 1.0
        k = 0
        for _ in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).to(self.est.device)
            for b0 in range(0, n - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                self.train_step(feat.index_select(0, idx).contiguous(), label.index_select(0, idx).contiguous(),
                                lr * decay ** k)
                k += 1
        return k


def features(est: Estimator, set_id: int, photons: DevicePhotons, i: int, want_counts: bool = False):
    """Network inputs (H x 36 bfloat16 bit patterns as int16) of set set_id's hit points from one
    batch of light vertices, tagged as iteration i; optionally the H x 32 ring counts."""
    H = est.n[set_id]
    feat = torch.empty((H, N_IN), dtype=torch.int16, device=est.device)
    counts = torch.empty((H, 32), dtype=torch.int32, device=est.device) if want_counts else None
    ws = est._workspace(hk.hk_workspace_bytes(est.ctx, photons.n, H))
    ph = photons.struct()
    hk.hk_mlp_features(est.ctx, set_id, est.states[set_id].data_ptr(), ph, iteration_code(i), feat.data_ptr(),
                       counts.data_ptr() if counts is not None else None, ws.data_ptr(), ws.numel(), est.stream)
    return feat, counts


def propose(est: Estimator, set_id: int, y: torch.Tensor, margin: float = 0.0):
    """Applies network outputs y (log(r / r1), original order) to the set's radii for its next
    iteration: r = clamp(r1 exp(y + margin), lb, r)."""
    hk.hk_mlp_propose(est.ctx, set_id, est.states[set_id].data_ptr(), y.contiguous().data_ptr(), margin, est.stream)


# ---------------------------------------------------------------------------------------------
# training data from plain runs, and the comparison of plain and learned runs at equal MSE
# ---------------------------------------------------------------------------------------------

def _ws_for(est: Estimator, set_id: int, batches):
    return est._workspace(max(est.workspace_for([b], [set_id]) for b in batches))


def plain_run(est: Estimator, set_id: int, w, batches, feature_its=()):
    """Plain iterations of one scene over the device batches; features taken before iterations in
    feature_its (1-based, from that iteration's batch). Returns (features by iteration, final radii)."""
    ks, p = w.kernels, w.params
    est.set_kernels(set_id, ks.pos, ks.nrm, r1=p.r1, rmin=p.rmin)
    _ws_for(est, set_id, batches)
    feats = {}
    for i, b in enumerate(batches, start=1):
        if i in feature_its:
            feats[i] = features(est, set_id, b, i)[0]
        est.iterate([set_id], [b])
    return feats, est.radii(set_id)


def training_set(est: Estimator, scenes, feature_its=(1, 2, 4, 8)):
    """Rows (features at each of feature_its, label log(r_final / r1)) of every hit point of every
    (workload, device batches) scene."""
    X, Y = [], []
    for w, batches in scenes:
        feats, r = plain_run(est, 0, w, batches, feature_its)
        lab = torch.log(r / float(np.float32(w.params.r1)))
        for i in feature_its:
            X.append(feats[i])
            Y.append(lab)
    return torch.cat(X).contiguous(), torch.cat(Y).contiguous()


def _mse(est, set_id, truth):
    L = est.radiance(set_id)
    return float(((L - truth) ** 2).mean())


def _run(est: Estimator, set_id: int, w, batches, truth, net: Optional[Network] = None, margin: float = 0.0):
    """One run over the batches (with the network's proposal before the first iteration when net is
    given): per-iteration MSE against truth and cumulative GPU milliseconds."""
    ks, p = w.kernels, w.params
    est.set_kernels(set_id, ks.pos, ks.nrm, r1=p.r1, rmin=p.rmin)
    _ws_for(est, set_id, batches)
    torch.cuda.synchronize()
    ev, mse = [], []
    for i, b in enumerate(batches, start=1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if net is not None and i == 1:
            f, _ = features(est, set_id, b, 1)
            propose(est, set_id, net.forward(f), margin)
        est.iterate([set_id], [b])
        e1.record()
        ev.append((e0, e1))
        mse.append(_mse(est, set_id, truth))
    torch.cuda.synchronize()
    ms = np.cumsum([a.elapsed_time(c) for a, c in ev])
    return dict(mse=mse, ms=ms.tolist(), radius_mean=float(est.radii(set_id).mean()))


def summarize(plain: dict, learned: dict) -> dict:
    """Equal-MSE comparison: iterations and GPU time the learned run needs to reach the plain run's
    final MSE."""
    target = plain["mse"][-1]
    reach = next((i for i, m in enumerate(learned["mse"]) if m <= target), None)
    return {"plain_final_mse": target, "learned_final_mse": learned["mse"][-1],
            "iterations": len(plain["mse"]), "plain_ms": plain["ms"][-1], "learned_ms": learned["ms"][-1],
            "learned_iters_to_plain_final_mse": None if reach is None else reach + 1,
            "learned_ms_to_plain_final_mse": None if reach is None else learned["ms"][reach]}


def compare(est: Estimator, net: Network, w, batches, truth: torch.Tensor, margin: float = 0.0, set_id: int = 0):
    """Plain run and learned run (proposal before the first iteration) of one scene."""
    plain = _run(est, set_id, w, batches, truth)
    learned = _run(est, set_id, w, batches, truth, net, margin)
    out = summarize(plain, learned)
    out["plain"], out["learned"] = plain, learned
    return out


def choose_margin(est: Estimator, net: Network, scenes, margins, set_id: int = 0):
    """The margin whose learned runs reach the plain runs' final MSE in the fewest iterations on the
    validation scenes ((workload, batches, truth) each), averaged over the scenes with a miss
    counted as one iteration past the end (a deterministic criterion: timings would make the choice
    vary from run to run); ties go to the lowest mean final MSE."""
    plains = [_run(est, set_id, w, b, t) for w, b, t in scenes]
    best, key_best, runs = None, None, {}
    for m in margins:
        ss = [summarize(p, _run(est, set_id, w, b, t, net, m)) for p, (w, b, t) in zip(plains, scenes)]
        runs[m] = ss
        its = [s["learned_iters_to_plain_final_mse"] or (s["iterations"] + 1) for s in ss]
        key = (float(np.mean(its)), float(np.mean([s["learned_final_mse"] for s in ss])))
        if key_best is None or key < key_best:
            best, key_best = m, key
    return best, runs


def truth_box(w) -> torch.Tensor:
    """Analytic radiance of a box-scene workload's hit points (direct light, f_r = 1/pi), 3 x H."""
    scn = w.info["scene"]
    L = scn.irradiance(w.kernels.pos, w.kernels.nrm) / math.pi
    return torch.from_numpy(np.repeat(L[None, :], 3, 0).astype(np.float32)).cuda()


def he_init(seed: int) -> np.ndarray:
    """He-normal weights and zero biases in the parameter order W1, b1, W2, b2, w3, b3 (float32)."""
    rng = np.random.Generator(np.random.Philox(np.random.SeedSequence(seed)))
    parts = [rng.normal(0, math.sqrt(2.0 / N_IN), (N_IN, 64)).ravel(), np.zeros(64),
             rng.normal(0, math.sqrt(2.0 / 64), (64, 64)).ravel(), np.zeros(64),
             rng.normal(0, math.sqrt(1.0 / 64), 64), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def experiment(est: Estimator, make_scene, train_seeds, val_seeds, test_seeds,
               margins=(0.5, 1.0, 1.5, 2.0, 2.5, 3.0),
               epoch_blocks: int = 4, epochs_per_block: int = 3, batch: int = 8192, lr: float = 2e-3,
               init_seed: int = 1, log=None):
    """Trains a network on plain runs of the training scenes (features at iterations 1, 2, 4, 8 ->
    log(r_final / r1)), picks the proposal margin on the validation scenes, and compares plain and
    learned runs of each held-out test scene at equal MSE. make_scene(seed) -> (workload, device
    batches). The top-level comparison fields are those of the first test scene; `scenes` lists
    every test scene and `summary` their mean and spread; `train_gpu_ms` is the GPU time of the
    training steps (gradient and Adam kernels), `features_gpu_ms` that of building the training rows
    (plain runs included)."""
    say = log or (lambda *a: None)
    seeds = [test_seeds] if isinstance(test_seeds, int) else list(test_seeds)
    X, Y = [], []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    feat_ms = 0.0
    for s in train_seeds:
        sc = make_scene(s)
        e0.record()
        x, y = training_set(est, [sc])
        e1.record()
        torch.cuda.synchronize()
        feat_ms += e0.elapsed_time(e1)
        X.append(x)
        Y.append(y)
        del sc
        say(f"training scene {s}: {x.shape[0]} rows")
    X, Y = torch.cat(X).contiguous(), torch.cat(Y).contiguous()
    net = Network(est, he_init(init_seed))
    e0.record()
    steps = 0
    for b in range(epoch_blocks):
        f = 0.4 ** b
        steps += net.train(X, Y, epochs=epochs_per_block, batch=min(batch, X.shape[0]), lr=lr * f, seed=b,
                           lr_final=0.5 * lr * f)
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    _, sq = net.grad(X, Y)
    rows = int(X.shape[0])
    train_mse, label_var = sq / rows, float(Y.var())
    say(f"trained: mse {train_mse:.4f} against label variance {label_var:.4f} ({steps} steps, {train_ms:.1f} ms)")
    del X, Y
    vseeds = [val_seeds] if isinstance(val_seeds, int) else list(val_seeds)
    vals = []
    for sd in vseeds:
        wv, bv = make_scene(sd)
        vals.append((wv, bv, truth_box(wv)))
    margin, val = choose_margin(est, net, vals, margins)
    del vals
    say(f"margin {margin} chosen on scenes {vseeds}")
    scenes = []
    for s in seeds:
        wt, bt = make_scene(s)
        r = compare(est, net, wt, bt, truth_box(wt), margin=margin)
        del bt
        t = r["learned_ms_to_plain_final_mse"]
        r["speedup_to_plain_final_mse"] = (r["plain_ms"] / t) if t else None
        r["seed"] = s
        scenes.append(r)
        say(f"scene {s}: plain final MSE {r['plain_final_mse']:.3e}, learned reaches it at iteration "
            f"{r['learned_iters_to_plain_final_mse']} ({r['speedup_to_plain_final_mse']})")
    out = dict(scenes[0])
    out.update(margin=margin, train_mse=train_mse, label_var=label_var, train_rows=rows, train_steps=steps,
               train_gpu_ms=train_ms, features_gpu_ms=feat_ms)
    out["validation"] = {str(m): [{k: v for k, v in r.items()} for r in rs] for m, rs in val.items()}
    out["scenes"] = scenes
    sp = [r["speedup_to_plain_final_mse"] for r in scenes if r["speedup_to_plain_final_mse"]]
    its = [r["learned_iters_to_plain_final_mse"] for r in scenes if r["learned_iters_to_plain_final_mse"]]
    out["summary"] = {
        "test_scenes": len(scenes), "reached": len(sp),
        "speedup_mean": float(np.mean(sp)) if sp else None, "speedup_min": float(min(sp)) if sp else None,
        "speedup_max": float(max(sp)) if sp else None, "speedup_std": float(np.std(sp)) if sp else None,
        "iterations_mean": float(np.mean(its)) if its else None,
        "iterations_min": int(min(its)) if its else None, "iterations_max": int(max(its)) if its else None,
    }
    return out
