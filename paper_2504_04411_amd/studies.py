"""Parameter studies on the box scene: MSE of the progressive estimate against the analytic direct
light as the shrink ratio k, the significance level alpha_F and the initial radius r1 vary (the
paper's studies of k, of the significance level and of the initial radius, here on a synthetic
scene with a known answer).

Every run goes through the library (one estimator context per setting); this module only sequences
the runs and computes the error metric.

    python -m paper_2504_04411_amd.studies [--res 512] [--photons 2000000] [--iters 64]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SETTINGS = {
    "k": [0.5, 0.6, 0.7, 0.8, 0.9],
    "alpha_f": [0.01, 0.05, 0.1, 0.2],
    "r1": [0.025, 0.05, 0.1],
}
DEFAULTS = dict(k=0.7, alpha_f=0.05, r1=0.05)


def _gen(args):
    seed, it, res, J = args
    from workloads import generators as G
    return it, G.config1(seed=seed, res=res, J=J).photons(it)


def run(res: int = 512, J: int = 2_000_000, iters: int = 64, seed: int = 1, workers: int = 16, log=None,
        settings=None):
    """One estimator run per setting (each parameter varied alone around DEFAULTS) on the same
    photon batches; MSE of the radiance against the analytic truth at iterations 8, 16, 32 (those
    below `iters`) and at the last one."""
    from workloads import generators as G
    say = log or (lambda *a: None)
    settings = SETTINGS if settings is None else settings
    w = G.config1(seed=seed, res=res, J=J)
    # the host batches are generated before this function touches the GPU; pass workers=1 from a
    # process that already holds a device context, so that nothing is forked from it
    host = [None] * iters
    jobs = [(seed, i, res, J) for i in range(iters)]
    if workers <= 1:
        for it, b in map(_gen, jobs):
            host[it] = b
    else:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            for it, b in ex.map(_gen, jobs):
                host[it] = b
    import torch
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    batches = [DevicePhotons.upload(b) for b in host]
    del host
    scene = w.info["scene"]
    truth_np = scene.irradiance(w.kernels.pos, w.kernels.nrm) / math.pi
    truth = torch.from_numpy(np.repeat(truth_np[None, :], 3, 0).astype(np.float32)).cuda()
    marks = [c for c in (8, 16, 32) if c < iters] + [iters]
    rows = []
    for name, values in settings.items():
        for v in values:
            prm = dict(DEFAULTS, **{name: v})
            r1 = prm["r1"]
            est = Estimator(r1, k=prm["k"], alpha_f=prm["alpha_f"], alpha=0.75, rmin=0.001 * r1)
            est.set_kernels(0, w.kernels.pos, w.kernels.nrm)
            est._workspace(max(est.workspace_for([b], [0]) for b in batches))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mse = {}
            for i, b in enumerate(batches, start=1):
                est.iterate([0], [b])
                if i in marks:
                    mse[i] = float(((est.radiance(0) - truth) ** 2).mean())
            torch.cuda.synchronize()
            r = est.radii(0)
            rows.append(dict(parameter=name, value=v, k=prm["k"], alpha_f=prm["alpha_f"], r1=r1,
                             mse={str(c): m for c, m in mse.items()}, mse_final=mse[iters],
                             radius_mean=float(r.mean()), radius_min=float(r.min()), radius_max=float(r.max()),
                             shrunk_frac=float((r < np.float32(r1)).float().mean()),
                             seconds=round(time.perf_counter() - t0, 3)))
            say(f"{name}={v}: final MSE {mse[iters]:.4e}, mean radius {rows[-1]['radius_mean']:.4f}")
            est.close()
    return dict(workload=f"box scene {res}x{res}, {J} light paths per iteration, {iters} iterations, seed {seed}; "
                         f"MSE of the radiance against the analytic direct light",
                defaults=DEFAULTS, marks=marks, rows=rows)


def markdown(result) -> str:
    marks = result["marks"]
    out = [f"Workload: {result['workload']}.", "",
           "| parameter | value | " + " | ".join(f"MSE @{c}" for c in marks) + " | mean radius |",
           "|---|---|" + "---|" * len(marks) + "---|"]
    for r in result["rows"]:
        out.append(f"| {r['parameter']} | {r['value']} | " + " | ".join(f"{r['mse'][str(c)]:.3e}" for c in marks)
                   + f" | {r['radius_mean']:.4f} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--res", type=int, default=512)
    ap.add_argument("--photons", type=int, default=2_000_000)
    ap.add_argument("--iters", type=int, default=64)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--json", default="")
    args = ap.parse_args()
    res = run(args.res, args.photons, args.iters, args.seed, log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    if args.json:
        with open(args.json, "w") as f:
            json.dump(res, f, indent=1)
    print(markdown(res), flush=True)


if __name__ == "__main__":
    main()
