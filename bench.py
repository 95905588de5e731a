"""Throughput of the hypothesis-tested progressive kernel estimator on one MI355X.

A step is one full iteration of the hot path (grid build, gather, grouped sums, F-test, radius and
estimate update) over one batch of light vertices. Default workload: the box scene, 512 x 512 hit
points on five faces of the unit box with per-point normals, 2M light sub-paths per iteration from a
point light with a spherical occluder, 64 iterations (the whole job is timed; warm-up iterations run
on a separate state first). Inputs are generated on the host, uploaded, and resident in HBM before
the timed region starts.

Prints one JSON line: value = queries/s (one query = one hit point in one iteration), with the
roofline of the dominant kernel (fused gather / test / update) and the CPU oracle timed on a bounded
sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Dominant-kernel work model per launch (VALU lane operations), from the hot-path measurement model:
# 150 per kernel (load state, F in float64, update), 35 per in-disk pair (map, group, compensated
# sums), 8 per candidate with 2.9 candidates per in-disk pair (uniform grid with cell = r).
OPS_PER_QUERY = 150.0
OPS_PER_PAIR = 35.0 + 8.0 * 2.9
# Vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit op per lane per clock
# (packed-FP32 and FMA doubling excluded; this build disables packed FP32).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published


def profiled_traffic(kname, tuning):
    """HBM bytes per launch of the gather kernel from the committed rocprofv3 summary (one record per
    tuning), or None when the kernel sources changed since the counters were taken (their hash is
    recorded there) or no record is of this instance of the kernel and this tuning."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "gather_update_box.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ["hk_gather.hip", "hk_internal.h", "hk_kernels.h", "hk_fquant.h"]:
        h.update(open(os.path.join(ROOT, "paper_2504_04411_amd", "csrc", f), "rb").read())
    want = [round(float(tuning[k]), 4) for k in ("cell_scale", "heavy_cost", "lanes_light", "lanes_heavy")]
    for m in re.finditer(r'^(\{"kernel": "gather_update_kernel".*\})$', open(path).read(), flags=re.M):
        rec = json.loads(m.group(1))
        if (h.hexdigest()[:16] == rec["source_sha256_16"] and rec.get("instance") == kname
                and [round(float(x), 4) for x in rec.get("tuning", [])] == want):
            return rec["traffic_bytes_per_launch"]
    return None


def _gen(args):
    seed, it, J = args
    from workloads import generators as G
    w = G.config1(seed=seed, J=J)
    b = w.photons(it)
    return it, b


def _gen3(args):
    seed, it, res, J, n = args
    from workloads import generators as G
    return it, G.config3(seed, res=res, J=J, n_iter=n).photons(it)


def learned_vs_plain(args, ex):
    """The learned radius proposal against the plain method at equal MSE on jittered box scenes:
    trained on seeds 30-33, margin picked on seed 34, compared on the held-out seed 39."""
    import torch
    from paper_2504_04411_amd import learned as Lr
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    from workloads import generators as G
    res, J, n = args.res, args.photons, 64

    def make_scene(seed):
        w = G.config3(seed, res=res, J=J, n_iter=n)
        out = [None] * n
        for it, b in ex.map(_gen3, [(seed, i, res, J, n) for i in range(n)]):
            out[it] = DevicePhotons.upload(b)
        return w, out

    p = G.config3(30, res=8, J=1000).params
    est = Estimator(p.r1, k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin)
    out = Lr.experiment(est, make_scene, (30, 31, 32, 33), 34, 39,
                        log=lambda m: print("# learned: " + m, file=sys.stderr, flush=True))
    est.close()
    torch.cuda.synchronize()
    keep = {k: out[k] for k in ("plain_final_mse", "learned_final_mse", "iterations", "plain_ms", "learned_ms",
                                "learned_iters_to_plain_final_mse", "learned_ms_to_plain_final_mse", "margin",
                                "train_mse", "label_var", "train_rows")}
    t = out["learned_ms_to_plain_final_mse"]
    keep["speedup_to_plain_final_mse"] = round(out["plain_ms"] / t, 3) if t else None
    keep["workload"] = (f"box scenes with jittered light and occluder, {res}x{res} hit points, {J} light paths per "
                        f"iteration, {n} iterations; trained on seeds 30-33, margin from seed 34, compared on seed 39; "
                        f"MSE of the radiance against the analytic direct light")
    return keep


def _gen2(args):
    s, it, J, edge, ca = args
    from workloads import generators as G
    return s, it, G.config2_photons(2, s, it, J, edge, ca)


def batched_sets(args, ex, n_iter=8):
    """Config 2 (16 independent planar sets of uneven size) through the batched launch: one
    hk_iterate call for all sets per iteration, against one call per set, and the batched iteration
    replayed from a captured graph against the same iteration run eagerly."""
    import torch
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    from workloads import generators as G
    meta = G.config2_sets(2)
    ws = G.config2(seed=2, n_iter=n_iter)
    n = len(ws)
    batches = [[None] * n for _ in range(n_iter)]
    jobs = [(s, it, J, edge, ca) for it in range(n_iter) for s, (_, J, edge, ca) in enumerate(meta)]
    for s, it, b in ex.map(_gen2, jobs):
        batches[it][s] = DevicePhotons.upload(b)
    p = ws[0].params
    est = Estimator(p.r1, k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin)
    ids = list(range(n))
    H = sum(w.kernels.n for w in ws)

    def reset():
        for s, w in enumerate(ws):
            est.set_kernels(s, w.kernels.pos, None, r1=w.params.r1, rmin=w.params.rmin)
        est._workspace(max(est.workspace_for(bb, ids) for bb in batches))
        torch.cuda.synchronize()

    def timed(fn):
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    reset()
    tuning = est.tuning()
    if not args.no_autotune:
        for it in range(2):
            est.iterate(ids, batches[it])
        tuning = est.autotune(ids, batches[2 % n_iter])
    out = {"workload": f"16 planar sets (config 2): {H} hit points and "
                       f"{sum(m[1] for m in meta)} light paths per iteration in all, {n_iter} iterations",
           "hit_points": H, "iterations": n_iter, "tuning": tuning}
    t = timed(lambda: [est.iterate(ids, batches[it]) for it in range(n_iter)])
    out["batched_queries_per_s"] = round(H * n_iter / t, 1)
    t = timed(lambda: [est.iterate([s], [batches[it][s]]) for it in range(n_iter) for s in ids])
    out["one_call_per_set_queries_per_s"] = round(H * n_iter / t, 1)
    t = timed(lambda: [est.iterate(ids, batches[0]) for _ in range(n_iter)])
    out["eager_repeated_batch_queries_per_s"] = round(H * n_iter / t, 1)
    reset()
    g = est.capture(ids, batches[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_iter):
        g.launch()
    torch.cuda.synchronize()
    out["graph_repeated_batch_queries_per_s"] = round(H * n_iter / (time.perf_counter() - t0), 1)
    g.close()
    est.close()
    return out


def generated_end_to_end(args, w, tuning):
    """The box workload with its light vertices generated on the device: every iteration is one
    replay of a graph that writes the batch (hk_emit_box) and runs the estimator on it. The
    generation kernel alone is timed with HIP events on the stream it runs on; it writes 36 bytes
    per slot (position, normal, flux) and reads nothing but its arguments."""
    import torch
    from paper_2504_04411_amd import hk
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    p = w.params
    sc = w.info["scene"]
    power = float(np.float32(4.0 * math.pi * sc.intensity))
    scene = hk.box_scene(sc.light, sc.sphere_c, sc.sphere_r, power)
    J, K, H = args.photons, args.steps, w.kernels.n
    est = Estimator(p.r1, k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin)
    est.set_tuning(tuning["cell_scale"], tuning["heavy_cost"], tuning["lanes_light"], tuning["lanes_heavy"])
    est.set_kernels(0, w.kernels.pos, w.kernels.nrm)
    mk = lambda: torch.empty((3, J), dtype=torch.float32, device="cuda")  # noqa: E731
    buf = DevicePhotons(J=J, pos=mk(), flux=mk(), nrm=mk())
    est._workspace(est.workspace_for([buf], [0]))
    est.emit_box(0, scene, args.seed, J, out=buf)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        est.emit_box(0, scene, args.seed, J, out=buf)
    e1.record()
    torch.cuda.synchronize()
    emit_ms = e0.elapsed_time(e1) / K
    g = est.capture_box([0], [scene], [args.seed], [buf])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        g.launch()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    truth = sc.irradiance(w.kernels.pos, w.kernels.nrm) / math.pi
    L = est.radiance(0).cpu().numpy()
    mse = float(((L - truth[None, :]) ** 2).mean())
    g.close()
    est.close()
    gbps = 36.0 * J / (emit_ms * 1e-3) / 1e9
    # vertex merging with the emission's partials, without and with the vertex connection to the
    # light (Eq. VCM-estimator), each one graph replay per iteration
    vcm = {}
    Hn = w.kernels.n
    ones = np.ones((3, Hn), np.float32)
    zeros = np.zeros((3, Hn), np.float32)
    for connect in (False, True):
        ev = Estimator(p.r1, mode="vcm", k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin)
        ev.set_tuning(tuning["cell_scale"], tuning["heavy_cost"], tuning["lanes_light"], tuning["lanes_heavy"])
        ev.set_kernels(0, w.kernels.pos, w.kernels.nrm, cam_beta=ones, cam_mis=zeros)
        vb = DevicePhotons(J=J, pos=mk(), flux=mk(), nrm=mk(), mis=mk())
        gv = ev.capture_box([0], [scene], [args.seed], [vb], connect=connect)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            gv.launch()
        torch.cuda.synchronize()
        dtv = time.perf_counter() - t0
        Lv = ev.radiance(0).cpu().numpy()
        vcm["merging_and_connection" if connect else "merging_only"] = {
            "queries_per_s": round(H * K / dtv, 1), "final_mse_vs_analytic": float(((Lv - truth[None, :]) ** 2).mean())}
        gv.close()
        ev.close()
    return {"workload": f"box scene, {args.res}x{args.res} hit points, {J} light sub-paths generated on the "
                        f"device per iteration (Philox4x32-10, seed {args.seed}), {K} iterations, one graph "
                        f"replay per iteration",
            "queries_per_s": round(H * K / dt, 1), "ms_per_iteration": round(dt / K * 1e3, 4),
            "final_mse_vs_analytic": mse,
            "vertex_merging": vcm,
            "emit": {"kernel": "emit_box_kernel", "avg_launch_ms": round(emit_ms, 4),
                     "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                  "frac": round(gbps / HBM_PEAK_GBPS, 4),
                                  "work_model": "36 bytes written per slot"}}}


def make_batches(seed, n, J, workers):
    out = [None] * n
    with ProcessPoolExecutor(max_workers=workers) as ex:
        for it, b in ex.map(_gen, [(seed, i, J) for i in range(n)]):
            out[it] = b
    return out


def cpu_baseline(w, batches, stride, nthreads):
    """The oracle as it stands (grid mode, OpenMP over kernels) on every `stride`-th kernel for all
    iterations; returns queries/s of that sample."""
    from oracle import oracle as O
    idx = np.arange(0, w.kernels.n, stride)
    ks = w.kernels.subset(idx)
    st = O.init_state(idx.size, w.params.r1)
    O.f_critical(np.array([b.J * (i + 1) for i, b in enumerate(batches)], float), w.params.alpha_f)  # warm cache
    t0 = time.perf_counter()
    for b in batches:
        O.iterate(w.params, ks, st, b, use_grid=True, nthreads=nthreads)
    dt = time.perf_counter() - t0
    return idx.size * len(batches) / dt, dt, idx.size


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--photons", type=int, default=2_000_000)
    ap.add_argument("--res", type=int, default=512)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-stride", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tuning")
    ap.add_argument("--tuning", default=None, metavar="CELL,HEAVY,LANES_LIGHT,LANES_HEAVY",
                    help="fixed tuning instead of the autotuner (profiling runs pin the autotuned setting)")
    ap.add_argument("--tune-at", type=int, default=32,
                    help="untimed iterations before the autotuner samples the state")
    ap.add_argument("--no-batched", action="store_true", help="skip the many-set (config 2) measurement")
    ap.add_argument("--no-generated", action="store_true",
                    help="skip the run with light vertices generated on the device")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the timed job, copy a MIB-sized device buffer once (reference for HBM "
                         "traffic counters: it reads and writes exactly MIB MiB)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is described but "
              "not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_04411_amd import hk
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    from workloads import generators as G

    hk.lib()
    torch.cuda.set_device(0)
    w = G.config1(seed=args.seed, res=args.res, J=args.photons)
    K, W = args.steps, args.warmup
    t0 = time.perf_counter()
    batches = make_batches(args.seed, max(K, W), args.photons, args.workers)
    print(f"# generated {len(batches)} batches in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = [DevicePhotons.upload(b) for b in batches]
    torch.cuda.synchronize()

    p = w.params
    est = Estimator(p.r1, k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin)
    est.set_kernels(0, w.kernels.pos, w.kernels.nrm)
    # untimed warm-up; the autotuner samples the state after `tune_at` iterations (the middle of the
    # timed run: at iteration 16 it preferred cells of 1.0 r, 2% slower than 0.7 r over 64 iterations),
    # then the timed run restarts from a fresh state
    fixed = args.tuning is not None
    n_pre = W if (args.no_autotune or fixed) else max(W, args.tune_at)
    for i in range(n_pre):
        est.iterate([0], [dev[i % len(dev)]])
    torch.cuda.synchronize()
    if fixed:
        cs, hc, ll, lh = args.tuning.split(",")
        est.set_tuning(float(cs), int(hc), int(ll), int(lh))
    tuning = est.tuning()
    if not (args.no_autotune or fixed):
        # settings timed on scratch copies of the warmed-up state with the next batch
        tuning = est.autotune([0], [dev[n_pre % len(dev)]])
        print(f"# autotuned: {tuning}", file=sys.stderr, flush=True)
    est.set_kernels(0, w.kernels.pos, w.kernels.nrm)         # fresh state for the timed job
    est._workspace(max(est.workspace_for([d], [0]) for d in dev))
    torch.cuda.synchronize()
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    est.profile(True)
    t0 = time.perf_counter()
    for i in range(K):
        est.iterate([0], [dev[i]])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = est.profile_read()
    stats = est.stats(0)
    radii = est.radii(0).cpu().numpy()
    H = w.kernels.n
    value = H * K / dt
    gather_s = prof["gather_ms"] / 1e3
    launch_ms = prof["gather_ms"] / max(prof["launches"], 1)
    ops = OPS_PER_QUERY * H * K + OPS_PER_PAIR * stats["pairs"]
    achieved = ops / gather_s / 1e12
    kname = f"gather_update_kernel<true,false,1,{tuning['lanes_light']},{tuning['lanes_heavy']}>"
    roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
            "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": profiled_traffic(kname, tuning),
            "kernel": kname, "avg_launch_ms": round(launch_ms, 4),
            "work_model": "150 ops/query + 58.2 ops/in-disk pair (VALU lane ops)"}
    out = {
        "metric": "photon-kernel queries/sec (gather+F-test+update) at 1 GPU",
        "value": round(value, 1), "unit": "queries/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(dt / K * 1e3, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"box scene, {args.res}x{args.res} hit points with normals, {args.photons} photons "
                               f"per iteration, point light and sphere occluder, {K} iterations",
                   "H": H, "J": args.photons, "iterations": K, "seed": args.seed},
        "gather_test_update_queries_per_s": round(H * K / gather_s, 1),
        "phase_ms_total": {"plan_and_grid": round(prof["grid_ms"], 3), "fcrit_wait": round(prof["fcrit_wait_ms"], 3),
                           "work_list": round(prof["list_ms"], 3), "gather_test_update": round(prof["gather_ms"], 3),
                           "tally": round(prof["tally_ms"], 3)},
        "tuning": dict(tuning, autotuned=not (args.no_autotune or fixed)),
        "pairs_per_query": round(stats["pairs"] / (H * K), 2),
        "candidates_per_pair": round(stats["candidates"] / max(stats["pairs"], 1), 3),
        "final_radius": {"mean": float(radii.mean()), "min": float(radii.min()),
                         "shrunk_frac": float((radii < np.float32(p.r1)).mean())},
        "roofline": roof,
    }
    if not args.no_generated:
        out["generated_end_to_end"] = generated_end_to_end(args, w, tuning)
    if not args.no_batched:
        with ProcessPoolExecutor(max_workers=args.workers) as ex:
            out["batched_sets"] = batched_sets(args, ex)
    if not args.no_learned:
        with ProcessPoolExecutor(max_workers=args.workers) as ex:
            out["learned_vs_plain"] = learned_vs_plain(args, ex)
    if not args.no_cpu_baseline:
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        q, secs, nk = cpu_baseline(w, batches[:K], args.cpu_stride, nthreads)
        out["cpu_baseline"] = {"value": round(q, 1), "unit": "queries/s", "cores": nthreads, "kind": "oracle",
                               "sample": f"oracle grid mode on every {args.cpu_stride}th hit point ({nk} kernels) "
                                         f"for all {K} iterations of the same inputs, {secs:.1f}s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
