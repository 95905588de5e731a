"""Throughput of the hypothesis-tested progressive kernel estimator on one MI355X.

A step is one full iteration of the hot path (grid build, gather, grouped sums, F-test, radius and
estimate update) over one batch of light vertices per hit-point set. The headline workload is the
largest one: 16 independent planar hit-point sets of uneven size (64^2 to 1024^2 hit points, 0.5M to
8M light paths each per iteration; 2.57M hit points and 41.6M light paths per iteration in all), one
batched call per iteration. Two more workloads are measured the same way and reported beside it: the
box scene (512 x 512 hit points with normals, 2M light paths from a point light with a spherical
occluder) and vertex merging at scale (1920 x 1080 camera vertices, 4M light vertices with MIS
partials). Inputs are generated on the host by spawned worker processes (nothing is forked from a
process that holds the GPU), uploaded, and resident in HBM before any timed region starts.

Every workload: W untimed warm-up iterations, the autotuner on the warmed state, then R repeats of
exactly K timed iterations, each from a fresh state; the median repeat is reported. HIP events on
the library's own stream time the phases; the dominant kernel (the fused gather / test / update)
gets a roofline. Prints one JSON line: value = queries/s of the headline workload (one query = one
hit point in one iteration).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Dominant-kernel VALU work model per launch (lane operations), the hot-path measurement model:
# 150 per hit point (load state, F in float64, update), 35 per in-disk pair (map, group, group
# sums), 8 per candidate with 2.9 candidates per in-disk pair (uniform grid with cell = r).
OPS_PER_QUERY = 150.0
OPS_PER_PAIR = 35.0 + 8.0 * 2.9
# Vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit op per lane per clock
# (packed-FP32 and FMA doubling excluded; this build disables packed FP32).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published
# Algorithmic bytes the gather / test / update must move per launch: every stored light vertex's
# payload read once (P_b bytes) and every hit point's geometry read (G_h) and statistics read and
# written once (2 x 232 bytes: twelve float64 (S, Q) pairs, the estimate pair, radius, counts).
STATE_RW = 2 * 232
WORKLOADS = {
    "sets": dict(P_b=24, G_h=12),       # planar sets: position + flux; position
    "box": dict(P_b=36, G_h=24),        # box: position + normal + flux; position + normal
    "merge": dict(P_b=48, G_h=48),      # merging: position + normal + throughput + partials; + camera
}


def profiled_traffic(workload, kname, tuning):
    """HBM bytes per launch of the gather kernel from the committed rocprofv3 summary (one record per
    workload, kernel instance and tuning), or None when the kernel sources changed since the counters
    were taken (their hash is recorded there) or no record matches."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "gather_traffic.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in ["hk_gather.hip", "hk_internal.h", "hk_kernels.h", "hk_fquant.h"]:
        h.update(open(os.path.join(ROOT, "paper_2504_04411_amd", "csrc", f), "rb").read())
    want = [round(float(tuning[k]), 4) for k in ("cell_scale", "heavy_cost", "lanes_light", "lanes_heavy")]
    for m in re.finditer(r'^(\{"kernel": "gather_update_kernel".*\})$', open(path).read(), flags=re.M):
        rec = json.loads(m.group(1))
        if (h.hexdigest()[:16] == rec["source_sha256_16"] and rec.get("instance") == kname
                and rec.get("workload") == workload
                and [round(float(x), 4) for x in rec.get("tuning", [])] == want):
            return rec["traffic_bytes_per_launch"]
    return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ------------------------------------------------------------------------------------------------
# workloads: hit-point sets and the batch descriptions the worker processes turn into light vertices
# ------------------------------------------------------------------------------------------------

def describe(name, args):
    """(workloads, batch specs per iteration, label) of a named workload."""
    from workloads import generators as G
    n = max(args.steps, args.warmup)
    if name == "sets":
        meta = G.config2_sets(2)
        ws = G.config2(seed=2)
        specs = [[("sets", 2, s, it, J, e, c) for s, (_, J, e, c) in enumerate(meta)] for it in range(n)]
        H = sum(w.kernels.n for w in ws)
        label = (f"16 planar hit-point sets of uneven size (config 2, seed 2): {H} hit points and "
                 f"{sum(m[1] for m in meta)} light paths per iteration in all, one batched call per iteration")
    elif name == "box":
        ws = [G.config1(seed=args.seed, res=args.res, J=args.photons)]
        specs = [[("box", args.seed, it, args.photons, args.res)] for it in range(n)]
        label = (f"box scene (config 1): {args.res}x{args.res} hit points with normals, {args.photons} light "
                 f"paths per iteration, point light and sphere occluder")
    elif name == "merge":
        ws = [G.config4(seed=4)]
        specs = [[("merge", 4, it, 4_000_000)] for it in range(n)]
        label = ("vertex merging at scale (config 4): 1920x1080 camera vertices, 4M light vertices per iteration "
                 "with throughput and MIS partials")
    else:
        raise ValueError(name)
    return ws, specs, label


def upload_batches(pool, specs):
    from paper_2504_04411_amd.estimator import DevicePhotons
    from workloads import generators as G
    flat = [s for it in specs for s in it]
    gen = pool.map(G.batch, flat)
    out = []
    for it in specs:
        out.append([DevicePhotons.upload(next(gen)) for _ in it])
    return out


def run_leg(name, args, pool):
    """Warm-up, autotune and R timed repeats of K iterations of one workload on the GPU."""
    import torch
    from paper_2504_04411_amd.estimator import Estimator
    ws, specs, label = describe(name, args)
    K, W, R = args.steps, args.warmup, args.repeats
    t0 = time.perf_counter()
    batches = upload_batches(pool, specs)
    torch.cuda.synchronize()
    print(f"# {name}: generated and uploaded {len(batches)} iterations of batches in "
          f"{time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    p = ws[0].params
    est = Estimator(p.r1, mode=p.mode, k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin)
    ids = list(range(len(ws)))
    H = sum(w.kernels.n for w in ws)

    def reset():
        for s, w in enumerate(ws):
            ks = w.kernels
            est.set_kernels(s, ks.pos, ks.nrm, None, ks.cam_beta, ks.cam_mis, r1=w.params.r1, rmin=w.params.rmin)

    reset()
    est._workspace(max(est.workspace_for(b, ids) for b in batches))
    fixed = args.tuning is not None
    if fixed:                       # a pinned setting (profiling runs) applies to the warm-up too
        cs, hc, ll, lh = args.tuning.split(",")
        est.set_tuning(float(cs), int(hc), int(ll), int(lh))
    n_pre = W if (args.no_autotune or fixed) else max(W, min(args.tune_at, K) if args.tune_at >= 0 else K // 2)
    for i in range(n_pre):
        est.iterate(ids, batches[i % len(batches)])
    torch.cuda.synchronize()
    tuning = est.tuning()
    if not (args.no_autotune or fixed):
        tuning = est.autotune(ids, batches[n_pre % len(batches)])
        print(f"# {name}: autotuned {tuning}", file=sys.stderr, flush=True)
    reps = []
    for r in range(R):
        reset()
        torch.cuda.synchronize()
        est.profile(True)
        t0 = time.perf_counter()
        for i in range(K):
            est.iterate(ids, batches[i])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = est.profile_read()
        est.profile(False)
        st = [est.stats(s) for s in ids]
        reps.append(dict(dt=dt, prof=prof, pairs=sum(x["pairs"] for x in st), cand=sum(x["candidates"] for x in st),
                         pairs_set=[x["pairs"] for x in st]))
    order = sorted(range(R), key=lambda i: reps[i]["dt"])
    med = reps[order[R // 2]]
    radii = np.concatenate([est.radii(s).cpu().numpy() for s in ids])
    r1s = np.concatenate([np.full(w.kernels.n, np.float32(w.params.r1)) for w in ws])
    prof = med["prof"]
    gather_s = prof["gather_ms"] / 1e3
    launch_ms = prof["gather_ms"] / max(prof["launches"], 1)
    ops = OPS_PER_QUERY * H * K + OPS_PER_PAIR * med["pairs"]
    alu = ops / gather_s / 1e12
    J = sum(b.J for b in batches[0])
    wl = WORKLOADS[name]
    # the iteration's algorithmic bytes, shared by its gather launches (one per batch of sets)
    per_it = max(prof["launches"], 1) / K
    bytes_launch = (J * wl["P_b"] + H * (wl["G_h"] + STATE_RW)) / per_it
    gbps = bytes_launch / (launch_ms * 1e-3) / 1e9 if launch_ms > 0 else 0.0
    nrm = ws[0].kernels.nrm is not None
    vcm = p.mode == "vcm"
    kname = (f"gather_update_kernel<{str(nrm).lower()},{str(vcm).lower()},1,{tuning['lanes_light']},"
             f"{tuning['lanes_heavy']}>")
    traffic = profiled_traffic(name, kname, tuning)
    alu_roof = {"bound": "alu", "achieved": round(alu, 3), "peak": round(VALU_PEAK_TOPS, 2), "unit": "TOP/s",
                "frac": round(alu / VALU_PEAK_TOPS, 4),
                "work_model": "150 ops/query + 58.2 ops/in-disk pair (VALU lane ops)"}
    hbm_roof = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(gbps / HBM_PEAK_GBPS, 4),
                "work_model": f"{wl['P_b']} B per light vertex + ({wl['G_h']} + {STATE_RW}) B per hit point per launch",
                "algorithmic_bytes_per_launch": int(bytes_launch)}
    # the two gather launches of a batch of several sets, each with its own sets' work: the first runs
    # beside the second phase's grid builds, the second alone
    phase_of = est.gather_phases(ids, batches[0])
    by_phase = []
    for ph_i in (0, 1):
        n_l = prof["launches_phase"][ph_i]
        if n_l == 0 or prof["launches_phase"][1] == 0:
            continue
        sel = [s for s in ids if phase_of[s] == ph_i]
        h_p = sum(ws[s].kernels.n for s in sel)
        ops_p = OPS_PER_QUERY * h_p * K + OPS_PER_PAIR * sum(med["pairs_set"][s] for s in sel)
        t_p = prof["gather_ms_phase"][ph_i] / 1e3
        by_phase.append({"phase": ph_i + 1, "sets": len(sel), "hit_points": h_p, "launches": n_l,
                         "avg_launch_ms": round(prof["gather_ms_phase"][ph_i] / n_l, 4),
                         "alu_achieved": round(ops_p / t_p / 1e12, 3),
                         "alu_frac": round(ops_p / t_p / 1e12 / VALU_PEAK_TOPS, 4),
                         "runs_beside": "the second phase's grid builds" if ph_i == 0 else "nothing"})
    out = {
        "workload": label, "hit_points": H, "light_paths_per_iteration": int(J), "iterations": K,
        "queries_per_s": round(H * K / med["dt"], 1), "ms_per_step": round(med["dt"] / K * 1e3, 4),
        "repeats_ms_per_step": [round(x["dt"] / K * 1e3, 4) for x in reps],
        "gather_test_update_queries_per_s": round(H * K / gather_s, 1),
        "phase_ms_per_step": {"plan_and_grid": round(prof["grid_ms"] / K, 4),
                              "fcrit_wait": round(prof["fcrit_wait_ms"] / K, 4),
                              "work_list": round(prof["list_ms"] / K, 4),
                              "gather_test_update": round(prof["gather_ms"] / K, 4),
                              "tally": round(prof["tally_ms"] / K, 4)},
        "tuning": dict(tuning, autotuned=not (args.no_autotune or fixed)),
        "pairs_per_query": round(med["pairs"] / (H * K), 2),
        "candidates_per_pair": round(med["cand"] / max(med["pairs"], 1), 3),
        "final_radius": {"mean_over_r1": float((radii / r1s).mean()), "shrunk_frac": float((radii < r1s).mean())},
        "dominant_kernel": {"kernel": kname, "avg_launch_ms": round(launch_ms, 4), "launches": int(prof["launches"])},
        "alu_roofline": alu_roof, "hbm_roofline": hbm_roof, "traffic": traffic,
    }
    if by_phase:
        out["gather_launches_by_phase"] = by_phase
    est.close()
    del batches
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out, ws, specs


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes, timed with HIP events on the current stream: the achievable
    read + write rate beside the published peak."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    del src, dst
    torch.cuda.empty_cache()
    t = statistics.median(ts)
    return {"bytes": nbytes, "gbps_read_plus_write": round(2 * nbytes / t / 1e9, 1),
            "frac_of_published": round(2 * nbytes / t / 1e9 / HBM_PEAK_GBPS, 4)}


def learned_vs_plain(args, pool):
    """The learned radius proposal against the plain method at equal MSE on jittered box scenes:
    trained on seeds 30-33, margin picked on seeds 34 and 35, compared on the held-out seeds 39-43."""
    import torch
    from paper_2504_04411_amd import learned as Lr
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    from workloads import generators as G
    res, J, n = args.res, args.photons, 64

    def make_scene(seed):
        w = G.config3(seed, res=res, J=J, n_iter=n)
        out = [DevicePhotons.upload(b) for b in pool.map(G.batch, [("jittered", seed, i, J, res) for i in range(n)])]
        return w, out

    p = G.config3(30, res=8, J=1000).params
    est = Estimator(p.r1, k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin)
    out = Lr.experiment(est, make_scene, (30, 31, 32, 33), (34, 35), tuple(range(39, 39 + args.learned_scenes)),
                        log=lambda m: print("# learned: " + m, file=sys.stderr, flush=True))
    est.close()
    torch.cuda.synchronize()
    keep = {k: out[k] for k in ("margin", "train_mse", "label_var", "train_rows", "train_steps", "train_gpu_ms",
                                "features_gpu_ms", "summary")}
    keep["scenes"] = [{k: r[k] for k in ("seed", "plain_final_mse", "learned_final_mse", "plain_ms",
                                         "learned_iters_to_plain_final_mse", "learned_ms_to_plain_final_mse",
                                         "speedup_to_plain_final_mse")} for r in out["scenes"]]
    keep["workload"] = (f"box scenes with jittered light and occluder, {res}x{res} hit points, {J} light paths per "
                        f"iteration, {n} iterations; trained on seeds 30-33, margin from seeds 34-35, compared on seeds "
                        f"39-{38 + args.learned_scenes}; MSE of the radiance against the analytic direct light")
    return keep


def generated_end_to_end(args, tuning):
    """The box workload with its light vertices generated on the device: every iteration is one
    replay of a graph that writes the batch (hk_emit_box) and runs the estimator on it. The
    generation kernel alone is timed with HIP events on the stream it runs on; it writes 36 bytes
    per slot (position, normal, flux) and reads nothing but its arguments."""
    import torch
    from paper_2504_04411_amd import hk
    from paper_2504_04411_amd.estimator import DevicePhotons, Estimator
    from workloads import generators as G
    w = G.config1(seed=args.seed, res=args.res, J=args.photons)
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
    ones = np.ones((3, H), np.float32)
    zeros = np.zeros((3, H), np.float32)
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


def batched_vs_per_set(args, ws, specs, pool, tuning):
    """The headline sets run as one batched call per iteration against one call per set, and a
    captured graph of one batched iteration replayed against the same iteration run eagerly."""
    import torch
    from paper_2504_04411_amd.estimator import Estimator
    n_it = min(args.steps, 8)
    batches = upload_batches(pool, specs[:n_it])
    p = ws[0].params
    est = Estimator(p.r1, k=p.k, alpha_f=p.alpha_f, alpha=p.alpha, rmin=p.rmin)
    est.set_tuning(tuning["cell_scale"], tuning["heavy_cost"], tuning["lanes_light"], tuning["lanes_heavy"])
    ids = list(range(len(ws)))
    H = sum(w.kernels.n for w in ws)

    def reset():
        for s, w in enumerate(ws):
            est.set_kernels(s, w.kernels.pos, None, r1=w.params.r1, rmin=w.params.rmin)
        est._workspace(max(est.workspace_for(b, ids) for b in batches))
        torch.cuda.synchronize()

    def timed(fn):
        reset()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    out = {"iterations": n_it}
    out["batched_queries_per_s"] = round(H * n_it / timed(lambda: [est.iterate(ids, batches[i]) for i in range(n_it)]), 1)
    out["one_call_per_set_queries_per_s"] = round(
        H * n_it / timed(lambda: [est.iterate([s], [batches[i][s]]) for i in range(n_it) for s in ids]), 1)
    out["eager_repeated_batch_queries_per_s"] = round(
        H * n_it / timed(lambda: [est.iterate(ids, batches[0]) for _ in range(n_it)]), 1)
    reset()
    g = est.capture(ids, batches[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_it):
        g.launch()
    torch.cuda.synchronize()
    out["graph_repeated_batch_queries_per_s"] = round(H * n_it / (time.perf_counter() - t0), 1)
    g.close()
    est.close()
    del batches
    torch.cuda.empty_cache()
    return out


def cpu_baseline(args, pool, ws, specs):
    """The oracle as it stands (grid mode, OpenMP over hit points) on a sample of the headline
    workload: every `stride`-th hit point of every set for the first `iters` iterations. The oracle
    builds each set's grid over all of the set's light vertices whatever the sample, so the sample is
    charged its share of that build (the build time of a one-hit-point gather, times the sampled
    fraction) plus its own gather and update. Returns queries/s on `threads` threads."""
    from oracle import oracle as O
    from workloads import generators as G
    iters = args.cpu_iters

    def run(threads, stride, n_it):
        subs = []
        for w in ws:
            idx = np.arange(0, w.kernels.n, stride)
            subs.append((w, w.kernels.subset(idx), w.kernels.subset(np.array([0])), idx.size / w.kernels.n))
        states = [O.init_state(ks.n, w.params.r1) for w, ks, _, _ in subs]
        ones = [O.init_state(1, w.params.r1) for w, _, _, _ in subs]
        flat = [s for it in specs[:n_it] for s in it]
        gen = pool.map(G.batch, flat)
        t_sample = t_grid_share = t_update = 0.0
        for it in range(n_it):
            for s, (w, ks, k1, frac) in enumerate(subs):
                ph = next(gen)
                O.f_critical(np.array([ph.J * (t + 1) for t in range(it + 1)], float), w.params.alpha_f)
                t0 = time.perf_counter()
                g = O.gather(ks, ph, states[s].r, use_grid=True, nthreads=threads)
                t1 = time.perf_counter()
                O.gather(k1, ph, ones[s].r, use_grid=True, nthreads=threads)
                t2 = time.perf_counter()
                O.iterate(w.params, ks, states[s], ph, gathered=g)
                t3 = time.perf_counter()
                t_sample += t1 - t0
                t_grid_share += (t2 - t1) * (1.0 - frac)
                t_update += t3 - t2
        nq = sum(ks.n for _, ks, _, _ in subs) * n_it
        charged = max(t_sample - t_grid_share, 1e-9) + t_update
        return nq / charged, charged, nq

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    q, secs, nq = run(threads, args.cpu_stride, iters)
    q1, secs1, nq1 = run(1, args.cpu_stride * 8, 1)
    return {"value": round(q, 1), "unit": "queries/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"oracle grid mode on one hit point in {args.cpu_stride} of each of the 16 sets ({nq // iters} "
                      f"hit points) for the first {iters} iterations of the same inputs, {secs:.1f}s charged "
                      f"(the sample's share of each set's grid build, its gather and its update)",
            "one_core": {"value": round(q1, 1), "sample": f"one hit point in {args.cpu_stride * 8}, first iteration "
                                                          f"({nq1} queries), {secs1:.1f}s charged"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed iterations per repeat (K)")
    ap.add_argument("--warmup", type=int, default=5, help="untimed iterations before the autotuner (W)")
    ap.add_argument("--repeats", type=int, default=5, help="timed repeats per workload; the median is reported")
    ap.add_argument("--photons", type=int, default=2_000_000, help="box scene: light paths per iteration")
    ap.add_argument("--res", type=int, default=512, help="box scene: hit points per side")
    ap.add_argument("--seed", type=int, default=1, help="box scene seed")
    ap.add_argument("--only", choices=["sets", "box", "merge"], default=None,
                    help="measure one workload only (profiling runs); it becomes the printed value")
    ap.add_argument("--cpu-stride", type=int, default=16)
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--learned-scenes", type=int, default=5, help="held-out scenes of the learned comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal comparison")
    ap.add_argument("--no-generated", action="store_true", help="skip the device-generated box run")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tuning")
    ap.add_argument("--tuning", default=None, metavar="CELL,HEAVY,LANES_LIGHT,LANES_HEAVY",
                    help="fixed tuning instead of the autotuner (profiling runs pin the autotuned setting)")
    ap.add_argument("--tune-at", type=int, default=-1,
                    help="untimed iterations before the autotuner samples the state (default: K / 2, the middle "
                         "of the timed run; at least W)")
    ap.add_argument("--workers", type=int, default=15,
                    help="batch-generating worker processes (<= 15; 0: generate in this process, as profiled "
                         "runs do, where every child process would load the profiler too)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the legs, copy a MIB-sized device buffer once (reference for HBM traffic "
                         "counters: it reads and writes exactly MIB MiB)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is described but "
              "not built", file=sys.stderr)
        sys.exit(2)

    # the batch generators run in spawned processes, started before anything touches the GPU
    from workloads import generators as G
    pool = G.spawn_pool(min(args.workers, 15))

    import torch
    from paper_2504_04411_amd import hk
    hk.lib()
    torch.cuda.set_device(0)
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    head = args.only or "sets"
    legs = [head] if args.only else ["sets", "box", "merge"]
    res = {}
    for name in legs:
        res[name] = run_leg(name, args, pool)
    main_out, ws, specs = res[head]
    dom = main_out["dominant_kernel"]
    roof = dict(main_out["alu_roofline"] if head != "merge" else main_out["hbm_roofline"])
    roof.update(traffic=main_out["traffic"], kernel=dom["kernel"], avg_launch_ms=dom["avg_launch_ms"])
    out = {
        "metric": "photon-kernel queries/sec (gather+F-test+update) at 1 GPU",
        "value": main_out["queries_per_s"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_out["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": main_out["workload"], "hit_points": main_out["hit_points"],
                   "light_paths_per_iteration": main_out["light_paths_per_iteration"], "iterations": args.steps,
                   "repeats": args.repeats, "statistic": "median of the repeats"},
        "roofline": roof,
        head: {k: v for k, v in main_out.items() if k not in ("workload",)},
    }
    for name in legs:
        if name != head:
            out[name] = res[name][0]
    out["copy_bandwidth"] = copy_bandwidth()
    if not args.only:
        out["sets"]["batched_vs_per_set"] = batched_vs_per_set(args, ws, specs, pool, res["sets"][0]["tuning"])
        if not args.no_generated:
            out["generated_end_to_end"] = generated_end_to_end(args, res["box"][0]["tuning"])
        if not args.no_learned:
            out["learned_vs_plain"] = learned_vs_plain(args, pool)
    if not args.no_cpu_baseline and head == "sets":
        out["cpu_baseline"] = cpu_baseline(args, pool, ws, specs)
    pool.shutdown()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
