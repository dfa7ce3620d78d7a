"""Benchmark of the short-range TreePM gravity hot path on one MI355X.

Workload: 64^3 = 262,144 equal-mass particles, 70% in 200 Plummer spheres on a
uniform background, PM mesh 128^3 (r_s = 1.25/128, r_cut = 4.5 r_s),
eps = 1/1920, Barnes-Hut theta = 0.5 (synthetic, seeded).

One step = tree build (keys, radix sort, octree, moments) + FP32 forward walk
+ FP32 adjoint walk and push-down, i.e. a differentiated force evaluation.
`value` = forward short-range interactions per second of whole step time.
Outside the timed region the same run measures the FP64 walk, the FP32 force
error against the FP64 oracle on a sample of targets, and the oracle itself on
the host (cpu_baseline).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "short-range interactions/s, FP32 vs FP64 at stated force error; fwd+adjoint"
FP32_PEAK_TFLOPS = 157.3           # MI355X FP32 vector peak
FLOP_PER_INTERACTION = 24          # algorithmic count per pair force
FLOP_PER_ADJOINT_INTERACTION = 48  # forward pair force plus its vector-Jacobian product
FLOP_PER_NODE_TEST = 13            # r^2 (5), opening angle (2), enlarged-cube guard (6)
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_clustered_262k.md")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "walk_clustered_262k_counters.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("walk.hip", "internal.h", "gpoly.h"):
        h.update(open(os.path.join(ROOT, "paper_2606_17145_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def committed_values(path):
    """The machine-readable `- key: value` lines of a committed counter summary, if it
    was taken on the current kernel source; else an empty dict."""
    if not os.path.exists(path):
        return {}
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    return vals if vals.get("kernel_source_sha256_16") == kernel_source_hash() else {}


def committed_traffic(phase):
    """HBM bytes per launch of `phase` (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    v = committed_values(TRAFFIC_FILE).get(f"{phase}_bytes_per_launch")
    return float(v) if v else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


BUILD_BYTES_PER_PARTICLE = 170     # algorithmic HBM bytes of the tree build (radix passes excluded)


def timed_ms(torch, fn, reps):
    """Median milliseconds of fn() over `reps` runs, HIP events on the current stream
    (the stream every library call of this script is launched on)."""
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def flip_rate(c32, c64):
    """Fraction of targets whose FP32 interaction counts differ from the FP64 ones."""
    a, b = c32.cpu().numpy(), c64.cpu().numpy()
    return float(np.mean(np.any(a != b, axis=1)))


def other_configs(torch, sg, WL, dev, reps):
    """The remaining workloads, each timed on its own: uniform_32k (FP64 reference
    case), clustered_2m_active (relative criterion, 10% active subset) and the
    zoom_6m 8-step FP32 rollout with and without tree reuse."""
    out = {}
    t = lambda a, **k: torch.tensor(a, device=dev, **k)   # noqa: E731

    # uniform 32^3, FP64 (and FP32 beside it)
    w = WL.uniform_32k()
    pos, mass, eps = t(w.pos), t(w.mass), t(w.eps)
    tree = sg.Tree()
    b_ms = timed_ms(torch, lambda: sg.tree_build(pos, mass, eps=eps, tree=tree), reps)
    res = {}
    f64 = timed_ms(torch, lambda: res.__setitem__("64", sg.shortrange_accel(tree, w.params("fp64"))), reps)
    f32 = timed_ms(torch, lambda: res.__setitem__("32", sg.shortrange_accel(tree, w.params("fp32"))), reps)
    inter = int(res["64"][1].cpu().numpy().astype(np.int64).sum())
    out["uniform_32k"] = {"n": w.n, "build_ms": b_ms, "walk_fp64_ms": f64, "walk_fp32_ms": f32,
                          "interactions": inter, "walk_fp64_interactions_per_s": inter / (f64 * 1e-3),
                          "walk_fp32_interactions_per_s": inter / (f32 * 1e-3),
                          "particles_per_s_build_plus_fp64_walk": w.n / ((b_ms + f64) * 1e-3),
                          "fp32_count_flip_rate": flip_rate(res["32"][1], res["64"][1])}
    log(f"bench: uniform_32k build {b_ms:.3f} ms, fp64 walk {f64:.3f} ms, fp32 walk {f32:.3f} ms")
    del tree

    # clustered 128^3, relative criterion, 209,715 active targets; a_old = |a| of the
    # FP64 Barnes-Hut walk of all particles (the same walk the oracle defines)
    w = WL.clustered_2m_active()
    pos, mass, eps = t(w.pos), t(w.mass), t(w.eps)
    tree = sg.Tree()
    b_ms = timed_ms(torch, lambda: sg.tree_build(pos, mass, eps=eps, tree=tree), reps)
    a_bh, _ = sg.shortrange_accel(tree, dict(w.params("fp64"), criterion="bh", theta=0.5), counts=False)
    a_old = a_bh.norm(dim=1).contiguous()
    del a_bh
    act = t(w.active)
    res = {}
    f32 = timed_ms(torch, lambda: res.__setitem__("32", sg.shortrange_accel(tree, w.params("fp32"), active=act,
                                                                           a_old=a_old)), reps)
    f64 = timed_ms(torch, lambda: res.__setitem__("64", sg.shortrange_accel(tree, w.params("fp64"), active=act,
                                                                           a_old=a_old)), reps)
    inter32 = int(res["32"][1].cpu().numpy().astype(np.int64).sum())
    inter64 = int(res["64"][1].cpu().numpy().astype(np.int64).sum())
    out["clustered_2m_active"] = {
        "n": w.n, "targets": int(w.active.size), "criterion": "relative", "alpha": w.alpha, "theta": w.theta,
        "build_ms": b_ms, "build_gbs_algorithmic": BUILD_BYTES_PER_PARTICLE * w.n / (b_ms * 1e-3) / 1e9,
        "walk_fp32_ms": f32, "walk_fp64_ms": f64, "interactions_fp32": inter32, "interactions_fp64": inter64,
        "walk_fp32_interactions_per_s": inter32 / (f32 * 1e-3),
        "walk_fp64_interactions_per_s": inter64 / (f64 * 1e-3),
        "fp32_over_fp64_walk_speedup": f64 / f32,
        "fp32_count_flip_rate": flip_rate(res["32"][1], res["64"][1]),
        "a_old": "|a| of the FP64 Barnes-Hut (theta 0.5) walk of all particles, on the device"}
    log(f"bench: clustered_2m_active build {b_ms:.3f} ms, fp32 walk {f32:.3f} ms, fp64 walk {f64:.3f} ms")
    del tree, res, a_old

    # zoom-in, 6,291,456 particles: 8 KDK steps FP32, forward rollout and its
    # gradient, rebuilding every evaluation and every second evaluation
    from paper_2606_17145_amd import rollout as RL
    w = WL.zoom_6m()
    pos, mass, eps = t(w.pos), t(w.mass), t(w.eps)
    vel, lw = t(w.extra["vel"]), t(w.extra["loss_w"])
    ns, dt = w.extra["n_steps"], w.extra["dt"]
    p = w.params("fp32")
    z = {"n": w.n, "steps": ns, "dt": dt, "precision": "fp32"}
    for k in (1, 2):
        fwd = timed_ms(torch, lambda: RL.kdk_rollout(pos, vel, mass, eps, p, ns, dt, rebuild_every=k), 2)
        grad = timed_ms(torch, lambda: RL.kdk_rollout_grad(pos, vel, mass, eps, p, ns, dt, lw, rebuild_every=k), 2)
        z[f"rebuild_every_{k}"] = {"forward_ms": fwd, "forward_and_gradient_ms": grad}
        log(f"bench: zoom_6m rollout rebuild_every={k}: forward {fwd:.1f} ms, gradient {grad:.1f} ms")
    x1, _ = RL.kdk_rollout(pos, vel, mass, eps, p, ns, dt)
    x2, _ = RL.kdk_rollout(pos, vel, mass, eps, p, ns, dt, rebuild_every=2)
    moved = (x1 - pos).norm(dim=1)
    z["reuse_position_difference_rel"] = float((x2 - x1).norm(dim=1).max() / moved.max())
    z["tree_reuse_forward_time_saved"] = 1.0 - z["rebuild_every_2"]["forward_ms"] / z["rebuild_every_1"]["forward_ms"]
    out["zoom_6m_rollout"] = z
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error-check", action="store_true")
    ap.add_argument("--no-other-configs", action="store_true",
                    help="skip the uniform_32k, clustered_2m_active and zoom_6m legs")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy a buffer of this size once before the run (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2606_17145_amd as sg
    from paper_2606_17145_amd import _lib
    from paper_2606_17145_amd import workloads as WL

    _lib.lib()   # fail loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = WL.clustered_262k()
    p32 = w.params("fp32")
    p64 = w.params("fp64")
    pos = torch.tensor(w.pos, device=dev)
    mass = torch.tensor(w.mass, device=dev)
    eps = torch.tensor(w.eps, device=dev)
    cot = torch.tensor(WL.adjoint_weights(w.n), device=dev, dtype=torch.float32)
    log(f"bench: {w.name} N={w.n}")

    tree = sg.Tree()

    def step(ev=None):
        if ev:
            ev[0].record()
        sg.tree_build(pos, mass, eps=eps, box=w.box, tree=tree)
        if ev:
            ev[1].record()
        acc, cnt = sg.shortrange_accel(tree, p32)
        if ev:
            ev[2].record()
        dx, dm = sg.shortrange_accel_adjoint(tree, p32, cot, list_token=tree.list_token)
        if ev:
            ev[3].record()
        return acc, cnt

    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    _lib.timing(True)      # HIP events around every phase, on the launch stream
    t0 = time.perf_counter()
    for k in range(args.steps):
        acc, cnt = step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phases = _lib.timing_read()
    _lib.timing(False)
    stats = tree.walk_stats()
    build_ms = np.mean([e[0].elapsed_time(e[1]) for e in evs])
    fwd_ms = np.mean([e[1].elapsed_time(e[2]) for e in evs])
    adj_ms = np.mean([e[2].elapsed_time(e[3]) for e in evs])
    ms_step = wall / args.steps * 1e3
    counts = cnt.cpu().numpy().astype(np.int64)
    inter = int(counts.sum())
    log(f"bench: step {ms_step:.3f} ms (build {build_ms:.3f}, fwd32 {fwd_ms:.3f}, adj32 {adj_ms:.3f}), "
        f"interactions {inter}")

    # FP64 leg (not in the step): same tree, FP64 walk
    e64 = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for _ in range(2):
        a64, c64 = sg.shortrange_accel(tree, p64)
    reps = max(3, args.steps // 2)
    t64 = []
    for _ in range(reps):
        e64[0].record()
        a64, c64 = sg.shortrange_accel(tree, p64)
        e64[1].record()
        torch.cuda.synchronize()
        t64.append(e64[0].elapsed_time(e64[1]))
    fwd64_ms = float(np.mean(t64))
    inter64 = int(c64.cpu().numpy().astype(np.int64).sum())
    flips = flip_rate(cnt, c64)
    log(f"bench: fwd64 {fwd64_ms:.3f} ms")

    # PM leg (not in the step): long-range force of the same particles on the 128^3 mesh
    pmh = sg.PM(128)
    for _ in range(2):
        a_pm = pmh.accel(pos, mass, box=w.box, r_s=w.r_s)
    torch.cuda.synchronize()
    _lib.timing(True)
    e_pm = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e_pm[0].record()
    for _ in range(reps):
        a_pm = pmh.accel(pos, mass, box=w.box, r_s=w.r_s)
    e_pm[1].record()
    torch.cuda.synchronize()
    pm_ms = e_pm[0].elapsed_time(e_pm[1]) / reps
    pm_phases = {k: ms / reps for k, (ms, n) in _lib.timing_read().items() if k.startswith("pm_") and n}
    _lib.timing(False)
    for _ in range(2):
        pm_dx, pm_dm = pmh.accel_adjoint(pos, mass, cot, box=w.box, r_s=w.r_s)
    torch.cuda.synchronize()
    _lib.timing(True)
    e_pm[0].record()
    for _ in range(reps):
        pm_dx, pm_dm = pmh.accel_adjoint(pos, mass, cot, box=w.box, r_s=w.r_s)
    e_pm[1].record()
    torch.cuda.synchronize()
    pm_adj_ms = e_pm[0].elapsed_time(e_pm[1]) / reps
    pm_adj_phases = {k: ms / reps for k, (ms, n) in _lib.timing_read().items() if k.startswith("pm_") and n}
    _lib.timing(False)
    del pmh
    log(f"bench: pm 128^3 {pm_ms:.3f} ms {pm_phases}; adjoint {pm_adj_ms:.3f} ms")

    # SPH density leg (not in the step): smoothing lengths and densities of the
    # same particles on the step's tree, 64 neighbours
    for _ in range(2):
        sph_h, sph_rho, sph_bad = sg.sph_density(tree, 64.0)
    torch.cuda.synchronize()
    _lib.timing(True)
    t_sph = time.perf_counter()
    for _ in range(reps):
        sph_h, sph_rho, sph_bad = sg.sph_density(tree, 64.0)
    torch.cuda.synchronize()
    sph_ms = (time.perf_counter() - t_sph) / reps * 1e3
    it_ms, it_n = _lib.timing_read()["sph_iter"]
    _lib.timing(False)
    log(f"bench: sph density {sph_ms:.3f} ms per call, {it_n / reps:.1f} iterations, "
        f"{it_ms / max(it_n, 1):.4f} ms per iteration, unconverged {sph_bad}")

    out = {
        "metric": METRIC,
        "value": inter / (ms_step * 1e-3),
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": "clustered_262k", "n": w.n, "spheres": 200, "cluster_fraction": 0.7,
                   "n_mesh": 128, "r_s": w.r_s, "r_cut": w.r_cut, "eps": float(w.eps[0]),
                   "theta": w.theta, "criterion": "bh", "step": "build + fp32 walk + fp32 adjoint",
                   "parallelism": "single GPU"},
        "phases_ms": {"tree_build": build_ms, "walk_fp32": fwd_ms, "adjoint_fp32": adj_ms, "walk_fp64": fwd64_ms},
        "interactions_per_step": inter,
        "walk_fp32_interactions_per_s": inter / (fwd_ms * 1e-3),
        "adjoint_fp32_interactions_per_s": inter / (adj_ms * 1e-3),
        "walk_fp64_interactions_per_s": inter64 / (fwd64_ms * 1e-3),
        "fp32_over_fp64_walk_speedup": fwd64_ms / fwd_ms,
        "fp32_count_flip_rate": flips,
        "particles_per_s": w.n / (ms_step * 1e-3),
    }
    # per-kernel average launch durations from the library's events
    avg = {k: (ms / n if n else 0.0) for k, (ms, n) in phases.items()}
    out["kernel_ms_per_launch"] = avg
    out["walk_stats"] = stats
    out["sph_density"] = {"n_ngb": 64, "ms_per_call": sph_ms, "iterations_per_call": it_n / reps,
                          "ms_per_iteration": it_ms / max(it_n, 1), "particles_per_s": w.n / (sph_ms * 1e-3),
                          "unconverged": sph_bad}
    out["pm_long_range"] = {"n_mesh": 128, "ms_per_call": pm_ms, "phases_ms_per_call": pm_phases,
                            "particles_per_s": w.n / (pm_ms * 1e-3), "adjoint_ms_per_call": pm_adj_ms,
                            "adjoint_phases_ms_per_call": pm_adj_phases}
    work = {"eval": FLOP_PER_INTERACTION * inter,
            "adjoint_eval": FLOP_PER_ADJOINT_INTERACTION * inter,
            "traverse": FLOP_PER_NODE_TEST * stats["node_tests"]}
    dom = max(work, key=lambda k: avg[k])
    achieved = work[dom] / (avg[dom] * 1e-3) / 1e12
    out["roofline"] = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                       "traffic": committed_traffic(dom)}
    # executed VALU FLOP (counters: 64 x (ADD + MUL + 2 FMA + TRANS) per launch) over the
    # live launch time, beside the algorithmic rate above
    cv = committed_values(COUNTERS_FILE)
    valu = {}
    for ph in ("traverse", "eval", "adjoint_eval"):
        f = cv.get(f"{ph}_valu_flop_per_launch")
        if f and avg[ph] > 0:
            ex = float(f) / (avg[ph] * 1e-3) / 1e12
            valu[ph] = {"executed_tflops": ex, "executed_frac": ex / FP32_PEAK_TFLOPS,
                        "valu_insts_per_simd_cycle": float(cv[f"{ph}_valu_insts_per_simd_cycle"]),
                        "algorithmic_tflops": work[ph] / (avg[ph] * 1e-3) / 1e12}
    out["valu_counters"] = valu or None

    if not args.no_other_configs:
        del tree
        torch.cuda.empty_cache()
        out["configs"] = other_configs(torch, sg, WL, dev, reps=max(3, args.steps // 4))

    if not args.no_error_check:
        from oracle import oracle as O
        ref = O.Tree(w.pos, w.mass, w.eps)
        sample = np.sort(np.random.default_rng(9).choice(w.n, 16384, replace=False))
        acc_ref, _ = O.walk(ref, p64, targets=sample)
        a32 = acc.double().cpu().numpy()[sample]
        nr = np.linalg.norm(acc_ref, axis=1)
        e32 = np.linalg.norm(a32 - acc_ref, axis=1) / np.maximum(nr, 1e-6 * np.median(nr))
        e64 = np.linalg.norm(a64.cpu().numpy()[sample] - acc_ref, axis=1) / np.maximum(nr, 1e-6 * np.median(nr))
        out["force_error"] = {"vs": "fp64 oracle", "sample_targets": int(sample.size),
                              "fp32_median": float(np.median(e32)), "fp32_p999": float(np.quantile(e32, 0.999)),
                              "fp64_max": float(e64.max())}
        log(f"bench: fp32 error median {np.median(e32):.2e} p99.9 {np.quantile(e32, 0.999):.2e}")

    if not args.no_cpu_baseline:
        # the oracle on the host: the whole step (tree build, walk and adjoint of all targets) in FP64
        from oracle import oracle as O
        O.use_native_build()     # -O3 -march=native for this host
        wt = WL.adjoint_weights(w.n)
        t0 = time.perf_counter()
        ref = O.Tree(w.pos, w.mass, w.eps)
        _, cs = O.walk(ref, p64)
        O.adjoint(ref, p64, wt)
        cpu_s = time.perf_counter() - t0
        cpu_model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo")
                          if ln.startswith("model name")), "unknown") if os.path.exists("/proc/cpuinfo") else "unknown"
        out["cpu_baseline"] = {"value": float(cs.sum()) / cpu_s, "unit": "interactions/s",
                               "cores": O.num_threads(), "host_cpus": os.cpu_count(),
                               "build": "gcc -O3 -march=native -ffp-contract=off -fopenmp",
                               "kind": "oracle", "cpu_model": cpu_model,
                               "sample": "the whole step on the same workload: FP64 oracle tree build of all "
                                         "262,144 particles, walk and adjoint of all 262,144 targets"}
        log(f"bench: oracle {cpu_s:.2f} s on {O.num_threads()} threads")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
