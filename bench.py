"""Benchmark: tree-force particles/s and interactions/s on one MI355X.

A step is one velocity-Verlet (kick-drift-kick) step of the whole hot path on
the N = 524,288 cloud (theta = 0.5, eps = 0.005, dt = 5e-5): enclosing cube,
keys (Hilbert order by default, --curve morton for Morton order), radix sort,
octree build, moments, groups, group walk (M2P + P2P) writing the forces in
the caller's order, and the two kicks.  Inputs are resident in HBM before the
timed region.

Prints ONE JSON line.  value = particles/s = N * steps / elapsed.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic FLOPs per interaction, counted from the FP32 evaluation code
# (add, sub, mul = 1; fma = 2; rsqrt = 1); forces only (no potential)
P2P_FLOPS = 19
M2P_FLOPS = 63
PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (packed) -- published peak
PEAK_FP64_TFLOPS = 78.6
WALK_SOURCES = ["paper_0709_3331_amd/csrc/walk.hip", "paper_0709_3331_amd/csrc/internal.h"]


def note(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def walk_source_hash():
    h = hashlib.sha256()
    for p in WALK_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# order of the keys for every solver and oracle tree of the run (ucp_curve)
CURVE = 1


def traffic_from_profile(precision):
    """HBM bytes per walk launch from the committed rocprofv3 counter summary,
    or None when the walk kernel or the key order changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", f"walk_{precision}_n524288_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except OSError:
        return None
    if d.get("walk_source_hash") != walk_source_hash() or d.get("curve") != CURVE:
        return None
    return d.get("hbm_bytes_per_launch")


def bench_ensemble(args, prec, dev):
    """64 independent clouds (N_c = 2 U[4096, 65536], sigma_c = U[0.5, 2]) built
    and walked together: one batched build and one persistent walk per Verlet
    step, the steps replayed from a hipGraph.  (G, L, group rule) come from the
    autotuner, run on this input."""
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import autotune, inputs
    from paper_0709_3331_amd.tree import TreeSolver

    ens, off, eprm = inputs.ensemble()
    clouds = len(off) - 1
    n = int(off[-1])
    x = torch.from_numpy(ens.x).to(dev)
    v = torch.from_numpy(ens.v).to(dev)
    q = torch.from_numpy(ens.q).to(dev)
    m = torch.from_numpy(ens.m).to(dev)
    offs = torch.from_numpy(off).to(dev)
    print(f"bench: ensemble of {clouds} clouds, N={n}: tuning", file=sys.stderr, flush=True)
    tuned = autotune.tune(x, q, offs, theta=eprm["theta"], eps=eprm["eps"], precision=prec,
                          candidates={"group_size": (32, 64), "list_len": (64, 128, 256),
                                      "group_mode": (1, 0), "leaf_cap": (8, 16, 24, 32)},
                          reps=2, use_cache=False)
    ts = TreeSolver(n, clouds, curve=CURVE, theta=eprm["theta"], eps=eprm["eps"], precision=prec,
                    group_size=tuned["group_size"], list_len=tuned["list_len"],
                    group_mode=tuned["group_mode"], leaf_cap=tuned["leaf_cap"])
    f = ts.tree_forces(x, q, offs)
    st = ts.stats()
    x0, v0, f0 = x.clone(), v.clone(), f.clone()

    def restore():
        for dst, src in ((x, x0), (v, v0), (f, f0)):
            dst.copy_(src)

    # one untimed call captures the step graphs; the timed call replays them
    # from the state the directly enqueued steps below start from too
    ts.step(x, v, f, q, m, eprm["dt"], 2, offsets=offs)
    restore()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ts.step(x, v, f, q, m, eprm["dt"], args.ensemble_steps, offsets=offs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ts.stats()
    # the walk time: the same steps enqueued directly with HIP events around
    # every walk launch (timing on bypasses the graphs)
    restore()
    ts.timing(True)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    ts.step(x, v, f, q, m, eprm["dt"], args.ensemble_steps, offsets=offs)
    torch.cuda.synchronize()
    e1 = time.perf_counter()
    wms, wc = ts.timing_read()
    balance = wave_balance(ts)
    ts.stats()
    ts.close()
    # the plain FP64 walk of the same batched build at the same setting
    t64 = TreeSolver(n, clouds, curve=CURVE, theta=eprm["theta"], eps=eprm["eps"],
                     precision=L.UCP_FP64, group_size=tuned["group_size"],
                     list_len=tuned["list_len"], group_mode=tuned["group_mode"],
                     leaf_cap=tuned["leaf_cap"])
    t64.tree_forces(x, q, offs)
    t64.timing(True)
    torch.cuda.synchronize()
    for _ in range(3):
        t64.tree_forces(x, q, offs)
    torch.cuda.synchronize()
    w64, c64 = t64.timing_read()
    t64.stats()
    t64.close()
    el = t1 - t0
    return {"clouds": clouds, "n_total": n, "steps": args.ensemble_steps,
            "path": "hipGraph replay of the batched step",
            "particles_per_s": n * args.ensemble_steps / el,
            "ms_per_step": 1e3 * el / args.ensemble_steps,
            "direct_enqueue_ms_per_step": 1e3 * (e1 - e0) / args.ensemble_steps,
            "walk_ms": wms / max(wc, 1),
            "walk_wave_balance": balance,
            "fp64_walk_ms": w64 / max(c64, 1),
            "split_speedup_walk": (w64 / max(c64, 1)) / (wms / max(wc, 1)),
            "interactions_per_particle": (st["p2p"] + st["m2p"]) / n,
            "tuned": {"group_size": tuned["group_size"], "list_len": tuned["list_len"],
                      "leaf_cap": tuned["leaf_cap"],
                      "group_mode": "chunk" if tuned["group_mode"] == 1 else "node",
                      "rel_force_err_vs_direct": tuned["rel_force_err_vs_direct"],
                      "per_particle_walk_err_vs_direct": tuned["per_particle_walk_err_vs_direct"],
                      "err_bound": tuned["err_bound"],
                      "rel_force_diff_vs_per_particle_fp64":
                          tuned.get("rel_force_diff_vs_per_particle_fp64"),
                      "candidates": {f"{'chunk' if r['group_mode'] == 1 else 'node'}/G{r['group_size']}/"
                                     f"L{r['list_len']}/cap{r['leaf_cap']}":
                                     {"walk_ms": round(r["walk_ms"], 4),
                                      "err_vs_direct": float("%.4g" % r["rel_force_err_vs_direct"]),
                                      "admitted": r["admitted"]}
                                     for r in tuned["candidates"]}}}


def _finite(v):
    """JSON has no NaN or infinity: report those as null."""
    return v if isinstance(v, float) and math.isfinite(v) else None


def wave_balance(ts):
    """Balance of the persistent walk in the last timed walk, from every
    wave's start and end.  More waves are launched than can be resident, so
    the waves that start with the launch take the groups and the rest start
    as those end, find the queues empty and stop.  Reported: the span of the
    walk, how many waves started with the launch, the spread of their end
    times, the share of their wave-time spent idle after their own end
    (the tail of the walk), and each compute unit's busy time (its first
    wave's start to its last wave's end) as min, mean, max and max / mean
    over the units."""
    import numpy as np
    t, unit = ts.wave_clock(units=True)
    span = float(t[:, 1].max())
    first = t[:, 0] <= 0.02 * span
    ends = t[first, 1]
    # per compute unit: busy from its first wave's start to its last wave's end
    cus, inv = np.unique(unit, return_inverse=True)
    busy = np.full(cus.shape[0], -np.inf)
    np.maximum.at(busy, inv, t[:, 1])
    start = np.full(cus.shape[0], np.inf)
    np.minimum.at(start, inv, t[:, 0])
    busy -= start
    return {"waves": int(t.shape[0]), "waves_at_launch": int(first.sum()), "span_us": span,
            "launch_wave_end_us": {"min": float(ends.min()), "p10": float(np.quantile(ends, 0.1)),
                                   "median": float(np.median(ends)), "max": float(ends.max())},
            "launch_wave_idle_share": float(np.mean(span - ends) / span),
            "per_cu_busy_us": {"cus": int(cus.shape[0]), "min": float(busy.min()),
                               "mean": float(busy.mean()), "max": float(busy.max()),
                               "max_over_mean": float(busy.max() / busy.mean())}}


def per_particle_rel(f, ref):
    """Per-particle relative force error |F_i - ref_i| / |ref_i|: median, 99th
    percentile and maximum (rows of ref that are NaN are skipped)."""
    import numpy as np
    m = ~np.isnan(ref[:, 0])
    r = np.linalg.norm(f[m] - ref[m], axis=1) / np.maximum(np.linalg.norm(ref[m], axis=1), 1e-300)
    return {"median": float(np.median(r)), "p99": float(np.quantile(r, 0.99)),
            "max": float(r.max()), "particles": int(m.sum())}


def cpu_info():
    """Model name of the host CPU and the cores this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "logical_cpus": os.cpu_count()}


def bench_accuracy_target(args, prec, x, v, q, m, n, eps, dt, tg, fd, target=1e-3):
    """The cheapest setting of (theta, leaf_cap) at G = 64 chunk groups whose
    relative RMS force error against the FP64 direct sum on the sampled
    targets meets `target`: every candidate is evaluated once for its error,
    and those that meet it are timed over whole Verlet steps (particles/s as
    in the headline, directly enqueued); the fastest is reported with its
    error."""
    import numpy as np
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd.tree import TreeSolver

    gm = L.UCP_GROUP_CHUNK if args.group_mode == "chunk" else L.UCP_GROUP_NODE
    rows = []
    for th in (0.3, 0.35, 0.4, 0.45, 0.5):
        for cap in (16, 24, 32, 48, 64):
            tt = TreeSolver(n, curve=CURVE, theta=th, eps=eps, precision=prec,
                            group_size=args.group_size, list_len=args.list_len, group_mode=gm,
                            leaf_cap=cap, walk_waves=args.walk_waves)
            fa = tt.tree_forces(x, q).cpu().numpy()
            err = float(np.linalg.norm(fa[tg] - fd) / np.linalg.norm(fd))
            row = {"theta": th, "leaf_cap": cap, "group_size": args.group_size,
                   "rel_force_err_vs_direct_sampled": err}
            if err <= target:
                xx, vv = x.clone(), v.clone()
                ff = tt.tree_forces(xx, q)
                tt.step(xx, vv, ff, q, m, dt, 1)
                tt.timing(True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                tt.step(xx, vv, ff, q, m, dt, 5)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                wm, wc = tt.timing_read()
                row["ms_per_step"] = 1e3 * (t1 - t0) / 5
                row["particles_per_s"] = n * 5 / (t1 - t0)
                row["walk_ms"] = wm / max(wc, 1)
            tt.stats()
            tt.close()
            rows.append(row)
    ok = [r for r in rows if "ms_per_step" in r]
    best = min(ok, key=lambda r: r["ms_per_step"]) if ok else None
    # the same with a margin: an error at most 3/4 of the target, which other
    # samples and states of the cloud keep below it
    okm = [r for r in ok if r["rel_force_err_vs_direct_sampled"] <= 0.75 * target]
    robust = min(okm, key=lambda r: r["ms_per_step"]) if okm else None
    # the plain FP64 walk at those settings: the split's speedup at equal
    # force accuracy (the two differ by ~1e-6, far below the tree's error)
    for r in (best, robust):
        if r is None or "fp64_walk_ms" in r:
            continue
        tt = TreeSolver(n, curve=CURVE, theta=r["theta"], eps=eps, precision=L.UCP_FP64,
                        group_size=args.group_size, list_len=args.list_len, group_mode=gm,
                        leaf_cap=r["leaf_cap"], walk_waves=args.walk_waves)
        tt.tree_forces(x, q)
        tt.timing(True)
        torch.cuda.synchronize()
        for _ in range(3):
            tt.tree_forces(x, q)
        torch.cuda.synchronize()
        wm, wc = tt.timing_read()
        tt.stats()
        tt.close()
        r["fp64_walk_ms"] = wm / max(wc, 1)
        r["split_speedup_walk"] = r["fp64_walk_ms"] / r["walk_ms"]
    return {"target_rel_rms_vs_direct": target, "cheapest": best, "cheapest_with_margin": robust,
            "candidates": [{k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}
                           for r in rows]}


def bench_seeds(args, prec, dev, seeds=(1, 2)):
    """The headline steps on the same workload drawn with other seeds (run to
    run variance of the input): ms per step and particles/s of graph replays,
    as the headline, and the walk time of the same steps enqueued directly."""
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import inputs
    from paper_0709_3331_amd.tree import TreeSolver

    gm = L.UCP_GROUP_CHUNK if args.group_mode == "chunk" else L.UCP_GROUP_NODE
    out = {}
    for sd in seeds:
        cl, prm = inputs.metric(sd)
        x = torch.from_numpy(cl.x).to(dev)
        v = torch.from_numpy(cl.v).to(dev)
        q = torch.from_numpy(cl.q).to(dev)
        m = torch.from_numpy(cl.m).to(dev)
        ts = TreeSolver(cl.n, curve=CURVE, theta=args.theta, eps=prm["eps"], precision=prec,
                        group_size=args.group_size, list_len=args.list_len, group_mode=gm,
                        leaf_cap=args.leaf_cap, walk_waves=args.walk_waves)
        f = ts.tree_forces(x, q)
        st = ts.stats()
        for _ in range(args.warmup):
            ts.step(x, v, f, q, m, prm["dt"], 1)
        x0, v0, f0 = x.clone(), v.clone(), f.clone()

        def restore():
            for dst, src in ((x, x0), (v, v0), (f, f0)):
                dst.copy_(src)

        # as the headline: graph replays of K steps, then the same steps from
        # the same state enqueued directly with the walk's HIP events
        ts.step(x, v, f, q, m, prm["dt"], 2)
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ts.step(x, v, f, q, m, prm["dt"], args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        restore()
        ts.timing(True)
        torch.cuda.synchronize()
        ts.step(x, v, f, q, m, prm["dt"], args.steps)
        torch.cuda.synchronize()
        wm, wc = ts.timing_read()
        ts.stats()
        ts.close()
        out[str(sd)] = {"ms_per_step": 1e3 * (t1 - t0) / args.steps,
                        "particles_per_s": cl.n * args.steps / (t1 - t0),
                        "walk_ms": wm / max(wc, 1),
                        "interactions_per_particle": (st["p2p"] + st["m2p"]) / cl.n}
    return out


def bench_large(args, prec, dev):
    """The N = 4,194,304 cloud (10% of the electrons hot, eps = 0.002,
    theta = 0.5): one force evaluation (build + walk) timed on its own, its
    particles/s, then 50 Verlet steps (dt = 5e-5), and the error of the
    forces against the FP64 oracle tree on every 997th walk group and against
    the FP64 direct sum on 1024 sampled targets."""
    import numpy as np
    import torch

    import oracle
    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import inputs
    from paper_0709_3331_amd.tree import TreeSolver

    cl, prm = inputs.large(0)
    n = cl.n
    print(f"bench: large cloud N={n}", file=sys.stderr, flush=True)
    gm = L.UCP_GROUP_CHUNK if args.group_mode == "chunk" else L.UCP_GROUP_NODE
    x = torch.from_numpy(cl.x).to(dev)
    v = torch.from_numpy(cl.v).to(dev)
    q = torch.from_numpy(cl.q).to(dev)
    m = torch.from_numpy(cl.m).to(dev)
    ts = TreeSolver(n, curve=CURVE, theta=prm["theta"], eps=prm["eps"], precision=prec,
                    group_size=args.group_size, list_len=args.list_len, group_mode=gm,
                    leaf_cap=args.leaf_cap, walk_waves=args.walk_waves)
    f = ts.tree_forces(x, q)
    st = ts.stats()
    f0 = f.cpu().numpy()
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ts.build(x, q)
        L.ucp_compute_forces(ts.h, f.data_ptr(), None, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ts.stats()
    eval_s = (t1 - t0) / reps
    ts.step(x, v, f, q, m, prm["dt"], 1)
    ts.timing(True)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    ts.step(x, v, f, q, m, prm["dt"], prm["steps"])
    torch.cuda.synchronize()
    s1 = time.perf_counter()
    wm, wc = ts.timing_read()
    ts.stats()
    ts.close()
    t = oracle.Tree(cl.x, cl.q, prm["theta"], prm["eps"], curve=CURVE, G=args.group_size,
                    group_mode=gm, leaf_cap=args.leaf_cap)
    ref = t.eval_groups(np.arange(0, t.ngroups, 997))["f"]
    mk = ~np.isnan(ref[:, 0])
    tg = np.sort(np.random.default_rng(0).choice(n, 1024, replace=False))
    fd, _ = oracle.direct_targets(cl.x, cl.q, prm["eps"], tg)
    return {"n": n, "eps": prm["eps"], "theta": prm["theta"],
            "force_eval_ms": 1e3 * eval_s, "force_eval_particles_per_s": n / eval_s,
            "steps": prm["steps"], "dt": prm["dt"],
            "ms_per_step": 1e3 * (s1 - s0) / prm["steps"],
            "particles_per_s": n * prm["steps"] / (s1 - s0),
            "walk_ms": wm / max(wc, 1),
            "interactions_per_particle": (st["p2p"] + st["m2p"]) / n,
            "rel_force_err_vs_oracle_tree_sampled": float(
                np.linalg.norm(f0[mk] - ref[mk]) / np.linalg.norm(ref[mk])),
            "per_particle_err_vs_oracle_tree_sampled": per_particle_rel(f0, ref),
            "rel_force_err_vs_direct_sampled": float(
                np.linalg.norm(f0[tg] - fd) / np.linalg.norm(fd)),
            "sampled_groups": int(len(range(0, t.ngroups, 997))), "sampled_targets": 1024}


def ensemble_steps(args, dev):
    """The 64-cloud ensemble's batched Verlet steps at the setting the
    autotuner picks for it (G = 64 chunk groups, L = 128, leaf capacity 24,
    the figures of the benchmark's ensemble section), enqueued directly with
    HIP events around every walk, for a kernel trace: --warmup untimed steps,
    then --steps timed ones."""
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import inputs
    from paper_0709_3331_amd.tree import TreeSolver

    ens, off, eprm = inputs.ensemble()
    clouds = len(off) - 1
    n = int(off[-1])
    x, v, q, m = (torch.from_numpy(a).to(dev) for a in (ens.x, ens.v, ens.q, ens.m))
    offs = torch.from_numpy(off).to(dev)
    prec = L.UCP_SPLIT if args.precision == "split" else L.UCP_FP64
    gm = L.UCP_GROUP_CHUNK if args.group_mode == "chunk" else L.UCP_GROUP_NODE
    ts = TreeSolver(n, clouds, curve=CURVE, theta=eprm["theta"], eps=eprm["eps"], precision=prec,
                    group_size=args.group_size, list_len=args.list_len, group_mode=gm,
                    leaf_cap=args.leaf_cap, walk_waves=args.walk_waves)
    f = ts.tree_forces(x, q, offs)
    ts.timing(True)
    for _ in range(args.warmup):
        ts.step(x, v, f, q, m, eprm["dt"], 1, offsets=offs)
    torch.cuda.synchronize()
    ts.timing_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts.step(x, v, f, q, m, eprm["dt"], 1, offsets=offs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wms, wc = ts.timing_read()
    ts.timing(False)
    st = ts.stats()
    ts.close()
    return {"workload": f"64-cloud ensemble, N={n} in all, eps={eprm['eps']}, theta={eprm['theta']}, "
                        f"G={args.group_size} ({args.group_mode} groups), L={args.list_len}, "
                        f"leaf_cap={args.leaf_cap}, one KDK Verlet step dt={eprm['dt']}",
            "n": n, "clouds": clouds, "precision": args.precision, "steps": args.steps,
            "warmup": args.warmup, "path": "directly enqueued steps",
            "ms_per_step": 1e3 * (t1 - t0) / args.steps, "walk_ms": wms / max(wc, 1),
            "interactions_per_particle": (st["m2p"] + st["p2p"]) / n}


def vjp_timing(args, dev):
    """The force VJP beside the forward walk on the N = 65,536 cloud of the
    differentiable rollout (theta = 0.5, eps = 0.01), same tree: --warmup
    untimed pairs, then --steps forward walks (HIP events around each walk
    launch) and --steps VJPs (torch events on the stream the library launches
    on, around the whole call: the adjoint walk with its preparation and the
    push down to the particles).  The cotangent u is standard normal."""
    import numpy as np
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import inputs
    from paper_0709_3331_amd.tree import TreeSolver

    cl, prm = inputs.adjoint(0)
    n = cl.n
    prec = L.UCP_SPLIT if args.precision == "split" else L.UCP_FP64
    x, q = (torch.from_numpy(a).to(dev) for a in (cl.x, cl.q))
    gm = L.UCP_GROUP_CHUNK if args.group_mode == "chunk" else L.UCP_GROUP_NODE
    ts = TreeSolver(n, curve=CURVE, theta=prm["theta"], eps=prm["eps"], precision=prec,
                    group_size=args.group_size, list_len=args.list_len, group_mode=gm,
                    leaf_cap=args.leaf_cap, walk_waves=args.walk_waves)
    ts.tree_forces(x, q)
    st = ts.stats()
    u = torch.from_numpy(np.random.default_rng(1).standard_normal((n, 3))).to(dev)
    for _ in range(args.warmup):
        ts.forces(n)
        ts.vjp(u)
    torch.cuda.synchronize()
    ts.timing(True)
    for _ in range(args.steps):
        ts.forces(n)
    torch.cuda.synchronize()
    fwd_tot, launches = ts.timing_read()
    fwd_ms = fwd_tot / max(launches, 1)
    ts.timing(False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        ts.vjp(u)
    e1.record()
    torch.cuda.synchronize()
    vjp_ms = e0.elapsed_time(e1) / args.steps
    ts.check()
    ts.close()
    return {"workload": f"N={n} Gaussian cloud (sigma=1), theta={prm['theta']}, eps={prm['eps']}, "
                        f"G={args.group_size} ({args.group_mode} groups), leaf_cap={args.leaf_cap}",
            "n": n, "precision": args.precision, "steps": args.steps, "warmup": args.warmup,
            "forward_walk_ms": fwd_ms, "forward_walk_launches": launches, "vjp_ms": vjp_ms,
            "vjp_over_forward_walk": vjp_ms / fwd_ms, "m2p": st["m2p"], "p2p": st["p2p"],
            "interactions_per_particle": (st["m2p"] + st["p2p"]) / n}


def bench_adjoint(prec, dev):
    """Differentiable rollout of the N = 65,536 cloud (eps = 0.01, checkpoint
    every 20 steps); loss = final ion kinetic energy; gradient with respect to
    sigma (x0 = sigma z) through the adjoint walk, reported beside central
    differences in sigma.  Cases:
      - the stated workload (theta = 0.5, dt = 1e-4) at 5, 20 and 200 steps;
      - theta = 0 (direct sum: no lists to change) at 5 steps, several h;
      - a resolved control, dt = 1e-6, 200 steps, at theta = 0.5 and at
        theta = 0, several h (h = 1e-4 is the workload's own).
    At theta > 0 the loss of a long rollout is only piecewise smooth in
    sigma: a perturbed run changes some interaction lists (an opening
    decision flips), and central differences over an h that spans such jumps
    do not converge to the derivative the adjoint returns; at theta = 0 there
    are no lists.
    The stated dt does not resolve electrons bound in the softened ion wells
    (omega dt ~ 4), so perturbations grow ~18x per step there and the finite
    differences stop being linear within a few steps unless h is tiny; in the
    resolved control they are.  Finite differences use the FP64 path; the
    stated 200-step workload is also timed in the benchmark precision.
    Nothing here is asserted; the gradient checks are tests."""
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import adjoint, inputs
    from paper_0709_3331_amd.tree import TreeSolver

    cl, prm = inputs.adjoint(0)
    n = cl.n
    z = torch.from_numpy(cl.x).to(dev)
    q = torch.from_numpy(cl.q).to(dev)
    m = torch.from_numpy(cl.m).to(dev)
    v0n = torch.from_numpy(cl.v).to(dev)
    solvers = {}

    def loss_of(ts, sigma, v0, dt, steps):
        xT, vT = adjoint.rollout(ts, sigma * z, v0, q, m, dt, steps, checkpoint_every=prm["ckpt"])
        return adjoint.ion_kinetic_energy(vT, q, m)

    # (theta, dt, steps, finite-difference steps h, precision); the finite
    # differences need the FP64 path: FP32 arithmetic makes the loss noisy at
    # the 1e-7 level, far above what 2h resolves
    fp64 = L.UCP_FP64
    cases = [(prm["theta"], prm["dt"], prm["steps"], (), prec),
             (prm["theta"], prm["dt"], 5, (1e-7, 1e-9, 1e-11), fp64),
             (prm["theta"], prm["dt"], 20, (1e-9, 1e-11), fp64),
             (0.0, prm["dt"], 5, (1e-7, 1e-9, 1e-11), fp64),
             (prm["theta"], 1e-6, prm["steps"], (1e-4, 1e-5, 1e-7, 1e-9), fp64),
             (0.0, 1e-6, prm["steps"], (1e-4, 1e-7, 1e-9), fp64)]
    out = {"n": n, "eps": prm["eps"], "checkpoint_every": prm["ckpt"], "cases": {}}
    for th, dt, steps, hs, pr in cases:
        if (th, pr) not in solvers:
            solvers[(th, pr)] = TreeSolver(n, curve=CURVE, theta=th, eps=prm["eps"], precision=pr)
        ts = solvers[(th, pr)]
        print(f"bench: adjoint rollout N={n} theta={th} dt={dt} steps={steps}", file=sys.stderr,
              flush=True)
        sigma = torch.tensor(1.0, dtype=torch.float64, device=dev, requires_grad=True)
        v0 = v0n.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = loss_of(ts, sigma, v0, dt, steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g = sigma.grad.item()
        fds = {}
        for h in hs:
            with torch.no_grad():
                lp = loss_of(ts, torch.tensor(1.0 + h, dtype=torch.float64, device=dev), v0n, dt,
                             steps).item()
                lm = loss_of(ts, torch.tensor(1.0 - h, dtype=torch.float64, device=dev), v0n, dt,
                             steps).item()
            fd = (lp - lm) / (2 * h)
            fds[f"{h:g}"] = {"central_difference": _finite(fd),
                             "rel_diff": _finite(abs(g - fd) / abs(fd)) if fd != 0 else None}
        name = "split" if pr == L.UCP_SPLIT else "fp64"
        out["cases"][f"theta={th:g},dt={dt:g},steps={steps},{name}"] = {
            "loss": _finite(loss.item()), "dL_dsigma": _finite(g), "fd": fds,
            "forward_s": t1 - t0, "backward_s": t2 - t1}
    for ts in solvers.values():
        ts.close()
    return out


def bench_other_curve(args, prec, cl, prm, dev):
    """The same workload with the other key order (Morton when the run uses
    Hilbert keys, and the reverse): the same K timed steps from the same
    initial state, with the step time, walk time and interactions."""
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd.tree import TreeSolver

    other = 1 - CURVE
    gm = L.UCP_GROUP_CHUNK if args.group_mode == "chunk" else L.UCP_GROUP_NODE
    x = torch.from_numpy(cl.x).to(dev)
    v = torch.from_numpy(cl.v).to(dev)
    q = torch.from_numpy(cl.q).to(dev)
    m = torch.from_numpy(cl.m).to(dev)
    ts = TreeSolver(cl.n, curve=other, theta=args.theta, eps=prm["eps"], precision=prec,
                    group_size=args.group_size, list_len=args.list_len, group_mode=gm,
                    leaf_cap=args.leaf_cap, walk_waves=args.walk_waves)
    f = ts.tree_forces(x, q)
    st0 = ts.stats()
    for _ in range(args.warmup):
        ts.step(x, v, f, q, m, prm["dt"], 1)
    ts.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ts.step(x, v, f, q, m, prm["dt"], args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wm, wc = ts.timing_read()
    ts.close()
    ms = 1e3 * (t1 - t0) / args.steps
    return {"curve": "hilbert" if other == 1 else "morton", "ms_per_step": ms,
            "particles_per_s": cl.n * args.steps / (t1 - t0), "walk_ms": wm / max(wc, 1),
            "interactions_per_particle": (st0["p2p"] + st0["m2p"]) / cl.n}


def bench_kelbg(args, prec, x, q, cl, plummer_walk_ms):
    """The same cloud and opening parameter under the Kelbg pair law of
    Eq. (3): electron-ion pairs through q q (1 - exp(-r/lambda)) / r with
    lambda = 0.005 (the length the Plummer runs use for eps), like pairs bare
    Coulomb (eps = 0) as in Sec. 2.1.  Walk time, interactions/s, the cost
    against the Plummer walk, and the force difference from the FP64 oracle
    tree on every 97th walk group."""
    import numpy as np
    import torch

    import oracle
    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd.tree import TreeSolver

    lam = 0.005
    gm = L.UCP_GROUP_CHUNK if args.group_mode == "chunk" else L.UCP_GROUP_NODE
    ts = TreeSolver(cl.n, curve=CURVE, theta=args.theta, eps=0.0, precision=prec, group_size=args.group_size,
                    list_len=args.list_len, group_mode=gm, leaf_cap=args.leaf_cap,
                    walk_waves=args.walk_waves, pair_law=L.UCP_PAIR_KELBG, lambda_ei=lam)
    f = ts.tree_forces(x, q)
    ts.timing(True)
    torch.cuda.synchronize()
    for _ in range(5):
        ts.tree_forces(x, q)
    torch.cuda.synchronize()
    wm, wc = ts.timing_read()
    st = ts.stats()
    ts.close()
    walk = wm / max(wc, 1)
    xs = x.cpu().numpy()   # the positions after the timed steps
    t = oracle.Tree(xs, cl.q, args.theta, 0.0, curve=CURVE, G=args.group_size, group_mode=gm,
                    leaf_cap=args.leaf_cap, pair_law=oracle.PAIR_KELBG, lambda_ei=lam)
    ref = t.eval_groups(np.arange(0, t.ngroups, 97))["f"]
    mask = ~np.isnan(ref[:, 0])
    fa = f.cpu().numpy()
    return {"lambda_ei": lam, "eps_like_pairs": 0.0, "walk_ms": walk,
            "interactions_per_s": (st["p2p"] + st["m2p"]) / (walk * 1e-3),
            "walk_cost_vs_plummer": walk / plummer_walk_ms,
            "rel_force_err_vs_oracle_tree_sampled": float(
                np.linalg.norm(fa[mask] - ref[mask]) / np.linalg.norm(ref[mask])),
            "sampled_particles": int(mask.sum())}


def opening_study(dev, dt=1e-6):
    """Opening-parameter study after Sec. 5.2 (Fig. 9): a cloud of 5e4 ions and
    5e4 electrons (sigma = 1, T_e = 1e-3, T_i = 1e-5, eps = 0.01) advanced
    1000 Verlet steps at each theta, its total energy E(t) = K + U (U from the
    tree potential at that theta) compared every 50 steps with the all-pairs
    run (theta = 0: no box is ever accepted) in FP64, and the cost of the
    steps set against theta = 0.1.  The default dt = 1e-6 is the resolved
    control: omega dt = 0.043 for an electron bound in a softened ion well
    (omega^2 = 1836 / eps^3), so the integrator's own energy error stays
    below the tree's; at dt = 1e-5 (omega dt = 0.43) the all-pairs run
    itself drifts by ~4% in 1000 steps."""
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import inputs
    from paper_0709_3331_amd.tree import TreeSolver

    cl = inputs.gaussian_cloud(100000, 1.0, 1e-3, 1e-5, 0)
    eps, dt, steps, every = 0.01, dt, 1000, 50
    q = torch.from_numpy(cl.q).to(dev)
    m = torch.from_numpy(cl.m).to(dev)

    def run(theta, prec):
        ts = TreeSolver(cl.n, curve=CURVE, theta=theta, eps=eps, precision=prec)
        x = torch.from_numpy(cl.x).to(dev)
        v = torch.from_numpy(cl.v).to(dev)
        f = ts.tree_forces(x, q)
        st = ts.stats()
        ipp = (st["p2p"] + st["m2p"]) / cl.n
        e0 = ts.energy(x, v, q, m).cpu().tolist()
        energies = [e0[2]]
        step_s = 0.0
        for _ in range(steps // every):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ts.step(x, v, f, q, m, dt, every)
            torch.cuda.synchronize()
            step_s += time.perf_counter() - t0
            energies.append(ts.energy(x, v, q, m)[2].item())
        ts.stats()
        ts.close()
        print(f"opening study: theta={theta:g} done, {1e3 * step_s / steps:.3f} ms/step",
              file=sys.stderr, flush=True)
        return energies, step_s / steps, ipp, e0

    e_ref, t_ref, _, c_ref = run(0.0, L.UCP_FP64)
    out = {"study": "opening parameter (Sec. 5.2, Fig. 9)", "n": cl.n, "eps": eps, "dt": dt,
           "steps": steps, "energy_every": every, "precision": "split",
           "reference": {"theta": 0.0, "precision": "fp64", "ms_per_step": 1e3 * t_ref,
                         "K_U_E_at_t0": c_ref[:3],
                         "energy_drift_max": _finite(max(abs(e - e_ref[0]) for e in e_ref)
                                                     / abs(e_ref[0]))},
           "theta": {}}
    base = None
    for th in (0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7):
        e, t, ipp, _ = run(th, L.UCP_SPLIT)
        err = [abs(a - b) / abs(b) for a, b in zip(e, e_ref)]
        base = base or t
        out["theta"][f"{th:g}"] = {
            "ms_per_step": 1e3 * t, "cost_vs_theta_0.1": t / base,
            "interactions_per_particle": ipp,
            "energy_err_vs_all_pairs_t0_pct": _finite(100 * err[0]),
            "energy_err_vs_all_pairs_max_pct": _finite(100 * max(err)),
            "energy_err_vs_all_pairs_final_pct": _finite(100 * err[-1]),
            "energy_drift_max_pct": _finite(100 * max(abs(a - e[0]) for a in e) / abs(e[0]))}
    return out


def relaxation_study(dev, clouds=16, n_c=10000, steps=10000, every=250, dt=2e-5, eps=0.05):
    """Relaxation of two-component clouds (after Sec. 5.3): `clouds` clouds of
    n_c particles (sigma = 1, T_e = 1e-3, T_i = 1e-5, seeds 0 .. clouds-1)
    advanced together by the batched Verlet step, with the tree (theta = 0.5)
    and with all pairs (theta = 0).  Every `every` steps the electron and ion
    temperatures T_s = m <|v|^2> / 3 (k_B = 1, mean over each cloud's species,
    then over clouds with the spread between clouds) are recorded.  eps = 0.05
    and dt = 2e-5 keep electrons bound in the softened ion wells resolved
    (omega dt = 0.08 for omega^2 = 1836 / eps^3).  Qualitative: the paper's
    physical parameters and figure data are not available."""
    import numpy as np
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import inputs
    from paper_0709_3331_amd.tree import TreeSolver

    cls = [inputs.gaussian_cloud(n_c, 1.0, 1e-3, 1e-5, s) for s in range(clouds)]
    x0 = np.concatenate([c.x for c in cls])
    v0 = np.concatenate([c.v for c in cls])
    q = torch.from_numpy(np.concatenate([c.q for c in cls])).to(dev)
    m = torch.from_numpy(np.concatenate([c.m for c in cls])).to(dev)
    off = torch.arange(0, clouds + 1, device=dev, dtype=torch.int64) * n_c
    n = clouds * n_c
    ion = (q > 0).reshape(clouds, n_c)

    def temps(v):
        k2 = (m * (v * v).sum(dim=1) / 3.0).reshape(clouds, n_c)
        te = (k2 * (~ion)).sum(dim=1) / (~ion).sum(dim=1)
        ti = (k2 * ion).sum(dim=1) / ion.sum(dim=1)
        return te.cpu().numpy(), ti.cpu().numpy()

    def run(theta):
        ts = TreeSolver(n, clouds, curve=CURVE, theta=theta, eps=eps, precision=L.UCP_SPLIT)
        x = torch.from_numpy(x0.copy()).to(dev)
        v = torch.from_numpy(v0.copy()).to(dev)
        f = ts.tree_forces(x, q, off)
        rows = []
        t0 = time.perf_counter()
        for k in range(steps // every + 1):
            if k:
                ts.step(x, v, f, q, m, dt, every, off)
            te, ti = temps(v)
            rows.append({"t": k * every * dt, "T_e": float(te.mean()), "T_e_spread": float(te.std()),
                         "T_i": float(ti.mean()), "T_i_spread": float(ti.std())})
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ts.stats()
        ts.close()
        print(f"relaxation study: theta={theta:g} done, {wall:.1f} s", file=sys.stderr, flush=True)
        return rows, wall

    tree, wt = run(0.5)
    pairs, wp = run(0.0)
    return {"study": "relaxation (Sec. 5.3)", "clouds": clouds, "n_per_cloud": n_c, "eps": eps,
            "dt": dt, "steps": steps, "record_every": every,
            "tree_theta_0.5": {"wall_s": wt, "series": tree},
            "all_pairs": {"wall_s": wp, "series": pairs}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["split", "fp64"], default="split")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--group-size", type=int, default=64)
    ap.add_argument("--list-len", type=int, default=128)
    ap.add_argument("--leaf-cap", type=int, default=24)
    ap.add_argument("--walk-waves", type=int, default=0)
    ap.add_argument("--group-mode", choices=["node", "chunk"], default="chunk")
    ap.add_argument("--curve", choices=["morton", "hilbert"], default="hilbert",
                    help="order of the keys, and so of the chunk groups")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparator run")
    ap.add_argument("--no-theta-sweep", action="store_true",
                    help="skip the theta = 0.3 / 0.7 accuracy and cost lines")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the batched 64-cloud ensemble measurement")
    ap.add_argument("--ensemble-steps", type=int, default=10)
    ap.add_argument("--no-species", action="store_true",
                    help="skip the per-species pseudo-particle measurement")
    ap.add_argument("--no-other-curve", action="store_true",
                    help="skip the same steps with the other key order")
    ap.add_argument("--no-kelbg", action="store_true",
                    help="skip the Kelbg pair-law measurement")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the differentiable 200-step rollout measurement")
    ap.add_argument("--no-accuracy-target", action="store_true",
                    help="skip the search for the cheapest setting that meets 1e-3 vs direct")
    ap.add_argument("--no-seeds", action="store_true",
                    help="skip the headline steps on the inputs of seeds 1 and 2")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the N = 4,194,304 cloud")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3 (no extras)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--study", choices=["opening", "relaxation"],
                    help="run a study instead of the benchmark and print its JSON line")
    ap.add_argument("--study-dt", type=float, default=1e-6, help="time step of the study")
    ap.add_argument("--workload", choices=["metric", "large", "adjoint", "ensemble"],
                    default="metric",
                    help="metric: the N=524,288 cloud (the benchmark); large: the N=4,194,304 "
                         "cloud (eps=0.002, 10%% hot electrons) under the same step protocol, "
                         "for profiling its build; adjoint: the N=65,536 cloud of the "
                         "differentiable rollout, --steps forward walks and force VJPs timed; "
                         "ensemble: the 64-cloud ensemble, --steps batched steps enqueued "
                         "directly at the autotuner's setting (these two print their own JSON "
                         "line instead of the benchmark's)")
    args = ap.parse_args()
    global CURVE
    CURVE = 1 if args.curve == "hilbert" else 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the method is not "
                          "sharded across GPUs in this build", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0709_3331_amd import _lib as L
    from paper_0709_3331_amd import inputs
    from paper_0709_3331_amd.tree import TreeSolver

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    command = "python bench.py " + " ".join(sys.argv[1:])
    if args.study == "opening":
        print(json.dumps({"command": command, **opening_study(dev, args.study_dt)}), flush=True)
        return
    if args.study == "relaxation":
        print(json.dumps({"command": command, **relaxation_study(dev)}), flush=True)
        return
    if args.workload == "adjoint":
        print(json.dumps({"command": command, **vjp_timing(args, dev)}), flush=True)
        return
    if args.workload == "ensemble":
        print(json.dumps({"command": command, **ensemble_steps(args, dev)}), flush=True)
        return
    cl, prm = inputs.metric(0) if args.workload == "metric" else inputs.large(0)
    n = cl.n
    theta, eps, dt = args.theta, prm["eps"], prm["dt"]
    prec = L.UCP_SPLIT if args.precision == "split" else L.UCP_FP64
    x = torch.from_numpy(cl.x).to(dev)
    v = torch.from_numpy(cl.v).to(dev)
    q = torch.from_numpy(cl.q).to(dev)
    m = torch.from_numpy(cl.m).to(dev)
    gm = L.UCP_GROUP_CHUNK if args.group_mode == "chunk" else L.UCP_GROUP_NODE
    ts = TreeSolver(n, curve=CURVE, theta=theta, eps=eps, precision=prec, group_size=args.group_size,
                    list_len=args.list_len, group_mode=gm, leaf_cap=args.leaf_cap,
                    walk_waves=args.walk_waves)
    print(f"bench: N={n} theta={theta} precision={args.precision}", file=sys.stderr, flush=True)

    # initial forces; interaction counts of one evaluation
    f = ts.tree_forces(x, q)
    st0 = ts.stats()
    for _ in range(args.warmup):
        ts.step(x, v, f, q, m, dt, 1)
    torch.cuda.synchronize()
    print("bench: warmup done", file=sys.stderr, flush=True)

    # the state the timed steps start from, so that the graph replays below
    # advance the same state (the cloud evolves from step to step, and so
    # does the walk's work)
    x0, v0, f0 = x.clone(), v.clone(), f.clone()
    # timed region: exactly K steps, walk kernels bracketed by HIP events on
    # the stream they are launched on
    ts.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ts.step(x, v, f, q, m, dt, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    walk_ms, walk_launches = ts.timing_read()
    balance = wave_balance(ts)
    ts.timing(False)
    st = ts.stats()
    graph = None
    if not args.profile:
        # the same K steps from the same state, replayed from the library's
        # captured graphs (which carry no timing events): one untimed call
        # captures them
        for dst, src in ((x, x0), (v, v0), (f, f0)):
            dst.copy_(src)
        ts.step(x, v, f, q, m, dt, 2)
        for dst, src in ((x, x0), (v, v0), (f, f0)):
            dst.copy_(src)
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        ts.step(x, v, f, q, m, dt, args.steps)
        torch.cuda.synchronize()
        g1 = time.perf_counter()
        graph = (g0, g1)
    # the accuracy figures below refer to the state the timed steps start from
    for dst, src in ((x, x0), (v, v0), (f, f0)):
        dst.copy_(src)
    # The headline times the library's default path for a call of many
    # steps, the replayed graphs; the directly enqueued run of the same steps
    # from the same state carries the HIP events that time the walk (timing
    # on bypasses the graphs), and is reported beside it.  A profiling run
    # has only the direct one.
    direct = {"ms_per_step": 1e3 * (t1 - t0) / args.steps,
              "particles_per_s": n * args.steps / (t1 - t0)}
    elapsed = (graph[1] - graph[0]) if graph else (t1 - t0)
    ms_per_step = 1e3 * elapsed / args.steps
    walk_avg_ms = walk_ms / max(walk_launches, 1)
    inter = st["p2p"] + st["m2p"]
    flops = P2P_FLOPS * st["p2p"] + M2P_FLOPS * st["m2p"]
    achieved = flops / (walk_avg_ms * 1e-3) / 1e12
    peak = PEAK_FP32_TFLOPS if prec == L.UCP_SPLIT else PEAK_FP64_TFLOPS
    result = {
        "metric": "tree-force particles/s & interactions/s at N=512K theta=0.5; rel force err vs FP64",
        "value": n * args.steps / elapsed,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-interactions/f64-accumulate" if prec == L.UCP_SPLIT else "f64",
        "data": "synthetic",
        "config": {"workload": (f"single two-component Gaussian cloud N=524288 (sigma=1, 5% halo "
                                f"shell 2-3 sigma)" if args.workload == "metric" else
                                f"single two-component Gaussian cloud N=4194304 (sigma=1, 10% of "
                                f"electrons hot)") + f", theta={theta:g}, eps={eps:g}, G={args.group_size} "
                               f"({args.group_mode} groups), "
                               f"leaf_cap={args.leaf_cap}, 63-bit {args.curve} keys, one KDK "
                               f"Verlet step dt={dt:g}",
                   "n": n, "theta": theta, "precision": args.precision,
                   "group_size": args.group_size, "group_mode": args.group_mode,
                   "curve": args.curve},
        "path": "hipGraph replay of the step" if graph else "directly enqueued steps",
        "direct_enqueue": direct,
        "interactions_per_s": inter / (walk_avg_ms * 1e-3),
        "interactions_per_particle": inter / n,
        "walk_ms": walk_avg_ms,
        "walk_wave_balance": balance,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": traffic_from_profile(args.precision)},
    }
    note(f"timed steps done, {ms_per_step:.4f} ms per step")
    if not args.profile and not args.no_compare:
        note("SPLIT against the FP64 GPU tree")
        # accuracy against the plain FP64 GPU tree at identical parameters and
        # against the FP64 oracle direct sum on sampled targets
        f_split = ts.tree_forces(x, q)
        ts64 = TreeSolver(n, curve=CURVE, theta=theta, eps=eps, precision=L.UCP_FP64,
                          group_size=args.group_size, list_len=args.list_len, group_mode=gm,
                          leaf_cap=args.leaf_cap, walk_waves=args.walk_waves)
        f64 = ts64.tree_forces(x, q)
        ts64.timing(True)
        torch.cuda.synchronize()
        for _ in range(3):
            ts64.tree_forces(x, q)
        torch.cuda.synchronize()
        w64, c64 = ts64.timing_read()
        a, b = f_split.cpu().numpy(), f64.cpu().numpy()
        result["rel_force_err_vs_fp64_gpu"] = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        result["fp64_walk_ms"] = w64 / max(c64, 1)
        result["split_speedup_walk"] = (w64 / max(c64, 1)) / walk_avg_ms
        ts64.close()
    if not args.profile and not args.no_cpu_baseline:
        import oracle
        note("accuracy against the oracle direct sum")
        xs = x.cpu().numpy()
        qs = cl.q
        fs = ts.tree_forces(x, q).cpu().numpy()
        rng = np.random.default_rng(0)
        tg = np.sort(rng.choice(n, 2048, replace=False))
        fd, _ = oracle.direct_targets(xs, qs, eps, tg)
        result["rel_force_err_vs_direct_sampled"] = float(
            np.linalg.norm(fs[tg] - fd) / np.linalg.norm(fd))
        result["meets_1e-3_vs_direct"] = result["rel_force_err_vs_direct_sampled"] <= 1e-3
        fdn = np.full_like(fs, np.nan)
        fdn[tg] = fd
        result["per_particle_err_vs_direct_sampled"] = per_particle_rel(fs, fdn)
        if not args.no_accuracy_target:
            note("cheapest setting that meets 1e-3 against the direct sum")
            result["accuracy_target"] = bench_accuracy_target(args, prec, x, v, q, m, n, eps, dt,
                                                              tg, fd)
        if not args.no_theta_sweep:
            note("theta sweep")
            # the other opening parameters of the same workload: walk time,
            # interactions per particle, error against the sampled direct sum
            sweep = {}
            for th in (0.3, 0.5, 0.7):
                tt = TreeSolver(n, curve=CURVE, theta=th, eps=eps, precision=prec, group_size=args.group_size,
                                list_len=args.list_len, group_mode=gm, leaf_cap=args.leaf_cap,
                                walk_waves=args.walk_waves)
                ft = tt.tree_forces(x, q)
                tt.timing(True)
                torch.cuda.synchronize()
                for _ in range(3):
                    tt.tree_forces(x, q)
                torch.cuda.synchronize()
                wm, wc = tt.timing_read()
                stt = tt.stats()
                fa = ft.cpu().numpy()
                sweep[f"{th:g}"] = {
                    "walk_ms": wm / max(wc, 1),
                    "interactions_per_particle": (stt["p2p"] + stt["m2p"]) / n,
                    "rel_force_err_vs_direct_sampled":
                        float(np.linalg.norm(fa[tg] - fd) / np.linalg.norm(fd))}
                tt.close()
            result["theta_sweep"] = sweep
        if not args.no_species:
            note("per-sign pseudo-particles")
            # the paper's pseudo-particles (one per sign at its centre of
            # charge, Eq. (5) with delta) against the quadrupole above
            spc = {}
            for th in (0.3, 0.5, 0.7):
                tt = TreeSolver(n, curve=CURVE, theta=th, eps=eps, precision=prec, group_size=args.group_size,
                                list_len=args.list_len, group_mode=gm, leaf_cap=args.leaf_cap,
                                walk_waves=args.walk_waves, expansion=L.UCP_EXPANSION_SPECIES)
                ft = tt.tree_forces(x, q)
                tt.timing(True)
                torch.cuda.synchronize()
                for _ in range(3):
                    tt.tree_forces(x, q)
                torch.cuda.synchronize()
                wm, wc = tt.timing_read()
                stt = tt.stats()
                fa = ft.cpu().numpy()
                spc[f"{th:g}"] = {
                    "walk_ms": wm / max(wc, 1),
                    "interactions_per_particle": (stt["p2p"] + stt["m2p"]) / n,
                    "m2p_per_particle": stt["m2p"] / n,
                    "rel_force_err_vs_direct_sampled":
                        float(np.linalg.norm(fa[tg] - fd) / np.linalg.norm(fd))}
                tt.close()
            result["species_pseudo_particles"] = spc
        note("oracle tree on the host (cpu_baseline)")
        c0 = time.perf_counter()
        ot = oracle.Tree(xs, qs, theta, eps, curve=CURVE, G=args.group_size, group_mode=gm,
                         leaf_cap=args.leaf_cap)
        ro = ot.eval(want_phi=False)
        c1 = time.perf_counter()
        result["rel_force_err_vs_oracle_tree"] = float(
            np.linalg.norm(fs - ro["f"]) / np.linalg.norm(ro["f"]))
        result["per_particle_err_vs_oracle_tree"] = per_particle_rel(fs, ro["f"])
        result["cpu_baseline"] = {
            "value": n / (c1 - c0), "unit": "particles/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": "one full FP64 oracle tree-force evaluation (build + walk, OpenMP over "
                      "groups) of the same N=524288 cloud at the same parameters; %.2f s" % (c1 - c0),
            **cpu_info()}
    if not args.profile and not args.no_other_curve:
        key = "morton_keys" if CURVE == 1 else "hilbert_keys"
        note("the other key order")
        result[key] = bench_other_curve(args, prec, cl, prm, dev)
    if not args.profile and not args.no_kelbg:
        note("Kelbg pair law")
        result["kelbg"] = bench_kelbg(args, prec, x, q, cl, walk_avg_ms)
    if not args.profile and not args.no_seeds:
        note("seed repeats")
        result["seed_repeats"] = bench_seeds(args, prec, dev)
    if not args.profile and not args.no_ensemble:
        result["ensemble"] = bench_ensemble(args, prec, dev)
    if not args.profile and not args.no_large:
        result["large"] = bench_large(args, prec, dev)
    if not args.profile and not args.no_adjoint:
        result["adjoint"] = bench_adjoint(prec, dev)
    if args.calib_copy:
        a = torch.ones(64 << 20, dtype=torch.float32, device=dev)   # 256 MiB
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        result["calib_copy_bytes"] = {"read": a.numel() * 4, "write": b.numel() * 4}
    ts.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
