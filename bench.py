#!/usr/bin/env python3
"""Tree-gravity throughput on one MI355X: particle-steps/s of full
drift-kick-drift steps (keys, sort, permute, topology, moments, walk, kick,
drift) through the C ABI, FP32-mixed grouped walk against the plain FP64
per-particle walk, each at its operating point: the opening angle and
launch shape (leaf size, group size, image split, waves per item, HIP-graph
replay) of paper_1110_4876_amd/operating_points.json, chosen by the
autotuner as the fastest meeting rms force error <= 1e-4 against the FP64
direct sum.  Every run checks that gate again, on targets the autotuner
never saw, at the start and at the end of the timed steps (--tune re-runs
the autotuner instead).

Default workload (the largest one-GPU configuration): 256 independent
shearing-sheet patches (N_p uniform on [2,000, 64,000], optical depth
uniform on [0.2, 1.0], seeds 0..255; radii dN/dR ~ R^-3 on [1, 4] m,
400 kg/m^3, Omega = 1.95e-4 s^-1, 3x3 ghost boxes, quadrupoles,
dt = 1e-3 2 pi / Omega) stepped together, one launch per kernel for all
patches, each step replayed from a captured HIP graph; 50 timed steps.
Other workloads: sheet50k (one patch of 50,000), sheet1m, plummer8m.
Synthetic and seeded.  Prints one JSON line on stdout; diagnostics go to
stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tree-gravity particle-steps/s, FP32-mixed vs FP64 plain, at rms force err ≤1e-4"
RMS_TARGET = 1e-4
# algorithmic work per term (flops; rsqrt counted as one): opening test 9,
# monopole (particle or cell) 20, quadrupole cell 56
FLOP_OPEN, FLOP_MONO, FLOP_QUAD = 9, 20, 56
PEAK_F64 = 78.6e12    # 256 CU x 64 FP64 FMA lanes x 2 flop x 2.4 GHz
PEAK_F32 = 157.3e12   # published, counts packed FP32 (dual FMA per lane)
# sources whose hash keys a stored traffic measurement (walk kernel + node record)
WALK_SRC = {"fp64": ("paper_1110_4876_amd/csrc/k_walk64.hip",
                     "paper_1110_4876_amd/csrc/rb_common.h"),
            "fp32": ("paper_1110_4876_amd/csrc/k_walk32.hip",
                     "paper_1110_4876_amd/csrc/rb_common.h")}
# workload -> (default steps, default warm-up steps)
KNOBS = ("theta", "leaf_size", "group_size", "split_images", "walk_waves")
DEFAULT_STEPS = {"sheet50k": (100, 10), "sheet1m": (10, 2), "plummer8m": (10, 2),
                 "batch256": (50, 5)}
# seed of the targets the accuracy gate is checked on (the autotuner tunes on
# seed 0, so the reported errors come from a sample it never saw)
GATE_SEED = 1000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_1110_4876_amd import inputs
    if name == "sheet50k":
        return (inputs.sheet(50000, seed=0),
                "sheet50k: shearing-sheet patch N=50000, tau=0.5, 3x3 images, quadrupole")
    if name == "sheet1m":
        return (inputs.sheet(1_000_000, seed=0),
                "sheet1m: shearing-sheet patch N=1000000, tau=0.5, 3x3 images, quadrupole")
    if name == "plummer8m":
        return (inputs.plummer(1 << 23, seed=0, b=0.001, quadrupole=True, dt=1e-4),
                "plummer8m: Plummer sphere N=8388608, b=0.001, open, quadrupole")
    if name == "batch256":
        return (inputs.batch(256, seed0=0),
                "batch256: 256 shearing-sheet patches, N_p ~ U{2000..64000}, "
                "tau_p ~ U(0.2, 1.0), 3x3 images, quadrupole")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(system, theta, seconds):
    """The oracle (FP64, insertion build, OpenMP walk) on a bounded sample."""
    import numpy as np
    import oracle
    pr0 = system.problems[0]
    if system.batch:
        # whole patches, one after another, full DKD steps
        done, t0 = 0, time.perf_counter()
        k = 0
        while True:
            pr = system.problems[k % len(system.problems)]
            op = oracle.make_params(**dict(pr.params, theta=theta))
            oracle.step(op, pr.state(), pr.m, 0.0, pr.dt, 1, use_tree=True)
            done += pr.n
            k += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
        return {"value": done / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(),
                "kind": "oracle",
                "sample": f"one full DKD step of each of the first {k} patches "
                          f"({done} particle-steps), theta={theta}"}
    if system.n <= 200_000:
        op = oracle.make_params(**dict(pr0.params, theta=theta))
        st = pr0.state()
        steps, t0 = 0, time.perf_counter()
        while True:
            st = oracle.step(op, st, pr0.m, steps * pr0.dt, pr0.dt, 1, use_tree=True)
            steps += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
        return {"value": system.n * steps / dt, "unit": "particle-steps/s",
                "cores": oracle.num_threads(), "kind": "oracle",
                "sample": f"{steps} full DKD steps of the same {system.n}-particle system "
                          f"with the oracle tree walk at theta={theta}"}
    # large systems: one tree build, then the walk for a sample of targets;
    # a step is estimated as build + walk time scaled to all particles
    op = oracle.make_params(**dict(pr0.params, theta=theta))
    t0 = time.perf_counter()
    tree = oracle.Tree(op, pr0.x, pr0.y, pr0.z, pr0.m, pr0.n_active)
    t_build = time.perf_counter() - t0
    k = 4096
    tg = np.sort(np.random.default_rng(1).choice(system.n, size=k, replace=False))
    t1 = time.perf_counter()
    tree.walk(s=0.0, targets=tg)
    t_walk = time.perf_counter() - t1
    per_step = t_build + t_walk * system.n / k
    return {"value": system.n / per_step, "unit": "particle-steps/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one oracle tree build ({t_build:.1f} s) plus the walk for {k} sampled "
                      f"targets ({t_walk:.2f} s), scaled to one step of all {system.n} "
                      f"particles, theta={theta}"}


def walk_source_sha(path):
    h = hashlib.sha256()
    for f in WALK_SRC[path]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def walk_kernel_name(path, walk_waves):
    if path == "fp64":
        return "k_walk64"
    return "k_walk32m" if walk_waves and walk_waves > 1 else "k_walk32"


def write_traffic(args, out_dir=None):
    """Turn four rocprofv3 --pmc runs (FETCH_SIZE and WRITE_SIZE, KiB per
    dispatch, for a plain device copy of known size and for the walk at the
    operating point given by the knob options) into HBM bytes per walk
    launch: each walk counter is scaled by true bytes / counter reading of
    the copy.  Writes walk_<path>_<workload>_traffic.json in out_dir
    (profiles/ by default) and returns the entry."""
    import csv
    import glob

    def values(d, counter, pat):
        out = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter and pat in r["Kernel_Name"]:
                        out.append(float(r["Counter_Value"]))
        if not out:
            raise SystemExit(f"no {counter} rows for {pat} under {d}")
        return out

    cf, cw, wf, ww = args.write_traffic
    path = args.precision if args.precision != "both" else "fp32"
    copy_bytes = (args.calibrate_copy or 512) << 20
    c_f = values(cf, "FETCH_SIZE", "copyBuffer")
    c_w = values(cw, "WRITE_SIZE", "copyBuffer")
    kname = walk_kernel_name(path, args.walk_waves)
    # the timed launches only: quadrupole on, interaction counters off (the
    # FP64 walk's name goes on with its schedule and record addressing)
    if kname == "k_walk64":
        full = "k_walk64<true, false, "
    elif kname == "k_walk32m":
        full = f"k_walk32m<true, false, {args.walk_waves}>"
    else:
        full = "k_walk32<true, false>"
    w_f = values(wf, "FETCH_SIZE", full)
    w_w = values(ww, "WRITE_SIZE", full)
    mean = lambda v: sum(v) / len(v)
    # the median over the launches: the steps' walks (the odd one at another
    # opening angle, for the theta 0.5 errors, does not move it)
    med = lambda v: sorted(v)[len(v) // 2]
    fs = copy_bytes / 1024 / mean(c_f)
    ws = copy_bytes / 1024 / mean(c_w)
    knobs = {"theta": args.theta, "leaf_size": args.leaf_size,
             "group_size": args.group_size, "split_images": args.split_images,
             "walk_waves": args.walk_waves}
    if path == "fp64":  # no groups or waves per item
        knobs["group_size"], knobs["walk_waves"] = None, None
    meta = {
        "kernel": kname, "workload": args.workload, "knobs": knobs,
        "sources": list(WALK_SRC[path]), "source_sha256": walk_source_sha(path),
        "kernel_instance": full,
        "fetch_kib_per_dispatch_raw": med(w_f), "write_kib_per_dispatch_raw": med(w_w),
        "fetch_kib_min_max": [min(w_f), max(w_f)], "write_kib_min_max": [min(w_w), max(w_w)],
        "copy_calibration": {"copy_bytes": copy_bytes, "fetch_kib_raw": mean(c_f),
                             "write_kib_raw": mean(c_w), "fetch_scale": fs, "write_scale": ws},
        "fetch_bytes_per_launch": med(w_f) * 1024 * fs,
        "write_bytes_per_launch": med(w_w) * 1024 * ws,
        "dispatches": len(w_f),
    }
    meta["bytes_per_launch"] = meta["fetch_bytes_per_launch"] + meta["write_bytes_per_launch"]
    out = os.path.join(out_dir or os.path.join(ROOT, "profiles"),
                       f"walk_{path}_{args.workload}_traffic.json")
    # one entry per operating point: a new measurement replaces the entry of
    # the same knobs
    entries = traffic_entries(out)
    entries = [e for e in entries if e.get("knobs") != meta["knobs"]] + [meta]
    with open(out, "w") as fh:
        json.dump({"entries": entries}, fh, indent=1)
    print(json.dumps(meta))
    return meta


def traffic_entries(path):
    """The stored walk traffic measurements of a file (none if absent)."""
    if not os.path.exists(path):
        return []
    d = json.load(open(path))
    return d["entries"] if "entries" in d else [d]


def build_traffic(args):
    """Turn rocprofv3 --pmc runs over every kernel of a bench run (FETCH_SIZE
    and WRITE_SIZE, plus the copy calibration runs) into HBM bytes per step
    of the build kernels: the dispatches between the walks of the second and
    the sixth timed step (four whole steps inside the timed call; a run of
    --warmup 1 --steps 6 or longer has them) grouped by kernel, each
    kernel's sum scaled by the copy's true bytes / counter reading and
    divided by the steps.  Prints one JSON object."""
    import csv
    import glob
    cf, cw, af, aw = args.build_traffic
    copy_bytes = (args.calibrate_copy or 512) << 20

    def rows(d, counter):
        out = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r["Counter_Name"] == counter:
                        out.append((int(r["Dispatch_Id"]), r["Kernel_Name"].split("(")[0]
                                    .replace("void ", ""), float(r["Counter_Value"])))
        return sorted(out)

    mean = lambda v: sum(v) / len(v)
    scale = {}
    for c, d in (("FETCH_SIZE", cf), ("WRITE_SIZE", cw)):
        v = [x for _, k, x in rows(d, c) if "copyBuffer" in k]
        scale[c] = copy_bytes / 1024 / mean(v)
    per_kernel = {}
    steps = None
    for c, d in (("FETCH_SIZE", af), ("WRITE_SIZE", aw)):
        rs = rows(d, c)

        def timed_walk(k):  # a walk launch without the interaction counters
            if not k.startswith("k_walk") or "<" not in k:
                return False
            targs = k[k.index("<") + 1:k.rindex(">")].split(", ")
            return len(targs) > 1 and targs[1] == "false"
        # walks: the first force evaluation (accuracy gate), the warm-up
        # step(s), then the timed steps
        walks = [i for i, (_, k, _) in enumerate(rs) if timed_walk(k)]
        lo, hi = walks[3], walks[7]
        window = rs[lo:hi]
        steps = 4
        for _, k, x in window:
            if k.startswith("k_walk") or "copyBuffer" in k or "fillBuffer" in k:
                continue
            e = per_kernel.setdefault(k, {"FETCH_SIZE": [], "WRITE_SIZE": []})
            e[c].append(x * 1024 * scale[c])
    out = {"steps": steps, "kernels": {}}
    tot = 0.0
    for k, e in sorted(per_kernel.items()):
        f = sum(e["FETCH_SIZE"]) / steps
        w = sum(e["WRITE_SIZE"]) / steps
        out["kernels"][k] = {"fetch_bytes_per_step": f, "write_bytes_per_step": w,
                             "dispatches_per_step": len(e["FETCH_SIZE"]) / steps}
        tot += f + w
    out["build_bytes_per_step"] = tot
    out["copy_scale"] = scale
    print(json.dumps(out))


def build_bytes(n, n_nodes, small_sort):
    """Algorithmic HBM bytes of one step's build (keys, sort, permute,
    topology, moments, kick and drift): per particle keys 36, sort 48 (bucket
    sort) or 192 (eight radix passes), permute 128, topology 30, drift and
    kick 96; moments 1.5 x 120 per node."""
    return n * (36 + (48 if small_sort else 192) + 128 + 30 + 96) + 180.0 * n_nodes


def collide_run(args, sysm, wdesc):
    """Collisional sheet: K steps, each one DKD step of FP32-mixed tree
    gravity and then collisions at the end of the step (search of Eq. (3),
    queue in random order, hard-sphere resolution with restitution), timed
    after W such steps from the initial state, so that the initial overlaps
    are gone.  Detector "tree": inside rb_step (rb_set_collisions), on the
    step's own tree, all K steps in one call; "tree-call": rb_collide after
    every one-step rb_step call (its own tree on the end-of-step positions);
    "sweep": rb_sweep likewise.  The search kernel is timed with HIP events
    on the context's stream."""
    import numpy as np
    import torch
    from paper_1110_4876_amd import autotune, rb
    if sysm.batch or "radius" not in sysm.problems[0].extra:
        raise SystemExit("--collide needs a single shearing-sheet workload with radii")
    pr = sysm.problems[0]
    n, dt = sysm.n, sysm.dt
    if args.theta:
        knobs = dict(theta=args.theta, leaf_size=args.leaf_size, group_size=args.group_size,
                     split_images=args.split_images, walk_waves=args.walk_waves)
    else:
        t_kick = 0.5 * dt
        tg = sysm.sample_targets(4096, 16, seed=0)
        cfg = autotune.tune(sysm, sysm.direct(tg, t_kick), tg, t_kick,
                            precision=rb.RB_FP32_MIXED, rms_target=RMS_TARGET, log=log)
        knobs = {k: cfg[k] for k in KNOBS}
    R = torch.as_tensor(pr.extra["radius"], dtype=torch.float64, device="cuda")
    eps = args.epsilon
    sweep = args.detector == "sweep"
    in_step = args.detector == "tree"

    def run(profile):
        ctx = sysm.create(rb.RB_FP32_MIXED, profile=profile, **knobs)
        try:
            X = sysm.clone()
            if in_step:
                rb.rb_set_collisions(ctx, R, eps, 1000)
                sysm.step(ctx, X, 0.0, args.warmup)
                rb.rb_sync(ctx)
                rb.rb_collision_counts(ctx)
                rb.rb_stats(ctx)  # discard warm-up timers
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sysm.step(ctx, X, args.warmup * dt, args.steps)
                torch.cuda.synchronize()
                secs = time.perf_counter() - t0
                pairs, resolved = rb.rb_collision_counts(ctx)
            else:
                def collide(k):
                    if sweep:
                        return rb.rb_sweep(ctx, sysm.parts(X), R, n, (k + 1) * dt, dt, eps,
                                           1000 + k)
                    return rb.rb_collide(ctx, sysm.parts(X), R, n, (k + 1) * dt, eps, 1000 + k)
                for k in range(args.warmup):
                    sysm.step(ctx, X, k * dt, 1)
                    collide(k)
                rb.rb_sync(ctx)
                rb.rb_stats(ctx)  # discard warm-up timers
                pairs = resolved = 0
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for k in range(args.warmup, args.warmup + args.steps):
                    sysm.step(ctx, X, k * dt, 1)
                    a, b = collide(k)
                    pairs += a
                    resolved += b
                torch.cuda.synchronize()
                secs = time.perf_counter() - t0
            s = rb.rb_stats(ctx)
            if sweep:
                n_nodes, n_live = 0, n
            else:
                rb.rb_tree_build(ctx, sysm.parts(X), n, n)  # (the node count of the end state)
                n_nodes, n_live = rb.rb_tree_info(ctx)
        finally:
            rb.rb_destroy(ctx)
        return secs, pairs, resolved, s, n_nodes, n_live

    # the timed run records no HIP events; a second run of the same steps
    # times the walk and the search kernels with events around them
    secs, pairs, resolved, _, n_nodes, n_live = run(0)
    _, pairs2, resolved2, s, _, _ = run(4)
    if (pairs2, resolved2) != (pairs, resolved):
        raise SystemExit(f"collision counts differ between two identical runs: "
                         f"{(pairs, resolved)} vs {(pairs2, resolved2)}")
    search_ms = s["ms"]["coll_search"] / max(1, s["calls"]["coll_search"])
    walk_ms = s["ms"]["walk"] / max(1, s["calls"]["walk"])
    # algorithmic bytes of one search.  Tree: every live particle's position,
    # radius and caller index read once (36 B), every cell record once
    # (32 B), every found pair written once (8 B).  Sweep: every particle's
    # sorted record read once (position, velocity, radius, interval end,
    # key, caller index: 76 B), every found pair written once (8 B).
    if sweep:
        algo = 76 * n_live + 8 * pairs / args.steps
    else:
        algo = 36 * n_live + 32 * n_nodes + 8 * pairs / args.steps
    achieved = algo / (search_ms * 1e-3)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        op = oracle.make_params(**dict(pr.params, theta=knobs["theta"]))
        st = pr.state()
        radius = np.asarray(pr.extra["radius"], dtype=np.float64)
        k, c0 = 0, time.perf_counter()
        while True:
            st = oracle.step(op, st, pr.m, k * dt, dt, 1, use_tree=True)
            if sweep:
                _, _, _, st = oracle.sweep(op, st, pr.m, radius, (k + 1) * dt, dt, eps,
                                           1000 + k)
            else:
                _, _, _, st = oracle.collide(op, st, pr.m, radius, (k + 1) * dt, eps, 1000 + k)
            k += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        cs = time.perf_counter() - c0
        cpu = {"value": n * k / cs, "unit": "particle-steps/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{k} collisional steps of the same {n}-particle sheet from the "
                         f"initial state (oracle tree gravity at theta={knobs['theta']}, "
                         f"brute-force {'trajectory' if sweep else 'overlap'} search, "
                         f"sequential queue)"}
    out = {
        "metric": "collisional-sheet particle-steps/s (FP32-mixed tree gravity DKD step + "
                  f"FP64 {'plane-sweep' if sweep else 'tree'} collision search and resolution)",
        "collision_path": {"tree": "inside rb_step, on the step's own tree",
                           "tree-call": "rb_collide after every step, own tree",
                           "sweep": "rb_sweep after every step"}[args.detector],
        "value": n * args.steps / secs,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wdesc + ", collisions at the end of every step, "
                   f"epsilon={eps}", "n": n, "images": 9, "detector": args.detector, **knobs},
        "collisions": {"pairs_per_step": pairs / args.steps,
                       "resolved_per_step": resolved / args.steps,
                       "search_ms": search_ms, "walk_ms": walk_ms,
                       "tree_nodes": n_nodes if not sweep else None},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": achieved / 8e12, "traffic": None,
                     "kernel": "k_sw_gather + k_sw_pairs" if sweep else "k_coll_detect"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def sweep_ring_run(args):
    """A narrow ring of 50,000 colliding particles around the origin (optical
    depth 0.5, width 0.01 of the radius, open box): K calls of rb_sweep along
    the azimuth over one time-step (detection and resolution), after W
    untimed calls; the x sweep and the tree search (rb_collide) timed the
    same way on the same state."""
    import numpy as np
    import torch
    from paper_1110_4876_amd import inputs, rb
    from paper_1110_4876_amd.system import System
    pr = inputs.ring(50000, seed=0)
    sysm = System(pr)
    n, dt = pr.n, pr.dt
    R = torch.as_tensor(pr.extra["radius"], dtype=torch.float64, device="cuda")
    steps = args.steps
    warm = args.warmup

    def run(kind, profile):
        ctx = sysm.create(rb.RB_FP64, profile=profile)
        try:
            X = sysm.clone()

            def call(k):
                if kind == "tree":
                    return rb.rb_collide(ctx, sysm.parts(X), R, n, 0.0, 0.5, 1000 + k)
                axis = rb.RB_SWEEP_PHI if kind == "phi" else rb.RB_SWEEP_X
                return rb.rb_sweep(ctx, sysm.parts(X), R, n, 0.0, dt, 0.5, 1000 + k,
                                   axis=axis)
            for k in range(warm):
                call(k)
            rb.rb_sync(ctx)
            rb.rb_stats(ctx)
            pairs = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for k in range(warm, warm + steps):
                pairs += call(k)[0]
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            s = rb.rb_stats(ctx)
        finally:
            rb.rb_destroy(ctx)
        return (secs, pairs / steps,
                s["ms"]["coll_search"] / max(1, s["calls"]["coll_search"]))
    # the timed runs record no HIP events; a second run of each times the
    # search kernels with events around them
    res = {}
    for k in ("phi", "x", "tree"):
        secs_k, pairs_k, _ = run(k, 0)
        res[k] = (secs_k, pairs_k, run(k, 4)[2])
    secs, pairs, search_ms = res["phi"]
    algo = 76 * n + 8 * pairs
    achieved = algo / (search_ms * 1e-3)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        op = oracle.make_params(**pr.params)
        radius = np.asarray(pr.extra["radius"], dtype=np.float64)
        k, c0 = 0, time.perf_counter()
        while True:
            oracle.sweep(op, pr.state(), pr.m, radius, 0.0, dt, 0.5, 1000 + k)
            k += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        cs = time.perf_counter() - c0
        cpu = {"value": n * k / cs, "unit": "particles/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"{k} calls of the oracle's trajectory collision search "
                         f"(brute force over all pairs) with resolution on the same ring"}
    out = {
        "metric": "ring collision-search particles/s (azimuthal plane sweep over one "
                  "time-step, FP64, with resolution)",
        "value": n * steps / secs,
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": secs * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ring50k: narrow ring N=50000 around the origin, tau=0.5, "
                               "width 0.01 r0, open box, dt = 1e-3 orbital period",
                   "n": n},
        "pairs_per_call": pairs,
        "compare_ms_per_call": {k: v[0] * 1e3 / steps for k, v in res.items()},
        "search_ms": {k: v[2] for k, v in res.items()},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": achieved / 8e12, "traffic": None,
                     "kernel": "k_sw_gather + k_sw_pairs_phi"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="batch256", choices=sorted(DEFAULT_STEPS))
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "fp32"])
    ap.add_argument("--theta", type=float, default=None,
                    help="fix theta (and the options below) instead of the workload's "
                         "operating point")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the operating point (leaf, group, image split, waves, "
                         "launch mode, theta) instead of taking it from "
                         "paper_1110_4876_amd/operating_points.json")
    ap.add_argument("--leaf-size", type=int, default=1)
    ap.add_argument("--group-size", type=int, default=64)
    ap.add_argument("--split-images", type=int, default=-1)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--walk-waves", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (the known-size "
                         "kernel that scales the HBM byte counters) and exit")
    ap.add_argument("--collide", action="store_true",
                    help="the collisional sheet instead: every step is a DKD step with "
                         "FP32-mixed tree gravity followed by the tree collision search and "
                         "hard-sphere resolution at the end of the step (own JSON line)")
    ap.add_argument("--epsilon", type=float, default=0.5,
                    help="coefficient of restitution of the collisional sheet")
    ap.add_argument("--detector", default="tree", choices=["tree", "tree-call", "sweep"],
                    help="collision detection of the collisional sheet: the octree search "
                         "inside rb_step on the step's own tree (tree), the same search as a "
                         "call after every step that builds its own tree (tree-call), or the "
                         "plane sweep along x over the step's trajectories (sweep)")
    ap.add_argument("--sweep-ring", action="store_true",
                    help="collision search on a narrow ring around the origin (50,000 "
                         "particles, open box): the azimuthal plane sweep, timed per call, "
                         "with the x sweep and the tree search on the same state beside it "
                         "(own JSON line)")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure this GPU's FP32 (unpacked) and FP64 FMA rates and "
                         "its streaming-copy HBM rate, print them as JSON and exit")
    ap.add_argument("--build-traffic", nargs=4, default=None,
                    metavar=("COPY_FETCH", "COPY_WRITE", "ALL_FETCH", "ALL_WRITE"),
                    help="only turn rocprofv3 --pmc folders of the copy calibration and of "
                         "a bench run over every kernel into the build's HBM bytes per step "
                         "(runs without a GPU) and exit")
    ap.add_argument("--write-traffic", nargs=4, default=None,
                    metavar=("COPY_FETCH", "COPY_WRITE", "WALK_FETCH", "WALK_WRITE"),
                    help="only turn four rocprofv3 --pmc output folders into the stored "
                         "walk traffic for the knobs given (runs without a GPU) and exit")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args)
        return
    if args.build_traffic:
        build_traffic(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    steps_d, warm_d = DEFAULT_STEPS[args.workload]
    args.steps = steps_d if args.steps is None else args.steps
    args.warmup = warm_d if args.warmup is None else args.warmup

    import torch
    from paper_1110_4876_amd import autotune, rb
    from paper_1110_4876_amd.metrics import force_errors
    from paper_1110_4876_amd.system import System

    torch.cuda.set_device(0)
    if args.peaks:
        f32, f64, hbm = (rb.rb_peak_probe(k) for k in (0, 1, 2))
        print(json.dumps({"fp32_unpacked_tflops": f32 / 1e12, "fp64_tflops": f64 / 1e12,
                          "hbm_copy_tbps": hbm / 1e12,
                          "published": {"fp32_packed_tflops": PEAK_F32 / 1e12,
                                        "fp64_tflops": PEAK_F64 / 1e12, "hbm_tbps": 8.0}}))
        return
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_read_bytes": nbytes, "copy_write_bytes": nbytes, "launches": 5}))
        return
    if args.sweep_ring:
        sweep_ring_run(args)
        return
    prob, wdesc = workload(args.workload)
    sysm = System(prob)
    n = sysm.n
    if args.collide:
        collide_run(args, sysm, wdesc)
        return
    gravity_run(args, sysm, wdesc)


def gravity_run(args, sysm, wdesc):
    """The headline: K timed DKD steps of each path (FP32-mixed and plain
    FP64) at its operating point, with the accuracy gate checked on an
    independent sample of targets at the start and at the end of the run."""
    import torch
    from paper_1110_4876_amd import autotune, rb
    from paper_1110_4876_amd.metrics import force_errors
    n = sysm.n
    t_kick = 0.5 * sysm.dt
    quad = bool(sysm.params["quadrupole"])
    # the gate sample: 4096 targets (16 per patch of a batch), drawn with a
    # seed the autotuner never sees, so the reported errors are not biased
    # by the selection of the operating point
    tg = sysm.sample_targets(4096, 16, seed=GATE_SEED)
    log(f"[{args.workload}] n={n}, {len(tg)} gate targets; FP64 direct-sum reference")
    ref = sysm.direct(tg, t_kick)

    def errors_at(prec, knobs, X, t, r):
        ctx = sysm.create(prec, **knobs)
        try:
            return force_errors(sysm.gravity(ctx, t, X).cpu().numpy()[tg], r)
        finally:
            rb.rb_destroy(ctx)

    def interactions(theta, t=None, X=None):
        """per-particle FP64 walk counts at theta, leaf 1 (the algorithmic work)"""
        ctx = sysm.create(rb.RB_FP64, theta=theta, leaf_size=1, profile=2)
        try:
            sysm.gravity(ctx, t_kick if t is None else t, X)
            s = rb.rb_stats(ctx)
            s["n_nodes"] = rb.rb_tree_info(ctx)[0]
        finally:
            rb.rb_destroy(ctx)
        flops = (FLOP_OPEN * s["open_tests"] + FLOP_MONO * s["pp"] +
                 (FLOP_QUAD if quad else FLOP_MONO) * s["cells"])
        return s, flops

    def executed(knobs, t=None, X=None):
        """the grouped FP32 walk's own evaluated list entries (all lanes)"""
        ctx = sysm.create(rb.RB_FP32_MIXED, profile=2, **knobs)
        try:
            sysm.gravity(ctx, t_kick if t is None else t, X)
            s = rb.rb_stats(ctx)
        finally:
            rb.rb_destroy(ctx)
        return s

    def simpson(a, m, b, keys):
        """the mean over the run of a count that varies smoothly, from its
        values at the start, the middle and the end (Simpson's rule)"""
        return {k: (a[k] + 4 * m[k] + b[k]) / 6 for k in keys}

    k_mid = args.steps // 2

    def timed(prec, knobs, use_graph, profile, mid=False):
        """warm-up, then exactly K steps from the initial state: in one call,
        or (mid) in two halves with a copy of the state between them"""
        ctx = sysm.create(prec, use_graph=use_graph, profile=profile, **knobs)
        M = None
        try:
            W = sysm.clone()
            sysm.step(ctx, W, 0.0, args.warmup)
            rb.rb_sync(ctx)
            rb.rb_stats(ctx)  # discard warm-up timers
            T = sysm.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if mid:
                sysm.step(ctx, T, 0.0, k_mid)
                M = {k: v.clone() for k, v in T.items()}
                sysm.step(ctx, T, k_mid * sysm.dt, args.steps - k_mid)
            else:
                sysm.step(ctx, T, 0.0, args.steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rb.rb_sync(ctx)
            s = rb.rb_stats(ctx)
        finally:
            rb.rb_destroy(ctx)
        return t1 - t0, s, T, M

    results = {}
    paths = ["fp64", "fp32"] if args.precision == "both" else [args.precision]
    for path in paths:
        prec = rb.RB_FP64 if path == "fp64" else rb.RB_FP32_MIXED
        source = "fixed"
        try:
            if args.theta:
                cfg = dict(theta=args.theta, leaf_size=args.leaf_size,
                           group_size=args.group_size, split_images=args.split_images,
                           walk_waves=args.walk_waves, use_graph=args.graph)
                source = "command line"
            elif args.tune:
                # tuned on its own sample (seed 0) and on a state from late in
                # a run as long as the timed one
                c0 = time.perf_counter()
                tg0 = sysm.sample_targets(4096, 16, seed=0)
                late = sysm.clone()
                ctx = sysm.create(rb.RB_FP64, theta=0.3)
                try:
                    sysm.step(ctx, late, 0.0, args.steps)
                    rb.rb_sync(ctx)
                finally:
                    rb.rb_destroy(ctx)
                t_late = (args.steps + 0.5) * sysm.dt
                checks = [(late, t_late, sysm.direct(tg0, t_late, late))]
                cfg = autotune.tune(sysm, sysm.direct(tg0, t_kick), tg0, t_kick, precision=prec,
                                    rms_target=RMS_TARGET, log=log, checks=checks)
                source = "autotuned"
                log(f"[{path}] tuned in {time.perf_counter() - c0:.1f} s")
            else:
                cfg = autotune.operating_point(args.workload, path)
            knobs = {k: cfg[k] for k in KNOBS}
            err = errors_at(prec, knobs, None, t_kick, ref)
            # the gate on the independent sample; a fixed point that misses
            # it steps down the autotuner's grid of opening angles
            tries = 0
            while err["rms"] > RMS_TARGET and source != "command line" and tries < 4:
                lower = [th for th in autotune.THETAS if th < knobs["theta"]]
                if not lower:
                    break
                log(f"[{path}] theta {knobs['theta']} misses the gate on the independent "
                    f"sample (rms {err['rms']:.3e}); trying {lower[0]}")
                knobs["theta"] = lower[0]
                source += ", lowered to meet the gate"
                err = errors_at(prec, knobs, None, t_kick, ref)
                tries += 1
            cfg.update(knobs)
        except (rb.RBError, RuntimeError) as ex:
            log(f"[{path}] unavailable: {ex}")
            continue
        use_graph = int(cfg.get("use_graph", 0))
        log(f"[{path}] theta={knobs['theta']} leaf={knobs['leaf_size']} "
            f"group={knobs['group_size']} split={knobs['split_images']} "
            f"waves={knobs['walk_waves']} graph={use_graph} ({source}): "
            f"rms={err['rms']:.3e} max={err['max']:.3e}")
        st0, flops0 = interactions(knobs["theta"])
        # The timed run records no HIP events (an event between two kernels
        # costs a few microseconds of idle GPU); the walk launches are timed
        # in a second, eager pass of the same K steps with HIP events around
        # every walk launch on the context's stream.
        secs, _, T, _ = timed(prec, knobs, use_graph, 0)
        _, s2, _, M = timed(prec, knobs, 0, 4, mid=k_mid > 0)
        if M is None:
            M = sysm.clone()
        t_mid = k_mid * sysm.dt + t_kick
        t_end = args.steps * sysm.dt + t_kick
        err_end = errors_at(prec, knobs, T, t_end, sysm.direct(tg, t_end, T))
        # The system evolves over the timed steps (a sheet's particles settle
        # into denser wakes) and a walk late in the run does more work than
        # an early one: the work of the timed walks is the mean of the counts
        # over the run, by Simpson's rule from the start, the middle and the
        # end of the run.
        stm, flopsm = interactions(knobs["theta"], t_mid, M)
        st1, flops1 = interactions(knobs["theta"], t_end, T)
        st = simpson(st0, stm, st1, ("open_tests", "cells", "pp", "n_nodes"))
        flops = (flops0 + 4 * flopsm + flops1) / 6
        if path == "fp32":
            ex = simpson(executed(knobs), executed(knobs, t_mid, M), executed(knobs, t_end, T),
                         ("list_cells", "list_pp"))
        del T, M
        # the nominal opening angle 0.5, same launch shape, initial state
        err_05 = errors_at(prec, dict(knobs, theta=0.5), None, t_kick, ref)
        ms_step = secs * 1e3 / args.steps
        walk_ms = s2["ms"]["walk"] / max(1, s2["calls"]["walk"])
        gate_ok = err["rms"] <= RMS_TARGET and err_end["rms"] <= RMS_TARGET
        r = dict(theta=knobs["theta"], leaf_size=knobs["leaf_size"],
                 group_size=knobs["group_size"] if path == "fp32" else None,
                 split_images=knobs["split_images"], use_graph=use_graph,
                 walk_waves=knobs["walk_waves"] if path == "fp32" else None,
                 operating_point=source,
                 errors=err, errors_end_of_run=err_end, accuracy_gate_met=gate_ok,
                 errors_at_theta_0_5=err_05, ms_per_step=ms_step,
                 particle_steps_per_s=n * args.steps / secs,
                 walk_ms=walk_ms, walk_launches=s2["calls"]["walk"],
                 interactions=dict(open_tests=st["open_tests"], cells=st["cells"],
                                   pp=st["pp"],
                                   note="mean over the timed run: Simpson's rule from the "
                                        "counts at its start, middle and end"),
                 interactions_start=dict(open_tests=st0["open_tests"], cells=st0["cells"],
                                         pp=st0["pp"]),
                 interactions_middle=dict(open_tests=stm["open_tests"], cells=stm["cells"],
                                          pp=stm["pp"]),
                 interactions_end_of_run=dict(open_tests=st1["open_tests"],
                                              cells=st1["cells"], pp=st1["pp"]),
                 algorithmic_flops_per_walk=flops,
                 algorithmic_tflops=flops / (walk_ms * 1e-3) / 1e12,
                 interactions_per_s=(st["cells"] + st["pp"]) / (walk_ms * 1e-3))
        if path == "fp32":
            ex_flops = (FLOP_QUAD if quad else FLOP_MONO) * ex["list_cells"] + \
                FLOP_MONO * ex["list_pp"]
            r["executed"] = dict(list_cells=ex["list_cells"], list_pp=ex["list_pp"],
                                 flops_per_walk=ex_flops,
                                 tflops=ex_flops / (walk_ms * 1e-3) / 1e12,
                                 interactions_per_s=(ex["list_cells"] + ex["list_pp"]) /
                                 (walk_ms * 1e-3),
                                 note="terms the grouped walk evaluates (every member of "
                                      "a group against its shared list), beside the "
                                      "per-particle algorithmic counts")
        # the build (everything but the walk) against HBM: algorithmic bytes
        # over the step time the walk leaves
        b_ms = ms_step - walk_ms
        b_bytes = build_bytes(n, st["n_nodes"], sysm_small_sort(sysm))
        r["build"] = dict(ms_per_step=b_ms, algorithmic_bytes=b_bytes,
                          achieved_GBps=b_bytes / (b_ms * 1e-3) / 1e9,
                          frac_of_hbm=b_bytes / (b_ms * 1e-3) / 8e12)
        results[path] = r
        log(f"[{path}] {ms_step:.3f} ms/step, walk {walk_ms:.3f} ms, "
            f"{r['particle_steps_per_s']:.3e} particle-steps/s, end-of-run rms "
            f"{err_end['rms']:.3e}, theta 0.5 rms {err_05['rms']:.3e}")

    if not results:
        raise SystemExit("no path produced a result")
    main_path = "fp32" if "fp32" in results else "fp64"
    r = results[main_path]
    peak = PEAK_F32 if main_path == "fp32" else PEAK_F64
    achieved = r["algorithmic_flops_per_walk"] / (r["walk_ms"] * 1e-3)
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"walk_{main_path}_{args.workload}_traffic.json")
    # only for the same kernel sources at the same operating point
    knobs = {k: r[k] for k in KNOBS}
    for meta in traffic_entries(tf):
        if (meta.get("source_sha256") == walk_source_sha(main_path) and
                meta.get("knobs") == knobs):
            traffic = meta.get("bytes_per_launch")
    traffic64 = None
    if "fp64" in results:
        knobs64 = {k: results["fp64"][k] for k in KNOBS}
        tf64 = os.path.join(ROOT, "profiles", f"walk_fp64_{args.workload}_traffic.json")
        for meta in traffic_entries(tf64):
            if (meta.get("source_sha256") == walk_source_sha("fp64") and
                    meta.get("knobs") == knobs64):
                traffic64 = meta.get("bytes_per_launch")
    if main_path == "fp64":
        traffic = traffic64
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                "kernel": walk_kernel_name(main_path, r["walk_waves"])}
    if "fp64" in results:
        r64 = results["fp64"]
        a64 = r64["algorithmic_flops_per_walk"] / (r64["walk_ms"] * 1e-3)
        r64["roofline"] = {"bound": "alu", "achieved": a64 / 1e12, "peak": PEAK_F64 / 1e12,
                           "unit": "TFLOP/s", "frac": a64 / PEAK_F64, "traffic": traffic64,
                           "kernel": walk_kernel_name("fp64", 1)}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sysm, r["theta"], args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": r["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if main_path == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": wdesc, "n": n, "patches": len(sysm.problems),
                   "images": 9 if sysm.params["boundary"] else 1,
                   "path": main_path, "theta": r["theta"], "quadrupole": quad,
                   "leaf_size": r["leaf_size"], "group_size": r["group_size"],
                   "split_images": r["split_images"], "walk_waves": r["walk_waves"],
                   "hip_graph": bool(r["use_graph"]),
                   "gate": f"rms <= {RMS_TARGET:g} vs FP64 direct sum on {len(tg)} targets "
                           f"(seed {GATE_SEED}) at the start and the end of the run"},
        "paths": results,
        "roofline": roofline,
        "build": r["build"],
        "cpu_baseline": cpu,
    }
    if "fp64" in results and "fp32" in results:
        out["speedup_fp32_vs_fp64"] = (results["fp32"]["particle_steps_per_s"] /
                                       results["fp64"]["particle_steps_per_s"])
    print(json.dumps(out), flush=True)


def sysm_small_sort(sysm):
    """whether every patch takes the bucket sort (at most 2^18 slots)"""
    return max(p.n for p in sysm.problems) <= (1 << 18)


if __name__ == "__main__":
    main()
