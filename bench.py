#!/usr/bin/env python3
"""Tree-gravity throughput on one MI355X: particle-steps/s of full
drift-kick-drift steps (keys, sort, permute, topology, moments, walk, kick,
drift) through the C ABI, FP32-mixed grouped walk against the plain FP64
per-particle walk, each at the largest opening angle whose rms force error
against the FP64 direct sum is <= 1e-4.

Default workload: one shearing-sheet ring patch of 50,000 particles
(radii dN/dR ~ R^-3 on [1, 4] m, 400 kg/m^3, optical depth 0.5,
Omega = 1.95e-4 s^-1, 3x3 ghost boxes, quadrupoles, dt = 1e-3 2 pi / Omega),
synthetic and seeded.  Prints one JSON line on stdout; diagnostics go to
stderr.
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

METRIC = "tree-gravity particle-steps/s, FP32-mixed vs FP64 plain, at rms force err ≤1e-4"
RMS_TARGET = 1e-4
THETAS = [0.7, 0.6, 0.55, 0.5, 0.47, 0.45, 0.42, 0.4, 0.37, 0.35, 0.32, 0.3, 0.28, 0.26,
          0.24, 0.22, 0.2, 0.18, 0.16, 0.14]
# algorithmic work per term (flops; rsqrt counted as one): opening test 9,
# monopole (particle or cell) 20, quadrupole cell 56
FLOP_OPEN, FLOP_MONO, FLOP_QUAD = 9, 20, 56
PEAK_F64 = 78.6e12    # 256 CU x 64 FP64 FMA lanes x 2 flop x 2.4 GHz
PEAK_F32 = 157.3e12   # published, counts packed FP32 (dual FMA per lane)
WALK_SRC = {"fp64": "paper_1110_4876_amd/csrc/k_walk64.hip",
            "fp32": "paper_1110_4876_amd/csrc/k_walk32.hip"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    from paper_1110_4876_amd import inputs
    if name == "sheet50k":
        return inputs.sheet(50000, seed=0), "sheet50k: shearing-sheet patch N=50000, tau=0.5, 3x3 images, quadrupole, 100-step run"
    if name == "sheet1m":
        return inputs.sheet(1_000_000, seed=0), "sheet1m: shearing-sheet patch N=1000000, tau=0.5, 3x3 images, quadrupole"
    if name == "plummer8m":
        return (inputs.plummer(1 << 23, seed=0, b=0.001, quadrupole=True, dt=1e-4),
                "plummer8m: Plummer sphere N=8388608, b=0.001, open, quadrupole")
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sheet50k")
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "fp32"])
    ap.add_argument("--theta", type=float, default=None,
                    help="fix theta (and the options below) instead of autotuning")
    ap.add_argument("--leaf-size", type=int, default=1)
    ap.add_argument("--group-size", type=int, default=64)
    ap.add_argument("--split-images", type=int, default=-1)
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1110_4876_amd import autotune, inputs, rb
    from paper_1110_4876_amd.metrics import force_errors

    torch.cuda.set_device(0)
    pr, wdesc = workload(args.workload)
    n = pr.n
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")  # noqa: E731
    X = {k: dev(getattr(pr, k)) for k in ("x", "y", "z", "vx", "vy", "vz", "m")}
    parts0 = rb.particles(X["x"], X["y"], X["z"], X["m"], X["vx"], X["vy"], X["vz"])
    t_kick = 0.5 * pr.dt
    tg = inputs.sample_targets(n, 4096, seed=0)
    tg_dev = torch.as_tensor(tg, device="cuda")

    # reference: FP64 direct sum (Eq. 1 over all images) on the samples
    ctx_ref = rb.rb_create(rb.params_from_problem(pr.params), n)
    ax = torch.empty(len(tg), dtype=torch.float64, device="cuda")
    ay, az = torch.empty_like(ax), torch.empty_like(ax)
    rb.rb_direct(ctx_ref, parts0, n, n, t_kick, tg_dev, ax, ay, az)
    rb.rb_sync(ctx_ref)
    ref = torch.stack([ax, ay, az], 1).cpu().numpy()
    rb.rb_destroy(ctx_ref)

    def accel(ctx):
        gx = torch.empty(n, dtype=torch.float64, device="cuda")
        gy, gz = torch.empty_like(gx), torch.empty_like(gx)
        rb.rb_gravity(ctx, parts0, n, n, t_kick, gx, gy, gz)
        rb.rb_sync(ctx)
        return torch.stack([gx, gy, gz], 1).cpu().numpy()[tg]

    def interactions(theta):
        """per-particle FP64 walk counts at theta (the algorithmic work)"""
        p = rb.params_from_problem(pr.params, theta=theta, profile=2)
        ctx = rb.rb_create(p, n)
        accel(ctx)
        s = rb.rb_stats(ctx)
        rb.rb_destroy(ctx)
        quad = bool(pr.params["quadrupole"])
        flops = (FLOP_OPEN * s["open_tests"] + FLOP_MONO * s["pp"] +
                 (FLOP_QUAD if quad else FLOP_MONO) * s["cells"])
        return s, flops

    results = {}
    paths = ["fp64", "fp32"] if args.precision == "both" else [args.precision]
    for path in paths:
        prec = rb.RB_FP64 if path == "fp64" else rb.RB_FP32_MIXED
        # operating point: the autotuner's fastest (leaf, group, image split,
        # launch mode) at its largest theta with rms error <= 1e-4; or a
        # fixed theta with the library defaults
        try:
            if args.theta:
                cfg = dict(theta=args.theta, leaf_size=args.leaf_size,
                           group_size=args.group_size, split_images=args.split_images,
                           use_graph=args.graph)
                ctx = rb.rb_create(rb.params_from_problem(
                    pr.params, precision=prec, **{k: v for k, v in cfg.items()
                                                  if k != "use_graph"}), n)
                err = force_errors(accel(ctx), ref)
                rb.rb_destroy(ctx)
            else:
                t0 = time.perf_counter()
                cfg = autotune.tune(pr, X, ref, tg, t_kick, precision=prec,
                                    rms_target=RMS_TARGET, log=log)
                err = cfg["errors"]
                log(f"[{path}] tuned in {time.perf_counter() - t0:.1f} s")
        except (rb.RBError, RuntimeError) as ex:
            log(f"[{path}] unavailable: {ex}")
            continue
        chosen = cfg["theta"]
        log(f"[{path}] theta={chosen} leaf={cfg['leaf_size']} group={cfg['group_size']} "
            f"split={cfg['split_images']} graph={cfg['use_graph']}: rms={err['rms']:.3e} "
            f"max={err['max']:.3e}")
        st, flops = interactions(chosen)
        # timed run: K steps in one call.  Eager launches carry HIP events
        # around every walk launch; a graph replay carries none, so its walk
        # launches are timed in a second, eager pass of the same K steps.
        tuned = dict(theta=chosen, leaf_size=cfg["leaf_size"], group_size=cfg["group_size"],
                     split_images=cfg["split_images"])

        def run(use_graph, profile):
            p = rb.params_from_problem(pr.params, precision=prec, use_graph=use_graph,
                                       profile=profile, **tuned)
            ctx = rb.rb_create(p, n)
            W = {k: v.clone() for k, v in X.items()}
            pw = rb.particles(W["x"], W["y"], W["z"], W["m"], W["vx"], W["vy"], W["vz"])
            rb.rb_step(ctx, pw, n, n, 0.0, pr.dt, args.warmup)
            rb.rb_sync(ctx)
            rb.rb_stats(ctx)  # discard warm-up timers
            T = {k: v.clone() for k, v in X.items()}
            pt = rb.particles(T["x"], T["y"], T["z"], T["m"], T["vx"], T["vy"], T["vz"])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rb.rb_step(ctx, pt, n, n, 0.0, pr.dt, args.steps)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rb.rb_sync(ctx)
            s = rb.rb_stats(ctx)
            rb.rb_destroy(ctx)
            return t0, t1, s

        t0, t1, s2 = run(cfg["use_graph"], 0 if cfg["use_graph"] else 4)
        if cfg["use_graph"]:
            _, _, s2 = run(0, 4)
        ms_step = (t1 - t0) * 1e3 / args.steps
        walk_ms = s2["ms"]["walk"] / max(1, s2["calls"]["walk"])
        results[path] = dict(theta=chosen, leaf_size=cfg["leaf_size"],
                             group_size=cfg["group_size"] if path == "fp32" else None,
                             split_images=cfg["split_images"], use_graph=cfg["use_graph"],
                             errors=err, ms_per_step=ms_step,
                             particle_steps_per_s=n * args.steps / (t1 - t0),
                             walk_ms=walk_ms, walk_launches=s2["calls"]["walk"],
                             interactions=dict(open_tests=st["open_tests"], cells=st["cells"],
                                               pp=st["pp"]),
                             algorithmic_flops_per_walk=flops)
        log(f"[{path}] theta={chosen} {ms_step:.3f} ms/step, walk {walk_ms:.3f} ms, "
            f"{results[path]['particle_steps_per_s']:.3e} particle-steps/s")

    if not results:
        raise SystemExit("no path produced a result")
    main_path = "fp32" if "fp32" in results else "fp64"
    r = results[main_path]
    peak = PEAK_F32 if main_path == "fp32" else PEAK_F64
    achieved = r["algorithmic_flops_per_walk"] / (r["walk_ms"] * 1e-3)
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"walk_{main_path}_{args.workload}_traffic.json")
    if os.path.exists(tf):
        meta = json.load(open(tf))
        src = open(os.path.join(ROOT, WALK_SRC[main_path]), "rb").read()
        if meta.get("source_sha256") == hashlib.sha256(src).hexdigest():
            traffic = meta.get("bytes_per_launch")
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                "kernel": "k_walk32" if main_path == "fp32" else "k_walk64"}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        op = oracle.make_params(**dict(pr.params, theta=r["theta"]))
        st0 = pr.state()
        steps = 0
        c0 = time.perf_counter()
        while True:
            st0 = oracle.step(op, st0, pr.m, steps * pr.dt, pr.dt, 1, use_tree=True)
            steps += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        c1 = time.perf_counter()
        cpu = {"value": n * steps / (c1 - c0), "unit": "particle-steps/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{steps} full DKD steps of the same {n}-particle patch with the "
                         f"oracle tree walk (FP64, insertion build, OpenMP over targets) "
                         f"at theta={r['theta']}"}

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
        "config": {"workload": wdesc, "n": n, "images": 9 if pr.params["boundary"] else 1,
                   "path": main_path, "theta": r["theta"],
                   "quadrupole": bool(pr.params["quadrupole"]),
                   "leaf_size": r["leaf_size"], "group_size": r["group_size"],
                   "split_images": r["split_images"], "hip_graph": bool(r["use_graph"])},
        "paths": {k: {kk: vv for kk, vv in v.items()} for k, v in results.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "fp64" in results and "fp32" in results:
        out["speedup_fp32_vs_fp64"] = (results["fp32"]["particle_steps_per_s"] /
                                       results["fp64"]["particle_steps_per_s"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
