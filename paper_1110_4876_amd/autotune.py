"""Autotuner for the tree walk: leaf size, walk group size (FP32-mixed path)
and image schedule, each at the largest opening angle that keeps the rms
force error at or below a target against a reference (normally the FP64
direct sum on sampled particles).  Candidates are timed with full drift-kick-drift steps
through the C ABI, so the build's share (which shrinks with larger leaves)
counts as much as the walk's.

The result is a plain dict; ``cache`` (a JSON path) stores results keyed by
the workload signature and the GPU architecture.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import rb
from .metrics import force_errors

THETAS = [0.7, 0.6, 0.55, 0.5, 0.47, 0.45, 0.42, 0.4, 0.37, 0.35, 0.32, 0.3, 0.28, 0.26,
          0.24, 0.22, 0.2, 0.18, 0.16, 0.14]


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName
    except Exception:  # pragma: no cover - informational only
        return "unknown"


def signature(problem) -> str:
    p = problem.params
    return (f"{problem.name}|n={problem.n}|W={p['W']:.6g}|b={p['b']:.3g}|quad={int(bool(p['quadrupole']))}"
            f"|bnd={p['boundary']}|ng={tuple(p['ng'])}")


def _accel(ctx, parts, n, t, targets):
    import torch
    ax = torch.empty(n, dtype=torch.float64, device="cuda")
    ay, az = torch.empty_like(ax), torch.empty_like(ax)
    rb.rb_gravity(ctx, parts, n, n, t, ax, ay, az)
    rb.rb_sync(ctx)
    return torch.stack([ax, ay, az], 1)[targets].cpu().numpy()


def tune(problem, dev, ref, targets, t_kick, precision=None, rms_target=1e-4,
         leafs=(1, 2, 4, 8), groups=(16, 32, 64), splits=(0, 1), graphs=(0, 1), steps=5,
         repeats=2, cache=None, log=None):
    """Search (leaf, group, split) x theta for one precision path (default
    FP32-mixed; the FP64 per-particle walk has no group size).

    dev: dict of device tensors x, y, z, vx, vy, vz, m (caller order).
    ref: reference accelerations at `targets` (rows), time t_kick.
    graphs: launch modes timed for each candidate (0 eager, 1 HIP-graph
    replay of the step); they do not change the result.
    Returns dict(leaf_size, group_size, split_images, use_graph, theta,
    ms_per_step, errors, table).
    """
    import torch
    if precision is None:
        precision = rb.RB_FP32_MIXED
    if precision == rb.RB_FP64:
        groups = (64,)
    key = f"{signature(problem)}|{_arch()}|prec={precision}|target={rms_target:g}"
    if cache and os.path.exists(cache):
        try:
            hit = json.load(open(cache)).get(key)
            if hit:
                return hit
        except (OSError, ValueError):
            pass
    n = problem.n
    parts = rb.particles(dev["x"], dev["y"], dev["z"], dev["m"], dev["vx"], dev["vy"], dev["vz"])
    tg = torch.as_tensor(np.asarray(targets, dtype=np.int64), device="cuda")
    table = []
    best = None
    for leaf in leafs:
        for group in groups:
            for split in splits:
                if problem.params["boundary"] == 0 and split:
                    continue  # one image: nothing to split
                chosen, err = None, None
                for th in THETAS:
                    p = rb.params_from_problem(problem.params, precision=precision,
                                               theta=th, leaf_size=leaf, group_size=group,
                                               split_images=split)
                    ctx = rb.rb_create(p, n)
                    try:
                        e = force_errors(_accel(ctx, parts, n, t_kick, tg), ref)
                    finally:
                        rb.rb_destroy(ctx)
                    if e["rms"] <= rms_target:
                        chosen, err = th, e
                        break
                if chosen is None:
                    continue
                for graph in graphs:
                    p = rb.params_from_problem(problem.params, precision=precision,
                                               theta=chosen, leaf_size=leaf, group_size=group,
                                               split_images=split, use_graph=graph)
                    ctx = rb.rb_create(p, n)
                    try:
                        work = {k: v.clone() for k, v in dev.items()}
                        wp = rb.particles(work["x"], work["y"], work["z"], work["m"],
                                          work["vx"], work["vy"], work["vz"])
                        rb.rb_step(ctx, wp, n, n, 0.0, problem.dt, 1)
                        rb.rb_sync(ctx)
                        times = []
                        for _ in range(repeats):
                            torch.cuda.synchronize()
                            t0 = time.perf_counter()
                            rb.rb_step(ctx, wp, n, n, 0.0, problem.dt, steps)
                            rb.rb_sync(ctx)
                            times.append((time.perf_counter() - t0) * 1e3 / steps)
                    finally:
                        rb.rb_destroy(ctx)
                    ms = min(times)
                    row = dict(leaf_size=leaf, group_size=group, split_images=split,
                               use_graph=graph, theta=chosen, ms_per_step=ms, rms=err["rms"],
                               max=err["max"])
                    table.append(row)
                    if log:
                        log(f"[tune] leaf={leaf} group={group} split={split} graph={graph} "
                            f"theta={chosen} rms={err['rms']:.2e} {ms:.3f} ms/step")
                    if best is None or ms < best["ms_per_step"]:
                        best = dict(row, errors=err)
    if best is None:
        raise RuntimeError("no candidate met the accuracy target")
    best["table"] = table
    if cache:
        try:
            data = json.load(open(cache)) if os.path.exists(cache) else {}
        except (OSError, ValueError):
            data = {}
        data[key] = best
        with open(cache, "w") as f:
            json.dump(data, f, indent=1)
    return best
