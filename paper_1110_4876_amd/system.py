"""A system on the GPU -- one particle set, or a batch of independent
shearing-sheet patches (one tree per root box, Sect. 2.3) -- driven through
the C ABI: context creation with parameter overrides, accelerations, steps
and the FP64 direct-sum reference.  Used by the autotuner and the benchmark.
"""
from __future__ import annotations

import numpy as np

from . import inputs, rb

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m")


class System:
    def __init__(self, problems):
        import torch
        self.batch = isinstance(problems, (list, tuple))
        probs = list(problems) if self.batch else [problems]
        self.problems = probs
        self.params = dict(probs[0].params)
        self.dt = probs[0].dt
        self.name = (f"batch{len(probs)}" if self.batch else probs[0].name)
        sizes = [p.n for p in probs]
        self.offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        self.n_active = self.n if self.batch else probs[0].n_active
        self.box_size = np.array([p.params["W"] for p in probs], dtype=np.float64)
        self.box_min = np.array([p.params["x0"] for p in probs], dtype=np.float64)
        self.X = {f: torch.as_tensor(np.ascontiguousarray(
            np.concatenate([getattr(p, f) for p in probs]), dtype=np.float64), device="cuda")
            for f in FIELDS}

    # ---- state --------------------------------------------------------------
    def clone(self) -> dict:
        return {k: v.clone() for k, v in self.X.items()}

    @staticmethod
    def parts(X) -> rb.rb_particles:
        return rb.particles(X["x"], X["y"], X["z"], X["m"], X["vx"], X["vy"], X["vz"])

    def signature(self) -> str:
        p = self.params
        return (f"{self.name}|n={self.n}|patches={len(self.problems)}|W0={p['W']:.6g}"
                f"|b={p['b']:.3g}|quad={int(bool(p['quadrupole']))}|bnd={p['boundary']}"
                f"|ng={tuple(p['ng'])}")

    # ---- calls through the C ABI --------------------------------------------
    def create(self, precision=rb.RB_FP64, **kw):
        p = rb.params_from_problem(self.params, precision=precision, **kw)
        if self.batch:
            return rb.rb_batch_create(p, self.offsets, self.box_size, self.box_min)
        return rb.rb_create(p, self.n)

    def gravity(self, ctx, t, X=None):
        """(n, 3) device tensor of tree accelerations at time t."""
        import torch
        X = self.X if X is None else X
        a = torch.empty((3, self.n), dtype=torch.float64, device="cuda")
        if self.batch:
            rb.rb_batch_gravity(ctx, self.parts(X), t, a[0], a[1], a[2])
        else:
            rb.rb_gravity(ctx, self.parts(X), self.n, self.n_active, t, a[0], a[1], a[2])
        rb.rb_sync(ctx)
        return a.t()

    def step(self, ctx, X, t, nsteps):
        if self.batch:
            rb.rb_batch_step(ctx, self.parts(X), t, self.dt, nsteps)
        else:
            rb.rb_step(ctx, self.parts(X), self.n, self.n_active, t, self.dt, nsteps)

    def direct(self, targets, t, X=None):
        """FP64 direct sum of Eq. (1) at the (global) target indices, on the
        GPU, for state X (default: the initial state); for a batch each
        target sees its own patch only."""
        import torch
        X = self.X if X is None else X
        targets = np.asarray(targets, dtype=np.int64)
        out = np.empty((len(targets), 3))
        for k, pr in enumerate(self.problems):
            lo, hi = int(self.offsets[k]), int(self.offsets[k + 1])
            sel = np.nonzero((targets >= lo) & (targets < hi))[0]
            if len(sel) == 0:
                continue
            ctx = rb.rb_create(rb.params_from_problem(pr.params), hi - lo)
            try:
                Xk = {f: v[lo:hi] for f, v in X.items()}
                tg = torch.as_tensor(targets[sel] - lo, device="cuda")
                a = torch.empty((3, len(sel)), dtype=torch.float64, device="cuda")
                n_act = (hi - lo) if self.batch else self.n_active
                rb.rb_direct(ctx, self.parts(Xk), hi - lo, n_act, t, tg, a[0], a[1], a[2])
                rb.rb_sync(ctx)
                out[sel] = a.t().cpu().numpy()
            finally:
                rb.rb_destroy(ctx)
        return out

    def sample_targets(self, per_system=4096, per_patch=16, seed=0):
        """Sampled targets without replacement: `per_system` for one system,
        `per_patch` from every patch of a batch (global indices)."""
        if not self.batch:
            return inputs.sample_targets(self.n, per_system, seed=seed)
        out = []
        for k in range(len(self.problems)):
            lo, hi = int(self.offsets[k]), int(self.offsets[k + 1])
            rng = np.random.default_rng(seed + k)
            out.append(lo + np.sort(rng.choice(hi - lo, size=min(per_patch, hi - lo),
                                               replace=False)))
        return np.concatenate(out).astype(np.int64)
