"""Helpers for the GPU tests: move a seeded problem to the device and call the
C ABI through the binding.  (Not a test module.)"""
import numpy as np
import torch

from paper_1110_4876_amd import rb


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


class Dev:
    """A problem's particles as device tensors plus the rb_particles struct."""

    def __init__(self, pr, with_v=True):
        self.x, self.y, self.z, self.m = dev(pr.x), dev(pr.y), dev(pr.z), dev(pr.m)
        if with_v:
            self.vx, self.vy, self.vz = dev(pr.vx), dev(pr.vy), dev(pr.vz)
            self.parts = rb.particles(self.x, self.y, self.z, self.m, self.vx, self.vy, self.vz)
        else:
            self.parts = rb.particles(self.x, self.y, self.z, self.m)
        self.n = len(pr.x)

    def state(self):
        return {k: getattr(self, k).cpu().numpy() for k in ("x", "y", "z", "vx", "vy", "vz")}


def make_ctx(pr, precision=rb.RB_FP64, capacity=None, **kw):
    p = rb.params_from_problem(pr.params, precision=precision, **kw)
    return rb.rb_create(p, capacity or max(pr.n, 1))


def gravity(ctx, d, n_active, t=0.0):
    ax = torch.empty(d.n, dtype=torch.float64, device="cuda")
    ay, az = torch.empty_like(ax), torch.empty_like(ax)
    rb.rb_gravity(ctx, d.parts, d.n, n_active, t, ax, ay, az)
    rb.rb_sync(ctx)
    return torch.stack([ax, ay, az], dim=1).cpu().numpy()


def direct(ctx, d, n_active, targets, t=0.0):
    tg = torch.as_tensor(np.asarray(targets, dtype=np.int64), device="cuda")
    ax = torch.empty(len(targets), dtype=torch.float64, device="cuda")
    ay, az = torch.empty_like(ax), torch.empty_like(ax)
    rb.rb_direct(ctx, d.parts, d.n, n_active, t, tg, ax, ay, az)
    rb.rb_sync(ctx)
    return torch.stack([ax, ay, az], dim=1).cpu().numpy()


def export(ctx, patch=0):
    nn, nl = rb.rb_tree_info(ctx)
    return rb.rb_tree_export(ctx, patch, nn, nl)


def rms_rel(a, ref):
    den = float(np.sum(ref * ref))
    return float(np.sqrt(np.sum((a - ref) ** 2) / den)) if den > 0 else float(np.abs(a).max())
