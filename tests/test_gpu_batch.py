"""Batched independent systems (one tree per root box, Sect. 2.3): every patch
of a batch gets exactly the tree, forces and trajectory it gets alone."""
import numpy as np
import pytest

from paper_1110_4876_amd import inputs

pytestmark = pytest.mark.gpu


def _patches(k=5, n_min=300, n_max=9000, seed0=10):
    return inputs.batch(k, n_min=n_min, n_max=n_max, seed0=seed0)


def _concat(ps):
    cat = lambda f: np.concatenate([getattr(p, f) for p in ps])  # noqa: E731
    from paper_1110_4876_amd.inputs import Problem
    off = np.concatenate([[0], np.cumsum([p.n for p in ps])]).astype(np.int64)
    big = Problem(cat("x"), cat("y"), cat("z"), cat("vx"), cat("vy"), cat("vz"), cat("m"),
                  dict(ps[0].params), int(off[-1]), ps[0].dt)
    return big, off


def _batch_ctx(ps, off, precision, **kw):
    from paper_1110_4876_amd import rb
    p = rb.params_from_problem(ps[0].params, precision=precision, **kw)
    W = np.array([q.params["W"] for q in ps])
    x0 = np.array([q.params["x0"] for q in ps])
    return rb.rb_batch_create(p, off, W, x0)


def test_batch_tree_equals_single():
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    ps = _patches()
    big, off = _concat(ps)
    ctx = _batch_ctx(ps, off, rb.RB_FP64)
    try:
        d = Dev(big, with_v=False)
        rb.rb_tree_build(ctx, d.parts, big.n, big.n)
        got = [export(ctx, k) for k in range(len(ps))]
    finally:
        rb.rb_destroy(ctx)
    for k, pr in enumerate(ps):
        c1 = make_ctx(pr)
        try:
            rb.rb_tree_build(c1, Dev(pr, with_v=False).parts, pr.n, pr.n)
            ref = export(c1)
        finally:
            rb.rb_destroy(c1)
        nn = len(ref["level"])
        for f in ("keys", "perm", "level", "prefix", "first", "count", "is_leaf", "M", "com"):
            np.testing.assert_array_equal(got[k][f][:len(ref[f])], ref[f], err_msg=f"patch {k} {f}")
        # no extra nodes: the export buffers beyond the patch's nodes stay empty
        assert np.all(got[k]["count"][nn:] == 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_gravity_and_step_equal_single(precision):
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    import torch
    ps = _patches()
    big, off = _concat(ps)
    t = 777.0
    ctx = _batch_ctx(ps, off, precision)
    try:
        d = Dev(big)
        ax = torch.empty(big.n, dtype=torch.float64, device="cuda")
        ay, az = torch.empty_like(ax), torch.empty_like(ax)
        rb.rb_batch_gravity(ctx, d.parts, t, ax, ay, az)
        rb.rb_sync(ctx)
        A = torch.stack([ax, ay, az], 1).cpu().numpy()
        rb.rb_batch_step(ctx, d.parts, 0.0, big.dt, 3)
        rb.rb_sync(ctx)
        S = d.state()
    finally:
        rb.rb_destroy(ctx)
    for k, pr in enumerate(ps):
        sl = slice(off[k], off[k + 1])
        c1 = make_ctx(pr, precision=precision)
        try:
            e = Dev(pr)
            bx = torch.empty(pr.n, dtype=torch.float64, device="cuda")
            by, bz = torch.empty_like(bx), torch.empty_like(bx)
            rb.rb_gravity(c1, e.parts, pr.n, pr.n, t, bx, by, bz)
            rb.rb_sync(c1)
            ref = torch.stack([bx, by, bz], 1).cpu().numpy()
            rb.rb_step(c1, e.parts, pr.n, pr.n, 0.0, pr.dt, 3)
            rb.rb_sync(c1)
            st = e.state()
        finally:
            rb.rb_destroy(c1)
        np.testing.assert_array_equal(A[sl], ref, err_msg=f"patch {k} forces")
        for f in st:
            np.testing.assert_array_equal(S[f][sl], st[f], err_msg=f"patch {k} {f}")


def test_batch_with_tiny_patches():
    # patches of 1-3 particles (boxes a few metres wide: particles leaving in
    # z are removed) behave exactly as when run alone
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    ps = _patches(4, n_min=1, n_max=3, seed0=50) + _patches(2, seed0=60)
    big, off = _concat(ps)
    ctx = _batch_ctx(ps, off, rb.RB_FP32_MIXED)
    try:
        d = Dev(big)
        rb.rb_batch_step(ctx, d.parts, 0.0, big.dt, 2)
        rb.rb_sync(ctx)
        S = d.state()
    finally:
        rb.rb_destroy(ctx)
    for k, pr in enumerate(ps):
        c1 = make_ctx(pr, precision=rb.RB_FP32_MIXED)
        try:
            e = Dev(pr)
            rb.rb_step(c1, e.parts, pr.n, pr.n, 0.0, pr.dt, 2)
            rb.rb_sync(c1)
            st = e.state()
        finally:
            rb.rb_destroy(c1)
        for f in st:
            np.testing.assert_array_equal(S[f][off[k]:off[k + 1]], st[f], err_msg=f"patch {k} {f}")
