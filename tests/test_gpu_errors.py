"""Deferred device errors: a node capacity too small for a clustered input
(RB_ECAPACITY) and a particle outside a periodic axis (RB_EOUTSIDE) are
reported by the next synchronising call; every kernel runs to its end, and
the same context then works on good input."""
import numpy as np
import pytest

from paper_1110_4876_amd import inputs

pytestmark = pytest.mark.gpu


def _pairs(n_pairs, seed):
    # particles in coincident pairs (1e-13 of the box apart): each pair's
    # branch runs down to the deepest level, about 15 nodes per pair
    pr = inputs.plummer(n_pairs, seed=seed)
    rep = lambda a: np.repeat(a, 2)  # noqa: E731
    x, y, z = rep(pr.x), rep(pr.y), rep(pr.z)
    x[1::2] += 1e-13 * 128
    m = np.full(2 * n_pairs, 0.5 / n_pairs)
    zero = np.zeros(2 * n_pairs)
    return inputs.Problem(x, y, z, zero, zero.copy(), zero.copy(), m, dict(pr.params),
                          2 * n_pairs, 1e-3)


def _good_after(orc, ctx, precision):
    # good input on the context that reported the error: the forces equal a
    # fresh context's bit for bit (and, FP64, the oracle's walk)
    from gpu_util import Dev, gravity, make_ctx, rms_rel
    from paper_1110_4876_amd import rb
    pr = inputs.plummer(2000, seed=3, b=0.01)
    a = gravity(ctx, Dev(pr, with_v=False), pr.n)
    fresh = make_ctx(pr, precision=precision, node_factor=1.5, capacity=4000)
    try:
        b = gravity(fresh, Dev(pr, with_v=False), pr.n)
    finally:
        rb.rb_destroy(fresh)
    np.testing.assert_array_equal(a, b)
    if precision == 0:
        ref = orc.bh(orc.make_params(**pr.params), pr.x, pr.y, pr.z, pr.m)
        assert rms_rel(a, ref) <= 1e-12


@pytest.mark.parametrize("precision", [0, 1])
def test_node_capacity_is_reported(orc, precision):
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    import torch
    pr = _pairs(1000, 4)
    ctx = make_ctx(pr, precision=precision, node_factor=1.5, capacity=4000)
    try:
        d = Dev(pr)
        a = torch.empty((3, pr.n), dtype=torch.float64, device="cuda")
        rb.rb_gravity(ctx, d.parts, d.n, d.n, 0.0, a[0], a[1], a[2])
        with pytest.raises(rb.RBError) as ex:
            rb.rb_sync(ctx)
        assert ex.value.code == rb.RB_ECAPACITY
        # the same through steps, eager and graph-replayed
        for graph in (0, 1):
            p = rb.params_from_problem(pr.params, precision=precision, node_factor=1.5,
                                       use_graph=graph)
            rb.rb_set_params(ctx, p)
            rb.rb_step(ctx, d.parts, d.n, d.n, 0.0, pr.dt, 2)
            with pytest.raises(rb.RBError) as ex:
                rb.rb_sync(ctx)
            assert ex.value.code == rb.RB_ECAPACITY
        # the error word is cleared once reported: the context works again
        rb.rb_sync(ctx)
        _good_after(orc, ctx, precision)
    finally:
        rb.rb_destroy(ctx)


@pytest.mark.parametrize("boundary", [inputs.PERIODIC, inputs.SHEAR])
def test_outside_periodic_axis_is_reported(orc, boundary):
    from gpu_util import Dev, gravity, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.sheet(3000, seed=8).with_params(boundary=boundary)
    W = pr.params["W"]
    bad = pr.with_params()
    bad.x = pr.x.copy()
    bad.x[17] = 0.5 * W + 3.0  # outside the box in x: never wrapped
    ctx = make_ctx(pr)
    try:
        with pytest.raises(rb.RBError) as ex:
            gravity(ctx, Dev(bad, with_v=False), bad.n)
        assert ex.value.code == rb.RB_EOUTSIDE
        # in a step, one wrap brings a particle back only from the
        # neighbouring box: one three boxes out stays outside
        far = pr.with_params()
        far.y = pr.y.copy()
        far.y[5] = 3.5 * W
        d = Dev(far)
        rb.rb_step(ctx, d.parts, d.n, d.n, 0.0, pr.dt, 1)
        with pytest.raises(rb.RBError) as ex:
            rb.rb_sync(ctx)
        assert ex.value.code == rb.RB_EOUTSIDE
        # good input afterwards: forces as the oracle's
        from gpu_util import rms_rel
        a = gravity(ctx, Dev(pr, with_v=False), pr.n, 100.0)
        p = orc.make_params(**pr.params)
        ref = orc.bh(p, pr.x, pr.y, pr.z, pr.m, s=orc.shear_offset(p, 100.0))
        assert rms_rel(a, ref) <= 1e-12
    finally:
        rb.rb_destroy(ctx)
