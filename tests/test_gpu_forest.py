"""Forests of root boxes (Sect. 2.3: an integer number of cubic root boxes
per axis, one tree per root box) on the GPU against the oracle's forest:
every root box's tree bit-exact, FP64 forces and interaction counts of the
per-particle walk, FP32-mixed against the direct sum, and steps across the
faces of elongated domains."""
import numpy as np
import pytest

from paper_1110_4876_amd import inputs

pytestmark = pytest.mark.gpu

TOL_BH = 1e-12


def _virtual(n_root):
    m = max(n_root)
    D = 0
    while (1 << D) < m:
        D += 1
    return D


def _plummer_forest(n, seed, n_root, W=64.0, **kw):
    # a Plummer sphere in a domain of n_root root boxes of side W centred on
    # the origin (open boundaries)
    pr = inputs.plummer(n, seed=seed, **kw)
    x0 = tuple(-0.5 * n_root[a] * W for a in range(3))
    return pr.with_params(W=W, x0=x0, n_root=tuple(n_root))


def _uniform_forest(n, seed, n_root, W=1.0, n_leaf=1):
    # uniform particles of masses U(0.5, 1.5) filling the domain, plus a tight
    # clump (deep cells) in one box
    rng = np.random.default_rng(seed)
    pts = [rng.uniform(0, n_root[a] * W, n) for a in range(3)]
    pts[0][:150] = 0.37 * W + rng.normal(0, 1e-4 * W, 150)
    pts[1][:150] = 0.61 * W + rng.normal(0, 1e-4 * W, 150)
    m = rng.uniform(0.5, 1.5, n)
    z = np.zeros(n)
    params = inputs.base_params(G=1.0, b=1e-3 * W, theta=0.5, quadrupole=True, W=W,
                                x0=(0.0, 0.0, 0.0), n_root=tuple(n_root), n_leaf=n_leaf)
    return inputs.Problem(pts[0], pts[1], pts[2], z.copy(), z.copy(), z.copy(), m, params,
                          n, 1e-3, 0.0, "uniform_forest")


CASES = [
    ("plummer_2x2x2", lambda: _plummer_forest(6000, 1, (2, 2, 2), quadrupole=True), 1, None),
    ("uniform_3x2x1", lambda: _uniform_forest(5000, 2, (3, 2, 1)), 1, None),
    ("uniform_3x2x1_leaf4", lambda: _uniform_forest(5000, 2, (3, 2, 1), n_leaf=4), 4, None),
    ("uniform_5x1x1_testparticles", lambda: _uniform_forest(4000, 3, (5, 1, 1)), 1, 3000),
    ("sheet_1x3x1", lambda: inputs.sheet(6000, seed=4, n_root=(1, 3, 1)), 1, None),
    ("sheet_4x1x1", lambda: inputs.sheet(6000, seed=5, n_root=(4, 1, 1)), 1, None),
]


def _dfs_skip_forest(e, roots):
    """next node after each subtree in depth-first order, root boxes in order"""
    nn = len(e["level"])
    skip = np.full(nn, -1, np.int64)
    import sys
    sys.setrecursionlimit(10000)

    def visit(v, after):
        skip[v] = after
        if e["is_leaf"][v]:
            return
        c0, nc = e["first_child"][v], e["n_child"][v]
        for k in range(nc):
            visit(c0 + k, c0 + k + 1 if k + 1 < nc else after)
    for k, r in enumerate(roots):
        visit(r, roots[k + 1] if k + 1 < len(roots) else -1)
    return skip


@pytest.mark.parametrize("name,maker,leaf,n_active", CASES, ids=[c[0] for c in CASES])
def test_forest_tree_matches_oracle(orc, name, maker, leaf, n_active):
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    pr = maker()
    na = pr.n if n_active is None else n_active
    D = _virtual(pr.params["n_root"])
    p = orc.make_params(**dict(pr.params, n_leaf=leaf))
    ref = orc.Tree(p, pr.x, pr.y, pr.z, pr.m, n_active=na).export()
    ctx = make_ctx(pr, leaf_size=leaf)
    try:
        d = Dev(pr, with_v=False)
        rb.rb_tree_build(ctx, d.parts, d.n, na)
        g = export(ctx)
    finally:
        rb.rb_destroy(ctx)
    np.testing.assert_array_equal(g["keys"], ref["keys"])
    np.testing.assert_array_equal(g["perm"], ref["perm"])
    # the cells above the root boxes come first (levels < D): never leaves
    nv = int(np.sum(g["level"] < D))
    assert not np.any(g["is_leaf"][:nv])
    assert np.all(g["level"][:nv] < D) and np.all(g["level"][nv:] >= D)
    for k in ("level", "prefix", "first", "count", "is_leaf"):
        np.testing.assert_array_equal(g[k][nv:], ref[k], err_msg=k)
    internal = ref["is_leaf"] == 0
    np.testing.assert_array_equal(g["n_child"][nv:][internal], ref["n_child"][internal])
    np.testing.assert_array_equal(g["first_child"][nv:][internal] - nv,
                                  ref["first_child"][internal])
    roots = np.nonzero(ref["level"] == D)[0]
    skip = _dfs_skip_forest(ref, list(roots))
    # a skip link may name a cell above the root boxes: the walk opens it and
    # goes on with its first root box
    gs = g["skip"][nv:].copy()
    for k in np.nonzero((gs >= 0) & (gs < nv))[0]:
        v = gs[k]
        while g["level"][v] < D:
            v = g["first_child"][v]
        gs[k] = v
    gs[gs >= 0] -= nv
    np.testing.assert_array_equal(gs, skip)
    np.testing.assert_array_equal(g["M"][nv:], ref["M"])
    np.testing.assert_array_equal(g["com"][nv:], ref["com"])
    if pr.params["quadrupole"]:
        scale = np.abs(ref["Q"]).max(axis=1, keepdims=True) + 1e-300
        assert (np.abs(g["Q"][nv:] - ref["Q"]) <= 1e-12 * scale).all()


@pytest.mark.parametrize("name,maker,leaf,n_active", CASES, ids=[c[0] for c in CASES])
def test_forest_fp64_walk_matches_oracle(orc, name, maker, leaf, n_active):
    from gpu_util import Dev, make_ctx, rms_rel
    from paper_1110_4876_amd import rb
    import torch
    pr = maker()
    na = pr.n if n_active is None else n_active
    t = 4321.0 if pr.params["boundary"] else 0.0
    p = orc.make_params(**dict(pr.params, n_leaf=leaf))
    T = orc.Tree(p, pr.x, pr.y, pr.z, pr.m, n_active=na)
    ref = T.walk(s=orc.shear_offset(p, t))
    for split in (0, 1):
        for sched in (1, 2, 3):
            ctx = make_ctx(pr, leaf_size=leaf, split_images=split, walk64_schedule=sched,
                           profile=2)
            try:
                d = Dev(pr, with_v=False)
                a = torch.empty((3, pr.n), dtype=torch.float64, device="cuda")
                rb.rb_gravity(ctx, d.parts, d.n, na, t, a[0], a[1], a[2])
                s = rb.rb_stats(ctx)
                a = a.t().cpu().numpy()
            finally:
                rb.rb_destroy(ctx)
            assert rms_rel(a, ref) <= TOL_BH, (split, sched, rms_rel(a, ref))
            for k in ("open_tests", "cells", "pp"):
                assert s[k] == T.stats[k], (split, sched, k, s[k], T.stats[k])


@pytest.mark.parametrize("name,maker", [(c[0], c[1]) for c in CASES if c[2] == 1],
                         ids=[c[0] for c in CASES if c[2] == 1])
def test_forest_fp32_meets_gate(orc, name, maker):
    from gpu_util import Dev, gravity, make_ctx
    from paper_1110_4876_amd import rb
    from paper_1110_4876_amd.metrics import force_errors
    pr = maker().with_params(theta=0.35)
    t = 4321.0 if pr.params["boundary"] else 0.0
    p = orc.make_params(**pr.params)
    tg = inputs.sample_targets(pr.n, 1024, seed=1)
    ref = orc.direct(p, pr.x, pr.y, pr.z, pr.m, s=orc.shear_offset(p, t), targets=tg)
    for waves in (1, 4):
        ctx = make_ctx(pr, precision=rb.RB_FP32_MIXED, walk_waves=waves)
        try:
            a = gravity(ctx, Dev(pr, with_v=False), pr.n, t)
        finally:
            rb.rb_destroy(ctx)
        e = force_errors(a[tg], ref)
        assert e["rms"] <= 1e-4, (waves, e)


def test_forest_of_eight_equals_one_box():
    # the 2x2x2 forest of boxes of side 64 covers the box of side 128 at the
    # same corner; its keys are the same and its trees are the big box's
    # level-1 subtrees, so the walks give identical forces (the big box's
    # root is never accepted by a particle inside it)
    from gpu_util import Dev, gravity, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.plummer(20000, seed=6, quadrupole=True)
    fr = _plummer_forest(20000, 6, (2, 2, 2), quadrupole=True)
    out = []
    for q in (pr, fr):
        for prec in (rb.RB_FP64, rb.RB_FP32_MIXED):
            ctx = make_ctx(q, precision=prec)
            try:
                out.append(gravity(ctx, Dev(q, with_v=False), q.n))
            finally:
                rb.rb_destroy(ctx)
    np.testing.assert_array_equal(out[0], out[2])
    np.testing.assert_array_equal(out[1], out[3])


def _run_steps(pr, t, nsteps, **kw):
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    ctx = make_ctx(pr, **kw)
    try:
        d = Dev(pr)
        rb.rb_step(ctx, d.parts, d.n, pr.n_active, t, pr.dt, nsteps)
        rb.rb_sync(ctx)
        return d.state()
    finally:
        rb.rb_destroy(ctx)


@pytest.mark.parametrize("n_root", [(1, 3, 1), (4, 1, 1), (2, 2, 1)])
def test_forest_sheet_steps_cross_the_faces(orc, n_root):
    # particles pushed across the x and y faces of an elongated shearing
    # sheet during the step re-enter with the domain's shear offset and
    # velocity jump (extents Lx, Ly), as in the oracle
    pr = inputs.sheet(4000, seed=7, n_root=n_root)
    W = pr.params["W"]
    Lx, Ly = n_root[0] * W, n_root[1] * W
    om = pr.params["omega"]
    pr.vx[:150] = np.sign(pr.x[:150]) * 0.5 * Lx / pr.dt
    pr.vy[:150] = -1.5 * om * pr.x[:150]
    pr.vy[150:300] = np.sign(pr.y[150:300]) * 0.5 * Ly / pr.dt
    p = orc.make_params(**pr.params)
    ref = orc.step(p, pr.state(), pr.m, 300.0, pr.dt, 2, use_tree=True)
    for prec in (0, 1):
        got = _run_steps(pr, 300.0, 2, precision=prec)
        tol = 1e-9 if prec == 0 else 1e-5
        for k in ("x", "y", "z"):
            np.testing.assert_allclose(got[k], ref[k], rtol=0, atol=tol * W, err_msg=(prec, k))


def test_forest_open_steps_remove_escapers(orc):
    pr = _plummer_forest(3000, 8, (3, 1, 2), W=40.0, b=0.05)
    pr.vx[:4] = 1e6  # out of the domain in the first drift
    p = orc.make_params(**pr.params)
    ref = orc.step(p, pr.state(), pr.m, 0.0, pr.dt, 3, use_tree=True)
    got = _run_steps(pr, 0.0, 3)
    assert np.all(np.isnan(got["x"][:4])) and np.all(np.isnan(ref["x"][:4]))
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        np.testing.assert_allclose(got[k][4:], ref[k][4:], rtol=1e-13, atol=1e-15, err_msg=k)


def test_forest_refused_where_unsupported():
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    import torch
    pr = inputs.sheet(3000, seed=9, n_root=(1, 2, 1))
    p = rb.params_from_problem(pr.params)
    with pytest.raises(rb.RBError) as ex:
        rb.rb_batch_create(p, np.array([0, pr.n]), np.array([pr.params["W"]]),
                           np.array([pr.params["x0"]]))
    assert ex.value.code == rb.RB_EUNSUPPORTED
    ctx = make_ctx(pr)
    try:
        d = Dev(pr)
        R = torch.as_tensor(pr.extra["radius"], device="cuda")
        with pytest.raises(rb.RBError) as ex:
            rb.rb_collide(ctx, d.parts, R, d.n, 0.0, 0.5, 1)
        assert ex.value.code == rb.RB_EUNSUPPORTED
    finally:
        rb.rb_destroy(ctx)
