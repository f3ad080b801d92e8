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


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_forces_match_oracle(orc, precision):
    # every patch of a batch against the oracle on that patch alone: the
    # FP64 walk against the oracle's walk (rms <= 1e-12), FP32-mixed against
    # the FP64 direct sum (rms <= 1e-4 at theta 0.35)
    from gpu_util import Dev, rms_rel
    from paper_1110_4876_amd import rb
    from paper_1110_4876_amd.metrics import force_errors
    import torch
    ps = [p.with_params(theta=0.35) for p in _patches(5, n_min=500, n_max=12000, seed0=70)]
    big, off = _concat(ps)
    t = 2345.0
    ctx = _batch_ctx(ps, off, precision)
    try:
        d = Dev(big, with_v=False)
        ax = torch.empty(big.n, dtype=torch.float64, device="cuda")
        ay, az = torch.empty_like(ax), torch.empty_like(ax)
        rb.rb_batch_gravity(ctx, d.parts, t, ax, ay, az)
        rb.rb_sync(ctx)
        A = torch.stack([ax, ay, az], 1).cpu().numpy()
    finally:
        rb.rb_destroy(ctx)
    for k, pr in enumerate(ps):
        p = orc.make_params(**pr.params)
        s = orc.shear_offset(p, t)
        a = A[off[k]:off[k + 1]]
        if precision == rb.RB_FP64:
            ref = orc.bh(p, pr.x, pr.y, pr.z, pr.m, s=s)
            assert rms_rel(a, ref) <= 1e-12, (k, rms_rel(a, ref))
        else:
            tg = inputs.sample_targets(pr.n, 512, seed=k)
            ref = orc.direct(p, pr.x, pr.y, pr.z, pr.m, s=s, targets=tg)
            e = force_errors(a[tg], ref)
            assert e["rms"] <= 1e-4, (k, e)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_graph_replay_equals_eager(precision):
    # a batch's step captured once as a HIP graph and replayed: every replay
    # (with eager work and synchronisations in between) equals eager launches
    from gpu_util import Dev
    from paper_1110_4876_amd import rb
    import torch
    ps = _patches(6, n_min=200, n_max=15000, seed0=80)
    big, off = _concat(ps)
    ce = _batch_ctx(ps, off, precision)
    cg = _batch_ctx(ps, off, precision, use_graph=1)
    try:
        a, b = Dev(big), Dev(big)
        for call in range(3):
            t0 = call * 3 * big.dt
            rb.rb_batch_step(ce, a.parts, t0, big.dt, 3)
            rb.rb_batch_step(cg, b.parts, t0, big.dt, 3)
            rb.rb_sync(ce)
            rb.rb_sync(cg)
            # eager work in between: a force evaluation on the graph context
            ax = torch.empty(big.n, dtype=torch.float64, device="cuda")
            ay, az = torch.empty_like(ax), torch.empty_like(ax)
            rb.rb_batch_gravity(cg, Dev(big, with_v=False).parts, 1.0, ax, ay, az)
            rb.rb_sync(cg)
            sa, sb = a.state(), b.state()
            for k in sa:
                np.testing.assert_array_equal(sa[k], sb[k], err_msg=f"call {call} {k}")
    finally:
        rb.rb_destroy(ce)
        rb.rb_destroy(cg)


_B256 = {}


def _batch256():
    if not _B256:
        ps = inputs.batch(256, seed0=0)
        big, off = _concat(ps)
        _B256.update(ps=ps, big=big, off=off)
    return _B256


@pytest.mark.parametrize("path", ["fp64", "fp32"])
def test_batch256_matches_oracle_per_patch(orc, path):
    # the 256-patch ensemble (N_p ~ U{2000..64000}, tau_p ~ U(0.2, 1.0),
    # seeds 0..255) at the benchmark's operating point and launch shape:
    # 16 sampled targets per patch.  FP64: the oracle's walk on each patch
    # (rms <= 1e-12 over all samples, and per patch); FP32-mixed: the FP64
    # direct sum (rms <= 1e-4).  Then two steps replayed from the captured
    # graph equal eager steps.
    from gpu_util import Dev, rms_rel
    from paper_1110_4876_amd import autotune, rb
    from paper_1110_4876_amd.metrics import force_errors
    import torch
    b = _batch256()
    ps, big, off = b["ps"], b["big"], b["off"]
    op = autotune.operating_point("batch256", path)
    prec = rb.RB_FP64 if path == "fp64" else rb.RB_FP32_MIXED
    kn = {k: op[k] for k in autotune.KNOBS}
    t = 0.5 * big.dt
    print(f"[batch256] {path} {kn} n={big.n}", flush=True)
    ctx = _batch_ctx(ps, off, prec, **kn)
    try:
        d = Dev(big, with_v=False)
        ax = torch.empty(big.n, dtype=torch.float64, device="cuda")
        ay, az = torch.empty_like(ax), torch.empty_like(ax)
        rb.rb_batch_gravity(ctx, d.parts, t, ax, ay, az)
        rb.rb_sync(ctx)
        A = torch.stack([ax, ay, az], 1).cpu().numpy()
    finally:
        rb.rb_destroy(ctx)
    got, ref = [], []
    for k, pr in enumerate(ps):
        p = orc.make_params(**dict(pr.params, theta=op["theta"]))
        s = orc.shear_offset(p, t)
        tg = inputs.sample_targets(pr.n, 16, seed=k)
        if path == "fp64":
            r = orc.Tree(p, pr.x, pr.y, pr.z, pr.m).walk(s=s, targets=tg)
            assert rms_rel(A[off[k] + tg], r) <= 1e-12, k
        else:
            r = orc.direct(p, pr.x, pr.y, pr.z, pr.m, s=s, targets=tg)
        got.append(A[off[k] + tg])
        ref.append(r)
    got, ref = np.concatenate(got), np.concatenate(ref)
    if path == "fp64":
        assert rms_rel(got, ref) <= 1e-12
    else:
        e = force_errors(got, ref)
        assert e["rms"] <= 1e-4, e
    # graph replay of the step at full size equals eager launches
    ce = _batch_ctx(ps, off, prec, **dict(kn, use_graph=0))
    cg = _batch_ctx(ps, off, prec, **dict(kn, use_graph=1))
    try:
        x, y = Dev(big), Dev(big)
        rb.rb_batch_step(ce, x.parts, 0.0, big.dt, 2)
        rb.rb_batch_step(cg, y.parts, 0.0, big.dt, 2)
        rb.rb_sync(ce)
        rb.rb_sync(cg)
        sx, sy = x.state(), y.state()
    finally:
        rb.rb_destroy(ce)
        rb.rb_destroy(cg)
    for k in sx:
        np.testing.assert_array_equal(sx[k], sy[k], err_msg=k)
