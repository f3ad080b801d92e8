"""Paths that only large systems take, checked against the oracle: the
large-node moments computed level by level over the whole chip (systems of
more than 2^22 slots, or forced on smaller ones by moments_level_log2), and
a Plummer sphere above 2^22 particles at full size (Sect. 4.2)."""
import numpy as np
import pytest

from paper_1110_4876_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [
    ("plummer5000_quad", lambda: inputs.plummer(5000, seed=3, quadrupole=True), 1, None),
    ("plummer5000_quad_leaf4", lambda: inputs.plummer(5000, seed=3, quadrupole=True), 4, None),
    ("sheet7000", lambda: inputs.sheet(7000, seed=1), 1, None),
    ("plummer3000_testparticles", lambda: inputs.plummer(3000, seed=4, quadrupole=True), 1, 2100),
]


def _tree(pr, leaf, na, **kw):
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    ctx = make_ctx(pr, leaf_size=leaf, **kw)
    try:
        d = Dev(pr, with_v=False)
        rb.rb_tree_build(ctx, d.parts, d.n, na)
        return export(ctx)
    finally:
        rb.rb_destroy(ctx)


def _check_tree(g, ref, quad):
    for k in ("keys", "perm", "level", "prefix", "first", "count", "is_leaf"):
        np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
    internal = ref["is_leaf"] == 0
    np.testing.assert_array_equal(g["n_child"][internal], ref["n_child"][internal])
    np.testing.assert_array_equal(g["first_child"][internal], ref["first_child"][internal])
    np.testing.assert_array_equal(g["M"], ref["M"])
    np.testing.assert_array_equal(g["com"], ref["com"])
    if quad:
        scale = np.abs(ref["Q"]).max(axis=1, keepdims=True) + 1e-300
        assert np.abs(g["Q"] - ref["Q"]).max() <= 1e-13 * scale.max()
        assert (np.abs(g["Q"] - ref["Q"]) <= 1e-12 * scale).all()


@pytest.mark.parametrize("name,maker,leaf,n_active", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("group", [16, 64])
def test_level_by_level_moments_match_oracle(orc, name, maker, leaf, n_active, group):
    # moments_level_log2 = 6: every system above 64 slots takes the
    # level-by-level large-node kernels; the tree equals the oracle's and the
    # one-workgroup path's
    pr = maker()
    na = pr.n if n_active is None else n_active
    p = orc.make_params(**dict(pr.params, n_leaf=leaf))
    ref = orc.Tree(p, pr.x, pr.y, pr.z, pr.m, n_active=na).export()
    g = _tree(pr, leaf, na, moments_level_log2=6, group_size=group)
    _check_tree(g, ref, pr.params["quadrupole"])
    d = _tree(pr, leaf, na, group_size=group)
    for k in ("M", "com", "Q", "skip"):
        np.testing.assert_array_equal(g[k], d[k], err_msg=k)


@pytest.mark.parametrize("precision", [0, 1])
def test_level_by_level_moments_in_steps(precision):
    # FP32-mixed steps keep FP64 records only where the walk needs them; the
    # level-by-level path must give the same steps as the one-workgroup path
    from gpu_util import Dev, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.sheet(9000, seed=12)
    out = []
    for lv in (0, 6):
        ctx = make_ctx(pr, precision=precision, moments_level_log2=lv)
        try:
            d = Dev(pr)
            rb.rb_step(ctx, d.parts, d.n, d.n, 0.0, pr.dt, 3)
            rb.rb_sync(ctx)
            out.append(d.state())
        finally:
            rb.rb_destroy(ctx)
    for k in out[0]:
        np.testing.assert_array_equal(out[0][k], out[1][k], err_msg=k)


_BIG = {}


def _big(orc):
    # a Plummer sphere of 4.5 * 2^20 particles (above 2^22: the large-node
    # moments run level by level), softening 0.001, quadrupoles
    if not _BIG:
        pr = inputs.plummer(4_718_592, seed=11, b=0.001, quadrupole=True, dt=1e-4)
        print(f"[large] oracle tree of {pr.n} particles", flush=True)
        p = orc.make_params(**dict(pr.params, theta=0.5))
        _BIG["pr"] = pr
        _BIG["tree"] = orc.Tree(p, pr.x, pr.y, pr.z, pr.m)
        _BIG["tg"] = inputs.sample_targets(pr.n, 4096, seed=0)
    return _BIG


def test_above_2p22_tree_and_fp64_walk_match_oracle(orc):
    from gpu_util import Dev, export, gravity, make_ctx, rms_rel
    from paper_1110_4876_amd import rb
    b = _big(orc)
    pr, T, tg = b["pr"], b["tree"], b["tg"]
    assert pr.n > (1 << 22)
    ref_a = T.walk(targets=tg)
    ctx = make_ctx(pr.with_params(theta=0.5))
    try:
        d = Dev(pr, with_v=False)
        a = gravity(ctx, d, pr.n)
        g = export(ctx)
    finally:
        rb.rb_destroy(ctx)
    assert rms_rel(a[tg], ref_a) <= 1e-12, rms_rel(a[tg], ref_a)
    # identical opening decisions leave only rounding in every particle
    err = np.linalg.norm(a[tg] - ref_a, axis=1) / np.linalg.norm(ref_a, axis=1)
    assert err.max() <= 1e-10, err.max()
    _check_tree(g, T.export(), True)


def test_above_2p22_fp32_mixed_meets_gate(orc):
    # FP32-mixed at the 2^23 Plummer workload's operating point against the
    # FP64 direct sum of Eq. (1) on 2048 sampled targets
    from gpu_util import Dev, gravity, make_ctx
    from paper_1110_4876_amd import autotune, rb
    from paper_1110_4876_amd.metrics import force_errors
    b = _big(orc)
    pr = b["pr"]
    op = autotune.operating_point("plummer8m", "fp32")
    tg = b["tg"][::2]
    p = orc.make_params(**pr.params)
    print(f"[large] oracle direct sum for {len(tg)} targets", flush=True)
    ref = orc.direct(p, pr.x, pr.y, pr.z, pr.m, targets=tg)
    for waves in sorted({1, op["walk_waves"]}):
        kn = {k: op[k] for k in autotune.KNOBS if k != "walk_waves"}
        ctx = make_ctx(pr, precision=rb.RB_FP32_MIXED, walk_waves=waves, **kn)
        try:
            a = gravity(ctx, Dev(pr, with_v=False), pr.n)
        finally:
            rb.rb_destroy(ctx)
        e = force_errors(a[tg], ref)
        assert e["rms"] <= 1e-4, (waves, e)
