"""GPU tree build (keys, sort, topology, moments) against the oracle's
insertion tree: Morton order and topology bit-exact, centre of mass bitwise,
quadrupoles to rounding."""
import numpy as np
import pytest

from paper_1110_4876_amd import inputs

pytestmark = pytest.mark.gpu

CASES = [
    ("plummer1024", lambda: inputs.plummer(1024, seed=0), 1, None),
    ("plummer5000_leaf4", lambda: inputs.plummer(5000, seed=3, quadrupole=True), 4, None),
    ("e1box1000_quad", lambda: inputs.e1_box(1000, 0, quadrupole=True), 1, None),
    ("sheet7000", lambda: inputs.sheet(7000, seed=1), 1, None),
    ("sheet7000_leaf8", lambda: inputs.sheet(7000, seed=1), 8, None),
    ("plummer3000_testparticles", lambda: inputs.plummer(3000, seed=4, quadrupole=True), 1, 2100),
]


def _dfs_skip(e):
    """next node after each subtree in depth-first octant order (-1 at end)"""
    nn = len(e["level"])
    skip = np.full(nn, -1, np.int64)

    def visit(v, after):
        skip[v] = after
        if e["is_leaf"][v]:
            return
        c0, nc = e["first_child"][v], e["n_child"][v]
        for k in range(nc):
            visit(c0 + k, c0 + k + 1 if k + 1 < nc else after)
    import sys
    sys.setrecursionlimit(10000)
    if nn:
        visit(0, -1)
    return skip


@pytest.mark.parametrize("name,maker,leaf,n_active", CASES, ids=[c[0] for c in CASES])
def test_tree_matches_oracle(orc, name, maker, leaf, n_active):
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    pr = maker()
    na = pr.n if n_active is None else n_active
    p = orc.make_params(**dict(pr.params, n_leaf=leaf))
    ref = orc.Tree(p, pr.x, pr.y, pr.z, pr.m, n_active=na).export()
    ctx = make_ctx(pr, leaf_size=leaf)
    try:
        d = Dev(pr, with_v=False)
        rb.rb_tree_build(ctx, d.parts, d.n, na)
        g = export(ctx)
    finally:
        rb.rb_destroy(ctx)
    for k in ("keys", "perm", "level", "prefix", "first", "count", "is_leaf"):
        np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
    internal = ref["is_leaf"] == 0
    np.testing.assert_array_equal(g["n_child"][internal], ref["n_child"][internal])
    np.testing.assert_array_equal(g["first_child"][internal], ref["first_child"][internal])
    np.testing.assert_array_equal(g["skip"], _dfs_skip(ref))
    # M and the centre of mass round identically (same summation order)
    np.testing.assert_array_equal(g["M"], ref["M"])
    np.testing.assert_array_equal(g["com"], ref["com"])
    if pr.params["quadrupole"]:
        scale = np.abs(ref["Q"]).max(axis=1, keepdims=True) + 1e-300
        assert np.abs(g["Q"] - ref["Q"]).max() <= 1e-13 * scale.max()
        assert (np.abs(g["Q"] - ref["Q"]) <= 1e-12 * scale).all()


def test_duplicate_positions_and_removed_particles(orc):
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.plummer(600, seed=5)
    pr.x[10:14] = pr.x[3]; pr.y[10:14] = pr.y[3]; pr.z[10:14] = pr.z[3]  # 5 equal keys
    pr.x[20] = np.nan                                                  # tombstone
    pr.x[21] = 100.0                                                   # outside: removed
    p = orc.make_params(**pr.params)
    ref = orc.Tree(p, pr.x, pr.y, pr.z, pr.m).export()
    ctx = make_ctx(pr)
    try:
        d = Dev(pr, with_v=False)
        rb.rb_tree_build(ctx, d.parts, d.n, d.n)
        nn, nl = rb.rb_tree_info(ctx)
        g = export(ctx)
    finally:
        rb.rb_destroy(ctx)
    assert nl == pr.n - 2
    for k in ("keys", "perm", "level", "prefix", "first", "count", "is_leaf"):
        np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
    np.testing.assert_array_equal(g["com"], ref["com"])


def test_single_and_tiny_systems(orc):
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    for n in (1, 2, 3, 65, 2049):
        pr = inputs.plummer(n, seed=n)
        p = orc.make_params(**pr.params)
        ref = orc.Tree(p, pr.x, pr.y, pr.z, pr.m).export()
        ctx = make_ctx(pr, capacity=4096)
        try:
            d = Dev(pr, with_v=False)
            rb.rb_tree_build(ctx, d.parts, d.n, d.n)
            g = export(ctx)
        finally:
            rb.rb_destroy(ctx)
        for k in ("perm", "level", "prefix", "first", "count", "is_leaf"):
            np.testing.assert_array_equal(g[k], ref[k], err_msg=f"n={n} {k}")


def test_tree_build_is_deterministic():
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.sheet(20000, seed=9)
    ctx = make_ctx(pr)
    try:
        d = Dev(pr, with_v=False)
        rb.rb_tree_build(ctx, d.parts, d.n, d.n)
        a = export(ctx)
        rb.rb_tree_build(ctx, d.parts, d.n, d.n)
        b = export(ctx)
    finally:
        rb.rb_destroy(ctx)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("n", [300_000, 700_000, 1_200_000])
def test_morton_order_at_large_sizes(orc, n):
    # the radix sort's larger tile shapes (2, 4 and 8 rows per wave) and the
    # topology at sizes beyond the oracle's insertion tree: sorted keys and
    # permutation equal a stable sort of the oracle's keys; node counts
    # per level equal the number of distinct prefixes of every level (with
    # leaf size 1 a prefix is a node iff its parent holds more than one)
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    pr = inputs.plummer(n, seed=9)
    # a few exact duplicates and removed particles exercise ties and sentinels
    pr.x[10:20] = pr.x[0]; pr.y[10:20] = pr.y[0]; pr.z[10:20] = pr.z[0]
    pr.x[30:33] = np.nan
    p = orc.make_params(**pr.params)
    k = orc.keys(p, pr.x, pr.y, pr.z)
    live = k != np.uint64(0xFFFFFFFFFFFFFFFF)
    order = np.argsort(k, kind="stable")
    ref_keys, ref_perm = k[order][: live.sum()], order[: live.sum()]
    ctx = make_ctx(pr)
    try:
        rb.rb_tree_build(ctx, Dev(pr, with_v=False).parts, pr.n, pr.n)
        g = export(ctx)
    finally:
        rb.rb_destroy(ctx)
    np.testing.assert_array_equal(g["keys"], ref_keys)
    np.testing.assert_array_equal(g["perm"], ref_perm)
    # nodes per level: a level-l prefix is a node iff its level-(l-1) parent
    # holds more than one particle
    lv = g["level"]
    for l in range(1, 22):
        sh = np.uint64(3 * (21 - l))
        pre = ref_keys >> sh
        par = ref_keys >> np.uint64(3 * (22 - l))
        up, pc = np.unique(par, return_counts=True)
        uniq = np.unique(pre)
        expect = int(np.isin(uniq >> np.uint64(3), up[pc > 1]).sum())
        assert int(np.sum(lv == l)) == expect, l


@pytest.mark.parametrize("n_dead", [0, 40, 700])
def test_clustered_ties_and_removed(orc, n_dead):
    # most particles inside one cell of level 4 (one bucket of the small-
    # system sort larger than a segment), runs of equal keys, and removed
    # particles in numbers below and above a segment: Morton order, ties in
    # index order, and the topology still equal the oracle's
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    rng = np.random.default_rng(17)
    pr = inputs.plummer(6000, seed=8)
    pr.x[:5000] = 3.0 + rng.uniform(0, 1.5, 5000)
    pr.y[:5000] = 3.0 + rng.uniform(0, 1.5, 5000)
    pr.z[:5000] = 3.0 + rng.uniform(0, 1.5, 5000)
    for j in range(0, 600, 6):  # runs of six equal keys
        pr.x[j + 1:j + 6] = pr.x[j]; pr.y[j + 1:j + 6] = pr.y[j]; pr.z[j + 1:j + 6] = pr.z[j]
    pr.x[5000:5000 + n_dead] = np.nan
    p = orc.make_params(**pr.params)
    ref = orc.Tree(p, pr.x, pr.y, pr.z, pr.m).export()
    ctx = make_ctx(pr)
    try:
        d = Dev(pr, with_v=False)
        rb.rb_tree_build(ctx, d.parts, d.n, d.n)
        nn, nl = rb.rb_tree_info(ctx)
        g = export(ctx)
    finally:
        rb.rb_destroy(ctx)
    assert nl == pr.n - n_dead
    for k in ("keys", "perm", "level", "prefix", "first", "count", "is_leaf"):
        np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
    np.testing.assert_array_equal(g["com"], ref["com"])


@pytest.mark.parametrize("level_log2", [None, 6])
def test_single_particle_leaves_are_point_masses(level_log2):
    # The FP64 walk evaluates a single-particle leaf through the cell terms;
    # they equal the point mass's term exactly only because the build puts
    # the leaf's centre of mass at the particle itself and leaves its
    # quadrupole exactly zero (Sect. 4.2: a leaf's moments are those of its
    # particles).  Both moment paths: groups and large nodes in one
    # workgroup, and level by level (forced above 64 slots).
    from gpu_util import Dev, export, make_ctx
    from paper_1110_4876_amd import rb
    kw = {} if level_log2 is None else dict(moments_level_log2=level_log2)
    for pr, leaf in ((inputs.sheet(20000, seed=2), 1),
                     (inputs.plummer(8000, seed=7, quadrupole=True), 4)):
        ctx = make_ctx(pr, leaf_size=leaf, **kw)
        try:
            d = Dev(pr, with_v=False)
            rb.rb_tree_build(ctx, d.parts, d.n, d.n)
            g = export(ctx)
        finally:
            rb.rb_destroy(ctx)
        one = (g["is_leaf"] != 0) & (g["count"] == 1)
        assert one.sum() > 100
        assert (g["Q"][one] == 0.0).all()
        src = g["perm"][g["first"][one]]
        pos = np.stack([pr.x[src], pr.y[src], pr.z[src]], axis=1)
        np.testing.assert_array_equal(g["com"][one], pos)
        np.testing.assert_array_equal(g["M"][one], pr.m[src])
