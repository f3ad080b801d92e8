"""Pins of the oracle's forest of root boxes (Sect. 2.3: the domain is an
integer number of cubic root boxes per axis, one tree per root box) and of
its tree reconstruction after the particles moved (Sect. 4.2), against brute
force, single-box trees, closed forms and the fresh build."""
import math

import numpy as np
import pytest

DEAD = np.uint64(2 ** 64 - 1)


def _virtual_levels(n_root):
    # levels above the root boxes: 2^D >= the most boxes along any axis
    return int(math.ceil(math.log2(max(n_root)))) if max(n_root) > 1 else 0


def _points(rng, n, n_root, W=1.0, x0=(0.0, 0.0, 0.0)):
    return [x0[a] + rng.uniform(0.0, n_root[a] * W, n) for a in range(3)]


def _brute_force_forest(keys, n_leaf, D):
    """Canonical nodes of every root box's tree by counting prefixes: the
    level-D prefix of an occupied root box is its root; a deeper prefix is a
    node iff its parent holds more than n_leaf particles; leaves hold at
    most n_leaf particles or lie on level 21."""
    keys = np.sort(keys[keys != DEAD])
    counts = {}
    for l in range(D, 22):
        pre = keys >> np.uint64(3 * (21 - l))
        u, c = np.unique(pre, return_counts=True)
        counts[l] = dict(zip(u.tolist(), c.tolist()))
    nodes = []
    for l in range(D, 22):
        for pre, c in sorted(counts[l].items()):
            if l > D and counts[l - 1][pre >> 3] <= n_leaf:
                continue
            nodes.append((l, pre, c, int(c <= n_leaf or l == 21)))
    return nodes


@pytest.mark.parametrize("n_root", [(2, 1, 1), (3, 2, 1), (4, 1, 1), (2, 2, 2), (5, 3, 1)])
@pytest.mark.parametrize("n_leaf", [1, 4])
def test_forest_topology_matches_brute_force(orc, n_root, n_leaf):
    rng = np.random.default_rng(sum(n_root) * 10 + n_leaf)
    x, y, z = _points(rng, 3000, n_root, W=2.0, x0=(-1.0, -3.0, 0.5))
    # a tight clump (deep cells) inside one box
    x[:200] = -1.0 + 1.3 + rng.normal(0, 1e-4, 200)
    p = orc.make_params(W=2.0, x0=(-1.0, -3.0, 0.5), n_leaf=n_leaf, n_root=n_root)
    T = orc.Tree(p, x, y, z, np.ones(3000))
    assert T.selfcheck()
    e = T.export()
    D = _virtual_levels(n_root)
    ref = _brute_force_forest(orc.keys(p, x, y, z), n_leaf, D)
    got = list(zip(e["level"].tolist(), e["prefix"].tolist(), e["count"].tolist(),
                   e["is_leaf"].tolist()))
    assert got == ref
    # one root per occupied box
    assert int(np.sum(e["level"] == D)) == len(np.unique(
        orc.keys(p, x, y, z) >> np.uint64(3 * (21 - D))))


@pytest.mark.parametrize("n_root", [(3, 2, 1), (4, 1, 1), (2, 2, 2)])
def test_root_box_of_a_particle(orc, n_root):
    # away from the faces, the root box named by a key's first D digits is
    # floor((x - x0) / W) on every axis
    rng = np.random.default_rng(3)
    W, x0 = 1.5, (2.0, -1.0, 0.0)
    D = _virtual_levels(n_root)
    cells = np.stack([rng.integers(0, n_root[a], 500) for a in range(3)], 1)
    frac = rng.uniform(0.01, 0.99, (500, 3))
    pts = np.array(x0) + (cells + frac) * W
    p = orc.make_params(W=W, x0=x0, n_root=n_root)
    k = orc.keys(p, pts[:, 0], pts[:, 1], pts[:, 2])
    pre = (k >> np.uint64(3 * (21 - D))).astype(np.int64)
    dec = np.zeros((500, 3), np.int64)
    for j in range(D):
        d = (pre >> (3 * (D - 1 - j))) & 7
        dec[:, 0] = dec[:, 0] * 2 + (d >> 2 & 1)
        dec[:, 1] = dec[:, 1] * 2 + (d >> 1 & 1)
        dec[:, 2] = dec[:, 2] * 2 + (d & 1)
    np.testing.assert_array_equal(dec, cells)
    # outside the domain: no key
    out = orc.keys(p, [x0[0] + n_root[0] * W + 1e-9], [0.0], [0.5])
    assert out[0] == DEAD


def test_forest_is_a_tree_per_root_box(orc):
    # a 2x1x1 forest of unit boxes at the origin (power-of-two scales, so
    # both quantisations are exact) has, in each box, the tree a single box
    # of side 1 at that box's corner builds from the box's particles; its
    # walk is the sum of the two single trees' walks
    rng = np.random.default_rng(7)
    n = 3000
    x, y, z = rng.uniform(0, 2, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)
    m = rng.uniform(0.5, 1.5, n)
    pf = orc.make_params(W=1.0, x0=(0.0, 0.0, 0.0), n_root=(2, 1, 1), quadrupole=True,
                         theta=0.6)
    F = orc.Tree(pf, x, y, z, m).export()
    for box in (0, 1):
        sel = np.nonzero((x >= box) & (x < box + 1))[0]
        ps = orc.make_params(W=1.0, x0=(float(box), 0.0, 0.0), quadrupole=True, theta=0.6)
        Ts = orc.Tree(ps, x[sel], y[sel], z[sel], m[sel])
        S = Ts.export()
        # the forest's nodes of this box: level + 1, prefix behind the box digit
        mine = (F["prefix"] >> (3 * (F["level"].astype(np.int64) - 1)).astype(np.uint64)) == \
            np.uint64(4 * box)
        mine &= F["level"] >= 1
        np.testing.assert_array_equal(F["level"][mine] - 1, S["level"])
        np.testing.assert_array_equal(
            F["prefix"][mine] - (np.uint64(4 * box) << (3 * (F["level"][mine].astype(np.int64)
                                                             - 1)).astype(np.uint64)),
            S["prefix"])
        np.testing.assert_array_equal(F["count"][mine], S["count"])
        np.testing.assert_array_equal(F["M"][mine], S["M"])
        np.testing.assert_array_equal(F["com"][mine], S["com"])
    full = orc.Tree(pf, x, y, z, m).walk()
    # the walk over both boxes is the sum of the two single-box walks: each
    # box's tree on every particle (targets indexed past the box's own
    # particles, so no target is taken for a member), members on themselves
    ref = np.zeros((n, 3))
    for box in (0, 1):
        sel = np.nonzero((x >= box) & (x < box + 1))[0]
        ps = orc.make_params(W=1.0, x0=(float(box), 0.0, 0.0), quadrupole=True, theta=0.6)
        Ts = orc.Tree(ps, x[sel], y[sel], z[sel], m[sel])
        k = len(sel)
        part = Ts.walk(x=np.concatenate([x[sel], x]), y=np.concatenate([y[sel], y]),
                       z=np.concatenate([z[sel], z]), targets=k + np.arange(n))
        part[sel] = Ts.walk(targets=np.arange(k))
        ref += part
    err = np.linalg.norm(full - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert err.max() <= 1e-13, err.max()


def test_forest_theta_zero_equals_direct_sum(orc):
    # theta = 0 opens every cell: the walk over all root boxes and ghost
    # images is the direct sum of Eq. (1) over the elongated domain's images
    from paper_1110_4876_amd import inputs
    rng = np.random.default_rng(11)
    n_root = (4, 1, 1)
    W = 10.0
    n = 1500
    x0 = (-0.5 * 4 * W, -0.5 * W, -0.5 * W)
    x, y = x0[0] + rng.uniform(0, 4 * W, n), x0[1] + rng.uniform(0, W, n)
    z = rng.normal(0, 0.5, n)
    m = rng.uniform(0.5, 1.5, n)
    for bnd in (inputs.PERIODIC, inputs.SHEAR):
        p = orc.make_params(W=W, x0=x0, n_root=n_root, boundary=bnd, ng=(1, 1), theta=0.0,
                            omega=0.01)
        s = orc.shear_offset(p, 37.0)
        a = orc.bh(p, x, y, z, m, s=s)
        d = orc.direct(p, x, y, z, m, s=s)
        assert np.sqrt(np.sum((a - d) ** 2) / np.sum(d ** 2)) <= 1e-13


def test_root_box_is_accepted_with_its_own_width(orc):
    # a compact cloud in root box 0 of a 3x1x1 forest of side W and a massless
    # target in box 2: box 0's tree root has width W, so at W / R < theta the
    # whole box acts through its monopole and quadrupole (closed form); were
    # the width that of a larger cell, the walk would open it
    rng = np.random.default_rng(2)
    W = 1.0
    n = 200
    c = np.array([0.5, 0.5, 0.5])
    pts = c + rng.normal(0, 0.05, (n, 3))
    m = rng.uniform(0.5, 1.5, n)
    tgt = np.array([2.9, 0.5, 0.5])
    R = np.linalg.norm(tgt - np.sum(m[:, None] * pts, 0) / m.sum())
    theta = 1.1 * W / R
    assert theta < 1.0
    x = np.concatenate([pts[:, 0], [tgt[0]]])
    y = np.concatenate([pts[:, 1], [tgt[1]]])
    z = np.concatenate([pts[:, 2], [tgt[2]]])
    mm = np.concatenate([m, [0.0]])
    p = orc.make_params(W=W, x0=(0.0, 0.0, 0.0), n_root=(3, 1, 1), theta=theta,
                        quadrupole=True)
    a = orc.bh(p, x, y, z, mm, n_active=n, targets=[n])[0]
    M = m.sum()
    com = np.sum(m[:, None] * pts, 0) / M
    sv = pts - com
    Q = np.einsum("i,ij,ik->jk", m, 3 * sv, sv) - np.eye(3) * np.sum(m * np.sum(sv * sv, 1))
    d = com - tgt
    r = np.linalg.norm(d)
    ref = M * d / r ** 3 - Q @ d / r ** 5 + 2.5 * (d @ Q @ d) * d / r ** 7
    assert np.linalg.norm(a - ref) <= 1e-13 * np.linalg.norm(ref)
    # at half that theta the box is opened and the answer moves closer to
    # the direct sum
    p2 = orc.make_params(W=W, x0=(0.0, 0.0, 0.0), n_root=(3, 1, 1), theta=0.5 * theta,
                         quadrupole=True)
    a2 = orc.bh(p2, x, y, z, mm, n_active=n, targets=[n])[0]
    dd = orc.direct(p2, x, y, z, mm, n_active=n, targets=[n])[0]
    assert np.linalg.norm(a2 - dd) < np.linalg.norm(a - dd)


def test_forest_shear_image_follows_the_drifted_particle(orc):
    # the geometry pin of the shear-periodic boundaries on an elongated
    # domain (Lx = 4 W, Ly = W): a particle wrapped across the +x face keeps
    # its ghost image in the domain copy at +Lx on the track of the same
    # particle drifted without the wrap
    W, om = 500.0, 2e-4
    Lx = 4 * W
    p = orc.make_params(G=1.0, W=W, x0=(-0.5 * Lx, -0.5 * W, -0.5 * W), n_root=(4, 1, 1),
                        boundary=orc.SHEAR, ng=(1, 1), drift=orc.EPICYCLE, omega=om)
    t1 = 0.31 * 2 * math.pi / om
    for slide in (20.0, 60.0, 150.0):
        tau = slide / (1.5 * om * Lx)
        x1 = 0.5 * Lx + 0.25
        src = dict(x=np.array([x1]), y=np.array([-100.0]), z=np.array([0.5]),
                   vx=np.array([0.02]), vy=np.array([-1.5 * om * x1 + 0.01]),
                   vz=np.array([0.0]))
        wr = orc.boundary(p, src, orc.shear_offset(p, t1))
        assert wr["x"][0] < 0
        free = orc.drift(p, src, tau)
        moved = orc.drift(p, wr, tau)
        s2 = orc.shear_offset(p, t1 + tau)
        tx, ty, tz = free["x"][0] + 0.8, free["y"][0], free["z"][0]
        a = orc.direct(p, [moved["x"][0], tx], [moved["y"][0], ty], [moved["z"][0], tz],
                       np.array([1.0, 0.0]), n_active=1, s=s2, targets=[1])[0]
        a_near = np.array([-0.8, 0.0, 0.0]) / 0.8 ** 3
        assert np.linalg.norm(a - a_near) <= 1e-4 * np.linalg.norm(a_near), slide


def test_forest_periodic_wrap_uses_the_domain(orc):
    # periodic boundaries on a 3x2x1 forest wrap at the domain's faces
    W = 2.0
    p = orc.make_params(W=W, x0=(0.0, 0.0, 0.0), n_root=(3, 2, 1), boundary=orc.PERIODIC,
                        ng=(1, 1))
    st = dict(x=np.array([6.5, -0.25, 3.0]), y=np.array([1.0, 2.0, 4.125]),
              z=np.array([0.5, 0.5, 0.5]), vx=np.ones(3), vy=np.ones(3), vz=np.ones(3))
    out = orc.boundary(p, st, 0.0)
    np.testing.assert_array_equal(out["x"], [0.5, 5.75, 3.0])
    np.testing.assert_array_equal(out["y"], [1.0, 2.0, 0.125])


def _same_tree(a, b):
    for k in ("level", "prefix", "first", "count", "is_leaf", "n_child", "first_child",
              "perm", "keys", "M", "com", "Q"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def _leaf_prefix_of_each(e, n):
    """(level, prefix) of the leaf holding each particle, from an export"""
    out = {}
    for v in np.nonzero(e["is_leaf"])[0]:
        for r in range(e["first"][v], e["first"][v] + e["count"][v]):
            out[int(e["perm"][r])] = (int(e["level"][v]), int(e["prefix"][v]))
    return out


@pytest.mark.parametrize("n_root", [(1, 1, 1), (3, 2, 1)])
@pytest.mark.parametrize("n_leaf", [1, 4])
@pytest.mark.parametrize("scale", [0.0, 1e-7, 1e-3, 0.05, 0.4])
def test_reconstruction_equals_fresh_build(orc, n_root, n_leaf, scale):
    # move the particles by ~scale box sides (some leave their cells, at 0.4
    # many change root box and some leave the open domain), reconstruct: the
    # tree is the fresh build's, bit for bit, and the particles re-inserted
    # are exactly those no longer inside their old leaf's cell
    rng = np.random.default_rng(int(scale * 1e7) % 1000 + 17 * n_leaf)
    n = 2500
    W = 1.0
    x, y, z = _points(rng, n, n_root, W=W)
    x[:100] = 0.2 + rng.normal(0, 1e-5, 100)  # deep cells
    m = rng.uniform(0.5, 1.5, n)
    p = orc.make_params(W=W, x0=(0.0, 0.0, 0.0), n_root=n_root, n_leaf=n_leaf,
                        quadrupole=True, theta=0.5)
    T = orc.Tree(p, x, y, z, m, n_active=n - 300)
    old = T.export()
    leaf_of = _leaf_prefix_of_each(old, n)
    x2 = x + rng.normal(0, scale * W, n)
    y2 = y + rng.normal(0, scale * W, n)
    z2 = z + rng.normal(0, scale * W, n)
    moved = T.update(x2, y2, z2)
    k2 = orc.keys(p, x2, y2, z2)
    expect = sum(1 for j, (l, pre) in leaf_of.items()
                 if k2[j] != DEAD and int(k2[j] >> np.uint64(3 * (21 - l))) != pre)
    assert moved == expect
    assert T.selfcheck()
    fresh = orc.Tree(p, x2, y2, z2, m, n_active=n - 300)
    _same_tree(T.export(), fresh.export())
    np.testing.assert_array_equal(T.walk(), fresh.walk())
    if scale == 0.0:
        assert moved == 0
