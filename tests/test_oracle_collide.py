"""Pins of the oracle's collisions (Sect. 5): the splitmix64 order against
published outputs, the hard-sphere resolution against closed forms and
conservation laws, detection against brute force on tiny inputs, and the
sequential (queue-order) semantics of several collisions on one particle."""
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def _open(orc, W=100.0):
    return orc.make_params(W=W, x0=(-W / 2, -W / 2, -W / 2), boundary=orc.OPEN)


def _state(x, v):
    x = np.asarray(x, float); v = np.asarray(v, float)
    return dict(x=x[:, 0].copy(), y=x[:, 1].copy(), z=x[:, 2].copy(),
                vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy())


def _v(s):
    return np.stack([s["vx"], s["vy"], s["vz"]], 1)


def test_splitmix64_published_outputs(orc):
    g = 0x9E3779B97F4A7C15
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    for k, h in rows:
        assert orc.splitmix64(int(k) * g) == int(h, 16)


def test_head_on_closed_form(orc):
    # 1-D collision along x: v1' = (m1 v1 + m2 v2 + m2 eps (v2 - v1)) / M,
    # v2' = (m1 v1 + m2 v2 - m1 eps (v2 - v1)) / M
    p = _open(orc)
    m = np.array([2.0, 3.0]); R = np.array([1.0, 1.5])
    v1, v2, eps = 0.7, -0.4, 0.5
    st = _state([[0, 0, 0], [2.0, 0, 0]], [[v1, 0, 0], [v2, 0, 0]])
    codes, npair, nres, out = orc.collide(p, st, m, R, 0.0, eps, 1234)
    assert npair == 1 and nres == 1 and int(codes[0]) == (0 << 35) | (1 << 7) | 0
    M = m.sum()
    e1 = (m[0] * v1 + m[1] * v2 + m[1] * eps * (v2 - v1)) / M
    e2 = (m[0] * v1 + m[1] * v2 - m[0] * eps * (v2 - v1)) / M
    assert abs(out["vx"][0] - e1) < 1e-15 and abs(out["vx"][1] - e2) < 1e-15
    assert out["vy"][0] == 0.0 and out["vz"][1] == 0.0
    # positions are untouched
    assert out["x"][1] == 2.0


def test_oblique_normal_reversed_tangent_kept(orc):
    p = _open(orc)
    rng = np.random.default_rng(3)
    for eps in (0.0, 0.3, 1.0):
        m = rng.uniform(0.5, 2.0, 2); R = np.array([1.0, 1.0])
        d = rng.normal(size=3); d *= 1.5 / np.linalg.norm(d)      # overlapping
        n = d / np.linalg.norm(d)
        v = rng.normal(size=(2, 3))
        u = v[1] - v[0]
        if u @ d >= 0:                                              # make them approach
            v[1] -= 2 * (u @ n) * n
            u = v[1] - v[0]
        st = _state([[0, 0, 0], d], v)
        _, npair, nres, out = orc.collide(p, st, m, R, 0.0, eps, 7)
        assert npair == 1 and nres == 1
        w = _v(out)
        u2 = w[1] - w[0]
        un, un2 = u @ n, u2 @ n
        assert abs(un2 + eps * un) < 1e-13 * (1 + abs(un))
        np.testing.assert_allclose(u2 - un2 * n, u - un * n, atol=1e-13)
        P0, P1 = m @ v, m @ w
        np.testing.assert_allclose(P1, P0, atol=1e-13)
        # kinetic energy lost: (1 - eps^2) mu un^2 / 2
        mu = m[0] * m[1] / m.sum()
        dE = 0.5 * (m @ (v * v).sum(1) - m @ (w * w).sum(1))
        assert abs(dE - 0.5 * mu * (1 - eps * eps) * un * un) < 1e-12


def test_separating_or_apart_pairs(orc):
    p = _open(orc)
    m = np.ones(2); R = np.ones(2)
    # overlapping but moving apart: queued, not resolved
    st = _state([[0, 0, 0], [1.0, 0, 0]], [[-0.1, 0, 0], [0.2, 0, 0]])
    _, npair, nres, out = orc.collide(p, st, m, R, 0.0, 0.5, 1)
    assert npair == 1 and nres == 0
    np.testing.assert_array_equal(_v(out), _v(st))
    # touching exactly (|d| = R_i + R_j) is not an overlap; apart is not either
    for dx in (2.0, 2.5):
        st = _state([[0, 0, 0], [dx, 0, 0]], [[1, 0, 0], [-1, 0, 0]])
        _, npair, nres, _ = orc.collide(p, st, m, R, 0.0, 0.5, 1)
        assert npair == 0 and nres == 0


def test_shear_image_pair(orc):
    # particle 0 at the -x edge overlaps the image (ix = -1, iy = 0) of
    # particle 1 at the +x edge; that image moves with the shear flow,
    # y velocity offset -3/2 Omega W ix = +3/2 Omega W
    W, om = 10.0, 0.2
    p = orc.make_params(W=W, x0=(-W / 2, -W / 2, -W / 2), boundary=orc.SHEAR, ng=(1, 1),
                        omega=om)
    m = np.array([1.0, 2.0]); R = np.array([0.5, 0.5])
    k = (-1 + 1) * 3 + (0 + 1)  # images: ix outer, iy inner, both in [-1, 1]

    def run(vx0, vx1):
        st = _state([[-4.8, 0.1, 0.0], [4.7, 0.1, 0.0]], [[vx0, 0.0, 0.0], [vx1, 0.0, 0.0]])
        return orc.collide(p, st, m, R, 0.0, 1.0, 5)
    # d = (4.7 - 10) - (-4.8) = -0.5 along x (the image sits left of 0)
    codes, npair, nres, _ = run(0.0, 0.0)
    assert npair == 1 and int(codes[0]) == (0 << 35) | (1 << 7) | k
    assert nres == 0            # u = (0, 3/2 Omega W, 0) is normal to d
    _, _, nres, _ = run(0.0, -0.3)
    assert nres == 0            # the image moves away from particle 0
    _, _, nres, out = run(0.0, 0.3)
    assert nres == 1            # the image approaches: 1-D elastic exchange in x
    M = m.sum()
    assert abs(out["vx"][0] - (2 * m[1] * 0.3) / M) < 1e-15
    assert abs(out["vx"][1] - ((m[1] - m[0]) * 0.3) / M) < 1e-15
    assert out["vy"][0] == 0.0 and out["vy"][1] == 0.0   # tangential: unchanged


def test_detection_brute_force_tiny(orc):
    rng = np.random.default_rng(11)
    W = 20.0
    for boundary, ng in ((orc.OPEN, (0, 0)), (orc.PERIODIC, (1, 1)), (orc.SHEAR, (1, 1))):
        p = orc.make_params(W=W, x0=(-W / 2, -W / 2, -W / 2), boundary=boundary, ng=ng,
                            omega=0.3)
        n = 60
        x = rng.uniform(-W / 2, W / 2, (n, 3)); x[:, 2] *= 0.1
        R = rng.uniform(0.5, 2.0, n)
        st = _state(x, np.zeros((n, 3)))
        t = 1.7
        codes, npair, _, _ = orc.collide(p, st, np.ones(n), R, t, 0.5, 9)
        s = orc.shear_offset(p, t) if boundary == orc.SHEAR else 0.0
        want = set()
        ks = [(0, 0)] if boundary == orc.OPEN else [(ix, iy) for ix in (-1, 0, 1) for iy in (-1, 0, 1)]
        for i in range(n):
            for j in range(i + 1, n):
                for k, (ix, iy) in enumerate(ks):
                    o = np.array([ix * W, iy * W - ix * s, 0.0])
                    if np.sum((x[j] + o - x[i]) ** 2) < (R[i] + R[j]) ** 2:
                        want.add((i << 35) | (j << 7) | k)
        assert npair == len(want) and set(int(c) for c in codes) == want


def test_queue_order_and_sequential_resolution(orc):
    # particle 1 overlaps 0 and 2; the result is the two pairwise collisions
    # applied one after the other in ascending splitmix64(seed + code)
    p = _open(orc)
    m = np.array([1.0, 1.5, 2.0]); R = np.array([1.0, 1.0, 1.0])
    x = [[-1.8, 0.0, 0.0], [0.0, 0.0, 0.0], [1.6, 0.3, 0.0]]
    v = [[1.0, 0.0, 0.0], [0.0, 0.2, 0.0], [-0.8, 0.1, 0.0]]
    eps = 0.4

    def pair(vv, i, j):
        d = np.array(x[j], float) - np.array(x[i], float)
        u = vv[j] - vv[i]
        if u @ d >= 0:
            return vv
        n = d / np.linalg.norm(d)
        f = (1 + eps) * (u @ n)
        M = m[i] + m[j]
        vv = vv.copy()
        vv[i] = vv[i] + (m[j] / M) * f * n
        vv[j] = vv[j] - (m[i] / M) * f * n
        return vv
    for seed in (1, 2, 3, 4):
        codes, npair, nres, out = orc.collide(p, _state(x, v), m, R, 0.0, eps, seed)
        assert npair == 2
        c01, c12 = (0 << 35) | (1 << 7), (1 << 35) | (2 << 7)
        first = c01 if orc.splitmix64(seed + c01) < orc.splitmix64(seed + c12) else c12
        assert int(codes[0]) == first
        vv = np.array(v, float)
        for c in ([c01, c12] if first == c01 else [c12, c01]):
            vv = pair(vv, c >> 35, (c >> 7) & ((1 << 28) - 1))
        np.testing.assert_allclose(_v(out), vv, atol=1e-14)


def test_momentum_conserved_many(orc):
    rng = np.random.default_rng(21)
    p = _open(orc, W=40.0)
    n = 400
    x = rng.uniform(-8, 8, (n, 3))
    v = rng.normal(size=(n, 3))
    m = rng.uniform(0.5, 3.0, n); R = rng.uniform(0.3, 1.0, n)
    _, npair, nres, out = orc.collide(p, _state(x, v), m, R, 0.0, 0.5, 99)
    assert npair > 100 and 0 < nres <= npair
    np.testing.assert_allclose(m @ _v(out), m @ v, atol=1e-11)
    # inelastic collisions never add kinetic energy
    assert m @ (_v(out) ** 2).sum(1) <= m @ (v ** 2).sum(1)
