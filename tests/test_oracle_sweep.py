"""Pins of the oracle's plane-sweep collisions (Sect. 5): the pairs whose
straight trajectories over the past time-step come within R_i + R_j.
Checked against closed forms of two-body encounters (a pass-through that
the overlap test misses, the segment's far end), the special cases that
reduce to the overlap test (dt = 0, no motion), and a dense time sampling
of every pair's trajectories on small open, periodic and shear boxes."""
import numpy as np


def _state(x, v):
    x = np.asarray(x, float); v = np.asarray(v, float)
    return dict(x=x[:, 0].copy(), y=x[:, 1].copy(), z=x[:, 2].copy(),
                vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy())


def _open(orc, W=100.0):
    return orc.make_params(W=W, x0=(-W / 2, -W / 2, -W / 2), boundary=orc.OPEN)


def test_pass_through_found_and_left_unresolved(orc):
    # two unit spheres that crossed each other half a step ago: 3 apart now,
    # separating at relative speed 6 (dt = 1); the overlap test misses them
    p = _open(orc)
    st = _state([[-1.5, 0, 0], [1.5, 0, 0]], [[-3.0, 0, 0], [3.0, 0, 0]])
    m = np.ones(2); R = np.ones(2)
    codes, npair, nres, out = orc.sweep(p, st, m, R, 0.0, 1.0, 0.5, 7)
    assert npair == 1 and int(codes[0]) == (0 << 35) | (1 << 7) | 0
    assert nres == 0  # separating now: the approach check leaves it
    np.testing.assert_array_equal(out["vx"], st["vx"])
    _, npair, _, _ = orc.collide(p, st, m, R, 0.0, 0.5, 7)
    assert npair == 0


def test_segment_far_end(orc):
    # closest approach of the infinite lines lies before the step began:
    # the distance at sigma = -dt decides.  Positions -+2, speeds -+1, R = 1:
    # at sigma = -dt the gap is 4 - 2 dt, contact needs it below 2
    p = _open(orc)
    st = _state([[-2.0, 0, 0], [2.0, 0, 0]], [[-1.0, 0, 0], [1.0, 0, 0]])
    m = np.ones(2); R = np.ones(2)
    for dt, want in ((0.99, 0), (1.0, 0), (1.01, 1), (3.0, 1)):
        _, npair, _, _ = orc.sweep(p, st, m, R, 0.0, dt, 0.5, 1)
        assert npair == want, dt


def test_oblique_miss_distance(orc):
    # parallel offset b in y: the closest approach is b whatever dt is
    p = _open(orc)
    m = np.ones(2); R = np.array([0.6, 0.4])
    for b, want in ((0.999, 1), (1.0, 0), (1.2, 0)):
        st = _state([[-5.0, 0, 0], [5.0, b, 0]], [[-2.0, 0, 0], [2.0, 0, 0]])
        _, npair, _, _ = orc.sweep(p, st, m, R, 0.0, 10.0, 0.5, 1)
        assert npair == want, b


def _random_system(rng, n, W):
    x = rng.uniform(-W / 2, W / 2, (n, 3)); x[:, 2] *= 0.1
    v = rng.normal(size=(n, 3)) * 0.8
    R = rng.uniform(0.3, 1.2, n)
    return x, v, R


def test_reduces_to_overlap_test(orc):
    rng = np.random.default_rng(21)
    W = 20.0
    p = orc.make_params(W=W, x0=(-W / 2, -W / 2, -W / 2), boundary=orc.SHEAR, ng=(1, 1),
                        omega=0.3)
    x, v, R = _random_system(rng, 80, W)
    m = rng.uniform(0.5, 2.0, 80)
    a = orc.collide(p, _state(x, v), m, R, 0.9, 0.5, 3)
    # dt = 0: the same pairs, queue and velocities
    b = orc.sweep(p, _state(x, v), m, R, 0.9, 0.0, 0.5, 3)
    assert a[1] == b[1] and a[2] == b[2]
    np.testing.assert_array_equal(a[0], b[0])
    for k in ("vx", "vy", "vz"):
        np.testing.assert_array_equal(a[3][k], b[3][k])
    # a longer step finds a superset
    c = orc.sweep(p, _state(x, v), m, R, 0.9, 2.0, 0.5, 3)
    assert set(int(q) for q in a[0]) <= set(int(q) for q in c[0]) and c[1] > a[1]


def test_dense_time_sampling(orc):
    # every pair and image: min over 5001 instants of |d + u sigma| on
    # [-dt, 0] against the threshold; pairs within 1e-6 of it are skipped
    rng = np.random.default_rng(5)
    W, dt = 20.0, 0.7
    sig = np.linspace(-dt, 0.0, 5001)
    for boundary, ng in ((orc.OPEN, (0, 0)), (orc.PERIODIC, (1, 1)), (orc.SHEAR, (1, 1))):
        om = 0.3
        p = orc.make_params(W=W, x0=(-W / 2, -W / 2, -W / 2), boundary=boundary, ng=ng,
                            omega=om)
        n = 40
        x, v, R = _random_system(rng, n, W)
        t = 2.3
        codes, npair, _, _ = orc.sweep(p, _state(x, v), np.ones(n), R, t, dt, 0.5, 9)
        got = set(int(c) for c in codes)
        assert npair == len(got)
        s = orc.shear_offset(p, t) if boundary == orc.SHEAR else 0.0
        ks = [(0, 0)] if boundary == orc.OPEN else [(ix, iy) for ix in (-1, 0, 1)
                                                     for iy in (-1, 0, 1)]
        checked = 0
        for i in range(n):
            for j in range(i + 1, n):
                for k, (ix, iy) in enumerate(ks):
                    o = np.array([ix * W, iy * W - ix * s, 0.0])
                    wy = -1.5 * om * W * ix if boundary == orc.SHEAR else 0.0
                    d = x[j] + o - x[i]
                    u = v[j] + np.array([0.0, wy, 0.0]) - v[i]
                    dist = np.sqrt(((d[None, :] + u[None, :] * sig[:, None]) ** 2).sum(1)).min()
                    lim = R[i] + R[j]
                    if abs(dist - lim) < 1e-6 * lim:
                        continue
                    code = (i << 35) | (j << 7) | k
                    assert (dist < lim) == (code in got), (boundary, i, j, k)
                    checked += dist < lim
        assert checked > 5
