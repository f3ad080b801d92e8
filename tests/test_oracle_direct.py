"""Pins of the oracle's direct summation (Eq. 1, Sect. 4.1) and ghost images
(Sect. 2.3) against closed forms, invariants and symmetry."""
import math

import numpy as np
import pytest

from paper_1110_4876_amd import inputs


def test_two_body_closed_form(orc):
    # a = G m r / (r^2 + b^2)^{3/2}, pointing at the other body
    G, b = 2.5, 0.3
    x = np.array([0.1, 0.7]); y = np.array([0.2, -0.1]); z = np.array([0.3, 0.4])
    m = np.array([1.5, 0.25])
    p = orc.make_params(G=G, b=b, W=4.0, x0=(-2, -2, -2))
    a = orc.direct(p, x, y, z, m)
    r = np.array([x[1] - x[0], y[1] - y[0], z[1] - z[0]])
    r2 = float(r @ r)
    expect0 = G * m[1] * r / (r2 + b * b) ** 1.5
    expect1 = -G * m[0] * r / (r2 + b * b) ** 1.5
    np.testing.assert_allclose(a[0], expect0, rtol=1e-14)
    np.testing.assert_allclose(a[1], expect1, rtol=1e-14)


def test_newton_third_law_open(orc):
    pr = inputs.plummer(512, seed=3, b=0.05)
    p = orc.make_params(**pr.params)
    a = orc.direct(p, pr.x, pr.y, pr.z, pr.m)
    f = pr.m[:, None] * a
    assert np.abs(f.sum(axis=0)).max() <= 1e-14 * np.abs(f).sum()


def test_newton_third_law_symmetric_images(orc):
    # periodic images form a symmetric set: momentum is still conserved
    pr = inputs.sheet(600, seed=1)
    p = orc.make_params(**dict(pr.params, boundary=orc.PERIODIC))
    a = orc.direct(p, pr.x, pr.y, pr.z, pr.m)
    f = pr.m[:, None] * a
    assert np.abs(f.sum(axis=0)).max() <= 1e-13 * np.abs(f).sum()


def test_lone_particle_in_periodic_images_feels_no_force(orc):
    # its ghost images sit symmetrically around it
    for bnd in (orc.PERIODIC, orc.SHEAR):
        p = orc.make_params(G=1.0, W=2.0, x0=(-1, -1, -1), boundary=bnd, ng=(1, 1),
                            omega=0.0)
        a = orc.direct(p, [0.3], [-0.2], [0.1], [1.0], s=0.0)
        assert np.abs(a).max() < 1e-15


def test_shear_images_reduce_to_periodic(orc):
    pr = inputs.sheet(400, seed=2)
    pp = orc.make_params(**dict(pr.params, boundary=orc.PERIODIC))
    ps = orc.make_params(**pr.params)
    ref = orc.direct(pp, pr.x, pr.y, pr.z, pr.m)
    a0 = orc.direct(ps, pr.x, pr.y, pr.z, pr.m, s=0.0)
    np.testing.assert_array_equal(a0, ref)
    # a non-zero offset moves the x-ghosts and changes the field
    a1 = orc.direct(ps, pr.x, pr.y, pr.z, pr.m, s=0.25 * pr.params["W"])
    assert np.abs(a1 - ref).max() > 1e-6 * np.abs(ref).max()


def test_shear_offset_definition(orc):
    # the box at +W slides with the mean flow vy = -1.5 Omega x: offset
    # 1.5 Omega W t, folded into [-W/2, W/2]
    pr = inputs.sheet(100, seed=0)
    p = orc.make_params(**pr.params)
    W, om = pr.params["W"], pr.params["omega"]
    for t in (0.0, 10.0, 1234.5, 3.3e4, 1e6):
        s = orc.shear_offset(p, t)
        assert abs(s) <= W / 2
        k = (1.5 * om * W * t - s) / W
        assert abs(k - round(k)) < 1e-9


def test_uniform_sphere_interior_field(orc):
    # shell theorem: inside a uniform sphere a_r = -G M r / R^3
    n, nt = 100_000, 400
    pr = inputs.uniform_sphere(n, seed=5, radius=1.0, mass=1.0, n_test=nt, b=0.0)
    p = orc.make_params(**pr.params)
    tg = np.arange(n, n + nt)
    a = orc.direct(p, pr.x, pr.y, pr.z, pr.m, n_active=n, targets=tg)
    pos = np.stack([pr.x[tg], pr.y[tg], pr.z[tg]], axis=1)
    r = np.linalg.norm(pos, axis=1)
    ar = np.sum(a * pos, axis=1) / r
    keep = (r > 0.15) & (r < 0.85)
    ratio = ar[keep] / (-r[keep])          # expect G M / R^3 = 1
    # a wrong sign, power or G factor moves this far outside the band
    assert abs(np.median(ratio) - 1.0) < 0.05
    assert abs(np.mean(ratio) - 1.0) < 4 * np.std(ratio) / math.sqrt(keep.sum()) + 0.02


def test_thin_shell_interior_field_vanishes(orc):
    rng = np.random.default_rng(11)
    n = 40_000
    c = rng.uniform(-1, 1, n); phi = rng.uniform(0, 2 * np.pi, n)
    s = np.sqrt(1 - c * c)
    x, y, z = s * np.cos(phi), s * np.sin(phi), c
    tx = np.array([0.0, 0.2, -0.3, 0.1]); ty = np.array([0.0, 0.1, 0.2, -0.4])
    tz = np.array([0.0, -0.3, 0.1, 0.2])
    X = np.concatenate([x, tx]); Y = np.concatenate([y, ty]); Z = np.concatenate([z, tz])
    m = np.concatenate([np.full(n, 1.0 / n), np.zeros(4)])
    p = orc.make_params(G=1.0, W=4.0, x0=(-2, -2, -2))
    a = orc.direct(p, X, Y, Z, m, n_active=n, targets=np.arange(n, n + 4))
    # field of the shell at its centre is 0; outside it would be ~1 / r^2
    assert np.abs(a).max() < 0.05
    # and outside the shell it is G M / r^2 towards the centre
    a_out = orc.direct(p, np.append(x, 1.8), np.append(y, 0.0), np.append(z, 0.0),
                       np.append(np.full(n, 1.0 / n), 0.0), n_active=n,
                       targets=np.array([n]))
    assert abs(a_out[0, 0] / (-1.0 / 1.8 ** 2) - 1.0) < 0.02


def test_test_particles_feel_but_do_not_source(orc):
    pr = inputs.plummer(300, seed=4, b=0.02)
    p = orc.make_params(**pr.params)
    na = 200
    a = orc.direct(p, pr.x, pr.y, pr.z, pr.m, n_active=na)
    a_massive_only = orc.direct(p, pr.x[:na], pr.y[:na], pr.z[:na], pr.m[:na])
    np.testing.assert_array_equal(a[:na], a_massive_only)
    assert np.all(np.linalg.norm(a[na:], axis=1) > 0)
