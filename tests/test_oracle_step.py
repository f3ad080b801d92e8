"""Pins of the oracle's drift-kick-drift step (Sect. 3), the epicycle drift
(Sect. 3.3) and the boundaries (Sect. 2.3) against closed forms, an
independent ODE integration and conservation laws."""
import math

import numpy as np
import pytest

from paper_1110_4876_amd import inputs


def _hill_rk4(state, omega, omega_z, T, nsub=4000):
    """Hill's equations without perturbation, by classical RK4."""
    y = np.array(state, dtype=np.float64)

    def f(u):
        x, yy, z, vx, vy, vz = u
        return np.array([vx, vy, vz, 2 * omega * vy + 3 * omega ** 2 * x,
                         -2 * omega * vx, -omega_z ** 2 * z])
    h = T / nsub
    for _ in range(nsub):
        k1 = f(y); k2 = f(y + 0.5 * h * k1); k3 = f(y + 0.5 * h * k2); k4 = f(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def test_epicycle_drift_matches_rk4(orc):
    om, omz = 1.3, 1.7
    p = orc.make_params(drift=orc.EPICYCLE, omega=om, omega_z=omz, boundary=orc.OPEN,
                        W=100.0, x0=(-50, -50, -50))
    st0 = dict(x=[0.3], y=[-0.2], z=[0.05], vx=[0.1], vy=[-0.7], vz=[0.02])
    tau = 0.9
    got = orc.drift(p, st0, tau)
    ref = _hill_rk4([0.3, -0.2, 0.05, 0.1, -0.7, 0.02], om, omz, tau)
    for k, name in enumerate(("x", "y", "z", "vx", "vy", "vz")):
        assert abs(got[name][0] - ref[k]) < 1e-12


def test_epicycle_period(orc):
    om = 0.8
    p = orc.make_params(drift=orc.EPICYCLE, omega=om, omega_z=om, W=100.0,
                        x0=(-50, -50, -50))
    # guiding centre at rest (C = 0): a pure epicycle closes after 2 pi / Omega
    st0 = dict(x=[0.4], y=[0.0], z=[0.1], vx=[0.0], vy=[-2 * om * 0.4], vz=[0.0])
    got = orc.drift(p, st0, 2 * math.pi / om)
    for name in ("x", "y", "z", "vx", "vy", "vz"):
        assert abs(got[name][0] - st0[name][0]) < 1e-12


def test_shear_flow_is_stationary(orc):
    pr = inputs.sheet(200, seed=0)
    om = pr.params["omega"]
    p = orc.make_params(**dict(pr.params, G=0.0))
    st = dict(x=pr.x, y=pr.y, z=np.zeros(pr.n), vx=np.zeros(pr.n), vy=-1.5 * om * pr.x,
              vz=np.zeros(pr.n))
    dt = pr.dt
    out = orc.drift(p, st, dt)
    np.testing.assert_allclose(out["x"], st["x"], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(out["y"], st["y"] - 1.5 * om * pr.x * dt, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(out["vy"], st["vy"], rtol=1e-12, atol=1e-15)


def test_leapfrog_energy_error_is_second_order(orc):
    pr = inputs.plummer(1024, seed=0, b=0.05)
    p = orc.make_params(**pr.params)
    e0 = orc.energy(p, pr.state(), pr.m)
    errs = []
    for dt in (4e-3, 2e-3, 1e-3):
        # T = 0.5: a time short against the crossing time keeps close
        # encounters rare, so the error is the smooth O(dt^2) term
        st = orc.step(p, pr.state(), pr.m, 0.0, dt, int(round(0.5 / dt)), use_tree=False)
        errs.append(abs(orc.energy(p, st, pr.m) - e0))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, (errs, r1, r2)


def test_leapfrog_is_time_reversible(orc):
    pr = inputs.plummer(256, seed=1, b=0.05)
    p = orc.make_params(**pr.params)
    fwd = orc.step(p, pr.state(), pr.m, 0.0, 1e-3, 50, use_tree=True)
    back = orc.step(p, fwd, pr.m, 0.05, -1e-3, 50, use_tree=True)
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(back[k], getattr(pr, k), rtol=0, atol=1e-12)


def test_single_step_dkd_sequence(orc):
    # one DKD step equals drift(dt/2), kick with the forces at the drifted
    # positions, drift(dt/2)
    pr = inputs.plummer(300, seed=2, b=0.02)
    p = orc.make_params(**pr.params)
    dt = pr.dt
    st = orc.step(p, pr.state(), pr.m, 0.0, dt, 1, use_tree=False)
    half = {k: getattr(pr, k) + getattr(pr, "v" + k) * dt / 2 for k in ("x", "y", "z")}
    a = orc.direct(p, half["x"], half["y"], half["z"], pr.m)
    v = {k: getattr(pr, "v" + k) + a[:, i] * dt for i, k in enumerate(("x", "y", "z"))}
    for k in ("x", "y", "z"):
        np.testing.assert_allclose(st[k], half[k] + v[k] * dt / 2, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(st["v" + k], v[k], rtol=1e-15, atol=1e-18)


def test_shear_wrap_keeps_guiding_centre_velocity(orc):
    # crossing the x face keeps vy + 1.5 Omega x unchanged and shifts y by
    # the box offset (box large enough that y needs no second wrap)
    pr = inputs.sheet(5000, seed=0)
    W, om = pr.params["W"], pr.params["omega"]
    p = orc.make_params(**pr.params)
    st = dict(x=np.array([0.5 * W + 1.0, -0.5 * W - 2.0]), y=np.array([10.0, -20.0]),
              z=np.array([0.0, 0.0]), vx=np.array([0.1, -0.1]),
              vy=np.array([-1.5 * om * (0.5 * W + 1.0), -1.5 * om * (-0.5 * W - 2.0)]),
              vz=np.array([0.0, 0.0]))
    s = 0.3 * W
    out = orc.boundary(p, st, s)
    np.testing.assert_allclose(out["x"], [-0.5 * W + 1.0, 0.5 * W - 2.0], rtol=1e-14)
    np.testing.assert_allclose(out["y"], [10.0 + s, -20.0 - s], rtol=1e-14)
    np.testing.assert_allclose(out["vy"] + 1.5 * om * out["x"], st["vy"] + 1.5 * om * st["x"],
                               rtol=1e-12, atol=1e-15)


def test_open_boundary_removes_leaving_particles(orc):
    p = orc.make_params(W=2.0, x0=(-1, -1, -1), boundary=orc.OPEN)
    st = dict(x=np.array([0.9, 0.0]), y=np.zeros(2), z=np.zeros(2), vx=np.array([1.0, 0.0]),
              vy=np.zeros(2), vz=np.zeros(2))
    out = orc.step(p, st, np.array([1e-9, 1e-9]), 0.0, 0.2, 1, use_tree=True)
    assert np.isnan(out["x"][0]) and out["vx"][0] == 0.0
    assert np.isfinite(out["x"][1])


def test_energy_closed_forms(orc):
    # two bodies: kinetic + softened pair potential written out by hand; a
    # massless test particle adds kinetic energy only (its mass is not a
    # source) and a removed particle (NaN position) adds nothing
    G, b = 0.7, 0.05
    p = orc.make_params(G=G, b=b, W=100.0, x0=(-50, -50, -50))
    st = {"x": np.array([0.0, 1.0, 2.0, np.nan]), "y": np.array([0.0, 0.5, 0.0, 0.0]),
          "z": np.array([0.0, -0.25, 0.0, 0.0]), "vx": np.array([1.0, 0.0, 0.3, 5.0]),
          "vy": np.array([0.0, -2.0, 0.0, 5.0]), "vz": np.array([0.5, 0.0, 0.0, 5.0])}
    m = np.array([2.0, 3.0, 4.0, 1.0])
    # particle 2 is a test particle (index >= n_active = 2); particle 3 is removed
    e = orc.energy(p, st, m, n_active=2)
    r2 = 1.0 + 0.25 + 0.0625
    ek = 0.5 * 2.0 * (1.0 + 0.25) + 0.5 * 3.0 * 4.0 + 0.5 * 4.0 * 0.09
    ep = -G * 2.0 * 3.0 / math.sqrt(r2 + b * b)
    assert abs(e - (ek + ep)) <= 1e-14 * abs(ek)


def test_periodic_wrap(orc):
    # plain periodic boundaries (Sect. 2.3): a particle leaving through an x
    # or y face re-enters through the opposite one, x -> x -+ W, with y (for
    # an x crossing), z and the velocity unchanged; z stays open
    W = 10.0
    p = orc.make_params(W=W, x0=(-5.0, -5.0, -5.0), boundary=orc.PERIODIC, ng=(1, 1),
                        omega=0.7)
    st = dict(x=np.array([5.0, 5.75, -5.25, 1.0, 2.0, 0.5]),
              y=np.array([1.0, -2.0, 3.0, 5.5, -5.125, 0.0]),
              z=np.array([0.5, 0.0, -1.0, 0.0, 0.0, 5.0]),
              vx=np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6]),
              vy=np.array([-0.1, -0.2, -0.3, -0.4, -0.5, -0.6]),
              vz=np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0]))
    out = orc.boundary(p, st, 1.234)  # the shear offset is ignored here
    np.testing.assert_array_equal(out["x"][:5], [-5.0, -4.25, 4.75, 1.0, 2.0])
    np.testing.assert_array_equal(out["y"][:5], [1.0, -2.0, 3.0, -4.5, 4.875])
    np.testing.assert_array_equal(out["z"][:5], st["z"][:5])
    for k in ("vx", "vy", "vz"):
        np.testing.assert_array_equal(out[k][:5], st[k][:5])
    # the last one left through the open z face: removed
    assert np.isnan(out["x"][5]) and out["vz"][5] == 0.0


def _sheet_params(orc, W=1000.0, omega=2e-4):
    return orc.make_params(G=1.0, b=0.0, W=W, x0=(-0.5 * W, -0.5 * W, -0.5 * W),
                           boundary=orc.SHEAR, ng=(1, 1), drift=orc.EPICYCLE, omega=omega)


def test_shear_ghost_image_is_the_unwrapped_neighbour(orc):
    # Geometry of the shear-periodic ghost boxes at a time with s != 0: a
    # source just outside the +x face, and a massless target d = 1 W/1000
    # away just inside it.  The boundary wraps the source to the -x side
    # (shifted in y by s); its ghost image in the box at +W must then sit
    # where the source was, so the target feels the same nearby source
    # before and after the wrap.  The image sets differ only by far images
    # (relative size (d/W)^2).  A flipped sign of the wrap's y shift, or of
    # the image offset, moves the nearby image by 2s and fails.
    W = 1000.0
    p = _sheet_params(orc, W)
    for s in (0.31 * W, -0.44 * W, 0.49 * W):
        for ys in (12.0, 0.5 * W - 0.4):  # the second one also wraps in y
            src = dict(x=np.array([0.5 * W + 0.3]), y=np.array([ys]), z=np.array([0.0]),
                       vx=np.zeros(1), vy=np.zeros(1), vz=np.zeros(1))
            wr = orc.boundary(p, src, s)
            assert wr["x"][0] < 0  # it was wrapped
            tx, ty = 0.5 * W - 0.7, ys - 0.2  # target 1.02 m from the source
            m = np.array([1.0, 0.0])
            before = orc.direct(p, [src["x"][0], tx], [src["y"][0], ty], [0.0, 0.0], m,
                                n_active=1, s=s, targets=[1])[0]
            after = orc.direct(p, [wr["x"][0], tx], [wr["y"][0], ty], [0.0, 0.0], m,
                               n_active=1, s=s, targets=[1])[0]
            near = np.array([0.5 * W + 0.3 - tx, ys - ty, 0.0])
            a_near = near / np.linalg.norm(near) ** 3
            assert np.linalg.norm(after - before) <= 1e-4 * np.linalg.norm(a_near)
            assert np.linalg.norm(after - a_near) <= 1e-4 * np.linalg.norm(a_near)


def test_shear_image_follows_the_drifted_particle(orc):
    # Hill's equations are invariant under the shear boost x -> x - W,
    # y -> y + (3/2) Omega W t + c, vy -> vy + (3/2) Omega W.  So a particle
    # wrapped across the +x face at t1 and then drifted with the epicycle
    # map must keep its ghost image in the box at +W on the track of the
    # same particle drifted without the wrap, at every later time t2 -- with
    # the images' shear offset s(t2).  This pins the direction of the shear
    # offset (relative to the mean flow vy = -(3/2) Omega x of the drift),
    # the wrap's y and vy shifts and the image offset together: flipping any
    # of them moves the image by 2 s(t1) ~ 0.6 W or by twice the slide.
    W, om = 1000.0, 2e-4
    p = _sheet_params(orc, W, om)
    t1 = 0.37 * 2 * math.pi / om
    # drift times over which the boxes slide by 20, 60 and 150 m against
    # each other: far more than d, while the particle stays near the box
    for slide in (20.0, 60.0, 150.0):
        tau = slide / (1.5 * om * W)
        x1 = 0.5 * W + 0.25
        src = dict(x=np.array([x1]), y=np.array([-100.0]), z=np.array([0.5]),
                   vx=np.array([0.02]), vy=np.array([-1.5 * om * x1 + 0.01]),
                   vz=np.array([0.0]))
        wr = orc.boundary(p, src, orc.shear_offset(p, t1))
        assert wr["x"][0] < 0
        free = orc.drift(p, src, tau)   # the unwrapped particle
        moved = orc.drift(p, wr, tau)   # the wrapped one
        t2 = t1 + tau
        s2 = orc.shear_offset(p, t2)
        # a massless target 0.8 m from the unwrapped particle's position:
        # the nearby source must be the wrapped particle's ghost image
        tx, ty, tz = free["x"][0] + 0.8, free["y"][0], free["z"][0]
        m = np.array([1.0, 0.0])
        a = orc.direct(p, [moved["x"][0], tx], [moved["y"][0], ty], [moved["z"][0], tz], m,
                       n_active=1, s=s2, targets=[1])[0]
        near = np.array([-0.8, 0.0, 0.0])
        a_near = near / 0.8 ** 3
        assert np.linalg.norm(a - a_near) <= 1e-4 * np.linalg.norm(a_near), (tau, a, a_near)
