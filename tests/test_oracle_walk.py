"""Pins of the oracle's tree walk (Sect. 4.2) and quadrupole term against the
direct sum, the multipole potential and the paper's accuracy claim
(Sect. 6.1)."""
import math

import numpy as np
import pytest

from paper_1110_4876_amd import inputs
from paper_1110_4876_amd.metrics import force_errors


def _err(a, ref):
    return force_errors(a, ref)


@pytest.mark.parametrize("maker", [
    lambda: inputs.plummer(1024, seed=0),
    lambda: inputs.e1_box(800, 1),
    lambda: inputs.sheet(1500, seed=3),
])
def test_theta_zero_equals_direct(orc, maker):
    # with theta = 0 no cell passes the opening test: every term is direct
    pr = maker()
    for quad in (False, True):
        p = orc.make_params(**dict(pr.params, theta=0.0, quadrupole=quad))
        s = orc.shear_offset(p, 123.0)
        ref = orc.direct(p, pr.x, pr.y, pr.z, pr.m, s=s)
        a = orc.bh(p, pr.x, pr.y, pr.z, pr.m, s=s)
        assert _err(a, ref)["rms"] < 1e-13
        assert orc.bh.last_stats["cells"] == 0


def test_bucket_leaves_theta_zero(orc):
    pr = inputs.plummer(1000, seed=2)
    p = orc.make_params(**dict(pr.params, theta=0.0, n_leaf=6))
    ref = orc.direct(p, pr.x, pr.y, pr.z, pr.m)
    assert _err(orc.bh(p, pr.x, pr.y, pr.z, pr.m), ref)["rms"] < 1e-13


def test_error_converges_as_theta_shrinks(orc):
    pr = inputs.plummer(2000, seed=1)
    ref = orc.direct(orc.make_params(**pr.params), pr.x, pr.y, pr.z, pr.m)
    for quad in (False, True):
        errs = []
        for th in (1.0, 0.7, 0.5, 0.3, 0.15):
            p = orc.make_params(**dict(pr.params, theta=th, quadrupole=quad))
            errs.append(_err(orc.bh(p, pr.x, pr.y, pr.z, pr.m), ref)["rms"])
        assert all(b < a for a, b in zip(errs, errs[1:])), errs
        assert errs[-1] < 0.02 * errs[0]


def _potential_field(M, com, Q, G, pos, h=1e-4):
    """-grad of Phi = -G M / r - (G/2) r.Q.r / r^5 by central differences."""
    def phi(r):
        d = r - com
        rr = math.sqrt(d @ d)
        return -G * M / rr - 0.5 * G * (d @ Q @ d) / rr ** 5
    g = np.zeros(3)
    for a in range(3):
        e = np.zeros(3); e[a] = h
        g[a] = -(phi(pos + e) - phi(pos - e)) / (2 * h)
    return g


def test_far_target_sees_root_multipole(orc):
    # a compact cloud near one corner, a massless target at the far corner:
    # the root passes the opening test and acts as one multipole
    rng = np.random.default_rng(4)
    n = 200
    cloud = rng.uniform(0.0, 0.05, (n, 3)) + 0.01
    m = rng.uniform(0.5, 1.5, n)
    tgt = np.array([[0.97, 0.96, 0.98]])
    P = np.vstack([cloud, tgt])
    mm = np.append(m, 0.0)
    for quad in (False, True):
        p = orc.make_params(G=1.3, W=1.0, x0=(0, 0, 0), theta=0.7, quadrupole=quad)
        t = orc.Tree(p, P[:, 0], P[:, 1], P[:, 2], mm, n_active=n)
        a = t.walk(targets=np.array([n]))[0]
        assert t.stats["cells"] >= 1
        M = m.sum()
        com = (m[:, None] * cloud).sum(0) / M
        Q = np.zeros((3, 3))
        if quad:
            s = cloud - com
            Q = 3 * np.einsum("i,ij,ik->jk", m, s, s) - np.eye(3) * np.sum(m * (s * s).sum(1))
        expect = _potential_field(M, com, Q, 1.3, tgt[0])
        np.testing.assert_allclose(a, expect, rtol=1e-7)


def test_quadrupole_convergence_order(orc):
    # a fixed cluster seen from distance R: the monopole error falls as
    # (s/R)^2, the quadrupole error at least as (s/R)^3 per doubling of R
    rng = np.random.default_rng(8)
    n = 64
    cluster = rng.normal(0.0, 0.01, (n, 3))
    cluster -= cluster.mean(0)
    m = rng.uniform(0.5, 1.5, n)
    res = {False: [], True: []}
    for R in (0.08, 0.16, 0.32, 0.64):
        tgt = np.array([[R, 0.6 * R, -0.3 * R]]) / math.sqrt(1.45)
        P = np.vstack([cluster, tgt])
        mm = np.append(m, 0.0)
        pe = orc.make_params(G=1.0, W=4.0, x0=(-2, -2, -2), theta=0.0)
        ref = orc.direct(pe, P[:, 0], P[:, 1], P[:, 2], mm, n_active=n, targets=np.array([n]))[0]
        for quad in (False, True):
            # theta so large that the root cell (cluster + massless target) is accepted
            p = orc.make_params(G=1.0, W=4.0, x0=(-2, -2, -2), theta=1000.0, quadrupole=quad)
            t = orc.Tree(p, P[:, 0], P[:, 1], P[:, 2], mm, n_active=n)
            a = t.walk(targets=np.array([n]))[0]
            res[quad].append(np.linalg.norm(a - ref) / np.linalg.norm(ref))
    mono = np.array(res[False]); quad = np.array(res[True])
    rm = mono[:-1] / mono[1:]
    rq = quad[:-1] / quad[1:]
    assert np.all((rm > 3.0) & (rm < 5.5)), rm
    assert np.all(rq > 7.0), rq
    assert np.all(quad < mono)


@pytest.mark.parametrize("theta,paper_ratio", [(0.5, 10.0), (0.1, 100.0)])
def test_e1_quadrupole_gain_matches_paper(orc, theta, paper_ratio):
    # Sect. 6.1: 1000 random particles of different masses in a box; the
    # quadrupole expansion is about one order of magnitude more accurate than
    # the monopole at theta ~ 0.5 and two orders at theta ~ 0.1
    pr = inputs.e1_box(1000, 0)
    pm = orc.make_params(**dict(pr.params, theta=theta, quadrupole=False))
    pq = orc.make_params(**dict(pr.params, theta=theta, quadrupole=True))
    ref = orc.direct(pm, pr.x, pr.y, pr.z, pr.m)
    em = _err(orc.bh(pm, pr.x, pr.y, pr.z, pr.m), ref)["paper"]
    eq = _err(orc.bh(pq, pr.x, pr.y, pr.z, pr.m), ref)["paper"]
    ratio = em / eq
    assert paper_ratio / 3.0 < ratio < paper_ratio * 3.0, ratio


def test_test_particles_in_tree(orc):
    pr = inputs.plummer(1500, seed=5)
    na = 1000
    p = orc.make_params(**dict(pr.params, theta=0.0))
    ref = orc.direct(p, pr.x, pr.y, pr.z, pr.m, n_active=na)
    a = orc.bh(p, pr.x, pr.y, pr.z, pr.m, n_active=na)
    assert _err(a, ref)["rms"] < 1e-13


def test_own_ghost_images_are_summed(orc):
    # a lone particle with ghosts: tree and direct agree (both zero by
    # symmetry), and a pair feels the images of both particles
    p = orc.make_params(G=1.0, W=2.0, x0=(-1, -1, -1), boundary=orc.PERIODIC, ng=(1, 1),
                        theta=0.0)
    x = np.array([0.3, -0.4]); y = np.array([0.1, 0.2]); z = np.array([0.0, 0.05])
    m = np.array([1.0, 2.0])
    ref = orc.direct(p, x, y, z, m)
    a = orc.bh(p, x, y, z, m)
    np.testing.assert_allclose(a, ref, rtol=1e-14, atol=1e-15)
