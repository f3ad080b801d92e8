"""Seeded synthetic inputs shared by the GPU path's tests, the benchmark and
the oracle's tests.

This module only draws initial conditions; it holds none of the gravity,
tree or integrator arithmetic.  Every generator uses
``numpy.random.default_rng(seed)`` (PCG64), and the order of the draws is
fixed in each docstring so that a problem is reproducible across machines.

Workloads (the paper's experiments use random particles and shearing-sheet
patches, Sect. 6.1 and Sect. 7; no dataset is involved):

* ``plummer``   -- equal-mass Plummer sphere (Aarseth, Henon & Wielen 1974),
                   G = M = a = 1, open boundaries, root box [-64, 64)^3.
* ``sheet``     -- shearing-sheet ring patch: radii from dN/dR ~ R^-3 on
                   [1, 4] m, density 400 kg/m^3, box side set by the optical
                   depth, shear-periodic in x, periodic in y.
* ``e1_box``    -- the force-accuracy set-up of Sect. 6.1: random particles
                   of different masses in a box.
* ``batch``     -- many independent sheet patches of uneven size.
* ``ring``      -- a narrow ring of colliding particles on circular orbits
                   around the origin, in an open box (a global simulation,
                   for the azimuthal plane sweep of Sect. 5).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

G_SI = 6.67430e-11

OPEN, PERIODIC, SHEAR = 0, 1, 2
LEAPFROG, EPICYCLE = 0, 1


@dataclass
class Problem:
    """Particles (FP64 SoA, caller order) plus the physical parameters."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray
    params: dict
    n_active: int
    dt: float
    t0: float = 0.0
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return len(self.x)

    def state(self) -> dict:
        return dict(x=self.x, y=self.y, z=self.z, vx=self.vx, vy=self.vy, vz=self.vz)

    def with_params(self, **kw) -> "Problem":
        p = dict(self.params)
        p.update(kw)
        return Problem(self.x, self.y, self.z, self.vx, self.vy, self.vz, self.m, p,
                       self.n_active, self.dt, self.t0, self.name, dict(self.extra))


def base_params(**kw) -> dict:
    p = dict(G=1.0, b=0.0, theta=0.5, quadrupole=False, n_leaf=1, group_size=64,
             W=1.0, x0=(0.0, 0.0, 0.0), boundary=OPEN, ng=(0, 0), drift=LEAPFROG,
             omega=0.0, omega_z=None, n_root=(1, 1, 1))
    p.update(kw)
    if p["omega_z"] is None:
        p["omega_z"] = p["omega"]
    return p


def _isotropic(rng, n):
    """Unit vectors: cos(polar) ~ U(-1, 1), azimuth ~ U(0, 2 pi)."""
    c = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(1.0 - c * c)
    return s * np.cos(phi), s * np.sin(phi), c


def plummer(n: int, seed: int = 0, b: float = 0.01, theta: float = 0.5,
            quadrupole: bool = False, dt: float = 1e-3, W: float = 128.0,
            n_leaf: int = 1) -> Problem:
    """Plummer sphere, total mass 1, scale radius 1, G = 1.

    Draw order: X ~ U(0, 0.999) (n values; r = (X^(-2/3) - 1)^(-1/2), which
    truncates at r ~ 38.7), position directions (2n), speed fractions q by
    rejection from q^2 (1 - q^2)^(7/2) (pairs of uniforms, 2 per trial,
    batches of n), velocity directions (2n).  Speed = q sqrt(2) (1 + r^2)^(-1/4).
    Positions and velocities are then shifted to the centre-of-mass frame.
    """
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 0.999, n)
    r = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    ux, uy, uz = _isotropic(rng, n)
    q = np.empty(0)
    while len(q) < n:
        a = rng.uniform(0.0, 1.0, n)
        g = rng.uniform(0.0, 0.1, n)
        q = np.concatenate([q, a[g < a * a * (1.0 - a * a) ** 3.5]])
    q = q[:n]
    v = q * math.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    wx, wy, wz = _isotropic(rng, n)
    m = np.full(n, 1.0 / n)
    x, y, z = r * ux, r * uy, r * uz
    vx, vy, vz = v * wx, v * wy, v * wz
    for arr in (x, y, z, vx, vy, vz):
        arr -= np.sum(m * arr) / np.sum(m)
    params = base_params(G=1.0, b=b, theta=theta, quadrupole=quadrupole, W=W,
                         x0=(-W / 2, -W / 2, -W / 2), boundary=OPEN, drift=LEAPFROG,
                         n_leaf=n_leaf)
    return Problem(x, y, z, vx, vy, vz, m, params, n, dt, 0.0, f"plummer{n}")


def sheet_from_rng(rng, n: int, tau: float = 0.5, omega: float = 1.95e-4,
                   rho: float = 400.0, r_min: float = 1.0, r_max: float = 4.0,
                   sigma_v: float = 0.01, theta: float = 0.5, quadrupole: bool = True,
                   ng=(1, 1), n_leaf: int = 1, n_root=(1, 1, 1)) -> Problem:
    """Shearing-sheet patch (Sect. 3.3, Sect. 7).

    Draw order: radii by inverse CDF of dN/dR ~ R^-3 on [r_min, r_max]
    (n uniforms), x ~ U(-Lx/2, Lx/2) and y ~ U(-Ly/2, Ly/2) (n each),
    z ~ N(0, R_i) (n), velocity dispersions N(0, sigma_v) for vx, vy, vz (n
    each).  The domain is n_root[0] x n_root[1] x n_root[2] cubic root boxes
    of side W (Sect. 2.3; elongated patches when they differ), with
    Lx Ly = n_root[0] n_root[1] W^2 = sum(pi R^2) / tau from the drawn radii;
    one box (the default) gives the square patch of side L = W.  vy also
    carries the mean shear flow -1.5 Omega x.  SI units, G = 6.67430e-11.
    """
    u = rng.uniform(0.0, 1.0, n)
    a2, b2 = r_min ** -2, r_max ** -2
    R = (a2 - u * (a2 - b2)) ** -0.5
    m = 4.0 / 3.0 * math.pi * R ** 3 * rho
    nx, ny, nz = (int(v) for v in n_root)
    W = math.sqrt(float(np.sum(math.pi * R * R)) / tau / (nx * ny))
    Lx, Ly, Lz = nx * W, ny * W, nz * W
    x = rng.uniform(-Lx / 2, Lx / 2, n)
    y = rng.uniform(-Ly / 2, Ly / 2, n)
    z = rng.normal(0.0, 1.0, n) * R
    vx = rng.normal(0.0, sigma_v, n)
    vy = rng.normal(0.0, sigma_v, n) - 1.5 * omega * x
    vz = rng.normal(0.0, sigma_v, n)
    params = base_params(G=G_SI, b=0.0, theta=theta, quadrupole=quadrupole, W=W,
                         x0=(-Lx / 2, -Ly / 2, -Lz / 2), boundary=SHEAR, ng=tuple(ng),
                         drift=EPICYCLE, omega=omega, omega_z=omega, n_leaf=n_leaf,
                         n_root=(nx, ny, nz))
    dt = 1e-3 * 2.0 * math.pi / omega
    return Problem(x, y, z, vx, vy, vz, m, params, n, dt, 0.0, f"sheet{n}",
                   dict(radius=R, tau=tau))


def sheet(n: int, seed: int = 0, **kw) -> Problem:
    return sheet_from_rng(np.random.default_rng(seed), n, **kw)


def ring(n: int, seed: int = 0, r0: float = 1.0, width: float = 0.01, tau: float = 0.5,
         GM: float = 1.0, sigma_rel: float = 2.0) -> Problem:
    """Narrow ring around a central mass GM at the origin (the central body
    itself is not a particle), open box.

    Draw order: radii by inverse CDF of dN/dR ~ R^-3 on [1, 4] (n uniforms,
    scaled below), orbital radius r ~ U(r0 - width/2, r0 + width/2) (n),
    azimuth ~ U(-pi, pi) (n), z ~ N(0, R_i) (n), velocity dispersions
    N(0, sigma) for the three components (n each), sigma = sigma_rel times
    the mean radius times the orbital frequency at r0.  The radii are scaled
    so that the ring's optical depth sum(pi R^2) / (2 pi r0 width) is tau.
    Velocities: circular Keplerian speed sqrt(GM / r) along the azimuth plus
    the dispersion.  Density 1 (masses 4/3 pi R^3).  dt is 1e-3 of the
    orbital period at r0.
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, n)
    Rt = (1.0 - u * (1.0 - 4.0 ** -2)) ** -0.5
    scale = math.sqrt(tau * 2.0 * math.pi * r0 * width / float(np.sum(math.pi * Rt * Rt)))
    R = Rt * scale
    r = rng.uniform(r0 - width / 2, r0 + width / 2, n)
    ph = rng.uniform(-math.pi, math.pi, n)
    z = rng.normal(0.0, 1.0, n) * R
    om = math.sqrt(GM / r0 ** 3)
    sig = sigma_rel * float(np.mean(R)) * om
    dv = rng.normal(0.0, sig, (3, n))
    vk = np.sqrt(GM / r)
    x, y = r * np.cos(ph), r * np.sin(ph)
    vx = -vk * np.sin(ph) + dv[0]
    vy = vk * np.cos(ph) + dv[1]
    vz = dv[2]
    m = 4.0 / 3.0 * math.pi * R ** 3
    W = 2.2 * (r0 + width)
    params = base_params(G=1.0, b=0.0, W=W, x0=(-W / 2, -W / 2, -W / 2), boundary=OPEN)
    dt = 1e-3 * 2.0 * math.pi / om
    return Problem(x, y, z, vx, vy, vz, m, params, n, dt, 0.0, f"ring{n}",
                   dict(radius=R, tau=tau))


def e1_box(n: int = 1000, seed: int = 0, theta: float = 0.5,
           quadrupole: bool = False) -> Problem:
    """Sect. 6.1: n random particles with different masses in a unit box.

    Draw order: x, y, z ~ U(0, 1) (n each), m ~ U(0.5, 1.5) (n).  G = 1,
    b = 0, no ghost boxes, root box [0, 1)^3.
    """
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, n)
    y = rng.uniform(0.0, 1.0, n)
    z = rng.uniform(0.0, 1.0, n)
    m = rng.uniform(0.5, 1.5, n)
    zero = np.zeros(n)
    params = base_params(G=1.0, b=0.0, theta=theta, quadrupole=quadrupole, W=1.0,
                         x0=(0.0, 0.0, 0.0), boundary=OPEN)
    return Problem(x, y, z, zero.copy(), zero.copy(), zero.copy(), m, params, n, 0.0,
                   0.0, f"e1box{n}")


def uniform_sphere(n: int, seed: int = 0, radius: float = 1.0, mass: float = 1.0,
                   n_test: int = 0, b: float = 0.0) -> Problem:
    """n massive particles uniform in a sphere, then n_test massless test
    particles uniform in the same sphere (indices >= n_active).

    Draw order: radii R u^(1/3) (n + n_test), directions (2 (n + n_test)).
    """
    rng = np.random.default_rng(seed)
    tot = n + n_test
    r = radius * rng.uniform(0.0, 1.0, tot) ** (1.0 / 3.0)
    ux, uy, uz = _isotropic(rng, tot)
    m = np.concatenate([np.full(n, mass / n), np.zeros(n_test)])
    zero = np.zeros(tot)
    W = 4.0 * radius
    params = base_params(G=1.0, b=b, W=W, x0=(-W / 2, -W / 2, -W / 2), boundary=OPEN)
    return Problem(r * ux, r * uy, r * uz, zero.copy(), zero.copy(), zero.copy(), m,
                   params, n, 0.0, 0.0, f"sphere{n}")


def batch(n_patch: int = 256, n_min: int = 2000, n_max: int = 64000,
          tau_min: float = 0.2, tau_max: float = 1.0, seed0: int = 0,
          **kw) -> list:
    """Independent sheet patches, patch p seeded with seed0 + p.

    Per patch the generator first draws N_p = integers(n_min, n_max + 1) and
    tau_p ~ U(tau_min, tau_max), then the patch's particles as in `sheet`.
    """
    out = []
    for p in range(n_patch):
        rng = np.random.default_rng(seed0 + p)
        n = int(rng.integers(n_min, n_max + 1))
        tau = float(rng.uniform(tau_min, tau_max))
        prob = sheet_from_rng(rng, n, tau=tau, **kw)
        prob.name = f"patch{p}"
        out.append(prob)
    return out


def sample_targets(n: int, k: int = 4096, seed: int = 0) -> np.ndarray:
    """k distinct particle indices (without replacement), sorted."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int64)
