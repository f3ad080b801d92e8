"""CPU FP64 oracle for Barnes-Hut tree gravity -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it, and it
shares no code with the GPU path: the arithmetic lives in ``rb_oracle.c``
(plain C, FP64, compiled with ``-ffp-contract=off``), this module only
marshals numpy arrays.

What each function follows in the paper (Rein & Liu 2012, REBOUND):
  * ``direct``  -- Eq. (1), direct summation (Sect. 4, 4.1), over the ghost
    boxes of Sect. 2.3;
  * ``tree`` / ``bh`` -- the octree of Sect. 4.2: insertion build, bottom-up
    mass, centre of mass and quadrupole (Hernquist 1987), walk with opening
    angle theta = w / R; one tree per cubic root box (``n_root`` boxes per
    axis, Sect. 2.3); ``Tree.update`` is the reconstruction after the
    particles moved (Sect. 4.2);
  * ``step`` -- the drift-kick-drift step of Sect. 3 with the leap-frog
    (Sect. 3.1) or exact epicycle (Sect. 3.3) drift and the boundaries of
    Sect. 2.3;
  * ``collide`` -- the collisions of Sect. 5 at the end of a step:
    overlapping pairs over the ghost boxes, a randomly ordered queue,
    hard-sphere resolution with a normal coefficient of restitution.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OPEN, PERIODIC, SHEAR = 0, 1, 2
LEAPFROG, EPICYCLE = 0, 1


def build(force: bool = True) -> str:
    """Compile rb_oracle.c into liboracle.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("G", ctypes.c_double),
        ("b", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("quadrupole", ctypes.c_int32),
        ("n_leaf", ctypes.c_int32),
        ("W", ctypes.c_double),
        ("x0", ctypes.c_double * 3),
        ("boundary", ctypes.c_int32),
        ("ng", ctypes.c_int32 * 2),
        ("drift", ctypes.c_int32),
        ("omega", ctypes.c_double),
        ("omega_z", ctypes.c_double),
        ("n_root", ctypes.c_int32 * 3),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(Params)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        vp = ctypes.c_void_p
        L.orc_keys.argtypes = [P, i64, vp, vp, vp, vp]
        L.orc_tree_build.argtypes = [P, i64, i64, vp, vp, vp, vp]
        L.orc_tree_build.restype = vp
        L.orc_tree_update.argtypes = [vp, vp, vp, vp]
        L.orc_tree_update.restype = i64
        L.orc_tree_free.argtypes = [vp]
        L.orc_tree_n_nodes.argtypes = [vp]
        L.orc_tree_n_nodes.restype = i64
        L.orc_tree_n_live.argtypes = [vp]
        L.orc_tree_n_live.restype = i64
        L.orc_tree_selfcheck.argtypes = [vp]
        L.orc_tree_selfcheck.restype = ctypes.c_int
        L.orc_tree_export.argtypes = [vp] * 13
        L.orc_bh.argtypes = [P, vp, i64, vp, vp, vp, ctypes.c_double, vp, i64, vp, vp, vp, vp]
        L.orc_direct.argtypes = [P, i64, i64, vp, vp, vp, vp, ctypes.c_double, vp, i64, vp, vp, vp]
        L.orc_shear_offset.argtypes = [P, ctypes.c_double]
        L.orc_shear_offset.restype = ctypes.c_double
        L.orc_drift.argtypes = [P, i64, vp, vp, vp, vp, vp, vp, ctypes.c_double]
        L.orc_boundary.argtypes = [P, i64, vp, vp, vp, vp, vp, vp, ctypes.c_double]
        L.orc_step.argtypes = [P, i64, i64, vp, vp, vp, vp, vp, vp, vp,
                               ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32]
        L.orc_energy.argtypes = [P, i64, i64, vp, vp, vp, vp, vp, vp, vp]
        L.orc_energy.restype = ctypes.c_double
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_splitmix64.argtypes = [ctypes.c_uint64]
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_collide.argtypes = [P, i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_uint64, vp, i64, vp]
        L.orc_collide.restype = i64
        L.orc_sweep.argtypes = [P, i64, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_uint64, vp, i64, vp]
        L.orc_sweep.restype = i64
        _lib = L
        del dp
    return _lib


def make_params(G=1.0, b=0.0, theta=0.5, quadrupole=False, n_leaf=1, W=1.0,
                x0=(0.0, 0.0, 0.0), boundary=OPEN, ng=(0, 0), drift=LEAPFROG,
                omega=0.0, omega_z=None, n_root=(1, 1, 1), **_ignored) -> Params:
    p = Params()
    p.G, p.b, p.theta = float(G), float(b), float(theta)
    p.quadrupole = int(bool(quadrupole))
    p.n_leaf = int(n_leaf)
    p.W = float(W)
    for a in range(3):
        p.x0[a] = float(x0[a])
    p.boundary = int(boundary)
    p.ng[0], p.ng[1] = int(ng[0]), int(ng[1])
    p.drift = int(drift)
    p.omega = float(omega)
    p.omega_z = float(omega if omega_z is None else omega_z)
    for a in range(3):
        p.n_root[a] = int(n_root[a])
    return p


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def keys(p: Params, x, y, z) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    out = np.empty(len(x), dtype=np.uint64)
    lib().orc_keys(ctypes.byref(p), len(x), _ptr(x), _ptr(y), _ptr(z), _ptr(out))
    return out


def shear_offset(p: Params, t: float) -> float:
    return float(lib().orc_shear_offset(ctypes.byref(p), float(t)))


class Tree:
    """Insertion-built octree with moments (Sect. 4.2)."""

    def __init__(self, p: Params, x, y, z, m, n_active=None):
        self.p = p
        self.x, self.y, self.z, self.m = _f64(x), _f64(y), _f64(z), _f64(m)
        n = len(self.x)
        self.n = n
        self.n_active = n if n_active is None else int(n_active)
        self.h = lib().orc_tree_build(ctypes.byref(p), n, self.n_active, _ptr(self.x),
                                      _ptr(self.y), _ptr(self.z), _ptr(self.m))

    def update(self, x, y, z) -> int:
        """Reconstruction after the particles moved (Sect. 4.2): returns the
        number of particles taken out and inserted again."""
        self.x, self.y, self.z = _f64(x), _f64(y), _f64(z)
        return int(lib().orc_tree_update(self.h, _ptr(self.x), _ptr(self.y), _ptr(self.z)))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_tree_free(h)
            self.h = None

    @property
    def n_nodes(self) -> int:
        return int(lib().orc_tree_n_nodes(self.h))

    @property
    def n_live(self) -> int:
        return int(lib().orc_tree_n_live(self.h))

    def selfcheck(self) -> bool:
        return bool(lib().orc_tree_selfcheck(self.h))

    def export(self) -> dict:
        nn, nl = self.n_nodes, self.n_live
        e = dict(
            level=np.zeros(nn, np.int8), prefix=np.zeros(nn, np.uint64),
            first=np.zeros(nn, np.int64), count=np.zeros(nn, np.int64),
            is_leaf=np.zeros(nn, np.int8), n_child=np.zeros(nn, np.int32),
            first_child=np.zeros(nn, np.int64), M=np.zeros(nn), com=np.zeros((nn, 3)),
            Q=np.zeros((nn, 6)), perm=np.zeros(nl, np.int64), keys=np.zeros(nl, np.uint64))
        order = ["level", "prefix", "first", "count", "is_leaf", "n_child", "first_child",
                 "M", "com", "Q", "perm", "keys"]
        lib().orc_tree_export(self.h, *[_ptr(e[k]) for k in order])
        return e

    def walk(self, s=0.0, targets=None, x=None, y=None, z=None):
        """Accelerations from the tree walk for `targets` (all when None)."""
        x = self.x if x is None else _f64(x)
        y = self.y if y is None else _f64(y)
        z = self.z if z is None else _f64(z)
        if targets is None:
            nt, tp, nout = 0, None, len(x)
        else:
            targets = np.ascontiguousarray(targets, dtype=np.int64)
            nt, tp, nout = len(targets), _ptr(targets), len(targets)
        ax, ay, az = np.zeros(nout), np.zeros(nout), np.zeros(nout)
        stats = np.zeros(3, np.int64)
        lib().orc_bh(ctypes.byref(self.p), self.h, len(x), _ptr(x), _ptr(y), _ptr(z),
                     float(s), tp, nt, _ptr(ax), _ptr(ay), _ptr(az), _ptr(stats))
        self.stats = dict(open_tests=int(stats[0]), cells=int(stats[1]), pp=int(stats[2]))
        return np.stack([ax, ay, az], axis=1)


def bh(p: Params, x, y, z, m, n_active=None, s=0.0, targets=None):
    """Barnes-Hut accelerations (builds the tree, walks it)."""
    t = Tree(p, x, y, z, m, n_active)
    a = t.walk(s=s, targets=targets)
    bh.last_stats = t.stats
    return a


def direct(p: Params, x, y, z, m, n_active=None, s=0.0, targets=None):
    """Eq. (1) by direct summation over all ghost images."""
    x, y, z, m = _f64(x), _f64(y), _f64(z), _f64(m)
    n = len(x)
    na = n if n_active is None else int(n_active)
    if targets is None:
        nt, tp, nout = 0, None, n
    else:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp, nout = len(targets), _ptr(targets), len(targets)
    ax, ay, az = np.zeros(nout), np.zeros(nout), np.zeros(nout)
    lib().orc_direct(ctypes.byref(p), n, na, _ptr(x), _ptr(y), _ptr(z), _ptr(m), float(s),
                     tp, nt, _ptr(ax), _ptr(ay), _ptr(az))
    return np.stack([ax, ay, az], axis=1)


def drift(p: Params, state: dict, tau: float) -> dict:
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    lib().orc_drift(ctypes.byref(p), len(s["x"]), *[_ptr(s[k]) for k in
                    ("x", "y", "z", "vx", "vy", "vz")], float(tau))
    return s


def boundary(p: Params, state: dict, s_off: float) -> dict:
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    lib().orc_boundary(ctypes.byref(p), len(s["x"]), *[_ptr(s[k]) for k in
                       ("x", "y", "z", "vx", "vy", "vz")], float(s_off))
    return s


def step(p: Params, state: dict, m, t0: float, dt: float, nsteps: int,
         n_active=None, use_tree=True) -> dict:
    """nsteps drift-kick-drift steps; returns a new state dict."""
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    m = _f64(m)
    n = len(m)
    na = n if n_active is None else int(n_active)
    lib().orc_step(ctypes.byref(p), n, na, *[_ptr(s[k]) for k in
                   ("x", "y", "z", "vx", "vy", "vz")], _ptr(m), float(t0), float(dt),
                   int(nsteps), int(bool(use_tree)))
    return s


def energy(p: Params, state: dict, m, n_active=None) -> float:
    s = {k: _f64(state[k]) for k in ("x", "y", "z", "vx", "vy", "vz")}
    m = _f64(m)
    n = len(m)
    na = n if n_active is None else int(n_active)
    return float(lib().orc_energy(ctypes.byref(p), n, na, *[_ptr(s[k]) for k in
                 ("x", "y", "z", "vx", "vy", "vz")], _ptr(m)))


def splitmix64(x: int) -> int:
    """The finalising mix of the splitmix64 generator (one output for state x)."""
    return int(lib().orc_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def collide(p: Params, state: dict, m, radius, t: float, eps: float, seed: int,
            cap: int = None):
    """Collisions at time t (Sect. 5): returns (codes in queue order, number
    of pairs, number resolved, new state).  A code is i 2^35 + j 2^7 + k for
    particles i < j overlapping through ghost image k of j."""
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    m, radius = _f64(m), _f64(radius)
    n = len(m)
    cap = 16 * n + 16 if cap is None else int(cap)
    codes = np.zeros(max(cap, 1), dtype=np.uint64)
    nres = np.zeros(1, dtype=np.int64)
    s_off = shear_offset(p, t)
    cnt = lib().orc_collide(ctypes.byref(p), n, *[_ptr(s[k]) for k in
                            ("x", "y", "z", "vx", "vy", "vz")], _ptr(m), _ptr(radius),
                            float(s_off), float(eps), ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                            _ptr(codes), cap, _ptr(nres))
    return codes[:min(int(cnt), cap)].copy(), int(cnt), int(nres[0]), s


def sweep(p: Params, state: dict, m, radius, t: float, dt: float, eps: float, seed: int,
          cap: int = None):
    """Collisions at time t as the plane sweep finds them (Sect. 5): pairs
    whose straight trajectories over the past time-step dt come within
    R_i + R_j; the same queue and resolution as collide().  Returns (codes in
    queue order, number of pairs, number resolved, new state)."""
    s = {k: _f64(state[k]).copy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    m, radius = _f64(m), _f64(radius)
    n = len(m)
    cap = 16 * n + 16 if cap is None else int(cap)
    codes = np.zeros(max(cap, 1), dtype=np.uint64)
    nres = np.zeros(1, dtype=np.int64)
    s_off = shear_offset(p, t)
    cnt = lib().orc_sweep(ctypes.byref(p), n, *[_ptr(s[k]) for k in
                          ("x", "y", "z", "vx", "vy", "vz")], _ptr(m), _ptr(radius),
                          float(s_off), float(dt), float(eps),
                          ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), _ptr(codes), cap, _ptr(nres))
    return codes[:min(int(cnt), cap)].copy(), int(cnt), int(nres[0]), s
